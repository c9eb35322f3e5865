// Small-state phase of one online DMD update (one workgroup, FP64).
//
// Brand's column append (the paper's reference [brand2006fast], used as in
// Sec. 2.3): with p = U^T x and rho the norm of the part of x outside
// span(U),
//     [U S W^T, x] = [U q] K blockdiag(W, 1)^T,   K = [[diag(sigma), p], [0, rho]],
// so an SVD K = U_k diag(sigma') V_k^T updates all three factors:
// U <- [U q] U_k, sigma <- sigma', W <- blockdiag(W, 1) V_k, each cut to the
// kept rank r'.  The right factor W is never stored; for chained pairs
// (y_j = x_{j+1}) the reduced operator A~ = U^T Y W S^-1 only needs the
// shifted product C = W[2:]^T W[:-1], the last row w of W and p_y = U^T y:
//     A~_ij = (sigma_i C_ij + p_y,i w_j) / sigma_j,
//     C <- V_k^T [[C, 0], [w^T, 0]] V_k,   w <- last row of V_k,
//     p_y <- U_k^T [U^T y; q^T y].
// The SVD of K is a one-sided (Hestenes) Jacobi iteration with a
// round-robin pair order, one 32-lane half-wavefront per column pair.
#include <hip/hip_runtime.h>
#include <math.h>

#include "odmd_internal.h"
#include "pass.h"

namespace odmd {

constexpr int LDK = MMAX + 1;        // LDS leading dimension of the core
constexpr int MAX_SWEEPS = 40;

__device__ __forceinline__ double halfwave_sum(double v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
  return v;
}

// Round-robin (circle) schedule: in round k of Mp-1 rounds, pair i of Mp/2.
__device__ __forceinline__ void rr_pair(int k, int i, int Mp, int& a, int& b) {
  if (i == 0) {
    a = k;
    b = Mp - 1;
  } else {
    a = (k + i) % (Mp - 1);
    b = (k - i + (Mp - 1)) % (Mp - 1);
  }
  if (b < a) { const int t = a; a = b; b = t; }
}

// One-sided Jacobi on the M columns of A (LDS, column-major, ld LDK), with
// the rotations accumulated in V.  On return the columns of A are mutually
// orthogonal: A = (A_in V) with ||A_j|| the singular values.
__device__ int jacobi_sweeps(double* A, double* V, double* d, int M, int* flag) {
  const int tid = threadIdx.x, hw = tid >> 5, hl = tid & 31;
  const int nhw = CORE_THREADS / 32;
  const int Mp = M + (M & 1);
  const int npair = Mp / 2;
  const double tolJ = 4.0 * sqrt((double)M) * 1.1102230246251565e-16;
  int sweep = 0;
  for (; sweep < MAX_SWEEPS; ++sweep) {
    for (int col = hw; col < M; col += nhw) {
      double s = 0.0;
      for (int row = hl; row < M; row += 32) s += A[col * LDK + row] * A[col * LDK + row];
      s = halfwave_sum(s);
      if (hl == 0) d[col] = s;
    }
    if (tid == 0) *flag = 0;
    __syncthreads();
    // Columns below the rounding floor of the largest one are numerically
    // zero (an exactly rank-deficient core, e.g. x in span(U)); rotating them
    // only reshuffles rounding noise, so they are left alone.
    double dmax = 0.0;
    for (int j = 0; j < M; ++j) dmax = fmax(dmax, d[j]);
    const double dfloor = dmax * (M * 2.220446049250313e-16) * (M * 2.220446049250313e-16);
    for (int round = 0; round < Mp - 1; ++round) {
      for (int pi = hw; pi < npair; pi += nhw) {
        int a, b;
        rr_pair(round, pi, Mp, a, b);
        if (b >= M) continue;
        double g = 0.0;
        for (int row = hl; row < M; row += 32) g += A[a * LDK + row] * A[b * LDK + row];
        g = halfwave_sum(g);
        const double al = d[a], be = d[b];
        if (fmin(al, be) > dfloor && fabs(g) > tolJ * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * g);
          const double az = fabs(zeta);
          double t = az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + zeta * zeta));
          if (zeta < 0.0) t = -t;
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          for (int row = hl; row < M; row += 32) {
            const double xa = A[a * LDK + row], xb = A[b * LDK + row];
            A[a * LDK + row] = c * xa - s * xb;
            A[b * LDK + row] = s * xa + c * xb;
            const double va = V[a * LDK + row], vb = V[b * LDK + row];
            V[a * LDK + row] = c * va - s * vb;
            V[b * LDK + row] = s * va + c * vb;
          }
          if (hl == 0) {
            d[a] = al - t * g;
            d[b] = be + t * g;
            *flag = 1;
          }
        }
      }
      __syncthreads();
    }
    const int rotated = *flag;
    __syncthreads();
    if (!rotated) break;
  }
  return sweep + 1;
}

__global__ __launch_bounds__(CORE_THREADS) void k_core(CoreArgs c) {
  DevState* __restrict__ st = c.st;
  __shared__ double sA[MMAX * LDK];
  __shared__ double sV[MMAX * LDK];
  __shared__ double red[CORE_THREADS];
  __shared__ double tot[PW];
  __shared__ double sd[MMAX + 1];
  __shared__ double p2[RMAX], pyr[RMAX], pyn[RMAX], wn[RMAX], sgn[RMAX];
  __shared__ int perm[MMAX + 1];
  __shared__ int flag;
  __shared__ double sc[8];
  __shared__ int si[4];

  const int tid = threadIdx.x;
  const int r = st->r, rs = st->rs, pending = st->pending;

  // 1. fixed-order reduction of the per-workgroup partial sums
  constexpr int NSPLIT = CORE_THREADS / PW;
  if (tid < NSPLIT * PW) {
    const int v = tid % PW, s = tid / PW;
    double acc = 0.0;
    for (int b = s; b < c.nblk; b += NSPLIT) acc += c.partials[(int64_t)b * PW + v];
    red[s * PW + v] = acc;
  }
  __syncthreads();
  if (tid < PW) {
    double t = 0.0;
    for (int s = 0; s < NSPLIT; ++s) t += red[s * PW + tid];
    tot[tid] = t;
  }
  __syncthreads();

  // 2. second projection p2 = U^T e and U^T y in the basis the pass used
  if (tid < r) {
    double a2, b2;
    if (pending) {
      a2 = st->g[tid] * tot[P_SEE];
      b2 = st->g[tid] * tot[P_SEY];
      for (int j = 0; j < rs; ++j) {
        a2 += st->G[tid * RMAX + j] * tot[P_SUE + j];
        b2 += st->G[tid * RMAX + j] * tot[P_SUY + j];
      }
    } else {
      a2 = tot[P_SUE + tid];
      b2 = tot[P_SUY + tid];
    }
    p2[tid] = a2;
    pyr[tid] = b2;
  }
  __syncthreads();

  // 3. checks, residual norm, growth test
  if (tid == 0) {
    const double ee = tot[P_EE], xx = tot[P_XX], ey = tot[P_EY], yy = tot[P_YY];
    double pp = 0.0, py2 = 0.0;
    for (int j = 0; j < r; ++j) {
      pp += p2[j] * p2[j];
      py2 += p2[j] * pyr[j];
    }
    int skip = 0;
    if (!(isfinite(ee) && isfinite(xx) && isfinite(ey) && isfinite(yy) && isfinite(pp) &&
          isfinite(py2))) {
      skip = ST_NONFINITE;
    } else if (st->m > 0 && xx != st->yy_prev) {
      skip = ST_SEQ;
    }
    double rho = sqrt(fmax(ee - pp, 0.0));
    const int grow = !skip && rho > 0.0 && rho > st->tol * sqrt(xx);
    if (!grow) rho = 0.0;
    sc[0] = rho;
    sc[1] = grow ? (ey - py2) / rho : 0.0;   // q^T y
    sc[2] = yy;
    si[0] = skip;
    si[1] = grow;
  }
  __syncthreads();
  const int skip = si[0];
  if (skip) {
    // The pass already wrote the rotated basis: it is now the stored one.
    if (tid < RMAX) st->a[tid] = tid < r ? st->py[tid] : 0.0;
    if (tid == 0) {
      st->status |= skip;
      st->rs = r;
      st->pending = 0;
      st->use_e = 0;
      st->beta = 0.0;
    }
    return;
  }
  const int grow = si[1];
  const double rho = sc[0], qy = sc[1];

  // 4. core K = [[diag(sigma), p], [0, rho]], p = p1 + p2 with p1 = cached p_y
  const int M = r + 1;
  for (int idx = tid; idx < M * M; idx += CORE_THREADS) {
    const int i = idx % M, j = idx / M;
    double v;
    if (j < r) v = (i == j) ? st->sigma[j] : 0.0;
    else v = (i < r) ? st->py[i] + p2[i] : rho;
    sA[j * LDK + i] = v;
    sV[j * LDK + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  // 5. SVD of the core
  const int sweeps = jacobi_sweeps(sA, sV, sd, M, &flag);

  // 6. singular values (exact column norms), descending order, truncation
  if (tid < M) {
    double s = 0.0;
    for (int i = 0; i < M; ++i) s += sA[tid * LDK + i] * sA[tid * LDK + i];
    sd[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < M) {
    const double me = sd[tid];
    int rank = 0;
    for (int k = 0; k < M; ++k) rank += (sd[k] > me) || (sd[k] == me && k < tid);
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    const double smax = sd[perm[0]];
    int rn = 0;
    if (smax > 0.0) {
      for (int k = 0; k < M; ++k) rn += sd[k] > st->tol * smax;
      rn = min(rn, c.r_max);
    }
    si[2] = rn;
  }
  __syncthreads();
  const int rn = si[2];
  if (rn == 0) {   // nothing kept (zero snapshots so far)
    if (tid == 0) {
      st->r = 0;
      st->rs = 0;
      st->pending = 0;
      st->use_e = 0;
      st->m += 1;
      st->yy_prev = sc[2];
      st->last_rho = rho;
      st->sweeps = sweeps;
      st->eig_valid = 0;
      if (sweeps > MAX_SWEEPS) st->status |= ST_NOCONV;
    }
    return;
  }

  // 7. U_k = (K V_k) diag(sigma')^-1 for kept columns; new p_y and signs
  //    U_k(i, jj) = sA[perm[jj]*LDK + i] / sd[perm[jj]]
  if (tid < rn) {
    const int pj = perm[tid];
    const double inv = 1.0 / sd[pj];
    double s = sA[pj * LDK + r] * qy;
    for (int i = 0; i < r; ++i) s += sA[pj * LDK + i] * pyr[i];
    pyn[tid] = s * inv;
    wn[tid] = sV[pj * LDK + r];
    sgn[tid] = sd[pj];
  }
  __syncthreads();

  // 8. rotation for the next pass: U' = U G + e g^T with
  //    G = U_k[:r, :r'] - (p2 / rho) U_k[r, :r'],  g = U_k[r, :r'] / rho
  const double irho = grow ? 1.0 / rho : 0.0;
  for (int idx = tid; idx < RMAX * RMAX; idx += CORE_THREADS) {
    const int j = idx % RMAX, k = idx / RMAX;   // row j of G (input column), column k
    double v = 0.0;
    if (j < r && k < rn) {
      const int pk = perm[k];
      const double inv = 1.0 / sd[pk];
      v = (sA[pk * LDK + j] - p2[j] * irho * sA[pk * LDK + r]) * inv;
    }
    st->G[k * RMAX + j] = v;
    if (c.basis_f32) st->G32[k * RMAX + j] = (float)v;
  }
  if (tid < RMAX) {
    double gk = 0.0;
    if (tid < rn) {
      const int pk = perm[tid];
      gk = sA[pk * LDK + r] * irho / sd[pk];
    }
    st->g[tid] = gk;
    if (c.basis_f32) st->g32[tid] = (float)gk;
    // a = G p1 with p1 = new p_y (the next x equals this y)
    double av = 0.0;
    if (tid < r) {
      for (int k = 0; k < rn; ++k) {
        const int pk = perm[k];
        av += (sA[pk * LDK + tid] - p2[tid] * irho * sA[pk * LDK + r]) / sd[pk] * pyn[k];
      }
    }
    st->a[tid] = av;
  }
  if (tid == 0) {
    double b = 0.0;
    for (int k = 0; k < rn; ++k) b += sA[perm[k] * LDK + r] * irho / sd[perm[k]] * pyn[k];
    st->beta = b;
  }
  __syncthreads();

  // 9. T = E V_k with E = [[C, 0], [w^T, 0]] (into sA, no longer needed)
  for (int idx = tid; idx < M * rn; idx += CORE_THREADS) {
    const int i = idx % M, bcol = idx / M;
    const int pb = perm[bcol];
    double s = 0.0;
    if (i < r) {
      for (int j = 0; j < r; ++j) s += st->C[j * RMAX + i] * sV[pb * LDK + j];
    } else {
      for (int j = 0; j < r; ++j) s += st->w[j] * sV[pb * LDK + j];
    }
    sA[bcol * LDK + i] = s;   // U_k is no longer read (synced above)
  }
  __syncthreads();

  // 10. C <- V_k^T T (kept block), sigma, w, p_y, A~
  for (int idx = tid; idx < rn * rn; idx += CORE_THREADS) {
    const int i = idx % rn, j = idx / rn;
    const int pi = perm[i];
    double s = 0.0;
    for (int k = 0; k < M; ++k) s += sV[pi * LDK + k] * sA[j * LDK + k];
    st->C[j * RMAX + i] = s;
    st->At[j * RMAX + i] = (sgn[i] * s + pyn[i] * wn[j]) / sgn[j];
  }
  if (tid < rn) {
    st->sigma[tid] = sgn[tid];
    st->w[tid] = wn[tid];
    st->py[tid] = pyn[tid];
  }
  if (tid == 0) {
    st->rs = r;
    st->r = rn;
    st->pending = 1;
    st->use_e = grow;
    st->m += 1;
    st->yy_prev = sc[2];
    st->last_rho = rho;
    st->sweeps = sweeps;
    st->eig_valid = 0;
    if (sweeps > MAX_SWEEPS) st->status |= ST_NOCONV;
  }
}

hipError_t launch_core(const CoreArgs& c, hipStream_t s) {
  hipLaunchKernelGGL(k_core, dim3(1), dim3(CORE_THREADS), 0, s, c);
  return hipGetLastError();
}

}  // namespace odmd
