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
// The SVD of K comes from its secular equation (below); a one-sided
// (Hestenes) Jacobi iteration with a round-robin pair order, one 32-lane
// half-wavefront per column pair, is the fallback.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "odmd_internal.h"
#include "pass.h"
#include "xlane.h"

namespace odmd {

constexpr int LDK = MMAX + 1;        // LDS leading dimension of the core
constexpr int LDQ = RMAX + 1;        // LDS row stride of Q (rows read by 16 lanes at once
                                     // fall in distinct banks)
constexpr int MAX_SWEEPS = 40;

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
__device__ __forceinline__ int jacobi_sweeps(double* A, double* V, double* d, int M, int* flag) {
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

// SVD of the core by its secular equation (used first; Jacobi is the fallback).
//
// K K^T = D^2 + z z^T with D = diag(sigma_1..sigma_r, 0) and z = [p; rho], so
// the squared singular values of K are the roots lambda of
//     f(lambda) = 1 + sum_j z_j^2 / (d_j^2 - lambda) = 0,
// one in each gap between consecutive d_j^2 and one above d_1^2.  With the
// roots known, left and right singular vectors have closed forms,
//     u_i[j] = z_j / (d_j^2 - lambda_i),   v_i[j] = d_j z_j / (d_j^2 - lambda_i),
// v_i[r] = -1 (then normalised).  Numerical orthogonality needs z replaced by
// the z~ for which the computed roots are exact (Loewner's formula, the
// Gu-Eisenstat construction), and every difference d_j^2 - lambda_i formed
// as (d_j - d_K)(d_j + d_K) - mu_i with lambda_i = d_K^2 + mu_i stored relative
// to its nearer pole d_K.  Entries of z below 8 eps max(|d|, |z|) are deflated
// (the pair (d_j, e_j) is already singular), as are poles closer than that
// (a Givens rotation moves their z weight onto one of them); the zero pole
// is never deflated: a zero rho is raised to that tolerance.  Each root is
// found by one 16-lane quarter-wavefront: bracketed iteration on the
// two-pole rational model of f (Li's "middle way"), from the root of a
// two-pole model with the other terms frozen, falling back to bisection.
constexpr int SEC_MAXIT = 64;
constexpr double SEC_EPS = 2.220446049250313e-16;
constexpr int SEC_TERMS = (MMAX + 15) / 16;   // secular terms per lane of a quarter-wave

struct SecShared {
  double dj[MMAX], zz[MMAX], zs[MMAX];   // live poles (descending), z^2, sign of z
  double rK[MMAX], mu[MMAX];             // root i: lambda_i = rK[i]^2 + mu[i]
  double zh[MMAX], nrm[2 * MMAX];
  double gc[MMAX], gs[MMAX], d[MMAX], z[MMAX];
  int J[MMAX], gi[MMAX], gj[MMAX], dflist[MMAX], live[MMAX];
  int nd, ndef, ngiv, fail;
  double tol;
};

// 1/x from the hardware reciprocal estimate and two Newton steps
// (r <- r + r (1 - x r)), each squaring the relative error: about 1 ulp,
// for the finite non-zero x of the secular terms
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}

// lambda_i - d_j^2 = (d_K^2 - d_j^2) + mu_i, with d_K the pole root i is stored against
__device__ __forceinline__ double lam_minus_d(const SecShared& S, int i, double dj) {
  const double dK = S.rK[i];
  return (dK - dj) * (dK + dj) + S.mu[i];
}

// Returns true on success; fills A (columns U_k * sigma'), V (V_k), column
// order arbitrary (the caller sorts by column norm), and the norms of A's
// columns into sdo (norms_ok: no tied-pole rotation touched them after).
__device__ __forceinline__ bool secular_svd(double* A, double* V, const double* sig, const double* pv, double rho,
                            int r, SecShared& S, double* sdo, bool& norms_ok) {
  const int tid = threadIdx.x;
  const int n = r + 1;

  // Set-up, by the first wavefront alone (one workgroup barrier at its
  // end): the tolerance 8 eps max(|d|, |z|), the poles and weights, the
  // deflation of tiny z (never the zero pole) keeping descending order, the
  // tied-pole check and merge, and the live poles' staging.  Lane t holds
  // entries t and t + 64.  Within one wavefront the LDS writes of one step
  // are seen by the next (the wave's LDS operations complete in order; the
  // wavefront fence keeps the compiler from reordering them).
  if (tid < 64) {
    const int j0 = tid, j1 = tid + 64;
    double m = 0.0;
    for (int j = tid; j < r; j += 64) m = fmax(m, fmax(fabs(sig[j]), fabs(pv[j])));
    if (tid == 0) m = fmax(m, fabs(rho));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    const double tl = 8.0 * SEC_EPS * m;
    const double rz = fabs(rho) <= tl ? tl : rho;
    const double d0 = j0 < r ? sig[j0] : 0.0, z0 = j0 < r ? pv[j0] : rz;
    const double d1 = j1 < r ? sig[j1] : 0.0, z1 = j1 < r ? pv[j1] : rz;
    if (j0 < n) {
      S.d[j0] = d0;
      S.z[j0] = z0;
    }
    if (j1 < n) {
      S.d[j1] = d1;
      S.z[j1] = z1;
    }
    const bool l0 = j0 < n && !(j0 < r && fabs(z0) <= tl);
    const bool l1 = j1 < n && !(j1 < r && fabs(z1) <= tl);
    const unsigned long long m0 = __ballot(l0), m1 = __ballot(l1);
    const unsigned long long lt = (tid == 0) ? 0ull : (~0ull >> (64 - tid));
    const int p0 = __popcll(m0 & lt), p1 = __popcll(m1 & lt);
    const int nl0 = __popcll(m0), nd0 = min(n, 64) - nl0;
    if (j0 < n) {
      if (l0) S.live[p0] = j0;
      else S.dflist[j0 - p0] = j0;
    }
    if (j1 < n) {
      if (l1) S.live[nl0 + p1] = j1;
      else S.dflist[nd0 + (j1 - 64 - p1)] = j1;
    }
    int nl = nl0 + __popcll(m1), ndef = n - nl;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // tied poles (rare): detected in parallel, merged serially by lane 0
    bool tie = false;
    for (int k = tid; k + 1 < nl; k += 64) {
      const int i = S.live[k], j = S.live[k + 1];
      tie = tie || (j != r && S.d[i] - S.d[j] <= tl);
    }
    int ngiv = 0;
    if (__ballot(tie)) {
      if (tid == 0) {
        int k = 0;
        while (k + 1 < nl) {
          const int i = S.live[k], j = S.live[k + 1];
          if (j != r && S.d[i] - S.d[j] <= tl) {
            const double h = hypot(S.z[i], S.z[j]);
            S.gc[ngiv] = S.z[i] / h;
            S.gs[ngiv] = S.z[j] / h;
            S.gi[ngiv] = i;
            S.gj[ngiv] = j;
            ++ngiv;
            S.z[i] = h;
            S.dflist[ndef++] = j;
            for (int t = k + 1; t + 1 < nl; ++t) S.live[t] = S.live[t + 1];
            --nl;
          } else {
            ++k;
          }
        }
      }
      nl = __shfl(nl, 0, 64);
      ndef = __shfl(ndef, 0, 64);
      ngiv = __shfl(ngiv, 0, 64);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int t = tid; t < nl; t += 64) {
      const int j = S.live[t];
      const double zj = S.z[j];
      S.J[t] = j;
      S.dj[t] = S.d[j];
      S.zz[t] = zj * zj;
      S.zs[t] = zj < 0.0 ? -1.0 : 1.0;
    }
    if (tid == 0) {
      S.tol = tl;
      S.fail = 0;
      S.nd = nl;
      S.ndef = ndef;
      S.ngiv = ngiv;
    }
  }
  __syncthreads();
  const int nd = S.nd;

  // roots: one 16-lane quarter-wave each, the lane's terms kept in registers
  const int qw = tid >> 4, ql = tid & 15;
  double tdj[SEC_TERMS], tzz[SEC_TERMS];
#pragma unroll
  for (int m = 0; m < SEC_TERMS; ++m) {
    const int k = ql + 16 * m;
    tdj[m] = k < nd ? S.dj[k] : 0.0;
    tzz[m] = k < nd ? S.zz[k] : 0.0;
  }
  for (int i = qw; i < nd; i += CORE_THREADS / 16) {
    if (nd == 1) {
      if (ql == 0) {
        S.rK[0] = S.dj[0];
        S.mu[0] = S.zz[0];
      }
      continue;
    }
    int K = 0;
    double fm = 0.0, half = 0.0;   // f at the midpoint of (d_i^2, d_{i-1}^2), half the gap
    if (i > 0) {
      const double dI = S.dj[i];
      half = 0.5 * (S.dj[i - 1] - dI) * (S.dj[i - 1] + dI);
#pragma unroll
      for (int m = 0; m < SEC_TERMS; ++m)
        if (ql + 16 * m < nd) fm += tzz[m] * recip((tdj[m] - dI) * (tdj[m] + dI) - half);
      fm = 1.0 + row_sum(fm);
      K = fm > 0.0 ? i : i - 1;
    }
    const double dK = S.dj[K];
    double lo, hi;
    if (i == 0) {
      double zsum = 0.0;
#pragma unroll
      for (int m = 0; m < SEC_TERMS; ++m) zsum += tzz[m];
      lo = 0.0;
      hi = row_sum(zsum);
    } else {
      lo = (S.dj[i] - dK) * (S.dj[i] + dK);
      hi = (S.dj[i - 1] - dK) * (S.dj[i - 1] + dK);
      if (K == i) hi *= 0.5;
      else lo *= 0.5;
    }
    const int ilo = i == 0 ? 1 : i, ihi = i == 0 ? 0 : i - 1;
    const double dlo = (S.dj[ilo] - dK) * (S.dj[ilo] + dK);
    const double dhi = (S.dj[ihi] - dK) * (S.dj[ihi] + dK);
    double dsh[SEC_TERMS];   // d_k^2 - d_K^2
#pragma unroll
    for (int m = 0; m < SEC_TERMS; ++m) dsh[m] = (tdj[m] - dK) * (tdj[m] + dK);
    double mu = 0.5 * (lo + hi);
    if (i > 0) {
      // Start from the root of the two-pole model: the two nearest terms
      // exact, the others frozen at their midpoint value c,
      //   c - z_K^2 / mu + z_O^2 / (del - mu) = 0
      //   <=>  c mu^2 - (c del + z_K^2 + z_O^2) mu + z_K^2 del = 0,
      // taken when it falls inside the bracket (else the midpoint).  A root
      // far from the bracket's middle (a wide gap between the kept and the
      // dropped directions) then needs a few iterations instead of ~9.
      const double zK = S.zz[K], zO = S.zz[K == i ? i - 1 : i];
      const double del = K == i ? dhi : dlo;
      const double c0 = fm + (S.zz[i] - S.zz[i - 1]) / half;
      const double qa = c0, qb = -(c0 * del + zK + zO), qc = zK * del;
      const double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        const double qq = -0.5 * (qb + (qb >= 0.0 ? sqrt(disc) : -sqrt(disc)));
        const double g1 = qa != 0.0 ? qq / qa : NAN;
        const double g2 = qq != 0.0 ? qc / qq : NAN;
        if (g1 > lo && g1 < hi) mu = g1;
        else if (g2 > lo && g2 < hi) mu = g2;
      }
    }
    int it = 0;
    const int nterm = (nd + 15) >> 4;   // term slots holding a live pole
    for (; it < SEC_MAXIT; ++it) {
      double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0;
#pragma unroll
      for (int m = 0; m < SEC_TERMS; ++m) {
        if (m >= nterm) break;            // uniform
        const int k = ql + 16 * m;
        if (k < nd) {
          const double rinv = recip(dsh[m] - mu);
          const double t = tzz[m] * rinv;
          if (k >= ilo) {
            psi += t;
            dpsi += t * rinv;
          } else {
            phi += t;
            dphi += t * rinv;
          }
        }
      }
      psi = row_sum(psi);
      phi = row_sum(phi);
      dpsi = row_sum(dpsi);
      dphi = row_sum(dphi);
      const double w = 1.0 + psi + phi;
      if (w > 0.0) hi = mu;
      else lo = mu;
      if (fabs(w) <= 8.0 * SEC_EPS * (1.0 + fabs(psi) + fabs(phi)) ||
          hi - lo <= 4.0 * SEC_EPS * fmax(fabs(lo), fabs(hi)))
        break;
      const double Dlo = dlo - mu, Dhi = dhi - mu, dw = dpsi + dphi;
      const double cq = w - Dlo * dpsi - Dhi * dphi;
      const double aq = (Dlo + Dhi) * w - Dlo * Dhi * dw;
      const double bq = Dlo * Dhi * w;
      // (the step only steers the iteration; the tests above decide
      // convergence, so reciprocals stand in for the divisions)
      double r1 = NAN, r2 = NAN;
      if (cq == 0.0) {
        if (aq != 0.0) r1 = bq * recip(aq);
      } else {
        const double disc = sqrt(fabs(aq * aq - 4.0 * bq * cq));
        const double qv = 0.5 * (aq + (aq >= 0.0 ? disc : -disc));
        r1 = qv * recip(cq);
        if (qv != 0.0) r2 = bq * recip(qv);
      }
      double eta;
      if (i == 0) eta = (r1 > Dhi) ? r1 : ((r2 > Dhi) ? r2 : NAN);
      else eta = (r1 > Dlo && r1 < Dhi) ? r1 : ((r2 > Dlo && r2 < Dhi) ? r2 : NAN);
      if (!(eta == eta) || w * eta >= 0.0) eta = -w * recip(dw);
      double nw = mu + eta;
      if (!(nw > lo && nw < hi)) nw = 0.5 * (lo + hi);
      mu = nw;
    }
    if (ql == 0) {
      S.rK[i] = dK;
      S.mu[i] = mu;
      if (it >= SEC_MAXIT || !isfinite(mu)) S.fail = 1;
    }
  }
  __syncthreads();
  if (S.fail) return false;

  // z~ from the computed roots (Loewner's formula), one quarter-wave per
  // entry, the product split over its 16 lanes
  for (int jj = qw; jj < nd; jj += CORE_THREADS / 16) {
    const double dj = S.dj[jj];
    double prod = 1.0;
    for (int i = ql; i < nd; i += 16) {
      const double di = S.dj[i];
      prod *= i == jj ? lam_minus_d(S, jj, dj) : lam_minus_d(S, i, dj) * recip((di - dj) * (di + dj));
    }
    prod = row_prod(prod);
    if (ql == 0) S.zh[jj] = S.zs[jj] * sqrt(fmax(prod, 0.0));
  }
  __syncthreads();
  // Vectors of the roots, one quarter-wave per column i: the unnormalised
  // entries on the live rows J[jj] (zero on the deflated rows), their norms,
  // then U columns of length sigma'_i and V columns of length 1, and the
  // finite check, with no barrier in between.
  for (int i = qw; i < nd; i += CORE_THREADS / 16) {
    double ea[SEC_TERMS], ev[SEC_TERMS];
    double sa = 0.0, sv = 0.0;
#pragma unroll
    for (int m = 0; m < SEC_TERMS; ++m) {
      const int jj = ql + 16 * m;
      ea[m] = 0.0;
      ev[m] = 0.0;
      if (jj < nd) {
        const double dj = S.dj[jj];
        const double a = S.zh[jj] * recip(-lam_minus_d(S, i, dj));   // z~_j / (d_j^2 - lambda_i)
        ea[m] = a;
        ev[m] = S.J[jj] == r ? -1.0 : dj * a;
        sa = __builtin_fma(a, a, sa);
        sv = __builtin_fma(ev[m], ev[m], sv);
      }
    }
    sa = row_sum(sa);
    sv = row_sum(sv);
    const double fa = sqrt(S.rK[i] * S.rK[i] + S.mu[i]) / sqrt(sa);
    const double fv = 1.0 / sqrt(sv);
    bool bad = false;
    double sn = 0.0;
#pragma unroll
    for (int m = 0; m < SEC_TERMS; ++m) {
      const int jj = ql + 16 * m;
      if (jj < nd) {
        const int row = S.J[jj];
        const double a = ea[m] * fa, v = ev[m] * fv;
        A[i * LDK + row] = a;
        V[i * LDK + row] = v;
        sn = __builtin_fma(a, a, sn);
        bad = bad || !isfinite(a) || !isfinite(v);
      }
    }
    sn = row_sum(sn);
    if (ql == 0) sdo[i] = sqrt(sn);          // the column norm of what A holds
    for (int t = ql; t < S.ndef; t += 16) {
      A[i * LDK + S.dflist[t]] = 0.0;
      V[i * LDK + S.dflist[t]] = 0.0;
    }
    if (bad) S.fail = 1;
  }
  // deflated pairs: (d_j, e_j, e_j)
  for (int t = tid; t < S.ndef; t += CORE_THREADS) sdo[nd + t] = fabs(sig[S.dflist[t]]);
  for (int idx = tid; idx < S.ndef * n; idx += CORE_THREADS) {
    const int t = idx / n, row = idx % n;
    const int j = S.dflist[t], col = nd + t;
    A[col * LDK + row] = row == j ? sig[j] : 0.0;
    V[col * LDK + row] = row == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // undo the tied-pole rotations on the rows of U_k and V_k (the caller
  // then takes the column norms again)
  norms_ok = S.ngiv == 0;
  if (S.ngiv > 0) {
    if (tid < 2 * n) {
      double* M = tid < n ? A : V;
      const int col = tid % n;
      bool bad = false;
      for (int g = S.ngiv - 1; g >= 0; --g) {
        const int i = S.gi[g], j = S.gj[g];
        const double cg = S.gc[g], sn = S.gs[g];
        const double ri = M[col * LDK + i], rj = M[col * LDK + j];
        M[col * LDK + i] = cg * ri - sn * rj;
        M[col * LDK + j] = sn * ri + cg * rj;
        bad = bad || !isfinite(M[col * LDK + i]) || !isfinite(M[col * LDK + j]);
      }
      if (bad) S.fail = 1;
    }
    __syncthreads();
  }
  return !S.fail;
}

// Stored-column count at which the next pass refolds: the capacity, or
// (fold_slack > 0) r' + fold_slack when that is smaller, so that a stream
// whose rank sits below its cap does not carry the whole capacity's
// pending columns through every pass.
__device__ __forceinline__ int fold_limit(const CoreArgs& c, int rn) {
  return c.fold_slack > 0 ? min(c.ct, rn + c.fold_slack) : c.ct;
}

typedef double d4_t __attribute__((ext_vector_type(4)));

// One 16 x 16 FP64 tile D = sum_{k < K} A(row, k) B(k, col) on the matrix
// cores, in the 16x16x4 operand layout: lane l holds row (and column) l % 16
// and k-step offset l / 16, and reads its elements at pa[k * sa] and
// pb[k * sb].  Every load is issued (a lane whose row or column is out of
// range, use_a / use_b false, or whose k is past K, reads k = 0 of a valid
// pointer and passes zero), so the loop has no divergent branches; two
// accumulators over alternate k-steps keep two products in flight, and the
// next eight k-steps' operands are loaded while these are multiplied.
template <int NB>
__device__ __forceinline__ d4_t mfma_tile_nb(const double* pa, int sa, bool use_a, const double* pb, int sb,
                                             bool use_b, int K, int l) {
  d4_t d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0;
  const int kl = l >> 4;
  // operands of the k-steps k0 + kl and k0 + kl + 4 (zero past K)
  auto load = [&](int k0, double& a0, double& b0, double& a1, double& b1) {
    const int ka = k0 + kl, kb = ka + 4;
    const bool va = ka < K, vb = kb < K;
    const int ia = va ? ka : 0, ib = vb ? kb : 0;
    a0 = pa[ia * sa];
    b0 = pb[ia * sb];
    a1 = pa[ib * sa];
    b1 = pb[ib * sb];
    a0 = use_a && va ? a0 : 0.0;
    b0 = use_b && va ? b0 : 0.0;
    a1 = use_a && vb ? a1 : 0.0;
    b1 = use_b && vb ? b1 : 0.0;
  };
  double a0, b0, a1, b1;
  load(0, a0, b0, a1, b1);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double na0, nb0, na1, nb1;
    load(8 * j + 8, na0, nb0, na1, nb1);   // the next k-steps' loads overlap these products
    d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, d1, 0, 0, 0);
    a0 = na0;
    b0 = nb0;
    a1 = na1;
    b1 = nb1;
  }
  return d0 + d1;
}

// The same product with a run-time loop over the blocks (fewer registers;
// the BF16 Gram correction's rarely taken products)
__device__ __forceinline__ d4_t mfma_tile_loop(const double* pa, int sa, bool use_a, const double* pb, int sb,
                                               bool use_b, int K, int l) {
  d4_t d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0;
  const int kl = l >> 4;
  auto load = [&](int k0, double& a0, double& b0, double& a1, double& b1) {
    const int ka = k0 + kl, kb = ka + 4;
    const bool va = ka < K, vb = kb < K;
    const int ia = va ? ka : 0, ib = vb ? kb : 0;
    a0 = pa[ia * sa];
    b0 = pb[ia * sb];
    a1 = pa[ib * sa];
    b1 = pb[ib * sb];
    a0 = use_a && va ? a0 : 0.0;
    b0 = use_b && va ? b0 : 0.0;
    a1 = use_a && vb ? a1 : 0.0;
    b1 = use_b && vb ? b1 : 0.0;
  };
  double a0, b0, a1, b1;
  load(0, a0, b0, a1, b1);
  for (int k0 = 0; k0 < K; k0 += 8) {
    double na0, nb0, na1, nb1;
    load(k0 + 8, na0, nb0, na1, nb1);
    d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, d1, 0, 0, 0);
    a0 = na0;
    b0 = nb0;
    a1 = na1;
    b1 = nb1;
  }
  return d0 + d1;
}

// The number of 8-step blocks is dispatched to a straight-line product (one
// uniform branch): a loop over a run-time K took about three times the
// matrix-core time of its products in isolation (2100 against 628 cycles for
// K = 40 on one wavefront), its load waits and branches breaking the
// pipelining.  The products and their order are those of the loop, bit for
// bit.
__device__ __forceinline__ d4_t mfma_tile(const double* pa, int sa, bool use_a, const double* pb,
                                          int sb, bool use_b, int K, int l) {
  static_assert(MMAX <= 72, "K of the core's products is at most 72");
  switch ((K + 7) >> 3) {
    case 1: return mfma_tile_nb<1>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 2: return mfma_tile_nb<2>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 3: return mfma_tile_nb<3>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 4: return mfma_tile_nb<4>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 5: return mfma_tile_nb<5>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 6: return mfma_tile_nb<6>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 7: return mfma_tile_nb<7>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 8: return mfma_tile_nb<8>(pa, sa, use_a, pb, sb, use_b, K, l);
    case 9: return mfma_tile_nb<9>(pa, sa, use_a, pb, sb, use_b, K, l);
    default: return d4_t{0.0, 0.0, 0.0, 0.0};   // K <= 0
  }
}

// General pairs (B = Y W held as T R): the right-factor bookkeeping of one
// update, in place of the chained pairs' shifted product.  With
// U' = [U q] U_k and B' = [B y] V_k (kept columns),
//     G' = U'^T B' = U_k^T E V_k,   E = [[G, U^T y], [q^T B, q^T y]],
//     R' = [[R, 0], [0, 1]] V_k,    A~ = G' diag(sigma')^-1.
// U_k(i, a) = sA[perm[a] * LDK + i] / sd[perm[a]], V_k(i, a) = sV[perm[a] *
// LDK + i]; sQ is free here (Q' is written) and receives E V_k.
__device__ __forceinline__ void general_tail(const CoreArgs& c, int r, int rn, int M, double qy,
                                          const double* sA, const double* sV, const double* sC,
                                          double* sQ, const double* sd, const double* sgn,
                                          const double* pyr, const double* qB, const int* perm) {
  DevState* __restrict__ st = c.st;
  DevState* __restrict__ tst = c.tst;
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int trefold = tst->refold;            // the T sweep left T[:, :r] = B (R = I)
  const int mTe = trefold ? r : tst->m;       // stored T columns before y; y sits in column mTe
  // E V_k[:, kept] (M x rn, K = M) into sQ[b * MMAX + i]
  {
    const int ntr = (M + 15) / 16, ntc = (rn + 15) / 16;
    for (int tile = wv; tile < ntr * ntc; tile += CORE_THREADS / 64) {
      const int i0 = 16 * (tile % ntr), b0 = 16 * (tile / ntr);
      const int ia = i0 + (l & 15), bb = b0 + (l & 15);
      const int pb = bb < rn ? perm[bb] : 0;
      // columns j < r of E on the matrix cores (row ia: row ia of G, stride
      // RMAX along j, or q^T B), then column r (U^T y, q^T y) times row r of
      // V_k as an outer-product term
      d4_t d = mfma_tile(ia < r ? sC + ia : qB, ia < r ? RMAX : 1, ia <= r, sV + pb * LDK, 1, bb < rn,
                         r, l);
      const double vr = bb < rn ? sV[pb * LDK + r] : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * v + (l >> 4);
        const double er = i < r ? pyr[i < r ? i : 0] : (i == r ? qy : 0.0);
        d[v] = __builtin_fma(er, vr, d[v]);
        if (i < M && bb < rn) sQ[bb * MMAX + i] = d[v];
      }
    }
  }
  // R' tiles in registers (R is read from the T state, rewritten in place
  // after the barrier below)
  constexpr int NRT = 4 * ((CMAX + 15) / 16);
  d4_t rt[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int tile = wv + 16 * h;
    d4_t d = {0.0, 0.0, 0.0, 0.0};
    if (tile < NRT) {
      const int c0 = 16 * (tile >> 2), k0 = 16 * (tile & 3);
      const int kb = k0 + (l & 15);
      const int pk = kb < rn ? perm[kb] : 0;
      if (!trefold) {
        // R (global, L2) for all k-steps first: one round of latency
        constexpr int KS = RMAX / 4;
        const int ca = c0 + (l & 15);
        double av[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int j = 4 * ks + (l >> 4);
          av[ks] = (j < r && ca < mTe) ? tst->Q[ca * RMAX + j] : 0.0;
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if (4 * ks < r) {
            const int j = 4 * ks + (l >> 4);
            const double bv = (j < r && kb < rn) ? sV[pk * LDK + j] : 0.0;
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], bv, d, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cr = c0 + 4 * v + (l >> 4);
        double out = 0.0;
        if (kb < rn) {
          if (cr < mTe) out = trefold ? sV[pk * LDK + cr] : d[v];
          else if (cr == mTe) out = sV[pk * LDK + r];
        }
        d[v] = out;
      }
    }
    rt[h] = d;
  }
  __syncthreads();
  // G' = U_k^T (E V_k) (rn x rn, K = M) and A~ = G' diag(sigma')^-1, each
  // tile formed transposed (as for C in the chained update: lane l holds
  // rows i0 + l%16, so the stores write 128-byte pieces)
  {
    const int nt = (rn + 15) / 16;
    for (int tile = wv; tile < nt * nt; tile += CORE_THREADS / 64) {
      const int i0 = 16 * (tile % nt), j0 = 16 * (tile / nt);
      const int ia = i0 + (l & 15), jb = j0 + (l & 15);
      const int pa = ia < rn ? perm[ia] : 0;
      const d4_t d = mfma_tile(sQ + (jb < rn ? jb : 0) * MMAX, 1, jb < rn, sA + pa * LDK, 1, ia < rn,
                               M, l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + 4 * v + (l >> 4);
        if (ia < rn && j < rn) {
          const double g = d[v] / sd[pa];
          st->C[j * RMAX + ia] = g;
          st->At[j * RMAX + ia] = g / sgn[j];
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int tile = wv + 16 * h;
    if (tile < NRT) {
      const int c0 = 16 * (tile >> 2), k0 = 16 * (tile & 3);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cr = c0 + 4 * v + (l >> 4);
        if (cr >= CMAX) continue;
        const int idx = cr * RMAX + k0 + (l & 15);
        tst->Q[idx] = rt[h][v];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    tst->m = mTe + 1;
    tst->r = rn;
    tst->refold = mTe + 1 >= fold_limit(c, rn);
  }
}

// BF16 basis after a refold: the refolded columns S' = fl(S Q) are not
// orthonormal (M = S'^T S' = I + E, ||E||_F about 1e-3).  The orthonormal
// basis of their span is S' M^-1/2; with the old basis U ~ S' (they differ
// by the rounding) the model X ~ U diag(sigma) W^T reads
// X ~ (S' M^-1/2) (M^1/2 diag(sigma)) W^T, so this update's core takes
// M^1/2 diag(sigma) as its top-left block (a general SVD; the right factor W
// and with it C and w are unchanged), inner products with the basis carry
// over as M^-1/2 S'^T v ~ M^-1/2 (U^T v), and Q = M^-1/2 (U = S'[:, :r] Q).
//   in:  the Gram records (sums in record order), p1 (pvec), p2, pyr.
//   out: sA = M^1/2 (ld LDK), sQ rows < r = M^-1/2, the three vectors
//        transformed; sV is scratch.
// M^1/2 and M^-1/2 come from the coupled Newton-Schulz iteration
// Y <- Y T, Z <- T Z, T = (3 I - Z Y) / 2 from Y = M, Z = I, quadratically
// convergent for ||I - M|| < 1 (Higham, Functions of Matrices, 2008, 6.3);
// its products are 16x16 FP64 matrix-core tiles, one per wave.
__device__ void gram_fix(const CoreArgs& c, int r, double* sA, double* sV, double* sQ, double* pvec,
                         double* p2, double* pyr) {
  const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
  const int nb = (r + 15) / 16;
  // 1. M from the records (fixed order), both triangles, into sA
  for (int e = tid; e < GRAM_REC; e += CORE_THREADS) {
    const int pp = e >> 8, ln = (e >> 2) & 63, v = e & 3;
    int I = 0, J = 0, k = pp;
    while (k >= GRAM_BLOCKS - I) { k -= GRAM_BLOCKS - I; ++I; }
    J = I + k;
    const int row = 16 * I + 4 * (ln >> 4) + v, col = 16 * J + (ln & 15);
    if (J < nb && row < r && col < r) {
      double t = 0.0;
      for (int w = 0; w < c.gnwg; ++w) t += c.grec[(int64_t)w * GRAM_REC + e];
      sA[col * LDK + row] = t;
      if (I != J) sA[row * LDK + col] = t;
    }
  }
  for (int idx = tid; idx < r * r; idx += CORE_THREADS) {
    const int i = idx % r, j = idx / r;
    sV[j * LDK + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // 2. Newton-Schulz: Y (sA) -> M^1/2, Z (sV) -> M^-1/2; T in sQ (ld LDQ)
  const int ti = wv & 3, tj = wv >> 2;           // one 16x16 tile per wave (16 waves)
  const int row0 = 16 * ti, col0 = 16 * tj;
  const bool tile_live = row0 < r && col0 < r;
  const int ra = row0 + (l & 15), cb = col0 + (l & 15);
  for (int it = 0; it < 12; ++it) {
    int far = 0;
    if (tile_live) {
      const d4_t d = mfma_tile_loop(sV + (ra < r ? ra : 0), LDK, ra < r, sA + (cb < r ? cb : 0) * LDK, 1,
                               cb < r, r, l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 4 * v + (l >> 4), j = cb;
        if (i < r && j < r) {
          const double t = ((i == j ? 3.0 : 0.0) - d[v]) * 0.5;
          sQ[j * LDQ + i] = t;
          far |= fabs(t - (i == j ? 1.0 : 0.0)) > 0x1p-50;
        }
      }
    }
    const int more = __syncthreads_or(far);
    d4_t yt = {0.0, 0.0, 0.0, 0.0}, tz = yt;
    if (tile_live) {
      yt = mfma_tile_loop(sA + (ra < r ? ra : 0), LDK, ra < r, sQ + (cb < r ? cb : 0) * LDQ, 1, cb < r, r, l);
      tz = mfma_tile_loop(sQ + (ra < r ? ra : 0), LDQ, ra < r, sV + (cb < r ? cb : 0) * LDK, 1, cb < r, r, l);
    }
    __syncthreads();
    if (tile_live) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + 4 * v + (l >> 4), j = cb;
        if (i < r && j < r) {
          sA[j * LDK + i] = yt[v];
          sV[j * LDK + i] = tz[v];
        }
      }
    }
    __syncthreads();
    if (!more) break;                            // T was I to 2^-50: Y, Z converged
  }
  // 3. p1, p2, U^T y in the orthonormal basis: M^-1/2 v (Z symmetric: row j
  //    of Z is column j), one quarter-wave per entry
  const int qw = tid >> 4, ql = tid & 15;       // 64 quarter-waves: entry qw of each vector
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if (qw < r) {
    for (int i = ql; i < r; i += 16) {
      const double w = sV[qw * LDK + i];
      t0 += w * pvec[i];
      t1 += w * p2[i];
      t2 += w * pyr[i];
    }
  }
  t0 = row_sum(t0);
  t1 = row_sum(t1);
  t2 = row_sum(t2);
  __syncthreads();
  if (qw < r && ql == 0) {
    pvec[qw] = t0;
    p2[qw] = t1;
    pyr[qw] = t2;
  }
  // 4. Q = M^-1/2 (rows < r of the refolded basis)
  for (int idx = tid; idx < r * r; idx += CORE_THREADS) {
    const int cc = idx / r, k2 = idx % r;
    sQ[cc * LDQ + k2] = sV[k2 * LDK + cc];
  }
  __syncthreads();
}

template <bool GENERAL>
__device__ __forceinline__ void core_update(const CoreArgs& c) {
  DevState* __restrict__ st = c.st;
  __shared__ double sA[MMAX * LDK];
  __shared__ double sV[MMAX * LDK];
  __shared__ double red[CORE_THREADS];
  __shared__ double tot[PW];
  __shared__ double sd[MMAX + 1];
  __shared__ double p2[RMAX], pyr[RMAX], pyn[RMAX], wn[RMAX], sgn[RMAX], ssig[RMAX], pvec[RMAX];
  __shared__ SecShared sec;
  __shared__ double sC[RMAX * RMAX];
  __shared__ double wk[RMAX], urk[RMAX], sw[RMAX], qB[RMAX], eB[RMAX], isg[RMAX];
  __shared__ int perm[MMAX + 1];
  __shared__ int flag;
  __shared__ double sc[8];
  __shared__ int si[4];
  __shared__ double sQ[CMAX * LDQ];    // Q (m x r), row c at sQ + c*LDQ
  static_assert(MMAX * MMAX <= CMAX * LDQ, "sQ holds E V_k for general pairs");

  const int tid = threadIdx.x;
  const int r = st->r, m = st->m, refolded = st->refold;

  // 0. stage Q and the shifted product C in LDS with coalesced passes, all
  //    of a thread's loads issued before its first store, and
  // 1. fixed-order reduction of the per-workgroup partial sums (compact
  //    records of pwc values, read as 16-byte pairs; sV is scratch here).
  //    The slot count does not depend on the record length, so every value
  //    is summed in the same order whatever bucket the pass ran with (x.x of
  //    a pair is then bit-equal to y.y of the pair before it).  A thread's
  //    records are read RU at a time, the first RU with Q and C, so that
  //    their latencies overlap.
  // the record length the pass wrote: its bucket, given by the launch or,
  // for passes that chose it on the device (c.rb = -kb), the variant of the
  // m the pass read (the pass leaves m as it found it)
  const int rbk = c.rb > 0 ? c.rb : live_variant(m, -c.rb);
  const int pwc = 2 * rbk + 6, pw2 = pwc / 2;
  constexpr int nslot = CORE_THREADS / (PW / 2);
  constexpr int RU = 10;
  const bool rth = tid < nslot * pw2;
  const int rg = rth ? tid % pw2 : 0, rsl = rth ? tid / pw2 : 0;
  const double2* __restrict__ rec = reinterpret_cast<const double2*>(c.partials);
  double2 rv[RU];
  int64_t macc0 = 0;
  double yyprev0 = 0.0, yhprev0 = 0.0, tol0 = 0.0;
  double ax = 0.0, ay = 0.0;
  // records rsl + (ch RU + i) nslot; past nblk a valid record is read and
  // not added
  auto load_records = [&](int ch) {
#pragma unroll
    for (int i = 0; i < RU; ++i) {
      const int b = rsl + (ch * RU + i) * nslot;
      rv[i] = rec[(int64_t)(b < c.nblk ? b : 0) * (PW / 2) + rg];
    }
  };
  auto add_records = [&](int ch) {
#pragma unroll
    for (int i = 0; i < RU; ++i)
      if (rsl + (ch * RU + i) * nslot < c.nblk) {
        ax += rv[i].x;
        ay += rv[i].y;
      }
  };
  {
    constexpr int NQ = (CMAX * RMAX + CORE_THREADS - 1) / CORE_THREADS;
    constexpr int NC = (RMAX * RMAX + CORE_THREADS - 1) / CORE_THREADS;
    double qv[NQ], cv[NC];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int idx = tid + i * CORE_THREADS;
      const int c0 = idx / RMAX, j = idx % RMAX;
      qv[i] = (idx < CMAX * RMAX && c0 < m && j < r) ? st->Q[idx] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int idx = tid + i * CORE_THREADS;
      const int j = idx % RMAX, k = idx / RMAX;
      cv[i] = (j < r && k < r) ? st->C[idx] : 0.0;
    }
    load_records(0);
    // the small state the later steps read, fetched with the rest: sigma
    // and p1 (the cached p_y, or U^T x of a general pair) into ssig / pvec,
    // and the scalars of the checks into tid 0's registers and sc[4]
    const bool sth = tid < RMAX && tid < r;
    const double sg = sth ? st->sigma[tid] : 0.0;
    const double p1v = sth ? (GENERAL ? st->p1[tid] : st->py[tid]) : 0.0;
    if (tid == 0) {
      macc0 = st->m_acc;
      yyprev0 = st->yy_prev;
      yhprev0 = st->yh_prev;
      tol0 = st->tol;
    }
    if (sth) {
      ssig[tid] = sg;
      pvec[tid] = p1v;
    }
    if (tid == 0) sc[4] = tol0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int idx = tid + i * CORE_THREADS;
      if (idx < CMAX * RMAX) sQ[idx / RMAX * LDQ + idx % RMAX] = qv[i];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) sC[tid + i * CORE_THREADS] = cv[i];
  }
  if (tid < RMAX) sw[tid] = tid < r ? st->w[tid] : 0.0;
  {
    add_records(0);
    for (int ch = 1; ch * RU * nslot < c.nblk; ++ch) {   // uniform
      load_records(ch);
      add_records(ch);
    }
    if (rth) {
      sV[rsl * pwc + 2 * rg] = ax;
      sV[rsl * pwc + 2 * rg + 1] = ay;
    }
    __syncthreads();
    if (tid < pwc) {
      double t = 0.0;
      for (int sl = 0; sl < nslot; ++sl) t += sV[sl * pwc + tid];
      const int rb = rbk;
      const int at = tid < rb ? P_SUE + tid : (tid < 2 * rb ? P_SUY + (tid - rb) : P_EE + (tid - 2 * rb));
      tot[at] = t;
    }
    __syncthreads();
  }

  // general pairs: e^T B = R^T T^T e from the T sweep's records (second
  // half, fixed-order sums; R and the T columns as that sweep read them)
  if constexpr (GENERAL) {
    const DevState* __restrict__ tst = c.tst;
    const int mT = tst->m;
    constexpr int NSL = CORE_THREADS / CMAX;
    double* part = sV;                       // scratch, as in step 1
    if (tid < NSL * CMAX) {
      const int it = tid % CMAX, sl = tid / CMAX;
      double t = 0.0;
      if (it < mT) {
#pragma unroll 16
        for (int b = sl; b < c.nblk; b += NSL) t += c.pt[(int64_t)b * PW + c.rbt + it];
      }
      part[sl * CMAX + it] = t;
    }
    __syncthreads();
    if (tid < CMAX) {
      double t = 0.0;
      for (int sl = 0; sl < NSL; ++sl) t += part[sl * CMAX + tid];
      red[tid] = t;
    }
    __syncthreads();
    if (tid < RMAX) {
      double t = 0.0;
      if (tid < r)
#pragma unroll 24
        for (int c0 = 0; c0 < mT; ++c0) t += tst->Q[c0 * RMAX + tid] * red[c0];
      eB[tid] = t;
    }
    __syncthreads();
  }

  // 2. second projection p2 = U^T e = Q^T S^T e and U^T y = Q^T S^T y, with
  //    the stored columns and the Q the pass read
  //    (one 16-lane quarter-wave per entry, the stored columns split over
  //    its lanes)
  {
    const int j = tid >> 4, jl = tid & 15;
    if (j < r) {
      double a2 = 0.0, b2 = 0.0;
      for (int c0 = jl; c0 < m; c0 += 16) {
        a2 = __builtin_fma(sQ[c0 * LDQ + j], tot[P_SUE + c0], a2);
        b2 = __builtin_fma(sQ[c0 * LDQ + j], tot[P_SUY + c0], b2);
      }
      a2 = row_sum(a2);
      b2 = row_sum(b2);
      if (jl == 0) {
        p2[j] = a2;
        pyr[j] = b2;
      }
    }
  }
  __syncthreads();
  // a refold pass left U = S[:, :r] (Q = I); the update below continues from it
  if (refolded) {
    for (int idx = tid; idx < CMAX * RMAX; idx += CORE_THREADS) {
      const int c0 = idx / RMAX, j = idx % RMAX;
      sQ[c0 * LDQ + j] = (c0 == j && j < r) ? 1.0 : 0.0;
    }
    __syncthreads();                   // step 3's phase reads Q
  }
  const int meff = refolded ? r : m;   // stored columns U is built from; e sits in column meff
  // a BF16 basis just refolded: carry the model over to the orthonormal
  // basis of the refolded columns (the core of this update is then general)
  const bool gfix = refolded && c.grec != nullptr && r > 0;
  if (gfix) gram_fix(c, r, sA, sV, sQ, pvec, p2, pyr);

  // 3. checks, residual norm, growth test (|p2|^2 and p2 . U^T y summed
  //    across the first wavefront, one entry per lane); in the same phase
  //    the second wavefront forms the core's p = p1 + p2 (step 4) and the
  //    rest (Q p2)[c] for the rotation (step 8) into red, one quarter-wave
  //    per row (a skipped update uses neither)
  if (tid >= 64 && tid < 128) {
    const int j = tid - 64;
    if (j < r) pvec[j] += p2[j];           // sigma and p1 were staged with Q
  } else if (tid >= 128) {
    const int q0 = (tid - 128) >> 4, l16 = tid & 15;
    for (int row = q0; row < CMAX; row += (CORE_THREADS - 128) / 16) {
      double t = 0.0;
      if (row < m || refolded)
        for (int j = l16; j < r; j += 16) t += sQ[row * LDQ + j] * p2[j];
      t = row_sum(t);
      if (l16 == 0) red[row] = t;
    }
  }
  if (tid < 64) {
    double pp = tid < r ? p2[tid] * p2[tid] : 0.0;
    double py2 = tid < r ? p2[tid] * pyr[tid] : 0.0;
    pp = add_half_pair(add_row_pair(row_sum(pp)));
    py2 = add_half_pair(add_row_pair(row_sum(py2)));
    if (tid == 0) {
      const double ee = tot[P_EE], xx = tot[P_XX], ey = tot[P_EY], yy = tot[P_YY];
      const double xh = tot[P_XH], yh = tot[P_YH];
      int skip = 0;
      if (!(isfinite(ee) && isfinite(xx) && isfinite(ey) && isfinite(yy) && isfinite(pp) &&
            isfinite(py2))) {
        skip = ST_NONFINITE;
      } else if (!GENERAL && macc0 > 0 && (xx != yyprev0 || xh != yhprev0)) {
        // x must be the previous pair's y: both fingerprints, summed in the
        // same fixed order by every pass of this stream, agree bit for bit
        skip = ST_SEQ;
      }
      double rho = sqrt(fmax(ee - pp, 0.0));
      const int grow = !skip && rho > 0.0 && rho > tol0 * sqrt(xx);
      if (!grow) rho = 0.0;
      sc[0] = rho;
      sc[1] = grow ? (ey - py2) / rho : 0.0;   // q^T y
      sc[2] = yy;
      sc[3] = yh;
      si[0] = skip;
      si[1] = grow;
    }
  }
  __syncthreads();
  const int skip = si[0];
  if (skip) {
    // The model is unchanged.  If the pass refolded, the stored columns now
    // hold U itself: Q = I, m = r and the next projection uses p_y directly.
    if (refolded) {
      for (int idx = tid; idx < CMAX * RMAX; idx += CORE_THREADS) {
        const int c0 = idx / RMAX, j = idx % RMAX;
        const double v = (c0 == j && j < r) ? 1.0 : 0.0;
        st->Q[idx] = v;
      }
      if (tid < CMAX) st->a[tid] = tid < r ? st->py[tid] : 0.0;
    }
    // Likewise for B = T R after a refolding T sweep: R = I, r columns.
    if (GENERAL && c.tst->refold) {
      DevState* __restrict__ tst = c.tst;
      for (int idx = tid; idx < CMAX * RMAX; idx += CORE_THREADS) {
        const int c0 = idx / RMAX, j = idx % RMAX;
        const double v = (c0 == j && j < r) ? 1.0 : 0.0;
        tst->Q[idx] = v;
      }
    }
    __syncthreads();
    if (tid == 0) {
      latch_status(st, skip);
      if (refolded) {
        st->m = r;
        st->refold = 0;
      }
      if (GENERAL && c.tst->refold) {
        c.tst->m = r;
        c.tst->refold = 0;
      }
    }
    return;
  }
  const int grow = si[1];
  const double rho = sc[0], qy = sc[1];

  // 4. core K = [[diag(sigma), p], [0, rho]], p = p1 + p2 with p1 the
  //    cached p_y (chained pairs) or U^T x from the projection sweep (p was
  //    formed in the phase of step 3)
  const int M = r + 1;
  // general pairs: q^T B = (e^T B - p2^T G) / rho with G = U^T B (in sC,
  // G(i, j) at sC[j * RMAX + i]), from the stored residual e = x - U p1
  // itself (no cancellation between x^T B and p^T G); zero when no
  // direction is added
  if (GENERAL && tid < r) {
    double t = 0.0;
    for (int i = 0; i < r; ++i) t += p2[i] * sC[tid * RMAX + i];
    qB[tid] = si[1] ? (eB[tid] - t) / sc[0] : 0.0;
  }

  // 5. SVD of the core: secular equation, one-sided Jacobi if that fails
  int sweeps = 0;
  bool have_norms = false;               // the secular solver left the column norms in sd
  if (gfix) {
    // K = [[M^1/2 diag(sigma), p], [0, rho]]: M^1/2 is in sA already
    for (int idx = tid; idx < M * M; idx += CORE_THREADS) {
      const int i = idx % M, j = idx / M;
      if (j < r) sA[j * LDK + i] = (i < r) ? sA[j * LDK + i] * ssig[j] : 0.0;
      else sA[j * LDK + i] = (i < r) ? pvec[i] : rho;
      sV[j * LDK + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    sweeps = jacobi_sweeps(sA, sV, sd, M, &flag);
  } else if (c.jacobi_only || !secular_svd(sA, sV, ssig, pvec, rho, r, sec, sd, have_norms)) {
    have_norms = false;
    for (int idx = tid; idx < M * M; idx += CORE_THREADS) {
      const int i = idx % M, j = idx / M;
      double v;
      if (j < r) v = (i == j) ? ssig[j] : 0.0;
      else v = (i < r) ? pvec[i] : rho;
      sA[j * LDK + i] = v;
      sV[j * LDK + i] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    sweeps = jacobi_sweeps(sA, sV, sd, M, &flag);
  }

  // 6. singular values (exact column norms), descending order, truncation
  //    (one 16-lane quarter-wave per column for the norm and for the rank;
  //    M = r + 1 may exceed the 64 quarter-waves)
  const int qcl = tid & 15;
  if (!have_norms) {                       // uniform
    for (int col = tid >> 4; col < M; col += CORE_THREADS / 16) {
      double s = 0.0;
      for (int i = qcl; i < M; i += 16) s = __builtin_fma(sA[col * LDK + i], sA[col * LDK + i], s);
      s = row_sum(s);
      if (qcl == 0) sd[col] = sqrt(s);
    }
    __syncthreads();
  }
  for (int col = tid >> 4; col < M; col += CORE_THREADS / 16) {
    const double me = sd[col];
    double rank = 0.0;
    for (int k = qcl; k < M; k += 16) rank += (sd[k] > me || (sd[k] == me && k < col)) ? 1.0 : 0.0;
    rank = row_sum(rank);
    if (qcl == 0) perm[(int)rank] = col;
  }
  __syncthreads();
  const double smax = sd[perm[0]];
  const int above = __syncthreads_count(tid < M && smax > 0.0 && sd[tid] > sc[4] * smax);
  const int rn = min(above, c.r_max);
  if (rn == 0) {   // nothing kept (zero snapshots so far)
    if (tid < CMAX) st->a[tid] = 0.0;
    if (GENERAL && tid == 0) {
      c.tst->m = 0;
      c.tst->r = 0;
      c.tst->refold = 0;
    }
    if (tid == 0) {
      st->r = 0;
      st->m = 0;
      st->refold = 0;
      st->m_acc += 1;
      st->yy_prev = sc[2];
      st->yh_prev = sc[3];
      st->last_rho = rho;
      st->sweeps = sweeps;
      st->eig_valid = 0;
      if (sweeps > MAX_SWEEPS) latch_status(st, ST_NOCONV);
    }
    return;
  }

  // 7. U_k = (K V_k) diag(sigma')^-1 for kept columns; new p_y and signs
  //    U_k(i, jj) = sA[perm[jj]*LDK + i] / sd[perm[jj]]
  //    (one 16-lane quarter-wave per kept column)
  {
    const int k = tid >> 4, kl = tid & 15;
    if (k < rn) {
      const int pj = perm[k];
      double s = 0.0;
      for (int i = kl; i < r; i += 16) s = __builtin_fma(sA[pj * LDK + i], pyr[i], s);
      s = row_sum(s);
      if (kl == 0) {
        const double inv = 1.0 / sd[pj];
        s = __builtin_fma(sA[pj * LDK + r], qy, s);
        pyn[k] = s * inv;
        wn[k] = sV[pj * LDK + r];
        sgn[k] = sd[pj];
        isg[k] = inv;                           // 1 / sigma'_k
        wk[k] = s * inv * inv;                  // p_y,k / sigma'_k
        urk[k] = sA[pj * LDK + r] * inv;        // U_k(r, k)
      }
    }
  }
  __syncthreads();

  // 8. The update's rotation U' = [U q] U_k[:, :r'] in the deferred form:
  //    U = S Q and q = (e - U p2) / rho with e stored as column meff, so
  //    U' = S Q' with Q' = [Q G; g^T] (rows < meff, then row meff), where
  //      G = U_k[:r, :r'] - (p2 / rho) U_k[r, :r'],   g = U_k[r, :r'] / rho.
  //    Q G is formed on the matrix cores straight from U_k (K V_k in sA):
  //      (Q G)[c, k] = ( (Q U')[c, k] - irho U'[r, k] (Q p2)[c] ) / sigma'_k
  //    with U'[i, k] = sA[perm[k] * LDK + i].
  const double irho = grow ? 1.0 / rho : 0.0;
  const int mnew = meff + grow;
  // G p_y into pvec (pvec is free after the SVD; the next pass's a needs
  // it; (Q p2)[c] is in red since step 3): one 16-lane quarter-wave per entry
  const int qw = tid >> 4, ql = tid & 15;
  {
    double bs = 0.0;                       // g . p_y up to 1/rho: U_k(r, :) p_y
    for (int k = ql; k < rn; k += 16) bs += urk[k] * pyn[k];
    const double bsum = row_sum(bs);
    for (int j = qw; j < RMAX; j += CORE_THREADS / 16) {
      // (G p_y)_j = sum_k U_k(j,k) p_y,k - (p2_j / rho) sum_k U_k(r,k) p_y,k
      double t = 0.0;
      if (j < r)
        for (int k = ql; k < rn; k += 16) t += sA[perm[k] * LDK + j] * wk[k];
      t = row_sum(t);
      if (ql == 0) pvec[j] = j < r ? t - p2[j] * irho * bsum : 0.0;
    }
  }
  __syncthreads();
  // Q' tiles: 16 x 16 blocks over the rows < mnew and the columns < r'
  // (readers of Q mask rows >= m and columns >= r, so the rest keeps stale
  // values), at most two per wave
  constexpr int NQT = 4 * ((CMAX + 15) / 16);
  static_assert(NQT <= 2 * (CORE_THREADS / 64), "two Q' tiles per wave at most");
  const int ncb = (rn + 15) >> 4, ntile = ((mnew + 15) >> 4) * ncb;
  d4_t qt[2];
  {
    const int wv = tid >> 6, l = tid & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tile = wv + 16 * h;
      d4_t d = {0.0, 0.0, 0.0, 0.0};
      if (tile < ntile) {
        const int c0 = 16 * (tile / ncb), k0 = 16 * (tile % ncb);
        const int kb = k0 + (l & 15), ca = c0 + (l & 15);
        const int pk = kb < rn ? perm[kb] : 0;
        d = mfma_tile(sQ + (ca < CMAX ? ca : 0) * LDQ, 1, ca < CMAX, sA + pk * LDK, 1, kb < rn, r, l);
        // element v of lane l: row c0 + 4 v + l/16, column k0 + l%16
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cr = c0 + 4 * v + (l >> 4);
          double out = 0.0;
          if (kb < rn) {
            const double inv = isg[kb];
            const double urr = sA[pk * LDK + r];
            if (cr < meff) out = (d[v] - irho * urr * red[cr]) * inv;
            else if (cr == meff && grow) out = urr * irho * inv;
          }
          d[v] = out;
        }
      }
      qt[h] = d;
    }
  }
  // next first-projection coefficients a = Q' p_y (rows < meff: Q (G p_y);
  // row meff: g . p_y), one quarter-wave per entry: by the wavefronts that
  // hold no Q' tile, while the others run their matrix-core tiles, or by
  // all of them after the tiles when every wavefront holds one
  {
    const int wv = tid >> 6;
    const int idle = ntile < CORE_THREADS / 64 ? CORE_THREADS / 64 - ntile : 0;
    const bool mine = idle > 0 ? wv >= ntile : true;
    const int q0 = idle > 0 ? qw - 4 * ntile : qw, nq = idle > 0 ? 4 * idle : CORE_THREADS / 16;
    if (mine) {
      for (int row = q0; row < CMAX; row += nq) {
        double t = 0.0;
        if (row < meff) {
          for (int j = ql; j < r; j += 16) t += sQ[row * LDQ + j] * pvec[j];
        } else if (row == meff && grow) {
          for (int k = ql; k < rn; k += 16) t += urk[k] * pyn[k];
        }
        t = row_sum(t);
        if (ql == 0) st->a[row] = row == meff && grow ? t * irho : t;
      }
    }
  }
  __syncthreads();   // every thread is done reading Q: write Q' in place
  {
    const int wv = tid >> 6, l = tid & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int tile = wv + 16 * h;
      if (tile < ntile) {
        const int c0 = 16 * (tile / ncb), k0 = 16 * (tile % ncb);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cr = c0 + 4 * v + (l >> 4);
          if (cr >= CMAX) continue;
          const int idx = cr * RMAX + k0 + (l & 15);
          st->Q[idx] = qt[h][v];
        }
      }
    }
  }

  if constexpr (GENERAL) {
    general_tail(c, r, rn, M, qy, sA, sV, sC, sQ, sd, sgn, pyr, qB, perm);
  } else {
  // 9. T = E V_k[:, kept] with E = [[C, 0], [w^T, 0]] (M x r, the zero
  //    last column dropped), on the matrix cores: 16 x 16 tiles of T, K = r,
  //    written into sA (U_k is no longer read)
  {
    const int wv = tid >> 6, l = tid & 63;
    const int ntr = (M + 15) / 16, ntc = (rn + 15) / 16;
    for (int tile = wv; tile < ntr * ntc; tile += CORE_THREADS / 64) {
      const int i0 = 16 * (tile % ntr), b0 = 16 * (tile / ntr);
      const int ia = i0 + (l & 15), bb = b0 + (l & 15);
      const int pb = bb < rn ? perm[bb] : 0;
      // row ia of E: row ia of C (stride RMAX along j) or w
      const d4_t d = mfma_tile(ia < r ? sC + ia : sw, ia < r ? RMAX : 1, ia <= r, sV + pb * LDK, 1,
                               bb < rn, r, l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * v + (l >> 4);
        if (i < M && bb < rn) sA[bb * LDK + i] = d[v];
      }
    }
  }
  __syncthreads();

  // 10. C <- V_k[:, kept]^T T (rn x rn, K = M) on the matrix cores; sigma,
  //     w, p_y and A~_ij = (sigma_i C_ij + p_y,i w_j) / sigma_j.  Each tile
  //     is formed transposed (T's columns as the first operand, the same
  //     products in the same order), so that lane l holds rows i0 + l%16 of
  //     columns j0 + 4 v + l/16: a store then writes 16 consecutive rows of
  //     a column (four 128-byte pieces instead of sixteen 32-byte ones)
  {
    const int wv = tid >> 6, l = tid & 63;
    const int nt = (rn + 15) / 16;
    for (int tile = wv; tile < nt * nt; tile += CORE_THREADS / 64) {
      const int i0 = 16 * (tile % nt), j0 = 16 * (tile / nt);
      const int ia = i0 + (l & 15), jb = j0 + (l & 15);
      const int pa = ia < rn ? perm[ia] : 0;
      const d4_t d = mfma_tile(sA + (jb < rn ? jb : 0) * LDK, 1, jb < rn, sV + pa * LDK, 1, ia < rn,
                               M, l);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + 4 * v + (l >> 4);
        if (ia < rn && j < rn) {
          st->C[j * RMAX + ia] = d[v];
          st->At[j * RMAX + ia] = (sgn[ia] * d[v] + pyn[ia] * wn[j]) * isg[j];
        }
      }
    }
  }
  }
  if (tid < rn) {
    st->sigma[tid] = sgn[tid];
    st->w[tid] = wn[tid];
    st->py[tid] = pyn[tid];
  }
  if (tid == 0) {
    st->r = rn;
    st->m = mnew;
    st->refold = mnew >= fold_limit(c, rn);
    st->m_acc += 1;
    st->yy_prev = sc[2];
    st->yh_prev = sc[3];
    st->last_rho = rho;
    st->sweeps = sweeps;
    st->eig_valid = 0;
    if (sweeps > MAX_SWEEPS) latch_status(st, ST_NOCONV);
  }
}

// One update of the small state, then the stored-column count it leaves,
// tagged with the update's sequence number, to the host-visible feedback
// word (the host sizes later launches from it).
template <bool GENERAL>
__device__ __forceinline__ void core_body(const CoreArgs& c) {
  core_update<GENERAL>(c);
  if (threadIdx.x == 0 && c.fb) {
    const unsigned mm = (unsigned)c.st->m;
    *reinterpret_cast<volatile unsigned*>(c.fb) = ((c.seq & 0xFFFFFFu) << 8) | (mm & 0xFFu);
  }
}

// chained pairs and general pairs (B = T R) as separate kernels, so that the
// chained kernel carries none of the general pairs' code
__global__ __launch_bounds__(CORE_THREADS) void k_core(CoreArgs c) { core_body<false>(c); }
__global__ __launch_bounds__(CORE_THREADS) void k_core_general(CoreArgs c) { core_body<true>(c); }

__global__ __launch_bounds__(CORE_THREADS) void k_core_batch(const CoreArgs* __restrict__ cs) {
  const CoreArgs c = cs[blockIdx.x];
  core_body<false>(c);
}

hipError_t launch_core_batch(const CoreArgs* cs, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_core_batch, dim3(count), dim3(CORE_THREADS), 0, s, cs);
  return hipGetLastError();
}

hipError_t launch_core(const CoreArgs& c, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (c.tst) hipExtLaunchKernelGGL(k_core_general, dim3(1), dim3(CORE_THREADS), 0, s, e0, e1, 0, c);
  else hipExtLaunchKernelGGL(k_core, dim3(1), dim3(CORE_THREADS), 0, s, e0, e1, 0, c);
  return hipGetLastError();
}

// General pairs, before the streaming pass: p1 = U^T x = Q^T S^T x and the
// pass coefficients a = Q p1, from the projection sweep's per-workgroup
// records (fixed-order sums, as in the small-state kernel).
__global__ __launch_bounds__(CORE_THREADS) void k_coef(CoefArgs c) {
  DevState* __restrict__ st = c.st;
  constexpr int NSL = CORE_THREADS / CMAX;   // partial-sum slots per column
  __shared__ double part[NSL][CMAX];
  __shared__ double v[CMAX];
  __shared__ double p1[RMAX];
  __shared__ double sQ[CMAX * RMAX];
  const int tid = threadIdx.x;
  const int r = st->r, m = st->m;
  // Q to LDS (all of a thread's loads issued together), record sums with
  // the loads of a slot overlapped
  {
    constexpr int NQ = (CMAX * RMAX + CORE_THREADS - 1) / CORE_THREADS;
    double qv[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int idx = tid + i * CORE_THREADS;
      qv[i] = (idx < CMAX * RMAX && idx / RMAX < m && idx % RMAX < r) ? st->Q[idx] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      if (tid + i * CORE_THREADS < CMAX * RMAX) sQ[tid + i * CORE_THREADS] = qv[i];
  }
  if (tid < NSL * CMAX) {
    const int it = tid % CMAX, sl = tid / CMAX;
    double t = 0.0;
    if (it < m) {
#pragma unroll 16
      for (int b = sl; b < c.nblk; b += NSL) t += c.pproj[(int64_t)b * PW + it];
    }
    part[sl][it] = t;
  }
  __syncthreads();
  if (tid < CMAX) {
    double t = 0.0;
    for (int sl = 0; sl < NSL; ++sl) t += part[sl][tid];
    v[tid] = t;
  }
  __syncthreads();
  if (tid < RMAX) {
    double a1 = 0.0;
    if (tid < r)
      for (int c0 = 0; c0 < m; ++c0) a1 += sQ[c0 * RMAX + tid] * v[c0];
    p1[tid] = a1;
    st->p1[tid] = a1;
  }
  __syncthreads();
  if (tid < CMAX) {
    double t = 0.0;
    if (tid < m)
      for (int j = 0; j < r; ++j) t += sQ[tid * RMAX + j] * p1[j];
    st->a[tid] = t;
  }
}

hipError_t launch_coef(const CoefArgs& c, hipStream_t s) {
  hipLaunchKernelGGL(k_coef, dim3(1), dim3(CORE_THREADS), 0, s, c);
  return hipGetLastError();
}

}  // namespace odmd
