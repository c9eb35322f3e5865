// Eigendecomposition of the reduced operator and prediction coefficients.
//
// Sec. 2.3: A~ = V Lambda V^-1, Phi = U V, and the prediction
// u(t) = Phi Lambda^(t/dt) Phi^+ u(0).  With U orthonormal and the anchor
// u(0) = x_a (the last snapshot), Phi^+ u(0) = V^-1 U^T x_a = V^-1 p_y =: b~,
// so the state k steps ahead is U c_k with c_k = Re(V (Lambda^k b~)).
//
// k_eig (one 64-lane wavefront, FP64):
//   1. Householder reduction of A~ to upper Hessenberg form H = Q^T A~ Q;
//   2. Francis double-shift QR iteration to the real Schur form T = Z^T A~ Z
//      (1x1 and standardised 2x2 diagonal blocks), accumulating Z;
//   3. eigenvectors of T by back-substitution (complex arithmetic), one lane
//      per eigenvalue, then V = Z X, unit 2-norm, largest entry real > 0;
//   4. order by |lambda| descending, then Im descending;
//   5. b~ = V^-1 p_y by Gaussian elimination with partial pivoting.
// k_predict_coef: c_k for a chunk of steps, folded with the basis
// coefficients (U = S[:, :m] Q, so U c = S (Q c)).
#include <hip/hip_runtime.h>
#include <math.h>

#include "odmd_internal.h"
#include "pass.h"

namespace odmd {

constexpr int LDH = RMAX + 1;
constexpr double EPS = 2.220446049250313e-16;

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
// Smith's algorithm for a / b
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double t = b.im / b.re, den = b.re + b.im * t;
    return {(a.re + a.im * t) / den, (a.im - a.re * t) / den};
  }
  const double t = b.re / b.im, den = b.re * t + b.im;
  return {(a.re * t + a.im) / den, (a.im * t - a.re) / den};
}
__device__ __forceinline__ double cabs2(cplx a) { return hypot(a.re, a.im); }

#define Hm(i, j) H[(j) * LDH + (i)]
#define Zm(i, j) Z[(j) * LDH + (i)]

// Apply the reflector P = I - tau v v^T (v = (1, v1, v2), or (1, v1) when
// three == false) to rows k.. of H from the left over columns [c0, n) and
// to columns k.. of H (rows [0, r1]) and of Z (all rows) from the right.
__device__ void apply_reflector(double* H, double* Z, int n, int k, double tau, double v1,
                                double v2, bool three, int c0, int r1) {
  const int t = threadIdx.x;
  if (t >= c0 && t < n) {
    double s = Hm(k, t) + v1 * Hm(k + 1, t);
    if (three) s += v2 * Hm(k + 2, t);
    s *= tau;
    Hm(k, t) -= s;
    Hm(k + 1, t) -= s * v1;
    if (three) Hm(k + 2, t) -= s * v2;
  }
  __syncthreads();
  if (t <= r1) {
    double s = Hm(t, k) + v1 * Hm(t, k + 1);
    if (three) s += v2 * Hm(t, k + 2);
    s *= tau;
    Hm(t, k) -= s;
    Hm(t, k + 1) -= s * v1;
    if (three) Hm(t, k + 2) -= s * v2;
  }
  if (t < n) {
    double s = Zm(t, k) + v1 * Zm(t, k + 1);
    if (three) s += v2 * Zm(t, k + 2);
    s *= tau;
    Zm(t, k) -= s;
    Zm(t, k + 1) -= s * v1;
    if (three) Zm(t, k + 2) -= s * v2;
  }
  __syncthreads();
}

// Reflector mapping (x, y, z) to (alpha, 0, 0): v = (1, v1, v2), tau.
__device__ __forceinline__ bool make_reflector(double x, double y, double z, double& tau,
                                               double& v1, double& v2, double& alpha) {
  const double sc = fmax(fabs(x), fmax(fabs(y), fabs(z)));
  if (sc == 0.0 || (y == 0.0 && z == 0.0)) return false;
  const double isc = 1.0 / sc;     // one division per quantity, not per entry
  x *= isc;
  y *= isc;
  z *= isc;
  const double nrm = sqrt(x * x + y * y + z * z);
  const double al = x >= 0.0 ? -nrm : nrm;
  const double iden = 1.0 / (x - al);
  v1 = y * iden;
  v2 = z * iden;
  tau = (al - x) / al;
  alpha = al * sc;
  return true;
}

__device__ __forceinline__ void eig_body(DevState* st) {
  if (st->eig_valid) return;
  __shared__ double H[RMAX * LDH];
  __shared__ double Z[RMAX * LDH];
  __shared__ double Xr[(RMAX + 1) * LDH];
  __shared__ double Xi[(RMAX + 1) * LDH];
  __shared__ double wr[RMAX], wi[RMAX], hv[RMAX];
  __shared__ int srank[RMAX];
  __shared__ int sfail;
  const int t = threadIdx.x;
  const int n = st->r;
  if (n == 0) {
    if (t == 0) {
      st->eig_valid = 1;
      st->eig_status = 0;
    }
    return;
  }
  for (int idx = t; idx < n * n; idx += 64) {
    const int i = idx % n, j = idx / n;
    Hm(i, j) = st->At[j * RMAX + i];
    Zm(i, j) = (i == j) ? 1.0 : 0.0;
  }
  if (t == 0) sfail = 0;
  __syncthreads();

  // 1. Hessenberg reduction
  for (int k = 0; k + 2 < n; ++k) {
    double x2 = 0.0;
    if (t > k + 1 && t < n) x2 = Hm(t, k) * Hm(t, k);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x2 += __shfl_xor(x2, o, 64);
    const double x0 = Hm(k + 1, k);
    if (x2 == 0.0) {
      __syncthreads();
      continue;
    }
    const double nrm = sqrt(x0 * x0 + x2);
    const double al = x0 >= 0.0 ? -nrm : nrm;
    const double v0 = x0 - al;
    const double beta = 2.0 / (v0 * v0 + x2);
    if (t < n) hv[t] = (t == k + 1) ? v0 : (t > k + 1 ? Hm(t, k) : 0.0);
    __syncthreads();
    if (t >= k && t < n) {          // left: rows k+1.., column t
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += hv[i] * Hm(i, t);
      s *= beta;
      for (int i = k + 1; i < n; ++i) Hm(i, t) -= s * hv[i];
    }
    __syncthreads();
    if (t < n) {                    // right: columns k+1.., row t (H and Z)
      double s = 0.0, sz = 0.0;
      for (int j = k + 1; j < n; ++j) {
        s += Hm(t, j) * hv[j];
        sz += Zm(t, j) * hv[j];
      }
      s *= beta;
      sz *= beta;
      for (int j = k + 1; j < n; ++j) {
        Hm(t, j) -= s * hv[j];
        Zm(t, j) -= sz * hv[j];
      }
    }
    __syncthreads();
    if (t > k + 1 && t < n) Hm(t, k) = 0.0;
    if (t == 0) Hm(k + 1, k) = al;
    __syncthreads();
  }

  // norm for deflation tests on zero diagonals
  double hn = 0.0;
  for (int idx = t; idx < n * n; idx += 64) hn = fmax(hn, fabs(Hm(idx % n, idx / n)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) hn = fmax(hn, __shfl_xor(hn, o, 64));
  if (hn == 0.0) hn = 1.0;

  // 2. Francis double-shift QR to real Schur form
  int hi = n - 1, its = 0, total = 0;
  while (hi >= 0) {
    // l = the largest index in [1, hi] whose subdiagonal entry is
    // negligible, else 0: every lane tests one entry, one ballot
    bool neg = false;
    if (t >= 1 && t <= hi) {
      double s = fabs(Hm(t - 1, t - 1)) + fabs(Hm(t, t));
      if (s == 0.0) s = hn;
      neg = fabs(Hm(t, t - 1)) <= EPS * s;
    }
    const unsigned long long mask = __ballot(neg);
    const int l = mask ? 63 - __builtin_clzll(mask) : 0;
    __syncthreads();
    if (l > 0 && t == 0) Hm(l, l - 1) = 0.0;
    __syncthreads();
    if (l == hi) {
      if (t == 0) {
        wr[hi] = Hm(hi, hi);
        wi[hi] = 0.0;
      }
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const int p = hi - 1, q = hi;
      const double a = Hm(p, p), b = Hm(p, q), c = Hm(q, p), d = Hm(q, q);
      const double pp = 0.5 * (a - d);
      const double disc = pp * pp + b * c;
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double zz = pp + (pp >= 0.0 ? sq : -sq);
        double la = d + zz, lb = (zz != 0.0) ? d - b * c / zz : d;
        // rotation whose first column is the eigenvector (zz, c) of la
        const double h = hypot(zz, c);
        __syncthreads();
        if (h > 0.0) {
          const double cs = zz / h, sn = c / h;
          if (t >= p && t < n) {      // rows p, q from the left (G^T)
            const double u = Hm(p, t), v = Hm(q, t);
            Hm(p, t) = cs * u + sn * v;
            Hm(q, t) = -sn * u + cs * v;
          }
          __syncthreads();
          if (t <= q) {               // columns p, q from the right
            const double u = Hm(t, p), v = Hm(t, q);
            Hm(t, p) = cs * u + sn * v;
            Hm(t, q) = -sn * u + cs * v;
          }
          if (t < n) {
            const double u = Zm(t, p), v = Zm(t, q);
            Zm(t, p) = cs * u + sn * v;
            Zm(t, q) = -sn * u + cs * v;
          }
          __syncthreads();
          if (t == 0) Hm(q, p) = 0.0;
          la = Hm(p, p);
          lb = Hm(q, q);
          __syncthreads();
        }
        if (t == 0) {
          wr[p] = la;
          wi[p] = 0.0;
          wr[q] = lb;
          wi[q] = 0.0;
        }
      } else {
        if (t == 0) {
          wr[p] = wr[q] = a - pp;        // (a + d) / 2
          wi[p] = sqrt(-disc);
          wi[q] = -sqrt(-disc);
        }
      }
      __syncthreads();
      hi -= 2;
      its = 0;
      continue;
    }
    if (total >= 30 * n) {
      if (t == 0) sfail = 1;
      break;
    }
    ++its;
    ++total;
    double s, tt;
    if (its == 10 || its == 20) {     // exceptional shift
      const double w = fabs(Hm(hi, hi - 1)) + fabs(Hm(hi - 1, hi - 2));
      s = 1.5 * w;
      tt = w * w;
    } else {
      s = Hm(hi - 1, hi - 1) + Hm(hi, hi);
      tt = Hm(hi - 1, hi - 1) * Hm(hi, hi) - Hm(hi - 1, hi) * Hm(hi, hi - 1);
    }
    double x = Hm(l, l) * Hm(l, l) + Hm(l, l + 1) * Hm(l + 1, l) - s * Hm(l, l) + tt;
    double y = Hm(l + 1, l) * (Hm(l, l) + Hm(l + 1, l + 1) - s);
    double z = Hm(l + 1, l) * Hm(l + 2, l + 1);
    for (int k = l; k <= hi - 1; ++k) {
      const bool three = k < hi - 1;
      double tau, v1, v2 = 0.0, al;
      const bool ok = make_reflector(x, y, three ? z : 0.0, tau, v1, v2, al);
      __syncthreads();
      if (ok) {
        const int c0 = k > l ? k - 1 : l;
        const int r1 = min(k + 3, hi);
        apply_reflector(H, Z, n, k, tau, v1, v2, three, c0, r1);
        if (k > l && t == 0) {
          Hm(k, k - 1) = al;
          Hm(k + 1, k - 1) = 0.0;
          if (three) Hm(k + 2, k - 1) = 0.0;
        }
        __syncthreads();
      }
      if (k < hi - 1) {
        x = Hm(k + 1, k);
        y = Hm(k + 2, k);
        z = (k + 3 <= hi) ? Hm(k + 3, k) : 0.0;
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // 3. eigenvectors of the quasi-triangular T by back-substitution
  const double smin = fmax(EPS * hn, 1e-300);
  if (t < n && !sfail) {
    const cplx lam = {wr[t], wi[t]};
    for (int i = 0; i < n; ++i) {
      Xr[t * LDH + i] = 0.0;
      Xi[t * LDH + i] = 0.0;
    }
    int start;
    if (wi[t] == 0.0) {
      Xr[t * LDH + t] = 1.0;
      start = t - 1;
    } else {
      const int p = (wi[t] > 0.0) ? t : t - 1;  // block (p, p+1)
      const int q = p + 1;
      const cplx a = {Hm(p, p), 0.0}, b = {Hm(p, q), 0.0};
      const cplx c = {Hm(q, p), 0.0}, d = {Hm(q, q), 0.0};
      cplx u1 = b, u2 = csub(lam, a);            // from row 1
      cplx w1 = csub(lam, d), w2 = c;            // from row 2
      if (cabs2(u1) + cabs2(u2) < cabs2(w1) + cabs2(w2)) {
        u1 = w1;
        u2 = w2;
      }
      Xr[t * LDH + p] = u1.re;
      Xi[t * LDH + p] = u1.im;
      Xr[t * LDH + q] = u2.re;
      Xi[t * LDH + q] = u2.im;
      start = p - 1;
    }
    int i = start;
    while (i >= 0) {
      const bool blk = i > 0 && Hm(i, i - 1) != 0.0;
      if (!blk) {
        cplx s = {0.0, 0.0};
        for (int j = i + 1; j < n; ++j) {
          const cplx xj = {Xr[t * LDH + j], Xi[t * LDH + j]};
          s = cadd(s, cmul({Hm(i, j), 0.0}, xj));
        }
        cplx den = csub({Hm(i, i), 0.0}, lam);
        if (cabs2(den) < smin) den = {smin, 0.0};
        const cplx xi = cdiv({-s.re, -s.im}, den);
        Xr[t * LDH + i] = xi.re;
        Xi[t * LDH + i] = xi.im;
        i -= 1;
      } else {
        const int i0 = i - 1;
        cplx s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
        for (int j = i + 1; j < n; ++j) {
          const cplx xj = {Xr[t * LDH + j], Xi[t * LDH + j]};
          s0 = cadd(s0, cmul({Hm(i0, j), 0.0}, xj));
          s1 = cadd(s1, cmul({Hm(i, j), 0.0}, xj));
        }
        const cplx m00 = csub({Hm(i0, i0), 0.0}, lam), m01 = {Hm(i0, i), 0.0};
        const cplx m10 = {Hm(i, i0), 0.0}, m11 = csub({Hm(i, i), 0.0}, lam);
        cplx det = csub(cmul(m00, m11), cmul(m01, m10));
        if (cabs2(det) < smin * smin) det = {smin * smin, 0.0};
        const cplx r0 = {-s0.re, -s0.im}, r1 = {-s1.re, -s1.im};
        const cplx x0 = cdiv(csub(cmul(r0, m11), cmul(m01, r1)), det);
        const cplx x1 = cdiv(csub(cmul(m00, r1), cmul(m10, r0)), det);
        Xr[t * LDH + i0] = x0.re;
        Xi[t * LDH + i0] = x0.im;
        Xr[t * LDH + i] = x1.re;
        Xi[t * LDH + i] = x1.im;
        i -= 2;
      }
      // rescale to keep the entries bounded
      double mx = 0.0;
      for (int j = max(i + 1, 0); j < n; ++j)
        mx = fmax(mx, fabs(Xr[t * LDH + j]) + fabs(Xi[t * LDH + j]));
      if (mx > 1e100) {
        const double f = 1.0 / mx;
        for (int j = 0; j < n; ++j) {
          Xr[t * LDH + j] *= f;
          Xi[t * LDH + j] *= f;
        }
      }
    }
  }
  __syncthreads();

  // V = Z X, normalised, stored at its rank in the output order
  if (t < n && !sfail) {
    const double ml = hypot(wr[t], wi[t]);
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double mj = hypot(wr[j], wi[j]);
      rank += (mj > ml) || (mj == ml && (wi[j] > wi[t] || (wi[j] == wi[t] && j < t)));
    }
    srank[t] = rank;
    double* __restrict__ vr = st->V_re + rank * RMAX;
    double* __restrict__ vi = st->V_im + rank * RMAX;
    double nrm2 = 0.0, best = -1.0;
    int ib = 0;
    for (int i = 0; i < n; ++i) {
      double ar = 0.0, ai = 0.0;
      for (int j = 0; j < n; ++j) {
        ar += Zm(i, j) * Xr[t * LDH + j];
        ai += Zm(i, j) * Xi[t * LDH + j];
      }
      vr[i] = ar;
      vi[i] = ai;
      const double m2 = ar * ar + ai * ai;
      nrm2 += m2;
      if (m2 > best) {
        best = m2;
        ib = i;
      }
    }
    // unit norm, largest-modulus entry real and positive: multiply by
    // conj(v_ib) / (|v_ib| ||v||)
    const double m = sqrt(best), f = 1.0 / sqrt(nrm2);
    const double pr = vr[ib] / m * f, pi = -vi[ib] / m * f;
    for (int i = 0; i < n; ++i) {
      const double ar = vr[i], ai = vi[i];
      vr[i] = ar * pr - ai * pi;
      vi[i] = i == ib ? 0.0 : ar * pi + ai * pr;
    }
    st->lam_re[rank] = wr[t];
    st->lam_im[rank] = wi[t];
  }
  __threadfence();
  __syncthreads();

  // 5. b~ = V^-1 p_y: Gaussian elimination with partial pivoting on [V | p_y]
  //    (reuses Xr/Xi as the complex augmented matrix, column-major)
  if (!sfail) {
    for (int idx = t; idx < n * (n + 1); idx += 64) {
      const int i = idx % n, j = idx / n;
      if (j < n) {
        Xr[j * LDH + i] = st->V_re[j * RMAX + i];
        Xi[j * LDH + i] = st->V_im[j * RMAX + i];
      } else {
        Xr[j * LDH + i] = st->py[i];
        Xi[j * LDH + i] = 0.0;
      }
    }
    __syncthreads();
    for (int cidx = 0; cidx < n; ++cidx) {
      // pivot: the largest modulus in rows cidx.., the first of equals
      // (one row per lane, then a butterfly over the wavefront)
      double best = -1.0;
      int piv = n;
      if (t >= cidx && t < n) {
        best = hypot(Xr[cidx * LDH + t], Xi[cidx * LDH + t]);
        piv = t;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int op = __shfl_xor(piv, o, 64);
        if (ob > best || (ob == best && op < piv)) {
          best = ob;
          piv = op;
        }
      }
      __syncthreads();
      if (piv != cidx) {
        for (int j = t; j <= n; j += 64) {
          const double ar = Xr[j * LDH + cidx], ai = Xi[j * LDH + cidx];
          Xr[j * LDH + cidx] = Xr[j * LDH + piv];
          Xi[j * LDH + cidx] = Xi[j * LDH + piv];
          Xr[j * LDH + piv] = ar;
          Xi[j * LDH + piv] = ai;
        }
      }
      __syncthreads();
      cplx dv = {Xr[cidx * LDH + cidx], Xi[cidx * LDH + cidx]};
      if (cabs2(dv) < 1e-300) dv = {1e-300, 0.0};
      if (t > cidx && t < n) {
        const cplx f = cdiv({Xr[cidx * LDH + t], Xi[cidx * LDH + t]}, dv);
        for (int j = cidx; j <= n; ++j) {
          const cplx u = cmul(f, {Xr[j * LDH + cidx], Xi[j * LDH + cidx]});
          Xr[j * LDH + t] -= u.re;
          Xi[j * LDH + t] -= u.im;
        }
      }
      __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {
      cplx dv = {Xr[i * LDH + i], Xi[i * LDH + i]};
      if (cabs2(dv) < 1e-300) dv = {1e-300, 0.0};
      const cplx xi = cdiv({Xr[n * LDH + i], Xi[n * LDH + i]}, dv);
      __syncthreads();
      if (t < i) {
        const cplx u = cmul({Xr[i * LDH + t], Xi[i * LDH + t]}, xi);
        Xr[n * LDH + t] -= u.re;
        Xi[n * LDH + t] -= u.im;
      }
      if (t == 0) {
        st->bt_re[i] = xi.re;
        st->bt_im[i] = xi.im;
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    st->eig_status = sfail;
    if (sfail) latch_status(st, ST_NOCONV);
    st->eig_valid = 1;
  }
}

// Coefficients of one chunk of predicted states: column kk (state
// a+k0+kk+1) of coefA is Q c_k, so that the state is S[:, :m] Q c_k.
__global__ __launch_bounds__(256) void k_predict_coef(DevState* st, int k0, int K) {
  __shared__ double zr[4][RMAX], zi[4][RMAX], cc[4][RMAX];
  const int col = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kk = blockIdx.x * 4 + col;
  const int n = st->r, m = st->m;
  const bool live = kk < K && n > 0 && st->eig_status == 0;
  const double kstep = (double)(k0 + kk + 1);
  if (live && l < n) {
    const double lr = st->lam_re[l], li = st->lam_im[l];
    const double mag = pow(hypot(lr, li), kstep);
    const double ang = kstep * atan2(li, lr);
    double sn, cs;
    sincos(ang, &sn, &cs);
    const cplx p = {mag * cs, mag * sn};
    const cplx z = cmul(p, {st->bt_re[l], st->bt_im[l]});
    zr[col][l] = z.re;
    zi[col][l] = z.im;
  }
  __syncthreads();
  if (live && l < n) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += st->V_re[j * RMAX + l] * zr[col][j] - st->V_im[j * RMAX + l] * zi[col][j];
    cc[col][l] = s;
  }
  __syncthreads();
  if (kk < K) {
    for (int c = l; c < CMAX; c += 64) {
      double v = 0.0;
      if (live && c < m)
        for (int k = 0; k < n; ++k) v += st->Q[c * RMAX + k] * cc[col][k];
      st->coefA[kk * CMAX + c] = v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n == 0 || st->eig_status != 0))
    latch_status(st, n == 0 ? ST_EMPTY : ST_NOCONV);
}

// Coefficients that materialise the basis: column k of U is S[:, :m] Q[:, k].
__global__ __launch_bounds__(256) void k_basis_coef(DevState* st) {
  const int m = st->m, r = st->r;
  for (int idx = threadIdx.x; idx < CMAX * RMAX; idx += 256) {
    const int c = idx % CMAX, k = idx / CMAX;
    st->coefA[k * CMAX + c] = (c < m && k < r) ? st->Q[c * RMAX + k] : 0.0;
  }
}

__global__ __launch_bounds__(64) void k_eig(DevState* st) { eig_body(st); }

// One workgroup per stream of a device-resident table of states.
__global__ __launch_bounds__(64) void k_eig_batch(DevState* const* __restrict__ sts) {
  eig_body(sts[blockIdx.x]);
}

hipError_t launch_eig(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_eig_batch(DevState* const* sts, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_batch, dim3(count), dim3(64), 0, s, sts);
  return hipGetLastError();
}

hipError_t launch_predict_coef(DevState* st, int k0, int steps, hipStream_t s) {
  hipLaunchKernelGGL(k_predict_coef, dim3((steps + 3) / 4), dim3(256), 0, s, st, k0, steps);
  return hipGetLastError();
}

hipError_t launch_basis_coef(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_coef, dim3(1), dim3(256), 0, s, st);
  return hipGetLastError();
}

}  // namespace odmd
