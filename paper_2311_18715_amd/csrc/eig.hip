// Eigendecomposition of the reduced operator and prediction coefficients.
//
// Sec. 2.3: A~ = V Lambda V^-1 and Phi = U V (the projected DMD modes), and
// the prediction u(t) = Phi Lambda^(t/dt) Phi^+ u(0).
//
// k_eig (one 64-lane wavefront, FP64), on demand for the eigenpairs:
//   1. Householder reduction of A~ to upper Hessenberg form H = Q^T A~ Q;
//   2. Francis double-shift QR iteration to the real Schur form T = Z^T A~ Z
//      (1x1 and standardised 2x2 diagonal blocks), accumulating Z;
//   3. eigenvectors of T by back-substitution (complex arithmetic), one lane
//      per eigenvalue, then V = Z X, unit 2-norm, largest entry real > 0;
//   4. order by |lambda| descending, then Im descending.
// k_power_coef: the prediction's coefficients for a chunk of steps, as
// powers of A~ applied to U^T x_a (equal to the eigenvector form at integer
// steps, see below), folded with the basis coefficients (U = S[:, :m] Q,
// so U c = S (Q c)).
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

// The value of v in the given lane (a wave-uniform index), in every lane.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/x and 1/sqrt(x): hardware estimates refined by two Newton steps each
__device__ __forceinline__ double recip_n(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsqrt_n(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  r = r * __builtin_fma(-h * r, r, 1.5);
  r = r * __builtin_fma(-h * r, r, 1.5);
  return r;
}

// Reflector mapping (x, y, z) to (alpha, 0, 0): v = (1, v1, v2), tau.
__device__ __forceinline__ bool make_reflector(double x, double y, double z, double& tau,
                                               double& v1, double& v2, double& alpha) {
  if (y == 0.0 && z == 0.0) return false;
  double ss = __builtin_fma(z, z, __builtin_fma(y, y, x * x));
  double sc = 1.0;
  if (!(ss > 0x1p-960 && ss < 0x1p960)) {     // rescale (rare): avoid under/overflow
    sc = fmax(fabs(x), fmax(fabs(y), fabs(z)));
    const double isc = 1.0 / sc;
    x *= isc;
    y *= isc;
    z *= isc;
    ss = __builtin_fma(z, z, __builtin_fma(y, y, x * x));
  }
  const double rn = rsqrt_n(ss);               // 1 / ||(x, y, z)||
  double nrm = ss * rn;
  nrm = __builtin_fma(0.5 * rn, __builtin_fma(-nrm, nrm, ss), nrm);
  const double al = x >= 0.0 ? -nrm : nrm;
  const double id = recip_n(x - al);           // |x - al| = |x| + nrm
  v1 = y * id;
  v2 = z * id;
  tau = __builtin_fma(fabs(x), rn, 1.0);       // (al - x) / al = 1 + |x| / nrm
  alpha = al * sc;
  return true;
}

// One step of the double-shift bulge chase: the reflector P = I - tau v v^T
// (v = (1, v1, v2); (1, v1) for the last step, THREE false) built from
// (x, y, z), applied as H <- P H P and Z <- Z P.  Every lane t is column t of
// the left application (rows k .. k+2, columns [c0, n) outside the 3 x 3
// block), row t of the right one (columns k .. k+2, rows [0, r1]) and row t
// of Z's.  Rows k .. k+2 meet both: those lanes apply the left reflector to
// their row of the 3 x 3 block (read by every lane) before the right one,
// and the column lanes leave the block to them, so no entry is written
// twice.  A lane outside a role reads and writes its own slots of dum
// instead (straight-line code, no divergent branches).  Returns this lane's
// new H(t, k) (rows <= r1), from which the next step's (x, y, z) are taken.
template <bool THREE, bool VECS>
__device__ __forceinline__ double bulge_step(double* H, double* Z, double* dum, int n, int l, int hi,
                                             int k, double x, double y, double z) {
  constexpr int nb = THREE ? 3 : 2;
  const int t = threadIdx.x;
  const int c0 = k > l ? k - 1 : l;
  const int r1 = THREE ? min(k + 3, hi) : hi;
  const bool col_live = t >= c0 && t < n && (t < k || t >= k + nb);
  const bool row_live = t <= r1;
  const bool z_live = t < n;
  double* pc = col_live ? &Hm(k, t) : dum + 9 * t;          // rows k .. k+nb-1, stride 1
  double* pr0 = row_live ? &Hm(t, k) : dum + 9 * t + 3;
  double* pr1 = row_live ? &Hm(t, k + 1) : dum + 9 * t + 4;
  double* pr2 = row_live ? &Hm(t, k + 2) : dum + 9 * t + 5;
  double* pz0 = z_live ? &Zm(t, k) : dum + 9 * t + 6;
  double* pz1 = z_live ? &Zm(t, k + 1) : dum + 9 * t + 7;
  double* pz2 = z_live ? &Zm(t, k + 2) : dum + 9 * t + 8;
  double b0[nb], b1[nb], b2[nb];                             // H(k .. k+2, k + c)
#pragma unroll
  for (int c = 0; c < nb; ++c) {
    b0[c] = Hm(k, k + c);
    b1[c] = Hm(k + 1, k + c);
    b2[c] = THREE ? Hm(k + 2, k + c) : 0.0;
  }
  double cv0 = pc[0], cv1 = pc[1], cv2 = THREE ? pc[2] : 0.0;
  double rv0 = *pr0, rv1 = *pr1, rv2 = THREE ? *pr2 : 0.0;
  double zv0 = VECS ? *pz0 : 0.0, zv1 = VECS ? *pz1 : 0.0, zv2 = VECS && THREE ? *pz2 : 0.0;
  double tau, v1, v2 = 0.0, al;
  if (!make_reflector(x, y, THREE ? z : 0.0, tau, v1, v2, al)) return rv0;   // uniform
  // column t, rows k .. k+2 (the bulge column k - 1 becomes (alpha, 0, 0))
  const double sc = tau * (cv0 + v1 * cv1 + v2 * cv2);
  const bool bulge = k > l && t == k - 1;
  cv0 = bulge ? al : cv0 - sc;
  cv1 = bulge ? 0.0 : cv1 - sc * v1;
  cv2 = bulge ? 0.0 : cv2 - sc * v2;
  // rows k .. k+2: row t of the block after the left application
  const int a = t - k;
  const bool in_blk = a >= 0 && a < nb;
  const double va = a == 1 ? v1 : (a == 2 ? v2 : 1.0);
#pragma unroll
  for (int c = 0; c < nb; ++c) {
    const double sb = tau * (b0[c] + v1 * b1[c] + v2 * b2[c]);
    const double ba = a == 1 ? b1[c] : (a == 2 ? b2[c] : b0[c]);
    const double nr = ba - sb * va;
    if (c == 0) rv0 = in_blk ? nr : rv0;
    if (c == 1) rv1 = in_blk ? nr : rv1;
    if (c == 2) rv2 = in_blk ? nr : rv2;
  }
  // row t, columns k .. k+2, and row t of Z
  const double sr = tau * (rv0 + v1 * rv1 + v2 * rv2);
  rv0 -= sr;
  rv1 -= sr * v1;
  rv2 -= sr * v2;
  if (VECS) {
    const double sz = tau * (zv0 + v1 * zv1 + v2 * zv2);
    zv0 -= sz;
    zv1 -= sz * v1;
    zv2 -= sz * v2;
  }
  pc[0] = cv0;
  pc[1] = cv1;
  if (THREE) pc[2] = cv2;
  *pr0 = rv0;
  *pr1 = rv1;
  if (THREE) *pr2 = rv2;
  if (VECS) {
    *pz0 = zv0;
    *pz1 = zv1;
    if (THREE) *pz2 = zv2;
  }
  return rv0;
}

// VECS false: eigenvalues only (no Z, eigenvectors or V); the cache level
// eig_valid is 1 after such a call and 2 after a call with vectors.
template <bool VECS>
__device__ __forceinline__ void eig_body(DevState* st) {
  if (st->eig_valid >= (VECS ? 2 : 1)) return;
  __shared__ double H[RMAX * LDH];
  __shared__ double Z[RMAX * LDH];
  __shared__ double Xr[(RMAX + 1) * LDH];
  __shared__ double Xi[(RMAX + 1) * LDH];
  __shared__ double wr[RMAX], wi[RMAX], hv[RMAX];
  __shared__ double dum[64 * 9];           // slots of lanes outside a role of a bulge step
  __shared__ int sfail;
  const int t = threadIdx.x;
  const int n = st->r;
  if (n == 0) {
    if (t == 0) {
      st->eig_valid = 2;
      st->eig_status = 0;
    }
    return;
  }
  for (int idx = t; idx < n * n; idx += 64) {
    const int i = idx % n, j = idx / n;
    Hm(i, j) = st->At[j * RMAX + i];
    if (VECS) Zm(i, j) = (i == j) ? 1.0 : 0.0;
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
      double s = 0.0, s2 = 0.0;
      int i = k + 1;
#pragma unroll 4
      for (; i + 1 < n; i += 2) {
        s = __builtin_fma(hv[i], Hm(i, t), s);
        s2 = __builtin_fma(hv[i + 1], Hm(i + 1, t), s2);
      }
      if (i < n) s = __builtin_fma(hv[i], Hm(i, t), s);
      s = (s + s2) * beta;
#pragma unroll 8
      for (int i = k + 1; i < n; ++i) Hm(i, t) -= s * hv[i];
    }
    __syncthreads();
    if (t < n) {                    // right: columns k+1.., row t (H and Z)
      double s = 0.0, sz = 0.0, s2 = 0.0, sz2 = 0.0;
      int j = k + 1;
#pragma unroll 4
      for (; j + 1 < n; j += 2) {
        s = __builtin_fma(Hm(t, j), hv[j], s);
        s2 = __builtin_fma(Hm(t, j + 1), hv[j + 1], s2);
        if (VECS) {
          sz = __builtin_fma(Zm(t, j), hv[j], sz);
          sz2 = __builtin_fma(Zm(t, j + 1), hv[j + 1], sz2);
        }
      }
      if (j < n) {
        s = __builtin_fma(Hm(t, j), hv[j], s);
        if (VECS) sz = __builtin_fma(Zm(t, j), hv[j], sz);
      }
      s = (s + s2) * beta;
      sz = (sz + sz2) * beta;
#pragma unroll 8
      for (int j = k + 1; j < n; ++j) {
        Hm(t, j) -= s * hv[j];
        if (VECS) Zm(t, j) -= sz * hv[j];
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
          if (VECS && t < n) {
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
    // Bulge chase: one barrier per step; the next step's (x, y, z), the new
    // H(k+1 .. k+3, k), come from the registers of the lanes of those rows.
    for (int k = l; k < hi - 1; ++k) {
      const double colk = bulge_step<true, VECS>(H, Z, dum, n, l, hi, k, x, y, z);
      x = readlane_d(colk, k + 1);
      y = readlane_d(colk, k + 2);
      z = (k + 3 <= hi) ? readlane_d(colk, k + 3) : 0.0;
      __syncthreads();
    }
    bulge_step<false, VECS>(H, Z, dum, n, l, hi, hi - 1, x, y, 0.0);
    __syncthreads();
  }
  __syncthreads();

  // 3. eigenvectors of the quasi-triangular T by back-substitution
  const double smin = fmax(EPS * hn, 1e-300);
  if (VECS && t < n && !sfail) {
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
    // running bound of the computed entries, for the rescaling test
    double mx = 0.0;
    for (int j = start + 1; j < n; ++j) mx = fmax(mx, fabs(Xr[t * LDH + j]) + fabs(Xi[t * LDH + j]));
    int i = start;
    while (i >= 0) {
      const bool blk = i > 0 && Hm(i, i - 1) != 0.0;
      // s = sum_{j > i} H(row, j) x_j for the one or two rows of this block
      // (H real: two real sums per row, two accumulators each)
      const int i0 = blk ? i - 1 : i;
      double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;   // row i0
      double u0r = 0.0, u0i = 0.0, u1r = 0.0, u1i = 0.0;   // row i (block only)
      int j = i + 1;
      for (; j + 1 < n; j += 2) {
        const double xr0 = Xr[t * LDH + j], xi0 = Xi[t * LDH + j];
        const double xr1 = Xr[t * LDH + j + 1], xi1 = Xi[t * LDH + j + 1];
        const double h0 = Hm(i0, j), h1 = Hm(i0, j + 1);
        s0r = __builtin_fma(h0, xr0, s0r);
        s0i = __builtin_fma(h0, xi0, s0i);
        s1r = __builtin_fma(h1, xr1, s1r);
        s1i = __builtin_fma(h1, xi1, s1i);
        if (blk) {                               // this lane's block row
          const double g0 = Hm(i, j), g1 = Hm(i, j + 1);
          u0r = __builtin_fma(g0, xr0, u0r);
          u0i = __builtin_fma(g0, xi0, u0i);
          u1r = __builtin_fma(g1, xr1, u1r);
          u1i = __builtin_fma(g1, xi1, u1i);
        }
      }
      if (j < n) {
        const double xr0 = Xr[t * LDH + j], xi0 = Xi[t * LDH + j];
        const double h0 = Hm(i0, j);
        s0r = __builtin_fma(h0, xr0, s0r);
        s0i = __builtin_fma(h0, xi0, s0i);
        if (blk) {
          const double g0 = Hm(i, j);
          u0r = __builtin_fma(g0, xr0, u0r);
          u0i = __builtin_fma(g0, xi0, u0i);
        }
      }
      if (!blk) {
        cplx den = csub({Hm(i, i), 0.0}, lam);
        if (cabs2(den) < smin) den = {smin, 0.0};
        const cplx xi = cdiv({-(s0r + s1r), -(s0i + s1i)}, den);
        Xr[t * LDH + i] = xi.re;
        Xi[t * LDH + i] = xi.im;
        mx = fmax(mx, fabs(xi.re) + fabs(xi.im));
        i -= 1;
      } else {
        const cplx m00 = csub({Hm(i0, i0), 0.0}, lam), m01 = {Hm(i0, i), 0.0};
        const cplx m10 = {Hm(i, i0), 0.0}, m11 = csub({Hm(i, i), 0.0}, lam);
        cplx det = csub(cmul(m00, m11), cmul(m01, m10));
        if (cabs2(det) < smin * smin) det = {smin * smin, 0.0};
        const cplx r0 = {-(s0r + s1r), -(s0i + s1i)}, r1 = {-(u0r + u1r), -(u0i + u1i)};
        const cplx x0 = cdiv(csub(cmul(r0, m11), cmul(m01, r1)), det);
        const cplx x1 = cdiv(csub(cmul(m00, r1), cmul(m10, r0)), det);
        Xr[t * LDH + i0] = x0.re;
        Xi[t * LDH + i0] = x0.im;
        Xr[t * LDH + i] = x1.re;
        Xi[t * LDH + i] = x1.im;
        mx = fmax(mx, fmax(fabs(x0.re) + fabs(x0.im), fabs(x1.re) + fabs(x1.im)));
        i -= 2;
      }
      // rescale to keep the entries bounded
      if (mx > 1e100) {
        const double f = 1.0 / mx;
        for (int jj = 0; jj < n; ++jj) {
          Xr[t * LDH + jj] *= f;
          Xi[t * LDH + jj] *= f;
        }
        mx = 1.0;
      }
    }
  }
  __syncthreads();

  // the eigenvalues at their rank in the output order; with vectors,
  // V = Z X normalised, at the same rank
  if (t < n) hv[t] = hypot(wr[t], wi[t]);    // |lambda| (hv is free after the reduction)
  __syncthreads();
  if (t < n && !sfail) {
    const double ml = hv[t];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double mj = hv[j];
      rank += (mj > ml) || (mj == ml && (wi[j] > wi[t] || (wi[j] == wi[t] && j < t)));
    }
    st->lam_re[rank] = wr[t];
    st->lam_im[rank] = wi[t];
    if (VECS) {
      double* __restrict__ vr = st->V_re + rank * RMAX;
      double* __restrict__ vi = st->V_im + rank * RMAX;
      // entries i0 .. i0+3 of Z X[:, t]: one load of x_j serves four rows of
      // Z (rows past n read row 0 and are not used)
      auto zx4 = [&](int i0, double (&ar)[4], double (&ai)[4]) {
        int ir[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar[u] = 0.0;
          ai[u] = 0.0;
          ir[u] = i0 + u < n ? i0 + u : 0;
        }
        for (int j = 0; j < n; ++j) {
          const double xr = Xr[t * LDH + j], xi = Xi[t * LDH + j];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double z = Zm(ir[u], j);
            ar[u] = __builtin_fma(z, xr, ar[u]);
            ai[u] = __builtin_fma(z, xi, ai[u]);
          }
        }
      };
      // first pass: the norm and the largest-modulus entry; the second forms
      // the entries again (bit for bit) and writes them normalised
      double nrm2 = 0.0, best = -1.0, vbr = 0.0, vbi = 0.0;
      int ib = 0;
      for (int i0 = 0; i0 < n; i0 += 4) {
        double ar[4], ai[4];
        zx4(i0, ar, ai);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (i0 + u < n) {
            const double m2 = ar[u] * ar[u] + ai[u] * ai[u];
            nrm2 += m2;
            if (m2 > best) {
              best = m2;
              ib = i0 + u;
              vbr = ar[u];
              vbi = ai[u];
            }
          }
        }
      }
      // unit norm, largest-modulus entry real and positive: multiply by
      // conj(v_ib) / (|v_ib| ||v||)
      const double m = sqrt(best), f = 1.0 / sqrt(nrm2);
      const double pr = vbr / m * f, pi = -vbi / m * f;
                                               // V[:, rank] = (Z X[:, t]) (pr + i pi)
      for (int i0 = 0; i0 < n; i0 += 4) {
        double ar[4], ai[4];
        zx4(i0, ar, ai);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u;
          if (i < n) {
            vr[i] = ar[u] * pr - ai[u] * pi;
            vi[i] = i == ib ? 0.0 : ar[u] * pi + ai[u] * pr;
          }
        }
      }
    }
  }
  __threadfence();
  __syncthreads();

  if (t == 0) {
    st->eig_status = sfail;
    if (sfail) latch_status(st, ST_NOCONV);
    st->eig_valid = VECS ? 2 : 1;
  }
}

// Prediction coefficients by powers of A~ (Sec. 2.3).  With U orthonormal,
// Phi = U V and the anchor x_a (Phi^+ x_a = V^-1 U^T x_a = V^-1 p_y), the
// state k steps ahead Phi Lambda^k Phi^+ x_a = U V Lambda^k V^-1 p_y equals
// U A~^k p_y: the same states without the eigendecomposition (and defined
// also where A~ has no full set of eigenvectors).  One workgroup forms
// c_k = A~^k p_y for one chunk of steps k0+1 .. k0+K by doubling: c_{k0+1}
// = A~ c_{k0}; with columns 1 .. w known and P = A~^w, columns w+1 .. 2w
// are P times columns 1 .. w, then P <- P^2.  The columns stay in LDS
// (leading dimension r | 1; the host sizes chunks by coef_chunk(r_max)),
// and are written out as Q c_k, the coefficients of the stored columns
// (U = S[:, :m] Q).  c_{k0+K} is kept in cfwd, where the next chunk starts.
// Products are 16 x 16 FP64 matrix-core tiles (16x16x4 operand layout:
// lane l supplies row or column l % 16 at k-step offset l / 16; element v
// of lane l's result is row 4 v + l / 16, column l % 16), spread over the
// workgroup's 16 wavefronts: a doubling's products and its squaring are
// one list of tiles.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int LP = RMAX + 1;            // leading dimension of the LDS matrices
constexpr int PC_THREADS = 1024;
constexpr int PC_NWV = PC_THREADS / 64;
constexpr int PC_NA = RMAX * RMAX / PC_THREADS;                    // A~ entries per thread
constexpr int PC_NQ = (CMAX * LP + PC_THREADS - 1) / PC_THREADS;   // Q entries per thread

struct PowerLds {
  double M[2 * RMAX * LP];              // A~^w and its square; then Q
  double col[PC_LCOL];                  // c_k of this chunk, column kk at kk * ldc
  double sv[RMAX];
};
static_assert(CMAX * LP <= 2 * RMAX * LP, "Q fits the power buffers");

// One 16 x 16 tile: sum over the k-steps s < 4 NT of A(s) B(s), where a(s)
// and b(s) give this lane's operands; two accumulators over alternate
// k-steps.  NT 16-row tiles cover the rank (entries past it are zero).
// The operands of a half of the k-steps (all of them for one or two
// tiles) are loaded before its products (the scheduling barrier keeps the
// compiler from spreading the loads between the products, where each pair
// of products waited for the next loads); halves keep a 1024-thread
// workgroup within 128 registers.
template <int NT, class FA, class FB>
__device__ __forceinline__ d4_t tile_sum(FA a, FB b) {
  constexpr int NH = NT > 2 ? 2 : 1;        // halves of the k-steps (fewer live operands)
  constexpr int KH = 4 * NT / NH;
  d4_t d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0;
#pragma unroll
  for (int hf = 0; hf < NH; ++hf) {
    double av[KH], bv[KH];
#pragma unroll
    for (int s = 0; s < KH; ++s) {
      av[s] = a(hf * KH + s);
      bv[s] = b(hf * KH + s);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KH; s += 2) {
      d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s + 1], bv[s + 1], d1, 0, 0, 0);
    }
  }
  return d0 + d1;
}

template <int NT>
__device__ __forceinline__ void power_body(DevState* st, PowerLds& S, int k0, int K, int koff, int n, int m) {
  const int t = threadIdx.x, l = t & 63, wv = t >> 6;
  const int lr = l & 15, lk = l >> 4;                // operand row/column, k-step offset
  const int ldc = n | 1;
  double* const out = st->coefA + koff * CMAX;       // column kk at out + kk * CMAX
  // every load of A~, Q and the start vector in flight at once
  double ra[PC_NA], rq[PC_NQ];
#pragma unroll
  for (int u = 0; u < PC_NA; ++u) {
    const int idx = t + u * PC_THREADS, i = idx % RMAX, j = idx / RMAX;
    const bool ok = i < n && j < n;
    const double x = st->At[ok ? j * RMAX + i : 0];
    ra[u] = ok ? x : 0.0;
  }
#pragma unroll
  for (int u = 0; u < PC_NQ; ++u) {
    const int idx = t + u * PC_THREADS, k = idx % LP, c = idx / LP;
    const bool ok = c < m && k < n;
    const double x = st->Q[ok ? c * RMAX + k : 0];
    rq[u] = ok ? x : 0.0;
  }
  const double s0 = t < n ? (k0 == 0 ? st->py[t] : st->cfwd[t]) : 0.0;
  double* P = S.M;
  double* P2 = S.M + RMAX * LP;
#pragma unroll
  for (int u = 0; u < PC_NA; ++u) {
    const int idx = t + u * PC_THREADS;
    P[(idx / RMAX) * LP + idx % RMAX] = ra[u];
  }
  if (t < RMAX) S.sv[t] = s0;
  __syncthreads();
  if (t < n) {                                       // c_{k0+1} = A~ c_{k0}
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 16 * NT; ++j) a[j & 3] = __builtin_fma(P[j * LP + t], S.sv[j], a[j & 3]);
    S.col[t] = (a[0] + a[1]) + (a[2] + a[3]);
  }
  __syncthreads();
  for (int w = 1; w < K; w *= 2) {
    // jobs: columns w .. w+cnt-1 = P (= A~^w) times columns 0 .. cnt-1, as
    // (16 columns, 16 rows) tiles; then, unless this is the last doubling,
    // the tiles of P2 = P P (= A~^2w)
    const int cnt = min(w, K - w);
    const int jp = (cnt + 15) / 16 * NT;
    const int js = 2 * w < K ? NT * NT : 0;
    for (int j = wv; j < jp + js; j += PC_NWV) {
      if (j < jp) {
        const int ct = j / NT, it = j % NT;
        const int c = ct * 16 + lr;
        const bool cv = c < cnt;
        const d4_t d = tile_sum<NT>(
            [&](int s) {
              const int k = 4 * s + lk;
              const bool ok = cv && k < n;
              const double x = S.col[ok ? c * ldc + k : 0];
              return ok ? x : 0.0;
            },
            [&](int s) { return P[(4 * s + lk) * LP + it * 16 + lr]; });
        const int i = it * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cc = ct * 16 + 4 * v + lk;
          if (cc < cnt && i < n) S.col[(w + cc) * ldc + i] = d[v];
        }
      } else {
        const int it = (j - jp) % NT, jt = (j - jp) / NT;
        const d4_t d = tile_sum<NT>([&](int s) { return P[(4 * s + lk) * LP + it * 16 + lr]; },
                                    [&](int s) { return P[(jt * 16 + lr) * LP + 4 * s + lk]; });
#pragma unroll
        for (int v = 0; v < 4; ++v) P2[(jt * 16 + lr) * LP + it * 16 + 4 * v + lk] = d[v];
      }
    }
    if (js) {
      double* const tmp = P;
      P = P2;
      P2 = tmp;
    }
    __syncthreads();
  }
  if (t < n) st->cfwd[t] = S.col[(K - 1) * ldc + t];
  double* const sQ = S.M;                            // the powers are done
#pragma unroll
  for (int u = 0; u < PC_NQ; ++u) {
    const int idx = t + u * PC_THREADS;
    if (idx < CMAX * LP) sQ[idx] = rq[u];
  }
  __syncthreads();
  // out column kk = Q c_kk, as (16 columns, 16 rows c) tiles over the rows
  // c < m (rounded up to 16); the rows above are zero
  const int CT = (m + 15) / 16;
  const int jf = (K + 15) / 16 * CT;
  for (int j = wv; j < jf; j += PC_NWV) {
    const int ct = j / CT, jt = j % CT;
    const int kk = ct * 16 + lr;
    const bool kv = kk < K;
    const int cq = jt * 16 + lr;
    const bool qv = cq < CMAX;
    const d4_t d = tile_sum<NT>(
        [&](int s) {
          const int k = 4 * s + lk;
          const bool ok = kv && k < n;
          const double x = S.col[ok ? kk * ldc + k : 0];
          return ok ? x : 0.0;
        },
        [&](int s) {
          const double q = sQ[(qv ? cq : 0) * LP + 4 * s + lk];
          return qv ? q : 0.0;
        });
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int kc = ct * 16 + 4 * v + lk;
      if (kc < K && qv) out[kc * CMAX + cq] = d[v];
    }
  }
  const int c0 = 16 * CT;
  if (c0 < CMAX)
    for (int idx = t; idx < K * (CMAX - c0); idx += PC_THREADS)
      out[(idx / (CMAX - c0)) * CMAX + c0 + idx % (CMAX - c0)] = 0.0;
}

__device__ __forceinline__ void power_entry(DevState* st, int k0, int K, int koff) {
  __shared__ PowerLds S;
  const int n = st->r, m = st->m;
  if (n == 0 || K > coef_chunk(n) || koff + K > COEF_CHUNK) {   // (the host sends neither)
    for (int idx = threadIdx.x; idx < K * CMAX && koff + idx / CMAX < COEF_CHUNK; idx += PC_THREADS)
      st->coefA[koff * CMAX + idx] = 0.0;
    if (threadIdx.x == 0) latch_status(st, n == 0 ? ST_EMPTY : ST_NOCONV);
    return;
  }
  switch ((n + 15) / 16) {
    case 1: power_body<1>(st, S, k0, K, koff, n, m); break;
    case 2: power_body<2>(st, S, k0, K, koff, n, m); break;
    case 3: power_body<3>(st, S, k0, K, koff, n, m); break;
    default: power_body<4>(st, S, k0, K, koff, n, m); break;
  }
}

__global__ __launch_bounds__(PC_THREADS) void k_power_coef(DevState* st, int k0, int K, int koff) {
  power_entry(st, k0, K, koff);
}

// The first chunk (k0 = 0) of several streams: one workgroup per entry of a
// device-resident table of states and step counts.
__global__ __launch_bounds__(PC_THREADS) void k_power_coef_batch(DevState* const* __restrict__ sts,
                                                                 const int* __restrict__ Ks) {
  power_entry(sts[blockIdx.x], 0, Ks[blockIdx.x], 0);
}

// Coefficients that materialise the basis: column k of U is S[:, :m] Q[:, k].
__global__ __launch_bounds__(256) void k_basis_coef(DevState* st) {
  const int m = st->m, r = st->r;
  for (int idx = threadIdx.x; idx < CMAX * RMAX; idx += 256) {
    const int c = idx % CMAX, k = idx / CMAX;
    st->coefA[k * CMAX + c] = (c < m && k < r) ? st->Q[c * RMAX + k] : 0.0;
  }
}

template <bool VECS>
__global__ __launch_bounds__(64) void k_eig(DevState* st) { eig_body<VECS>(st); }

hipError_t launch_eig(DevState* st, bool vectors, hipStream_t s) {
  if (vectors) hipLaunchKernelGGL(k_eig<true>, dim3(1), dim3(64), 0, s, st);
  else hipLaunchKernelGGL(k_eig<false>, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_power_coef(DevState* st, int k0, int steps, int koff, hipStream_t s) {
  hipLaunchKernelGGL(k_power_coef, dim3(1), dim3(PC_THREADS), 0, s, st, k0, steps, koff);
  return hipGetLastError();
}

hipError_t launch_power_coef_batch(DevState* const* sts, const int* steps, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_power_coef_batch, dim3(count), dim3(PC_THREADS), 0, s, sts, steps);
  return hipGetLastError();
}

hipError_t launch_basis_coef(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_coef, dim3(1), dim3(256), 0, s, st);
  return hipGetLastError();
}

}  // namespace odmd
