// Internal layout shared by the HIP kernels and the host runtime.
//
// Per stream the device holds:
//   Us  stored basis, column-major, column j at Us + j*ld (ld = n rounded up
//       to 64 elements), storage type TS (double or float);
//   Es  stored residual e of the last pass (n elements of TS);
//   partials  per-workgroup partial sums of the streaming pass;
//   DevState  the small FP64 state below.
//
// The logical basis U (the paper's L, Sec. 2.3) is either Us[:, :r] or, when
// a rotation is pending, Us G + Es g^T: the rotation of an update is applied
// lazily by the next streaming pass (or folded into prediction coefficients),
// so every update reads and writes the basis once.
#pragma once
#include <stdint.h>

namespace odmd {

constexpr int RMAX = 64;          // rank cap
constexpr int MMAX = RMAX + 1;    // core size (r + 1)
constexpr int PW = 2 * RMAX + 6;  // partial-sum record per workgroup
constexpr int PASS_THREADS = 256;
constexpr int PASS_MAX_BLOCKS = 512;
constexpr int CORE_THREADS = 1024;
constexpr int COEF_CHUNK = 512;   // prediction steps per coefficient chunk

// partial-sum record layout (doubles)
constexpr int P_SUE = 0;             // Us^T e        [0, RMAX)
constexpr int P_SEE = RMAX;          // Es . e
constexpr int P_EE = RMAX + 1;       // e . e
constexpr int P_XX = RMAX + 2;       // x . x
constexpr int P_SUY = RMAX + 3;      // Us^T y        [RMAX+3, 2RMAX+3)
constexpr int P_SEY = 2 * RMAX + 3;  // Es . y
constexpr int P_EY = 2 * RMAX + 4;   // e . y
constexpr int P_YY = 2 * RMAX + 5;   // y . y

// latched status bits
constexpr int ST_NONFINITE = 1;
constexpr int ST_SEQ = 2;
constexpr int ST_NOCONV = 4;
constexpr int ST_EMPTY = 8;

struct DevState {
  // scalars (int block first, then doubles)
  int r;          // logical rank
  int rs;         // columns of Us that the logical basis is built from
  int pending;    // 1: U = Us G + Es g^T ; 0: U = Us[:, :r]
  int use_e;      // pending and g != 0 (Es enters the basis)
  int status;     // latched error bits
  int sweeps;     // Jacobi sweeps of the last core SVD
  int eig_valid;  // eigen cache belongs to the current model
  int eig_status; // 0 ok, else iteration cap hit
  long long m;    // accepted pairs
  double tol;     // effective tolerance
  double yy_prev; // y.y of the last accepted pair (chaining fingerprint)
  double last_rho;
  double beta;    // g . p1 for the next pass
  double pad_[3];
  // vectors and matrices; matrices column-major with leading dim RMAX
  double sigma[RMAX];
  double w[RMAX];
  double py[RMAX];      // U^T y_last: cached projection of the next x
  double a[RMAX];       // G p1 for the next pass (length rs)
  double g[RMAX];       // length r
  double G[RMAX * RMAX];      // rs x r: G[j + k*RMAX]
  float G32[RMAX * RMAX];     // FP32 copy for FP32 storage
  float g32[RMAX];
  double C[RMAX * RMAX];      // r x r shifted product W[2:]^T W[:-1]
  double At[RMAX * RMAX];     // A~ (r x r)
  // eigen cache
  double lam_re[RMAX], lam_im[RMAX];
  double V_re[RMAX * RMAX], V_im[RMAX * RMAX];
  // prediction coefficients of one chunk: rows j < rs, columns steps
  double coefA[RMAX * COEF_CHUNK];
  double coefB[COEF_CHUNK];
  double bt_re[RMAX], bt_im[RMAX];   // b~ = V^-1 p_y
};

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace odmd
