"""Plain FP64 CPU oracle for online DMD -- TEST INFRASTRUCTURE ONLY.

This module is the correctness reference for the GPU library.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does, and it shares no code with the HIP
implementation (it imports nothing from the package).

What it computes (Sec. 2.3 of the paper, "Online DMD"):

* the DMD matrix A = U+ (U-)^+ ~ U+ R S^-1 L^* from the truncated SVD
  U- = L S R^* of the input snapshot matrix;
* the reduced operator  A~ = L^* U+ R S^-1  (r x r);
* its eigendecomposition A~ = V Lambda V^-1 and the projected modes
  Phi = L V;
* the prediction u(t) = Phi Lambda^(t/dt) Phi^+ u(0);
* the online form: one snapshot pair appended per step, with the SVD of the
  snapshot matrix updated by Brand's rank-1 column append (the paper keeps
  to Brand's original algorithm, reference [brand2006fast]).

Notation used below (the paper's symbols in brackets): x_j, y_j = x_{j+1}
are the columns of X [U-] and Y [U+]; U [L] is the n x r left basis, sigma
[diag S] the singular values, W [R] the right singular vectors (m x r,
never stored by the online method).

Readings where the paper is silent (each listed in the design notes):
  * rank choice: r' = min(r_max, #{sigma'_i > tol * sigma'_1});
  * rank growth: a new direction is kept only if rho > tol * ||x||, else the
    update is rank-preserving (rho = 0, q = 0);
  * the shifted-product bookkeeping for chained pairs (y_j = x_{j+1}):
    C = W[2:m]^T W[1:m-1], w = W[m, :], p_y = U^T y_m, from which
    A~_ij = (sigma_i C_ij + p_y,i w_j) / sigma_j;
  * prediction anchor: the last y seen, b = V^-1 U^T y_last, output rows are
    the states a+1 .. a+steps.

Every function here is written for clarity, not speed: textbook CGS2 with
explicit passes, LAPACK (numpy.linalg) for the small SVD and eigenproblem.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "OnlineDMD", "OnlineDMDF1", "batch_dmd", "eig_sorted", "rollout",
    "rollout_power", "NonFiniteInput", "UnchainedPair", "subspace_angle",
    "match_eigs",
]


class NonFiniteInput(ValueError):
    """A snapshot holds NaN or Inf; the state is left unchanged."""


class UnchainedPair(ValueError):
    """x_k is not the y of the previous accepted pair (chained form only)."""


def _cgs2(U: np.ndarray, x: np.ndarray, tol: float):
    """Classical Gram-Schmidt with one reorthogonalisation pass.

    Returns the coefficients p = U^T x (two passes summed), the norm rho of
    the part of x outside span(U), and the unit direction q of that part.
    The direction is kept only if rho > tol * ||x||; otherwise the update is
    rank-preserving and rho = 0, q = 0.
    """
    p1 = U.T @ x
    e1 = x - U @ p1
    p2 = U.T @ e1
    e = e1 - U @ p2
    rho = float(np.linalg.norm(e))
    if rho > tol * np.linalg.norm(x) and rho > 0.0:
        return p1 + p2, rho, e / rho
    return p1 + p2, 0.0, np.zeros_like(x)


def _core_svd(sigma: np.ndarray, p: np.ndarray, rho: float):
    """SVD of the (r+1) x (r+1) core K = [[diag(sigma), p], [0, rho]].

    Brand's column append: [U S W^T, x] = [U q] K blockdiag(W, 1)^T, so the
    SVD of the small K gives the update of all three factors.  numpy returns
    singular values in descending order.
    """
    r = sigma.shape[0]
    K = np.zeros((r + 1, r + 1))
    K[:r, :r] = np.diag(sigma)
    K[:r, r] = p
    K[r, r] = rho
    Uk, s, VkT = np.linalg.svd(K)
    return Uk, s, VkT.T


def _truncation_rank(s: np.ndarray, r_max: int, tol: float) -> int:
    if s.size == 0 or not s[0] > 0.0:
        return 0
    return int(min(r_max, np.count_nonzero(s > tol * s[0])))


def _shifted_product_update(C: np.ndarray, w: np.ndarray, Vk: np.ndarray, rn: int):
    """New C = W'[2:]^T W'[:-1] and w = last row of W' for W' = blockdiag(W, 1) V_k.

    The shifted product of the extended factor blockdiag(W, 1), rows 2..m+1
    against rows 1..m, is [[C, 0], [w^T, 0]]; the new last row of W' is the
    last row of V_k.  Both are then cut to the kept rank.
    """
    r = C.shape[0]
    E = np.zeros((r + 1, r + 1))
    E[:r, :r] = C
    E[r, :r] = w
    return (Vk.T @ E @ Vk)[:rn, :rn], Vk[r, :rn].copy()


class OnlineDMD:
    """Online DMD by rank-1 column appends, chained pairs (y_j = x_{j+1}).

    Parameters follow the library's create call: state dimension n, rank
    cap r_max, relative tolerance tol (used for both the rank-growth test
    and the truncation).  With ``store_history`` the oracle also keeps W and
    Y so that C and A~ can be checked against their definitions.
    """

    def __init__(self, n: int, r_max: int, tol: float, store_history: bool = False):
        if n < 1 or r_max < 1 or not (0.0 <= tol < 1.0):
            raise ValueError("bad arguments")
        self.n, self.r_max, self.tol = int(n), int(r_max), float(tol)
        self.U = np.zeros((self.n, 0))
        self.sigma = np.zeros(0)
        self.C = np.zeros((0, 0))
        self.w = np.zeros(0)
        self.p_y = np.zeros(0)
        self.m = 0                       # accepted pairs
        self.y_last = None
        self.store_history = store_history
        self.W = np.zeros((0, 0))
        self.Y = []
        self.last_rho = 0.0

    @property
    def r(self) -> int:
        return self.sigma.shape[0]

    def update(self, x: np.ndarray, y: np.ndarray) -> None:
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        y = np.asarray(y, dtype=np.float64).reshape(-1)
        if x.shape[0] != self.n or y.shape[0] != self.n:
            raise ValueError("snapshot length")
        if not (np.all(np.isfinite(x)) and np.all(np.isfinite(y))):
            raise NonFiniteInput("non-finite snapshot")
        if self.y_last is not None and not np.array_equal(x, self.y_last):
            raise UnchainedPair("x_k differs from the previous x_k+1")

        U, r = self.U, self.r
        p, rho, q = _cgs2(U, x, self.tol)
        self.last_rho = rho

        Uk, s, Vk = _core_svd(self.sigma, p, rho)
        rn = _truncation_rank(s, self.r_max, self.tol)

        Cn, wn = _shifted_product_update(self.C, self.w, Vk, rn)

        Un = np.hstack([U, q[:, None]]) @ Uk[:, :rn]
        self.U = Un
        self.sigma = s[:rn].copy()
        self.C = Cn
        self.w = wn
        self.p_y = Un.T @ y              # plain definition, one explicit pass
        self.m += 1
        self.y_last = y.copy()
        if self.store_history:
            Wext = np.zeros((self.W.shape[0] + 1, r + 1))
            Wext[:-1, :r] = self.W
            Wext[-1, r] = 1.0
            self.W = (Wext @ Vk)[:, :rn]
            self.Y.append(y.copy())

    def atilde(self) -> np.ndarray:
        """A~_ij = (sigma_i C_ij + p_y,i w_j) / sigma_j  (chained-pair form)."""
        s = self.sigma
        return (s[:, None] * self.C + np.outer(self.p_y, self.w)) / s[None, :]

    def atilde_from_history(self) -> np.ndarray:
        """A~ = U^T Y W S^-1 straight from the stored Y and W (Sec. 2.3)."""
        if not self.store_history:
            raise RuntimeError("history not stored")
        Y = np.stack(self.Y, axis=1)
        return self.U.T @ Y @ self.W / self.sigma[None, :]

    def shifted_product_from_history(self) -> np.ndarray:
        """W[2:m]^T W[1:m-1] from the stored W (the C the recursion keeps)."""
        return self.W[1:].T @ self.W[:-1]

    def eigs(self):
        return eig_sorted(self.atilde())

    def predict(self, steps: int) -> np.ndarray:
        """States x_{a+1} .. x_{a+steps} (rows), anchored at the last y."""
        lam, V = self.eigs()
        return rollout(self.U, V, lam, self.p_y, steps)


class OnlineDMDF1:
    """Online DMD for general (not necessarily chained) pairs.

    Keeps B = Y W (n x r) instead of the shifted product C, and forms
    A~ = U^T B S^-1 straight from the definition; B follows the right factor
    through B <- ([B y] V_k)[:, :r'].  The left factor, sigma and the
    rank rules are those of the chained form; p_y = U^T y of the last pair
    anchors the rollout.
    """

    def __init__(self, n: int, r_max: int, tol: float):
        self.n, self.r_max, self.tol = int(n), int(r_max), float(tol)
        self.U = np.zeros((self.n, 0))
        self.B = np.zeros((self.n, 0))
        self.sigma = np.zeros(0)
        self.p_y = np.zeros(0)

    @property
    def r(self) -> int:
        return self.sigma.shape[0]

    def update(self, x, y) -> None:
        x = np.asarray(x, dtype=np.float64).reshape(-1)
        y = np.asarray(y, dtype=np.float64).reshape(-1)
        if not (np.all(np.isfinite(x)) and np.all(np.isfinite(y))):
            raise NonFiniteInput("non-finite snapshot")
        p, rho, q = _cgs2(self.U, x, self.tol)
        Uk, s, Vk = _core_svd(self.sigma, p, rho)
        rn = _truncation_rank(s, self.r_max, self.tol)
        self.U = np.hstack([self.U, q[:, None]]) @ Uk[:, :rn]
        self.B = np.hstack([self.B, y[:, None]]) @ Vk[:, :rn]
        self.sigma = s[:rn].copy()
        self.p_y = self.U.T @ y

    def atilde(self) -> np.ndarray:
        """A~ = U^T B S^-1 = U^T Y W S^-1 (Sec. 2.3), B = Y W."""
        return (self.U.T @ self.B) / self.sigma[None, :]

    def eigs(self):
        return eig_sorted(self.atilde())

    def predict(self, steps: int) -> np.ndarray:
        """States after the last y seen, as for chained pairs."""
        lam, V = self.eigs()
        return rollout(self.U, V, lam, self.p_y, steps)


def batch_dmd(X: np.ndarray, Y: np.ndarray, r_max: int, tol: float):
    """Exact DMD from all snapshots at once (the O(N n r) route).

    X = U S W^T (thin SVD), truncated at r = min(r_max, #{s_i > tol s_1});
    A~ = U^T Y W S^-1.  Returns (U, s, A~).
    """
    U, s, WT = np.linalg.svd(X, full_matrices=False)
    r = _truncation_rank(s, r_max, tol)
    U, s, W = U[:, :r], s[:r], WT[:r].T
    return U, s, U.T @ Y @ W / s[None, :]


def eig_sorted(A: np.ndarray):
    """Eigenpairs of A (LAPACK dgeev through numpy).

    Columns of V have unit 2-norm; each column's largest-modulus entry is
    made real and positive.  Order: |lambda| descending, then Im descending.
    """
    lam, V = np.linalg.eig(A)
    lam = lam.astype(np.complex128)
    V = V.astype(np.complex128)
    for j in range(V.shape[1]):
        v = V[:, j] / np.linalg.norm(V[:, j])
        k = int(np.argmax(np.abs(v)))
        V[:, j] = v * (np.conj(v[k]) / abs(v[k]))
    order = np.lexsort((-lam.imag, -np.abs(lam)))
    return lam[order], V[:, order]


def rollout(U, V, lam, p_y, steps: int) -> np.ndarray:
    """x^_{a+k} = Re(U V Lambda^k b), b = V^-1 p_y, k = 1..steps.

    Returns a (steps, n) array.  This is u(t) = Phi Lambda^(t/dt) Phi^+ u(0)
    with Phi = U V and u(0) the anchor whose projection is p_y
    (Phi^+ u(0) = V^-1 U^T u(0) because U has orthonormal columns).
    """
    b = np.linalg.solve(V, p_y.astype(np.complex128))
    k = np.arange(1, steps + 1)
    coeff = (lam[None, :] ** k[:, None]) * b[None, :]      # (steps, r)
    return np.real(coeff @ V.T @ U.T)


def rollout_power(U, A, p_y, steps: int) -> np.ndarray:
    """Same states through powers of A~: x^_{a+k} = U A~^k U^T u(0)."""
    out = np.empty((steps, U.shape[0]))
    c = p_y.copy()
    for k in range(steps):
        c = A @ c
        out[k] = U @ c
    return out


def subspace_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle (radians) between span(A) and span(B).

    With orthonormal bases Qa, Qb (thin QR), the principal angles theta_i
    have cosines = singular values of Qa^T Qb and sines = singular values of
    (I - Qa Qa^T) Qb (Bjorck and Golub, 1973).  The largest angle is taken
    as atan2(largest sine, smallest cosine): the sine alone loses accuracy
    near pi/2 and the cosine alone near 0, the pair is accurate at both ends.
    If B has more columns than A, some direction of span(B) lies outside
    span(A) and the smallest cosine is 0.
    """
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    s_max = float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))
    cos = np.linalg.svd(qa.T @ qb, compute_uv=False)
    c_min = 0.0 if qb.shape[1] > qa.shape[1] else float(np.min(cos))
    return float(np.arctan2(s_max, c_min))


def match_eigs(ref: np.ndarray, got: np.ndarray) -> np.ndarray:
    """Greedy nearest matching; returns got reordered to pair with ref."""
    got = list(got)
    out = []
    for z in ref:
        k = int(np.argmin([abs(z - g) for g in got]))
        out.append(got.pop(k))
    return np.asarray(out)
