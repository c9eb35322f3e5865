"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle against mathematics the paper fixes (Sec. 2.3):
closed forms, brute force on tiny inputs, planted truth, invariants and
special cases.  A plausible mistake in the oracle (a dropped term of A~, a
transposed shifted product, a wrong row of W, a sign error in the
projection) fails at least one of them; ``test_planted_mistakes_are_caught``
plants such mistakes and checks that.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def run_online(X, r_max, tol, cls=O.OnlineDMD, **kw):
    o = cls(X.shape[0], r_max, tol, **kw)
    for k in range(X.shape[1] - 1):
        o.update(X[:, k], X[:, k + 1])
    return o


def proj_pinv_operator(X):
    """P_X Y X^+ with X = snapshots 0..m-1, Y = 1..m, P_X the orthogonal
    projector onto range(X), all from pinv (no SVD of our own)."""
    Xm, Y = X[:, :-1], X[:, 1:]
    Xp = np.linalg.pinv(Xm)
    return (Xm @ Xp) @ Y @ Xp


def rel_eig_err(ref, got):
    m = O.match_eigs(ref, got)
    return np.max(np.abs(m - ref) / np.maximum(np.abs(ref), 1e-300))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_golden_closed_forms(case):
    """Hand-derived eigenvalues of tiny exactly-linear systems."""
    X = np.asarray(case["snapshots"], dtype=np.float64).T
    ref = np.asarray(case["eigs_re"]) + 1j * np.asarray(case["eigs_im"])
    tol_eig = 1e-6 if case["name"] == "shear_3d" else 1e-12   # defective: sqrt(eps)
    o = run_online(X, r_max=X.shape[0], tol=1e-12)
    lam, _ = o.eigs()
    assert lam.shape == ref.shape
    assert np.max(np.abs(O.match_eigs(ref, lam) - ref)) < tol_eig
    _, _, Ab = O.batch_dmd(X[:, :-1], X[:, 1:], X.shape[0], 1e-12)
    assert np.max(np.abs(O.match_eigs(ref, np.linalg.eigvals(Ab)) - ref)) < tol_eig


def test_first_update_closed_form():
    """m = 1: U = x/||x||, sigma = ||x||, A~ = x.y / ||x||^2."""
    g = np.random.default_rng(1)
    x, y = g.standard_normal(37), g.standard_normal(37)
    o = O.OnlineDMD(37, 5, 1e-10)
    o.update(x, y)
    assert o.r == 1
    np.testing.assert_allclose(o.sigma[0], np.linalg.norm(x), rtol=1e-15)
    np.testing.assert_allclose(np.abs(o.U[:, 0]), np.abs(x) / np.linalg.norm(x), rtol=1e-14)
    np.testing.assert_allclose(o.atilde()[0, 0], x @ y / (x @ x), rtol=1e-14)


def test_scalar_least_squares_ratio():
    """n = 1: A~ is the least-squares ratio sum x_j y_j / sum x_j^2."""
    g = np.random.default_rng(2)
    X = g.standard_normal((1, 50))
    o = run_online(X, 4, 1e-12)
    x, y = X[0, :-1], X[0, 1:]
    assert o.r == 1
    np.testing.assert_allclose(o.atilde()[0, 0], x @ y / (x @ x), rtol=1e-13)
    np.testing.assert_allclose(o.sigma[0], np.linalg.norm(x), rtol=1e-13)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("n,m", [(40, 12), (200, 30), (512, 64)])
def test_batch_svd_agreement_no_truncation(n, m):
    """Incremental SVD equals the SVD of the full snapshot matrix (rank < r_max)."""
    g = np.random.default_rng(n + m)
    X = g.standard_normal((n, m + 1))
    o = run_online(X, r_max=m + 1, tol=1e-13)
    U, s, _ = np.linalg.svd(X[:, :-1], full_matrices=False)
    assert o.r == m
    np.testing.assert_allclose(o.sigma, s, rtol=1e-12)
    assert O.subspace_angle(o.U, U[:, :m]) < 1e-11
    # projected operator P_X Y X^+ by pseudo-inverse, against U A~ U^T
    A = proj_pinv_operator(X)
    P = o.U @ o.atilde() @ o.U.T
    assert np.max(np.abs(P - A)) < 1e-9 * np.max(np.abs(A))


def test_atilde_definition_from_history():
    """Recursion for C, w, p_y equals A~ = U^T Y W S^-1 and W[2:]^T W[:-1].

    Without truncation the chained-pair recursion is exact (well-conditioned
    random stream, every sigma far above rounding).
    """
    g = np.random.default_rng(11)
    X = g.standard_normal((80, 31))
    o = run_online(X, 40, 1e-12, store_history=True)
    assert o.r == 30
    np.testing.assert_allclose(o.C, o.shifted_product_from_history(), atol=1e-13)
    np.testing.assert_allclose(o.w, o.W[-1], atol=1e-14)
    A1, A2 = o.atilde(), o.atilde_from_history()
    assert np.max(np.abs(A1 - A2)) < 1e-12 * np.max(np.abs(A2))


def test_planted_wake_noise_free_eigs():
    """Noise-free wake stream: rank 21 and the planted spectrum."""
    s = synth.wake(nx=30, ny=20, noise=0.0)
    X = s.snapshots(0, 120)
    o = run_online(X, 30, 1e-10, store_history=True)
    assert o.r == 21
    np.testing.assert_allclose(o.C, o.shifted_product_from_history(), atol=1e-13)
    pl = s.planted_eigs()
    lam = O.match_eigs(pl, np.linalg.eigvals(o.atilde()))
    # decayed transients leave sigma ~ 1e-9 sigma_1: accuracy set by conditioning
    assert np.max(np.abs(lam[:11] - pl[:11])) < 1e-6
    assert np.max(np.abs(lam - pl)) < 1e-3


def test_atilde_recursion_under_noise_truncation():
    """Truncating only noise directions: the recursion's A~ differs from the
    definition by truncation error, which leaves the planted spectrum alone."""
    s = synth.wake(nx=30, ny=20, noise=1e-6)
    X = s.snapshots(0, 150)
    o = run_online(X, 30, 1e-8, store_history=True)
    assert o.r == 30
    np.testing.assert_allclose(o.C, o.shifted_product_from_history(), atol=1e-12)
    np.testing.assert_allclose(o.w, o.W[-1], atol=1e-13)
    pl = s.planted_eigs()[:11]               # mean flow and shedding harmonics
    l1 = O.match_eigs(pl, np.linalg.eigvals(o.atilde()))
    l2 = O.match_eigs(pl, np.linalg.eigvals(o.atilde_from_history()))
    _, _, Ab = O.batch_dmd(X[:, :-1], X[:, 1:], 30, 1e-8)
    l3 = O.match_eigs(pl, np.linalg.eigvals(Ab))
    # all three forms carry the same noise-level bias (~1e-5 on the weakest
    # harmonic at noise 1e-6); none may stray further than that
    assert np.max(np.abs(l1 - l2)) < 2e-5
    assert np.max(np.abs(l1 - pl)) < 5e-5
    assert np.max(np.abs(l1 - pl)) < 3.0 * np.max(np.abs(l3 - pl))


def test_batch_dmd_projection_matches_pinv():
    g = np.random.default_rng(9)
    X = g.standard_normal((60, 21))
    U, s, Ab = O.batch_dmd(X[:, :-1], X[:, 1:], 30, 1e-14)
    A = proj_pinv_operator(X)
    assert np.max(np.abs(U @ Ab @ U.T - A)) < 1e-10 * np.max(np.abs(A))


# ---------------------------------------------------------------- planted truth

def test_planted_small_eigs_rank_rollout():
    """Exact low-rank linear data: rank 6, planted eigenvalues, future states."""
    s = synth.planted_small()
    X = s.snapshots(0, 400)
    o = run_online(X, 20, 1e-8)
    assert o.r == 6
    lam, V = o.eigs()
    assert rel_eig_err(s.planted_eigs(), lam) < 1e-12
    assert np.linalg.norm(o.U.T @ o.U - np.eye(6)) < 1e-12
    pred = o.predict(500)
    fut = s.clean(400, 900).T
    err = np.linalg.norm(pred - fut, axis=1) / np.linalg.norm(fut, axis=1)
    assert err.max() < 1e-10
    # same states through powers of A~
    pw = O.rollout_power(o.U, o.atilde(), o.p_y, 50)
    assert np.max(np.abs(pw - pred[:50])) < 1e-10 * np.max(np.abs(pred[:50]))


def test_planted_wake_leading_eigs_with_noise():
    s = synth.wake(nx=60, ny=40, noise=1e-6)
    X = s.snapshots(0, 300)
    o = run_online(X, 40, 1e-8)
    lam, _ = o.eigs()
    pl = s.planted_eigs()
    m = O.match_eigs(pl, lam)
    # mean flow and shedding harmonics (on the unit circle) to noise level
    assert np.max(np.abs(m[:11] - pl[:11])) < 1e-6
    assert np.linalg.norm(o.U.T @ o.U - np.eye(o.r)) < 1e-12


def test_f1_equals_f2_without_truncation():
    s = synth.planted_small(n=300)
    X = s.snapshots(0, 80)
    a = run_online(X, 20, 1e-10)
    b = run_online(X, 20, 1e-10, cls=O.OnlineDMDF1)
    la, lb = np.linalg.eigvals(a.atilde()), np.linalg.eigvals(b.atilde())
    assert rel_eig_err(la, lb) < 1e-11


def run_pairs(X, Y, r_max, tol, cls=O.OnlineDMDF1):
    o = cls(X.shape[0], r_max, tol)
    for j in range(X.shape[1]):
        o.update(X[:, j], Y[:, j])
    return o


def test_f1_general_pairs_recover_planted_eigs():
    """Unchained pairs of one exact linear map: the spectrum on the planted
    subspace is recovered whatever the pairing (closed form)."""
    s = synth.planted_small(n=300)
    X, Y = synth.restarted_pairs(s, 6, 15, seed=17)
    o = run_pairs(X, Y, 20, 1e-10)
    assert o.r == 6
    assert rel_eig_err(s.planted_eigs(), np.linalg.eigvals(o.atilde())) < 1e-11
    # the chained form refuses these pairs
    with pytest.raises(O.UnchainedPair):
        run_pairs(X, Y, 20, 1e-10, cls=O.OnlineDMD)


@pytest.mark.parametrize("n,m", [(60, 25), (300, 48)])
def test_f1_general_pairs_match_pinv_operator(n, m):
    """Independent random x_j, y_j, no truncation: U A~ U^T equals the
    projected operator P_X Y X^+ formed by pseudo-inverse (brute force)."""
    g = np.random.default_rng(3 * n + m)
    X, Y = g.standard_normal((n, m)), g.standard_normal((n, m))
    o = run_pairs(X, Y, m + 2, 1e-13)
    assert o.r == m
    Xp = np.linalg.pinv(X)
    A = (X @ Xp) @ Y @ Xp
    P = o.U @ o.atilde() @ o.U.T
    assert np.max(np.abs(P - A)) < 1e-10 * np.max(np.abs(A))
    # rollout anchored at the last y: x^_1 = U A~ U^T y_last
    np.testing.assert_allclose(o.predict(1)[0], A @ Y[:, -1], rtol=0, atol=1e-9 * np.max(np.abs(A @ Y[:, -1])))


def test_f1_planted_mistake_is_caught():
    """B rotated with the left factor U_k instead of V_k (a plausible
    transposition) breaks the pseudo-inverse pin."""
    class BadF1(O.OnlineDMDF1):
        def update(self, x, y):
            p, rho, q = O._cgs2(self.U, x, self.tol)
            Uk, s, Vk = O._core_svd(self.sigma, p, rho)
            rn = O._truncation_rank(s, self.r_max, self.tol)
            self.U = np.hstack([self.U, q[:, None]]) @ Uk[:, :rn]
            self.B = np.hstack([self.B, y[:, None]]) @ Uk[:, :rn]
            self.sigma = s[:rn].copy()
            self.p_y = self.U.T @ y

    g = np.random.default_rng(9)
    X, Y = g.standard_normal((60, 25)), g.standard_normal((60, 25))
    o = run_pairs(X, Y, 27, 1e-13, cls=BadF1)
    Xp = np.linalg.pinv(X)
    A = (X @ Xp) @ Y @ Xp
    assert np.max(np.abs(o.U @ o.atilde() @ o.U.T - A)) > 1e-3 * np.max(np.abs(A))


# ---------------------------------------------------------------- invariants

def test_scaling_invariance():
    s = synth.wake(nx=20, ny=20, noise=1e-6)
    X = s.snapshots(0, 60)
    a = run_online(X, 12, 1e-8)
    b = run_online(3.5 * X, 12, 1e-8)
    np.testing.assert_allclose(b.sigma, 3.5 * a.sigma, rtol=1e-10)
    assert rel_eig_err(np.linalg.eigvals(a.atilde()), np.linalg.eigvals(b.atilde())) < 1e-9


def test_row_permutation_and_sign_invariance():
    s = synth.wake(nx=20, ny=20, noise=1e-6)
    X = s.snapshots(0, 60)
    g = np.random.default_rng(3)
    perm = g.permutation(X.shape[0])
    sign = np.where(g.random(X.shape[0]) < 0.5, -1.0, 1.0)
    a = run_online(X, 12, 1e-8)
    b = run_online(sign[:, None] * X[perm], 12, 1e-8)
    np.testing.assert_allclose(b.sigma, a.sigma, rtol=1e-10)
    assert rel_eig_err(np.linalg.eigvals(a.atilde()), np.linalg.eigvals(b.atilde())) < 1e-9


# ---------------------------------------------------------------- special cases

def test_orthogonal_new_direction_appends_sigma():
    """x orthogonal to span(U): K is diagonal and sigma' = sigma U {||x||}."""
    n = 10
    E = np.eye(n)
    o = O.OnlineDMD(n, 5, 1e-12)
    o.update(3.0 * E[:, 0], 2.0 * E[:, 1])
    o.update(2.0 * E[:, 1], 1.0 * E[:, 2])
    np.testing.assert_allclose(o.sigma, [3.0, 2.0], rtol=1e-15)
    o.update(1.0 * E[:, 2], 0.5 * E[:, 3])
    np.testing.assert_allclose(o.sigma, [3.0, 2.0, 1.0], rtol=1e-15)


def test_in_span_keeps_rank_and_zero_vector():
    """x in span(U): rank unchanged; x = 0: no growth, sigma unchanged, w = 0."""
    n = 8
    E = np.eye(n)
    o = O.OnlineDMD(n, 5, 1e-10)
    o.update(E[:, 0], E[:, 1])
    o.update(E[:, 1], E[:, 0] + E[:, 1])
    r0 = o.r
    o.update(E[:, 0] + E[:, 1], np.zeros(n))
    assert o.r == r0
    s0 = o.sigma.copy()
    o.update(np.zeros(n), np.zeros(n))
    assert o.r == r0
    np.testing.assert_allclose(o.sigma, s0, rtol=1e-15)
    assert np.all(o.w == 0.0)


def test_zero_first_snapshot_stays_empty():
    o = O.OnlineDMD(6, 3, 1e-8)
    o.update(np.zeros(6), np.ones(6))
    assert o.r == 0


def test_rank_capped_by_n():
    g = np.random.default_rng(4)
    X = g.standard_normal((3, 30))
    o = run_online(X, 10, 1e-12)
    assert o.r == 3
    A = X[:, 1:] @ np.linalg.pinv(X[:, :-1])      # X spans R^3: no projection
    assert np.max(np.abs(o.U @ o.atilde() @ o.U.T - A)) < 1e-10 * np.max(np.abs(A))


def test_errors():
    o = O.OnlineDMD(4, 2, 1e-8)
    with pytest.raises(O.NonFiniteInput):
        o.update(np.array([1.0, np.nan, 0, 0]), np.ones(4))
    o.update(np.ones(4), np.arange(4.0))
    with pytest.raises(O.UnchainedPair):
        o.update(np.ones(4), np.ones(4))
    with pytest.raises(ValueError):
        O.OnlineDMD(0, 2, 1e-8)


# ---------------------------------------------------------------- eig / rollout

def test_eig_sorted_known_spectrum():
    """Block-diagonal rotation-scaling blocks plus reals, hidden by a similarity."""
    g = np.random.default_rng(5)
    ref = []
    D = np.zeros((7, 7))
    for i, (rad, th) in enumerate([(0.9, 0.3), (0.5, 1.1)]):
        c, s_ = rad * np.cos(th), rad * np.sin(th)
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[c, -s_], [s_, c]]
        ref += [rad * np.exp(1j * th), rad * np.exp(-1j * th)]
    for i, v in enumerate([1.0, -0.7, 0.2]):
        D[4 + i, 4 + i] = v
        ref.append(v)
    S = g.standard_normal((7, 7))
    A = S @ D @ np.linalg.inv(S)
    lam, V = O.eig_sorted(A)
    assert rel_eig_err(np.asarray(ref), lam) < 1e-12
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, rtol=1e-14)
    assert np.max(np.abs(A @ V - V * lam[None, :])) < 1e-12
    assert np.all(np.diff(np.abs(lam)) <= 1e-15)


# ---------------------------------------------------------------- properties

@settings(max_examples=25, deadline=None)
@given(n=st.integers(2, 40), m=st.integers(1, 15), seed=st.integers(0, 10_000))
def test_property_matches_batch_when_not_truncated(n, m, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, m + 1))
    o = run_online(X, r_max=64, tol=1e-12)
    s = np.linalg.svd(X[:, :-1], compute_uv=False)
    k = min(n, m)
    assert o.r == k
    np.testing.assert_allclose(o.sigma, s[:k], rtol=1e-10)
    assert np.linalg.norm(o.U.T @ o.U - np.eye(k)) < 1e-12
    A = proj_pinv_operator(X)
    assert np.max(np.abs(o.U @ o.atilde() @ o.U.T - A)) < 1e-8 * max(1.0, np.max(np.abs(A)))


# ---------------------------------------------------------------- self-test of the pins

def test_planted_mistakes_are_caught(monkeypatch):
    """Plant plausible mistakes in the oracle; each must break the 1e-12
    planted-eigenvalue pin by orders of magnitude."""
    s = synth.planted_small(n=200)
    X = s.snapshots(0, 120)

    def planted_error(atilde):
        monkeypatch.setattr(O.OnlineDMD, "atilde", atilde)
        o = run_online(X, 20, 1e-8)
        err = rel_eig_err(s.planted_eigs(), np.linalg.eigvals(o.atilde()))
        monkeypatch.undo()
        return err

    good = planted_error(O.OnlineDMD.atilde)
    assert good < 1e-12
    # dropped p_y w^T term
    assert planted_error(lambda o: o.sigma[:, None] * o.C / o.sigma[None, :]) > 1e-9
    # transposed shifted product
    assert planted_error(lambda o: (o.sigma[:, None] * o.C.T + np.outer(o.p_y, o.w))
                         / o.sigma[None, :]) > 1e-9
    # sigma on the wrong side
    assert planted_error(lambda o: (o.sigma[None, :] * o.C + np.outer(o.p_y, o.w))
                         / o.sigma[:, None]) > 1e-9


def test_planted_mistakes_in_update_are_caught(monkeypatch):
    s = synth.planted_small(n=200)
    X = s.snapshots(0, 120)
    good_cgs2, good_state = O._cgs2, O._shifted_product_update

    def bad_cgs2(U, x, tol):                 # sign error in the first projection
        p1 = U.T @ x
        e1 = x + U @ p1
        p2 = U.T @ e1
        e = e1 - U @ p2
        rho = float(np.linalg.norm(e))
        if rho > tol * np.linalg.norm(x):
            return p1 + p2, rho, e / rho
        return p1 + p2, 0.0, np.zeros_like(x)

    def bad_state(C, w, Vk, rn):             # first row of V_k taken as the new w
        Cn, _ = good_state(C, w, Vk, rn)
        return Cn, Vk[0, :rn].copy()

    for bad, name in [(bad_cgs2, "_cgs2"), (bad_state, "_shifted_product_update")]:
        monkeypatch.setattr(O, name, bad)
        o = run_online(X, 20, 1e-8)
        monkeypatch.undo()
        assert rel_eig_err(s.planted_eigs(), np.linalg.eigvals(o.atilde())) > 1e-9 \
            or o.r != 6


# ---------------------------------------------------------------- principal angles

def _axis_pair(theta):
    """span{e1, e2} against span{e1, cos(theta) e2 + sin(theta) e3} in R^4:
    principal angles 0 and theta, exactly representable bases."""
    A = np.zeros((4, 2))
    A[0, 0] = A[1, 1] = 1.0
    B = np.zeros((4, 2))
    B[0, 0] = 1.0
    B[1, 1], B[2, 1] = np.cos(theta), np.sin(theta)
    return A, B


def _embedded_pair(thetas, n=40, seed=7):
    """Two k-dimensional subspaces of R^n at the principal angles ``thetas``
    (Bjorck-Golub canonical form rotated by a random orthogonal matrix),
    each given by a non-orthonormal basis (a random well-conditioned right
    factor), so the function must orthonormalise before measuring."""
    g = np.random.Generator(np.random.PCG64(seed))
    k = len(thetas)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    c, s = np.cos(thetas), np.sin(thetas)
    A = Q[:, :k]
    B = Q[:, :k] * c[None, :] + Q[:, k:2 * k] * s[None, :]
    MA = np.eye(k) + 0.3 * g.standard_normal((k, k)) / np.sqrt(k)
    MB = np.eye(k) + 0.3 * g.standard_normal((k, k)) / np.sqrt(k)
    return A @ MA, B @ MB


@pytest.mark.parametrize("theta", [1e-9, 1e-4, 1e-3, 0.7, np.pi / 2 - 1e-6])
def test_subspace_angle_known_angle(theta):
    """The largest principal angle of an exactly known pair, to 1e-12
    relative at every scale from 1e-9 rad to pi/2 - 1e-6."""
    A, B = _axis_pair(theta)
    assert abs(O.subspace_angle(A, B) - theta) <= 1e-12 * theta
    assert abs(O.subspace_angle(B, A) - theta) <= 1e-12 * theta


def test_subspace_angle_several_angles_and_basis_invariance():
    """Several nonzero angles: the largest one is returned (not the smallest,
    not a norm over all of them), whatever bases span the two subspaces."""
    for thetas in ([0.3, 0.5, 0.1], [1e-6, 2e-6, 5e-7], [1.2, 0.0, 0.4, 1.5]):
        A, B = _embedded_pair(np.asarray(thetas))
        got = O.subspace_angle(A, B)
        assert abs(got - max(thetas)) <= 1e-12 * max(thetas) + 1e-14, (thetas, got)
    A, _ = _embedded_pair(np.array([0.2, 0.3]))
    assert O.subspace_angle(A, A @ np.array([[2.0, 1.0], [0.0, 3.0]])) <= 1e-14
    # a direction of span(B) outside span(A) when B is larger: pi/2
    A, _ = _axis_pair(0.0)
    assert abs(O.subspace_angle(A[:, :1], A) - np.pi / 2) <= 1e-15


def test_subspace_angle_planted_mistakes_are_caught(monkeypatch):
    """Plausible wrong versions of the function fail the pins above."""
    def cosine_form(A, B):
        qa, _ = np.linalg.qr(A)
        qb, _ = np.linalg.qr(B)
        c = np.linalg.svd(qa.T @ qb, compute_uv=False)
        return float(np.arccos(min(1.0, np.min(c))))

    def frobenius_sine(A, B):
        qa, _ = np.linalg.qr(A)
        qb, _ = np.linalg.qr(B)
        return float(np.arcsin(min(1.0, np.linalg.norm(qb - qa @ (qa.T @ qb)))))

    def smallest_angle(A, B):
        qa, _ = np.linalg.qr(A)
        qb, _ = np.linalg.qr(B)
        c = np.linalg.svd(qa.T @ qb, compute_uv=False)
        s = np.sqrt(np.maximum(0.0, 1.0 - c ** 2))
        return float(np.arctan2(np.min(s), np.max(c)))

    def no_orthonormalisation(A, B):
        s = np.linalg.norm(B - A @ (A.T @ B), 2)
        c = np.linalg.svd(A.T @ B, compute_uv=False)
        return float(np.arctan2(s, np.min(c)))

    for bad in (cosine_form, frobenius_sine, smallest_angle, no_orthonormalisation,
                lambda A, B: 0.0):
        monkeypatch.setattr(O, "subspace_angle", bad)
        failed = False
        for theta in (1e-9, 1e-4, 0.7, np.pi / 2 - 1e-6):
            A, B = _axis_pair(theta)
            failed |= abs(O.subspace_angle(A, B) - theta) > 1e-12 * theta
        for thetas in ([0.3, 0.5, 0.1], [1.2, 0.0, 0.4, 1.5]):
            A, B = _embedded_pair(np.asarray(thetas))
            failed |= abs(O.subspace_angle(A, B) - max(thetas)) > 1e-12 * max(thetas) + 1e-14
        monkeypatch.undo()
        assert failed, bad


def _jordan_stream(n=1500, steps=41, seed=29):
    """x_k = P M^k c with M = diag(J, 0.99 R(0.3)), J = [[0.97, 1], [0, 0.97]]
    (a Jordan block: the operator on span P has no full set of
    eigenvectors)."""
    g = np.random.default_rng(seed)
    P = g.standard_normal((n, 4)) / np.sqrt(n)
    M = np.zeros((4, 4))
    M[:2, :2] = [[0.97, 1.0], [0.0, 0.97]]
    c, s = np.cos(0.3), np.sin(0.3)
    M[2:, 2:] = 0.99 * np.array([[c, -s], [s, c]])
    z = np.array([1.0, 1.0, 1.0, 0.5])
    X = np.empty((n, steps + 60))
    for k in range(steps + 60):
        X[:, k] = P @ z
        z = M @ z
    return X[:, :steps], X[:, steps:]


def test_power_rollout_on_a_defective_operator():
    """Where A~ has no full set of eigenvectors the eigenvector form of the
    prediction loses accuracy (V nearly singular), while U A~^k U^T x_a is
    still the exact continuation of linear data: rollout_power matches the
    true future states to 1e-10."""
    X, fut = _jordan_stream()
    o = run_online(X, 8, 1e-10)
    assert o.r == 4
    _, V = np.linalg.eig(o.atilde())
    assert np.linalg.cond(V) > 1e5                     # numerically defective
    pw = O.rollout_power(o.U, o.atilde(), o.p_y, 60)
    err = np.linalg.norm(pw - fut.T, axis=1) / np.linalg.norm(fut, axis=0).max()
    assert err.max() < 1e-10
