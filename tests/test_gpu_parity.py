"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Inputs come from the seeded generators in paper_2311_18715_amd.synth and
feed both sides.  Tolerances (FP64 path): eigenvalues 1e-10 relative
(eigenvalues with |lambda| >= 1e-2 max|lambda|), singular values 1e-11
relative, orthogonality ||U^T U - I||_F <= 1e-12, rollouts 1e-9 relative.
"""
import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import ODMD, OdmdError


def dev(X, dtype=None):
    """Snapshots as rows of a device tensor: row k is x_k."""
    return torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dtype or torch.float64)


def run_both(X, r_max, tol, steps=None, basis="f64", check_every=0):
    m = X.shape[1] - 1 if steps is None else steps
    g = ODMD(X.shape[0], r_max, tol, basis=basis)
    o = O.OnlineDMD(X.shape[0], r_max, g.info().tol_eff)
    Xd = dev(X, torch.float64 if basis == "f64" else torch.float32)
    Xo = X if basis == "f64" else Xd.double().cpu().numpy().T
    for k in range(m):
        g.update(Xd[k], Xd[k + 1])
        o.update(Xo[:, k], Xo[:, k + 1])
        if check_every and (k % check_every == 0 or k == m - 1):
            s = g.state()
            assert s["r"] == o.r, f"rank differs at step {k}"
            np.testing.assert_allclose(s["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    g.sync()
    return g, o


def rel_eig_err(ref, got, floor=1e-2):
    big = np.abs(ref) >= floor * np.abs(ref).max()
    m = O.match_eigs(ref[big], got)
    return np.max(np.abs(m - ref[big]) / np.abs(ref[big]))


def orth_err(g):
    U = g.basis_matrix()
    return torch.linalg.norm(U.T @ U - torch.eye(U.shape[1], dtype=U.dtype, device=U.device)).item()


@pytest.fixture(params=["secular", "jacobi"])
def core_svd(request, monkeypatch):
    """Run a test with each small-SVD solver of the core."""
    if request.param == "jacobi":
        monkeypatch.setenv("ODMD_CORE_SVD", "jacobi")
    else:
        monkeypatch.delenv("ODMD_CORE_SVD", raising=False)
    return request.param


def test_planted_small_every_step(core_svd):
    """n=4096, rank 6, r_max 20, tol 1e-8, 399 pairs: rank and sigma each step."""
    s = synth.planted_small()
    X = s.snapshots(0, 400)
    g, o = run_both(X, 20, 1e-8, check_every=1)
    assert g.info().r == 6
    lam, V = g.eigs()
    lo, Vo = o.eigs()
    assert rel_eig_err(lo, lam) < 1e-10
    assert rel_eig_err(s.planted_eigs(), lam) < 1e-10
    # eigenvectors: unit norm, A~ V = V Lambda with the GPU's own A~
    st = g.state()
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, rtol=1e-12)
    assert np.max(np.abs(st["atilde"] @ V - V * lam[None, :])) < 1e-10
    assert orth_err(g) < 1e-12
    # U A~ U^T is basis-independent: compare on random probes
    U = g.basis_matrix().cpu().numpy()
    P = np.random.default_rng(0).standard_normal((X.shape[0], 4))
    Pg = U @ (st["atilde"] @ (U.T @ P))
    Po = o.U @ (o.atilde() @ (o.U.T @ P))
    assert np.max(np.abs(Pg - Po)) < 1e-10 * np.max(np.abs(Po))


@pytest.mark.parametrize("steps", [1, 4, 5, 16, 17, 129, 1100])
def test_rollout_lengths_against_the_oracle(steps):
    """Rollouts of every length class of the read-out: a few states (one
    row per lane), one to eight 16-state blocks, several 128-state blocks,
    and more states than one coefficient chunk (512 at this rank cap), with
    the coefficients' serial start (up to 16 steps) and doubling: each state within
    1e-9 of the oracle's, relative to the largest state (the planted modes
    decay: the last of 1100 states is 1e-9 of the first), on a ragged n."""
    s = synth.random_planted(3001, 6, seed=913, noise=1e-9)
    X = s.snapshots(0, 61)
    g, o = run_both(X, 12, 1e-8)
    pg = g.predict(steps).cpu().numpy()
    po = o.predict(steps)
    assert pg.shape == po.shape == (steps, 3001)
    err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1).max()
    assert err.max() < 1e-9


@pytest.mark.parametrize("r_max,steps", [(24, 50), (40, 600), (64, 400)])
def test_rollout_chunks_of_higher_ranks_against_the_oracle(r_max, steps):
    """The prediction's coefficients are formed as powers of A~ applied to
    U^T x_a, a chunk of steps at a time whose length falls with the rank cap
    (r_max 40: 272 steps, 64: 160): a noisy wake stream at ranks 24, 40 and
    64 (two to four 16-row tiles), rollouts across two and three chunks,
    each state within 1e-9 of the oracle's eigenvector-form rollout relative
    to the largest state, on a ragged n."""
    s = synth.wake(nx=61, ny=39, noise=1e-6)
    X = s.snapshots(0, 200)
    g, o = run_both(X, r_max, 1e-8)
    assert g.info().r == o.r == r_max
    pg = g.predict(steps).cpu().numpy()
    po = o.predict(steps)
    err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1).max()
    assert err.max() < 1e-9


def test_planted_small_rollout():
    s = synth.planted_small()
    X = s.snapshots(0, 400)
    g, o = run_both(X, 20, 1e-8)
    pred = g.predict(500)
    g.sync()
    pg = pred.cpu().numpy()
    po = o.predict(500)
    fut = s.clean(400, 900).T
    err_o = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1)
    err_f = np.linalg.norm(pg - fut, axis=1) / np.linalg.norm(fut, axis=1)
    assert err_o.max() < 1e-9
    assert err_f.max() < 1e-9


@pytest.mark.parametrize("nx,ny,r_max", [(60, 40, 40), (173, 97, 32), (7, 5, 24)])
def test_wake_ragged_sizes(nx, ny, r_max, core_svd):
    """Noisy wake stream, n not a multiple of the tile size, truncation active."""
    s = synth.wake(nx=nx, ny=ny, noise=1e-6)
    X = s.snapshots(0, 200)
    g, o = run_both(X, r_max, 1e-8, check_every=25)
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    # planted (mean flow and shedding harmonics) eigenvalues agree to 1e-10
    pl = s.planted_eigs()[:11]
    mg, mo = O.match_eigs(pl, lam), O.match_eigs(pl, lo)
    assert np.max(np.abs(mg - mo) / np.abs(mo)) < 1e-10
    assert orth_err(g) < 1e-12


def test_determinism_bitwise():
    s = synth.wake(nx=50, ny=30, noise=1e-6)
    X = s.snapshots(0, 80)
    Xd = dev(X)
    runs = []
    for _ in range(2):
        g = ODMD(X.shape[0], 24, 1e-8)
        for k in range(79):
            g.update(Xd[k], Xd[k + 1])
        st = g.state()
        runs.append((st["sigma"], st["atilde"], g.basis_matrix().cpu().numpy()))
        g.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_scalar_and_tiny_streams():
    g = np.random.default_rng(7)
    X = g.standard_normal((1, 40))
    gp, o = run_both(X, 1, 1e-12)
    st = gp.state()
    x, y = X[0, :-1], X[0, 1:]
    np.testing.assert_allclose(st["atilde"][0, 0], x @ y / (x @ x), rtol=1e-13)
    # n below one tile, rank cap = n
    X = g.standard_normal((9, 30))
    gp, o = run_both(X, 9, 1e-12, check_every=3)
    assert gp.info().r == 9
    A = X[:, 1:] @ np.linalg.pinv(X[:, :-1])
    U = gp.basis_matrix().cpu().numpy()
    assert np.max(np.abs(U @ gp.state()["atilde"] @ U.T - A)) < 1e-10 * np.max(np.abs(A))


def test_rank_cap_64(core_svd):
    g = np.random.default_rng(8)
    X = g.standard_normal((3000, 90))
    gp, o = run_both(X, 64, 1e-12, check_every=10)
    assert gp.info().r == 64
    assert orth_err(gp) < 1e-12
    lam, _ = gp.eigs()
    assert rel_eig_err(np.linalg.eigvals(o.atilde()), lam, floor=0.1) < 1e-9


def test_zero_snapshots_and_empty_model(core_svd):
    n = 700
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    g = ODMD(n, 8, 1e-8)
    g.update(z, z)                      # zero first snapshot: stays empty
    g.sync()
    assert g.info().r == 0
    with pytest.raises(OdmdError) as e:
        g.eigs()
    assert e.value.name == "EEMPTY"
    g.predict(3)
    with pytest.raises(OdmdError):
        g.sync()                        # latched EEMPTY from the prediction
    g.update(z, x)                      # chained (x_k = previous x_k+1 = 0)
    g.update(x, 2 * x)
    g.sync()
    assert g.info().r == 1
    g.update(2 * x, z)                  # in span: rank unchanged
    g.update(z, z)                      # zero pair: rank unchanged, w -> 0
    g.sync()
    st = g.state()
    assert st["r"] == 1 and st["w"][0] == 0.0


def test_nonfinite_and_unchained_are_skipped():
    s = synth.planted_small(n=1000)
    X = s.snapshots(0, 30)
    Xd = dev(X)
    g = ODMD(1000, 10, 1e-8)
    for k in range(20):
        g.update(Xd[k], Xd[k + 1])
    g.sync()
    before = g.state()
    bad = Xd[21].clone()
    bad[17] = float("nan")
    g.update(Xd[20], bad)
    with pytest.raises(OdmdError) as e:
        g.sync()
    assert e.value.name == "ENONFINITE"
    after = g.state()
    np.testing.assert_array_equal(before["sigma"], after["sigma"])
    g.update(Xd[5], Xd[6])              # does not chain to the last accepted pair
    with pytest.raises(OdmdError) as e:
        g.sync()
    assert e.value.name == "ESEQ"
    # equal norms, not the previous y: sign-flipped, two entries swapped,
    # the entries reversed (x.x unchanged; the hashed fingerprint differs)
    flip = -Xd[20]
    swap = Xd[20].clone()
    swap[[3, 700]] = swap[[700, 3]]
    rev = torch.flip(Xd[20], dims=[0])
    for x in (flip, swap, rev):
        nx, n20 = float(x @ x), float(Xd[20] @ Xd[20])
        assert abs(nx - n20) <= 1e-13 * n20
        g.update(x, Xd[21])
        with pytest.raises(OdmdError) as e:
            g.sync()
        assert e.value.name == "ESEQ"
    np.testing.assert_array_equal(before["sigma"], g.state()["sigma"])
    # the stream resumes where it was and matches an oracle that skipped both
    o = O.OnlineDMD(1000, 10, 1e-8)
    for k in range(25):
        o.update(X[:, k], X[:, k + 1])
    for k in range(20, 25):
        g.update(Xd[k], Xd[k + 1])
    g.sync()
    np.testing.assert_allclose(g.state()["sigma"], o.sigma, rtol=1e-12)


def test_full_size_wake_prefix():
    """n = 160,000 (400 x 200 grid), r_max 40, the launch the benchmark times:
    the first 120 updates element by element against the oracle, then
    properties that hold at any length."""
    s = synth.wake(nx=400, ny=200, noise=1e-6)
    X = s.snapshots(0, 121)
    g, o = run_both(X, 40, 1e-8, check_every=20)
    st = g.state()
    assert st["r"] == o.r
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    pl = s.planted_eigs()[:11]
    assert np.max(np.abs(O.match_eigs(pl, lam) - O.match_eigs(pl, lo))) < 1e-10
    assert orth_err(g) < 1e-12
    pg = g.predict(5).cpu().numpy()
    po = o.predict(5)
    assert np.max(np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1)) < 1e-9


def test_refold_limit_follows_the_rank():
    """FP64/FP32 bases refold once r + 16 columns are stored, below the
    capacity (here 48); a BF16 basis only at the capacity.  The oracle's
    values are kept.  The stream (Gaussian modes, rank 27, cap 30) keeps
    appending directions that truncation then drops, so the stored columns
    grow at a steady rank."""
    n, rank, r_max, steps = 90992, 27, 30, 120
    gen = synth.DevicePlanted(torch, n, rank, seed=231118715 + 1)
    X64 = gen.chunk(0, steps + 1)
    X = X64.cpu().numpy().T
    o = O.OnlineDMD(n, r_max, 1e-8)
    for k in range(steps):
        o.update(X[:, k], X[:, k + 1])
    for basis in ("f64", "f32", "bf16"):
        g = ODMD(n, r_max, 1e-8, basis=basis)
        Xd = X64 if basis == "f64" else X64.float()
        peak, over = 0, 0
        for k in range(steps):
            g.update(Xd[k], Xd[k + 1])
            info = g.info()
            peak = max(peak, info.stored)
            over = max(over, info.stored - info.r)
        assert info.capacity == 48
        assert peak <= 48, (basis, peak)
        if basis != "bf16":
            assert over <= 16, (basis, over)
        if basis == "f64":
            assert over == 16 and peak < 48, (peak, over)     # refolded below the capacity
            st = g.state()
            assert st["r"] == o.r
            np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
        g.close()


def _basis_invariant_err(g, o, n, seed=3):
    """max |U A~ U^T P - U_o A~_o U_o^T P| over random probes P, relative:
    the DMD operator on span(U) does not depend on the basis chosen inside
    ties of equal singular values."""
    U = g.basis_matrix().cpu().numpy()
    P = np.random.default_rng(seed).standard_normal((n, 4))
    Pg = U @ (g.state()["atilde"] @ (U.T @ P))
    Po = o.U @ (o.atilde() @ (o.U.T @ P))
    return np.max(np.abs(Pg - Po)) / np.max(np.abs(Po))


def test_tied_singular_values_and_orthogonal_appends(core_svd):
    """Special cases of the core (Sec. 2.3's rank-1 append with a core
    K = [[diag sigma, p], [0, rho]]):
      * x orthogonal to span(U) with the norm of every earlier snapshot:
        p = 0 and rho = sigma_i, so K is diagonal with all values tied (every
        secular term deflates);
      * then a snapshot mixing all earlier directions plus a new one: p has
        nonzero entries on exactly tied poles, which the secular solver must
        merge by rotations before it solves;
      * then ordinary snapshots.
    Compared with the oracle by invariants (sorted sigma, the operator
    U A~ U^T on probes, orthogonality), since the singular vectors inside a
    tie are not unique."""
    n, k = 5000, 12
    X = np.zeros((n, k + 8))
    rows = np.random.default_rng(11).permutation(n)[:k + 1]
    for j in range(k):
        X[rows[j], j] = 3.0                     # equal norms, orthogonal
    a = np.random.default_rng(12).standard_normal(k)
    X[rows[:k], k] = a                          # mixes every tied direction
    X[rows[k], k] = 0.5                         # plus a new one
    X[:, k + 1:] = np.random.default_rng(13).standard_normal((n, 7))
    g, o = run_both(X, 24, 1e-12, steps=k - 1)
    st = g.state()
    assert st["r"] == o.r == k - 1
    np.testing.assert_allclose(st["sigma"], 3.0, rtol=1e-14)      # all tied
    for steps in (k, k + 1, X.shape[1] - 1):                        # the merge, then more
        g, o = run_both(X, 24, 1e-12, steps=steps)
        st = g.state()
        assert st["r"] == o.r
        np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-12, atol=1e-14 * o.sigma[0])
        assert orth_err(g) < 1e-12
        assert _basis_invariant_err(g, o, n) < 1e-10
        g.close()


def test_full_size_wake_all_updates():
    """The benchmark's stream exactly (wake on a 400 x 200 grid, n =
    160,000, noise 1e-6, r_max 40, tol 1e-8, all 1999 updates, the launch
    the benchmark times) against the oracle: rank and sigma every 200
    updates, then the eigenvalues of the planted modes present in the data
    (mean flow, shedding harmonics), orthogonality and a 500-state
    rollout."""
    s = synth.wake(nx=400, ny=200, noise=1e-6)
    X = s.snapshots(0, 2000)
    print("wake n=160000: 1999 updates against the oracle", flush=True)
    g, o = run_both(X, 40, 1e-8, check_every=200)
    st = g.state()
    assert st["r"] == o.r == 40
    np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    pl = s.planted_eigs()[:11]
    mg, mo = O.match_eigs(pl, lam), O.match_eigs(pl, lo)
    assert np.max(np.abs(mg - mo) / np.abs(mo)) < 1e-10
    # the other eigenvalues belong to noise directions (reading: the 1e-10
    # tolerance applies to the planted ones).  A~_ij carries 1/sigma_j, so
    # rounding in the columns of the noise directions (sigma_j down to
    # 1e-6 sigma_1) is amplified; the operator on the directions above the
    # noise, U_k A~_kk U_k^T with sigma_k >= 1e-4 sigma_1, must agree to 1e-10
    print(f"all eigenvalues with |lambda| >= 1e-2 max: {rel_eig_err(lo, lam):.2e}; "
          f"whole operator on probes: {_basis_invariant_err(g, o, X.shape[0]):.2e}", flush=True)
    k = int(np.sum(o.sigma >= 1e-4 * o.sigma[0]))
    assert k >= 11
    U = g.basis_matrix().cpu().numpy()[:, :k]
    P = np.random.default_rng(5).standard_normal((X.shape[0], 4))
    Pg = U @ (st["atilde"][:k, :k] @ (U.T @ P))
    Po = o.U[:, :k] @ (o.atilde()[:k, :k] @ (o.U[:, :k].T @ P))
    assert np.max(np.abs(Pg - Po)) < 1e-10 * np.max(np.abs(Po))
    assert orth_err(g) < 1e-12
    pg = g.predict(500).cpu().numpy()
    po = o.predict(500)
    err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1)
    print(f"rollout over 500 states: max relative difference {err.max():.2e}", flush=True)
    assert err.max() < 1e-9


def test_prediction_on_a_defective_operator():
    """A stream whose operator has a Jordan block (A~ without a full set of
    eigenvectors: cond(V) about 2e8).  The GPU forms the prediction from
    powers of A~, so it stays the exact continuation of the linear data:
    60 states within 1e-10 of the true future (relative to the largest
    state) and of the oracle's power-form rollout, where the eigenvector
    form of the oracle is off by about 2e-9."""
    from test_oracle_pins import _jordan_stream
    X, fut = _jordan_stream()
    g, o = run_both(X, 8, 1e-10)
    assert g.info().r == o.r == 4
    pg = g.predict(60).cpu().numpy()
    scale = np.linalg.norm(fut, axis=0).max()
    assert np.linalg.norm(pg - fut.T, axis=1).max() < 1e-10 * scale
    pw = O.rollout_power(o.U, o.atilde(), o.p_y, 60)
    assert np.linalg.norm(pg - pw, axis=1).max() < 1e-10 * scale


def test_rank_one_stream_rollout_across_chunks():
    """x_k = 0.9^k v: rank 1 (one 16-row tile, a 1 x 1 A~), 1100 predicted
    states (three read-out launches, coefficient launches of 512) equal
    0.9^(a+k) v to 1e-12 of the largest state."""
    n = 2048 + 37
    v = np.random.default_rng(5).standard_normal(n)
    X = np.stack([0.9 ** k * v for k in range(12)], axis=1)
    g, o = run_both(X, 4, 1e-10)
    assert g.info().r == o.r == 1
    pg = g.predict(1100).cpu().numpy()
    fut = np.stack([0.9 ** (11 + k) * v for k in range(1, 1101)])
    assert np.abs(pg - fut).max() < 1e-12 * np.abs(fut).max()


@pytest.mark.parametrize("steps", [271, 272, 273, 512, 513, 784])
def test_rollout_at_chunk_boundaries(steps):
    """Rank cap 40: coefficient launches of 272 steps, read-out launches of
    512 states.  Rollouts that end just before, on and just after each
    boundary match the oracle's state by state (1e-9 of the largest state)."""
    s = synth.wake(nx=61, ny=39, noise=1e-6)
    X = s.snapshots(0, 120)
    g, o = run_both(X, 40, 1e-8)
    assert g.info().r == o.r == 40
    pg = g.predict(steps).cpu().numpy()
    po = o.predict(steps)
    err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1).max()
    assert err.max() < 1e-9


def test_eigenvalues_alone_equal_those_with_vectors():
    """odmd_eigs without vectors runs the eigensolver without Z, the
    eigenvectors and V: its eigenvalues equal those of a call with vectors
    bit for bit (Z does not enter H's iteration), a call with vectors after
    a values-only call recomputes, a values-only call after it reuses the
    cache, and an update invalidates both."""
    s = synth.wake(nx=61, ny=39, noise=1e-6)
    X = s.snapshots(0, 122)
    g, o = run_both(X, 40, 1e-8, steps=120)
    lam1 = g.eigs(vectors=False)[0]
    lam2, V = g.eigs(vectors=True)
    assert np.array_equal(lam1, lam2)
    assert np.array_equal(g.eigs(vectors=False)[0], lam2)
    A = g.state()["atilde"]
    assert np.linalg.norm(A @ V - V * lam2[None, :]) < 1e-10 * np.linalg.norm(A)
    Xd = dev(X, torch.float64)
    g.update(Xd[120], Xd[121])
    lam3 = g.eigs(vectors=False)[0]
    lam4, _ = g.eigs(vectors=True)
    assert np.array_equal(lam3, lam4) and not np.array_equal(lam3, lam1)
