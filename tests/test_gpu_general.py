"""General (unchained) pairs on the GPU against the FP64 oracle's general
form (B = Y W, A~ = U^T B S^-1, Sec. 2.3).

Inputs: restarted trajectories of one planted operator (seeded synth
generators), so that x_k of a pair differs from the previous x_k1 at
every segment start.  Tolerances as for chained pairs (FP64): eigenvalues
1e-10 relative on |lambda| >= 1e-2 max|lambda|, singular values 1e-11
relative, orthogonality 1e-12, rollouts 1e-9 relative; FP32 basis 1e-4 on
the eigenvalues of the modes above the noise.
"""
import ctypes

import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import ODMD, OdmdError, update_batch


def dev(X, dtype=torch.float64 if torch is not None else None):
    return torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dtype)


def rel_eig_err(ref, got, floor=1e-2):
    big = np.abs(ref) >= floor * np.abs(ref).max()
    m = O.match_eigs(ref[big], got)
    return np.max(np.abs(m - ref[big]) / np.abs(ref[big]))


def run_pairs(X, Y, r_max, tol, basis="f64", check_every=0):
    dt = torch.float64 if basis == "f64" else torch.float32
    g = ODMD(X.shape[0], r_max, tol, basis=basis, pairs="general")
    o = O.OnlineDMDF1(X.shape[0], r_max, g.info().tol_eff)
    Xd, Yd = dev(X, dt), dev(Y, dt)
    Xo, Yo = Xd.double().cpu().numpy().T, Yd.double().cpu().numpy().T
    for j in range(X.shape[1]):
        g.update(Xd[j], Yd[j])
        o.update(Xo[:, j], Yo[:, j])
        if check_every and (j % check_every == 0 or j == X.shape[1] - 1):
            s = g.state()
            assert s["r"] == o.r, f"rank differs at pair {j}"
            np.testing.assert_allclose(s["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    g.sync()
    return g, o


def test_planted_restarted_pairs_every_step():
    """n = 4096, rank 6, 8 segments x 20 pairs, noise-free: rank and sigma
    after every pair, A~ against the oracle's and the planted spectrum."""
    s = synth.planted_small()
    X, Y = synth.restarted_pairs(s, 8, 20, seed=41)
    g, o = run_pairs(X, Y, 20, 1e-8, check_every=1)
    assert g.info().r == 6
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    assert rel_eig_err(lo, lam) < 1e-10
    assert rel_eig_err(s.planted_eigs(), lam) < 1e-10
    st = g.state()
    U = g.basis_matrix().cpu().numpy()
    assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) < 1e-12
    # U A~ U^T is basis-independent: compare on probes
    P = np.random.default_rng(1).standard_normal((U.shape[0], 4))
    a = U @ (st["atilde"] @ (U.T @ P))
    b = o.U @ (o.atilde() @ (o.U.T @ P))
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(b))
    pg, po = g.predict(50).cpu().numpy(), o.predict(50)
    assert np.max(np.abs(pg - po)) < 1e-9 * np.max(np.abs(po))


@pytest.mark.parametrize("nx,ny,r_max,segments,length", [
    (61, 37, 24, 10, 14),      # n = 4514: ragged last tile; both stored sets refold
    (400, 200, 40, 6, 25),     # n = 160,000, the benchmark's stream size and launch shape
])
def test_noisy_wake_restarted_pairs(nx, ny, r_max, segments, length):
    """Wake-shaped operator with noise 1e-6, truncation at r_max, stored
    column sets of both U and B refolding several times."""
    s = synth.wake(nx=nx, ny=ny, noise=1e-6)
    X, Y = synth.restarted_pairs(s, segments, length, seed=43)
    g, o = run_pairs(X, Y, r_max, 1e-8, check_every=7)
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    # the eigenvalues of the planted modes (noise directions, some of them
    # larger in modulus than the weakest transients, differ at the
    # truncation boundary and are not compared)
    pl = s.planted_eigs()
    mg, mo = O.match_eigs(pl, lam), O.match_eigs(pl, lo)
    assert np.max(np.abs(mg - mo) / np.abs(mo)) < 1e-10
    st = g.state()
    np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    U = g.basis_matrix().cpu().numpy()
    assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) < 1e-12
    pg, po = g.predict(20).cpu().numpy(), o.predict(20)
    err = np.linalg.norm(pg - po, axis=1) / np.linalg.norm(po, axis=1)
    assert err.max() < 1e-9


def test_chained_stream_through_general_handle():
    """A chained stream through a general handle gives the chained form's
    model (F1 and F2 agree without truncation)."""
    s = synth.planted_small(n=3000)
    X = s.snapshots(0, 150)
    Xd = dev(X)
    a = ODMD(X.shape[0], 16, 1e-8)
    b = ODMD(X.shape[0], 16, 1e-8, pairs="general")
    for k in range(X.shape[1] - 1):
        a.update(Xd[k], Xd[k + 1])
        b.update(Xd[k], Xd[k + 1])
    a.sync()
    b.sync()
    la, _ = a.eigs()
    lb, _ = b.eigs()
    assert a.info().r == b.info().r == 6
    assert rel_eig_err(la, lb) < 1e-11
    pa, pb = a.predict(30).cpu().numpy(), b.predict(30).cpu().numpy()
    assert np.max(np.abs(pa - pb)) < 1e-9 * np.max(np.abs(pa))


def test_fp32_general_pairs():
    """FP32 basis (FP64 residuals, projections and small problems) against
    the FP64 oracle on the same FP32-rounded pairs: 1e-4 relative on the
    eigenvalues of the modes above the noise."""
    s = synth.wake(nx=150, ny=100, noise=1e-5)
    X, Y = synth.restarted_pairs(s, 8, 20, seed=47)
    g, o = run_pairs(X, Y, 40, 1e-8, basis="f32")
    lam, _ = g.eigs()
    lo, _ = o.eigs()
    pl = s.planted_eigs()
    persist = pl[np.abs(np.abs(pl) - 1.0) < 1e-12]
    mg, mo = O.match_eigs(persist, lam), O.match_eigs(persist, lo)
    assert np.max(np.abs(mg - mo) / np.abs(mo)) < 1e-4


def test_general_edge_cases():
    """Zero first pair (stays empty), a pair with x in span(U) (rank kept),
    non-finite input latched, batch launch refused."""
    n = 777
    g = ODMD(n, 8, 1e-8, pairs="general")
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    g.update(z, z)
    g.sync()
    assert g.info().r == 0
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, 6))
    Xd = dev(X)
    g.update(Xd[0], Xd[1])
    g.update(Xd[2], Xd[3])
    g.update(Xd[0] * 2.0, Xd[4])           # x in span(U): rank unchanged
    g.sync()
    o = O.OnlineDMDF1(n, 8, 1e-8)
    o.update(np.zeros(n), np.zeros(n))
    o.update(X[:, 0], X[:, 1])
    o.update(X[:, 2], X[:, 3])
    o.update(2.0 * X[:, 0], X[:, 4])
    assert g.info().r == o.r == 2
    np.testing.assert_allclose(g.state()["atilde"].shape, (2, 2))
    la, _ = g.eigs()
    lo, _ = o.eigs()
    assert rel_eig_err(lo, la) < 1e-10
    bad = Xd[5].clone()
    bad[3] = float("nan")
    g.update(bad, Xd[1])
    with pytest.raises(OdmdError) as e:
        g.sync()
    assert e.value.name == "ENONFINITE"
    h = ODMD(n, 8, 1e-8, pairs="general")
    with pytest.raises(OdmdError) as e:
        update_batch([h], [Xd[0]], [Xd[1]])
    assert e.value.name == "EINVAL"
