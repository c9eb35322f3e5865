"""Launch shapes of the streaming pass: explicit and tuned shapes.

Any valid shape (workgroup size, rows per workgroup, workgroup cap) must
give the oracle's results: one workgroup for all rows, one per 16-row unit,
and shapes between, over sizes that end in a ragged tile.  Handles with
tuned shapes must batch bit for bit like their own launches, and the
autotuner must return one of its candidates.
"""
import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd import odmd as B
    from paper_2311_18715_amd.odmd import ODMD, update_batch

SHAPES = [None, (256, 16, 65536), (512, 16, 65536), (512, 2048, 1024), (256, 128, 7),
          (512, 1 << 24, 1), (256, 16, 1)]


def _stream(n, rank, steps, seed):
    s = synth.random_planted(n, rank, seed=seed)
    X = s.snapshots(0, steps + 1)
    return X, torch.from_numpy(np.ascontiguousarray(X.T)).cuda()


@pytest.mark.parametrize("n,rank,r_max", [(20011, 12, 24), (777, 6, 10)])
def test_every_shape_matches_the_oracle(n, rank, r_max):
    steps = 45                       # spans two refolds at r_max = 24 (capacity 40)
    X, Xd = _stream(n, rank, steps, seed=31 + n)
    o = O.OnlineDMD(n, r_max, 1e-10)
    for k in range(steps):
        o.update(X[:, k], X[:, k + 1])
    lam_o = np.sort_complex(o.eigs()[0])
    ref = None
    for shape in SHAPES:
        g = ODMD(n, r_max, 1e-10, shape=shape)
        for k in range(steps):
            g.update(Xd[k], Xd[k + 1])
        g.sync()
        info = g.info()
        t, rpb, cap = shape or B.default_shape(n)
        assert info.threads == t
        assert info.nblocks == min(-(-n // rpb), cap), shape
        st = g.state()
        assert st["r"] == o.r, shape
        np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
        lam = np.sort_complex(g.eigs(vectors=False)[0])
        np.testing.assert_allclose(lam, lam_o, rtol=1e-10, atol=1e-12)
        if ref is None:
            ref = st
        else:                        # shapes change the order of the sums only
            np.testing.assert_allclose(st["sigma"], ref["sigma"], rtol=1e-12)
        g.close()


def test_shaped_batch_equals_individual_bitwise():
    specs = [(20011, 12, 24, "f64", (256, 128, 1024)), (5000, 8, 16, "f32", (512, 2048, 256)),
             (64, 4, 8, "f64", (256, 16, 65536)), (9000, 10, 33, "f32", None),
             (3000, 6, 16, "f64", (512, 256, 3))]
    steps = 30
    data = [_stream(n, rank, steps, seed=70 + i) for i, (n, rank, _, _, _) in enumerate(specs)]
    data = [(X, Xd if b == "f64" else Xd.float()) for (X, Xd), (_, _, _, b, _) in zip(data, specs)]
    A = [ODMD(n, rm, 1e-10, basis=b, shape=sh) for (n, _, rm, b, sh) in specs]
    C = [ODMD(n, rm, 1e-10, basis=b, shape=sh) for (n, _, rm, b, sh) in specs]
    for k in range(steps):
        update_batch(A, [Xd[k] for _, Xd in data], [Xd[k + 1] for _, Xd in data])
        for g, (_, Xd) in zip(C, data):
            g.update(Xd[k], Xd[k + 1])
    for a, c, spec in zip(A, C, specs):
        sa, sc = a.state(), c.state()
        for key in ("sigma", "atilde", "p_y", "C", "w"):
            assert np.array_equal(sa[key], sc[key]), (spec, key)
        assert torch.equal(a.basis_matrix(), c.basis_matrix()), spec


@pytest.mark.parametrize("basis,streams", [("f64", 1), ("f32", 3)])
def test_autotune_returns_a_working_candidate(basis, streams):
    n, r_max = 5000, 16
    shape, us_best, us_default = B.autotune(n, r_max, basis, streams=streams)
    t, rpb, cap = shape
    assert t in (256, 512)
    assert shape == B.default_shape(n) or (rpb in (128, 256, 512, 1024, 2048)
                                           and cap in (256, 512, 1024))
    assert 0.0 < us_best <= us_default
    # the tuned shape serves a stream (the oracle's result, as above)
    X, Xd = _stream(n, 6, 20, seed=5)
    tol = 1e-10
    if basis == "f32":
        # FP32 snapshots: a tolerance above their own rounding (2^-24), which
        # the method would otherwise keep as new directions
        Xd, tol = Xd.float(), 1e-6
    g = ODMD(n, r_max, tol, basis=basis, shape=shape)
    for k in range(20):
        g.update(Xd[k], Xd[k + 1])
    g.sync()
    assert g.info().r == 6


def test_shape_by_objective_uses_the_shipped_table():
    from paper_2311_18715_amd import autotune
    for n, r_max, basis, objective in [(160000, 40, "f64", "latency"), (10000, 16, "f64", "latency"),
                                       (150000, 30, "f32", "throughput"), (77, 4, "f32", "throughput")]:
        g = ODMD(n, r_max, 1e-10, basis=basis, shape=objective)
        want = autotune.lookup(n, r_max, basis, objective=objective)
        assert g.shape == want
        t, rpb, cap = want or B.default_shape(n)
        info = g.info()
        assert (info.threads, info.nblocks) == (t, min(-(-n // rpb), cap))
        g.close()


def test_fp32_two_rows_per_lane_matches_one_row():
    """FP32 storage at a ragged n past the two-rows-per-lane threshold: the
    512-thread shape (two rows per lane, whole 128-byte lines) against the
    256-thread shape (one row per lane) on the same pairs.  Different sum
    orders, so the two agree to FP32-storage rounding: equal rank, sigma
    within 1e-6 sigma_1, eigenvalues within 2e-5 of each other and 1e-4 of
    the planted ones (80 pairs: with 40, the FP64 oracle itself is 4e-3 off
    on these FP32-rounded snapshots), rollouts within 1e-5.  A batch of two two-row handles equals their
    own launches bit for bit."""
    n, rank, r_max, steps = (1 << 21) + 17, 9, 16, 80
    gen = synth.DevicePlanted(torch, n, rank, seed=2718, dtype=torch.float32)
    X = gen.chunk(0, steps + 1)
    two = ODMD(n, r_max, 1e-6, basis="f32")
    one = ODMD(n, r_max, 1e-6, basis="f32", shape=(256, 512, 512))
    assert two.info().threads == 512 and one.info().threads == 256
    for k in range(steps):
        two.update(X[k], X[k + 1])
        one.update(X[k], X[k + 1])
    st, so = two.state(), one.state()
    assert st["r"] == so["r"] == rank
    np.testing.assert_allclose(st["sigma"], so["sigma"], rtol=0, atol=1e-6 * so["sigma"][0])
    lams = [g.eigs(vectors=False)[0] for g in (two, one)]
    for lam in lams:
        got = O.match_eigs(gen.planted, lam)
        assert np.max(np.abs(got - gen.planted) / np.abs(gen.planted)) < 1e-4
    d = np.abs(O.match_eigs(lams[1], lams[0]) - lams[1]) / np.abs(lams[1])
    assert d.max() < 2e-5, d.max()
    pt, po = two.predict(20), one.predict(20)
    err = (torch.linalg.norm((pt - po).double(), dim=1) / torch.linalg.norm(po.double(), dim=1)).max()
    assert float(err) < 1e-5, float(err)
    # batched two-row launches equal the handles' own launches
    A = [ODMD(n, r_max, 1e-6, basis="f32") for _ in range(2)]
    C = [ODMD(n, r_max, 1e-6, basis="f32") for _ in range(2)]
    for k in range(12):
        update_batch(A, [X[k], X[k + 1]], [X[k + 1], X[k + 2]])
        C[0].update(X[k], X[k + 1])
        C[1].update(X[k + 1], X[k + 2])
    for a, c in zip(A, C):
        sa, sc = a.state(), c.state()
        for key in ("sigma", "atilde", "p_y", "C", "w"):
            assert np.array_equal(sa[key], sc[key]), key
        assert torch.equal(a.basis_matrix(), c.basis_matrix())
    for g in [two, one] + A + C:
        g.close()


def test_profile_kernel_and_latency_samples():
    """Timed updates: events around each kernel give pass and core
    durations; latency-only updates give NaN for those and their pass start
    to core end; timing changes no result."""
    X, Xd = _stream(20011, 8, 40, seed=77)
    g, h = ODMD(20011, 16, 1e-8), ODMD(20011, 16, 1e-8)
    g.profile(64)
    g.profile(0)
    for k in range(40):
        if k == 10:
            g.profile_latency(False)
            g.profile(64)
        elif k == 20:
            g.profile_latency(True)
        elif k == 30:
            g.profile(0)
        g.update(Xd[k], Xd[k + 1])
        h.update(Xd[k], Xd[k + 1])
    a, b, u = g.profile_samples()
    assert len(a) == 20
    assert np.all(a[:10] > 0) and np.all(b[:10] > 0)
    assert np.all(u[:10] >= np.maximum(a[:10], b[:10]))
    assert np.all(np.isnan(a[10:])) and np.all(np.isnan(b[10:]))
    assert np.all(u[10:] > 0) and np.all(np.isfinite(u))
    lam_g, lam_h = g.eigs(vectors=False)[0], h.eigs(vectors=False)[0]
    assert np.array_equal(lam_g, lam_h)
    g.close()
    h.close()
