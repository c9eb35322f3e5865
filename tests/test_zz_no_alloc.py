"""The batched update without allocation (odmd_update_batch_noalloc)
against odmd_update_batch: same handles' shapes, same pairs, results equal
bit for bit, on two calls in a row, the second with a smaller input (fewer
streams, one of them the same as before); FP64 streams also against the
oracle.  The streams mix storage types, both launch shapes (n below and
above 131072) and several live-column buckets, so the fixed tables hold
several pass launches."""
import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import (ODMD, OdmdError, update_batch,
                                           update_batch_noalloc)

SPECS = [  # (n, planted rank, r_max, basis)
    (3000, 6, 16, "f64"), (140001, 12, 24, "f64"), (20000, 30, 64, "f32"),
    (777, 10, 12, "f32"), (150000, 8, 16, "bf16"), (9001, 20, 40, "f64"),
]


def _data(steps):
    out = []
    for i, (n, rank, rmax, basis) in enumerate(SPECS):
        X = synth.random_planted(n, rank, seed=4000 + i).snapshots(0, steps + 1)
        dt = torch.float64 if basis == "f64" else torch.float32
        out.append((X, torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dt)))
    return out


def _same(a, b, tag):
    a.sync()
    b.sync()
    sa, sb = a.state(), b.state()
    assert sa["r"] == sb["r"], tag
    for key in ("sigma", "atilde", "p_y", "C", "w"):
        assert np.array_equal(sa[key], sb[key]), (tag, key)
    assert torch.equal(a.basis_matrix(), b.basis_matrix()), tag


def test_noalloc_batch_equals_update_batch_on_two_calls():
    s1, s2 = 30, 20
    data = _data(s1 + s2)
    print(f"noalloc: {len(SPECS)} streams, {s1} steps, then 3 streams, {s2} steps", flush=True)
    A = [ODMD(n, rmax, 1e-10, basis=b) for (n, _, rmax, b) in SPECS]
    B = [ODMD(n, rmax, 1e-10, basis=b) for (n, _, rmax, b) in SPECS]
    # first call: every stream
    for k in range(s1):
        xs = [Xd[k] for _, Xd in data]
        ys = [Xd[k + 1] for _, Xd in data]
        update_batch(A, xs, ys)
        update_batch_noalloc(B, xs, ys)
    for i, (a, b) in enumerate(zip(A, B)):
        _same(a, b, ("first", SPECS[i]))
    # second call, smaller: three streams (a different mix of types and shapes)
    sub = [1, 3, 5]
    for k in range(s1, s1 + s2):
        xs = [data[i][1][k] for i in sub]
        ys = [data[i][1][k + 1] for i in sub]
        update_batch([A[i] for i in sub], xs, ys)
        update_batch_noalloc([B[i] for i in sub], xs, ys)
    for i in range(len(SPECS)):
        _same(A[i], B[i], ("second", SPECS[i]))
    # FP64 streams of the second call against the oracle
    for i in sub:
        n, _, rmax, basis = SPECS[i]
        if basis != "f64":
            continue
        X = data[i][0]
        o = O.OnlineDMD(n, rmax, 1e-10)
        for k in range(s1 + s2):
            o.update(X[:, k], X[:, k + 1])
        st = B[i].state()
        assert st["r"] == o.r
        np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    for g in A + B:
        g.close()


def test_noalloc_batch_rejects_duplicates_and_general_pairs():
    X = synth.random_planted(1000, 6, seed=5).snapshots(0, 3)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    a = ODMD(1000, 8, 1e-10)
    g = ODMD(1000, 8, 1e-10, pairs="general")
    with pytest.raises(OdmdError):
        update_batch_noalloc([a, a], [Xd[0], Xd[0]], [Xd[1], Xd[1]])
    with pytest.raises(OdmdError):
        update_batch_noalloc([a, g], [Xd[0], Xd[0]], [Xd[1], Xd[1]])
    update_batch_noalloc([a], [Xd[0]], [Xd[1]])
    a.sync()
    assert a.info().r == 1
    a.close()
    g.close()
