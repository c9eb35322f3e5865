"""Batched form: one fused update of many streams equals per-stream updates.

Streams differ in size (ragged, several rank buckets) and storage type; the
batched launch must reproduce each stream's own launch bit for bit (same
partition, same reduction order), and the FP64 streams must match the
oracle.
"""
import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import ODMD, update_batch

SPECS = [  # (n, planted rank, r_max, basis)
    (3000, 6, 16, "f64"), (777, 10, 12, "f64"), (20000, 30, 64, "f64"),
    (5000, 12, 40, "f32"), (12345, 20, 24, "f32"), (64, 4, 8, "f64"), (9000, 26, 33, "f32"),
]


def make_streams(steps):
    data = []
    for i, (n, rank, rmax, basis) in enumerate(SPECS):
        s = synth.random_planted(n, rank, seed=1000 + i)
        X = s.snapshots(0, steps + 1)
        dt = torch.float64 if basis == "f64" else torch.float32
        data.append((X, torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dt)))
    return data


def test_batch_equals_individual_bitwise():
    steps = 40
    data = make_streams(steps)
    A = [ODMD(n, rmax, 1e-10, basis=b) for (n, _, rmax, b) in SPECS]
    B = [ODMD(n, rmax, 1e-10, basis=b) for (n, _, rmax, b) in SPECS]
    for k in range(steps):
        update_batch(A, [Xd[k] for _, Xd in data], [Xd[k + 1] for _, Xd in data])
        for g, (_, Xd) in zip(B, data):
            g.update(Xd[k], Xd[k + 1])
    for a, b, (X, _), spec in zip(A, B, data, SPECS):
        a.sync()
        b.sync()
        sa, sb = a.state(), b.state()
        assert sa["r"] == sb["r"]
        for key in ("sigma", "atilde", "p_y", "C", "w"):
            assert np.array_equal(sa[key], sb[key]), (spec, key)
        assert torch.equal(a.basis_matrix(), b.basis_matrix()), spec
        if spec[3] == "f64":
            o = O.OnlineDMD(X.shape[0], spec[2], 1e-10)
            for k in range(steps):
                o.update(X[:, k], X[:, k + 1])
            assert sa["r"] == o.r
            np.testing.assert_allclose(sa["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])


def test_batch_of_one_and_validation():
    s = synth.random_planted(1000, 8, seed=7)
    X = s.snapshots(0, 11)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    a, b = ODMD(1000, 8, 1e-10), ODMD(1000, 8, 1e-10)
    for k in range(10):
        update_batch([a], [Xd[k]], [Xd[k + 1]])
        b.update(Xd[k], Xd[k + 1])
    assert np.array_equal(a.state()["atilde"], b.state()["atilde"])
    with pytest.raises(Exception):
        update_batch([a, a], [Xd[0], Xd[0]], [Xd[1], Xd[1]])    # duplicate handle


def test_predict_batch_equals_individual():
    from paper_2311_18715_amd.odmd import predict_batch
    steps = 25
    data = make_streams(steps)
    A = [ODMD(n, rmax, 1e-10, basis=b) for (n, _, rmax, b) in SPECS]
    for k in range(steps):
        update_batch(A, [Xd[k] for _, Xd in data], [Xd[k + 1] for _, Xd in data])
    # 17 + i states, and a long rollout for every third stream: more states
    # than one coefficient launch holds at its rank cap (the batched launch
    # forms the first chunk, the rest follow per stream) and than one
    # read-out launch (512)
    ks = [17 + i if i % 3 else 600 + 7 * i for i in range(len(A))]
    one = [g.predict(k) for g, k in zip(A, ks)]
    many = predict_batch(A, ks)
    for a, b in zip(one, many):
        assert torch.equal(a, b)
    with pytest.raises(Exception):
        predict_batch([A[0], A[0]], [3, 3])
