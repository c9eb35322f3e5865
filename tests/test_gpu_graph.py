"""Plans and HIP-graph replay of the batched step.

A plan fixes one batched step (handles and snapshot buffers); launching it
eagerly must equal odmd_update_batch bit for bit, and a graph captured
from its launch must equal the eager launches on every replay, with eager
work and synchronisations between replays.  The FP64 streams must match
the oracle.
"""
import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import ODMD, Plan, OdmdError, update_batch

SPECS = [  # (n, planted rank, r_max, basis, shape)
    (20011, 12, 24, "f64", None), (3000, 6, 16, "f32", None), (777, 5, 10, "f64", (256, 16, 65536)),
    (150000, 10, 40, "f32", None), (64, 4, 8, "f64", None),
]
STEPS = 36


def _data():
    out = []
    for i, (n, rank, _, basis, _) in enumerate(SPECS):
        X = synth.random_planted(n, rank, seed=400 + i).snapshots(0, STEPS + 1)
        dt = torch.float64 if basis == "f64" else torch.float32
        out.append((X, torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dt)))
    return out


def _models(stream):
    return [ODMD(n, rm, 1e-10, basis=b, stream=stream, shape=sh) for (n, _, rm, b, sh) in SPECS]


def _equal(a, b):
    sa, sb = a.state(), b.state()
    if sa["r"] != sb["r"]:
        return False
    return all(np.array_equal(sa[k], sb[k]) for k in ("sigma", "atilde", "p_y", "C", "w")) and \
        torch.equal(a.basis_matrix(), b.basis_matrix())


class _Buffers:
    """Two fixed snapshot buffers per stream: pair k reads buf[k % 2] and
    buf[(k + 1) % 2]; x_{k+1} is written into buf[(k + 1) % 2] first."""

    def __init__(self, data):
        self.buf = [[torch.empty_like(Xd[0]) for _ in range(2)] for _, Xd in data]
        self.data = data

    def fill(self, k):
        for b, (_, Xd) in zip(self.buf, self.data):
            if k == 0:
                b[0].copy_(Xd[0])
            b[(k + 1) % 2].copy_(Xd[k + 1])

    def plans(self, models):
        return [Plan(models, [b[j] for b in self.buf], [b[1 - j] for b in self.buf]) for j in (0, 1)]


def test_plan_equals_update_batch_and_oracle():
    S = torch.cuda.Stream()
    data = _data()
    A, Bm = _models(S), _models(S)
    with torch.cuda.stream(S):
        bufs = _Buffers(data)
        plans = bufs.plans(A)
        for k in range(STEPS):
            bufs.fill(k)
            plans[k % 2].launch()
            update_batch(Bm, [b[k % 2] for b in bufs.buf], [b[(k + 1) % 2] for b in bufs.buf])
    S.synchronize()
    for a, b, (X, _), spec in zip(A, Bm, data, SPECS):
        a.sync()
        assert _equal(a, b), spec
        if spec[3] == "f64":
            o = O.OnlineDMD(X.shape[0], spec[2], 1e-10)
            for k in range(STEPS):
                o.update(X[:, k], X[:, k + 1])
            st = a.state()
            assert st["r"] == o.r
            np.testing.assert_allclose(st["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    # a plan keeps its handles alive
    with pytest.raises(OdmdError):
        A[0].close()
    for p in plans:
        p.close()
    for m in A + Bm:
        m.close()


def test_graph_replay_equals_eager_launches():
    S = torch.cuda.Stream()
    data = _data()
    E, G = _models(S), _models(S)
    with torch.cuda.stream(S):
        be, bg = _Buffers(data), _Buffers(data)
        pe, pg = be.plans(E), bg.plans(G)
    S.synchronize()
    graphs = []
    for p in pg:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=S):
            p.launch()
        graphs.append(g)
    for k in range(STEPS):
        with torch.cuda.stream(S):
            be.fill(k)
            bg.fill(k)
            pe[k % 2].launch()
            graphs[k % 2].replay()
        S.synchronize()                     # eager work and a wait between replays
        if k % 5 == 4 or k == STEPS - 1:
            for e, g, spec in zip(E, G, SPECS):
                assert _equal(e, g), (k, spec)
    for p in pe + pg:
        p.close()
    for m in E + G:
        m.close()


def test_captured_single_stream_updates_and_prediction():
    """odmd_update and odmd_predict captured directly (no plan): replays
    equal eager calls bit for bit, and the batched entry points refuse
    capture."""
    n, rank, r_max, steps, pred = 20011, 12, 24, 40, 30
    X = synth.random_planted(n, rank, seed=77).snapshots(0, steps + 1)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    S = torch.cuda.Stream()
    e = ODMD(n, r_max, 1e-10, stream=S)
    g = ODMD(n, r_max, 1e-10, stream=S)
    buf = [torch.empty_like(Xd[0]) for _ in range(2)]
    out_g = torch.empty((pred, n), dtype=torch.float64, device="cuda")
    S.synchronize()
    graphs = []
    for j in (0, 1):
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=S):
            g.update(buf[j], buf[1 - j])
        graphs.append(gr)
    gp = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gp, stream=S):
        with pytest.raises(OdmdError):           # refused before anything is enqueued
            update_batch([g], [buf[0]], [buf[1]])
        g.predict(pred, out=out_g)
    for k in range(steps):
        with torch.cuda.stream(S):
            if k == 0:
                buf[0].copy_(Xd[0])
            buf[(k + 1) % 2].copy_(Xd[k + 1])
            e.update(Xd[k], Xd[k + 1])
            graphs[k % 2].replay()
        S.synchronize()
        if k % 7 == 6 or k == steps - 1:
            assert _equal(e, g), k
    with torch.cuda.stream(S):
        out_e = e.predict(pred)
        gp.replay()
    S.synchronize()
    assert torch.equal(out_e, out_g)
    o = O.OnlineDMD(n, r_max, 1e-10)
    for k in range(steps):
        o.update(X[:, k], X[:, k + 1])
    np.testing.assert_allclose(g.state()["sigma"], o.sigma, rtol=1e-11, atol=1e-13 * o.sigma[0])
    e.close()
    g.close()


def test_plan_argument_checks():
    S = torch.cuda.Stream()
    a = ODMD(1000, 8, 1e-10, stream=S)
    b = ODMD(1000, 8, 1e-10, stream=S)
    gen = ODMD(1000, 8, 1e-10, stream=S, pairs="general")
    other = ODMD(1000, 8, 1e-10)                     # another stream
    x = torch.zeros(1000, dtype=torch.float64, device="cuda")
    with pytest.raises(OdmdError):
        Plan([gen], [x], [x])                         # general pairs: per-handle updates only
    with pytest.raises(OdmdError):
        Plan([a, a], [x, x], [x, x])                  # duplicate handle
    with pytest.raises(OdmdError):
        Plan([a, other], [x, x], [x, x])              # handles on different streams
    p = Plan([a, b], [x, x], [x, x])
    with pytest.raises(OdmdError):
        b.close()                                     # held by the plan
    p.close()
    for m in (a, b, gen, other):
        m.close()
