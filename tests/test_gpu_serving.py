"""Serving loop on the GPU: streams of different size, rank cap and storage
type arrive interleaved, wait for admission under a memory budget, share
batched rounds, and each one's predictions equal, bit for bit, those of the
same stream run alone through plain updates."""
import numpy as np
import pytest

from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.odmd import ODMD
    from paper_2311_18715_amd.serving import Server

SPECS = [  # (n, planted rank, r_max, basis, updates)
    (3000, 6, 16, "f32", 60), (777, 10, 12, "f64", 45), (20000, 30, 64, "f32", 70),
    (5000, 12, 40, "f64", 50), (12345, 20, 24, "f32", 65), (64, 4, 8, "f64", 30),
    (9000, 26, 33, "f32", 55), (40000, 8, 32, "f32", 40),
]
PRED_AT = {0: [20], 2: [35], 3: [10, 30], 6: [50]}   # predictions after these updates
STEPS = 9


def streams():
    out = []
    for i, (n, rank, rmax, basis, m) in enumerate(SPECS):
        s = synth.random_planted(n, rank, seed=4000 + i, noise=1e-7)
        X = s.snapshots(0, m + 1)
        dt = torch.float64 if basis == "f64" else torch.float32
        out.append(torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dt))
    return out


def script(seed=5):
    """Interleaved arrival order: (stream, update index or 'predict')."""
    rng = np.random.default_rng(seed)
    pos = [0] * len(SPECS)
    events = []
    while any(pos[i] < SPECS[i][4] for i in range(len(SPECS))):
        i = int(rng.integers(len(SPECS)))
        if pos[i] >= SPECS[i][4]:
            continue
        events.append((i, pos[i]))
        pos[i] += 1
        if pos[i] in PRED_AT.get(i, []):
            events.append((i, "predict"))
    for i in range(len(SPECS)):
        events.append((i, "predict"))          # a final prediction per stream
    return events


def test_mix_equals_alone_under_admission():
    data = streams()
    events = script()
    # alone: each stream by itself, plain per-stream updates
    alone = {}
    for i, (n, _, rmax, basis, m) in enumerate(SPECS):
        g = ODMD(n, rmax, 1e-8, basis=basis)
        outs = []
        for k in range(m):
            g.update(data[i][k], data[i][k + 1])
            if k + 1 in PRED_AT.get(i, []):
                outs.append(g.predict(STEPS).cpu().numpy())
        outs.append(g.predict(STEPS).cpu().numpy())
        g.sync()
        alone[i] = outs
        g.close()
    # mix: all streams through the server; the budget holds about half of them
    need = [ODMD.state_bytes(n, rmax, basis) for (n, _, rmax, basis, _) in SPECS]
    budget = int(0.5 * sum(need)) + max(need)
    S = Server(budget)
    for i, (n, _, rmax, basis, _) in enumerate(SPECS):
        S.open(i, n, rmax, 1e-8, basis)
    assert any(not S.admitted(i) for i in range(len(SPECS)))   # admission binds
    preds = {i: [] for i in range(len(SPECS))}
    for j, (i, what) in enumerate(events):
        if what == "predict":
            preds[i].append(S.submit_predict(i, STEPS))
        else:
            S.submit_update(i, data[i][what], data[i][what + 1])
        if len(preds[i]) == len(PRED_AT.get(i, [])) + 1:
            S.close(i)                          # its last request is queued
        if j % 3 == 2:
            S.pump()                             # requests keep arriving between rounds
    S.drain()
    assert S.peak_used <= budget
    assert max(S.batch_sizes) > 1                # rounds really mixed streams
    for i in range(len(SPECS)):
        got = [r.out.cpu().numpy() for r in preds[i]]
        assert all(r.done and r.error is None for r in preds[i])
        assert len(got) == len(alone[i])
        for a, b in zip(got, alone[i]):
            assert np.array_equal(a, b), f"stream {i} differs alone vs in the mix"
    lat = S.latency_us("update")
    assert lat["count"] == sum(s[4] for s in SPECS)


def test_device_errors_reach_the_requests_of_their_stream():
    """A non-chaining pair of one stream in a mixed round: the device skips
    it and latches ESEQ; that stream's request of the round carries the
    error, the other streams' requests do not, and later rounds are clean.
    odmd_peek_status sees the latched bits without a device call."""
    data = streams()[:3]
    S = Server(10 ** 10, max_layers=1)
    for i in range(3):
        n, _, rmax, basis, _ = SPECS[i]
        S.open(i, n, rmax, 1e-8, basis)
    first = [S.submit_update(i, data[i][0], data[i][1]) for i in range(3)]
    S.drain()
    assert all(r.done and r.error is None for r in first)
    ok0 = S.submit_update(0, data[0][1], data[0][2])
    bad = S.submit_update(1, data[1][5], data[1][6])      # does not chain to x_1
    ok2 = S.submit_update(2, data[2][1], data[2][2])
    S.drain()
    assert ok0.error is None and ok2.error is None
    assert bad.error == "ESEQ"
    later = S.submit_update(1, data[1][1], data[1][2])    # the chain resumes
    S.drain()
    assert later.done and later.error is None
    # peek: latched by a finished update, cleared by sync
    n, _, rmax, basis, _ = SPECS[1]
    g = ODMD(n, rmax, 1e-8, basis=basis)
    g.update(data[1][0], data[1][1])
    g.update(data[1][3], data[1][4])                      # unchained
    torch.cuda.synchronize()
    assert g.peek_status() == 6                            # ESEQ
    with pytest.raises(Exception):
        g.sync()
    assert g.peek_status() == 0
    g.close()


def test_release_without_waiting_reuses_memory_safely():
    """Handles on caller workspaces released without waiting (odmd_release)
    while their updates are still queued; their workspaces go back to
    torch's allocator at once and their pinned words to the library's pool.
    Handles made right after (reusing both) match a handle made on a quiet
    device bit for bit."""
    n, rank, rmax, m = 20011, 8, 16, 30
    s = synth.random_planted(n, rank, seed=4321, noise=1e-7)
    Xd = torch.from_numpy(np.ascontiguousarray(s.snapshots(0, m + 1).T)).cuda()
    ref = ODMD(n, rmax, 1e-8)
    for k in range(m):
        ref.update(Xd[k], Xd[k + 1])
    lam_ref = ref.eigs(vectors=False)[0]
    sig_ref = ref.state()["sigma"]
    ref.close()
    nbytes = ODMD.state_bytes(n, rmax, "f64")
    for _ in range(3):
        hs = []
        for i in range(40):
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            g = ODMD(n, rmax, 1e-8, workspace=ws)
            for k in range(6):
                g.update(Xd[k], Xd[k + 1])
            hs.append(g)
        for g in hs:
            g.close(wait=False)               # their updates are still queued
        del hs, g, ws
        outs = []
        for i in range(4):
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            g = ODMD(n, rmax, 1e-8, workspace=ws)
            for k in range(m):
                g.update(Xd[k], Xd[k + 1])
            outs.append((g.eigs(vectors=False)[0], g.state()["sigma"]))
            g.close(wait=False)
        for lam, sig in outs:
            assert np.array_equal(lam, lam_ref) and np.array_equal(sig, sig_ref)


def test_prediction_arenas_hold_the_same_states():
    """keep_outputs=False: a round's predictions are written into views of
    one of the server's preallocated arenas (rotated over max_inflight + 1
    rounds).  Taken right after their round, they equal the predictions of
    the same streams run alone, bit for bit, round after round (every arena
    reused several times); a prediction larger than an arena gets its own
    tensor."""
    import types
    from paper_2311_18715_amd import odmd as B
    data = streams()[:4]
    calls = []

    def predict_batch(models, steps, outs=None):
        res = B.predict_batch(models, steps, outs=outs)
        calls.append((outs is not None, list(models), res))
        return res

    proxy = types.SimpleNamespace(**{k: getattr(B, k) for k in dir(B) if not k.startswith("__")})
    proxy.predict_batch = predict_batch
    # arenas of 4 MB: the four streams' 9-state predictions (about 1.3 MB)
    # fit; a 64-state prediction of the n = 20000 stream (5.1 MB) does not
    S = Server(10 ** 10, backend=proxy, keep_outputs=False, max_inflight=2, pred_bytes=4 << 20)
    twins = []
    for i in range(4):
        n, _, rmax, basis, _ = SPECS[i]
        S.open(i, n, rmax, 1e-8, basis)
        twins.append(ODMD(n, rmax, 1e-8, basis=basis))
    for k in range(12):
        for i in range(4):
            S.submit_update(i, data[i][k], data[i][k + 1])
            S.submit_predict(i, STEPS)
            twins[i].update(data[i][k], data[i][k + 1])
        before = len(calls)
        S.pump()
        torch.cuda.synchronize()
        assert len(calls) == before + 1
        used_arena, models, outs = calls[-1]
        assert used_arena and len(outs) == 4
        got = [o.clone() for o in outs]
        for i, g in enumerate(got):
            assert torch.equal(g, twins[i].predict(STEPS)), f"round {k}, stream {i}"
    S.submit_predict(2, 64)
    S.pump()
    torch.cuda.synchronize()
    used_arena, models, outs = calls[-1]
    assert not used_arena and torch.equal(outs[0], twins[2].predict(64))
    S.drain()
    assert all(r.done and r.error is None and r.out is None for r in S.completed)
    for t in twins:
        t.close()
