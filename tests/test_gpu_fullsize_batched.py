"""The batched and serving forms at their full workload sizes.

Batched mix: 256 streams, n log-uniform in [1e4, 1e6], planted rank in
{6..30}, r_max in {16..64}, FP32 storage with the tuned launch shapes, all
advanced together by odmd_update_batch (the benchmark's launch
configuration).  Sampled streams (the smallest, the largest, and the first
whose planted rank exceeds its cap) must equal their own per-stream
updates bit for bit and match the FP64 oracle run on the same (FP32)
snapshots within FP32 storage error.

Serving mix: 1024 streams, n log-uniform in [1e4, 2e6], r_max in
{16, 32, 64}, FP32 or BF16 storage, under a 200 GB budget (everything
admitted) and a 20 GB budget (admission binds); sampled streams'
predictions must equal those of the stream run alone, bit for bit.
"""
import math
import sys

import numpy as np
import pytest

from oracle import odmd_oracle as O
from paper_2311_18715_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd import autotune
    from paper_2311_18715_amd.odmd import ODMD, handle_array, update_batch_ptrs
    from paper_2311_18715_amd.serving import Server


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def test_batched_mix_full_size():
    steps, chunk = 60, 20
    descs = synth.batched_streams(256)
    table = autotune.load_table()
    shapes = [autotune.lookup(n, rm, "f32", objective="throughput", table=table)
              for (n, _, rm, _) in descs]
    ns = [d[0] for d in descs]
    trunc = next(i for i, (_, rank, rm, _) in enumerate(descs) if rank > rm)
    sample = sorted({int(np.argmin(ns)), int(np.argmax(ns)), trunc})
    _say(f"batched mix: 256 streams, {sum(ns)} rows, sampled {sample}")
    gens = [synth.DevicePlanted(torch, n, rank, seed) for (n, rank, _, seed) in descs]
    models = [ODMD(n, rm, 1e-8, basis="f32", shape=sh) for (n, _, rm, _), sh in zip(descs, shapes)]
    alone = {i: ODMD(descs[i][0], descs[i][2], 1e-8, basis="f32", shape=shapes[i]) for i in sample}
    H = handle_array(models)
    nb = np.array(ns, dtype=np.uint64) * np.uint64(4)
    host = {i: [] for i in sample}
    for k0 in range(0, steps, chunk):
        X = [g.chunk(k0, chunk + 1).float() for g in gens]
        base = np.array([x.data_ptr() for x in X], dtype=np.uint64)
        for k in range(chunk):
            update_batch_ptrs(H, base + np.uint64(k) * nb, base + np.uint64(k + 1) * nb)
            for i in sample:
                alone[i].update(X[i][k], X[i][k + 1])
        for i in sample:
            host[i].append(X[i][:chunk + (k0 + chunk == steps)].double().cpu().numpy())
        torch.cuda.synchronize()
        del X
        _say(f"batched mix: {k0 + chunk} steps")
    for g in models:
        g.sync()                      # no latched error in any stream
    for (n, rank, rm, _), g in zip(descs, models):
        st = g.state()
        # at most r_max directions; above the FP32 resolution floor at most
        # the planted rank (FP32 rounding of the snapshots may add
        # directions near the 1e-8 tolerance)
        assert 1 <= st["r"] <= rm
        assert int(np.sum(st["sigma"] >= 2.0 ** -20 * st["sigma"][0])) <= min(rank, rm)
    for i in sample:
        n, rank, rm, _ = descs[i]
        a, b = models[i].state(), alone[i].state()
        for key in ("sigma", "atilde", "p_y", "C", "w"):
            assert np.array_equal(a[key], b[key]), (i, key)
        assert torch.equal(models[i].basis_matrix(), alone[i].basis_matrix()), i
        Xh = np.concatenate(host[i], axis=0).T            # (n, steps + 1), the FP32 snapshots
        o = O.OnlineDMD(n, rm, 1e-8)
        for k in range(steps):
            o.update(Xh[:, k], Xh[:, k + 1])
        r = min(a["r"], o.r)
        # FP32 storage perturbs the snapshot matrix by about 1e-7 of its norm;
        # singular values move by no more than that (Weyl)
        err = np.max(np.abs(a["sigma"][:r] - o.sigma[:r])) / o.sigma[0]
        _say(f"stream {i} (n={n}, rank {rank}, r_max {rm}): r {a['r']} / oracle {o.r}, "
             f"sigma error {err:.2e}")
        assert err < 1e-5, i
        # eigenvalues within the FP32 tolerance (1e-4 relative, |lambda| >=
        # 1e-2 max|lambda|) for the model truncated at the FP32 resolution
        # floor, sigma_i >= 2^-20 sigma_1 (the full ranks may differ by
        # rounding-decided directions near the tolerance)
        k = int(np.sum(a["sigma"] >= 2.0 ** -20 * a["sigma"][0]))
        ko = int(np.sum(o.sigma >= 2.0 ** -20 * o.sigma[0]))
        assert k == ko and abs(a["r"] - o.r) <= 2, i
        lam = np.linalg.eigvals(a["atilde"][:k, :k])
        lo = np.linalg.eigvals(o.atilde()[:k, :k])
        big = lo[np.abs(lo) >= 1e-2 * np.abs(lo).max()]
        eerr = np.max(np.abs(O.match_eigs(big, lam) - big) / np.abs(big))
        _say(f"stream {i}: eigenvalues above the FP32 floor ({k}) vs oracle {eerr:.2e}")
        assert eerr < 1e-4, i
    for g in list(alone.values()) + models:
        g.close()


def _serving_specs(count=1024, seed=231118715 + 11):
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(1e4), math.log(2e6)))))
        out.append((n, int(g.integers(6, 31)), int(g.choice([16, 32, 64])),
                    "bf16" if g.random() < 0.5 else "f32", seed + 100 + i))
    return out


@pytest.mark.parametrize("budget_gb", [200, 20])
def test_serving_mix_full_size(budget_gb):
    updates, pred_steps = 12, 100
    specs = _serving_specs()
    _say(f"serving mix: 1024 streams, {sum(s[0] for s in specs)} rows, budget {budget_gb} GB")
    data = []
    for (n, rank, _, _, seed) in specs:
        gen = synth.DevicePlanted(torch, n, rank, seed, dtype=torch.float32)
        data.append(gen.chunk(0, updates + 1))
        del gen
    torch.cuda.synchronize()
    sample = [0, 1, int(np.argmax([s[0] for s in specs]))]
    budget = budget_gb << 30
    need = [ODMD.state_bytes(n, rm, basis) for (n, _, rm, basis, _) in specs]
    S = Server(budget)
    for i, (n, _, rm, basis, _) in enumerate(specs):
        S.open(i, n, rm, 1e-8, basis)
    admitted = sum(S.admitted(i) for i in range(len(specs)))
    _say(f"serving mix: state {sum(need) / 2 ** 30:.1f} GB, admitted at once {admitted}")
    if sum(need) <= budget:
        assert admitted == len(specs)
    else:
        assert admitted < len(specs)                   # admission binds
    # requests come from admitted, unfinished streams (a simulation sends
    # snapshots once it holds a slot); rounds run every 64 requests, and
    # whenever no admitted stream is left to send
    rng = np.random.default_rng(5)
    pos = [0] * len(specs)
    preds = {}
    live = set(range(len(specs)))
    adm = sorted(i for i in live if S.admitted(i))
    j = 0
    while live:
        if not adm:
            S.pump()
            torch.cuda.synchronize()
            adm = sorted(i for i in live if S.admitted(i))
            continue
        i = adm[int(rng.integers(len(adm)))]
        S.submit_update(i, data[i][pos[i]], data[i][pos[i] + 1])
        pos[i] += 1
        if pos[i] == updates:
            if i in sample:
                preds[i] = S.submit_predict(i, pred_steps)
            S.close(i)
            live.discard(i)
            adm.remove(i)
        j += 1
        if j % 64 == 0:
            S.pump()
            adm = sorted(i for i in live if S.admitted(i))
    S.drain()
    assert S.peak_used <= budget
    assert S.latency_us("update")["count"] == updates * len(specs)
    assert max(S.batch_sizes) > 1
    for i in sample:
        n, _, rm, basis, _ = specs[i]
        r = preds[i]
        assert r.done and r.error is None, i
        g = ODMD(n, rm, 1e-8, basis=basis)
        for k in range(updates):
            g.update(data[i][k], data[i][k + 1])
        ref = g.predict(pred_steps)
        g.sync()
        assert torch.equal(r.out, ref), f"stream {i} differs alone vs in the mix"
        g.close()
    _say(f"serving mix: {len(S.batch_sizes)} rounds, mean batch {np.mean(S.batch_sizes):.0f}")
