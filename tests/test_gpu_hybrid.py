"""Hybrid FOM/DMD time stepping on the GPU (the workflow of Sec. 2.1):
the general-pair DMD replaces most full-order steps of a periodically
forced implicit heat equation, and the hybrid trajectory stays on the
full-order one."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2311_18715_amd.hybrid import HeatFOM, run_hybrid
    from paper_2311_18715_amd.odmd import ODMD


@pytest.mark.parametrize("nx,ny", [(48, 48), (400, 400)])
def test_hybrid_tracks_fom_and_avoids_calls(nx, ny):
    fom = HeatFOM(torch, nx, ny)
    u0 = fom.initial_state()
    final = 240
    # full-order reference
    ref = u0
    for k in range(final):
        ref = fom.step(ref, k)
    eps = 1e-8
    r = run_hybrid(fom, u0, final, lambda n: ODMD(n, 16, 1e-10, pairs="general"),
                   eps_dmd=eps, horizon=32, check_convergence=False)
    assert r.kinds[0] == "fom"
    assert all((res <= eps) == acc for _, res, acc in r.checks)
    assert sum(acc for _, _, acc in r.checks) == r.kinds.count("dmd")
    accepted = r.kinds.count("dmd")
    assert accepted + r.fom_calls == final
    assert r.fom_fraction_avoided > 0.5, r.fom_fraction_avoided
    err = float(torch.linalg.norm(r.final - ref) / torch.linalg.norm(ref))
    assert err < 1e-6, err


def test_hybrid_convergence_exit():
    fom = HeatFOM(torch, 48, 48)
    u0 = fom.initial_state()
    final = 400
    ref = u0
    for k in range(final):
        ref = fom.step(ref, k)
    r = run_hybrid(fom, u0, final, lambda n: ODMD(n, 16, 1e-10, pairs="general"),
                   eps_dmd=1e-30, horizon=8, conv_eps=1e-9, conv_window=5)
    # every prediction is refused (eps below rounding), so the exit comes from
    # the eigenvalue test, well before the final step
    assert r.converged_at is not None and r.converged_at < final // 2
    err = float(torch.linalg.norm(r.final - ref) / torch.linalg.norm(ref))
    assert err < 1e-6, err
