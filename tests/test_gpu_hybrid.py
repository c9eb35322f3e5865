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


class _OracleGeneralDMD:
    """The oracle's general-pair online DMD (OnlineDMDF1) behind the
    interface run_hybrid drives (update, predict, eigs, info), for a run of
    the same loop with the CPU oracle in place of the library."""

    class _Info:
        def __init__(self, r):
            self.r = r

    def __init__(self, n, r_max, tol):
        from oracle import odmd_oracle as O
        self.O = O
        self.o = O.OnlineDMDF1(n, r_max, tol)

    def update(self, x, y):
        self.o.update(x.double().cpu().numpy(), y.double().cpu().numpy())

    def info(self):
        return self._Info(self.o.r)

    def eigs(self, vectors=True):
        lam, V = self.o.eigs()
        return lam, (V if vectors else None)

    def predict(self, steps):
        return torch.from_numpy(np.ascontiguousarray(self.o.predict(steps))).cuda()


def test_hybrid_loop_matches_the_loop_on_the_oracle():
    """The hybrid workflow (Sec. 2.1, Fig. 1; residual acceptance of Sec. 2.2)
    run twice on the heat stand-in: once with the library's general-pair
    handle and once with the oracle's general-pair DMD.  Every accept /
    reject decision and every full-order call must be the same, and the
    final states must agree to 1e-9 relative."""
    fom_a, fom_b = HeatFOM(torch, 48, 48), HeatFOM(torch, 48, 48)
    u0 = fom_a.initial_state()
    final, eps, r_max, tol = 240, 1e-8, 16, 1e-10
    ra = run_hybrid(fom_a, u0, final, lambda n: ODMD(n, r_max, tol, pairs="general"),
                    eps_dmd=eps, horizon=32, check_convergence=False)
    rb = run_hybrid(fom_b, u0, final, lambda n: _OracleGeneralDMD(n, r_max, tol),
                    eps_dmd=eps, horizon=32, check_convergence=False)
    assert ra.kinds == rb.kinds
    assert [(k, acc) for k, _, acc in ra.checks] == [(k, acc) for k, _, acc in rb.checks]
    assert ra.fom_calls == rb.fom_calls and ra.fom_calls < final // 2
    # the residuals of the checked predictions differ far less than their
    # distance to the threshold: no decision was close
    ra_res = np.array([res for _, res, _ in ra.checks])
    rb_res = np.array([res for _, res, _ in rb.checks])
    diff = np.abs(ra_res - rb_res)
    margin = np.abs(rb_res - eps)
    assert np.all(diff < 1e-2 * margin)
    err = float(torch.linalg.norm(ra.final - rb.final) / torch.linalg.norm(rb.final))
    print(f"hybrid loop: {ra.fom_calls} full-order calls in {final} steps; residuals "
          f"differ by at most {diff.max():.1e} (smallest margin to eps {margin.min():.1e}); "
          f"final state library vs oracle {err:.2e}")
    assert err < 1e-9
