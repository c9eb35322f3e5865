"""Decision logic of the hybrid FOM/DMD loop on the CPU, with stand-ins that
record what the loop asks of the full-order model and of the DMD."""
import numpy as np

from paper_2311_18715_amd.hybrid import run_hybrid


class FakeFOM:
    """States are scalars in length-1 arrays; the FOM doubles the state.
    A prediction's residual is read from a table keyed by the step."""

    def __init__(self, bad_steps):
        self.n = 1
        self.bad = set(bad_steps)
        self.calls = []

    def step(self, u, k):
        self.calls.append(k)
        return u * 2.0

    def residual(self, u_prev, u_next, k):
        return 1.0 if k in self.bad else 0.0


class FakeDMD:
    def __init__(self, n, eig_seq=None):
        self.pairs = []
        self.eig_seq = eig_seq

    class _I:
        r = 1

    def info(self):
        return self._I()

    def update(self, x, y):
        self.pairs.append((float(x[0]), float(y[0])))

    def predict(self, steps):
        y = self.pairs[-1][1]
        return np.array([[y * 3.0 ** (j + 1)] for j in range(steps)])   # distinguishable states

    def eigs(self, vectors=False):
        k = len(self.pairs)
        return (np.array([1.0 + (self.eig_seq[k - 1] if self.eig_seq else 1.0 / k)]), None)


def test_accept_reject_and_unchained_updates():
    fom = FakeFOM(bad_steps={3, 4})
    made = []

    def make(n):
        made.append(FakeDMD(n))
        return made[-1]

    r = run_hybrid(fom, np.array([1.0]), 8, make, eps_dmd=0.5, horizon=4, check_convergence=False)
    d = made[0]
    # step 0: FOM (initialises); steps 1, 2 accepted; 3 and 4 rejected -> FOM;
    # 5, 6, 7 accepted
    assert r.kinds == ["fom", "dmd", "dmd", "fom", "fom", "dmd", "dmd", "dmd"]
    assert fom.calls == [0, 3, 4]
    assert r.fom_calls == 3
    # the DMD sees only FOM pairs; the second one starts from an accepted
    # prediction (unchained): x = 2 * 3 * 3 = 18, not the previous y = 2
    assert d.pairs == [(1.0, 2.0), (18.0, 36.0), (36.0, 72.0)]
    # accepted states are consumed in rollout order from the last FOM snapshot
    assert float(r.final[0]) == 72.0 * 27.0
    assert abs(r.fom_fraction_avoided - 5.0 / 8.0) < 1e-15


def test_convergence_exit_predicts_final_state():
    fom = FakeFOM(bad_steps=set(range(100)))       # every prediction rejected
    made = []

    def make(n):
        made.append(FakeDMD(n, eig_seq=[0.5, 0.25, 0.25, 0.25, 0.25]))
        return made[-1]

    r = run_hybrid(fom, np.array([1.0]), 50, make, eps_dmd=0.5, horizon=4,
                   conv_eps=1e-12, conv_window=3)
    # eigenvalue unchanged over updates 3, 4, 5 -> converged after step 5
    assert r.converged_at == 5
    assert r.fom_calls == 5
    assert r.kinds[:5] == ["fom"] * 5 and r.kinds[5:] == ["skip"] * 45
    # final state: rollout from the last FOM snapshot (2^5 = 32) to step 50
    assert float(r.final[0]) == 32.0 * 3.0 ** 45
