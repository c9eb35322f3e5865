"""Host logic of the serving loop (admission, ordering, batching), on the CPU
with a stand-in backend that records what the scheduler asks of the device."""
import itertools

import numpy as np
import pytest

from paper_2311_18715_amd.serving import Server


class _Ptr:
    _ids = itertools.count(1)

    def __init__(self):
        self._p = next(self._ids) * 4096

    def data_ptr(self):
        return self._p


class FakeTorch:
    uint8 = "uint8"

    class cuda:
        class Event:
            def record(self):
                pass

            def query(self):
                return True

            def synchronize(self):
                pass

        @staticmethod
        def synchronize():
            pass

    @staticmethod
    def empty(nbytes, dtype=None, device=None):
        return _Ptr()


class FakeBackend:
    """ODMD stand-in: state_bytes = 8 n r_max; records each batched update
    and prediction in the order the scheduler issues them."""

    def __init__(self):
        self.log = []
        self.live = set()
        B = self

        class ODMD:
            _next = itertools.count(1)

            def __init__(self, n, r_max, tol, basis="f32", workspace=None, shape=None):
                self.n, self.id, self.shape = n, next(ODMD._next), shape
                self.handle = type("H", (), {"value": self.id})()
                B.live.add(self.id)
                B.models[self.id] = self

            @staticmethod
            def state_bytes(n, r_max, basis="f32", io=None, shape=None):
                # a shape with more workgroups holds more partial-sum records
                return 8 * n * r_max + (0 if shape is None else 1024 * shape[2])

            def predict(self, steps):
                B.log.append(("predict", self.id, steps))
                return np.zeros((steps, self.n))

            def peek_status(self):
                return B.errors.get(self.id, 0)

            def sync(self):
                B.log.append(("sync", self.id))
                B.errors.pop(self.id, None)

            def close(self, wait=True):
                B.live.discard(self.id)

        self.models = {}
        self.errors = {}             # model id -> latched status code
        self.ODMD = ODMD

    @staticmethod
    def status_name(code):
        return {4: "ENONFINITE", 6: "ESEQ"}.get(code, str(code))

    def predict_batch(self, models, steps, outs=None):
        return [m.predict(s) for m, s in zip(models, steps)]

    def handle_array(self, models):
        return np.array([m.handle.value for m in models], dtype=np.uint64)

    def update_batch_ptrs(self, H, xp, yp):
        self.log.append(("batch", tuple(int(h) for h in H), tuple(int(x) for x in xp)))


def make(budget, **kw):
    B = FakeBackend()
    return Server(budget, backend=B, torch_module=FakeTorch, **kw), B


def test_admission_fifo_and_budget():
    S, B = make(budget=8 * 100 * 10 * 2)          # room for two n=100, r_max=10 streams
    assert S.open(1, 100, 10, 1e-8)
    assert S.open(2, 100, 10, 1e-8)
    assert not S.open(3, 100, 10, 1e-8)           # waits
    assert not S.open(4, 50, 10, 1e-8)            # waits behind 3 (FIFO), though it would fit later
    assert S.used == 2 * 8000 and not S.admitted(3)
    S.close(1)
    S.pump()                                      # 1 has no work: released
    S.pump()                                      # 3 admitted into the freed room
    assert S.admitted(3) and not S.admitted(4)
    assert S.used <= S.budget and S.peak_used <= S.budget
    S.close(2)
    S.pump()
    S.pump()
    assert S.admitted(4)
    with pytest.raises(ValueError):
        S.open(9, 10_000, 64, 1e-8)               # larger than the whole budget


def test_rounds_keep_stream_order_and_batch_heads():
    S, B = make(budget=10**9)
    for sid in range(3):
        S.open(sid, 100 + sid, 8, 1e-8)
    xs = {sid: [_Ptr() for _ in range(4)] for sid in range(3)}
    reqs = []
    for k in range(3):
        for sid in range(3):
            reqs.append(S.submit_update(sid, xs[sid][k], xs[sid][k + 1]))
    pr = S.submit_predict(1, 7)
    S.drain()
    batches = [e for e in B.log if e[0] == "batch"]
    # one batched launch per layer: the k-th update of every stream together
    assert len(batches) == 3 and all(len(b[1]) == 3 for b in batches)
    assert S.rounds == 1
    for k, b in enumerate(batches):
        assert b[2] == tuple(xs[sid][k].data_ptr() for sid in range(3))
    # the prediction of stream 1 runs after its three updates
    order = [e[0] for e in B.log]
    assert order.index("predict") == len(order) - 1
    assert all(r.done for r in reqs) and pr.done and pr.out.shape == (7, 101)


def test_late_arrivals_join_the_next_round():
    S, B = make(budget=10**9)
    S.open(0, 10, 4, 1e-8)
    S.open(1, 10, 4, 1e-8)
    p = [_Ptr() for _ in range(4)]
    S.submit_update(0, p[0], p[1])
    S.pump()                                       # first round: stream 0 only
    S.submit_update(1, p[2], p[3])                 # arrives while the first round runs
    S.submit_update(0, p[1], p[2])
    S.pump()                                       # second round: both
    batches = [e for e in B.log if e[0] == "batch"]
    assert [len(b[1]) for b in batches] == [1, 2]


def test_blocked_admission_is_reported():
    S, B = make(budget=8 * 100 * 10)
    S.open(1, 100, 10, 1e-8)
    S.open(2, 100, 10, 1e-8)                      # waits; stream 1 stays open and idle
    S.submit_update(2, _Ptr(), _Ptr())
    with pytest.raises(RuntimeError):
        S.drain()


def test_stream_shapes_reach_the_handles():
    S, B = make(budget=10 ** 9)
    S.open(0, 100, 8, 1e-8)
    S.open(1, 100, 8, 1e-8, shape=(256, 1024, 512))
    assert B.models[S.streams[0].model.id].shape is None
    assert B.models[S.streams[1].model.id].shape == (256, 1024, 512)
    # the budget counts the shaped stream's own bytes
    assert S.used == 2 * 8 * 100 * 8 + 1024 * 512


def test_layers_bound_a_round_and_keep_order():
    """At most max_layers leading updates of a stream per round, then at
    most one prediction; predictions go after the round's update layers."""
    S, B = make(budget=10 ** 9, max_layers=2)
    S.open(0, 10, 4, 1e-8)
    S.open(1, 10, 4, 1e-8)
    p = [_Ptr() for _ in range(7)]
    for k in range(5):
        S.submit_update(0, p[k], p[k + 1])
    S.submit_update(1, p[0], p[1])
    S.submit_predict(1, 3)
    S.submit_update(1, p[1], p[2])               # after the prediction: next round
    S.pump()                                      # round 1: layers 0 and 1, then the prediction
    assert [(e[0], len(e[1]) if e[0] == "batch" else e[1]) for e in B.log] == \
        [("batch", 2), ("batch", 1), ("predict", S.streams[1].model.id)]
    assert len(S.streams[0].queue) == 3 and len(S.streams[1].queue) == 1
    S.drain()
    xs = [b[2] for b in B.log if b[0] == "batch"]
    stream0 = [x[0] for x in xs]                  # stream 0 is first in every batch it is in
    assert stream0 == [p[k].data_ptr() for k in range(5)]
    assert S.rounds == 3


def test_prediction_output_per_round_is_bounded():
    """Predictions past the round's output budget wait for the next round."""
    S, B = make(budget=10 ** 9, pred_bytes=100 * 8 * 10)
    for sid in range(3):
        S.open(sid, 10, 4, 1e-8)
        S.submit_update(sid, _Ptr(), _Ptr())
        S.submit_predict(sid, 100)                # 8000 bytes each: one per round
    S.pump()
    assert sum(1 for e in B.log if e[0] == "predict") == 1
    S.drain()
    assert sum(1 for e in B.log if e[0] == "predict") == 3 and S.rounds == 3


def test_latched_errors_reach_that_rounds_requests():
    """An error the device latched for one stream in a round is reported on
    that stream's requests of the round only, and cleared (odmd_sync)."""
    S, B = make(budget=10 ** 9)
    S.open(0, 10, 4, 1e-8)
    S.open(1, 10, 4, 1e-8)
    p = [_Ptr() for _ in range(4)]
    a = S.submit_update(0, p[0], p[1])
    b = S.submit_update(1, p[2], p[3])
    c = S.submit_predict(1, 2)
    B.errors[S.streams[1].model.id] = 6           # stream 1's update did not chain
    S.drain()
    assert a.done and a.error is None
    assert b.done and b.error == "ESEQ" and c.error == "ESEQ"
    assert ("sync", S.streams[1].model.id) in B.log and not B.errors
    d = S.submit_update(1, p[3], p[0])
    S.drain()
    assert d.done and d.error is None
