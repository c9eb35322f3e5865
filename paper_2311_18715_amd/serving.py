"""Continuous-batching request loop over many online-DMD streams.

Many concurrent simulations each feed one stream: snapshot pairs to append
(updates, Sec. 2.3) and requests for predicted states (the O(N r) rollout).
Every stream's state (stored basis, sigma, A~, ...) stays resident on the
device.  A stream is admitted when its device bytes (odmd_state_bytes) fit
in the memory budget; otherwise it waits, in arrival order, until closed
streams free enough.

Each scheduling round takes, from every admitted stream with queued
requests, its leading updates (up to ``max_layers``) and a prediction that
follows them: the k-th updates of the streams form layer k, one batched
update each (odmd_update_batch: one pass launch per group of like streams,
one small-state launch for all), and all the round's predictions follow as
one batched prediction.  Everything goes to one device stream in that
order, so a stream's requests run strictly in order and every result equals
the one the stream would get alone (the batched launches are bitwise equal
to per-stream launches).
Requests that arrive while a round runs on the device join a later round.

The device work of a round is recorded with one event; a request's latency
runs from its submission to the host's observation that its round finished.
Errors the device latches for a stream in a round (an update skipped for a
non-finite or unchained pair, a prediction of an empty model, an iteration
cap) are read then, without a device call, and reported on that round's
requests of the stream (the error is then cleared).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    """One update or prediction request.  ``out`` holds the predicted states
    (steps x n device tensor) of a prediction once ``done``."""
    kind: str                       # "update" | "predict"
    sid: int
    x: object = None
    y: object = None
    steps: int = 0
    out: object = None
    t_submit: float = 0.0
    t_done: float = 0.0
    done: bool = False
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


@dataclasses.dataclass
class _Stream:
    sid: int
    n: int
    r_max: int
    tol: float
    basis: str
    bytes: int
    model: object = None
    workspace: object = None
    queue: Deque[Request] = dataclasses.field(default_factory=collections.deque)
    closing: bool = False
    shape: Optional[tuple] = None     # pass launch shape; None: the library default


class Server:
    """Request loop with HBM-budget admission and continuous batching.

    budget_bytes bounds the sum of the admitted streams' device state
    (odmd_state_bytes); prediction outputs are not part of it: with
    keep_outputs (the default) they are allocated per request, without it
    they are views of max_inflight + 1 arenas of pred_bytes each, allocated
    when the server starts (40 GB with the defaults).  ``backend`` is the module that provides ODMD,
    handle_array and update_batch_ptrs (the library binding; a stand-in can
    be passed for host-only tests of the scheduling logic)."""

    def __init__(self, budget_bytes: int, backend=None, torch_module=None,
                 clock: Callable[[], float] = time.perf_counter, max_layers: int = 8,
                 max_inflight: int = 4, keep_outputs: bool = True, pred_bytes: int = 8 << 30):
        if backend is None:
            from paper_2311_18715_amd import odmd as backend
        if torch_module is None:
            import torch as torch_module
        if max_layers < 1:
            raise ValueError("max_layers must be at least 1")
        self.B, self.torch, self.clock = backend, torch_module, clock
        self.max_layers = int(max_layers)
        # rounds in flight before pump() waits for the oldest (bounds the
        # prediction outputs held on the device); keep_outputs=False drops a
        # prediction's states once its round is done (load generators)
        self.max_inflight = max(1, int(max_inflight))
        self.keep_outputs = bool(keep_outputs)
        self.pred_bytes = int(pred_bytes)    # prediction output per round (FP64 bound)
        # keep_outputs=False: a round's prediction outputs are views of one
        # of max_inflight + 1 arenas of pred_bytes (a round reuses the arena
        # of a round that has finished), instead of an allocation each,
        # which under memory churn made the allocator synchronise
        self._arenas: List = []
        if not self.keep_outputs:            # allocated up front, not inside the request loop
            self._arenas = [self.torch.empty(self.pred_bytes, dtype=self.torch.uint8, device="cuda")
                            for _ in range(self.max_inflight + 1)]
        self.active: Dict[int, _Stream] = {}    # admitted streams with queued work or closing
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self.streams: Dict[int, _Stream] = {}
        self.waiting: Deque[_Stream] = collections.deque()
        self.inflight: List = []          # (event, [requests], {sid: stream}) per round
        self.completed: List[Request] = []
        self.rounds = 0
        self.batch_sizes: List[int] = []
        # host seconds spent in pump() and, inside it, in the library's
        # batched update and prediction calls (which also wait when their
        # staging buffers are still in use by queued device work)
        self.host_s = {"pump": 0.0, "update_batch": 0.0, "predict_batch": 0.0}

    # ---- streams -------------------------------------------------------
    def open(self, sid: int, n: int, r_max: int, tol: float, basis: str = "f32",
             shape=None) -> bool:
        """Register a stream; returns True if it was admitted at once.

        shape: (threads, rows_per_block, max_blocks) of the stream's pass
        (a tuned one), or None for the library's default."""
        if sid in self.streams:
            raise ValueError(f"stream {sid} already open")
        kw = {} if shape is None else {"shape": tuple(shape)}
        nbytes = int(self.B.ODMD.state_bytes(n, r_max, basis, **kw))
        if nbytes <= 0 or nbytes > self.budget:
            raise ValueError(f"stream {sid} cannot fit the budget ({nbytes} bytes)")
        st = _Stream(sid, int(n), int(r_max), float(tol), basis, nbytes,
                     shape=None if shape is None else tuple(shape))
        self.streams[sid] = st
        self.waiting.append(st)
        self._admit()
        return st.model is not None

    def close(self, sid: int) -> None:
        """Close a stream once its queued requests are served."""
        st = self.streams[sid]
        st.closing = True
        if st.model is not None:
            self.active[sid] = st

    def admitted(self, sid: int) -> bool:
        return self.streams[sid].model is not None

    def _admit(self) -> None:
        while self.waiting and self.used + self.waiting[0].bytes <= self.budget:
            st = self.waiting.popleft()
            ws = self.torch.empty(st.bytes + 256, dtype=self.torch.uint8, device="cuda")
            st.workspace = ws
            kw = {} if st.shape is None else {"shape": st.shape}
            st.model = self.B.ODMD(st.n, st.r_max, st.tol, basis=st.basis, workspace=ws, **kw)
            self.used += st.bytes
            self.peak_used = max(self.peak_used, self.used)
            if st.queue or st.closing:
                self.active[st.sid] = st

    def _release(self, st: _Stream) -> None:
        # no wait: the workspace goes back to torch's allocator on the
        # handles' stream, which orders its reuse after the queued work
        st.model.close(wait=False)
        st.model = None
        st.workspace = None
        self.used -= st.bytes
        del self.streams[st.sid]
        self.active.pop(st.sid, None)

    # ---- requests ------------------------------------------------------
    def _enqueue(self, r: Request) -> Request:
        st = self.streams[r.sid]
        st.queue.append(r)
        if st.model is not None:
            self.active[r.sid] = st
        return r

    def submit_update(self, sid: int, x, y) -> Request:
        return self._enqueue(Request("update", sid, x=x, y=y, t_submit=self.clock()))

    def submit_predict(self, sid: int, steps: int) -> Request:
        return self._enqueue(Request("predict", sid, steps=int(steps), t_submit=self.clock()))

    # ---- scheduling ----------------------------------------------------
    def pump(self) -> int:
        """One round: for every admitted stream with queued requests, its
        leading updates (at most max_layers of them) and, if one follows, a
        prediction.  The k-th updates of the streams form layer k (one
        batched launch per layer); the predictions go last, in one batched
        call (one coefficient launch for all), each after its own stream's
        updates.  Predictions past pred_bytes of output in the
        round wait for the next one.  Returns the number of requests
        launched."""
        t_pump = self.clock()
        self.poll()
        while len(self.inflight) >= self.max_inflight:
            self.inflight[0][0].synchronize()
            self.poll()
        self._admit()
        layers: List[list] = []              # per layer: [(st, r)] updates
        preds: List[tuple] = []
        pred_bytes = 0
        members: Dict[int, _Stream] = {}
        taken: Dict[int, int] = {}
        for st in list(self.active.values()):
            if not st.queue:
                if st.closing:
                    self._release(st)
                else:
                    del self.active[st.sid]
                continue
            j = 0
            q = st.queue
            while j < len(q) and j < self.max_layers and q[j].kind == "update":
                if j == len(layers):
                    layers.append([])
                layers[j].append((st, q[j]))
                j += 1
            if j < len(q) and q[j].kind == "predict":
                nb = q[j].steps * st.n * 8
                if not preds or pred_bytes + nb <= self.pred_bytes:
                    preds.append((st, q[j]))
                    pred_bytes += nb
                    j += 1
            if j:
                members[st.sid] = st
                taken[st.sid] = j
        launched = []
        for ups in layers:
            H = self.B.handle_array([st.model for st, _ in ups])
            xp = np.fromiter((r.x.data_ptr() for _, r in ups), dtype=np.uint64, count=len(ups))
            yp = np.fromiter((r.y.data_ptr() for _, r in ups), dtype=np.uint64, count=len(ups))
            t = self.clock()
            self.B.update_batch_ptrs(H, xp, yp)
            self.host_s["update_batch"] += self.clock() - t
            launched.extend(r for _, r in ups)
            self.batch_sizes.append(len(ups))
        if preds:
            t = self.clock()
            try:
                outs = self.B.predict_batch([st.model for st, _ in preds],
                                            [r.steps for _, r in preds],
                                            **self._arena_outs(preds))
            except Exception as e:
                outs = [None] * len(preds)
                for _, r in preds:
                    r.error = str(e)
            self.host_s["predict_batch"] += self.clock() - t
            for (_, r), o in zip(preds, outs):
                r.out = o
            launched.extend(r for _, r in preds)
        for sid, j in taken.items():
            q = members[sid].queue
            for _ in range(j):
                q.popleft()
        if launched:
            ev = self.torch.cuda.Event()
            ev.record()
            self.inflight.append((ev, launched, members))
            self.rounds += 1
        self.host_s["pump"] += self.clock() - t_pump
        return len(launched)

    def _arena_outs(self, preds) -> dict:
        """outs= for predict_batch from this round's arena, or {} (new
        tensors) when outputs are kept or the round's outputs exceed it."""
        if self.keep_outputs:
            return {}
        sizes = [(r.steps, st.n, st.model.dtype) for st, r in preds]
        nbytes = [s * n * (8 if dt == self.torch.float64 else 4) for s, n, dt in sizes]
        offs, o = [], 0
        for b in nbytes:
            offs.append(o)
            o += (b + 255) // 256 * 256
        if o > self.pred_bytes:
            return {}
        k = self.rounds % (self.max_inflight + 1)
        while len(self._arenas) <= k:
            self._arenas.append(self.torch.empty(self.pred_bytes, dtype=self.torch.uint8, device="cuda"))
        a = self._arenas[k]
        return {"outs": [a[o:o + b].view(dt).view(s, n) for o, b, (s, n, dt) in zip(offs, nbytes, sizes)]}

    def poll(self) -> None:
        """Mark the requests of finished rounds done, with the errors their
        streams latched on the device in that round."""
        keep = []
        now = None
        for ev, reqs, members in self.inflight:
            if ev.query():
                now = now if now is not None else self.clock()
                bad = {}
                for sid, st in members.items():
                    if st.model is None:
                        continue
                    code = st.model.peek_status()
                    if code:
                        bad[sid] = self.B.status_name(code)
                        try:
                            st.model.sync()          # clears the latched error
                        except Exception:
                            pass
                for r in reqs:
                    r.t_done, r.done = now, True
                    if r.sid in bad and r.error is None:
                        r.error = bad[r.sid]
                    if not self.keep_outputs:
                        r.out = None
                    r.x = r.y = None
                    self.completed.append(r)
            else:
                keep.append((ev, reqs, members))
        self.inflight = keep

    def idle(self) -> bool:
        return not self.inflight and not self.waiting and \
            all(not st.queue for st in self.active.values())

    def drain(self) -> None:
        """Run rounds until every queued request is done.  Raises if queued
        work waits for admission that no open stream will ever make room
        for (the caller must close streams)."""
        while True:
            launched = self.pump()
            if self.idle():
                break
            if not any(st.queue for st in self.active.values()):
                # only waits for the device, or for admission, are left
                self.torch.cuda.synchronize()
                self.poll()
                if launched == 0 and not self.inflight:
                    self.pump()        # releases closing streams, admits waiting ones
                    if not any(st.queue for st in self.active.values()) and self.waiting:
                        raise RuntimeError("admission blocked: the budget is held by open "
                                           "streams with no queued work; close some")
        self.torch.cuda.synchronize()
        self.poll()

    def latency_us(self, kind: str = "update") -> Dict[str, float]:
        lat = np.array([r.latency for r in self.completed if r.kind == kind]) * 1e6
        if lat.size == 0:
            return {"p50": float("nan"), "p99": float("nan"), "count": 0}
        return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                "count": int(lat.size)}
