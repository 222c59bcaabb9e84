"""Continuous-batching request loop for Wilson-loop requests.

A request is one model (hopping list) with a k-plane, a band window and a
kind (plain, spin-resolved or nested Wilson loop, or the Berry flux per
plaquette of the occupied space or of its spin sectors). Requests arrive at any
time. The engine

* admits a waiting request as soon as its device footprint (resident
  eigenvectors, one eigensolver chunk of Hamiltonians, the eigensolver's and
  the loop stage's workspace) fits the HBM budget next to the requests already
  admitted, first come first served with skip-ahead for smaller requests;
* keeps every admitted request's eigenvectors resident on the device until
  its loop stage has run;
* packs the pending k-points of the admitted requests that share (N, bands,
  precision) into one batched eigensolver launch (continuous batching: a
  request that arrives while others run joins at the next launch);
* runs work on several GPU lanes at once: a lane is a host thread with a
  library context and a stream of its own, so launches of different sizes
  (different keys), and loop stages, overlap on the device; one key is
  diagonalized on one lane at a time;
* runs a request's loop stage as soon as all its k-points are diagonalized
  (on whichever lane is free: it waits on the eigensolver's stream event),
  frees its memory and records its latency;
* stops a request that is cancelled (``Engine.cancel``) or outlives its
  ``timeout`` (seconds from submission): a waiting one is never admitted, an
  admitted one gets no further eigensolver launches and no loop stage, and
  its memory is freed once its launch in flight (if any) has ended; either
  way the request completes with ``RequestCancelled`` / ``RequestTimeout`` as
  its error and the other requests are unaffected;
* writes one JSON line per completed request (``log_path``): its sizes,
  precision, kind, outcome, queueing time, latency and status flags.

The engine holds no arithmetic of the method: the executor runs the library
calls (``GpuExecutor``), or simulates their duration (``FakeExecutor``, used to
test admission, batching and the lanes on a CPU).
"""
from __future__ import annotations

import collections
import itertools
import json
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _lib as L

KIND_WILSON, KIND_SPIN, KIND_NESTED = "wilson", "spin", "nested"
KIND_FLUX, KIND_SPIN_FLUX = "flux", "spin_flux"


class RequestCancelled(Exception):
    """The request was cancelled before its result was computed."""


class RequestTimeout(RequestCancelled):
    """The request outlived its timeout before its result was computed."""


@dataclass
class Request:
    hoplist: object
    kappa: np.ndarray          # (n_perp, n_par, 3)
    lo: int
    hi: int
    kind: str = KIND_WILSON
    spin_diag: Optional[np.ndarray] = None
    precision: int = L.BE_FP64
    window: tuple = (0.0, 0.5)
    tag: str = ""
    timeout: Optional[float] = None  # seconds from submission; None: no limit
    rid: int = -1
    t_submit: float = 0.0
    t_admit: Optional[float] = None
    t_done: float = 0.0
    result: Optional[dict] = None
    error: Optional[BaseException] = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def N(self) -> int:
        return int(self.hoplist.N)

    @property
    def m(self) -> int:
        return self.hi - self.lo

    @property
    def n_k(self) -> int:
        return int(self.kappa.shape[0] * self.kappa.shape[1])

    @property
    def key(self):
        return (self.N, self.lo, self.hi, self.precision)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


def resident_bytes(req: Request) -> int:
    """Eigenvectors (c128, N x m per k-point), eigenvalues and status words."""
    return req.n_k * (req.N * max(req.m, 1) * 16 + (req.m + 2) * 8 + 4)


class Engine:
    """Admission, batching and scheduling over the executor's lanes."""

    def __init__(self, executor, hbm_budget: int, clock: Callable[[], float] = time.perf_counter,
                 on_event: Optional[Callable[[dict], None]] = None, log_path: Optional[str] = None,
                 policy: str = "fifo"):
        if policy not in ("fifo", "srpt"):
            raise ValueError("policy must be 'fifo' (oldest request first) or 'srpt' (least remaining work first)")
        self.policy = policy
        self.ex = executor
        self.on_event = on_event  # called after every task (progress reporting)
        self.log_path = log_path  # JSON lines, one per completed request
        self._log_lock = threading.Lock()
        self.budget = int(hbm_budget)
        self.clock = clock
        self._cv = threading.Condition()
        self._queue: collections.deque = collections.deque()
        self._active: Dict[int, dict] = {}
        self._ids = itertools.count()
        self._busy_keys = set()
        self.used = 0
        self.peak_used = 0
        self.completed: List[Request] = []
        self.step_log: List[dict] = []
        self._to_log: List[Request] = []  # stopped before admission, logged outside the lock
        self._stop = False
        self._threads: List[threading.Thread] = []

    # ------------------------------------------------------------ API
    def submit(self, req: Request) -> Request:
        if self.ex.footprint(req) > self.budget:
            raise ValueError("request does not fit the HBM budget even alone")
        with self._cv:
            req.rid = next(self._ids)
            req.t_submit = self.clock()
            self._queue.append(req)
            self._cv.notify_all()
        return req

    def pending(self) -> int:
        with self._cv:
            return len(self._queue) + len(self._active)

    def cancel(self, req: Request) -> bool:
        """Stop a request that has not started its loop stage. Returns False
        when it is already finishing or done."""
        with self._cv:
            ok = self._stop_request(req, RequestCancelled(f"request {req.rid} cancelled"))
            self._cv.notify_all()
        if ok and req.done.is_set():
            self._log(req)
        return ok

    # ------------------------------------------------------------ stopping
    def _stop_request(self, req: Request, exc: RequestCancelled) -> bool:
        """(Lock held.) A waiting request completes at once; an admitted one
        takes no further k-points and skips its loop stage, and completes when
        its launch in flight (if any) has ended."""
        if req in self._queue:
            self._queue.remove(req)
            req.error = exc
            req.t_done = self.clock()
            self.completed.append(req)
            req.done.set()
            return True
        a = self._active.get(req.rid)
        if a is None or a["finishing"] or a["req"] is not req:
            return False
        if req.error is None:
            req.error = exc
        a["next_k"] = req.n_k
        return True

    def _expire(self):
        """(Lock held.) Stop the requests that outlived their timeout."""
        now = self.clock()
        late = [r for r in list(self._queue) + [a["req"] for a in self._active.values()]
                if r.timeout is not None and now - r.t_submit > r.timeout and r.error is None]
        for r in late:
            queued = r in self._queue
            if self._stop_request(r, RequestTimeout(f"request {r.rid} exceeded its timeout of {r.timeout} s")) \
                    and queued:
                self._to_log.append(r)

    def log_record(self, req: Request) -> dict:
        """The request's JSON-lines record."""
        out = req.result or {}
        st = out.get("status")
        status = int(np.bitwise_or.reduce(np.asarray(st, dtype=np.int64).ravel())) if st is not None else None
        outcome = ("ok" if req.error is None else "timeout" if isinstance(req.error, RequestTimeout)
                   else "cancelled" if isinstance(req.error, RequestCancelled) else "error")
        return {"rid": req.rid, "tag": req.tag, "kind": req.kind, "N": req.N, "m": req.m, "k_points": req.n_k,
                "precision": int(req.precision), "outcome": outcome,
                "error": None if req.error is None else f"{type(req.error).__name__}: {req.error}",
                "t_submit": req.t_submit, "queue_s": (req.t_admit - req.t_submit) if req.t_admit is not None else None,
                "latency_s": req.latency, "status": status, "eig_status": out.get("eig_status")}

    def _log(self, req: Request):
        if not self.log_path:
            return
        line = json.dumps(self.log_record(req))
        with self._log_lock, open(self.log_path, "a") as f:
            f.write(line + "\n")

    def step(self, lane: int = 0) -> bool:
        """Take and run one task on `lane` in the calling thread (admission
        included). Returns False when there was nothing to do."""
        with self._cv:
            task = self._take_task()
        self._flush_log()
        if task is None:
            return False
        self._run_task(task, lane)
        return True

    def _flush_log(self):
        with self._cv:
            reqs, self._to_log = self._to_log, []
        for r in reqs:
            self._log(r)

    def run_until_idle(self, lane: int = 0):
        while self.step(lane) or self.pending():
            pass

    def start(self):
        """One worker thread per executor lane."""
        self._stop = False
        self._threads = [threading.Thread(target=self._worker, args=(k,), daemon=True)
                         for k in range(self.ex.n_lanes)]
        for t in self._threads:
            t.start()

    def stop(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        self._threads = []

    # ------------------------------------------------------------ scheduling
    def _worker(self, lane: int):
        while True:
            with self._cv:
                task = self._take_task()
                while task is None and not self._stop:
                    self._cv.wait(0.05)
                    task = self._take_task()
            self._flush_log()
            if task is None:
                return
            self._run_task(task, lane)

    def _admit(self):
        for req in list(self._queue):
            fp = self.ex.footprint(req)
            if self.used + fp > self.budget:
                continue  # skip ahead: a smaller request may still fit
            self._queue.remove(req)
            self._active[req.rid] = {"req": req, "state": None, "next_k": 0, "fp": fp, "inflight": 0,
                                     "finishing": False}
            req.t_admit = self.clock()
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)

    def _take_task(self):
        """Next task (caller holds the lock): a loop stage of a request whose
        k-points are all diagonalized, else an eigensolver launch of a request
        whose key is not running on another lane (the oldest one, or with
        policy "srpt" the one with the least remaining eigensolver work,
        pending k-points times N^3), packed with the other admitted requests of
        that key."""
        self._expire()
        self._admit()
        act = list(self._active.values())
        for a in act:
            if not a["finishing"] and a["inflight"] == 0 and a["next_k"] >= a["req"].n_k:
                a["finishing"] = True
                return ("loop", a)
        order = act
        if self.policy == "srpt":
            order = sorted(act, key=lambda a: (a["req"].n_k - a["next_k"]) * float(a["req"].N) ** 3)
        for a in order:
            r = a["req"]
            if a["next_k"] >= r.n_k or r.key in self._busy_keys:
                continue
            budget = self.ex.chunk_for(r)
            parts = []
            for b in act:
                if budget <= 0:
                    break
                rb = b["req"]
                if rb.key != r.key or b["next_k"] >= rb.n_k:
                    continue
                take = min(budget, rb.n_k - b["next_k"])
                parts.append((b, b["next_k"], b["next_k"] + take))
                b["next_k"] += take
                b["inflight"] += 1
                budget -= take
            self._busy_keys.add(r.key)
            return ("eig", parts)
        return None

    def _run_task(self, task, lane: int):
        kind, payload = task
        if kind == "eig":
            parts = payload
            err = None
            t_start = self.clock()
            try:
                for b, _, _ in parts:
                    if b["state"] is None:
                        b["state"] = self.ex.prepare(b["req"], lane)
                        b["state"]["rid"] = b["req"].rid
                self.ex.run_eig([(b["state"], k0, k1) for b, k0, k1 in parts], lane)
            except BaseException as e:  # noqa: BLE001 - reported on the request
                err = e
            with self._cv:
                ev = {"kind": "eig", "t0": t_start, "t": self.clock(), "lane": lane, "N": parts[0][0]["req"].N,
                      "requests": [b["req"].rid for b, _, _ in parts], "k_points": sum(k1 - k0 for _, k0, k1 in parts)}
                self.step_log.append(ev)
                for b, _, _ in parts:
                    b["inflight"] -= 1
                    if err is not None:
                        b["req"].error = err
                        b["next_k"] = b["req"].n_k
                self._busy_keys.discard(parts[0][0]["req"].key)
                self._cv.notify_all()
            if self.on_event:
                self.on_event(ev)
        else:
            a = payload
            req = a["req"]
            try:
                if req.error is None:
                    req.result = self.ex.finish(a["state"], lane)
            except BaseException as e:  # noqa: BLE001
                req.error = e
            finally:
                if a["state"] is not None:
                    self.ex.release(a["state"], lane)
            with self._cv:
                del self._active[req.rid]
                self.used -= a["fp"]
                req.t_done = self.clock()
                self.completed.append(req)
                self._cv.notify_all()
            self._log(req)
            req.done.set()
            if self.on_event:
                self.on_event({"kind": "done", "lane": lane, "N": req.N, "request": req.rid, "tag": req.tag,
                               "latency": req.latency})


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "n": 0}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": int(lat.size)}


# ---------------------------------------------------------------- executors
class GpuExecutor:
    """Runs requests through the library on one device, on n_lanes lanes (a
    library context and a torch stream each; a lane is used by one host
    thread at a time). Eigensolver launches take up to chunk_for(req)
    k-points: as many Hamiltonians as fit h_bytes (at most chunk_cap)."""

    def __init__(self, n_lanes: int = 2, h_bytes: int = 16 << 30, chunk_cap: int = 2048, device: int = 0):
        import torch
        self.torch = torch
        self.n_lanes = int(n_lanes)
        self.h_bytes = int(h_bytes)
        self.chunk_cap = int(chunk_cap)
        self.device = device
        self.lanes = []
        for _ in range(self.n_lanes):
            self.lanes.append((L.Context(device), torch.cuda.Stream(device=device)))
        self._H = {}          # key -> [H buffer, event after its last use]
        self._chunk = {}      # (N, precision) -> Hamiltonians per launch
        self._key_users = collections.Counter()
        self._lock = threading.Lock()

    @staticmethod
    def _hb(req):
        return 8 if L.c64_input(req.precision) else 16

    def chunk_for(self, req: Request) -> int:
        """Hamiltonians per eigensolver launch for the request's key: the same
        for every request of a key, since the key's buffer holds that many;
        a whole number of the eigensolver's device rounds where it holds at
        least one (a launch of 404 order-2304 matrices would run as two
        rounds of 202 on 256 compute units; 256 fill one)."""
        key = (req.N, req.precision)
        if key not in self._chunk:
            per = req.N * req.N * self._hb(req)
            c = int(max(1, min(self.chunk_cap, self.h_bytes // per)))
            r = self.lanes[0][0].eigh_round(req.N, req.precision)
            self._chunk[key] = c // r * r if c >= r else c
        return self._chunk[key]

    def footprint(self, req: Request) -> int:
        """Resident eigenvectors, one chunk of Hamiltonians (one buffer per
        key, used by one lane at a time), the eigensolver's workspace for a
        chunk (panel vectors and the tridiagonal solver's four N x m FP64
        arrays per matrix) and the loop stage's."""
        c = self.chunk_for(req)
        m = max(req.m, 1)
        mp = max(64, (m + 63) // 64 * 64)
        # the eigensolver works in sub-batches of at most 48 GiB of workspace
        eig_ws = min(48 << 30, min(c, req.n_k) * (req.N * 96 * self._hb(req) + 4 * req.N * mp * 8 + req.N * m * 8
                                                  + m * m * 8))
        n_lines = req.n_k // max(1, req.kappa.shape[1]) if req.kappa.ndim == 3 else req.n_k
        # overlap/polar/product buffers (passes of at most 4 GiB), the Wilson
        # matrices' eigenproblems (at most 4 GiB, plus the eigensolver's own)
        loop_ws = (min(6 << 30, req.n_k * 3 * m * m * 16) + min(6 << 30, n_lines * 5 * m * m * 16)
                   + req.n_k * req.N * m * 16 * (1 if req.kind in (KIND_SPIN, KIND_SPIN_FLUX) else 0))
        return int(resident_bytes(req) + c * req.N * req.N * self._hb(req) + eig_ws + loop_ws)

    def _hbuf(self, req, stream):
        """The key's Hamiltonian buffer, ready for use on `stream` (which waits
        for the buffer's last use on another lane's stream)."""
        torch = self.torch
        with self._lock:
            ent = self._H.get(req.key)
            if ent is None:
                dt = torch.complex64 if L.c64_input(req.precision) else torch.complex128
                ent = [torch.empty((self.chunk_for(req), req.N, req.N), dtype=dt, device=self.device), None]
                self._H[req.key] = ent
        if ent[1] is not None:
            stream.wait_event(ent[1])
        ent[0].record_stream(stream)
        return ent

    def prepare(self, req: Request, lane: int) -> dict:
        torch = self.torch
        ctx, stream = self.lanes[lane]
        with self._lock:
            self._key_users[req.key] += 1
        with torch.cuda.stream(stream):
            plan = ctx.hk_plan([req.hoplist])
            kap = torch.from_numpy(np.ascontiguousarray(req.kappa.reshape(-1, 3), dtype=np.float64)).to(
                self.device, non_blocking=False)
            U = torch.empty((req.n_k, max(req.m, 1), req.N), dtype=torch.complex128, device=self.device)
            ev = torch.empty((req.n_k, req.m + 2), dtype=torch.float64, device=self.device)
            st = torch.empty(req.n_k, dtype=torch.int32, device=self.device)
        return {"req": req, "plan": plan, "kap": kap, "U": U, "ev": ev, "st": st, "event": None, "alloc_stream": stream}

    def run_eig(self, parts, lane: int):
        """parts: list of (state, k0, k1), all with the same (N, bands,
        precision). Builds the chunk's Hamiltonians on the lane's stream and
        diagonalizes them into the requests' own buffers."""
        torch = self.torch
        ctx, stream = self.lanes[lane]
        r0 = parts[0][0]["req"]
        N, prec = r0.N, r0.precision
        dcode = L.BE_C64 if L.c64_input(prec) else L.BE_C128
        with torch.cuda.stream(stream):
            hent = self._hbuf(r0, stream)
            H = hent[0]
            total = sum(k1 - k0 for _, k0, k1 in parts)
            if total > H.shape[0]:  # the kernels would write past the key's buffer
                raise ValueError(f"launch of {total} k-points exceeds the key's buffer of {H.shape[0]}")
            n = 0
            for st, k0, k1 in parts:
                if st["event"] is not None:
                    stream.wait_event(st["event"])
                for k in ("U", "ev", "st", "kap"):
                    st[k].record_stream(stream)
                ctx.build_hk(st["plan"], 0, 1, st["kap"][k0:k1], H[n:], N * N, N, dcode)
                n += k1 - k0
            n = 0
            for st, k0, k1 in parts:
                c = k1 - k0
                ctx.eigh_batched(H[n:], dcode, N, N, N * N, c, r0.lo, r0.hi, prec, st["ev"][k0:], st["U"][k0:], N,
                                 st["U"].stride(0), st["st"][k0:])
                n += c
                ev = torch.cuda.Event()
                ev.record(stream)
                st["event"] = ev
            hent[1] = ev  # the buffer's last use

    def finish(self, st, lane: int) -> dict:
        from . import pipeline as P
        torch = self.torch
        ctx, stream = self.lanes[lane]
        r: Request = st["req"]
        with torch.cuda.stream(stream):
            if st["event"] is not None:
                stream.wait_event(st["event"])
            for k in ("U", "ev", "st"):
                st[k].record_stream(stream)
            g = P.EigGrid(st["U"], st["ev"], st["st"], r.N, r.m, r.N, 1, r.kappa.shape[1], r.kappa.shape[0])
            if r.kind == KIND_SPIN:
                out = P.spin(ctx, g, np.asarray(r.spin_diag)[None], precision=r.precision)
            elif r.kind == KIND_NESTED:
                out = P.nested(ctx, g, r.window)
            elif r.kind == KIND_FLUX:
                out = P.flux(ctx, g)
            elif r.kind == KIND_SPIN_FLUX:
                out = P.spin_flux(ctx, g, np.asarray(r.spin_diag)[None], precision=r.precision)
            else:
                out = P.wilson(ctx, g)
            out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
            out["eig_status"] = int((st["st"].cpu().numpy() != 0).any())
        return out

    def release(self, st, lane: int):
        st["plan"].close()
        for k in ("U", "ev", "st", "kap"):
            st[k] = None
        key = st["req"].key
        with self._lock:
            self._key_users[key] -= 1
            if self._key_users[key] <= 0:
                del self._key_users[key]
                self._H.pop(key, None)   # no admitted request uses the key any more


class FakeExecutor:
    """Simulated executor for CPU tests: sleeps for a time proportional to the
    work of each call and records what it was asked to do, and on which lane."""

    def __init__(self, flops_per_s: float = 1e12, sleep: bool = True, n_lanes: int = 1, chunk_k: int = 2048):
        self.rate = flops_per_s
        self.sleep = sleep
        self.n_lanes = n_lanes
        self.chunk_k = chunk_k
        self.calls = []
        self.live = 0
        self.running = collections.Counter()
        self.overlaps = 0
        self._lock = threading.Lock()

    def chunk_for(self, req):
        return self.chunk_k

    def footprint(self, req):
        return resident_bytes(req) + self.chunk_for(req) * req.N * req.N * 16

    def prepare(self, req, lane):
        with self._lock:
            self.live += 1
        return {"req": req, "done_k": 0}

    def run_eig(self, parts, lane):
        keys = {p[0]["req"].key for p in parts}
        assert len(keys) == 1, "a launch mixes incompatible requests"
        key = keys.pop()
        N = parts[0][0]["req"].N
        nk = sum(p[2] - p[1] for p in parts)
        with self._lock:
            assert self.running[key] == 0, "one key runs on two lanes at once"
            self.running[key] += 1
            if sum(self.running.values()) > 1:
                self.overlaps += 1
            for st, k0, k1 in parts:
                assert k0 == st["done_k"], "k-points must be processed in order, once"
                st["done_k"] = k1
            self.calls.append(("eig", [p[0]["rid"] for p in parts], nk, lane))
        if self.sleep:
            time.sleep(nk * 10.0 * N ** 3 / self.rate)
        with self._lock:
            self.running[key] -= 1

    def finish(self, st, lane):
        r = st["req"]
        assert st["done_k"] == r.n_k
        with self._lock:
            self.calls.append(("loop", st["rid"], lane))
        return {"rid": st["rid"], "n_k": r.n_k}

    def release(self, st, lane):
        with self._lock:
            self.live -= 1


def served_precision(kind: str) -> int:
    """Eigensolver precision of the served workload's request types: the mixed
    path for the BHZ supercells (about 1e-7 rad from FP64), the refined mixed
    path for the 96-orbital model, whose small gaps (0.045 against a bandwidth
    of 66) take the mixed path's phase error above 1e-6 rad."""
    return L.BE_MIXED_FP32_REFINED if kind == "w96" else L.BE_MIXED_FP32


def poisson_arrivals(rate_hz: float, n: int, seed) -> np.ndarray:
    """Arrival times of a Poisson stream (exponential gaps), seconds from 0."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def drive(engine: Engine, requests: List[Request], arrivals: np.ndarray, clock=time.perf_counter):
    """Submit requests at their arrival times while the engine's lanes run
    (those arriving at time 0 are queued before the lanes start)."""
    t0 = clock()
    pending = []
    for req, ta in zip(requests, arrivals):
        if ta <= 0.0:
            engine.submit(req)
        else:
            pending.append((req, ta))
    engine.start()
    try:
        for req, ta in pending:
            while clock() - t0 < ta:
                time.sleep(min(0.001, max(0.0, ta - (clock() - t0))))
            engine.submit(req)
        for req in requests:
            req.done.wait()
    finally:
        engine.stop()
    return clock() - t0
