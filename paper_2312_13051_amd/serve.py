"""Continuous-batching request loop for Wilson-loop requests.

A request is one model (hopping list) with a k-plane, a band window and a
kind (plain, spin-resolved or nested Wilson loop, or the Berry flux per
plaquette of the occupied space or of its spin sectors). Requests arrive at any
time. The engine

* admits a waiting request as soon as its device footprint (resident
  eigenvectors plus its share of the Hamiltonian buffer) fits the HBM budget
  next to the requests already admitted, first come first served with
  skip-ahead for smaller requests;
* keeps every admitted request's eigenvectors resident on the device until
  its Wilson loop has run;
* packs, at every step, the pending k-points of all admitted requests that
  share (N, bands, precision) into one batched eigensolver launch (continuous
  batching: a request that arrives while others run joins at the next step);
* runs a request's Wilson-loop stage as soon as all its k-points are
  diagonalized, frees its memory and records its latency.

The engine holds no arithmetic of the method: the executor runs the library
calls (``GpuExecutor``), or simulates their duration (``FakeExecutor``, used to
test admission and batching on a CPU).
"""
from __future__ import annotations

import collections
import itertools
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _lib as L

KIND_WILSON, KIND_SPIN, KIND_NESTED = "wilson", "spin", "nested"
KIND_FLUX, KIND_SPIN_FLUX = "flux", "spin_flux"


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
    rid: int = -1
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    result: Optional[dict] = None
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
    def latency(self) -> float:
        return self.t_done - self.t_submit


def footprint_bytes(req: Request, chunk_k: int) -> int:
    """Device bytes a request holds while admitted: its resident eigenvectors
    (c128, N x m per k-point), eigenvalues, and at most chunk_k Hamiltonians."""
    hb = 8 if req.precision == L.BE_MIXED_FP32 else 16
    resident = req.n_k * (req.N * max(req.m, 1) * 16 + (req.m + 2) * 8 + 4)
    h = min(chunk_k, req.n_k) * req.N * req.N * hb
    return int(resident + h)


class Engine:
    def __init__(self, executor, hbm_budget: int, chunk_k: int = 2048, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.chunk_k = int(chunk_k)
        self.clock = clock
        self._lock = threading.Lock()
        self._queue: collections.deque = collections.deque()
        self._active: Dict[int, dict] = {}
        self._ids = itertools.count()
        self.used = 0
        self.peak_used = 0
        self.completed: List[Request] = []
        self.step_log: List[dict] = []
        self._stop = threading.Event()
        self._thread: Optional[threading.Thread] = None

    # ------------------------------------------------------------ API
    def submit(self, req: Request) -> Request:
        if footprint_bytes(req, self.chunk_k) > self.budget:
            raise ValueError("request does not fit the HBM budget even alone")
        with self._lock:
            req.rid = next(self._ids)
            req.t_submit = self.clock()
            self._queue.append(req)
        return req

    def pending(self) -> int:
        with self._lock:
            return len(self._queue) + len(self._active)

    def step(self) -> bool:
        """One scheduling step. Returns False when there was nothing to do."""
        self._admit()
        with self._lock:
            active = list(self._active.values())
        if not active:
            return False
        # requests whose k-points are all diagonalized: run the loop stage
        ready = [a for a in active if a["next_k"] >= a["req"].n_k]
        for a in ready:
            self._finish(a)
        todo = [a for a in active if a["next_k"] < a["req"].n_k]
        if not todo:
            return True
        # continuous batching: pack pending k-points of compatible requests,
        # oldest first, up to chunk_k k-points per eigensolver launch
        key0 = self._key(todo[0]["req"])
        group = [a for a in todo if self._key(a["req"]) == key0]
        budget = self.chunk_k
        parts = []
        for a in group:
            if budget <= 0:
                break
            r = a["req"]
            take = min(budget, r.n_k - a["next_k"])
            parts.append((a["state"], a["next_k"], a["next_k"] + take))
            a["next_k"] += take
            budget -= take
        self.ex.run_eig(parts)
        self.step_log.append({"t": self.clock(), "requests": [p[0]["rid"] for p in parts],
                              "k_points": sum(p[2] - p[1] for p in parts)})
        return True

    def run_until_idle(self):
        while self.step() or self.pending():
            pass

    def start(self):
        self._stop.clear()
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def stop(self):
        self._stop.set()
        if self._thread:
            self._thread.join()

    # ------------------------------------------------------------ internals
    @staticmethod
    def _key(r: Request):
        return (r.N, r.lo, r.hi, r.precision)

    def _loop(self):
        while not self._stop.is_set():
            if not self.step():
                time.sleep(0.0005)

    def _admit(self):
        with self._lock:
            waiting = list(self._queue)
        for req in waiting:
            fp = footprint_bytes(req, self.chunk_k)
            if self.used + fp > self.budget:
                continue  # skip ahead: a smaller request may still fit
            state = self.ex.prepare(req)
            state["rid"] = req.rid
            with self._lock:
                self._queue.remove(req)
                self._active[req.rid] = {"req": req, "state": state, "next_k": 0, "fp": fp}
            req.t_admit = self.clock()
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)

    def _finish(self, a):
        req = a["req"]
        req.result = self.ex.finish(a["state"])
        self.ex.release(a["state"])
        with self._lock:
            del self._active[req.rid]
        self.used -= a["fp"]
        req.t_done = self.clock()
        self.completed.append(req)
        req.done.set()


def latency_stats(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "n": 0}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": int(lat.size)}


# ---------------------------------------------------------------- executors
class GpuExecutor:
    """Runs requests through the library on one device."""

    def __init__(self, ctx: L.Context, chunk_k: int = 2048):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.chunk_k = chunk_k
        self._H = {}

    def _hbuf(self, N, prec):
        torch = self.torch
        dt = torch.complex64 if prec == L.BE_MIXED_FP32 else torch.complex128
        key = (N, prec)
        if key not in self._H:
            self._H[key] = torch.empty((self.chunk_k, N, N), dtype=dt, device="cuda")
        return self._H[key]

    def prepare(self, req: Request) -> dict:
        torch = self.torch
        plan = self.ctx.hk_plan([req.hoplist])
        kap = torch.from_numpy(np.ascontiguousarray(req.kappa.reshape(-1, 3), dtype=np.float64)).cuda()
        U = torch.empty((req.n_k, max(req.m, 1), req.N), dtype=torch.complex128, device="cuda")
        ev = torch.empty((req.n_k, req.m + 2), dtype=torch.float64, device="cuda")
        st = torch.empty(req.n_k, dtype=torch.int32, device="cuda")
        return {"req": req, "plan": plan, "kap": kap, "U": U, "ev": ev, "st": st}

    def run_eig(self, parts):
        """parts: list of (state, k0, k1), all with the same (N, bands, precision)."""
        torch = self.torch
        r0 = parts[0][0]["req"]
        N, prec = r0.N, r0.precision
        dcode = L.BE_C64 if prec == L.BE_MIXED_FP32 else L.BE_C128
        H = self._hbuf(N, prec)
        n = 0
        for st, k0, k1 in parts:
            self.ctx.build_hk(st["plan"], 0, 1, st["kap"][k0:k1], H[n:], N * N, N, dcode)
            n += k1 - k0
        if len(parts) == 1:
            st, k0, k1 = parts[0]
            self.ctx.eigh_batched(H, dcode, N, N, N * N, n, r0.lo, r0.hi, prec, st["ev"][k0:], st["U"][k0:], N,
                                  st["U"].stride(0), st["st"][k0:])
            return
        m = max(r0.m, 1)
        U = torch.empty((n, m, N), dtype=torch.complex128, device="cuda")
        ev = torch.empty((n, r0.m + 2), dtype=torch.float64, device="cuda")
        sts = torch.empty(n, dtype=torch.int32, device="cuda")
        self.ctx.eigh_batched(H, dcode, N, N, N * N, n, r0.lo, r0.hi, prec, ev, U, N, U.stride(0), sts)
        n = 0
        for st, k0, k1 in parts:
            c = k1 - k0
            st["U"][k0:k1].copy_(U[n:n + c])
            st["ev"][k0:k1].copy_(ev[n:n + c])
            st["st"][k0:k1].copy_(sts[n:n + c])
            n += c

    def finish(self, st) -> dict:
        from . import pipeline as P
        r: Request = st["req"]
        g = P.EigGrid(st["U"], st["ev"], st["st"], r.N, r.m, r.N, 1, r.kappa.shape[1], r.kappa.shape[0])
        if r.kind == KIND_SPIN:
            out = P.spin(self.ctx, g, np.asarray(r.spin_diag)[None], precision=r.precision)
        elif r.kind == KIND_NESTED:
            out = P.nested(self.ctx, g, r.window)
        elif r.kind == KIND_FLUX:
            out = P.flux(self.ctx, g)
        elif r.kind == KIND_SPIN_FLUX:
            out = P.spin_flux(self.ctx, g, np.asarray(r.spin_diag)[None], precision=r.precision)
        else:
            out = P.wilson(self.ctx, g)
        out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
        out["eig_status"] = int((st["st"].cpu().numpy() != 0).any())
        return out

    def release(self, st):
        st["plan"].close()
        for k in ("U", "ev", "st", "kap"):
            st[k] = None


class FakeExecutor:
    """Simulated executor for CPU tests: sleeps for a time proportional to the
    work of each call and records what it was asked to do."""

    def __init__(self, flops_per_s: float = 1e12, sleep: bool = True):
        self.rate = flops_per_s
        self.sleep = sleep
        self.calls = []
        self.live = 0

    def prepare(self, req):
        self.live += 1
        return {"req": req, "done_k": 0}

    def run_eig(self, parts):
        keys = {(p[0]["req"].N, p[0]["req"].lo, p[0]["req"].hi, p[0]["req"].precision) for p in parts}
        assert len(keys) == 1, "a launch mixes incompatible requests"
        N = parts[0][0]["req"].N
        nk = sum(p[2] - p[1] for p in parts)
        for st, k0, k1 in parts:
            assert k0 == st["done_k"], "k-points must be processed in order, once"
            st["done_k"] = k1
        self.calls.append(("eig", [p[0]["rid"] for p in parts], nk))
        if self.sleep:
            time.sleep(nk * 10.0 * N ** 3 / self.rate)

    def finish(self, st):
        r = st["req"]
        assert st["done_k"] == r.n_k
        self.calls.append(("loop", st["rid"]))
        return {"rid": st["rid"], "n_k": r.n_k}

    def release(self, st):
        self.live -= 1


def poisson_arrivals(rate_hz: float, n: int, seed) -> np.ndarray:
    """Arrival times of a Poisson stream (exponential gaps), seconds from 0."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def drive(engine: Engine, requests: List[Request], arrivals: np.ndarray, clock=time.perf_counter):
    """Submit requests at their arrival times while the engine thread runs."""
    engine.start()
    t0 = clock()
    for req, ta in zip(requests, arrivals):
        while clock() - t0 < ta:
            time.sleep(min(0.001, max(0.0, ta - (clock() - t0))))
        engine.submit(req)
    for req in requests:
        req.done.wait()
    engine.stop()
    return clock() - t0
