"""Continuous-batching reconstruction server.

Requests are FISTA reconstructions (Sec. 2.3) on possibly different
geometries and library precisions.  The unit of GPU work is one batched
FISTA iteration of one (geometry, precision) class through `pat_fista_step`:
every request carries its own iteration counter and momentum sequence, so
requests join a class batch at the next iteration boundary after they are
admitted and leave it the moment their last iteration is done.  Each class
runs on its own stream, so batches of different classes overlap on the
device.  A slot's iteration count advances when its iteration is launched,
so its result is taken (in stream order, right after its last iteration)
and its row handed on at launch time; a class may therefore have up to
``depth`` iterations queued, which it does while it is the only class with
work: the GPU then runs the next iteration while the host handles the last
one.  With several classes busy their streams keep the device fed, and one
queued iteration per class lets requests that arrive join the very next
one.  The kernel library of every class is built once and cached; a
request is admitted only if the HBM it needs (its slot in the class's state
pool, plus the library and workspace when the class is new) fits the
budget, evicting libraries of idle classes when necessary.

The scheduler is written against a small backend interface (``HipBackend``
here; the tests plug in a CPU float64 backend) so its logic can be checked
without a GPU.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import torch

from .op import Geometry, Operator


@dataclass
class Request:
    geom: Geometry
    d: torch.Tensor                # [nt, ny, nx] data (device or host)
    niter: int = 50
    h_dtype: str = "f32"
    lam: float = 0.0
    nonneg: bool = True
    tau: float | None = None       # None: 1/L from 30 power iterations of the class
    rid: int = -1
    t_arrival: float | None = None
    t_admit: float | None = None
    t_done: float | None = None
    x: torch.Tensor | None = None  # result x_niter
    status: str = "pending"        # pending | running | done | nonfinite | rejected

    @property
    def key(self):
        return (self.geom, self.h_dtype)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


@dataclass
class _Slot:
    req: Request
    k: int = 0          # iterations done
    t: float = 1.0      # FISTA t_k


@dataclass
class _Class:
    key: tuple
    op: object
    tau: float
    cap: int = 0
    pool: dict = field(default_factory=dict)   # x, z, d, bad
    ws: object = None
    active: list = field(default_factory=list)  # slot i <-> row i of the pool
    inflight: list = field(default_factory=list)  # queued iterations: (event, [(request, x, flag)])
    keep: list = field(default_factory=list)    # (pool, ws, bytes, events): replaced buffers kept
                                                # alive until the iterations queued before end
    last_used: float = 0.0
    bytes_lib: int = 0
    bytes_ws1: int = 0      # the operator's own one-object workspace (A^T d at admission, step size)
    bytes_pool: int = 0
    bytes_keep: int = 0     # replaced pools kept alive until the iterations using them end


class HipBackend:
    """GPU backend: libpat operators, torch-owned buffers, one stream per class.

    normal=True (default) steps requests with the per-frequency normal
    operator: a slot keeps A^T d (formed once at admission) instead of d, and
    an iteration costs one z-spectrum, one nz x nz contraction and one inverse
    spectrum; normal=False takes the explicit A then A^T every iteration.
    Libraries without Gram blocks always take the explicit step: the linear
    (zero-padded) boundary and scan-grid sampling, whose cropping or sampling
    between A and A^T breaks the per-frequency structure of A^T A."""

    def __init__(self, device: int = 0, normal: bool = True):
        self.device = torch.device("cuda", device)
        self.normal = normal
        self._flags = None   # pinned host ring of the non-finite flags of finished slots
        self._next_flag = 0

    def library_bytes(self, geom, h_dtype) -> int:
        from .op import h_bytes
        return h_bytes(geom, h_dtype)

    def build(self, geom, h_dtype, stream):
        with torch.cuda.stream(stream):
            op = Operator(geom, h_dtype, device=self.device.index)
        return op

    def step_size(self, op, stream) -> float:
        from . import inputs
        with torch.cuda.stream(stream):
            v0 = torch.from_numpy(inputs.gaussian_random(op.x_shape, seed=1002).astype("float32")).to(self.device)
            L, _ = op.power_norm(v0, 30)
        return 1.0 / L

    def uses_normal(self, op) -> bool:
        return self.normal and op.has_gram

    def slot_bytes(self, op) -> int:
        g = op.geom
        if self.uses_normal(op):
            return 4 * g.nx * g.ny * 3 * g.nz + 4
        return 4 * (2 * g.nz * g.ny * g.nx + g.nt * (g.ny // g.sy) * (g.nx // g.sx)) + 4

    def workspace_bytes(self, op, cap) -> int:
        return op.workspace_bytes(cap)

    def new_stream(self):
        return torch.cuda.Stream(device=self.device)

    def alloc_pool(self, op, cap, stream):
        g = op.geom
        data = "b" if self.uses_normal(op) else "d"
        dshape = op.x_shape if self.uses_normal(op) else op.d_shape
        with torch.cuda.stream(stream):
            return {"x": torch.zeros((cap,) + op.x_shape, device=self.device),
                    "z": torch.zeros((cap,) + op.x_shape, device=self.device),
                    data: torch.zeros((cap,) + dshape, device=self.device),
                    "bad": torch.zeros(cap, dtype=torch.int32, device=self.device)}, \
                torch.empty(op.workspace_bytes(cap), dtype=torch.uint8, device=self.device)

    def load_row(self, pool, i, d, stream, op=None):
        with torch.cuda.stream(stream):
            if "b" in pool:
                op.apply_AT(d.to(self.device, non_blocking=True), out=pool["b"][i])
            else:
                pool["d"][i].copy_(d, non_blocking=True)
            pool["x"][i].zero_()
            pool["z"][i].zero_()
            pool["bad"][i].zero_()

    def move_row(self, pool, src, dst, stream):
        with torch.cuda.stream(stream):
            for name in pool:
                pool[name][dst].copy_(pool[name][src])

    def copy_rows(self, old, new, n, stream):
        with torch.cuda.stream(stream):
            for name in old:
                new[name][:n].copy_(old[name][:n])

    def step(self, op, pool, ws, n, betas, taus, lams, nonnegs, stream):
        with torch.cuda.stream(stream):
            if "b" in pool:
                op.fista_step_normal(pool["b"][:n], pool["x"][:n], pool["z"][:n], betas, taus, lams,
                                     nonnegs, nonfinite=pool["bad"][:n], ws=ws)
            else:
                op.fista_step(pool["d"][:n], pool["x"][:n], pool["z"][:n], betas, taus, lams, nonnegs,
                              nonfinite=pool["bad"][:n], ws=ws)

    def mark(self, stream):
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def take_result(self, pool, i, stream):
        """x_i and its non-finite flag, copied in stream order; the flag lands
        in pinned host memory and is read only after a later mark() is done
        (4,096 entries: far more results than can be queued at once)."""
        if self._flags is None:
            self._flags = torch.zeros(4096, dtype=torch.int32, pin_memory=True)
        j = self._next_flag % self._flags.numel()
        self._next_flag += 1
        flag = self._flags[j:j + 1]
        with torch.cuda.stream(stream):
            x = pool["x"][i].clone()
            flag.copy_(pool["bad"][i:i + 1], non_blocking=True)
        return x, flag


class Server:
    def __init__(self, backend=None, hbm_budget: int = 64 << 30, max_batch: int = 16,
                 clock=time.perf_counter, depth: int = 2):
        self.be = backend if backend is not None else HipBackend()
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.depth = max(1, int(depth))   # iterations queued per class
        self.clock = clock
        self.classes: dict[tuple, _Class] = {}
        self.pending: list[Request] = []
        self.finished: list[Request] = []
        self.used = 0
        self.peak = 0
        self.batch_hist: dict[int, int] = {}
        self.streams: dict[tuple, object] = {}
        self._ws1: dict[tuple, int] = {}   # one-object workspace of each class built so far
        self._rid = 0

    # ------------------------------------------------------------ submit
    def submit(self, req: Request) -> Request:
        if req.rid < 0:
            req.rid = self._rid
            self._rid += 1
        if req.t_arrival is None:
            req.t_arrival = self.clock()
        self.pending.append(req)
        return req

    # -------------------------------------------------------- accounting
    def _charge(self, n: int):
        self.used += n
        self.peak = max(self.peak, self.used)

    def _evict_idle(self, need: int, keep_key) -> bool:
        idle = sorted((c for c in self.classes.values()
                       if c.key != keep_key and not c.active and not c.inflight
                       and not any(r.key == c.key for r in self.pending)),
                      key=lambda c: c.last_used)
        for c in idle:
            if self.used + need <= self.budget:
                break
            self._charge(-(c.bytes_lib + c.bytes_ws1 + c.bytes_pool + c.bytes_keep))
            del self.classes[c.key]
        return self.used + need <= self.budget

    def _stream(self, key):
        if key not in self.streams:
            self.streams[key] = self.be.new_stream()
        return self.streams[key]

    def _open_class(self, req: Request):
        key = req.key
        lib = self.be.library_bytes(req.geom, req.h_dtype)
        if lib > self.budget:
            req.status = "rejected"
            return None
        # the operator keeps a workspace for one object (A^T d of each admitted
        # request, the power iteration of the step size), charged with the
        # library; its size is known once the class has been built
        need = lib + self._ws1.get(key, 0)
        if self.used + need > self.budget and not self._evict_idle(need, key):
            return None
        st = self._stream(key)
        op = self.be.build(req.geom, req.h_dtype, st)
        ws1 = self._ws1[key] = self.be.workspace_bytes(op, 1)
        if lib + ws1 + self.be.slot_bytes(op) + self.be.workspace_bytes(op, 1) > self.budget:
            req.status = "rejected"       # one request of this class can never fit
            return None
        if self.used + lib + ws1 > self.budget and not self._evict_idle(lib + ws1, key):
            return None                   # built but not admitted (first build only)
        cls = _Class(key=key, op=op, tau=self.be.step_size(op, st), bytes_lib=lib, bytes_ws1=ws1)
        self._charge(lib + ws1)
        self.classes[key] = cls
        return cls

    def _grow(self, cls: _Class) -> bool:
        new_cap = min(self.max_batch, max(1, 2 * cls.cap))
        if new_cap <= cls.cap:
            return False
        need = new_cap * self.be.slot_bytes(cls.op) + self.be.workspace_bytes(cls.op, new_cap)
        # the old pool stays alive (and charged) until the iterations queued
        # on it have ended, so the new one is charged in full
        if self.used + need > self.budget and not self._evict_idle(need, cls.key):
            return False
        st = self._stream(cls.key)
        pool, ws = self.be.alloc_pool(cls.op, new_cap, st)
        if cls.cap:
            self.be.copy_rows(cls.pool, pool, len(cls.active), st)
            cls.keep.append((cls.pool, cls.ws, cls.bytes_pool, [ev for ev, _ in cls.inflight]))
        cls.bytes_keep += cls.bytes_pool
        cls.pool, cls.ws, cls.cap = pool, ws, new_cap
        self._charge(need)
        cls.bytes_pool = need
        return True

    # ------------------------------------------------------------ ticks
    def _admit(self):
        still = []
        for req in self.pending:
            cls = self.classes.get(req.key)
            if cls is None:
                cls = self._open_class(req)
                if cls is None:
                    if req.status != "rejected":
                        still.append(req)
                    else:
                        self.finished.append(req)
                    continue
            if len(cls.active) >= cls.cap and not self._grow(cls):
                still.append(req)
                continue
            i = len(cls.active)
            st = self._stream(cls.key)
            self.be.load_row(cls.pool, i, req.d, st, op=cls.op)
            cls.active.append(_Slot(req))
            req.status = "running"
            req.t_admit = self.clock()
            if req.tau is None:
                req.tau = cls.tau
        self.pending = still

    def _retire(self, cls: _Class):
        # queued iterations end in order; their finished requests complete
        now = None
        while cls.inflight and self.be.done(cls.inflight[0][0]):
            _, results = cls.inflight.pop(0)
            now = self.clock() if now is None else now
            for req, x, flag in results:
                req.x = x
                req.t_done = now
                req.status = "nonfinite" if bool(flag) else "done"
                self.finished.append(req)
        still = []
        for entry in cls.keep:
            if all(self.be.done(ev) for ev in entry[3]):
                self._charge(-entry[2])
                cls.bytes_keep -= entry[2]
            else:
                still.append(entry)
        cls.keep = still

    def _launch(self, cls: _Class, depth: int):
        st = self._stream(cls.key)
        while cls.active and len(cls.inflight) < depth:
            n = len(cls.active)
            betas, taus, lams, nns = [], [], [], []
            for s in cls.active:
                t_next = (1.0 + math.sqrt(1.0 + 4.0 * s.t * s.t)) / 2.0
                betas.append((s.t - 1.0) / t_next)
                s.t = t_next
                taus.append(s.req.tau)
                lams.append(s.req.lam)
                nns.append(s.req.nonneg)
            self.be.step(cls.op, cls.pool, cls.ws, n, betas, taus, lams, nns, st)
            # slots whose last iteration this is: result taken right behind
            # it on the stream, row handed to the last active slot
            results = []
            for i in range(n - 1, -1, -1):
                s = cls.active[i]
                s.k += 1
                if s.k < s.req.niter:
                    continue
                x, flag = self.be.take_result(cls.pool, i, st)
                results.append((s.req, x, flag))
                last = len(cls.active) - 1
                if i != last:
                    self.be.move_row(cls.pool, last, i, st)
                    cls.active[i] = cls.active[last]
                cls.active.pop()
            cls.inflight.append((self.be.mark(st), results))
            cls.last_used = self.clock()
            self.batch_hist[n] = self.batch_hist.get(n, 0) + 1

    def poll(self) -> bool:
        """One scheduler tick.  Returns True while work remains."""
        for cls in list(self.classes.values()):
            if cls.inflight or cls.keep:
                self._retire(cls)
        self._admit()
        working = sum(1 for c in self.classes.values() if c.active or c.inflight)
        depth = self.depth if working <= 1 else 1
        for cls in self.classes.values():
            self._launch(cls, depth)
        busy = any(c.active or c.inflight for c in self.classes.values())
        return busy or bool(self.pending)

    def run_until_idle(self, sleep: float = 0.0):
        while self.poll():
            if sleep:
                time.sleep(sleep)

    # ------------------------------------------------------------ stats
    def stats(self) -> dict:
        lat = sorted(r.latency for r in self.finished if r.latency is not None)
        out = {"completed": len(lat), "hbm_peak_bytes": self.peak, "batch_hist": dict(self.batch_hist)}
        if lat:
            out["p50_s"] = _pct(lat, 50)
            out["p99_s"] = _pct(lat, 99)
            span = max(r.t_done for r in self.finished if r.t_done) - min(r.t_arrival for r in self.finished)
            out["recon_per_s"] = len(lat) / span if span > 0 else float("inf")
        return out


def _pct(sorted_vals, p):
    if not sorted_vals:
        return None
    k = (len(sorted_vals) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return sorted_vals[lo] + (sorted_vals[hi] - sorted_vals[lo]) * (k - lo)


def run_fifo(backend, requests, clock=time.perf_counter):
    """Baseline: one request at a time in arrival order, no batching; requests
    arrive on their own schedule (t_arrival) and wait for the GPU."""
    srv = Server(backend, hbm_budget=1 << 62, max_batch=1, clock=clock)
    order = sorted(requests, key=lambda r: r.t_arrival)
    for r in order:
        while clock() < r.t_arrival:
            pass
        srv.submit(r)
        srv.run_until_idle()
    return srv
