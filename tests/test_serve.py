"""Scheduler logic of the continuous-batching server (CPU, float64 fake device)."""
import numpy as np

from oracle import hlib, operators as ops, solvers
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry
from paper_2603_28150_amd.serve import Request, Server, run_fifo


class _Ev:
    def __init__(self, t):
        self.t = t


class CpuBackend:
    """Same interface as HipBackend; every step runs at once in float64 and
    the library/slot sizes are the real ones of the float32 layouts."""

    def __init__(self, clock):
        self.clock = clock
        self.built = []

    def _og(self, g):
        return OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim)

    def library_bytes(self, geom, h_dtype):
        nh = geom.nx // 2 + 1
        return nh * geom.ny * geom.nz * geom.nt * (4 if h_dtype == "f32" else 2)

    def build(self, geom, h_dtype, stream):
        self.built.append((geom, h_dtype))

        class Op:
            pass
        op = Op()
        op.geom = geom
        op.Hh = hlib.H_half(self._og(geom))
        op.x_shape = (geom.nz, geom.ny, geom.nx)
        op.d_shape = (geom.nt, geom.ny, geom.nx)
        return op

    def step_size(self, op, stream):
        return 1.0 / solvers.norm_exact(op.Hh)

    def slot_bytes(self, op):
        g = op.geom
        return 4 * g.nx * g.ny * (2 * g.nz + g.nt)

    def workspace_bytes(self, op, cap):
        return 0

    def new_stream(self):
        return None

    def alloc_pool(self, op, cap, stream):
        return {"x": np.zeros((cap,) + op.x_shape), "z": np.zeros((cap,) + op.x_shape),
                "d": np.zeros((cap,) + op.d_shape), "bad": np.zeros(cap, dtype=int)}, None

    def load_row(self, pool, i, d, stream, op=None):
        pool["d"][i] = d
        pool["x"][i] = 0
        pool["z"][i] = 0
        pool["bad"][i] = 0

    def move_row(self, pool, src, dst, stream):
        for k in pool:
            pool[k][dst] = pool[k][src]

    def copy_rows(self, old, new, n, stream):
        for k in old:
            new[k][:n] = old[k][:n]

    def step(self, op, pool, ws, n, betas, taus, lams, nonnegs, stream):
        for i in range(n):
            x_prev, z = pool["x"][i].copy(), pool["z"][i].copy()
            with np.errstate(all="ignore"):
                x = solvers.fista(lambda v: ops.A_fft(op.Hh, v), lambda v: ops.AT_fft(op.Hh, v),
                                  pool["d"][i], op.x_shape, 1, taus[i], lams[i], nonneg=nonnegs[i],
                                  momentum=False, z0=z, x_prev0=x_prev)[0]
                pool["z"][i] = x + betas[i] * (x - x_prev)
            pool["x"][i] = x
            if not np.all(np.isfinite(x)):
                pool["bad"][i] = 1
        return _Ev(self.clock())

    def mark(self, stream):
        return _Ev(self.clock())

    def done(self, ev):
        return True

    def take_result(self, pool, i, stream):
        return pool["x"][i].copy(), bool(pool["bad"][i])


G1 = Geometry.paper_like(16, 16, 8, 24)
G2 = Geometry.paper_like(32, 16, 6, 20)


def _req(g, seed, niter, **kw):
    o = OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c)
    Hh = hlib.H_half(o)
    p0 = inputs.gaussian_blobs((g.nz, g.ny, g.nx), seed=seed)
    clean = ops.A_fft(Hh, p0)
    d = clean + inputs.NOISE_20DB * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=seed + 1)
    return Request(geom=g, d=d, niter=niter, **kw), Hh


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def _standalone(Hh, d, niter, tau, lam=0.0, nonneg=True):
    return solvers.fista(lambda v: ops.A_fft(Hh, v), lambda v: ops.AT_fft(Hh, v), d,
                         (d.shape[0] and Hh.shape[2], Hh.shape[0], 2 * (Hh.shape[1] - 1)),
                         niter, tau, lam, nonneg=nonneg)[-1]


def test_mixed_requests_equal_standalone_fista():
    clock = Clock()
    srv = Server(CpuBackend(clock), hbm_budget=1 << 40, max_batch=4, clock=clock)
    reqs = []
    for i, (g, n) in enumerate([(G1, 5), (G2, 7), (G1, 9), (G1, 3), (G2, 4), (G1, 6)]):
        r, Hh = _req(g, 100 + 10 * i, n, lam=0.01 * (i % 2))
        reqs.append((r, Hh))
        srv.submit(r)
        srv.poll()                      # requests arrive while others run
    srv.run_until_idle()
    for r, Hh in reqs:
        assert r.status == "done"
        ref = _standalone(Hh, r.d, r.niter, r.tau, r.lam)
        assert np.array_equal(r.x, ref), r.rid
    st = srv.stats()
    assert st["completed"] == 6 and st["p99_s"] >= st["p50_s"] > 0
    assert max(st["batch_hist"]) > 1     # batching did happen


def test_admission_respects_the_hbm_budget():
    clock = Clock()
    be = CpuBackend(clock)
    lib1, lib2 = be.library_bytes(G1, "f32"), be.library_bytes(G2, "f32")
    slot1 = 4 * 16 * 16 * (2 * 8 + 24)
    slot2 = 4 * 32 * 16 * (2 * 6 + 20)
    # room for the G1 library with two slots, or the G2 library with one
    budget = max(lib1 + 2 * slot1, lib2 + slot2) + 1000
    assert lib1 + 4 * slot1 > budget and lib1 + lib2 + slot2 > budget
    srv = Server(be, hbm_budget=budget, max_batch=8, clock=clock)
    r1, _ = _req(G1, 1, 4)
    r2, _ = _req(G1, 2, 4)
    r3, _ = _req(G1, 3, 4)
    r4, _ = _req(G2, 4, 3)
    for r in (r1, r2, r3, r4):
        srv.submit(r)
    srv.poll()
    assert srv.used <= srv.budget
    assert r3.status == "pending" and r4.status == "pending"   # no room yet
    srv.run_until_idle()
    assert all(r.status == "done" for r in (r1, r2, r3, r4))
    assert srv.peak <= srv.budget
    assert be.built.count((G1, "f32")) >= 1 and (G2, "f32") in be.built


def test_oversized_request_is_rejected():
    clock = Clock()
    srv = Server(CpuBackend(clock), hbm_budget=1000, clock=clock)
    r, _ = _req(G1, 5, 2)
    srv.submit(r)
    srv.run_until_idle()
    assert r.status == "rejected" and r.x is None


def test_nonfinite_request_is_isolated():
    clock = Clock()
    srv = Server(CpuBackend(clock), hbm_budget=1 << 40, max_batch=4, clock=clock)
    good, Hh = _req(G1, 7, 6)
    bad, _ = _req(G1, 8, 80)
    srv.submit(good)
    srv.submit(bad)
    srv.poll()
    bad.tau = 1e6 * good.tau            # far beyond 2/L: the iterate overflows
    srv.run_until_idle()
    assert good.status == "done"
    assert np.array_equal(good.x, _standalone(Hh, good.d, 6, good.tau))
    assert bad.status == "nonfinite"


def test_fifo_baseline_runs_one_at_a_time():
    clock = Clock()
    reqs = [_req(G1, 20 + i, 3)[0] for i in range(3)]
    for i, r in enumerate(reqs):
        r.t_arrival = 0.0
    srv = run_fifo(CpuBackend(clock), reqs, clock=clock)
    assert set(srv.batch_hist) == {1}
    assert all(r.status == "done" for r in reqs)


class WsBackend(CpuBackend):
    """CpuBackend whose operators also hold workspaces (of known sizes)."""

    def workspace_bytes(self, op, cap):
        return 1000 * cap + 500


def test_accounting_charges_workspaces_and_replaced_pools():
    # the operator's own one-object workspace is charged with its library,
    # a pool replaced while growing stays charged until the step that used it
    # has ended, and what is charged after the work drains is exactly what
    # the classes still hold
    clock = Clock()
    be = WsBackend(clock)
    srv = Server(be, hbm_budget=1 << 40, max_batch=4, clock=clock)
    reqs = [_req(G1, 30 + i, 10 + i)[0] for i in range(4)]   # all four overlap: the pool grows to 4
    growth = []
    for r in reqs:
        srv.submit(r)
        srv.poll()
        growth.append(srv.used)
    cls = srv.classes[(G1, "f32")]
    assert cls.bytes_ws1 == 1500
    srv.run_until_idle()
    assert all(r.status == "done" for r in reqs)
    assert cls.bytes_keep == 0 and not cls.keep
    held = sum(c.bytes_lib + c.bytes_ws1 + c.bytes_pool for c in srv.classes.values())
    assert srv.used == held
    slot = be.slot_bytes(cls.op)
    # the peak saw the old pool and the new one together at least once
    assert srv.peak >= cls.bytes_lib + cls.bytes_ws1 + cls.bytes_pool + (2 * slot + be.workspace_bytes(None, 2))


def test_class_waiting_for_memory_is_not_rebuilt_every_tick():
    # the budget fits G1's class and G2's library, but not G2's library with
    # its workspace: G2 is built once, found not to fit, and then waits without
    # being built again each tick until G1 goes idle and is evicted
    clock = Clock()
    be = WsBackend(clock)
    lib1, lib2 = be.library_bytes(G1, "f32"), be.library_bytes(G2, "f32")
    slot1 = 4 * 16 * 16 * (2 * 8 + 24)
    held1 = lib1 + 1500 + slot1 + 1500               # library, own workspace, one slot + its workspace
    budget = held1 + lib2 + 700                       # G2's library fits, with its 1,500-byte workspace not
    srv = Server(be, hbm_budget=budget, max_batch=1, clock=clock)
    r1, _ = _req(G1, 40, 30)   # still running after the polls below (two iterations queued per poll)
    srv.submit(r1)
    srv.poll()
    r2, _ = _req(G2, 41, 3)
    srv.submit(r2)
    for _ in range(8):
        srv.poll()
    assert r2.status == "pending" and r1.status == "running"
    assert be.built.count((G2, "f32")) == 1
    srv.run_until_idle()
    assert r1.status == "done" and r2.status == "done"
    assert be.built.count((G2, "f32")) == 2 and srv.peak <= budget


class LateBackend(CpuBackend):
    """CpuBackend whose queued iterations report done only on the second
    query, so that several stay queued on a class at once."""

    def __init__(self, clock):
        super().__init__(clock)
        self.asked = set()

    def done(self, ev):
        if id(ev) in self.asked:
            return True
        self.asked.add(id(ev))
        return False


def test_queued_iterations_respect_the_depth_and_the_results():
    # a class keeps at most `depth` iterations queued (it queues more than
    # one only while it is the only class with work); iteration counts advance at
    # launch, results are taken right after a request's last iteration and
    # its row handed on, so every result equals the standalone FISTA bit for
    # bit whatever the depth
    for depth in (1, 2, 3):
        clock = Clock()
        srv = Server(LateBackend(clock), hbm_budget=1 << 40, max_batch=3, clock=clock, depth=depth)
        reqs = []
        peak = 0

        def check():
            nonlocal peak
            for c in srv.classes.values():
                assert len(c.inflight) <= depth
                peak = max(peak, len(c.inflight))
        for i, (g, n) in enumerate([(G1, 4), (G1, 7), (G2, 5), (G1, 2), (G1, 6)]):
            r, Hh = _req(g, 300 + 10 * i, n)
            reqs.append((r, Hh))
            srv.submit(r)
            srv.poll()
            check()
        while srv.poll():
            check()
        assert peak == depth
        for r, Hh in reqs:
            assert r.status == "done"
            assert np.array_equal(r.x, _standalone(Hh, r.d, r.niter, r.tau)), (depth, r.rid)
        if depth > 1:
            assert max(srv.batch_hist) > 1
