"""GPU parity at the lengths the workloads run, through the C ABI.

* 100 FISTA iterations free-running (Sec. 2.3, eq. 12-15), every iterate
  against the FP64 oracle, on a grid that takes the benchmark's kernel paths:
  square (one library slab per radial class, eight-member work items, large
  classes split over several items) with 512 time samples (A's rows split
  over two workgroups), 20 dB noise, the step from 30 power iterations.
* The serving classes (64^2 x 64 x 256 and 128^2 x 96 x 384, FP32 and BF16
  libraries): 50-iteration reconstructions served in one continuous-batching
  run, each result against the oracle (BF16 against the oracle applying the
  same quantised library, and against the exact one).

Bars: relative l2 1e-5 (FP32, and BF16 against the quantised oracle), 5e-3
(BF16 against the exact oracle).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle_threads
from oracle import operators as ops, quant, solvers
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import inputs
from paper_2603_28150_amd.op import Geometry, Operator
from paper_2603_28150_amd.serve import HipBackend, Request, Server

pytestmark = pytest.mark.gpu


def og(g: Geometry) -> OGeom:
    return OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim)


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def data_20db(A, shape, seed):
    """Vascular phantom (40 tubes), its data plus 20 dB Gaussian noise."""
    p0 = inputs.vascular_phantom(shape, seed=seed)
    clean = A(p0)
    return clean + inputs.NOISE_20DB * np.sqrt(np.mean(clean ** 2)) * inputs.noise_like(clean.shape, seed=seed + 1)


def test_fista_100_iterations_free_running_every_iterate():
    g = Geometry.paper_like(64, 64, 64, 512)
    Hh = oracle_threads.H_half(og(g))
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    shape = (g.nz, g.ny, g.nx)
    d = data_20db(A, shape, seed=1201)
    op = Operator(g)
    info = op.info()
    assert info["members_max"] == 8 and info["nitems"] > info["nclass"]   # radial fold, split classes
    # step size: 30 power iterations on A^T A from a seeded random start,
    # the same on both sides
    v0 = inputs.gaussian_random(shape, seed=1002)
    Lo = solvers.power_iteration(A, AT, v0, 30)
    L, trace = op.power_norm(dev(v0), 30)
    assert np.max(np.abs(np.array(trace) - Lo) / np.array(Lo)) < 1e-5
    tau = float(np.float32(1.0 / Lo[-1]))
    K = 100
    xs = solvers.fista(A, AT, d, shape, K, tau, 0.0, nonneg=True)
    dd = dev(d)
    errs = [rel(host(op.recon_fista(dd, k, tau, 0.0, nonneg=True)), xs[k - 1]) for k in range(1, K + 1)]
    print("FISTA 64x64x64x512 free-running rel. l2 error at k = 1, 10, 20, ..., 100:",
          " ".join(f"{errs[k - 1]:.2e}" for k in [1] + list(range(10, K + 1, 10))), flush=True)
    assert max(errs) < 1e-5, errs
    # teacher-forced: one oracle step from the GPU's own state (x_{k-1}, z_k),
    # stepped by the batched entry point with the Gram-block gradient
    atd = op.apply_AT(dd)[None]
    x = torch.zeros((1,) + shape, device="cuda")
    z = torch.zeros_like(x)
    betas = solvers.momentum_weights(K)
    states = {}
    for k in range(1, K + 1):
        if k in (1, 2, 25, 50, 99, 100):
            states[k] = [host(x[0]), host(z[0])]
        op.fista_step_normal(atd, x, z, [betas[k - 1]], [tau], [0.0], [True])
        if k in states:
            states[k].append(host(x[0]))

    def forced(k):
        xp, zp, xg = states[k]
        xo = solvers.fista(A, AT, d, shape, 1, tau, 0.0, nonneg=True, z0=zp, x_prev0=xp, k0=k - 1)[0]
        return rel(xg, xo)

    with ThreadPoolExecutor(len(states)) as ex:
        forced_errs = dict(zip(states, ex.map(forced, states)))
    assert max(forced_errs.values()) < 1e-5, forced_errs
    assert rel(states[100][2], host(op.recon_fista(dd, K, tau, 0.0, nonneg=True))) < 1e-5


@pytest.mark.parametrize("shape", [(64, 64, 64, 256), (128, 128, 96, 384)],
                         ids=["64x64x64x256", "128x128x96x384"])
def test_served_fifty_iterations_match_oracle(shape):
    g = Geometry.paper_like(*shape)
    Hh = oracle_threads.H_half(og(g))
    Hq, _ = quant.quantise(Hh, "bf16")
    xshape = (g.nz, g.ny, g.nx)
    A = lambda v: ops.A_fft(Hh, v)
    AT = lambda v: ops.AT_fft(Hh, v)
    ds = [data_20db(A, xshape, seed) for seed in (1301, 1311)]
    v0 = inputs.gaussian_random(xshape, seed=1002)
    tau = float(np.float32(1.0 / solvers.power_iteration(A, AT, v0, 30)[-1]))
    # both classes (FP32 and BF16 library) in one server: two requests each,
    # batched per class, the classes on their own streams
    srv = Server(HipBackend(), hbm_budget=32 << 30, max_batch=16)
    reqs = [srv.submit(Request(geom=g, d=dev(d), niter=50, h_dtype=kind, tau=tau))
            for kind in ("f32", "bf16") for d in ds]
    srv.run_until_idle()
    torch.cuda.synchronize()
    assert all(r.status == "done" for r in reqs)
    assert max(srv.stats()["batch_hist"]) == 2

    def traj(args):
        H, d = args
        return solvers.fista(lambda v: ops.A_fft(H, v), lambda v: ops.AT_fft(H, v), d, xshape, 50, tau,
                             0.0, nonneg=True)[-1]

    jobs = [(Hh, ds[0]), (Hh, ds[1]), (Hq, ds[0]), (Hq, ds[1])]
    with ThreadPoolExecutor(len(jobs)) as ex:
        exact0, exact1, quant0, quant1 = ex.map(traj, jobs)
    exact, quantised = [exact0, exact1], [quant0, quant1]
    for i in range(2):
        xf, xb = host(reqs[i].x), host(reqs[2 + i].x)
        e_f32, e_q, e_bx = rel(xf, exact[i]), rel(xb, quantised[i]), rel(xb, exact[i])
        print(f"served {shape} request {i}: FP32 vs oracle {e_f32:.2e}, BF16 vs quantised oracle {e_q:.2e}, "
              f"BF16 vs exact oracle {e_bx:.2e}", flush=True)
        assert e_f32 < 1e-5
        assert e_q < 1e-5
        assert e_bx < 5e-3
