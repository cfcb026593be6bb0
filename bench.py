#!/usr/bin/env python3
"""Benchmark of the planar photoacoustic operator on one MI355X.

Step = one forward A and one adjoint A^T (the pair every gradient of the
reconstruction needs, eq. 15) at 256 x 256 x 128 depths x 512 time samples,
float32, on a seeded synthetic vascular phantom (40 polyline tubes) resident
in HBM.  Each apply is issued as its three steps through the C ABI
(spectrum -> contraction -> inverse spectrum; the same kernels pat_apply_A
launches) so that HIP events around the contraction, the dominant kernel,
give its duration inside the timed region.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the operator runs on one GPU
(the multi-GPU sharding is a design note, not code).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A+Aᵀ applies/s at 256²×128×512, % HBM roofline; served recon p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BIG = dict(nx=256, ny=256, nz=128, nt=512)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def contraction_bytes(info: dict, nk: int, nz: int, nt: int, adjoint: bool, B: int = 1) -> int:
    """Algorithmic bytes of one contraction launch: every stored class slab
    of the library once (slab_bytes: one slab serves all frequencies of its
    symmetry class), the input spectrum read once and the output spectrum
    written once (nk frequencies; unused spectrum rows are neither read nor
    written)."""
    slab = info["slab_bytes_AT"] if adjoint else info["slab_bytes_A"]
    return slab + B * nk * (nz + nt) * 8


def reread_bytes(info: dict, adjoint: bool) -> int:
    """Library bytes the work items read beyond one read of every slab: a
    class with more members than an item holds is split into items that each
    stream its slab (the later reads meant to hit the XCD's L2)."""
    if adjoint:
        return info["read_bytes_AT"] - info["slab_bytes_AT"]
    return info["read_bytes_A"] - info["slab_bytes_A"]


def fista_algorithmic_bytes(info: dict, nk: int, nz: int, nt: int, nxy: int, niter: int) -> int:
    """What 100 iterations of the Gram-block FISTA must move at least: A^T d
    once (one adjoint contraction's algorithmic bytes plus d read and A^T d's
    spectrum written), then per iteration the Gram blocks once, the spectrum
    of A^T d read, and the update's object arrays (z and x_{k-1} read, x_k
    and z_{k+1} written: 16 bytes per voxel; the gradient never leaves the
    chip)."""
    n = nz * nxy
    setup = contraction_bytes(info, nk, nz, nt, True) + 4 * nt * nxy
    return setup + niter * (info["gram_bytes"] + 8 * nz * nk + 16 * n)


def fista_gram_bytes(info: dict, nk: int, nz: int, nt: int, nxy: int, niter: int) -> int:
    """Bytes that pat_recon_fista's passes move with the Gram-block gradient
    (periodic boundary, one object, nxy = nx * ny sensor points, the update
    fused into the inverse transform as at fast sizes with rows of whole
    16-byte units, no trace):
    set-up: the spectrum of d (row pass: d in, intermediate out; column pass:
    intermediate in, spectrum out), one A^T contraction, x and z cleared, and
    z read by the first iteration's row pass;
    per iteration: the spectrum of z (its row pass done by the previous
    update: the column pass moves two spectrum-sized arrays), the Gram
    contraction (blocks, z^ and (A^T d)^ in, result out), the inverse
    spectrum's column pass (two spectrum-sized passes) and its row pass with
    the update and the next row pass (one spectrum-sized array in and one
    out; x, z in and out)."""
    n = nz * nxy
    setup = 4 * nt * nxy + 24 * nt * nk + contraction_bytes(info, nk, nz, nt, True) + 8 * n + 4 * n
    per_iter = 16 * n + 72 * nz * nk + info["gram_bytes"]
    return setup + niter * per_iter


def time_pairs(op, x, steps, warmup, B=1):
    """Times `steps` A+A^T pairs built from stage calls; returns
    (seconds total, mean contraction ms for A, for A^T)."""
    import torch
    g = op.geom
    Sz, St = B * g.nz, B * g.nt
    Xs = op.spectrum_buffer(Sz)
    Ds = op.spectrum_buffer(St)
    y = torch.empty((B,) + op.d_shape if B > 1 else op.d_shape, dtype=torch.float32, device=op.device)
    gx = torch.empty_like(x)

    def pair(ev=None):
        if ev: ev[0].record()
        op.spectrum(x, Sz, Xs, B_ws=B)
        if ev: ev[1].record()
        op.contract(Xs, Ds, adjoint=False, B=B)
        if ev: ev[2].record()
        op.inverse_spectrum(Ds, St, y, B_ws=B)
        if ev: ev[3].record()
        op.spectrum(y, St, Ds, B_ws=B)
        if ev: ev[4].record()
        op.contract(Ds, Xs, adjoint=True, B=B)
        if ev: ev[5].record()
        op.inverse_spectrum(Xs, Sz, gx, B_ws=B)
        if ev: ev[6].record()

    for _ in range(warmup):
        pair()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        pair(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(6)] for e in evs])
    el = per.mean(axis=0)
    log("  stage ms (spec_z, contract_A, ispec_t, spec_t, contract_AT, ispec_z): "
        + ", ".join(f"{v:.3f}" for v in el))
    time_pairs.last = {"pair_ms": per.sum(axis=1), "stage_ms": el}
    return t1 - t0, float(el[1]), float(el[4])


# transverse frequencies (m, p) where GPU outputs are compared with the oracle:
# DC, axes, Nyquist corners, multi-member classes and random ones
SAMPLE_M = np.array([0, 128, 0, 128, 3, 7, 100, 41, 128, 17])
SAMPLE_P = np.array([0, 0, 128, 128, 250, 3, 9, 200, 77, 17])


def spectra_at(y, M=SAMPLE_M, P=SAMPLE_P) -> np.ndarray:
    """2D DFT over (x, y) of GPU output slices at the sampled frequencies,
    float64: [B, K, n] (y: [B, n, ny, nx] device tensor)."""
    import torch
    out = []
    for b in range(y.shape[0]):
        F = torch.fft.rfft2(y[b].double())            # [n, ny, nx/2+1]
        out.append(F[:, torch.as_tensor(P), torch.as_tensor(M)].T.cpu().numpy())
    return np.stack(out)


def oracle_accuracy(samples: dict) -> dict:
    """Relative error per object of GPU outputs against the float64 oracle at
    the sampled frequencies (|| D_gpu - D_oracle || / || D_oracle || over
    those frequencies and all time samples)."""
    from oracle import hlib, operators as ops
    from oracle.geometry import paper_like
    g = paper_like(**BIG)
    Hk = hlib.H_hat(g, SAMPLE_M, SAMPLE_P)
    out = {}
    for name, (x64s, D) in samples.items():
        errs = []
        for b in range(len(x64s)):
            Do = ops.A_at_freqs(Hk, x64s[b], SAMPLE_M, SAMPLE_P)
            errs.append(float(np.linalg.norm(D[b] - Do) / np.linalg.norm(Do)))
        out[name] = {"max": max(errs), "median": float(np.median(errs)), "per_object": errs}
    return out


def oracle_library(g, threads: int) -> np.ndarray:
    """The oracle's half-spectrum library (its direct q-sums, FP64), the
    frequencies split into blocks that `threads` host threads compute (numpy
    releases the GIL in the cosines and matrix products; BLAS held to one
    thread per caller).  float64 [Ny, Nx/2+1, Nz, Nt]."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import hlib
    nh = g.nx // 2 + 1
    nk = g.ny * nh
    out = np.empty((nk, g.nz, g.nt))
    k = np.arange(nk)
    m, p = k % nh, k // nh
    block = 128

    def run(s0):
        out[s0:s0 + block] = hlib.H_hat(g, m[s0:s0 + block], p[s0:s0 + block], chunk=block)

    with threadpool_limits(1), ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(0, nk, block)))
    return out.reshape(g.ny, nh, g.nz, g.nt)


def cpu_baseline(x64: np.ndarray, runs: int = 3) -> dict:
    """The FP64 oracle on the host at the full 256x256x128x512 size: its
    half-spectrum library built once (time measured), then `runs` forward +
    adjoint pairs, each A and A^T in full (the oracle's numpy transforms and
    per-frequency products, one thread); median and mean over the runs (the
    paper reports the mean of three runs, Sec. 3.2).  Beside it, the FFT form
    of the operator on every host core with the same library (FP64, FP32)."""
    from threadpoolctl import threadpool_limits
    from oracle import operators as ops
    from oracle.geometry import paper_like
    from paper_2603_28150_amd import inputs
    g = paper_like(**BIG)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    Hh = oracle_library(g, cores)
    t_build = time.perf_counter() - t0
    log(f"  oracle library: {t_build:.1f} s on {cores} threads ({Hh.nbytes / 1e9:.1f} GB)")
    r64 = inputs.gaussian_random((g.nt, g.ny, g.nx), seed=8)
    tA, tAT = [], []
    with threadpool_limits(1):
        for _ in range(runs):
            t0 = time.perf_counter()
            ops.A_fft(Hh, x64)
            t1 = time.perf_counter()
            ops.AT_fft(Hh, r64)
            t2 = time.perf_counter()
            tA.append(t1 - t0)
            tAT.append(t2 - t1)
    pair = [a + b for a, b in zip(tA, tAT)]
    log(f"  oracle A+AT: median {np.median(pair):.2f} s, mean {np.mean(pair):.2f} s per pair")
    out = {"value": 1.0 / float(np.median(pair)), "unit": "A+Aᵀ pairs/s", "cores": 1, "kind": "oracle",
           "sample": f"{runs} full forward+adjoint pairs of the oracle (FP64, numpy transforms and "
                     f"per-frequency products, one thread) at 256x256x128x512 with its half-spectrum "
                     f"library in host memory; value = 1 / median pair time",
           "median_s_per_pair": float(np.median(pair)), "mean_s_per_pair": float(np.mean(pair)),
           "A_s": tA, "AT_s": tAT,
           "oracle_library_build_s": t_build, "oracle_library_build_threads": cores,
           "oracle_library_GB": Hh.nbytes / 1e9,
           "cpu": host_cpu()}
    out["fft_path"] = cpu_fft_path(x64, r64, Hh, cores, runs)
    return out


def host_cpu() -> dict:
    """CPU model, logical cores and RAM of the host (Linux /proc)."""
    model, mem = platform.processor() or platform.machine(), None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "ram_GiB": mem}


def cpu_fft_path(x64: np.ndarray, r64: np.ndarray, Hh: np.ndarray, cores: int, runs: int) -> dict:
    """The FFT form of the operator on the host with the precomputed library,
    FP64 and FP32, on every core: scipy's pocketfft transforms (workers =
    cores) and the per-frequency products on `cores` threads over blocks of
    frequencies.  `runs` full pairs each, median reported; 100-iteration
    FISTA estimated as 100 explicit-gradient pairs."""
    from concurrent.futures import ThreadPoolExecutor
    import scipy.fft as sf
    from threadpoolctl import threadpool_limits
    nz, ny, nx = x64.shape
    nt = r64.shape[0]
    nh = nx // 2 + 1
    nk = ny * nh
    out = {}
    blocks = [(s0, min(nk, s0 + 512)) for s0 in range(0, nk, 512)]
    for dt, ct, name in ((np.float64, np.complex128, "fp64"), (np.float32, np.complex64, "fp32")):
        H = Hh.reshape(nk, nz, nt) if dt is np.float64 else Hh.reshape(nk, nz, nt).astype(np.float32)
        x, r = x64.astype(dt), r64.astype(dt)

        def contract(Xk, adjoint):
            res = np.empty((nk, nz if adjoint else nt), ct)

            def run(bk):
                s0, s1 = bk
                if adjoint:
                    Rs = np.stack([Xk[s0:s1].real, Xk[s0:s1].imag], axis=2)
                    G = np.matmul(H[s0:s1], Rs)
                    res[s0:s1] = G[:, :, 0] + 1j * G[:, :, 1]
                else:
                    Xs = np.stack([Xk[s0:s1].real, Xk[s0:s1].imag], axis=1)
                    D = np.matmul(Xs, H[s0:s1])
                    res[s0:s1] = D[:, 0, :] + 1j * D[:, 1, :]

            with ThreadPoolExecutor(cores) as ex:
                list(ex.map(run, blocks))
            return res

        pairs = []
        with threadpool_limits(1):
            for _ in range(runs):
                t0 = time.perf_counter()
                X = sf.rfft2(x, workers=cores).reshape(nz, nk).T
                D = contract(X, False)
                sf.irfft2(D.T.reshape(nt, ny, nh), s=(ny, nx), workers=cores)
                R = sf.rfft2(r, workers=cores).reshape(nt, nk).T
                G = contract(R, True)
                sf.irfft2(G.T.reshape(nz, ny, nh), s=(ny, nx), workers=cores)
                pairs.append(time.perf_counter() - t0)
        med = float(np.median(pairs))
        out[name] = {"pairs_per_s": 1.0 / med, "s_per_pair": pairs, "fista100_s_estimate": 100.0 * med}
        log(f"  FFT path {name}: {1.0 / med:.2f} pairs/s on {cores} cores")
        del H
    out["cores"] = cores
    out["how"] = (f"scipy.fft rfft2/irfft2 of every slice ({cores} workers) and the per-frequency products "
                  f"on {cores} threads, library precomputed in host memory, {runs} full pairs each, median; "
                  f"FISTA estimate = 100 explicit-gradient iterations (one pair each), proximal step not counted")
    return out


CONTRACT_SRC = os.path.join(ROOT, "paper_2603_28150_amd", "csrc", "contract.hip")


def source_sha256(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def profile_traffic(kernel_bytes: int):
    """HBM traffic of the contraction from the committed rocprofv3 PMC summary,
    or None when there is none or it was taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "contract_fp32_256x256x128x512_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_sha256") != source_sha256(CONTRACT_SRC):
        return None
    return d.get("traffic_bytes_per_launch")


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Device-to-device copy rate (bytes read + written per second, GB/s): the
    achievable denominator next to the 8 TB/s specification."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16/FP16/batch/FISTA forms")
    ap.add_argument("--forms", default=",".join(FORMS),
                    help="comma-separated subset of the forms to run: " + ", ".join(FORMS))
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="measured requests per serving run (after 20 warm-up requests)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a device copy of 1 GiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the operator runs on one GPU only (no multi-GPU path); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_28150_amd import inputs
    from paper_2603_28150_amd.op import Geometry, Operator

    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.ones(1 << 28, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    geom = Geometry.paper_like(**BIG)
    t0 = time.perf_counter()
    op = Operator(geom, "f32")
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    info = op.info()
    log(f"library built in {t_build:.3f} s: {info}")
    # the same library by one k-space stepping run (reciprocity build), timed
    # beside a second closed-form build (both after the first, which also
    # loads the code object), and compared at the sampled frequencies
    builds = {}
    for name in ("step", "closed"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o2 = Operator(Geometry.paper_like(**BIG, build=name), "f32")
        torch.cuda.synchronize()
        builds[name] = time.perf_counter() - t0
        if name == "step":
            nh = geom.nx // 2 + 1
            step_diff = max(float((o2.export_H(int(p * nh + m), 1) - op.export_H(int(p * nh + m), 1)).abs().max())
                            for m, p in zip(SAMPLE_M, SAMPLE_P))
        del o2
        torch.cuda.empty_cache()
    log(f"library build: closed form {builds['closed']:.3f} s, k-space stepper {builds['step']:.3f} s, "
        f"largest difference at the sampled frequencies {step_diff:.2e}")
    x64 = inputs.vascular_phantom(op.x_shape, seed=1001)
    x = torch.from_numpy(x64.astype(np.float32)).cuda()

    secs, tA, tAT = time_pairs(op, x, args.steps, args.warmup)
    tp = time_pairs.last
    ms_step = secs / args.steps * 1e3
    copy_gbs = copy_bandwidth()
    value = args.steps / secs
    bA = contraction_bytes(info, op.nk, geom.nz, geom.nt, False)
    bAT = contraction_bytes(info, op.nk, geom.nz, geom.nt, True)
    achieved = (bA + bAT) / ((tA + tAT) * 1e-3) / 1e9
    log(f"A+AT: {ms_step:.3f} ms/pair, contraction A {tA:.3f} ms, AT {tAT:.3f} ms, {achieved:.0f} GB/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "A+Aᵀ pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded vascular phantom, 40 tubes)",
        "config": {"workload": "planar PAT operator: one A + one A^T, 256x256 transverse, "
                               "128 depths, 512 time samples, FP32 kernel library, batch 1",
                   "nx": 256, "ny": 256, "nz": 128, "nt": 512, "batch": 1,
                   "library_classes": info["nclass"], "library_build_s": builds["closed"],
                   "library_build_step_s": builds["step"], "library_step_vs_closed_max_abs": step_diff},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profile_traffic(bA),
                     "kernel": "k_contract (A and A^T, mean of both)",
                     "algorithmic_bytes_per_launch": (bA + bAT) / 2,
                     "reread_bytes_per_launch": (reread_bytes(info, False) + reread_bytes(info, True)) / 2,
                     "ms_per_launch": (tA + tAT) / 2,
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "timing": {"median_ms_per_pair": float(np.median(tp["pair_ms"])),
                   "min_ms_per_pair": float(np.min(tp["pair_ms"])),
                   "stage_ms": dict(zip(["spectrum_z", "contract_A", "inverse_spectrum_t",
                                         "spectrum_t", "contract_AT", "inverse_spectrum_z"],
                                        [float(v) for v in tp["stage_ms"]]))},
        # the paper's own speed figures, with the hardware it states (context,
        # not a baseline for this metric: other machine, other workload)
        "paper_context": {"claim": "forward operator two to three orders of magnitude faster than a k-Wave "
                                   "solve; 256^3 grid, 1000 time steps: ~1e3 s (k-Wave) vs a few s",
                          "hardware": "MATLAB, CPU only, 2x AMD EPYC 7662 (2x64 cores), 2 TiB RAM",
                          "source": "Sec. 3.2 (runtime comparison, Fig. 2)"},
    }

    samples = {}
    if not args.no_forms:
        out["forms"] = forms(op, x, x64, args, samples)
    if not args.no_serve:
        del op
        torch.cuda.empty_cache()
        out["serving"] = serving(args)
    if not args.no_cpu:
        log("cpu baseline (the oracle at full size) ...")
        out["cpu_baseline"] = cpu_baseline(x64)
        if samples:
            out["accuracy_vs_oracle"] = oracle_accuracy(samples)
            log(f"accuracy: { {k: v['max'] for k, v in out['accuracy_vs_oracle'].items()} }")
    print(json.dumps(out), flush=True)


FORMS = ("fista", "b1_16bit", "batch16", "linear", "paper_grids", "autograd")


def forms(op, x, x64, args, samples: dict) -> dict:
    """Secondary numbers on the same GPU: FISTA (Gram and explicit gradient),
    16-bit libraries, batches of 16, the autograd fit.  GPU output spectra at
    the sampled frequencies go to `samples` for the oracle comparison."""
    import math
    import torch
    from paper_2603_28150_amd import autograd, inputs
    from paper_2603_28150_amd.op import Geometry, Operator
    res = {}
    g = op.geom
    sel = set(args.forms.split(","))
    unknown = sel - set(FORMS)
    if unknown:
        raise SystemExit(f"bench.py: unknown forms {sorted(unknown)}")
    if "fista" in sel:
        # 100-iteration FISTA with the step from 30 power iterations, 20 dB noise
        clean = op.apply_A(x)
        samples["f32_b1"] = ([x64], spectra_at(clean[None]))
        sig = float(torch.sqrt(torch.mean(clean * clean)))
        noise = torch.from_numpy(inputs.noise_like(op.d_shape, seed=1501).astype(np.float32)).cuda()
        d = clean + inputs.NOISE_20DB * sig * noise
        v0 = torch.from_numpy(inputs.gaussian_random(op.x_shape, seed=1002).astype(np.float32)).cuda()
        t0 = time.perf_counter()
        L, _ = op.power_norm(v0, 30)
        t_pow = time.perf_counter() - t0
        op.recon_fista(d, 2, 1.0 / L)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.recon_fista(d, 100, 1.0 / L, 0.0, nonneg=True)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        res["fista100_fp32_s"] = t_f
        fb = fista_gram_bytes(op.info(), op.nk, g.nz, g.nt, g.nx * g.ny, 100)
        fa = fista_algorithmic_bytes(op.info(), op.nk, g.nz, g.nt, g.nx * g.ny, 100)
        res["fista100_traffic_GB"] = fb / 1e9
        res["fista100_traffic_frac_of_peak"] = fb / t_f / 1e9 / HBM_PEAK_GBS
        res["fista100_algorithmic_GB"] = fa / 1e9
        res["fista100_algorithmic_frac_of_peak"] = fa / t_f / 1e9 / HBM_PEAK_GBS
        res["power30_s"] = t_pow
        # the same iterations with the explicit gradient A^T (A z - d): two applies each
        xs = torch.zeros((1,) + op.x_shape, device="cuda")
        zs = torch.zeros_like(xs)
        ws = op.workspace(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tk = 1.0
        for _ in range(100):
            tn = (1.0 + math.sqrt(1.0 + 4.0 * tk * tk)) / 2.0
            op.fista_step(d[None], xs, zs, [(tk - 1.0) / tn], [1.0 / L], [0.0], [True], ws=ws)
            tk = tn
        torch.cuda.synchronize()
        res["fista100_explicit_fp32_s"] = time.perf_counter() - t0
        log(f"FISTA 100 it: {t_f:.3f} s (Gram; {res['fista100_traffic_GB']:.1f} GB moved by its passes, "
            f"{res['fista100_traffic_frac_of_peak']:.0%} of HBM peak; {res['fista100_algorithmic_GB']:.1f} GB "
            f"algorithmic, {res['fista100_algorithmic_frac_of_peak']:.0%}), "
            f"{res['fista100_explicit_fp32_s']:.3f} s (explicit); power 30 it {t_pow:.3f} s")
        del xs, zs, d, noise, clean
    if "b1_16bit" in sel:
        # 16-bit libraries, batch 1
        for kind in ("bf16", "f16"):
            o = Operator(g, kind)
            inf = o.info()
            secs, tA, tAT = time_pairs(o, x, max(5, args.steps // 2), 2)
            b = contraction_bytes(inf, o.nk, g.nz, g.nt, False) + contraction_bytes(inf, o.nk, g.nz, g.nt, True)
            res[f"{kind}_pairs_per_s"] = max(5, args.steps // 2) / secs
            res[f"{kind}_contract_GBs"] = b / ((tA + tAT) * 1e-3) / 1e9
            samples[f"{kind}_b1"] = ([x64], spectra_at(o.apply_A(x)[None]))
            log(f"{kind}: {res[f'{kind}_pairs_per_s']:.1f} pairs/s, contraction {res[f'{kind}_contract_GBs']:.0f} GB/s")
            del o
            torch.cuda.empty_cache()
    if "batch16" in sel:
        # batch of 16 objects, FP32 and BF16 libraries
        xb64 = [inputs.vascular_phantom(op.x_shape, seed=2001 + b) for b in range(16)]
        xb = torch.from_numpy(np.stack(xb64).astype(np.float32)).cuda()
        for kind in ("f32", "bf16"):
            o = op if kind == "f32" else Operator(g, kind)
            secs, tA, tAT = time_pairs(o, xb, 3, 1, B=16)
            inf = o.info()
            b = (contraction_bytes(inf, o.nk, g.nz, g.nt, False, B=16) +
                 contraction_bytes(inf, o.nk, g.nz, g.nt, True, B=16))
            res[f"batch16_{kind}_object_pairs_per_s"] = 16 * 3 / secs
            res[f"batch16_{kind}_contract_ms"] = [tA, tAT]
            res[f"batch16_{kind}_contract_GBs"] = b / ((tA + tAT) * 1e-3) / 1e9
            samples[f"{kind}_b16"] = (xb64, spectra_at(o.apply_A(xb)))
            log(f"batch16 {kind}: {res[f'batch16_{kind}_object_pairs_per_s']:.1f} object-pairs/s, contraction "
                f"A {tA:.3f} ms, AT {tAT:.3f} ms, {res[f'batch16_{kind}_contract_GBs']:.0f} GB/s algorithmic")
            if o is not op:
                del o
            torch.cuda.empty_cache()
        del xb
    if "linear" in sel:
        # zero-padded linear convolution (Sec. 2.3): same object and data grids,
        # transforms and library on the doubled 512^2 grid
        gl = Geometry.paper_like(g.nx, g.ny, g.nz, g.nt, boundary="linear")
        t0 = time.perf_counter()
        ol = Operator(gl, "f32")
        torch.cuda.synchronize()
        res["linear_library_build_s"] = time.perf_counter() - t0
        infl = ol.info()
        secs, tA, tAT = time_pairs(ol, x, max(5, args.steps // 2), 2)
        bl = contraction_bytes(infl, ol.nk, g.nz, g.nt, False) + contraction_bytes(infl, ol.nk, g.nz, g.nt, True)
        res["linear_pairs_per_s"] = max(5, args.steps // 2) / secs
        res["linear_contract_GBs"] = bl / ((tA + tAT) * 1e-3) / 1e9
        res["linear_library_GiB"] = (infl["slab_bytes_A"] + infl["slab_bytes_AT"]) / 2**30
        log(f"linear (512^2 transforms): {res['linear_pairs_per_s']:.1f} pairs/s, "
            f"contraction {res['linear_contract_GBs']:.0f} GB/s, library {res['linear_library_GiB']:.1f} GiB")
        del ol
        torch.cuda.empty_cache()
    if "paper_grids" in sel:
        # the paper's grid shapes on the linear boundary (Sec. 3.3-3.4): the in vivo
        # 384 x 326 x 96 grid at 50 um (384 samples chosen here) on 768^2
        # transforms, the wire phantom 202 x 202 x 37 at 10 um (256 samples) on 432^2
        # and the wire grid on the periodic boundary, whose 202-point axes run
        # chirp-z transforms (512-point convolutions)
        for name, gp in (("invivo_384x326x96x384", Geometry.paper_like(384, 326, 96, 384, dx=50e-6, boundary="linear")),
                         ("wire_202x202x37x256", Geometry.paper_like(202, 202, 37, 256, dx=10e-6, boundary="linear")),
                         ("wire_periodic_chirpz_202x202x37x256", Geometry.paper_like(202, 202, 37, 256, dx=10e-6))):
            t0 = time.perf_counter()
            op_ = Operator(gp, "f32")
            torch.cuda.synchronize()
            build_s = time.perf_counter() - t0
            inf_ = op_.info()
            xp = torch.from_numpy(inputs.vascular_phantom(op_.x_shape, seed=4101).astype(np.float32)).cuda()
            secs, tA, tAT = time_pairs(op_, xp, 5, 2)
            bp = (contraction_bytes(inf_, op_.nk, gp.nz, gp.nt, False) +
                  contraction_bytes(inf_, op_.nk, gp.nz, gp.nt, True))
            res[f"{name}_pairs_per_s"] = 5 / secs
            res[f"{name}_contract_GBs"] = bp / ((tA + tAT) * 1e-3) / 1e9
            res[f"{name}_library_GiB"] = (inf_["slab_bytes_A"] + inf_["slab_bytes_AT"]) / 2**30
            res[f"{name}_library_build_s"] = build_s
            log(f"{name} ({gp.boundary}, {op_.nk} transverse frequencies): {res[f'{name}_pairs_per_s']:.1f} pairs/s, "
                f"contraction {res[f'{name}_contract_GBs']:.0f} GB/s, library {res[f'{name}_library_GiB']:.1f} GiB, "
                f"build {build_s:.2f} s")
            del op_, xp
            torch.cuda.empty_cache()
    if "autograd" in sel:
        # differentiable form: 200 Adam steps on 1/2 ||A x - y||^2 + 1e-3 TV(x), 128^2 x 64 x 256
        ga = Geometry.paper_like(128, 128, 64, 256)
        oa = Operator(ga, "f32")
        xa = torch.from_numpy(inputs.vascular_phantom(oa.x_shape, seed=3001).astype(np.float32)).cuda()
        ya = oa.apply_A(xa)
        autograd.fit_adam_tv(oa, ya, steps=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, losses = autograd.fit_adam_tv(oa, ya, steps=200)
        torch.cuda.synchronize()
        res["autograd_adam200_128x128x64x256_s"] = time.perf_counter() - t0
        res["autograd_loss_first_last"] = [losses[0], losses[-1]]
        log(f"autograd 200 Adam steps: {res['autograd_adam200_128x128x64x256_s']:.2f} s, "
            f"loss {losses[0]:.4g} -> {losses[-1]:.4g}")
        del oa, xa, ya
        torch.cuda.empty_cache()
    return res


def serving(args) -> dict:
    """Poisson streams of 50-iteration FISTA reconstructions over three
    geometries x {FP32, BF16} libraries (seeded vascular phantoms, 20 dB
    noise): 20 warm-up requests, then the measured ones.  The same stream is
    served by (i) the plain FIFO: one request at a time, no batching, explicit
    A then A^T each iteration; (ii) the same FIFO with the per-frequency
    normal operator (the gradient form alone, no batching); (iii) continuous
    batching with the normal operator; (iv) the same with a 24 GiB HBM
    budget so that admission binds.  A saturating stream (400 req/s) compares batching
    with a FIFO of the same step.  Libraries are pre-built (cache warm; the
    cold build time is reported apart); latency = completion - arrival."""
    import torch
    from paper_2603_28150_amd import inputs
    from paper_2603_28150_amd.op import Geometry
    from paper_2603_28150_amd.serve import HipBackend, Request, Server
    geoms = [Geometry.paper_like(64, 64, 64, 256), Geometry.paper_like(128, 128, 96, 384),
             Geometry.paper_like(256, 256, 128, 512)]
    classes = [(g, k) for g in geoms for k in ("f32", "bf16")]
    rng = np.random.default_rng(4001)
    n_warm = 20
    n = n_warm + args.serve_requests
    which = rng.integers(0, len(classes), n)
    be_n, be_x = HipBackend(normal=True), HipBackend(normal=False)
    warm = Server(be_n, hbm_budget=200 << 30, max_batch=16)
    t0 = time.perf_counter()
    for g, k in classes:
        warm.submit(Request(geom=g, d=torch.zeros((g.nt, g.ny, g.nx), device="cuda"), niter=1, h_dtype=k))
    warm.run_until_idle()
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    clean = {}
    for ci, (g, k) in enumerate(classes):
        op = warm.classes[(g, k)].op
        clean[ci] = []
        for j in range(4):
            p0 = torch.from_numpy(inputs.vascular_phantom((g.nz, g.ny, g.nx), seed=5000 + 10 * ci + j)
                                  .astype(np.float32)).cuda()
            clean[ci].append(op.apply_A(p0))
    reqs_data = []
    for r in range(n):
        ci = int(which[r])
        g, k = classes[ci]
        c = clean[ci][r % 4]
        sig = float(torch.sqrt(torch.mean(c * c)))
        noise = torch.from_numpy(inputs.noise_like((g.nt, g.ny, g.nx), seed=5000 + r).astype(np.float32)).cuda()
        reqs_data.append((g, k, c + inputs.NOISE_20DB * sig * noise))
    torch.cuda.synchronize()

    def fresh(backend, max_batch, budget=200 << 30):
        srv = Server(backend, hbm_budget=budget, max_batch=max_batch)
        for key, cls in warm.classes.items():   # warm library cache, empty slots
            cls.cap, cls.pool, cls.ws, cls.active, cls.inflight, cls.bytes_pool = 0, {}, None, [], [], 0
            cls.keep, cls.bytes_keep = [], 0
            srv.classes[key] = cls
        srv.used = sum(c.bytes_lib + c.bytes_ws1 for c in warm.classes.values())
        return srv

    def run(srv, rate, fifo):
        gaps = np.random.default_rng(4002).exponential(1.0 / rate, n)
        reqs = [Request(geom=g, d=d, niter=50, h_dtype=k) for g, k, d in reqs_data]
        t = time.perf_counter()
        for r, gap in zip(reqs, gaps):
            t += gap
            r.t_arrival = t
        i = 0
        while i < n or srv.poll():
            now = time.perf_counter()
            while i < n and reqs[i].t_arrival <= now and (not fifo or not srv.poll()):
                srv.submit(reqs[i])
                i += 1
            if fifo:
                srv.run_until_idle()
            elif i < n and not srv.poll():
                time.sleep(max(0.0, min(1e-3, reqs[i].t_arrival - time.perf_counter())))
        torch.cuda.synchronize()
        st = srv.stats()
        meas = [r for r in reqs[n_warm:] if r.latency is not None]
        lat = sorted(r.latency for r in meas)
        span = max(r.t_done for r in meas) - min(r.t_arrival for r in reqs[n_warm:]) if meas else 0.0
        out = {"p50_s": float(np.percentile(lat, 50)) if lat else None,
               "p99_s": float(np.percentile(lat, 99)) if lat else None,
               "recon_per_s": len(meas) / span if span > 0 else None,
               "completed": len(meas),
               "rejected": sum(r.status == "rejected" for r in reqs[n_warm:]),
               "hbm_peak_GiB": st["hbm_peak_bytes"] / 2**30}
        if not fifo:
            out["batch_hist"] = {str(b): c for b, c in sorted(st["batch_hist"].items())}
        for r in reqs:
            r.x = None
        return out

    out = {"library_cache_cold_build_s": t_cold, "requests_measured": n - n_warm,
           "requests_warmup": n_warm, "iterations": 50,
           "classes": [f"{g.nx}x{g.ny}x{g.nz}x{g.nt}/{k}" for g, k in classes],
           "library_cache_GiB": sum(c.bytes_lib for c in warm.classes.values()) / 2**30}
    out["rate_20"] = {"fifo_plain": run(fresh(be_x, 1), 20.0, True),
                      "fifo_normal": run(fresh(be_n, 1), 20.0, True),
                      "batching": run(fresh(be_n, 16), 20.0, False),
                      "batching_budget_24GiB": run(fresh(be_n, 16, 24 << 30), 20.0, False)}
    log(f"serving at 20 req/s: {out['rate_20']}")
    out["rate_400"] = {"fifo_normal": run(fresh(be_n, 1), 400.0, True),
                       "batching": run(fresh(be_n, 16), 400.0, False),
                       "batching_budget_24GiB": run(fresh(be_n, 16, 24 << 30), 400.0, False)}
    log(f"serving at 400 req/s: {out['rate_400']}")
    return out


if __name__ == "__main__":
    main()
