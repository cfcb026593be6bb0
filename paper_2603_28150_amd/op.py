"""Operator handle over libpat.so with torch-owned device buffers.

torch supplies device memory and streams only; every step of A, A^T, the
power iteration and FISTA runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib


@dataclass(frozen=True)
class Geometry:
    """Discrete planar geometry (mirrors pat_geometry; SI units)."""
    nx: int
    ny: int
    nz: int
    nt: int
    dx: float
    dy: float
    dz: float
    dt: float
    c: float
    nz_sim: int = 0
    boundary: str = "periodic"     # "periodic" or "linear" (zero-padded, Sec. 2.3)
    ir: tuple = ()                 # sensor response taps (causal FIR along t), () = ideal
    sx: int = 1                    # scan grid: data at every sx-th column ...
    sy: int = 1                    # ... and sy-th row of the sensor grid
    build: str = "closed"          # library build: "closed" form or one k-space "step"ping run

    @staticmethod
    def paper_like(nx, ny, nz, nt, dx=100e-6, c=1500.0, cfl=0.3, nz_sim=0,
                   boundary="periodic", ir=(), sx=1, sy=1, build="closed") -> "Geometry":
        """dx = dy = dz, dt = cfl * dx / c (the physics of the synthetic workloads)."""
        return Geometry(nx, ny, nz, nt, dx, dx, dx, cfl * dx / c, c, nz_sim, boundary,
                        tuple(float(v) for v in ir), sx, sy, build)

    def to_c(self, h_dtype: str) -> _lib.Geometry:
        g = _lib.Geometry(self.nx, self.ny, self.nz, self.nt, self.dx, self.dy, self.dz,
                          self.dt, self.c, self.nz_sim, _lib.HDTYPES[h_dtype],
                          _lib.BOUNDARIES[self.boundary], len(self.ir), None, self.sx, self.sy,
                          _lib.BUILDS[self.build])
        if self.ir:
            g.ir = (C.c_double * len(self.ir))(*self.ir)   # kept alive by the struct
        return g


# transform sizes of the library's FFTs (include/pat.h, pat_geometry.nx)
FFT_SIZES = (16, 32, 48, 64, 72, 96, 108, 128, 144, 192, 216, 256, 288, 384, 432, 512, 576, 768, 864, 1024)


def transform_size(n: int, boundary: str) -> int:
    """Transform grid size along one axis: n (periodic), or the smallest of
    FFT_SIZES >= max(16, 2 n) (linear)."""
    if boundary != "linear":
        return n
    return min(p for p in FFT_SIZES if p >= max(16, 2 * n))


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class Context:
    """pat_ctx for one GPU; one per device per process is enough."""
    _by_device: dict[int, "Context"] = {}

    def __init__(self, device: int = 0):
        lib = _lib.load()
        h = C.c_void_p()
        _lib.check(lib.pat_ctx_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    @classmethod
    def get(cls, device: int = 0) -> "Context":
        if device not in cls._by_device:
            cls._by_device[device] = Context(device)
        return cls._by_device[device]


def h_bytes(geom: Geometry, h_dtype: str = "f32") -> int:
    g = geom.to_c(h_dtype)
    hb, sb = C.c_size_t(), C.c_size_t()
    _lib.call("pat_H_bytes", C.byref(g), C.byref(hb), C.byref(sb))
    return hb.value


class Operator:
    """A, A^T and FISTA for one geometry; owns its kernel library on the GPU."""

    def __init__(self, geom: Geometry, h_dtype: str = "f32", device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP operator needs a GPU")
        self.geom = geom
        self.h_dtype = h_dtype
        self.device = torch.device("cuda", device)
        self.ctx = Context.get(device)
        g = geom.to_c(h_dtype)
        hb, sb = C.c_size_t(), C.c_size_t()
        _lib.call("pat_H_bytes", C.byref(g), C.byref(hb), C.byref(sb))
        self.h_buf = torch.empty(hb.value, dtype=torch.uint8, device=self.device)
        # build scratch (the stepped build's record), released once the build
        # is enqueued: the caching allocator hands it out again only to work
        # ordered after the build on this stream
        scratch = torch.empty(max(sb.value, 16), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _lib.call("pat_H_build", self.ctx.handle, C.byref(g), _ptr(self.h_buf), hb.value,
                  _ptr(scratch), sb.value, _stream(self.device), C.byref(h))
        del scratch
        self.handle = h
        self._ws: dict[tuple[int, int], torch.Tensor] = {}
        # Gram blocks (periodic boundary, unsampled data): the normal-operator
        # gradient of recon_fista and fista_step_normal
        self.has_gram = self.info()["gram_bytes"] > 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _lib.load().pat_op_destroy(h)
            except Exception:
                pass
            self.handle = None

    # ------------------------------------------------------------ buffers
    @property
    def x_shape(self):
        return (self.geom.nz, self.geom.ny, self.geom.nx)

    @property
    def d_shape(self):
        return (self.geom.nt, self.geom.ny // self.geom.sy, self.geom.nx // self.geom.sx)

    @property
    def nk(self) -> int:
        """Half-spectrum frequencies of the transform grid (the padded grid
        of the linear boundary)."""
        fx, fy = transform_size(self.geom.nx, self.geom.boundary), transform_size(self.geom.ny, self.geom.boundary)
        return fy * (fx // 2 + 1)

    def info(self) -> dict:
        """Stored-library shape: nk, nclass, members_max, nz_sim, slab bytes per layout."""
        i = _lib.OpInfo()
        _lib.call("pat_get_info", self.handle, C.byref(i))
        return {f: getattr(i, f) for f, _ in _lib.OpInfo._fields_}

    # ---------------------------------------------------- stage-level calls
    def spectrum(self, f: torch.Tensor, S: int, out: torch.Tensor, B_ws: int = 1) -> torch.Tensor:
        """Step (i): half spectrum (rows of spectrum_stride(S) complex64 values
        as float pairs, see spectrum_rows) of S real slices."""
        ws = self.workspace(B_ws)
        _lib.call("pat_spectrum", self.handle, _ptr(f), _ptr(out), S, _ptr(ws), ws.numel(),
                  _stream(self.device))
        return out

    def inverse_spectrum(self, spec: torch.Tensor, S: int, out: torch.Tensor, sub=None,
                         B_ws: int = 1) -> torch.Tensor:
        """Step (iii): S real slices from a half spectrum, divided by nx*ny, minus sub."""
        ws = self.workspace(B_ws)
        _lib.call("pat_inverse_spectrum", self.handle, _ptr(spec), _ptr(out), S,
                  _ptr(sub) if sub is not None else None, _ptr(ws), ws.numel(),
                  _stream(self.device))
        return out

    def contract(self, spec_in: torch.Tensor, spec_out: torch.Tensor, adjoint: bool, B: int = 1):
        """Step (ii): per-frequency contraction with H^ (adjoint: sum over time)."""
        _lib.call("pat_contract", self.handle, int(bool(adjoint)), _ptr(spec_in), _ptr(spec_out),
                  B, _stream(self.device))
        return spec_out

    def spectrum_rows(self):
        """Frequency index k of every spectrum row (-1: unused row)."""
        n = self.info()["spec_rows"]
        arr = (C.c_int32 * n)()
        _lib.call("pat_spectrum_rows", self.handle, arr)
        return list(arr)

    @staticmethod
    def spectrum_stride(S: int) -> int:
        """Row stride (complex elements) of a spectrum array of S slices."""
        n = C.c_int32()
        _lib.call("pat_spectrum_stride", S, C.byref(n))
        return n.value

    def spectrum_buffer(self, S: int) -> torch.Tensor:
        """Spectrum array [spec_rows][stride][2] for S slices; entries s >= S
        of a row are padding."""
        rs = self.spectrum_stride(S)
        return torch.empty((self.info()["spec_rows"], rs, 2), dtype=torch.float32, device=self.device)

    def workspace_bytes(self, B: int = 1) -> int:
        n = C.c_size_t()
        _lib.call("pat_workspace_bytes", self.handle, B, C.byref(n))
        return n.value

    def workspace(self, B: int = 1) -> torch.Tensor:
        key = (B, _stream(self.device))
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(self.workspace_bytes(B), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def _check(self, t: torch.Tensor, shape, name: str) -> torch.Tensor:
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if tuple(t.shape[-3:]) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., {shape})")
        return t

    # ---------------------------------------------------------- operators
    def apply_A(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """y = A x for x of shape [nz, ny, nx] or [B, nz, ny, nx]."""
        self._check(x, self.x_shape, "x")
        B = 1 if x.dim() == 3 else x.shape[0]
        if out is None:
            out = torch.empty(x.shape[:-3] + self.d_shape, dtype=torch.float32, device=self.device)
        self._check(out, self.d_shape, "out")
        ws = self.workspace(B)
        _lib.call("pat_apply_A", self.handle, _ptr(x), _ptr(out), B, _ptr(ws), ws.numel(),
                  _stream(self.device))
        return out

    def apply_AT(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """x = A^T y for y of shape [nt, ny, nx] or [B, nt, ny, nx]."""
        self._check(y, self.d_shape, "y")
        B = 1 if y.dim() == 3 else y.shape[0]
        if out is None:
            out = torch.empty(y.shape[:-3] + self.x_shape, dtype=torch.float32, device=self.device)
        self._check(out, self.x_shape, "out")
        ws = self.workspace(B)
        _lib.call("pat_apply_AT", self.handle, _ptr(y), _ptr(out), B, _ptr(ws), ws.numel(),
                  _stream(self.device))
        return out

    def power_norm(self, v0: torch.Tensor, niter: int = 30):
        """(L_niter, [L_1..L_niter]) of the power iteration on A^T A (synchronises)."""
        self._check(v0, self.x_shape, "v0")
        ws = self.workspace(1)
        L = C.c_double()
        tr = (C.c_double * niter)()
        _lib.call("pat_power_norm", self.handle, _ptr(v0), niter, C.byref(L), tr, _ptr(ws),
                  ws.numel(), _stream(self.device))
        return L.value, list(tr)

    def recon_fista(self, d: torch.Tensor, niter: int, tau: float, lam: float = 0.0,
                    nonneg: bool = True, momentum: bool = True, trace: bool = False,
                    out: torch.Tensor | None = None):
        """x_niter of FISTA (x_0 = 0); with trace=True also 1/2||A z_k - d||^2 per step."""
        self._check(d, self.d_shape, "d")
        if out is None:
            out = torch.empty(self.x_shape, dtype=torch.float32, device=self.device)
        self._check(out, self.x_shape, "out")
        tr = torch.empty(max(niter, 1), dtype=torch.float32, device=self.device) if trace else None
        ws = self.workspace(1)
        _lib.call("pat_recon_fista", self.handle, _ptr(d), _ptr(out), niter, float(tau),
                  float(lam), int(bool(nonneg)), int(bool(momentum)),
                  _ptr(tr) if tr is not None else None, _ptr(ws), ws.numel(), _stream(self.device))
        return (out, tr[:niter]) if trace else out

    def fista_step(self, d, x, z, beta, tau, lam, nonneg, nonfinite=None, ws=None) -> None:
        """One batched FISTA iteration in place on x and z ([B, nz, ny, nx]).
        ws: optional workspace tensor (at least workspace_bytes(B))."""
        B = x.shape[0]
        self._check(d, self.d_shape, "d")
        self._check(x, self.x_shape, "x")
        self._check(z, self.x_shape, "z")
        cb = (C.c_double * B)(*[float(b) for b in beta])
        ct = (C.c_float * B)(*[float(t) for t in tau])
        cl = (C.c_float * B)(*[float(v) for v in lam])
        cn = (C.c_int32 * B)(*[int(bool(v)) for v in nonneg])
        if ws is None:
            ws = self.workspace(B)
        _lib.call("pat_fista_step", self.handle, B, _ptr(d), _ptr(x), _ptr(z), cb, ct, cl, cn,
                  _ptr(nonfinite) if nonfinite is not None else None, _ptr(ws), ws.numel(),
                  _stream(self.device))

    def fista_step_normal(self, atd, x, z, beta, tau, lam, nonneg, nonfinite=None, ws=None) -> None:
        """One batched FISTA iteration with the per-frequency normal operator;
        atd = A^T d of every object ([B, nz, ny, nx])."""
        B = x.shape[0]
        self._check(atd, self.x_shape, "atd")
        self._check(x, self.x_shape, "x")
        self._check(z, self.x_shape, "z")
        cb = (C.c_double * B)(*[float(b) for b in beta])
        ct = (C.c_float * B)(*[float(t) for t in tau])
        cl = (C.c_float * B)(*[float(v) for v in lam])
        cn = (C.c_int32 * B)(*[int(bool(v)) for v in nonneg])
        if ws is None:
            ws = self.workspace(B)
        _lib.call("pat_fista_step_normal", self.handle, B, _ptr(atd), _ptr(x), _ptr(z), cb, ct, cl, cn,
                  _ptr(nonfinite) if nonfinite is not None else None, _ptr(ws), ws.numel(),
                  _stream(self.device))

    def adjoint_check(self, x: torch.Tensor, y: torch.Tensor) -> float:
        self._check(x, self.x_shape, "x")
        self._check(y, self.d_shape, "y")
        ws = self.workspace(1)
        r = C.c_double()
        _lib.call("pat_adjoint_check", self.handle, _ptr(x), _ptr(y), C.byref(r), _ptr(ws),
                  ws.numel(), _stream(self.device))
        return r.value

    def export_H(self, k0: int = 0, nk: int | None = None) -> torch.Tensor:
        """Dequantised H^ for half-spectrum frequencies k0..k0+nk-1: [nk, nz, nt]."""
        if nk is None:
            nk = self.nk - k0
        out = torch.empty((nk, self.geom.nz, self.geom.nt), dtype=torch.float32, device=self.device)
        _lib.call("pat_H_export", self.handle, k0, nk, _ptr(out), _stream(self.device))
        return out
