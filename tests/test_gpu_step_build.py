"""The library built by one k-space time-stepping run (pat_geometry.build =
PAT_BUILD_STEP): a unit point source stepped with the exact propagator in
float64, the field recorded on every depth plane (by reciprocity the
library, Sec. 3.2), against the closed-form build and the FP64 oracle.

Bars: library 1e-7 of its largest value (float32 storage), the same bar
against the closed-form library; 16-bit libraries equal up to rare
last-place differences; A and A^T through either library 1e-5 relative l2.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import hlib, operators as ops
from oracle.geometry import Geometry as OGeom
from paper_2603_28150_amd import _lib, inputs
from paper_2603_28150_amd.op import Context, Geometry, Operator

pytestmark = pytest.mark.gpu

GEOMS = {
    "tiny": Geometry.paper_like(32, 32, 16, 64),                           # radial classes
    "ragged": Geometry(32, 16, 13, 37, 1e-4, 1.3e-4, 1e-4, 2e-8, 1500.0),   # quadrant classes, ragged
    "mid": Geometry.paper_like(64, 64, 40, 130),                           # several time blocks
}


def og(g):
    return OGeom(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim)


def stepped(g):
    return Geometry(g.nx, g.ny, g.nz, g.nt, g.dx, g.dy, g.dz, g.dt, g.c, g.nz_sim, g.boundary, g.ir,
                    g.sx, g.sy, "step")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", list(GEOMS))
def test_stepped_library_equals_closed_form_and_oracle(name):
    g = GEOMS[name]
    opc, ops_ = Operator(g), Operator(stepped(g))
    Hs, Hc = host(ops_.export_H()), host(opc.export_H())
    Ho = hlib.H_half(og(g)).reshape(Hs.shape)
    top = np.abs(Ho).max()
    assert np.abs(Hs - Ho).max() <= 1e-7 * top
    assert np.abs(Hs - Hc).max() <= 1e-7 * top
    x = inputs.gaussian_blobs(opc.x_shape, seed=41)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    assert rel(host(ops_.apply_A(xd)), ops.A_fft(hlib.H_half(og(g)), x)) < 1e-5
    d = inputs.gaussian_random(opc.d_shape, seed=42)
    dd = torch.from_numpy(d.astype(np.float32)).cuda()
    assert rel(host(ops_.apply_AT(dd)), host(opc.apply_AT(dd))) < 1e-5


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_stepped_16bit_library_equals_closed_form(kind):
    g = GEOMS["tiny"]
    Hs, Hc = host(Operator(stepped(g), kind).export_H()), host(Operator(g, kind).export_H())
    ulp = 2.0 ** -8 if kind == "bf16" else 2.0 ** -11
    top = np.abs(Hc).max()
    big = np.abs(Hc) > 1e-12 * top
    diff = np.abs(Hs - Hc)
    assert np.all(diff[~big] <= 1e-12 * top)
    assert np.mean(diff[big] > 0) < 1e-3
    assert np.all(diff[big] <= ulp * np.abs(Hc[big]) * 1.01)


def test_stepped_library_with_sensor_response():
    taps = (0.25, 0.5, 0.25, -0.1, 0.05)
    g = Geometry.paper_like(32, 32, 16, 64, ir=taps)
    Hs = host(Operator(stepped(g)).export_H())
    Ho = hlib.with_sensor_response(hlib.H_half(og(g)), taps).reshape(Hs.shape)
    assert np.abs(Hs - Ho).max() <= 1e-7 * np.abs(Ho).max()


def test_stepped_build_in_blocks_of_classes():
    # scratch for three classes' records: the stepper runs the classes in
    # ragged blocks of three and lands on the same library; scratch below one
    # record is refused before any launch
    g = GEOMS["mid"]
    L = _lib.load()
    ctx = Context.get(0)
    cg = stepped(g).to_c("f32")
    hb, sb = C.c_size_t(), C.c_size_t()
    assert L.pat_H_bytes(C.byref(cg), C.byref(hb), C.byref(sb)) == 0
    nq = og(g).nq
    per = g.nt * (nq // 2 + 1) * 8
    assert sb.value % per == 0 and sb.value >= per
    hbuf = torch.empty(hb.value, dtype=torch.uint8, device="cuda")
    scratch = torch.empty(3 * per, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    stream = torch.cuda.current_stream().cuda_stream
    assert L.pat_H_build(ctx.handle, C.byref(cg), hbuf.data_ptr(), hb.value, scratch.data_ptr(), per - 8,
                         stream, C.byref(h)) == -1
    assert b"scratch too small" in L.pat_last_error()
    assert L.pat_H_build(ctx.handle, C.byref(cg), hbuf.data_ptr(), hb.value, scratch.data_ptr(), 3 * per,
                         stream, C.byref(h)) == 0
    info = _lib.OpInfo()
    assert L.pat_get_info(h, C.byref(info)) == 0
    assert info.nclass % 3 != 0                       # the last block is ragged
    nk = info.nk
    out = torch.empty((nk, g.nz, g.nt), device="cuda")
    assert L.pat_H_export(h, 0, nk, out.data_ptr(), stream) == 0
    Hc = host(Operator(g).export_H())
    assert np.abs(host(out) - Hc).max() <= 1e-7 * np.abs(Hc).max()
    assert L.pat_op_destroy(h) == 0


@pytest.mark.parametrize("g", [Geometry.paper_like(24, 16, 6, 30, boundary="linear"),      # 48 x 32 periods
                               Geometry.paper_like(34, 34, 8, 40)],                       # chirp-z axes
                         ids=["linear", "chirpz"])
def test_stepped_build_on_other_transform_grids(g):
    # the stepped build is a property of the library alone: the same on the
    # padded grid of the linear boundary and on chirp-z axes
    Hs, Hc = host(Operator(stepped(g)).export_H()), host(Operator(g).export_H())
    assert np.abs(Hs - Hc).max() <= 1e-7 * np.abs(Hc).max()
