// C ABI of libpat.so: argument checking, kernel-library layout, workspace
// layout and the order of launches for each call of include/pat.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pat_internal.hpp"

struct pat_ctx {
  int device;
  void* scratch;  // this device's address of the static scratch (pat_apply_A_noalloc)
};

struct pat_op {
  pat_ctx* ctx;
  pat_geometry g;
  int nq;
  int fx, fy;   // transform grid (2 nx x 2 ny for the linear boundary)
  int sx, sy;   // scan-grid sampling of the data (1: every grid point)
  int nh, nk;   // half-spectrum columns fx/2+1 and frequencies fy*nh
  int G;        // member slots per work item (8: radial float32, 4: radial 16-bit, 2: quadrant fold)
  int nclass;   // stored slabs
  int nitem;    // contraction work items (each reads one slab)
  int vec;      // storage elements per 16-byte load
  int sA_row, sT_row;
  int ntA, ksA, ntT, ksT;  // 16-bit fragment tiling
  char* hbuf;
  int nrows;          // spectrum rows: nitem * G, item-major
  int32_t* members;   // [nitem][G]
  int32_t* item_slab; // [nitem]
  int32_t* kclass;    // [nk] slab of frequency k
  int32_t* rowmap;    // [nk] spectrum row of frequency k
  int32_t* cls_freq;  // [nclass][2]
  float* inv_scale;   // [nz]
  unsigned long long* amax;  // [nz]
  void* slabA;        // FP32: [nclass][nz][sA_row]; 16-bit: MFMA fragments (n, k = l)
  void* slabT;        // FP32: [nclass][nt][sT_row]; 16-bit: MFMA fragments (l, k = n)
  void* rowA;         // [nclass][nz][sA_row] rows of the storage type (= slabA for FP32)
  void* rowT;         // [nclass][nt][sT_row] rows of the storage type (= slabT for FP32)
  float* gram;        // [nclass][nz][sG_row]  Gram blocks of the library
  int32_t* kexpA;     // FP32: [nclass][nt] exponent of each [n][l] row (A's k rows), else null
  int32_t* kexpT;     // FP32: [nclass][nz] exponent of each [l][n] row (A^T's k rows), else null
  int sG_row;
  pat::FftChirp chirp;  // chirp-z tables of axes that are not fast FFT sizes
  std::vector<float2> h_cz;  // their host copy: c and the kernel DFT, x then y
  std::vector<int32_t> h_members, h_kclass, h_cls_freq, h_rowmap, h_item_slab;
  std::vector<double> h_ir;  // sensor response taps folded into the library
};

namespace pat {

// Scratch of pat_apply_A_noalloc: a file-scope device array, so that the
// entry point needs no allocation.  Each GPU the library runs on holds its
// own copy (at its own address) until the process ends.  Host code must not
// use the symbol itself as a device address: pat_ctx_create looks the
// address up once per device (hipGetSymbolAddress, that device current) and
// every use goes through the pointer kept in the context.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char g_scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// address of g_scratch on `device` (which must be current)
static pat_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    PAT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(g_scratch)));
    if (!p) return fail(PAT_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return PAT_OK;
}

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

pat_status fail(pat_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

pat_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PAT_OK;
  return fail(PAT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------- geometry rules

// transform sizes the FFT kernels provide: 2^a 3^b, b <= 3, multiples of 4
// in [16, 1024], at least 48 when b > 0
static bool fft_size(int v) {
  static const int sizes[] = {16,  32,  48,  64,  72,  96,  108, 128, 144, 192,
                              216, 256, 288, 384, 432, 512, 576, 768, 864, 1024};
  for (int s : sizes)
    if (v == s) return true;
  return false;
}

// other even lengths in [16, 512] (the paper's 202 and 326 among them) run as
// chirp-z transforms: a circular convolution of length chirp_m(n), the
// smallest power of two >= 2n - 1
static bool chirp_size(int v) { return !fft_size(v) && v >= 16 && v <= 512 && v % 2 == 0; }
static int chirp_m(int n) {
  int m = 64;
  while (m < 2 * n - 1) m <<= 1;
  return m;
}

// c[k] = exp(i pi k^2 / n), k < n, then the m-point DFT of the even kernel
// b[j] = c[|j|] (|j| < n, j taken mod m) divided by m; float64, rounded once
static void chirp_tables(int n, int m, std::vector<float2>& out) {
  const double pi = 3.141592653589793238462643383279502884;
  std::vector<double> cr(n), ci(n);
  for (int k = 0; k < n; ++k) {
    const long long r = ((long long)k * k) % (2LL * n);  // exact phase reduction
    cr[k] = std::cos(pi * (double)r / n);
    ci[k] = std::sin(pi * (double)r / n);
    out.push_back(make_float2((float)cr[k], (float)ci[k]));
  }
  std::vector<double> br(m, 0.0), bi(m, 0.0);
  for (int j = 0; j < n; ++j) {
    br[j] = cr[j];
    bi[j] = ci[j];
    if (j > 0) {
      br[m - j] = cr[j];
      bi[m - j] = ci[j];
    }
  }
  for (int k = 0; k < m; ++k) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < m; ++j) {
      if (br[j] == 0.0 && bi[j] == 0.0) continue;
      const long long e = ((long long)k * j) % m;
      const double a = -2.0 * pi * (double)e / m;
      const double ca = std::cos(a), sa = std::sin(a);
      sr += br[j] * ca - bi[j] * sa;
      si += br[j] * sa + bi[j] * ca;
    }
    out.push_back(make_float2((float)(sr / m), (float)(si / m)));
  }
}

static int default_nq(const pat_geometry& g) {
  const double reach = std::ceil(g.c * g.dt * (double)(g.nt - 1) / g.dz);
  const long long need = (long long)g.nz + (long long)reach + 1;
  int nq = 1;
  while (nq < need) nq <<= 1;
  return nq;
}

// build scratch of the stepped library build: the record of as many classes
// as fit in 256 MiB (at least one); none for the closed form
static size_t step_scratch_bytes(const pat_geometry& g, int nclass) {
  if (g.build != PAT_BUILD_STEP) return 0;
  const size_t per = step_class_bytes(g.nt, g.nz_sim ? g.nz_sim : default_nq(g));
  const size_t block = std::max<size_t>(1, std::min<size_t>((size_t)nclass, (size_t(256) << 20) / per));
  return block * per;
}

// scan-grid sampling steps (0 in a zero-initialised geometry means 1)
static int scan_sx(const pat_geometry& g) { return g.sx > 1 ? g.sx : 1; }
static int scan_sy(const pat_geometry& g) { return g.sy > 1 ? g.sy : 1; }
static bool sampled(const pat_geometry& g) { return scan_sx(g) > 1 || scan_sy(g) > 1; }

// linear boundary: the transform grid is the smallest transform size holding
// twice the window (so that no offset inside the window wraps), at least 16
static int linear_size(int n) {
  int p = n > 8 ? 2 * n : 16;
  while (!fft_size(p)) ++p;
  return p;
}

// the periodic grid the transforms and the library live on
static pat_geometry transform_geometry(const pat_geometry& g) {
  pat_geometry t = g;
  if (g.boundary == PAT_BOUNDARY_LINEAR) {
    t.nx = linear_size(g.nx);
    t.ny = linear_size(g.ny);
  }
  return t;
}

static pat_status check_geometry(const pat_geometry* g) {
  if (!g) return fail(PAT_EINVAL, "geometry is null");
  if (g->nz < 1 || g->nt < 1) return fail(PAT_EINVAL, "nz and nt must be >= 1");
  if (!(g->dx > 0 && g->dy > 0 && g->dz > 0 && g->dt > 0 && g->c > 0))
    return fail(PAT_EINVAL, "dx, dy, dz, dt and c must be > 0");
  if (g->nz_sim != 0 && g->nz_sim < g->nz) return fail(PAT_EINVAL, "nz_sim must be 0 or >= nz");
  if (g->h_dtype < PAT_H_F32 || g->h_dtype > PAT_H_F16) return fail(PAT_EINVAL, "unknown h_dtype");
  if (g->boundary != PAT_BOUNDARY_PERIODIC && g->boundary != PAT_BOUNDARY_LINEAR)
    return fail(PAT_EINVAL, "unknown boundary");
  if (g->boundary == PAT_BOUNDARY_PERIODIC &&
      (!(fft_size(g->nx) || chirp_size(g->nx)) || !(fft_size(g->ny) || chirp_size(g->ny))))
    return fail(PAT_EUNSUPPORTED, "periodic: nx and ny must be transform sizes (16, 32, 48, 64, 72, 96, 108, 128, "
                                  "144, 192, 216, 256, 288, 384, 432, 512, 576, 768, 864, 1024) or even "
                                  "lengths in [16, 512] (chirp-z)");
  if (g->boundary == PAT_BOUNDARY_PERIODIC && (chirp_size(g->nx) || chirp_size(g->ny)) &&
      (g->sx > 1 || g->sy > 1))
    return fail(PAT_EUNSUPPORTED, "scan-grid sampling needs fast transform sizes (no chirp-z axis)");
  if (g->boundary == PAT_BOUNDARY_LINEAR && (g->nx < 4 || g->nx > 512 || g->ny < 1 || g->ny > 512))
    return fail(PAT_EUNSUPPORTED, "linear: nx must be in [4, 512] and ny in [1, 512]");
  if (g->nz > 2048 || g->nt > 2048) return fail(PAT_EUNSUPPORTED, "nz and nt must be <= 2048");
  if (g->n_ir < 0 || g->n_ir > kMaxIr) return fail(PAT_EUNSUPPORTED, "n_ir must be in [0, 64]");
  if (g->sx < 0 || g->sy < 0) return fail(PAT_EINVAL, "sx and sy must be >= 0");
  if (g->build != PAT_BUILD_CLOSED && g->build != PAT_BUILD_STEP) return fail(PAT_EINVAL, "unknown build");
  if (g->nx % scan_sx(*g) || g->ny % scan_sy(*g))
    return fail(PAT_EUNSUPPORTED, "sx must divide nx and sy must divide ny");
  if (g->n_ir > 0) {
    if (!g->ir) return fail(PAT_EINVAL, "ir is null while n_ir > 0");
    for (int j = 0; j < g->n_ir; ++j)
      if (!std::isfinite(g->ir[j])) return fail(PAT_EINVAL, "sensor response taps must be finite");
  }
  return PAT_OK;
}

// -------------------------------------------------------- frequency classes
// H^ depends on (m, p) only through kx^2 + ky^2, so one stored slab serves a
// whole symmetry class of half-spectrum frequencies:
//   quadrant fold (any grid):          (|m~|, |p~|), <= 2 members
//   radial fold (nx = ny, dx = dy):    all frequencies with equal m~^2 + p~^2
// A work item of the contraction is one slab with up to G member
// frequencies (a class with more members than G is split into several items
// that read the same slab, adjacent in item order, so that the contraction
// runs them on one XCD and the second read hits its L2); its members occupy
// spectrum rows item*G .. item*G+G-1.  G = 8 for float32 libraries; 16-bit
// libraries take G = 4 so that a batch of 16 objects (64 member-object
// pairs) stays in two matrix-core column groups of 32 pairs, and the VALU
// kernel (8 values per 16-byte load) keeps its accumulators in registers.
struct Classes {
  int G = 2;
  std::vector<int32_t> freq;       // [nslab][2] representative |m~|, |p~|
  std::vector<int32_t> item_slab;  // [nitem]
  std::vector<int32_t> members;    // [nitem][G]
  std::vector<int32_t> kclass;     // [nk] slab of frequency k
  std::vector<int32_t> rowmap;     // [nk] spectrum row of frequency k
  int n() const { return (int)freq.size() / 2; }
  int nitem() const { return (int)item_slab.size(); }
};

static Classes make_classes(const pat_geometry& g) {
  Classes C;
  const int nh = g.nx / 2 + 1, hx = g.nx / 2, hy = g.ny / 2;
  const bool square = g.nx == g.ny && g.dx == g.dy;
  const int nk = g.ny * nh;
  // members of the half spectrum with |m~| = m, |p~| = pa
  auto members_of = [&](int m, int pa, std::vector<int32_t>& out) {
    const int p1 = pa, p2 = (g.ny - pa) % g.ny;
    out.push_back(p1 * nh + m);
    if (p2 != p1) out.push_back(p2 * nh + m);
  };
  std::vector<std::vector<int32_t>> groups;  // member list per slab
  if (square) {
    std::vector<int> slot_of_r(2 * hx * hx + 1, -1);
    for (int a = 0; a <= hx; ++a)
      for (int b = a; b <= hx; ++b) {
        int gi = slot_of_r[a * a + b * b];
        if (gi < 0) {
          gi = (int)groups.size();
          groups.emplace_back();
          C.freq.push_back(a);
          C.freq.push_back(b);
          slot_of_r[a * a + b * b] = gi;
        }
        members_of(a, b, groups[gi]);
        if (a != b) members_of(b, a, groups[gi]);
      }
    C.G = g.h_dtype == PAT_H_F32 ? 8 : 4;
  } else {
    for (int m = 0; m <= hx; ++m)
      for (int pa = 0; pa <= hy; ++pa) {
        groups.emplace_back();
        C.freq.push_back(m);
        C.freq.push_back(pa);
        members_of(m, pa, groups.back());
      }
    C.G = 2;
  }
  C.kclass.assign(nk, -1);
  C.rowmap.assign(nk, -1);
  for (int gi = 0; gi < (int)groups.size(); ++gi) {
    const auto& mem = groups[gi];
    for (size_t i0 = 0; i0 < mem.size(); i0 += C.G) {
      const int item = (int)C.item_slab.size();
      C.item_slab.push_back(gi);
      for (int s = 0; s < C.G; ++s) {
        const size_t i = i0 + s;
        const int k = i < mem.size() ? mem[i] : -1;
        C.members.push_back(k);
        if (k >= 0) {
          C.kclass[k] = gi;
          C.rowmap[k] = item * C.G + s;
        }
      }
    }
  }
  return C;
}

struct HLayout {
  size_t off_cz, bytes_cz;
  size_t off_members, off_items, off_kclass, off_rowmap, off_freq, off_inv, off_amax, off_ir, off_A,
      off_T, off_Ar, off_Tr, off_G, off_X, total;
  size_t bytes_A, bytes_T, bytes_Ar, bytes_Tr, bytes_G, bytes_X;
  int sG_row;
  int nclass, nitem, G, vec, sA_row, sT_row;
  int ntA, ksA, ntT, ksT;
};

static HLayout h_layout(const pat_geometry& g, const Classes& C) {
  HLayout L;
  L.nclass = C.n();
  L.nitem = C.nitem();
  L.G = C.G;
  const size_t esz = g.h_dtype == PAT_H_F32 ? 4 : 2;
  L.vec = (int)(16 / esz);
  L.sA_row = (int)align_up((size_t)g.nt, (size_t)L.vec);
  L.sT_row = (int)align_up((size_t)g.nz, (size_t)L.vec);
  // 16-bit libraries are stored as MFMA fragments: 32 output rows x 16 k
  L.ntA = (g.nt + 31) / 32;
  L.ksA = (g.nz + 15) / 16;
  L.ntT = (g.nz + 31) / 32;
  L.ksT = (g.nt + 15) / 16;
  // rows [slab][l][n] and [slab][n][l] of the storage type, for the VALU
  // contraction; 16-bit libraries add both layouts as MFMA fragments for
  // batches (the FP32 rows serve every batch size)
  L.bytes_Ar = (size_t)L.nclass * g.nz * L.sA_row * esz;
  L.bytes_Tr = (size_t)L.nclass * g.nt * L.sT_row * esz;
  if (g.h_dtype == PAT_H_F32) {
    L.bytes_A = 0;
    L.bytes_T = 0;
  } else {
    L.bytes_A = (size_t)L.nclass * L.ntA * L.ksA * 1024;
    L.bytes_T = (size_t)L.nclass * L.ntT * L.ksT * 1024;
  }
  const int nk = g.ny * (g.nx / 2 + 1);
  size_t o = 0;
  L.off_members = o; o = align_up(o + (size_t)L.nitem * L.G * 4, 256);
  L.off_items = o;   o = align_up(o + (size_t)L.nitem * 4, 256);
  L.off_kclass = o;  o = align_up(o + (size_t)nk * 4, 256);
  L.off_rowmap = o;  o = align_up(o + (size_t)nk * 4, 256);
  L.off_freq = o;    o = align_up(o + (size_t)L.nclass * 8, 256);
  L.off_inv = o;     o = align_up(o + (size_t)g.nz * 4, 256);
  L.off_amax = o;    o = align_up(o + (size_t)g.nz * 8, 256);
  L.off_ir = o;      o = align_up(o + (size_t)g.n_ir * 8, 256);
  L.bytes_cz = 0;  // chirp-z tables (periodic axes only: the linear periods are fast sizes)
  if (chirp_size(g.nx)) L.bytes_cz += (size_t)(g.nx + chirp_m(g.nx)) * 8;
  if (chirp_size(g.ny)) L.bytes_cz += (size_t)(g.ny + chirp_m(g.ny)) * 8;
  L.off_cz = o;      o = align_up(o + L.bytes_cz, 256);
  L.sG_row = (int)align_up((size_t)g.nz, 4);
  // Gram blocks serve the normal-operator gradient, which only the periodic,
  // unsampled operator has (see pat_recon_fista)
  L.bytes_G = (g.boundary == PAT_BOUNDARY_PERIODIC && !sampled(g))
                  ? (size_t)L.nclass * g.nz * L.sG_row * 4 : 0;
  L.off_Ar = o;      o = align_up(o + L.bytes_Ar, 256);
  L.off_Tr = o;      o = align_up(o + L.bytes_Tr, 256);
  L.off_A = o;       o = align_up(o + L.bytes_A, 256);
  L.off_T = o;       o = align_up(o + L.bytes_T, 256);
  L.off_G = o;       o = align_up(o + L.bytes_G, 256);
  // float32 libraries: the power-of-two exponent of every k row of both
  // layouts ([n][l] rows for A, [l][n] rows for A^T), for the batched
  // contraction's float16 terms
  L.bytes_X = g.h_dtype == PAT_H_F32 ? (size_t)L.nclass * (g.nt + g.nz) * 4 : 0;
  L.off_X = o;       o = align_up(o + L.bytes_X, 256);
  L.total = o;
  return L;
}

// ------------------------------------------------------------- workspace
struct Work {
  float2 *Xs, *Ds, *T, *Bs, *Gs;
  float *V, *U, *Z, *R;
  double* part64;
  float* part32;
  double* s64;   // 8 doubles
  float* s32;    // 8 floats + trace of the power iteration
  size_t total;
};
constexpr int kMaxPowerIter = 4096;

// Workspace of a batch of B objects.  The spectra of B*nz and B*nt slices
// and the transforms' intermediate come first: they are all one apply of A
// uses (apply_only: the layout stops there, the other buffers are null).
static Work work_layout(const pat_op* op, int B, char* base, bool apply_only = false) {
  const pat_geometry& g = op->g;
  const size_t nxy = (size_t)g.nx * g.ny;
  const size_t Sz = (size_t)B * g.nz, St = (size_t)B * g.nt;
  Work w;
  std::memset(&w, 0, sizeof(w));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + o : nullptr;
    o = align_up(o + bytes, 256);
    return p;
  };
  const size_t rz = spec_stride((int)Sz), rt = spec_stride((int)St);
  w.Xs = (float2*)take((size_t)op->nrows * rz * 8);  // nrows = nitem * G
  w.Ds = (float2*)take((size_t)op->nrows * rt * 8);
  w.T = (float2*)take((size_t)g.ny * op->nh * std::max(rz, rt) * 8);
  if (apply_only) {
    w.total = o;
    return w;
  }
  w.Bs = (float2*)take((size_t)op->nrows * rz * 8);
  w.Gs = (float2*)take((size_t)op->nrows * rz * 8);
  w.V = (float*)take(Sz * nxy * 4);
  w.U = (float*)take(Sz * nxy * 4);
  w.Z = (float*)take(Sz * nxy * 4);
  w.R = (float*)take(St * nxy * 4);
  w.part64 = (double*)take(kRedBlocks * 8);
  w.part32 = (float*)take(kRedBlocks * 4);
  w.s64 = (double*)take(8 * 8);
  w.s32 = (float*)take((8 + kMaxPowerIter) * 4);
  w.total = o;
  return w;
}

static bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

// a batch of B objects: B >= 1 and at most 2^30 slices per spectrum row
static pat_status check_batch(const pat_op* op, int B) {
  if (B < 1) return fail(PAT_EINVAL, "batch B must be >= 1");
  if ((long long)B * std::max(op->g.nz, op->g.nt) > (1LL << 30))
    return fail(PAT_EINVAL, "batch too large: B * max(nz, nt) must be <= 2^30");
  return PAT_OK;
}

static pat_status check_op_call(pat_op* op, int B, void* ws, size_t ws_bytes, Work* w) {
  if (!op) return fail(PAT_EINVAL, "operator is null");
  PAT_TRY(check_batch(op, B));
  if (!ws || misaligned(ws)) return fail(PAT_EINVAL, "workspace is null or not 16-byte aligned");
  *w = work_layout(op, B, (char*)ws);
  if (ws_bytes < w->total)
    return fail(PAT_EINVAL, "workspace too small: need " + std::to_string(w->total) + " bytes");
  PAT_HIP(hipSetDevice(op->ctx->device));
  return PAT_OK;
}

static pat_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(PAT_EINVAL, std::string(name) + " is null");
  if (misaligned(p)) return fail(PAT_EINVAL, std::string(name) + " is not 16-byte aligned");
  return PAT_OK;
}

// 1 / (points of the transform grid): the inverse DFT normalisation
static float inv_area(const pat_op* op) { return 1.0f / (float)((long long)op->fx * op->fy); }

// step (ii): per-frequency contraction of B spectra
static pat_status run_contract(pat_op* op, bool adjoint, const float2* in, float2* out, int B,
                               hipStream_t st) {
  const pat_geometry& g = op->g;
  ContractArgs a;
  a.members = op->members;
  a.item_slab = op->item_slab;
  a.in = in;
  a.out = out;
  a.out_sub = nullptr;
  a.nitem = op->nitem;
  const float* sc = g.h_dtype == PAT_H_F32 ? nullptr : op->inv_scale;
  // one object: the VALU kernel on the row layouts streams the library at
  // the FP32 kernel's rate; batches go to the matrix cores (one slab read
  // serves every object; FP32 values enter as two float16 terms, scaled by
  // a power of two per row)
  const bool f32 = g.h_dtype == PAT_H_F32;
  if (B > 1) {
    MfmaArgs m;
    m.krows = nullptr;
    m.k_srow = 0;
    m.k_slab = 0;
    m.kexp = nullptr;
    m.frag = nullptr;
    m.members = op->members;
    m.item_slab = op->item_slab;
    m.in = in;
    m.out = out;
    m.G = op->G;
    m.B = B;
    m.nitem = op->nitem;
    if (!adjoint) {
      if (f32) {
        m.krows = static_cast<const float*>(op->rowT);  // [n][l]: runs along k = l
        m.k_srow = op->sT_row;
        m.k_slab = (long long)g.nt * op->sT_row;
        m.kexp = op->kexpA;
      } else {
        m.frag = op->slabA;
      }
      m.K = g.nz;
      m.N = g.nt;
      m.ntiles = op->ntA;
      m.ksteps = op->ksA;
      m.in_scale = sc;
      m.out_scale = nullptr;
    } else {
      if (f32) {
        m.krows = static_cast<const float*>(op->rowA);  // [l][n]: runs along k = n
        m.k_srow = op->sA_row;
        m.k_slab = (long long)g.nz * op->sA_row;
        m.kexp = op->kexpT;
      } else {
        m.frag = op->slabT;
      }
      m.K = g.nt;
      m.N = g.nz;
      m.ntiles = op->ntT;
      m.ksteps = op->ksT;
      m.in_scale = nullptr;
      m.out_scale = sc;
    }
    m.in_rs = spec_stride(B * m.K);
    m.out_rs = spec_stride(B * m.N);
    return contract_mfma(m, g.h_dtype, st);
  }
  if (!adjoint) {
    a.slab = op->rowA;
    a.in_scale = sc;
    a.out_scale = nullptr;
    a.ni = g.nz;
    a.nj = g.nt;
    a.s_row = op->sA_row;
  } else {
    a.slab = op->rowT;
    a.in_scale = nullptr;
    a.out_scale = sc;
    a.ni = g.nt;
    a.nj = g.nz;
    a.s_row = op->sT_row;
  }
  a.slab_elems = (long long)a.ni * a.s_row;
  a.in_rs = spec_stride(B * a.ni);
  a.out_rs = spec_stride(B * a.nj);
  return contract(a, g.h_dtype, op->G, B, st);
}

// Gram contraction: out = G z^ - sub per frequency, B spectra of nz slices
static pat_status run_gram(pat_op* op, const float2* in, float2* out, const float2* sub, int B,
                           hipStream_t st) {
  const pat_geometry& g = op->g;
  ContractArgs a;
  a.slab = op->gram;
  a.members = op->members;
  a.item_slab = op->item_slab;
  a.in = in;
  a.out = out;
  a.in_scale = nullptr;
  a.out_scale = nullptr;
  a.out_sub = sub;
  a.ni = g.nz;
  a.nj = g.nz;
  a.s_row = op->sG_row;
  a.slab_elems = (long long)g.nz * op->sG_row;
  a.in_rs = spec_stride(B * g.nz);
  a.out_rs = spec_stride(B * g.nz);
  a.nitem = op->nitem;
  return contract(a, PAT_H_F32, op->G, B, st);
}

// y = A x (- sub), B objects
// (rows_done: the forward transform's first pass on x is already in w.T)
static pat_status run_A(pat_op* op, const float* x, float* y, int B, const float* sub, const Work& w,
                        hipStream_t st, bool rows_done = false) {
  const pat_geometry& g = op->g;
  if (rows_done)
    PAT_TRY(fft2_r2c_cols(w.T, w.Xs, op->fx, op->fy, g.ny, B * g.nz, op->rowmap, op->chirp, st));
  else
    PAT_TRY(fft2_r2c(x, w.T, w.Xs, op->fx, op->fy, g.nx, g.ny, 1, 1, B * g.nz, op->rowmap, op->chirp, st));
  PAT_TRY(run_contract(op, false, w.Xs, w.Ds, B, st));
  return fft2_c2r(w.Ds, w.T, y, op->fx, op->fy, g.nx, g.ny, op->sx, op->sy, B * g.nt, inv_area(op), sub,
                  op->rowmap, op->chirp, st);
}

// x = A^T y, B data sets
static pat_status run_AT(pat_op* op, const float* y, float* x, int B, const Work& w, hipStream_t st) {
  const pat_geometry& g = op->g;
  PAT_TRY(fft2_r2c(y, w.T, w.Ds, op->fx, op->fy, g.nx, g.ny, op->sx, op->sy, B * g.nt, op->rowmap, op->chirp, st));
  PAT_TRY(run_contract(op, true, w.Ds, w.Xs, B, st));
  return fft2_c2r(w.Xs, w.T, x, op->fx, op->fy, g.nx, g.ny, 1, 1, B * g.nz, inv_area(op), nullptr,
                  op->rowmap, op->chirp, st);
}

// FISTA update with the gradient A^T r of B objects (r: data-shaped), the
// update in the last pass of A^T's inverse transform when that pass allows
// it (fft2_c2r_fista_ok), else A^T into the workspace and a separate update
// (Tnext != null: also the next iteration's first forward pass on the new z,
// see fft2_c2r_fista; only where fft2_c2r_fista_ok holds)
static pat_status run_AT_update(pat_op* op, const float* r, float* x, float* z, int B,
                                const FistaBatch& p, int32_t* nonfinite, const Work& w, hipStream_t st,
                                float2* Tnext = nullptr) {
  const pat_geometry& g = op->g;
  if (!fft2_c2r_fista_ok(g.nx, op->chirp, B * g.nz, g.nz)) {
    PAT_TRY(run_AT(op, r, w.U, B, w, st));
    return fista_update(x, z, w.U, (long long)g.nz * g.nx * g.ny, B, p, nonfinite, st);
  }
  PAT_TRY(fft2_r2c(r, w.T, w.Ds, op->fx, op->fy, g.nx, g.ny, op->sx, op->sy, B * g.nt, op->rowmap, op->chirp, st));
  PAT_TRY(run_contract(op, true, w.Ds, w.Xs, B, st));
  return fft2_c2r_fista(w.Xs, w.T, z, x, op->fx, op->fy, g.nx, g.ny, B * g.nz, g.nz, inv_area(op), nullptr,
                        op->rowmap, op->chirp, p, nonfinite, Tnext, st);
}

// FISTA update with the Gram-path gradient: the inverse transform of the
// spectra gs (G z^ - b^, or G z^ with sub = A^T d subtracted after the
// transform), the update fused into the transform's last pass when it
// allows it
static pat_status gram_update(pat_op* op, const float2* gs, const float* sub, float* x, float* z, int B,
                              const FistaBatch& p, int32_t* nonfinite, const Work& w, hipStream_t st,
                              float2* Tnext = nullptr) {
  const pat_geometry& g = op->g;
  if (!fft2_c2r_fista_ok(g.nx, op->chirp, B * g.nz, g.nz)) {
    PAT_TRY(fft2_c2r(gs, w.T, w.U, op->fx, op->fy, g.nx, g.ny, 1, 1, B * g.nz, inv_area(op), sub,
                     op->rowmap, op->chirp, st));
    return fista_update(x, z, w.U, (long long)g.nz * g.nx * g.ny, B, p, nonfinite, st);
  }
  return fft2_c2r_fista(gs, w.T, z, x, op->fx, op->fy, g.nx, g.ny, B * g.nz, g.nz, inv_area(op), sub,
                        op->rowmap, op->chirp, p, nonfinite, Tnext, st);
}

}  // namespace pat

using namespace pat;

// =================================================================== ABI
extern "C" {

const char* pat_status_str(pat_status s) {
  switch (s) {
    case PAT_OK: return "PAT_OK";
    case PAT_EINVAL: return "PAT_EINVAL";
    case PAT_EUNSUPPORTED: return "PAT_EUNSUPPORTED";
    case PAT_ENOMEM: return "PAT_ENOMEM";
    case PAT_EHIP: return "PAT_EHIP";
    case PAT_ENONFINITE: return "PAT_ENONFINITE";
  }
  return "PAT_UNKNOWN";
}

const char* pat_last_error(void) { return g_last_error.c_str(); }

pat_status pat_ctx_create(int device, pat_ctx** out) {
  if (!out) return fail(PAT_EINVAL, "out is null");
  *out = nullptr;
  int n = 0;
  PAT_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n || device >= kMaxDevices) return fail(PAT_EINVAL, "no such HIP device");
  hipDeviceProp_t prop;
  PAT_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PAT_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", not gfx950");
  PAT_HIP(hipSetDevice(device));
  PAT_TRY(fft_init_device());
  void* scratch = nullptr;
  PAT_TRY(scratch_address(device, &scratch));
  pat_ctx* c = new (std::nothrow) pat_ctx;
  if (!c) return fail(PAT_ENOMEM, "host allocation failed");
  c->device = device;
  c->scratch = scratch;
  *out = c;
  return PAT_OK;
}

void pat_ctx_destroy(pat_ctx* ctx) { delete ctx; }

pat_status pat_H_bytes(const pat_geometry* geom, size_t* h_bytes, size_t* scratch_bytes) {
  PAT_TRY(check_geometry(geom));
  if (!h_bytes) return fail(PAT_EINVAL, "h_bytes is null");
  const pat_geometry tg = transform_geometry(*geom);
  Classes C = make_classes(tg);
  *h_bytes = h_layout(tg, C).total;
  if (scratch_bytes) *scratch_bytes = step_scratch_bytes(*geom, C.n());
  return PAT_OK;
}

pat_status pat_H_build(pat_ctx* ctx, const pat_geometry* geom, void* h_buf, size_t h_bytes,
                       void* scratch, size_t scratch_bytes, void* stream, pat_op** out) {
  if (!ctx || !out) return fail(PAT_EINVAL, "ctx or out is null");
  *out = nullptr;
  PAT_TRY(check_geometry(geom));
  PAT_TRY(check_ptr(h_buf, "h_buf"));
  const pat_geometry tg = transform_geometry(*geom);
  Classes C = make_classes(tg);
  HLayout L = h_layout(tg, C);
  if (h_bytes < L.total)
    return fail(PAT_EINVAL, "h_buf too small: need " + std::to_string(L.total) + " bytes");
  if (geom->build == PAT_BUILD_STEP) {
    PAT_TRY(check_ptr(scratch, "scratch"));
    const int nq = geom->nz_sim ? geom->nz_sim : default_nq(*geom);
    if (scratch_bytes < step_class_bytes(geom->nt, nq))
      return fail(PAT_EINVAL, "scratch too small for the stepped build: need at least " +
                                  std::to_string(step_class_bytes(geom->nt, nq)) + " bytes");
  }
  for (int32_t kc : C.kclass)
    if (kc < 0) return fail(PAT_EINVAL, "internal: frequency without class");
  PAT_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;

  pat_op* op = new (std::nothrow) pat_op;
  if (!op) return fail(PAT_ENOMEM, "host allocation failed");
  op->ctx = ctx;
  op->g = *geom;
  op->h_ir.assign(geom->ir, geom->ir + geom->n_ir);
  op->g.ir = nullptr;  // not retained: the taps live in h_ir and in the library
  op->nq = geom->nz_sim ? geom->nz_sim : default_nq(*geom);
  op->g.nz_sim = op->nq;
  op->fx = tg.nx;
  op->fy = tg.ny;
  op->sx = scan_sx(*geom);
  op->sy = scan_sy(*geom);
  op->nh = op->fx / 2 + 1;
  op->nk = op->fy * op->nh;
  op->G = L.G;
  op->nclass = L.nclass;
  op->nitem = L.nitem;
  op->vec = L.vec;
  op->sA_row = L.sA_row;
  op->sT_row = L.sT_row;
  op->ntA = L.ntA;
  op->ksA = L.ksA;
  op->ntT = L.ntT;
  op->ksT = L.ksT;
  op->hbuf = (char*)h_buf;
  op->nrows = L.nitem * L.G;
  op->members = (int32_t*)(op->hbuf + L.off_members);
  op->item_slab = (int32_t*)(op->hbuf + L.off_items);
  op->kclass = (int32_t*)(op->hbuf + L.off_kclass);
  op->rowmap = (int32_t*)(op->hbuf + L.off_rowmap);
  op->cls_freq = (int32_t*)(op->hbuf + L.off_freq);
  op->inv_scale = (float*)(op->hbuf + L.off_inv);
  op->amax = (unsigned long long*)(op->hbuf + L.off_amax);
  op->rowA = op->hbuf + L.off_Ar;
  op->rowT = op->hbuf + L.off_Tr;
  const bool f32 = geom->h_dtype == PAT_H_F32;
  op->slabA = f32 ? op->rowA : op->hbuf + L.off_A;
  op->slabT = f32 ? op->rowT : op->hbuf + L.off_T;
  op->gram = L.bytes_G ? (float*)(op->hbuf + L.off_G) : nullptr;
  op->kexpA = L.bytes_X ? (int32_t*)(op->hbuf + L.off_X) : nullptr;
  op->kexpT = L.bytes_X ? op->kexpA + (size_t)L.nclass * geom->nt : nullptr;
  op->sG_row = L.sG_row;
  op->h_members = std::move(C.members);
  op->h_kclass = std::move(C.kclass);
  op->h_cls_freq = std::move(C.freq);
  op->h_rowmap = std::move(C.rowmap);
  op->h_item_slab = std::move(C.item_slab);

  auto bail = [&](pat_status s) {
    delete op;
    return s;
  };
  pat_status s;
  // zero everything first: slab padding must read as zero
  if ((s = fill_zero(h_buf, L.total, st)) != PAT_OK) return bail(s);
  if ((s = hip_check(hipMemcpyAsync(op->members, op->h_members.data(), op->h_members.size() * 4,
                                    hipMemcpyHostToDevice, st), "upload members")) != PAT_OK)
    return bail(s);
  if ((s = hip_check(hipMemcpyAsync(op->kclass, op->h_kclass.data(), op->h_kclass.size() * 4,
                                    hipMemcpyHostToDevice, st), "upload classes")) != PAT_OK)
    return bail(s);
  if ((s = hip_check(hipMemcpyAsync(op->cls_freq, op->h_cls_freq.data(), op->h_cls_freq.size() * 4,
                                    hipMemcpyHostToDevice, st), "upload frequencies")) != PAT_OK)
    return bail(s);
  if ((s = hip_check(hipMemcpyAsync(op->rowmap, op->h_rowmap.data(), op->h_rowmap.size() * 4,
                                    hipMemcpyHostToDevice, st), "upload row map")) != PAT_OK)
    return bail(s);
  if ((s = hip_check(hipMemcpyAsync(op->item_slab, op->h_item_slab.data(), op->h_item_slab.size() * 4,
                                    hipMemcpyHostToDevice, st), "upload items")) != PAT_OK)
    return bail(s);
  double* d_ir = reinterpret_cast<double*>(op->hbuf + L.off_ir);
  if (geom->n_ir > 0 &&
      (s = hip_check(hipMemcpyAsync(d_ir, op->h_ir.data(), op->h_ir.size() * 8, hipMemcpyHostToDevice, st),
                     "upload sensor response")) != PAT_OK)
    return bail(s);
  if (L.bytes_cz) {  // chirp-z tables of the transform axes that need them
    float2* d_cz = reinterpret_cast<float2*>(op->hbuf + L.off_cz);
    const int nxg = op->fx, nyg = op->fy;
    if (chirp_size(nxg)) {
      chirp_tables(nxg, chirp_m(nxg), op->h_cz);
      op->chirp.cx = d_cz;
      op->chirp.bx = d_cz + nxg;
      op->chirp.mx = chirp_m(nxg);
    }
    if (chirp_size(nyg)) {
      const size_t o0 = op->h_cz.size();
      chirp_tables(nyg, chirp_m(nyg), op->h_cz);
      op->chirp.cy = d_cz + o0;
      op->chirp.by = d_cz + o0 + nyg;
      op->chirp.my = chirp_m(nyg);
    }
    if ((s = hip_check(hipMemcpyAsync(d_cz, op->h_cz.data(), op->h_cz.size() * sizeof(float2),
                                      hipMemcpyHostToDevice, st), "upload chirp-z tables")) != PAT_OK)
      return bail(s);
  }
  HBuildArgs a;
  a.ir = geom->n_ir > 0 ? d_ir : nullptr;
  a.n_ir = geom->n_ir;
  a.cls_freq = op->cls_freq;
  a.nclass = op->nclass;
  a.nx = op->fx;
  a.ny = op->fy;
  a.nz = geom->nz;
  a.nt = geom->nt;
  a.nq = op->nq;
  a.dx = geom->dx;
  a.dy = geom->dy;
  a.dz = geom->dz;
  a.dt = geom->dt;
  a.c = geom->c;
  a.slabA = op->slabA;
  a.slabT = op->slabT;
  a.rowA = op->rowA;
  a.rowT = op->rowT;
  a.sA_row = op->sA_row;
  a.sT_row = op->sT_row;
  a.ntA = op->ntA;
  a.ksA = op->ksA;
  a.ntT = op->ntT;
  a.ksT = op->ksT;
  a.amax = op->amax;
  a.inv_scale = op->inv_scale;
  a.hdtype = geom->h_dtype;
  a.ptab = geom->build == PAT_BUILD_STEP ? static_cast<double*>(scratch) : nullptr;
  a.ptab_bytes = geom->build == PAT_BUILD_STEP ? scratch_bytes : 0;
  a.c0 = 0;
  if ((s = hbuild(a, st)) != PAT_OK) return bail(s);
  if (f32) {
    if ((s = row_exponents(static_cast<const float*>(op->rowT), (long long)op->nclass * geom->nt, geom->nz,
                           op->sT_row, op->kexpA, st)) != PAT_OK)
      return bail(s);
    if ((s = row_exponents(static_cast<const float*>(op->rowA), (long long)op->nclass * geom->nz, geom->nt,
                           op->sA_row, op->kexpT, st)) != PAT_OK)
      return bail(s);
  }
  GramArgs ga;
  ga.slabA = op->slabA;
  ga.inv_scale = op->inv_scale;
  ga.gram = op->gram;
  ga.nslab = op->nclass;
  ga.nz = geom->nz;
  ga.nt = geom->nt;
  ga.sA_row = op->sA_row;
  ga.ntA = op->ntA;
  ga.ksA = op->ksA;
  ga.sG_row = op->sG_row;
  ga.hdtype = geom->h_dtype;
  if (op->gram && (s = gram_build(ga, st)) != PAT_OK) return bail(s);
  *out = op;
  return PAT_OK;
}

pat_status pat_op_destroy(pat_op* op) {
  delete op;
  return PAT_OK;
}

pat_status pat_H_export(pat_op* op, int32_t k0, int32_t nk, float* out, void* stream) {
  if (!op) return fail(PAT_EINVAL, "operator is null");
  if (k0 < 0 || nk < 0 || (long long)k0 + nk > op->nk) return fail(PAT_EINVAL, "frequency range out of bounds");
  if (nk == 0) return PAT_OK;
  PAT_TRY(check_ptr(out, "out"));
  PAT_HIP(hipSetDevice(op->ctx->device));
  return hexport(op->slabA, op->g.h_dtype, op->kclass, op->inv_scale, k0, nk, op->g.nz, op->g.nt,
                 op->sA_row, op->ntA, op->ksA, out, (hipStream_t)stream);
}

pat_status pat_get_info(const pat_op* op, pat_op_info* info) {
  if (!op || !info) return fail(PAT_EINVAL, "null argument");
  const pat_geometry tg = transform_geometry(op->g);
  Classes C = make_classes(tg);
  const HLayout L = h_layout(tg, C);
  info->nk = op->nk;
  info->nclass = op->nclass;
  info->members_max = op->G;
  info->nz_sim = op->nq;
  info->slab_bytes_A = L.bytes_Ar;
  info->slab_bytes_AT = L.bytes_Tr;
  info->nitems = op->nitem;
  info->read_bytes_A = L.bytes_Ar / op->nclass * op->nitem;
  info->read_bytes_AT = L.bytes_Tr / op->nclass * op->nitem;
  info->spec_rows = op->nrows;
  info->gram_bytes = L.bytes_G;
  return PAT_OK;
}

pat_status pat_spectrum_rows(const pat_op* op, int32_t* k_of_row) {
  if (!op || !k_of_row) return fail(PAT_EINVAL, "null argument");
  for (int r = 0; r < op->nrows; ++r) k_of_row[r] = op->h_members[r];
  return PAT_OK;
}

pat_status pat_spectrum_stride(int32_t S, int32_t* stride) {
  if (!stride) return fail(PAT_EINVAL, "null argument");
  if (S < 1 || S > (1 << 30)) return fail(PAT_EINVAL, "S must be in [1, 2^30]");
  *stride = spec_stride(S);
  return PAT_OK;
}

pat_status pat_workspace_bytes(const pat_op* op, int32_t B, size_t* bytes) {
  if (!op || !bytes) return fail(PAT_EINVAL, "null argument");
  PAT_TRY(check_batch(op, B));
  *bytes = work_layout(op, B, nullptr).total;
  return PAT_OK;
}

pat_status pat_apply_A(pat_op* op, const float* x, float* y, int32_t B, void* ws, size_t ws_bytes,
                       void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, B, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(y, "y"));
  return run_A(op, x, y, B, nullptr, w, (hipStream_t)stream);
}

pat_status pat_apply_AT(pat_op* op, const float* y, float* x, int32_t B, void* ws, size_t ws_bytes,
                        void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, B, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(y, "y"));
  return run_AT(op, y, x, B, w, (hipStream_t)stream);
}

pat_status pat_apply_A_noalloc(pat_op* op, const float* x, float* y, int32_t B, void* stream) {
  if (!op) return fail(PAT_EINVAL, "operator is null");
  PAT_TRY(check_batch(op, B));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(y, "y"));
  const size_t need = work_layout(op, B, nullptr, true).total;
  if (need > kNoAllocBytes)
    return fail(PAT_EUNSUPPORTED, "this apply needs " + std::to_string(need) +
                                      " bytes of scratch, more than the " + std::to_string(kNoAllocBytes) +
                                      " of the static scratch: use pat_apply_A with a workspace");
  if (!op->ctx->scratch) return fail(PAT_EHIP, "the context has no scratch address");
  PAT_HIP(hipSetDevice(op->ctx->device));
  // nothing in the scratch needs to start at zero: every spectrum row and
  // intermediate element an apply reads was written earlier in the same apply
  const Work w = work_layout(op, B, static_cast<char*>(op->ctx->scratch), true);
  return run_A(op, x, y, B, nullptr, w, (hipStream_t)stream);
}

// workspace rows of T (complex) available for S slices
static pat_status check_stage(pat_op* op, int S, void* ws, size_t ws_bytes, Work* w) {
  if (!op) return fail(PAT_EINVAL, "operator is null");
  if (S < 1 || S > (1 << 30)) return fail(PAT_EINVAL, "S must be in [1, 2^30]");
  const int per = std::max(op->g.nz, op->g.nt);
  const int B = (S + per - 1) / per;
  return check_op_call(op, B, ws, ws_bytes, w);
}

pat_status pat_spectrum(pat_op* op, const float* f, float* spec, int32_t S, void* ws,
                        size_t ws_bytes, void* stream) {
  Work w;
  PAT_TRY(check_stage(op, S, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(f, "f"));
  PAT_TRY(check_ptr(spec, "spec"));
  return fft2_r2c(f, w.T, (float2*)spec, op->fx, op->fy, op->g.nx, op->g.ny, 1, 1, S, op->rowmap,
                  op->chirp, (hipStream_t)stream);
}

pat_status pat_inverse_spectrum(pat_op* op, const float* spec, float* f, int32_t S, const float* sub,
                                void* ws, size_t ws_bytes, void* stream) {
  Work w;
  PAT_TRY(check_stage(op, S, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(f, "f"));
  PAT_TRY(check_ptr(spec, "spec"));
  if (sub) PAT_TRY(check_ptr(sub, "sub"));
  return fft2_c2r((const float2*)spec, w.T, f, op->fx, op->fy, op->g.nx, op->g.ny, 1, 1, S,
                  inv_area(op), sub, op->rowmap, op->chirp, (hipStream_t)stream);
}

pat_status pat_contract(pat_op* op, int32_t adjoint, const float* in, float* out, int32_t B,
                        void* stream) {
  if (!op) return fail(PAT_EINVAL, "operator is null");
  PAT_TRY(check_batch(op, B));
  PAT_TRY(check_ptr(in, "in"));
  PAT_TRY(check_ptr(out, "out"));
  PAT_HIP(hipSetDevice(op->ctx->device));
  return run_contract(op, adjoint != 0, (const float2*)in, (float2*)out, B, (hipStream_t)stream);
}

pat_status pat_power_norm(pat_op* op, const float* v0, int32_t niter, double* L_out,
                          double* L_trace, void* ws, size_t ws_bytes, void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, 1, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(v0, "v0"));
  if (!L_out) return fail(PAT_EINVAL, "L_out is null");
  if (niter < 1 || niter > kMaxPowerIter) return fail(PAT_EINVAL, "niter must be in [1, 4096]");
  hipStream_t st = (hipStream_t)stream;
  const pat_geometry& g = op->g;
  const long long n = (long long)g.nz * g.nx * g.ny;
  float* Ls = w.s32 + 8;
  PAT_TRY(dot_f32(v0, v0, n, w.part32, w.s32, 1.f, st));
  PAT_TRY(scale_rsqrt(w.V, v0, n, w.s32, st));
  for (int i = 0; i < niter; ++i) {
    if (op->gram) {
      // A^T A v per frequency through the Gram blocks: one forward transform,
      // one nz x nz contraction, one inverse transform
      PAT_TRY(fft2_r2c(w.V, w.T, w.Xs, op->fx, op->fy, g.nx, g.ny, 1, 1, g.nz, op->rowmap, op->chirp, st));
      PAT_TRY(run_gram(op, w.Xs, w.Gs, nullptr, 1, st));
      PAT_TRY(fft2_c2r(w.Gs, w.T, w.U, op->fx, op->fy, g.nx, g.ny, 1, 1, g.nz, inv_area(op), nullptr,
                       op->rowmap, op->chirp, st));
    } else {
      PAT_TRY(run_A(op, w.V, w.R, 1, nullptr, w, st));
      PAT_TRY(run_AT(op, w.R, w.U, 1, w, st));
    }
    PAT_TRY(dot_f32(w.V, w.U, n, w.part32, Ls + i, 1.f, st));
    PAT_TRY(dot_f32(w.U, w.U, n, w.part32, w.s32 + 1, 1.f, st));
    PAT_TRY(scale_rsqrt(w.V, w.U, n, w.s32 + 1, st));
  }
  std::vector<float> hL(niter);
  PAT_HIP(hipMemcpyAsync(hL.data(), Ls, niter * sizeof(float), hipMemcpyDeviceToHost, st));
  PAT_HIP(hipStreamSynchronize(st));
  *L_out = hL[niter - 1];
  if (L_trace)
    for (int i = 0; i < niter; ++i) L_trace[i] = hL[i];
  return PAT_OK;
}

pat_status pat_recon_fista(pat_op* op, const float* d, float* x, int32_t niter, float tau,
                           float lambda, int32_t nonneg, int32_t momentum, float* trace, void* ws,
                           size_t ws_bytes, void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, 1, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(d, "d"));
  PAT_TRY(check_ptr(x, "x"));
  if (niter < 0) return fail(PAT_EINVAL, "niter must be >= 0");
  if (!(tau > 0.f) || !(lambda >= 0.f)) return fail(PAT_EINVAL, "tau must be > 0 and lambda >= 0");
  hipStream_t st = (hipStream_t)stream;
  const pat_geometry& g = op->g;
  const long long n = (long long)g.nz * g.nx * g.ny;
  const long long nd = (long long)g.nt * (g.nx / op->sx) * (g.ny / op->sy);
  const float inv = inv_area(op);
  // The periodic operator is block diagonal in the transverse frequency, so
  // A^T A is too and the gradient is formed per frequency with the Gram
  // blocks.  The linear boundary (crop) and the scan-grid sampling act on
  // the data between A and A^T and couple frequencies: their gradient is
  // taken explicitly, A then A^T.
  const bool normal = op->gram != nullptr;
  if (normal) {
    // b^ = spectrum of A^T d (the adjoint up to its inverse transform), once
    PAT_TRY(fft2_r2c(d, w.T, w.Ds, op->fx, op->fy, g.nx, g.ny, op->sx, op->sy, g.nt, op->rowmap, op->chirp, st));
    PAT_TRY(run_contract(op, true, w.Ds, w.Bs, 1, st));
    if (trace) {
      PAT_TRY(fft2_c2r(w.Bs, w.T, w.V, op->fx, op->fy, g.nx, g.ny, 1, 1, g.nz, inv, nullptr, op->rowmap, op->chirp, st));  // b = A^T d
      PAT_TRY(dot_f64(d, d, nd, w.part64, w.s64 + 2, st));
    }
  } else if (trace) {
    PAT_TRY(fill_zero(w.s64, 3 * sizeof(double), st));  // the trace is 1/2 <r, r> alone
  }
  PAT_TRY(fill_zero(x, n * 4, st));
  PAT_TRY(fill_zero(w.Z, n * 4, st));
  double t = 1.0;
  FistaBatch p;
  std::memset(&p, 0, sizeof(p));
  const bool chain = !trace && fft2_c2r_fista_ok(g.nx, op->chirp, g.nz, g.nz);
  bool rows_done = false;  // w.T holds the first forward pass on z
  for (int k = 1; k <= niter; ++k) {
    double beta = 0.0;
    if (momentum) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      beta = (t - 1.0) / tn;
      t = tn;
    }
    p.o[0].tau = tau;
    p.o[0].thr = tau * lambda;
    p.o[0].beta = (float)beta;
    p.o[0].nonneg = nonneg ? 1 : 0;
    // Without a trace, the update of every iteration but the last also runs
    // the next iteration's first forward pass on the new z (into w.T)
    float2* next = (chain && k < niter) ? w.T : nullptr;
    if (normal) {
      // gradient A^T (A z - d) = A^T A z - A^T d, per frequency: G z^ - b^
      if (rows_done)
        PAT_TRY(fft2_r2c_cols(w.T, w.Xs, op->fx, op->fy, g.ny, g.nz, op->rowmap, op->chirp, st));
      else
        PAT_TRY(fft2_r2c(w.Z, w.T, w.Xs, op->fx, op->fy, g.nx, g.ny, 1, 1, g.nz, op->rowmap, op->chirp, st));
      PAT_TRY(run_gram(op, w.Xs, w.Gs, w.Bs, 1, st));
      if (trace) {
        // the data term needs the gradient itself:
        // 1/2 ||A z - d||^2 = 1/2 (<z, g> - <z, b> + ||d||^2), float64 sums
        PAT_TRY(fft2_c2r(w.Gs, w.T, w.U, op->fx, op->fy, g.nx, g.ny, 1, 1, g.nz, inv, nullptr, op->rowmap, op->chirp, st));
        PAT_TRY(dot_f64(w.Z, w.U, n, w.part64, w.s64 + 0, st));
        PAT_TRY(dot_f64(w.Z, w.V, n, w.part64, w.s64 + 1, st));
        PAT_TRY(trace_combine(trace + (k - 1), w.s64, st));
        PAT_TRY(fista_update(x, w.Z, w.U, n, 1, p, nullptr, st));
      } else {
        PAT_TRY(gram_update(op, w.Gs, nullptr, x, w.Z, 1, p, nullptr, w, st, next));
      }
    } else {
      // explicit: residual r = A z - d (fused into the inverse transform), g = A^T r
      PAT_TRY(run_A(op, w.Z, w.R, 1, d, w, st, rows_done));
      if (trace) {
        PAT_TRY(dot_f64(w.R, w.R, nd, w.part64, w.s64 + 0, st));
        PAT_TRY(trace_combine(trace + (k - 1), w.s64, st));
      }
      PAT_TRY(run_AT_update(op, w.R, x, w.Z, 1, p, nullptr, w, st, next));
    }
    rows_done = next != nullptr;
  }
  return PAT_OK;
}

pat_status pat_fista_step(pat_op* op, int32_t B, const float* d, float* x, float* z,
                          const double* beta, const float* tau, const float* lambda,
                          const int32_t* nonneg, int32_t* nonfinite, void* ws, size_t ws_bytes,
                          void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, B, ws, ws_bytes, &w));
  if (B > 32) return fail(PAT_EINVAL, "B must be <= 32");
  PAT_TRY(check_ptr(d, "d"));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(z, "z"));
  if (!beta || !tau || !lambda || !nonneg) return fail(PAT_EINVAL, "per-object parameters are null");
  hipStream_t st = (hipStream_t)stream;
  FistaBatch p;
  std::memset(&p, 0, sizeof(p));
  for (int b = 0; b < B; ++b) {
    if (!(tau[b] > 0.f) || !(lambda[b] >= 0.f)) return fail(PAT_EINVAL, "tau must be > 0 and lambda >= 0");
    p.o[b].tau = tau[b];
    p.o[b].thr = tau[b] * lambda[b];
    p.o[b].beta = (float)beta[b];
    p.o[b].nonneg = nonneg[b] ? 1 : 0;
  }
  PAT_TRY(run_A(op, z, w.R, B, d, w, st));
  return run_AT_update(op, w.R, x, z, B, p, nonfinite, w, st);
}

pat_status pat_fista_step_normal(pat_op* op, int32_t B, const float* atd, float* x, float* z,
                                 const double* beta, const float* tau, const float* lambda,
                                 const int32_t* nonneg, int32_t* nonfinite, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (op && !op->gram)
    return fail(PAT_EUNSUPPORTED,
                "the normal-operator step needs Gram blocks: periodic boundary, unsampled data");
  Work w;
  PAT_TRY(check_op_call(op, B, ws, ws_bytes, &w));
  if (B > 32) return fail(PAT_EINVAL, "B must be <= 32");
  PAT_TRY(check_ptr(atd, "atd"));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(z, "z"));
  if (!beta || !tau || !lambda || !nonneg) return fail(PAT_EINVAL, "per-object parameters are null");
  hipStream_t st = (hipStream_t)stream;
  FistaBatch p;
  std::memset(&p, 0, sizeof(p));
  for (int b = 0; b < B; ++b) {
    if (!(tau[b] > 0.f) || !(lambda[b] >= 0.f)) return fail(PAT_EINVAL, "tau must be > 0 and lambda >= 0");
    p.o[b].tau = tau[b];
    p.o[b].thr = tau[b] * lambda[b];
    p.o[b].beta = (float)beta[b];
    p.o[b].nonneg = nonneg[b] ? 1 : 0;
  }
  const pat_geometry& g = op->g;
  PAT_TRY(fft2_r2c(z, w.T, w.Xs, op->fx, op->fy, g.nx, g.ny, 1, 1, B * g.nz, op->rowmap, op->chirp, st));
  PAT_TRY(run_gram(op, w.Xs, w.Gs, nullptr, B, st));
  return gram_update(op, w.Gs, atd, x, z, B, p, nonfinite, w, st);  // gradient A^T A z - A^T d
}

pat_status pat_adjoint_check(pat_op* op, const float* x, const float* y, double* rel_out, void* ws,
                             size_t ws_bytes, void* stream) {
  Work w;
  PAT_TRY(check_op_call(op, 1, ws, ws_bytes, &w));
  PAT_TRY(check_ptr(x, "x"));
  PAT_TRY(check_ptr(y, "y"));
  if (!rel_out) return fail(PAT_EINVAL, "rel_out is null");
  hipStream_t st = (hipStream_t)stream;
  const pat_geometry& g = op->g;
  const long long n = (long long)g.nz * g.nx * g.ny;
  const long long nd = (long long)g.nt * (g.nx / op->sx) * (g.ny / op->sy);
  PAT_TRY(run_A(op, x, w.R, 1, nullptr, w, st));
  PAT_TRY(run_AT(op, y, w.U, 1, w, st));
  PAT_TRY(dot_f64(w.R, y, nd, w.part64, w.s64 + 0, st));
  PAT_TRY(dot_f64(x, w.U, n, w.part64, w.s64 + 1, st));
  PAT_TRY(dot_f64(w.R, w.R, nd, w.part64, w.s64 + 2, st));
  PAT_TRY(dot_f64(y, y, nd, w.part64, w.s64 + 3, st));
  double h[4];
  PAT_HIP(hipMemcpyAsync(h, w.s64, sizeof(h), hipMemcpyDeviceToHost, st));
  PAT_HIP(hipStreamSynchronize(st));
  *rel_out = std::fabs(h[0] - h[1]) / std::sqrt(h[2] * h[3]);
  return PAT_OK;
}

}  // extern "C"
