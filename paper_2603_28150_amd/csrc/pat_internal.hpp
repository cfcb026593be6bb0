// Internal declarations shared by the translation units of libpat.so.
// Not part of the ABI (see include/pat.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pat.h"

namespace pat {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
pat_status fail(pat_status s, const std::string& msg);
pat_status hip_check(hipError_t e, const char* what);
#define PAT_TRY(expr)                       \
  do {                                      \
    pat_status _s = (expr);                 \
    if (_s != PAT_OK) return _s;            \
  } while (0)
#define PAT_HIP(expr) PAT_TRY(::pat::hip_check((expr), #expr))
// After a launch: reports launch-configuration errors.
#define PAT_LAUNCHED(what) PAT_TRY(::pat::hip_check(hipGetLastError(), what))

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// --------------------------------------------------------------- 2D FFTs
// Row stride (complex elements) of frequency-major arrays holding S slices:
// S rounded up to 64, plus 32, i.e. an odd multiple of 256 bytes and never a
// power of two.  Power-of-two strides (4 KB .. 64 KB at the usual slice
// counts) map the rows read or written together onto the same few HBM
// channels and halve the column pass's bandwidth.
inline int spec_stride(int S) { return (S + 63) / 64 * 64 + 32; }

// Slice layouts (S slices, element type float / float2, rs = spec_stride(S)):
//   real slices      f[s][nyw/sy][nxw/sx]
//   half spectrum    X[row(p*nh + m) * rs + s] (frequency rows, slice fastest;
//                    nh = nx/2 + 1; row() is the class-major row map, or the
//                    identity when rowmap is null)
//   row-transformed  T[(j*nh + m) * rs + s]   (y not yet transformed)
// Forward transforms are unnormalised; the inverse multiplies by `scale`.
pat_status fft_init_device();  // uploads the twiddle table to the current device
// Chirp-z tables of an axis whose length n is not a fast FFT size: c[n]
// (exp(i pi k^2 / n), k < n) and the m-point DFT of the chirp kernel over m
// (m a power of two >= 2n - 1), device arrays; m = 0: the axis uses the fast
// transforms.
struct FftChirp {
  const float2* cx = nullptr;
  const float2* bx = nullptr;
  int mx = 0;
  const float2* cy = nullptr;
  const float2* by = nullptr;
  int my = 0;
};
// f holds S slices covering the nxw x nyw window of the fx x fy transform
// grid (fast sizes, or chirp-z lengths), sampled every sx columns and sy rows:
// f[s][nyw/sy][nxw/sx].  Zero-padding and zero-filling on the way in,
// cropping and sampling on the way out.
// An axis with chirp-z tables (ch.mx / ch.my > 0) must be covered whole and
// unsampled.
pat_status fft2_r2c(const float* f, float2* T, float2* X, int fx, int fy, int nxw, int nyw, int sx,
                    int sy, int S, const int32_t* rowmap, const FftChirp& ch, hipStream_t st);
// f = scale * c2r(X) - sub (sub may be null; same layout as f)
pat_status fft2_c2r(const float2* X, float2* T, float* f, int fx, int fy, int nxw, int nyw, int sx,
                    int sy, int S, float scale, const float* sub, const int32_t* rowmap,
                    const FftChirp& ch, hipStream_t st);

// ------------------------------------------------------ contraction (VALU)
// out[t*G+g][obj*nj + j] = sum_i slab_s[i][j] * in[t*G+g][obj*ni + i] (* scales)
// for every work item t, its slab s = item_slab[t] and member slots g < G
// (members[t*G+g] < 0: empty; filled slots come first).
struct ContractArgs {
  const void* slab;          // [nslab][ni][s_row] of the storage type
  const int32_t* members;    // [nitem][G]
  const int32_t* item_slab;  // [nitem]
  const float2* in;          // [nitem*G][in_rs]  item-major spectrum rows
  float2* out;               // [nitem*G][out_rs]
  const float* in_scale;   // [ni] or null
  const float* out_scale;  // [nj] or null
  const float2* out_sub;   // null, or rows like out: out = result - out_sub
  int ni, nj, s_row;
  long long slab_elems;    // ni * s_row
  int in_rs, out_rs;
  int nitem;
};
pat_status contract(const ContractArgs& a, int hdtype, int G, int B, hipStream_t st);

// ------------------------------------------------------ contraction (MFMA)
// out[c*G+g][b*N + n] = sum_k X[c*G+g][b*K + k] * S_c(k, n) for 16-bit slabs
// stored as 32 x 16 bf16/f16 fragments in MFMA B-operand lane order:
// fragment (tile, kstep) of class c holds S_c(kstep*16 + 8*(lane/32) + e,
// tile*32 + lane%32) at 16-byte unit lane, element e.
struct MfmaArgs {
  const void* frag;          // 16-bit libraries: [nslab][ntiles][ksteps][64] 16-byte units (else null)
  const int32_t* members;    // [nitem][G]
  const int32_t* item_slab;  // [nitem]
  const float2* in;          // [nitem*G][in_rs]
  float2* out;               // [nitem*G][out_rs]
  const float* in_scale;     // [K] or null
  const float* out_scale;    // [N] or null
  int K, N, ntiles, ksteps, in_rs, out_rs, G, B, nitem;
  const float* krows;        // float32 libraries: [nslab][N][k_srow] rows along k (else null)
  int k_srow;
  long long k_slab;          // N * k_srow
  const int32_t* kexp;       // float32 libraries: [nslab][N] exponent e of each k row, max |row| 2^e < 2^15
};
pat_status contract_mfma(const MfmaArgs& a, int hdtype, hipStream_t st);
// exponent e of each of nrows rows of K floats (row stride srow): the power
// of two that takes the row's largest magnitude m to m 2^e in [2^14, 2^15)
// (0 for all-zero rows)
pat_status row_exponents(const float* rows, long long nrows, int K, int srow, int32_t* ex, hipStream_t st);

// ------------------------------------------------------------- H^ build
struct HBuildArgs {
  const int32_t* cls_freq;  // [C][2]: |m~|, |p~| (x and y frequency indices)
  int nclass, nx, ny, nz, nt, nq;
  double dx, dy, dz, dt, c;
  void* slabA;              // FP32: [C][nz][sA_row] (n fastest); 16-bit: fragments (n, k=l)
  void* slabT;              // FP32: [C][nt][sT_row] (l fastest); 16-bit: fragments (l, k=n)
  void* rowA;               // [C][nz][sA_row] rows of the storage type (= slabA for FP32)
  void* rowT;               // [C][nt][sT_row] rows of the storage type (= slabT for FP32)
  int sA_row, sT_row;
  int ntA, ksA, ntT, ksT;   // fragment tiling of the 16-bit layouts
  unsigned long long* amax; // [nz] bit patterns of max |H^| per depth
  float* inv_scale;         // [nz] 1/s_l
  int hdtype;
  const double* ir;         // [n_ir] sensor response taps (device), or null
  int n_ir;                 // 0: ideal sensors
  // stepped build: the recorded fields of classes c0 .. c0 + ncb - 1,
  // ptab[(c - c0) * nt + n][q] (q < nq/2 + 1, weighted by w_q / nq); null:
  // closed form
  double* ptab;
  size_t ptab_bytes;
  int c0;
};
constexpr int kMaxIr = 64;  // longest sensor response folded into the library
pat_status hbuild(const HBuildArgs& a, hipStream_t st);
// bytes of the stepped build's record of one class
inline size_t step_class_bytes(int nt, int nq) { return (size_t)nt * (nq / 2 + 1) * 8; }
struct GramArgs {
  const void* slabA;        // stored library, [l][n] rows (FP32) or fragments (16-bit)
  const float* inv_scale;   // [nz]
  float* gram;              // [nslab][nz][sG_row]
  int nslab, nz, nt, sA_row, ntA, ksA, sG_row, hdtype;
};
pat_status gram_build(const GramArgs& a, hipStream_t st);

pat_status hexport(const void* slabA, int hdtype, const int32_t* kclass, const float* inv_scale,
                   int k0, int nk, int nz, int nt, int sA_row, int ntA, int ksA, float* out,
                   hipStream_t st);

// ------------------------------------------------------- vector kernels
pat_status fill_zero(void* p, size_t bytes, hipStream_t st);
// partial sums of a*b (or a*a when b == a) over n floats into part[nblk]; float or double accumulation
pat_status dot_f32(const float* a, const float* b, long long n, float* part, float* result,
                   float post_scale, hipStream_t st);
pat_status dot_f64(const float* a, const float* b, long long n, double* part, double* result,
                   hipStream_t st);
// out[0] = (s[0] - s[1] + s[2]) / 2
pat_status trace_combine(float* out, const double* s, hipStream_t st);
// dst = src / sqrt(*nrm2)
pat_status scale_rsqrt(float* dst, const float* src, long long n, const float* nrm2, hipStream_t st);

struct FistaObj {
  float tau, thr, beta;
  int nonneg;
};
struct FistaBatch {
  FistaObj o[32];
};
// per object b: x_old = x; x = prox(z - tau g); z = x + beta (x - x_old)
pat_status fista_update(float* x, float* z, const float* g, long long n_per_obj, int B,
                        const FistaBatch& p, int32_t* nonfinite, hipStream_t st);
// fft2_c2r (unsampled) and fista_update in one: the gradient of slice s is
// g = scale * c2r(X) - sub, of object s / per_obj, and x, z (slices like
// the inverse transform's output) are updated in its last pass without g
// being stored.  Needs a fast x axis, nxw % 4 == 0 and per_obj a multiple
// of 16 unless S == per_obj (EUNSUPPORTED otherwise; fft2_c2r_fista_ok says
// beforehand).  Tnext != null: also the next iteration's forward row pass on
// the new z (unsampled slices, as fft2_r2c's first pass writes it), in the
// layout of T; Tnext may be T.
bool fft2_c2r_fista_ok(int nxw, const FftChirp& ch, int S, int per_obj);
pat_status fft2_c2r_fista(const float2* X, float2* T, float* z, float* x, int fx, int fy, int nxw,
                          int nyw, int S, int per_obj, float scale, const float* sub,
                          const int32_t* rowmap, const FftChirp& ch, const FistaBatch& p,
                          int32_t* nonfinite, float2* Tnext, hipStream_t st);
// the second (column) pass of fft2_r2c alone, for unsampled slices whose
// first pass is already in T (from fft2_c2r_fista with Tnext)
pat_status fft2_r2c_cols(const float2* T, float2* X, int fx, int fy, int nyw, int S, const int32_t* rowmap,
                         const FftChirp& ch, hipStream_t st);

constexpr int kRedBlocks = 512;

}  // namespace pat
