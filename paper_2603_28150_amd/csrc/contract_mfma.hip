// Per-frequency contraction on the matrix cores, for 16-bit kernel libraries
// and for batches of objects (step (ii) of Sec. 3.2).
//
// For one symmetry class c the members' spectra of B objects form the columns
// of a real matrix (re and im parts of every (member, object) pair), and the
// contraction is a real GEMM against the class slab:
//     A  :  out[col][n] = sum_l X[col][l]  H^[l][n]
//     A^T:  out[col][l] = sum_n R[col][n]  H^[l][n]
// i.e. out (cols x N) = X (cols x K) * S (K x N) with S the slab seen along the
// output index.  The slab is the B operand of v_mfma_f32_32x32x16_bf16 and is
// stored pre-tiled in the exact lane order the instruction consumes (1 KB per
// 32 x 16 fragment), so every wave load is one contiguous, fully coalesced
// kilobyte streamed once from HBM.  The spectra are the A operand: staged in
// LDS as bfloat16 hi + lo pairs (x = hi + lo to 2^-17 relative), so the only
// significant error left is the library's own 16-bit rounding.  A float16
// library value is split exactly into two bfloat16 values on the fly (an
// 11-bit significand is the sum of an 8-bit and a 3-bit one), so both 16-bit
// formats run on the bf16 MFMA with float32 accumulation and no overflow risk.
// Output columns come out of the accumulators as (re, im) pairs along the
// slab's output index: 256-byte contiguous stores.
#include "pat_internal.hpp"

namespace pat {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;      // waves per workgroup
constexpr int kKC = 8;         // k-steps (of 16) per staged chunk
constexpr int kMT = 4;         // most 32-column tiles per launch group (64 pairs)
constexpr int kTerms = 2;      // hi + lo split of the spectra

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

union Frag {
  u32x4 u;
  bf16x8 b;
  unsigned short s[8];
};

// float16 fragment -> two bfloat16 fragments whose sum is exact
__device__ __forceinline__ void split_f16(const Frag& in, Frag& hi, Frag& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    _Float16 h;
    __builtin_memcpy(&h, &in.s[e], 2);
    const float f = (float)h;
    const unsigned short a = bf16_rne(f);
    hi.s[e] = a;
    lo.s[e] = bf16_rne(f - bf16_to_f(a));
  }
}

// Stages the spectra of k-chunk ch (the A operand) into LDS, split hi + lo.
// Work item = (pair, 8 consecutive k): 8 complex values in, four 16-byte
// fragment units out (re and im columns, hi and lo terms).
template <int MT>
__device__ __forceinline__ void stage_chunk(const MfmaArgs& a, u32x4* lds, int c, int p0, int gp,
                                            int ch, int tid) {
  const int k0 = ch * kKC * 16;
  constexpr int items = MT * 16 * kKC * 2;  // pairs x k-octets
  for (int it = tid; it < items; it += kWaves * 64) {
    const int pl = it / (kKC * 2), ko = it % (kKC * 2);
    float2 v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = make_float2(0.f, 0.f);
    if (pl < gp) {
      const int pair = p0 + pl;
      const int g = pair / a.B, b = pair % a.B;
      if (a.members[c * a.G + g] >= 0) {
        const float2* src = a.in + (size_t)(c * a.G + g) * a.in_rs + (size_t)b * a.K;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + ko * 8 + e;
          if (k < a.K) {
            v[e] = src[k];
            if (a.in_scale) {
              const float sc = a.in_scale[k];
              v[e].x *= sc;
              v[e].y *= sc;
            }
          }
        }
      }
    }
    const int ks = ko >> 1, half = ko & 1;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      const int col = 2 * pl + part;
      const int mt = col >> 5, r = col & 31;
      Frag hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = part ? v[e].y : v[e].x;
        hi.s[e] = bf16_rne(x);
        lo.s[e] = bf16_rne(x - bf16_to_f(hi.s[e]));
      }
      const int unit = (ks * MT + mt) * 64 + r + 32 * half;
      lds[unit] = hi.u;
      lds[kKC * MT * 64 + unit] = lo.u;
    }
  }
}

template <bool F16, int MT>
__global__ __launch_bounds__(512, MT == 4 ? 2 : 4) void k_contract_mfma(MfmaArgs a) {
  extern __shared__ u32x4 lds[];  // [term][ks][mt][lane] 16-byte units
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int c = blockIdx.x, cg = blockIdx.y;  // c: work item
  const int npairs = a.G * a.B;
  const int p0 = cg * (kMT * 16);
  const int gp = min(MT * 16, npairs - p0);  // pairs in this launch group
  // waves -> (N-tile, k-part): a wave owns one N-tile per pass; when there
  // are fewer N-tiles than waves, waves sharing a tile split its k-steps
  int kparts = 1;
  while (kparts < kWaves && a.ntiles * kparts * 2 <= kWaves) kparts *= 2;
  const int kpart = w % kparts;
  const int wslot = w / kparts;
  const int wstride = kWaves / kparts;
  const int nchunks = (a.ksteps + kKC - 1) / kKC;
  const u32x4* slab = reinterpret_cast<const u32x4*>(a.frag) + (size_t)a.item_slab[c] * a.ntiles * a.ksteps * 64;
  bool staged = false;  // LDS holds chunk 0 (kept only when there is one chunk)

  for (int tile0 = 0; tile0 < a.ntiles; tile0 += wstride) {
    const int tile = tile0 + wslot;
    const bool has = tile < a.ntiles;
    f32x16 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x16(0.f);

    for (int ch = 0; ch < nchunks; ++ch) {
      const int nks = min(kKC, a.ksteps - ch * kKC);
      if (!(staged && nchunks == 1)) {
        __syncthreads();
        stage_chunk<MT>(a, lds, c, p0, gp, ch, tid);
        __syncthreads();
        staged = true;
      }
      // this wave's slab fragments of the chunk, all loads issued up front
      Frag fr[kKC];
#pragma unroll
      for (int s = 0; s < kKC; ++s) {
        const int ks = kpart + s * kparts;
        if (has && s * kparts < kKC && ks < nks)
          fr[s].u = __builtin_nontemporal_load(slab + ((size_t)tile * a.ksteps + ch * kKC + ks) * 64 + lane);
        else
          fr[s].u = u32x4(0);
      }
      if (has) {
#pragma unroll
        for (int s = 0; s < kKC; ++s) {
          const int ks = kpart + s * kparts;
          if (s * kparts >= kKC || ks >= nks) break;
          if constexpr (!F16) {
#pragma unroll
            for (int m = 0; m < MT; ++m) {
              Frag ah, al;
              ah.u = lds[(ks * MT + m) * 64 + lane];
              al.u = lds[(kKC * MT + ks * MT + m) * 64 + lane];
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, fr[s].b, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, fr[s].b, acc[m], 0, 0, 0);
            }
          } else {
            Frag hh, hl;
            split_f16(fr[s], hh, hl);
#pragma unroll
            for (int m = 0; m < MT; ++m) {
              Frag ah, al;
              ah.u = lds[(ks * MT + m) * 64 + lane];
              al.u = lds[(kKC * MT + ks * MT + m) * 64 + lane];
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, hh.b, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, hh.b, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, hl.b, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, hl.b, acc[m], 0, 0, 0);
            }
          }
        }
      }
    }

    // add the k-parts of waves sharing an N-tile (one column tile at a time)
    if (kparts > 1) {
      float* red = reinterpret_cast<float*>(lds);
      staged = false;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v) red[(w * 16 + v) * 64 + lane] = acc[m][v];
        __syncthreads();
        if (kpart == 0) {
          for (int p = 1; p < kparts; ++p)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[m][v] += red[((w + p) * 16 + v) * 64 + lane];
        }
      }
    }

    // store (re, im) pairs along the output index
    const int row = tile * 32 + (lane & 31);
    if (has && kpart == 0 && row < a.N) {
      const float sc = a.out_scale ? a.out_scale[row] : 1.f;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);  // even: the re part
          const int pl = (m * 32 + i) >> 1;
          if (pl >= gp) continue;
          const int pair = p0 + pl;
          const int g = pair / a.B, b = pair % a.B;
          if (a.members[c * a.G + g] < 0) continue;
          // streamed out: not read again by this kernel
          typedef float v2f __attribute__((ext_vector_type(2)));
          __builtin_nontemporal_store(v2f{acc[m][v] * sc, acc[m][v + 1] * sc},
                                      reinterpret_cast<v2f*>(a.out + (size_t)(c * a.G + g) * a.out_rs +
                                                             (size_t)b * a.N + row));
        }
      }
    }
  }
}

template <int MT>
static void launch_mt(const MfmaArgs& a, int hdtype, dim3 grid, hipStream_t st) {
  const size_t lds = (size_t)kTerms * kKC * MT * 64 * 16;
  const size_t red = (size_t)kWaves * 16 * 64 * 4;  // k-part reduction buffer
  const size_t bytes = lds > red ? lds : red;
  if (hdtype == PAT_H_F16)
    k_contract_mfma<true, MT><<<grid, kWaves * 64, bytes, st>>>(a);
  else
    k_contract_mfma<false, MT><<<grid, kWaves * 64, bytes, st>>>(a);
}

pat_status contract_mfma(const MfmaArgs& a, int hdtype, hipStream_t st) {
  if (a.nitem == 0 || a.B == 0) return PAT_OK;
  const int npairs = a.G * a.B;
  const int groups = (npairs + kMT * 16 - 1) / (kMT * 16);
  const int cols = 2 * (groups > 1 ? kMT * 16 : npairs);  // columns of the widest group
  dim3 grid(a.nitem, groups);
  if (cols <= 32)
    launch_mt<1>(a, hdtype, grid, st);
  else if (cols <= 64)
    launch_mt<2>(a, hdtype, grid, st);
  else
    launch_mt<4>(a, hdtype, grid, st);
  PAT_LAUNCHED("contraction (MFMA)");
  return PAT_OK;
}

}  // namespace pat
