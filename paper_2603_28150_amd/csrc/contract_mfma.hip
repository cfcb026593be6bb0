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
constexpr int kMT = 4;         // 32-column tiles per launch group (64 pairs)
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

// Stages the spectra of k-chunk ch (A operand), split hi + lo, into LDS.
__device__ __forceinline__ void stage_chunk(const MfmaArgs& a, unsigned short* lds16, int c,
                                            int p0, int gp, int ch, int tid) {
  const int k0 = ch * kKC * 16;
  for (int idx = tid; idx < kMT * 16 * kKC * 16; idx += kWaves * 64) {
    const int pl = idx / (kKC * 16), kk = idx % (kKC * 16);
    const int k = k0 + kk;
    float2 v = make_float2(0.f, 0.f);
    if (pl < gp && k < a.K) {
      const int pair = p0 + pl;
      const int g = pair / a.B, b = pair % a.B;
      if (a.members[c * a.G + g] >= 0) {
        v = a.in[(size_t)(c * a.G + g) * a.in_rs + (size_t)b * a.K + k];
        if (a.in_scale) {
          const float s = a.in_scale[k];
          v.x *= s;
          v.y *= s;
        }
      }
    }
    const int ks = kk >> 4, half = (kk >> 3) & 1, e = kk & 7;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      const int col = 2 * pl + part;
      const int mt = col >> 5, r = col & 31;
      const float x = part ? v.y : v.x;
      const unsigned short hi = bf16_rne(x);
      const unsigned short lo = bf16_rne(x - bf16_to_f(hi));
      const int unit = (ks * kMT + mt) * 64 + r + 32 * half;
      lds16[(size_t)unit * 8 + e] = hi;
      lds16[((size_t)kKC * kMT * 64 + unit) * 8 + e] = lo;
    }
  }
}

template <bool F16>
__global__ __launch_bounds__(512) void k_contract_mfma(MfmaArgs a) {
  extern __shared__ u32x4 lds[];  // [term][ks][mt][lane] 16-byte units
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int c = blockIdx.x, cg = blockIdx.y;
  const int npairs = a.G * a.B;
  const int p0 = cg * (kMT * 16);
  const int gp = min(kMT * 16, npairs - p0);  // pairs in this launch group
  const int MT = (2 * gp + 31) / 32;
  // waves -> (N-tile, k-part): a wave owns one N-tile per pass; when there
  // are fewer N-tiles than waves, waves sharing a tile split its k-steps
  int kparts = 1;
  while (kparts < kWaves && a.ntiles * kparts * 2 <= kWaves) kparts *= 2;
  const int kpart = w % kparts;
  const int wslot = w / kparts;
  const int wstride = kWaves / kparts;
  const int nchunks = (a.ksteps + kKC - 1) / kKC;
  unsigned short* lds16 = reinterpret_cast<unsigned short*>(lds);
  const u32x4* slab = reinterpret_cast<const u32x4*>(a.frag) + (size_t)c * a.ntiles * a.ksteps * 64;
  bool staged = false;  // LDS holds chunk 0 (only kept when there is one chunk)

  for (int tile0 = 0; tile0 < a.ntiles; tile0 += wstride) {
    const int tile = tile0 + wslot;
    const bool has = wslot < wstride && tile < a.ntiles;
    f32x16 acc[kMT];
#pragma unroll
    for (int m = 0; m < kMT; ++m) acc[m] = f32x16(0.f);

    for (int ch = 0; ch < nchunks; ++ch) {
      if (!(staged && nchunks == 1)) {
        __syncthreads();
        stage_chunk(a, lds16, c, p0, gp, ch, tid);
        __syncthreads();
        staged = true;
      }
      const int nks = min(kKC, a.ksteps - ch * kKC);
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
            for (int m = 0; m < kMT; ++m) {
              if (m >= MT) continue;
              Frag ah, al;
              ah.u = lds[(ks * kMT + m) * 64 + lane];
              al.u = lds[(kKC * kMT + ks * kMT + m) * 64 + lane];
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, fr[s].b, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, fr[s].b, acc[m], 0, 0, 0);
            }
          } else {
            Frag hh, hl;
            split_f16(fr[s], hh, hl);
#pragma unroll
            for (int m = 0; m < kMT; ++m) {
              if (m >= MT) continue;
              Frag ah, al;
              ah.u = lds[(ks * kMT + m) * 64 + lane];
              al.u = lds[(kKC * kMT + ks * kMT + m) * 64 + lane];
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
      for (int m = 0; m < kMT; ++m) {
        if (m >= MT) break;
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
      for (int m = 0; m < kMT; ++m) {
        if (m >= MT) continue;
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);  // even: the re part
          const int pl = (m * 32 + i) >> 1;
          if (pl >= gp) continue;
          const int pair = p0 + pl;
          const int g = pair / a.B, b = pair % a.B;
          if (a.members[c * a.G + g] < 0) continue;
          a.out[(size_t)(c * a.G + g) * a.out_rs + (size_t)b * a.N + row] =
              make_float2(acc[m][v] * sc, acc[m][v + 1] * sc);
        }
      }
    }
  }
}

pat_status contract_mfma(const MfmaArgs& a, int hdtype, hipStream_t st) {
  if (a.nclass == 0 || a.B == 0) return PAT_OK;
  const int groups = (a.G * a.B + kMT * 16 - 1) / (kMT * 16);
  const size_t lds = (size_t)kTerms * kKC * kMT * 64 * 16;  // 64 KB; >= the k-part buffer
  dim3 grid(a.nclass, groups);
  if (hdtype == PAT_H_F16)
    k_contract_mfma<true><<<grid, kWaves * 64, lds, st>>>(a);
  else
    k_contract_mfma<false><<<grid, kWaves * 64, lds, st>>>(a);
  PAT_LAUNCHED("contraction (MFMA)");
  return PAT_OK;
}

}  // namespace pat
