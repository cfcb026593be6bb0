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
//
// Float32 libraries (batches of objects) run on v_mfma_f32_32x32x16_f16
// instead.  The B operand comes from the stored rows that run along k (the
// [n][l] rows for A, the [l][n] rows for A^T): each lane reads 8 consecutive
// floats, scales them by its row's power of two (computed with the library,
// so that the row's largest magnitude lies in [2^14, 2^15)) and splits each
// into two float16 terms, h = h1 + h2 to 2^-22 relative.  The spectra are
// staged as float16 hi + lo pairs in the same way, scaled by a power of two
// per (member, object) pair: the smallest exponent over the k-chunks staged
// so far, so no value overflows; when a later chunk lowers it, the pair's
// accumulated sums are scaled down by the same power of two first (exact).
// Three MFMAs per step: hi h1, hi h2 and lo h1; the product left out (lo
// h2) is below 2^-22 of the step's largest.  Both scales come off in the
// epilogue (exact powers of two).
//
// Workgroups: the (item, column group) units are dealt to the XCDs in eight
// contiguous ranges, so the column groups of one item, and the items a large
// class is split into, run on the same XCD at about the same time and its L2
// serves the slab to all of them.
#include "pat_internal.hpp"

namespace pat {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;      // waves per workgroup
constexpr int kKC = 8;         // k-steps (of 16) per staged chunk
constexpr int kTerms = 2;      // hi + lo split of the spectra
constexpr int kMinBlocks = 3;  // workgroups per CU the registers are sized for (2 at MT = 4)

// two floats -> two bfloat16 (round to nearest even) packed low, high
__device__ __forceinline__ unsigned pk_bf16(float a, float b) {
  const bf16x2 h = __builtin_convertvector((f32x2){a, b}, bf16x2);
  unsigned u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}
__device__ __forceinline__ float lo_f(unsigned u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float hi_f(unsigned u) { return __uint_as_float(u & 0xffff0000u); }

// (a, b) -> hi + lo bfloat16 pairs: a = hi.a + lo.a to 2^-17 relative
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
  hi = pk_bf16(a, b);
  lo = pk_bf16(a - lo_f(hi), b - hi_f(hi));
}

union Frag {
  u32x4 u;
  bf16x8 b;
  f16x8 h;
  unsigned short s[8];
};

// (a, b) -> hi + lo float16 pairs (round to nearest even): a = hi.a + lo.a
// to 2^-22 relative while |a| < 2^15 and hi.a is a normal number
__device__ __forceinline__ void split2_f16(float a, float b, unsigned& hi, unsigned& lo) {
  const f32x2 x = {a, b};
  const f16x2 h = __builtin_convertvector(x, f16x2);
  const f32x2 hf = __builtin_convertvector(h, f32x2);
  const f16x2 l = __builtin_convertvector((f32x2){x[0] - hf[0], x[1] - hf[1]}, f16x2);
  __builtin_memcpy(&hi, &h, 4);
  __builtin_memcpy(&lo, &l, 4);
}

enum { kSrcBf16 = 0, kSrcF16 = 1, kSrcF32 = 2 };

// 8 float32 values (two 16-byte units) times 2^e -> two float16 fragments,
// h1 + h2 = h 2^e to 2^-22 relative
__device__ __forceinline__ void split_f32(const u32x4 (&raw)[2], int e, Frag& b1, Frag& b2) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float x0 = ldexpf(__uint_as_float(raw[j >> 1][2 * (j & 1)]), e);
    const float x1 = ldexpf(__uint_as_float(raw[j >> 1][2 * (j & 1) + 1]), e);
    unsigned h, l;
    split2_f16(x0, x1, h, l);
    b1.u[j] = h;
    b2.u[j] = l;
  }
}

// float16 fragment -> two bfloat16 fragments whose sum is exact
__device__ __forceinline__ void split_f16(const Frag& in, Frag& hi, Frag& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    _Float16 h0, h1;
    __builtin_memcpy(&h0, &in.s[2 * j], 2);
    __builtin_memcpy(&h1, &in.s[2 * j + 1], 2);
    unsigned a, b;
    split2((float)h0, (float)h1, a, b);
    hi.u[j] = a;
    lo.u[j] = b;
  }
}

// Workgroup barrier that orders LDS accesses only: waves share nothing
// through global memory here, so a barrier need not wait for the wave's
// outstanding global loads and stores (a full __syncthreads() would).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS position, within its 64-unit fragment row, of the A-operand unit that
// lane `idx` of k-step ks reads: the unit index XOR (2 ks + idx/32), a value
// below 16, so the bit that selects the k half is kept and each 16-lane
// quarter of a read still covers all 16 four-bank groups.  The staging loop
// below writes, from 16 consecutive lanes, the units of one column for every
// (k-step, k half); unswizzled those sit 512 bytes apart, all in one bank
// group (a 16-way conflict); swizzled they fall in 16 different groups.
__device__ __forceinline__ int a_unit(int ks, int idx) { return idx ^ ((2 * ks + (idx >> 5)) & 15); }

// Stages the spectra of k-chunk ch (the A operand) into LDS, split hi + lo.
// Work item = (pair, 8 consecutive k): 8 complex values in, four 16-byte
// fragment units out (re and im columns, hi and lo terms).  Consecutive lanes
// take consecutive k-octets of one pair, so the global loads of 16 lanes are
// one contiguous kilobyte of a spectrum row.  A thread's items go in rounds
// of two, every load of a round (and of its per-depth scales) issued before
// the first is used: one memory latency per chunk up to 32-pair groups, two
// for 64-pair groups (whose four items would not fit the registers at once).
// in_off[pl]: offset of pair pl's spectrum row in a.in (float2 units), -1
// for a pair outside the group or in an empty member slot (staged as zeros).
// 16-bit libraries: bfloat16 terms, the spectra times the library's
// per-depth scales when it has them.  Float32 libraries: float16 terms of
// the spectra times 2^e, e per pair the running minimum over the chunks of
// the tile (reset by `first`) of the exponent that takes the chunk's largest
// magnitude of the pair into [2^14, 2^15); etab[pair] receives e and
// etab[MT*16 + pair] the change of e from the last chunk (0 or negative).
template <int MT, int SRC>
__device__ __forceinline__ void stage_chunk(const MfmaArgs& a, u32x4* lds, const long long* in_off, int ch,
                                            int tid, int* etab, bool first) {
  constexpr bool SCALED = SRC != kSrcF32;
  const int k0 = ch * kKC * 16;
  constexpr int items = MT * 16 * kKC * 2;  // pairs x k-octets
  constexpr int per_all = items / (kWaves * 64);  // items per thread
  static_assert(items % (kWaves * 64) == 0, "whole items per thread");
  constexpr int per = per_all < 2 ? per_all : 2;  // items per round trip
#pragma unroll
  for (int r0 = 0; r0 < per_all; r0 += per) {
    float4 q[per][4];  // 8 complex values per item
    float4 sq[SCALED ? per : 1][2];  // their 8 scales
#pragma unroll
    for (int r = 0; r < per; ++r) {
      const int it = tid + (r0 + r) * kWaves * 64;
      const int pl = it / (kKC * 2), ko = it % (kKC * 2);
      const int kb = k0 + ko * 8;
#pragma unroll
      for (int e = 0; e < 4; ++e) q[r][e] = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (SCALED) sq[r][0] = sq[r][1] = make_float4(1.f, 1.f, 1.f, 1.f);
      const long long off = in_off[pl];
      if (off < 0) continue;
      const float2* src = a.in + off;
      if (kb + 8 <= a.K) {  // 64 aligned bytes
        const float4* s4 = reinterpret_cast<const float4*>(src + kb);
#pragma unroll
        for (int e = 0; e < 4; ++e) q[r][e] = s4[e];
        if constexpr (SCALED) {
          if (a.in_scale) {
            const float4* c4 = reinterpret_cast<const float4*>(a.in_scale + kb);
            sq[r][0] = c4[0];
            sq[r][1] = c4[1];
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (kb + e < a.K) {
            const float2 v = src[kb + e];
            if (e & 1) {
              q[r][e >> 1].z = v.x;
              q[r][e >> 1].w = v.y;
            } else {
              q[r][e >> 1].x = v.x;
              q[r][e >> 1].y = v.y;
            }
            if constexpr (SCALED) sq[r][e >> 2][e & 3] = a.in_scale ? a.in_scale[kb + e] : 1.f;
          }
      }
    }
#pragma unroll
    for (int r = 0; r < per; ++r) {
      const int it = tid + (r0 + r) * kWaves * 64;
      const int pl = it / (kKC * 2), ko = it % (kKC * 2);
      float2 v[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[2 * e] = make_float2(q[r][e].x, q[r][e].y);
        v[2 * e + 1] = make_float2(q[r][e].z, q[r][e].w);
      }
      if (SCALED && a.in_scale) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float sc = sq[SCALED ? r : 0][e >> 2][e & 3];
          v[e].x *= sc;
          v[e].y *= sc;
        }
      }
      if constexpr (SRC == kSrcF32) {
        // the pair's largest magnitude in this chunk: its 16 k-octets are
        // the items of 16 consecutive lanes (one round, aligned to 16)
        float mx = 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fmaxf(fabsf(v[e].x), fabsf(v[e].y)));
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        int E;
        (void)frexpf(mx, &E);  // mx < 2^E (E = 0 for zero)
        const int eo = first ? 15 - E : etab[pl];
        const int en = min(eo, 15 - E);
        if ((tid & 15) == 0) {
          etab[pl] = en;
          etab[MT * 16 + pl] = en - eo;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          v[e].x = ldexpf(v[e].x, en);
          v[e].y = ldexpf(v[e].y, en);
        }
      }
      const int ks = ko >> 1, half = ko & 1;
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const int col = 2 * pl + part;
        const int mt = col >> 5, rr = col & 31;
        Frag hi, lo;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          unsigned h, l;
          const float x0 = part ? v[2 * j].y : v[2 * j].x;
          const float x1 = part ? v[2 * j + 1].y : v[2 * j + 1].x;
          if constexpr (SRC == kSrcF32)
            split2_f16(x0, x1, h, l);
          else
            split2(x0, x1, h, l);
          hi.u[j] = h;
          lo.u[j] = l;
        }
        const int unit = (ks * MT + mt) * 64 + a_unit(ks, rr + 32 * half);
        lds[unit] = hi.u;
        lds[kKC * MT * 64 + unit] = lo.u;
      }
    }
  }  // rounds of items
}

// LDS: the staged chunk (or the k-part reduction buffer, whichever is
// larger)
template <int MT>
constexpr size_t table_offset() {
  constexpr size_t units = (size_t)kTerms * kKC * MT * 64 * 16;
  constexpr size_t red = (size_t)kWaves * 16 * 64 * 4;
  return units > red ? units : red;
}
// then the pair offset tables (input rows, output rows: 64-bit, -1 for no
// pair), then for float32 libraries the exponent table of stage_chunk
template <int MT>
constexpr size_t offs_bytes() { return (size_t)2 * MT * 16 * sizeof(long long); }
template <int MT>
constexpr size_t etab_bytes() { return (size_t)2 * MT * 16 * sizeof(int); }

// ALIGNED: K a multiple of 16 and N of 32 (float32 rows read without bounds
// branches)
template <int SRC, int MT, bool ALIGNED>
__global__ __launch_bounds__(kWaves * 64, MT >= 4 ? 2 : kMinBlocks) void k_contract_mfma(MfmaArgs a, int groups) {
  extern __shared__ u32x4 lds[];  // [term][ks][mt][lane] 16-byte units
  long long* offs = reinterpret_cast<long long*>(reinterpret_cast<char*>(lds) + table_offset<MT>());
  int* etab = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + table_offset<MT>() + offs_bytes<MT>());
  constexpr int KB = SRC == kSrcF32 ? kKC / 4 : kKC / 2;  // k-steps per batch of B loads
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  int c, cg;  // work item, column group
  {
    // units (item, column group) in item order, cut into eight contiguous
    // ranges, one per XCD (workgroups go to the XCDs round-robin by index):
    // the groups of an item and the items a large class is split into run
    // on one XCD together and share the slab through its L2
    const int units = a.nitem * groups;
    const int per_xcd = (units + 7) >> 3;
    const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (u >= units) return;  // whole workgroup: padding of the grid
    c = u / groups;
    cg = u - c * groups;
  }
  // filled member slots of the item, read once here: the loops below read
  // the LDS offset tables instead of the member table (a global load after
  // a store waits for that store on the in-order counter; LDS reads do not)
  unsigned gmask = 0;
#pragma unroll
  for (int g = 0; g < 8; ++g)
    if (g < a.G && a.members[c * a.G + g] >= 0) gmask |= 1u << g;
  const int npairs = a.G * a.B;
  const int p0 = cg * (MT * 16);
  const int gp = min(MT * 16, npairs - p0);  // pairs in this launch group
  // row offsets of the group's pairs (one division per pair and workgroup,
  // not one per load and store); read after the first staging barrier
  if (tid < MT * 16) {
    long long oi = -1, oo = -1;
    if (tid < gp) {
      const int pair = p0 + tid;
      const int g = pair / a.B, b = pair % a.B;
      if ((gmask >> g) & 1u) {
        oi = (long long)(c * a.G + g) * a.in_rs + (long long)b * a.K;
        oo = (long long)(c * a.G + g) * a.out_rs + (long long)b * a.N;
      }
    }
    offs[tid] = oi;
    offs[MT * 16 + tid] = oo;
  }
  // waves -> (N-tile, k-part): a wave owns one N-tile per pass; when there
  // are fewer N-tiles than waves, waves sharing a tile split its k-steps
  int kparts = 1;
  while (kparts < kWaves && a.ntiles * kparts * 2 <= kWaves) kparts *= 2;
  const int kpart = w % kparts;
  const int wslot = w / kparts;
  const int wstride = kWaves / kparts;
  const int nchunks = (a.ksteps + kKC - 1) / kKC;
  const u32x4* slab = SRC == kSrcF32 ? nullptr
                                      : reinterpret_cast<const u32x4*>(a.frag) +
                                            (size_t)a.item_slab[c] * a.ntiles * a.ksteps * 64;
  const float* krow = SRC == kSrcF32 ? a.krows + (size_t)a.item_slab[c] * a.k_slab : nullptr;
  bool staged = false;  // LDS holds chunk 0 (kept only when there is one chunk)
  int lsx = 0;  // float32: exponent of this lane's library row in the current tile

  // The B operands of one batch of KB k-steps (16-bit fragments, or float32
  // rows: 8 floats per lane and k-step).
  struct BBatch {
    Frag fr[KB];
    u32x4 raw[KB][2];
  };
  // Issues the loads of batch (tile, chunk ch, first k-step s0) of this wave.
  // K-steps out of range (and every k-step of a tile past the end) get zeros
  // (16-bit tiles, unaligned rows) or row 0 (aligned rows); mma_batch skips
  // them either way.
  auto load_batch = [&](BBatch& o, int tile, int ch, int s0) {
    const bool has = tile < a.ntiles;
    const int nks = min(kKC, a.ksteps - ch * kKC);
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      const int ks = kpart + (s0 + s) * kparts;
      const bool ok = has && (s0 + s) * kparts < kKC && ks < nks;
      if constexpr (SRC != kSrcF32) {
        // plain loads: the other column groups of the item (and the other
        // items of a split class) read the same fragments next, from the
        // XCD's L2.  (Loaded under a branch: branch-free, the compiler
        // moves the last load of a batch behind the first products, and the
        // wave then waits twice per batch.)
        if (ok)
          o.fr[s].u = slab[((size_t)tile * a.ksteps + ch * kKC + ks) * 64 + lane];
        else
          o.fr[s].u = u32x4(0);
      } else if constexpr (ALIGNED) {
        // K a multiple of 16 and N of 32: every in-range row segment is a
        // whole 32 bytes; out of range, row 0 is read and never used (no
        // branch hides a load from the wait counter, and no select forces
        // a wait right after the load)
        const int n = tile * 32 + (lane & 31);
        const int k0 = (ch * kKC + ks) * 16 + 8 * (lane >> 5);
        const u32x4* src = reinterpret_cast<const u32x4*>(krow + (ok ? (size_t)n * a.k_srow + k0 : (size_t)0));
        o.raw[s][0] = src[0];
        o.raw[s][1] = src[1];
      } else {
        const int n = tile * 32 + (lane & 31);
        const int k0 = (ch * kKC + ks) * 16 + 8 * (lane >> 5);
        o.raw[s][0] = u32x4(0);
        o.raw[s][1] = u32x4(0);
        if (ok && n < a.N) {
          const float* src = krow + (size_t)n * a.k_srow + k0;
          if (k0 + 8 <= a.K) {
            // plain loads: the 128-byte lines serve two k-steps
            o.raw[s][0] = *reinterpret_cast<const u32x4*>(src);
            o.raw[s][1] = *(reinterpret_cast<const u32x4*>(src) + 1);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (k0 + e < a.K) o.raw[s][e >> 2][e & 3] = __float_as_uint(src[e]);
          }
        }
      }
    }
  };
  // The products of one loaded batch with the staged spectra.
  auto mma_batch = [&](const BBatch& o, int ch, int s0, f32x16 (&acc)[MT]) {
    const int nks = min(kKC, a.ksteps - ch * kKC);
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      const int ks = kpart + (s0 + s) * kparts;
      if ((s0 + s) * kparts >= kKC || ks >= nks) break;
      if constexpr (SRC == kSrcBf16) {
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          Frag ah, al;
          ah.u = lds[(ks * MT + m) * 64 + a_unit(ks, lane)];
          al.u = lds[(kKC * MT + ks * MT + m) * 64 + a_unit(ks, lane)];
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, o.fr[s].b, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, o.fr[s].b, acc[m], 0, 0, 0);
        }
      } else if constexpr (SRC == kSrcF16) {
        Frag hh, hl;
        split_f16(o.fr[s], hh, hl);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          Frag ah, al;
          ah.u = lds[(ks * MT + m) * 64 + a_unit(ks, lane)];
          al.u = lds[(kKC * MT + ks * MT + m) * 64 + a_unit(ks, lane)];
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, hh.b, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, hh.b, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah.b, hl.b, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al.b, hl.b, acc[m], 0, 0, 0);
        }
      } else {
        Frag b1, b2;
        split_f32(o.raw[s], lsx, b1, b2);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          Frag ah, al;
          ah.u = lds[(ks * MT + m) * 64 + a_unit(ks, lane)];
          al.u = lds[(kKC * MT + ks * MT + m) * 64 + a_unit(ks, lane)];
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah.h, b1.h, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah.h, b2.h, acc[m], 0, 0, 0);
          acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al.h, b1.h, acc[m], 0, 0, 0);
        }
      }
    }
  };

  // float32 rows: two batches in flight per wave, the loads of the next
  // batch (in the next chunk, or the next tile at the end of one) issued
  // before the products of the current one, and a tile's stores after the
  // loads of the next tile's first batch, so that waiting for those loads
  // does not wait for the stores.  16-bit tiles: one batch at a time (the
  // second buffer, with the depth scales of the staging, would spill).
  constexpr bool kPipe = SRC == kSrcF32;
  static_assert(kKC % (2 * KB) == 0, "an even number of batches per chunk");
  BBatch bA, bB;
  if constexpr (kPipe) load_batch(bA, wslot, 0, 0);
  for (int tile0 = 0; tile0 < a.ntiles; tile0 += wstride) {
    const int tile = tile0 + wslot;
    const bool has = tile < a.ntiles;
    // output row of this lane and its scale, read before the tile's loads
    const int row = tile * 32 + (lane & 31);
    const float sc = SRC != kSrcF32 && a.out_scale && has && row < a.N ? a.out_scale[row] : 1.f;
    if constexpr (SRC == kSrcF32) lsx = has && row < a.N ? a.kexp[(size_t)a.item_slab[c] * a.N + row] : 0;
    f32x16 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = f32x16(0.f);

    for (int ch = 0; ch < nchunks; ++ch) {
      if (!(staged && nchunks == 1)) {
        lds_barrier();
        stage_chunk<MT, SRC>(a, lds, offs, ch, tid, etab, ch == 0);
        lds_barrier();
        staged = true;
      }
      if (SRC == kSrcF32 && ch > 0) {
        // a pair whose exponent this chunk lowered: its sums so far times
        // the same power of two (accumulator row i of tile m is column
        // 32 m + i, pair 16 m + i/2; lane half h holds rows 8 q + 4 h + 0..3)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int2 d = *reinterpret_cast<const int2*>(etab + MT * 16 + m * 16 + 4 * q + 2 * (lane >> 5));
            acc[m][4 * q] = ldexpf(acc[m][4 * q], d.x);
            acc[m][4 * q + 1] = ldexpf(acc[m][4 * q + 1], d.x);
            acc[m][4 * q + 2] = ldexpf(acc[m][4 * q + 2], d.y);
            acc[m][4 * q + 3] = ldexpf(acc[m][4 * q + 3], d.y);
          }
      }
      if constexpr (!kPipe) {
#pragma unroll 1
        for (int s0 = 0; s0 < kKC; s0 += KB) {
          load_batch(bA, tile, ch, s0);
          if (has) mma_batch(bA, ch, s0, acc);
        }
        continue;
      }
#pragma unroll 1
      for (int s0 = 0; s0 < kKC; s0 += 2 * KB) {
        // bA holds batch s0
        load_batch(bB, tile, ch, s0 + KB);
        if (has) mma_batch(bA, ch, s0, acc);
        int nt = tile, nc = ch, ns = s0 + 2 * KB;
        if (ns >= kKC) {
          ns = 0;
          if (++nc >= nchunks) {
            nc = 0;
            nt = tile + wstride;
          }
        }
        load_batch(bA, nt, nc, ns);
        if (has) mma_batch(bB, ch, s0 + KB, acc);
      }
    }

    // add the k-parts of waves sharing an N-tile (one column tile at a time)
    if (kparts > 1) {
      float* red = reinterpret_cast<float*>(lds);
      staged = false;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        lds_barrier();
#pragma unroll
        for (int v = 0; v < 16; ++v) red[(w * 16 + v) * 64 + lane] = acc[m][v];
        lds_barrier();
        if (kpart == 0) {
          for (int p = 1; p < kparts; ++p)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[m][v] += red[((w + p) * 16 + v) * 64 + lane];
        }
      }
    }

    // per-row output scale (1 when there is none; float32: 2^-(pair's
    // exponent + library row's exponent)), applied here on straight-line
    // code (the empty asm keeps the compiler from sinking the products into
    // the conditional stores below, where each store would first wait for
    // the scale's load and so for every earlier store)
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if constexpr (SRC == kSrcF32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int2 e = *reinterpret_cast<const int2*>(etab + m * 16 + 4 * q + 2 * (lane >> 5));
          acc[m][4 * q] = ldexpf(acc[m][4 * q], -(e.x + lsx));
          acc[m][4 * q + 1] = ldexpf(acc[m][4 * q + 1], -(e.x + lsx));
          acc[m][4 * q + 2] = ldexpf(acc[m][4 * q + 2], -(e.y + lsx));
          acc[m][4 * q + 3] = ldexpf(acc[m][4 * q + 3], -(e.y + lsx));
        }
      } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[m][v] *= sc;
      }
      asm volatile("" : "+v"(acc[m]));
    }

    // store (re, im) pairs along the output index
    // (accumulator rows 8 q + 4 h + {0, 1} and {2, 3} of tile m: the re
    // and im parts of pairs 16 m + 4 q + 2 h and the one after it)
    if (has && kpart == 0 && row < a.N) {
      typedef float v2f __attribute__((ext_vector_type(2)));
      typedef long long i64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        i64x2 o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          o[q] = *reinterpret_cast<const i64x2*>(offs + MT * 16 + m * 16 + 4 * q + 2 * (lane >> 5));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // streamed out: not read again by this kernel
          if (o[q][0] >= 0)
            __builtin_nontemporal_store(v2f{acc[m][4 * q], acc[m][4 * q + 1]},
                                        reinterpret_cast<v2f*>(a.out + o[q][0] + row));
          if (o[q][1] >= 0)
            __builtin_nontemporal_store(v2f{acc[m][4 * q + 2], acc[m][4 * q + 3]},
                                        reinterpret_cast<v2f*>(a.out + o[q][1] + row));
        }
      }
    }
  }
}

template <int MT>
static void launch_mt(const MfmaArgs& a, int src, int groups, hipStream_t st) {
  const size_t bytes = table_offset<MT>() + offs_bytes<MT>() + (src == kSrcF32 ? etab_bytes<MT>() : 0);
  dim3 grid((unsigned)(((long long)a.nitem * groups + 7) / 8 * 8));
  if (src == kSrcF32 && a.K % 16 == 0 && a.N % 32 == 0)
    k_contract_mfma<kSrcF32, MT, true><<<grid, kWaves * 64, bytes, st>>>(a, groups);
  else if (src == kSrcF32)
    k_contract_mfma<kSrcF32, MT, false><<<grid, kWaves * 64, bytes, st>>>(a, groups);
  else if constexpr (MT < 4) {  // 16-bit tiles take groups of up to 32 pairs
    if (src == kSrcF16)
      k_contract_mfma<kSrcF16, MT, false><<<grid, kWaves * 64, bytes, st>>>(a, groups);
    else
      k_contract_mfma<kSrcBf16, MT, false><<<grid, kWaves * 64, bytes, st>>>(a, groups);
  }
}

// one wave per row: the row's largest magnitude m, then e = 15 - E with
// m = f 2^E, 1/2 <= f < 1 (E = 0 when m is zero).  Rows start on 16-byte
// boundaries and their stride is a multiple of 4 floats, so every 4-float
// load that starts below K stays inside the row's stride.
__global__ __launch_bounds__(256) void k_row_exp(const float* rows, long long nrows, int K, int srow, int32_t* ex) {
  const long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nrows) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const float* p = rows + r * srow;
  float mx = 0.f;
  for (int k = 4 * lane; k < K; k += 256) {
    const float4 v = *reinterpret_cast<const float4*>(p + k);
    mx = fmaxf(mx, fabsf(v.x));
    if (k + 1 < K) mx = fmaxf(mx, fabsf(v.y));
    if (k + 2 < K) mx = fmaxf(mx, fabsf(v.z));
    if (k + 3 < K) mx = fmaxf(mx, fabsf(v.w));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if (lane == 0) {
    int E;
    (void)frexpf(mx, &E);
    ex[r] = 15 - E;
  }
}

pat_status row_exponents(const float* rows, long long nrows, int K, int srow, int32_t* ex, hipStream_t st) {
  if (nrows == 0) return PAT_OK;
  if (!rows || !ex || K < 0 || srow < K || srow % 4 != 0 || (reinterpret_cast<uintptr_t>(rows) & 15u) != 0)
    return fail(PAT_EINVAL, "row exponents: rows must be 16-byte aligned with a stride of whole 4-float units");
  const long long blocks = (nrows + 3) / 4;
  if (blocks > 0x7fffffffLL) return fail(PAT_EUNSUPPORTED, "row exponents: too many rows");
  k_row_exp<<<dim3((unsigned)blocks), 256, 0, st>>>(rows, nrows, K, srow, ex);
  PAT_LAUNCHED("row exponents");
  return PAT_OK;
}

pat_status contract_mfma(const MfmaArgs& a, int hdtype, hipStream_t st) {
  if (a.nitem == 0 || a.B == 0) return PAT_OK;
  const int src = hdtype == PAT_H_F16 ? kSrcF16 : hdtype == PAT_H_F32 ? kSrcF32 : kSrcBf16;
  if (src == kSrcF32 && (!a.krows || !a.kexp))
    return fail(PAT_EINVAL, "float32 contraction on the matrix cores needs the k rows and their exponents");
  if (src != kSrcF32 && !a.frag) return fail(PAT_EINVAL, "16-bit contraction needs the operand tiles");
  if (a.G < 1 || a.G > 8) return fail(PAT_EINVAL, "work items hold 1 to 8 member slots");
  const int npairs = a.G * a.B;
  // column groups of 64 pairs for float32 rows (every group splits the
  // slab's values into float16 terms and reads the slab once: half as often as
  // with 32-pair groups; measured 8-10 % faster at B = 16), 32 for 16-bit
  // tiles (64 measured 1-3 % slower), 16 when there are no more pairs
  const int MT = npairs <= 16 ? 1 : src == kSrcF32 && npairs >= 64 ? 4 : 2;
  const int groups = (npairs + MT * 16 - 1) / (MT * 16);
  if (((long long)a.nitem * groups + 7) / 8 * 8 > 0x7fffffffLL) return fail(PAT_EUNSUPPORTED, "contraction grid too large");
  if (MT == 1)
    launch_mt<1>(a, src, groups, st);
  else if (MT == 4)
    launch_mt<4>(a, src, groups, st);
  else
    launch_mt<2>(a, src, groups, st);
  PAT_LAUNCHED("contraction (MFMA)");
  return PAT_OK;
}

}  // namespace pat
