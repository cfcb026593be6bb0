// Per-frequency multiply-accumulate of the operator (step (ii) of Sec. 3.2).
//
// For every transverse frequency k:
//   A   :  D^[k, n] = sum_l H^[k, l, n] X^[k, l]          (sum over depth)
//   A^T :  G^[k, l] = sum_n conj(H^[k, l, n]) R^[k, n]    (sum over time)
// H^ is real and identical for all frequencies of one symmetry class, so the
// library keeps one slab per class in two layouts, [l][n] for A and [n][l] for
// A^T.  Both products then have the same shape: the summed index i runs over
// slab rows, the kept index j runs along a row, and one workgroup (or, for
// long rows, two, each taking half of every row) streams one slab exactly once
// while applying it to every member frequency of its work item (up to eight).  Streaming the slab is the whole cost (it is >95 % of the bytes
// an apply moves), so the kernel is built around 16-byte non-temporal loads
// of whole rows: lanes of a row group cover one row, row groups take
// interleaved rows, and a short LDS tree adds the row-group partial sums at
// the end.  Accumulation is float32 for every storage type.
#include <type_traits>

#include "dft.hpp"
#include "pat_internal.hpp"

namespace pat {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int kRowParts = 2;  // workgroups per item and object for long rows

template <typename HT> struct Slab;

template <> struct Slab<float> {
  static constexpr int VEC = 4;
  typedef v4f raw_t;
  __device__ static __forceinline__ float get(const raw_t& r, int v) { return r[v]; }
};

struct bf16_t { unsigned short bits; };
struct f16_t { unsigned short bits; };

template <> struct Slab<bf16_t> {
  static constexpr int VEC = 8;
  typedef v4u raw_t;
  __device__ static __forceinline__ float get(const raw_t& r, int v) {
    const unsigned w = r[v >> 1];
    const unsigned b = (v & 1) ? (w & 0xFFFF0000u) : (w << 16);
    return __uint_as_float(b);
  }
};

template <> struct Slab<f16_t> {
  static constexpr int VEC = 8;
  typedef v4u raw_t;
  __device__ static __forceinline__ float get(const raw_t& r, int v) {
    const unsigned w = r[v >> 1];
    const unsigned short h = (v & 1) ? (unsigned short)(w >> 16) : (unsigned short)(w & 0xFFFFu);
    _Float16 x;
    __builtin_memcpy(&x, &h, 2);
    return (float)x;
  }
};

// One work item: GG active member slots (GG <= G, the slot count of the
// spectrum rows).  Uniform per workgroup.
// float32 slabs with rows of one chunk per lane: two rows per register
// buffer instead of four, so that the kernel fits 128 registers and four
// waves per SIMD (measured faster on short rows, neutral on long ones)
template <typename HT, int JPT>
constexpr bool kLowRegs = std::is_same<HT, float>::value && JPT == 1;

template <typename HT, int G, int GG, int JPT>
__device__ __forceinline__ void contract_item(const ContractArgs& a, int lr_log2, int t, int b, int j0,
                                              int njl, const int (&kg)[G], float4* smem_raw) {
  typedef Slab<HT> SL;
  typedef typename SL::raw_t raw_t;
  constexpr int VEC = SL::VEC;
  constexpr int U = kLowRegs<HT, JPT> ? 2 : 4 / JPT;  // rows per register buffer
  constexpr int NS = JPT * VEC * GG * 2;    // accumulators per thread
  float2* xin = reinterpret_cast<float2*>(smem_raw);
  float* red = reinterpret_cast<float*>(smem_raw);
  const int tid = threadIdx.x;
  const int Lr = 1 << lr_log2, R = 256 >> lr_log2;
  const int lr = tid & (Lr - 1), rg = tid >> lr_log2;

  // this workgroup's part of the rows: elements j0 .. j0 + njl - 1
  const HT* slab = reinterpret_cast<const HT*>(a.slab) + (size_t)a.item_slab[t] * a.slab_elems + j0;
  const int nchunks = (njl + VEC - 1) / VEC;
  bool cl[JPT];
  const HT* colp[JPT];
#pragma unroll
  for (int jj = 0; jj < JPT; ++jj) {
    const int ch = lr + jj * Lr;
    cl[jj] = ch < nchunks;
    colp[jj] = slab + (size_t)min(ch, nchunks - 1) * VEC;  // clamped: always a valid address
  }

  // Rows in flight: the loads of the next U rows are issued before the FMAs
  // of the current ones (two register buffers), so that every wave keeps
  // memory requests outstanding while it computes.  Loads are unconditional
  // (rows and chunks clamped into the slab, the value zeroed by a select) so
  // that no branch hides them from the wait counter.
  auto load_rows = [&](raw_t (&raw)[U][JPT], int i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * R;
      const int ic = min(i, a.ni - 1);
#pragma unroll
      for (int jj = 0; jj < JPT; ++jj) {
        const raw_t v = __builtin_nontemporal_load(
            reinterpret_cast<const raw_t*>(colp[jj] + (size_t)ic * a.s_row));
        raw[u][jj] = (i < a.ni && cl[jj]) ? v : raw_t(0);
      }
    }
  };
  raw_t ra[U][JPT], rb[U][JPT];
  load_rows(ra, rg);  // the first rows travel while the member vectors are staged

  // member input vectors -> LDS xin[i][g], with the optional per-row scale;
  // 16-byte loads along each member row when the row length is even
  if ((a.ni & 1) == 0) {
    // batches of kStage loads per thread, all issued before their LDS stores
    // (one memory latency per batch instead of one per load); consecutive
    // lanes take consecutive members of one k pair, so that the LDS stores
    // are contiguous (the loads still cover whole 128-byte lines per wave)
    constexpr int kStage = 8;
    const int h = a.ni >> 1;
    const int total = GG * h;
    for (int base = tid; base < total; base += 256 * kStage) {
      float4 v[kStage];
      float2 sv[kStage];  // the per-row scales of the pair, loaded with it
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int idx = base + q * 256;
        v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        sv[q] = make_float2(1.f, 1.f);
        if (idx < total) {
          const int g = idx % GG, i = 2 * (idx / GG);
          int k = -1;
#pragma unroll
          for (int gg = 0; gg < GG; ++gg) k = (gg == g) ? kg[gg] : k;
          if (k >= 0)
            v[q] = *reinterpret_cast<const float4*>(a.in + (size_t)(t * G + g) * a.in_rs + (size_t)b * a.ni + i);
          if (a.in_scale) sv[q] = *reinterpret_cast<const float2*>(a.in_scale + i);
        }
      }
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int idx = base + q * 256;
        if (idx >= total) break;
        const int g = idx % GG, i = 2 * (idx / GG);
        float4 w = v[q];
        if (a.in_scale) w = make_float4(w.x * sv[q].x, w.y * sv[q].x, w.z * sv[q].y, w.w * sv[q].y);
        xin[i * GG + g] = make_float2(w.x, w.y);
        xin[(i + 1) * GG + g] = make_float2(w.z, w.w);
      }
    }
  } else {
    for (int idx = tid; idx < a.ni * GG; idx += 256) {
      const int i = idx / GG, g = idx % GG;
      int k = -1;
#pragma unroll
      for (int gg = 0; gg < GG; ++gg) k = (gg == g) ? kg[gg] : k;
      float2 v = make_float2(0.f, 0.f);
      if (k >= 0) {
        v = a.in[(size_t)(t * G + g) * a.in_rs + (size_t)b * a.ni + i];
        if (a.in_scale) v = cscale(v, a.in_scale[i]);
      }
      xin[idx] = v;
    }
  }
  __syncthreads();

  float acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.f;

  auto fma_rows = [&](const raw_t (&raw)[U][JPT], int i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * R;
      if (i >= a.ni) break;
      float2 xv[GG];
#pragma unroll
      for (int g = 0; g < GG; ++g) xv[g] = xin[i * GG + g];
#pragma unroll
      for (int jj = 0; jj < JPT; ++jj) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const float h = SL::get(raw[u][jj], v);
#pragma unroll
          for (int g = 0; g < GG; ++g) {
            float* p = &acc[((jj * VEC + v) * GG + g) * 2];
            p[0] = fmaf(h, xv[g].x, p[0]);
            p[1] = fmaf(h, xv[g].y, p[1]);
          }
        }
      }
    }
  };
  for (int i0 = rg; i0 < a.ni; i0 += 2 * R * U) {
    load_rows(rb, i0 + R * U);
    fma_rows(ra, i0);
    if (i0 + R * U >= a.ni) break;
    load_rows(ra, i0 + 2 * R * U);
    fma_rows(rb, i0 + R * U);
  }

  // add the partial sums of the R row groups (fixed order: deterministic)
  for (int half = R >> 1; half >= 1; half >>= 1) {
    __syncthreads();
    const int span = half * Lr;
    if (rg >= half && rg < 2 * half) {
      const int w = (rg - half) * Lr + lr;
#pragma unroll
      for (int s = 0; s < NS; ++s) red[s * span + w] = acc[s];
    }
    __syncthreads();
    if (rg < half) {
      const int w = rg * Lr + lr;
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s] += red[s * span + w];
    }
  }

  // float32, whole 16-byte pairs per lane and nothing to subtract: row group
  // 0 stores its sums directly (each lane four consecutive outputs per
  // member, the lanes of a member row contiguous), without a pass through
  // LDS (A and A^T 1.5 % faster; the 16-bit kernels, eight outputs per lane,
  // measured 4 % slower that way and keep the pass through LDS)
  if (std::is_same<HT, float>::value && a.out_sub == nullptr && (a.nj & 1) == 0 && njl % VEC == 0) {
    if (rg != 0) return;
    if (a.out_scale) {
      // per-row output scales, all loaded before the first use and applied
      // here, so that no load is outstanding at the stores below
      float scv[JPT][VEC];
#pragma unroll
      for (int jj = 0; jj < JPT; ++jj)
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          scv[jj][v] = a.out_scale[j0 + min((lr + jj * Lr) * VEC + v, njl - 1)];
#pragma unroll
      for (int jj = 0; jj < JPT; ++jj)
#pragma unroll
        for (int v = 0; v < VEC; ++v)
#pragma unroll
          for (int g = 0; g < GG; ++g) {
            float* q = &acc[((jj * VEC + v) * GG + g) * 2];
            q[0] *= scv[jj][v];
            q[1] *= scv[jj][v];
          }
    }
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) {
      const int cj = (lr + jj * Lr) * VEC;
      if (cj >= njl) continue;
#pragma unroll
      for (int g = 0; g < GG; ++g) {
        if (kg[g] < 0) continue;
        v4f* dst = reinterpret_cast<v4f*>(a.out + (size_t)(t * G + g) * a.out_rs + (size_t)b * a.nj + j0 + cj);
#pragma unroll
        for (int v = 0; v < VEC; v += 2) {
          const float* q0 = &acc[((jj * VEC + v) * GG + g) * 2];
          const float* q1 = &acc[((jj * VEC + v + 1) * GG + g) * 2];
          __builtin_nontemporal_store(v4f{q0[0], q0[1], q1[0], q1[1]}, dst + v / 2);
        }
      }
    }
    return;
  }

  // stage the member rows in LDS, then store each row contiguously (whole
  // cache lines per store instruction)
  __syncthreads();
  float2* ob = reinterpret_cast<float2*>(smem_raw);
  if (rg == 0) {
    // per-row output scales: every load issued before the first is used
    float scv[JPT][VEC];
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int j = (lr + jj * Lr) * VEC + v;
        scv[jj][v] = a.out_scale ? a.out_scale[j0 + min(j, njl - 1)] : 1.f;
      }
#pragma unroll
    for (int jj = 0; jj < JPT; ++jj) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int j = (lr + jj * Lr) * VEC + v;
        if (j >= njl) continue;
        const float sc = scv[jj][v];
#pragma unroll
        for (int g = 0; g < GG; ++g) {
          const float* p = &acc[((jj * VEC + v) * GG + g) * 2];
          ob[g * njl + j] = make_float2(p[0] * sc, p[1] * sc);
        }
      }
    }
  }
  __syncthreads();
  if ((njl & 1) == 0 && (a.nj & 1) == 0) {
    // two complex values (16 bytes) per store, non-temporal: the rows are
    // not read again by this kernel
    // groups of kOut elements per thread: the values of a group (and the
    // subtracted ones) are all read into separate registers before its
    // first store; a load issued after a store, or a register rewritten
    // while a store still reads it, waits for that store on the in-order
    // memory counter
    constexpr int kOut = 2;
    const int h = njl >> 1;
    for (int e0 = tid; e0 < GG * h; e0 += 256 * kOut) {
      float4 val[kOut], sub[kOut];
      bool ok[kOut];
#pragma unroll
      for (int q = 0; q < kOut; ++q) {
        const int e = e0 + q * 256;
        const int g = e / h, j = 2 * (e - g * h);
        int k = -1;
#pragma unroll
        for (int gg = 0; gg < GG; ++gg) k = (gg == g) ? kg[gg] : k;
        ok[q] = e < GG * h && k >= 0;
        sub[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        val[q] = sub[q];
        if (ok[q]) {
          val[q] = *reinterpret_cast<const float4*>(ob + g * njl + j);
          if (a.out_sub)
            sub[q] = *reinterpret_cast<const float4*>(a.out_sub + (size_t)(t * G + g) * a.out_rs +
                                                      (size_t)b * a.nj + j0 + j);
        }
      }
      // differences on straight-line code (the empty asm keeps them out of
      // the conditional stores, where each store would wait again)
      v4f d[kOut];
#pragma unroll
      for (int q = 0; q < kOut; ++q) {
        d[q] = v4f{val[q].x - sub[q].x, val[q].y - sub[q].y, val[q].z - sub[q].z, val[q].w - sub[q].w};
        asm volatile("" : "+v"(d[q]));
      }
#pragma unroll
      for (int q = 0; q < kOut; ++q) {
        const int e = e0 + q * 256;
        const int g = e / h, j = 2 * (e - g * h);
        if (ok[q]) {
          const size_t o = (size_t)(t * G + g) * a.out_rs + (size_t)b * a.nj + j0 + j;
          __builtin_nontemporal_store(d[q], reinterpret_cast<v4f*>(a.out + o));
        }
      }
    }
  } else {
    for (int e = tid; e < GG * njl; e += 256) {
      const int g = e / njl, j = e - g * njl;
      int k = -1;
#pragma unroll
      for (int gg = 0; gg < GG; ++gg) k = (gg == g) ? kg[gg] : k;
      if (k >= 0) {
        const size_t o = (size_t)(t * G + g) * a.out_rs + (size_t)b * a.nj + j0 + j;
        a.out[o] = a.out_sub ? csub(ob[e], a.out_sub[o]) : ob[e];
      }
    }
  }
}

// Workgroups -> (item t, object b, row part).  One object: JS workgroups per
// item, each streaming 1/JS of every slab row (shorter workgroups, a shorter
// tail); a batch: one workgroup per item and object.  Workgroups are dealt to
// the eight XCDs round-robin by index, so the units (item, part or object),
// in item order, are cut into eight contiguous ranges, one per XCD, each
// taken in order: the B objects of an item, and the items a large class is
// split into (adjacent, reading the same slab), run on one XCD at about the
// same time, and every read of a slab after the first comes from that XCD's
// L2 instead of HBM.
__device__ __forceinline__ bool item_of_block(int nitem, int B, int JS, int& t, int& b, int& part) {
  const int per_item = B == 1 ? JS : B;
  const int units = nitem * per_item;
  const int per_xcd = (units + 7) >> 3;
  const int u = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (u >= units) return false;
  t = u / per_item;
  const int rem = u - t * per_item;
  part = B == 1 ? rem : 0;
  b = B == 1 ? 0 : rem;
  return true;
}

template <typename HT, int G, int JPT>
__global__ __launch_bounds__(256, (kLowRegs<HT, JPT> ? 4 : 1)) void k_contract(ContractArgs a, int lr_log2, int B, int JS, int chpart) {
  extern __shared__ float4 smem_raw[];
  int t, b, part;
  if (!item_of_block(a.nitem, B, JS, t, b, part)) return;  // whole workgroup: padding of the grid
  constexpr int VEC = Slab<HT>::VEC;
  const int j0 = part * chpart * VEC;
  const int njl = min(a.nj - j0, chpart * VEC);
  int kg[G];
#pragma unroll
  for (int g = 0; g < G; ++g) kg[g] = a.members[t * G + g];
  if constexpr (G > 4) {
    if (kg[4] < 0) {  // at most four members: the cheaper body
      contract_item<HT, G, 4, JPT>(a, lr_log2, t, b, j0, njl, kg, smem_raw);
      return;
    }
  }
  contract_item<HT, G, G, JPT>(a, lr_log2, t, b, j0, njl, kg, smem_raw);
}

template <typename HT, int G>
static pat_status launch_t(const ContractArgs& a, int B, hipStream_t st) {
  constexpr int VEC = Slab<HT>::VEC;
  // one object: rows of 128 or more 16-byte chunks are split over kRowParts
  // workgroups per item (halves of 1 KB and more still stream well; shorter
  // parts measured slower)
  const int JS = (B == 1 && (a.nj + VEC - 1) / VEC >= 128) ? kRowParts : 1;
  const int chpart = ((a.nj + VEC - 1) / VEC + JS - 1) / JS;  // 16-byte chunks per part
  const int nchunks = chpart;
  int lr_log2 = 0;
  while ((1 << lr_log2) < nchunks && lr_log2 < 8) ++lr_log2;
  const int Lr = 1 << lr_log2, R = 256 / Lr;
  const int jpt = (nchunks + Lr - 1) / Lr;
  if (jpt > 2) return fail(PAT_EUNSUPPORTED, "contraction row longer than 512 vectors");
  const int ns = jpt * VEC * G * 2;
  size_t red_bytes = R > 1 ? (size_t)(R / 2) * Lr * ns * sizeof(float) : 0;
  size_t in_bytes = (size_t)a.ni * G * sizeof(float2);
  size_t out_bytes = (size_t)chpart * VEC * G * sizeof(float2);
  size_t lds = red_bytes > in_bytes ? red_bytes : in_bytes;
  lds = lds > out_bytes ? lds : out_bytes;
  if (lds > 160 * 1024) return fail(PAT_EUNSUPPORTED, "contraction input vector does not fit in LDS");
  const long long nblk = ((long long)a.nitem * (B == 1 ? JS : B) + 7) / 8 * 8;
  if (nblk > 0x7fffffffLL) return fail(PAT_EUNSUPPORTED, "contraction grid too large");
  dim3 grid((unsigned)nblk);
  if (jpt == 1)
    k_contract<HT, G, 1><<<grid, 256, lds, st>>>(a, lr_log2, B, JS, chpart);
  else
    k_contract<HT, G, 2><<<grid, 256, lds, st>>>(a, lr_log2, B, JS, chpart);
  PAT_LAUNCHED("contraction");
  return PAT_OK;
}

pat_status contract(const ContractArgs& a, int hdtype, int G, int B, hipStream_t st) {
  if (a.nitem == 0 || B == 0) return PAT_OK;
  if (G == 8) {  // radial fold: float32 libraries only
    if (hdtype == PAT_H_F32) return launch_t<float, 8>(a, B, st);
    return fail(PAT_EUNSUPPORTED, "8-member work items need a float32 library");
  }
  if (G == 4) {
    if (hdtype == PAT_H_F32) return launch_t<float, 4>(a, B, st);
    if (hdtype == PAT_H_BF16) return launch_t<bf16_t, 4>(a, B, st);
    return launch_t<f16_t, 4>(a, B, st);
  }
  if (hdtype == PAT_H_F32) return launch_t<float, 2>(a, B, st);
  if (hdtype == PAT_H_BF16) return launch_t<bf16_t, 2>(a, B, st);
  return launch_t<f16_t, 2>(a, B, st);
}

}  // namespace pat
