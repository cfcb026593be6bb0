// Kernel library build: the sensor-plane response of a unit point absorber at
// each depth, in the transverse Fourier domain (the depth-indexed impulse
// responses of Sec. 2.1, built once and reused by every apply, Sec. 3.2).
//
// On the grid that is periodic in x, y and z (z-period nq = nz_sim) the exact
// semi-discrete solution of the wave equation with zero initial velocity is
// cos(c t |k|) times the initial spectrum.  Restricted to the sensor plane:
//
//   H^[l, n] = (1/nq) sum_{q} cos(n c dt |k(q)|) cos(2 pi q l / nq)
//            = sum_{q=0}^{floor(nq/2)} w_q/nq cos(n theta_q) cos(2 pi q l / nq),
//
// with theta_q = c dt sqrt(kx^2 + ky^2 + kz(q)^2), w_q = 2 for the pairs
// {q, -q} and 1 for q = 0 and the Nyquist plane; the imaginary parts cancel
// in pairs, so H^ is real.  Phases reach several hundred radians, so the
// whole build runs in float64 and rounds once (to float32, then to 16 bits
// for the reduced-precision forms).  A sensor response r (causal FIR) is
// folded in along t: H^'[l, n] = sum_j r_j H^[l, n - j].
//
// Two ways to obtain the time factor: evaluated directly (closed form), or
// by one k-space time-stepping run from a unit point source at the origin,
// P^0 = 1, P^1 = cos(theta) P^0, P^{n+1} = 2 cos(theta) P^n - P^{n-1} (the
// exact propagator with zero initial velocity, float64), whose field on depth
// plane l at step n is the inverse z-DFT sum above: by reciprocity the field
// at depth l due to a source on the sensor plane is the sensor-plane
// response to a source at depth l (the single-simulation library of
// Sec. 3.2).  The stepper records the field of a block of classes in build
// scratch; the depth sum then reads the record instead of the cosines.
#include <algorithm>
#include <cmath>

#include "pat_internal.hpp"

namespace pat {

constexpr int kNT = 64;   // time samples per workgroup
constexpr int kLP = 64;   // depths per pass (4 groups x 16)
constexpr int kQB = 32;   // q values per LDS chunk
constexpr int kMaxNq = 4096;

__device__ __forceinline__ int ceil_log2_d(double v) {
  int e;
  const double f = frexp(v, &e);  // v = f 2^e, 0.5 <= f < 1
  return f == 0.5 ? e - 1 : e;
}

__device__ __forceinline__ double depth_scale(const unsigned long long* amax, int l, int hdtype) {
  if (hdtype == PAT_H_F32) return 1.0;
  const double m = __longlong_as_double((long long)amax[l]);
  if (!(m > 0.0)) return 1.0;
  const int e = hdtype == PAT_H_BF16 ? 0 : 15;
  return ldexp(1.0, e - ceil_log2_d(m));
}

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ unsigned short to_f16(float f) {
  _Float16 h = (_Float16)f;
  unsigned short b;
  __builtin_memcpy(&b, &h, 2);
  return b;
}

// MODE 0: per-depth max |H^| only, 1: write the slabs.  FIR: fold the sensor
// response into the time axis.  The library is linear in the time factor
// cos(n theta_q), so the filter acts on that factor: each q-chunk also
// evaluates it at the n_ir - 1 earlier samples (zero before t = 0) and
// filters in LDS before the depth sum.
// Stepped time factor of class a.c0 + blockIdx.y for the wavenumbers
// q = 0 .. nq/2 (one thread each): P^n(q) for n < nt, weighted by w_q / nq,
// into ptab[(blockIdx.y * nt + n) * (nq/2 + 1) + q].
__global__ __launch_bounds__(256) void k_hstep(HBuildArgs a) {
  const int Qn = a.nq / 2 + 1;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Qn) return;
  const int c = a.c0 + blockIdx.y;
  const double two_pi = 6.283185307179586476925286766559;
  const double kx = two_pi * a.cls_freq[2 * c] / (a.nx * a.dx);
  const double ky = two_pi * a.cls_freq[2 * c + 1] / (a.ny * a.dy);
  const double kz = two_pi * q / (a.nq * a.dz);
  const double theta = a.c * a.dt * sqrt(kx * kx + ky * ky + kz * kz);
  const double two_cos = 2.0 * cos(theta);
  const double w = ((q == 0 || 2 * q == a.nq) ? 1.0 : 2.0) / a.nq;
  double* rec = a.ptab + (size_t)blockIdx.y * a.nt * Qn + q;
  double prev = 1.0;             // P^0: unit point source (flat spectrum)
  double cur = 0.5 * two_cos;    // P^1 = cos(theta) P^0: zero initial velocity
  rec[0] = w * prev;
  for (int n = 1; n < a.nt; ++n) {
    rec[(size_t)n * Qn] = w * cur;
    const double next = fma(two_cos, cur, -prev);
    prev = cur;
    cur = next;
  }
}

template <int MODE, bool FIR, bool STEP>
__global__ __launch_bounds__(256) void k_hbuild(HBuildArgs a) {
  __shared__ double ctab[kMaxNq];
  __shared__ double P[kQB * kNT];
  __shared__ float tile[kNT * (kLP + 1)];
  __shared__ double Praw[FIR ? kQB * (kNT + kMaxIr - 1) : 1];
  __shared__ double irs[FIR ? kMaxIr : 1];
  const int tid = threadIdx.x;
  const int nl = tid & (kNT - 1), lg = tid >> 6;
  const int c = a.c0 + blockIdx.y;
  const int n = blockIdx.x * kNT + nl;
  const double* rec = STEP ? a.ptab + (size_t)blockIdx.y * a.nt * (a.nq / 2 + 1) : nullptr;
  const int nq = a.nq;
  const int Qn = nq / 2 + 1;
  const double two_pi = 6.283185307179586476925286766559;

  for (int r = tid; r < nq; r += 256) ctab[r] = cos(two_pi * (double)r / (double)nq);
  if constexpr (FIR)
    for (int j = tid; j < a.n_ir; j += 256) irs[j] = a.ir[j];

  const int fx = a.cls_freq[2 * c], fy = a.cls_freq[2 * c + 1];
  const double kx = two_pi * fx / (a.nx * a.dx);
  const double ky = two_pi * fy / (a.ny * a.dy);
  const double kperp2 = kx * kx + ky * ky;
  const double cdt = a.c * a.dt;
  const double inv_nq = 1.0 / nq;

  for (int l0 = 0; l0 < a.nz; l0 += kLP) {
    double acc[16];
    int idx[16], stp[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      acc[u] = 0.0;
      idx[u] = 0;
      stp[u] = (l0 + lg + 4 * u) % nq;
    }
    for (int q0 = 0; q0 < Qn; q0 += kQB) {
      __syncthreads();
      if constexpr (!FIR) {
        for (int e = tid; e < kQB * kNT; e += 256) {
          const int qq = e / kNT, nn = e % kNT;
          const int q = q0 + qq, ng = blockIdx.x * kNT + nn;
          double v = 0.0;
          if (q < Qn && ng < a.nt) {
            if constexpr (STEP) {
              v = rec[(size_t)ng * Qn + q];
            } else {
              const double kz = two_pi * q / (nq * a.dz);
              const double theta = cdt * sqrt(kperp2 + kz * kz);
              const double w = (q == 0 || 2 * q == nq) ? 1.0 : 2.0;
              v = w * inv_nq * cos((double)ng * theta);
            }
          }
          P[e] = v;
        }
      } else {
        const int L = a.n_ir, W = kNT + L - 1;
        const int nbase = blockIdx.x * kNT - (L - 1);
        for (int e = tid; e < kQB * W; e += 256) {
          const int qq = e / W, nr = e % W;
          const int q = q0 + qq, ng = nbase + nr;
          double v = 0.0;
          if (q < Qn && ng >= 0 && ng < a.nt) {
            if constexpr (STEP) {
              v = rec[(size_t)ng * Qn + q];
            } else {
              const double kz = two_pi * q / (nq * a.dz);
              const double theta = cdt * sqrt(kperp2 + kz * kz);
              const double w = (q == 0 || 2 * q == nq) ? 1.0 : 2.0;
              v = w * inv_nq * cos((double)ng * theta);
            }
          }
          Praw[qq * W + nr] = v;
        }
        __syncthreads();
        for (int e = tid; e < kQB * kNT; e += 256) {
          const int qq = e / kNT, nn = e % kNT;
          const double* pr = Praw + qq * W + nn + (L - 1);
          double v = 0.0;
          for (int j = 0; j < L; ++j) v = fma(irs[j], pr[-j], v);
          P[e] = v;
        }
      }
      __syncthreads();
      const int qe = (Qn - q0) < kQB ? (Qn - q0) : kQB;
      for (int qq = 0; qq < qe; ++qq) {
        const double p = P[qq * kNT + nl];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          acc[u] = fma(p, ctab[idx[u]], acc[u]);
          idx[u] += stp[u];
          if (idx[u] >= nq) idx[u] -= nq;
        }
      }
    }

    if (MODE == 0) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int l = l0 + lg + 4 * u;
        double m = (n < a.nt) ? fabs(acc[u]) : 0.0;
        for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if (nl == 0 && l < a.nz)
          atomicMax(&a.amax[l], (unsigned long long)__double_as_longlong(m));
      }
    } else {
      // [l][n] rows: lanes along n, coalesced; the scaled values also go to
      // the LDS tile for the transposed and the fragment layouts
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int ll = lg + 4 * u, l = l0 + ll;
        float f = 0.f;
        if (l < a.nz) f = (float)(acc[u] * depth_scale(a.amax, l, a.hdtype));
        tile[nl * (kLP + 1) + ll] = f;
        if (l < a.nz && n < a.nt) {
          const size_t o = ((size_t)c * a.nz + l) * a.sA_row + n;
          if (a.hdtype == PAT_H_F32) reinterpret_cast<float*>(a.rowA)[o] = f;
          else if (a.hdtype == PAT_H_BF16) reinterpret_cast<unsigned short*>(a.rowA)[o] = to_bf16(f);
          else reinterpret_cast<unsigned short*>(a.rowA)[o] = to_f16(f);
        }
      }
      __syncthreads();
      // [n][l] rows: transpose through LDS so that lanes run along l
      for (int e = tid; e < kNT * kLP; e += 256) {
        const int nn = e / kLP, ll = e % kLP;
        const int ng = blockIdx.x * kNT + nn, l = l0 + ll;
        if (ng >= a.nt || l >= a.nz) continue;
        const float f = tile[nn * (kLP + 1) + ll];
        const size_t o = ((size_t)c * a.nt + ng) * a.sT_row + l;
        if (a.hdtype == PAT_H_F32) reinterpret_cast<float*>(a.rowT)[o] = f;
        else if (a.hdtype == PAT_H_BF16) reinterpret_cast<unsigned short*>(a.rowT)[o] = to_bf16(f);
        else reinterpret_cast<unsigned short*>(a.rowT)[o] = to_f16(f);
      }
      if (a.hdtype != PAT_H_F32) {
        // 16-bit library: MFMA fragments for both directions, from the tile
        const int n0 = blockIdx.x * kNT;
        for (int dir = 0; dir < 2; ++dir) {
          // dir 0: rows n, k = l (forward);  dir 1: rows l, k = n (adjoint)
          const int nt = dir == 0 ? a.ntA : a.ntT, ks = dir == 0 ? a.ksA : a.ksT;
          const int rt0 = (dir == 0 ? n0 : l0) / 32, kt0 = (dir == 0 ? l0 : n0) / 16;
          unsigned short* dst = reinterpret_cast<unsigned short*>(dir == 0 ? a.slabA : a.slabT);
          for (int unit = tid; unit < 8 * 64; unit += 256) {
            const int f = unit >> 6, L = unit & 63;
            const int rt = f >> 2, kt = f & 3;
            if (rt0 + rt >= nt || kt0 + kt >= ks) continue;
            const int r = rt * 32 + (L & 31), k = kt * 16 + 8 * (L >> 5);
            unsigned short v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float x = dir == 0 ? tile[r * (kLP + 1) + k + e] : tile[(k + e) * (kLP + 1) + r];
              v[e] = a.hdtype == PAT_H_BF16 ? to_bf16(x) : to_f16(x);
            }
            uint4 pk;
            pk.x = v[0] | ((unsigned)v[1] << 16);
            pk.y = v[2] | ((unsigned)v[3] << 16);
            pk.z = v[4] | ((unsigned)v[5] << 16);
            pk.w = v[6] | ((unsigned)v[7] << 16);
            const size_t o = (((size_t)c * nt + rt0 + rt) * ks + kt0 + kt) * 64 + L;
            reinterpret_cast<uint4*>(dst)[o] = pk;
          }
        }
      }
    }
  }
}

__global__ void k_scales(const unsigned long long* amax, float* inv_scale, int nz, int hdtype) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nz) inv_scale[l] = (float)(1.0 / depth_scale(amax, l, hdtype));
}

template <int MODE>
static pat_status launch_depth_sum(const HBuildArgs& a, int ncls, hipStream_t st) {
  dim3 grid((a.nt + kNT - 1) / kNT, ncls);
  const bool fir = a.n_ir > 0, step = a.ptab != nullptr;
  if (step && fir) k_hbuild<MODE, true, true><<<grid, 256, 0, st>>>(a);
  else if (step) k_hbuild<MODE, false, true><<<grid, 256, 0, st>>>(a);
  else if (fir) k_hbuild<MODE, true, false><<<grid, 256, 0, st>>>(a);
  else k_hbuild<MODE, false, false><<<grid, 256, 0, st>>>(a);
  PAT_LAUNCHED(MODE == 0 ? "H build (max pass)" : "H build");
  return PAT_OK;
}

// one pass over all classes (MODE 0: per-depth maxima, 1: the slabs); the
// stepped build records and sums one block of classes at a time
template <int MODE>
static pat_status build_pass(const HBuildArgs& a, hipStream_t st) {
  if (!a.ptab) return launch_depth_sum<MODE>(a, a.nclass, st);
  const size_t per = step_class_bytes(a.nt, a.nq);
  const int block = (int)std::min<size_t>((size_t)a.nclass, a.ptab_bytes / per);
  if (block < 1) return fail(PAT_EINVAL, "build scratch holds less than one class's record");
  const int Qn = a.nq / 2 + 1;
  for (int c0 = 0; c0 < a.nclass; c0 += block) {
    HBuildArgs b = a;
    b.c0 = c0;
    const int ncls = std::min(block, a.nclass - c0);
    k_hstep<<<dim3((Qn + 255) / 256, ncls), 256, 0, st>>>(b);
    PAT_LAUNCHED("H build (k-space stepper)");
    PAT_TRY(launch_depth_sum<MODE>(b, ncls, st));
  }
  return PAT_OK;
}

pat_status hbuild(const HBuildArgs& a, hipStream_t st) {
  if (a.nq > kMaxNq) return fail(PAT_EUNSUPPORTED, "nz_sim above 4096 is not supported");
  if (a.n_ir < 0 || a.n_ir > kMaxIr || (a.n_ir > 0 && !a.ir))
    return fail(PAT_EINVAL, "sensor response: 0..64 taps");
  if (a.hdtype != PAT_H_F32) PAT_TRY(build_pass<0>(a, st));
  k_scales<<<(a.nz + 127) / 128, 128, 0, st>>>(a.amax, a.inv_scale, a.nz, a.hdtype);
  PAT_LAUNCHED("H build (scales)");
  return build_pass<1>(a, st);
}

// ------------------------------------------------------------ export
__global__ void k_hexport(const void* slabA, int hdtype, const int32_t* kclass,
                          const float* inv_scale, int k0, int nz, int nt, int sA_row, int ntA,
                          int ksA, float* out) {
  const int kk = blockIdx.x;
  const int c = kclass[k0 + kk];
  for (int e = threadIdx.x; e < nz * nt; e += blockDim.x) {
    const int l = e / nt, n = e % nt;
    float f;
    if (hdtype == PAT_H_F32) {
      f = reinterpret_cast<const float*>(slabA)[((size_t)c * nz + l) * sA_row + n];
    } else {
      // fragment (n/32, l/16), lane n%32 + 32*((l%16)/8), element l%8
      const size_t o = ((((size_t)c * ntA + n / 32) * ksA + l / 16) * 64 + (n & 31) + 32 * ((l >> 3) & 1)) * 8 + (l & 7);
      const unsigned short b = reinterpret_cast<const unsigned short*>(slabA)[o];
      if (hdtype == PAT_H_BF16) {
        f = __uint_as_float((unsigned)b << 16);
      } else {
        _Float16 h;
        __builtin_memcpy(&h, &b, 2);
        f = (float)h;
      }
    }
    out[(size_t)kk * nz * nt + e] = f * inv_scale[l];
  }
}

pat_status hexport(const void* slabA, int hdtype, const int32_t* kclass, const float* inv_scale,
                   int k0, int nk, int nz, int nt, int sA_row, int ntA, int ksA, float* out,
                   hipStream_t st) {
  if (nk <= 0) return PAT_OK;
  k_hexport<<<nk, 256, 0, st>>>(slabA, hdtype, kclass, inv_scale, k0, nz, nt, sA_row, ntA, ksA,
                                out);
  PAT_LAUNCHED("H export");
  return PAT_OK;
}


// ------------------------------------------------------- normal operator
// Gram blocks of the stored (dequantised) library: G_s[l][l'] =
// sum_n H^_s[l][n] H^_s[l'][n], accumulated in float64 and rounded once.  A^T A
// is block diagonal in the transverse Fourier basis with these blocks, so the
// gradient of the data term, A^T (A z - d) = A^T A z - A^T d (eq. 15), can be
// formed per frequency from the spectrum of z alone.
constexpr int kGN = 32;   // time samples per LDS chunk

__device__ __forceinline__ float lib_value(const GramArgs& a, int s, int l, int n) {
  if (a.hdtype == PAT_H_F32)
    return reinterpret_cast<const float*>(a.slabA)[((size_t)s * a.nz + l) * a.sA_row + n];
  const size_t o = ((((size_t)s * a.ntA + n / 32) * a.ksA + l / 16) * 64 + (n & 31) + 32 * ((l >> 3) & 1)) * 8 + (l & 7);
  const unsigned short b = reinterpret_cast<const unsigned short*>(a.slabA)[o];
  float f;
  if (a.hdtype == PAT_H_BF16) {
    f = __uint_as_float((unsigned)b << 16);
  } else {
    _Float16 h;
    __builtin_memcpy(&h, &b, 2);
    f = (float)h;
  }
  return f * a.inv_scale[l];
}

// workgroup = (slab, 64 x 64 output tile); thread = 4 x 4 outputs
__global__ __launch_bounds__(256) void k_gram(GramArgs a) {
  __shared__ double hi[64][kGN + 1], hj[64][kGN + 1];
  const int s = blockIdx.z;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  double acc[4][4] = {};
  for (int n0 = 0; n0 < a.nt; n0 += kGN) {
    __syncthreads();
    for (int e = tid; e < 64 * kGN; e += 256) {
      const int r = e / kGN, nn = e % kGN;
      const int n = n0 + nn;
      hi[r][nn] = (i0 + r < a.nz && n < a.nt) ? (double)lib_value(a, s, i0 + r, n) : 0.0;
      hj[r][nn] = (j0 + r < a.nz && n < a.nt) ? (double)lib_value(a, s, j0 + r, n) : 0.0;
    }
    __syncthreads();
    for (int nn = 0; nn < kGN; ++nn) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = hi[ti + 16 * u][nn];
        y[u] = hj[tj + 16 * u][nn];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(x[u], y[v], acc[u][v]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ti + 16 * u, j = j0 + tj + 16 * v;
      if (i < a.nz && j < a.nz) a.gram[((size_t)s * a.nz + i) * a.sG_row + j] = (float)acc[u][v];
    }
}

pat_status gram_build(const GramArgs& a, hipStream_t st) {
  if (a.nslab == 0) return PAT_OK;
  const int nb = (a.nz + 63) / 64;
  dim3 grid(nb, nb, a.nslab);
  k_gram<<<grid, 256, 0, st>>>(a);
  PAT_LAUNCHED("Gram blocks");
  return PAT_OK;
}

}  // namespace pat
