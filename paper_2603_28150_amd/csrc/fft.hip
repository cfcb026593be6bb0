// Batched 2D transverse FFTs (gfx950) for the transform sizes 2^a 3^b of
// PAT_FFT_SIZES: powers of two 16..1024 and 48..864 with b = 1..3 (radix-3
// stages; every size a multiple of 4 so that rows move as 16-byte units).
//
// Step (i) and step (iii) of the FFT realisation of the operator (Sec. 3.2):
// every depth or time slice is transformed over (x, y).  Each 1D transform
// is a four-step FFT, N = N1 * N2: every thread does one N1-point DFT in
// registers, multiplies by the twiddles, and after a single LDS exchange does
// one N2-point DFT.  Two passes move the data through HBM:
//   rows:    real rows (x) <-> half spectrum along x, transposed so that the
//            slice index is fastest, pairs of real rows packed into one
//            complex transform;
//   columns: complex transforms along y on the frequency-major layout, slices
//            fastest, so that loads and stores are contiguous across threads.
// Twiddles exp(-2 pi i e / N) of every size N are tabulated on the host in
// float64 and rounded once to float32.
//
// Transform sizes and data extents are separate: slices cover an nx_d x ny_d
// window of the fx x fy transform grid (nx_d <= fx, ny_d <= fy), sampled at
// every sx-th column and sy-th row (the slices store (nx_d/sx) x (ny_d/sy)
// values).  Points outside the window or between samples are zeros that are
// never read (forward) and never written (inverse), so the zero-padded
// linear convolution and the scan-grid sampling cost no extra HBM traffic.
#include <cmath>
#include <vector>

#include "dft.hpp"
#include "pat_internal.hpp"

namespace pat {

#define PAT_FFT_SIZES(X) \
  X(16) X(32) X(48) X(64) X(72) X(96) X(108) X(128) X(144) X(192) X(216) X(256) X(288) X(384) \
  X(432) X(512) X(576) X(768) X(864) X(1024)

#define PAT_SIZE_ENTRY(N) N,
constexpr int kFftSizes[] = {PAT_FFT_SIZES(PAT_SIZE_ENTRY)};
#undef PAT_SIZE_ENTRY

// twiddles of every size, one contiguous table per size (a block reads its
// N values as whole cache lines)
constexpr int tw_offset(int n) {
  int o = 0;
  for (int s : kFftSizes) {
    if (s == n) return o;
    o += s;
  }
  return -1;
}
constexpr int tw_total() {
  int o = 0;
  for (int s : kFftSizes) o += s;
  return o;
}
__device__ float2 g_tw[tw_total()];

pat_status fft_init_device() {
  std::vector<float2> host(tw_total());
  const double two_pi = 6.283185307179586476925286766559;
  for (int n : kFftSizes)
    for (int e = 0; e < n; ++e) {
      const double a = two_pi * e / (double)n;
      host[tw_offset(n) + e] = make_float2((float)std::cos(a), (float)-std::sin(a));
    }
  PAT_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host.data(), sizeof(float2) * host.size(), 0,
                            hipMemcpyHostToDevice));
  return PAT_OK;
}

// exp(DIR 2 pi i e / N), e < N, into LDS
template <int N, int DIR>
__device__ __forceinline__ void load_twiddles(float2* tw, int tid, int nthreads) {
  constexpr int off = tw_offset(N);
  static_assert(off >= 0, "no twiddles for this size");
  for (int e = tid; e < N; e += nthreads) {
    const float2 w = g_tw[off + e];
    tw[e] = DIR < 0 ? w : cconj(w);
  }
}

// block -> (row j, slice block sb) of a row pass over a (ny x nsb) grid:
// rows fastest within tiles of tj rows, the tiles one after another
__device__ __forceinline__ void row_block(int tj, int& j, int& sb) {
  const int ny = gridDim.x, nsb = gridDim.y;
  const long long L = (long long)blockIdx.y * ny + blockIdx.x;
  const int tile = (int)(L / ((long long)tj * nsb));
  const int tjj = min(tj, ny - tile * tj);
  const int in = (int)(L - (long long)tile * tj * nsb);
  j = tile * tj + in % tjj;
  sb = in / tjj;
}

// ------------------------------------------------------------- columns (y)
// out[orow(p)*rs + s] = sum_j exp(DIR 2 pi i p j / N) in[irow(j)*rs + s]
// irow / orow: the spectrum side uses the class-major row map so that the
// contraction reads and writes contiguous rows; the other side is compact:
// only rows j = istride*j' with j' < nin are present (the others are zeros),
// at row j'*nh + m, and only rows p = ostride*p' with p' < nout are written,
// at row p'*nh + m.
// slices per block: 16 contiguous 8-byte values per spectrum row fill a
// 128-byte line (8 or 4 slices ran the 512- to 1024-point passes 1.3-1.7x
// slower); up to 16 * 32 threads and 147 KB of LDS at 1024 points
template <int N> struct ColSB { static constexpr int value = 16; };

template <int N, int DIR>
__global__ __launch_bounds__(512) void k_fft_cols(const float2* __restrict__ in,
                                                  float2* __restrict__ out, int nh, int S,
                                                  int rs, const int32_t* __restrict__ imap,
                                                  const int32_t* __restrict__ omap, int sfast,
                                                  int nin, int istride, int nout, int ostride) {
  constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
  constexpr int SB = ColSB<N>::value;
  constexpr int PAD = N + 1;   // LDS stride per slice (complex)
  constexpr int NT = SB * N1;  // threads
  __shared__ float2 tw[N];
  __shared__ float2 ex[SB * PAD];
  __shared__ int rin[N], rout[N];
  const int tid = threadIdx.x;
  const int s = tid % SB, t = tid / SB;
  // grid order: slice blocks fastest for very wide rows (adjacent workgroups
  // share rows), frequency columns fastest otherwise (spreads channels)
  const int m = sfast ? blockIdx.y : blockIdx.x;
  const int sg = (sfast ? blockIdx.x : blockIdx.y) * SB + s;
  const bool live = sg < S;
  load_twiddles<N, DIR>(tw, tid, NT);
  for (int y = tid; y < N; y += NT) {
    const bool iv = imap || (y % istride == 0 && y / istride < nin);
    const bool ov = omap || (y % ostride == 0 && y / ostride < nout);
    rin[y] = !iv ? -1 : imap ? imap[y * nh + m] : (y / istride) * nh + m;
    rout[y] = !ov ? -1 : omap ? omap[y * nh + m] : (y / ostride) * nh + m;
  }
  __syncthreads();
  if (t < N2) {
    float2 v[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int y = t + N2 * n1;
      v[n1] = (live && rin[y] >= 0) ? in[(size_t)rin[y] * rs + sg] : make_float2(0.f, 0.f);
    }
    dft<N1, DIR>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) ex[s * PAD + t * N1 + k1] = cmul(v[k1], tw[t * k1]);
  }
  __syncthreads();
  float2 v[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) v[n2] = ex[s * PAD + n2 * N1 + t];
  dft<N2, DIR>(v);
  if (live) {
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int p = t + N1 * k2;
      if (rout[p] >= 0) out[(size_t)rout[p] * rs + sg] = v[k2];
    }
  }
}

// ---------------------------------------------------------- rows, r2c (x)
// Forward transforms of a block's Q packed sequences, in LDS at
// ex[q * PAD + n] = f[2q][n] + i f[2q+1][n] (n < N, written before a
// barrier; tw holds the forward twiddles), and the stores of the two real
// half spectra of each, slice-fastest: T[(j*NH + m)*rs + s0 + sl].
template <int N, int Q>
__device__ __forceinline__ void r2c_rows_from_lds(float2* ex, const float2* tw, float2* __restrict__ T,
                                                  int j, int s0, int S, int rs) {
  constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
  constexpr int PX = Split<N>::N1 + 1;
  constexpr int PAD = Split<N>::N2 * PX + 1;
  constexpr int NT = Q * N1;
  constexpr int NH = N / 2 + 1;
  const int tid = threadIdx.x;
  const int t = tid % N1, q = tid / N1;
  float2 v[N1];
  if (t < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = ex[q * PAD + t + N2 * n1];
  }
  __syncthreads();
  if (t < N2) {
    dft<N1, -1>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) ex[q * PAD + t * PX + k1] = cmul(v[k1], tw[t * k1]);
  }
  __syncthreads();
  float2 w[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) w[n2] = ex[q * PAD + n2 * PX + t];
  dft<N2, -1>(w);
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) ex[q * PAD + t + N1 * k2] = w[k2];
  __syncthreads();
  // separate the two packed real transforms and store slice-fastest
  for (int idx = tid; idx < NH * 2 * Q; idx += NT) {
    const int m = idx / (2 * Q), sl = idx % (2 * Q);
    const int s = s0 + sl;
    if (s >= S) continue;
    const int qq = sl >> 1;
    const float2 zm = ex[qq * PAD + m];
    const float2 zc = cconj(ex[qq * PAD + (m == 0 ? 0 : N - m)]);
    float2 r;
    if ((sl & 1) == 0) {
      r = make_float2(0.5f * (zm.x + zc.x), 0.5f * (zm.y + zc.y));
    } else {
      const float2 d = csub(zm, zc);
      r = make_float2(0.5f * d.y, -0.5f * d.x);
    }
    T[(size_t)(j * NH + m) * rs + s] = r;
  }
}

// T[(j*nh + m)*rs + s] = sum_{i < nxc} exp(-2 pi i m sx i / N) f[s][j][i],  m = 0..N/2,
// for the ny rows j of slices f[s][ny][nxc]: sample i sits at transform
// column sx*i, every other column of the length-N row is zero
// The 2Q rows of a block are read with 16-byte loads into LDS, packed in
// pairs as z = f[2q] + i f[2q+1]; after the transform the two real spectra are
// separated and written slice-fastest (contiguous across threads).
// GEN: rows of any length (element loads) or scan-grid sampling; the common
// case (16-byte aligned rows, every column) compiles to plain vector loads
template <int N, int Q, bool GEN>  // Q packed complex sequences = 2Q real slices per block
__global__ __launch_bounds__(256) void k_fft_rows_r2c(const float* __restrict__ f,
                                                      float2* __restrict__ T, int ny, int nxd,
                                                      int sx, int S, int rs, int tj) {
  constexpr int N1 = Split<N>::N1;
  // per packed sequence: N values in natural order, or the N2 x N1 exchange
  // with rows padded to N1 + 1 (lanes write their N1 outputs to separate banks)
  constexpr int PX = Split<N>::N1 + 1;
  constexpr int PAD = Split<N>::N2 * PX + 1;
  constexpr int NT = Q * N1;
  __shared__ float2 tw[N];
  __shared__ float2 ex[Q * PAD];
  const int tid = threadIdx.x;
  int j, sb;
  row_block(tj, j, sb);
  const int s0 = sb * 2 * Q;
  load_twiddles<N, -1>(tw, tid, NT);
  // rows of the block: 2Q rows x N/4 float4, every load issued before any LDS
  // store; adjacent lanes take the two rows of a packed pair at the same
  // column (their re and im floats are adjacent in LDS: few bank conflicts),
  // and each row is still read as whole lines across the wave
  constexpr int LIT = (2 * Q * (N / 4) + NT - 1) / NT;
  float4 ld[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int u = tid + it * NT;
    const int row = 2 * (u / (N / 2)) + (u & 1), c4 = (u % (N / 2)) >> 1;
    const int s = s0 + row;
    ld[it] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (u < 2 * Q * (N / 4) && s < S && 4 * c4 < nxd) {
      const float* src = f + ((size_t)s * ny + j) * nxd;
      if (!GEN || (nxd & 3) == 0) {
        ld[it] = reinterpret_cast<const float4*>(src)[c4];
      } else {  // rows not 16-byte aligned: element loads, zeros past the row
        const int i0 = 4 * c4;
        ld[it].x = src[i0];
        if (i0 + 1 < nxd) ld[it].y = src[i0 + 1];
        if (i0 + 2 < nxd) ld[it].z = src[i0 + 2];
        if (i0 + 3 < nxd) ld[it].w = src[i0 + 3];
      }
    }
  }
  if (GEN && sx > 1) {  // samples land sx columns apart: clear the row buffers first
    for (int e = tid; e < Q * PAD; e += NT) ex[e] = make_float2(0.f, 0.f);
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int u = tid + it * NT;
    if (u >= 2 * Q * (N / 4)) break;
    const int row = 2 * (u / (N / 2)) + (u & 1), c4 = (u % (N / 2)) >> 1;
    if (!GEN || sx == 1) {
      float* z = reinterpret_cast<float*>(ex + (row >> 1) * PAD + 4 * c4) + (row & 1);
      z[0] = ld[it].x;
      z[2] = ld[it].y;
      z[4] = ld[it].z;
      z[6] = ld[it].w;
    } else if (4 * c4 < nxd) {
      float* z = reinterpret_cast<float*>(ex + (row >> 1) * PAD) + (row & 1);
      const int i0 = 4 * c4 * sx;
      z[2 * i0] = ld[it].x;
      if (4 * c4 + 1 < nxd) z[2 * (i0 + sx)] = ld[it].y;
      if (4 * c4 + 2 < nxd) z[2 * (i0 + 2 * sx)] = ld[it].z;
      if (4 * c4 + 3 < nxd) z[2 * (i0 + 3 * sx)] = ld[it].w;
    }
  }
  __syncthreads();
  r2c_rows_from_lds<N, Q>(ex, tw, T, j, s0, S, rs);
}

// ---------------------------------------------------------- rows, c2r (x)
// LDS of the c2r row kernels: twiddles, and one buffer for the half spectra,
// the exchange between the two DFT stages and the real rows
template <int N, int Q>
struct C2rLds {
  static constexpr int NH = N / 2 + 1;
  static constexpr int PAD = Split<N>::N2 * (Split<N>::N1 + 1) + 1;
  static constexpr int BUF0 = (2 * Q * NH > Q * PAD) ? 2 * Q * NH : Q * PAD;
  static constexpr int BUF = (BUF0 * 2 > 2 * Q * (N + 4)) ? BUF0 : (2 * Q * (N + 4) + 1) / 2;
};

// Unscaled inverse transforms of row j of the block's 2Q half-spectrum
// slices s0 .. s0+2Q-1 (F Hermitian-extended from m = 0..N/2, imaginary
// parts of m = 0, N/2 dropped); on return (after a barrier) real row sl is
// in LDS at rows[sl * (N + 4)].
template <int N, int Q>
__device__ __forceinline__ float* c2r_rows_to_lds(const float2* __restrict__ T, int j, int s0, int S,
                                                  int rs, float2* tw, float2* buf) {
  constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
  constexpr int PX = Split<N>::N1 + 1;  // exchange row stride, see k_fft_rows_r2c
  constexpr int PAD = Split<N>::N2 * PX + 1;
  constexpr int NT = Q * N1;
  constexpr int NH = N / 2 + 1;
  const int tid = threadIdx.x;
  constexpr int LIT = (NH * 2 * Q + NT - 1) / NT;
  float2 ld[LIT];
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    const int m = idx / (2 * Q), sl = idx % (2 * Q);
    const int s = s0 + sl;
    ld[it] = (idx < NH * 2 * Q && s < S) ? T[(size_t)(j * NH + m) * rs + s] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int it = 0; it < LIT; ++it) {
    const int idx = tid + it * NT;
    if (idx >= NH * 2 * Q) break;
    const int m = idx / (2 * Q), sl = idx % (2 * Q);
    float2 F = ld[it];
    if (m == 0 || m == N / 2) F.y = 0.f;
    buf[sl * NH + m] = F;
  }
  load_twiddles<N, +1>(tw, tid, NT);
  __syncthreads();
  const int t = tid % N1, q = tid / N1;
  float2 v[N1];
  if (t < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int i = t + N2 * n1;
      float2 fa, fb;
      if (i <= N / 2) {
        fa = buf[(2 * q) * NH + i];
        fb = buf[(2 * q + 1) * NH + i];
      } else {
        fa = cconj(buf[(2 * q) * NH + N - i]);
        fb = cconj(buf[(2 * q + 1) * NH + N - i]);
      }
      v[n1] = make_float2(fa.x - fb.y, fa.y + fb.x);  // Fa + i Fb
    }
    dft<N1, +1>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmul(v[k1], tw[t * k1]);
  }
  __syncthreads();
  if (t < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) buf[q * PAD + t * PX + k1] = v[k1];
  }
  __syncthreads();
  float2 w[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) w[n2] = buf[q * PAD + n2 * PX + t];
  dft<N2, +1>(w);
  __syncthreads();
  // real rows 2q (re) and 2q+1 (im) into LDS, then 16-byte row stores
  float* rows = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) {
    const int i = t + N1 * k2;
    rows[(2 * q) * (N + 4) + i] = w[k2].x;
    rows[(2 * q + 1) * (N + 4) + i] = w[k2].y;
  }
  __syncthreads();
  return rows;
}

// f[s][j][i] = scale * sum_{m=0}^{N-1} exp(+2 pi i m i / N) F[m] - sub[s][j][i],
// stored for the samples i = 0..nxc-1 at transform columns sx*i (slices
// f[s][ny][nxc]; the rest of the period is not stored)
template <int N, int Q, bool GEN>
__global__ __launch_bounds__(256) void k_fft_rows_c2r(const float2* __restrict__ T,
                                                      float* __restrict__ f, int ny, int nxd,
                                                      int sx, int S, int rs, float scale,
                                                      const float* __restrict__ sub, int tj) {
  constexpr int NT = Q * Split<N>::N1;
  __shared__ float2 tw[N];
  __shared__ float2 buf[C2rLds<N, Q>::BUF];
  const int tid = threadIdx.x;
  int j, sb;
  row_block(tj, j, sb);
  const int s0 = sb * 2 * Q;
  float* rows = c2r_rows_to_lds<N, Q>(T, j, s0, S, rs, tw, buf);
  constexpr int SIT = (2 * Q * (N / 4) + NT - 1) / NT;
  float4 sb4[SIT];
  if (sub) {
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int u = tid + it * NT;
      const int row = u / (N / 4), c4 = u % (N / 4);
      const int s = s0 + row;
      sb4[it] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (u < 2 * Q * (N / 4) && s < S && 4 * c4 < nxd) {
        const float* src = sub + ((size_t)s * ny + j) * nxd;
        if (!GEN || (nxd & 3) == 0) {
          sb4[it] = reinterpret_cast<const float4*>(src)[c4];
        } else {
          const int i0 = 4 * c4;
          sb4[it].x = src[i0];
          if (i0 + 1 < nxd) sb4[it].y = src[i0 + 1];
          if (i0 + 2 < nxd) sb4[it].z = src[i0 + 2];
          if (i0 + 3 < nxd) sb4[it].w = src[i0 + 3];
        }
      }
    }
  }
#pragma unroll
  for (int it = 0; it < SIT; ++it) {
    const int u = tid + it * NT;
    const int row = u / (N / 4), c4 = u % (N / 4);
    const int s = s0 + row;
    if (u >= 2 * Q * (N / 4) || s >= S || 4 * c4 >= nxd) continue;
    float4 r;
    const int i0 = 4 * c4;
    if (!GEN || sx == 1) {
      r = *reinterpret_cast<const float4*>(rows + row * (N + 4) + i0);
    } else {
      // samples past the row end read in-range LDS and are not stored
      const float* rr = rows + row * (N + 4);
      r = make_float4(rr[i0 * sx], rr[min(i0 + 1, nxd - 1) * sx], rr[min(i0 + 2, nxd - 1) * sx],
                      rr[min(i0 + 3, nxd - 1) * sx]);
    }
    float4 v = make_float4(r.x * scale, r.y * scale, r.z * scale, r.w * scale);
    if (sub) {
      v.x -= sb4[it].x;
      v.y -= sb4[it].y;
      v.z -= sb4[it].z;
      v.w -= sb4[it].w;
    }
    float* dst = f + ((size_t)s * ny + j) * nxd;
    if (!GEN || (nxd & 3) == 0) {
      reinterpret_cast<float4*>(dst)[c4] = v;
    } else {
      dst[i0] = v.x;
      if (i0 + 1 < nxd) dst[i0 + 1] = v.y;
      if (i0 + 2 < nxd) dst[i0 + 2] = v.z;
      if (i0 + 3 < nxd) dst[i0 + 3] = v.w;
    }
  }
}

// ------------------------------------------------- chirp-z (Bluestein) sizes
// A transform length N that is not among the fast sizes (even, 16..512) runs
// as a circular convolution of length M, a power of two >= 2N - 1.  With
// c[n] = exp(i pi n^2 / N):
//   forward  X[k] = conj(c[k]) sum_n (x[n] conj(c[n])) c[k - n]
//   inverse  x[n] = c[n] sum_k (X[k] c[k]) conj(c[n - k])
// (from 2nk = n^2 + k^2 - (k - n)^2).  The convolution is an M-point forward
// FFT, a product with the M-point DFT of the chirp kernel (tabulated on the
// host in float64 with 1/M folded in; the kernel is even, so the inverse
// direction uses its conjugate), and an M-point inverse FFT.

// In-place M-point FFT of one LDS sequence, natural order in and out; t <
// Split<M>::N1 is the thread's index within its sequence.  Every thread of the
// block calls it (it synchronises the block).
template <int M, int DIR>
__device__ __forceinline__ void lds_fft(float2* seq, const float2* tw, int t) {
  constexpr int N1 = Split<M>::N1, N2 = Split<M>::N2, PX = N1 + 1;
  float2 v[N1];
  if (t < N2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = seq[t + N2 * n1];
    dft<N1, DIR>(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = cmul(v[k1], DIR < 0 ? tw[t * k1] : cconj(tw[t * k1]));
  }
  __syncthreads();
  if (t < N2) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) seq[t * PX + k1] = v[k1];
  }
  __syncthreads();
  float2 w[N2];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) w[n2] = seq[n2 * PX + t];
  dft<N2, DIR>(w);
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < N2; ++k2) seq[t + N1 * k2] = w[k2];
  __syncthreads();
}

constexpr int kChirpMaxN = 512;  // longest chirp-z transform

// rows, r2c, length N by chirp-z: the 2Q real rows of slices s0.. at row j
// (f[s][ny][N]) packed in pairs as in k_fft_rows_r2c; T as there
template <int M, int Q>
__global__ __launch_bounds__(256) void k_fft_rows_r2c_cz(const float* __restrict__ f,
                                                         float2* __restrict__ T, int ny, int N,
                                                         int S, int rs, const float2* __restrict__ cz,
                                                         const float2* __restrict__ bz) {
  constexpr int N1 = Split<M>::N1, N2 = Split<M>::N2, PX = N1 + 1;
  constexpr int PAD = N2 * PX + 1;
  constexpr int NT = Q * N1;  // Q * M = N2 * NT elements, N2 per thread
  __shared__ float2 tw[M];
  __shared__ float2 ex[Q * PAD];
  const int tid = threadIdx.x;
  const int t = tid % N1, q = tid / N1;
  const int j = blockIdx.x;
  const int s0 = blockIdx.y * 2 * Q;
  const int NH = N / 2 + 1;
  load_twiddles<M, -1>(tw, tid, NT);
  float2 z[N2];
#pragma unroll
  for (int it = 0; it < N2; ++it) {
    const int e = tid + it * NT;
    const int qq = e / M, n = e % M;
    const int s = s0 + 2 * qq;
    float a = 0.f, b = 0.f;
    if (n < N) {
      if (s < S) a = f[((size_t)s * ny + j) * N + n];
      if (s + 1 < S) b = f[((size_t)(s + 1) * ny + j) * N + n];
    }
    z[it] = make_float2(a, b);
  }
#pragma unroll
  for (int it = 0; it < N2; ++it) {
    const int e = tid + it * NT;
    const int qq = e / M, n = e % M;
    ex[qq * PAD + n] = n < N ? cmul(z[it], cconj(cz[n])) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft<M, -1>(ex + q * PAD, tw, t);
  // pointwise passes: every table load of the pass issued before its first
  // use (Q * M = N2 * NT elements, N2 per thread)
  {
    float2 c[N2];
#pragma unroll
    for (int it = 0; it < N2; ++it) c[it] = bz[(tid + it * NT) % M];
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT, qq = e / M, n = e % M;
      ex[qq * PAD + n] = cmul(ex[qq * PAD + n], c[it]);
    }
  }
  __syncthreads();
  lds_fft<M, +1>(ex + q * PAD, tw, t);
  {
    float2 c[N2];
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT;
      c[it] = e < Q * N ? cz[e % N] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT;
      if (e < Q * N) {
        const int qq = e / N, n = e % N;
        ex[qq * PAD + n] = cmul(ex[qq * PAD + n], cconj(c[it]));
      }
    }
  }
  __syncthreads();
  // separate the two packed real transforms and store slice-fastest
  for (int idx = tid; idx < NH * 2 * Q; idx += NT) {
    const int m = idx / (2 * Q), sl = idx % (2 * Q);
    const int s = s0 + sl;
    if (s >= S) continue;
    const int qq = sl >> 1;
    const float2 zm = ex[qq * PAD + m];
    const float2 zc = cconj(ex[qq * PAD + (m == 0 ? 0 : N - m)]);
    float2 r;
    if ((sl & 1) == 0) {
      r = make_float2(0.5f * (zm.x + zc.x), 0.5f * (zm.y + zc.y));
    } else {
      const float2 d = csub(zm, zc);
      r = make_float2(0.5f * d.y, -0.5f * d.x);
    }
    T[(size_t)(j * NH + m) * rs + s] = r;
  }
}

// rows, c2r, length N by chirp-z: f = scale * (real rows of the Hermitian
// half spectra in T) - sub, as k_fft_rows_c2r without sampling
template <int M, int Q>
__global__ __launch_bounds__(256) void k_fft_rows_c2r_cz(const float2* __restrict__ T,
                                                         float* __restrict__ f, int ny, int N, int S,
                                                         int rs, float scale,
                                                         const float* __restrict__ sub,
                                                         const float2* __restrict__ cz,
                                                         const float2* __restrict__ bz) {
  constexpr int N1 = Split<M>::N1, N2 = Split<M>::N2, PX = N1 + 1;
  constexpr int PAD = N2 * PX + 1;
  constexpr int NT = Q * N1;
  constexpr int NHMAX = M / 4 + 1;  // N <= M / 2
  __shared__ float2 tw[M];
  __shared__ float2 ex[Q * PAD];
  __shared__ float2 hb[2 * Q * NHMAX];
  const int tid = threadIdx.x;
  const int t = tid % N1, q = tid / N1;
  const int j = blockIdx.x;
  const int s0 = blockIdx.y * 2 * Q;
  const int NH = N / 2 + 1;
  // every global load of a pass is issued before its first use: the half
  // spectra (N <= M / 2, so NH <= M / 4 + 1), then the tables c and the
  // kernel DFT, then c and the subtrahend of the output pass
  {
    constexpr int HIT = ((M / 4 + 1) * 2 * Q + NT - 1) / NT;
    float2 hv[HIT];
#pragma unroll
    for (int it = 0; it < HIT; ++it) {
      const int idx = tid + it * NT;
      const int m = idx / (2 * Q), sl = idx % (2 * Q);
      hv[it] = (idx < NH * 2 * Q && s0 + sl < S) ? T[(size_t)(j * NH + m) * rs + s0 + sl] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < HIT; ++it) {
      const int idx = tid + it * NT;
      if (idx < NH * 2 * Q) {
        const int m = idx / (2 * Q), sl = idx % (2 * Q);
        float2 F = hv[it];
        if (m == 0 || m == N / 2) F.y = 0.f;
        hb[sl * NH + m] = F;
      }
    }
  }
  load_twiddles<M, -1>(tw, tid, NT);
  __syncthreads();
  // z = Fa + i Fb over the full period (Hermitian extension), times c
  {
    float2 c[N2];
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int i = (tid + it * NT) % M;
      c[it] = i < N ? cz[i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT, qq = e / M, i = e % M;
      float2 v = make_float2(0.f, 0.f);
      if (i < N) {
        float2 fa, fb;
        if (i <= N / 2) {
          fa = hb[(2 * qq) * NH + i];
          fb = hb[(2 * qq + 1) * NH + i];
        } else {
          fa = cconj(hb[(2 * qq) * NH + N - i]);
          fb = cconj(hb[(2 * qq + 1) * NH + N - i]);
        }
        v = cmul(make_float2(fa.x - fb.y, fa.y + fb.x), c[it]);
      }
      ex[qq * PAD + i] = v;
    }
  }
  __syncthreads();
  lds_fft<M, -1>(ex + q * PAD, tw, t);
  {
    float2 c[N2];
#pragma unroll
    for (int it = 0; it < N2; ++it) c[it] = bz[(tid + it * NT) % M];
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT, qq = e / M, n = e % M;
      ex[qq * PAD + n] = cmul(ex[qq * PAD + n], cconj(c[it]));
    }
  }
  __syncthreads();
  lds_fft<M, +1>(ex + q * PAD, tw, t);
  // real rows 2q (re) and 2q+1 (im)
  {
    float2 c[N2], sv[N2];
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT;
      c[it] = sv[it] = make_float2(0.f, 0.f);
      if (e < Q * N) {
        const int qq = e / N, n = e % N;
        const int s = s0 + 2 * qq;
        c[it] = cz[n];
        if (sub) {
          if (s < S) sv[it].x = sub[((size_t)s * ny + j) * N + n];
          if (s + 1 < S) sv[it].y = sub[((size_t)(s + 1) * ny + j) * N + n];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < N2; ++it) {
      const int e = tid + it * NT;
      if (e >= Q * N) continue;
      const int qq = e / N, n = e % N;
      const int s = s0 + 2 * qq;
      const float2 v = cmul(ex[qq * PAD + n], c[it]);
      if (s < S) f[((size_t)s * ny + j) * N + n] = v.x * scale - sv[it].x;
      if (s + 1 < S) f[((size_t)(s + 1) * ny + j) * N + n] = v.y * scale - sv[it].y;
    }
  }
}

// columns, length N by chirp-z: out[orow(p)*rs + s] = sum_j exp(DIR 2 pi i p j / N)
// in[irow(j)*rs + s], maps as in k_fft_cols (full columns, no strides)
template <int M, int DIR>
__global__ __launch_bounds__(512) void k_fft_cols_cz(const float2* __restrict__ in,
                                                     float2* __restrict__ out, int nh, int S, int rs,
                                                     const int32_t* __restrict__ imap,
                                                     const int32_t* __restrict__ omap, int sfast,
                                                     int N, const float2* __restrict__ cz,
                                                     const float2* __restrict__ bz) {
  constexpr int N1 = Split<M>::N1, N2 = Split<M>::N2, PX = N1 + 1;
  constexpr int SB = 16;
  constexpr int PAD = N2 * PX + 1;
  constexpr int NT = SB * N1;
  __shared__ float2 tw[M];
  __shared__ float2 ex[SB * PAD];
  __shared__ int rin[kChirpMaxN], rout[kChirpMaxN];
  const int tid = threadIdx.x;
  const int s = tid % SB, t = tid / SB;
  const int m = sfast ? blockIdx.y : blockIdx.x;
  const int sg = (sfast ? blockIdx.x : blockIdx.y) * SB + s;
  const bool live = sg < S;
  load_twiddles<M, -1>(tw, tid, NT);
  for (int y = tid; y < N; y += NT) {
    rin[y] = imap ? imap[y * nh + m] : y * nh + m;
    rout[y] = omap ? omap[y * nh + m] : y * nh + m;
  }
  __syncthreads();
  float2 z[N2];  // y = t + N1 * i, i < N2 covers the period
#pragma unroll
  for (int i = 0; i < N2; ++i) {
    const int y = t + N1 * i;
    z[i] = (live && y < N && rin[y] >= 0) ? in[(size_t)rin[y] * rs + sg] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int i = 0; i < N2; ++i) {
    const int y = t + N1 * i;
    ex[s * PAD + y] = y < N ? cmul(z[i], DIR < 0 ? cconj(cz[y]) : cz[y]) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft<M, -1>(ex + s * PAD, tw, t);
#pragma unroll
  for (int i = 0; i < N2; ++i) {
    const int y = t + N1 * i;
    ex[s * PAD + y] = cmul(ex[s * PAD + y], DIR < 0 ? bz[y] : cconj(bz[y]));
  }
  __syncthreads();
  lds_fft<M, +1>(ex + s * PAD, tw, t);
  if (live) {
#pragma unroll
    for (int i = 0; i < N2; ++i) {
      const int p = t + N1 * i;
      if (p < N && rout[p] >= 0)
        out[(size_t)rout[p] * rs + sg] = cmul(ex[s * PAD + p], DIR < 0 ? cconj(cz[p]) : cz[p]);
    }
  }
}

// ------------------------------------------------------------- launchers
template <int N, int DIR>
static void launch_cols(const float2* in, float2* out, int nh, int S, int rs, const int32_t* imap,
                        const int32_t* omap, int nin, int istride, int nout, int ostride,
                        hipStream_t st) {
  constexpr int SB = ColSB<N>::value;
  const int sfast = S >= 2048;
  const int nsb = (S + SB - 1) / SB;
  dim3 grid = sfast ? dim3(nsb, nh) : dim3(nh, nsb);
  k_fft_cols<N, DIR><<<grid, SB * Split<N>::N1, 0, st>>>(in, out, nh, S, rs, imap, omap, sfast,
                                                         nin, istride, nout, ostride);
}

template <int DIR>
static pat_status cols(const float2* in, float2* out, int fy, int nh, int S, int rs,
                       const int32_t* imap, const int32_t* omap, int nin, int istride, int nout,
                       int ostride, hipStream_t st) {
#define PAT_COLS(N) launch_cols<N, DIR>(in, out, nh, S, rs, imap, omap, nin, istride, nout, ostride, st)
  switch (fy) {
#define PAT_CASE(N) \
    case N: PAT_COLS(N); break;
    PAT_FFT_SIZES(PAT_CASE)
#undef PAT_CASE
    default: return fail(PAT_EUNSUPPORTED, "transform size along y is not one of the FFT sizes");
  }
#undef PAT_COLS
  PAT_LAUNCHED("fft columns");
  return PAT_OK;
}

// Rows per tile of a row pass's block order.  The resident workgroups of a
// pass over 2,048 slices or more (batches) cover 4 rows of many slice blocks
// at a time instead of every row of a few slice blocks: the spectrum side's
// rows are then written in long runs (measured: B = 16 object-pairs +1.5 %
// with 4 rows per tile, +1 % with 1 or 16); fewer slices keep the row-major
// order (the whole pass fits a few rounds of workgroups).
static int row_tile(int nyc, int S) { return S >= 2048 ? 4 : nyc; }

template <int N, int Q>
static void rows_r2c(const float* f, float2* T, int nyc, int nxc, int sx, int S, int rs,
                     hipStream_t st) {
  dim3 grid(nyc, (S + 2 * Q - 1) / (2 * Q));
  const int tj = row_tile(nyc, S);
  if (sx == 1 && (nxc & 3) == 0)
    k_fft_rows_r2c<N, Q, false><<<grid, Q * Split<N>::N1, 0, st>>>(f, T, nyc, nxc, sx, S, rs, tj);
  else
    k_fft_rows_r2c<N, Q, true><<<grid, Q * Split<N>::N1, 0, st>>>(f, T, nyc, nxc, sx, S, rs, tj);
}

// The same inverse transform with the FISTA update as its epilogue: the
// transform is the gradient g = scale * c2r(X) - sub of slice s, of object
// b = s / per_obj (every row block lies inside one object), and on the
// stored columns (nxd of them, whole 16-byte units)
//     x_old = x; x = prox(z - tau_b g); z = x + beta_b (x - x_old)
// exactly as k_fista_update, without storing g.  NEXT: the block then runs
// the next iteration's forward row pass on its rows of the new z (zero past
// nxd), Tn[(j*NH + m)*rs + s] as k_fft_rows_r2c writes it; Tn may be T (the
// block rewrites exactly the entries it read).
template <int N, int Q, bool NEXT>
__global__ __launch_bounds__(256) void k_fft_rows_c2r_fista(const float2* T, float* __restrict__ z,
                                                            float* __restrict__ x, int ny, int nxd, int S,
                                                            int rs, float scale, const float* __restrict__ sub,
                                                            int per_obj, FistaBatch p,
                                                            int32_t* __restrict__ nonfinite, float2* Tn) {
  constexpr int NT = Q * Split<N>::N1;
  constexpr int SIT = (2 * Q * (N / 4) + NT - 1) / NT;
  __shared__ float2 tw[N];
  __shared__ float2 buf[C2rLds<N, Q>::BUF];
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const int s0 = blockIdx.y * 2 * Q;
  const int ob = s0 / per_obj;
  const FistaObj o = p.o[ob];
  float* rows = c2r_rows_to_lds<N, Q>(T, j, s0, S, rs, tw, buf);
  // the update's operands, all loads issued before the first use
  float4 zz[SIT], xx[SIT], sb[SIT];
#pragma unroll
  for (int it = 0; it < SIT; ++it) {
    const int u = tid + it * NT;
    const int row = u / (N / 4), c4 = u % (N / 4);
    const int s = s0 + row;
    zz[it] = xx[it] = sb[it] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (u < 2 * Q * (N / 4) && s < S && 4 * c4 < nxd) {
      const size_t off = ((size_t)s * ny + j) * nxd + 4 * c4;
      zz[it] = *reinterpret_cast<const float4*>(z + off);
      xx[it] = *reinterpret_cast<const float4*>(x + off);
      if (sub) sb[it] = *reinterpret_cast<const float4*>(sub + off);
    }
  }
  auto upd = [&](float r, float sv, float zv, float xo, float& xn, float& zn) {
    const float g = r * scale - sv;
    const float v = zv - o.tau * g;
    if (o.nonneg) {
      xn = fmaxf(v - o.thr, 0.f);
    } else {
      const float m = fmaxf(fabsf(v) - o.thr, 0.f);
      xn = copysignf(m, v);
    }
    zn = xn + o.beta * (xn - xo);
  };
  bool bad = false;
#pragma unroll
  for (int it = 0; it < SIT; ++it) {
    const int u = tid + it * NT;
    const int row = u / (N / 4), c4 = u % (N / 4);
    const int s = s0 + row;
    if (u >= 2 * Q * (N / 4) || s >= S || 4 * c4 >= nxd) {
      zz[it] = make_float4(0.f, 0.f, 0.f, 0.f);  // the next row pass sees zeros there
      continue;
    }
    const float4 r = *reinterpret_cast<const float4*>(rows + row * (N + 4) + 4 * c4);
    float4 xn, zn;
    upd(r.x, sb[it].x, zz[it].x, xx[it].x, xn.x, zn.x);
    upd(r.y, sb[it].y, zz[it].y, xx[it].y, xn.y, zn.y);
    upd(r.z, sb[it].z, zz[it].z, xx[it].z, xn.z, zn.z);
    upd(r.w, sb[it].w, zz[it].w, xx[it].w, xn.w, zn.w);
    bad |= !(isfinite(xn.x) && isfinite(xn.y) && isfinite(xn.z) && isfinite(xn.w));
    const size_t off = ((size_t)s * ny + j) * nxd + 4 * c4;
    *reinterpret_cast<float4*>(x + off) = xn;
    *reinterpret_cast<float4*>(z + off) = zn;
    zz[it] = zn;
  }
  if (bad && nonfinite) nonfinite[ob] = 1;
  if constexpr (NEXT) {
    // rows of the new z into LDS, packed in pairs as k_fft_rows_r2c packs
    // them (the buffer is free once every thread has read its rows)
    constexpr int PAD = C2rLds<N, Q>::PAD;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int u = tid + it * NT;
      if (u >= 2 * Q * (N / 4)) break;
      const int row = u / (N / 4), c4 = u % (N / 4);
      float* zp = reinterpret_cast<float*>(buf + (row >> 1) * PAD + 4 * c4) + (row & 1);
      zp[0] = zz[it].x;
      zp[2] = zz[it].y;
      zp[4] = zz[it].z;
      zp[6] = zz[it].w;
    }
    load_twiddles<N, -1>(tw, tid, NT);
    __syncthreads();
    r2c_rows_from_lds<N, Q>(buf, tw, Tn, j, s0, S, rs);
  }
}

template <int N, int Q>
static void rows_c2r(const float2* T, float* f, int nyc, int nxc, int sx, int S, int rs, float scale,
                     const float* sub, hipStream_t st) {
  dim3 grid(nyc, (S + 2 * Q - 1) / (2 * Q));
  const int tj = row_tile(nyc, S);
  if (sx == 1 && (nxc & 3) == 0)
    k_fft_rows_c2r<N, Q, false><<<grid, Q * Split<N>::N1, 0, st>>>(T, f, nyc, nxc, sx, S, rs, scale, sub, tj);
  else
    k_fft_rows_c2r<N, Q, true><<<grid, Q * Split<N>::N1, 0, st>>>(T, f, nyc, nxc, sx, S, rs, scale, sub, tj);
}

template <int N, int Q>
static void rows_c2r_fista(const float2* T, float* z, float* x, int nyc, int nxc, int S, int rs,
                           float scale, const float* sub, int per_obj, const FistaBatch& p,
                           int32_t* nonfinite, float2* Tn, hipStream_t st) {
  dim3 grid(nyc, (S + 2 * Q - 1) / (2 * Q));
  if (Tn)
    k_fft_rows_c2r_fista<N, Q, true><<<grid, Q * Split<N>::N1, 0, st>>>(T, z, x, nyc, nxc, S, rs, scale, sub,
                                                                       per_obj, p, nonfinite, Tn);
  else
    k_fft_rows_c2r_fista<N, Q, false><<<grid, Q * Split<N>::N1, 0, st>>>(T, z, x, nyc, nxc, S, rs, scale, sub,
                                                                        per_obj, p, nonfinite, nullptr);
}

// 8 packed sequences (16 real slices) per row block: small enough for several
// resident workgroups per CU, large enough for full 16-byte row loads
constexpr int kRowQ = 8;
#define PAT_ROWS(fn, N, ...) (fn<N, kRowQ>(__VA_ARGS__))

static bool extents_ok(int fx, int fy, int nxw, int nyw, int sx, int sy) {
  if (sx < 1 || sy < 1 || nxw > fx || nyw > fy || nxw % sx || nyw % sy) return false;
  return nxw / sx >= 1 && nyw / sy >= 1;
}

template <int M, int Q>
static void rows_r2c_cz(const float* f, float2* T, int ny, int N, int S, int rs, const float2* cz,
                        const float2* bz, hipStream_t st) {
  dim3 grid(ny, (S + 2 * Q - 1) / (2 * Q));
  k_fft_rows_r2c_cz<M, Q><<<grid, Q * Split<M>::N1, 0, st>>>(f, T, ny, N, S, rs, cz, bz);
}

template <int M, int Q>
static void rows_c2r_cz(const float2* T, float* f, int ny, int N, int S, int rs, float scale,
                        const float* sub, const float2* cz, const float2* bz, hipStream_t st) {
  dim3 grid(ny, (S + 2 * Q - 1) / (2 * Q));
  k_fft_rows_c2r_cz<M, Q><<<grid, Q * Split<M>::N1, 0, st>>>(T, f, ny, N, S, rs, scale, sub, cz, bz);
}

template <int M, int DIR>
static void launch_cols_cz(const float2* in, float2* out, int nh, int S, int rs, const int32_t* imap,
                           const int32_t* omap, int N, const float2* cz, const float2* bz,
                           hipStream_t st) {
  constexpr int SB = 16;
  const int sfast = S >= 2048;
  const int nsb = (S + SB - 1) / SB;
  dim3 grid = sfast ? dim3(nsb, nh) : dim3(nh, nsb);
  k_fft_cols_cz<M, DIR><<<grid, SB * Split<M>::N1, 0, st>>>(in, out, nh, S, rs, imap, omap, sfast, N,
                                                            cz, bz);
}

#define PAT_CHIRP_M(X) X(64) X(128) X(256) X(512) X(1024)

template <int DIR>
static pat_status cols_cz(const float2* in, float2* out, int fy, int nh, int S, int rs,
                          const int32_t* imap, const int32_t* omap, const float2* cz, const float2* bz,
                          int M, hipStream_t st) {
  if (fy > kChirpMaxN || 2 * fy - 1 > M) return fail(PAT_EINVAL, "chirp-z: table length does not fit");
  switch (M) {
#define PAT_CASE(MM) \
    case MM: launch_cols_cz<MM, DIR>(in, out, nh, S, rs, imap, omap, fy, cz, bz, st); break;
    PAT_CHIRP_M(PAT_CASE)
#undef PAT_CASE
    default: return fail(PAT_EUNSUPPORTED, "chirp-z convolution length must be a power of two in [64, 1024]");
  }
  PAT_LAUNCHED("fft columns (chirp-z)");
  return PAT_OK;
}

pat_status fft2_r2c(const float* f, float2* T, float2* X, int fx, int fy, int nxw, int nyw, int sx,
                    int sy, int S, const int32_t* rowmap, const FftChirp& ch, hipStream_t st) {
  if (S <= 0) return PAT_OK;
  if (!extents_ok(fx, fy, nxw, nyw, sx, sy))
    return fail(PAT_EINVAL, "fft: data extent or sampling does not fit the transform");
  const int nh = fx / 2 + 1;
  const int rs = spec_stride(S);
  const int nxc = nxw / sx, nyc = nyw / sy;
  if ((ch.mx && (nxw != fx || sx != 1)) || (ch.my && (nyw != fy || sy != 1)))
    return fail(PAT_EUNSUPPORTED, "fft: chirp-z axes take whole, unsampled slices");
  if (ch.mx) {
    if (fx > kChirpMaxN || 2 * fx - 1 > ch.mx) return fail(PAT_EINVAL, "chirp-z: table length does not fit");
    switch (ch.mx) {
#define PAT_CASE(MM) \
      case MM: rows_r2c_cz<MM, kRowQ>(f, T, nyc, fx, S, rs, ch.cx, ch.bx, st); break;
      PAT_CHIRP_M(PAT_CASE)
#undef PAT_CASE
      default: return fail(PAT_EUNSUPPORTED, "chirp-z convolution length must be a power of two in [64, 1024]");
    }
    PAT_LAUNCHED("fft rows r2c (chirp-z)");
    if (ch.my) return cols_cz<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, ch.cy, ch.by, ch.my, st);
    return cols<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, nyc, sy, fy, 1, st);
  }
  switch (fx) {
#define PAT_CASE(N) \
    case N: PAT_ROWS(rows_r2c, N, f, T, nyc, nxc, sx, S, rs, st); break;
    PAT_FFT_SIZES(PAT_CASE)
#undef PAT_CASE
    default: return fail(PAT_EUNSUPPORTED, "transform size along x is not one of the FFT sizes");
  }
  PAT_LAUNCHED("fft rows r2c");
  if (ch.my) return cols_cz<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, ch.cy, ch.by, ch.my, st);
  return cols<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, nyc, sy, fy, 1, st);
}

pat_status fft2_c2r(const float2* X, float2* T, float* f, int fx, int fy, int nxw, int nyw, int sx,
                    int sy, int S, float scale, const float* sub, const int32_t* rowmap,
                    const FftChirp& ch, hipStream_t st) {
  if (S <= 0) return PAT_OK;
  if (!extents_ok(fx, fy, nxw, nyw, sx, sy))
    return fail(PAT_EINVAL, "fft: data extent or sampling does not fit the transform");
  const int nh = fx / 2 + 1;
  const int rs = spec_stride(S);
  const int nxc = nxw / sx, nyc = nyw / sy;
  if ((ch.mx && (nxw != fx || sx != 1)) || (ch.my && (nyw != fy || sy != 1)))
    return fail(PAT_EUNSUPPORTED, "fft: chirp-z axes take whole, unsampled slices");
  if (ch.my)
    PAT_TRY(cols_cz<+1>(X, T, fy, nh, S, rs, rowmap, nullptr, ch.cy, ch.by, ch.my, st));
  else
    PAT_TRY(cols<+1>(X, T, fy, nh, S, rs, rowmap, nullptr, fy, 1, nyc, sy, st));
  if (ch.mx) {
    if (fx > kChirpMaxN || 2 * fx - 1 > ch.mx) return fail(PAT_EINVAL, "chirp-z: table length does not fit");
    switch (ch.mx) {
#define PAT_CASE(MM) \
      case MM: rows_c2r_cz<MM, kRowQ>(T, f, nyc, fx, S, rs, scale, sub, ch.cx, ch.bx, st); break;
      PAT_CHIRP_M(PAT_CASE)
#undef PAT_CASE
      default: return fail(PAT_EUNSUPPORTED, "chirp-z convolution length must be a power of two in [64, 1024]");
    }
    PAT_LAUNCHED("fft rows c2r (chirp-z)");
    return PAT_OK;
  }
  switch (fx) {
#define PAT_CASE(N) \
    case N: PAT_ROWS(rows_c2r, N, T, f, nyc, nxc, sx, S, rs, scale, sub, st); break;
    PAT_FFT_SIZES(PAT_CASE)
#undef PAT_CASE
    default: return fail(PAT_EUNSUPPORTED, "transform size along x is not one of the FFT sizes");
  }
  PAT_LAUNCHED("fft rows c2r");
  return PAT_OK;
}


pat_status fft2_r2c_cols(const float2* T, float2* X, int fx, int fy, int nyw, int S, const int32_t* rowmap,
                         const FftChirp& ch, hipStream_t st) {
  if (S <= 0) return PAT_OK;
  if (nyw < 1 || nyw > fy || (ch.my && nyw != fy))
    return fail(PAT_EINVAL, "fft: data extent does not fit the transform");
  const int nh = fx / 2 + 1;
  const int rs = spec_stride(S);
  if (ch.my) return cols_cz<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, ch.cy, ch.by, ch.my, st);
  return cols<-1>(T, X, fy, nh, S, rs, nullptr, rowmap, nyw, 1, fy, 1, st);
}

bool fft2_c2r_fista_ok(int nxw, const FftChirp& ch, int S, int per_obj) {
  return !ch.mx && (nxw & 3) == 0 && per_obj >= 1 && (S == per_obj || per_obj % (2 * kRowQ) == 0);
}

pat_status fft2_c2r_fista(const float2* X, float2* T, float* z, float* x, int fx, int fy, int nxw,
                          int nyw, int S, int per_obj, float scale, const float* sub,
                          const int32_t* rowmap, const FftChirp& ch, const FistaBatch& p,
                          int32_t* nonfinite, float2* Tnext, hipStream_t st) {
  if (S <= 0) return PAT_OK;
  if (!extents_ok(fx, fy, nxw, nyw, 1, 1))
    return fail(PAT_EINVAL, "fft: data extent does not fit the transform");
  if (!fft2_c2r_fista_ok(nxw, ch, S, per_obj))
    return fail(PAT_EUNSUPPORTED, "fft: the fused update needs a fast x axis, rows of whole 16-byte "
                                  "units and row blocks inside one object");
  const int nh = fx / 2 + 1;
  const int rs = spec_stride(S);
  if (ch.my && nyw != fy) return fail(PAT_EUNSUPPORTED, "fft: chirp-z axes take whole, unsampled slices");
  if (ch.my)
    PAT_TRY(cols_cz<+1>(X, T, fy, nh, S, rs, rowmap, nullptr, ch.cy, ch.by, ch.my, st));
  else
    PAT_TRY(cols<+1>(X, T, fy, nh, S, rs, rowmap, nullptr, fy, 1, nyw, 1, st));
  switch (fx) {
#define PAT_CASE(N) \
    case N: PAT_ROWS(rows_c2r_fista, N, T, z, x, nyw, nxw, S, rs, scale, sub, per_obj, p, nonfinite, Tnext, st); break;
    PAT_FFT_SIZES(PAT_CASE)
#undef PAT_CASE
    default: return fail(PAT_EUNSUPPORTED, "transform size along x is not one of the FFT sizes");
  }
  PAT_LAUNCHED("fft rows c2r + FISTA update");
  return PAT_OK;
}

}  // namespace pat
