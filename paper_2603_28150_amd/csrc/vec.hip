// Element-wise and reduction kernels around the operator: buffer clearing,
// dot products (float32 tree sums; float64 for the adjoint check only),
// normalisation for the power iteration, and the fused FISTA update
// (proximal step of Sec. 2.3 plus the momentum extrapolation).
#include "pat_internal.hpp"

namespace pat {

__global__ void k_fill_zero(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

pat_status fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return PAT_OK;
  const size_t n16 = bytes / 16;
  int blocks = (int)((n16 + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_fill_zero<<<blocks, 256, 0, st>>>(reinterpret_cast<uint4*>(p), n16,
                                      reinterpret_cast<unsigned char*>(p) + n16 * 16, bytes % 16);
  PAT_LAUNCHED("fill");
  return PAT_OK;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot_part(const float* __restrict__ a,
                                                  const float* __restrict__ b, long long n,
                                                  T* __restrict__ part) {
  __shared__ T sh[256];
  T s = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    s += (T)a[i] * (T)b[i];
  const T tot = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot_final(const T* __restrict__ part, int np,
                                                   T* __restrict__ result, T post) {
  __shared__ T sh[256];
  T s = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  const T tot = block_sum(s, sh);
  if (threadIdx.x == 0) result[0] = tot * post;
}

pat_status dot_f32(const float* a, const float* b, long long n, float* part, float* result,
                   float post_scale, hipStream_t st) {
  k_dot_part<float><<<kRedBlocks, 256, 0, st>>>(a, b, n, part);
  PAT_LAUNCHED("dot partials");
  k_dot_final<float><<<1, 256, 0, st>>>(part, kRedBlocks, result, post_scale);
  PAT_LAUNCHED("dot final");
  return PAT_OK;
}

pat_status dot_f64(const float* a, const float* b, long long n, double* part, double* result,
                   hipStream_t st) {
  k_dot_part<double><<<kRedBlocks, 256, 0, st>>>(a, b, n, part);
  PAT_LAUNCHED("dot64 partials");
  k_dot_final<double><<<1, 256, 0, st>>>(part, kRedBlocks, result, 1.0);
  PAT_LAUNCHED("dot64 final");
  return PAT_OK;
}

__global__ void k_scale_rsqrt(float* __restrict__ dst, const float* __restrict__ src, long long n,
                              const float* __restrict__ nrm2) {
  const float s = 1.0f / sqrtf(nrm2[0]);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i] * s;
}

pat_status scale_rsqrt(float* dst, const float* src, long long n, const float* nrm2,
                       hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_scale_rsqrt<<<(int)blocks, 256, 0, st>>>(dst, src, n, nrm2);
  PAT_LAUNCHED("normalise");
  return PAT_OK;
}

__global__ void k_trace_combine(float* out, const double* s) {
  out[0] = (float)(0.5 * (s[0] - s[1] + s[2]));
}

pat_status trace_combine(float* out, const double* s, hipStream_t st) {
  k_trace_combine<<<1, 1, 0, st>>>(out, s);
  PAT_LAUNCHED("trace");
  return PAT_OK;
}

// x_old = x; v = z - tau g; x = prox(v); z = x + beta (x - x_old)
__global__ __launch_bounds__(256) void k_fista_update(float* __restrict__ x, float* __restrict__ z,
                                                      const float* __restrict__ g,
                                                      long long n_per_obj, FistaBatch p,
                                                      int32_t* __restrict__ nonfinite) {
  const int b = blockIdx.y;
  const FistaObj o = p.o[b];
  float* xb = x + (size_t)b * n_per_obj;
  float* zb = z + (size_t)b * n_per_obj;
  const float* gb = g + (size_t)b * n_per_obj;
  bool bad = false;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_per_obj; i += stride) {
    const float xo = xb[i];
    const float v = zb[i] - o.tau * gb[i];
    float xn;
    if (o.nonneg) {
      xn = fmaxf(v - o.thr, 0.f);
    } else {
      const float m = fmaxf(fabsf(v) - o.thr, 0.f);
      xn = copysignf(m, v);
    }
    bad |= !isfinite(xn);
    xb[i] = xn;
    zb[i] = xn + o.beta * (xn - xo);
  }
  if (bad && nonfinite) nonfinite[b] = 1;
}

pat_status fista_update(float* x, float* z, const float* g, long long n_per_obj, int B,
                        const FistaBatch& p, int32_t* nonfinite, hipStream_t st) {
  long long blocks = (n_per_obj + 1023) / 1024;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  dim3 grid((unsigned)blocks, B);
  k_fista_update<<<grid, 256, 0, st>>>(x, z, g, n_per_obj, p, nonfinite);
  PAT_LAUNCHED("fista update");
  return PAT_OK;
}

}  // namespace pat
