/*
 * pat.h -- C ABI of the MI355X planar photoacoustic operator library (libpat.so).
 *
 * The library implements the depth-dependent, transverse shift-invariant
 * forward operator of arXiv 2603.28150 (Sec. 2.1-2.2, eq. 6-8),
 *
 *     d(r_perp, t_n) = sum_l  h_l(., t_n)  (*)_perp  x(., z_l)          (A)
 *
 * its adjoint for the Euclidean inner products (eq. 9-11),
 *
 *     g(r_perp, z_l) = sum_n  h_l(., t_n)  (star)_perp  d(., t_n)       (A^T)
 *
 * and the accelerated proximal-gradient (FISTA) solution of the inverse
 * problem of Sec. 2.3 (eq. 12-15),
 *
 *     x^ = argmin 1/2 ||A x - d||^2 + lambda ||x||_1 + i_{R+}(x).
 *
 * Both operators run as in the FFT realisation of Sec. 3.2: a 2D transverse
 * FFT of every input slice, a per-frequency multiply-accumulate against the
 * kernel library H^[k, l, n], and a 2D inverse FFT of every output slice.
 * The kernel library is built on the GPU from the exact discrete solution of
 * the homogeneous wave equation (eq. 1-2) on a grid periodic in x, y and z:
 *     H^[(m,p), l, n] = (1/nz_sim) sum_q cos(c t_n |k(m,p,q)|) exp(-2 pi i q l / nz_sim)
 * (real-valued; see pat_H_build).
 *
 * Conventions for every call:
 *  - Arrays are float32, C-contiguous with x fastest:
 *      objects  x [B][nz][ny][nx]      data  d [B][nt][ny][nx].
 *    Index l = 0 is the sensor plane (depth z_l = l*dz) and sample n is at
 *    time t_n = n*dt (n = 0 included).  The transverse boundary is periodic.
 *  - Device pointers must be 16-byte aligned; "device" means memory of the
 *    context's GPU.  The caller owns every buffer.  The library never
 *    allocates device memory: kernel-library storage and workspace come from
 *    the caller, sized by pat_H_bytes / pat_workspace_bytes.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *    only enqueues work on `stream` and returns, except the ones marked
 *    "synchronises", which return host scalars.
 *  - Errors are returned as pat_status; nothing is thrown across the ABI and
 *    nothing aborts.  pat_last_error() gives a message for the calling thread.
 *  - A pat_op is immutable after pat_H_build and may be used from several
 *    host threads and streams at once, each with its own workspace.
 */
#ifndef PAT_H_
#define PAT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pat_ctx pat_ctx; /* one GPU */
typedef struct pat_op pat_op;   /* one geometry + its kernel library */

typedef enum {
  PAT_OK = 0,
  PAT_EINVAL = -1,       /* bad argument: null/misaligned pointer, buffer too small, B < 1, ... */
  PAT_EUNSUPPORTED = -2, /* valid but unsupported: nx or ny outside the supported sizes, ... */
  PAT_ENOMEM = -3,       /* host allocation failed */
  PAT_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
  PAT_ENONFINITE = -5    /* a non-finite value was detected where a check was requested */
} pat_status;

/* Storage type of the kernel library.  FP32 is the plain operator.  The
 * 16-bit forms store H^ * s_l rounded to bfloat16 / float16 (nearest even,
 * via float32) with a per-depth power-of-two scale
 *     s_l = 2^(e - ceil(log2 max_{k,n} |H^[k,l,n]|)),  e = 0 (BF16), 15 (FP16),
 * and accumulate in float32; A pre-scales the depth spectrum by 1/s_l and
 * A^T post-scales it, so both use the same dequantised H^ and stay adjoint. */
typedef enum { PAT_H_F32 = 0, PAT_H_BF16 = 1, PAT_H_F16 = 2 } pat_hdtype;

/* Transverse boundary of the convolution.  PERIODIC: circular at nx x ny.
 * LINEAR: the zero-padded linear convolution of Sec. 2.3 (the object and the
 * data live on nx x ny; the transforms and the library are taken on the
 * px x py periodic grid, px the smallest transform size (see nx below)
 * >= max(16, 2 nx), and likewise py; the object is zero-padded and the data
 * cropped, so that A^T
 * stays the exact adjoint).  That library is the free-space response on the
 * nx x ny window as long as the wavefront does not travel round the period
 * within the record, c*dt*(nt-1) < (px-nx+1)*dx and (py-ny+1)*dy. */
typedef enum { PAT_BOUNDARY_PERIODIC = 0, PAT_BOUNDARY_LINEAR = 1 } pat_boundary;

typedef struct {
  int32_t nx, ny;  /* transverse grid (x fastest).  Periodic: the fast
                      transform sizes 16, 32, 48, 64, 72, 96, 108, 128, 144,
                      192, 216, 256, 288, 384, 432, 512, 576, 768, 864, 1024
                      (2^a 3^b, b <= 3), or any other even length in [16, 512]
                      (chirp-z transforms: a circular convolution of
                      power-of-two length >= 2n - 1; no scan-grid sampling
                      then).  Linear: any nx in [4, 512], ny in [1, 512] */
  int32_t nz, nt;  /* depths and time samples, >= 1 */
  double dx, dy, dz, dt, c; /* spacings [m], time step [s], sound speed [m/s]; all > 0 */
  int32_t nz_sim;  /* z-period of the simulated medium in grid points: 0 selects
                      the smallest power of two >= nz + ceil(c*dt*(nt-1)/dz) + 1,
                      otherwise it must be >= nz */
  int32_t h_dtype; /* pat_hdtype */
  int32_t boundary; /* pat_boundary */
  /* Temporal response of the sensors (the ideal point sensors of Sec. 2.1
   * when n_ir = 0): a causal FIR filter of n_ir <= 64 taps ir[0..n_ir-1]
   * (host float64, read by pat_H_bytes and pat_H_build only and copied into
   * the library), folded into the library along t:
   *     H^'[k, l, n] = sum_{j <= min(n, n_ir-1)} ir[j] H^[k, l, n-j],
   * so A returns the filtered data and A^T applies the matching correlation
   * at no cost per apply. */
  int32_t n_ir;
  const double* ir;
  /* Scan grid: the data are recorded at every sx-th column and sy-th row of
   * the nx x ny sensor grid (a sampling operator S after A, zero-filling S^T
   * before A^T), so data arrays are [nt][ny/sy][nx/sx].  sx must divide nx
   * with nx/sx a multiple of 4, sy must divide ny; 0 or 1: every point. */
  int32_t sx, sy;
  /* How pat_H_build computes the library (pat_build; 0 = closed form). */
  int32_t build;
} pat_geometry;

/* Library build.  CLOSED: the time factor cos(n c dt |k|) of every wavenumber
 * evaluated directly.  STEP: one k-space time-stepping run from a unit point
 * source, P^0 = 1, P^1 = cos(theta) P^0, P^{n+1} = 2 cos(theta) P^n - P^{n-1}
 * (theta = c dt |k|, the exact propagator of eq. 1-2 with zero initial
 * velocity, float64), the field recorded on every depth plane at every step;
 * by reciprocity (the library discussion of Sec. 3.2) the plane at depth l is
 * the sensor-plane response to a source at depth l.  Both store the same
 * library up to float64 rounding; STEP needs build scratch (pat_H_bytes). */
typedef enum { PAT_BUILD_CLOSED = 0, PAT_BUILD_STEP = 1 } pat_build;

/* ---------------------------------------------------------------- context */

/* Binds `device` (a HIP device ordinal, which must be a gfx950 GPU), uploads
 * the FFT twiddle tables to it, and returns a context.  Host memory only. */
pat_status pat_ctx_create(int device, pat_ctx** out);
void pat_ctx_destroy(pat_ctx* ctx);

/* ----------------------------------------------------------- kernel library */

/* Bytes of device memory the kernel library of `geom` needs (h_bytes), and
 * of scratch for building it (scratch_bytes: 0 for the closed form; for the
 * stepped build, the recorded fields of a block of symmetry classes, at most
 * 256 MiB plus one class; pat_H_build accepts any scratch that holds one
 * class's record, nt x (nz_sim/2 + 1) float64 values, and steps that many
 * classes per pass).  Host only. */
pat_status pat_H_bytes(const pat_geometry* geom, size_t* h_bytes, size_t* scratch_bytes);

/* Builds the kernel library of `geom` into the caller's device buffer h_buf
 * (>= h_bytes) on `stream`, and returns the operator handle in *out.
 * The library is the sensor-plane response of a unit point absorber at
 * each depth (Sec. 2.1; the library of Sec. 3.2), computed exactly on the
 * periodic grid in float64 on the GPU (cosine phases up to c*t*|k|, then the
 * depth sum) and stored in geom->h_dtype.  H^ is real and depends on
 * (kx, ky) only through kx^2 + ky^2, so it is stored once per symmetry class
 * of transverse frequencies: (|kx|, |ky|), or every frequency with the same
 * kx^2 + ky^2 when nx = ny and dx = dy; the layout inside h_buf is private.  h_buf must stay alive
 * and unmodified while the operator is in use; pat_op_destroy does not free
 * it.  Asynchronous: the operator may be used on `stream` at once, on other
 * streams after `stream` has been synchronised. */
pat_status pat_H_build(pat_ctx* ctx, const pat_geometry* geom, void* h_buf, size_t h_bytes,
                       void* scratch, size_t scratch_bytes, void* stream, pat_op** out);

pat_status pat_op_destroy(pat_op* op);

/* Writes the dequantised library for the r2c half-spectrum frequencies
 * k0 .. k0+nk-1 (k = p*(nx/2+1) + m, with m the x index and p the y index of
 * the 2D DFT) as a dense float32 device array out[nk][nz][nt].  For tests
 * and for users who want the kernels. */
pat_status pat_H_export(pat_op* op, int32_t k0, int32_t nk, float* out, void* stream);

/* Shape of the stored library: nk half-spectrum frequencies, nclass stored
 * slabs (symmetry classes: frequencies with equal kx^2 + ky^2 share one), the
 * z-period used, and the bytes of one stored row layout (the library keeps
 * two, rows along n for A and along l for A^T; a 16-bit library also keeps
 * both as matrix-core operand tiles, padded to 32 x 16, for batches).  The
 * contraction runs over nitems work items of up to members_max frequencies;
 * each streams one slab, so one apply of one object reads read_bytes_A (or
 * read_bytes_AT) of library.  gram_bytes: the Gram blocks kept for the
 * normal-operator gradient (one nz x nz float32 block per class), 0 when the
 * library has none (see pat_recon_fista). */
typedef struct {
  int32_t nk, nclass, members_max, nz_sim;
  size_t slab_bytes_A, slab_bytes_AT;
  int32_t spec_rows; /* rows of a spectrum array (see pat_spectrum) = nitems * members_max */
  int32_t nitems;
  size_t read_bytes_A, read_bytes_AT;
  size_t gram_bytes;
} pat_op_info;
pat_status pat_get_info(const pat_op* op, pat_op_info* info);

/* Frequency of every spectrum row: host array k_of_row[spec_rows]; -1 marks
 * rows no frequency maps to.  Host only. */
pat_status pat_spectrum_rows(const pat_op* op, int32_t* k_of_row);

/* Row stride, in complex elements, of a spectrum array holding S slices
 * (see pat_spectrum): S rounded up to a multiple of 64, plus 32 (an odd
 * multiple of 256 bytes).  The padding keeps rows from being a power of two
 * long, which would put the rows the transforms touch together on the same
 * HBM channels.  EINVAL for S outside [1, 2^30].  Host only. */
pat_status pat_spectrum_stride(int32_t S, int32_t* stride);

/* Workspace bytes every call below needs for a batch of B objects.  Here and
 * in every call taking B: EINVAL unless 1 <= B and B * max(nz, nt) <= 2^30
 * (slices per spectrum row). */
pat_status pat_workspace_bytes(const pat_op* op, int32_t B, size_t* bytes);

/* ------------------------------------------------------------- operators */

/* y = A x for B objects (eq. 7-8): x [B][nz][ny][nx] -> y [B][nt][ny/sy][nx/sx]
 * (y [B][nt][ny][nx] without scan-grid sampling; likewise everywhere below). */
pat_status pat_apply_A(pat_op* op, const float* x, float* y, int32_t B,
                       void* ws, size_t ws_bytes, void* stream);

/* y = A x exactly as pat_apply_A (same kernels, same results), for callers
 * that cannot allocate device memory or pass a workspace: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * spectra live in a static scratch array of 128 MiB that the library holds on
 * every GPU it runs on until the process ends; nothing is allocated per call.
 * EUNSUPPORTED when the B objects' spectra do not fit (pat_apply_A's
 * workspace minus its FISTA buffers: e.g. B = 1 up to 128 x 128 x 96 x 384,
 * B = 4 at 64 x 64 x 64 x 256); EINVAL as pat_apply_A.  All calls on one GPU
 * share its scratch: calls that overlap in time on that GPU (several
 * streams, several host threads) race and must be serialised by the caller;
 * calls in sequence on one stream are safe. */
pat_status pat_apply_A_noalloc(pat_op* op, const float* x, float* y, int32_t B, void* stream);

/* x = A^T y for B data sets (eq. 11): y [B][nt][ny/sy][nx/sx] -> x [B][nz][ny][nx]. */
pat_status pat_apply_AT(pat_op* op, const float* y, float* x, int32_t B,
                        void* ws, size_t ws_bytes, void* stream);

/* The three steps of an apply (Sec. 3.2), for callers that work in the
 * transverse Fourier domain.  Spectra are complex64 (interleaved re, im
 * float pairs), one row per r2c half-spectrum frequency, slice index fastest:
 *     spec[r*rs + s],  r = 0 .. spec_rows-1,  s = b*n + i < S,
 * rs = pat_spectrum_stride(S), S = B*n (n = nz for object spectra, nt for
 * data spectra); a spectrum array holds spec_rows*rs complex values and the
 * padding s >= S of each row is neither read nor written.  Rows are ordered by
 * symmetry class, members of a class adjacent, so that the contraction
 * streams contiguous rows; row r holds frequency k = k_of_row[r] from
 * pat_spectrum_rows (k = p*(nx/2+1) + m; -1 marks an unused row, whose
 * content is undefined).  pat_apply_A is pat_spectrum(x, B*nz) -> pat_contract(0) ->
 * pat_inverse_spectrum(B*nt), and pat_apply_AT the same with nz and nt
 * swapped and pat_contract(1); the calls launch the same kernels.
 *
 * The stage calls act on the full sensor grid: for a geometry with a scan
 * grid, S and S^T are applied by pat_apply_A / pat_apply_AT only.
 * pat_spectrum: unnormalised 2D DFT over (x, y) of S real slices f[S][ny][nx]
 * (step (i)); pat_inverse_spectrum: f = IDFT2(spec) / (nx*ny) - sub for S
 * slices (step (iii); sub may be NULL, else it has the layout of f).  Both need
 * a workspace sized by pat_workspace_bytes for some B with S <= B*max(nz, nt).
 * pat_contract (step (ii)): adjoint == 0: out[k][b*nt+n] = sum_l H^[k,l,n] in[k][b*nz+l];
 * adjoint != 0: out[k][b*nz+l] = sum_n conj(H^[k,l,n]) in[k][b*nt+n]; rows of
 * in and out have the strides of B*nz and B*nt slices; no workspace.  B = 1
 * runs on the vector units in float32; B >= 2 on the matrix cores, accumulated
 * in float32: with a float32 library the spectra and library values enter as
 * pairs of float16 terms under power-of-two scales (2^-22 relative), with a
 * 16-bit library the spectra as bfloat16 hi + lo pairs (2^-17 relative); an
 * object's result in a batch agrees with its B = 1 result to about 1e-6
 * relative (l2), not bit for bit. */
pat_status pat_spectrum(pat_op* op, const float* f, float* spec, int32_t S, void* ws,
                        size_t ws_bytes, void* stream);
pat_status pat_inverse_spectrum(pat_op* op, const float* spec, float* f, int32_t S, const float* sub,
                                void* ws, size_t ws_bytes, void* stream);
pat_status pat_contract(pat_op* op, int32_t adjoint, const float* in, float* out, int32_t B,
                        void* stream);

/* Step-size estimate by power iteration on A^T A (synchronises):
 * v = v0/||v0||; repeat niter times: w = A^T A v, L_i = <v, w>, v = w/||w||.
 * Writes L_niter to *L_out and, if L_trace != NULL, every L_i to the host
 * array L_trace[niter].  v0: device [nz][ny][nx], not modified.  A^T A is
 * block diagonal in the transverse frequency (Sec. 3.2), so the iteration
 * never leaves the frequencies v0 contains: start from a random vector (a
 * constant v0 yields the k = 0 block's norm only, an underestimate).  Where
 * the library has Gram blocks (see pat_recon_fista) w is formed through
 * them, else as A^T (A v). */
pat_status pat_power_norm(pat_op* op, const float* v0, int32_t niter, double* L_out,
                          double* L_trace, void* ws, size_t ws_bytes, void* stream);

/* FISTA for one object (Sec. 2.3): x_0 = 0, z_1 = x_0, t_1 = 1; for k = 1..niter:
 *     x_k     = prox(z_k - tau * A^T (A z_k - d)),
 *     z_{k+1} = x_k + beta_k (x_k - x_{k-1}),  beta_k = (t_k - 1)/t_{k+1},
 *     t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2   (beta_k = 0 if momentum == 0),
 * with prox(v) = max(v - tau*lambda, 0) if nonneg, else soft-thresholding.
 * d: device [nt][ny][nx]; x: device [nz][ny][nx], receives x_niter.
 * Periodic boundary, unsampled data: the gradient A^T (A z - d) =
 * A^T A z - A^T d (eq. 15) is formed per transverse frequency with the Gram
 * blocks H^_k^T H^_k of the library (built with it, float64 sums of the
 * stored values): one spectrum of z, one nz x nz contraction and one inverse
 * spectrum per iteration, A^T d once.  Linear boundary or scan-grid
 * sampling: the cropping or sampling between A and A^T couples the
 * frequencies, so the gradient is A^T r with r = A z - d, two applies.
 * trace: NULL or a device float array [niter] that receives
 * 1/2 ||A z_k - d||^2, the data term at the point where the gradient of
 * step k is taken (periodic: as 1/2 (<z, g> - <z, A^T d> + ||d||^2) with
 * float64 sums, absolute error of order 1e-7 * ||d||^2; linear: 1/2 <r, r>).
 * The momentum weights are computed on the host in float64.  Asynchronous. */
pat_status pat_recon_fista(pat_op* op, const float* d, float* x, int32_t niter,
                           float tau, float lambda, int32_t nonneg, int32_t momentum,
                           float* trace, void* ws, size_t ws_bytes, void* stream);

/* One FISTA iteration for B independent problems that share the operator
 * (the unit of work of a continuous-batching server).  Object b's arrays are
 * slices b of the batched arrays d [B][nt][ny][nx], x and z [B][nz][ny][nx];
 * x holds x_{k-1} on entry and x_k on exit, z holds z_k on entry and z_{k+1}
 * on exit.  beta, tau, lambda: host arrays [B] (beta_k of each object's own
 * iteration counter); nonneg: host int array [B].  B <= 32.  If
 * nonfinite != NULL (device int [B]), entry b is set to 1 when x_k of
 * object b contains a non-finite value and left unchanged otherwise. */
pat_status pat_fista_step(pat_op* op, int32_t B, const float* d, float* x, float* z,
                          const double* beta, const float* tau, const float* lambda,
                          const int32_t* nonneg, int32_t* nonfinite,
                          void* ws, size_t ws_bytes, void* stream);

/* The same iteration with the gradient formed per frequency through the Gram
 * blocks of the library (see pat_recon_fista): atd [B][nz][ny][nx] holds
 * A^T d of each object (one pat_apply_AT when the problem is set up), so the
 * data themselves are not needed; x, z, beta, tau, lambda, nonneg and
 * nonfinite as in pat_fista_step.  Per iteration: one spectrum of z, one
 * nz x nz contraction, one inverse spectrum and the update.  Only for
 * libraries with Gram blocks: periodic boundary, unsampled data
 * (EUNSUPPORTED otherwise). */
pat_status pat_fista_step_normal(pat_op* op, int32_t B, const float* atd, float* x, float* z,
                                 const double* beta, const float* tau, const float* lambda,
                                 const int32_t* nonneg, int32_t* nonfinite,
                                 void* ws, size_t ws_bytes, void* stream);

/* Adjoint check with float64 dot products on the GPU (synchronises):
 * *rel_out = |<A x, y> - <x, A^T y>| / (||A x|| ||y||).
 * x: device [nz][ny][nx], y: device [nt][ny][nx]. */
pat_status pat_adjoint_check(pat_op* op, const float* x, const float* y, double* rel_out,
                             void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ diagnostics */

const char* pat_status_str(pat_status s);
/* Message of the last failing call on the calling thread ("" if none). */
const char* pat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PAT_H_ */
