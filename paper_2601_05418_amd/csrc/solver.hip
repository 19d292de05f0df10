// Reconstruction on top of the compressed operator (Section 3.4).
//
// CG solves the normal equations of Eq. 16.  Dot products are FP64 and
// deterministic: every partial-producing kernel runs on the same fixed grid,
// each block writes one partial, and every consumer block re-sums the full
// partial array in the same order.  Scalars are never stored and re-read
// across blocks; the squared-residual partials alternate between two slots.
//
// FISTA solves Eq. 17 with the wavelet term.  A separable Haar transform of
// L levels acts independently on 2^L x 2^L tiles (every level only combines
// pixels inside such a tile), so the gradient step, the wavelet
// soft-threshold and the momentum update are one pass with one tile per
// thread, held in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "devutil.h"
#include "fft.h"
#include "plan.h"

namespace gpjc {

static constexpr int kRedBlocks = 240;  // fixed grid of every partial-producing kernel

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum (256 threads); result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// Sum of nb partials, same order in every block; result returned to all threads.
__device__ inline double sum_partials(const double* __restrict__ p, int nb, double* sh) {
  double v = 0.0;
  if (threadIdx.x < 64)
    for (int i = threadIdx.x; i < nb; i += 64) v += p[i];
  if (threadIdx.x < 64) v = wave_sum(v);
  if (threadIdx.x == 0) sh[4] = v;
  __syncthreads();
  const double r = sh[4];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_fill_zero(float2* __restrict__ v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_copy(const float2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// CG state on the device: the squared-residual partials alternate between two
// slots of red_rr (slot t & 1 after t iterations), and the iteration count t
// lives in device memory (incremented by k_cg_q), so one iteration is the
// same launch sequence every time and can be captured once and replayed.
__device__ inline double* rr_slot(double* base, int nb, int t) { return base + (t & 1) * nb; }

// Resets the numeric flag and the iteration counter (a kernel, not a memset,
// so that a captured solve holds no memset nodes).
__global__ void k_cg_reset(int* __restrict__ flag, int* __restrict__ iter) {
  if (threadIdx.x == 0) {
    *flag = 0;
    *iter = 0;
  }
}

// The CG vector kernels are written as bodies over one block index blk of
// a fixed grid of nb blocks, so that the per-plan kernels (blk = blockIdx.x)
// and the batch's work-list kernels (any block taking item (slice, blk))
// perform identical arithmetic in identical order.

// r = b - A x (A x given as partial images), p = r, partial <r, r> into slot t.
__device__ inline void cg_start_body(const float2* __restrict__ part, int nchunk, const float2* __restrict__ bvec,
                                     float2* __restrict__ r, float2* __restrict__ p, double* __restrict__ red_rr,
                                     int nb, const int* __restrict__ iter, size_t n, int blk, double* sh) {
  double acc = 0.0;
  for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x) {
    const float2 v = csub(bvec[i], sum_chunks(part, nchunk, n, i));
    r[i] = v;
    p[i] = v;
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_slot(red_rr, nb, *iter)[blk] = s;
}

// hist[t] = sqrt(sum of slot t's partials); one block.
__device__ inline void store_norm_body(const double* __restrict__ red_rr, int nb, const int* __restrict__ iter,
                                       double* __restrict__ hist, double* sh) {
  const int t = *iter;
  const double s = sum_partials(red_rr + (t & 1) * nb, nb, sh);
  if (threadIdx.x == 0) hist[t] = sqrt(s);
}

// q = A p (from partials), partial Re <p, q>; block 0 advances the iteration
// count (no other block of the same launch reads it).
__device__ inline void cg_q_body(const float2* __restrict__ part, int nchunk, const float2* __restrict__ p,
                                 float2* __restrict__ q, double* __restrict__ red_pq, int* __restrict__ iter, int nb,
                                 size_t n, int blk, double* sh) {
  double acc = 0.0;
  for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x) {
    const float2 v = sum_chunks(part, nchunk, n, i);
    q[i] = v;
    const float2 pv = p[i];
    acc += (double)pv.x * v.x + (double)pv.y * v.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red_pq[blk] = s;
  if (blk == 0 && threadIdx.x == 0) *iter += 1;
}

// alpha = rr / pq; x += alpha p; r -= alpha q; partial <r, r> into slot t
// (the old residual is in slot t - 1).
__device__ inline void cg_update_body(const double* __restrict__ red_pq, double* __restrict__ red_rr, int nb,
                                      const int* __restrict__ iter, float2* __restrict__ x, float2* __restrict__ r,
                                      const float2* __restrict__ p, const float2* __restrict__ q, size_t n,
                                      int* __restrict__ flag, int blk, double* sh) {
  const int t = *iter;
  const double pq = sum_partials(red_pq, nb, sh);
  const double rr = sum_partials(rr_slot(red_rr, nb, t - 1), nb, sh);
  if (!isfinite(pq) || !isfinite(rr)) {
    if (blk == 0 && threadIdx.x == 0) *flag = 1;
  }
  const double alpha = (pq > 0.0 && rr > 0.0) ? rr / pq : 0.0;
  const float a = (float)alpha;
  double acc = 0.0;
  for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x) {
    const float2 pv = p[i], qv = q[i];
    float2 xv = x[i], rv = r[i];
    xv = make_float2(fmaf(a, pv.x, xv.x), fmaf(a, pv.y, xv.y));
    rv = make_float2(fmaf(-a, qv.x, rv.x), fmaf(-a, qv.y, rv.y));
    x[i] = xv;
    r[i] = rv;
    acc += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_slot(red_rr, nb, t)[blk] = s;
}

// beta = rr_t / rr_{t-1}; p = r + beta p; hist[t] = ||r||.
__device__ inline void cg_dir_body(const double* __restrict__ red_rr, int nb, const int* __restrict__ iter,
                                   const float2* __restrict__ r, float2* __restrict__ p, size_t n,
                                   double* __restrict__ hist, int blk, double* sh) {
  const int t = *iter;
  const double rn = sum_partials(red_rr + (t & 1) * nb, nb, sh);
  const double ro = sum_partials(red_rr + ((t - 1) & 1) * nb, nb, sh);
  const float beta = (float)((ro > 0.0) ? rn / ro : 0.0);
  for (size_t i = (size_t)blk * blockDim.x + threadIdx.x; i < n; i += (size_t)nb * blockDim.x) {
    const float2 rv = r[i], pv = p[i];
    p[i] = make_float2(fmaf(beta, pv.x, rv.x), fmaf(beta, pv.y, rv.y));
  }
  if (blk == 0 && threadIdx.x == 0) hist[t] = sqrt(rn);
}

__global__ __launch_bounds__(256) void k_cg_start(const float2* __restrict__ part, int nchunk,
                                                  const float2* __restrict__ bvec, float2* __restrict__ r,
                                                  float2* __restrict__ p, double* __restrict__ red_rr, int nb,
                                                  const int* __restrict__ iter, size_t n) {
  __shared__ double sh[8];
  cg_start_body(part, nchunk, bvec, r, p, red_rr, nb, iter, n, blockIdx.x, sh);
}
__global__ void k_store_norm(const double* __restrict__ red_rr, int nb, const int* __restrict__ iter,
                             double* __restrict__ hist) {
  __shared__ double sh[8];
  store_norm_body(red_rr, nb, iter, hist, sh);
}
__global__ __launch_bounds__(256) void k_cg_q(const float2* __restrict__ part, int nchunk, const float2* __restrict__ p,
                                              float2* __restrict__ q, double* __restrict__ red_pq, int* __restrict__ iter,
                                              size_t n) {
  __shared__ double sh[8];
  cg_q_body(part, nchunk, p, q, red_pq, iter, gridDim.x, n, blockIdx.x, sh);
}
__global__ __launch_bounds__(256) void k_cg_update(const double* __restrict__ red_pq, double* __restrict__ red_rr,
                                                   int nb, const int* __restrict__ iter, float2* __restrict__ x,
                                                   float2* __restrict__ r, const float2* __restrict__ p,
                                                   const float2* __restrict__ q, size_t n, int* __restrict__ flag) {
  __shared__ double sh[8];
  cg_update_body(red_pq, red_rr, nb, iter, x, r, p, q, n, flag, blockIdx.x, sh);
}
__global__ __launch_bounds__(256) void k_cg_dir(const double* __restrict__ red_rr, int nb, const int* __restrict__ iter,
                                                const float2* __restrict__ r, float2* __restrict__ p, size_t n,
                                                double* __restrict__ hist) {
  __shared__ double sh[8];
  cg_dir_body(red_rr, nb, iter, r, p, n, hist, blockIdx.x, sh);
}

// Work-list forms for a batch: the items are (slice, block) pairs, slice
// major, taken by a persistent grid in strides of its size.  Every item is
// one block of the per-plan kernel above on that slice's vectors, so each
// slice's reductions keep their fixed order and a batched solve equals the
// separate ones bit for bit.  The store-norm step has one item per slice.
__global__ __launch_bounds__(256) void k_cg_list(const CgSlice* __restrict__ sl, int nslice, int op) {
  __shared__ double sh[8];
  const int nb = kRedBlocks;
  const int items = op == kCgListNorm ? nslice : nslice * nb;
  for (int w = blockIdx.x; w < items; w += gridDim.x) {
    const int si = op == kCgListNorm ? w : w / nb;
    const int blk = op == kCgListNorm ? 0 : w - si * nb;
    const CgSlice d = sl[si];
    double* red_pq = d.red;
    double* red_rr = d.red + nb;
    int* iter = d.flag + 1;
    switch (op) {
      case kCgListQ: cg_q_body(d.part, d.nchunk, d.p, d.q, red_pq, iter, nb, d.n, blk, sh); break;
      case kCgListUpdate: cg_update_body(red_pq, red_rr, nb, iter, d.x, d.r, d.p, d.q, d.n, d.flag, blk, sh); break;
      case kCgListDir: cg_dir_body(red_rr, nb, iter, d.r, d.p, d.n, d.hist, blk, sh); break;
      case kCgListStart: cg_start_body(d.part, d.nchunk, d.b, d.r, d.p, red_rr, nb, iter, d.n, blk, sh); break;
      default: store_norm_body(red_rr, nb, iter, d.hist, sh); break;
    }
  }
}

static int fill_zero(const Plan& pl, float2* v, size_t n) {
  hipLaunchKernelGGL(k_fill_zero, dim3(kRedBlocks), dim3(256), 0, pl.stream, v, n);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

static int copy_vec(const Plan& pl, const float2* a, float2* b, size_t n) {
  hipLaunchKernelGGL(k_copy, dim3(kRedBlocks), dim3(256), 0, pl.stream, a, b, n);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// The solve in three parts so that a batch can capture cg_iteration once.
int cg_setup(Plan& pl, Store st, bool refine, const float2* y, const float2* x0) {
  const size_t n = pl.img_elems();
  const int nb = kRedBlocks;
  // With refinement, b and every true residual come from the FP32 operator,
  // so the iterates converge to the FP32 solution; only the search
  // directions see the reduced-precision operator.
  const Store sb = refine ? Store::F32 : st;
  int* iter = pl.flag + 1;
  hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(64), 0, pl.stream, pl.flag, iter);
  GPJC_HIP(hipGetLastError());
  // b = E'^H y
  GPJC_TRY(op_adjoint_part(pl, sb, y));
  GPJC_TRY(launch_combine(pl, pl.vb));
  GPJC_TRY(copy_vec(pl, x0, pl.vx, n));
  // r0 = b - A x0
  GPJC_TRY(op_normal_part(pl, sb, pl.vx));
  hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, pl.vb, pl.vr, pl.vp,
                     pl.red + nb, nb, iter, n);
  hipLaunchKernelGGL(k_store_norm, dim3(1), dim3(256), 0, pl.stream, pl.red + nb, nb, iter, pl.hist);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int cg_op_part(const Plan& pl, Store st, int phase) {
  return phase == 0 ? op_normal_part(pl, st, pl.vp) : op_normal_part(pl, Store::F32, pl.vx);
}

CgSlice cg_slice_of(const Plan& pl) {
  CgSlice d;
  d.part = pl.part;
  d.b = pl.vb;
  d.x = pl.vx;
  d.r = pl.vr;
  d.p = pl.vp;
  d.q = pl.vq;
  d.red = pl.red;
  d.flag = pl.flag;
  d.hist = pl.hist;
  d.n = pl.img_elems();
  d.nchunk = pl.f1h_nchunk;
  return d;
}

int launch_cg_list(const CgSlice* d_list, int nslice, int op, int grid, hipStream_t s) {
  const int items = op == kCgListNorm ? nslice : nslice * kRedBlocks;
  hipLaunchKernelGGL(k_cg_list, dim3(std::max(1, std::min(grid, items))), dim3(256), 0, s, d_list, nslice, op);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int cg_iteration(const Plan& pl, Store st, bool refresh) {
  const size_t n = pl.img_elems();
  const int nb = kRedBlocks;
  int* iter = pl.flag + 1;
  double* red_pq = pl.red;
  double* red_rr = pl.red + nb;
  GPJC_TRY(op_normal_part(pl, st, pl.vp));
  {
    StageScope sc(pl, GPJC_STAGE_SOLVER);
    hipLaunchKernelGGL(k_cg_q, dim3(nb), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, pl.vp, pl.vq, red_pq, iter,
                       n);
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(256), 0, pl.stream, red_pq, red_rr, nb, iter, pl.vx, pl.vr, pl.vp,
                       pl.vq, n, pl.flag);
  }
  GPJC_HIP(hipGetLastError());
  if (refresh) {
    GPJC_TRY(op_normal_part(pl, Store::F32, pl.vx));
    StageScope sc(pl, GPJC_STAGE_SOLVER);
    hipLaunchKernelGGL(k_cg_start, dim3(nb), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, pl.vb, pl.vr, pl.vp,
                       red_rr, nb, iter, n);
    hipLaunchKernelGGL(k_store_norm, dim3(1), dim3(256), 0, pl.stream, red_rr, nb, iter, pl.hist);
  } else {
    StageScope sc(pl, GPJC_STAGE_SOLVER);
    hipLaunchKernelGGL(k_cg_dir, dim3(nb), dim3(256), 0, pl.stream, red_rr, nb, iter, pl.vr, pl.vp, n, pl.hist);
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// Copies the result out; queues the history (h_resid, iters + 1 entries, may
// be NULL) and the numeric flag (h_flag) to the host without synchronising.
int cg_finish(const Plan& pl, float2* x, int iters, double* h_resid, int* h_flag) {
  GPJC_TRY(copy_vec(pl, pl.vx, x, pl.img_elems()));
  if (h_resid)
    GPJC_HIP(hipMemcpyAsync(h_resid, pl.hist, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost, pl.stream));
  GPJC_HIP(hipMemcpyAsync(h_flag, pl.flag, sizeof(int), hipMemcpyDeviceToHost, pl.stream));
  return GPJC_OK;
}

bool cg_refresh_at(int it, int iters, int refine_every, Store st) {
  return refine_every > 0 && is_16bit(st) && (it + 1) % refine_every == 0 && it + 1 < iters;
}

int run_cg(Plan& pl, Store st, const float2* y, float2* x, int iters, int refine_every, double* h_resid) {
  const bool refine = refine_every > 0 && is_16bit(st);
  GPJC_TRY(cg_setup(pl, st, refine, y, x));
  for (int it = 0; it < iters; ++it) GPJC_TRY(cg_iteration(pl, st, cg_refresh_at(it, iters, refine_every, st)));
  int flag = 0;
  GPJC_TRY(cg_finish(pl, x, iters, h_resid, &flag));
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  if (flag) return fail(GPJC_E_NUMERIC, "CG: non-finite residual or curvature");
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// One gradient step on 1/2 ||E' x - y||^2 and its backward, for unrolled
// reconstruction: x_out = x - alpha (E'^H E' x - b) with b = E'^H y.
// For a real loss L and upstream gradient g = dL/dx_out (the conjugate
// Wirtinger convention, dL = Re <g, dx_out>):
//   dL/dx     = (I - alpha E'^H E') g      (E'^H E' is Hermitian, alpha real)
//   dL/db     = alpha g
//   dL/dalpha = -Re <g, E'^H E' x - b>
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gd_update(const float2* __restrict__ part, int nchunk,
                                                   const float2* __restrict__ x, const float2* __restrict__ b,
                                                   const float* __restrict__ alpha, float2* __restrict__ x_out,
                                                   float2* __restrict__ r_out, size_t n) {
  const float a = *alpha;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 r = csub(sum_chunks(part, nchunk, n, i), b[i]);
    const float2 xv = x[i];
    x_out[i] = make_float2(fmaf(-a, r.x, xv.x), fmaf(-a, r.y, xv.y));
    if (r_out) r_out[i] = r;
  }
}

__global__ __launch_bounds__(256) void k_gd_backward(const float2* __restrict__ part, int nchunk,
                                                     const float2* __restrict__ g, const float2* __restrict__ r,
                                                     const float* __restrict__ alpha, float2* __restrict__ gx,
                                                     float2* __restrict__ gb, double* __restrict__ red, size_t n) {
  __shared__ double sh[8];
  const float a = *alpha;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 q = sum_chunks(part, nchunk, n, i);
    const float2 gv = g[i];
    if (gx) gx[i] = make_float2(fmaf(-a, q.x, gv.x), fmaf(-a, q.y, gv.y));
    if (gb) gb[i] = make_float2(a * gv.x, a * gv.y);
    const float2 rv = r[i];
    acc += (double)gv.x * rv.x + (double)gv.y * rv.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__global__ void k_store_neg_sum(const double* __restrict__ red, int nb, float* __restrict__ out) {
  __shared__ double sh[8];
  const double s = sum_partials(red, nb, sh);
  if (threadIdx.x == 0) *out = (float)(-s);
}

int run_gd_step(const Plan& pl, Store st, const float2* x, const float2* b, const float* alpha, float2* x_out,
                float2* r_out) {
  GPJC_TRY(op_normal_part(pl, st, x));
  StageScope sc(pl, GPJC_STAGE_SOLVER);
  hipLaunchKernelGGL(k_gd_update, dim3(kRedBlocks), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, x, b, alpha,
                     x_out, r_out, pl.img_elems());
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int run_gd_step_backward(const Plan& pl, Store st, const float2* g, const float* alpha, const float2* r, float2* gx,
                         float2* gb, float* galpha) {
  GPJC_TRY(op_normal_part(pl, st, g));
  StageScope sc(pl, GPJC_STAGE_SOLVER);
  hipLaunchKernelGGL(k_gd_backward, dim3(kRedBlocks), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, g, r, alpha,
                     gx, gb, pl.red, pl.img_elems());
  hipLaunchKernelGGL(k_store_neg_sum, dim3(1), dim3(256), 0, pl.stream, pl.red, kRedBlocks, galpha);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// FISTA
// ---------------------------------------------------------------------------
template <int LEV>
__device__ inline void haar_tile(float2 (&c)[1 << LEV][1 << LEV], bool inverse) {
  constexpr int S = 1 << LEV;
  constexpr float rs = 0.70710678118654752440f;
  if (!inverse) {
#pragma unroll
    for (int lev = 0; lev < LEV; ++lev) {
      const int h = S >> lev;
      // along x (rows i < h)
#pragma unroll
      for (int i = 0; i < S; ++i) {
        if (i < h) {
          float2 t[S];
#pragma unroll
          for (int j = 0; j < S / 2; ++j)
            if (j < h / 2) {
              t[j] = cscale(cadd(c[i][2 * j], c[i][2 * j + 1]), rs);
              t[j + h / 2] = cscale(csub(c[i][2 * j], c[i][2 * j + 1]), rs);
            }
#pragma unroll
          for (int j = 0; j < S; ++j)
            if (j < h) c[i][j] = t[j];
        }
      }
      // along y (columns j < h)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        if (j < h) {
          float2 t[S];
#pragma unroll
          for (int i = 0; i < S / 2; ++i)
            if (i < h / 2) {
              t[i] = cscale(cadd(c[2 * i][j], c[2 * i + 1][j]), rs);
              t[i + h / 2] = cscale(csub(c[2 * i][j], c[2 * i + 1][j]), rs);
            }
#pragma unroll
          for (int i = 0; i < S; ++i)
            if (i < h) c[i][j] = t[i];
        }
      }
    }
  } else {
#pragma unroll
    for (int lev = LEV - 1; lev >= 0; --lev) {
      const int h = S >> lev;
      // along y
#pragma unroll
      for (int j = 0; j < S; ++j) {
        if (j < h) {
          float2 t[S];
#pragma unroll
          for (int i = 0; i < S / 2; ++i)
            if (i < h / 2) {
              const float2 lo = c[i][j], hi = c[i + h / 2][j];
              t[2 * i] = cscale(cadd(lo, hi), rs);
              t[2 * i + 1] = cscale(csub(lo, hi), rs);
            }
#pragma unroll
          for (int i = 0; i < S; ++i)
            if (i < h) c[i][j] = t[i];
        }
      }
      // along x
#pragma unroll
      for (int i = 0; i < S; ++i) {
        if (i < h) {
          float2 t[S];
#pragma unroll
          for (int j = 0; j < S / 2; ++j)
            if (j < h / 2) {
              const float2 lo = c[i][j], hi = c[i][j + h / 2];
              t[2 * j] = cscale(cadd(lo, hi), rs);
              t[2 * j + 1] = cscale(csub(lo, hi), rs);
            }
#pragma unroll
          for (int j = 0; j < S; ++j)
            if (j < h) c[i][j] = t[j];
        }
      }
    }
  }
}

// Haar transform of a 2^L x 2^L tile held one coefficient per lane (lane
// e = i * S + j for tile row i, column j).  Level l combines lanes whose row
// and column are multiples of 2^l: along x with the lane 2^l columns away,
// then along y with the lane 2^l rows away; the average stays on the lane
// with the lower index, the difference moves to the other.  After L levels
// lane 0 holds the tile's low-pass coefficient and every other lane one
// detail coefficient -- the Mallat coefficient set, stored permuted.
template <int LEV>
__device__ inline float2 haar_lanes(float2 v, int i, int j, bool inverse) {
  constexpr int S = 1 << LEV;
  constexpr float rs = 0.70710678118654752440f;
  auto step = [&](int mask, bool hi, bool active) {
    const float2 o = make_float2(__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64));
    if (!active) return;
    if (!inverse) v = hi ? cscale(csub(o, v), rs) : cscale(cadd(v, o), rs);
    else v = hi ? cscale(csub(o, v), rs) : cscale(cadd(v, o), rs);
  };
  if (!inverse) {
#pragma unroll
    for (int l = 0; l < LEV; ++l) {
      const int st = 1 << l;
      const bool act = (i % st == 0) && (j % st == 0);
      step(st, (j & st) != 0, act);       // along x
      step(st * S, (i & st) != 0, act);   // along y
    }
  } else {
#pragma unroll
    for (int l = LEV - 1; l >= 0; --l) {
      const int st = 1 << l;
      const bool act = (i % st == 0) && (j % st == 0);
      step(st * S, (i & st) != 0, act);   // along y
      step(st, (j & st) != 0, act);       // along x
    }
  }
  return v;
}

// v = y - (A y - b) / L; x = W^H soft(W v, thr) (final low-pass untouched);
// y <- x + mom (x - x_prev); x_prev <- x.  One lane per pixel, 2^L x 2^L
// pixels per tile, whole tiles per wave.
template <int LEV>
__global__ __launch_bounds__(256) void k_fista_step(const float2* __restrict__ part, int nchunk,
                                                    const float2* __restrict__ bvec, const float2* __restrict__ tvg,
                                                    float lam_tv, float2* __restrict__ yv,
                                                    float2* __restrict__ xprev, int nx, int ny, int B, float invL,
                                                    float thr, float mom) {
  constexpr int S = 1 << LEV, T = S * S;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int tile = gid / T, e = gid - tile * T;
  const int i = e / S, j = e - i * S;
  const int tx_n = nx / S, ty_n = ny / S;
  const int ntiles = B * tx_n * ty_n;
  const bool valid = tile < ntiles;
  const int tt = valid ? tile : 0;
  const int b = tt / (tx_n * ty_n);
  const int rem = tt - b * tx_n * ty_n;
  const int ty = rem / tx_n, tx = rem - ty * tx_n;
  const size_t n = (size_t)B * nx * ny;
  const size_t idx = ((size_t)b * ny + ty * S + i) * nx + tx * S + j;
  float2 g = csub(sum_chunks(part, nchunk, n, idx), bvec[idx]);
  if (lam_tv != 0.f) {
    const float2 t = tvg[idx];
    g = make_float2(fmaf(lam_tv, t.x, g.x), fmaf(lam_tv, t.y, g.y));
  }
  const float2 yy = yv[idx];
  float2 c = make_float2(fmaf(-invL, g.x, yy.x), fmaf(-invL, g.y, yy.y));
  c = haar_lanes<LEV>(c, i, j, false);
  if (e != 0) {
    const float mag = sqrtf(c.x * c.x + c.y * c.y);
    c = cscale(c, mag > thr ? 1.0f - thr / mag : 0.0f);
  }
  c = haar_lanes<LEV>(c, i, j, true);
  if (valid) {
    const float2 xo = xprev[idx];
    yv[idx] = make_float2(fmaf(mom, c.x - xo.x, c.x), fmaf(mom, c.y - xo.y, c.y));
    xprev[idx] = c;
  }
}

template <int LEV>
static int launch_fista_step(const Plan& pl, float invL, float thr, float mom, float lam_tv) {
  StageScope sc(pl, GPJC_STAGE_SOLVER);
  const size_t lanes = pl.img_elems();
  hipLaunchKernelGGL(k_fista_step<LEV>, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, pl.stream, pl.part,
                     pl.f1h_nchunk, pl.vb, pl.vq, lam_tv, pl.vp, pl.vx, pl.nx, pl.ny, pl.B, invL, thr, mom);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// Smoothed total variation (Eq. 17's TV term): TV_eps(x) = sum over pixels of
// sqrt(|Dx x|^2 + |Dy x|^2 + eps^2), forward differences with a zero
// difference at the last column / row of each image.
// ---------------------------------------------------------------------------
// q = D x / m at pixel (i, j) of image b (zero outside the image)
__device__ inline void tv_q(const float2* __restrict__ x, int b, int i, int j, int nx, int ny, float eps2,
                            float2* qx, float2* qy) {
  if (i < 0 || j < 0) {
    *qx = *qy = make_float2(0.f, 0.f);
    return;
  }
  const float2* xb = x + (size_t)b * ny * nx;
  const float2 c = xb[(size_t)i * nx + j];
  const float2 dx = j + 1 < nx ? csub(xb[(size_t)i * nx + j + 1], c) : make_float2(0.f, 0.f);
  const float2 dy = i + 1 < ny ? csub(xb[(size_t)(i + 1) * nx + j], c) : make_float2(0.f, 0.f);
  const float inv = rsqrtf(dx.x * dx.x + dx.y * dx.y + dy.x * dy.x + dy.y * dy.y + eps2);
  *qx = cscale(dx, inv);
  *qy = cscale(dy, inv);
}

// g = D^H (D x / m): the gradient of TV_eps at x
__global__ __launch_bounds__(256) void k_tv_grad(const float2* __restrict__ x, float2* __restrict__ g, int nx, int ny,
                                                 int B, float eps2) {
  const size_t n = (size_t)B * ny * nx;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % nx);
    const int i = (int)((idx / nx) % ny);
    const int b = (int)(idx / ((size_t)nx * ny));
    float2 qx, qy, qxl, qyl, qxu, qyu;
    tv_q(x, b, i, j, nx, ny, eps2, &qx, &qy);
    tv_q(x, b, i, j - 1, nx, ny, eps2, &qxl, &qyl);
    tv_q(x, b, i - 1, j, nx, ny, eps2, &qxu, &qyu);
    // (D^H q)[i][j] = qx[i][j-1] - qx[i][j] + qy[i-1][j] - qy[i][j]  (qx = 0 at j = nx-1, qy = 0 at i = ny-1)
    g[idx] = make_float2(qxl.x - qx.x + qyu.x - qy.x, qxl.y - qx.y + qyu.y - qy.y);
  }
}

// partial sums of TV_eps(x) on the fixed grid
__global__ __launch_bounds__(256) void k_tv_value(const float2* __restrict__ x, double* __restrict__ red, int nx,
                                                  int ny, int B, double eps2) {
  __shared__ double sh[8];
  const size_t n = (size_t)B * ny * nx;
  double acc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx % nx);
    const int i = (int)((idx / nx) % ny);
    const float2 c = x[idx];
    const float2 dx = j + 1 < nx ? csub(x[idx + 1], c) : make_float2(0.f, 0.f);
    const float2 dy = i + 1 < ny ? csub(x[idx + nx], c) : make_float2(0.f, 0.f);
    acc += sqrt((double)dx.x * dx.x + (double)dx.y * dx.y + (double)dy.x * dy.x + (double)dy.y * dy.y + eps2);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// FISTA objective of an iterate x (Eq. 17 with the wavelet term, in the
// 1/2 ||E' x - y||^2 + lambda ||W x||_1 form, final low-pass band not
// penalised), accumulated in FP64 on the fixed reduction grid.
// ---------------------------------------------------------------------------
// partial sums of |d - y|^2 over the data vector
__global__ __launch_bounds__(256) void k_resid2(const float2* __restrict__ d, const float2* __restrict__ y,
                                                double* __restrict__ red, size_t n) {
  __shared__ double sh[8];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 a = d[i], b = y[i];
    const double re = (double)a.x - b.x, im = (double)a.y - b.y;
    acc += re * re + im * im;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// partial sums of |c| over the detail coefficients of W img (one 2^L x 2^L
// tile per thread, tiles strided over the fixed grid)
template <int LEV>
__global__ __launch_bounds__(256) void k_wavelet_l1(const float2* __restrict__ img, int nx, int ny, int B,
                                                    double* __restrict__ red) {
  constexpr int S = 1 << LEV;
  __shared__ double sh[8];
  const int tx_n = nx / S, ty_n = ny / S;
  const int ntiles = B * tx_n * ty_n;
  double acc = 0.0;
  for (int tile = blockIdx.x * blockDim.x + threadIdx.x; tile < ntiles; tile += gridDim.x * blockDim.x) {
    const int b = tile / (tx_n * ty_n);
    const int rem = tile - b * tx_n * ty_n;
    const int ty = rem / tx_n, tx = rem - ty * tx_n;
    float2 c[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) c[i][j] = img[((size_t)b * ny + ty * S + i) * nx + tx * S + j];
    haar_tile<LEV>(c, false);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (i | j) acc += sqrt((double)c[i][j].x * c[i][j].x + (double)c[i][j].y * c[i][j].y);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// *out = 1/2 sum(red_d) + lambda sum(red_w) + lambda_tv sum(red_t); single block
__global__ void k_store_obj(const double* __restrict__ red_d, const double* __restrict__ red_w,
                            const double* __restrict__ red_t, int nb, double lambda, double lambda_tv,
                            double* __restrict__ out) {
  __shared__ double sh[8];
  const double d = sum_partials(red_d, nb, sh);
  const double w = sum_partials(red_w, nb, sh);
  const double t = lambda_tv != 0.0 ? sum_partials(red_t, nb, sh) : 0.0;
  if (threadIdx.x == 0) *out = 0.5 * d + lambda * w + lambda_tv * t;
}

__global__ __launch_bounds__(256) void k_norm2(const float2* __restrict__ v, double* __restrict__ red, size_t n);

// *flag = 1 if the sum of the nb partials is not finite, else 0; single block
__global__ void k_flag_nonfinite(const double* __restrict__ red, int nb, int* __restrict__ flag) {
  __shared__ double sh[8];
  const double s = sum_partials(red, nb, sh);
  if (threadIdx.x == 0) *flag = isfinite(s) ? 0 : 1;
}

static size_t data_elems(const Plan& pl) {
  return pl.compressed ? (size_t)pl.B * pl.np * pl.K * pl.ms : (size_t)pl.B * pl.nc * pl.ms * pl.nt;
}

// Objective of x = pl.vx into *out (device): forward application into pl.vd,
// then the two reductions.
static int fista_objective(const Plan& pl, Store st, const float2* y, int levels, double lambda, double lam_tv,
                           double eps, double* out) {
  GPJC_TRY(op_forward(pl, st, pl.vx, pl.vd));
  const int nb = kRedBlocks;
  double* red_d = pl.red;
  double* red_w = pl.red + nb;
  double* red_t = pl.red + 2 * nb;
  if (lam_tv != 0.0)
    hipLaunchKernelGGL(k_tv_value, dim3(nb), dim3(256), 0, pl.stream, pl.vx, red_t, pl.nx, pl.ny, pl.B, eps * eps);
  hipLaunchKernelGGL(k_resid2, dim3(nb), dim3(256), 0, pl.stream, pl.vd, y, red_d, data_elems(pl));
  switch (levels) {
    case 1: hipLaunchKernelGGL(k_wavelet_l1<1>, dim3(nb), dim3(256), 0, pl.stream, pl.vx, pl.nx, pl.ny, pl.B, red_w); break;
    case 2: hipLaunchKernelGGL(k_wavelet_l1<2>, dim3(nb), dim3(256), 0, pl.stream, pl.vx, pl.nx, pl.ny, pl.B, red_w); break;
    default: hipLaunchKernelGGL(k_wavelet_l1<3>, dim3(nb), dim3(256), 0, pl.stream, pl.vx, pl.nx, pl.ny, pl.B, red_w); break;
  }
  hipLaunchKernelGGL(k_store_obj, dim3(1), dim3(256), 0, pl.stream, red_d, red_w, red_t, nb, lambda, lam_tv, out);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int run_fista(Plan& pl, Store st, const float2* y, float2* x, int iters, double lambda, double lam_tv, double eps,
              double lip, int levels, double* h_obj) {
  const size_t n = pl.img_elems();
  GPJC_TRY(op_adjoint_part(pl, st, y));
  GPJC_TRY(launch_combine(pl, pl.vb));
  GPJC_TRY(fill_zero(pl, pl.vx, n));  // x_{k-1}
  GPJC_TRY(fill_zero(pl, pl.vp, n));  // y_k
  const float invL = (float)(1.0 / lip);
  const float thr = (float)(lambda / lip);
  double t = 1.0;
  const float ltv = (float)lam_tv;
  for (int it = 0; it < iters; ++it) {
    GPJC_TRY(op_normal_part(pl, st, pl.vp));
    if (lam_tv != 0.0) {
      StageScope sc(pl, GPJC_STAGE_SOLVER);
      hipLaunchKernelGGL(k_tv_grad, dim3(kRedBlocks), dim3(256), 0, pl.stream, pl.vp, pl.vq, pl.nx, pl.ny, pl.B,
                         (float)(eps * eps));
      GPJC_HIP(hipGetLastError());
    }
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    const float mom = (float)((t - 1.0) / tn);
    t = tn;
    switch (levels) {
      case 1: GPJC_TRY(launch_fista_step<1>(pl, invL, thr, mom, ltv)); break;
      case 2: GPJC_TRY(launch_fista_step<2>(pl, invL, thr, mom, ltv)); break;
      default: GPJC_TRY(launch_fista_step<3>(pl, invL, thr, mom, ltv)); break;
    }
    if (h_obj) GPJC_TRY(fista_objective(pl, st, y, levels, lambda, lam_tv, eps, pl.hist + it));
  }
  GPJC_TRY(copy_vec(pl, pl.vx, x, n));
  // numeric status: the squared norm of the result, summed in FP64, must be finite
  hipLaunchKernelGGL(k_norm2, dim3(kRedBlocks), dim3(256), 0, pl.stream, pl.vx, pl.red, n);
  hipLaunchKernelGGL(k_flag_nonfinite, dim3(1), dim3(256), 0, pl.stream, pl.red, kRedBlocks, pl.flag);
  GPJC_HIP(hipGetLastError());
  int flag = 0;
  GPJC_HIP(hipMemcpyAsync(&flag, pl.flag, sizeof(int), hipMemcpyDeviceToHost, pl.stream));
  if (h_obj) GPJC_HIP(hipMemcpyAsync(h_obj, pl.hist, sizeof(double) * iters, hipMemcpyDeviceToHost, pl.stream));
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  if (flag) return fail(GPJC_E_NUMERIC, "FISTA: non-finite iterate");
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// Power iteration for the largest eigenvalue of the normal operator.
// ---------------------------------------------------------------------------
// partial sums of |v|^2
__global__ __launch_bounds__(256) void k_norm2(const float2* __restrict__ v, double* __restrict__ red, size_t n) {
  __shared__ double sh[8];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 a = v[i];
    acc += (double)a.x * a.x + (double)a.y * a.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

// v_out = v_in / sqrt(sum partials)
__global__ __launch_bounds__(256) void k_scale_unit(const float2* __restrict__ vin, float2* __restrict__ vout,
                                                    const double* __restrict__ red, int nb, size_t n) {
  __shared__ double sh[8];
  const double s = sum_partials(red, nb, sh);
  const float inv = (float)(s > 0.0 ? 1.0 / sqrt(s) : 0.0);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    vout[i] = cscale(vin[i], inv);
}

// q = A v (partials); partial Re <v, q> and |q|^2
__global__ __launch_bounds__(256) void k_power_q(const float2* __restrict__ part, int nchunk,
                                                 const float2* __restrict__ v, float2* __restrict__ q,
                                                 double* __restrict__ red_vq, double* __restrict__ red_qq, size_t n) {
  __shared__ double sh[8];
  double a1 = 0.0, a2 = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 w = sum_chunks(part, nchunk, n, i);
    q[i] = w;
    const float2 a = v[i];
    a1 += (double)a.x * w.x + (double)a.y * w.y;
    a2 += (double)w.x * w.x + (double)w.y * w.y;
  }
  const double s1 = block_sum(a1, sh);
  if (threadIdx.x == 0) red_vq[blockIdx.x] = s1;
  const double s2 = block_sum(a2, sh);
  if (threadIdx.x == 0) red_qq[blockIdx.x] = s2;
}

__global__ void k_store_sum(const double* __restrict__ red, int nb, double* __restrict__ out) {
  __shared__ double sh[8];
  const double s = sum_partials(red, nb, sh);
  if (threadIdx.x == 0) *out = s;
}

int run_power_iteration(Plan& pl, Store st, const float2* x0, int iters, double* h_lambda) {
  const size_t n = pl.img_elems();
  const int nb = kRedBlocks;
  double* red_a = pl.red;
  double* red_b = pl.red + nb;
  hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(256), 0, pl.stream, x0, red_a, n);
  hipLaunchKernelGGL(k_scale_unit, dim3(nb), dim3(256), 0, pl.stream, x0, pl.vp, red_a, nb, n);
  GPJC_HIP(hipGetLastError());
  GPJC_HIP(hipMemsetAsync(pl.hist, 0, sizeof(double), pl.stream));
  for (int it = 0; it < iters; ++it) {
    GPJC_TRY(op_normal_part(pl, st, pl.vp));
    hipLaunchKernelGGL(k_power_q, dim3(nb), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, pl.vp, pl.vq, red_a,
                       red_b, n);
    hipLaunchKernelGGL(k_scale_unit, dim3(nb), dim3(256), 0, pl.stream, pl.vq, pl.vp, red_b, nb, n);
    if (it == iters - 1) hipLaunchKernelGGL(k_store_sum, dim3(1), dim3(256), 0, pl.stream, red_a, nb, pl.hist);
    GPJC_HIP(hipGetLastError());
  }
  GPJC_HIP(hipMemcpyAsync(h_lambda, pl.hist, sizeof(double), hipMemcpyDeviceToHost, pl.stream));
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// max |W x| over all Haar coefficients (per-tile transform, block maxima).
// ---------------------------------------------------------------------------
template <int LEV>
__global__ __launch_bounds__(64) void k_wavelet_absmax(const float2* __restrict__ img, int nx, int ny, int B,
                                                       double* __restrict__ red) {
  constexpr int S = 1 << LEV;
  const int tx_n = nx / S, ty_n = ny / S;
  const int tile = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.f;
  if (tile < B * tx_n * ty_n) {
    const int b = tile / (tx_n * ty_n);
    const int rem = tile - b * tx_n * ty_n;
    const int ty = rem / tx_n, tx = rem - ty * tx_n;
    float2 c[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) c[i][j] = img[((size_t)b * ny + ty * S + i) * nx + tx * S + j];
    haar_tile<LEV>(c, false);
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) m = fmaxf(m, sqrtf(c[i][j].x * c[i][j].x + c[i][j].y * c[i][j].y));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off, 64));
  if (threadIdx.x == 0) red[blockIdx.x] = m;
}

int run_wavelet_absmax(Plan& pl, const float2* img, int levels, double* h_out) {
  const int S = 1 << levels;
  const int tiles = pl.B * (pl.nx / S) * (pl.ny / S);
  const int blocks = (tiles + 63) / 64;
  if (blocks > 4096) return fail(GPJC_E_UNSUPPORTED, "image too large for the wavelet maximum");
  switch (levels) {
    case 1: hipLaunchKernelGGL(k_wavelet_absmax<1>, dim3(blocks), dim3(64), 0, pl.stream, img, pl.nx, pl.ny, pl.B, pl.red); break;
    case 2: hipLaunchKernelGGL(k_wavelet_absmax<2>, dim3(blocks), dim3(64), 0, pl.stream, img, pl.nx, pl.ny, pl.B, pl.red); break;
    default: hipLaunchKernelGGL(k_wavelet_absmax<3>, dim3(blocks), dim3(64), 0, pl.stream, img, pl.nx, pl.ny, pl.B, pl.red); break;
  }
  GPJC_HIP(hipGetLastError());
  std::vector<double> h(blocks);
  GPJC_HIP(hipMemcpyAsync(h.data(), pl.red, sizeof(double) * blocks, hipMemcpyDeviceToHost, pl.stream));
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  *h_out = m;
  return GPJC_OK;
}

}  // namespace gpjc
