// Reconstruction algorithm #1 (Section 3.4, Eq. 16): hybrid-space least
// squares over aliased sets, each solved by LSQR (Paige and Saunders).
//
// With a regular R-fold phase-encode mask and no calibration lines (lines with
// (ky - Ny/2) divisible by R, Ms = Ny / R of them), the zero-filled inverse DFT
// of the acquired lines is periodic in y with period Ms and holds
// (1/R) sum_q Z[yr + q Ms]: the image rows yr + q Ms (q < R) fold onto one
// another, and Eq. 16 splits into Ms independent problems (per image), one per
// aliased set yr:
//
//   M_yr rho_yr = h_yr,   M_yr v = R^(-1/2) sum_q Z_v[:, :, yr + q Ms],
//   h_yr = R^(1/2) zf[:, :, yr],
//
// with Z_v the column stages of the operator (readout model and group
// contraction per image column, without the phase-encode DFT) and zf the
// zero-filled inverse DFT of the data.  Every set runs its own LSQR
// recurrence; all sets advance together, one operator application per
// direction and iteration.  Per set, work-groups of k_lsqr_u / k_lsqr_v own
// the set's elements, reduce its norms in FP64 in a fixed order and update its
// scalars, so each set's iterates are those of an LSQR run on that set alone.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "devutil.h"
#include "fft.h"
#include "plan.h"

namespace gpjc {

namespace {

// Per-set scalars: sc[kAlpha * nsets + s] etc.
enum { kAlpha = 0, kBeta = 1, kRhoBar = 2, kPhiBar = 3 };

__device__ inline double wg_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double t = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return t;
}

// Data side of one set s = (b, yr); elements e = (p, k).
//   start:  ubar = R^(1/2) zf[b][p][yr][k]            (zf: FP32 Z^T of the data)
//   else:   ubar = R^(-1/2) sum_q sum_split Zp[..][b][p][k][yr + q Ms] - alpha u
//   beta = ||ubar||, u = ubar / beta (zero if beta = 0), and the adjoint's input
//   Z^T[b][p][yr + q Ms][k] = R^(-1/2) u for every q.
template <Store ST>
__global__ __launch_bounds__(256) void k_lsqr_u(int start, const float2* __restrict__ zf, const float2* __restrict__ Zp,
                                                int ksplit, size_t zstride, float2* __restrict__ u, void* __restrict__ Zt,
                                                double* __restrict__ sc, int nsets, int np, int K, int kp, int ny,
                                                int ms, int R) {
  __shared__ double sh[4];
  const int s = blockIdx.x, b = s / ms, yr = s - b * ms;
  const int ne = np * K;
  const float rs = rsqrtf((float)R), r1 = sqrtf((float)R);
  const float alpha = start ? 0.f : (float)sc[kAlpha * nsets + s];
  float2* us = u + (size_t)s * ne;
  double acc = 0.0;
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int p = e / K, k = e - p * K;
    float2 v;
    if (start) {
      v = cscale(zf[(((size_t)b * np + p) * ny + yr) * kp + k], r1);
    } else {
      float2 f = make_float2(0.f, 0.f);
      const size_t base = (((size_t)b * np + p) * K + k) * ny + yr;
      for (int sp = 0; sp < ksplit; ++sp)
        for (int q = 0; q < R; ++q) f = cadd(f, Zp[sp * zstride + base + (size_t)q * ms]);
      const float2 uo = us[e];
      v = make_float2(f.x * rs - alpha * uo.x, f.y * rs - alpha * uo.y);
    }
    us[e] = v;
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double beta = sqrt(wg_sum(acc, sh));
  const float inv = beta > 0.0 ? (float)(1.0 / beta) : 0.f;
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int p = e / K, k = e - p * K;
    const float2 v = cscale(us[e], inv);
    us[e] = v;
    const float2 z = cscale(v, rs);
    for (int q = 0; q < R; ++q) store_zt<ST>(Zt, ((size_t)b * np + p) * ny + yr + (size_t)q * ms, kp, k, z);
  }
  if (threadIdx.x == 0) sc[kBeta * nsets + s] = beta;
}

// Image side of one set s = (b, yr); elements (q, x) of rows y = yr + q Ms.
//   start:  vbar = E^H-columns(u) (the partial images), alpha = ||vbar||,
//           v = vbar / alpha, w = v, x = 0, phibar = beta, rhobar = alpha
//   else:   vbar = E^H-columns(u) - beta v, alpha' = ||vbar||, v' = vbar / alpha',
//           rho = hypot(rhobar, beta), c = rhobar / rho, s = beta / rho,
//           theta = s alpha', rhobar = -c alpha', phi = c phibar, phibar = s phibar,
//           x += (phi / rho) w, w = v' - (theta / rho) w.
__global__ __launch_bounds__(256) void k_lsqr_v(int start, const float2* __restrict__ part, int nchunk,
                                                float2* __restrict__ v, float2* __restrict__ w, float2* __restrict__ x,
                                                double* __restrict__ sc, int nsets, int nx, int ny, int ms, int R,
                                                size_t nimg) {
  __shared__ double sh[4];
  __shared__ float coef[3];  // 1 / alpha', phi / rho, theta / rho
  const int s = blockIdx.x, b = s / ms, yr = s - b * ms;
  const int ne = R * nx;
  const float beta = (float)sc[kBeta * nsets + s];
  double acc = 0.0;
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int q = e / nx, xx = e - q * nx;
    const size_t i = ((size_t)b * ny + yr + (size_t)q * ms) * nx + xx;
    float2 vb = sum_chunks(part, nchunk, nimg, i);
    if (!start) {
      const float2 vo = v[i];
      vb = make_float2(vb.x - beta * vo.x, vb.y - beta * vo.y);
    }
    v[i] = vb;
    acc += (double)vb.x * vb.x + (double)vb.y * vb.y;
  }
  const double alpha = sqrt(wg_sum(acc, sh));
  if (threadIdx.x == 0) {
    coef[0] = alpha > 0.0 ? (float)(1.0 / alpha) : 0.f;
    if (start) {
      coef[1] = coef[2] = 0.f;
      sc[kPhiBar * nsets + s] = sc[kBeta * nsets + s];
      sc[kRhoBar * nsets + s] = alpha;
    } else {
      const double rhobar = sc[kRhoBar * nsets + s], phibar = sc[kPhiBar * nsets + s], bt = sc[kBeta * nsets + s];
      const double rho = hypot(rhobar, bt);
      if (rho > 0.0) {
        const double c = rhobar / rho, sn = bt / rho;
        const double theta = sn * alpha;
        const double phi = c * phibar;
        coef[1] = (float)(phi / rho);
        coef[2] = (float)(theta / rho);
        sc[kRhoBar * nsets + s] = -c * alpha;
        sc[kPhiBar * nsets + s] = sn * phibar;
      } else {
        coef[1] = coef[2] = 0.f;
      }
    }
    sc[kAlpha * nsets + s] = alpha;
  }
  __syncthreads();
  const float ia = coef[0], fx = coef[1], fw = coef[2];
  for (int e = threadIdx.x; e < ne; e += 256) {
    const int q = e / nx, xx = e - q * nx;
    const size_t i = ((size_t)b * ny + yr + (size_t)q * ms) * nx + xx;
    const float2 vn = cscale(v[i], ia);
    v[i] = vn;
    if (start) {
      w[i] = vn;
      x[i] = make_float2(0.f, 0.f);
    } else {
      const float2 wo = w[i], xo = x[i];
      x[i] = make_float2(fmaf(fx, wo.x, xo.x), fmaf(fx, wo.y, xo.y));
      w[i] = make_float2(fmaf(-fw, wo.x, vn.x), fmaf(-fw, wo.y, vn.y));
    }
  }
}

// hist[t] = sqrt(sum over sets of phibar^2) (fixed order); flag if not finite.
__global__ void k_lsqr_resid(const double* __restrict__ sc, int nsets, double* __restrict__ hist, int t,
                             int* __restrict__ flag) {
  __shared__ double sh[4];
  double a = 0.0;
  for (int s = threadIdx.x; s < nsets; s += 256) {
    const double p = sc[kPhiBar * nsets + s];
    a += p * p;
  }
  const double r = sqrt(wg_sum(a, sh));
  if (threadIdx.x == 0) {
    hist[t] = r;
    if (!isfinite(r)) *flag = 1;
  }
}

__global__ __launch_bounds__(256) void k_copy_image(const float2* __restrict__ a, float2* __restrict__ b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_flag_clear(int* __restrict__ flag) {
  if (threadIdx.x == 0) *flag = 0;
}

template <Store ST>
int lsqr_u(const Plan& pl, bool start, int ms, int R, int ksplit) {
  StageScope scope(pl, GPJC_STAGE_SOLVER);
  const int nsets = pl.B * ms;
  const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
  void* zt = ST == Store::F32 ? static_cast<void*>(pl.Zt) : static_cast<void*>(pl.Zt16);
  hipLaunchKernelGGL((k_lsqr_u<ST>), dim3(nsets), dim3(256), 0, pl.stream, start ? 1 : 0, pl.Zt, pl.Zp,
                     ksplit, zs, pl.vd, zt, pl.red, nsets, pl.np, pl.K, pl.Kp, pl.ny, ms, R);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int lsqr_u_st(const Plan& pl, Store st, bool start, int ms, int R) {
  const int ks = pl.cfg(st).ksplit;  // partials of Z the compressing contraction of st wrote
  switch (storage_of(st)) {
    case Store::F32: return lsqr_u<Store::F32>(pl, start, ms, R, ks);
    case Store::BF16: return lsqr_u<Store::BF16>(pl, start, ms, R, ks);
    default: return lsqr_u<Store::F16>(pl, start, ms, R, ks);
  }
}

int lsqr_v(const Plan& pl, bool start, int ms, int R, int t) {
  StageScope scope(pl, GPJC_STAGE_SOLVER);
  const int nsets = pl.B * ms;
  hipLaunchKernelGGL(k_lsqr_v, dim3(nsets), dim3(256), 0, pl.stream, start ? 1 : 0, pl.part, pl.f1h_nchunk, pl.vr,
                     pl.vp, pl.vx, pl.red, nsets, pl.nx, pl.ny, ms, R, pl.img_elems());
  hipLaunchKernelGGL(k_lsqr_resid, dim3(1), dim3(256), 0, pl.stream, pl.red, nsets, pl.hist, t, pl.flag);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

}  // namespace

// R of a regular mask without calibration lines: lines with (ky - Ny/2)
// divisible by R and no others; 0 if the mask is not of that form.
int regular_accel(const Plan& pl) {
  if (pl.ms < 1 || pl.ny % pl.ms) return 0;
  const int R = pl.ny / pl.ms;
  for (int i = 0; i < pl.ny; ++i) {
    const int d = ((i - pl.ny / 2) % R + R) % R;
    if ((d == 0) != (pl.mask_h[i] != 0)) return 0;
  }
  return R;
}

int run_lsqr(Plan& pl, Store st, const float2* y, float2* xout, int iters, double* h_resid) {
  const int R = regular_accel(pl);
  const int ms = pl.ms;
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, pl.stream, pl.flag);
  // 1. inverse DFT along the phase encodes (zero-filled): FP32 Z^T
  GPJC_TRY(launch_pe_adj(pl, y, Store::F32));
  // start: beta_1 u_1 = h, alpha_1 v_1 = M^H u_1
  GPJC_TRY(lsqr_u_st(pl, st, true, ms, R));
  GPJC_TRY(op_adj_columns(pl, st));
  GPJC_TRY(lsqr_v(pl, true, ms, R, 0));
  // 2. the sets' LSQR iterations, all sets together
  for (int it = 0; it < iters; ++it) {
    GPJC_TRY(op_fwd_columns(pl, st, pl.vr));
    GPJC_TRY(lsqr_u_st(pl, st, false, ms, R));
    GPJC_TRY(op_adj_columns(pl, st));
    GPJC_TRY(lsqr_v(pl, false, ms, R, it + 1));
  }
  // 3. the assembled image
  hipLaunchKernelGGL(k_copy_image, dim3(240), dim3(256), 0, pl.stream, pl.vx, xout, pl.img_elems());
  GPJC_HIP(hipGetLastError());
  int flag = 0;
  GPJC_HIP(hipMemcpyAsync(&flag, pl.flag, sizeof(int), hipMemcpyDeviceToHost, pl.stream));
  if (h_resid)
    GPJC_HIP(hipMemcpyAsync(h_resid, pl.hist, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost, pl.stream));
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  if (flag) return fail(GPJC_E_NUMERIC, "LSQR: non-finite residual");
  return GPJC_OK;
}

}  // namespace gpjc
