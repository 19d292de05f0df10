// Stages of the hybrid-space Wave operator E' and their adjoints.
//
//   F1   readout: coil weighting, zero-padded oversampled readout DFT, PSF
//        (the readout model of Section 2.3 for a modulation that repeats on
//        every phase-encode step);
//   F2   group contraction: Z_p = A_{g(p)} W_p over the Nc x P virtual
//        channels of every patch (Eqs. 13-14 applied to hybrid data);
//   F3   phase-encode DFT and line selection (Section 3.4: the phase-encode
//        dimension is reconstructed by FFT).
//
// Readout DFT: with t = q*os + s (q < Nx, s < os) and the zero padding, the
// centred length-Nt DFT of a length-Nx line splits into os length-Nx DFTs:
//   X[q os + s] = post[t] * FFT_Nx(u[x] * twin[s][x])[q],
//   twin[s][x] = (-1)^x exp(-2 pi i s x / Nt),
//   post[t]    = (-1)^(Nx/2) (-1)^q exp(i pi s / os) / sqrt(Nt),
// and post[t] is folded into the PSF once per plan (psfp).
#include <hip/hip_runtime.h>

#include <cmath>

#include "devutil.h"
#include "fft.h"
#include "fft2.h"
#include "plan.h"

namespace gpjc {

__device__ inline void wg_sync() { __syncthreads(); }

// ---------------------------------------------------------------------------
// Tables: psfp, twin, FFT twiddles (FP64 evaluation, rounded once).
// ---------------------------------------------------------------------------
__global__ void k_prep_tables(const float2* __restrict__ psf, float2* __restrict__ psfp, float2* __restrict__ twin,
                              float2* __restrict__ twx, float2* __restrict__ twy, int nx, int ny, int os) {
  const int nt = os * nx;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double inv_sqrt_nt = 1.0 / sqrt((double)nt);
  const double sgn_nx = ((nx / 2) & 1) ? -1.0 : 1.0;
  for (size_t i = gid; i < (size_t)ny * nt; i += stride) {
    const int t = (int)(i % nt);
    const int q = t / os, s = t - q * os;
    double sn, cs;
    sincospi((double)s / os, &sn, &cs);
    const double sg = sgn_nx * ((q & 1) ? -1.0 : 1.0) * inv_sqrt_nt;
    const double pr = sg * cs, pi = sg * sn;
    const float2 v = psf[i];
    psfp[i] = make_float2((float)(v.x * pr - v.y * pi), (float)(v.x * pi + v.y * pr));
  }
  for (size_t i = gid; i < (size_t)os * nx; i += stride) {
    const int s = (int)(i / nx), x = (int)(i % nx);
    const long m = ((long)s * x) % nt;
    double sn, cs;
    sincospi(-2.0 * (double)m / nt, &sn, &cs);
    const double sg = (x & 1) ? -1.0 : 1.0;
    twin[i] = make_float2((float)(sg * cs), (float)(sg * sn));
  }
  for (size_t i = gid; i < (size_t)nx; i += stride) {
    double sn, cs;
    sincospi(-2.0 * (double)i / nx, &sn, &cs);
    twx[i] = make_float2((float)cs, (float)sn);
  }
  for (size_t i = gid; i < (size_t)ny; i += stride) {
    double sn, cs;
    sincospi(-2.0 * (double)i / ny, &sn, &cs);
    twy[i] = make_float2((float)cs, (float)sn);
  }
}

int launch_prep_tables(Plan& pl) {
  hipLaunchKernelGGL(k_prep_tables, dim3(256), dim3(256), 0, pl.stream, pl.psf, pl.psfp, pl.twin, pl.tw_x,
                     pl.tw_y, pl.nx, pl.ny, pl.os);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// t / os for t < 2^16 and a small runtime os, through a float reciprocal:
// (t + 0.5) / os stays at least 0.5 / os away from every integer, far more
// than the float rounding of the product.
__device__ inline int div_os(int t, float inv_os) { return (int)(((float)t + 0.5f) * inv_os); }

// ---------------------------------------------------------------------------
// F1: W[b][n][y][t] = psfp[y][t] * FFT_Nx(coil * img * twin[s])[q]
// grid (row blocks, nc, B); `rows` image rows per work-group.  LDS lines are
// padded (fft.h): line (r, s) holds the s-th sub-transform of row r.
// ---------------------------------------------------------------------------
template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_fwd(const float2* __restrict__ img, const float2* __restrict__ coils,
                                                     const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                     const float2* __restrict__ tw, void* __restrict__ W, int ny,
                                                     int nc, int os, float inv_os, int rows) {
  constexpr int LS = fline(NX);
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  const int nt = os * NX;
  const int n = blockIdx.y, b = blockIdx.z;
  const int y0 = blockIdx.x * rows;
  const int nr = min(rows, ny - y0);
  float2* twl = sm;
  float2* bufA = sm + NX;
  float2* bufB = bufA + rows * os * LS;
  for (int i = tid; i < NX; i += 256) twl[i] = tw[i];
  const float2* cp = coils + ((size_t)n * ny + y0) * NX;
  const float2* ip = img + ((size_t)b * ny + y0) * NX;
  for (int i = tid; i < nr * NX; i += 256) {
    const int r = i / NX, x = i - r * NX;
    const float2 u = cmul(cp[i], ip[i]);
    float2* dst = bufA + r * os * LS + fpad(x);
    for (int s = 0; s < os; ++s) dst[s * LS] = cmul(u, twin[s * NX + x]);
  }
  // PSF samples of the first row are fetched before the transform so their
  // latency overlaps it (nt <= 16 * 256 samples per row).
  constexpr int PF = 16;
  float2 pv[PF];
  const float2* ps0 = psfp + (size_t)y0 * nt;
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const int t = tid + 256 * k;
    if (t < nt) pv[k] = ps0[t];
  }
  __syncthreads();
  const float2* res = fft_lines<NX>(bufA, bufB, twl, nr * os, LS, tid, 256, wg_sync);
  for (int r = 0; r < nr; ++r) {
    const size_t ob = (((size_t)b * nc + n) * ny + y0 + r) * nt;
    const float2* ps = psfp + (size_t)(y0 + r) * nt;
    const float2* rr = res + r * os * LS;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int t = tid + 256 * k;
      if (t < nt) {
        const int q = div_os(t, inv_os), s = t - q * os;
        const float2 psv = r == 0 ? pv[k] : ps[t];
        store_c<ST>(W, ob + t, cmul(psv, rr[s * LS + fpad(q)]));
      }
    }
  }
}

// F1^H for one image row and a chunk of coils: conj PSF, inverse readout DFT,
// crop, sum over the chunk of conj(coil) * line.  grid (ny, nchunk, B).
template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_adj(const void* __restrict__ W, const float2* __restrict__ coils,
                                                     const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                     const float2* __restrict__ tw, float2* __restrict__ part, int ny,
                                                     int nc, int os, float inv_os, int cb, int cpc, int B) {
  constexpr int LS = fline(NX);
  extern __shared__ float2 sm[];
  constexpr int PER = (NX + 255) / 256;
  const int tid = threadIdx.x;
  const int nt = os * NX;
  const int y = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z;
  float2* twl = sm;
  float2* bufA = sm + NX;
  float2* bufB = bufA + cb * os * LS;
  for (int i = tid; i < NX; i += 256) twl[i] = tw[i];
  float2 acc[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) acc[e] = make_float2(0.f, 0.f);
  const int nb = chunk * cpc, ne = min(nc, nb + cpc);
  const float2* ps = psfp + (size_t)y * nt;
  for (int n0 = nb; n0 < ne; n0 += cb) {
    const int ncb = min(cb, ne - n0);
    for (int c = 0; c < ncb; ++c) {
      const size_t wb = (((size_t)b * nc + n0 + c) * ny + y) * nt;
      float2* dst = bufA + c * os * LS;
      for (int t = tid; t < nt; t += 256) {
        const int q = div_os(t, inv_os), s = t - q * os;
        dst[s * LS + fpad(q)] = cmulc(ps[t], load_c<ST>(W, wb + t));  // conj(conj(psf) * w)
      }
    }
    __syncthreads();
    const float2* res = fft_lines<NX>(bufA, bufB, twl, ncb * os, LS, tid, 256, wg_sync);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int x = tid + e * 256;
      if (x < NX) {
        for (int c = 0; c < ncb; ++c) {
          float2 v = make_float2(0.f, 0.f);
          const float2* rc = res + c * os * LS + fpad(x);
          for (int s = 0; s < os; ++s) v = cadd(v, cmul(rc[s * LS], twin[s * NX + x]));
          // v holds conj of the cropped line; acc += conj(coil) * line
          const float2 cv = coils[((size_t)(n0 + c) * ny + y) * NX + x];
          acc[e] = cadd(acc[e], cconj(cmul(v, cv)));
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int x = tid + e * 256;
    if (x < NX) part[(((size_t)chunk * B + b) * ny + y) * NX + x] = acc[e];
  }
}

// ---------------------------------------------------------------------------
// Two-pass form of F1 (N = N1 N2, see fft2.h).  One work-group takes one
// image row and cb coils, i.e. cb * os sub-transforms of length NX; the first
// pass is an N1-point DFT per (coil, sub-transform, i2) in registers, the
// second an N2-point DFT per (coil, sub-transform, k1).  The launch keeps
// cb * os * N1 <= blockDim.x so every second-pass item has its own thread,
// which lets results overwrite the exchange buffer after one barrier.  The
// PSF row is read once for all cb coils; the pre-twiddle table (os x NX) is
// read through the L1 cache, shared by all work-groups of a CU.
// ---------------------------------------------------------------------------
__device__ inline int udiv(int a, int b) { return (int)(((float)a + 0.5f) / (float)b); }  // a < 2^16, b small
constexpr int kPsfRegs = 8;  // readout samples per thread held in registers by k_readout_fwd2 / _adj2
constexpr int kSetupRegs = 2;  // coil x image elements per thread and round of loads in k_readout_fwd2

template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_fwd2(const float2* __restrict__ img, const float2* __restrict__ coils,
                                                      const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                      const float2* __restrict__ tw, void* __restrict__ W, int ny,
                                                      int nc, int os, int cb) {
  using S = Split<NX>;
  constexpr int N1 = S::N1, N2 = S::N2, AS = N1 + 1;
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nt = os * NX;
  const int y = blockIdx.x, n0 = blockIdx.y * cb, b = blockIdx.z;
  const int ncb = min(cb, nc - n0);
  float2* twl = sm;         // [NX]       exp(-2 pi i m / NX)
  float2* u = twl + NX;     // [cb][NX]   coil * image
  float2* A = u + cb * NX;  // [cb][os][N2][AS], then the output rows [cb][nt]
  const float2* ip = img + ((size_t)b * ny + y) * NX;
  {
    // The set-up loads (coil and image rows, twiddles) are issued before any
    // is used: kSetupRegs elements per thread, clamped indices; a loop takes
    // the rest of rows longer than that (cb NX > kSetupRegs blockDim).
    const int tot = ncb * NX;
    float2 cv[kSetupRegs], iv[kSetupRegs];
#pragma unroll
    for (int k = 0; k < kSetupRegs; ++k) {
      const int i = min(tid + k * nthr, tot - 1), c = i / NX, x = i - c * NX;
      cv[k] = coils[((size_t)(n0 + c) * ny + y) * NX + x];
      iv[k] = ip[x];
    }
    const float2 twv = tw[min(tid, NX - 1)];
#pragma unroll
    for (int k = 0; k < kSetupRegs; ++k) {
      const int i = tid + k * nthr;
      if (i < tot) u[i] = cmul(cv[k], iv[k]);
    }
    for (int i = tid + kSetupRegs * nthr; i < tot; i += nthr) {
      const int c = i / NX, x = i - c * NX;
      u[i] = cmul(coils[((size_t)(n0 + c) * ny + y) * NX + x], ip[x]);
    }
    if (tid < NX) twl[tid] = twv;
    for (int i = tid + nthr; i < NX; i += nthr) twl[i] = tw[i];
  }
  __syncthreads();
  const int items1 = ncb * os * N2;
  for (int it = tid; it < items1; it += nthr) {
    const int r = it / N2, i2 = it - r * N2;  // r = c * os + s
    const int c = udiv(r, os), s = r - c * os;
    float2 v[N1];
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) v[i1] = cmul(u[c * NX + i2 + N2 * i1], twin[s * NX + i2 + N2 * i1]);
    rdft<N1>(v);
    float2* dst = A + (r * N2 + i2) * AS;
    dst[0] = v[0];
    int m = i2;
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      dst[k1] = cmul(v[k1], twl[m]);
      m += i2;
      m = m >= NX ? m - NX : m;
    }
  }
  __syncthreads();
  // The PSF samples of the output phase are loaded here, behind the second
  // pass.  Loads and stores retire in issue order, so a load issued between
  // the output stores could only be waited for together with them.
  const float2* ps = psfp + (size_t)y * nt;
  float2 pv[kPsfRegs];
#pragma unroll
  for (int k = 0; k < kPsfRegs; ++k) pv[k] = ps[min(tid + k * nthr, nt - 1)];  // past the end: dropped
  const int items2 = ncb * os * N1;
  const bool act = tid < items2;
  float2 w[N2];
  int r2 = 0, k1 = 0;
  if (act) {
    r2 = tid / N1;
    k1 = tid - r2 * N1;
    const float2* src = A + r2 * N2 * AS + k1;
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) w[i2] = src[i2 * AS];
    rdft<N2>(w);
  }
  __syncthreads();
  if (act) {
    const int c = udiv(r2, os), s = r2 - c * os;
    float2* o = A + c * nt + s;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) o[(k1 + N1 * k2) * os] = w[k2];
  }
  __syncthreads();
  for (int c = 0; c < ncb; ++c) {
    const size_t row = (((size_t)b * nc + n0 + c) * ny + y) * nt;
    const float2* ar = A + c * nt;
#pragma unroll
    for (int k = 0; k < kPsfRegs; ++k) {
      const int t = tid + k * nthr;
      if (t < nt) store_c<ST>(W, row + t, cmul(pv[k], ar[t]));
    }
  }
  for (int t = tid + kPsfRegs * nthr; t < nt; t += nthr) {
    const float2 p = ps[t];
    for (int c = 0; c < ncb; ++c)
      store_c<ST>(W, (((size_t)b * nc + n0 + c) * ny + y) * nt + t, cmul(p, A[c * nt + t]));
  }
}

// Two-pass form of F1^H: one work-group per image row and cb coils, leaving
// one partial image per coil group.  The inputs conj(psf) w are scattered to
// sub-transform rows (padded to os (mod 32) slots so consecutive samples land
// on consecutive banks); the inverse DFT of length NX per sub-transform is
// taken as conj(FFT(conj(.))) with the two passes of the forward form; the
// sum over sub-transforms of the pre-twiddled results and the coil
// combination follow.  Pre-twiddles are read from the (L1-resident) table.
// Grid (kAdjRowBlock x chunks, row blocks, B): the chunks of kAdjRowBlock
// consecutive rows are consecutive work-groups, so they find each row's PSF
// in L2 (sweeping all rows of one chunk after another took a volume's PSF,
// Nz Ny Nt samples, from HBM once per chunk), while the W rows read at one
// time stay kAdjRowBlock consecutive rows of each coil.
constexpr int kAdjRowBlock = 16;
template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_adj2(const void* __restrict__ W, const float2* __restrict__ coils,
                                                      const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                      const float2* __restrict__ tw, float2* __restrict__ part, int ny,
                                                      int nc, int os, int cb, int B) {
  using S = Split<NX>;
  constexpr int N1 = S::N1, N2 = S::N2, AS = N1 + 1;
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nt = os * NX;
  const int nxp = NX + ((os - NX % 32) % 32 + 32) % 32;
  const int y = blockIdx.y * kAdjRowBlock + blockIdx.x % kAdjRowBlock;
  const int chunk = blockIdx.x / kAdjRowBlock, b = blockIdx.z;
  if (y >= ny) return;  // the last row block's spare work-groups
  const int n0 = chunk * cb, ncb = min(cb, nc - n0);
  float2* twl = sm;       // [NX]
  float2* X = twl + NX;   // [cb][os][nxp] inputs, then [cb][os][N2][AS], then [cb][os][NX] results
  const float2 twv = tw[min(tid, NX - 1)];  // stored below, behind the sample loads
  const float2* ps = psfp + (size_t)y * nt;
  // kPsfRegs samples per thread and coil are loaded before any is used, so
  // that many loads are in flight instead of one sample's.  Samples past the
  // row end load the last sample (no branch around a load) and are dropped.
  float2 pv[kPsfRegs];
  int xo[kPsfRegs];  // LDS slot (s, q) of sample t, without the coil offset
#pragma unroll
  for (int k = 0; k < kPsfRegs; ++k) {
    const int t = tid + k * nthr;
    const int q = udiv(t, os), s = t - q * os;
    pv[k] = ps[min(t, nt - 1)];
    xo[k] = s * nxp + q;
  }
  for (int c = 0; c < ncb; ++c) {
    const size_t row = (((size_t)b * nc + n0 + c) * ny + y) * nt;
    float2 wv[kPsfRegs];
#pragma unroll
    for (int k = 0; k < kPsfRegs; ++k) wv[k] = load_c<ST>(W, row + min(tid + k * nthr, nt - 1));
#pragma unroll
    for (int k = 0; k < kPsfRegs; ++k)
      if (tid + k * nthr < nt) X[c * os * nxp + xo[k]] = cmulc(pv[k], wv[k]);
  }
  for (int t = tid + kPsfRegs * nthr; t < nt; t += nthr) {
    const int q = udiv(t, os), s = t - q * os;
    const float2 p = ps[t];
    for (int c = 0; c < ncb; ++c)
      X[(c * os + s) * nxp + q] = cmulc(p, load_c<ST>(W, (((size_t)b * nc + n0 + c) * ny + y) * nt + t));
  }
  if (tid < NX) twl[tid] = twv;
  for (int i = tid + nthr; i < NX; i += nthr) twl[i] = tw[i];
  __syncthreads();
  const int items1 = ncb * os * N2;  // <= blockDim.x
  float2 v[N1];
  int r1 = 0, i2 = 0;
  const bool act1 = tid < items1;
  if (act1) {
    r1 = tid / N2;
    i2 = tid - r1 * N2;
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) v[i1] = X[r1 * nxp + i2 + N2 * i1];
  }
  __syncthreads();
  if (act1) {
    rdft<N1>(v);
    float2* dst = X + (r1 * N2 + i2) * AS;
    dst[0] = v[0];
    int m = i2;
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      dst[k1] = cmul(v[k1], twl[m]);
      m += i2;
      m = m >= NX ? m - NX : m;
    }
  }
  __syncthreads();
  const int items2 = ncb * os * N1;  // <= blockDim.x
  float2 w[N2];
  int r2 = 0, k1 = 0;
  const bool act2 = tid < items2;
  if (act2) {
    r2 = tid / N1;
    k1 = tid - r2 * N1;
    const float2* src = X + r2 * N2 * AS + k1;
#pragma unroll
    for (int j = 0; j < N2; ++j) w[j] = src[j * AS];
    rdft<N2>(w);
  }
  __syncthreads();
  if (act2) {
    // the inverse sub-transform is conj(w); keep twin * w, whose sum over s is
    // the conjugate of the pre-twiddled sum
    const int s = r2 - udiv(r2, os) * os;
    float2* o = X + r2 * NX;
    const float2* tws = twin + s * NX;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int x = k1 + N1 * k2;
      o[x] = cmul(w[k2], tws[x]);
    }
  }
  __syncthreads();
  float2* pp = part + (((size_t)chunk * B + b) * ny + y) * NX;
  for (int x = tid; x < NX; x += nthr) {
    float2 acc = make_float2(0.f, 0.f);
    for (int c = 0; c < ncb; ++c) {
      float2 v2 = make_float2(0.f, 0.f);
      for (int s = 0; s < os; ++s) v2 = cadd(v2, X[(c * os + s) * NX + x]);
      acc = cadd(acc, cconj(cmul(v2, coils[((size_t)(n0 + c) * ny + y) * NX + x])));
    }
    pp[x] = acc;
  }
}

__global__ void k_combine(const float2* __restrict__ part, int nchunk, size_t n, float2* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = sum_chunks(part, nchunk, n, i);
}

// ---------------------------------------------------------------------------
// F3 on compressed lines Z[l][y], l = (b, p, k), y contiguous.
// post(ky) = (-1)^(Ny/2) (-1)^ky / sqrt(Ny); pre-twiddle (-1)^y.
// ---------------------------------------------------------------------------
template <int NY>
__device__ inline float pe_post(int ky) {
  const float s = (((NY / 2) + ky) & 1) ? -1.f : 1.f;
  return s * (1.0f / sqrtf((float)NY));
}

// Sums over the k-split partials of elements i = tid + 256 it (it < IT) of
// the nel consecutive elements at base, in partial order (the same values as
// adding them one by one).  The loads of kSumBatch partials of all IT
// elements are issued before any is added, so they are in flight together.
constexpr int kSumBatch = 3;
template <int IT>
__device__ inline void sum_partials(float2 (&a)[IT], const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                    size_t base, int nel, int tid) {
#pragma unroll
  for (int it = 0; it < IT; ++it) a[it] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < ksplit; k0 += kSumBatch) {
    float2 v[kSumBatch][IT];
#pragma unroll
    for (int h = 0; h < kSumBatch; ++h)
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = min(tid + 256 * it, nel - 1);  // past the end: a valid element, dropped by the caller
        v[h][it] = k0 + h < ksplit ? Zp[(size_t)(k0 + h) * zstride + base + i] : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int h = 0; h < kSumBatch; ++h)
#pragma unroll
      for (int it = 0; it < IT; ++it) a[it] = cadd(a[it], v[h][it]);
  }
}

template <int NY>
__device__ inline void load_z_lines(float2* A, const float2* __restrict__ Zp, int ksplit, size_t zstride, int l0,
                                    int nl, int tid) {
  constexpr int LS = fline(NY);
  constexpr int IT = 4;  // elements per thread and round of loads
  const int nel = nl * NY;
  for (int i0 = 0; i0 < nel; i0 += IT * 256) {
    float2 a[IT];
    sum_partials<IT>(a, Zp, ksplit, zstride, (size_t)l0 * NY + i0, nel - i0, tid);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = i0 + tid + 256 * it;
      if (i < nel) {
        const int li = i / NY, y = i - li * NY;
        A[li * LS + fpad(y)] = (y & 1) ? make_float2(-a[it].x, -a[it].y) : a[it];
      }
    }
  }
}

template <int NY>
__global__ __launch_bounds__(256) void k_pe_fwd(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                float2* __restrict__ out, const int* __restrict__ lines, int ms,
                                                int nlines, int lpb, const float2* __restrict__ tw) {
  constexpr int LS = fline(NY);
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * LS;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  load_z_lines<NY>(A, Zp, ksplit, zstride, l0, nl, tid);
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, LS, tid, 256, wg_sync);
  for (int i = tid; i < nl * ms; i += 256) {
    const int li = i / ms, m = i - li * ms;
    const int ky = lines[m];
    out[(size_t)l0 * ms + i] = cscale(res[li * LS + fpad(ky)], pe_post<NY>(ky));
  }
}

// Adjoint: zero-fill, inverse DFT; writes Zt[(b,p)][y][k] (k contiguous, stride kp), stored as ST.
template <int NY, Store ST>
__global__ __launch_bounds__(256) void k_pe_adj(const float2* __restrict__ in, void* __restrict__ Zt,
                                                const int* __restrict__ lines, int ms, int nlines, int lpb, int K,
                                                int kp, const float2* __restrict__ tw) {
  constexpr int LS = fline(NY);
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * LS;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  for (int i = tid; i < nl * LS; i += 256) A[i] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int i = tid; i < nl * ms; i += 256) {
    const int li = i / ms, m = i - li * ms;
    const int ky = lines[m];
    A[li * LS + fpad(ky)] = cscale(cconj(in[(size_t)l0 * ms + i]), pe_post<NY>(ky));
  }
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, LS, tid, 256, wg_sync);
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, li = i - y * nl;
    const int l = l0 + li;
    const int bp = l / K, k = l - bp * K;
    float2 v = cconj(res[li * LS + fpad(y)]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    store_zt<ST>(Zt, (size_t)bp * NY + y, kp, k, v);
  }
}

// Normal y-stage: (-1)^y conj(FFT(conj(mask/Ny * FFT((-1)^y z)))) -> Zt.
template <int NY, Store ST>
__global__ __launch_bounds__(256) void k_pe_normal(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                   void* __restrict__ Zt, const float* __restrict__ maskf,
                                                   int nlines, int lpb, int K, int kp,
                                                   const float2* __restrict__ tw) {
  constexpr int LS = fline(NY);
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * LS;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  load_z_lines<NY>(A, Zp, ksplit, zstride, l0, nl, tid);
  __syncthreads();
  float2* res = fft_lines<NY>(A, Bf, twl, nl, LS, tid, 256, wg_sync);
  const float inv = 1.0f / (float)NY;
  for (int i = tid; i < nl * NY; i += 256) {
    const int li = i / NY, ky = i - li * NY;
    float2& v = res[li * LS + fpad(ky)];
    v = cconj(cscale(v, maskf[ky] * inv));
  }
  __syncthreads();
  float2* other = (res == A) ? Bf : A;
  const float2* res2 = fft_lines<NY>(res, other, twl, nl, LS, tid, 256, wg_sync);
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, li = i - y * nl;
    const int l = l0 + li;
    const int bp = l / K, k = l - bp * K;
    float2 v = cconj(res2[li * LS + fpad(y)]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    store_zt<ST>(Zt, (size_t)bp * NY + y, kp, k, v);
  }
}

// Two-pass form of the normal y-stage for NY = N1 N2, L lines per
// work-group (256 threads).  All threads first sum the k-split partials of
// the lines into LDS (coalesced along y).  Per line, the forward transform's
// first pass (N1-point DFTs of stride-N2 subsequences, twiddled), one
// exchange, its second pass (N2-point DFTs) -- which leaves each thread the
// spectrum subsequence ky = k1 + N1 k2 -- then mask / NY and conjugation, and,
// in the same registers, the first pass of the second transform taken the
// other way round (N2-point DFTs over k2, twiddled), one more exchange, and
// N1-point DFTs giving y = m2 + N2 n1.
template <int NY>
struct PeNormal2Geo {
  static constexpr int N1 = Split<NY>::N1, N2 = Split<NY>::N2, AS = N1 + 1;
  static constexpr int L = 64 / (N1 > N2 ? N1 : N2) > 0 ? 64 / (N1 > N2 ? N1 : N2) : 1;  // lines per work-group
  static constexpr int NYP = NY + 1;
};

template <int NY, Store ST>
__global__ __launch_bounds__(256) void k_pe_normal2(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                    void* __restrict__ Zt, const float* __restrict__ maskf, int nlines,
                                                    int K, int kp, const float2* __restrict__ tw) {
  using Gm = PeNormal2Geo<NY>;
  constexpr int N1 = Gm::N1, N2 = Gm::N2, AS = Gm::AS, L = Gm::L, NYP = Gm::NYP;
  __shared__ float2 twl[NY];
  __shared__ float2 Zs[L * NYP];
  __shared__ float2 E[L * N2 * AS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * L;
  const int nl = min(L, nlines - l0);
  {
    constexpr int IT = (L * NY + 255) / 256;
    float2 a[IT];
    sum_partials<IT>(a, Zp, ksplit, zstride, (size_t)l0 * NY, nl * NY, tid);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = tid + 256 * it;
      if (i < nl * NY) {
        const int ln = i / NY, y = i - ln * NY;
        Zs[ln * NYP + y] = (y & 1) ? make_float2(-a[it].x, -a[it].y) : a[it];
      }
    }
  }
  __syncthreads();
  if (tid < nl * N2) {  // forward, first pass: item (line, i2)
    const int ln = tid / N2, i2 = tid - ln * N2;
    float2 v[N1];
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) v[i1] = Zs[ln * NYP + i2 + N2 * i1];
    rdft<N1>(v);
    float2* dst = E + (ln * N2 + i2) * AS;
    dst[0] = v[0];
    int m = i2;
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      dst[k1] = cmul(v[k1], twl[m]);
      m += i2;
      m = m >= NY ? m - NY : m;
    }
  }
  __syncthreads();
  // forward second pass, mask, and the second transform's first pass: item (line, k1)
  float2 w[N2];
  int ln2 = 0, k1 = 0;
  const bool act2 = tid < nl * N1;
  if (act2) {
    ln2 = tid / N1;
    k1 = tid - ln2 * N1;
    const float2* src = E + ln2 * N2 * AS + k1;
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) w[i2] = src[i2 * AS];
    rdft<N2>(w);  // w[k2] = F[k1 + N1 k2]
    const float inv = 1.0f / (float)NY;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) w[k2] = cconj(cscale(w[k2], maskf[k1 + N1 * k2] * inv));
    rdft<N2>(w);  // over k2: w[m2] = sum_k2 g[k1 + N1 k2] w_N2^{k2 m2}
  }
  __syncthreads();
  if (act2) {
    float2* dst = E + ln2 * N2 * AS + k1;
    int m = 0;
#pragma unroll
    for (int m2 = 0; m2 < N2; ++m2) {
      dst[m2 * AS] = cmul(w[m2], twl[m]);  // twiddle w_NY^{k1 m2}
      m += k1;
      m = m >= NY ? m - NY : m;
    }
  }
  __syncthreads();
  if (tid < nl * N2) {  // second transform, last pass: item (line, m2)
    const int ln = tid / N2, m2 = tid - ln * N2;
    float2 v[N1];
    const float2* src = E + (ln * N2 + m2) * AS;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = src[n1];
    rdft<N1>(v);  // v[n1] = G[m2 + N2 n1]
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int y = m2 + N2 * n1;
      float2 r = cconj(v[n1]);
      if (y & 1) r = make_float2(-r.x, -r.y);
      Zs[ln * NYP + y] = r;
    }
  }
  __syncthreads();
  // transposed store, k fastest within each (b, p)
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, ln = i - y * nl;
    const int l = l0 + ln;
    const int bp = l / K, k = l - bp * K;
    store_zt<ST>(Zt, (size_t)bp * NY + y, kp, k, Zs[ln * NYP + y]);
  }
}

// ---------------------------------------------------------------------------
// F3 on uncompressed columns W[(b,n)][y][t] (stride nt).  Work-group: one
// (b, n) and `tb` consecutive t.
// ---------------------------------------------------------------------------
template <int NY, Store ST>
__global__ __launch_bounds__(256) void k_pe_cols(const void* __restrict__ Win, void* __restrict__ Wout,
                                                 const float2* __restrict__ in_s, float2* __restrict__ out_s,
                                                 const int* __restrict__ lines, const float* __restrict__ maskf,
                                                 int ms, int nt, int tb, int mode, const float2* __restrict__ tw) {
  // mode 0: forward W -> out_s [(b,n)][ms][nt]; 1: adjoint in_s -> Wout; 2: normal Win -> Wout
  constexpr int LS = fline(NY);
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + tb * LS;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int t0 = blockIdx.x * tb;
  const int ntb = min(tb, nt - t0);
  const size_t bn = blockIdx.y;
  if (mode == 1) {
    for (int i = tid; i < ntb * LS; i += 256) A[i] = make_float2(0.f, 0.f);
    __syncthreads();
    for (int i = tid; i < ms * ntb; i += 256) {
      const int m = i / ntb, c = i - m * ntb;
      const int ky = lines[m];
      A[c * LS + fpad(ky)] = cscale(cconj(in_s[(bn * ms + m) * nt + t0 + c]), pe_post<NY>(ky));
    }
  } else {
    for (int i = tid; i < NY * ntb; i += 256) {
      const int y = i / ntb, c = i - y * ntb;
      float2 v = load_c<ST>(Win, (bn * NY + y) * nt + t0 + c);
      A[c * LS + fpad(y)] = (y & 1) ? make_float2(-v.x, -v.y) : v;
    }
  }
  __syncthreads();
  float2* res = fft_lines<NY>(A, Bf, twl, ntb, LS, tid, 256, wg_sync);
  if (mode == 0) {
    for (int i = tid; i < ms * ntb; i += 256) {
      const int m = i / ntb, c = i - m * ntb;
      const int ky = lines[m];
      out_s[(bn * ms + m) * nt + t0 + c] = cscale(res[c * LS + fpad(ky)], pe_post<NY>(ky));
    }
    return;
  }
  if (mode == 2) {
    const float inv = 1.0f / (float)NY;
    for (int i = tid; i < ntb * NY; i += 256) {
      const int c = i / NY, ky = i - c * NY;
      float2& v = res[c * LS + fpad(ky)];
      v = cconj(cscale(v, maskf[ky] * inv));
    }
    __syncthreads();
    float2* other = (res == A) ? Bf : A;
    res = fft_lines<NY>(res, other, twl, ntb, LS, tid, 256, wg_sync);
  }
  for (int i = tid; i < NY * ntb; i += 256) {
    const int y = i / ntb, c = i - y * ntb;
    float2 v = cconj(res[c * LS + fpad(y)]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    store_c<ST>(Wout, (bn * NY + y) * nt + t0 + c, v);
  }
}

// ---------------------------------------------------------------------------
// Centred DFTs along the columns of uncompressed planes, in place, two-pass
// register form (as k_pe_normal2).  Element e of column c of plane q sits at
// W[q pstride + e estride + c], c < ncols: for a slice, planes (b, n) with
// columns t (estride = ncols = Nt); for a volume's y pass, planes (b, n, z)
// likewise; for its z pass, planes (b, n) with columns y Nt + t (estride =
// ncols = Ny Nt).  Work-group: L consecutive columns of one plane; lane ln =
// tid % L owns column c0 + ln, so every global access is an L-sample row
// segment.  The first pass reads its stride-N2 inputs straight from W and the
// last pass writes straight back; only the exchanges go through LDS, laid out
// with the column index fastest.  N = N1 N2, L max(N1, N2) <= 256.
// ---------------------------------------------------------------------------
template <int N, int N1_>
struct Cols2Geo {
  static constexpr int N1 = N1_, N2 = N / N1_;
  static constexpr int L = 256 / (N1 > N2 ? N1 : N2);  // columns per work-group
};

// N1 <= sqrt(N) as large as possible with 256 divisible by N / N1 (so every
// thread has an item in the first pass); the slice's factors otherwise.
constexpr int cols_n1(int n) {
  int best = 1;
  for (int d = 2; d * d <= n; ++d)
    if (n % d == 0 && n / d <= 32 && 256 % (n / d) == 0 && reg_dft_ok(d) && reg_dft_ok(n / d)) best = d;
  return best > 1 ? best : split_n1(n);
}

// F^H M F per column: mask maskf[k mstride + c / cdiv] at frequency k of
// column c (a slice: mstride 1, cdiv = ncols; a volume's z pass: mstride Ny,
// cdiv Nt, the mask row of the column's ky).
template <int NY, int N1_>
__global__ __launch_bounds__(256) void k_pe_cols_normal2(float2* __restrict__ W, size_t pstride, size_t estride,
                                                         int ncols, const float* __restrict__ maskf, int mstride,
                                                         int cdiv, const float2* __restrict__ tw) {
  using Gm = Cols2Geo<NY, N1_>;
  constexpr int N1 = Gm::N1, N2 = Gm::N2, L = Gm::L;
  __shared__ float2 twl[NY];
  __shared__ float2 E[N1 * N2 * L];  // element (i2, k1) of column ln at (i2 N1 + k1) L + ln
  const int tid = threadIdx.x;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int c0 = blockIdx.x * L;
  const int ln = tid % L, it = tid / L;
  const bool colok = c0 + ln < ncols;
  const int moff = colok ? (c0 + ln) / cdiv : 0;
  float2* col = W + (size_t)blockIdx.y * pstride + c0 + ln;  // element y of this column at col[y estride]
  float2 v[N1];
  if (it < N2) {  // forward, first pass: item (ln, i2 = it)
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) {
      const int y = it + N2 * i1;
      const float2 a = colok ? col[(size_t)y * estride] : make_float2(0.f, 0.f);
      v[i1] = (y & 1) ? make_float2(-a.x, -a.y) : a;
    }
  }
  __syncthreads();  // twiddle table
  if (it < N2) {
    rdft<N1>(v);
    E[(it * N1) * L + ln] = v[0];
    int m = it;
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      E[(it * N1 + k1) * L + ln] = cmul(v[k1], twl[m]);
      m += it;
      m = m >= NY ? m - NY : m;
    }
  }
  __syncthreads();
  // forward second pass, mask, and the second transform's first pass: item (ln, k1 = it)
  float2 w[N2];
  const bool act2 = it < N1;
  if (act2) {
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) w[i2] = E[(i2 * N1 + it) * L + ln];
    rdft<N2>(w);  // w[k2] = F[k1 + N1 k2]
    const float inv = 1.0f / (float)NY;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2)
      w[k2] = cconj(cscale(w[k2], maskf[(size_t)(it + N1 * k2) * mstride + moff] * inv));
    rdft<N2>(w);
  }
  __syncthreads();
  if (act2) {
    int m = 0;
#pragma unroll
    for (int m2 = 0; m2 < N2; ++m2) {
      E[(m2 * N1 + it) * L + ln] = cmul(w[m2], twl[m]);  // twiddle w_NY^{k1 m2}
      m += it;
      m = m >= NY ? m - NY : m;
    }
  }
  __syncthreads();
  if (it < N2 && colok) {  // second transform, last pass: item (ln, m2 = it)
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = E[(it * N1 + n1) * L + ln];
    rdft<N1>(v);  // v[n1] = G[m2 + N2 n1]
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) {
      const int y = it + N2 * n1;
      float2 r = cconj(v[n1]);
      if (y & 1) r = make_float2(-r.x, -r.y);
      col[(size_t)y * estride] = r;
    }
  }
}

// The centred DFT (inverse = 0) or its inverse (1) of every column.  Forward:
// x[e] (-1)^e in, X[k] pe_post(k) out; inverse: conj(X[k]) pe_post(k) in,
// conj(.) (-1)^e out.
template <int N, int N1_>
__global__ __launch_bounds__(256) void k_cols2(float2* __restrict__ W, size_t pstride, size_t estride, int ncols,
                                               int inverse, const float2* __restrict__ tw) {
  using Gm = Cols2Geo<N, N1_>;
  constexpr int N1 = Gm::N1, N2 = Gm::N2, L = Gm::L;
  __shared__ float2 twl[N];
  __shared__ float2 E[N1 * N2 * L];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += 256) twl[i] = tw[i];
  const int c0 = blockIdx.x * L;
  const int ln = tid % L, it = tid / L;
  const bool colok = c0 + ln < ncols;
  float2* col = W + (size_t)blockIdx.y * pstride + c0 + ln;
  float2 v[N1];
  if (it < N2) {  // first pass: item (ln, i2 = it)
#pragma unroll
    for (int i1 = 0; i1 < N1; ++i1) {
      const int e = it + N2 * i1;
      const float2 a = colok ? col[(size_t)e * estride] : make_float2(0.f, 0.f);
      v[i1] = inverse ? cscale(cconj(a), pe_post<N>(e)) : ((e & 1) ? make_float2(-a.x, -a.y) : a);
    }
  }
  __syncthreads();  // twiddle table
  if (it < N2) {
    rdft<N1>(v);
    E[(it * N1) * L + ln] = v[0];
    int m = it;
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      E[(it * N1 + k1) * L + ln] = cmul(v[k1], twl[m]);
      m += it;
      m = m >= N ? m - N : m;
    }
  }
  __syncthreads();
  if (it < N1 && colok) {  // second pass: item (ln, k1 = it), outputs k1 + N1 k2
    float2 w[N2];
#pragma unroll
    for (int i2 = 0; i2 < N2; ++i2) w[i2] = E[(i2 * N1 + it) * L + ln];
    rdft<N2>(w);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int e = it + N1 * k2;
      float2 r;
      if (inverse) {
        r = cconj(w[k2]);
        if (e & 1) r = make_float2(-r.x, -r.y);
      } else {
        r = cscale(w[k2], pe_post<N>(e));
      }
      col[(size_t)e * estride] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side sizing of the two-pass readout forms (complex elements of LDS).
// ---------------------------------------------------------------------------
size_t two_pass_lds_fwd(int nx, int os, int cb) {
  const int n1 = split_n1(nx), n2 = nx / n1;
  const size_t a = (size_t)cb * os * n2 * (n1 + 1), o = (size_t)cb * os * nx;
  return (size_t)nx + (size_t)cb * nx + (a > o ? a : o);
}
size_t two_pass_lds_adj(int nx, int os, int cb) {
  const int n1 = split_n1(nx), n2 = nx / n1;
  const size_t in = (size_t)nx + ((os - nx % 32) % 32 + 32) % 32, ex = (size_t)n2 * (n1 + 1);
  return (size_t)nx + (size_t)cb * os * (in > ex ? in : ex);
}
// Coils per work-group of the two-pass forward form (0 = not applicable):
// every second-pass item needs its own thread (at most 256) and the LDS must
// fit in 64 KiB.
int two_pass_coils(int nx, int os, int nc, int* threads) {
  const int n1 = split_n1(nx), n2 = nx / n1;
  if (n1 <= 1 || n2 <= 1 || n2 > 32) return 0;
  for (int cb = std::min(nc, 4); cb >= 1; --cb) {
    const int items = cb * os * std::max(n1, n2);
    if (items > 256) continue;
    if (two_pass_lds_fwd(nx, os, cb) * 8 > 65536) continue;
    *threads = 256;  // the load, scatter and output phases take every thread (measured faster than items)
    return cb;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Launch dispatch over the instantiated FFT lengths.
// ---------------------------------------------------------------------------

bool fft_size_supported(int n) {
#define GPJC_CASE(N) \
  if (n == N) return true;
  GPJC_FFT_SIZES(GPJC_CASE)
#undef GPJC_CASE
  return false;
}

template <template <int> class F, class... Args>
static int dispatch_n(int n, Args&&... args) {
#define GPJC_CASE(N) \
  if (n == N) return F<N>::run(args...);
  GPJC_FFT_SIZES(GPJC_CASE)
#undef GPJC_CASE
  return fail(GPJC_E_UNSUPPORTED, "FFT length " + std::to_string(n) + " not built");
}

template <Store ST>
struct ReadoutFwd {
  template <int NX>
  struct L {
    static int run(const Plan& pl, const float2* img) {
      StageScope sc(pl, GPJC_STAGE_READOUT_FWD, true);
      if constexpr (Split<NX>::ok) {
        if (pl.f2_cb > 0) {
          const size_t lds = two_pass_lds_fwd(NX, pl.os, pl.f2_cb) * sizeof(float2);
          dim3 grid(pl.ny, (pl.nc + pl.f2_cb - 1) / pl.f2_cb, pl.B);
          sc.launch(k_readout_fwd2<NX, ST>, grid, dim3(pl.f2_threads), lds, pl.stream, img, pl.coils, pl.psfp,
                    pl.twin, pl.tw_x, (void*)pl.W, pl.ny, pl.nc, pl.os, pl.f2_cb);
          GPJC_HIP(hipGetLastError());
          return GPJC_OK;
        }
      }
      const int rows = pl.f1_rows;
      const size_t lds = (size_t)(NX + 2 * rows * pl.os * fline(NX)) * sizeof(float2);
      dim3 grid((pl.ny + rows - 1) / rows, pl.nc, pl.B);
      sc.launch(k_readout_fwd<NX, ST>, grid, dim3(256), lds, pl.stream, img, pl.coils, pl.psfp, pl.twin, pl.tw_x,
                (void*)pl.W, pl.ny, pl.nc, pl.os, 1.0f / pl.os, rows);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

template <Store ST>
struct ReadoutAdj {
  template <int NX>
  struct L {
    static int run(const Plan& pl) {
      StageScope sc(pl, GPJC_STAGE_READOUT_ADJ, true);
      if constexpr (Split<NX>::ok) {
        if (pl.f2_adj) {
          const size_t lds = two_pass_lds_adj(NX, pl.os, pl.f2_cb) * sizeof(float2);
          const dim3 grid(kAdjRowBlock * pl.f1h_nchunk, (pl.ny + kAdjRowBlock - 1) / kAdjRowBlock, pl.B);
          sc.launch(k_readout_adj2<NX, ST>, grid, dim3(pl.f2_threads), lds, pl.stream, (const void*)pl.W, pl.coils,
                    pl.psfp, pl.twin, pl.tw_x, pl.part, pl.ny, pl.nc, pl.os, pl.f2_cb, pl.B);
          GPJC_HIP(hipGetLastError());
          return GPJC_OK;
        }
      }
      const size_t lds = (size_t)(NX + 2 * pl.f1h_cb * pl.os * fline(NX)) * sizeof(float2);
      dim3 grid(pl.ny, pl.f1h_nchunk, pl.B);
      sc.launch(k_readout_adj<NX, ST>, grid, dim3(256), lds, pl.stream, (const void*)pl.W, pl.coils, pl.psfp,
                pl.twin, pl.tw_x, pl.part, pl.ny, pl.nc, pl.os, 1.0f / pl.os, pl.f1h_cb, pl.f1h_cpc, pl.B);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

template <int NY>
struct PeFwd {
  static int run(const Plan& pl, float2* out, int ksplit) {
    StageScope sc(pl, GPJC_STAGE_PE_FWD);
    const int nlines = pl.B * pl.np * pl.K;
    const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * fline(NY)) * sizeof(float2);
    const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
    hipLaunchKernelGGL(k_pe_fwd<NY>, dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream, pl.Zp,
                       ksplit, zs, out, pl.lines, pl.ms, nlines, pl.f3_lpb, pl.tw_y);
    GPJC_HIP(hipGetLastError());
    return GPJC_OK;
  }
};

// Z^T in the storage the expanding contraction reads for precision st.
static void* zt_for(const Plan& pl, Store st) {
  return st == Store::F32 ? static_cast<void*>(pl.Zt) : static_cast<void*>(pl.Zt16);
}

template <Store ST>
struct PeAdj {
  template <int NY>
  struct L {
    static int run(const Plan& pl, const float2* in) {
      StageScope sc(pl, GPJC_STAGE_PE_ADJ);
      const int nlines = pl.B * pl.np * pl.K;
      const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * fline(NY)) * sizeof(float2);
      hipLaunchKernelGGL((k_pe_adj<NY, ST>), dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream,
                         in, zt_for(pl, ST), pl.lines, pl.ms, nlines, pl.f3_lpb, pl.K, pl.Kp, pl.tw_y);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

template <Store ST>
struct PeNormal {
  template <int NY>
  struct L {
    static int run(const Plan& pl, int ksplit) {
      StageScope sc(pl, GPJC_STAGE_PE_NORMAL, true);
      const int nlines = pl.B * pl.np * pl.K;
      if constexpr (Split<NY>::ok) {
        constexpr int lines = PeNormal2Geo<NY>::L;
        const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
        sc.launch(k_pe_normal2<NY, ST>, dim3((nlines + lines - 1) / lines), dim3(256), 0, pl.stream,
                  (const float2*)pl.Zp, ksplit, zs, zt_for(pl, ST), (const float*)pl.maskf, nlines, pl.K,
                  pl.Kp, (const float2*)pl.tw_y);
        GPJC_HIP(hipGetLastError());
        return GPJC_OK;
      }
      const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * fline(NY)) * sizeof(float2);
      const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
      sc.launch(k_pe_normal<NY, ST>, dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream,
                (const float2*)pl.Zp, ksplit, zs, zt_for(pl, ST), (const float*)pl.maskf, nlines,
                pl.f3_lpb, pl.K, pl.Kp, (const float2*)pl.tw_y);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

template <Store ST>
struct PeCols {
  template <int NY>
  struct L {
    static int run(const Plan& pl, int mode, const float2* in_s, float2* out_s) {
      StageScope sc(pl, GPJC_STAGE_PE_COLS);
      if constexpr (ST == Store::F32 && Split<NY>::ok) {
        if (mode == 2) {
          constexpr int N1 = Split<NY>::N1, L = Cols2Geo<NY, N1>::L;
          hipLaunchKernelGGL((k_pe_cols_normal2<NY, N1>), dim3((pl.nt + L - 1) / L, pl.B * pl.nc), dim3(256), 0,
                             pl.stream, pl.W, (size_t)NY * pl.nt, (size_t)pl.nt, pl.nt, (const float*)pl.maskf, 1,
                             pl.nt, (const float2*)pl.tw_y);
          GPJC_HIP(hipGetLastError());
          return GPJC_OK;
        }
      }
      const int tb = pl.f3_tb;
      const size_t lds = (size_t)(NY + 2 * tb * fline(NY)) * sizeof(float2);
      dim3 grid((pl.nt + tb - 1) / tb, pl.B * pl.nc);
      hipLaunchKernelGGL((k_pe_cols<NY, ST>), grid, dim3(256), lds, pl.stream, (const void*)pl.W, (void*)pl.W, in_s,
                         out_s, pl.lines, pl.maskf, pl.ms, pl.nt, tb, mode, pl.tw_y);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

// The passes of a volume's uncompressed phase-encode stage over W, in place
// (pe3d.hip orders them): 0 y forward, 1 y inverse, over lines of Ny at
// stride Nt in every (b, n, z) row block; 2 z forward, 3 z inverse, 4 z
// forward, 2D mask, inverse, over the columns (y, t) of every (b, n) plane
// at stride Ny Nt.  N is Ny for the y passes, Nz for the z passes.
template <int N>
struct Cols3 {
  static int run(const Plan& pl, int pass) {
    constexpr int N1 = cols_n1(N), L = Cols2Geo<N, N1>::L;
    const bool ypass = pass < 2;
    const size_t ncols = ypass ? (size_t)pl.nt : (size_t)pl.ny2 * pl.nt;  // also the element stride
    const size_t pstride = ypass ? (size_t)pl.ny2 * pl.nt : (size_t)pl.ny * pl.nt;
    const int planes = ypass ? pl.B * pl.nc * pl.nz : pl.B * pl.nc;
    const float2* tw = ypass ? pl.tw_y3 : pl.tw_z3;
    const dim3 grid((unsigned)((ncols + L - 1) / L), planes);
    if (pass == 4)
      hipLaunchKernelGGL((k_pe_cols_normal2<N, N1>), grid, dim3(256), 0, pl.stream, pl.W, pstride, ncols, (int)ncols,
                         (const float*)pl.maskf3, pl.ny2, pl.nt, tw);
    else
      hipLaunchKernelGGL((k_cols2<N, N1>), grid, dim3(256), 0, pl.stream, pl.W, pstride, ncols, (int)ncols, pass & 1,
                         tw);
    GPJC_HIP(hipGetLastError());
    return GPJC_OK;
  }
};

int launch_pe3_cols_pass(const Plan& pl, int pass) { return dispatch_n<Cols3>(pass < 2 ? pl.ny2 : pl.nz, pl, pass); }

int launch_readout_fwd(const Plan& pl, const float2* img, Store st) {
  switch (storage_of(st)) {
    case Store::F32: return dispatch_n<ReadoutFwd<Store::F32>::L>(pl.nx, pl, img);
    case Store::BF16: return dispatch_n<ReadoutFwd<Store::BF16>::L>(pl.nx, pl, img);
    default: return dispatch_n<ReadoutFwd<Store::F16>::L>(pl.nx, pl, img);
  }
}

int launch_readout_adj(const Plan& pl, Store st) {
  switch (storage_of(st)) {
    case Store::F32: return dispatch_n<ReadoutAdj<Store::F32>::L>(pl.nx, pl);
    case Store::BF16: return dispatch_n<ReadoutAdj<Store::BF16>::L>(pl.nx, pl);
    default: return dispatch_n<ReadoutAdj<Store::F16>::L>(pl.nx, pl);
  }
}

int launch_combine(const Plan& pl, float2* out) {
  StageScope sc(pl, GPJC_STAGE_COMBINE);
  const size_t n = pl.img_elems();
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(k_combine, dim3(blocks), dim3(256), 0, pl.stream, pl.part, pl.f1h_nchunk, n, out);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// The split st's compressing contraction used is the number of partials of Z
// the phase-encode stage sums.
int launch_pe_fwd(const Plan& pl, float2* out, Store st) {
  if (pl.nz > 1) return launch_pe3_fwd(pl, out, st);
  return dispatch_n<PeFwd>(pl.ny, pl, out, pl.cfg(st).ksplit);
}
int launch_pe_adj(const Plan& pl, const float2* in, Store st) {
  if (pl.nz > 1) return launch_pe3_adj(pl, in, st);
  switch (storage_of(st)) {
    case Store::F32: return dispatch_n<PeAdj<Store::F32>::L>(pl.ny, pl, in);
    case Store::BF16: return dispatch_n<PeAdj<Store::BF16>::L>(pl.ny, pl, in);
    default: return dispatch_n<PeAdj<Store::F16>::L>(pl.ny, pl, in);
  }
}
int launch_pe_normal(const Plan& pl, Store st) {
  if (pl.nz > 1) return launch_pe3_normal(pl, st);
  const int ks = pl.cfg(st).ksplit;
  switch (storage_of(st)) {
    case Store::F32: return dispatch_n<PeNormal<Store::F32>::L>(pl.ny, pl, ks);
    case Store::BF16: return dispatch_n<PeNormal<Store::BF16>::L>(pl.ny, pl, ks);
    default: return dispatch_n<PeNormal<Store::F16>::L>(pl.ny, pl, ks);
  }
}

int launch_pe_cols_fwd(const Plan& pl, float2* out) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 0, (const float2*)nullptr, out);
}
int launch_pe_cols_adj(const Plan& pl, const float2* in) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 1, in, (float2*)nullptr);
}
int launch_pe_cols_normal(const Plan& pl) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 2, (const float2*)nullptr, (float2*)nullptr);
}

// ---------------------------------------------------------------------------
// Whole operators
// ---------------------------------------------------------------------------
int op_forward(const Plan& pl, Store st, const float2* img, float2* out) {
  if (pl.general) {
    GPJC_TRY(launch_explicit_fwd(pl, img));
    return launch_pe_fwd(pl, out, Store::F32);
  }
  if (!pl.compressed) {
    GPJC_TRY(launch_readout_fwd(pl, img, Store::F32));
    return pl.nz > 1 ? launch_pe3_cols_fwd(pl, out) : launch_pe_cols_fwd(pl, out);
  }
  GPJC_TRY(launch_readout_fwd(pl, img, st));
  GPJC_TRY(launch_group_compress(pl, st));
  return launch_pe_fwd(pl, out, st);
}

int op_adjoint_part(const Plan& pl, Store st, const float2* in) {
  if (pl.general) {
    GPJC_TRY(launch_pe_adj(pl, in, Store::F32));
    return launch_explicit_adj(pl);
  }
  if (!pl.compressed) {
    GPJC_TRY(pl.nz > 1 ? launch_pe3_cols_adj(pl, in) : launch_pe_cols_adj(pl, in));
    return launch_readout_adj(pl, Store::F32);
  }
  GPJC_TRY(launch_pe_adj(pl, in, st));
  GPJC_TRY(launch_group_expand(pl, st));
  return launch_readout_adj(pl, st);
}

int op_fwd_columns(const Plan& pl, Store st, const float2* img) {
  if (pl.general) return launch_explicit_fwd(pl, img);
  GPJC_TRY(launch_readout_fwd(pl, img, st));
  return launch_group_compress(pl, st);
}

int op_adj_columns(const Plan& pl, Store st) {
  if (pl.general) return launch_explicit_adj(pl);
  GPJC_TRY(launch_group_expand(pl, st));
  return launch_readout_adj(pl, st);
}

int op_normal_part(const Plan& pl, Store st, const float2* img) {
  if (pl.general) {
    GPJC_TRY(launch_explicit_fwd(pl, img));
    GPJC_TRY(launch_pe_normal(pl, Store::F32));
    return launch_explicit_adj(pl);
  }
  if (!pl.compressed) {
    GPJC_TRY(launch_readout_fwd(pl, img, Store::F32));
    GPJC_TRY(pl.nz > 1 ? launch_pe3_cols_normal(pl) : launch_pe_cols_normal(pl));
    return launch_readout_adj(pl, Store::F32);
  }
  GPJC_TRY(launch_readout_fwd(pl, img, st));
  GPJC_TRY(launch_group_compress(pl, st));
  GPJC_TRY(launch_pe_normal(pl, st));
  GPJC_TRY(launch_group_expand(pl, st));
  return launch_readout_adj(pl, st);
}

}  // namespace gpjc
