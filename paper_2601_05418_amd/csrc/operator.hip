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

#include "fft.h"
#include "plan.h"

namespace gpjc {

// ---------------------------------------------------------------------------
// Reduced-precision storage of complex values (round to nearest even).
// ---------------------------------------------------------------------------
__device__ inline uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline uint32_t f32_to_f16_bits(float f) {
  _Float16 h = (_Float16)f;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_bits_to_f32(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

template <Store ST>
__device__ inline void store_c(void* base, size_t i, float2 v) {
  if constexpr (ST == Store::F32) {
    reinterpret_cast<float2*>(base)[i] = v;
  } else if constexpr (ST == Store::BF16) {
    reinterpret_cast<uint32_t*>(base)[i] = f32_to_bf16_bits(v.x) | (f32_to_bf16_bits(v.y) << 16);
  } else {
    reinterpret_cast<uint32_t*>(base)[i] = f32_to_f16_bits(v.x) | (f32_to_f16_bits(v.y) << 16);
  }
}
template <Store ST>
__device__ inline float2 load_c(const void* base, size_t i) {
  if constexpr (ST == Store::F32) {
    return reinterpret_cast<const float2*>(base)[i];
  } else {
    const uint32_t w = reinterpret_cast<const uint32_t*>(base)[i];
    if constexpr (ST == Store::BF16) return make_float2(bf16_bits_to_f32(w & 0xffffu), bf16_bits_to_f32(w >> 16));
    else return make_float2(f16_bits_to_f32(w & 0xffffu), f16_bits_to_f32(w >> 16));
  }
}

__device__ inline void wg_sync() { __syncthreads(); }

// Work-group id remapped so that consecutive logical tiles share one XCD
// (work-groups are dealt round-robin over the 8 XCDs, each with its own L2).
__device__ inline int xcd_logical(int linear, int total) {
  const int per = total / 8, rem = total % 8;
  const int xcd = linear % 8, slot = linear / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

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

// ---------------------------------------------------------------------------
// F1: W[b][n][y][t] = psfp[y][t] * FFT_Nx(coil * img * twin[s])[q]
// grid (row blocks, nc, B); `rows` image rows per work-group.
// ---------------------------------------------------------------------------
template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_fwd(const float2* __restrict__ img, const float2* __restrict__ coils,
                                                     const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                     const float2* __restrict__ tw, void* __restrict__ W, int ny,
                                                     int nc, int os, int rows) {
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  const int nt = os * NX;
  const int n = blockIdx.y, b = blockIdx.z;
  const int y0 = blockIdx.x * rows;
  const int nr = min(rows, ny - y0);
  float2* twl = sm;
  float2* bufA = sm + NX;
  float2* bufB = bufA + rows * os * NX;
  for (int i = tid; i < NX; i += 256) twl[i] = tw[i];
  const float2* cp = coils + ((size_t)n * ny + y0) * NX;
  const float2* ip = img + ((size_t)b * ny + y0) * NX;
  for (int i = tid; i < nr * NX; i += 256) {
    const int r = i / NX, x = i - r * NX;
    const float2 u = cmul(cp[i], ip[i]);
    float2* dst = bufA + r * os * NX + x;
    for (int s = 0; s < os; ++s) dst[s * NX] = cmul(u, twin[s * NX + x]);
  }
  __syncthreads();
  const float2* res = fft_lines<NX>(bufA, bufB, twl, nr * os, NX, tid, 256, wg_sync);
  const size_t obase = (((size_t)b * nc + n) * ny + y0) * nt;
  const float2* ps = psfp + (size_t)y0 * nt;
  for (int i = tid; i < nr * nt; i += 256) {
    const int r = i / nt, t = i - r * nt;
    const int q = t / os, s = t - q * os;
    store_c<ST>(W, obase + i, cmul(ps[i], res[(r * os + s) * NX + q]));
  }
}

// F1^H for one image row and a chunk of coils: conj PSF, inverse readout DFT,
// crop, sum over the chunk of conj(coil) * line.  grid (ny, nchunk, B).
template <int NX, Store ST>
__global__ __launch_bounds__(256) void k_readout_adj(const void* __restrict__ W, const float2* __restrict__ coils,
                                                     const float2* __restrict__ psfp, const float2* __restrict__ twin,
                                                     const float2* __restrict__ tw, float2* __restrict__ part, int ny,
                                                     int nc, int os, int cb, int cpc, int B) {
  extern __shared__ float2 sm[];
  constexpr int PER = (NX + 255) / 256;
  const int tid = threadIdx.x;
  const int nt = os * NX;
  const int y = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z;
  float2* twl = sm;
  float2* bufA = sm + NX;
  float2* bufB = bufA + cb * os * NX;
  for (int i = tid; i < NX; i += 256) twl[i] = tw[i];
  float2 acc[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) acc[e] = make_float2(0.f, 0.f);
  const int nb = chunk * cpc, ne = min(nc, nb + cpc);
  const float2* ps = psfp + (size_t)y * nt;
  for (int n0 = nb; n0 < ne; n0 += cb) {
    const int ncb = min(cb, ne - n0);
    for (int i = tid; i < ncb * nt; i += 256) {
      const int c = i / nt, t = i - c * nt;
      const int q = t / os, s = t - q * os;
      const float2 w = load_c<ST>(W, (((size_t)b * nc + n0 + c) * ny + y) * nt + t);
      bufA[(c * os + s) * NX + q] = cmulc(ps[t], w);  // conj(conj(psf) * w)
    }
    __syncthreads();
    const float2* res = fft_lines<NX>(bufA, bufB, twl, ncb * os, NX, tid, 256, wg_sync);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int x = tid + e * 256;
      if (x < NX) {
        for (int c = 0; c < ncb; ++c) {
          float2 v = make_float2(0.f, 0.f);
          for (int s = 0; s < os; ++s) v = cadd(v, cmul(res[(c * os + s) * NX + x], twin[s * NX + x]));
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

__global__ void k_combine(const float2* __restrict__ part, int nchunk, size_t n, float2* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float2 v = part[i];
    for (int c = 1; c < nchunk; ++c) v = cadd(v, part[c * n + i]);
    out[i] = v;
  }
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

template <int NY>
__device__ inline void load_z_lines(float2* A, const float2* __restrict__ Zp, int ksplit, size_t zstride, int l0,
                                    int nl, int tid) {
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i % NY;
    const size_t g = (size_t)l0 * NY + i;
    float2 v = Zp[g];
    for (int ks = 1; ks < ksplit; ++ks) v = cadd(v, Zp[ks * zstride + g]);
    A[i] = (y & 1) ? make_float2(-v.x, -v.y) : v;
  }
}

template <int NY>
__global__ __launch_bounds__(256) void k_pe_fwd(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                float2* __restrict__ out, const int* __restrict__ lines, int ms,
                                                int nlines, int lpb, const float2* __restrict__ tw) {
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * NY;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  load_z_lines<NY>(A, Zp, ksplit, zstride, l0, nl, tid);
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, NY, tid, 256, wg_sync);
  for (int i = tid; i < nl * ms; i += 256) {
    const int li = i / ms, m = i - li * ms;
    const int ky = lines[m];
    out[(size_t)l0 * ms + i] = cscale(res[li * NY + ky], pe_post<NY>(ky));
  }
}

// Adjoint: zero-fill, inverse DFT; writes Zt[(b,p)][y][k] (k contiguous, stride kp).
template <int NY>
__global__ __launch_bounds__(256) void k_pe_adj(const float2* __restrict__ in, float2* __restrict__ Zt,
                                                const int* __restrict__ lines, int ms, int nlines, int lpb, int K,
                                                int kp, const float2* __restrict__ tw) {
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * NY;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  for (int i = tid; i < nl * NY; i += 256) A[i] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int i = tid; i < nl * ms; i += 256) {
    const int li = i / ms, m = i - li * ms;
    const int ky = lines[m];
    A[li * NY + ky] = cscale(cconj(in[(size_t)l0 * ms + i]), pe_post<NY>(ky));
  }
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, NY, tid, 256, wg_sync);
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, li = i - y * nl;
    const int l = l0 + li;
    const int bp = l / K, k = l - bp * K;
    float2 v = cconj(res[li * NY + y]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    Zt[((size_t)bp * NY + y) * kp + k] = v;
  }
}

// Normal y-stage: (-1)^y conj(FFT(conj(mask/Ny * FFT((-1)^y z)))) -> Zt.
template <int NY>
__global__ __launch_bounds__(256) void k_pe_normal(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                   float2* __restrict__ Zt, const float* __restrict__ maskf,
                                                   int nlines, int lpb, int K, int kp,
                                                   const float2* __restrict__ tw) {
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  float2* twl = sm;
  float2* A = sm + NY;
  float2* Bf = A + lpb * NY;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, nlines - l0);
  load_z_lines<NY>(A, Zp, ksplit, zstride, l0, nl, tid);
  __syncthreads();
  float2* res = fft_lines<NY>(A, Bf, twl, nl, NY, tid, 256, wg_sync);
  const float inv = 1.0f / (float)NY;
  for (int i = tid; i < nl * NY; i += 256) {
    const int ky = i % NY;
    res[i] = cconj(cscale(res[i], maskf[ky] * inv));
  }
  __syncthreads();
  float2* other = (res == A) ? Bf : A;
  const float2* res2 = fft_lines<NY>(res, other, twl, nl, NY, tid, 256, wg_sync);
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, li = i - y * nl;
    const int l = l0 + li;
    const int bp = l / K, k = l - bp * K;
    float2 v = cconj(res2[li * NY + y]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    Zt[((size_t)bp * NY + y) * kp + k] = v;
  }
}

// ---------------------------------------------------------------------------
// F3 on uncompressed columns W[(b,n)][y][t] (stride nt).  Work-group: one
// (b, n) and `tb` consecutive t.  LDS lines padded to NY + 1.
// ---------------------------------------------------------------------------
template <int NY, Store ST>
__global__ __launch_bounds__(256) void k_pe_cols(const void* __restrict__ Win, void* __restrict__ Wout,
                                                 const float2* __restrict__ in_s, float2* __restrict__ out_s,
                                                 const int* __restrict__ lines, const float* __restrict__ maskf,
                                                 int ms, int nt, int tb, int mode, const float2* __restrict__ tw) {
  // mode 0: forward W -> out_s [(b,n)][ms][nt]; 1: adjoint in_s -> Wout; 2: normal Win -> Wout
  extern __shared__ float2 sm[];
  constexpr int LS = NY + 1;
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
      A[c * LS + ky] = cscale(cconj(in_s[(bn * ms + m) * nt + t0 + c]), pe_post<NY>(ky));
    }
  } else {
    for (int i = tid; i < NY * ntb; i += 256) {
      const int y = i / ntb, c = i - y * ntb;
      float2 v = load_c<ST>(Win, (bn * NY + y) * nt + t0 + c);
      A[c * LS + y] = (y & 1) ? make_float2(-v.x, -v.y) : v;
    }
  }
  __syncthreads();
  float2* res = fft_lines<NY>(A, Bf, twl, ntb, LS, tid, 256, wg_sync);
  if (mode == 0) {
    for (int i = tid; i < ms * ntb; i += 256) {
      const int m = i / ntb, c = i - m * ntb;
      const int ky = lines[m];
      out_s[(bn * ms + m) * nt + t0 + c] = cscale(res[c * LS + ky], pe_post<NY>(ky));
    }
    return;
  }
  if (mode == 2) {
    const float inv = 1.0f / (float)NY;
    for (int i = tid; i < ntb * NY; i += 256) {
      const int c = i / NY, ky = i - c * NY;
      res[c * LS + ky] = cconj(cscale(res[c * LS + ky], maskf[ky] * inv));
    }
    __syncthreads();
    float2* other = (res == A) ? Bf : A;
    res = fft_lines<NY>(res, other, twl, ntb, LS, tid, 256, wg_sync);
  }
  for (int i = tid; i < NY * ntb; i += 256) {
    const int y = i / ntb, c = i - y * ntb;
    float2 v = cconj(res[c * LS + y]);
    if (y & 1) v = make_float2(-v.x, -v.y);
    store_c<ST>(Wout, (bn * NY + y) * nt + t0 + c, v);
  }
}

// ---------------------------------------------------------------------------
// Group contraction on FP32 MFMA (v_mfma_f32_16x16x4_f32).
//
// A complex product C = A B is carried as one real product of the expanded
// matrices [[Ar, -Ai], [Ai, Ar]] acting on interleaved (re, im) columns, so
// both operands are read straight from their natural interleaved layouts.
// Both operands are walked along the contraction index kk with one float4
// per lane: in a block of 16 kk, lane (i, q) (i = lane % 16, q = lane / 16)
// holds kk = kb + 4q .. kb + 4q + 3 of its row i and feeds element e to the
// e-th MFMA, so the four MFMAs together cover all 16 kk.
// Work-group 256 = 2 x 2 waves, wave tile 32 x 32, work-group tile 64 x 64.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct GemmCompressArgs {
  const float* A;   // [G][M][KD], M = 2K rows (k, re/im), KD = 2 ns
  const float* in;  // float view of [B][nc][N][nt] complex
  float2* out;      // [ksplit][B][np][K][N]
  const int* pgroup;
  int M, N, KD, nc, nt, P, np, K, B, ksplit, kchunk;
  size_t split_stride;
};

__global__ __launch_bounds__(256) void k_gemm_compress_f32(GemmCompressArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int tiles_n = (a.N + 63) / 64, tiles_m = (a.M + 63) / 64;
  const int total = tiles_n * tiles_m * a.B * a.np * a.ksplit;
  const int logical = xcd_logical(blockIdx.x, total);
  const int tn = logical % tiles_n;
  int rest = logical / tiles_n;
  const int tm = rest % tiles_m;
  const int z = rest / tiles_m;
  const int ks = z % a.ksplit, bp = z / a.ksplit;
  const int b = bp / a.np, p = bp - b * a.np;
  const int g = a.pgroup[p];
  const int row0 = tm * 64 + (wave >> 1) * 32;
  const int col0 = tn * 64 + (wave & 1) * 32;
  const int twoP = 2 * a.P;
  const size_t coil_stride = (size_t)a.N * a.nt * 2;

  const float* arow[2];
  bool va[2];
  const float* brow[2];
  bool vb[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int r = row0 + 16 * m + li;
    va[m] = r < a.M;
    arow[m] = a.A + ((size_t)g * a.M + (va[m] ? r : 0)) * a.KD;
    const int c = col0 + 16 * m + li;
    vb[m] = c < a.N;
    brow[m] = a.in + (((size_t)b * a.nc) * a.N + (vb[m] ? c : 0)) * a.nt * 2 + (size_t)p * twoP;
  }
  floatx4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[m][c] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int kbeg = ks * a.kchunk;
  const int kend = min(a.KD, kbeg + a.kchunk);
  for (int kb = kbeg; kb < kend; kb += 16) {
    const int kk = kb + 4 * lq;
    const bool vk = kk < kend;
    const int n = kk / twoP;
    const int jj = kk - n * twoP;
    floatx4 av[2], bv[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      av[m] = (va[m] && vk) ? *reinterpret_cast<const floatx4*>(arow[m] + kk) : floatx4{0.f, 0.f, 0.f, 0.f};
      bv[m] = (vb[m] && vk) ? *reinterpret_cast<const floatx4*>(brow[m] + n * coil_stride + jj)
                            : floatx4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m][e], bv[c][e], acc[m][c], 0, 0, 0);
  }
  // acc[m][c][r] = C[row0 + 16 m + 4 lq + r][col0 + 16 c + li]; rows pair up as (k, re), (k, im).
  float2* out = a.out + ks * a.split_stride + ((size_t)b * a.np + p) * a.K * a.N;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int row = row0 + 16 * m + 4 * lq;
      const int col = col0 + 16 * c + li;
      if (col < a.N) {
        if (row < a.M) out[(size_t)(row >> 1) * a.N + col] = make_float2(acc[m][c][0], acc[m][c][1]);
        if (row + 2 < a.M) out[(size_t)((row >> 1) + 1) * a.N + col] = make_float2(acc[m][c][2], acc[m][c][3]);
      }
    }
}

struct GemmExpandArgs {
  const float* Zt;  // [B][np][ny][KD] floats, KD = 2 kp
  const float* AH;  // [G][N][KD], N = 2 ns
  void* W;          // [B][nc][ny][nt] complex (storage per Store)
  const int* pgroup;
  int M, N, KD, nc, nt, P, np, B;
};

template <Store ST>
__global__ __launch_bounds__(256) void k_gemm_expand_f32(GemmExpandArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int tiles_n = (a.N + 63) / 64, tiles_m = (a.M + 63) / 64;
  const int total = tiles_n * tiles_m * a.B * a.np;
  const int logical = xcd_logical(blockIdx.x, total);
  const int tn = logical % tiles_n;
  int rest = logical / tiles_n;
  const int tm = rest % tiles_m;
  const int bp = rest / tiles_m;
  const int b = bp / a.np, p = bp - b * a.np;
  const int g = a.pgroup[p];
  const int row0 = tm * 64 + (wave >> 1) * 32;
  const int col0 = tn * 64 + (wave & 1) * 32;

  const float* arow[2];
  bool va[2];
  const float* brow[2];
  bool vb[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int r = row0 + 16 * m + li;
    va[m] = r < a.M;
    arow[m] = a.Zt + ((size_t)bp * a.M + (va[m] ? r : 0)) * a.KD;
    const int c = col0 + 16 * m + li;
    vb[m] = c < a.N;
    brow[m] = a.AH + ((size_t)g * a.N + (vb[m] ? c : 0)) * a.KD;
  }
  floatx4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[m][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int kb = 0; kb < a.KD; kb += 16) {
    const int kk = kb + 4 * lq;
    floatx4 av[2], bv[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      av[m] = va[m] ? *reinterpret_cast<const floatx4*>(arow[m] + kk) : floatx4{0.f, 0.f, 0.f, 0.f};
      bv[m] = vb[m] ? *reinterpret_cast<const floatx4*>(brow[m] + kk) : floatx4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m][e], bv[c][e], acc[m][c], 0, 0, 0);
  }
  // C[y][col], col = (n, j, re/im) -> W[b][n][y][p P + j]
  const int twoP = 2 * a.P;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = col0 + 16 * c + li;
    if (col >= a.N) continue;
    const int n = col / twoP, jj = col - n * twoP;
    const size_t cbase = ((size_t)b * a.nc + n) * a.M;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int y = row0 + 16 * m + 4 * lq + r;
        if (y < a.M) {
          const size_t fi = (cbase + y) * (size_t)a.nt * 2 + (size_t)p * twoP + jj;
          if constexpr (ST == Store::F32) {
            reinterpret_cast<float*>(a.W)[fi] = acc[m][c][r];
          } else if constexpr (ST == Store::BF16) {
            reinterpret_cast<uint16_t*>(a.W)[fi] = (uint16_t)f32_to_bf16_bits(acc[m][c][r]);
          } else {
            reinterpret_cast<uint16_t*>(a.W)[fi] = (uint16_t)f32_to_f16_bits(acc[m][c][r]);
          }
        }
      }
  }
}

// Real forms of the bank: Aexp [G][2K][2ns] (compressing), AH [G][2ns][2kp] (expanding).
__global__ void k_expand_bank(const double2* __restrict__ A, float* __restrict__ Aexp, float* __restrict__ AH, int G,
                              int K, int kp, int ns) {
  const size_t total = (size_t)G * K * ns;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % ns);
    const int k = (int)((idx / ns) % K);
    const int g = (int)(idx / ((size_t)ns * K));
    const double2 v = A[idx];
    const float ar = (float)v.x, ai = (float)v.y;
    float* e0 = Aexp + ((size_t)g * 2 * K + 2 * k) * 2 * ns;
    float* e1 = e0 + 2 * ns;
    e0[2 * i] = ar;
    e0[2 * i + 1] = -ai;
    e1[2 * i] = ai;
    e1[2 * i + 1] = ar;
    float* h0 = AH + ((size_t)g * 2 * ns + 2 * i) * 2 * kp;
    float* h1 = h0 + 2 * kp;
    h0[2 * k] = ar;
    h0[2 * k + 1] = ai;
    h1[2 * k] = -ai;
    h1[2 * k + 1] = ar;
  }
}

// ---------------------------------------------------------------------------
// Launch dispatch over the instantiated FFT lengths.
// ---------------------------------------------------------------------------
#define GPJC_FFT_SIZES(X) \
  X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(160) X(192) X(224) X(256) X(320) X(384) X(448) X(512)

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
      StageScope sc(pl, GPJC_STAGE_READOUT_FWD);
      const int rows = pl.f1_rows;
      const size_t lds = (size_t)(NX + 2 * rows * pl.os * NX) * sizeof(float2);
      dim3 grid((pl.ny + rows - 1) / rows, pl.nc, pl.B);
      hipLaunchKernelGGL((k_readout_fwd<NX, ST>), grid, dim3(256), lds, pl.stream, img, pl.coils, pl.psfp, pl.twin,
                         pl.tw_x, (void*)pl.W, pl.ny, pl.nc, pl.os, rows);
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
      StageScope sc(pl, GPJC_STAGE_READOUT_ADJ);
      const size_t lds = (size_t)(NX + 2 * pl.f1h_cb * pl.os * NX) * sizeof(float2);
      dim3 grid(pl.ny, pl.f1h_nchunk, pl.B);
      hipLaunchKernelGGL((k_readout_adj<NX, ST>), grid, dim3(256), lds, pl.stream, (const void*)pl.W, pl.coils,
                         pl.psfp, pl.twin, pl.tw_x, pl.part, pl.ny, pl.nc, pl.os, pl.f1h_cb, pl.f1h_cpc, pl.B);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

template <int NY>
struct PeFwd {
  static int run(const Plan& pl, float2* out) {
    StageScope sc(pl, GPJC_STAGE_PE_FWD);
    const int nlines = pl.B * pl.np * pl.K;
    const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * NY) * sizeof(float2);
    const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
    hipLaunchKernelGGL(k_pe_fwd<NY>, dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream, pl.Zp,
                       pl.gemm_ksplit, zs, out, pl.lines, pl.ms, nlines, pl.f3_lpb, pl.tw_y);
    GPJC_HIP(hipGetLastError());
    return GPJC_OK;
  }
};

template <int NY>
struct PeAdj {
  static int run(const Plan& pl, const float2* in) {
    StageScope sc(pl, GPJC_STAGE_PE_ADJ);
    const int nlines = pl.B * pl.np * pl.K;
    const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * NY) * sizeof(float2);
    hipLaunchKernelGGL(k_pe_adj<NY>, dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream, in,
                       pl.Zt, pl.lines, pl.ms, nlines, pl.f3_lpb, pl.K, pl.Kp, pl.tw_y);
    GPJC_HIP(hipGetLastError());
    return GPJC_OK;
  }
};

template <int NY>
struct PeNormal {
  static int run(const Plan& pl) {
    StageScope sc(pl, GPJC_STAGE_PE_NORMAL);
    const int nlines = pl.B * pl.np * pl.K;
    const size_t lds = (size_t)(NY + 2 * pl.f3_lpb * NY) * sizeof(float2);
    const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
    hipLaunchKernelGGL(k_pe_normal<NY>, dim3((nlines + pl.f3_lpb - 1) / pl.f3_lpb), dim3(256), lds, pl.stream,
                       pl.Zp, pl.gemm_ksplit, zs, pl.Zt, pl.maskf, nlines, pl.f3_lpb, pl.K, pl.Kp, pl.tw_y);
    GPJC_HIP(hipGetLastError());
    return GPJC_OK;
  }
};

template <Store ST>
struct PeCols {
  template <int NY>
  struct L {
    static int run(const Plan& pl, int mode, const float2* in_s, float2* out_s) {
      StageScope sc(pl, GPJC_STAGE_PE_COLS);
      const int tb = pl.f3_tb;
      const size_t lds = (size_t)(NY + 2 * tb * (NY + 1)) * sizeof(float2);
      dim3 grid((pl.nt + tb - 1) / tb, pl.B * pl.nc);
      hipLaunchKernelGGL((k_pe_cols<NY, ST>), grid, dim3(256), lds, pl.stream, (const void*)pl.W, (void*)pl.W, in_s,
                         out_s, pl.lines, pl.maskf, pl.ms, pl.nt, tb, mode, pl.tw_y);
      GPJC_HIP(hipGetLastError());
      return GPJC_OK;
    }
  };
};

int launch_readout_fwd(const Plan& pl, const float2* img, Store st) {
  switch (st) {
    case Store::F32: return dispatch_n<ReadoutFwd<Store::F32>::L>(pl.nx, pl, img);
    case Store::BF16: return dispatch_n<ReadoutFwd<Store::BF16>::L>(pl.nx, pl, img);
    default: return dispatch_n<ReadoutFwd<Store::F16>::L>(pl.nx, pl, img);
  }
}

int launch_readout_adj(const Plan& pl, Store st) {
  switch (st) {
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

int launch_pe_fwd(const Plan& pl, float2* out) { return dispatch_n<PeFwd>(pl.ny, pl, out); }
int launch_pe_adj(const Plan& pl, const float2* in) { return dispatch_n<PeAdj>(pl.ny, pl, in); }
int launch_pe_normal(const Plan& pl) { return dispatch_n<PeNormal>(pl.ny, pl); }

int launch_pe_cols_fwd(const Plan& pl, float2* out) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 0, (const float2*)nullptr, out);
}
int launch_pe_cols_adj(const Plan& pl, const float2* in) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 1, in, (float2*)nullptr);
}
int launch_pe_cols_normal(const Plan& pl) {
  return dispatch_n<PeCols<Store::F32>::L>(pl.ny, pl, 2, (const float2*)nullptr, (float2*)nullptr);
}

static int gemm_compress(const Plan& pl, const float* in, int ncol, float2* out, int ksplit) {
  StageScope sc(pl, GPJC_STAGE_GROUP_COMPRESS);
  GemmCompressArgs a;
  a.A = pl.Aexp;
  a.in = in;
  a.out = out;
  a.pgroup = pl.pgroup;
  a.M = 2 * pl.K;
  a.N = ncol;
  a.KD = 2 * pl.ns;
  a.nc = pl.nc;
  a.nt = pl.nt;
  a.P = pl.P;
  a.np = pl.np;
  a.K = pl.K;
  a.B = pl.B;
  a.ksplit = ksplit;
  a.kchunk = ((a.KD + ksplit - 1) / ksplit + 15) / 16 * 16;
  a.split_stride = (size_t)pl.B * pl.np * pl.K * ncol;
  const int total = ((ncol + 63) / 64) * ((a.M + 63) / 64) * pl.B * pl.np * ksplit;
  hipLaunchKernelGGL(k_gemm_compress_f32, dim3(total), dim3(256), 0, pl.stream, a);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_group_compress(const Plan& pl, Store st) {
  if (st != Store::F32) return fail(GPJC_E_UNSUPPORTED, "reduced-precision contraction not built");
  return gemm_compress(pl, reinterpret_cast<const float*>(pl.W), pl.ny, pl.Zp, pl.gemm_ksplit);
}

int launch_compress_data(const Plan& pl, const float2* ksp, float2* out) {
  return gemm_compress(pl, reinterpret_cast<const float*>(ksp), pl.ms, out, 1);
}

int launch_group_expand(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_GROUP_EXPAND);
  GemmExpandArgs a;
  a.Zt = reinterpret_cast<const float*>(pl.Zt);
  a.AH = pl.AH;
  a.W = pl.W;
  a.pgroup = pl.pgroup;
  a.M = pl.ny;
  a.N = 2 * pl.ns;
  a.KD = 2 * pl.Kp;
  a.nc = pl.nc;
  a.nt = pl.nt;
  a.P = pl.P;
  a.np = pl.np;
  a.B = pl.B;
  const int total = ((a.N + 63) / 64) * ((a.M + 63) / 64) * pl.B * pl.np;
  if (st != Store::F32) return fail(GPJC_E_UNSUPPORTED, "reduced-precision contraction not built");
  hipLaunchKernelGGL(k_gemm_expand_f32<Store::F32>, dim3(total), dim3(256), 0, pl.stream, a);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_expand_bank(Plan& pl) {
  GPJC_HIP(hipMemsetAsync(pl.AH, 0, (size_t)pl.G * 2 * pl.ns * 2 * pl.Kp * sizeof(float), pl.stream));
  const size_t total = (size_t)pl.G * pl.K * pl.ns;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_expand_bank, dim3(blocks), dim3(256), 0, pl.stream, pl.A128, pl.Aexp, pl.AH, pl.G, pl.K,
                     pl.Kp, pl.ns);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// ---------------------------------------------------------------------------
// Whole operators
// ---------------------------------------------------------------------------
int op_forward(const Plan& pl, Store st, const float2* img, float2* out) {
  if (!pl.compressed) {
    GPJC_TRY(launch_readout_fwd(pl, img, Store::F32));
    return launch_pe_cols_fwd(pl, out);
  }
  GPJC_TRY(launch_readout_fwd(pl, img, st));
  GPJC_TRY(launch_group_compress(pl, st));
  return launch_pe_fwd(pl, out);
}

int op_adjoint_part(const Plan& pl, Store st, const float2* in) {
  if (!pl.compressed) {
    GPJC_TRY(launch_pe_cols_adj(pl, in));
    return launch_readout_adj(pl, Store::F32);
  }
  GPJC_TRY(launch_pe_adj(pl, in));
  GPJC_TRY(launch_group_expand(pl, st));
  return launch_readout_adj(pl, st);
}

int op_normal_part(const Plan& pl, Store st, const float2* img) {
  if (!pl.compressed) {
    GPJC_TRY(launch_readout_fwd(pl, img, Store::F32));
    GPJC_TRY(launch_pe_cols_normal(pl));
    return launch_readout_adj(pl, Store::F32);
  }
  GPJC_TRY(launch_readout_fwd(pl, img, st));
  GPJC_TRY(launch_group_compress(pl, st));
  GPJC_TRY(launch_pe_normal(pl));
  GPJC_TRY(launch_group_expand(pl, st));
  return launch_readout_adj(pl, st);
}

}  // namespace gpjc
