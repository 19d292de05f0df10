// Phase-encode stage of 3D volumes (Section 3.4: both phase-encoding
// dimensions are reconstructed by FFT).  Rows of the readout and contraction
// stages are (z, y) pairs, row = z * Ny + y, so the compressed hybrid data of
// patch p and rank k form an Nz x Ny plane Z[b][p][k][z][y].  The stage takes
// the centred unitary 2D DFT of every plane and keeps the acquired (kz, ky)
// points of the 2D mask (raster order, kz major): a y pass over lines of Ny
// contiguous values, then a z pass over columns of stride Ny, both in LDS
// with the mixed-radix Stockham passes; T holds the planes between passes.
//
//   forward  Zp -> y-DFT -> T -> z-DFT -> T -> gather -> S'
//   normal   Zp -> y-DFT -> T -> z-DFT, mask, inverse z-DFT -> T -> inverse y-DFT -> Z^T
//   adjoint  S' -> scatter (zero fill) -> T -> inverse z-DFT -> T -> inverse y-DFT -> Z^T
//
// The uncompressed operator takes the same 2D DFT of every (coil, sample)
// plane of the readout-stage output W [b][n][z Ny + y][t], in place, with
// the two-pass column kernels of operator.hip: a y pass over lines of Ny at
// stride Nt, a z pass over the (y, t) columns of each (b, n) plane at stride
// Ny Nt; whole rows of Nt samples are gathered to, or scattered from,
// S [b][n][Ms][Nt].
//
// Centred DFT of length N from an unnormalised FFT: x[i] (-1)^i in, then
// X[k] (-1)^(N/2 + k) / sqrt(N) out; the inverse is conj(F(conj(.))).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "devutil.h"
#include "fft.h"
#include "plan.h"

namespace gpjc {

namespace {

__device__ inline void sync3() { __syncthreads(); }

template <int N>
__device__ inline float post3(int k) {
  const float s = (((N / 2) + k) & 1) ? -1.f : 1.f;
  return s * (1.0f / sqrtf((float)N));
}

template <int N>
constexpr int lines3() {
  // lines per work-group: two padded LDS buffers of fline(N) per line plus the
  // twiddles within 64 KiB, at most 16
  constexpr int l = (8192 - N) / (2 * fline(N));
  return l > 16 ? 16 : (l < 1 ? 1 : l);
}

// y pass, forward, from the k-split partials of Zp: lines (b, p, k, z).
template <int NY>
__global__ __launch_bounds__(256) void k3_y_fwd(const float2* __restrict__ Zp, int ksplit, size_t zstride,
                                                float2* __restrict__ T, int nlines, const float2* __restrict__ tw) {
  constexpr int LS = fline(NY), L = lines3<NY>();
  __shared__ float2 twl[NY];
  __shared__ float2 A[L * LS], Bf[L * LS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int l0 = blockIdx.x * L, nl = min(L, nlines - l0);
  // The partials are summed in order, and the loads of kSum3 of them for
  // kIt3 elements are issued before any is added.
  constexpr int kIt3 = 4, kSum3 = 3;
  const int nel = nl * NY;
  for (int i0 = 0; i0 < nel; i0 += kIt3 * 256) {
    float2 a[kIt3];
#pragma unroll
    for (int it = 0; it < kIt3; ++it) a[it] = make_float2(0.f, 0.f);
    for (int s0 = 0; s0 < ksplit; s0 += kSum3) {
      float2 v[kSum3][kIt3];
#pragma unroll
      for (int h = 0; h < kSum3; ++h)
#pragma unroll
        for (int it = 0; it < kIt3; ++it) {
          const int i = min(i0 + tid + 256 * it, nel - 1);  // past the end: a valid element, not stored
          v[h][it] = s0 + h < ksplit ? Zp[(size_t)(s0 + h) * zstride + (size_t)l0 * NY + i] : make_float2(0.f, 0.f);
        }
#pragma unroll
      for (int h = 0; h < kSum3; ++h)
#pragma unroll
        for (int it = 0; it < kIt3; ++it) a[it] = cadd(a[it], v[h][it]);
    }
#pragma unroll
    for (int it = 0; it < kIt3; ++it) {
      const int i = i0 + tid + 256 * it;
      if (i < nel) {
        const int li = i / NY, y = i - li * NY;
        A[li * LS + fpad(y)] = (y & 1) ? make_float2(-a[it].x, -a[it].y) : a[it];
      }
    }
  }
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, LS, tid, 256, sync3);
  for (int i = tid; i < nl * NY; i += 256) {
    const int li = i / NY, k = i - li * NY;
    T[(size_t)l0 * NY + i] = cscale(res[li * LS + fpad(k)], post3<NY>(k));
  }
}

// z pass over columns (b, p, k, y) of T (stride ny between z), L consecutive
// y of one plane per work-group.  mode 0: forward; 1: forward, mask
// maskf[kz * ny + ky], inverse; 2: inverse.
template <int NZ>
__global__ __launch_bounds__(256) void k3_z(float2* __restrict__ T, int ny, int ncols, int mode,
                                            const float* __restrict__ maskf, const float2* __restrict__ tw) {
  constexpr int LS = fline(NZ), L = lines3<NZ>();
  __shared__ float2 twl[NZ];
  __shared__ float2 A[L * LS], Bf[L * LS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NZ; i += 256) twl[i] = tw[i];
  const int cpp = (ny + L - 1) / L;  // column groups per plane
  const int plane = blockIdx.x / cpp, y0 = (blockIdx.x - plane * cpp) * L;
  const int nl = min(L, ny - y0);
  float2* Tp = T + (size_t)plane * NZ * ny;
  const bool inv_in = mode == 2;
  for (int i = tid; i < nl * NZ; i += 256) {
    const int z = i / nl, c = i - z * nl;
    float2 v = Tp[(size_t)z * ny + y0 + c];
    if (inv_in) v = cconj(v);
    A[c * LS + fpad(z)] = (z & 1) ? make_float2(-v.x, -v.y) : v;
  }
  __syncthreads();
  float2* res = fft_lines<NZ>(A, Bf, twl, nl, LS, tid, 256, sync3);
  if (mode == 1) {
    // mask in k-space, then the inverse: conj, (-1)^kz, FFT
    float2* other = res == A ? Bf : A;
    for (int i = tid; i < nl * NZ; i += 256) {
      const int c = i / NZ, kz = i - c * NZ;
      const float m = maskf[(size_t)kz * ny + y0 + c];
      const float2 v = cscale(res[c * LS + fpad(kz)], post3<NZ>(kz) * m);
      other[c * LS + fpad(kz)] = (kz & 1) ? make_float2(-v.x, v.y) : make_float2(v.x, -v.y);  // conj, (-1)^kz
    }
    __syncthreads();
    float2* res2 = fft_lines<NZ>(other, res, twl, nl, LS, tid, 256, sync3);
    for (int i = tid; i < nl * NZ; i += 256) {
      const int z = i / nl, c = i - z * nl;
      Tp[(size_t)z * ny + y0 + c] = cconj(cscale(res2[c * LS + fpad(z)], post3<NZ>(z)));
    }
    return;
  }
  for (int i = tid; i < nl * NZ; i += 256) {
    const int z = i / nl, c = i - z * nl;
    float2 v = cscale(res[c * LS + fpad(z)], post3<NZ>(z));
    Tp[(size_t)z * ny + y0 + c] = inv_in ? cconj(v) : v;
  }
}

// y pass, inverse, lines (b, p, k, z) of T -> Z^T rows (z * ny + y), k
// fastest.  A work-group takes L consecutive k of one (b, p, z), so its
// stores for each y are L consecutive elements of a Z^T row.
template <int NY, Store ST>
__global__ __launch_bounds__(256) void k3_y_inv(const float2* __restrict__ T, void* __restrict__ Zt, int nz, int K,
                                                int kp, const float2* __restrict__ tw) {
  constexpr int LS = fline(NY), L = lines3<NY>();
  __shared__ float2 twl[NY];
  __shared__ float2 A[L * LS], Bf[L * LS];
  const int tid = threadIdx.x;
  for (int i = tid; i < NY; i += 256) twl[i] = tw[i];
  const int kblocks = (K + L - 1) / L;
  const int z = blockIdx.x % nz, rest = blockIdx.x / nz;  // consecutive groups read neighbouring lines of T
  const int kb = rest % kblocks, bp = rest / kblocks;
  const int k0 = kb * L, nl = min(L, K - k0);
  const float2* Tl = T + (((size_t)bp * K + k0) * nz + z) * NY;  // line li at Tl + li nz NY
  for (int i = tid; i < nl * NY; i += 256) {
    const int li = i / NY, y = i - li * NY;
    const float2 v = cconj(Tl[(size_t)li * nz * NY + y]);
    A[li * LS + fpad(y)] = (y & 1) ? make_float2(-v.x, -v.y) : v;
  }
  __syncthreads();
  const float2* res = fft_lines<NY>(A, Bf, twl, nl, LS, tid, 256, sync3);
  const size_t row0 = (size_t)bp * nz * NY + (size_t)z * NY;
  for (int i = tid; i < nl * NY; i += 256) {
    const int y = i / nl, li = i - y * nl;
    const float2 v = cconj(cscale(res[li * LS + fpad(y)], post3<NY>(y)));
    store_zt<ST>(Zt, row0 + y, kp, k0 + li, v);
  }
}

// out[bpk][m] = T[bpk][pts[m]]
__global__ __launch_bounds__(256) void k3_gather(const float2* __restrict__ T, const int* __restrict__ pts, int ms,
                                                 int rows, size_t nplanes, float2* __restrict__ out) {
  const size_t n = nplanes * ms;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t pl = i / ms;
    const int m = (int)(i - pl * ms);
    out[i] = T[pl * rows + pts[m]];
  }
}

// T[bpk][r] = S'[bpk][sel[r]] where the point is acquired, 0 elsewhere
__global__ __launch_bounds__(256) void k3_scatter(const float2* __restrict__ in, const int* __restrict__ sel, int ms,
                                                  int rows, size_t nplanes, float2* __restrict__ T) {
  const size_t n = nplanes * rows;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t pl = i / rows;
    const int r = (int)(i - pl * rows);
    const int m = sel[r];
    T[i] = m >= 0 ? in[pl * ms + m] : make_float2(0.f, 0.f);
  }
}

// out[q][m][t] = W[q][pts[m]][t] over the planes q = (b, n): the acquired rows
__global__ __launch_bounds__(256) void k3_gather_rows(const float2* __restrict__ W, const int* __restrict__ pts, int ms,
                                                      int rows, int nt, int nout, float2* __restrict__ out) {
  for (int o = blockIdx.x; o < nout; o += gridDim.x) {
    const int q = o / ms, m = o - q * ms;
    const float2* src = W + ((size_t)q * rows + pts[m]) * nt;
    float2* dst = out + (size_t)o * nt;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) dst[t] = src[t];
  }
}

// W[q][r][t] = S[q][sel[r]][t] where row r is acquired, 0 elsewhere
__global__ __launch_bounds__(256) void k3_scatter_rows(const float2* __restrict__ in, const int* __restrict__ sel,
                                                       int ms, int rows, int nt, int nw, float2* __restrict__ W) {
  for (int o = blockIdx.x; o < nw; o += gridDim.x) {
    const int q = o / rows, r = o - q * rows;
    const int m = sel[r];
    float2* dst = W + (size_t)o * nt;
    if (m >= 0) {
      const float2* src = in + ((size_t)q * ms + m) * nt;
      for (int t = threadIdx.x; t < nt; t += blockDim.x) dst[t] = src[t];
    } else {
      for (int t = threadIdx.x; t < nt; t += blockDim.x) dst[t] = make_float2(0.f, 0.f);
    }
  }
}

template <int N>
struct YFwd {
  static int run(const Plan& pl, int ksplit, size_t zstride) {
    constexpr int L = lines3<N>();
    const int nlines = pl.B * pl.np * pl.K * pl.nz;
    hipLaunchKernelGGL(k3_y_fwd<N>, dim3((nlines + L - 1) / L), dim3(256), 0, pl.stream, pl.Zp, ksplit, zstride,
                       pl.T3, nlines, pl.tw_y3);
    return GPJC_OK;
  }
};
template <int N>
struct ZPass {
  static int run(const Plan& pl, int mode) {
    constexpr int L = lines3<N>();
    const int nplanes = pl.B * pl.np * pl.K;
    const int cpp = (pl.ny2 + L - 1) / L;
    hipLaunchKernelGGL(k3_z<N>, dim3(nplanes * cpp), dim3(256), 0, pl.stream, pl.T3, pl.ny2, nplanes * pl.ny2, mode,
                       pl.maskf3, pl.tw_z3);
    return GPJC_OK;
  }
};
template <Store ST>
struct YInv {
  template <int N>
  struct L {
    static int run(const Plan& pl) {
      constexpr int LL = lines3<N>();
      const int groups = pl.B * pl.np * pl.nz * ((pl.K + LL - 1) / LL);  // (b, p, block of k, z)
      void* zt = ST == Store::F32 ? static_cast<void*>(pl.Zt) : static_cast<void*>(pl.Zt16);
      hipLaunchKernelGGL((k3_y_inv<N, ST>), dim3(groups), dim3(256), 0, pl.stream, pl.T3, zt, pl.nz, pl.K, pl.Kp,
                         pl.tw_y3);
      return GPJC_OK;
    }
  };
};

template <template <int> class F, class... Args>
int dispatch3(int n, Args&&... args) {
#define GPJC_CASE3(N) \
  if (n == N) return F<N>::run(args...);
  GPJC_FFT_SIZES(GPJC_CASE3)
#undef GPJC_CASE3
  return fail(GPJC_E_UNSUPPORTED, "3D phase-encode length " + std::to_string(n) + " not built");
}

int y_inv(const Plan& pl, Store st) {
  switch (storage_of(st)) {
    case Store::F32: return dispatch3<YInv<Store::F32>::L>(pl.ny2, pl);
    case Store::BF16: return dispatch3<YInv<Store::BF16>::L>(pl.ny2, pl);
    default: return dispatch3<YInv<Store::F16>::L>(pl.ny2, pl);
  }
}

}  // namespace

int launch_pe3_fwd(const Plan& pl, float2* out, Store st) {
  StageScope sc(pl, GPJC_STAGE_PE_FWD);
  const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
  GPJC_TRY(dispatch3<YFwd>(pl.ny2, pl, pl.cfg(st).ksplit, zs));
  GPJC_TRY(dispatch3<ZPass>(pl.nz, pl, 0));
  const size_t nplanes = (size_t)pl.B * pl.np * pl.K;
  hipLaunchKernelGGL(k3_gather, dim3(2048), dim3(256), 0, pl.stream, pl.T3, pl.pts3, pl.ms, pl.ny, nplanes, out);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_pe3_adj(const Plan& pl, const float2* in, Store st) {
  StageScope sc(pl, GPJC_STAGE_PE_ADJ);
  const size_t nplanes = (size_t)pl.B * pl.np * pl.K;
  hipLaunchKernelGGL(k3_scatter, dim3(2048), dim3(256), 0, pl.stream, in, pl.sel3, pl.ms, pl.ny, nplanes, pl.T3);
  GPJC_TRY(dispatch3<ZPass>(pl.nz, pl, 2));
  GPJC_TRY(y_inv(pl, st));
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_pe3_normal(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_PE_NORMAL);
  const size_t zs = (size_t)pl.B * pl.np * pl.K * pl.ny;
  GPJC_TRY(dispatch3<YFwd>(pl.ny2, pl, pl.cfg(st).ksplit, zs));
  GPJC_TRY(dispatch3<ZPass>(pl.nz, pl, 1));
  GPJC_TRY(y_inv(pl, st));
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_pe3_cols_fwd(const Plan& pl, float2* out) {
  StageScope sc(pl, GPJC_STAGE_PE_COLS);
  GPJC_TRY(launch_pe3_cols_pass(pl, 0));
  GPJC_TRY(launch_pe3_cols_pass(pl, 2));
  const int nout = pl.B * pl.nc * pl.ms;
  hipLaunchKernelGGL(k3_gather_rows, dim3(std::min(nout, 8192)), dim3(256), 0, pl.stream, pl.W, pl.pts3, pl.ms, pl.ny,
                     pl.nt, nout, out);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_pe3_cols_adj(const Plan& pl, const float2* in) {
  StageScope sc(pl, GPJC_STAGE_PE_COLS);
  const int nw = pl.B * pl.nc * pl.ny;
  hipLaunchKernelGGL(k3_scatter_rows, dim3(std::min(nw, 8192)), dim3(256), 0, pl.stream, in, pl.sel3, pl.ms, pl.ny,
                     pl.nt, nw, pl.W);
  GPJC_TRY(launch_pe3_cols_pass(pl, 3));
  GPJC_TRY(launch_pe3_cols_pass(pl, 1));
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_pe3_cols_normal(const Plan& pl) {
  StageScope sc(pl, GPJC_STAGE_PE_COLS);
  GPJC_TRY(launch_pe3_cols_pass(pl, 0));
  GPJC_TRY(launch_pe3_cols_pass(pl, 4));
  GPJC_TRY(launch_pe3_cols_pass(pl, 1));
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

// Host tables of a 3D plan: raster indices of the acquired points, the point
// index of every row (or -1), the mask as floats, twiddles of Ny and Nz.
int setup_pe3(Plan& pl, const uint8_t* mask2) {
  const int rows = pl.ny;
  std::vector<int> pts, sel(rows, -1);
  std::vector<float> mf(rows, 0.f);
  for (int r = 0; r < rows; ++r)
    if (mask2[r]) {
      sel[r] = (int)pts.size();
      pts.push_back(r);
      mf[r] = 1.f;
    }
  auto tw = [](int n) {
    std::vector<float2> t(n);
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)n;
      t[m] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    return t;
  };
  const std::vector<float2> ty = tw(pl.ny2), tz = tw(pl.nz);
  GPJC_HIP(hipMemcpyAsync(pl.pts3, pts.data(), sizeof(int) * pts.size(), hipMemcpyHostToDevice, pl.stream));
  GPJC_HIP(hipMemcpyAsync(pl.sel3, sel.data(), sizeof(int) * rows, hipMemcpyHostToDevice, pl.stream));
  GPJC_HIP(hipMemcpyAsync(pl.maskf3, mf.data(), sizeof(float) * rows, hipMemcpyHostToDevice, pl.stream));
  GPJC_HIP(hipMemcpyAsync(pl.tw_y3, ty.data(), sizeof(float2) * ty.size(), hipMemcpyHostToDevice, pl.stream));
  GPJC_HIP(hipMemcpyAsync(pl.tw_z3, tz.data(), sizeof(float2) * tz.size(), hipMemcpyHostToDevice, pl.stream));
  GPJC_HIP(hipStreamSynchronize(pl.stream));  // host vectors go out of scope
  return GPJC_OK;
}

}  // namespace gpjc
