// Explicit compressed readout model for a general modulation map
// exp(-i k_m(t, x, y)) (nonlinear B0 fields, e.g. a local B0 coil array,
// Section 3.1; Eqs. 1-3), where no readout point-spread function exists.
//
// The modulation repeats on every phase-encode step, so the phase-encode
// dimension stays Fourier (Section 2.3) and each image column y has a dense
// readout model E_y[(n, t)][x] = c_n(x, y) exp(-i k_m(t, x, y)) F[t][x].
// Compression stores, per column, E'_y = blockdiag_p(A_g(p)) E_y (Eq. 14),
// the compressed readout matrices of Section 5 / Table S2:
//
//   E'[y][p][k][x] = sum_{n,j} A_g(p)[k][n][j] c_n(x, y) b[pP + j][y][x] F[pP + j][x],
//   F[t][x] = exp(-2 pi i (t - Nt/2)(x - Nx/2) / Nt) / sqrt(Nt),
//
// built once per bank (FP64 accumulation, stored FP32) and applied as
//   forward  Z[b][p][k][y]  = sum_x E'[y][(p, k)][x] img[b][y][x]      (then the
//            phase-encode stage, shared with the Wave operator)
//   adjoint  img[b][y][x]   = sum_{(p,k)} conj(E'[y][(p, k)][x]) Z[b][p][k][y].
// Both applications stream E' (Ny Np K Nx complex values) once per image
// batch: HBM-bound, which is why compression pays here -- the stored model
// shrinks with K / (Nc P).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"
#include "fft.h"
#include "plan.h"
#include "zcomplex.h"

namespace gpjc {

namespace {

constexpr int kBuildRows = 16;  // rows k per work-group of the build

// Work-group: one column y, one patch p, kBuildRows rows k; threads stride over
// x.  The bank entries are the same for every thread (scalar loads).
__global__ __launch_bounds__(256) void k_build_explicit(const double2* __restrict__ A, const float2* __restrict__ coils,
                                                        const float2* __restrict__ bmod, const int* __restrict__ pgroup,
                                                        int nc, int nx, int ny, int nt, int P, int np, int K,
                                                        float2* __restrict__ Ec) {
  const int y = blockIdx.x, p = blockIdx.y, k0 = blockIdx.z * kBuildRows;
  const int g = pgroup[p];
  const int ns = nc * P;
  const double inv = 1.0 / sqrt((double)nt);
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    double2 acc[kBuildRows];
#pragma unroll
    for (int q = 0; q < kBuildRows; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int j = 0; j < P; ++j) {
      const int t = p * P + j;
      const double2 fb = zscale(zmul(zroot((long)(t - nt / 2) * (x - nx / 2), nt), z_of(bmod[((size_t)t * ny + y) * nx + x])),
                                inv);
      for (int n = 0; n < nc; ++n) {
        const double2 e = zmul(fb, z_of(coils[((size_t)n * ny + y) * nx + x]));
        const double2* Ar = A + ((size_t)g * K + k0) * ns + n * P + j;
#pragma unroll
        for (int q = 0; q < kBuildRows; ++q)
          if (k0 + q < K) acc[q] = zadd(acc[q], zmul(Ar[(size_t)q * ns], e));
      }
    }
#pragma unroll
    for (int q = 0; q < kBuildRows; ++q)
      if (k0 + q < K) Ec[(((size_t)y * np + p) * K + k0 + q) * nx + x] = make_float2((float)acc[q].x, (float)acc[q].y);
  }
}

// Forward: one wave per row (rows strided over the work-group's four waves),
// lanes along x in 16-byte pairs of complex values, XB pairs per lane; BC
// images (up to 8, one pass over E' per 8 images) from b0 on.  Each row's sums are reduced across the wave in a fixed
// butterfly order.
template <int BC, int XB>
__global__ __launch_bounds__(256) void k_explicit_fwd(const float2* __restrict__ Ec, const float2* __restrict__ img,
                                                      int b0, int B, int nx, int ny, int rows, int rpw,
                                                      float2* __restrict__ Z) {
  const int y = blockIdx.y, r_beg = blockIdx.x * rpw, r_end = min(rows, r_beg + rpw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int npair = nx / 2;
  floatx4 xv[BC][XB];
#pragma unroll
  for (int b = 0; b < BC; ++b)
#pragma unroll
    for (int i = 0; i < XB; ++i) {
      const int q = lane + 64 * i;
      xv[b][i] = (b0 + b < B && q < npair)
                     ? reinterpret_cast<const floatx4*>(img + ((size_t)(b0 + b) * ny + y) * nx)[q]
                     : floatx4{0.f, 0.f, 0.f, 0.f};
    }
  for (int r = r_beg + wave; r < r_end; r += 4) {
    const floatx4* er = reinterpret_cast<const floatx4*>(Ec + ((size_t)y * rows + r) * nx);
    floatx4 e[XB];
#pragma unroll
    for (int i = 0; i < XB; ++i) {
      const int q = lane + 64 * i;
      e[i] = q < npair ? er[q] : floatx4{0.f, 0.f, 0.f, 0.f};
    }
    float ar[BC], ai[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      ar[b] = 0.f;
      ai[b] = 0.f;
#pragma unroll
      for (int i = 0; i < XB; ++i) {
        const floatx4 v = xv[b][i], m = e[i];
        ar[b] += m[0] * v[0] - m[1] * v[1] + m[2] * v[2] - m[3] * v[3];
        ai[b] += m[0] * v[1] + m[1] * v[0] + m[2] * v[3] + m[3] * v[2];
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        ar[b] += __shfl_xor(ar[b], off, 64);
        ai[b] += __shfl_xor(ai[b], off, 64);
      }
    if (lane == 0)
#pragma unroll
      for (int b = 0; b < BC; ++b)
        if (b0 + b < B) Z[((size_t)(b0 + b) * rows + r) * ny + y] = make_float2(ar[b], ai[b]);
  }
}

// Forward for several images at once: G lanes per row, so a wave takes 64 / G
// rows per step; lane g reads the 16-byte pairs g, g + G, ... of its row (G
// consecutive pairs per load instruction and row), and the BC image rows of
// column y sit in LDS, where the row groups of a wave read the same pairs.
// Each row's sums are reduced over its G lanes in a fixed butterfly order: the
// cross-lane work per row is log2(G) steps instead of the six of a whole-wave
// reduction, for 2 BC values each.  A lane takes RPL rows RW apart at once, so
// each image value it reads from LDS serves RPL rows.
template <int BC, int G, int RPL>
__global__ __launch_bounds__(256) void k_explicit_fwd_g(const float2* __restrict__ Ec, const float2* __restrict__ img,
                                                        int b0, int B, int nx, int ny, int rows, int rpw,
                                                        float2* __restrict__ Z) {
  extern __shared__ floatx4 xs[];  // [BC][nx / 2] pairs of image values
  constexpr int RW = 64 / G;       // rows per wave and step for each of a lane's RPL rows
  const int y = blockIdx.y, r_beg = blockIdx.x * rpw, r_end = min(rows, r_beg + rpw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane % G, rl = lane / G;
  const int npair = nx / 2;
  for (int i = tid; i < BC * npair; i += 256) {
    const int b = i / npair, q = i - b * npair;
    xs[i] = b0 + b < B ? reinterpret_cast<const floatx4*>(img + ((size_t)(b0 + b) * ny + y) * nx)[q]
                       : floatx4{0.f, 0.f, 0.f, 0.f};
  }
  __syncthreads();
  for (int r0 = r_beg + wave * RW * RPL; r0 < r_end; r0 += 4 * RW * RPL) {
    // a lane's rows r0 + rl + j RW share every image value it reads from LDS
    const floatx4* er[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j)  // rows past the end read the last row and are not written
      er[j] = reinterpret_cast<const floatx4*>(Ec + ((size_t)y * rows + min(r0 + rl + j * RW, r_end - 1)) * nx);
    float ar[RPL][BC], ai[RPL][BC];
#pragma unroll
    for (int j = 0; j < RPL; ++j)
#pragma unroll
      for (int b = 0; b < BC; ++b) ar[j][b] = ai[j][b] = 0.f;
#pragma unroll 2
    for (int q = g; q < npair; q += G) {
      floatx4 m[RPL];
#pragma unroll
      for (int j = 0; j < RPL; ++j) m[j] = er[j][q];
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        const floatx4 v = xs[b * npair + q];
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          ar[j][b] += m[j][0] * v[0] - m[j][1] * v[1] + m[j][2] * v[2] - m[j][3] * v[3];
          ai[j][b] += m[j][0] * v[1] + m[j][1] * v[0] + m[j][2] * v[3] + m[j][3] * v[2];
        }
      }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
      for (int j = 0; j < RPL; ++j)
#pragma unroll
        for (int b = 0; b < BC; ++b) {
          ar[j][b] += __shfl_xor(ar[j][b], off, 64);
          ai[j][b] += __shfl_xor(ai[j][b], off, 64);
        }
    if (g == 0)
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int r = r0 + rl + j * RW;
        if (r < r_end)
#pragma unroll
          for (int b = 0; b < BC; ++b)
            if (b0 + b < B) Z[((size_t)(b0 + b) * rows + r) * ny + y] = make_float2(ar[j][b], ai[j][b]);
      }
  }
}

constexpr int kAdjRows = 512;  // rows per chunk of the adjoint (LDS staging of Z)

// Adjoint: work-group (chunk c of the rows, column y).  A thread owns one x
// (or, for nx < 256, one x of one of nsub row subsets); the chunk's Z values
// of BC images sit in LDS.  Subsets are summed in a fixed order at the end.
// Writes the chunk's partial image part[c][b][y][x].
template <int BC>
__global__ __launch_bounds__(256) void k_explicit_adj(const float2* __restrict__ Ec, const float2* __restrict__ Zt,
                                                      int b0, int B, int nx, int ny, int np, int K, int kp, int rc,
                                                      float2* __restrict__ part) {
  const int c = blockIdx.x, y = blockIdx.y;
  const int rows = np * K;
  const int r_beg = c * rc, nr = max(0, min(rows, r_beg + rc) - r_beg);
  __shared__ float2 zs[BC][kAdjRows];
  __shared__ float2 red[256 * BC];
  const int tid = threadIdx.x;
  for (int i = tid; i < BC * nr; i += 256) {
    const int b = i / nr, rr = i - b * nr;
    const int r = r_beg + rr, p = r / K, k = r - p * K;
    zs[b][rr] = b0 + b < B ? Zt[(((size_t)(b0 + b) * np + p) * ny + y) * kp + k] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int nsub = nx < 256 ? 256 / nx : 1;
  const int sub = tid / (nx < 256 ? nx : 256);
  const size_t nimg = (size_t)ny * nx;
  for (int x0 = 0; x0 < nx; x0 += 256) {
    const int x = x0 + (nx < 256 ? tid % nx : tid);
    const bool act = sub < nsub && x < nx;
    float2 acc[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) acc[b] = make_float2(0.f, 0.f);
    if (act) {
      // eight rows' loads in flight before their products (rows past the
      // chunk load row nr - 1 and are weighted by zero)
      const float2* col = Ec + ((size_t)y * rows + r_beg) * nx + x;
      for (int r0 = sub; r0 < nr; r0 += 8 * nsub) {
        float2 e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = col[(size_t)min(r0 + u * nsub, nr - 1) * nx];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = r0 + u * nsub;
          if (rr < nr) {
#pragma unroll
            for (int b = 0; b < BC; ++b) {
              const float2 z = zs[b][rr];
              acc[b].x += e[u].x * z.x + e[u].y * z.y;  // conj(e) z
              acc[b].y += e[u].x * z.y - e[u].y * z.x;
            }
          }
        }
      }
    }
    if (nsub > 1) {
#pragma unroll
      for (int b = 0; b < BC; ++b) red[b * 256 + tid] = acc[b];
      __syncthreads();
      if (sub == 0 && act) {
        for (int s = 1; s < nsub; ++s)
#pragma unroll
          for (int b = 0; b < BC; ++b) acc[b] = cadd(acc[b], red[b * 256 + s * nx + tid]);
      }
      __syncthreads();
    }
    if (sub == 0 && act)
#pragma unroll
      for (int b = 0; b < BC; ++b)
        if (b0 + b < B) part[((size_t)c * B + b0 + b) * nimg + (size_t)y * nx + x] = acc[b];
  }
}

// Adjoint for several images at once: as k_explicit_adj, but a thread owns a
// pair of neighbouring x (16-byte loads of E') and the chunk's Z values sit in
// LDS row-major, [row][image], so one 16-byte LDS read gives two images of a
// row: per row and thread, one load, BC / 2 LDS reads and 8 BC multiply-adds.
template <int BC>
__global__ __launch_bounds__(256) void k_explicit_adj_p(const float2* __restrict__ Ec, const float2* __restrict__ Zt,
                                                        int b0, int B, int nx, int ny, int np, int K, int kp, int rc,
                                                        float2* __restrict__ part) {
  static_assert(BC % 2 == 0, "images in pairs");
  const int c = blockIdx.x, y = blockIdx.y;
  const int rows = np * K;
  const int r_beg = c * rc, nr = max(0, min(rows, r_beg + rc) - r_beg);
  __shared__ floatx4 zs[kAdjRows * BC / 2];  // [row][image pair]
  __shared__ floatx4 red[256 * BC / 2];
  const int tid = threadIdx.x;
  for (int i = tid; i < BC * nr; i += 256) {
    const int rr = i / BC, b = i - rr * BC;
    const int r = r_beg + rr, p = r / K, k = r - p * K;
    const float2 z = b0 + b < B ? Zt[(((size_t)(b0 + b) * np + p) * ny + y) * kp + k] : make_float2(0.f, 0.f);
    reinterpret_cast<float2*>(zs)[rr * BC + b] = z;
  }
  __syncthreads();
  const int npair = nx / 2;
  const int nsub = npair < 256 ? 256 / npair : 1;
  const int sub = tid / (npair < 256 ? npair : 256);
  const size_t nimg = (size_t)ny * nx;
  for (int q0 = 0; q0 < npair; q0 += 256) {
    const int q = q0 + (npair < 256 ? tid % npair : tid);
    const bool act = sub < nsub && q < npair;
    floatx4 acc[BC];  // per image: (x0 re, x0 im, x1 re, x1 im)
#pragma unroll
    for (int b = 0; b < BC; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
    if (act) {
      const floatx4* col = reinterpret_cast<const floatx4*>(Ec + ((size_t)y * rows + r_beg) * nx) + q;
      for (int r0 = sub; r0 < nr; r0 += 8 * nsub) {
        floatx4 e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = col[(size_t)min(r0 + u * nsub, nr - 1) * npair];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = r0 + u * nsub;
          if (rr < nr) {
#pragma unroll
            for (int h = 0; h < BC / 2; ++h) {
              const floatx4 z = zs[rr * (BC / 2) + h];  // images 2h and 2h + 1
#pragma unroll
              for (int w = 0; w < 2; ++w) {
                const float zr = z[2 * w], zi = z[2 * w + 1];
                floatx4& a = acc[2 * h + w];
                a[0] += e[u][0] * zr + e[u][1] * zi;  // conj(e) z, first x
                a[1] += e[u][0] * zi - e[u][1] * zr;
                a[2] += e[u][2] * zr + e[u][3] * zi;  // second x
                a[3] += e[u][2] * zi - e[u][3] * zr;
              }
            }
          }
        }
      }
    }
    if (nsub > 1) {
      for (int h = 0; h < BC / 2; ++h) {
        __syncthreads();
        red[tid * 2] = acc[2 * h];
        red[tid * 2 + 1] = acc[2 * h + 1];
        __syncthreads();
        if (sub == 0 && act)
          for (int s2 = 1; s2 < nsub; ++s2) {
            const floatx4 u0 = red[(s2 * npair + tid) * 2], u1 = red[(s2 * npair + tid) * 2 + 1];
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
              acc[2 * h][e2] += u0[e2];
              acc[2 * h + 1][e2] += u1[e2];
            }
          }
      }
    }
    if (sub == 0 && act)
#pragma unroll
      for (int b = 0; b < BC; ++b)
        if (b0 + b < B)
          reinterpret_cast<floatx4*>(part + ((size_t)c * B + b0 + b) * nimg + (size_t)y * nx)[q] = acc[b];
  }
}

template <int BC>
void launch_fwd_bc(const Plan& pl, const float2* img, int b0, int xb, dim3 grid, int rpw) {
  const int rows = pl.np * pl.K;
  switch (xb) {
    case 1: hipLaunchKernelGGL((k_explicit_fwd<BC, 1>), grid, dim3(256), 0, pl.stream, pl.Ec, img, b0, pl.B, pl.nx, pl.ny, rows, rpw, pl.Zp); break;
    case 2: hipLaunchKernelGGL((k_explicit_fwd<BC, 2>), grid, dim3(256), 0, pl.stream, pl.Ec, img, b0, pl.B, pl.nx, pl.ny, rows, rpw, pl.Zp); break;
    default: hipLaunchKernelGGL((k_explicit_fwd<BC, 4>), grid, dim3(256), 0, pl.stream, pl.Ec, img, b0, pl.B, pl.nx, pl.ny, rows, rpw, pl.Zp); break;
  }
}

}  // namespace

// Rows of the forward per work-group: 16 per wave for one or two images; 64
// per wave for more (k_explicit_fwd_g, which stages the image rows once per
// work-group).
constexpr int kFwdRowsPerWg = 64;
constexpr int kFwdRowsPerWgMulti = 256;
constexpr int kFwdLanesPerRow = 8;
constexpr int kFwdRowsPerLane = 2;  // rows a lane of the grouped forward takes together

int explicit_chunks(int rows, int ny, int B) {
  const int bp = (B + 7) / 8;
  int c = (2048 + ny * bp - 1) / (ny * bp);
  c = std::max(c, (rows + kAdjRows - 1) / kAdjRows);
  return std::max(1, std::min(c, rows));
}

size_t explicit_bytes(int nx, int ny, int np, int K) { return (size_t)ny * np * K * nx * sizeof(float2); }

int launch_build_explicit(const Plan& pl) {
  const dim3 grid(pl.ny, pl.np, (pl.K + kBuildRows - 1) / kBuildRows);
  hipLaunchKernelGGL(k_build_explicit, grid, dim3(256), 0, pl.stream, pl.A128, pl.coils, pl.bmod, pl.pgroup, pl.nc,
                     pl.nx, pl.ny, pl.nt, pl.P, pl.np, pl.K, pl.Ec);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_explicit_fwd(const Plan& pl, const float2* img) {
  StageScope sc(pl, GPJC_STAGE_EXPLICIT_FWD);
  const int rows = pl.np * pl.K;
  const int xb = (pl.nx / 2 + 63) / 64;  // 16-byte pairs per lane
  if (xb > 4) return fail(GPJC_E_UNSUPPORTED, "explicit model: nx above 512");
  const dim3 grid((rows + kFwdRowsPerWg - 1) / kFwdRowsPerWg, pl.ny);
  const dim3 grid_m((rows + kFwdRowsPerWgMulti - 1) / kFwdRowsPerWgMulti, pl.ny);
  for (int b0 = 0; b0 < pl.B; b0 += 8) {
    const int left = pl.B - b0;
    if (left == 1) {
      launch_fwd_bc<1>(pl, img, b0, xb, grid, kFwdRowsPerWg);
    } else if (left == 2) {
      launch_fwd_bc<2>(pl, img, b0, xb, grid, kFwdRowsPerWg);
    } else if (left <= 4) {
      hipLaunchKernelGGL((k_explicit_fwd_g<4, kFwdLanesPerRow, kFwdRowsPerLane>), grid_m, dim3(256),
                         4 * (pl.nx / 2) * sizeof(floatx4), pl.stream, pl.Ec, img, b0, pl.B, pl.nx, pl.ny, rows,
                         kFwdRowsPerWgMulti, pl.Zp);
    } else {
      hipLaunchKernelGGL((k_explicit_fwd_g<8, kFwdLanesPerRow, kFwdRowsPerLane>), grid_m, dim3(256),
                         8 * (pl.nx / 2) * sizeof(floatx4), pl.stream, pl.Ec, img, b0, pl.B, pl.nx, pl.ny, rows,
                         kFwdRowsPerWgMulti, pl.Zp);
    }
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_explicit_adj(const Plan& pl) {
  StageScope sc(pl, GPJC_STAGE_EXPLICIT_ADJ);
  const int rows = pl.np * pl.K;
  const int nchunk = pl.f1h_nchunk;
  const int rc = (rows + nchunk - 1) / nchunk;
  if (rc > kAdjRows) return fail(GPJC_E_UNSUPPORTED, "explicit model: rows per chunk above the LDS stage");
  const dim3 grid(nchunk, pl.ny);
  for (int b0 = 0; b0 < pl.B; b0 += 8) {
    const int left = pl.B - b0;
    if (left == 1)
      hipLaunchKernelGGL((k_explicit_adj<1>), grid, dim3(256), 0, pl.stream, pl.Ec, pl.Zt, b0, pl.B, pl.nx, pl.ny, pl.np,
                         pl.K, pl.Kp, rc, pl.part);
    else if (left == 2)
      hipLaunchKernelGGL((k_explicit_adj<2>), grid, dim3(256), 0, pl.stream, pl.Ec, pl.Zt, b0, pl.B, pl.nx, pl.ny, pl.np,
                         pl.K, pl.Kp, rc, pl.part);
    else if (left <= 4)
      hipLaunchKernelGGL((k_explicit_adj_p<4>), grid, dim3(256), 0, pl.stream, pl.Ec, pl.Zt, b0, pl.B, pl.nx, pl.ny,
                         pl.np, pl.K, pl.Kp, rc, pl.part);
    else
      hipLaunchKernelGGL((k_explicit_adj_p<8>), grid, dim3(256), 0, pl.stream, pl.Ec, pl.Zt, b0, pl.B, pl.nx, pl.ny,
                         pl.np, pl.K, pl.Kp, rc, pl.part);
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

}  // namespace gpjc
