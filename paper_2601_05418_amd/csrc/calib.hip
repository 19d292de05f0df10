// Calibration of the compression bank (Section 2.4, Eqs. 6-12), all FP64.
//
// 1. Whitening (Eq. 12's T): Psi = Q Q^H (Cholesky), T = Q^{-1}; the coil
//    maps are whitened, cw = T c.
// 2. Gram (Eqs. 9-11): for group g with first member patch at sample t0,
//      e_r[(n, j)] = cw_n(r) psf[iy][t0 + j] exp(-2 pi i j (ix - Nx/2) / Nt)
//    (the readout DFT row of Eq. 6 without its per-pixel factor
//    exp(-2 pi i (t0 - Nt/2)(ix - Nx/2) / Nt) and 1/sqrt(Nt): a unit-modulus
//    scalar per pixel and a constant, both cancelling in e e^H / ||e||^2), and
//      P_g = sum_{r in ROI} w_r e_r e_r^H,  w_r = 1 / ||e_r||^2
//          = 1 / (sum_n |cw_n(r)|^2 * sum_j |psf[iy][t0 + j]|^2).
//    The sum is evaluated in separated form.  With r = (iy, ix), the pixel's
//    weight, coil and phase factors depend on ix only through
//      Q_nm(iy, d) = sum_ix wc(r) cw_n(r) conj(cw_m(r)) exp(-2 pi i d (ix - Nx/2) / Nt),
//    wc(r) = 1 / sum_n |cw_n(r)|^2, d = j - k in (-P, P), which no group
//    depends on; then
//      P_g[(n, j), (m, k)] = sum_iy q_g(iy) psf[iy][t0 + j] conj(psf[iy][t0 + k]) Q_nm(iy, j - k),
//    q_g(iy) = 1 / sum_j |psf[iy][t0 + j]|^2.  Same matrix (FP64, summation
//    order aside) for about 1/90 of the direct sum's work on 224 x 224.
// 3. Eigen-decomposition (Eq. 8): every eigenvalue and the eigenvectors of
//    the K largest, by Householder reduction to tridiagonal form, bisection
//    and inverse iteration (eigen.hip).
// 4. Selection (Eq. 12): eigenvalues in decreasing order, each of the first K
//    eigenvectors scaled by a unit phase so that its
//    largest-magnitude entry (lowest index on ties) is real positive,
//    A_g = [u_1 ... u_K]^H (T (x) I_P).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "fft.h"
#include "plan.h"
#include "zcomplex.h"

namespace gpjc {

namespace {

constexpr int kPair = 32;  // Gram rows are padded to a multiple of this (row stride of H)

// ---------------------------------------------------------------------------
// Whitening factor: T = Q^{-1}, Psi = Q Q^H, one work-group, global scratch.
// ---------------------------------------------------------------------------
__global__ void k_whiten_factor(const float2* __restrict__ psi, double2* __restrict__ Lc, double2* __restrict__ T,
                                int nc, int* __restrict__ flag) {
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < nc * nc; i += nth) {
    const float2 v = psi[i];
    Lc[i] = make_double2(v.x, v.y);
  }
  __syncthreads();
  __shared__ double diag;
  for (int j = 0; j < nc; ++j) {
    if (tid == 0) {
      double d = Lc[j * nc + j].x;
      for (int k = 0; k < j; ++k) d -= zabs2(Lc[j * nc + k]);
      if (!(d > 0.0)) {
        *flag = 1;
        d = 1.0;
      }
      diag = sqrt(d);
      Lc[j * nc + j] = make_double2(diag, 0.0);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < nc; i += nth) {
      double2 s = Lc[i * nc + j];
      for (int k = 0; k < j; ++k) s = zsub(s, zmulc(Lc[i * nc + k], Lc[j * nc + k]));
      Lc[i * nc + j] = zscale(s, 1.0 / diag);
    }
    __syncthreads();
  }
  // T = L^{-1}: forward substitution, one column per thread.
  for (int c = tid; c < nc; c += nth) {
    for (int i = 0; i < nc; ++i) {
      double2 s = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int k = c; k < i; ++k) s = zsub(s, zmul(Lc[i * nc + k], T[k * nc + c]));
      T[i * nc + c] = i < c ? make_double2(0.0, 0.0) : zscale(s, 1.0 / Lc[i * nc + i].x);
    }
  }
}

// cw[n][r] = sum_m T[n][m] c[m][r] (T = I if null); wc[r] = 1 / sum_n |cw_n|^2
// inside the ROI, 0 elsewhere or for a zero vector.
__global__ void k_calib_maps(const float2* __restrict__ coils, const double2* __restrict__ T,
                             const uint8_t* __restrict__ roi, double2* __restrict__ cw, double* __restrict__ wc,
                             int nc, int npix) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < npix; r += gridDim.x * blockDim.x) {
    double en = 0.0;
    for (int n = 0; n < nc; ++n) {
      double2 v;
      if (T) {
        v = make_double2(0.0, 0.0);
        for (int m = 0; m < nc; ++m) {
          const float2 c = coils[(size_t)m * npix + r];
          v = zadd(v, zmul(T[n * nc + m], make_double2(c.x, c.y)));
        }
      } else {
        const float2 c = coils[(size_t)n * npix + r];
        v = make_double2(c.x, c.y);
      }
      cw[(size_t)n * npix + r] = v;
      en += zabs2(v);
    }
    const bool in = roi ? roi[r] != 0 : true;
    wc[r] = (in && en > 0.0) ? 1.0 / en : 0.0;
  }
}

// ph[dd][ix] = exp(-2 pi i (dd - P + 1)(ix - nx/2) / nt), dd < 2P - 1;
// qinv[g][iy] = 1 / sum_j |psf[iy][t0_g + j]|^2.
__global__ void k_calib_tables(const float2* __restrict__ psf, const int* __restrict__ t0s, double2* __restrict__ ph,
                               double* __restrict__ qinv, int P, int nx, int ny, int nt, int G) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  const int nd = 2 * P - 1;
  for (int i = gid; i < nd * nx; i += stride) {
    const int dd = i / nx, ix = i % nx;
    long m = ((long)(dd - P + 1) * (ix - nx / 2)) % nt;  // exact reduction of the angle
    if (m < 0) m += nt;
    double sn, cs;
    sincospi(-2.0 * (double)m / nt, &sn, &cs);
    ph[i] = make_double2(cs, sn);
  }
  for (int i = gid; i < G * ny; i += stride) {
    const int g = i / ny, iy = i % ny;
    double s = 0.0;
    for (int j = 0; j < P; ++j) {
      const float2 v = psf[(size_t)iy * nt + t0s[g] + j];
      s += (double)v.x * v.x + (double)v.y * v.y;
    }
    qinv[i] = s > 0.0 ? 1.0 / s : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Gram, separated form (see the header).
// k_gram_q: Q[(n nc + m)][iy][dd] = sum_ix wc cw_n conj(cw_m) ph[dd][ix].
// Work-group: one row iy, one coil n and a chunk of kQO * 256 outputs (m, dd);
// pixels are staged qx at a time in LDS (all coils' maps, the weighted map of
// coil n, the phase rows), qx chosen by the host to fit the LDS budget.
// ---------------------------------------------------------------------------
constexpr int kQO = 8;            // outputs per thread
constexpr size_t kGramLds = 65536;  // LDS budget of the two Gram kernels (bytes)

__global__ __launch_bounds__(256) void k_gram_q(const double2* __restrict__ cw, const double* __restrict__ wc,
                                                const double2* __restrict__ ph, double2* __restrict__ Q, int nc,
                                                int nx, int ny, int nd, int qx) {
  const int iy = blockIdx.x, n = blockIdx.y;
  const int npix = nx * ny;
  extern __shared__ double2 smq[];
  const int qs = qx + 1;           // LDS row stride: an odd number of 16-byte slots, so rows fall on distinct banks
  double2* cwm = smq;              // [nc][qs]
  double2* an = cwm + nc * qs;     // [qx]  wc * cw_n
  double2* phs = an + qx;          // [nd][qs]
  const int tid = threadIdx.x;
  const int nout = nc * nd;
  int om[kQO], od[kQO];
  bool ok[kQO];
  double2 acc[kQO];
#pragma unroll
  for (int q = 0; q < kQO; ++q) {
    const int o = blockIdx.z * (kQO * 256) + tid + 256 * q;
    ok[q] = o < nout;
    om[q] = ok[q] ? o / nd : 0;
    od[q] = ok[q] ? o - om[q] * nd : 0;
    acc[q] = make_double2(0.0, 0.0);
  }
  const size_t rowpix = (size_t)iy * nx;
  for (int x0 = 0; x0 < nx; x0 += qx) {
    const int nxc = min(qx, nx - x0);
    for (int i = tid; i < nc * qx; i += 256) {
      const int m = i / qx, x = i - m * qx;
      cwm[m * qs + x] = x < nxc ? cw[(size_t)m * npix + rowpix + x0 + x] : make_double2(0.0, 0.0);
    }
    for (int x = tid; x < qx; x += 256)
      an[x] = x < nxc ? zscale(cw[(size_t)n * npix + rowpix + x0 + x], wc[rowpix + x0 + x]) : make_double2(0.0, 0.0);
    for (int i = tid; i < nd * qx; i += 256) {
      const int dd = i / qx, x = i - dd * qx;
      phs[dd * qs + x] = x < nxc ? ph[(size_t)dd * nx + x0 + x] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int x = 0; x < nxc; ++x) {
      const double2 a = an[x];
#pragma unroll
      for (int q = 0; q < kQO; ++q)
        if (ok[q]) acc[q] = zadd(acc[q], zmul(zmulc(a, cwm[om[q] * qs + x]), phs[od[q] * qs + x]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kQO; ++q)
    if (ok[q]) Q[(((size_t)n * nc + om[q]) * ny + iy) * nd + od[q]] = acc[q];
}

// k_gram_assemble: the block (n, m), m >= n, of P_g; the block (m, n) is its
// conjugate transpose.  Work-group: one coil pair, one group and a tile of
// 4 * 256 outputs (j, k); rows iy are staged ay at a time in LDS (the
// q-weighted PSF samples of the patch, the plain ones, and Q_nm).
constexpr int kAO = 4;  // outputs per thread

__global__ __launch_bounds__(256) void k_gram_assemble(const double2* __restrict__ Q, const float2* __restrict__ psf,
                                                       const double* __restrict__ qinv, const int* __restrict__ t0s,
                                                       double2* __restrict__ H, int nc, int P, int ny, int nt, int nsp,
                                                       int ntile, int ay) {
  const int n = blockIdx.x, m = blockIdx.y;
  if (m < n) return;
  const int g = blockIdx.z / ntile, tile = blockIdx.z - g * ntile;
  const int nd = 2 * P - 1, t0 = t0s[g];
  extern __shared__ double2 sma[];
  double2* pj = sma;             // [ay][P]  q_g(iy) psf[iy][t0 + j]
  double2* pk = pj + ay * P;     // [ay][P]  psf[iy][t0 + k]
  double2* qs = pk + ay * P;     // [ay][nd] Q_nm(iy, .)
  const int tid = threadIdx.x;
  int oj[kAO], ok_[kAO];
  bool ok[kAO];
  double2 acc[kAO];
#pragma unroll
  for (int q = 0; q < kAO; ++q) {
    const int o = tile * (kAO * 256) + tid + 256 * q;
    ok[q] = o < P * P;
    oj[q] = ok[q] ? o / P : 0;
    ok_[q] = ok[q] ? o - oj[q] * P : 0;
    acc[q] = make_double2(0.0, 0.0);
  }
  const double2* Qnm = Q + ((size_t)n * nc + m) * ny * nd;
  const double* qg = qinv + (size_t)g * ny;
  for (int y0 = 0; y0 < ny; y0 += ay) {
    const int nyc = min(ay, ny - y0);
    for (int i = tid; i < ay * P; i += 256) {
      const int r = i / P, j = i - r * P;
      double2 a = make_double2(0.0, 0.0), b = a;
      if (r < nyc) {
        const float2 v = psf[(size_t)(y0 + r) * nt + t0 + j];
        b = make_double2(v.x, v.y);
        a = zscale(b, qg[y0 + r]);
      }
      pj[i] = a;
      pk[i] = b;
    }
    for (int i = tid; i < ay * nd; i += 256) {
      const int r = i / nd, dd = i - r * nd;
      qs[i] = r < nyc ? Qnm[(size_t)(y0 + r) * nd + dd] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int r = 0; r < nyc; ++r) {
#pragma unroll
      for (int q = 0; q < kAO; ++q)
        if (ok[q])
          acc[q] = zadd(acc[q], zmul(zmulc(pj[r * P + oj[q]], pk[r * P + ok_[q]]), qs[r * nd + oj[q] - ok_[q] + P - 1]));
    }
    __syncthreads();
  }
  double2* Hg = H + (size_t)g * nsp * nsp;
#pragma unroll
  for (int q = 0; q < kAO; ++q)
    if (ok[q]) {
      const int a = n * P + oj[q], b = m * P + ok_[q];
      Hg[(size_t)a * nsp + b] = acc[q];
      if (m != n) Hg[(size_t)b * nsp + a] = zconj(acc[q]);
    }
}

// ---------------------------------------------------------------------------
// Gram of a general modulation map exp(-i k_m(t, x, y)), which does not
// factor into a readout PSF (Section 3.1): the direct form of Eq. 10 over
// the pixels.  Per group, k_gen_channels writes the weighted composite
// vectors (patch-common phase dropped: it is one unit scalar per pixel and
// cancels in e e^H)
//   u[(n, j)][r] = sqrt(w_r) cw_n(r) b[t0 + j][r] exp(-2 pi i j (ix - nx/2) / nt),
//   w_r = wc(r) / sum_j |b[t0 + j][r]|^2  (= 1 / |e_r|^2 inside the ROI),
// and k_gram_direct forms H_g = sum_r u_r u_r^H.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gen_channels(const double2* __restrict__ cw, const double* __restrict__ wc,
                                                      const float2* __restrict__ bmod, int t0, int P, int nc, int nx,
                                                      int npix, int nt, double2* __restrict__ u) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < npix; r += gridDim.x * blockDim.x) {
    const int ix = r % nx;
    double eb = 0.0;
    for (int j = 0; j < P; ++j) eb += zabs2(z_of(bmod[(size_t)(t0 + j) * npix + r]));
    const double sw = (wc[r] > 0.0 && eb > 0.0) ? sqrt(wc[r] / eb) : 0.0;
    for (int j = 0; j < P; ++j) {
      const double2 f = zscale(zmul(z_of(bmod[(size_t)(t0 + j) * npix + r]), zroot((long)j * (ix - nx / 2), nt)), sw);
      for (int n = 0; n < nc; ++n) u[(size_t)(n * P + j) * npix + r] = zmul(cw[(size_t)n * npix + r], f);
    }
  }
}

// H[a][b] = sum_r u[a][r] conj(u[b][r]) for a 32 x 32 tile pair (ta <= tb;
// the mirrored tile is written as the conjugate transpose).  256 threads,
// 2 x 2 outputs each; pixels staged 32 at a time in LDS.
__global__ __launch_bounds__(256) void k_gram_direct(const double2* __restrict__ u, int ns, int npix,
                                                     double2* __restrict__ H, int nsp) {
  const int ta = blockIdx.x, tb = blockIdx.y;
  if (ta > tb) return;
  __shared__ double2 Ua[32][33], Ub[32][33];
  const int tid = threadIdx.x;
  const int i0 = (tid >> 4) * 2, j0 = (tid & 15) * 2;
  double2 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int r0 = 0; r0 < npix; r0 += 32) {
    for (int i = tid; i < 32 * 32; i += 256) {
      const int row = i >> 5, c = i & 31;
      const int ra = ta * 32 + row, rb = tb * 32 + row, px = r0 + c;
      Ua[row][c] = (ra < ns && px < npix) ? u[(size_t)ra * npix + px] : make_double2(0.0, 0.0);
      Ub[row][c] = (rb < ns && px < npix) ? u[(size_t)rb * npix + px] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 32; ++c) {
      const double2 a0 = Ua[i0][c], a1 = Ua[i0 + 1][c], b0 = Ub[j0][c], b1 = Ub[j0 + 1][c];
      acc[0][0] = zadd(acc[0][0], zmulc(a0, b0));
      acc[0][1] = zadd(acc[0][1], zmulc(a0, b1));
      acc[1][0] = zadd(acc[1][0], zmulc(a1, b0));
      acc[1][1] = zadd(acc[1][1], zmulc(a1, b1));
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int ra = ta * 32 + i0 + a, rb = tb * 32 + j0 + b;
      if (ra < ns && rb < ns) {
        H[(size_t)ra * nsp + rb] = acc[a][b];
        if (ta != tb) H[(size_t)rb * nsp + ra] = zconj(acc[a][b]);
      }
    }
}

// Phase-normalise the eigenvectors of the K largest eigenvalues (U rows, in
// decreasing eigenvalue order) and write A_g = [u_1 ... u_K]^H (T (x) I_P).
// One work-group per group.
__global__ __launch_bounds__(256) void k_select_rows(const double2* __restrict__ U, const double2* __restrict__ T,
                                                     double2* __restrict__ A, double2* __restrict__ rowbuf, int ns,
                                                     int K, int nc, int P) {
  const int g = blockIdx.x, tid = threadIdx.x;
  __shared__ double best_v[256];
  __shared__ int best_i[256];
  double2* row = rowbuf + (size_t)g * ns;
  for (int k = 0; k < K; ++k) {
    const double2* u = U + ((size_t)g * K + k) * ns;
    double bv = -1.0;
    int bi = 0;
    for (int a = tid; a < ns; a += 256) {
      const double m = zabs2(u[a]);
      if (m > bv) {
        bv = m;
        bi = a;
      }
    }
    best_v[tid] = bv;
    best_i[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const double v2 = best_v[tid + s];
        const int i2 = best_i[tid + s];
        if (v2 > best_v[tid] || (v2 == best_v[tid] && i2 < best_i[tid])) {
          best_v[tid] = v2;
          best_i[tid] = i2;
        }
      }
      __syncthreads();
    }
    const double2 um = u[best_i[0]];
    const double mu = sqrt(zabs2(um));
    const double2 ph = mu > 0.0 ? zscale(zconj(um), 1.0 / mu) : make_double2(1.0, 0.0);
    for (int a = tid; a < ns; a += 256) row[a] = zconj(zmul(u[a], ph));
    __syncthreads();
    double2* Ak = A + ((size_t)g * K + k) * ns;
    for (int a = tid; a < ns; a += 256) {
      if (T) {
        const int n = a / P, j = a - n * P;
        double2 s = make_double2(0.0, 0.0);
        for (int m = 0; m < nc; ++m) s = zadd(s, zmul(row[m * P + j], T[m * nc + n]));
        Ak[a] = s;
      } else {
        Ak[a] = row[a];
      }
    }
    __syncthreads();
  }
}

template <class T>
int dmalloc(T** p, size_t n) {
  GPJC_HIP(hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)));
  return GPJC_OK;
}

// Calibration workspaces.  Three modes: device allocations freed when the
// call returns (the default); carving from a caller-provided region (arena,
// 256-byte aligned pieces, nothing allocated); or measuring only (no arena,
// measure set: pointers stay null and `used` totals the bytes an arena needs).
struct Scratch {
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  bool measure = false;
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  int alloc(T** p, size_t n) {
    *p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (arena || measure) {
      const size_t off = (used + 255) / 256 * 256;
      used = off + bytes;
      if (measure) return GPJC_OK;
      if (used > cap) return fail(GPJC_E_UNSUPPORTED, "calibration workspace exceeds the static scratch");
      *p = reinterpret_cast<T*>(arena + off);
      return GPJC_OK;
    }
    GPJC_TRY(dmalloc(p, std::max<size_t>(n, 1)));
    ptrs.push_back(*p);
    return GPJC_OK;
  }
};

// Workspace pointers of one calibration.
struct CalibBufs {
  double2 *T = nullptr, *Lc = nullptr, *cw, *ph = nullptr, *Qg = nullptr, *u = nullptr, *H, *rowbuf;
  double *wc, *qinv;
  int *t0s, *flag;
  TriEigBufs te;
};

int alloc_calib(Scratch& s, const Plan& pl, bool whiten, CalibBufs& b) {
  const int G = pl.G, ns = pl.ns, P = pl.P;
  const int npix = pl.nx * pl.ny;
  const int nsp = (ns + kPair - 1) / kPair * kPair;
  const int nd = 2 * P - 1;
  GPJC_TRY(s.alloc(&b.cw, (size_t)pl.nc * npix));
  GPJC_TRY(s.alloc(&b.wc, (size_t)npix));
  if (pl.general) {  // the weighted composite vectors of one group at a time
    GPJC_TRY(s.alloc(&b.u, (size_t)ns * npix));
  } else {
    GPJC_TRY(s.alloc(&b.ph, (size_t)nd * pl.nx));
    GPJC_TRY(s.alloc(&b.Qg, (size_t)pl.nc * pl.nc * pl.ny * nd));
  }
  GPJC_TRY(s.alloc(&b.qinv, (size_t)G * pl.ny));
  GPJC_TRY(s.alloc(&b.t0s, (size_t)G));
  GPJC_TRY(s.alloc(&b.H, (size_t)G * nsp * nsp));
  GPJC_TRY(s.alloc(&b.flag, 2));
  GPJC_TRY(s.alloc(&b.rowbuf, (size_t)G * ns));
  const size_t gn = (size_t)G * ns, gk = gn * pl.K;
  TriEigBufs& t = b.te;
  GPJC_TRY(s.alloc(&t.d, gn));
  GPJC_TRY(s.alloc(&t.tau, gn));
  GPJC_TRY(s.alloc(&t.f, gn));
  GPJC_TRY(s.alloc(&t.f2, gn));
  GPJC_TRY(s.alloc(&t.eig, gn));
  GPJC_TRY(s.alloc(&t.bounds, (size_t)G * 3));
  GPJC_TRY(s.alloc(&t.e, gn));
  GPJC_TRY(s.alloc(&t.vb, 2 * gn));
  GPJC_TRY(s.alloc(&t.wb, gn));
  GPJC_TRY(s.alloc(&t.pb, gn));
  GPJC_TRY(s.alloc(&t.cb, gn));
  GPJC_TRY(s.alloc(&t.ph, gn));
  GPJC_TRY(s.alloc(&t.pd, gn));
  GPJC_TRY(s.alloc(&t.pt, gn * ((ns + 15) / 16)));
  GPJC_TRY(s.alloc(&t.lm, gk));
  GPJC_TRY(s.alloc(&t.u0, gk));
  GPJC_TRY(s.alloc(&t.u1, gk));
  GPJC_TRY(s.alloc(&t.u2, gk));
  GPJC_TRY(s.alloc(&t.x, gk));
  GPJC_TRY(s.alloc(&t.sw, gk));
  GPJC_TRY(s.alloc(&t.U, gk));
  if (whiten) {
    GPJC_TRY(s.alloc(&b.Lc, (size_t)pl.nc * pl.nc));
    GPJC_TRY(s.alloc(&b.T, (size_t)pl.nc * pl.nc));
  }
  return GPJC_OK;
}

}  // namespace

static int calibrate_in(Plan& pl, Scratch& s, const uint8_t* roi, const float2* noise_cov, double* h_eig,
                        double2* A_out) {
  const int G = pl.G, ns = pl.ns, P = pl.P;
  const int npix = pl.nx * pl.ny;
  const int nsp = (ns + kPair - 1) / kPair * kPair;
  CalibBufs bufs;
  GPJC_TRY(alloc_calib(s, pl, noise_cov != nullptr, bufs));
  double2 *T = bufs.T, *Lc = bufs.Lc, *cw = bufs.cw, *ph = bufs.ph, *Qg = bufs.Qg, *H = bufs.H, *rowbuf = bufs.rowbuf;
  double *wc = bufs.wc, *qinv = bufs.qinv;
  int *t0s = bufs.t0s, *flag = bufs.flag;  // flag[0]: whitening, flag[1]: eigensolver
  const int nd = 2 * P - 1;
  hipStream_t st = pl.stream;

  std::vector<int> t0h(G, -1);
  for (int p = 0; p < pl.np; ++p)
    if (t0h[pl.pgroup_h[p]] < 0) t0h[pl.pgroup_h[p]] = p * P;
  GPJC_HIP(hipMemcpyAsync(t0s, t0h.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  GPJC_HIP(hipMemsetAsync(flag, 0, 2 * sizeof(int), st));

  if (noise_cov) {
    hipLaunchKernelGGL(k_whiten_factor, dim3(1), dim3(256), 0, st, noise_cov, Lc, T, pl.nc, flag);
    GPJC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_calib_maps, dim3(std::min(1024, (npix + 255) / 256)), dim3(256), 0, st, pl.coils, T, roi, cw,
                     wc, pl.nc, npix);
  if (!pl.general)
    hipLaunchKernelGGL(k_calib_tables, dim3(64), dim3(256), 0, st, pl.psf, t0s, ph, qinv, P, pl.nx, pl.ny, pl.nt, G);
  if (pl.general) {
    const int nt32 = (ns + 31) / 32;
    for (int g = 0; g < G; ++g) {
      hipLaunchKernelGGL(k_gen_channels, dim3(std::min(1024, (npix + 255) / 256)), dim3(256), 0, st, cw, wc, pl.bmod,
                         t0h[g], P, pl.nc, pl.nx, npix, pl.nt, bufs.u);
      hipLaunchKernelGGL(k_gram_direct, dim3(nt32, nt32), dim3(256), 0, st, bufs.u, ns, npix,
                         H + (size_t)g * nsp * nsp, nsp);
    }
    GPJC_HIP(hipGetLastError());
  } else {
    const int nout = pl.nc * nd;
    const dim3 gq(pl.ny, pl.nc, (nout + kQO * 256 - 1) / (kQO * 256));
    // pixels / rows per LDS chunk: 16, fewer when the staged rows would not fit
    // LDS of k_gram_q: (nc + nd) rows of qx + 1 slots and one row of qx
    const size_t qrow = sizeof(double2) * (size_t)(pl.nc + 1 + nd), arow = sizeof(double2) * (size_t)(2 * P + nd);
    const int qx = (int)std::min<size_t>(16, kGramLds / qrow - 1), ay = (int)std::min<size_t>(16, kGramLds / arow);
    if (qx < 1 || ay < 1) return fail(GPJC_E_UNSUPPORTED, "calibration: coil count or patch length too large");
    const size_t lq = qrow * (qx + 1);
    hipLaunchKernelGGL(k_gram_q, gq, dim3(256), lq, st, cw, wc, ph, Qg, pl.nc, pl.nx, pl.ny, nd, qx);
    GPJC_HIP(hipGetLastError());
    const int ntile = (P * P + kAO * 256 - 1) / (kAO * 256);
    const dim3 ga(pl.nc, pl.nc, G * ntile);
    const size_t la = arow * ay;
    hipLaunchKernelGGL(k_gram_assemble, ga, dim3(256), la, st, Qg, pl.psf, qinv, t0s, H, pl.nc, P, pl.ny, pl.nt, nsp,
                       ntile, ay);
    GPJC_HIP(hipGetLastError());
  }

  // Eigenvalues and the K leading eigenvectors (Eq. 8), then A_g (Eq. 12).
  GPJC_TRY(tri_eigen(st, H, nsp, ns, G, pl.K, bufs.te, flag + 1));
  hipLaunchKernelGGL(k_select_rows, dim3(G), dim3(256), 0, st, bufs.te.U, T, pl.A128, rowbuf, ns, pl.K, pl.nc, P);
  GPJC_HIP(hipGetLastError());
  int hflag[2] = {0, 0};
  GPJC_HIP(hipMemcpyAsync(hflag, flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  GPJC_HIP(hipStreamSynchronize(st));
  if (hflag[0]) return fail(GPJC_E_NUMERIC, "calibration: noise covariance is not positive definite");
  if (hflag[1])
    return fail(GPJC_E_NUMERIC, "calibration: non-finite Gram, or an eigenvector failed its residual check");
  GPJC_TRY(launch_expand_bank(pl));
  if (pl.general) GPJC_TRY(launch_build_explicit(pl));
  pl.have_bank = true;
  if (A_out)
    GPJC_HIP(hipMemcpyAsync(A_out, pl.A128, sizeof(double2) * (size_t)G * pl.K * ns, hipMemcpyDeviceToDevice, st));
  if (h_eig)
    GPJC_HIP(hipMemcpyAsync(h_eig, bufs.te.eig, sizeof(double) * (size_t)G * ns, hipMemcpyDeviceToHost, st));
  GPJC_HIP(hipStreamSynchronize(st));
  return GPJC_OK;
}

int run_calibrate(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out) {
  Scratch s;  // device allocations, freed on return
  return calibrate_in(pl, s, roi, noise_cov, h_eig, A_out);
}

// ---------------------------------------------------------------------------
// Calibration without device allocation: the workspaces are carved from a
// file-scope device array of kStaticScratchBytes.  Each GPU holds its own copy
// until the process ends; its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current (in
// host code the array's name is not a device address).  Calls that overlap on
// one GPU share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static int static_scratch(int device, char** out) {
  if (device < 0 || device >= 64) return fail(GPJC_E_UNSUPPORTED, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    GPJC_HIP(hipGetDevice(&cur));
    if (cur != device) GPJC_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) GPJC_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !ptr)
      return fail(GPJC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[device]);
  return GPJC_OK;
}

int run_calibrate_static(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out) {
  Scratch need;
  need.measure = true;
  CalibBufs dummy;
  GPJC_TRY(alloc_calib(need, pl, noise_cov != nullptr, dummy));
  if (need.used > kStaticScratchBytes)
    return fail(GPJC_E_UNSUPPORTED, "calibration needs " + std::to_string(need.used) +
                                        " bytes of workspace; the static scratch holds " +
                                        std::to_string(kStaticScratchBytes));
  Scratch s;
  GPJC_TRY(static_scratch(pl.device, &s.arena));
  s.cap = kStaticScratchBytes;
  return calibrate_in(pl, s, roi, noise_cov, h_eig, A_out);
}

}  // namespace gpjc
