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
// 3. Eigen-decomposition (Eq. 8) by block-cyclic Jacobi: the matrix (padded
//    to a multiple of 32 with decoupled diagonal entries -1, below every
//    eigenvalue of the PSD P_g) is cut into blocks of 16; each round pairs
//    the blocks by a round-robin tournament, diagonalises every 32 x 32 pair
//    problem with complex Jacobi rotations in LDS, orders its eigenvalues
//    decreasingly (the larger ones to the lower-indexed block), and applies
//    the result to the whole matrix (H <- Q^H H Q) and to the eigenvector
//    accumulator (U <- U Q).  Couplings below a threshold derived from the
//    stopping tolerance are not rotated, and pair problems that need neither
//    a rotation nor a reordering are skipped by the update kernels.  Sweeps
//    repeat until the off-diagonal Frobenius norm is below 1e-13 of the
//    total.
// 4. Selection (Eq. 12): eigenvalues in decreasing order (ties by index),
//    each of the first K eigenvectors scaled by a unit phase so that its
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

// Round-robin tournament over n players (n even): step s in [0, n-1), pair i
// in [0, n/2); every pair of players meets exactly once in n-1 steps.
__host__ __device__ inline void rr_pair(int n, int s, int i, int* p, int* q) {
  if (i == 0) {
    *p = s;
    *q = n - 1;
  } else {
    const int m = n - 1;
    *p = (s + i) % m;
    *q = (s - i + m) % m;
  }
  if (*p > *q) {
    const int t = *p;
    *p = *q;
    *q = t;
  }
}

constexpr int kBlk = 16;     // Jacobi block
constexpr int kPair = 32;    // pair problem size
constexpr int kLd = 33;      // LDS row stride of 32 x 32 tiles
// Inner sweeps per pair problem and round.  The pair problem need not be
// diagonalised to rounding: the outer sweeps revisit every coupling, and two
// inner sweeps gave the fewest total operations on Ns = 1024 (the outer sweep
// count stays at 10-11 from 1 to 15 inner sweeps).
constexpr int kInnerSweeps = 2;

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

// Padded entries: zero coupling, diagonal -1; U = I.
__global__ void k_jac_init(double2* __restrict__ H, double2* __restrict__ U, int ns, int nsp, int G) {
  const size_t total = (size_t)G * nsp * nsp;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int b = (int)(i % nsp), a = (int)((i / nsp) % nsp);
    if (a >= ns || b >= ns) H[i] = make_double2(a == b ? -1.0 : 0.0, 0.0);
    U[i] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
}

__device__ inline int pair_index(int I, int J, int l) { return l < kBlk ? I * kBlk + l : J * kBlk + (l - kBlk); }

// Diagonalise the 32 x 32 problem of block pair `pr` in round `round`: complex
// Jacobi rotations in round-robin order, 16 disjoint rotations per step.  A
// step computes the 16 rotations, then every thread applies them to one 2 x 2
// block of M (M <- J^H M J, rows of pair t / 16, columns of pair t % 16) and to
// two row pairs of V (V <- V J).  Writes V with its columns ordered by
// decreasing eigenvalue and whether it differs from the identity.
__global__ __launch_bounds__(256) void k_jac_solve(const double2* __restrict__ H, double2* __restrict__ Vout,
                                                   int* __restrict__ rot, const int* __restrict__ active,
                                                   const double* __restrict__ thr2, int nsp, int nb, int round,
                                                   double tol) {
  const int g = blockIdx.y, pr = blockIdx.x;
  if (!active[g]) return;
  const double th2 = thr2[g];
  int I, J;
  rr_pair(nb, round, pr, &I, &J);
  __shared__ double2 M[kPair][kLd];
  __shared__ double2 V[kPair][kLd];
  __shared__ double prm_c[kPair / 2], prm_s[kPair / 2];
  __shared__ double2 prm_u[kPair / 2];
  __shared__ int prm_p[kPair / 2], prm_q[kPair / 2];
  __shared__ double red[8];
  __shared__ int done, rotated;
  __shared__ int rank[kPair];
  const int tid = threadIdx.x;
  if (tid == 0) rotated = 0;
  const double2* Hg = H + (size_t)g * nsp * nsp;
  for (int e = tid; e < kPair * kPair; e += 256) {
    const int a = e / kPair, b = e % kPair;
    M[a][b] = Hg[(size_t)pair_index(I, J, a) * nsp + pair_index(I, J, b)];
    V[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int bi = tid / (kPair / 2), bj = tid % (kPair / 2);  // 2 x 2 block of M owned in a step
  for (int sweep = 0; sweep < kInnerSweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < kPair * kPair; e += 256) {
      const int a = e / kPair, b = e % kPair;
      const double v = zabs2(M[a][b]);
      tot += v;
      if (a != b) off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      tot += __shfl_down(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = off;
      red[4 + (tid >> 6)] = tot;
    }
    __syncthreads();
    if (tid == 0) {
      const double o = red[0] + red[1] + red[2] + red[3], t = red[4] + red[5] + red[6] + red[7];
      done = (o <= tol * tol * t || o <= th2) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int s = 0; s < kPair - 1; ++s) {
      if (tid < kPair / 2) {
        int p, q;
        rr_pair(kPair, s, tid, &p, &q);
        const double a = M[p][p].x, b = M[q][q].x;
        const double2 c = M[p][q];
        // |c| by a scaled hypot: re^2 + im^2 of a decayed coupling can fall
        // into the subnormal range, and the phase c / |c| would then no
        // longer have unit modulus (the rotation would not be unitary).
        const double mc = hypot(c.x, c.y);
        double cs = 1.0, sn = 0.0;
        double2 u = make_double2(1.0, 0.0);
        if (mc > 1e-300 && mc * mc > th2) {
          rotated = 1;
          const double zeta = (b - a) / (2.0 * mc);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = t * cs;
          u = make_double2(c.x / mc, c.y / mc);
        }
        prm_c[tid] = cs;
        prm_s[tid] = sn;
        prm_u[tid] = u;
        prm_p[tid] = p;
        prm_q[tid] = q;
      }
      __syncthreads();
      // The rotation of pair i mixes columns p, q as
      //   X[:, p] <- cs X[:, p] - sn conj(u) X[:, q],  X[:, q] <- sn X[:, p] + cs conj(u) X[:, q]
      // and, from the left (J^H), rows p, q as
      //   M[p, :] <- cs M[p, :] - sn u M[q, :],        M[q, :] <- sn M[p, :] + cs u M[q, :].
      {
        const int pa = prm_p[bi], qa = prm_q[bi], pb = prm_p[bj], qb = prm_q[bj];
        const double ca = prm_c[bi], sa = prm_s[bi], cb = prm_c[bj], sb = prm_s[bj];
        const double2 ua = prm_u[bi], ubc = zconj(prm_u[bj]);
        const double2 m00 = M[pa][pb], m01 = M[pa][qb], m10 = M[qa][pb], m11 = M[qa][qb];
        // columns
        const double2 n00 = zsub(zscale(m00, cb), zscale(zmul(m01, ubc), sb));
        const double2 n01 = zadd(zscale(m00, sb), zscale(zmul(m01, ubc), cb));
        const double2 n10 = zsub(zscale(m10, cb), zscale(zmul(m11, ubc), sb));
        const double2 n11 = zadd(zscale(m10, sb), zscale(zmul(m11, ubc), cb));
        // rows
        M[pa][pb] = zsub(zscale(n00, ca), zscale(zmul(n10, ua), sa));
        M[qa][pb] = zadd(zscale(n00, sa), zscale(zmul(n10, ua), ca));
        M[pa][qb] = zsub(zscale(n01, ca), zscale(zmul(n11, ua), sa));
        M[qa][qb] = zadd(zscale(n01, sa), zscale(zmul(n11, ua), ca));
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = bi + (kPair / 2) * h;  // row of V
        const int pb = prm_p[bj], qb = prm_q[bj];
        const double cb = prm_c[bj], sb = prm_s[bj];
        const double2 ubc = zconj(prm_u[bj]);
        const double2 vp = V[k][pb], vq = V[k][qb];
        V[k][pb] = zsub(zscale(vp, cb), zscale(zmul(vq, ubc), sb));
        V[k][qb] = zadd(zscale(vp, sb), zscale(zmul(vq, ubc), cb));
      }
      __syncthreads();
    }
  }
  // Eigenvalues of the pair problem in decreasing order (ties by position):
  // column a of V moves to column rank[a], so the larger eigenvalues settle
  // in the lower-indexed block.  Without this ordering the graded spectrum
  // of P_g converges only linearly over the sweeps.
  if (tid < kPair) {
    const double la = M[tid][tid].x;
    int r = 0;
    for (int b = 0; b < kPair; ++b) {
      const double lb = M[b][b].x;
      r += (lb > la) || (lb == la && b < tid);
    }
    rank[tid] = r;
  }
  __syncthreads();
  if (tid < kPair && rank[tid] != tid) rotated = 1;
  __syncthreads();
  double2* Vg = Vout + ((size_t)g * (nb / 2) + pr) * kPair * kPair;
  for (int e = tid; e < kPair * kPair; e += 256) {
    const int a = e / kPair, b = e % kPair;
    Vg[a * kPair + rank[b]] = V[a][b];
  }
  if (tid == 0) rot[g * (nb / 2) + pr] = rotated;
}

// One 16 x 16 block of a complex 32 x 32 x 32 product on the FP64 16x16x4
// MFMA.  The complex product takes four real products (re = ar br - ai bi,
// im = ar bi + ai br).  Operand lanes: A[l % 16][l / 16], B[l / 16][l % 16];
// result lane l, register r: C[4 r + l / 16][l % 16].
//
// Register fragments of a 32 x 32 row-major tile T for k-steps k0 = 0, 4, ..:
//   as B operand of column block bj:        frag[s] = T[4 s + l / 16][16 bj + l % 16]
//   as A operand of (T^H), row block bi:    frag[s] = conj(T[4 s + l / 16][16 bi + l % 16])
// Both read the same elements; the conjugation is applied at use.
typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ inline void zfrag_load(const double2* __restrict__ T, int blk, double2 (&f)[kPair / 4]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < kPair / 4; ++s) f[s] = T[(4 * s + (l >> 4)) * kPair + 16 * blk + (l & 15)];
}

// C = X[16 bi + ., :] * B, B given as fragments of column block bj; X in LDS.
__device__ inline void zmma_lds_frag(const double2 (*X)[kLd], const double2 (&fb)[kPair / 4], int bi, dx4& cr,
                                     dx4& ci) {
  const int l = threadIdx.x & 63;
  const int li = l & 15, lk = l >> 4;
  cr = dx4{0.0, 0.0, 0.0, 0.0};
  ci = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < kPair / 4; ++s) {
    const double2 a = X[16 * bi + li][4 * s + lk];
    const double2 b = fb[s];
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
  }
}

// H <- V_a^H H V_b on the tile of pair a (rows) x pair b (cols), a <= b, one
// wave per tile with neither LDS nor barriers; the mirrored tile (b, a) is
// written as the conjugate transpose.
// - Y = X V_b, X the tile: per 16 x 16 block (q, bj), operand fragments of X
//   are read from H directly, those of V_b from the rotation blocks.
// - Z = V_a^H Y: the result registers of Y's blocks are already the B
//   operand fragments of this product (register r of block q holds rows
//   4 (4 q + r) + l / 16, i.e. k-step 4 q + r).
// The wave reads the whole tile before it writes any of it, so the update
// in place needs no synchronisation.  A side whose rotation is the identity
// is skipped.
__global__ __launch_bounds__(64) void k_jac_apply_h(double2* __restrict__ H, const double2* __restrict__ Vall,
                                                    const int* __restrict__ rot, const int* __restrict__ active,
                                                    int nsp, int nb, int round) {
  const int g = blockIdx.y;
  if (!active[g]) return;
  const int npair = nb / 2;
  const int a = blockIdx.x / npair, b = blockIdx.x % npair;
  if (b < a) return;
  const bool ra = rot[g * npair + a] != 0, rb = rot[g * npair + b] != 0;
  if (!ra && !rb) return;  // both sides identity
  int Ia, Ja, Ib, Jb;
  rr_pair(nb, round, a, &Ia, &Ja);
  rr_pair(nb, round, b, &Ib, &Jb);
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  double2* Hg = H + (size_t)g * nsp * nsp;
  const double2* Va = Vall + ((size_t)g * npair + a) * kPair * kPair;
  const double2* Vb = Vall + ((size_t)g * npair + b) * kPair * kPair;
  dx4 yr[2][2], yi[2][2];  // Y block (q, bj): register r holds Y[16 q + 4 r + l / 16][16 bj + l % 16]
  if (rb) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      double2 fb[kPair / 4];
      zfrag_load(Vb, bj, fb);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const size_t row = (size_t)pair_index(Ia, Ja, 16 * q + li) * nsp;
        dx4 cr = dx4{0.0, 0.0, 0.0, 0.0}, ci = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < kPair / 4; ++s) {
          const double2 x = Hg[row + pair_index(Ib, Jb, 4 * s + lk)];
          const double2 v = fb[s];
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, v.x, cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.y, v.y, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, v.y, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, v.x, ci, 0, 0, 0);
        }
        yr[q][bj] = cr;
        yi[q][bj] = ci;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double2 x = Hg[(size_t)pair_index(Ia, Ja, 16 * q + 4 * r + lk) * nsp + pair_index(Ib, Jb, 16 * bj + li)];
          yr[q][bj][r] = x.x;
          yi[q][bj][r] = x.y;
        }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {  // row block of Z
    double2 fa[kPair / 4];
    if (ra) zfrag_load(Va, q, fa);
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      dx4 cr = yr[q][bj], ci = yi[q][bj];
      if (ra) {
        cr = dx4{0.0, 0.0, 0.0, 0.0};
        ci = dx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < kPair / 4; ++s) {
          const double2 u = make_double2(fa[s].x, -fa[s].y);  // (V_a^H)[16 q + l % 16][4 s + l / 16]
          const double yre = yr[s / 4][bj][s % 4], yim = yi[s / 4][bj][s % 4];
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(u.x, yre, cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-u.y, yim, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(u.x, yim, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(u.y, yre, ci, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ra_i = pair_index(Ia, Ja, 16 * q + 4 * r + lk), cb_i = pair_index(Ib, Jb, 16 * bj + li);
        Hg[(size_t)ra_i * nsp + cb_i] = make_double2(cr[r], ci[r]);
        if (a != b) Hg[(size_t)cb_i * nsp + ra_i] = make_double2(cr[r], -ci[r]);
      }
    }
  }
}

// U[:, pair b] <- U[:, pair b] V_b, kURows rows per work-group in tiles of 32.
constexpr int kURows = 128;
__global__ __launch_bounds__(256) void k_jac_apply_u(double2* __restrict__ U, const double2* __restrict__ Vall,
                                                     const int* __restrict__ rot, const int* __restrict__ active,
                                                     int nsp, int nb, int round) {
  const int g = blockIdx.z;
  if (!active[g]) return;
  const int npair = nb / 2;
  const int b = blockIdx.y;
  if (!rot[g * npair + b]) return;
  int Ib, Jb;
  rr_pair(nb, round, b, &Ib, &Jb);
  __shared__ double2 X[kPair][kLd];
  const int tid = threadIdx.x;
  const int w = tid >> 6, bi = w >> 1, bj = w & 1, l = tid & 63;
  double2* Ug = U + (size_t)g * nsp * nsp;
  double2 fb[kPair / 4];
  zfrag_load(Vall + ((size_t)g * npair + b) * kPair * kPair, bj, fb);
  const int col = pair_index(Ib, Jb, 16 * bj + (l & 15));
  const int rend = min(nsp, (int)(blockIdx.x + 1) * kURows);
  for (int r0 = blockIdx.x * kURows; r0 < rend; r0 += kPair) {
    for (int e = tid; e < kPair * kPair; e += 256) {
      const int i = e / kPair, j = e % kPair;
      X[i][j] = Ug[(size_t)(r0 + i) * nsp + pair_index(Ib, Jb, j)];
    }
    __syncthreads();
    dx4 cr, ci;
    zmma_lds_frag(X, fb, bi, cr, ci);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Ug[(size_t)(r0 + 16 * bi + 4 * r + (l >> 4)) * nsp + col] = make_double2(cr[r], ci[r]);
    __syncthreads();
  }
}

// Per group: partial sums of |H_ab|^2 off the diagonal and in total (real entries only).
__global__ __launch_bounds__(256) void k_jac_norms(const double2* __restrict__ H, double* __restrict__ part, int ns,
                                                   int nsp) {
  const int g = blockIdx.y;
  const double2* Hg = H + (size_t)g * nsp * nsp;
  double off = 0.0, tot = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < (size_t)ns * ns; e += (size_t)gridDim.x * 256) {
    const int a = (int)(e / ns), b = (int)(e % ns);
    const double v = zabs2(Hg[(size_t)a * nsp + b]);
    tot += v;
    if (a != b) off += v;
  }
  __shared__ double red[8];
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_down(off, o, 64);
    tot += __shfl_down(tot, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = off;
    red[4 + (threadIdx.x >> 6)] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[((size_t)g * gridDim.x + blockIdx.x) * 2] = red[0] + red[1] + red[2] + red[3];
    part[((size_t)g * gridDim.x + blockIdx.x) * 2 + 1] = red[4] + red[5] + red[6] + red[7];
  }
}

// Order eigenpairs, phase-normalise the first K vectors, write A_g (and the
// sorted eigenvalues).  One work-group per group.
__global__ __launch_bounds__(256) void k_select(const double2* __restrict__ H, const double2* __restrict__ U,
                                                const double2* __restrict__ T, double2* __restrict__ A,
                                                double* __restrict__ eig, double2* __restrict__ rowbuf, int ns,
                                                int nsp, int K, int nc, int P) {
  const int g = blockIdx.x, tid = threadIdx.x;
  const double2* Hg = H + (size_t)g * nsp * nsp;
  const double2* Ug = U + (size_t)g * nsp * nsp;
  extern __shared__ int order[];  // [ns]
  __shared__ double best_v[256];
  __shared__ int best_i[256];
  for (int a = tid; a < ns; a += 256) {
    const double la = Hg[(size_t)a * nsp + a].x;
    int rank = 0;
    for (int b = 0; b < ns; ++b) {
      const double lb = Hg[(size_t)b * nsp + b].x;
      rank += (lb > la) || (lb == la && b < a);
    }
    order[rank] = a;
    eig[(size_t)g * ns + rank] = la;
  }
  __syncthreads();
  double2* row = rowbuf + (size_t)g * ns;
  for (int k = 0; k < K; ++k) {
    const int col = order[k];
    double bv = -1.0;
    int bi = 0;
    for (int a = tid; a < ns; a += 256) {
      const double m = zabs2(Ug[(size_t)a * nsp + col]);
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
    const double2 um = Ug[(size_t)best_i[0] * nsp + col];
    const double mu = sqrt(zabs2(um));
    const double2 ph = mu > 0.0 ? zscale(zconj(um), 1.0 / mu) : make_double2(1.0, 0.0);
    // row k of U^H after the phase: conj(u * ph)
    for (int a = tid; a < ns; a += 256) row[a] = zconj(zmul(Ug[(size_t)a * nsp + col], ph));
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
  double2 *T = nullptr, *Lc = nullptr, *cw, *ph = nullptr, *Qg = nullptr, *u = nullptr, *H, *U, *V, *rowbuf;
  double *wc, *qinv, *norms, *eigd, *thr2;
  int *t0s, *active, *rot, *flag;
};
constexpr int kNormBlocks = 64;

int alloc_calib(Scratch& s, const Plan& pl, bool whiten, CalibBufs& b) {
  const int G = pl.G, ns = pl.ns, P = pl.P;
  const int npix = pl.nx * pl.ny;
  const int nsp = (ns + kPair - 1) / kPair * kPair;
  const int npair = nsp / kBlk / 2;
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
  GPJC_TRY(s.alloc(&b.U, (size_t)G * nsp * nsp));
  GPJC_TRY(s.alloc(&b.V, (size_t)G * npair * kPair * kPair));
  GPJC_TRY(s.alloc(&b.active, (size_t)G));
  GPJC_TRY(s.alloc(&b.thr2, (size_t)G));
  GPJC_TRY(s.alloc(&b.rot, (size_t)G * npair));
  GPJC_TRY(s.alloc(&b.flag, 1));
  GPJC_TRY(s.alloc(&b.eigd, (size_t)G * ns));
  GPJC_TRY(s.alloc(&b.rowbuf, (size_t)G * ns));
  GPJC_TRY(s.alloc(&b.norms, (size_t)G * kNormBlocks * 2));
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
  const int nb = nsp / kBlk;
  const int npair = nb / 2;
  CalibBufs bufs;
  GPJC_TRY(alloc_calib(s, pl, noise_cov != nullptr, bufs));
  double2 *T = bufs.T, *Lc = bufs.Lc, *cw = bufs.cw, *ph = bufs.ph, *Qg = bufs.Qg, *H = bufs.H, *U = bufs.U,
          *V = bufs.V, *rowbuf = bufs.rowbuf;
  double *wc = bufs.wc, *qinv = bufs.qinv, *norms = bufs.norms, *eigd = bufs.eigd, *thr2 = bufs.thr2;
  int *t0s = bufs.t0s, *active = bufs.active, *rot = bufs.rot, *flag = bufs.flag;
  const int nd = 2 * P - 1;
  const int norm_blocks = kNormBlocks;
  hipStream_t st = pl.stream;

  std::vector<int> t0h(G, -1);
  for (int p = 0; p < pl.np; ++p)
    if (t0h[pl.pgroup_h[p]] < 0) t0h[pl.pgroup_h[p]] = p * P;
  GPJC_HIP(hipMemcpyAsync(t0s, t0h.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  std::vector<int> ones(G, 1);
  GPJC_HIP(hipMemcpyAsync(active, ones.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  GPJC_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));

  if (noise_cov) {
    hipLaunchKernelGGL(k_whiten_factor, dim3(1), dim3(256), 0, st, noise_cov, Lc, T, pl.nc, flag);
    GPJC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_calib_maps, dim3(std::min(1024, (npix + 255) / 256)), dim3(256), 0, st, pl.coils, T, roi, cw,
                     wc, pl.nc, npix);
  if (!pl.general)
    hipLaunchKernelGGL(k_calib_tables, dim3(64), dim3(256), 0, st, pl.psf, t0s, ph, qinv, P, pl.nx, pl.ny, pl.nt, G);
  hipLaunchKernelGGL(k_jac_init, dim3(2048), dim3(256), 0, st, H, U, ns, nsp, G);
  GPJC_HIP(hipGetLastError());
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

  const char* venv = std::getenv("GPJC_VERBOSE");
  const bool verbose = venv && venv[0] && venv[0] != '0';
  const double tol = 1e-13;
  // Sweep cap; GPJC_JACOBI_SWEEP_CAP (1..40) lowers it, so a caller can force
  // the non-convergence status from the host.
  int max_sweeps = 40;
  if (const char* cap = std::getenv("GPJC_JACOBI_SWEEP_CAP")) {
    const int c = std::atoi(cap);
    if (c >= 1 && c < max_sweeps) max_sweeps = c;
  }
  std::vector<double> hn((size_t)G * norm_blocks * 2);
  std::vector<int> act(G, 1);
  std::vector<double> th2(G, 0.0);
  bool converged = false;
  for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
    hipLaunchKernelGGL(k_jac_norms, dim3(norm_blocks, G), dim3(256), 0, st, H, norms, ns, nsp);
    GPJC_HIP(hipGetLastError());
    GPJC_HIP(hipMemcpyAsync(hn.data(), norms, sizeof(double) * hn.size(), hipMemcpyDeviceToHost, st));
    GPJC_HIP(hipStreamSynchronize(st));
    int nact = 0;
    for (int g = 0; g < G; ++g) {
      double off = 0.0, tot = 0.0;
      for (int b = 0; b < norm_blocks; ++b) {
        off += hn[((size_t)g * norm_blocks + b) * 2];
        tot += hn[((size_t)g * norm_blocks + b) * 2 + 1];
      }
      if (!std::isfinite(off) || !std::isfinite(tot)) return fail(GPJC_E_NUMERIC, "calibration: non-finite Gram");
      act[g] = off > tol * tol * tot ? 1 : 0;
      // Threshold Jacobi: couplings with |h_pq|^2 <= tol^2 ||H||_F^2 / ns^2
      // are not rotated.  A sweep that rotates nothing therefore leaves
      // off(H) below tol^2 ||H||_F^2, so the sweeps cannot stall.
      th2[g] = tol * tol * tot / ((double)ns * ns);
      nact += act[g];
    }
    if (verbose) {
      double worst = 0.0;
      for (int g = 0; g < G; ++g) {
        double off = 0.0, tot = 0.0;
        for (int b = 0; b < norm_blocks; ++b) {
          off += hn[((size_t)g * norm_blocks + b) * 2];
          tot += hn[((size_t)g * norm_blocks + b) * 2 + 1];
        }
        worst = std::max(worst, std::sqrt(off / tot));
      }
      std::fprintf(stderr, "[gpjc] calibrate sweep %d: %d groups active, worst off/total %.3e\n", sweep, nact, worst);
    }
    if (nact == 0) {
      converged = true;
      break;
    }
    if (sweep == max_sweeps) break;
    GPJC_HIP(hipMemcpyAsync(active, act.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
    GPJC_HIP(hipMemcpyAsync(thr2, th2.data(), sizeof(double) * G, hipMemcpyHostToDevice, st));
    for (int round = 0; round < nb - 1; ++round) {
      hipLaunchKernelGGL(k_jac_solve, dim3(npair, G), dim3(256), 0, st, H, V, rot, active, thr2, nsp, nb, round,
                         1e-15);
      hipLaunchKernelGGL(k_jac_apply_h, dim3(npair * npair, G), dim3(64), 0, st, H, V, rot, active, nsp, nb, round);
      hipLaunchKernelGGL(k_jac_apply_u, dim3((nsp + kURows - 1) / kURows, npair, G), dim3(256), 0, st, U, V, rot,
                         active, nsp, nb, round);
    }
    GPJC_HIP(hipGetLastError());
  }
  if (!converged) return fail(GPJC_E_NUMERIC, "calibration: Jacobi did not converge within the sweep cap");

  const size_t lds = sizeof(int) * (size_t)ns;
  hipLaunchKernelGGL(k_select, dim3(G), dim3(256), lds, st, H, U, T, pl.A128, eigd, rowbuf, ns, nsp, pl.K, pl.nc, P);
  GPJC_HIP(hipGetLastError());
  int hflag = 0;
  GPJC_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  GPJC_HIP(hipStreamSynchronize(st));
  if (hflag) return fail(GPJC_E_NUMERIC, "calibration: noise covariance is not positive definite");
  GPJC_TRY(launch_expand_bank(pl));
  if (pl.general) GPJC_TRY(launch_build_explicit(pl));
  pl.have_bank = true;
  if (A_out)
    GPJC_HIP(hipMemcpyAsync(A_out, pl.A128, sizeof(double2) * (size_t)G * pl.K * ns, hipMemcpyDeviceToDevice, st));
  if (h_eig) GPJC_HIP(hipMemcpyAsync(h_eig, eigd, sizeof(double) * (size_t)G * ns, hipMemcpyDeviceToHost, st));
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
