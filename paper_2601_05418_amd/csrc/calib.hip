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
// 3. Eigen-decomposition (Eq. 8) by block-cyclic Jacobi: the matrix (padded
//    to a multiple of 32 with decoupled diagonal entries -1, below every
//    eigenvalue of the PSD P_g) is cut into blocks of 16; each round pairs
//    the blocks by a round-robin tournament, diagonalises every 32 x 32 pair
//    problem with complex Jacobi rotations in LDS, and applies the rotations
//    to the whole matrix (H <- Q^H H Q) and to the eigenvector accumulator
//    (U <- U Q).  Sweeps repeat until the off-diagonal Frobenius norm is
//    below 1e-13 of the total.
// 4. Selection (Eq. 12): eigenvalues in decreasing order (ties by index),
//    each of the first K eigenvectors scaled by a unit phase so that its
//    largest-magnitude entry (lowest index on ties) is real positive,
//    A_g = [u_1 ... u_K]^H (T (x) I_P).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fft.h"
#include "plan.h"

namespace gpjc {

namespace {

__device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ inline double2 zmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ inline double2 zcmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

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

// dtab[j][ix] = exp(-2 pi i j (ix - nx/2) / nt); qinv[g][iy] = 1 / sum_j |psf[iy][t0_g + j]|^2.
__global__ void k_calib_tables(const float2* __restrict__ psf, const int* __restrict__ t0s, double2* __restrict__ dtab,
                               double* __restrict__ qinv, int P, int nx, int ny, int nt, int G) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  for (int i = gid; i < P * nx; i += stride) {
    const int j = i / nx, ix = i % nx;
    const long m = ((long)j * (ix - nx / 2)) % nt;
    double sn, cs;
    sincospi(-2.0 * (double)m / nt, &sn, &cs);
    dtab[i] = make_double2(cs, sn);
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
// Gram: one 64 x 64 tile (ta <= tb) of P_g per work-group, 4 x 4 complex
// accumulators per thread, virtual channels synthesised per pixel chunk.
// ---------------------------------------------------------------------------
constexpr int kGT = 64;   // tile
constexpr int kGR = 16;   // pixels per chunk

__global__ __launch_bounds__(256) void k_gram(const double2* __restrict__ cw, const double* __restrict__ wc,
                                              const float2* __restrict__ psf, const double2* __restrict__ dtab,
                                              const double* __restrict__ qinv, const int* __restrict__ t0s,
                                              double2* __restrict__ H, int P, int nx, int ny, int nt, int ns,
                                              int nsp, int ntile) {
  const int ta = blockIdx.x / ntile, tb = blockIdx.x % ntile;
  if (tb < ta) return;
  const int g = blockIdx.y;
  const int t0 = t0s[g];
  const int npix = nx * ny;
  __shared__ double2 eA[kGT][kGR + 1];
  __shared__ double2 eB[kGT][kGR + 1];
  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  const double* qg = qinv + (size_t)g * ny;
  for (int r0 = 0; r0 < npix; r0 += kGR) {
    for (int e = tid; e < 2 * kGT * kGR; e += 256) {
      const int side = e / (kGT * kGR);
      const int rem = e - side * kGT * kGR;
      const int a = rem / kGR, rr = rem - a * kGR;
      const int idx = (side ? tb : ta) * kGT + a;
      const int r = r0 + rr;
      double2 v = make_double2(0.0, 0.0);
      if (idx < ns && r < npix) {
        const int n = idx / P, j = idx - n * P;
        const int iy = r / nx, ix = r - iy * nx;
        const float2 pf = psf[(size_t)iy * nt + t0 + j];
        v = zmul(zmul(cw[(size_t)n * npix + r], make_double2(pf.x, pf.y)), dtab[j * nx + ix]);
        if (side == 0) v = zscale(v, wc[r] * qg[iy]);
      }
      if (side) eB[a][rr] = v;
      else eA[a][rr] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kGR; ++rr) {
      double2 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = eA[ty + 16 * i][rr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = eB[tx + 16 * j][rr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x = fma(av[i].x, bv[j].x, fma(av[i].y, bv[j].y, acc[i][j].x));
          acc[i][j].y = fma(av[i].y, bv[j].x, fma(-av[i].x, bv[j].y, acc[i][j].y));
        }
    }
    __syncthreads();
  }
  double2* Hg = H + (size_t)g * nsp * nsp;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int al = ta * kGT + ty + 16 * i, be = tb * kGT + tx + 16 * j;
      if (al < ns && be < ns) {
        Hg[(size_t)al * nsp + be] = acc[i][j];
        if (ta != tb) Hg[(size_t)be * nsp + al] = zconj(acc[i][j]);
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

// Diagonalise the 32 x 32 problem of block pair `pr` in round `round`; V out.
__global__ __launch_bounds__(256) void k_jac_solve(const double2* __restrict__ H, double2* __restrict__ Vout,
                                                   const int* __restrict__ active, int nsp, int nb, int round,
                                                   double tol) {
  const int g = blockIdx.y, pr = blockIdx.x;
  if (!active[g]) return;
  int I, J;
  rr_pair(nb, round, pr, &I, &J);
  __shared__ double2 M[kPair][kLd];
  __shared__ double2 V[kPair][kLd];
  __shared__ double prm_c[kPair / 2], prm_s[kPair / 2];
  __shared__ double2 prm_u[kPair / 2];
  __shared__ int prm_p[kPair / 2], prm_q[kPair / 2];
  __shared__ double red[8];
  __shared__ int done;
  const int tid = threadIdx.x;
  const double2* Hg = H + (size_t)g * nsp * nsp;
  for (int e = tid; e < kPair * kPair; e += 256) {
    const int a = e / kPair, b = e % kPair;
    M[a][b] = Hg[(size_t)pair_index(I, J, a) * nsp + pair_index(I, J, b)];
    V[a][b] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 15; ++sweep) {
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
      done = (o <= tol * tol * t) ? 1 : 0;
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
        if (mc > 1e-300) {
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
      // columns of M and V: X[:, p] = cs X[:, p] - sn conj(u) X[:, q]; X[:, q] = sn X[:, p] + cs conj(u) X[:, q]
      for (int e = tid; e < 2 * (kPair / 2) * kPair; e += 256) {
        const int which = e / ((kPair / 2) * kPair);
        const int rem = e - which * (kPair / 2) * kPair;
        const int i = rem / kPair, k = rem % kPair;
        const int p = prm_p[i], q = prm_q[i];
        const double cs = prm_c[i], sn = prm_s[i];
        const double2 uc = zconj(prm_u[i]);
        double2(*X)[kLd] = which ? V : M;
        const double2 xp = X[k][p], xq = X[k][q];
        X[k][p] = zsub(zscale(xp, cs), zscale(zmul(xq, uc), sn));
        X[k][q] = zadd(zscale(xp, sn), zscale(zmul(xq, uc), cs));
      }
      __syncthreads();
      // rows of M: M[p, :] = cs M[p, :] - sn u M[q, :]; M[q, :] = sn M[p, :] + cs u M[q, :]
      for (int e = tid; e < (kPair / 2) * kPair; e += 256) {
        const int i = e / kPair, k = e % kPair;
        const int p = prm_p[i], q = prm_q[i];
        const double cs = prm_c[i], sn = prm_s[i];
        const double2 u = prm_u[i];
        const double2 mp = M[p][k], mq = M[q][k];
        M[p][k] = zsub(zscale(mp, cs), zscale(zmul(mq, u), sn));
        M[q][k] = zadd(zscale(mp, sn), zscale(zmul(mq, u), cs));
      }
      __syncthreads();
    }
  }
  double2* Vg = Vout + ((size_t)g * (nb / 2) + pr) * kPair * kPair;
  for (int e = tid; e < kPair * kPair; e += 256) Vg[e] = V[e / kPair][e % kPair];
}

// H <- Q^H H Q on the tile of pair a (rows) x pair b (cols), a <= b.
__global__ __launch_bounds__(256) void k_jac_apply_h(double2* __restrict__ H, const double2* __restrict__ Vall,
                                                     const int* __restrict__ active, int nsp, int nb, int round) {
  const int g = blockIdx.y;
  if (!active[g]) return;
  const int npair = nb / 2;
  const int a = blockIdx.x / npair, b = blockIdx.x % npair;
  if (b < a) return;
  int Ia, Ja, Ib, Jb;
  rr_pair(nb, round, a, &Ia, &Ja);
  rr_pair(nb, round, b, &Ib, &Jb);
  __shared__ double2 X[kPair][kLd];
  __shared__ double2 Va[kPair][kLd];
  __shared__ double2 Vb[kPair][kLd];
  const int tid = threadIdx.x;
  double2* Hg = H + (size_t)g * nsp * nsp;
  const double2* Vga = Vall + ((size_t)g * npair + a) * kPair * kPair;
  const double2* Vgb = Vall + ((size_t)g * npair + b) * kPair * kPair;
  for (int e = tid; e < kPair * kPair; e += 256) {
    const int i = e / kPair, j = e % kPair;
    X[i][j] = Hg[(size_t)pair_index(Ia, Ja, i) * nsp + pair_index(Ib, Jb, j)];
    Va[i][j] = Vga[e];
    Vb[i][j] = Vgb[e];
  }
  __syncthreads();
  // thread owns rows ti, ti+16 and cols tj, tj+16
  const int ti = tid / 16, tj = tid % 16;
  double2 t[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < kPair; ++k) s = zadd(s, zmul(X[ti + 16 * u][k], Vb[k][tj + 16 * v]));
      t[u][v] = s;
    }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) X[ti + 16 * u][tj + 16 * v] = t[u][v];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = ti + 16 * u, j = tj + 16 * v;
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < kPair; ++k) s = zadd(s, zcmul(Va[k][i], X[k][j]));
      const int gi = pair_index(Ia, Ja, i), gj = pair_index(Ib, Jb, j);
      Hg[(size_t)gi * nsp + gj] = s;
      if (a != b) Hg[(size_t)gj * nsp + gi] = zconj(s);
    }
}

// U[:, pair b] <- U[:, pair b] V_b on 32 rows per work-group.
__global__ __launch_bounds__(256) void k_jac_apply_u(double2* __restrict__ U, const double2* __restrict__ Vall,
                                                     const int* __restrict__ active, int nsp, int nb, int round) {
  const int g = blockIdx.z;
  if (!active[g]) return;
  const int npair = nb / 2;
  const int b = blockIdx.y, r0 = blockIdx.x * kPair;
  int Ib, Jb;
  rr_pair(nb, round, b, &Ib, &Jb);
  __shared__ double2 X[kPair][kLd];
  __shared__ double2 Vb[kPair][kLd];
  const int tid = threadIdx.x;
  double2* Ug = U + (size_t)g * nsp * nsp;
  const double2* Vgb = Vall + ((size_t)g * npair + b) * kPair * kPair;
  for (int e = tid; e < kPair * kPair; e += 256) {
    const int i = e / kPair, j = e % kPair;
    X[i][j] = Ug[(size_t)(r0 + i) * nsp + pair_index(Ib, Jb, j)];
    Vb[i][j] = Vgb[e];
  }
  __syncthreads();
  const int ti = tid / 16, tj = tid % 16;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = ti + 16 * u, j = tj + 16 * v;
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < kPair; ++k) s = zadd(s, zmul(X[i][k], Vb[k][j]));
      Ug[(size_t)(r0 + i) * nsp + pair_index(Ib, Jb, j)] = s;
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

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  int alloc(T** p, size_t n) {
    *p = nullptr;
    GPJC_TRY(dmalloc(p, std::max<size_t>(n, 1)));
    ptrs.push_back(*p);
    return GPJC_OK;
  }
};

}  // namespace

int run_calibrate(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out) {
  const int G = pl.G, ns = pl.ns, P = pl.P;
  const int npix = pl.nx * pl.ny;
  const int nsp = (ns + kPair - 1) / kPair * kPair;
  const int nb = nsp / kBlk;
  const int npair = nb / 2;
  Scratch s;
  double2 *T = nullptr, *Lc = nullptr, *cw, *dtab, *H, *U, *V, *rowbuf;
  double *wc, *qinv, *norms, *eigd;
  int *t0s, *active, *flag;
  GPJC_TRY(s.alloc(&cw, (size_t)pl.nc * npix));
  GPJC_TRY(s.alloc(&wc, (size_t)npix));
  GPJC_TRY(s.alloc(&dtab, (size_t)P * pl.nx));
  GPJC_TRY(s.alloc(&qinv, (size_t)G * pl.ny));
  GPJC_TRY(s.alloc(&t0s, (size_t)G));
  GPJC_TRY(s.alloc(&H, (size_t)G * nsp * nsp));
  GPJC_TRY(s.alloc(&U, (size_t)G * nsp * nsp));
  GPJC_TRY(s.alloc(&V, (size_t)G * npair * kPair * kPair));
  GPJC_TRY(s.alloc(&active, (size_t)G));
  GPJC_TRY(s.alloc(&flag, 1));
  GPJC_TRY(s.alloc(&eigd, (size_t)G * ns));
  GPJC_TRY(s.alloc(&rowbuf, (size_t)G * ns));
  const int norm_blocks = 64;
  GPJC_TRY(s.alloc(&norms, (size_t)G * norm_blocks * 2));
  hipStream_t st = pl.stream;

  std::vector<int> t0h(G, -1);
  for (int p = 0; p < pl.np; ++p)
    if (t0h[pl.pgroup_h[p]] < 0) t0h[pl.pgroup_h[p]] = p * P;
  GPJC_HIP(hipMemcpyAsync(t0s, t0h.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  std::vector<int> ones(G, 1);
  GPJC_HIP(hipMemcpyAsync(active, ones.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  GPJC_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));

  if (noise_cov) {
    GPJC_TRY(s.alloc(&Lc, (size_t)pl.nc * pl.nc));
    GPJC_TRY(s.alloc(&T, (size_t)pl.nc * pl.nc));
    hipLaunchKernelGGL(k_whiten_factor, dim3(1), dim3(256), 0, st, noise_cov, Lc, T, pl.nc, flag);
    GPJC_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_calib_maps, dim3(std::min(1024, (npix + 255) / 256)), dim3(256), 0, st, pl.coils, T, roi, cw,
                     wc, pl.nc, npix);
  hipLaunchKernelGGL(k_calib_tables, dim3(64), dim3(256), 0, st, pl.psf, t0s, dtab, qinv, P, pl.nx, pl.ny, pl.nt, G);
  hipLaunchKernelGGL(k_jac_init, dim3(2048), dim3(256), 0, st, H, U, ns, nsp, G);
  GPJC_HIP(hipGetLastError());
  const int ntile = (ns + kGT - 1) / kGT;
  hipLaunchKernelGGL(k_gram, dim3(ntile * ntile, G), dim3(256), 0, st, cw, wc, pl.psf, dtab, qinv, t0s, H, P, pl.nx,
                     pl.ny, pl.nt, ns, nsp, ntile);
  GPJC_HIP(hipGetLastError());

  const char* venv = std::getenv("GPJC_VERBOSE");
  const bool verbose = venv && venv[0] && venv[0] != '0';
  const double tol = 1e-13;
  const int max_sweeps = 40;
  std::vector<double> hn((size_t)G * norm_blocks * 2);
  std::vector<int> act(G, 1);
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
    for (int round = 0; round < nb - 1; ++round) {
      hipLaunchKernelGGL(k_jac_solve, dim3(npair, G), dim3(256), 0, st, H, V, active, nsp, nb, round, 1e-15);
      hipLaunchKernelGGL(k_jac_apply_h, dim3(npair * npair, G), dim3(256), 0, st, H, V, active, nsp, nb, round);
      hipLaunchKernelGGL(k_jac_apply_u, dim3(nsp / kPair, npair, G), dim3(256), 0, st, U, V, active, nsp, nb, round);
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
  pl.have_bank = true;
  if (A_out)
    GPJC_HIP(hipMemcpyAsync(A_out, pl.A128, sizeof(double2) * (size_t)G * pl.K * ns, hipMemcpyDeviceToDevice, st));
  if (h_eig) GPJC_HIP(hipMemcpyAsync(h_eig, eigd, sizeof(double) * (size_t)G * ns, hipMemcpyDeviceToHost, st));
  GPJC_HIP(hipStreamSynchronize(st));
  return GPJC_OK;
}

}  // namespace gpjc
