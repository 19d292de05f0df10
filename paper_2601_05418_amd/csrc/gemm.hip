// Group contraction of the compressed operator (Eqs. 13-14 applied to hybrid
// data) on MFMA:
//
//   compress  Z_p[k][y]          = sum_{n,j} A_g[k][n][j] W[n][y][p P + j]
//   expand    W[n][y][p P + j]   = sum_k conj(A_g[k][n][j]) Z_p[k][y]
//
// A complex product is one real product of the expanded matrix
// [[Ar, -Ai], [Ai, Ar]] with interleaved (re, im) columns, so both operands
// are read in their natural interleaved layouts and the contraction index kk
// is contiguous in memory for both.
//
// FP32 (v_mfma_f32_16x16x4_f32): in a block of 16 kk, lane (i, q)
// (i = lane % 16, q = lane / 16) holds kk = kb + 4q .. kb + 4q + 3 of row i
// as one float4 and feeds element e to the e-th MFMA; the four MFMAs
// together cover the 16 kk.
// BF16 / FP16 (v_mfma_f32_16x16x32_{bf16,f16}): in a block of 32 kk, lane
// (i, q) holds kk = kb + 8q .. kb + 8q + 7 of row i (16 bytes), one MFMA per
// block, FP32 accumulation.
// Either way one 16-byte load per lane and operand tile feeds a block, and
// loads run kDepth - 1 blocks ahead of the MFMAs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "devutil.h"
#include "plan.h"

namespace gpjc {

namespace {

constexpr floatx4 kZero4 = {0.f, 0.f, 0.f, 0.f};
constexpr int kDepth = 3;  // register ring depth of the operand pipeline

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Operand element type and contraction block per storage precision.
template <Store ST>
struct Mma {
  using E = uint16_t;
  static constexpr int KB = 32;  // kk per block
  static constexpr int LW = 8;   // kk per lane per block
  static constexpr int NE = 1;   // MFMAs per block and tile pair
};
template <>
struct Mma<Store::F32> {
  using E = float;
  static constexpr int KB = 16;
  static constexpr int LW = 4;
  static constexpr int NE = 4;
};

// One MFMA step: 16-byte lane operands a, b (bit containers), step e of the block.
template <Store ST>
__device__ inline floatx4 mma_step(const floatx4& a, const floatx4& b, int e, const floatx4& c) {
  if constexpr (ST == Store::F32) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], c, 0, 0, 0);
  } else if constexpr (ST == Store::BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
  }
}

struct CompressArgs {
  const void* A;    // [G][M][KD] elements, M = 2K rows (k, re/im), KD = 2 ns
  const void* in;   // element view of [B][nc][N][nt] complex
  float2* out;      // [ksplit][B][np][K][N]
  const int* pgroup;
  const void* zeros;  // >= 16 zero bytes: the source of every masked-out load
  int M, N, KD, nc, nt, P, np, K, B, ksplit, kchunk;
  size_t split_stride;
};

// Work-group tile (WM*MT*16) x (WN*NT*16); wave tile (MT*16) x (NT*16).
template <int WM, int WN, int MT, int NT, Store ST>
__global__ __launch_bounds__(64 * WM * WN) void k_compress(CompressArgs a) {
  using E = typename Mma<ST>::E;
  constexpr int KB = Mma<ST>::KB, LW = Mma<ST>::LW, NE = Mma<ST>::NE;
  constexpr int TM = WM * MT * 16, TN = WN * NT * 16;
  const E* Ab = static_cast<const E*>(a.A);
  const E* inb = static_cast<const E*>(a.in);
  const E* zeros = static_cast<const E*>(a.zeros);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int wm = wave / WN, wn = wave % WN;
  const int tiles_n = (a.N + TN - 1) / TN, tiles_m = (a.M + TM - 1) / TM;
  const int total = tiles_n * tiles_m * a.B * a.np * a.ksplit;
  const int logical = xcd_logical(blockIdx.x, total);
  const int tn = logical % tiles_n;
  const int rest = logical / tiles_n;
  const int tm = rest % tiles_m, z = rest / tiles_m;
  const int ks = z % a.ksplit, bp = z / a.ksplit;
  const int b = bp / a.np, p = bp - b * a.np;
  const int g = a.pgroup[p];
  const int row0 = tm * TM + wm * MT * 16, col0 = tn * TN + wn * NT * 16;
  const int twoP = 2 * a.P;
  const size_t coil_stride = (size_t)a.N * a.nt * 2;

  const E* arow[MT];
  bool va[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int r = row0 + 16 * m + li;
    va[m] = r < a.M;
    arow[m] = Ab + ((size_t)g * a.M + (va[m] ? r : 0)) * a.KD;
  }
  const E* brow[NT];
  bool vb[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    const int cc = col0 + 16 * c + li;
    vb[c] = cc < a.N;
    brow[c] = inb + ((size_t)b * a.nc * a.N + (vb[c] ? cc : 0)) * a.nt * 2 + (size_t)p * twoP;
  }
  floatx4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[m][c] = kZero4;

  const int kbeg = ks * a.kchunk;
  const int kend = min(a.KD, kbeg + a.kchunk);
  // lane position in the contraction: kk = n * 2P + jj
  int kk = kbeg + LW * lq;
  int n = kk / twoP;
  int jj = kk - n * twoP;
  // Masked-out operands are read from the zero buffer (the address is
  // selected, never the loaded value, so no load has to complete before
  // the MFMAs of the current block are issued).
  auto load = [&](floatx4(&xa)[MT], floatx4(&xb)[NT]) {
    const bool vk = kk < kend;
    const size_t kb_off = (size_t)n * coil_stride + jj;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      xa[m] = *reinterpret_cast<const floatx4*>((va[m] && vk) ? arow[m] + kk : zeros);
#pragma unroll
    for (int c = 0; c < NT; ++c)
      xb[c] = *reinterpret_cast<const floatx4*>((vb[c] && vk) ? brow[c] + kb_off : zeros);
  };
  // Ring of kDepth register buffers with compile-time indices: block s is
  // multiplied while blocks s+1 .. s+kDepth-1 are in flight.  Blocks past
  // kend load zeros, so the ring may run over the end of the chunk.
  auto advance = [&]() {
    kk += KB;
    jj += KB;
#pragma unroll
    for (int w = 0; w < 4; ++w) {  // 2P >= KB / 4, so at most four coil wraps per block
      const bool wrap = jj >= twoP;
      jj = wrap ? jj - twoP : jj;
      n += wrap ? 1 : 0;
    }
  };
  floatx4 ra[kDepth][MT], rb[kDepth][NT];
#pragma unroll
  for (int s = 0; s < kDepth - 1; ++s) {
    load(ra[s], rb[s]);
    advance();
  }
  for (int kb = kbeg; kb < kend; kb += KB * kDepth) {
#pragma unroll
    for (int s = 0; s < kDepth; ++s) {
      load(ra[(s + kDepth - 1) % kDepth], rb[(s + kDepth - 1) % kDepth]);
      advance();
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int c = 0; c < NT; ++c) acc[m][c] = mma_step<ST>(ra[s][m], rb[s][c], e, acc[m][c]);
    }
  }
  // acc[m][c][r] = C[row0 + 16 m + 4 lq + r][col0 + 16 c + li]; rows pair up as (k, re), (k, im).
  float2* out = a.out + ks * a.split_stride + ((size_t)b * a.np + p) * a.K * a.N;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const int row = row0 + 16 * m + 4 * lq;
      const int col = col0 + 16 * c + li;
      if (col < a.N) {
        if (row < a.M) out[(size_t)(row >> 1) * a.N + col] = make_float2(acc[m][c][0], acc[m][c][1]);
        if (row + 2 < a.M) out[(size_t)((row >> 1) + 1) * a.N + col] = make_float2(acc[m][c][2], acc[m][c][3]);
      }
    }
}

struct ExpandArgs {
  const void* Zt;   // [B][np][M][KD] elements, M = ny, KD = 2 kp
  const void* AH;   // [G][N][KD], N = 2 ns
  void* W;          // [B][nc][ny][nt] complex (storage per Store)
  const int* pgroup;
  const void* zeros;
  int M, N, KD, nc, nt, P, np, B;
};

template <int WM, int WN, int MT, int NT, Store ST>
__global__ __launch_bounds__(64 * WM * WN) void k_expand(ExpandArgs a) {
  using E = typename Mma<ST>::E;
  constexpr int KB = Mma<ST>::KB, LW = Mma<ST>::LW, NE = Mma<ST>::NE;
  constexpr int TM = WM * MT * 16, TN = WN * NT * 16;
  const E* Zb = static_cast<const E*>(a.Zt);
  const E* Hb = static_cast<const E*>(a.AH);
  const E* zeros = static_cast<const E*>(a.zeros);
  constexpr int LDT = TN + 4;
  __shared__ float tile[TM * LDT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int wm = wave / WN, wn = wave % WN;
  const int tiles_n = (a.N + TN - 1) / TN, tiles_m = (a.M + TM - 1) / TM;
  const int total = tiles_n * tiles_m * a.B * a.np;
  const int logical = xcd_logical(blockIdx.x, total);
  const int tn = logical % tiles_n;
  const int rest = logical / tiles_n;
  const int tm = rest % tiles_m, bp = rest / tiles_m;
  const int b = bp / a.np, p = bp - b * a.np;
  const int g = a.pgroup[p];
  const int row0 = tm * TM + wm * MT * 16, col0 = tn * TN + wn * NT * 16;

  const E* arow[MT];
  bool va[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int r = row0 + 16 * m + li;
    va[m] = r < a.M;
    arow[m] = Zb + ((size_t)bp * a.M + (va[m] ? r : 0)) * a.KD;
  }
  const E* brow[NT];
  bool vb[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    const int cc = col0 + 16 * c + li;
    vb[c] = cc < a.N;
    brow[c] = Hb + ((size_t)g * a.N + (vb[c] ? cc : 0)) * a.KD;
  }
  floatx4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[m][c] = kZero4;
  int kk = LW * lq;
  auto load = [&](floatx4(&xa)[MT], floatx4(&xb)[NT]) {
    const bool vk = kk < a.KD;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      xa[m] = *reinterpret_cast<const floatx4*>((va[m] && vk) ? arow[m] + kk : zeros);
#pragma unroll
    for (int c = 0; c < NT; ++c)
      xb[c] = *reinterpret_cast<const floatx4*>((vb[c] && vk) ? brow[c] + kk : zeros);
  };
  floatx4 ra[kDepth][MT], rb[kDepth][NT];
#pragma unroll
  for (int s = 0; s < kDepth - 1; ++s) {
    load(ra[s], rb[s]);
    kk += KB;
  }
  for (int kb = 0; kb < a.KD; kb += KB * kDepth) {
#pragma unroll
    for (int s = 0; s < kDepth; ++s) {
      load(ra[(s + kDepth - 1) % kDepth], rb[(s + kDepth - 1) % kDepth]);
      kk += KB;
#pragma unroll
      for (int e = 0; e < NE; ++e)
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int c = 0; c < NT; ++c) acc[m][c] = mma_step<ST>(ra[s][m], rb[s][c], e, acc[m][c]);
    }
  }
  // stage the tile in LDS, then write whole W row segments
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        tile[(wm * MT * 16 + 16 * m + 4 * lq + r) * LDT + wn * NT * 16 + 16 * c + li] = acc[m][c][r];
  __syncthreads();
  const int twoP = 2 * a.P;
  const int rbase = tm * TM, cbase = tn * TN;
  for (int e = threadIdx.x; e < TM * (TN / 4); e += 64 * WM * WN) {
    const int rl = e / (TN / 4), cl = (e - rl * (TN / 4)) * 4;
    const int y = rbase + rl, col = cbase + cl;
    if (y >= a.M || col >= a.N) continue;
    const int n = col / twoP, jj = col - n * twoP;
    const size_t fi = (((size_t)b * a.nc + n) * a.M + y) * (size_t)a.nt * 2 + (size_t)p * twoP + jj;
    const float* src = tile + rl * LDT + cl;
    if constexpr (ST == Store::F32) {
      *reinterpret_cast<floatx4*>(reinterpret_cast<float*>(a.W) + fi) = floatx4{src[0], src[1], src[2], src[3]};
    } else {
      uint2 v;
      v.x = to_bits16<ST>(src[0]) | (to_bits16<ST>(src[1]) << 16);
      v.y = to_bits16<ST>(src[2]) | (to_bits16<ST>(src[3]) << 16);
      *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(a.W) + fi) = v;
    }
  }
}

// Real forms of the bank: Aexp [G][2K][2ns] (compressing), AH [G][2ns][2kp]
// (expanding), in FP32 and, when the 16-bit copies exist, rounded once more
// (nearest even) to BF16 (index 0) and FP16 (index 1) in the same layouts.
struct BankOut {
  float* Aexp;
  float* AH;
  uint16_t* Aexp16[2];
  uint16_t* AH16[2];
};

__device__ inline void put16(uint16_t* const (&dst)[2], size_t i, float v) {
  if (dst[0]) dst[0][i] = (uint16_t)f32_to_bf16_bits(v);
  if (dst[1]) dst[1][i] = (uint16_t)f32_to_f16_bits(v);
}

__global__ void k_expand_bank(const double2* __restrict__ A, BankOut o, int G, int K, int kp, int ns) {
  const size_t total = (size_t)G * K * ns;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % ns);
    const int k = (int)((idx / ns) % K);
    const int g = (int)(idx / ((size_t)ns * K));
    const double2 v = A[idx];
    const float ar = (float)v.x, ai = (float)v.y;
    const size_t e0 = ((size_t)g * 2 * K + 2 * k) * 2 * ns + 2 * i, e1 = e0 + 2 * ns;
    const float ev[4] = {ar, -ai, ai, ar};  // e0, e0 + 1, e1, e1 + 1
    const size_t ei[4] = {e0, e0 + 1, e1, e1 + 1};
    const size_t h0 = ((size_t)g * 2 * ns + 2 * i) * 2 * kp + 2 * k, h1 = h0 + 2 * kp;
    const float hv[4] = {ar, ai, -ai, ar};
    const size_t hi[4] = {h0, h0 + 1, h1, h1 + 1};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      o.Aexp[ei[r]] = ev[r];
      o.AH[hi[r]] = hv[r];
      put16(o.Aexp16, ei[r], ev[r]);
      put16(o.AH16, hi[r], hv[r]);
    }
  }
}

// Tile-shape tables (waves WM x WN, wave tile MT x NT blocks of 16).
struct Shape {
  int wm, wn, mt, nt;
};
constexpr Shape kCompressShapes[] = {{4, 1, 2, 2}, {4, 1, 2, 4}, {2, 2, 2, 2}, {1, 4, 2, 2}, {2, 2, 2, 4}};
constexpr Shape kExpandShapes[] = {{1, 4, 2, 2}, {1, 4, 2, 4}, {2, 2, 2, 4}, {1, 4, 1, 4}, {2, 2, 2, 2}};
constexpr int kNumCompress = sizeof(kCompressShapes) / sizeof(Shape);
constexpr int kNumExpand = sizeof(kExpandShapes) / sizeof(Shape);

template <int V, Store ST>
void launch_compress_v(dim3 grid, hipStream_t st, const CompressArgs& a) {
  constexpr Shape S = kCompressShapes[V];
  hipLaunchKernelGGL((k_compress<S.wm, S.wn, S.mt, S.nt, ST>), grid, dim3(64 * S.wm * S.wn), 0, st, a);
}
template <int V, Store ST>
void launch_expand_v(dim3 grid, hipStream_t st, const ExpandArgs& a) {
  constexpr Shape S = kExpandShapes[V];
  hipLaunchKernelGGL((k_expand<S.wm, S.wn, S.mt, S.nt, ST>), grid, dim3(64 * S.wm * S.wn), 0, st, a);
}

template <Store ST>
void compress_variant(int v, dim3 grid, hipStream_t st, const CompressArgs& a) {
  switch (v) {
    case 0: launch_compress_v<0, ST>(grid, st, a); break;
    case 1: launch_compress_v<1, ST>(grid, st, a); break;
    case 2: launch_compress_v<2, ST>(grid, st, a); break;
    case 3: launch_compress_v<3, ST>(grid, st, a); break;
    default: launch_compress_v<4, ST>(grid, st, a); break;
  }
}
template <Store ST>
void expand_variant(int v, dim3 grid, hipStream_t st, const ExpandArgs& a) {
  switch (v) {
    case 0: launch_expand_v<0, ST>(grid, st, a); break;
    case 1: launch_expand_v<1, ST>(grid, st, a); break;
    case 2: launch_expand_v<2, ST>(grid, st, a); break;
    case 3: launch_expand_v<3, ST>(grid, st, a); break;
    default: launch_expand_v<4, ST>(grid, st, a); break;
  }
}

int bank16_index(const Plan& pl, Store st) {
  const int i = st == Store::BF16 ? 0 : 1;
  if (!pl.Aexp16[i] || !pl.AH16[i] || !pl.Zt16)
    return fail(GPJC_E_UNSUPPORTED, "16-bit contractions need patch_len divisible by 4");
  return i;
}

int gemm_compress(const Plan& pl, Store st, const void* in, int ncol, float2* out, int ksplit) {
  CompressArgs a;
  if (st == Store::F32) {
    a.A = pl.Aexp;
  } else {
    const int i = bank16_index(pl, st);
    if (i < 0) return i;
    a.A = pl.Aexp16[i];
  }
  a.in = in;
  a.out = out;
  a.pgroup = pl.pgroup;
  a.zeros = pl.zeros;
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
  const int kb = st == Store::F32 ? Mma<Store::F32>::KB : Mma<Store::BF16>::KB;
  a.kchunk = ((a.KD + ksplit - 1) / ksplit + kb - 1) / kb * kb;
  a.split_stride = (size_t)pl.B * pl.np * pl.K * ncol;
  const Shape S = kCompressShapes[pl.gemm_cvar];
  const int TM = S.wm * S.mt * 16, TN = S.wn * S.nt * 16;
  const dim3 grid(((ncol + TN - 1) / TN) * ((a.M + TM - 1) / TM) * pl.B * pl.np * ksplit);
  switch (st) {
    case Store::F32: compress_variant<Store::F32>(pl.gemm_cvar, grid, pl.stream, a); break;
    case Store::BF16: compress_variant<Store::BF16>(pl.gemm_cvar, grid, pl.stream, a); break;
    default: compress_variant<Store::F16>(pl.gemm_cvar, grid, pl.stream, a); break;
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

}  // namespace

int gemm_compress_variants() { return kNumCompress; }
int gemm_expand_variants() { return kNumExpand; }
int compress_tile_rows(const Plan& pl) {
  const Shape S = kCompressShapes[pl.gemm_cvar];
  return S.wm * S.mt * 16;
}
int compress_tile_cols(const Plan& pl) {
  const Shape S = kCompressShapes[pl.gemm_cvar];
  return S.wn * S.nt * 16;
}

int launch_group_compress(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_GROUP_COMPRESS);
  return gemm_compress(pl, st, pl.W, pl.ny, pl.Zp, pl.gemm_ksplit);
}

int launch_compress_data(const Plan& pl, const float2* ksp, float2* out) {
  StageScope sc(pl, GPJC_STAGE_GROUP_COMPRESS);
  return gemm_compress(pl, Store::F32, ksp, pl.ms, out, 1);
}

int launch_group_expand(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_GROUP_EXPAND);
  ExpandArgs a;
  if (st == Store::F32) {
    a.Zt = pl.Zt;
    a.AH = pl.AH;
  } else {
    const int i = bank16_index(pl, st);
    if (i < 0) return i;
    a.Zt = pl.Zt16;
    a.AH = pl.AH16[i];
  }
  a.W = pl.W;
  a.pgroup = pl.pgroup;
  a.zeros = pl.zeros;
  a.M = pl.ny;
  a.N = 2 * pl.ns;
  a.KD = 2 * pl.Kp;
  a.nc = pl.nc;
  a.nt = pl.nt;
  a.P = pl.P;
  a.np = pl.np;
  a.B = pl.B;
  const Shape S = kExpandShapes[pl.gemm_evar];
  const int TM = S.wm * S.mt * 16, TN = S.wn * S.nt * 16;
  const dim3 grid(((a.N + TN - 1) / TN) * ((a.M + TM - 1) / TM) * pl.B * pl.np);
  switch (st) {
    case Store::F32: expand_variant<Store::F32>(pl.gemm_evar, grid, pl.stream, a); break;
    case Store::BF16: expand_variant<Store::BF16>(pl.gemm_evar, grid, pl.stream, a); break;
    default: expand_variant<Store::F16>(pl.gemm_evar, grid, pl.stream, a); break;
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

int launch_expand_bank(Plan& pl) {
  const size_t nh = (size_t)pl.G * 2 * pl.ns * 2 * pl.Kp;
  GPJC_HIP(hipMemsetAsync(pl.AH, 0, nh * sizeof(float), pl.stream));
  BankOut o{pl.Aexp, pl.AH, {pl.Aexp16[0], pl.Aexp16[1]}, {pl.AH16[0], pl.AH16[1]}};
  for (int i = 0; i < 2; ++i)
    if (pl.AH16[i]) GPJC_HIP(hipMemsetAsync(pl.AH16[i], 0, nh * sizeof(uint16_t), pl.stream));
  const size_t total = (size_t)pl.G * pl.K * pl.ns;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_expand_bank, dim3(blocks), dim3(256), 0, pl.stream, pl.A128, o, pl.G, pl.K, pl.Kp, pl.ns);
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

}  // namespace gpjc
