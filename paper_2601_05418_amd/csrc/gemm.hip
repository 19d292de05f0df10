// Group contraction of the compressed operator (Eqs. 13-14 applied to hybrid
// data) on MFMA:
//
//   compress  Z_p[k][y]          = sum_{n,j} A_g[k][n][j] W[n][y][p P + j]
//   expand    W[n][y][p P + j]   = sum_k conj(A_g[k][n][j]) Z_p[k][y]
//
// Both operands are read in their natural interleaved (re, im) layouts, so
// the contraction index kk is contiguous in memory for both.  The bank is
// stored in expanded real form, rows [Ar, -Ai] and [Ai, Ar] interleaved per
// complex row (compressing) and [Ar, Ai], [-Ai, Ar] per complex column
// (expanding).  Two ways of forming the complex product:
// - expanded: one real product with the expanded bank, four real
//   multiplications per complex one (16-bit types and the general forms);
// - three-multiplication (FP32 LDS-staged forms): only the first expanded
//   row of each pair is read, conj(A) (compressing) or A (expanding), and
//   three real products t1, t2, t3 are combined at the end (block_mma).
//
// BF16X6 keeps FP32 storage and runs the contraction on the BF16 MFMA: each
// FP32 operand is split, as it is staged into LDS, into three BF16 pieces
// x = x0 + x1 + x2 (x0 the nearest BF16 to x, x1 the nearest to x - x0, x2
// the nearest to what remains; the remainders are exact in FP32) and the six
// piece products whose orders sum to at most two (00, 01, 10, 02, 11, 20) are
// accumulated in FP32 (the split-operand emulation of a wider product by
// narrow ones, as in Ootomo and Yokota, 2022, and Henry et al., 2019).  The
// dropped products and the last piece's rounding are below 2^-26 of each
// product, under FP32's own rounding of the result.  The bank is read in its
// FP32 form, one row of each expanded pair, and the other row is derived in
// registers ((u, v) -> (-v, u) per complex element, exact on the pieces).
//
// In the 16-bit expanding contraction the phase-encode output Z^T is carried
// as a hi + lo pair of 16-bit values (hi = rn(z), lo = rn(z - hi)): its rows
// hold both parts one after the other and meet the same bank row twice, so
// Z^T adds no rounding beyond the bank's and W's.
//
// Two families of kernels, chosen per launch:
// - LDS-staged (k_compress_lds, k_expand_lds): the work-group loads k-tiles of
//   one 128-byte line per row cooperatively into LDS and the waves read their
//   MFMA fragments from there; 32x32x2 FP32 in the three-multiplication form,
//   or 16x16x32 BF16 / FP16 with FP32 accumulation.  Every geometry whose
//   operands stay below 2 GiB.
// - General (k_compress, k_expand): per-lane addressing with masks, for
//   operands of 2 GiB or more.  In a block of 16 kk (FP32,
//   v_mfma_f32_16x16x4_f32) lane (i, q) (i = lane % 16, q = lane / 16) holds
//   kk = kb + 4q .. kb + 4q + 3 of row i and feeds element e to the e-th MFMA;
//   in a block of 32 kk (16-bit, v_mfma_f32_16x16x32_*) it holds 8 elements and
//   feeds one MFMA.
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
typedef float floatx16 __attribute__((ext_vector_type(16)));

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
template <>
struct Mma<Store::BF16X6> {  // staged form only; the data are FP32
  using E = float;
  static constexpr int KB = 32;
  static constexpr int LW = 8;
  static constexpr int NE = 1;
};

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int kPieces = 3;  // BF16 pieces per FP32 operand in BF16X6

// The kPieces BF16 pieces of four FP32 values, four per 8-byte word: piece q
// is the nearest-even BF16 of what pieces 0..q-1 leave of each value.
__device__ inline void split_pieces(const floatx4& v, uint2 (&p)[kPieces]) {
  floatx4 r = v;
#pragma unroll
  for (int q = 0; q < kPieces; ++q) {
    const bf16x4 h = __builtin_convertvector(r, bf16x4);
    p[q] = __builtin_bit_cast(uint2, h);
    if (q + 1 < kPieces) r -= __builtin_convertvector(h, floatx4);
  }
}
// Pieces of the partner row of an expanded pair: (u, v) -> (-v, u) for each
// complex element held as two BF16 halves of a word.
__device__ inline uint2 partner_pieces(uint2 p) {
  return make_uint2(__builtin_rotateleft32(p.x, 16) ^ 0x8000u, __builtin_rotateleft32(p.y, 16) ^ 0x8000u);
}

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
  int M, N, KD, nc, nt, P, np, K, B, ksplit, kchunk;  // the FP32 staged form is launched with M = K
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
  // With P odd (FP32) a lane's four floats are two complex elements that may
  // lie in two coils: the data operand is read as two 8-byte halves, the
  // second at the next sample or the next coil's first one, or from the zero
  // buffer at or past kend.
  const bool odd = ST == Store::F32 && (twoP & 2);
  auto load = [&](floatx4(&xa)[MT], floatx4(&xb)[NT]) {
    const bool vk = kk < kend;
    const size_t kb_off = (size_t)n * coil_stride + jj;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      xa[m] = *reinterpret_cast<const floatx4*>((va[m] && vk) ? arow[m] + kk : zeros);
    if (odd) {
      const bool vk1 = kk + 2 < kend;
      const size_t kb1 = jj + 2 < twoP ? kb_off + 2 : kb_off + coil_stride - jj;
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const float2 h0 = *reinterpret_cast<const float2*>((vb[c] && vk) ? brow[c] + kb_off : zeros);
        const float2 h1 = *reinterpret_cast<const float2*>((vb[c] && vk1) ? brow[c] + kb1 : zeros);
        xb[c] = floatx4{h0.x, h0.y, h1.x, h1.y};
      }
    } else {
#pragma unroll
      for (int c = 0; c < NT; ++c)
        xb[c] = *reinterpret_cast<const floatx4*>((vb[c] && vk) ? brow[c] + kb_off : zeros);
    }
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

// Writes four consecutive output floats src[0..3] of row y, starting at
// float column col of the (n, j) index (two floats per complex column), to
// W[b][n][y][p P + j].  With 2P a multiple of four they are one 16-byte
// segment of one coil's patch.  With P odd (FP32 only) the two complex values
// are stored one by one, each in its own coil, and a value at or past ncolf
// (the floats of one row) is skipped.
template <Store ST>
__device__ inline void store_w_quad(void* W, const float* src, int b, int y, int col, int ncolf, int M, int nc,
                                    int nt, int P, int p) {
  const int twoP = 2 * P;
  if constexpr (ST == Store::F32) {
    if (twoP & 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = col + 2 * h;
        if (c >= ncolf) break;
        const int n = c / twoP, jj = c - n * twoP;
        const size_t fi = (((size_t)b * nc + n) * M + y) * (size_t)nt * 2 + (size_t)p * twoP + jj;
        *reinterpret_cast<float2*>(reinterpret_cast<float*>(W) + fi) = make_float2(src[2 * h], src[2 * h + 1]);
      }
      return;
    }
  }
  const int n = col / twoP, jj = col - n * twoP;
  const size_t fi = (((size_t)b * nc + n) * M + y) * (size_t)nt * 2 + (size_t)p * twoP + jj;
  if constexpr (ST == Store::F32) {
    *reinterpret_cast<floatx4*>(reinterpret_cast<float*>(W) + fi) = floatx4{src[0], src[1], src[2], src[3]};
  } else {
    uint2 v;
    v.x = to_bits16<ST>(src[0]) | (to_bits16<ST>(src[1]) << 16);
    v.y = to_bits16<ST>(src[2]) | (to_bits16<ST>(src[3]) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(W) + fi) = v;
  }
}

struct ExpandArgs {
  const void* Zt;   // [B][np][M][KD] elements, M = ny; KD = 2 kp (FP32) or 4 kp (16-bit hi | lo)
  const void* AH;   // [G][N][KDB], N = 2 ns, KDB = 2 kp
  void* W;          // [B][nc][ny][nt] complex (storage per Store)
  const int* pgroup;
  const void* zeros;
  int M, N, KD, KDB, nc, nt, P, np, B;  // the FP32 staged form is launched with N = ns
  // 16-bit: Z^T rows hold a hi part and a lo part of 2 kp elements each, and
  // both meet the same bank row: contraction element kk reads bank element
  // kk - kwrap once kk >= kwrap (kwrap = 2 kp; 0 = no wrap).
  int kwrap;
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
    brow[c] = Hb + ((size_t)g * a.N + (vb[c] ? cc : 0)) * a.KDB;
  }
  floatx4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[m][c] = kZero4;
  int kk = LW * lq;
  auto load = [&](floatx4(&xa)[MT], floatx4(&xb)[NT]) {
    const bool vk = kk < a.KD;
    const int kb = (a.kwrap && kk >= a.kwrap) ? kk - a.kwrap : kk;
#pragma unroll
    for (int m = 0; m < MT; ++m)
      xa[m] = *reinterpret_cast<const floatx4*>((va[m] && vk) ? arow[m] + kk : zeros);
#pragma unroll
    for (int c = 0; c < NT; ++c)
      xb[c] = *reinterpret_cast<const floatx4*>((vb[c] && vk) ? brow[c] + kb : zeros);
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
  const int rbase = tm * TM, cbase = tn * TN;
  for (int e = threadIdx.x; e < TM * (TN / 4); e += 64 * WM * WN) {
    const int rl = e / (TN / 4), cl = (e - rl * (TN / 4)) * 4;
    const int y = rbase + rl, col = cbase + cl;
    if (y >= a.M || col >= a.N) continue;
    store_w_quad<ST>(a.W, tile + rl * LDT + cl, b, y, col, a.N, a.M, a.nc, a.nt, a.P, p);
  }
}

// ---------------------------------------------------------------------------
// Buffer-addressed loads of the staged forms: a thread keeps 32-bit byte
// offsets into a buffer resource per operand region; rows, columns and chunks
// out of range get offsets >= 2^31, and buffer loads beyond the descriptor's
// extent return zeros.  Each operand region must stay below 2^31 bytes.
// ---------------------------------------------------------------------------
constexpr uint32_t kOOB = 0x80000000u;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline floatx4 bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ inline float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// MFMA geometry of the staged forms: FP32 uses the 32 x 32 x 2
// instruction (four independent 32 x 32 accumulators sustain close to the
// FP32 peak, the 16 x 16 x 4 form does not), the 16-bit types the 16 x 16 x 32
// one.  A lane (i, h) (i = lane % T, h = lane / T) holds LW consecutive
// contraction elements kb + LW h .. of its row / column; the result register
// r of a lane holds row row_of(r, h) and column i of the T x T tile.
template <Store ST>
struct Geo {
  static constexpr int T = 16, KB = 32, LW = 8, NE = 1, NR = 4;
  using Acc = floatx4;
  __device__ static int row_of(int r, int h) { return 4 * h + r; }
  __device__ static Acc step(const floatx4& a, const floatx4& b, int, const Acc& c) { return mma_step<ST>(a, b, 0, c); }
};
template <>
struct Geo<Store::F32> {
  static constexpr int T = 32, KB = 8, LW = 4, NE = 4, NR = 16;
  using Acc = floatx16;
  __device__ static int row_of(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }
  __device__ static Acc step(const floatx4& a, const floatx4& b, int e, const Acc& c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], c, 0, 0, 0);
  }
};

template <>
struct Geo<Store::BF16X6> {
  static constexpr int T = 16, KB = 32, LW = 8, NE = 1, NR = 4;
  using Acc = floatx4;
  __device__ static int row_of(int r, int h) { return 4 * h + r; }
};

// One k-tile of the BF16X6 product: piece fragments fa[m][q], fb[c][q] (eight
// BF16 of one row each); every accumulator takes the six products of pieces
// whose orders sum to at most kPieces - 1, larger orders first.
template <int MT, int NT>
__device__ inline void split_mma(const floatx4 (&fa)[MT][kPieces], const floatx4 (&fb)[NT][kPieces],
                                 floatx4 (&acc)[MT][NT]) {
#pragma unroll
  for (int s = kPieces - 1; s >= 0; --s)
#pragma unroll
    for (int q = 0; q <= s; ++q)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < NT; ++c)
          acc[m][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, fa[m][q]),
                                                               __builtin_bit_cast(bf16x8, fb[c][s - q]), acc[m][c],
                                                               0, 0, 0);
}

// ---------------------------------------------------------------------------
// Compressing contraction staged through LDS.  The operand layout of an MFMA
// spans 16 or 32 rows per load instruction, so register-direct loads touch
// that many cache lines each; here the work-group loads k-tiles of one
// 128-byte line per row (32 FP32 or 64 16-bit elements) cooperatively, eight
// lanes per row, into LDS, and the waves read their MFMA fragments from
// there (32x32x2 FP32, or 16x16x32 BF16 / FP16 with FP32 accumulation).  The next PF k-tiles are
// prefetched into registers while the current one is multiplied.  Row
// stride 36 floats (144 bytes, an odd multiple of 16): the 16-byte fragment
// reads of one pass fall on distinct bank groups.  Needs 2P a multiple of the
// 16-byte chunk (a chunk never crosses a coil) and the k-split chunk a
// multiple of the k-tile.
// ---------------------------------------------------------------------------
// One MFMA block of a wave's k-tile product: row fragments fa[MT] and
// column fragments fb[NT] into acc.  In FP32 each fragment holds two
// interleaved complex elements and the block is the three-multiplication
// complex product conj(X) Y, X being the bank operand (the rows when XR):
//   t1 += Xr Yr,  t2 += Xi Yi,  t3 += (Xr - Xi)(Yr + Yi),
// from which re = t1 + t2 and im = t3 - t1 + t2.  It takes three real
// products where the expanded 2 x 2 block form takes four.  The 16-bit types
// take the expanded form, one MFMA per block.
template <Store ST, bool XR, int MT, int NT, int NA>
__device__ inline void block_mma(const floatx4 (&fa)[MT], const floatx4 (&fb)[NT],
                                 typename Geo<ST>::Acc (&acc)[NA][MT][NT]) {
  if constexpr (ST == Store::F32) {
    static_assert(NA == 3, "three accumulators per tile");
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float sa[MT], sb[NT];
#pragma unroll
      for (int m = 0; m < MT; ++m) sa[m] = XR ? fa[m][2 * h] - fa[m][2 * h + 1] : fa[m][2 * h] + fa[m][2 * h + 1];
#pragma unroll
      for (int c = 0; c < NT; ++c) sb[c] = XR ? fb[c][2 * h] + fb[c][2 * h + 1] : fb[c][2 * h] - fb[c][2 * h + 1];
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          acc[0][m][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m][2 * h], fb[c][2 * h], acc[0][m][c], 0, 0, 0);
          acc[1][m][c] =
              __builtin_amdgcn_mfma_f32_32x32x2f32(fa[m][2 * h + 1], fb[c][2 * h + 1], acc[1][m][c], 0, 0, 0);
          acc[2][m][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa[m], sb[c], acc[2][m][c], 0, 0, 0);
        }
    }
  } else {
    static_assert(NA == 1, "one accumulator per tile");
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[0][m][c] = Geo<ST>::step(fa[m], fb[c], 0, acc[0][m][c]);
  }
}

template <int WM, int WN, int MT, int NT, int PF, Store ST, bool ODD>
__global__ __launch_bounds__(64 * WM * WN) void k_compress_lds(CompressArgs a) {
  constexpr bool SPL = ST == Store::BF16X6;
  static_assert(!ODD || ST == Store::F32 || SPL, "odd patch lengths are built for FP32 data only");
  using G = Geo<ST>;
  using E = typename Mma<ST>::E;
  constexpr int T = G::T, NR = G::NR;
  constexpr int ES = (int)sizeof(E);
  // k-tile elements per row; LDS row stride in floats (BF16X6: the pieces of
  // a row's k-tile one after the other, 16 floats each)
  constexpr int KT = 128 / ES, LS = SPL ? 16 * kPieces + 4 : 36;
  // FP32 takes the three-multiplication form: a.M counts complex rows k, and
  // row k is bank row 2k, conj(A_g[k]) interleaved.
  constexpr bool C3 = ST == Store::F32;
  constexpr int RS = C3 ? 2 : 1, NA = C3 ? 3 : 1;  // bank rows per kernel row; accumulators per tile
  constexpr int JB = SPL ? 1 : 128 / (G::KB * ES), JF = G::KB * ES / 4;  // MFMA blocks per k-tile, floats per block
  constexpr int TM = WM * MT * T, TN = WN * NT * T, NTHR = 64 * WM * WN;
  // bank rows loaded per k-tile (BF16X6: the first row of each expanded pair)
  constexpr int TA = SPL ? TM / 2 : TM;
  constexpr int AR = TA * 8 / NTHR, BR = TN * 8 / NTHR;  // 16-byte chunks per thread per k-tile
  static_assert(AR * NTHR == TA * 8 && BR * NTHR == TN * 8, "tile rows must split evenly over the threads");
  __shared__ floatx4 smem[(TM + TN) * LS / 4];
  float* As = reinterpret_cast<float*>(smem);
  float* Bs = As + TM * LS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane % T, lh = lane / T;
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
  const int twoP = 2 * a.P;
  const size_t cstride = (size_t)a.N * a.nt * 2;

  const int kbeg = ks * a.kchunk;
  const int kend = min(a.KD, kbeg + a.kchunk);
  const int nst = max(0, (kend - kbeg + KT - 1) / KT);

  const E* Ab = static_cast<const E*>(a.A) + (size_t)g * RS * a.M * a.KD;
  const __amdgpu_buffer_rsrc_t rA = make_rsrc(Ab, (uint32_t)((size_t)RS * a.M * a.KD * ES));
  // The data operand's buffer starts at the first coil of this k-chunk and
  // spans the coils it touches, so 32-bit offsets reach any data size whose
  // per-chunk span fits (the host picks the split for that).
  const int nn0 = kend > kbeg ? kbeg / twoP : 0;
  const int nspan = kend > kbeg ? (kend - 1) / twoP - nn0 + 1 : 0;
  const E* Bb = static_cast<const E*>(a.in) + ((size_t)b * a.nc + nn0) * cstride + (size_t)p * twoP;
  const __amdgpu_buffer_rsrc_t rB =
      make_rsrc(Bb, nspan ? (uint32_t)((nspan * cstride - (size_t)p * twoP) * ES) : 0u);
  // This thread's 16-byte chunk along the contraction: element kk of the
  // (coil, in-patch sample) index, i.e. coil nn, sample jj.  With 2P a
  // multiple of the chunk a chunk never straddles a coil; k-tiles may, so the
  // coil advance is per thread.  Chunks at or past kend read zeros.  ODD (P
  // odd, FP32): a chunk holds two complex elements that may lie in two
  // coils, so the data operand is fetched as two 8-byte halves, the second
  // at offset d1 from the first (the next sample, or the next coil's first
  // one); a second half at or past kend reads zeros, and the bank's matching
  // half then meets a zero factor.
  const int c16 = tid & 7;
  int kk = kbeg + (KT / 8) * c16;
  int jj = kk % twoP;
  const int nn = kk / twoP;
  uint32_t va[AR], vb[BR];
#pragma unroll
  for (int r = 0; r < AR; ++r) {
    const int lr = (tid >> 3) + r * (NTHR / 8);
    const int row = tm * TM + (SPL ? 2 * lr : lr);
    va[r] = row < a.M ? (uint32_t)(((size_t)row * RS * a.KD + kk) * ES) : kOOB;
  }
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    const int cc = tn * TN + (tid >> 3) + r * (NTHR / 8);
    vb[r] = cc < a.N ? (uint32_t)(((size_t)cc * a.nt * 2 + (size_t)(nn - nn0) * cstride + jj) * ES) : kOOB;
  }
  const uint32_t wrap = (uint32_t)((cstride - (size_t)twoP) * ES);  // end of a coil's patch -> next coil's
  floatx4 pa[PF][AR], pb[PF][BR];  // PF k-tiles of loads in flight
  auto fetch = [&](floatx4(&xa)[AR], floatx4(&xb)[BR]) {
    const bool in = kk < kend;
#pragma unroll
    for (int r = 0; r < AR; ++r) xa[r] = bload(rA, in ? va[r] : kOOB);
    if constexpr (ODD) {
      const uint32_t d1 = (uint32_t)((jj + 2 < twoP ? (size_t)2 : cstride - (size_t)twoP + 2) * ES);
      const bool in1 = kk + 2 < kend;
#pragma unroll
      for (int r = 0; r < BR; ++r) {
        const float2 h0 = bload2(rB, in ? vb[r] : kOOB);
        const float2 h1 = bload2(rB, in1 ? vb[r] + d1 : kOOB);
        xb[r] = floatx4{h0.x, h0.y, h1.x, h1.y};
      }
    } else {
#pragma unroll
      for (int r = 0; r < BR; ++r) xb[r] = bload(rB, in ? vb[r] : kOOB);
    }
    kk += KT;
    jj += KT;
    uint32_t inc = KT * ES;
    while (jj >= twoP) {
      jj -= twoP;
      inc += wrap;
    }
#pragma unroll
    for (int r = 0; r < AR; ++r) va[r] += KT * ES;
#pragma unroll
    for (int r = 0; r < BR; ++r) vb[r] += inc;
  };
  typename G::Acc acc[NA][MT][NT];
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[q][m][c][r] = 0.f;
#pragma unroll
  for (int f = 0; f < PF; ++f)
    if (f < nst) fetch(pa[f], pb[f]);
  for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
    for (int f = 0; f < PF; ++f) {
      const int st = st0 + f;
      if (st >= nst) break;
      __syncthreads();  // the previous k-tile has been read
      if constexpr (SPL) {
#pragma unroll
        for (int r = 0; r < AR; ++r) {
          uint2 pc[kPieces];
          split_pieces(pa[f][r], pc);
          float* row = As + 2 * ((tid >> 3) + r * (NTHR / 8)) * LS + 2 * c16;
#pragma unroll
          for (int q = 0; q < kPieces; ++q) {
            *reinterpret_cast<uint2*>(row + 16 * q) = pc[q];
            *reinterpret_cast<uint2*>(row + LS + 16 * q) = partner_pieces(pc[q]);
          }
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
          uint2 pc[kPieces];
          split_pieces(pb[f][r], pc);
          float* row = Bs + ((tid >> 3) + r * (NTHR / 8)) * LS + 2 * c16;
#pragma unroll
          for (int q = 0; q < kPieces; ++q) *reinterpret_cast<uint2*>(row + 16 * q) = pc[q];
        }
      } else {
#pragma unroll
        for (int r = 0; r < AR; ++r)
          *reinterpret_cast<floatx4*>(As + ((tid >> 3) + r * (NTHR / 8)) * LS + 4 * c16) = pa[f][r];
#pragma unroll
        for (int r = 0; r < BR; ++r)
          *reinterpret_cast<floatx4*>(Bs + ((tid >> 3) + r * (NTHR / 8)) * LS + 4 * c16) = pb[f][r];
      }
      __syncthreads();
      if (st + PF < nst) fetch(pa[f], pb[f]);
      if constexpr (SPL) {
        floatx4 fa[MT][kPieces], fb[NT][kPieces];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int q = 0; q < kPieces; ++q)
            fa[m][q] = *reinterpret_cast<const floatx4*>(As + (wm * MT * T + T * m + li) * LS + 16 * q + 4 * lh);
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
          for (int q = 0; q < kPieces; ++q)
            fb[c][q] = *reinterpret_cast<const floatx4*>(Bs + (wn * NT * T + T * c + li) * LS + 16 * q + 4 * lh);
        split_mma<MT, NT>(fa, fb, acc[0]);
      } else {
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          floatx4 fa[MT], fb[NT];
#pragma unroll
          for (int m = 0; m < MT; ++m)
            fa[m] = *reinterpret_cast<const floatx4*>(As + (wm * MT * T + T * m + li) * LS + JF * j + 4 * lh);
#pragma unroll
          for (int c = 0; c < NT; ++c)
            fb[c] = *reinterpret_cast<const floatx4*>(Bs + (wn * NT * T + T * c + li) * LS + JF * j + 4 * lh);
          block_mma<ST, true>(fa, fb, acc);
        }
      }
    }
  }
  float2* out = a.out + ks * a.split_stride + ((size_t)b * a.np + p) * a.K * a.N;
  const int row0 = tm * TM + wm * MT * T, col0 = tn * TN + wn * NT * T;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const int col = col0 + T * c + li;
      if constexpr (C3) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int row = row0 + T * m + G::row_of(r, lh);
          const float t1 = acc[0][m][c][r], t2 = acc[1][m][c][r], t3 = acc[2][m][c][r];
          if (col < a.N && row < a.M) out[(size_t)row * a.N + col] = make_float2(t1 + t2, t3 - t1 + t2);
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; r += 2) {
          const int row = row0 + T * m + G::row_of(r, lh);
          if (col < a.N && row < a.M)
            out[(size_t)(row >> 1) * a.N + col] = make_float2(acc[0][m][c][r], acc[0][m][c][r + 1]);
        }
      }
    }
}

// Expanding contraction staged through LDS, as k_compress_lds: both
// operands (Z^T rows and rows of the real-form bank) are contiguous along the
// contraction, which has 2 Kp elements (a multiple of the k-tile).  The output tile
// is staged through the same LDS to write whole W row segments.
template <int WM, int WN, int MT, int NT, int PF, Store ST>
__global__ __launch_bounds__(64 * WM * WN) void k_expand_lds(ExpandArgs a) {
  constexpr bool SPL = ST == Store::BF16X6;
  using G = Geo<ST>;
  using E = typename Mma<ST>::E;
  constexpr int T = G::T, NR = G::NR;
  constexpr int ES = (int)sizeof(E);
  constexpr int KT = 128 / ES, LS = SPL ? 16 * kPieces + 4 : 36;
  // FP32 takes the three-multiplication form: a.N counts complex columns
  // (n, j), and column i is bank row 2i, A_g[:, i] interleaved.
  constexpr bool C3 = ST == Store::F32;
  constexpr int RS = C3 ? 2 : 1, NA = C3 ? 3 : 1, CF = C3 ? 2 : 1;  // CF: output floats per column
  constexpr int JB = SPL ? 1 : 128 / (G::KB * ES), JF = G::KB * ES / 4;
  constexpr int TM = WM * MT * T, TN = WN * NT * T, NTHR = 64 * WM * WN;
  constexpr int TB = SPL ? TN / 2 : TN;  // bank rows loaded per k-tile (BF16X6: first row of each pair)
  constexpr int AR = TM * 8 / NTHR, BR = TB * 8 / NTHR;
  static_assert(AR * NTHR == TM * 8 && BR * NTHR == TB * 8, "tile rows must split evenly over the threads");
  constexpr int LDT = CF * TN + 4;
  constexpr int SM = ((TM + TN) * LS > TM * LDT ? (TM + TN) * LS : TM * LDT);
  __shared__ floatx4 smem[SM / 4];
  float* As = reinterpret_cast<float*>(smem);
  float* Bs = As + TM * LS;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane % T, lh = lane / T;
  const int wm = wave / WN, wn = wave % WN;
  const int tiles_n = (a.N + TN - 1) / TN, tiles_m = (a.M + TM - 1) / TM;
  const int total = tiles_n * tiles_m * a.B * a.np;
  const int logical = xcd_logical(blockIdx.x, total);
  const int tn = logical % tiles_n;
  const int rest = logical / tiles_n;
  const int tm = rest % tiles_m, bp = rest / tiles_m;
  const int b = bp / a.np, p = bp - b * a.np;
  const int g = a.pgroup[p];

  const __amdgpu_buffer_rsrc_t rA = make_rsrc(static_cast<const E*>(a.Zt) + (size_t)bp * a.M * a.KD,
                                              (uint32_t)((size_t)a.M * a.KD * ES));
  const __amdgpu_buffer_rsrc_t rB = make_rsrc(static_cast<const E*>(a.AH) + (size_t)g * RS * a.N * a.KDB,
                                              (uint32_t)((size_t)RS * a.N * a.KDB * ES));
  const int nst = a.KD / KT;
  const int c16 = tid & 7;
  int kc = (KT / 8) * c16;  // this thread's chunk position along the contraction
  uint32_t va[AR], vb[BR];
#pragma unroll
  for (int r = 0; r < AR; ++r) {
    const int row = tm * TM + (tid >> 3) + r * (NTHR / 8);
    va[r] = row < a.M ? (uint32_t)(((size_t)row * a.KD + (KT / 8) * c16) * ES) : kOOB;
  }
#pragma unroll
  for (int r = 0; r < BR; ++r) {
    const int lr = (tid >> 3) + r * (NTHR / 8);
    const int cc = tn * TN + (SPL ? 2 * lr : lr);
    const int kb0 = (a.kwrap && kc >= a.kwrap) ? kc - a.kwrap : kc;  // a chunk may start in the lo part
    vb[r] = cc < a.N ? (uint32_t)(((size_t)cc * RS * a.KDB + kb0) * ES) : kOOB;
  }
  floatx4 pa[PF][AR], pb[PF][BR];  // PF k-tiles of loads in flight
  auto fetch = [&](floatx4(&xa)[AR], floatx4(&xb)[BR]) {
#pragma unroll
    for (int r = 0; r < AR; ++r) xa[r] = bload(rA, va[r]);
#pragma unroll
    for (int r = 0; r < BR; ++r) xb[r] = bload(rB, vb[r]);
#pragma unroll
    for (int r = 0; r < AR; ++r) va[r] += KT * ES;
    // the bank offset returns to the row start where the lo part begins
    const uint32_t back = (a.kwrap && kc < a.kwrap && kc + KT >= a.kwrap) ? (uint32_t)(a.kwrap * ES) : 0u;
    kc += KT;
#pragma unroll
    for (int r = 0; r < BR; ++r) vb[r] += KT * ES - back;
  };
  typename G::Acc acc[NA][MT][NT];
#pragma unroll
  for (int q = 0; q < NA; ++q)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[q][m][c][r] = 0.f;
#pragma unroll
  for (int f = 0; f < PF; ++f)
    if (f < nst) fetch(pa[f], pb[f]);
  for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
    for (int f = 0; f < PF; ++f) {
      const int st = st0 + f;
      if (st >= nst) break;
      __syncthreads();
      if constexpr (SPL) {
#pragma unroll
        for (int r = 0; r < AR; ++r) {
          uint2 pc[kPieces];
          split_pieces(pa[f][r], pc);
          float* row = As + ((tid >> 3) + r * (NTHR / 8)) * LS + 2 * c16;
#pragma unroll
          for (int q = 0; q < kPieces; ++q) *reinterpret_cast<uint2*>(row + 16 * q) = pc[q];
        }
#pragma unroll
        for (int r = 0; r < BR; ++r) {
          uint2 pc[kPieces];
          split_pieces(pb[f][r], pc);
          float* row = Bs + 2 * ((tid >> 3) + r * (NTHR / 8)) * LS + 2 * c16;
#pragma unroll
          for (int q = 0; q < kPieces; ++q) {
            *reinterpret_cast<uint2*>(row + 16 * q) = pc[q];
            *reinterpret_cast<uint2*>(row + LS + 16 * q) = partner_pieces(pc[q]);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < AR; ++r)
          *reinterpret_cast<floatx4*>(As + ((tid >> 3) + r * (NTHR / 8)) * LS + 4 * c16) = pa[f][r];
#pragma unroll
        for (int r = 0; r < BR; ++r)
          *reinterpret_cast<floatx4*>(Bs + ((tid >> 3) + r * (NTHR / 8)) * LS + 4 * c16) = pb[f][r];
      }
      __syncthreads();
      if (st + PF < nst) fetch(pa[f], pb[f]);
      if constexpr (SPL) {
        floatx4 fa[MT][kPieces], fb[NT][kPieces];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int q = 0; q < kPieces; ++q)
            fa[m][q] = *reinterpret_cast<const floatx4*>(As + (wm * MT * T + T * m + li) * LS + 16 * q + 4 * lh);
#pragma unroll
        for (int c = 0; c < NT; ++c)
#pragma unroll
          for (int q = 0; q < kPieces; ++q)
            fb[c][q] = *reinterpret_cast<const floatx4*>(Bs + (wn * NT * T + T * c + li) * LS + 16 * q + 4 * lh);
        split_mma<MT, NT>(fa, fb, acc[0]);
      } else {
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          floatx4 fa[MT], fb[NT];
#pragma unroll
          for (int m = 0; m < MT; ++m)
            fa[m] = *reinterpret_cast<const floatx4*>(As + (wm * MT * T + T * m + li) * LS + JF * j + 4 * lh);
#pragma unroll
          for (int c = 0; c < NT; ++c)
            fb[c] = *reinterpret_cast<const floatx4*>(Bs + (wn * NT * T + T * c + li) * LS + JF * j + 4 * lh);
          block_mma<ST, false>(fa, fb, acc);
        }
      }
    }
  }
  __syncthreads();  // the operand tiles are dead; the LDS now stages the output tile
  float* tile = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        float* t = tile + (wm * MT * T + T * m + G::row_of(r, lh)) * LDT + CF * (wn * NT * T + T * c + li);
        if constexpr (C3) {
          const float t1 = acc[0][m][c][r], t2 = acc[1][m][c][r], t3 = acc[2][m][c][r];
          *reinterpret_cast<float2*>(t) = make_float2(t1 + t2, t3 - t1 + t2);
        } else {
          *t = acc[0][m][c][r];
        }
      }
  __syncthreads();
  constexpr int TF = CF * TN;  // output tile width in floats
  const int rbase = tm * TM, cbase = CF * tn * TN, ncolf = CF * a.N;
  for (int e = tid; e < TM * (TF / 4); e += NTHR) {
    const int rl = e / (TF / 4), cl = (e - rl * (TF / 4)) * 4;
    const int y = rbase + rl, col = cbase + cl;
    if (y >= a.M || col >= ncolf) continue;
    store_w_quad<storage_of(ST)>(a.W, tile + rl * LDT + cl, b, y, col, ncolf, a.M, a.nc, a.nt, a.P, p);
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

// Tile-shape tables: waves WM x WN per work-group, wave tile MT x NT MFMA
// tiles, depth.  kCompressLds / kExpandLds: LDS-staged FP32 (32 x 32 tiles
// of complex rows / columns, depth = k-tiles of register prefetch); the *16
// tables: LDS-staged 16-bit (16 x 16 tiles).  Index 0 is the default of its
// class.  The general forms (operands of 2 GiB or more) use one fixed shape.
struct Shape {
  int wm, wn, mt, nt, depth;
};
constexpr int kNumShapes = 8;
constexpr Shape kCompressLds[kNumShapes] = {{2, 2, 1, 1, 1}, {2, 1, 1, 1, 2}, {2, 1, 1, 1, 1}, {2, 1, 1, 2, 1},
                                            {4, 1, 1, 1, 1}, {2, 4, 1, 1, 1}, {1, 2, 1, 1, 1}, {1, 4, 1, 1, 1}};
constexpr Shape kExpandLds[kNumShapes] = {{1, 2, 1, 1, 1}, {1, 4, 1, 1, 1}, {1, 2, 1, 1, 2}, {2, 2, 1, 1, 1},
                                          {1, 1, 1, 1, 1}, {1, 2, 1, 2, 1}, {2, 1, 1, 1, 1}, {1, 4, 1, 1, 2}};
constexpr Shape kCompressLds16[kNumShapes] = {{4, 1, 2, 4, 1}, {2, 2, 4, 2, 1}, {2, 1, 4, 2, 1}, {4, 1, 2, 2, 1},
                                              {2, 1, 4, 4, 1}, {4, 2, 2, 2, 1}, {1, 4, 2, 2, 1}, {2, 2, 2, 2, 1}};
constexpr Shape kExpandLds16[kNumShapes] = {{2, 2, 2, 2, 1}, {1, 2, 2, 2, 1}, {1, 4, 2, 2, 1}, {2, 4, 2, 2, 1},
                                            {1, 4, 2, 4, 1}, {1, 2, 2, 4, 1}, {1, 4, 2, 2, 2}, {2, 2, 2, 4, 1}};
// BF16X6 (16 x 16 tiles of expanded rows / columns; the bank operand loads
// half the rows of its tile, so TM / 2 (compressing) or TN / 2 (expanding)
// rows must split evenly over the threads).  A k-tile is short work for the
// MFMA here (six 16 x 16 x 32 products per tile pair), so the loads run two
// to four k-tiles ahead.  Index 0 of each: measured best on the 224 x 224,
// 32-coil slice (with a split of 3 for the compressing one).
constexpr Shape kCompressSplit[kNumShapes] = {{4, 1, 2, 4, 2}, {4, 1, 2, 4, 3}, {4, 1, 2, 4, 4}, {2, 2, 2, 2, 3},
                                              {4, 2, 2, 2, 3}, {4, 1, 2, 2, 3}, {1, 2, 2, 2, 3}, {2, 2, 2, 2, 4}};
constexpr Shape kExpandSplit[kNumShapes] = {{2, 2, 2, 2, 2}, {2, 2, 2, 2, 3}, {2, 2, 2, 2, 4}, {1, 4, 2, 2, 3},
                                            {2, 4, 2, 2, 3}, {2, 2, 2, 4, 3}, {2, 2, 4, 2, 3}, {1, 2, 2, 2, 3}};
constexpr Shape kCompressGeneral = {4, 1, 2, 2, 3};
constexpr Shape kExpandGeneral = {1, 4, 2, 2, 3};

// Whether the LDS-staged and buffer-addressed forms apply.  The staged forms
// take k-tiles of one 128-byte line per row.
int staged_ktile(Store st) { return storage_of(st) == Store::F32 ? 32 : 64; }
size_t elem_bytes(Store st) { return storage_of(st) == Store::F32 ? 4 : 2; }
// Coils that the widest k-chunk of a split touches (the staged compressing
// form addresses the data operand from the first of them).
int chunk_coil_span(int KD, int kchunk, int ksplit, int twoP) {
  int span = 0;
  for (int ks = 0; ks < ksplit; ++ks) {
    const int kbeg = ks * kchunk, kend = std::min(KD, kbeg + kchunk);
    if (kend > kbeg) span = std::max(span, (kend - 1) / twoP - kbeg / twoP + 1);
  }
  return span;
}
bool compress_span_fits(size_t coil_elems, int span, size_t esz) { return (size_t)span * coil_elems * esz < kOOB; }
bool compress_staged(const CompressArgs& a, Store st) {
  const size_t esz = elem_bytes(st);
  const int span = chunk_coil_span(a.KD, a.kchunk, a.ksplit, 2 * a.P);
  // FP32 data take any P (odd P through the two-half data loads), 16-bit types 2P a multiple of 8
  return (esz == 4 || (2 * a.P) % (int)(16 / esz) == 0) && a.kchunk % staged_ktile(st) == 0 &&
         compress_span_fits((size_t)a.N * a.nt * 2, span, esz) && (size_t)a.M * a.KD * esz < kOOB;
}
// 2 kp is a multiple of 32, so KD (2 kp FP32, 4 kp 16-bit) is always a whole
// number of k-tiles; the staged form needs 32-bit buffer offsets.
bool expand_staged(const ExpandArgs& a, Store st) {
  const size_t esz = elem_bytes(st);
  return a.KD % staged_ktile(st) == 0 && (size_t)a.M * a.KD * esz < kOOB && (size_t)a.N * a.KDB * esz < kOOB;
}

int tiles(int n, int t) { return (n + t - 1) / t; }

template <int V, Store ST>
void launch_compress_v(StageScope& sc, hipStream_t s, const CompressArgs& a) {
  const int rest = a.B * a.np * a.ksplit;
  if (compress_staged(a, ST)) {
    constexpr Shape S = ST == Store::F32 ? kCompressLds[V] : ST == Store::BF16X6 ? kCompressSplit[V] : kCompressLds16[V];
    constexpr int T = Geo<ST>::T;
    CompressArgs c = a;
    if (ST == Store::F32) c.M = a.K;  // complex rows of the three-multiplication form
    const dim3 grid(tiles(c.N, S.wn * S.nt * T) * tiles(c.M, S.wm * S.mt * T) * rest);
    if constexpr (storage_of(ST) == Store::F32) {
      if (a.P & 1) {
        sc.launch(k_compress_lds<S.wm, S.wn, S.mt, S.nt, S.depth, ST, true>, grid, dim3(64 * S.wm * S.wn),
                           0, s, c);
        return;
      }
    }
    sc.launch(k_compress_lds<S.wm, S.wn, S.mt, S.nt, S.depth, ST, false>, grid, dim3(64 * S.wm * S.wn), 0,
                       s, c);
  } else {
    // operands of 2 GiB or more: BF16X6 takes the FP32 general form
    constexpr Shape S = kCompressGeneral;
    const dim3 grid(tiles(a.N, S.wn * S.nt * 16) * tiles(a.M, S.wm * S.mt * 16) * rest);
    sc.launch(k_compress<S.wm, S.wn, S.mt, S.nt, storage_of(ST)>, grid, dim3(64 * S.wm * S.wn), 0, s, a);
  }
}
template <int V, Store ST>
void launch_expand_v(StageScope& sc, hipStream_t s, const ExpandArgs& a) {
  const int rest = a.B * a.np;
  if (expand_staged(a, ST)) {
    constexpr Shape S = ST == Store::F32 ? kExpandLds[V] : ST == Store::BF16X6 ? kExpandSplit[V] : kExpandLds16[V];
    constexpr int T = Geo<ST>::T;
    ExpandArgs e = a;
    if (ST == Store::F32) e.N = a.N / 2;  // complex columns of the three-multiplication form
    const dim3 grid(tiles(e.N, S.wn * S.nt * T) * tiles(e.M, S.wm * S.mt * T) * rest);
    sc.launch(k_expand_lds<S.wm, S.wn, S.mt, S.nt, S.depth, ST>, grid, dim3(64 * S.wm * S.wn), 0, s, e);
  } else {
    constexpr Shape S = kExpandGeneral;
    const dim3 grid(tiles(a.N, S.wn * S.nt * 16) * tiles(a.M, S.wm * S.mt * 16) * rest);
    sc.launch(k_expand<S.wm, S.wn, S.mt, S.nt, storage_of(ST)>, grid, dim3(64 * S.wm * S.wn), 0, s, a);
  }
}

template <Store ST>
void compress_variant(int v, StageScope& sc, hipStream_t s, const CompressArgs& a) {
  switch (v) {
    case 0: launch_compress_v<0, ST>(sc, s, a); break;
    case 1: launch_compress_v<1, ST>(sc, s, a); break;
    case 2: launch_compress_v<2, ST>(sc, s, a); break;
    case 3: launch_compress_v<3, ST>(sc, s, a); break;
    case 4: launch_compress_v<4, ST>(sc, s, a); break;
    case 5: launch_compress_v<5, ST>(sc, s, a); break;
    case 6: launch_compress_v<6, ST>(sc, s, a); break;
    default: launch_compress_v<7, ST>(sc, s, a); break;
  }
}
template <Store ST>
void expand_variant(int v, StageScope& sc, hipStream_t s, const ExpandArgs& a) {
  switch (v) {
    case 0: launch_expand_v<0, ST>(sc, s, a); break;
    case 1: launch_expand_v<1, ST>(sc, s, a); break;
    case 2: launch_expand_v<2, ST>(sc, s, a); break;
    case 3: launch_expand_v<3, ST>(sc, s, a); break;
    case 4: launch_expand_v<4, ST>(sc, s, a); break;
    case 5: launch_expand_v<5, ST>(sc, s, a); break;
    case 6: launch_expand_v<6, ST>(sc, s, a); break;
    default: launch_expand_v<7, ST>(sc, s, a); break;
  }
}
static_assert(kNumShapes == 8, "the variant switches list every shape");

int bank16_index(const Plan& pl, Store st) {
  const int i = st == Store::BF16 ? 0 : 1;
  if (!pl.Aexp16[i] || !pl.AH16[i] || !pl.Zt16)
    return fail(GPJC_E_UNSUPPORTED, "16-bit contractions need patch_len divisible by 4");
  return i;
}

// The staged forms take k-tiles of 32 (FP32) or 64 (16-bit) elements.
int compress_kchunk(int KD, int ksplit, Store st) {
  const int kb = staged_ktile(st);
  return ((KD + ksplit - 1) / ksplit + kb - 1) / kb * kb;
}

int kblock(Store st) { return st == Store::F32 ? Geo<Store::F32>::KB : Geo<Store::BF16>::KB; }

int gemm_compress(const Plan& pl, StageScope& sc, Store st, const void* in, int ncol, float2* out, int ksplit,
                  int cvar) {
  CompressArgs a;
  if (storage_of(st) == Store::F32) {
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
  a.kchunk = compress_kchunk(a.KD, ksplit, st);
  a.split_stride = (size_t)pl.B * pl.np * pl.K * ncol;
  switch (st) {
    case Store::F32: compress_variant<Store::F32>(cvar, sc, pl.stream, a); break;
    case Store::BF16X6: compress_variant<Store::BF16X6>(cvar, sc, pl.stream, a); break;
    case Store::BF16: compress_variant<Store::BF16>(cvar, sc, pl.stream, a); break;
    default: compress_variant<Store::F16>(cvar, sc, pl.stream, a); break;
  }
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

}  // namespace

int gemm_compress_variants() { return kNumShapes; }
int gemm_expand_variants() { return kNumShapes; }

// Defaults: for the compressing contraction the work-group shape with the
// tallest row tile that pads at most 1/8 of its rows (FP32: 64 or 32 of the K
// complex rows; 16-bit and BF16X6: 128, 64 or 32 of the 2K real rows), else
// the shortest; for the expanding one shape 0; and a split giving about 504
// work-groups.
int compress_shape_for_rows(int rows, Store st) {
  const bool f32 = st == Store::F32;
  const int n = f32 ? 2 : 3;
  const int order16[3] = {0, 7, 6}, orderx6[3] = {0, 3, 6};
  const int* order = st == Store::BF16X6 ? orderx6 : order16;
  const int tile[3] = {f32 ? 64 : 128, f32 ? 32 : 64, 32};
  for (int i = 0; i < n; ++i) {
    const int padded = (rows + tile[i] - 1) / tile[i] * tile[i];
    if (8 * (padded - rows) <= padded) return order[i];
  }
  return order[n - 1];
}
void default_gemm_config(Plan& pl) {
  for (const Store st : {Store::F32, Store::BF16, Store::BF16X6}) {
    Plan::GemmCfg& g = pl.cfg(st);
    const int rows = st == Store::F32 ? pl.K : 2 * pl.K;  // complex rows in FP32, real rows otherwise
    g.cvar = compress_shape_for_rows(rows, st);
    g.evar = 0;
    const Shape S = st == Store::F32 ? kCompressLds[g.cvar] : st == Store::BF16X6 ? kCompressSplit[g.cvar]
                                                                                  : kCompressLds16[g.cvar];
    const int T = st == Store::F32 ? 32 : 16;
    const long t = (long)tiles(pl.ny, S.wn * S.nt * T) * tiles(rows, S.wm * S.mt * T) * pl.B * pl.np;
    // work-groups: measured best for E'^H E' on the 224 x 224, 32-coil slice
    // (the phase-encode stage reads one partial of Z per split)
    const long target = 504;
    int ks = (int)std::max<long>(1, (target + t - 1) / t);
    ks = std::min(std::min(ks, std::max(1, 2 * pl.ns / 128)), kMaxKsplit);
    // a split whose k-chunks the staged form can address (large volumes)
    while (ks < kMaxKsplit && !compress_split_staged(pl, st, ks)) ++ks;
    g.ksplit = ks;
  }
}

bool compress_split_staged(const Plan& pl, Store st, int ksplit) {
  return compress_span_fits((size_t)pl.ny * pl.nt * 2,
                            chunk_coil_span(2 * pl.ns, compress_kchunk(2 * pl.ns, ksplit, st), ksplit, 2 * pl.P),
                            elem_bytes(st));
}

int launch_group_compress(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_GROUP_COMPRESS, true);
  return gemm_compress(pl, sc, st, pl.W, pl.ny, pl.Zp, pl.cfg(st).ksplit, pl.cfg(st).cvar);
}

int launch_compress_data(const Plan& pl, const float2* ksp, float2* out) {
  StageScope sc(pl, GPJC_STAGE_GROUP_COMPRESS, true);
  return gemm_compress(pl, sc, Store::F32, ksp, pl.ms, out, 1, pl.cfg(Store::F32).cvar);
}

int launch_group_expand(const Plan& pl, Store st) {
  StageScope sc(pl, GPJC_STAGE_GROUP_EXPAND, true);
  ExpandArgs a;
  if (storage_of(st) == Store::F32) {
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
  a.KDB = 2 * pl.Kp;
  a.KD = storage_of(st) == Store::F32 ? 2 * pl.Kp : 4 * pl.Kp;
  a.kwrap = storage_of(st) == Store::F32 ? 0 : 2 * pl.Kp;
  a.nc = pl.nc;
  a.nt = pl.nt;
  a.P = pl.P;
  a.np = pl.np;
  a.B = pl.B;
  switch (st) {
    case Store::F32: expand_variant<Store::F32>(pl.cfg(st).evar, sc, pl.stream, a); break;
    case Store::BF16X6: expand_variant<Store::BF16X6>(pl.cfg(st).evar, sc, pl.stream, a); break;
    case Store::BF16: expand_variant<Store::BF16>(pl.cfg(st).evar, sc, pl.stream, a); break;
    default: expand_variant<Store::F16>(pl.cfg(st).evar, sc, pl.stream, a); break;
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
