// C ABI of libgpjc: argument validation, plan set-up and dispatch.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fft.h"
#include "fft2.h"
#include "plan.h"


namespace gpjc {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static bool debug_sync() {
  static const bool on = [] {
    const char* e = std::getenv("GPJC_DEBUG_SYNC");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

// Status of a queued call; with GPJC_DEBUG_SYNC set, also waits and reports
// errors raised by the kernels.
static int finish(const Plan& pl, int status) {
  if (status != GPJC_OK || !debug_sync()) return status;
  GPJC_HIP(hipStreamSynchronize(pl.stream));
  GPJC_HIP(hipGetLastError());
  return GPJC_OK;
}

template <class T>
static int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return GPJC_OK;
  GPJC_HIP(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
  return GPJC_OK;
}

static void free_plan(Plan* pl) {
  void* bufs[] = {pl->coils, pl->psf,  pl->psfp, pl->twin, pl->tw_x, pl->tw_y, pl->lines, pl->pgroup,
                  pl->maskf, pl->zeros, pl->A128, pl->Aexp, pl->AH,   pl->W,    pl->Zp,   pl->Zt,    pl->part,
                  pl->vx,    pl->vr,   pl->vp,   pl->vq,   pl->vb,   pl->vd,   pl->red,  pl->hist,  pl->flag,
                  pl->bmod,  pl->Ec,   pl->T3,   pl->pts3, pl->sel3, pl->maskf3, pl->tw_y3, pl->tw_z3};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int i = 0; i < 2; ++i) {
    if (pl->Aexp16[i]) (void)hipFree(pl->Aexp16[i]);
    if (pl->AH16[i]) (void)hipFree(pl->AH16[i]);
  }
  if (pl->Zt16) (void)hipFree(pl->Zt16);
  for (hipEvent_t e : pl->timing.ev) (void)hipEventDestroy(e);
  pl->timing.ev.clear();
}

static int validate_geom(const gpjc_geom* g) {
  if (!g) return fail(GPJC_E_INVAL, "geom is NULL");
  if (g->nx < 2 || g->ny < 2 || (g->nx & 1) || (g->ny & 1))
    return fail(GPJC_E_INVAL, "nx and ny must be even and >= 2");
  if (g->nc < 1) return fail(GPJC_E_INVAL, "nc must be >= 1");
  if (g->os < 1) return fail(GPJC_E_INVAL, "os must be >= 1");
  if (g->batch < 1) return fail(GPJC_E_INVAL, "batch must be >= 1");
  if (!g->mask) return fail(GPJC_E_INVAL, "mask is NULL");
  int ms = 0;
  for (int i = 0; i < g->ny; ++i) ms += g->mask[i] != 0;
  if (ms == 0) return fail(GPJC_E_INVAL, "mask selects no phase-encode line");
  if ((long)g->os * g->nx > (1L << 20) || (long)g->nc * g->ny * g->nx > (1L << 30))
    return fail(GPJC_E_INVAL, "os * nx or nc * ny * nx out of range");
  if (g->compressed) {
    const int nt = g->os * g->nx;
    if (g->patch_len < 1 || nt % g->patch_len)
      return fail(GPJC_E_INVAL, "patch_len must divide nt = os * nx");
    if (g->n_groups < 1) return fail(GPJC_E_INVAL, "n_groups must be >= 1");
    if (!g->patch_group) return fail(GPJC_E_INVAL, "patch_group is NULL");
    const long ns = (long)g->nc * g->patch_len;
    if (g->k < 1 || g->k > ns) return fail(GPJC_E_INVAL, "k must lie in [1, nc * patch_len]");
    const int np = nt / g->patch_len;
    std::vector<int> used(g->n_groups, 0);
    for (int p = 0; p < np; ++p) {
      const int v = g->patch_group[p];
      if (v < 0 || v >= g->n_groups) return fail(GPJC_E_INVAL, "patch_group value out of [0, n_groups)");
      used[v] = 1;
    }
    for (int v = 0; v < g->n_groups; ++v)
      if (!used[v]) return fail(GPJC_E_INVAL, "group " + std::to_string(v) + " has no patch");
  }
  return GPJC_OK;
}

static int check_supported(const gpjc_geom* g) {
  if (!fft_size_supported(g->nx) || !fft_size_supported(g->ny))
    return fail(GPJC_E_UNSUPPORTED, "nx / ny must be one of the built FFT lengths");
  return GPJC_OK;
}

static constexpr int kLdsSlots = 8192;  // float2 slots per work-group (64 KiB)

// Every kernel keeps its LDS within 64 KiB; shapes that cannot are rejected.
static int check_lds(const gpjc_geom* g) {
  const long line = 2L * g->os * fline(g->nx) + g->nx;  // one image row of the readout stages
  if (line > kLdsSlots) return fail(GPJC_E_UNSUPPORTED, "os * nx too large for the readout stages");
  if ((long)g->os * g->nx > 16 * 256) return fail(GPJC_E_UNSUPPORTED, "readout longer than 4096 samples");
  if (2L * fline(g->ny) + g->ny > kLdsSlots) return fail(GPJC_E_UNSUPPORTED, "ny too large for the phase-encode stages");
  return GPJC_OK;
}

static void choose_launch(Plan& pl) {
  const int lds_f2 = kLdsSlots;
  const int lsx = fline(pl.nx), lsy = fline(pl.ny);
  // readout forward: one image row per work-group once there are enough rows
  int rows = std::max(1, (lds_f2 - pl.nx) / (2 * pl.os * lsx));
  rows = std::min(rows, std::max(1, pl.ny * pl.nc * pl.B / 4096));
  pl.f1_rows = std::max(1, std::min(rows, pl.ny));
  // the two-pass register-FFT form where its work-group fits
  pl.f2_threads = 256;
  pl.f2_cb = two_pass_coils(pl.nx, pl.os, pl.nc, &pl.f2_threads);

  // readout adjoint: coils transformed together (up to 2, LDS permitting),
  // and enough coil chunks for about 2048 work-groups (each chunk leaves one
  // partial image)
  int cb = std::max(1, (lds_f2 - pl.nx) / (2 * pl.os * lsx));
  cb = std::min(std::min(cb, 2), pl.nc);
  int nchunk = (2048 + pl.ny * pl.B - 1) / (pl.ny * pl.B);
  nchunk = std::max(1, std::min(nchunk, (pl.nc + cb - 1) / cb));
  int cpc = (pl.nc + nchunk - 1) / nchunk;
  cpc = (cpc + cb - 1) / cb * cb;
  pl.f1h_cb = cb;
  pl.f1h_cpc = cpc;
  pl.f1h_nchunk = (pl.nc + cpc - 1) / cpc;
  // two-pass adjoint: one coil group (f2_cb coils) per work-group and partial image
  pl.f2_adj = pl.f2_cb > 0 && (long)pl.f2_cb * pl.os * std::max(split_n1(pl.nx), pl.nx / split_n1(pl.nx)) <= pl.f2_threads &&
              two_pass_lds_adj(pl.nx, pl.os, pl.f2_cb) * 8 <= 65536;
  if (pl.f2_adj) {
    pl.f1h_cpc = pl.f2_cb;
    pl.f1h_nchunk = (pl.nc + pl.f2_cb - 1) / pl.f2_cb;
  }

  const int lpb_max = std::max(1, std::min(32, (lds_f2 - pl.ny) / (2 * lsy)));
  const int nlines = pl.compressed ? pl.B * pl.np * pl.K : 1;
  pl.f3_lpb = std::max(1, std::min(lpb_max, nlines / 1024));
  pl.f3_tb = std::max(1, std::min(16, (lds_f2 - pl.ny) / (2 * lsy)));

  if (pl.compressed) default_gemm_config(pl);
  if (pl.general) {
    // the explicit adjoint leaves one partial image per chunk of rows (p, k);
    // the explicit forward writes Z whole, so the phase-encode stage reads one split
    pl.f1h_nchunk = explicit_chunks(pl.np * pl.K, pl.ny, pl.B);
    for (Plan::GemmCfg& g : pl.gemm) g.ksplit = 1;
  }
}

static int setup_plan(Plan& pl, const gpjc_geom* g, const gpjc_c64* d_coils, const gpjc_c64* d_psf,
                      const gpjc_c64* d_bmod, hipStream_t stream) {
  pl.general = d_bmod != nullptr;
  pl.nx = g->nx;
  pl.ny = g->ny;
  pl.nc = g->nc;
  pl.os = g->os;
  pl.nt = g->os * g->nx;
  pl.B = g->batch;
  pl.compressed = g->compressed ? 1 : 0;
  pl.stream = stream;
  pl.mask_h.assign(g->mask, g->mask + g->ny);
  for (int i = 0; i < g->ny; ++i)
    if (g->mask[i]) pl.lines_h.push_back(i);
  pl.ms = (int)pl.lines_h.size();
  if (pl.compressed) {
    pl.P = g->patch_len;
    pl.np = pl.nt / pl.P;
    pl.G = g->n_groups;
    pl.K = g->k;
    pl.Kp = (pl.K + 15) / 16 * 16;  // whole 32-element blocks of the 16-bit expanding contraction
    pl.ns = pl.nc * pl.P;
    pl.pgroup_h.assign(g->patch_group, g->patch_group + pl.np);
  }
  GPJC_HIP(hipGetDevice(&pl.device));
  choose_launch(pl);

  const size_t npix = (size_t)pl.ny * pl.nx;
  GPJC_TRY(dalloc(&pl.coils, (size_t)pl.nc * npix));
  GPJC_TRY(dalloc(&pl.psf, (size_t)pl.ny * pl.nt));
  GPJC_TRY(dalloc(&pl.psfp, (size_t)pl.ny * pl.nt));
  GPJC_TRY(dalloc(&pl.twin, (size_t)pl.os * pl.nx));
  GPJC_TRY(dalloc(&pl.tw_x, (size_t)pl.nx));
  GPJC_TRY(dalloc(&pl.tw_y, (size_t)pl.ny));
  GPJC_TRY(dalloc(&pl.lines, (size_t)pl.ms));
  GPJC_TRY(dalloc(&pl.maskf, (size_t)pl.ny));
  GPJC_TRY(dalloc(&pl.zeros, 64));
  GPJC_HIP(hipMemsetAsync(pl.zeros, 0, 64 * sizeof(float), stream));
  if (!pl.general) GPJC_TRY(dalloc(&pl.W, (size_t)pl.B * pl.nc * pl.ny * pl.nt));
  GPJC_TRY(dalloc(&pl.part, (size_t)pl.f1h_nchunk * pl.B * npix));
  const size_t ni = pl.img_elems();
  GPJC_TRY(dalloc(&pl.vx, ni));
  GPJC_TRY(dalloc(&pl.vr, ni));
  GPJC_TRY(dalloc(&pl.vp, ni));
  GPJC_TRY(dalloc(&pl.vq, ni));
  GPJC_TRY(dalloc(&pl.vb, ni));
  GPJC_TRY(dalloc(&pl.vd, pl.compressed ? (size_t)pl.B * pl.np * pl.K * pl.ms : (size_t)pl.B * pl.nc * pl.ms * pl.nt));
  GPJC_TRY(dalloc(&pl.red, 4096));
  pl.hist_cap = 100001;
  GPJC_TRY(dalloc(&pl.hist, (size_t)pl.hist_cap));
  GPJC_TRY(dalloc(&pl.flag, 4));
  if (pl.compressed) {
    GPJC_TRY(dalloc(&pl.pgroup, (size_t)pl.np));
    GPJC_TRY(dalloc(&pl.A128, (size_t)pl.G * pl.K * pl.ns));
    // 16 floats of tail: with Ns odd, a contraction chunk at the end of the
    // last row reads two floats past it (their data factor is zero)
    GPJC_TRY(dalloc(&pl.Aexp, (size_t)pl.G * 2 * pl.K * 2 * pl.ns + 16));
    GPJC_HIP(hipMemsetAsync(pl.Aexp + (size_t)pl.G * 2 * pl.K * 2 * pl.ns, 0, 16 * sizeof(float), stream));
    GPJC_TRY(dalloc(&pl.AH, (size_t)pl.G * 2 * pl.ns * 2 * pl.Kp));
    GPJC_TRY(dalloc(&pl.Zp, (size_t)kMaxKsplit * pl.B * pl.np * pl.K * pl.ny));
    GPJC_TRY(dalloc(&pl.Zt, (size_t)pl.B * pl.np * pl.ny * pl.Kp));
    GPJC_HIP(hipMemsetAsync(pl.Zt, 0, sizeof(float2) * (size_t)pl.B * pl.np * pl.ny * pl.Kp, stream));
    if (pl.general) {
      GPJC_TRY(dalloc(&pl.bmod, (size_t)pl.nt * npix));
      GPJC_TRY(dalloc(&pl.Ec, explicit_bytes(pl.nx, pl.ny, pl.np, pl.K) / sizeof(float2)));
    }
    if (pl.P % 4 == 0 && !pl.general) {  // 16-bit contractions: bank copies and a 16-bit Z^T (pads stay zero)
      for (int i = 0; i < 2; ++i) {
        GPJC_TRY(dalloc(&pl.Aexp16[i], (size_t)pl.G * 2 * pl.K * 2 * pl.ns));
        GPJC_TRY(dalloc(&pl.AH16[i], (size_t)pl.G * 2 * pl.ns * 2 * pl.Kp));
      }
      GPJC_TRY(dalloc(&pl.Zt16, (size_t)pl.B * pl.np * pl.ny * 2 * pl.Kp));
      GPJC_HIP(hipMemsetAsync(pl.Zt16, 0, sizeof(uint32_t) * (size_t)pl.B * pl.np * pl.ny * 2 * pl.Kp, stream));
    }
    GPJC_HIP(hipMemcpyAsync(pl.pgroup, pl.pgroup_h.data(), sizeof(int) * pl.np, hipMemcpyHostToDevice, stream));
  }
  std::vector<float> mf(pl.ny);
  for (int i = 0; i < pl.ny; ++i) mf[i] = pl.mask_h[i] ? 1.f : 0.f;
  GPJC_HIP(hipMemcpyAsync(pl.maskf, mf.data(), sizeof(float) * pl.ny, hipMemcpyHostToDevice, stream));
  GPJC_HIP(hipMemcpyAsync(pl.lines, pl.lines_h.data(), sizeof(int) * pl.ms, hipMemcpyHostToDevice, stream));
  GPJC_HIP(hipMemcpyAsync(pl.coils, d_coils, sizeof(float2) * pl.nc * npix, hipMemcpyDeviceToDevice, stream));
  if (pl.general) {
    // no readout PSF: a unit table keeps the shared set-up uniform
    const std::vector<float2> ones((size_t)pl.ny * pl.nt, make_float2(1.f, 0.f));
    GPJC_HIP(hipMemcpyAsync(pl.psf, ones.data(), sizeof(float2) * ones.size(), hipMemcpyHostToDevice, stream));
    GPJC_HIP(hipMemcpyAsync(pl.bmod, d_bmod, sizeof(float2) * (size_t)pl.nt * npix, hipMemcpyDeviceToDevice, stream));
    GPJC_HIP(hipStreamSynchronize(stream));  // `ones` is a host temporary
  } else {
    GPJC_HIP(hipMemcpyAsync(pl.psf, d_psf, sizeof(float2) * pl.ny * pl.nt, hipMemcpyDeviceToDevice, stream));
  }
  GPJC_TRY(launch_prep_tables(pl));
  GPJC_HIP(hipMemsetAsync(pl.hist, 0, sizeof(double) * pl.hist_cap, stream));

  if (pl.compressed && pl.G < pl.np && pl.P > 1 && pl.general) {
    // the same rule for a general map: member patches' map blocks agree
    const size_t blk = (size_t)pl.P * npix;
    std::vector<float2> h((size_t)pl.nt * npix);
    GPJC_HIP(hipMemcpyAsync(h.data(), pl.bmod, sizeof(float2) * h.size(), hipMemcpyDeviceToHost, stream));
    GPJC_HIP(hipStreamSynchronize(stream));
    std::vector<int> first(pl.G, -1);
    for (int p = 0; p < pl.np; ++p) {
      const int g0 = pl.pgroup_h[p];
      if (first[g0] < 0) {
        first[g0] = p;
        continue;
      }
      const float2* a = h.data() + (size_t)p * blk;
      const float2* b = h.data() + (size_t)first[g0] * blk;
      for (size_t i = 0; i < blk; ++i)
        if (std::hypot(a[i].x - b[i].x, a[i].y - b[i].y) > 1e-6)
          return fail(GPJC_E_INVAL, "patch " + std::to_string(p) + " does not share the modulation of group " +
                                        std::to_string(g0));
    }
  }
  if (pl.compressed && pl.G < pl.np && pl.P > 1 && !pl.general) {
    // One matrix per group is only valid if every member sees the same
    // modulation.  (With P = 1 a patch's channels differ from another's by one
    // unit phase per pixel, which cancels in Eq. 7: every grouping is legal.)
    std::vector<float2> h((size_t)pl.ny * pl.nt);
    GPJC_HIP(hipMemcpyAsync(h.data(), pl.psf, sizeof(float2) * h.size(), hipMemcpyDeviceToHost, stream));
    GPJC_HIP(hipStreamSynchronize(stream));
    std::vector<int> first(pl.G, -1);
    for (int p = 0; p < pl.np; ++p) {
      const int g0 = pl.pgroup_h[p];
      if (first[g0] < 0) {
        first[g0] = p;
        continue;
      }
      const int q = first[g0];
      for (int y = 0; y < pl.ny; ++y)
        for (int j = 0; j < pl.P; ++j) {
          const float2 a = h[(size_t)y * pl.nt + p * pl.P + j], b = h[(size_t)y * pl.nt + q * pl.P + j];
          if (std::hypot(a.x - b.x, a.y - b.y) > 1e-6)
            return fail(GPJC_E_INVAL, "patch " + std::to_string(p) + " does not share the modulation of group " +
                                          std::to_string(g0));
        }
    }
  }
  GPJC_HIP(hipStreamSynchronize(stream));
  return GPJC_OK;
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static int check_plan(const gpjc_plan* plan) {
  if (!plan) return fail(GPJC_E_INVAL, "plan is NULL");
  return GPJC_OK;
}

static bool known_prec(int prec) {
  return prec == GPJC_FP32 || prec == GPJC_BF16 || prec == GPJC_FP16 || prec == GPJC_BF16X6;
}
static Store store_of_prec(int prec) {
  return prec == GPJC_FP32 ? Store::F32 : prec == GPJC_BF16 ? Store::BF16 : prec == GPJC_FP16 ? Store::F16 : Store::BF16X6;
}

// BF16X6 is accepted by every plan: plans without group contractions (the
// uncompressed and modulation-map operators) run their FP32 path for it.
int check_prec(const Plan& pl, int prec, Store* st) {
  if (!known_prec(prec)) return fail(GPJC_E_INVAL, "unknown precision");
  const bool b16 = prec == GPJC_BF16 || prec == GPJC_FP16;
  if (b16 && !pl.compressed) return fail(GPJC_E_UNSUPPORTED, "the uncompressed operator is FP32 only");
  if (b16 && pl.general)
    return fail(GPJC_E_UNSUPPORTED, "the explicit readout model of a modulation-map plan is FP32 only");
  if (b16 && pl.P % 4) return fail(GPJC_E_UNSUPPORTED, "16-bit contractions need patch_len divisible by 4");
  *st = store_of_prec(prec);
  return GPJC_OK;
}

int check_bank(const Plan& pl) {
  if (pl.compressed && !pl.have_bank)
    return fail(GPJC_E_STATE, "no compression bank: call gpjc_calibrate or gpjc_set_compression first");
  return GPJC_OK;
}

}  // namespace gpjc

using namespace gpjc;

extern "C" {

int gpjc_plan_create(const gpjc_geom* geom, const gpjc_c64* d_coils, const gpjc_c64* d_psf, void* hip_stream,
                     gpjc_plan** out) {
  TraceRange trace("gpjc_plan_create");
  if (!out) return fail(GPJC_E_INVAL, "out is NULL");
  *out = nullptr;
  GPJC_TRY(validate_geom(geom));
  if (!d_coils || !d_psf) return fail(GPJC_E_INVAL, "coil maps or PSF is NULL");
  if (!aligned(d_coils, 8) || !aligned(d_psf, 8)) return fail(GPJC_E_INVAL, "coil maps / PSF not 8-byte aligned");
  GPJC_TRY(check_supported(geom));
  GPJC_TRY(check_lds(geom));
  gpjc_plan* pl = new (std::nothrow) gpjc_plan();
  if (!pl) return fail(GPJC_E_NOMEM, "host allocation failed");
  const int s = setup_plan(*pl, geom, d_coils, d_psf, nullptr, reinterpret_cast<hipStream_t>(hip_stream));
  if (s != GPJC_OK) {
    free_plan(pl);
    delete pl;
    return s;
  }
  *out = pl;
  return GPJC_OK;
}

int gpjc_plan_create_3d(const gpjc_geom* geom, int nz, const uint8_t* mask2, const gpjc_c64* d_coils,
                        const gpjc_c64* d_psf, void* hip_stream, gpjc_plan** out) {
  TraceRange trace("gpjc_plan_create_3d");
  if (!out) return fail(GPJC_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!geom) return fail(GPJC_E_INVAL, "geom is NULL");
  if (nz < 2) return fail(GPJC_E_INVAL, "nz must be >= 2 (use gpjc_plan_create for a 2D slice)");
  if (!mask2) return fail(GPJC_E_INVAL, "mask2 is NULL");
  if ((long)nz * geom->ny > 65535L * 16) return fail(GPJC_E_INVAL, "nz * ny out of range");
  if (!geom->compressed && ((long)geom->batch * geom->nc * nz > 65535 ||
                            (long)geom->batch * geom->nc * nz * geom->ny >= (1L << 31)))
    return fail(GPJC_E_UNSUPPORTED, "batch * nc * nz too large for the uncompressed volume operator");
  if (!fft_size_supported(geom->nx) || !fft_size_supported(geom->ny) || !fft_size_supported(nz))
    return fail(GPJC_E_UNSUPPORTED, "nx, ny and nz must be built FFT lengths");
  // the 2D machinery on (z, y) rows
  gpjc_geom g2 = *geom;
  g2.ny = nz * geom->ny;
  g2.mask = mask2;
  GPJC_TRY(validate_geom(&g2));
  if (!d_coils || !d_psf) return fail(GPJC_E_INVAL, "coil maps or PSF is NULL");
  if (!aligned(d_coils, 8) || !aligned(d_psf, 8)) return fail(GPJC_E_INVAL, "coil maps / PSF not 8-byte aligned");
  const long line = 2L * geom->os * fline(geom->nx) + geom->nx;
  if (line > kLdsSlots || (long)geom->os * geom->nx > 16 * 256)
    return fail(GPJC_E_UNSUPPORTED, "os * nx too large for the readout stages");
  gpjc_plan* pl = new (std::nothrow) gpjc_plan();
  if (!pl) return fail(GPJC_E_NOMEM, "host allocation failed");
  int s = setup_plan(*pl, &g2, d_coils, d_psf, nullptr, reinterpret_cast<hipStream_t>(hip_stream));
  if (s == GPJC_OK) {
    Plan& p = *pl;
    p.nz = nz;
    p.ny2 = geom->ny;
    if (p.compressed) s = dalloc(&p.T3, (size_t)p.B * p.np * p.K * p.ny);
    if (s == GPJC_OK) s = dalloc(&p.pts3, (size_t)p.ms);
    if (s == GPJC_OK) s = dalloc(&p.sel3, (size_t)p.ny);
    if (s == GPJC_OK) s = dalloc(&p.maskf3, (size_t)p.ny);
    if (s == GPJC_OK) s = dalloc(&p.tw_y3, (size_t)p.ny2);
    if (s == GPJC_OK) s = dalloc(&p.tw_z3, (size_t)nz);
    if (s == GPJC_OK) s = setup_pe3(p, mask2);
  }
  if (s != GPJC_OK) {
    free_plan(pl);
    delete pl;
    return s;
  }
  *out = pl;
  return GPJC_OK;
}

int gpjc_plan_create_bmap(const gpjc_geom* geom, const gpjc_c64* d_coils, const gpjc_c64* d_bmod, void* hip_stream,
                          gpjc_plan** out) {
  TraceRange trace("gpjc_plan_create_bmap");
  if (!out) return fail(GPJC_E_INVAL, "out is NULL");
  *out = nullptr;
  GPJC_TRY(validate_geom(geom));
  if (!geom->compressed) return fail(GPJC_E_INVAL, "a modulation-map plan must be compressed");
  if (!d_coils || !d_bmod) return fail(GPJC_E_INVAL, "coil maps or modulation map is NULL");
  if (!aligned(d_coils, 8) || !aligned(d_bmod, 8)) return fail(GPJC_E_INVAL, "coil maps / map not 8-byte aligned");
  if (geom->nx > 512) return fail(GPJC_E_UNSUPPORTED, "modulation-map plans: nx above 512");
  GPJC_TRY(check_supported(geom));
  GPJC_TRY(check_lds(geom));
  gpjc_plan* pl = new (std::nothrow) gpjc_plan();
  if (!pl) return fail(GPJC_E_NOMEM, "host allocation failed");
  const int s = setup_plan(*pl, geom, d_coils, nullptr, d_bmod, reinterpret_cast<hipStream_t>(hip_stream));
  if (s != GPJC_OK) {
    free_plan(pl);
    delete pl;
    return s;
  }
  *out = pl;
  return GPJC_OK;
}

int gpjc_plan_destroy(gpjc_plan* plan) {
  if (!plan) return GPJC_OK;
  (void)hipStreamSynchronize(plan->stream);
  free_plan(plan);
  delete plan;
  return GPJC_OK;
}

int gpjc_set_stream(gpjc_plan* plan, void* hip_stream) {
  GPJC_TRY(check_plan(plan));
  plan->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return GPJC_OK;
}

int gpjc_calibrate(gpjc_plan* plan, const uint8_t* d_roi, const gpjc_c64* d_noise_cov, double* h_eigvals,
                   gpjc_c128* d_A_out) {
  TraceRange trace("gpjc_calibrate");
  GPJC_TRY(check_plan(plan));
  if (!plan->compressed) return fail(GPJC_E_INVAL, "calibration needs a compressed plan");
  return finish(*plan, run_calibrate(*plan, d_roi, reinterpret_cast<const float2*>(d_noise_cov), h_eigvals,
                                     reinterpret_cast<double2*>(d_A_out)));
}

int gpjc_calibrate_static(gpjc_plan* plan, const uint8_t* d_roi, const gpjc_c64* d_noise_cov, double* h_eigvals,
                          gpjc_c128* d_A_out) {
  TraceRange trace("gpjc_calibrate_static");
  GPJC_TRY(check_plan(plan));
  if (!plan->compressed) return fail(GPJC_E_INVAL, "calibration needs a compressed plan");
  return finish(*plan, run_calibrate_static(*plan, d_roi, reinterpret_cast<const float2*>(d_noise_cov), h_eigvals,
                                            reinterpret_cast<double2*>(d_A_out)));
}

int gpjc_set_compression(gpjc_plan* plan, const gpjc_c128* d_A) {
  TraceRange trace("gpjc_set_compression");
  GPJC_TRY(check_plan(plan));
  if (!plan->compressed) return fail(GPJC_E_INVAL, "compression bank needs a compressed plan");
  if (!d_A || !aligned(d_A, 16)) return fail(GPJC_E_INVAL, "bank pointer NULL or not 16-byte aligned");
  GPJC_HIP(hipMemcpyAsync(plan->A128, d_A, sizeof(double2) * (size_t)plan->G * plan->K * plan->ns,
                          hipMemcpyDeviceToDevice, plan->stream));
  GPJC_TRY(launch_expand_bank(*plan));
  if (plan->general) GPJC_TRY(launch_build_explicit(*plan));
  plan->have_bank = true;
  return finish(*plan, GPJC_OK);
}

int gpjc_compress(const gpjc_plan* plan, const gpjc_c64* d_ksp, gpjc_c64* d_out) {
  TraceRange trace("gpjc_compress");
  GPJC_TRY(check_plan(plan));
  if (!plan->compressed) return fail(GPJC_E_INVAL, "gpjc_compress needs a compressed plan");
  if (!d_ksp || !d_out) return fail(GPJC_E_INVAL, "NULL buffer");
  if (!aligned(d_ksp, 16) || !aligned(d_out, 8)) return fail(GPJC_E_INVAL, "k-space must be 16-byte aligned");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, launch_compress_data(*plan, reinterpret_cast<const float2*>(d_ksp),
                                            reinterpret_cast<float2*>(d_out)));
}

int gpjc_forward(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_img, gpjc_c64* d_out) {
  TraceRange trace("gpjc_forward");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_img || !d_out || !aligned(d_img, 8) || !aligned(d_out, 8))
    return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, op_forward(*plan, st, reinterpret_cast<const float2*>(d_img), reinterpret_cast<float2*>(d_out)));
}

int gpjc_adjoint(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_in, gpjc_c64* d_img) {
  TraceRange trace("gpjc_adjoint");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_in || !d_img || !aligned(d_in, 8) || !aligned(d_img, 8))
    return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  GPJC_TRY(check_bank(*plan));
  GPJC_TRY(op_adjoint_part(*plan, st, reinterpret_cast<const float2*>(d_in)));
  return finish(*plan, launch_combine(*plan, reinterpret_cast<float2*>(d_img)));
}

int gpjc_normal(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_img, gpjc_c64* d_out) {
  TraceRange trace("gpjc_normal");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_img || !d_out || !aligned(d_img, 8) || !aligned(d_out, 8))
    return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  GPJC_TRY(check_bank(*plan));
  GPJC_TRY(op_normal_part(*plan, st, reinterpret_cast<const float2*>(d_img)));
  return finish(*plan, launch_combine(*plan, reinterpret_cast<float2*>(d_out)));
}

int gpjc_gd_step(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_x, const gpjc_c64* d_b,
                 const float* d_alpha, gpjc_c64* d_x_out, gpjc_c64* d_r_out) {
  TraceRange trace("gpjc_gd_step");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_x || !d_b || !d_alpha || !d_x_out) return fail(GPJC_E_INVAL, "NULL buffer");
  if (!aligned(d_x, 8) || !aligned(d_b, 8) || !aligned(d_x_out, 8) || !aligned(d_r_out, 8) || !aligned(d_alpha, 4))
    return fail(GPJC_E_INVAL, "misaligned buffer");
  if (d_x_out == d_x || d_x_out == d_b) return fail(GPJC_E_INVAL, "d_x_out must not alias d_x or d_b");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_gd_step(*plan, st, reinterpret_cast<const float2*>(d_x), reinterpret_cast<const float2*>(d_b),
                                   d_alpha, reinterpret_cast<float2*>(d_x_out), reinterpret_cast<float2*>(d_r_out)));
}

int gpjc_gd_step_backward(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_g, const float* d_alpha,
                          const gpjc_c64* d_r, gpjc_c64* d_gx_out, gpjc_c64* d_gb_out, float* d_galpha_out) {
  TraceRange trace("gpjc_gd_step_backward");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_g || !d_alpha || !d_r || !d_galpha_out) return fail(GPJC_E_INVAL, "NULL buffer");
  if (!aligned(d_g, 8) || !aligned(d_r, 8) || !aligned(d_gx_out, 8) || !aligned(d_gb_out, 8) ||
      !aligned(d_alpha, 4) || !aligned(d_galpha_out, 4))
    return fail(GPJC_E_INVAL, "misaligned buffer");
  if (d_gx_out && (d_gx_out == d_g || d_gx_out == d_r)) return fail(GPJC_E_INVAL, "d_gx_out must not alias inputs");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_gd_step_backward(*plan, st, reinterpret_cast<const float2*>(d_g), d_alpha,
                                            reinterpret_cast<const float2*>(d_r), reinterpret_cast<float2*>(d_gx_out),
                                            reinterpret_cast<float2*>(d_gb_out), d_galpha_out));
}

int gpjc_recon_cg(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters, int refine_every,
                  double* h_resid) {
  TraceRange trace("gpjc_recon_cg");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_y || !d_x || !aligned(d_y, 8) || !aligned(d_x, 8)) return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  if (iters < 0 || iters + 1 > plan->hist_cap) return fail(GPJC_E_INVAL, "iters out of range");
  if (refine_every < 0) return fail(GPJC_E_INVAL, "refine_every must be >= 0");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_cg(*plan, st, reinterpret_cast<const float2*>(d_y), reinterpret_cast<float2*>(d_x), iters,
                              refine_every, h_resid));
}

int gpjc_recon_fista(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters, double lambda,
                     double lipschitz, int haar_levels, double* h_obj) {
  TraceRange trace("gpjc_recon_fista");
  return gpjc_recon_fista_tv(plan, prec, d_y, d_x, iters, lambda, 0.0, 1.0, lipschitz, haar_levels, h_obj);
}

int gpjc_recon_fista_tv(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters, double lambda,
                        double lambda_tv, double tv_eps, double lipschitz, int haar_levels, double* h_obj) {
  TraceRange trace("gpjc_recon_fista_tv");
  if (!(lambda_tv >= 0.0) || !std::isfinite(lambda_tv)) return fail(GPJC_E_INVAL, "lambda_tv must be >= 0");
  if (!(tv_eps > 0.0) || !std::isfinite(tv_eps)) return fail(GPJC_E_INVAL, "tv_eps must be positive");
  if (plan && plan->nz > 1 && lambda_tv != 0.0)
    return fail(GPJC_E_UNSUPPORTED, "the total-variation term is built for 2D slices");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_y || !d_x || !aligned(d_y, 8) || !aligned(d_x, 8)) return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  if (iters < 0) return fail(GPJC_E_INVAL, "iters must be >= 0");
  if (!(lipschitz > 0.0) || !std::isfinite(lipschitz)) return fail(GPJC_E_INVAL, "lipschitz must be positive");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(GPJC_E_INVAL, "lambda must be >= 0");
  if (haar_levels < 1 || haar_levels > 3) return fail(GPJC_E_UNSUPPORTED, "haar_levels must be 1, 2 or 3");
  const int t = 1 << haar_levels;
  // 3D volumes: the 2D Haar transform of every z partition (tiles never cross one)
  const int rows_per_image = plan->nz > 1 ? plan->ny2 : plan->ny;
  if (plan->nx % t || rows_per_image % t) return fail(GPJC_E_INVAL, "nx and ny must be divisible by 2^haar_levels");
  if (h_obj && iters > plan->hist_cap) return fail(GPJC_E_INVAL, "iters too large for the objective history");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_fista(*plan, st, reinterpret_cast<const float2*>(d_y), reinterpret_cast<float2*>(d_x),
                                 iters, lambda, lambda_tv, tv_eps, lipschitz, haar_levels, h_obj));
}

int gpjc_recon_lsqr(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters,
                    double* h_resid) {
  TraceRange trace("gpjc_recon_lsqr");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!plan->compressed) return fail(GPJC_E_UNSUPPORTED, "algorithm #1 is built for compressed plans");
  if (!d_y || !d_x || !aligned(d_y, 8) || !aligned(d_x, 8)) return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  if (iters < 0 || iters + 1 > plan->hist_cap) return fail(GPJC_E_INVAL, "iters out of range");
  if (plan->nz > 1) return fail(GPJC_E_UNSUPPORTED, "algorithm #1 is built for 2D slices");
  if (!regular_accel(*plan))
    return fail(GPJC_E_UNSUPPORTED, "algorithm #1 needs a regular R-fold mask without calibration lines");
  if (4L * plan->B * plan->ms > 4096) return fail(GPJC_E_UNSUPPORTED, "more than 1024 aliased sets");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_lsqr(*plan, st, reinterpret_cast<const float2*>(d_y), reinterpret_cast<float2*>(d_x), iters,
                                h_resid));
}

int gpjc_power_iteration(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_x0, int iters, double* h_lambda) {
  TraceRange trace("gpjc_power_iteration");
  GPJC_TRY(check_plan(plan));
  Store st;
  GPJC_TRY(check_prec(*plan, prec, &st));
  if (!d_x0 || !aligned(d_x0, 8) || !h_lambda) return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  if (iters < 1) return fail(GPJC_E_INVAL, "iters must be >= 1");
  GPJC_TRY(check_bank(*plan));
  return finish(*plan, run_power_iteration(*plan, st, reinterpret_cast<const float2*>(d_x0), iters, h_lambda));
}

int gpjc_wavelet_absmax(gpjc_plan* plan, const gpjc_c64* d_img, int haar_levels, double* h_out) {
  TraceRange trace("gpjc_wavelet_absmax");
  GPJC_TRY(check_plan(plan));
  if (!d_img || !aligned(d_img, 8) || !h_out) return fail(GPJC_E_INVAL, "NULL or misaligned buffer");
  if (haar_levels < 1 || haar_levels > 3) return fail(GPJC_E_UNSUPPORTED, "haar_levels must be 1, 2 or 3");
  const int t = 1 << haar_levels;
  // 3D volumes: the 2D Haar transform of every z partition (tiles never cross one)
  const int rows_per_image = plan->nz > 1 ? plan->ny2 : plan->ny;
  if (plan->nx % t || rows_per_image % t) return fail(GPJC_E_INVAL, "nx and ny must be divisible by 2^haar_levels");
  return finish(*plan, run_wavelet_absmax(*plan, reinterpret_cast<const float2*>(d_img), haar_levels, h_out));
}

int gpjc_stage_timing(gpjc_plan* plan, int enable) {
  return gpjc_stage_timing_select(plan, enable ? (1u << GPJC_STAGE_COUNT) - 1u : 0u);
}

int gpjc_stage_timing_select(gpjc_plan* plan, unsigned stage_mask) {
  GPJC_TRY(check_plan(plan));
  if (stage_mask >> GPJC_STAGE_COUNT) return fail(GPJC_E_INVAL, "stage mask names an unknown stage");
  Timing& t = plan->timing;
  const bool enable = stage_mask != 0;
  if (enable) {
    if (t.ev.empty()) {
      const int cap = 16384;
      t.ev.resize(2 * cap);
      for (auto& e : t.ev) GPJC_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      t.stage.assign(cap, 0);
    }
    t.used = 0;
  }
  t.on = enable;
  t.mask = stage_mask;
  return GPJC_OK;
}

int gpjc_stage_times(gpjc_plan* plan, double* h_ms, int* h_launches) {
  GPJC_TRY(check_plan(plan));
  if (!h_ms || !h_launches) return fail(GPJC_E_INVAL, "NULL output");
  for (int i = 0; i < GPJC_STAGE_COUNT; ++i) {
    h_ms[i] = 0.0;
    h_launches[i] = 0;
  }
  Timing& t = plan->timing;
  if (t.used == 0) return GPJC_OK;
  GPJC_HIP(hipEventSynchronize(t.ev[2 * (t.used - 1) + 1]));
  for (int k = 0; k < t.used; ++k) {
    float ms = 0.f;
    GPJC_HIP(hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]));
    h_ms[t.stage[k]] += ms;
    h_launches[t.stage[k]] += 1;
  }
  return GPJC_OK;
}

int gpjc_set_gemm_config(gpjc_plan* plan, gpjc_prec prec, int compress_variant, int expand_variant, int ksplit) {
  GPJC_TRY(check_plan(plan));
  if (!plan->compressed) return fail(GPJC_E_INVAL, "GEMM configuration needs a compressed plan");
  if (plan->general) return fail(GPJC_E_UNSUPPORTED, "modulation-map plans have no group contraction to configure");
  if (!known_prec(prec)) return fail(GPJC_E_INVAL, "unknown precision");
  if (compress_variant < 0 || compress_variant >= gemm_compress_variants() || expand_variant < 0 ||
      expand_variant >= gemm_expand_variants())
    return fail(GPJC_E_INVAL, "unknown GEMM variant");
  if (ksplit < 1 || ksplit > kMaxKsplit) return fail(GPJC_E_INVAL, "ksplit out of range");
  Plan::GemmCfg& c = plan->cfg(store_of_prec(prec));
  c.cvar = compress_variant;
  c.evar = expand_variant;
  c.ksplit = ksplit;
  ++plan->config_gen;
  return GPJC_OK;
}

int gpjc_get_gemm_config(const gpjc_plan* plan, gpjc_prec prec, int* compress_variant, int* expand_variant,
                         int* ksplit, int* n_compress_variants, int* n_expand_variants) {
  GPJC_TRY(check_plan(plan));
  if (!known_prec(prec)) return fail(GPJC_E_INVAL, "unknown precision");
  const Plan::GemmCfg& c = plan->cfg(store_of_prec(prec));
  if (compress_variant) *compress_variant = c.cvar;
  if (expand_variant) *expand_variant = c.evar;
  if (ksplit) *ksplit = c.ksplit;
  if (n_compress_variants) *n_compress_variants = gemm_compress_variants();
  if (n_expand_variants) *n_expand_variants = gemm_expand_variants();
  return GPJC_OK;
}

const char* gpjc_status_string(int status) {
  switch (status) {
    case GPJC_OK: return "ok";
    case GPJC_E_INVAL: return "invalid argument";
    case GPJC_E_STATE: return "invalid state";
    case GPJC_E_NOMEM: return "out of device memory";
    case GPJC_E_DEVICE: return "HIP runtime error";
    case GPJC_E_UNSUPPORTED: return "unsupported";
    case GPJC_E_NUMERIC: return "numerical failure";
    default: return "unknown status";
  }
}

const char* gpjc_last_error(void) { return g_last_error.c_str(); }

const char* gpjc_runtime_path(void) {
  static std::string path;
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&hipGetDeviceCount), &info) && info.dli_fname) path = info.dli_fname;
  return path.c_str();
}

}  // extern "C"
