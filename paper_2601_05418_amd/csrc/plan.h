// Internal plan state and launcher prototypes shared by the HIP sources.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gpjc.h"

namespace gpjc {

// Status helper: records the message and returns the code.
int fail(int code, const std::string& msg);

#define GPJC_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::gpjc::fail(e_ == hipErrorOutOfMemory ? GPJC_E_NOMEM : GPJC_E_DEVICE, \
                          std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define GPJC_TRY(expr)        \
  do {                        \
    int s_ = (expr);          \
    if (s_ != GPJC_OK) return s_; \
  } while (0)

// Arithmetic of a precision: FP32, the 16-bit storage types, and BF16X6 (FP32
// storage everywhere; the group contractions run on the BF16 MFMA with every
// FP32 operand split into three BF16 pieces).
enum class Store { F32 = 0, BF16 = 1, F16 = 2, BF16X6 = 3 };
// The type hybrid data, Z and the phase-encode stage are stored in.
constexpr Store storage_of(Store st) { return st == Store::BF16X6 ? Store::F32 : st; }
// Whether a precision stores 16-bit values (and so takes FP32 refinement in CG).
constexpr bool is_16bit(Store st) { return st == Store::BF16 || st == Store::F16; }

// HIP-event timing of stage launches (enabled on request).
struct Timing {
  bool on = false;
  unsigned mask = 0;  // bit s set: stage s is timed
  int used = 0;
  std::vector<hipEvent_t> ev;  // 2 per launch
  std::vector<int> stage;
};

struct Plan {
  // geometry
  int nx = 0, ny = 0, nc = 0, os = 0, nt = 0, P = 0, np = 0, G = 0, K = 0, Kp = 0, ns = 0, ms = 0;
  int B = 1, compressed = 1;
  std::vector<int> pgroup_h;
  std::vector<uint8_t> mask_h;
  std::vector<int> lines_h;
  hipStream_t stream = nullptr;
  int device = 0;

  // launch configuration
  int f1_rows = 1;          // image rows per readout-forward workgroup
  int f2_cb = 0;            // coils per work-group of the two-pass readout forward (0 = Stockham form)
  int f2_threads = 256;     // threads per work-group of the two-pass readout forms
  bool f2_adj = false;      // the adjoint uses the two-pass form too (one coil group per work-group)
  int f1h_cb = 1;           // coils transformed together in the readout adjoint
  int f1h_nchunk = 1;       // coil chunks (partial images) in the readout adjoint
  int f1h_cpc = 1;          // coils per chunk
  int f3_lpb = 1;           // phase-encode lines per workgroup
  int f3_tb = 1;            // readout columns per uncompressed phase-encode workgroup
  // group-contraction configuration per precision class ([0] FP32, [1] BF16 / FP16,
  // [2] BF16X6): tile shape of the compressing and expanding contractions, split of
  // the compressing one (the phase-encode stage sums that many partials of Z)
  struct GemmCfg {
    int cvar = 0, evar = 0, ksplit = 1;
  };
  GemmCfg gemm[3];
  static int cfg_index(Store st) { return st == Store::F32 ? 0 : st == Store::BF16X6 ? 2 : 1; }
  const GemmCfg& cfg(Store st) const { return gemm[cfg_index(st)]; }
  GemmCfg& cfg(Store st) { return gemm[cfg_index(st)]; }
  long config_gen = 0;      // bumped whenever the launch configuration changes

  // 3D volumes (gpjc_plan_create_3d): rows are (z, y) pairs, ny = nz * ny2;
  // the phase-encode stage is the 2D DFT over (z, y) with a 2D mask
  int nz = 1, ny2 = 0;
  float2* T3 = nullptr;     // [B][np][K][nz][ny2] planes between the 2D-DFT passes (compressed plans)
  int* pts3 = nullptr;      // [ms] row (kz * ny2 + ky) of each acquired point
  int* sel3 = nullptr;      // [ny] acquired-point index of every row, or -1
  float* maskf3 = nullptr;  // [ny] 0 / 1
  float2* tw_y3 = nullptr;  // [ny2] exp(-2 pi i m / ny2)
  float2* tw_z3 = nullptr;  // [nz]

  // general modulation map (plans from gpjc_plan_create_bmap): no readout PSF;
  // the compressed readout matrices are stored per phase-encode column
  bool general = false;
  float2* bmod = nullptr;   // [nt][ny][nx] exp(-i k_m(t, x, y))
  float2* Ec = nullptr;     // [ny][np][K][nx] E'_y, rebuilt with every bank

  // device: geometry tables
  float2* coils = nullptr;  // [nc][ny][nx]
  float2* psf = nullptr;    // [ny][nt] as given
  float2* psfp = nullptr;   // [ny][nt] psf times the readout post-twiddle
  float2* twin = nullptr;   // [os][nx] readout pre-twiddle
  float2* tw_x = nullptr;   // [nx] exp(-2 pi i m / nx)
  float2* tw_y = nullptr;   // [ny]
  int* lines = nullptr;     // [ms]
  int* pgroup = nullptr;    // [np]
  float* maskf = nullptr;   // [ny] 0 / 1
  float* zeros = nullptr;   // [64] zero-filled; source of masked-out loads

  // device: compression bank
  bool have_bank = false;
  double2* A128 = nullptr;  // [G][K][ns]
  float* Aexp = nullptr;    // [G][2K][2ns]   real form for compressing
  float* AH = nullptr;      // [G][2ns][2Kp]  real form for expanding
  // 16-bit copies of Aexp / AH, index 0 = BF16, 1 = FP16 (same layouts)
  uint16_t* Aexp16[2] = {nullptr, nullptr};
  uint16_t* AH16[2] = {nullptr, nullptr};

  // device: workspaces
  float2* W = nullptr;      // [B][nc][ny][nt] (also holds 16-bit W)
  float2* Zp = nullptr;     // [ksplit][B][np][K][ny]
  float2* Zt = nullptr;     // [B][np][ny][Kp]
  uint32_t* Zt16 = nullptr; // [B][np][ny][2 Kp] 16-bit (re, im) pairs, hi then lo, for the 16-bit contractions
  float2* part = nullptr;   // [f1h_nchunk][B][ny][nx]

  // device: solver state
  float2 *vx = nullptr, *vr = nullptr, *vp = nullptr, *vq = nullptr, *vb = nullptr;
  float2* vd = nullptr;     // one data vector (gpjc_forward's output layout): FISTA objective
  double* red = nullptr;    // reduction partials
  double* hist = nullptr;   // [hist_cap]
  int* flag = nullptr;      // numeric status flag
  int hist_cap = 0;
  int red_blocks = 0;

  mutable Timing timing;

  size_t img_elems() const { return (size_t)B * ny * nx; }
};

// Times one stage launch while timing is on.  A stage of one kernel launches
// it through launch(), which hands the event pair to the kernel's own
// dispatch (hipExtLaunchKernel records them at the kernel's start and end,
// with no marker packets around it); a stage of several kernels is bracketed
// by event records before and after.
struct StageScope {
  const Plan& pl;
  int slot = -1;
  bool single = false, consumed = false;
  StageScope(const Plan& p, int st, bool one_kernel = false) : pl(p), single(one_kernel) {
    Timing& t = p.timing;
    if (t.on && ((t.mask >> st) & 1u) && t.used < (int)t.stage.size()) {
      slot = t.used++;
      t.stage[slot] = st;
      if (!single) (void)hipEventRecord(t.ev[2 * slot], p.stream);
    }
  }
  template <typename F, typename... A>
  void launch(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, A... args) {
    if (slot >= 0 && single && !consumed) {
      hipExtLaunchKernelGGL(kernel, grid, block, lds, s, pl.timing.ev[2 * slot], pl.timing.ev[2 * slot + 1], 0,
                            args...);
      consumed = true;
    } else {
      kernel<<<grid, block, lds, s>>>(args...);
    }
  }
  ~StageScope() {
    if (slot < 0) return;
    if (single && !consumed) (void)hipEventRecord(pl.timing.ev[2 * slot], pl.stream);
    if (!single || !consumed) (void)hipEventRecord(pl.timing.ev[2 * slot + 1], pl.stream);
  }
};

// A named range around one library call, for tracing tools (rocprofv3
// --marker-trace shows it; without a tool attached it costs a function call).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Argument checks shared by the entry points (api.hip).
int check_prec(const Plan& pl, int prec, Store* st);
int check_bank(const Plan& pl);

// ---- operator stages (operator.hip) ----
int launch_prep_tables(Plan& pl);
int launch_readout_fwd(const Plan& pl, const float2* img, Store st);
int launch_readout_adj(const Plan& pl, Store st);
int launch_combine(const Plan& pl, float2* out);
int launch_group_compress(const Plan& pl, Store st);
int launch_group_expand(const Plan& pl, Store st);
int launch_pe_fwd(const Plan& pl, float2* out, Store st);
int launch_pe_adj(const Plan& pl, const float2* in, Store st);
int launch_pe_normal(const Plan& pl, Store st);
int launch_pe_cols_fwd(const Plan& pl, float2* out);
int launch_pe_cols_adj(const Plan& pl, const float2* in);
int launch_pe_cols_normal(const Plan& pl);
// volumes: one pass over W in place; 0 / 1 y forward / inverse, 2 / 3 z forward / inverse, 4 z normal
int launch_pe3_cols_pass(const Plan& pl, int pass);
int launch_expand_bank(Plan& pl);
// Whether the staged compressing forms can address the readout-stage output
// of a plan with this split (else it runs on the general form).
bool compress_split_staged(const Plan& pl, Store st, int ksplit);
// Tile shapes built per precision class, and the default configuration of a plan.
int gemm_compress_variants();
int gemm_expand_variants();
constexpr int kMaxKsplit = 8;
void default_gemm_config(Plan& pl);
int launch_compress_data(const Plan& pl, const float2* ksp, float2* out);

// Whole operators: images in, images (as partial sums in pl.part) or data out.
int op_forward(const Plan& pl, Store st, const float2* img, float2* out);
int op_adjoint_part(const Plan& pl, Store st, const float2* in);  // result in pl.part
int op_normal_part(const Plan& pl, Store st, const float2* img);  // result in pl.part
// The column stages alone (compressed plans): readout model and group
// contraction per image column, without the phase-encode DFT.
int op_fwd_columns(const Plan& pl, Store st, const float2* img);  // img -> Zp (split partials)
int op_adj_columns(const Plan& pl, Store st);                      // Z^T -> pl.part

// ---- reconstruction algorithm #1 (hybrid.hip) ----
int regular_accel(const Plan& pl);  // R of a regular mask without calibration lines, else 0
int run_lsqr(Plan& pl, Store st, const float2* y, float2* x, int iters, double* h_resid);

// ---- Hermitian eigensolver of the calibration (eigen.hip) ----
// Workspaces of tri_eigen for G matrices of size n and K wanted vectors.
struct TriEigBufs {
  double *d, *tau, *f, *f2, *eig, *bounds;  // [G][n] each (bounds [G][3]); eig: every eigenvalue, descending
  double2 *e, *vb, *wb, *pb, *cb, *ph, *pd; // [G][n] each (vb [2][G][n])
  double2* pt;                              // [G][ceil(n / 16)][n]
  double *lm, *u0, *u1, *u2, *x;            // [G][n][K] each
  unsigned char* sw;                        // [G][n][K]
  double2* U;                               // [G][K][n]: eigenvectors of the K largest eigenvalues
};
// Eigenvalues and the K leading eigenvectors of G Hermitian n x n matrices
// (H: [G][ld][ld], overwritten).  *flag is set when an eigenvector fails its
// residual check.  n <= 2048.
int tri_eigen(hipStream_t st, double2* H, int ld, int n, int G, int K, const TriEigBufs& b, int* flag);

// ---- calibration (calib.hip) ----
int run_calibrate(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out);
// The same calibration with its workspaces in the library's static device
// scratch (kStaticScratchBytes per GPU): no device allocation.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
int run_calibrate_static(Plan& pl, const uint8_t* roi, const float2* noise_cov, double* h_eig, double2* A_out);

// ---- solvers (solver.hip) ----
int run_cg(Plan& pl, Store st, const float2* y, float2* x, int iters, int refine_every, double* h_resid);
// CG in parts (a batch captures one iteration once and replays it):
int cg_setup(Plan& pl, Store st, bool refine, const float2* y, const float2* x0);
int cg_iteration(const Plan& pl, Store st, bool refresh);
int cg_finish(const Plan& pl, float2* x, int iters, double* h_resid, int* h_flag);
bool cg_refresh_at(int it, int iters, int refine_every, Store st);
// The operator part of an iteration: A p (phase 0) or the refresh's FP32 A x
// (phase 1), leaving partial images in pl.part.
int cg_op_part(const Plan& pl, Store st, int phase);
// One slice's CG vectors for the batch's work-list kernels.
struct CgSlice {
  const float2* part;
  const float2* b;
  float2 *x, *r, *p, *q;
  double* red;   // [pq partials][two rr slots]
  int* flag;     // numeric flag; flag[1] is the iteration count
  double* hist;
  size_t n;
  int nchunk;
};
CgSlice cg_slice_of(const Plan& pl);
// Work-list steps over every slice of a batch (same arithmetic and order as
// the per-plan kernels): after phase 0, Q then UPDATE, then DIR; a refresh
// iteration runs phase 1 after UPDATE, then START and NORM.
enum CgListOp { kCgListQ = 0, kCgListUpdate = 1, kCgListDir = 2, kCgListStart = 3, kCgListNorm = 4 };
int launch_cg_list(const CgSlice* d_list, int nslice, int op, int grid, hipStream_t s);

// ---- GEMM tile autotuning (tune.hip) ----
int autotune(Plan& pl, Store st, const char* cache_path, int* h_choice);
int run_fista(Plan& pl, Store st, const float2* y, float2* x, int iters, double lambda, double lam_tv, double eps,
              double lip, int levels, double* h_obj);

int run_power_iteration(Plan& pl, Store st, const float2* x0, int iters, double* h_lambda);
int run_gd_step(const Plan& pl, Store st, const float2* x, const float2* b, const float* alpha, float2* x_out,
                float2* r_out);
int run_gd_step_backward(const Plan& pl, Store st, const float2* g, const float* alpha, const float2* r, float2* gx,
                         float2* gb, float* galpha);
int run_wavelet_absmax(Plan& pl, const float2* img, int levels, double* h_out);

// ---- phase-encode stage of 3D volumes (pe3d.hip) ----
int launch_pe3_fwd(const Plan& pl, float2* out, Store st);
int launch_pe3_adj(const Plan& pl, const float2* in, Store st);
int launch_pe3_normal(const Plan& pl, Store st);
// the same stage on the uncompressed W [B][nc][nz ny2][nt], in place
int launch_pe3_cols_fwd(const Plan& pl, float2* out);
int launch_pe3_cols_adj(const Plan& pl, const float2* in);
int launch_pe3_cols_normal(const Plan& pl);
int setup_pe3(Plan& pl, const uint8_t* mask2);

// ---- explicit readout model for general modulation maps (explicit.hip) ----
int launch_build_explicit(const Plan& pl);
int launch_explicit_fwd(const Plan& pl, const float2* img);  // img -> Zp (split 0)
int launch_explicit_adj(const Plan& pl);                      // Zt -> part
int explicit_chunks(int rows, int ny, int B);
size_t explicit_bytes(int nx, int ny, int np, int K);

// Sizing of the two-pass readout forms (operator.hip).
size_t two_pass_lds_fwd(int nx, int os, int cb);
size_t two_pass_lds_adj(int nx, int os, int cb);
int two_pass_coils(int nx, int os, int nc, int* threads);

// Lengths the FFT kernels are instantiated for.
bool fft_size_supported(int n);

}  // namespace gpjc

// The opaque handle of the C ABI is the plan itself.
struct gpjc_plan : gpjc::Plan {};
