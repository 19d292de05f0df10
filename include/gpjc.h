/*
 * libgpjc -- group-patch joint compression of B0- and RF-modulated k-space
 * and the compressed Wave encoding operator, for AMD Instinct MI355X
 * (gfx950).
 *
 * The method: arXiv 2601.05418, Section 2.4 (Eqs. 6-15).  A readout line of
 * Nt = os * nx samples is cut into patches of P consecutive samples; patch p
 * belongs to group g(p).  For each group the Nc * P products of coil map,
 * modulation phase and readout DFT row (Eq. 6) form "virtual channels"; the
 * top-K eigenvectors of their normalised Gram matrix P_g (Eqs. 7-11) give the
 * compression matrix A_g (Eqs. 8, 12), applied to every patch of the group
 * (Eqs. 13, 14) to form the reduced model S' = E' rho (Eq. 15).
 * Reconstruction solves Eq. 16 (least squares, here by CG on the normal
 * equations) or Eq. 17 with the wavelet term (FISTA), Section 3.4.
 *
 * Operator conventions (the paper leaves FFT centring and scaling open; this
 * library uses centred unitary DFTs):
 *   W[n][y][t]  = psf[y][t] * sum_x F_Nt[t][x + (Nt-Nx)/2] coils[n][y][x] img[y][x]
 *   Z[p][k][y]  = sum_{n,j} A[g(p)][k][n][j] W[n][y][p*P + j]
 *   S'[p][k][m] = sum_y F_Ny[line_m][y] Z[p][k][y]
 * with F_N[k][i] = exp(-2 pi i (k - N/2)(i - N/2) / N) / sqrt(N) and line_m
 * the m-th set entry of the phase-encode mask (ascending).  The uncompressed
 * operator (geom.compressed = 0) skips Z: S[n][m][t] = sum_y F_Ny[line_m][y] W[n][y][t].
 *
 * Memory: every d_* argument is a device pointer, every h_* argument a host
 * pointer.  The caller owns all buffers passed in; they must stay valid until
 * the work queued on the plan's stream has completed.  Complex data are
 * interleaved (re, im) and 8-byte (c64) / 16-byte (c128) aligned; buffers
 * read with vector loads (gpjc_compress input) must be 16-byte aligned.
 * The plan owns its copies of coil maps and PSF, the compression bank and all
 * workspaces; they are allocated by gpjc_plan_create / gpjc_calibrate /
 * gpjc_set_compression and freed by gpjc_plan_destroy.  gpjc_forward,
 * gpjc_adjoint, gpjc_normal and the recon calls allocate nothing.
 *
 * Errors: every call returns GPJC_OK (0) or a negative status.  Arguments are
 * validated before anything is launched, so a failing call leaves its outputs
 * untouched (except GPJC_E_DEVICE / GPJC_E_NUMERIC raised after launch).
 * gpjc_last_error() returns a thread-local message for the last failure.
 * Calls are asynchronous on the plan's stream unless they return host data
 * (h_* outputs), which synchronise.  A plan is used by one thread at a time.
 */
#ifndef GPJC_H
#define GPJC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } gpjc_c64;
typedef struct { double re, im; } gpjc_c128;

/* Arithmetic of the group contraction and PSF product inside the operator.
 * FP32: everything FP32 (FP32 MFMA; the group contractions form each complex
 * product from three real products).  BF16 / FP16 (compressed plans with
 * patch_len % 4 == 0, else GPJC_E_UNSUPPORTED): the operands of both group
 * contractions are rounded to BF16 / FP16 (round to nearest even) and
 * contracted on MFMA with FP32 accumulation -- the compression matrices and
 * the hybrid data W after the PSF product (forward) and after the expanding
 * contraction (adjoint).  The phase-encode output Z^T feeding the expanding
 * contraction is carried as a hi + lo pair of 16-bit values (hi = rn(z),
 * lo = rn(z - hi)), so it adds almost no rounding of its own.  FFTs, coil
 * products and the phase-encode stage compute in FP32.  FP16 needs every stored value below 65504 in magnitude
 * (non-finite results surface as GPJC_E_NUMERIC in the solvers).
 * BF16X6: FP32 storage and FP32 accuracy, with both group contractions on the
 * BF16 MFMA: every FP32 operand is split into three BF16 pieces (each the
 * nearest-even BF16 of what the earlier pieces leave) and the six piece
 * products whose orders sum to at most two are accumulated in FP32; what it
 * drops is below 2^-26 of each product.  Any patch_len; plans without group
 * contractions (uncompressed, modulation-map) run their FP32 path for it.
 * Section 2.4, Eqs. 13-14, for the contractions themselves. */
typedef enum { GPJC_FP32 = 0, GPJC_BF16 = 1, GPJC_FP16 = 2, GPJC_BF16X6 = 3 } gpjc_prec;

enum {
  GPJC_OK = 0,
  GPJC_E_INVAL = -1,       /* bad argument, geometry or group partition */
  GPJC_E_STATE = -2,       /* compressed operator used before a bank exists */
  GPJC_E_NOMEM = -3,       /* device allocation failed */
  GPJC_E_DEVICE = -4,      /* HIP runtime error (message in gpjc_last_error) */
  GPJC_E_UNSUPPORTED = -5, /* size or mode this build does not provide */
  GPJC_E_NUMERIC = -6      /* NaN/Inf in a solver, or eigensolver did not converge */
};

/* Geometry of a plan (Section 2.3, Fig. 3A; Section 3.3).  The host arrays
 * are copied at plan creation. */
typedef struct {
  int32_t nx, ny;              /* image matrix, readout x fastest; both even */
  int32_t nc;                  /* receive coils */
  int32_t os;                  /* readout oversampling; nt = os * nx */
  int32_t patch_len;           /* P; nt % P == 0 */
  int32_t n_groups;            /* G */
  const int32_t* patch_group;  /* host [nt / P], values in [0, G), every group used */
  int32_t k;                   /* kept rank per group, 1 <= K <= nc * P */
  const uint8_t* mask;         /* host [ny], nonzero = phase-encode line acquired */
  int32_t batch;               /* B images sharing the geometry and maps */
  int32_t compressed;          /* 1 = E' (Eq. 15), 0 = uncompressed E (Eq. 4) */
} gpjc_geom;

typedef struct gpjc_plan gpjc_plan;

/* Create a plan.  d_coils [nc][ny][nx] c64 (E_RF of Eq. 6), d_psf [ny][nt]
 * c64 = exp(-i k_m(t, y)) (E_NG of Eq. 6, Eqs. 1 and 3 for Wave), both
 * copied.  hip_stream: a hipStream_t (NULL = default stream).  Checks that
 * every group's member patches see identical PSF columns (max abs difference
 * <= 1e-6), the condition under which one matrix serves all of them
 * (Section 2.3); GPJC_E_INVAL otherwise.  Synchronises. */
int gpjc_plan_create(const gpjc_geom* geom, const gpjc_c64* d_coils, const gpjc_c64* d_psf,
                     void* hip_stream, gpjc_plan** out);
/* Create a plan for a 3D volume with two phase-encode dimensions (Section
 * 3.4: both are reconstructed by FFT; Table S2, Figs. 8-9): geom->ny is the
 * in-plane phase-encode size, nz the second; images are [B][nz][ny][nx],
 * d_coils [nc][nz][ny][nx], d_psf [nz][ny][nt] (e.g. the Wave-CAIPI corkscrew
 * exp(-i k_m(t, y, z))), mask2 host [nz][ny] (nonzero = (kz, ky) acquired;
 * geom->mask is ignored).  The readout stage, group contraction and
 * calibration act on the nz * ny rows (z, y) as on the rows of a slice; the
 * phase-encode stage is the centred unitary 2D DFT over (z, y), and data
 * (gpjc_forward's output, gpjc_compress's input lines) list the acquired
 * points in raster order (kz major, ky fastest): Ms = number of them.
 * geom->compressed = 0 gives the uncompressed E (data [B][nc][Ms][nt]), whose
 * phase-encode stage takes the 2D DFT of every (coil, readout sample) plane
 * of the readout-stage output in place; it needs batch * nc * nz <= 65535
 * (GPJC_E_UNSUPPORTED otherwise).  nx, ny, nz built FFT lengths.  CG, FISTA
 * with the Haar term (2D Haar of every z partition), batching, autotuning and
 * the 16-bit precisions work as for slices; algorithm #1 and the TV term are
 * built for slices (GPJC_E_UNSUPPORTED).  Synchronises. */
int gpjc_plan_create_3d(const gpjc_geom* geom, int nz, const uint8_t* mask2, const gpjc_c64* d_coils,
                        const gpjc_c64* d_psf, void* hip_stream, gpjc_plan** out);

/* Create a plan for a general modulation map (Section 3.1: nonlinear B0
 * fields such as a local B0 coil array; Eqs. 1-3), d_bmod [nt][ny][nx] c64 =
 * exp(-i k_m(t, x, y)), which need not factor into a readout PSF.  The
 * phase-encode dimension stays Fourier (the modulation repeats on every
 * phase-encode step, Section 2.3), and each image column y has the dense
 * readout model E_y[(n, t)][x] = c_n(x, y) exp(-i k_m(t, x, y)) F_Nt[t][x].
 * Compressed plans only (geom->compressed = 1), FP32 only.  Calibration
 * (Eqs. 6-12) forms each P_g directly over the pixels; every bank
 * (gpjc_calibrate / gpjc_set_compression) is turned into the explicit
 * compressed readout matrices E'_y = blockdiag_p(A_g(p)) E_y (Eq. 14), stored
 * per column ([ny][Np][K][nx] c64, ny * Np * K * nx * 8 bytes, owned by the
 * plan), which gpjc_forward / gpjc_adjoint / gpjc_normal and the solvers
 * apply, each followed or preceded by the phase-encode DFT and mask as for
 * the Wave operator.  Group legality: member patches' map blocks must agree
 * within 1e-6 (any grouping is legal for P = 1).  d_bmod is copied;
 * synchronises. */
int gpjc_plan_create_bmap(const gpjc_geom* geom, const gpjc_c64* d_coils, const gpjc_c64* d_bmod,
                          void* hip_stream, gpjc_plan** out);
int gpjc_plan_destroy(gpjc_plan* plan);
/* Switch the stream later calls are queued on. */
int gpjc_set_stream(gpjc_plan* plan, void* hip_stream);

/* Calibrate the compression bank (Eqs. 6-12): per group, FP64 Gram matrix of
 * the composite maps over the ROI (d_roi [ny][nx] uint8, NULL = all pixels
 * with a nonzero vector), Hermitian eigen-decomposition (Householder
 * tridiagonalisation, bisection for every eigenvalue, inverse iteration for
 * the K leading eigenvectors), descending order, each
 * eigenvector phase-normalised (largest-magnitude entry real positive), first
 * K rows of U^H, times T (x) I_P with T = Q^{-1}, Psi = Q Q^H from
 * d_noise_cov [nc][nc] c64 (NULL = identity).  Outputs (optional):
 * h_eigvals [G][nc*P] descending, d_A_out [G][K][nc][P] c128.
 * Synchronises.  Compressed plans only; Ns = nc*P <= 2048.  GPJC_E_NUMERIC
 * if the Gram is not finite, the noise covariance is not positive definite,
 * or a kept eigenvector fails its residual check ||T y - lambda y|| <=
 * 1e-9 ||T|| after the inverse iteration (3 steps; the environment variable
 * GPJC_INVIT_ITERS = 0..8 sets the count). */
int gpjc_calibrate(gpjc_plan* plan, const uint8_t* d_roi, const gpjc_c64* d_noise_cov,
                   double* h_eigvals, gpjc_c128* d_A_out);

/* gpjc_calibrate for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with every calibration workspace carved
 * from a static device array of 64 MiB (one per GPU, held by the library
 * until the process ends) instead of being allocated.  Allocates nothing.
 * GPJC_E_UNSUPPORTED (before anything is queued) if the workspaces exceed
 * 64 MiB: about 16 groups of Ns = 128 (the 64 x 64, 8-coil slice) fit,
 * high-field slices do not.  Calls that overlap on one GPU share the array
 * and race; the array keeps the last call's contents, and every part a call
 * reads is written by that call first. */
int gpjc_calibrate_static(gpjc_plan* plan, const uint8_t* d_roi, const gpjc_c64* d_noise_cov,
                          double* h_eigvals, gpjc_c128* d_A_out);

/* Install an externally computed bank d_A [G][K][nc][P] c128 (copied):
 * the matrices A_g of Eq. 12 that Eqs. 13-14 apply, e.g. a bank exported by
 * gpjc_calibrate (d_A_out) and reused, as the compression matrices are
 * computed once and reused (Section 2.4).  d_A is 16-byte aligned. */
int gpjc_set_compression(gpjc_plan* plan, const gpjc_c128* d_A);

/* Eq. 13: d_ksp [B][nc][Ms][nt] c64 (acquired lines, ascending; 16-byte
 * aligned) -> d_out [B][Np][K][Ms] c64, Np = nt / P. */
int gpjc_compress(const gpjc_plan* plan, const gpjc_c64* d_ksp, gpjc_c64* d_out);

/* E' (compressed plan): d_img [B][ny][nx] -> d_out [B][Np][K][Ms].
 * E  (uncompressed plan): d_img -> d_out [B][nc][Ms][nt]. */
int gpjc_forward(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_img, gpjc_c64* d_out);
/* Conjugate transpose of gpjc_forward. */
int gpjc_adjoint(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_in, gpjc_c64* d_img);
/* E'^H E' (or E^H E): d_img [B][ny][nx] -> d_out [B][ny][nx]. */
int gpjc_normal(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_img, gpjc_c64* d_out);

/* CG on the normal equations E'^H E' x = E'^H y (Eq. 16's minimiser),
 * d_y in gpjc_forward's output layout, d_x [B][ny][nx] holds x0 on entry and
 * the result on exit; all B images form one joint system.  Dot products are
 * accumulated in FP64 with a fixed reduction order.  With prec != FP32 and
 * refine_every > 0, b = E'^H y and r0 come from the FP32 operator, the
 * search directions from the prec operator, and every refine_every
 * iterations the residual is recomputed as b - E'^H E' x with the FP32
 * operator and the search restarted (iterative refinement: the iterates
 * converge to the FP32 solution).
 * h_resid [iters+1] (optional) receives ||r_k||_2; synchronises if given.
 * GPJC_E_NUMERIC if a residual or step is NaN/Inf (checked at the end). */
int gpjc_recon_cg(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x,
                  int iters, int refine_every, double* h_resid);

/* One gradient-descent step on 1/2 ||E' x - y||^2 (Eq. 16's objective),
 * for unrolled reconstruction networks: with b = E'^H y precomputed (d_b,
 * gpjc_adjoint's output layout [B][ny][nx]) and the step size in device
 * memory (d_alpha, one float, so a learnable step needs no host sync),
 *   d_r_out = E'^H E' x - b          (optional, the residual of the step)
 *   d_x_out = x - alpha * (E'^H E' x - b).
 * d_x_out must not alias d_x or d_b. */
int gpjc_gd_step(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_x, const gpjc_c64* d_b,
                 const float* d_alpha, gpjc_c64* d_x_out, gpjc_c64* d_r_out);
/* Backward of gpjc_gd_step for a real loss L, given g = dL/dx_out (the
 * conjugate-Wirtinger gradient PyTorch uses: dL = Re <g, dx_out>) and the
 * step's residual d_r:
 *   d_gx_out     = g - alpha E'^H E' g     (dL/dx; optional)
 *   d_gb_out     = alpha g                 (dL/db; optional)
 *   d_galpha_out = -Re <g, r>              (dL/dalpha, one float on the device,
 *                                          FP64 fixed-order reduction). */
int gpjc_gd_step_backward(const gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_g, const float* d_alpha,
                          const gpjc_c64* d_r, gpjc_c64* d_gx_out, gpjc_c64* d_gb_out, float* d_galpha_out);

/* FISTA (Section 3.4, Eq. 17 with the wavelet term, TV weight 0) on
 * 1/2 ||E' x - y||^2 + lambda ||W x||_1, W the orthonormal separable Haar
 * transform with haar_levels levels (1..3, nx and ny divisible by
 * 2^levels; the final low-pass band is not penalised), step 1 / lipschitz,
 * x_0 = 0.  d_x [B][ny][nx] receives the last iterate.  h_obj [iters]
 * (optional, iters <= 100001) receives the objective of each iterate x_k,
 * accumulated in FP64 with a fixed reduction order; its data term applies
 * E' in precision prec once more per iteration.  Synchronises at the end;
 * GPJC_E_NUMERIC if the result holds NaN/Inf. */
int gpjc_recon_fista(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters,
                     double lambda, double lipschitz, int haar_levels, double* h_obj);

/* FISTA on the full Eq. 17 (Section 3.4): 1/2 ||E' x - y||^2 +
 * lambda_tv TV_eps(x) + lambda ||W x||_1, with the total variation in the
 * smooth approximation TV_eps(x) = sum over pixels of
 * sqrt(|Dx x|^2 + |Dy x|^2 + tv_eps^2) (Dx, Dy forward differences, zero at
 * the last column / row of each image), whose gradient
 * D^H (D x / sqrt(|D x|^2 + tv_eps^2)) joins the gradient step; the wavelet
 * term stays the proximal step.  lipschitz must bound ||E'^H E'|| +
 * 8 lambda_tv / tv_eps.  Otherwise as gpjc_recon_fista (which is the
 * lambda_tv = 0 case); h_obj includes the TV term. */
int gpjc_recon_fista_tv(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters,
                        double lambda, double lambda_tv, double tv_eps, double lipschitz, int haar_levels,
                        double* h_obj);

/* Reconstruction algorithm #1 (Section 3.4, Fig. 6A): hybrid-space least
 * squares (Eq. 16) for a regular R-fold mask without calibration lines (the
 * acquired lines are exactly those with (ky - Ny/2) divisible by R; else
 * GPJC_E_UNSUPPORTED).  The zero-filled inverse DFT of d_y along the phase
 * encodes folds image rows yr + q Ny/R (q < R) onto each other, so Eq. 16
 * splits into Ny/R independent readout problems per image (unknowns: R Nx
 * pixels; data: the Np K compressed samples of one line), each solved by LSQR
 * (Paige and Saunders) from zero for `iters` iterations; all sets advance
 * together through the operator's column stages, and each set's norms and
 * scalars are its own (FP64, fixed reduction order), so each set follows its
 * own LSQR recurrence.  d_y in gpjc_forward's layout, d_x [B][ny][nx] receives
 * the assembled image.  h_resid [iters+1] (optional) receives
 * sqrt(sum over sets of the LSQR residual estimate^2) = ||E' x_k - y||.
 * Compressed plans (Wave or modulation map), at most 1024 sets (B Ny/R).
 * Synchronises; GPJC_E_NUMERIC on a non-finite residual. */
int gpjc_recon_lsqr(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_y, gpjc_c64* d_x, int iters,
                    double* h_resid);

/* Largest eigenvalue of E'^H E' (the Lipschitz constant of FISTA's
 * gradient) by power iteration from the caller's start d_x0 [B][ny][nx]
 * (normalised first): v <- A v / ||A v||, lambda_k = <v_{k-1}, A v_{k-1}>.
 * Returns the last lambda in *h_lambda; synchronises. */
int gpjc_power_iteration(gpjc_plan* plan, gpjc_prec prec, const gpjc_c64* d_x0, int iters, double* h_lambda);

/* max over all coefficients of |W x| for d_img [B][ny][nx], W the
 * orthonormal Haar transform of haar_levels levels (FISTA's lambda is
 * chosen relative to this for x = E'^H y).  Synchronises. */
int gpjc_wavelet_absmax(gpjc_plan* plan, const gpjc_c64* d_img, int haar_levels, double* h_out);

/* Per-stage kernel timing with HIP events on the plan's stream.  While
 * enabled, every stage launch is bracketed by an event pair (up to 16384
 * launches); gpjc_stage_times synchronises and returns, per stage id, the
 * summed milliseconds and the number of timed launches.  Enabling resets the
 * record. */
enum {
  GPJC_STAGE_READOUT_FWD = 0,   /* F1 */
  GPJC_STAGE_GROUP_COMPRESS,    /* F2 (and Eq. 13 on k-space) */
  GPJC_STAGE_PE_NORMAL,         /* fused phase-encode normal stage */
  GPJC_STAGE_PE_FWD,            /* phase-encode forward */
  GPJC_STAGE_PE_ADJ,            /* phase-encode adjoint */
  GPJC_STAGE_GROUP_EXPAND,      /* F2^H */
  GPJC_STAGE_READOUT_ADJ,       /* F1^H */
  GPJC_STAGE_PE_COLS,           /* uncompressed phase-encode stages */
  GPJC_STAGE_COMBINE,           /* partial-image sums */
  GPJC_STAGE_SOLVER,            /* CG / FISTA vector kernels */
  GPJC_STAGE_EXPLICIT_FWD,      /* explicit readout matrices, forward */
  GPJC_STAGE_EXPLICIT_ADJ,      /* explicit readout matrices, adjoint */
  GPJC_STAGE_COUNT
};
int gpjc_stage_timing(gpjc_plan* plan, int enable);
/* As gpjc_stage_timing, but only the stages whose bit (1 << stage id) is set
 * in stage_mask are bracketed; 0 disables timing.  Each event pair adds a few
 * microseconds between launches, so a throughput measurement times only the
 * stage it reports.  GPJC_E_INVAL for bits at or above GPJC_STAGE_COUNT. */
int gpjc_stage_timing_select(gpjc_plan* plan, unsigned stage_mask);
int gpjc_stage_times(gpjc_plan* plan, double* h_ms, int* h_launches);

/* Work-group tile shape of the two group contractions and the contraction
 * split of the compressing one (1..8), for one precision class: FP32, the
 * two 16-bit types together (BF16 and FP16 share one setting), or BF16X6.  Variant
 * numbers index per-class tables of built shapes.  The defaults come from
 * the plan's sizes; gpjc_autotune times the variants and installs the
 * fastest.  Changes only speed, never results beyond FP32 summation order. */
int gpjc_set_gemm_config(gpjc_plan* plan, gpjc_prec prec, int compress_variant, int expand_variant, int ksplit);
int gpjc_get_gemm_config(const gpjc_plan* plan, gpjc_prec prec, int* compress_variant, int* expand_variant,
                         int* ksplit, int* n_compress_variants, int* n_expand_variants);

/* Tile autotuning of the group contractions: times every built tile shape
 * of both contractions on the plan's own buffers, each split of the
 * compressing one together with the phase-encode stage that reads its
 * partials back, and installs the fastest, as gpjc_set_gemm_config would.  Results are cached
 * per (precision, Ns, K, Ny, B*Np) bucket for the process and, if cache_path
 * is not NULL, in that text file (appended; read on first use), so later
 * plans of the same bucket -- in this or another process -- skip the timing.
 * h_choice [4] (optional): compress variant, expand variant, split, and 1 if
 * the bucket was found in the cache.  Overwrites the plan's operator
 * workspaces; synchronises. */
int gpjc_autotune(gpjc_plan* plan, gpjc_prec prec, const char* cache_path, int* h_choice);

/* Batches of independent slices (Section 3.4 solves independent
 * subproblems in parallel): n plans of any geometries, reconstructed
 * together.  A batch keeps one captured HIP graph per precision holding one
 * CG iteration of every slice and replays it for every iteration; slices are
 * spread over `lanes` streams (0 = 4, at most 16 and n), longest first, so
 * their kernels overlap.  The plans stay owned by the caller and must
 * outlive the batch; a plan may belong to one batch at a time, and must not
 * be used on its own while a batch call runs.  Changing a plan's tile
 * configuration makes the next batch call capture again. */
typedef struct gpjc_batch gpjc_batch;
int gpjc_batch_create(gpjc_plan* const* plans, int n, int lanes, gpjc_batch** out);
int gpjc_batch_destroy(gpjc_batch* batch);
/* Number of streams; h_lane_of [n] (optional) receives each slice's stream. */
int gpjc_batch_lanes(const gpjc_batch* batch, int* h_lane_of);
/* gpjc_recon_cg for every slice i on d_y[i] / d_x[i] (host arrays of n
 * device pointers), one schedule for all: the same result, bit for bit, as
 * n separate gpjc_recon_cg calls with the same plans.  h_resid [n][iters+1]
 * (optional).  Waits for work already queued on the plans' streams, and
 * returns when the batch is done.  GPJC_E_NUMERIC names the first failing
 * slice. */
int gpjc_batch_recon_cg(gpjc_batch* batch, gpjc_prec prec, const gpjc_c64* const* d_y, gpjc_c64* const* d_x,
                        int iters, int refine_every, double* h_resid);
/* gpjc_autotune for every plan of the batch. */
int gpjc_batch_autotune(gpjc_batch* batch, gpjc_prec prec, const char* cache_path);

const char* gpjc_status_string(int status);
const char* gpjc_last_error(void);
/* Path of the HIP runtime library this build is bound to in this process. */
const char* gpjc_runtime_path(void);

#ifdef __cplusplus
}
#endif

#endif /* GPJC_H */
