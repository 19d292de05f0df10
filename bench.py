#!/usr/bin/env python3
"""Benchmark of the compressed Wave operator and reconstruction on one GPU.

Workload: the 2D high-field slice -- 224 x 224 image, 32 coils with B1
phase, readout oversampling 6 (1344 samples), Wave 7 cycles / +-6 rad, 42
patches of 32 samples each its own group (1024 virtual channels), K = 64
(16x joint compression), R = 4 with 16 calibration lines, noise at SNR 30.

One step = one FISTA reconstruction of the slice (50 iterations, 3-level
Haar, lambda = 1e-3 max|W E'^H S'|, step 1/L with L from 50 power
iterations x 1.01): E'^H S' once, then 50 applications of E'^H E' and the
fused gradient / wavelet-prox / momentum update.  value = E'^H E'
applications per second over the timed steps (50 per step).  Calibration
(Gram + eigen-decomposition) and compression of the acquired k-space are
timed once, outside the steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "compressed E^H E applications/s and s/slice recon vs plain FP32, at <=1e-4 NRMSE"
ITERS = 50
LEVELS = 3

PEAKS = {"hbm": 8.0e12, "fp32": 157.3e12, "bf16": 2.5e15, "fp16": 2.5e15, "bf16x6": 2.5e15}
DTYPES = {"fp32": "f32", "bf16": "bf16", "fp16": "f16", "bf16x6": "f32 (bf16x6 contractions)"}

# Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a
# plain copy) for the FP32 operator on this workload, with the hash of the
# sources each kernel is built from when the counters were taken.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "highfield_op_hbm_traffic.md")
STAGE_SOURCES = {
    "readout_fwd": ("operator.hip", "fft.h", "fft2.h", "devutil.h"),
    "readout_adj": ("operator.hip", "fft.h", "fft2.h", "devutil.h"),
    "pe_normal": ("operator.hip", "fft.h", "fft2.h", "devutil.h"),
    "group_compress": ("gemm.hip", "devutil.h"),
    "group_expand": ("gemm.hip", "devutil.h"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_work(g, stage, prec, ksplit_read=1):
    """Algorithmic work of one launch of a stage: (bound, amount, unit)."""
    B, nx, ny, nc, nt = 1, g.nx, g.ny, g.nc, g.nt
    wbytes = 8 if prec in ("fp32", "bf16x6") else 4
    if stage in ("group_compress", "group_expand"):
        if prec == "fp32":  # arithmetic intensity ~50 flop/B, above the FP32 MFMA ridge (~20)
            return "mfma", 8.0 * B * g.k * nc * nt * ny, "flop"
        if prec == "bf16x6":
            # FP32 W once, one FP32 row of each expanded bank pair once, Z once in FP32;
            # the six BF16 products issue 6 x 8 flops per complex multiply-add, about
            # 0.9 of the HBM time at the BF16 peak: HBM-bound
            bank = 4.0 * g.n_groups * g.k * 2 * g.ns
            return "hbm", 8.0 * B * nc * ny * nt + bank + 8.0 * B * g.n_patches * g.k * ny, "byte"
        # 16-bit operands: ~90 flop/B, far below the BF16/FP16 ridge (~300): HBM-bound.
        # W (16-bit) once, the 16-bit real-form bank once, Z in FP32 (compress) / 16-bit (expand).
        bank = 2.0 * g.n_groups * (2 * g.k) * (2 * g.ns)
        z = (8.0 if stage == "group_compress" else 4.0) * B * g.n_patches * g.k * ny
        return "hbm", wbytes * B * nc * ny * nt + bank + z, "byte"
    if stage in ("readout_fwd", "readout_adj"):
        return "hbm", 8.0 * (B * nx * ny + nc * nx * ny + ny * nt) + wbytes * B * nc * ny * nt, "byte"
    if stage == "pe_normal":
        return "hbm", 16.0 * B * g.n_patches * g.k * ny, "byte"
    if stage == "solver":
        return "hbm", 10 * 8.0 * B * nx * ny, "byte"
    return "hbm", 8.0 * B * nx * ny, "byte"


def source_hash(files):
    import hashlib
    m = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2601_05418_amd", "csrc", f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(stage):
    """Bytes per launch from the committed counter summary, or None when the
    kernel's sources changed since the counters were taken."""
    if stage not in STAGE_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    want = source_hash(STAGE_SOURCES[stage])
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and f[0] == "traffic-bytes" and f[1] == stage and f[3] == "src":
                return float(f[2]) if f[4] == want else None
    return None


def batch_bench(steps, warmup, prec, tune_path):
    """64 uneven slices (random matrix size, coils, oversampling, patch length,
    compression factor and acceleration), batched CG-20 with the iteration
    captured in one HIP graph; random orthonormal banks and random data (the
    cost does not depend on them).  Tiles are autotuned per bucket first."""
    import numpy as np
    import torch

    from paper_2601_05418_amd import gpjc, synth
    slices = synth.batch_draws(64, 0)
    rng = np.random.default_rng(77)
    plans, ys = [], []
    for sl in slices:
        g = sl.geom
        p = gpjc.Plan.from_slice(sl)
        p.set_compression(torch.as_tensor(synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng)).cuda())
        plans.append(p)
        ys.append(torch.as_tensor(np.ascontiguousarray(synth.unit_noise(p.data_shape(), rng), np.complex64)).cuda())
    batch = gpjc.Batch(plans)
    t = time.perf_counter()
    batch.autotune(prec, tune_path)
    t_tune = time.perf_counter() - t
    iters = 20
    for _ in range(warmup):
        batch.recon_cg(ys, iters, prec=prec)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        batch.recon_cg(ys, iters, prec=prec)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    # the same solves one plan at a time, without the graph
    t = time.perf_counter()
    for p, y in zip(plans, ys):
        p.recon_cg(y, iters, prec=prec)
    torch.cuda.synchronize()
    dt_sep = time.perf_counter() - t
    w_bytes = sum(p.nc * p.ny * p.nt * 8 for p in plans)
    gemm_f = sum(8.0 * p.k * p.nc * p.nt * p.ny for p in plans)
    batch.close()
    return {
        "workload": "64 uneven slices (N 128-256, 16-32 coils, os 6/8, P 16-48, 12-20x compression, R 3-5 + 8 ACS), "
                    f"batched CG-{iters}",
        "slices": 64, "cg_iters": iters, "precision": prec,
        "s_per_batch": dt, "s_per_slice": dt / 64,
        "op_apps_per_s_aggregate": 64 * (iters + 1) / dt,
        "s_per_batch_one_plan_at_a_time": dt_sep,
        "autotune_s": t_tune,
        "W_total_GB": w_bytes / 1e9, "contraction_GFLOP_per_direction": gemm_f / 1e9,
    }


def unrolled_bench(steps, warmup, prec):
    """Unrolled reconstruction network: 8 images of 256 x 256, 32 coils, os 8
    (2048 samples), 64 groups of 32 samples, K = 80, R = 4; 10 gradient steps
    with learnable step sizes, checkpointed every 2 steps; one training step
    = forward + backward of 1/2 ||x_10 - x_true||^2 (random orthonormal bank)."""
    import numpy as np
    import torch

    from paper_2601_05418_amd import autograd as ga
    from paper_2601_05418_amd import gpjc, synth
    slices = synth.unrolled_slices(8, 0)
    sl = slices[0]
    g = sl.geom
    rng = np.random.default_rng(41)
    plan = gpjc.Plan.from_slice(sl, batch=8)
    plan.set_compression(torch.as_tensor(synth.orthonormal_bank(g.n_groups, g.k, g.nc, g.patch_len, rng)).cuda())
    truth = torch.as_tensor(np.ascontiguousarray(np.stack([s.image for s in slices]), np.complex64)).cuda()
    y = plan.forward(truth)
    x0 = torch.as_tensor(np.ascontiguousarray(synth.unit_noise(plan.image_shape(), rng), np.complex64)).cuda()
    lip = plan.power_iteration(x0, 30, prec=prec) * 1.01
    net = ga.UnrolledGD(plan, steps=10, alpha0=1.0 / lip, checkpoint_every=2, prec=prec)

    def train_step():
        net.zero_grad(set_to_none=True)
        loss = 0.5 * (net(y) - truth).abs().pow(2).sum()
        loss.backward()
        return loss

    for _ in range(warmup):
        train_step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        loss = train_step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    plan.close()
    return {
        "workload": "unrolled GD, 8 x 256x256, 32 coils, os 8, 64 groups of 32, K=80, R=4; 10 steps, "
                    "checkpoint every 2; forward + backward",
        "precision": prec, "s_per_training_step": dt,
        "normal_equivalents_per_step": 30, "op_apps_per_s": 30 * 8 / dt,
        "final_loss": float(loss.detach()),
    }


def explicit_bench(reps=20):
    """The explicit compressed readout model on a local-B0-array slice (a
    nonlinear modulation map, no readout PSF): 224 x 224, 32 coils, os 6
    (1344 samples), an 8-coil local B0 array with 7 cycles per readout and
    +-6 rad.  Joint compression: 42 patches of 32 samples on the 6 groups of
    one modulation period, K = 64 (16x).  RF-only compression: P = 1, one
    group for every sample, K = 10 (3.2x) -- the comparison of Table S2.
    Reported: explicit-matrix size, build and calibration time, and E'^H E'
    applications per image per second for 1 and 8 images per application,
    with the HBM rate of the explicit forward / adjoint kernels."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2601_05418_amd import gpjc, synth
    dev = torch.device("cuda:0")
    base = synth.local_b0_slice(0, n=224, nc=32, os_=6, patch_len=32, k=64, accel=4, acs=16, cycles=7,
                                phase_max=6.0, periodic=True)
    g = base.geom
    rf_geom = dataclasses.replace(g, patch_len=1, patch_group=np.zeros(g.nt, np.int32), n_groups=1, k=10)
    out = {"workload": "local-B0 slice 224x224, 32 coils, os 6 (1344 samples), 8-coil B0 array, 7 cycles, "
                       "+-6 rad, R=4+16 ACS; joint P=32 (6 periodic groups), K=64 vs RF-only P=1, K=10"}
    for name, geom in (("joint_16x", g), ("rf_only_3.2x", rf_geom)):
        sl = dataclasses.replace(base, geom=geom)
        rows = geom.n_patches * geom.k
        ebytes = 8.0 * geom.ny * rows * geom.nx
        res = {"patch_len": geom.patch_len, "groups": geom.n_groups, "k": geom.k,
               "compression_factor": geom.nc * geom.patch_len / geom.k, "explicit_matrix_GB": ebytes / 1e9}
        for batch in (1, 8):
            plan = gpjc.Plan.from_map_slice(sl, batch=batch)
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.calibrate()
            torch.cuda.synchronize()
            if batch == 1:
                res["calibrate_and_build_s"] = time.perf_counter() - t
            x = torch.as_tensor(np.ascontiguousarray(np.broadcast_to(sl.image, (batch, g.ny, g.nx)),
                                                     np.complex64)).to(dev)
            o = torch.empty_like(x)
            for _ in range(3):
                plan.normal(x, out=o)
            plan.stage_timing(True, stages=["explicit_fwd", "explicit_adj"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                plan.normal(x, out=o)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            st = plan.stage_times()
            plan.stage_timing(False)
            kb = {}
            for stg in ("explicit_fwd", "explicit_adj"):
                ms, n = st[stg]
                sec = ms / n / 1e3
                byts = ebytes + 8.0 * batch * (geom.ny * geom.nx + rows * geom.ny)
                kb[stg] = {"us_per_launch": sec * 1e6, "GB_per_s": byts / sec / 1e9, "hbm_frac": byts / sec / 8e12}
            res[f"batch{batch}"] = {"ms_per_application": dt * 1e3, "image_applications_per_s": batch / dt,
                                    "kernels": kb}
            plan.close()
            torch.cuda.empty_cache()
        out[name] = res
        log(f"explicit {name}: {res['explicit_matrix_GB']:.2f} GB, "
            f"B=1 {res['batch1']['ms_per_application']:.3f} ms, B=8 {res['batch8']['ms_per_application']:.3f} ms")
    out["joint_speedup_over_rf_only"] = {
        f"batch{b}": out["joint_16x"][f"batch{b}"]["image_applications_per_s"]
        / out["rf_only_3.2x"][f"batch{b}"]["image_applications_per_s"] for b in (1, 8)}
    return out


def solvers_bench(steps=3):
    """The other reconstruction algorithms of Section 3.4 on the high-field
    slice (224 x 224, 32 coils, 42 groups of 32, K = 64), GPU calibration and
    compression of the acquired data:
    - algorithm #1, LSQR-20 over the 56 aliased sets of a regular R = 4 mask
      without calibration lines, beside CG-20 on the same data (both Eq. 16);
    - FISTA-50 on Eq. 17 with smoothed TV (lambda_tv = 2e-3, eps = 1e-2 of
      max|b|) and the Haar term (lambda = 1e-3 max|W b|) on a variable-density
      Poisson-disc mask (~4x, 16 centre lines), compressed and plain operator."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2601_05418_amd import gpjc, synth
    dev = torch.device("cuda:0")
    out = {}

    def acquire(sl):
        full = gpjc.Plan.from_slice(sl, compressed=False)
        img = torch.as_tensor(np.ascontiguousarray(sl.image[None], np.complex64)).to(dev)
        s_h = full.forward(img).cpu().numpy().astype(np.complex128)
        rng = np.random.default_rng(3)
        noise = synth.unit_noise(s_h.shape, rng)
        full.close()
        return torch.as_tensor(np.ascontiguousarray(s_h + synth.scaled_noise(s_h, noise, 30.0), np.complex64)).to(dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    base = synth.highfield_slice(0)
    g = base.geom
    ky = np.arange(g.ny) - g.ny // 2
    reg = dataclasses.replace(base, geom=dataclasses.replace(g, mask=(ky % 4 == 0).astype(np.uint8)))
    ksp = acquire(reg)
    plan = gpjc.Plan.from_slice(reg)
    plan.calibrate()
    y = plan.compress(ksp)
    out["lsqr_alg1"] = {
        "workload": "224x224, 32 coils, 42 groups of 32, K=64, regular R=4 without calibration lines (56 aliased "
                    "sets of 4x224 unknowns, 2688 samples each), SNR 30",
        "lsqr20_s_per_slice": timed(lambda: plan.recon_lsqr(y, 20)),
        "cg20_s_per_slice_same_data": timed(lambda: plan.recon_cg(y, 20)),
    }
    plan.close()
    log(f"algorithm #1 LSQR-20: {out['lsqr_alg1']['lsqr20_s_per_slice'] * 1e3:.2f} ms")

    mask = synth.poisson_disc_mask(g.ny, 4, np.random.default_rng(9), center=16)
    pd = dataclasses.replace(base, geom=dataclasses.replace(g, mask=mask))
    ksp = acquire(pd)
    plan = gpjc.Plan.from_slice(pd)
    plan.calibrate()
    y = plan.compress(ksp)
    unc = gpjc.Plan.from_slice(pd, compressed=False)
    res = {"workload": f"224x224, 32 coils, 42 groups of 32, K=64, variable-density Poisson-disc mask "
                       f"({int(mask.sum())} of {g.ny} lines), SNR 30; FISTA-50 with TV + 3-level Haar"}
    x0 = torch.as_tensor(np.ascontiguousarray(synth.unit_noise((1, g.ny, g.nx), np.random.default_rng(1)),
                                              np.complex64)).to(dev)
    for name, p, data in (("compressed", plan, y), ("uncompressed", unc, ksp)):
        b = p.adjoint(data)
        amax = float(b.abs().max())
        lam = 1e-3 * p.wavelet_absmax(b, LEVELS)
        lam_tv, eps = 2e-3 * amax, 1e-2 * amax
        lip = p.power_iteration(x0, 30) * 1.01 + 8 * lam_tv / eps
        res[f"{name}_s_per_slice"] = timed(lambda: p.recon_fista_tv(data, ITERS, lam, lam_tv, eps, lip, LEVELS))
    res["speedup_of_compressed"] = res["uncompressed_s_per_slice"] / res["compressed_s_per_slice"]
    out["fista_tv_poisson_disc"] = res
    plan.close()
    unc.close()
    log(f"FISTA-TV-50 PD: compressed {res['compressed_s_per_slice'] * 1e3:.2f} ms, "
        f"uncompressed {res['uncompressed_s_per_slice'] * 1e3:.2f} ms")
    return out


def volume_bench(steps=3):
    """A 3D Wave-CAIPI volume close to the 3D ex vivo case of Table S2
    (180 x 180 x 80, 32 coils, os 8): 192 x 192 x 64, 32 coils, os 8 (1536
    samples), corkscrew PSF with 8 cycles and +-6 rad, 48 patches of 32 on the
    6 groups of one period, K = 56 (18x), CAIPI 4 x 3 shift 1 with a 16 x 16
    centre.  Calibration, tile autotuning, E'^H E' per volume (FP32, BF16), CG-20, and the
    uncompressed FP32 E^H E of the same volume; a stage-timed application of
    each operator."""
    import numpy as np
    import torch

    from paper_2601_05418_amd import gpjc, synth
    dev = torch.device("cuda:0")
    v = synth.volume(0, n=192, nz=64, nc=32, os_=8, patch_len=32, k=56, ry=4, rz=3, shift=1, acs=16, cycles=8,
                     phase=6.0, periodic=True)
    g = v.geom
    plan = gpjc.Plan.from_volume(v)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.calibrate()
    torch.cuda.synchronize()
    t_cal = time.perf_counter() - t
    for prec in ("fp32", "bf16"):
        plan.autotune(prec)  # contraction tiles for the volume's shapes (under a second each)
    x = torch.as_tensor(np.ascontiguousarray(v.image[None], np.complex64)).to(dev)
    o = torch.empty_like(x)
    res = {"workload": f"3D Wave-CAIPI {g.nx}x{g.ny}x{v.nz}, {g.nc} coils, os {g.os} ({g.nt} samples), "
                       f"{g.n_patches} patches of {g.patch_len} on {g.n_groups} periodic groups, K={g.k} "
                       f"({g.ns / g.k:.0f}x), CAIPI 4x3 shift 1 + 16x16 centre ({v.ms} of {g.ny * v.nz} points)",
           "calibrate_s": t_cal, "W_GB": 8.0 * g.nc * g.ny * v.nz * g.nt / 1e9}
    for prec in ("fp32", "bf16"):
        for _ in range(2):
            plan.normal(x, prec=prec, out=o)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            plan.normal(x, prec=prec, out=o)
        torch.cuda.synchronize()
        res[f"normal_ms_{prec}"] = (time.perf_counter() - t) / steps * 1e3
    y = plan.forward(x)
    plan.recon_cg(y, 2)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.recon_cg(y, 20)
    torch.cuda.synchronize()
    res["cg20_s_per_volume"] = time.perf_counter() - t

    def staged(p, prec):
        p.stage_timing(True)
        p.normal(x, prec=prec, out=o)
        torch.cuda.synchronize()
        st = p.stage_times()
        p.stage_timing(False)
        return {k: round(v[0], 4) for k, v in st.items() if v[1]}

    res["stages_ms_fp32"] = staged(plan, "fp32")
    plan.close()
    log(f"3D volume: calibrate {t_cal:.2f} s, E'^H E' {res['normal_ms_fp32']:.2f} ms, "
        f"CG-20 {res['cg20_s_per_volume']:.3f} s")
    full = gpjc.Plan.from_volume(v, compressed=False)
    for _ in range(2):
        full.normal(x, out=o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        full.normal(x, out=o)
    torch.cuda.synchronize()
    res["uncompressed_fp32"] = {"normal_ms": (time.perf_counter() - t) / steps * 1e3,
                                "stages_ms": staged(full, "fp32")}
    full.close()
    for prec in ("fp32", "bf16"):
        res["uncompressed_fp32"][f"speedup_of_compressed_{prec}"] = \
            res["uncompressed_fp32"]["normal_ms"] / res[f"normal_ms_{prec}"]
    # Against the roofline, from the stage-timed applications: the volume's
    # rows (z, y) take the place of a slice's rows y in the work model.
    import dataclasses
    gv = dataclasses.replace(g, ny=g.ny * v.nz)
    roof = {}
    for stage in ("readout_fwd", "group_compress", "group_expand", "readout_adj"):
        ms = res["stages_ms_fp32"].get(stage)
        bound, work, unit = stage_work(gv, stage, "fp32")
        if ms:
            rate = work / (ms * 1e-3) / (1e12 if unit == "flop" else 1e9)
            peak = PEAKS["fp32"] / 1e12 if bound == "mfma" else PEAKS["hbm"] / 1e9
            roof[stage] = {"bound": bound, "achieved": rate, "peak": peak,
                           "unit": "TFLOP/s" if unit == "flop" else "GB/s", "frac": rate / peak}
    w_bytes = 8.0 * g.nc * g.ny * v.nz * g.nt
    ms = res["uncompressed_fp32"]["stages_ms"].get("pe_cols")
    if ms:
        roof["uncompressed_pe_cols"] = {
            "bound": "hbm", "passes": 3, "moved_GB": 3 * 2 * w_bytes / 1e9, "algorithmic_GB": 2 * w_bytes / 1e9,
            "achieved_moved": 3 * 2 * w_bytes / (ms * 1e-3) / 1e9, "achieved": 2 * w_bytes / (ms * 1e-3) / 1e9,
            "peak": PEAKS["hbm"] / 1e9, "unit": "GB/s", "frac": 2 * w_bytes / (ms * 1e-3) / PEAKS["hbm"]}
    res["roofline"] = roof
    log(f"3D volume, uncompressed: E^H E {res['uncompressed_fp32']['normal_ms']:.2f} ms")
    return res


def cpu_baseline(sl, budget_s, gpu_normal=None):
    """The oracle on the host cores, on a bounded sample of the workload:
    E'^H E' applications for about budget_s seconds (the unit of `value`),
    the wavelet prox of one FISTA iteration, and the Gram + eigen-selection
    of one of the slice's groups.  FISTA-50 and calibration of the whole
    slice are extrapolated from these (50 applications + 50 proxes; G times
    one group).  gpu_normal(bank, x) -> the GPU's FP32 E'^H E' x with the same
    bank; its distance to the first oracle application is reported."""
    import numpy as np

    from oracle import compression as oc
    from oracle import encoding as oe
    from oracle import solvers as osv
    g = sl.geom
    rng = np.random.default_rng(0)
    bank = np.empty((g.n_groups, g.k, g.nc, g.patch_len), complex)
    for i in range(g.n_groups):
        q, _ = np.linalg.qr(rng.standard_normal((g.ns, g.k)) + 1j * rng.standard_normal((g.ns, g.k)))
        bank[i] = q.conj().T.reshape(g.k, g.nc, g.patch_len)
    r64 = lambda a: np.asarray(a, np.complex64).astype(np.complex128)  # the values the GPU holds
    coils, psf = r64(sl.coils), r64(sl.psf)
    x = r64(sl.image)
    first = None
    n = 0
    t0 = time.perf_counter()
    c0 = os.times()
    while True:
        y = oe.normal(x, coils, psf, g.mask, g.os, bank, g.patch_group, g.patch_len)
        if first is None:
            first = (x, y)
        x = y / np.linalg.norm(y)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    wall = time.perf_counter() - t0
    t = time.perf_counter()
    osv.wavelet_prox(x, 1e-3, LEVELS)
    t_prox = time.perf_counter() - t
    t = time.perf_counter()
    e = oc.virtual_channels(coils, psf, g.os, g.patch_len, 0)
    oc.compression_matrix(oc.gram(e), g.k, g.patch_len)
    t_group = time.perf_counter() - t
    c1 = os.times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    wall_all = time.perf_counter() - t0
    try:
        import threadpoolctl
        blas = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        blas = None
    out = {
        "value": n / wall,
        "unit": "E'^H E' applications/s",
        "cores": len(os.sched_getaffinity(0)),
        "threads_used": round(cpu / wall_all, 2),
        "kind": "oracle",
        "sample": f"{n} FP64 NumPy applications of E'^H E' ({wall:.1f} s), one wavelet prox and the Gram + "
                  f"eigen-selection of 1 of {g.n_groups} groups, on the same {g.nx}x{g.ny} / {g.nc}-coil slice "
                  f"(random orthonormal bank); BLAS threads {blas}, np.fft single-threaded",
        "fista50_s_per_slice_extrapolated": ITERS * (wall / n + t_prox),
        "calibrate_s_extrapolated": g.n_groups * t_group,
        "calibrate_one_group_s": t_group,
    }
    if gpu_normal is not None:
        xin, yref = first
        out["gpu_fp32_normal_rel_l2_vs_oracle"] = float(np.linalg.norm(gpu_normal(bank, xin) - yref)
                                                        / np.linalg.norm(yref))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "fp16", "bf16x6"])
    ap.add_argument("--periodic", action="store_true", help="map the 42 patches onto the 6 of one wave period")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-slice batched CG measurement")
    ap.add_argument("--no-unrolled", action="store_true", help="skip the unrolled-network training step")
    ap.add_argument("--no-explicit", action="store_true", help="skip the explicit-model (local B0 map) measurement")
    ap.add_argument("--no-solvers", action="store_true", help="skip the algorithm #1 and FISTA-TV measurements")
    ap.add_argument("--no-volume", action="store_true", help="skip the 3D volume measurement")
    ap.add_argument("--tune-cache", default=None, help="tile autotuning cache file")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (reference for byte counters)")
    ap.add_argument("--op-only", type=int, default=0, metavar="N",
                    help="only calibrate and run N applications of E'^H E' (for profiler runs)")
    ap.add_argument("--volume-only", action="store_true",
                    help="only run the 3D volume measurement and print its record (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs on a single "
              "MI355X; the multi-GPU sharding is a design in the documentation only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_05418_amd import gpjc, synth

    dev = torch.device("cuda:0")
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "copies": 5}), flush=True)
        return
    if args.volume_only:
        print(json.dumps({"volume_3d": volume_bench()}), flush=True)
        return
    sl = synth.highfield_slice(0, periodic=args.periodic)
    g = sl.geom
    log(f"workload: {g.nx}x{g.ny}, nc={g.nc}, nt={g.nt}, P={g.patch_len}, G={g.n_groups}, K={g.k}, Ms={g.ms}")

    # acquired k-space: uncompressed operator on the GPU, then noise at SNR 30
    full = gpjc.Plan.from_slice(sl, compressed=False)
    img = torch.as_tensor(np.ascontiguousarray(sl.image[None], np.complex64)).to(dev)
    s_h = full.forward(img).cpu().numpy().astype(np.complex128)
    full.close()
    noisy = s_h + synth.scaled_noise(s_h, sl.noise[None], sl.snr)
    ksp = torch.as_tensor(np.ascontiguousarray(noisy, np.complex64)).to(dev)

    plan = gpjc.Plan.from_slice(sl)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.calibrate()
    torch.cuda.synchronize()
    t_cal = time.perf_counter() - t
    log(f"calibrate: {t_cal:.3f} s")
    y = plan.compress(ksp)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        plan.compress(ksp, out=y)
    torch.cuda.synchronize()
    t_comp = (time.perf_counter() - t) / 10

    if args.op_only:
        xin = torch.as_tensor(np.ascontiguousarray(sl.image[None], np.complex64)).to(dev)
        out = torch.empty_like(xin)
        for _ in range(args.op_only):
            plan.normal(xin, prec=args.prec, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"op_only_applications": args.op_only}), flush=True)
        return

    b = plan.adjoint(y, prec=args.prec)
    lam = 1e-3 * plan.wavelet_absmax(b, LEVELS)
    rng = np.random.default_rng(1)
    x0 = torch.as_tensor(np.ascontiguousarray(synth.unit_noise((1, g.ny, g.nx), rng), np.complex64)).to(dev)
    lip = plan.power_iteration(x0, 50, prec=args.prec) * 1.01
    log(f"lambda {lam:.4e}, L {lip:.4e}")
    # The oracle's stored FISTA-50 run of this slice (tests/golden, written by
    # a script that calls only the oracle): with its lambda and L the GPU runs
    # the same schedule, and its result is compared with the stored iterate.
    gold = None
    gold_path = os.path.join(ROOT, "tests", "golden", "highfield_fista50.npz")
    if not args.periodic and os.path.exists(gold_path):
        gold = np.load(gold_path)
        lam_gpu, lip_gpu = lam, lip
        lam, lip = float(gold["lam"]), float(gold["lip"])
        log(f"using the stored oracle's lambda {lam:.4e} and L {lip:.4e}")

    x = torch.empty((1, g.ny, g.nx), dtype=torch.complex64, device=dev)
    # Untimed pass with every stage timed by HIP events: the per-stage
    # breakdown, and the dominant kernel.  A single-kernel stage hands its
    # event pair to the kernel's own dispatch (the events mark the kernel's
    # start and end); the timed steps time only the dominant kernel.
    plan.stage_timing(True)
    plan.recon_fista(y, ITERS, lam, lip, LEVELS, prec=args.prec, out=x)
    torch.cuda.synchronize()
    stages = plan.stage_times()
    plan.stage_timing(False)
    per_stage = {k: {"ms_per_launch": (v[0] / v[1] if v[1] else 0.0), "launches": v[1], "ms_total": v[0]}
                 for k, v in stages.items() if v[1]}
    dom = max(per_stage, key=lambda k: per_stage[k]["ms_total"])
    for i in range(args.warmup):
        plan.recon_fista(y, ITERS, lam, lip, LEVELS, prec=args.prec, out=x)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")
    plan.stage_timing(True, stages=[dom])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        plan.recon_fista(y, ITERS, lam, lip, LEVELS, prec=args.prec, out=x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    live = plan.stage_times()[dom]
    plan.stage_timing(False)
    ms_per_step = 1e3 * dt / args.steps
    value = ITERS * args.steps / dt
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms per slice, {value:.1f} E'^H E' per s")
    accuracy = {}
    if gold is not None:
        xr = x.cpu().numpy()[0].astype(np.complex128)
        ref = gold["x"].astype(np.complex128)
        mag = np.abs(ref)
        accuracy = {
            "fista50_nrmse_vs_stored_oracle": float(np.sqrt(np.mean(np.abs(xr - ref) ** 2)) / (mag.max() - mag.min())),
            "lambda_rel_diff_gpu_vs_oracle": abs(lam_gpu - lam) / lam,
            "lipschitz_rel_diff_gpu_vs_oracle": abs(lip_gpu - lip) / lip,
            "note": "GPU FISTA-50 (its own calibration, the oracle's lambda and L) against the oracle's FP64 run "
                    "stored in tests/golden/highfield_fista50.npz; NRMSE normalised by the reference's range",
        }
        log(f"FISTA-50 NRMSE vs stored oracle: {accuracy['fista50_nrmse_vs_stored_oracle']:.2e}")

    # operator alone
    out = torch.empty_like(x)
    for _ in range(5):
        plan.normal(x, prec=args.prec, out=out)
    torch.cuda.synchronize()
    t = time.perf_counter()
    nop = 100
    for _ in range(nop):
        plan.normal(x, prec=args.prec, out=out)
    torch.cuda.synchronize()
    op_rate = nop / (time.perf_counter() - t)

    def op_rate_of(pl, prec, n=100):
        for _ in range(5):
            pl.normal(x, prec=prec, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            pl.normal(x, prec=prec, out=out)
        torch.cuda.synchronize()
        return n / (time.perf_counter() - t0)

    # the same operator with 16-bit operands (FP32 accumulation), and the
    # uncompressed FP32 operator on the same slice
    variants = {args.prec: op_rate}
    for pr in ("fp32", "bf16", "fp16", "bf16x6"):
        if pr != args.prec:
            variants[pr] = op_rate_of(plan, pr)
    unc = gpjc.Plan.from_slice(sl, compressed=False)
    variants["uncompressed_fp32"] = op_rate_of(unc, "fp32")
    log("E'^H E' per s: " + ", ".join(f"{k} {v:.0f}" for k, v in variants.items()))
    # the same FISTA-50 reconstruction with the uncompressed FP32 operator on
    # the acquired k-space
    b_u = unc.adjoint(ksp)
    lam_u = 1e-3 * unc.wavelet_absmax(b_u, LEVELS)
    lip_u = unc.power_iteration(x0, 50) * 1.01
    x_u = torch.empty_like(x)
    for _ in range(max(1, args.warmup)):
        unc.recon_fista(ksp, ITERS, lam_u, lip_u, LEVELS, out=x_u)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        unc.recon_fista(ksp, ITERS, lam_u, lip_u, LEVELS, out=x_u)
    torch.cuda.synchronize()
    dt_u = (time.perf_counter() - t) / args.steps
    uncomp = {"s_per_slice": dt_u, "apps_per_s": ITERS / dt_u, "op_apps_per_s": variants["uncompressed_fp32"],
              "speedup_of_compressed": dt_u / (ms_per_step / 1e3)}
    unc.close()
    log(f"uncompressed FP32 FISTA-{ITERS}: {dt_u * 1e3:.3f} ms per slice")
    # The same reconstruction with the contractions in BF16X6 (FP32 storage,
    # FP32-accurate split-BF16 products), timed the same way
    split_run = None
    if args.prec == "fp32":
        xs = torch.empty_like(x)
        for _ in range(max(1, args.warmup)):
            plan.recon_fista(y, ITERS, lam, lip, LEVELS, prec="bf16x6", out=xs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.recon_fista(y, ITERS, lam, lip, LEVELS, prec="bf16x6", out=xs)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t) / args.steps
        split_run = {"s_per_slice": dt_s, "apps_per_s": ITERS / dt_s, "op_apps_per_s": variants["bf16x6"],
                     "speedup_vs_fp32_compressed": (ms_per_step / 1e3) / dt_s,
                     "speedup_vs_uncompressed_fp32": dt_u / dt_s}
        if gold is not None:
            xr = xs.cpu().numpy()[0].astype(np.complex128)
            ref = gold["x"].astype(np.complex128)
            mag = np.abs(ref)
            split_run["fista50_nrmse_vs_stored_oracle"] = float(
                np.sqrt(np.mean(np.abs(xr - ref) ** 2)) / (mag.max() - mag.min()))
        log(f"BF16X6 FISTA-{ITERS}: {dt_s * 1e3:.3f} ms per slice")

    bound, work, kind = stage_work(g, dom, args.prec)
    avg_s = live[0] / live[1] / 1e3  # measured over the timed steps
    if bound == "mfma":
        peak = PEAKS[args.prec]
        roof = {"bound": "mfma", "achieved": work / avg_s / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s"}
        # work counts 8 real flops per complex multiply-add; the FP32 contractions
        # form the product with three real multiplications, so they issue 3/4 of it
        issued = 0.75 * work if dom in ("group_compress", "group_expand") else work
        roof["issued_frac"] = issued / avg_s / peak
    else:
        peak = PEAKS["hbm"]
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": peak / 1e9, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # counters were taken on the FP32 operator of the 42-group workload
    roof["traffic"] = measured_traffic(dom) if (args.prec == "fp32" and not args.periodic) else None
    roof["traffic_unit"] = "bytes per launch"
    roof["kernel"] = dom
    roof["work_per_launch"] = work
    roof["work_unit"] = kind
    roof["timed_launches"] = live[1]

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "E'^H E' applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.prec],
        "data": "synthetic",
        "config": {
            "workload": f"2D high-field slice {g.nx}x{g.ny}, {g.nc} coils, os {g.os} ({g.nt} samples), "
                        f"{g.n_patches} patches of {g.patch_len}, {g.n_groups} groups, K={g.k}, R=4+16 ACS, "
                        f"SNR 30; step = FISTA-{ITERS} with {LEVELS}-level Haar",
            "nx": g.nx, "ny": g.ny, "nc": g.nc, "os": g.os, "patch_len": g.patch_len,
            "groups": g.n_groups, "k": g.k, "ms": g.ms, "fista_iters": ITERS, "precision": args.prec,
        },
        "s_per_slice": ms_per_step / 1e3,
        "op_apps_per_s": op_rate,
        "op_apps_per_s_by_variant": variants,
        "uncompressed_fp32": uncomp,
        # the reduced-precision forms against the plain FP32 compressed operator
        "op_speedup_vs_fp32": {k: variants[k] / variants["fp32"] for k in ("bf16", "fp16", "bf16x6")
                               if "fp32" in variants},
        "fp32_accurate_bf16x6": split_run,
        "calibrate_s": t_cal,
        "compress_s": t_comp,
        "stages": per_stage,
        "stages_note": "one untimed FISTA step with every stage timed by HIP events (single-kernel stages by "
                       "events on the kernel's own dispatch, hipExtLaunchKernel; the others by event records "
                       "around them); the timed steps time only the roofline kernel, the same way",
        "roofline": roof,
        "accuracy": accuracy,
        "cpu_baseline": None,
    }
    if not args.no_batch:
        log("batched CG over 64 uneven slices ...")
        plan.close()
        result["batch"] = batch_bench(max(1, args.steps // 2), 1, args.prec, args.tune_cache)
        log(f"batch: {result['batch']['s_per_batch']:.3f} s per 64 slices")
    if not args.no_unrolled:
        log("unrolled network training step ...")
        result["unrolled"] = unrolled_bench(max(1, args.steps // 2), 1, args.prec)
        log(f"unrolled: {result['unrolled']['s_per_training_step'] * 1e3:.1f} ms per training step")
    if not args.no_explicit:
        log("explicit readout model on a local-B0 map ...")
        result["explicit_local_b0"] = explicit_bench()
    if not args.no_solvers:
        log("algorithm #1 and FISTA-TV ...")
        result["solvers"] = solvers_bench()
    if not args.no_volume:
        log("3D volume ...")
        result["volume_3d"] = volume_bench()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")

        def gpu_normal(bank, xin):
            p = gpjc.Plan.from_slice(sl)
            p.set_compression(torch.as_tensor(bank).to(dev))
            xt = torch.as_tensor(np.ascontiguousarray(xin[None], np.complex64)).to(dev)
            out_np = p.normal(xt).cpu().numpy()[0].astype(np.complex128)
            p.close()
            return out_np

        result["cpu_baseline"] = cpu_baseline(sl, args.cpu_seconds, gpu_normal)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
