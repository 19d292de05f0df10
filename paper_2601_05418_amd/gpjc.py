"""Python binding of libgpjc (ctypes).

Argument marshalling only: every step of the operator, calibration and
reconstruction runs in the library's HIP kernels.  PyTorch provides device
memory (tensors) and the stream.  torch is imported before the library is
loaded so that libgpjc binds to the same HIP runtime instance as torch and
device pointers can be shared.

The function names mirror the C ABI in include/gpjc.h.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpjc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "gpjc.h")

FP32, BF16, FP16, BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "bf16x6": BF16X6}

STAGES = ("readout_fwd", "group_compress", "pe_normal", "pe_fwd", "pe_adj", "group_expand", "readout_adj",
          "pe_cols", "combine", "solver", "explicit_fwd", "explicit_adj")

GPJC_OK = 0
GPJC_E_INVAL = -1
GPJC_E_STATE = -2
GPJC_E_NOMEM = -3
GPJC_E_DEVICE = -4
GPJC_E_UNSUPPORTED = -5
GPJC_E_NUMERIC = -6


class GpjcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libgpjc status {status}: {message}")
        self.status = status


class _Geom(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nc", ctypes.c_int32), ("os", ctypes.c_int32),
        ("patch_len", ctypes.c_int32), ("n_groups", ctypes.c_int32),
        ("patch_group", ctypes.POINTER(ctypes.c_int32)), ("k", ctypes.c_int32),
        ("mask", ctypes.POINTER(ctypes.c_uint8)), ("batch", ctypes.c_int32), ("compressed", ctypes.c_int32),
    ]


_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "gpjc_plan_create": (_I, [ctypes.POINTER(_Geom), _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    "gpjc_plan_create_bmap": (_I, [ctypes.POINTER(_Geom), _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    "gpjc_plan_create_3d": (_I, [ctypes.POINTER(_Geom), _I, _VP, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    "gpjc_plan_destroy": (_I, [_VP]),
    "gpjc_set_stream": (_I, [_VP, _VP]),
    "gpjc_calibrate": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "gpjc_calibrate_static": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "gpjc_set_compression": (_I, [_VP, _VP]),
    "gpjc_compress": (_I, [_VP, _VP, _VP]),
    "gpjc_forward": (_I, [_VP, _I, _VP, _VP]),
    "gpjc_adjoint": (_I, [_VP, _I, _VP, _VP]),
    "gpjc_normal": (_I, [_VP, _I, _VP, _VP]),
    "gpjc_recon_cg": (_I, [_VP, _I, _VP, _VP, _I, _I, _VP]),
    "gpjc_recon_fista": (_I, [_VP, _I, _VP, _VP, _I, _D, _D, _I, _VP]),
    "gpjc_recon_lsqr": (_I, [_VP, _I, _VP, _VP, _I, _VP]),
    "gpjc_recon_fista_tv": (_I, [_VP, _I, _VP, _VP, _I, _D, _D, _D, _D, _I, _VP]),
    "gpjc_power_iteration": (_I, [_VP, _I, _VP, _I, _VP]),
    "gpjc_wavelet_absmax": (_I, [_VP, _VP, _I, _VP]),
    "gpjc_stage_timing": (_I, [_VP, _I]),
    "gpjc_stage_timing_select": (_I, [_VP, ctypes.c_uint]),
    "gpjc_stage_times": (_I, [_VP, _VP, _VP]),
    "gpjc_set_gemm_config": (_I, [_VP, _I, _I, _I, _I]),
    "gpjc_get_gemm_config": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP]),
    "gpjc_gd_step": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP]),
    "gpjc_gd_step_backward": (_I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
    "gpjc_autotune": (_I, [_VP, _I, ctypes.c_char_p, _VP]),
    "gpjc_batch_create": (_I, [_VP, _I, _I, ctypes.POINTER(_VP)]),
    "gpjc_batch_destroy": (_I, [_VP]),
    "gpjc_batch_lanes": (_I, [_VP, _VP]),
    "gpjc_batch_recon_cg": (_I, [_VP, _I, _VP, _VP, _I, _I, _VP]),
    "gpjc_batch_autotune": (_I, [_VP, _I, ctypes.c_char_p]),
    "gpjc_status_string": (ctypes.c_char_p, [_I]),
    "gpjc_last_error": (ctypes.c_char_p, []),
    "gpjc_runtime_path": (ctypes.c_char_p, []),
}

_lib = None


def header_symbols(path: str = HEADER_PATH):
    """Names of the functions declared in include/gpjc.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpjc_[a-z0-9_]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load libgpjc.so (built in-tree).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def runtime_path() -> str:
    return load().gpjc_runtime_path().decode()


def _check(status: int):
    if status != GPJC_OK:
        raise GpjcError(status, load().gpjc_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    """Device pointer of an output tensor (must be contiguous)."""
    if t is None:
        return None
    if not t.is_contiguous() or t.is_conj() or t.is_neg():
        raise ValueError("output tensor must be contiguous and not a conjugate / negative view")
    return ctypes.c_void_p(t.data_ptr())


def _materialise(t: torch.Tensor) -> torch.Tensor:
    """Contiguous tensor whose memory holds its values: lazily conjugated or
    negated views (PyTorch's conj / neg bits) are resolved, as the library
    reads raw memory."""
    return t.resolve_conj().resolve_neg().contiguous()


def _dev_tensor(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return _materialise(x.to(device=device, dtype=dtype))
    return _materialise(torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype))


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class Plan:
    """A libgpjc plan: geometry, coil maps, PSF, compression bank, workspaces.

    coils [nc][ny][nx] and psf [ny][nt] (complex, host or device) are copied.
    """

    def __init__(self, nx, ny, nc, os_, coils, psf, mask, patch_len=0, patch_group=None, n_groups=0, k=0,
                 batch=1, compressed=True, device="cuda:0", stream=None, bmod=None, nz=1):
        """psf [ny][nt] (Wave) or, with psf None, bmod [nt][ny][nx] (a general
        modulation map, gpjc_plan_create_bmap); nz > 1: a 3D volume with
        mask [nz][ny], coils [nc][nz][ny][nx], psf [nz][ny][nt]
        (gpjc_plan_create_3d)."""
        self.lib = load()
        self.device = torch.device(device)
        self.nx, self.ny, self.nc, self.os = int(nx), int(ny), int(nc), int(os_)
        self.nt = self.os * self.nx
        self.batch = int(batch)
        self.compressed = bool(compressed)
        self.nz = int(nz)
        self.mask = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        self.ms = int((self.mask != 0).sum())
        self.patch_len = int(patch_len)
        self.k = int(k)
        self.n_groups = int(n_groups)
        self.np_ = self.nt // self.patch_len if self.compressed and self.patch_len else 0
        pg = np.zeros(max(self.np_, 1), np.int32) if patch_group is None else patch_group
        self.patch_group = np.ascontiguousarray(np.asarray(pg, dtype=np.int32))
        g = _Geom(self.nx, self.ny, self.nc, self.os, self.patch_len, self.n_groups,
                  self.patch_group.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.k,
                  self.mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), self.batch, int(self.compressed))
        c = _dev_tensor(coils, torch.complex64, self.device)
        self.general = bmod is not None
        p = _dev_tensor(bmod if self.general else psf, torch.complex64, self.device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        handle = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        if self.nz > 1:
            _check(self.lib.gpjc_plan_create_3d(ctypes.byref(g), self.nz,
                                                self.mask.ctypes.data_as(ctypes.c_void_p), _ptr(c), _ptr(p),
                                                ctypes.c_void_p(st), ctypes.byref(handle)))
        else:
            create = self.lib.gpjc_plan_create_bmap if self.general else self.lib.gpjc_plan_create
            _check(create(ctypes.byref(g), _ptr(c), _ptr(p), ctypes.c_void_p(st), ctypes.byref(handle)))
        self.handle = handle
        self._inputs = []

    @classmethod
    def from_slice(cls, sl, batch=1, compressed=True, **kw):
        g = sl.geom
        return cls(g.nx, g.ny, g.nc, g.os, sl.coils, sl.psf, g.mask, g.patch_len, g.patch_group, g.n_groups,
                   g.k, batch=batch, compressed=compressed, **kw)

    @classmethod
    def from_volume(cls, v, batch=1, compressed=True, **kw):
        """A plan for a 3D volume (synth.Volume)."""
        g = v.geom
        return cls(g.nx, g.ny, g.nc, g.os, v.coils, v.psf, v.mask2, g.patch_len, g.patch_group, g.n_groups, g.k,
                   batch=batch, compressed=compressed, nz=v.nz, **kw)

    @classmethod
    def from_map_slice(cls, sl, batch=1, **kw):
        """A plan for a slice with a general modulation map (synth.MapSlice)."""
        g = sl.geom
        return cls(g.nx, g.ny, g.nc, g.os, sl.coils, None, g.mask, g.patch_len, g.patch_group, g.n_groups, g.k,
                   batch=batch, compressed=True, bmod=sl.bmod, **kw)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gpjc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- shapes ----
    @property
    def ns(self):
        return self.nc * self.patch_len

    def data_shape(self):
        if self.compressed:
            return (self.batch, self.np_, self.k, self.ms)
        return (self.batch, self.nc, self.ms, self.nt)

    def image_shape(self):
        if self.nz > 1:
            return (self.batch, self.nz, self.ny, self.nx)
        return (self.batch, self.ny, self.nx)

    def _empty(self, shape, dtype=torch.complex64):
        return torch.empty(shape, dtype=dtype, device=self.device)

    def _in(self, t: torch.Tensor, dtype=torch.complex64):
        """Pointer to an input, made contiguous on the plan's device; the
        tensor is kept referenced until the next call so a temporary copy
        outlives the queued work."""
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.ascontiguousarray(t))
        t = _materialise(t.to(device=self.device, dtype=dtype))
        self._inputs.append(t)
        return ctypes.c_void_p(t.data_ptr())

    def _begin(self):
        self._inputs = []

    # ---- calls ----
    def set_stream(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib.gpjc_set_stream(self.handle, ctypes.c_void_p(st)))

    def calibrate(self, roi=None, noise_cov=None, want_eigvals=False, want_bank=False):
        roi_t = None if roi is None else _dev_tensor(np.asarray(roi, np.uint8), torch.uint8, self.device)
        cov_t = None if noise_cov is None else _dev_tensor(noise_cov, torch.complex64, self.device)
        eig = np.zeros((self.n_groups, self.ns), np.float64) if want_eigvals else None
        bank = self._empty((self.n_groups, self.k, self.nc, self.patch_len), torch.complex128) if want_bank else None
        _check(self.lib.gpjc_calibrate(self.handle, _ptr(roi_t), _ptr(cov_t),
                                       None if eig is None else eig.ctypes.data_as(ctypes.c_void_p),
                                       _ptr(bank)))
        return eig, bank

    def calibrate_static(self, roi=None, noise_cov=None, want_eigvals=False, want_bank=False):
        """calibrate() through gpjc_calibrate_static: the workspaces live in
        the library's static device scratch, nothing is allocated."""
        roi_t = None if roi is None else _dev_tensor(np.asarray(roi, np.uint8), torch.uint8, self.device)
        cov_t = None if noise_cov is None else _dev_tensor(noise_cov, torch.complex64, self.device)
        eig = np.zeros((self.n_groups, self.ns), np.float64) if want_eigvals else None
        bank = self._empty((self.n_groups, self.k, self.nc, self.patch_len), torch.complex128) if want_bank else None
        _check(self.lib.gpjc_calibrate_static(self.handle, _ptr(roi_t), _ptr(cov_t),
                                              None if eig is None else eig.ctypes.data_as(ctypes.c_void_p),
                                              _ptr(bank)))
        return eig, bank

    def set_compression(self, bank):
        self._begin()
        _check(self.lib.gpjc_set_compression(self.handle, self._in(bank, torch.complex128)))

    def compress(self, ksp, out=None):
        self._begin()
        out = self._empty((self.batch, self.np_, self.k, self.ms)) if out is None else out
        _check(self.lib.gpjc_compress(self.handle, self._in(ksp), _ptr(out)))
        return out

    def forward(self, img, prec="fp32", out=None):
        out = self._empty(self.data_shape()) if out is None else out
        self._begin()
        _check(self.lib.gpjc_forward(self.handle, _prec(prec), self._in(img), _ptr(out)))
        return out

    def adjoint(self, y, prec="fp32", out=None):
        out = self._empty(self.image_shape()) if out is None else out
        self._begin()
        _check(self.lib.gpjc_adjoint(self.handle, _prec(prec), self._in(y), _ptr(out)))
        return out

    def normal(self, img, prec="fp32", out=None):
        out = self._empty(self.image_shape()) if out is None else out
        self._begin()
        _check(self.lib.gpjc_normal(self.handle, _prec(prec), self._in(img), _ptr(out)))
        return out

    def recon_cg(self, y, iters, x0=None, prec="fp32", refine_every=0, want_resid=False):
        x = torch.zeros(self.image_shape(), dtype=torch.complex64, device=self.device) if x0 is None \
            else x0.clone().contiguous()
        hist = np.zeros(iters + 1, np.float64) if want_resid else None
        self._begin()
        _check(self.lib.gpjc_recon_cg(self.handle, _prec(prec), self._in(y), _ptr(x), int(iters), int(refine_every),
                                      None if hist is None else hist.ctypes.data_as(ctypes.c_void_p)))
        return (x, hist) if want_resid else x

    def recon_fista(self, y, iters, lam, lipschitz, levels=3, prec="fp32", out=None, want_obj=False):
        """FISTA-L1; with want_obj also the objective after every iteration
        (returns (x, objectives))."""
        x = self._empty(self.image_shape()) if out is None else out
        obj = np.zeros(int(iters), np.float64) if want_obj else None
        self._begin()
        _check(self.lib.gpjc_recon_fista(self.handle, _prec(prec), self._in(y), _ptr(x), int(iters), float(lam),
                                         float(lipschitz), int(levels),
                                         None if obj is None else obj.ctypes.data_as(ctypes.c_void_p)))
        return (x, obj) if want_obj else x

    def recon_fista_tv(self, y, iters, lam, lam_tv, tv_eps, lipschitz, levels=3, prec="fp32", out=None,
                       want_obj=False):
        """FISTA on Eq. 17 with the smoothed TV term (gpjc_recon_fista_tv)."""
        x = self._empty(self.image_shape()) if out is None else out
        obj = np.zeros(int(iters), np.float64) if want_obj else None
        self._begin()
        _check(self.lib.gpjc_recon_fista_tv(self.handle, _prec(prec), self._in(y), _ptr(x), int(iters), float(lam),
                                            float(lam_tv), float(tv_eps), float(lipschitz), int(levels),
                                            None if obj is None else obj.ctypes.data_as(ctypes.c_void_p)))
        return (x, obj) if want_obj else x

    def recon_lsqr(self, y, iters, prec="fp32", want_resid=False):
        """Reconstruction algorithm #1: LSQR over the aliased sets of a regular
        mask; returns the image (and the residual norm per iteration)."""
        x = self._empty(self.image_shape())
        hist = np.zeros(int(iters) + 1, np.float64) if want_resid else None
        self._begin()
        _check(self.lib.gpjc_recon_lsqr(self.handle, _prec(prec), self._in(y), _ptr(x), int(iters),
                                        None if hist is None else hist.ctypes.data_as(ctypes.c_void_p)))
        return (x, hist) if want_resid else x

    def power_iteration(self, x0, iters=50, prec="fp32"):
        self._begin()
        lam = ctypes.c_double()
        _check(self.lib.gpjc_power_iteration(self.handle, _prec(prec), self._in(x0), int(iters), ctypes.byref(lam)))
        return lam.value

    def wavelet_absmax(self, img, levels=3):
        self._begin()
        out = ctypes.c_double()
        _check(self.lib.gpjc_wavelet_absmax(self.handle, self._in(img), int(levels), ctypes.byref(out)))
        return out.value

    def stage_timing(self, enable=True, stages=None):
        """Bracket stage launches with HIP events: all stages, or only the
        named ones (names from STAGES) when `stages` is given."""
        if stages is None:
            _check(self.lib.gpjc_stage_timing(self.handle, int(bool(enable))))
            return
        mask = 0
        for name in stages:
            mask |= 1 << STAGES.index(name)
        _check(self.lib.gpjc_stage_timing_select(self.handle, mask if enable else 0))

    def stage_times(self):
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int * len(STAGES))()
        _check(self.lib.gpjc_stage_times(self.handle, ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}

    def set_gemm_config(self, compress_variant, expand_variant, ksplit, prec="fp32"):
        _check(self.lib.gpjc_set_gemm_config(self.handle, _prec(prec), int(compress_variant), int(expand_variant),
                                             int(ksplit)))

    def gemm_config(self, prec="fp32"):
        v = [ctypes.c_int() for _ in range(5)]
        _check(self.lib.gpjc_get_gemm_config(self.handle, _prec(prec), *[ctypes.byref(x) for x in v]))
        return {"compress": v[0].value, "expand": v[1].value, "ksplit": v[2].value,
                "n_compress": v[3].value, "n_expand": v[4].value}

    def gd_step(self, x, b, alpha, prec="fp32", want_residual=True):
        """x - alpha (E'^H E' x - b) and the residual E'^H E' x - b; alpha is a
        one-element float32 device tensor."""
        self._begin()
        xo = self._empty(self.image_shape())
        r = self._empty(self.image_shape()) if want_residual else None
        _check(self.lib.gpjc_gd_step(self.handle, _prec(prec), self._in(x), self._in(b),
                                     self._in(alpha, torch.float32), _ptr(xo), _ptr(r)))
        return xo, r

    def gd_step_backward(self, g, alpha, r, prec="fp32", want_gx=True, want_gb=True):
        """(dL/dx, dL/db, dL/dalpha) of gd_step for upstream gradient g."""
        self._begin()
        gx = self._empty(self.image_shape()) if want_gx else None
        gb = self._empty(self.image_shape()) if want_gb else None
        ga = torch.empty((), dtype=torch.float32, device=self.device)
        _check(self.lib.gpjc_gd_step_backward(self.handle, _prec(prec), self._in(g), self._in(alpha, torch.float32),
                                              self._in(r), _ptr(gx), _ptr(gb), _ptr(ga)))
        return gx, gb, ga

    def autotune(self, prec="fp32", cache_path=None):
        """Times the contraction tile shapes on this plan and installs the
        fastest; returns the choice and whether the bucket came from the cache."""
        ch = (ctypes.c_int * 4)()
        path = None if cache_path is None else os.fsencode(cache_path)
        torch.cuda.synchronize(self.device)
        _check(self.lib.gpjc_autotune(self.handle, _prec(prec), path, ch))
        return {"compress": ch[0], "expand": ch[1], "ksplit": ch[2], "cached": bool(ch[3])}


class Batch:
    """Independent slices (one Plan each, any geometries) reconstructed
    together: one captured HIP graph replays a CG iteration of every slice."""

    def __init__(self, plans, lanes=0):
        self.lib = load()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        handle = ctypes.c_void_p()
        _check(self.lib.gpjc_batch_create(arr, len(self.plans), int(lanes), ctypes.byref(handle)))
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gpjc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lanes(self):
        lane_of = (ctypes.c_int * len(self.plans))()
        n = self.lib.gpjc_batch_lanes(self.handle, lane_of)
        if n < 0:
            _check(n)
        return n, list(lane_of)

    def recon_cg(self, ys, iters, xs=None, prec="fp32", refine_every=0, want_resid=False):
        """ys: one data tensor per slice (the plan's data_shape()); xs: initial
        images (copied) or None for zeros.  Returns the images (and residual
        histories [n][iters+1])."""
        n = len(self.plans)
        if len(ys) != n or (xs is not None and len(xs) != n):
            raise ValueError("one input per slice")
        yin, xout = [], []
        for i, p in enumerate(self.plans):
            yin.append(_dev_tensor(ys[i], torch.complex64, p.device))
            x = torch.zeros(p.image_shape(), dtype=torch.complex64, device=p.device) if xs is None \
                else _dev_tensor(xs[i], torch.complex64, p.device).clone()
            xout.append(x)
        ya = (ctypes.c_void_p * n)(*[t.data_ptr() for t in yin])
        xa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xout])
        hist = np.zeros((n, iters + 1), np.float64) if want_resid else None
        torch.cuda.synchronize()
        _check(self.lib.gpjc_batch_recon_cg(self.handle, _prec(prec), ya, xa, int(iters), int(refine_every),
                                            None if hist is None else hist.ctypes.data_as(ctypes.c_void_p)))
        return (xout, hist) if want_resid else xout

    def autotune(self, prec="fp32", cache_path=None):
        path = None if cache_path is None else os.fsencode(cache_path)
        torch.cuda.synchronize()
        _check(self.lib.gpjc_batch_autotune(self.handle, _prec(prec), path))

