"""octmc: orthogonal-raster OCT/OCTA 3-D motion correction on MI355X (gfx950).

Thin ctypes binding of the C ABI in include/octmc.h (liboctmc.so, built
in-tree by paper_2010_06931_amd.build).  The binding only marshals arguments:
every step of the registration runs in the library's HIP kernels.  PyTorch
supplies device memory and streams.  There is no fallback: if the library is
missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboctmc.so")

F32, BF16, F16 = 0, 1, 2
_DTYPES = {"f32": F32, "float32": F32, "bf16": BF16, "bfloat16": BF16, "f16": F16, "float16": F16}
MEM_HOST, MEM_DEVICE = 0, 1
CHECK_NAN = 0x1
DETECT_INVALID = 0x2
ENFACE_PROJECT = 0x4
PREALIGN = 0x8
MULTI_PAIRWISE = 0x10
HOST_LINE_SEARCH = 0x20
MAX_LEVELS = 8

TERM_F, TERM_DATA, TERM_STR, TERM_ANG, TERM_REG, TERM_MEAN, TERM_STR05, TERM_ANG05, TERM_ETA, TERM_GP = range(10)
NTERMS = 10
TERM_NAMES = ("F", "data", "str", "ang", "reg", "mean", "str05", "ang05", "eta", "gp")

STATUS = {0: "OK", -1: "E_INVALID", -2: "E_SHAPE", -3: "E_DTYPE", -4: "E_OOM", -5: "E_DEVICE", -6: "E_NAN",
          -7: "E_BUSY"}

# exported symbols of include/octmc.h (checked by the CPU test suite)
SYMBOLS = ("octmc_version", "octmc_last_error", "octmc_params_default", "octmc_create", "octmc_destroy",
           "octmc_pair_create", "octmc_pair_destroy", "octmc_pair_levels", "octmc_pair_level_shape",
           "octmc_validity_from_octa", "octmc_enface_project", "octmc_enface_workspace_size", "octmc_prealign_eval",
           "octmc_prealign",
           "octmc_pair_prealignment", "octmc_resample_axial", "octmc_multi_create", "octmc_multi_destroy",
           "octmc_multi_eval", "octmc_multi_register", "octmc_eval",
           "octmc_eval_profile", "octmc_eval_batched", "octmc_eval_noalloc", "octmc_register", "octmc_merge",
           "octmc_request_footprint", "octmc_server_create", "octmc_server_submit", "octmc_server_poll",
           "octmc_server_status", "octmc_server_destroy")
SERVE_GROUPED, SERVE_STREAMS = 0, 1


class Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("delta0", C.c_double), ("eps_huber", C.c_double),
                ("eps_reg", C.c_double), ("flyback_frac", C.c_double), ("mean_weight", C.c_double),
                ("levels", C.c_int32), ("iters_per_level", C.c_int32), ("lbfgs_m", C.c_int32),
                ("ls_max_evals", C.c_int32), ("c1", C.c_double), ("c2", C.c_double),
                ("merge_kappa", C.c_double), ("merge_tau", C.c_double), ("flags", C.c_uint32),
                ("prealign_iters", C.c_int32), ("gamma_tilt", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Shape(C.Structure):
    _fields_ = [("w", C.c_int32), ("h", C.c_int32), ("d", C.c_int32), ("dtype", C.c_int), ("mem", C.c_int)]


class Report(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("iters", C.c_int32 * MAX_LEVELS), ("evals", C.c_int32 * MAX_LEVELS),
                ("ls_fail", C.c_int32 * MAX_LEVELS), ("eta", C.c_double * MAX_LEVELS),
                ("f_start", C.c_double * MAX_LEVELS), ("f_end", C.c_double * MAX_LEVELS)]

    def as_list(self):
        n = self.nlevels
        return [dict(iters=self.iters[k], evals=self.evals[k], ls_fail=self.ls_fail[k], eta=self.eta[k],
                     f_start=self.f_start[k], f_end=self.f_end[k]) for k in range(n)]


class Request(C.Structure):
    _fields_ = [("params", Params), ("shape", Shape)] + \
               [(n, C.c_void_p) for n in ("oct_x", "oct_y", "octa_x", "octa_y", "enface_x", "enface_y", "valid_x",
                                          "valid_y", "disp_out", "merged_oct", "merged_octa")] + \
               [("tag", C.c_uint64)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("bytes_reserved", C.c_uint64), ("bytes_used", C.c_uint64), ("report", Report),
                ("error", C.c_char * 160)]

    def as_dict(self):
        return dict(id=self.id, tag=self.tag, status=self.status, t_submit=self.t_submit, t_admit=self.t_admit,
                    t_done=self.t_done, bytes_reserved=self.bytes_reserved, bytes_used=self.bytes_used,
                    report=self.report.as_list(), error=self.error.decode(errors="replace"))


class OctmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"octmc {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded liboctmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_06931_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.octmc_version.restype = C.c_char_p
        L.octmc_last_error.restype = C.c_char_p
        L.octmc_params_default.argtypes = [C.POINTER(Params)]
        L.octmc_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.octmc_destroy.argtypes = [vp]
        L.octmc_pair_create.argtypes = [vp, C.POINTER(Params), C.POINTER(Shape)] + [vp] * 8 + [vp, C.POINTER(vp)]
        L.octmc_pair_destroy.argtypes = [vp]
        L.octmc_pair_level_shape.argtypes = [vp, C.c_int32] + [C.POINTER(C.c_int32)] * 3
        L.octmc_pair_levels.argtypes = [vp, C.POINTER(C.c_int32)]
        L.octmc_validity_from_octa.argtypes = [vp, C.POINTER(Shape), vp, C.c_int32, vp, vp]
        L.octmc_enface_project.argtypes = [vp, C.POINTER(Shape), vp, vp, C.c_int32, vp, C.POINTER(C.c_double), vp, vp,
                                           C.POINTER(C.c_double), vp, C.c_uint64, vp]
        L.octmc_enface_workspace_size.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_uint64)]
        dpp = C.POINTER(C.c_double)
        L.octmc_prealign_eval.argtypes = [vp, C.c_int32, dpp, C.c_double, dpp, dpp, dpp, vp]
        L.octmc_prealign.argtypes = [vp, C.c_double, C.c_int32, dpp, C.POINTER(Report), vp]
        L.octmc_pair_prealignment.argtypes = [vp, dpp, vp, vp]
        L.octmc_resample_axial.argtypes = [vp, C.POINTER(Shape), vp, vp, vp, vp]
        L.octmc_multi_create.argtypes = [vp, C.POINTER(Params), C.POINTER(Shape), C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp,
                                         C.POINTER(vp)]
        L.octmc_multi_destroy.argtypes = [vp]
        L.octmc_multi_eval.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32, vp]
        L.octmc_multi_register.argtypes = [vp, vp, vp, vp, C.POINTER(Report), vp]
        L.octmc_eval.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32, vp]
        L.octmc_eval_profile.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32, C.POINTER(C.c_float), vp]
        L.octmc_eval_batched.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, vp, vp, vp, C.c_int32, vp]
        L.octmc_eval_noalloc.argtypes = [vp, C.POINTER(Params), C.POINTER(Shape)] + [vp] * 10 + [C.c_int32, vp]
        L.octmc_register.argtypes = [vp, vp, vp, vp, C.POINTER(Report), vp]
        L.octmc_merge.argtypes = [vp, vp, vp, vp, vp]
        L.octmc_request_footprint.argtypes = [C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.octmc_server_create.argtypes = [vp, C.c_uint64, C.c_int32, C.c_int32, C.POINTER(vp)]
        L.octmc_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.octmc_server_poll.argtypes = [vp, C.POINTER(Completion), C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
        L.octmc_server_status.argtypes = [vp] + [C.POINTER(C.c_int32)] * 3
        L.octmc_server_destroy.argtypes = [vp]
        for name in SYMBOLS:
            if name not in ("octmc_version", "octmc_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise OctmcError(rc, lib().octmc_last_error().decode())


def version() -> str:
    return lib().octmc_version().decode()


def default_params(**overrides) -> Params:
    p = Params()
    _check(lib().octmc_params_default(C.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _f32(t, device):
    if t is None:
        return None
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=torch.float32).contiguous()


class Context:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0):
        self.device = device
        self._h = C.c_void_p()
        _check(lib().octmc_create(device, C.byref(self._h)))

    def close(self):
        if self._h:
            lib().octmc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


_default_ctx = {}


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def eval_noalloc(sx, sy, ax, ay, vx, vy, disp, eta, terms, grad=None, *, dtype: str = "f32",
                 params: Params | None = None, eta_mode: int = 1, ctx: Context | None = None, stream=None):
    """octmc_eval_noalloc: one evaluation on caller-owned device tensors with
    the library's static scratch; neither this wrapper nor the library
    allocates device memory.  sx, sy [h][w][d] in the storage type (float32,
    bfloat16 or float16 tensors), ax, ay [h][w], vx [h], vy [w], disp and
    grad [2][h][w][3] float32, eta float64[1] (written for eta_mode 0, read
    for 1), terms float64[NTERMS]."""
    ctx = ctx or context(0)
    h, w, d = sx.shape
    want = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    for t in (sx, sy):
        if t.dtype != want or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (h, w, d):
            raise ValueError(f"volumes must be contiguous {want} cuda tensors of one shape")
    prm = params if params is not None else default_params()
    shape = Shape(w, h, d, _DTYPES[dtype], MEM_DEVICE)
    _check(lib().octmc_eval_noalloc(ctx._h, C.byref(prm), C.byref(shape), _ptr(sx), _ptr(sy), _ptr(ax), _ptr(ay),
                                    _ptr(vx), _ptr(vy), _ptr(disp), _ptr(eta), _ptr(terms), _ptr(grad), eta_mode,
                                    _stream(stream)))
    return terms, grad


class Pair:
    """One orthogonal scan pair resident on the GPU (pyramid of every input).

    sx, sy: structural volumes [h][w][d]; ox, oy: OCTA volumes (optional);
    ax, ay: en face images [h][w] (optional if ox, oy are given); vx[h], vy[w]:
    B-scan validity (optional).  Tensors may live on the host or on the device;
    the library copies them."""

    def __init__(self, sx, sy, *, ox=None, oy=None, ax=None, ay=None, vx=None, vy=None, params: Params | None = None,
                 dtype: str = "f32", ctx: Context | None = None, stream=None, detect_invalid: bool = False,
                 project_enface: bool = False, prealign: bool = False, host_line_search: bool = False,
                 **param_overrides):
        self.ctx = ctx or context(0)
        dev = torch.device("cuda", self.ctx.device)
        self.params = params if params is not None else default_params()
        for k, v in param_overrides.items():
            setattr(self.params, k, v)
        if detect_invalid:  # validity from the OCTA volumes (Sec. 2.2) when vx, vy are not given
            self.params.flags |= DETECT_INVALID
        if project_enface:  # en face images by the projection of Sec. 2.3 when ax, ay are not given
            self.params.flags |= ENFACE_PROJECT
        if prealign:  # stage-1 rough axial prealignment before ingest
            self.params.flags |= PREALIGN
        if host_line_search:  # L-BFGS decisions on the host (the device form gives the same bits)
            self.params.flags |= HOST_LINE_SEARCH
        sx, sy = _f32(sx, dev), _f32(sy, dev)
        h, w, d = sx.shape
        if sy.shape != sx.shape:
            raise ValueError("sx and sy differ in shape")
        self.shape = Shape(w, h, d, _DTYPES[dtype], MEM_DEVICE)
        self.dtype = dtype
        ins = [sx, sy, _f32(ox, dev), _f32(oy, dev), _f32(ax, dev), _f32(ay, dev), _f32(vx, dev), _f32(vy, dev)]
        self._h = C.c_void_p()
        _check(lib().octmc_pair_create(self.ctx._h, C.byref(self.params), C.byref(self.shape),
                                       *[_ptr(t) for t in ins], _stream(stream), C.byref(self._h)))
        self.has_octa = ox is not None

    @property
    def levels(self) -> int:
        """Pyramid levels the pair holds (resolved when created with levels=0)."""
        n = C.c_int32()
        _check(lib().octmc_pair_levels(self._h, C.byref(n)))
        return n.value

    def level_shape(self, level: int):
        w, h, d = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().octmc_pair_level_shape(self._h, level, C.byref(w), C.byref(h), C.byref(d)))
        return w.value, h.value, d.value

    def eval(self, level: int, disp: torch.Tensor, *, grad: bool | torch.Tensor = True, terms=None,
             eta_mode: int = 1, stream=None):
        """Objective terms (float64[NTERMS], device) and gradient (like disp)."""
        w, h, d = self.level_shape(level)
        if disp.shape != (2, h, w, 3) or disp.dtype != torch.float32 or not disp.is_cuda:
            raise ValueError(f"disp must be a float32 cuda tensor of shape (2, {h}, {w}, 3)")
        disp = disp.contiguous()
        if terms is None:
            terms = torch.empty(NTERMS, dtype=torch.float64, device=disp.device)
        g = None
        if grad is True:
            g = torch.empty_like(disp)
        elif isinstance(grad, torch.Tensor):
            g = grad
        _check(lib().octmc_eval(self._h, level, _ptr(disp), _ptr(terms), _ptr(g), eta_mode, _stream(stream)))
        return terms, g

    def eval_profile(self, level: int, disp: torch.Tensor, *, grad: torch.Tensor | None = None, terms=None,
                     eta_mode: int = 1, stream=None):
        """octmc_eval with HIP events between its kernels; returns the stage
        times in ms: (displacement sum, structural kernel, combine)."""
        if terms is None:
            terms = torch.empty(NTERMS, dtype=torch.float64, device=disp.device)
        ms = (C.c_float * 3)()
        _check(lib().octmc_eval_profile(self._h, level, _ptr(disp), _ptr(terms), _ptr(grad), eta_mode, ms,
                                        _stream(stream)))
        return list(ms)

    def prealign_eval(self, level: int, theta, gamma_tilt: float = 1.0, stream=None):
        """Stage-1 objective at level `level` and theta (2 (h + w) values):
        (terms dict, T, gradient with respect to theta as numpy float64)."""
        w, h, _ = self.level_shape(level)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).ravel())
        if th.size != 2 * (w + h):
            raise ValueError(f"theta needs {2 * (w + h)} values at level {level}")
        terms = np.zeros(NTERMS)
        g = np.zeros_like(th)
        T = C.c_double()
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        _check(lib().octmc_prealign_eval(self._h, level, dp(th), float(gamma_tilt), dp(terms), C.byref(T), dp(g),
                                         _stream(stream)))
        return dict(zip(TERM_NAMES, terms.tolist())), T.value, g

    def prealign(self, gamma_tilt: float = 1.0, iters_per_level: int = 100, stream=None):
        """The stage-1 solve on this pair's pyramid: theta at the finest level
        and the per-level report."""
        th = np.zeros(2 * (self.shape.w + self.shape.h))
        rep = Report()
        _check(lib().octmc_prealign(self._h, float(gamma_tilt), int(iters_per_level),
                                    th.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep), _stream(stream)))
        return th, rep.as_list()

    def prealignment(self, stream=None):
        """Stage-1 result of a pair created with prealign=True: theta (numpy)
        and the axial field dz [2][h][w] (device)."""
        th = np.zeros(2 * (self.shape.w + self.shape.h))
        dz = torch.empty((2, self.shape.h, self.shape.w), dtype=torch.float32,
                         device=torch.device("cuda", self.ctx.device))
        _check(lib().octmc_pair_prealignment(self._h, th.ctypes.data_as(C.POINTER(C.c_double)), _ptr(dz),
                                             _stream(stream)))
        return th, dz

    def register(self, *, merged: bool = False, stream=None):
        """Full solve.  Returns (disp [2][h][w][3], merged_oct or None,
        merged_octa or None, per-level report list)."""
        h, w, d = self.shape.h, self.shape.w, self.shape.d
        dev = torch.device("cuda", self.ctx.device)
        disp = torch.empty((2, h, w, 3), dtype=torch.float32, device=dev)
        mo = torch.empty((h, w, d), dtype=torch.float32, device=dev) if merged else None
        ma = torch.empty((h, w, d), dtype=torch.float32, device=dev) if (merged and self.has_octa) else None
        rep = Report()
        _check(lib().octmc_register(self._h, _ptr(disp), _ptr(mo), _ptr(ma), C.byref(rep), _stream(stream)))
        return disp, mo, ma, rep.as_list()

    def merge(self, disp: torch.Tensor, *, octa: bool = False, stream=None):
        h, w, d = self.shape.h, self.shape.w, self.shape.d
        mo = torch.empty((h, w, d), dtype=torch.float32, device=disp.device)
        ma = torch.empty((h, w, d), dtype=torch.float32, device=disp.device) if octa else None
        _check(lib().octmc_merge(self._h, _ptr(disp.contiguous()), _ptr(mo), _ptr(ma), _stream(stream)))
        return mo, ma

    def close(self):
        if getattr(self, "_h", None):
            lib().octmc_pair_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def validity_from_octa(vol: torch.Tensor, scan: int, *, ctx: Context | None = None, stream=None) -> torch.Tensor:
    """Input validity of one OCTA volume [h][w][d] (Sec. 2.2): one 0/1 value per
    B-scan, rows j for the X-fast scan (scan 0), columns i for the Y-fast scan
    (scan 1)."""
    ctx = ctx or context(0)
    dev = torch.device("cuda", ctx.device)
    vol = _f32(vol, dev)
    h, w, d = vol.shape
    out = torch.empty(h if scan == 0 else w, dtype=torch.float32, device=dev)
    shape = Shape(w, h, d, F32, MEM_DEVICE)
    _check(lib().octmc_validity_from_octa(ctx._h, C.byref(shape), _ptr(vol), int(scan), _ptr(out), _stream(stream)))
    return out


class Multi:
    """n >= 2 raster scans registered jointly (two-volume terms over all
    pairs).  vols: structural volumes [h][w][d]; orients: 0 (X-fast) or 1
    (Y-fast) per volume; octa, enface, valid: lists of n or None.
    pairwise=True evaluates the structural term pair by pair instead of the
    fused pass that resamples each volume once (n = 3 or 4)."""

    def __init__(self, vols, orients, *, octa=None, enface=None, valid=None, params: Params | None = None,
                 dtype: str = "f32", ctx: Context | None = None, stream=None, detect_invalid: bool = False,
                 project_enface: bool = False, pairwise: bool = False, host_line_search: bool = False,
                 **param_overrides):
        self.ctx = ctx or context(0)
        dev = torch.device("cuda", self.ctx.device)
        self.params = params if params is not None else default_params()
        for k, v in param_overrides.items():
            setattr(self.params, k, v)
        if detect_invalid:
            self.params.flags |= DETECT_INVALID
        if project_enface:
            self.params.flags |= ENFACE_PROJECT
        if pairwise:
            self.params.flags |= MULTI_PAIRWISE
        if host_line_search:  # L-BFGS decisions on the host (the device form gives the same bits)
            self.params.flags |= HOST_LINE_SEARCH
        n = len(vols)
        self._has_octa = octa is not None
        S = [_f32(v, dev) for v in vols]
        h, w, d = S[0].shape
        self.n = n
        self.shape = Shape(w, h, d, _DTYPES[dtype], MEM_DEVICE)
        lists = {}
        for name, lst in (("octa", octa), ("enface", enface), ("valid", valid)):
            lists[name] = None if lst is None else [_f32(x, dev) for x in lst]
        self._keep = (S, lists)
        arr = lambda ts: None if ts is None else (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        orient = (C.c_int32 * n)(*[int(o) for o in orients])
        self._h = C.c_void_p()
        _check(lib().octmc_multi_create(self.ctx._h, C.byref(self.params), C.byref(self.shape), n, orient, arr(S),
                                        arr(lists["octa"]), arr(lists["enface"]), arr(lists["valid"]),
                                        _stream(stream), C.byref(self._h)))
        self._keep = None  # the library copied the inputs

    def level_shape(self, level: int):
        w, h, d = self.shape.w, self.shape.h, self.shape.d
        for _ in range(level):
            w, h, d = (w + 1) // 2, (h + 1) // 2, (d + 1) // 2
        return w, h, d

    def eval(self, level: int, disp: torch.Tensor, *, grad: bool = True, eta_mode: int = 1, stream=None):
        """n-volume objective terms (float64[NTERMS], device) and gradient."""
        w, h, _ = self.level_shape(level)
        if disp.shape != (self.n, h, w, 3) or disp.dtype != torch.float32 or not disp.is_cuda:
            raise ValueError(f"disp must be a float32 cuda tensor of shape ({self.n}, {h}, {w}, 3)")
        disp = disp.contiguous()
        terms = torch.empty(NTERMS, dtype=torch.float64, device=disp.device)
        g = torch.empty_like(disp) if grad else None
        _check(lib().octmc_multi_eval(self._h, level, _ptr(disp), _ptr(terms), _ptr(g), eta_mode, _stream(stream)))
        return terms, g

    def register(self, *, merged: bool = False, stream=None):
        """Joint solve: (disp [n][h][w][3], merged_oct or None, merged_octa or None, report)."""
        h, w, d = self.shape.h, self.shape.w, self.shape.d
        dev = torch.device("cuda", self.ctx.device)
        disp = torch.empty((self.n, h, w, 3), dtype=torch.float32, device=dev)
        mo = torch.empty((h, w, d), dtype=torch.float32, device=dev) if merged else None
        ma = torch.empty_like(mo) if merged and self._has_octa else None
        rep = Report()
        _check(lib().octmc_multi_register(self._h, _ptr(disp), _ptr(mo), _ptr(ma), C.byref(rep), _stream(stream)))
        return disp, mo, ma, rep.as_list()

    def close(self):
        if getattr(self, "_h", None):
            lib().octmc_multi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def resample_axial(vol: torch.Tensor, dz: torch.Tensor, *, ctx: Context | None = None, stream=None) -> torch.Tensor:
    """vol [h][w][d] resampled along depth by the per-A-scan field dz [h][w]
    (Catmull-Rom, clamped): out(i, j, k) = vol(i, j, k + dz(i, j))."""
    ctx = ctx or context(0)
    dev = torch.device("cuda", ctx.device)
    v, z = _f32(vol, dev), _f32(dz, dev)
    h, w, d = v.shape
    if z.shape != (h, w):
        raise ValueError("dz must be [h][w]")
    out = torch.empty_like(v)
    shape = Shape(w, h, d, F32, MEM_DEVICE)
    _check(lib().octmc_resample_axial(ctx._h, C.byref(shape), _ptr(v), _ptr(z), _ptr(out), _stream(stream)))
    return out


def enface_workspace_size(w: int, h: int, d: int) -> int:
    n = C.c_uint64()
    _check(lib().octmc_enface_workspace_size(int(w), int(h), int(d), C.byref(n)))
    return n.value


def enface_project(oct_vol: torch.Tensor, octa_vol: torch.Tensor, scan: int, valid: torch.Tensor | None = None, *,
                   fixed=None, details: bool = False, workspace: torch.Tensor | None = None, out=None,
                   ctx: Context | None = None, stream=None):
    """Segmentation-free en face projection (Sec. 2.3) of one scan: float32
    [h][w] on the device.  oct_vol, octa_vol: [h][w][d]; valid: one value per
    B-scan (rows for scan 0, columns for scan 1) or None; fixed: (p5, p95) in
    place of the percentiles.  With details=True also returns the per-A-scan
    voxel counts (int32 [h][w]) and (p5, p95, threshold, OCT threshold).
    workspace: a device tensor of at least enface_workspace_size bytes; with
    it (and details=False) the call is asynchronous on the stream."""
    ctx = ctx or context(0)
    dev = torch.device("cuda", ctx.device)
    o, a = _f32(oct_vol, dev), _f32(octa_vol, dev)
    if o.dim() != 3 or o.shape != a.shape:
        raise ValueError("oct_vol and octa_vol must be [h][w][d] volumes of one shape")
    h, w, d = a.shape
    v = _f32(valid, dev)
    if v is not None and v.numel() != (h if scan == 0 else w):
        raise ValueError("valid needs one value per B-scan")
    if out is None:
        out = torch.empty((h, w), dtype=torch.float32, device=dev)
    elif out.shape != (h, w) or out.dtype != torch.float32 or out.device != dev or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [h][w] tensor on the context's device")
    cnt = torch.empty((h, w), dtype=torch.int32, device=dev) if details else None
    stats = (C.c_double * 4)() if details else None
    fx = None if fixed is None else (C.c_double * 2)(float(fixed[0]), float(fixed[1]))
    shape = Shape(w, h, d, F32, MEM_DEVICE)
    wb = 0 if workspace is None else workspace.numel() * workspace.element_size()
    if workspace is not None and (not workspace.is_cuda or not workspace.is_contiguous()):
        raise ValueError("workspace must be a contiguous device tensor")
    _check(lib().octmc_enface_project(ctx._h, C.byref(shape), _ptr(o), _ptr(a), int(scan), _ptr(v), fx, _ptr(out),
                                      _ptr(cnt), stats, _ptr(workspace), wb, _stream(stream)))
    return (out, cnt, tuple(stats)) if details else out


def eval_batched(pairs, level: int, disp: torch.Tensor, *, grad: bool = True, eta_mode: int = 1, stream=None):
    """One grouped evaluation over pairs sharing the level shape.
    disp: [B][2][h][w][3] float32 cuda.  Returns terms [B][NTERMS], grad."""
    B = len(pairs)
    if B < 1:
        raise ValueError("need at least one pair")
    w, h, d = pairs[0].level_shape(level)
    if disp.shape != (B, 2, h, w, 3) or disp.dtype != torch.float32 or not disp.is_cuda:
        raise ValueError(f"disp must be a float32 cuda tensor of shape ({B}, 2, {h}, {w}, 3)")
    disp = disp.contiguous()
    terms = torch.empty((B, NTERMS), dtype=torch.float64, device=disp.device)
    g = torch.empty_like(disp) if grad else None
    arr = (C.c_void_p * B)(*[p._h for p in pairs])
    _check(lib().octmc_eval_batched(arr, B, level, _ptr(disp), _ptr(terms), _ptr(g), eta_mode, _stream(stream)))
    return terms, g


def terms_dict(terms: torch.Tensor) -> dict:
    t = terms.detach().cpu().tolist()
    return dict(zip(TERM_NAMES, t))


class OctmcObjective(torch.autograd.Function):
    """F(D) of B pairs as a differentiable function of their displacements.

    forward(D, pairs, level) evaluates the objective (Eq. 1 without the tilt
    term) of every pair in one grouped launch and returns F as float64 [B];
    the gradient the same launch computes (the hand-written adjoint of the
    resampling, loss and regulariser) is kept, and backward returns it scaled
    by the incoming dF.  eta of each pair's level is used as stored (Eq. 10
    fixes it per level; it carries no gradient): set it first with
    eval(..., eta_mode=0) or eval_batched(..., eta_mode=0).

        F = OctmcObjective.apply(D, pairs, level)   # D: [B][2][h][w][3] float32 cuda
        F.sum().backward()                           # D.grad = dF/dD
    """

    @staticmethod
    def forward(ctx, D, pairs, level):
        terms, g = eval_batched(list(pairs), int(level), D.detach(), grad=True, eta_mode=1)
        ctx.save_for_backward(g)
        return terms[:, TERM_F].clone()

    @staticmethod
    def backward(ctx, gF):
        (g,) = ctx.saved_tensors
        scale = gF.to(device=g.device, dtype=torch.float32).reshape(-1, *([1] * (g.dim() - 1)))
        return scale * g, None, None


def objective(D: torch.Tensor, pairs, level: int = 0) -> torch.Tensor:
    """F of every pair (float64 [B]), differentiable with respect to D."""
    return OctmcObjective.apply(D, tuple(pairs), level)


def register(x_oct, y_oct, x_octa=None, y_octa=None, *, enface_x=None, enface_y=None, valid_x=None, valid_y=None,
             params: Params | None = None, dtype: str = "f32", merged: bool = True, **param_overrides):
    """Register one orthogonal scan pair and merge it.

    x_oct, y_oct: structural volumes [h][w][d] in the common frame (the Y-fast
    scan transposed by the caller); x_octa, y_octa: OCTA volumes or None;
    enface_*: en face images [h][w] (needed when no OCTA volumes are given);
    valid_*: B-scan validity.  Returns (disp [2][h][w][3], merged_oct,
    merged_octa, per-level report)."""
    P = Pair(x_oct, y_oct, ox=x_octa, oy=y_octa, ax=enface_x, ay=enface_y, vx=valid_x, vy=valid_y, params=params,
             dtype=dtype, **param_overrides)
    try:
        return P.register(merged=merged)
    finally:
        P.close()


class Server:
    """Continuous-batching registration server on one device (see
    octmc_server_create).  Tensors passed to submit() are kept alive until
    their completion has been polled."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 8, mode: int = SERVE_STREAMS,
                 ctx: Context | None = None):
        self.ctx = ctx or context(0)
        self._h = C.c_void_p()
        _check(lib().octmc_server_create(self.ctx._h, int(hbm_budget_bytes), int(max_active), int(mode),
                                         C.byref(self._h)))
        self._keep = {}

    @staticmethod
    def _request(sx, sy, disp_out, *, ox=None, oy=None, ax=None, ay=None, vx=None, vy=None, merged_oct=None,
                 merged_octa=None, params: Params | None = None, dtype: str = "f32", tag: int = 0,
                 **param_overrides):
        dev = disp_out.device
        sx, sy = _f32(sx, dev), _f32(sy, dev)
        h, w, d = sx.shape
        if disp_out.shape != (2, h, w, 3) or disp_out.dtype != torch.float32 or not disp_out.is_cuda:
            raise ValueError(f"disp_out must be a float32 cuda tensor of shape (2, {h}, {w}, 3)")
        prm = params if params is not None else default_params()
        for k, v in param_overrides.items():
            setattr(prm, k, v)
        keep = [sx, sy, _f32(ox, dev), _f32(oy, dev), _f32(ax, dev), _f32(ay, dev), _f32(vx, dev), _f32(vy, dev),
                disp_out, merged_oct, merged_octa]
        r = Request()
        r.params = prm
        r.shape = Shape(w, h, d, _DTYPES[dtype], MEM_DEVICE)
        for name, t in zip(("oct_x", "oct_y", "octa_x", "octa_y", "enface_x", "enface_y", "valid_x", "valid_y",
                            "disp_out", "merged_oct", "merged_octa"), keep):
            setattr(r, name, None if t is None else t.data_ptr())
        r.tag = int(tag)
        return r, keep

    @staticmethod
    def footprint(sx, sy, disp_out, **kw) -> int:
        r, _ = Server._request(sx, sy, disp_out, **kw)
        b = C.c_uint64()
        _check(lib().octmc_request_footprint(C.byref(r), C.byref(b)))
        return b.value

    def submit(self, sx, sy, disp_out, **kw) -> int:
        """Queue one request (keywords as Pair plus disp_out / merged_oct /
        merged_octa device outputs and a tag); returns its id."""
        r, keep = self._request(sx, sy, disp_out, **kw)
        rid = C.c_uint64()
        torch.cuda.current_stream().synchronize()  # inputs written on torch's stream are complete
        _check(lib().octmc_server_submit(self._h, C.byref(r), C.byref(rid)))
        self._keep[rid.value] = keep
        return rid.value

    def poll(self, max_n: int = 64, wait_ms: int = 0):
        out = (Completion * max_n)()
        n = C.c_int32()
        _check(lib().octmc_server_poll(self._h, out, max_n, int(wait_ms), C.byref(n)))
        res = []
        for k in range(n.value):
            c = out[k].as_dict()
            self._keep.pop(c["id"], None)
            res.append(c)
        return res

    def status(self):
        q, a, d = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().octmc_server_status(self._h, C.byref(q), C.byref(a), C.byref(d)))
        return dict(queued=q.value, active=a.value, done=d.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().octmc_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
