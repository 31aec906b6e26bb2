"""Python access to the FP64 CPU oracle (oracle/octmc_oracle.c).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
baseline leg import this package.  The product path (paper_2010_06931_amd)
never imports it and shares no code with it.

Every array handed to the C code is converted to contiguous float64 first;
displacement fields are [2][h][w][3] (scan, row j, column i, (dx, dy, dz)).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "octmc_oracle.c")
_LIB = os.path.join(_HERE, "liboctmc_oracle.so")

T_F, T_DATA, T_STR, T_ANG, T_REG, T_MEAN, T_STR05, T_ANG05 = range(8)
TERM_NAMES = ("F", "data", "str", "ang", "reg", "mean", "str05", "ang05")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("delta0", C.c_double), ("eps_h", C.c_double),
                ("eps_r", C.c_double), ("flyback_frac", C.c_double), ("mean_weight", C.c_double),
                ("levels", C.c_int), ("iters", C.c_int), ("lbfgs_m", C.c_int), ("ls_max_evals", C.c_int),
                ("c1", C.c_double), ("c2", C.c_double), ("merge_kappa", C.c_double),
                ("merge_tau", C.c_double), ("store", C.c_int)]


@dataclass
class Params:
    alpha: float = 1.0
    delta0: float = 0.5
    eps_h: float = 1e-3
    eps_r: float = 0.1
    flyback_frac: float = 0.25
    mean_weight: float = 1.0
    levels: int = 3
    iters: int = 100
    lbfgs_m: int = 5
    ls_max_evals: int = 20
    c1: float = 1e-4
    c2: float = 0.9
    merge_kappa: float = 1.0
    merge_tau: float = 0.05
    store: int = 0  # structural storage in the solve: 0 exact, 1 bfloat16, 2 binary16

    def c(self) -> _Params:
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)})


class _Report(C.Structure):
    _fields_ = [("iters", C.c_int), ("evals", C.c_int), ("ls_fail", C.c_int), ("converged", C.c_int),
                ("f_start", C.c_double), ("f_end", C.c_double)]


_FG = C.CFUNCTYPE(C.c_int, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double))
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_hermite_taps.argtypes = [C.c_double, dp, dp]
        L.orc_sample1.argtypes = [dp, C.c_int, C.c_double, dp]
        L.orc_sample2.argtypes = [dp, C.c_int, C.c_int, C.c_double, C.c_double, dp]
        L.orc_sample3.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.orc_pseudo_huber.argtypes = [C.c_double, C.c_double, dp]
        L.orc_eval.argtypes = [dp] * 6 + [C.c_int] * 3 + [dp, C.POINTER(_Params), C.c_double, dp, dp]
        L.orc_eval.restype = C.c_int
        L.orc_data_ascans.argtypes = [dp] * 6 + [C.c_int] * 3 + [dp, C.POINTER(_Params), C.c_double,
                                                                C.POINTER(C.c_int64), C.c_int, dp, dp]
        L.orc_eta_from_terms.argtypes = [C.c_double, C.c_double]
        L.orc_eta_from_terms.restype = C.c_double
        L.orc_pyr_down3.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp]
        L.orc_pyr_down3_f32.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp]
        L.orc_pyr_down3_f32.restype = None
        L.orc_pyr_down2.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_pyr_down1.argtypes = [dp, C.c_int, dp]
        L.orc_upsample.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int, C.c_int]
        L.orc_lbfgs.argtypes = [C.c_int, dp, _FG, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_double, C.POINTER(_Report)]
        L.orc_lbfgs.restype = C.c_int
        L.orc_register.argtypes = [dp] * 6 + [C.c_int] * 3 + [C.POINTER(_Params), dp, dp]
        L.orc_register.restype = C.c_int
        L.orc_density.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_merge.argtypes = [dp] * 6 + [C.c_int] * 3 + [dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.orc_enface_mean.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp]
        L.orc_substitute_invalid.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, C.c_int]
        L.orc_median3.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp]
        L.orc_median3.restype = None
        L.orc_rank_line.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orc_rank_line.restype = None
        L.orc_quantile_valid.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_double]
        L.orc_quantile_valid.restype = C.c_double
        L.orc_enface_project.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp]
        L.orc_enface_project.restype = None
        L.orc_tilt_expand.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_tilt_expand.restype = None
        L.orc_tilt_reduce.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_tilt_reduce.restype = None
        L.orc_tilt_term.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_double, dp]
        L.orc_tilt_term.restype = C.c_double
        L.orc_prealign_eval.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, dp, C.POINTER(_Params), C.c_double, dp,
                                        dp]
        L.orc_prealign_eval.restype = C.c_double
        L.orc_tilt_upsample.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int, C.c_int]
        L.orc_tilt_upsample.restype = None
        L.orc_prealign.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.POINTER(_Params), C.c_double, C.c_int, dp,
                                   dp]
        L.orc_prealign.restype = C.c_int
        L.orc_resample_z.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_resample_z.restype = None
        dpp = C.POINTER(dp)
        ip = C.POINTER(C.c_int)
        L.orc_eval_multi.argtypes = [C.c_int, dpp, dpp, dpp, ip, C.c_int, C.c_int, C.c_int, dp,
                                     C.POINTER(_Params), dp, dp, dp, dp]
        L.orc_eval_multi.restype = C.c_int
        L.orc_upsample_multi.argtypes = [C.c_int, dp, C.c_int, C.c_int, dp, C.c_int, C.c_int]
        L.orc_upsample_multi.restype = None
        L.orc_register_multi.argtypes = [C.c_int, dpp, dpp, dpp, ip, C.c_int, C.c_int, C.c_int, C.POINTER(_Params),
                                         dp, dp]
        L.orc_register_multi.restype = C.c_int
        L.orc_merge_multi.argtypes = [C.c_int, dpp, dpp, dpp, ip, C.c_int, C.c_int, C.c_int, dp, C.c_double,
                                      C.c_double, dp, dp]
        L.orc_merge_multi.restype = None
        L.orc_validity.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orc_validity.restype = None
        L.orc_set_progress.argtypes = [C.c_int]
        L.orc_set_progress.restype = None
        L.orc_round_storage.argtypes = [dp, C.c_size_t, C.c_int]
        L.orc_round_storage.restype = None
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def set_progress(every: int) -> None:
    """Print the L-BFGS step count and objective to stderr every `every`
    accepted steps of any oracle solve (0: off).  Printing only."""
    lib().orc_set_progress(int(every))


def set_threads(n: int) -> int:
    """Host threads of the oracle's parallel loops (timing only; results do not
    depend on it).  Returns the count in effect."""
    return int(lib().orc_set_threads(int(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ----------------------------------------------------------------------------
# small building blocks

def hermite_taps(t: float):
    w = np.zeros(4)
    dw = np.zeros(4)
    lib().orc_hermite_taps(float(t), _p(w), _p(dw))
    return w, dw


def sample1(v, x: float):
    v = _f64(v)
    out = np.zeros(2)
    lib().orc_sample1(_p(v), v.shape[0], float(x), _p(out))
    return out


def sample2(img, x: float, y: float):
    img = _f64(img)
    out = np.zeros(3)
    lib().orc_sample2(_p(img), img.shape[1], img.shape[0], float(x), float(y), _p(out))
    return out


def sample3(vol, x: float, y: float, z: float):
    vol = _f64(vol)
    out = np.zeros(4)
    h, w, d = vol.shape
    lib().orc_sample3(_p(vol), w, h, d, float(x), float(y), float(z), _p(out))
    return out


def pseudo_huber(x: float, eps: float):
    out = np.zeros(2)
    lib().orc_pseudo_huber(float(x), float(eps), _p(out))
    return out


# ----------------------------------------------------------------------------
# objective

@dataclass
class Level:
    """One pyramid level of a pair, all float64 numpy arrays."""
    sx: np.ndarray
    sy: np.ndarray
    ax: np.ndarray
    ay: np.ndarray
    vx: np.ndarray
    vy: np.ndarray

    @property
    def whd(self):
        h, w, d = self.sx.shape
        return w, h, d


def level_from(sx, sy, ax, ay, vx=None, vy=None) -> Level:
    sx, sy, ax, ay = _f64(sx), _f64(sy), _f64(ax), _f64(ay)
    h, w, _ = sx.shape
    vx = np.ones(h) if vx is None else _f64(vx)
    vy = np.ones(w) if vy is None else _f64(vy)
    return Level(sx, sy, ax, ay, vx, vy)


def level_from_pair(pair) -> Level:
    return level_from(pair.sx, pair.sy, pair.ax, pair.ay, pair.vx, pair.vy)


def evaluate(lv: Level, D, params: Params | None = None, eta: float = 1.0, grad: bool = True):
    """Objective terms (dict) and gradient ([2][h][w][3] float64 or None)."""
    params = params or Params()
    D = _f64(D)
    w, h, d = lv.whd
    assert D.shape == (2, h, w, 3)
    terms = np.zeros(8)
    g = np.zeros_like(D) if grad else None
    pc = params.c()
    rc = lib().orc_eval(_p(lv.sx), _p(lv.sy), _p(lv.ax), _p(lv.ay), _p(lv.vx), _p(lv.vy), w, h, d,
                        _p(D), C.byref(pc), float(eta), _p(terms), _p(g) if grad else None)
    if rc:
        raise RuntimeError(f"orc_eval failed ({rc})")
    return dict(zip(TERM_NAMES, terms.tolist())), g


def data_ascans(lv: Level, D, ascans, params: Params | None = None, eta: float = 1.0):
    """Data term pieces and data gradient of selected A-scans (index j w + i):
    part [n][5] = (eta-weighted data, S_str, S_ang, S_str05, S_ang05 summands),
    grad [n][6] = (d/d d^X, d/d d^Y)."""
    params = params or Params()
    D = _f64(D)
    w, h, d = lv.whd
    lst = np.ascontiguousarray(ascans, dtype=np.int64)
    part = np.zeros((lst.size, 5))
    g = np.zeros((lst.size, 6))
    pc = params.c()
    lib().orc_data_ascans(_p(lv.sx), _p(lv.sy), _p(lv.ax), _p(lv.ay), _p(lv.vx), _p(lv.vy), w, h, d, _p(D),
                          C.byref(pc), float(eta), lst.ctypes.data_as(C.POINTER(C.c_int64)), lst.size,
                          _p(part), _p(g))
    return part, g


def eta_from_terms(s_str05: float, s_ang05: float) -> float:
    return lib().orc_eta_from_terms(float(s_str05), float(s_ang05))


def eta_at(lv: Level, D, params: Params | None = None) -> float:
    t, _ = evaluate(lv, D, params, 1.0, grad=False)
    return eta_from_terms(t["str05"], t["ang05"])


# ----------------------------------------------------------------------------
# pyramid, solve, merge

def pyr_down3(vol):
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2, (d + 1) // 2))
    lib().orc_pyr_down3(_p(vol), w, h, d, _p(out))
    return out


def pyr_down3_f32(vol):
    """The 2 x 2 x 2 box of pyr_down3 in single precision (depth, then x,
    then y), for pyramids rounded to a 16-bit storage type."""
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2, (d + 1) // 2))
    lib().orc_pyr_down3_f32(_p(vol), w, h, d, _p(out))
    return out


def pyr_down2(img):
    img = _f64(img)
    h, w = img.shape
    out = np.zeros(((h + 1) // 2, (w + 1) // 2))
    lib().orc_pyr_down2(_p(img), w, h, _p(out))
    return out


def pyr_down1(v):
    v = _f64(v)
    out = np.zeros((v.shape[0] + 1) // 2)
    lib().orc_pyr_down1(_p(v), v.shape[0], _p(out))
    return out


def pyramid(lv: Level, levels: int, store: int = 0):
    """Pyramid levels of a pair.  store = 1 (bfloat16) or 2 (binary16): the
    structural levels are built in single precision from the unrounded level
    above and each is then rounded to the storage type, as a solve with that
    storage sees them (level 0 included)."""
    down = pyr_down3_f32 if store else pyr_down3
    out = [lv]
    for _ in range(1, levels):
        p = out[-1]
        out.append(Level(down(p.sx), down(p.sy), pyr_down2(p.ax), pyr_down2(p.ay),
                         pyr_down1(p.vx), pyr_down1(p.vy)))
    if store:
        out = [Level(round_storage(q.sx, store), round_storage(q.sy, store), q.ax, q.ay, q.vx, q.vy) for q in out]
    return out


def upsample(Dc, wf: int, hf: int):
    Dc = _f64(Dc)
    _, hc, wc, _ = Dc.shape
    out = np.zeros((2, hf, wf, 3))
    lib().orc_upsample(_p(Dc), wc, hc, _p(out), wf, hf)
    return out


def lbfgs(fg, x0, m=5, max_iter=100, ls_max_evals=20, c1=1e-4, c2=0.9):
    """Minimise a Python objective fg(x) -> (f, g) with the oracle's L-BFGS."""
    x = _f64(x0).copy()
    n = x.size

    def cb(_ctx, xp, fp, gp):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            f, g = fg(xv)
            fp[0] = float(f)
            np.ctypeslib.as_array(gp, shape=(n,))[:] = np.asarray(g, dtype=np.float64).ravel()
            return 0
        except Exception:  # noqa: BLE001 - reported through the return code
            return 1

    cfun = _FG(cb)
    rep = _Report()
    rc = lib().orc_lbfgs(n, _p(x), cfun, None, m, max_iter, ls_max_evals, c1, c2, C.byref(rep))
    if rc:
        raise RuntimeError(f"orc_lbfgs failed ({rc})")
    return x, dict(iters=rep.iters, evals=rep.evals, ls_fail=rep.ls_fail, converged=rep.converged,
                   f_start=rep.f_start, f_end=rep.f_end)


def register(lv: Level, params: Params | None = None):
    """Full multi-resolution solve; returns D ([2][h][w][3]) and per-level
    reports (coarsest first)."""
    params = params or Params()
    w, h, d = lv.whd
    D = np.zeros((2, h, w, 3))
    rep = np.zeros((params.levels, 5))
    pc = params.c()
    rc = lib().orc_register(_p(lv.sx), _p(lv.sy), _p(lv.ax), _p(lv.ay), _p(lv.vx), _p(lv.vy), w, h, d,
                            C.byref(pc), _p(D), _p(rep))
    if rc:
        raise RuntimeError(f"orc_register failed ({rc})")
    reps = [dict(eta=r[0], f_start=r[1], f_end=r[2], iters=int(r[3]), evals=int(r[4])) for r in rep]
    return D, reps


def density(D):
    D = _f64(D)
    _, h, w, _ = D.shape
    out = np.zeros((2, h, w))
    lib().orc_density(_p(D), w, h, _p(out))
    return out


def merge(sx, sy, D, ox=None, oy=None, vx=None, vy=None, kappa=1.0, tau=0.05):
    sx, sy, D = _f64(sx), _f64(sy), _f64(D)
    h, w, d = sx.shape
    octa = ox is not None
    ox = _f64(ox) if octa else np.zeros(1)
    oy = _f64(oy) if octa else np.zeros(1)
    vx = np.ones(h) if vx is None else _f64(vx)
    vy = np.ones(w) if vy is None else _f64(vy)
    m_oct = np.zeros((h, w, d))
    m_octa = np.zeros((h, w, d)) if octa else None
    rho = np.zeros((2, h, w))
    wt = np.zeros((2, h, w))
    lib().orc_merge(_p(sx), _p(sy), _p(ox), _p(oy), _p(vx), _p(vy), w, h, d, _p(D), float(kappa), float(tau),
                    _p(m_oct), _p(m_octa) if octa else None, _p(rho), _p(wt))
    return m_oct, m_octa, rho, wt


def enface_mean(vol):
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.zeros((h, w))
    lib().orc_enface_mean(_p(vol), w, h, d, _p(out))
    return out


def substitute_invalid(vol, valid, V: int):
    vol = _f64(vol).copy()
    valid = _f64(valid)
    h, w, d = vol.shape
    lib().orc_substitute_invalid(_p(vol), w, h, d, _p(valid), int(V))
    return vol


def round_storage(v, store: int):
    """v rounded to bfloat16 (store = 1) or binary16 (store = 2), to nearest
    with ties to even, as float64."""
    v = _f64(v).copy()
    lib().orc_round_storage(_p(v), v.size, int(store))
    return v


def validity(vol, V: int):
    """Input validity of one OCTA volume [h][w][d] (Sec. 2.2): one value per
    B-scan (rows j for V = 0, columns i for V = 1)."""
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.zeros(h if V == 0 else w)
    lib().orc_validity(_p(vol), w, h, d, int(V), _p(out))
    return out


def median3(vol):
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.empty_like(vol)
    lib().orc_median3(_p(vol), w, h, d, _p(out))
    return out


def rank_line(vol, axis: int, half: int = 7, rank: int = 2):
    """Rank filter along x (axis 0) or y (axis 1) of a [h][w][d] volume."""
    vol = _f64(vol)
    h, w, d = vol.shape
    out = np.empty_like(vol)
    lib().orc_rank_line(_p(vol), w, h, d, int(axis), int(half), int(rank), _p(out))
    return out


def quantile_valid(vol, V: int, valid, q: float) -> float:
    vol = _f64(vol)
    h, w, d = vol.shape
    return lib().orc_quantile_valid(_p(vol), w, h, d, int(V), _p(_f64(valid)), float(q))


def enface_project(oct_vol, octa_vol, V: int, valid=None, fixed=None, details=False):
    """Segmentation-free en face projection (Sec. 2.3) of scan V: [h][w].
    fixed: optional (p5, p95) normalisation mapping.  With details=True also
    returns the per-A-scan voxel counts and (p5, p95, thr_r, thr_s)."""
    o, a = _f64(oct_vol), _f64(octa_vol)
    h, w, d = a.shape
    valid = np.ones(h if V == 0 else w) if valid is None else _f64(valid)
    out = np.zeros((h, w))
    cnt = np.zeros((h, w))
    st = np.zeros(4)
    fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.float64)
    lib().orc_enface_project(_p(o), _p(a), w, h, d, int(V), _p(valid), None if fx is None else _p(fx), _p(out),
                             _p(cnt), _p(st))
    return (out, cnt, st) if details else out


# ----------------------------------------------------------------------------
# Stage 1, rough axial prealignment.  theta: X-fast B-scans (h rows) then
# Y-fast B-scans (w columns), (z_b, t_b) each: 2 (h + w) values.

def tilt_expand(theta, w: int, h: int):
    th = _f64(theta)
    D = np.zeros((2, h, w, 3))
    lib().orc_tilt_expand(_p(th), w, h, _p(D))
    return D


def tilt_reduce(G):
    G = _f64(G)
    _, h, w, _ = G.shape
    out = np.zeros(2 * (w + h))
    lib().orc_tilt_reduce(_p(G), w, h, _p(out))
    return out


def tilt_term(theta, w: int, h: int, d: int, gamma_t: float = 1.0):
    th = _f64(theta)
    g = np.zeros(2 * (w + h))
    T = lib().orc_tilt_term(_p(th), w, h, d, float(gamma_t), _p(g))
    return T, g


def prealign_eval(sx, sy, theta, params: Params | None = None, gamma_t: float = 1.0):
    """Stage-1 objective F + T at theta: (terms dict with "T" and "F1", gradient)."""
    params = params or Params()
    sx, sy, th = _f64(sx), _f64(sy), _f64(theta)
    h, w, d = sx.shape
    terms = np.zeros(9)
    g = np.zeros(2 * (w + h))
    pc = params.c()
    f1 = lib().orc_prealign_eval(_p(sx), _p(sy), w, h, d, _p(th), C.byref(pc), float(gamma_t), _p(terms), _p(g))
    t = dict(zip(TERM_NAMES, terms[:8].tolist()))
    t["T"] = float(terms[8])
    t["F1"] = float(f1)
    return t, g


def tilt_upsample(theta_c, wc: int, hc: int, wf: int, hf: int):
    tc = _f64(theta_c)
    out = np.zeros(2 * (wf + hf))
    lib().orc_tilt_upsample(_p(tc), wc, hc, _p(out), wf, hf)
    return out


def prealign(sx, sy, params: Params | None = None, gamma_t: float = 1.0, iters: int = 100):
    """The stage-1 solve on the pyramid: theta at the finest level and
    per-level reports (coarsest first)."""
    params = params or Params()
    sx, sy = _f64(sx), _f64(sy)
    h, w, d = sx.shape
    th = np.zeros(2 * (w + h))
    rep = np.zeros((params.levels, 4))
    pc = params.c()
    rc = lib().orc_prealign(_p(sx), _p(sy), w, h, d, C.byref(pc), float(gamma_t), int(iters), _p(th), _p(rep))
    if rc:
        raise RuntimeError(f"orc_prealign failed ({rc})")
    return th, [dict(f_start=r[0], f_end=r[1], iters=int(r[2]), evals=int(r[3])) for r in rep]


def resample_z(vol, dz):
    vol, dz = _f64(vol), _f64(dz)
    h, w, d = vol.shape
    out = np.zeros_like(vol)
    lib().orc_resample_z(_p(vol), w, h, d, _p(dz), _p(out))
    return out


# ----------------------------------------------------------------------------
# More than two volumes.  vols: list of n structural volumes [h][w][d];
# orient: 0 (X-fast) or 1 (Y-fast) per volume; enface: n images [h][w];
# valid: n vectors (h values for X-fast, w for Y-fast) or None (all valid).

class Multi:
    def __init__(self, vols, orient, enface, valid=None):
        self.S = [_f64(v) for v in vols]
        self.A = [_f64(a) for a in enface]
        self.orient = [int(o) for o in orient]
        h, w, d = self.S[0].shape
        self.whd = (w, h, d)
        self.V = [np.ones(h if o == 0 else w) for o in self.orient] if valid is None else \
            [_f64(v) for v in valid]
        self._keep = (self.S, self.A, self.V)

    def ptrs(self, arrs):
        return (C.POINTER(C.c_double) * len(arrs))(*[_p(a) for a in arrs])

    def orient_c(self):
        return (C.c_int * len(self.orient))(*self.orient)


def pair_index(n: int):
    """The pairs (P, Q), P < Q, in the order the multi-volume functions use."""
    return [(P, Q) for P in range(n) for Q in range(P + 1, n)]


def evaluate_multi(mv: Multi, D, params: Params | None = None, eta=None, grad: bool = True):
    """n-volume objective: (terms dict, per-pair (S_str05, S_ang05), gradient [n][h][w][3])."""
    params = params or Params()
    D = _f64(D)
    n = len(mv.S)
    w, h, d = mv.whd
    assert D.shape == (n, h, w, 3)
    np_ = n * (n - 1) // 2
    eta = np.ones(np_) if eta is None else _f64(eta)
    terms = np.zeros(8)
    p05 = np.zeros((np_, 2))
    g = np.zeros_like(D) if grad else None
    pc = params.c()
    rc = lib().orc_eval_multi(n, mv.ptrs(mv.S), mv.ptrs(mv.A), mv.ptrs(mv.V), mv.orient_c(), w, h, d, _p(D),
                              C.byref(pc), _p(eta), _p(terms), _p(p05), _p(g) if grad else None)
    if rc:
        raise RuntimeError(f"orc_eval_multi failed ({rc})")
    return dict(zip(TERM_NAMES, terms.tolist())), p05, g


def upsample_multi(Dc, wf: int, hf: int):
    Dc = _f64(Dc)
    n, hc, wc, _ = Dc.shape
    out = np.zeros((n, hf, wf, 3))
    lib().orc_upsample_multi(n, _p(Dc), wc, hc, _p(out), wf, hf)
    return out


def register_multi(mv: Multi, params: Params | None = None):
    params = params or Params()
    n = len(mv.S)
    w, h, d = mv.whd
    D = np.zeros((n, h, w, 3))
    rep = np.zeros((params.levels, 4))
    pc = params.c()
    rc = lib().orc_register_multi(n, mv.ptrs(mv.S), mv.ptrs(mv.A), mv.ptrs(mv.V), mv.orient_c(), w, h, d,
                                  C.byref(pc), _p(D), _p(rep))
    if rc:
        raise RuntimeError(f"orc_register_multi failed ({rc})")
    return D, [dict(f_start=r[0], f_end=r[1], iters=int(r[2]), evals=int(r[3])) for r in rep]


def merge_multi(mv: Multi, D, octa=None, kappa: float = 1.0, tau: float = 0.05):
    """Merged OCT (and OCTA, from the given OCTA volumes with invalid B-scans
    already replaced) of n registered volumes."""
    D = _f64(D)
    n = len(mv.S)
    w, h, d = mv.whd
    mo = np.zeros((h, w, d))
    O = [_f64(o) for o in octa] if octa is not None else None
    ma = np.zeros((h, w, d)) if O is not None else None
    lib().orc_merge_multi(n, mv.ptrs(mv.S), mv.ptrs(O) if O is not None else None, mv.ptrs(mv.V), mv.orient_c(),
                          w, h, d, _p(D), float(kappa), float(tau), _p(mo), _p(ma) if ma is not None else None)
    return mo, ma
