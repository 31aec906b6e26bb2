"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself:
closed forms, invariants the paper states, special cases that reduce to a
library routine (scipy's cubic Hermite spline), finite differences, exact
constructions (integer shifts) and brute force on tiny inputs.
"""
import math

import numpy as np
import pytest
import torch
from scipy.interpolate import CubicHermiteSpline

import synth

RNG = np.random.default_rng(7)


# ---------------------------------------------------------------------------
# scipy-based separable interpolation: the library pin of the interpolator.

def _scipy_axis_interp(arr, axis, x, deriv=False, pad=8):
    """Cubic Hermite interpolation of `arr` along `axis` at position x with
    central-difference knot slopes and constant extension beyond the ends."""
    ap = np.pad(arr, [(pad, pad) if a == axis else (0, 0) for a in range(arr.ndim)], mode="edge")
    n = ap.shape[axis]
    knots = np.arange(n, dtype=float) - pad
    slopes = np.zeros_like(ap)
    sl = [slice(None)] * ap.ndim
    up, dn, mid = list(sl), list(sl), list(sl)
    up[axis], dn[axis], mid[axis] = slice(2, None), slice(None, -2), slice(1, -1)
    slopes[tuple(mid)] = 0.5 * (ap[tuple(up)] - ap[tuple(dn)])
    sp = CubicHermiteSpline(knots, ap, slopes, axis=axis)
    if deriv:
        sp = sp.derivative()
    return sp(x)


def scipy_sample3(vol, x, y, z):
    """Value and the three partial derivatives at (x, y, z) of a [h][w][d]
    volume, by successive 1-D scipy interpolation along z, x and y."""
    out = []
    for dx, dy, dz in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        a = _scipy_axis_interp(vol, 2, z, deriv=bool(dz))      # -> [h][w]
        a = _scipy_axis_interp(a, 1, x, deriv=bool(dx))        # -> [h]
        a = _scipy_axis_interp(a, 0, y, deriv=bool(dy))        # -> scalar
        out.append(float(a))
    return np.array(out)


def scipy_sample2(img, x, y):
    out = []
    for dx, dy in [(0, 0), (1, 0), (0, 1)]:
        a = _scipy_axis_interp(img, 1, x, deriv=bool(dx))
        a = _scipy_axis_interp(a, 0, y, deriv=bool(dy))
        out.append(float(a))
    return np.array(out)


# ---------------------------------------------------------------------------
# interpolator (Eq. 2 "Hermitian interpolation", C1 per the text after Eq. 5)

@pytest.mark.parametrize("t", [0.0, 0.1, 0.25, 0.5, 0.73, 0.999])
def test_taps_partition_and_polynomial_reproduction(orc, t):
    w, dw = orc.hermite_taps(t)
    offs = np.array([-1.0, 0.0, 1.0, 2.0])
    assert abs(w.sum() - 1) < 1e-15
    assert abs(dw.sum()) < 1e-14
    # linear and quadratic fields are reproduced exactly, with their slopes
    assert abs((offs * w).sum() - t) < 1e-14
    assert abs((offs ** 2 * w).sum() - t * t) < 1e-14
    assert abs((offs * dw).sum() - 1) < 1e-14
    assert abs((offs ** 2 * dw).sum() - 2 * t) < 1e-14
    # cubics are not (central-difference tangents are not exact for x^3;
    # the error vanishes at the knots and, by symmetry, at t = 1/2)
    if t not in (0.0, 0.5):
        assert abs((offs ** 3 * w).sum() - t ** 3) > 1e-6


def test_taps_at_knot(orc):
    w, dw = orc.hermite_taps(0.0)
    np.testing.assert_array_equal(w, [0, 1, 0, 0])
    np.testing.assert_allclose(dw, [-0.5, 0, 0.5, 0], atol=0)


def test_sample1_matches_scipy_and_is_c1(orc):
    v = RNG.normal(size=23)
    for x in [-4.2, -0.5, 0.0, 0.3, 5.5, 11.01, 21.7, 22.0, 25.3]:
        ref_v = float(_scipy_axis_interp(v, 0, x))
        ref_d = float(_scipy_axis_interp(v, 0, x, deriv=True))
        got = orc.sample1(v, x)
        assert abs(got[0] - ref_v) < 1e-12, x
        assert abs(got[1] - ref_d) < 1e-12, x
    for n in range(0, 22):  # C1 across every knot, including clamped ones
        left = orc.sample1(v, n - 1e-9)
        right = orc.sample1(v, n)
        assert abs(left[0] - right[0]) < 1e-7
        assert abs(left[1] - right[1]) < 1e-7
        assert right[0] == v[n]  # exact at knots


def test_sample1_constant_extension(orc):
    v = RNG.normal(size=9)
    assert orc.sample1(v, -3.5)[0] == pytest.approx(v[0], abs=1e-15)
    assert orc.sample1(v, -3.5)[1] == pytest.approx(0.0, abs=1e-15)
    assert orc.sample1(v, 12.25)[0] == pytest.approx(v[-1], abs=1e-15)


def test_sample2_sample3_match_scipy(orc):
    img = RNG.normal(size=(9, 11))
    vol = RNG.normal(size=(7, 9, 10))
    for x, y in [(3.3, 4.6), (-1.2, 0.4), (10.7, 8.9), (5.0, 2.0)]:
        np.testing.assert_allclose(orc.sample2(img, x, y), scipy_sample2(img, x, y), atol=1e-12)
    for x, y, z in [(3.3, 4.6, 2.2), (-1.7, 0.25, -2.5), (8.9, 6.6, 9.7), (4.0, 3.0, 5.0), (2.5, 7.5, 11.2)]:
        np.testing.assert_allclose(orc.sample3(vol, x, y, z), scipy_sample3(vol, x, y, z), atol=1e-12)


# ---------------------------------------------------------------------------
# loss (Eq. 4)

def test_pseudo_huber_closed_forms(orc):
    eps = 1e-3
    assert orc.pseudo_huber(0.0, eps).tolist() == [0.0, 0.0]
    L, dL = orc.pseudo_huber(eps, eps)
    assert L == pytest.approx(eps * (math.sqrt(2) - 1), rel=1e-15)
    assert dL == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    L, dL = orc.pseudo_huber(-3 * eps, eps)
    assert L == pytest.approx(eps * (math.sqrt(10) - 1), rel=1e-14)
    assert dL == pytest.approx(-3 / math.sqrt(10), rel=1e-14)
    # far from 0 the loss approaches |x| - eps + eps^2 / (2|x|) (robust to outliers)
    L, dL = orc.pseudo_huber(5.0, eps)
    assert L == pytest.approx(5.0 - eps + eps * eps / 10, abs=1e-12)
    assert dL == pytest.approx(1.0, abs=1e-7)
    # small residuals are quadratic: L ~ x^2 / (2 eps), no cancellation
    L, _ = orc.pseudo_huber(1e-9, eps)
    assert L == pytest.approx(1e-18 / (2 * eps), rel=1e-10)


# ---------------------------------------------------------------------------
# brute force of the whole objective on a tiny pair through scipy

def _brute_objective(sx, sy, ax, ay, vx, vy, D, delta0, eps, eta):
    """Eqs. 2-9 on a tiny pair with every interpolant taken from scipy."""
    h, w, d = sx.shape

    def L(r):
        return eps * (np.sqrt(1 + (r / eps) ** 2) - 1)

    data = s_str = s_ang = 0.0
    for j in range(h):
        for i in range(w):
            dX, dY = D[0, j, i], D[1, j, i]
            lam = 0.0
            for k in range(d):
                ix = scipy_sample3(sx, i + dX[0], j + dX[1], k + dX[2])[0]
                iy = scipy_sample3(sy, i + dY[0], j + dY[1], k + dY[2])[0]
                lam += L(ix - iy)
            ra = scipy_sample2(ax, i + dX[0], j + dX[1])[0] - scipy_sample2(ay, i + dY[0], j + dY[1])[0]
            tvx = min(max(float(_scipy_axis_interp(vx, 0, j + dX[1])), 0.0), 1.0)
            tvy = min(max(float(_scipy_axis_interp(vy, 0, i + dY[0])), 0.0), 1.0)
            delta = delta0 * tvx * tvy
            s_str += (1 - delta) * lam
            s_ang += delta * d * L(ra)
            data += eta * (1 - delta) * lam + delta * d * L(ra) / eta
    return data, s_str, s_ang


def test_objective_matches_scipy_brute_force(orc):
    rng = np.random.default_rng(3)
    h = w = 5
    d = 6
    sx, sy = rng.uniform(0, 1, (h, w, d)), rng.uniform(0, 1, (h, w, d))
    ax, ay = rng.uniform(0, 1, (h, w)), rng.uniform(0, 1, (h, w))
    vx = np.array([1, 1, 0, 1, 1.0])
    vy = np.array([1, 0.5, 1, 1, 1.0])
    D = rng.uniform(-1.5, 1.5, (2, h, w, 3))
    lv = orc.level_from(sx, sy, ax, ay, vx, vy)
    p = orc.Params(alpha=0.0, mean_weight=0.0, delta0=0.5)
    eta = 1.37
    t, _ = orc.evaluate(lv, D, p, eta, grad=False)
    data, s_str, s_ang = _brute_objective(sx, sy, ax, ay, vx, vy, D, 0.5, 1e-3, eta)
    assert t["data"] == pytest.approx(data, rel=1e-12)
    assert t["str"] == pytest.approx(s_str, rel=1e-12)
    assert t["ang"] == pytest.approx(s_ang, rel=1e-12)
    assert t["F"] == pytest.approx(data, rel=1e-12)


# ---------------------------------------------------------------------------
# invariants the paper states

def _tiny_pair(seed=0, h=12, d=16):
    rng = np.random.default_rng(seed)
    sx = rng.uniform(0, 1, (h, h, d))
    sy = rng.uniform(0, 1, (h, h, d))
    ax = rng.uniform(0, 1, (h, h))
    ay = rng.uniform(0, 1, (h, h))
    return sx, sy, ax, ay


def test_zero_data_term_identical_inputs(orc):
    sx, _, ax, _ = _tiny_pair()
    lv = orc.level_from(sx, sx, ax, ax)
    p = orc.Params(alpha=0.0, mean_weight=0.0)
    t, g = orc.evaluate(lv, np.zeros((2, 12, 12, 3)), p, 1.3)
    assert t["data"] == 0.0 and t["str"] == 0.0 and t["ang"] == 0.0
    assert np.all(g == 0.0)
    # any field that moves both scans the same way keeps the term at zero
    D1 = np.random.default_rng(1).uniform(-2, 2, (12, 12, 3))
    t, g = orc.evaluate(lv, np.stack([D1, D1]), p, 0.7)
    assert t["data"] == 0.0
    assert np.all(g == 0.0)


def test_integer_shift_resamples_exactly(orc):
    """S^Y(q) = S^X(q + s) for an integer s: d^Y = d^X - s aligns the scans
    exactly, for any fractional d^X (same taps, same weights)."""
    rng = np.random.default_rng(5)
    n, d, s = 24, 26, np.array([2, -1, 3])
    o = 4
    big = np.zeros((n + 2 * o,) * 2 + (d + 2 * o,))
    big2d = np.zeros((n + 2 * o,) * 2)
    # content only where both crops have a zero band of >= 4 samples, so the
    # clamped edges of both scans see zeros as well
    lo = o + np.maximum(0, s) + 4
    hi = o + np.minimum(0, s) + np.array([n, n, d]) - 4
    big[lo[1]:hi[1], lo[0]:hi[0], lo[2]:hi[2]] = rng.uniform(0.1, 1, (hi - lo)[[1, 0, 2]])
    big2d[lo[1]:hi[1], lo[0]:hi[0]] = rng.uniform(0.1, 1, (hi - lo)[[1, 0]])
    sx = big[o:o + n, o:o + n, o:o + d]
    sy = big[o + s[1]:o + s[1] + n, o + s[0]:o + s[0] + n, o + s[2]:o + s[2] + d]
    ax = big2d[o:o + n, o:o + n]
    ay = big2d[o + s[1]:o + s[1] + n, o + s[0]:o + s[0] + n]
    lv = orc.level_from(sx, sy, ax, ay)
    dX = np.broadcast_to(np.array([0.37, -0.21, 0.64]), (n, n, 3))
    D = np.stack([dX, dX - s])
    t, _ = orc.evaluate(lv, D, orc.Params(alpha=0.0, mean_weight=0.0), 1.0, grad=False)
    # zero up to the rounding of the fractional parts of i + dx and i - 2 + dx
    assert t["data"] < 1e-18
    # and a different fractional offset between the scans is not aligned
    D[1, :, :, 0] += 0.5
    t, _ = orc.evaluate(lv, D, orc.Params(alpha=0.0, mean_weight=0.0), 1.0, grad=False)
    assert t["data"] > 1.0


def test_transpose_symmetry(orc):
    """Transposing both scans (i <-> j), swapping the X/Y roles and the x/y
    displacement components maps the problem onto itself: R -> -R."""
    sx, sy, ax, ay = _tiny_pair(2)
    vx = np.array([1, 1, 1, 0.2, 0, 0.7, 1, 1, 1, 1, 1, 1.0])
    vy = np.array([1, 0.6, 1, 1, 1, 1, 1, 1, 0, 1, 1, 1.0])
    D = np.random.default_rng(4).uniform(-1.5, 1.5, (2, 12, 12, 3))
    p = orc.Params()
    lv = orc.level_from(sx, sy, ax, ay, vx, vy)
    t1, g1 = orc.evaluate(lv, D, p, 1.1)
    lvT = orc.level_from(sy.transpose(1, 0, 2), sx.transpose(1, 0, 2), ay.T, ax.T, vy, vx)
    DT = np.stack([D[1].transpose(1, 0, 2)[..., [1, 0, 2]], D[0].transpose(1, 0, 2)[..., [1, 0, 2]]])
    t2, g2 = orc.evaluate(lvT, DT, p, 1.1)
    for k in t1:
        assert t2[k] == pytest.approx(t1[k], rel=1e-12, abs=1e-12), k
    g1T = np.stack([g1[1].transpose(1, 0, 2)[..., [1, 0, 2]], g1[0].transpose(1, 0, 2)[..., [1, 0, 2]]])
    np.testing.assert_allclose(g2, g1T, rtol=1e-10, atol=1e-10)


def test_delta0_zero_is_oct_only(orc):
    """With delta0 = 0 the en face images have no influence and the data term
    is eta times the OCT-only similarity (Eq. 3); the paper compares against
    exactly that configuration."""
    sx, sy, ax, ay = _tiny_pair(3)
    D = np.random.default_rng(6).uniform(-1, 1, (2, 12, 12, 3))
    p0 = orc.Params(delta0=0.0)
    t1, g1 = orc.evaluate(orc.level_from(sx, sy, ax, ay), D, p0, 1.7)
    t2, g2 = orc.evaluate(orc.level_from(sx, sy, 5 * ay, -ax), D, p0, 1.7)
    assert t1["F"] == t2["F"]
    np.testing.assert_array_equal(g1, g2)
    t3, _ = orc.evaluate(orc.level_from(sx, sy, ax, ay), D, orc.Params(delta0=0.0, alpha=0, mean_weight=0), 1.0,
                         grad=False)
    assert t1["data"] == pytest.approx(1.7 * t3["data"], rel=1e-14)
    assert t1["ang"] == 0.0


def test_invalid_scans_remove_angiographic_term(orc):
    """v = 0 makes delta = 0: the angiographic term vanishes and the
    structural term becomes the basic one (Sec. 2.4)."""
    sx, sy, ax, ay = _tiny_pair(4)
    D = np.random.default_rng(8).uniform(-1, 1, (2, 12, 12, 3))
    z = np.zeros(12)
    t, _ = orc.evaluate(orc.level_from(sx, sy, ax, ay, z, None), D, orc.Params(), 1.0, grad=False)
    assert t["ang"] == 0.0
    t0, _ = orc.evaluate(orc.level_from(sx, sy, ax, ay), D, orc.Params(delta0=0.0), 1.0, grad=False)
    assert t["str"] == pytest.approx(t0["str"], rel=1e-14)


def test_eta_equalises_terms(orc):
    p = synth.make_pair("tiny", n=24, d=32)
    lv = orc.level_from_pair(p)
    t, _ = orc.evaluate(lv, np.zeros((2, 24, 24, 3)), orc.Params(), 1.0, grad=False)
    eta = orc.eta_from_terms(t["str05"], t["ang05"])
    # eta S_str = S_ang / eta: both equal the geometric mean (Eq. 10)
    assert eta * t["str05"] == pytest.approx(t["ang05"] / eta, rel=1e-14)
    assert eta * t["str05"] == pytest.approx(math.sqrt(t["str05"] * t["ang05"]), rel=1e-14)
    assert orc.eta_from_terms(0.0, 3.0) == 1.0


# ---------------------------------------------------------------------------
# gradient

def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(11)
    pair = synth.make_pair("tiny", n=16, d=24)
    vx = np.ones(16)
    vx[5] = 0.0
    vy = np.ones(16)
    vy[9] = 0.3
    lv = orc.level_from(pair.sx, pair.sy, pair.ax, pair.ay, vx, vy)
    D = pair.d_gt.numpy() + rng.normal(0, 0.3, (2, 16, 16, 3))
    p = orc.Params(alpha=0.7, mean_weight=2.0)
    eta = 0.9
    _, g = orc.evaluate(lv, D, p, eta)
    h = 1e-5
    idx = [tuple(int(v) for v in rng.integers([0, 0, 0, 0], [2, 16, 16, 3])) for _ in range(40)]
    for ix in idx:
        # keep sample positions away from knots, where the spline's third
        # derivative jumps and central differences lose accuracy
        base = (ix[2], ix[1], 0)[ix[3]] + D[ix]
        frac = base - math.floor(base)
        if min(frac, 1 - frac) < 1e-3:
            D[ix] += 0.01
    _, g = orc.evaluate(lv, D, p, eta)
    for ix in idx:
        Dp, Dm = D.copy(), D.copy()
        Dp[ix] += h
        Dm[ix] -= h
        fp = orc.evaluate(lv, Dp, p, eta, grad=False)[0]["F"]
        fm = orc.evaluate(lv, Dm, p, eta, grad=False)[0]["F"]
        fd = (fp - fm) / (2 * h)
        assert fd == pytest.approx(g[ix], rel=2e-6, abs=2e-4 * max(1.0, abs(g).max() * 1e-3)), ix


# ---------------------------------------------------------------------------
# regulariser and mean term: closed forms

def test_regulariser_closed_forms(orc):
    n, d = 10, 7
    sx = np.zeros((n, n, d))
    lv = orc.level_from(sx, sx, np.zeros((n, n)), np.zeros((n, n)))
    p = orc.Params(alpha=1.0, mean_weight=0.0, eps_r=0.1, flyback_frac=0.25)
    # a constant field costs nothing
    D = np.broadcast_to(np.array([0.3, -0.2, 1.1]), (2, n, n, 3)).copy()
    t, _ = orc.evaluate(lv, D, p, grad=False)
    assert t["reg"] == 0.0
    # a single jump J inside an X-fast B-scan (between (3, 4) and (4, 4))
    eps = 0.1
    D = np.zeros((2, n, n, 3))
    D[0, 4, 4:, 0] = eps     # from A-scan (4, 4) on in time: rest of row 4 ...
    D[0, 5:, :, 0] = eps     # ... and every later B-scan
    t, _ = orc.evaluate(lv, D, p, grad=False)
    assert t["reg"] == pytest.approx(d * eps * (math.sqrt(2) - 1), rel=1e-13)
    # the same jump across a B-scan boundary is weighted by 1/sqrt(1 + f)
    f = math.floor(0.25 * n + 0.5)  # round half up: 2.5 -> 3
    D = np.zeros((2, n, n, 3))
    D[0, 5:, :, 0] = eps
    t, _ = orc.evaluate(lv, D, p, grad=False)
    assert t["reg"] == pytest.approx(d * eps * (math.sqrt(2) - 1) / math.sqrt(1 + f), rel=1e-13)
    # Y-fast: a jump between (i=2, j=7) and (i=2, j=8)
    D = np.zeros((2, n, n, 3))
    D[1, 8:, 2, 1] = eps
    D[1, :, 3:, 1] = eps
    t, _ = orc.evaluate(lv, D, p, grad=False)
    assert t["reg"] == pytest.approx(d * eps * (math.sqrt(2) - 1), rel=1e-13)


def test_mean_term_closed_form(orc):
    n, d = 8, 5
    sx = np.zeros((n, n, d))
    lv = orc.level_from(sx, sx, np.zeros((n, n)), np.zeros((n, n)))
    c = np.array([0.5, -1.5, 2.0])
    D = np.broadcast_to(c, (2, n, n, 3)).copy()
    p = orc.Params(alpha=0.0, mean_weight=1.7)
    t, g = orc.evaluate(lv, D, p)
    na = n * n
    assert t["mean"] == pytest.approx(2 * 1.7 * d * na * (c ** 2).sum(), rel=1e-14)
    np.testing.assert_allclose(g, np.broadcast_to(2 * 1.7 * d * c, g.shape), rtol=1e-14)


# ---------------------------------------------------------------------------
# pyramid and level transition

def test_pyramid_closed_forms(orc):
    rng = np.random.default_rng(2)
    # constants stay constant, including odd sizes
    v = np.full((5, 7, 9), 2.5)
    np.testing.assert_array_equal(orc.pyr_down3(v), np.full((3, 4, 5), 2.5))
    # a field linear in the coordinates: the coarse sample is the value at the
    # centre of its 2x2x2 block (fine position 2I + 1/2), for even sizes
    j, i, k = np.meshgrid(np.arange(8), np.arange(6), np.arange(10), indexing="ij")
    lin = 0.3 * i - 1.2 * j + 0.7 * k + 4
    J, I, K = np.meshgrid(np.arange(4), np.arange(3), np.arange(5), indexing="ij")
    np.testing.assert_allclose(orc.pyr_down3(lin), 0.3 * (2 * I + .5) - 1.2 * (2 * J + .5) + 0.7 * (2 * K + .5) + 4,
                               atol=1e-13)
    # odd sizes: the last coarse sample averages the last fine one with itself
    a = rng.normal(size=(3, 3, 3))
    assert orc.pyr_down3(a)[1, 1, 1] == pytest.approx(a[2, 2, 2], abs=1e-15)
    np.testing.assert_allclose(orc.pyr_down1(np.array([1.0, 3, 5, 9, 11])), [2, 7, 11])
    np.testing.assert_allclose(orc.pyr_down2(np.arange(6.0).reshape(2, 3)), [[2.0, 3.5]])
    # even sizes keep the mean
    b = rng.normal(size=(6, 8, 4))
    assert orc.pyr_down3(b).mean() == pytest.approx(b.mean(), abs=1e-14)


def test_pyramid_single_precision_for_rounded_storage(orc):
    """The single-precision box of 16-bit storage pyramids: exact where every
    partial sum is representable (dyadic inputs), within the error bound of
    three levels of float32 additions (3 u times the mean of |x|, u = 2^-24)
    of the pinned float64 box elsewhere, ragged sizes included; and a rounded
    pyramid's levels are the storage rounding of those single-precision
    levels (level 0 the rounded input)."""
    rng = np.random.default_rng(5)
    dy = rng.integers(-64, 64, size=(5, 7, 9)) / 8.0
    np.testing.assert_array_equal(orc.pyr_down3_f32(dy), orc.pyr_down3(dy))
    for shape in ((6, 8, 10), (5, 7, 9), (1, 3, 2)):
        v = rng.random(shape).astype(np.float32).astype(np.float64) * 3.0
        v = v.astype(np.float32).astype(np.float64)
        a, b = orc.pyr_down3_f32(v), orc.pyr_down3(v)
        assert np.all(a.astype(np.float32).astype(np.float64) == a)  # single-precision values
        # the mean of |x| over each block bounds the block's |values|
        bound = 3 * 2.0 ** -24 * orc.pyr_down3(np.abs(v)) * (1 + 1e-12)
        assert np.all(np.abs(a - b) <= bound + 2.0 ** -24 * np.abs(b))
    lv = orc.level_from(rng.random((6, 6, 8)).astype(np.float32), rng.random((6, 6, 8)).astype(np.float32),
                        np.zeros((6, 6)), np.zeros((6, 6)))
    pr = orc.pyramid(lv, 3, store=1)
    assert np.array_equal(pr[0].sx, orc.round_storage(lv.sx, 1))
    np.testing.assert_array_equal(pr[1].sy, orc.round_storage(orc.pyr_down3_f32(lv.sy), 1))
    np.testing.assert_array_equal(pr[2].sx, orc.round_storage(orc.pyr_down3_f32(orc.pyr_down3_f32(lv.sx)), 1))


def test_upsample_closed_forms(orc):
    c = np.broadcast_to(np.array([0.5, -0.25, 1.5]), (2, 4, 5, 3)).copy()
    np.testing.assert_allclose(orc.upsample(c, 10, 8), np.broadcast_to(2 * c[0, 0, 0], (2, 8, 10, 3)))
    # a linear coarse field a*I + b*J maps to 2 (a (i - 1/2)/2 + b (j - 1/2)/2)
    # away from the clamped border
    J, I = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
    lin = np.zeros((2, 6, 6, 3))
    lin[..., 0] = 0.4 * I - 0.7 * J
    up = orc.upsample(lin, 12, 12)
    j, i = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    exp = 0.4 * (i - 0.5) - 0.7 * (j - 0.5)
    sl = (slice(1, 11), slice(1, 11))
    np.testing.assert_allclose(up[0][sl][..., 0], exp[sl], atol=1e-13)


# ---------------------------------------------------------------------------
# L-BFGS

def test_lbfgs_quadratic_closed_form(orc):
    rng = np.random.default_rng(9)
    n = 40
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.normal(size=n)
    x, rep = orc.lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(n), m=5, max_iter=200)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-9)


def test_lbfgs_rosenbrock(orc):
    def fg(x):
        f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
        return f, g

    x, rep = orc.lbfgs(fg, np.array([-1.2, 1.0]), m=5, max_iter=500)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-6)


def test_lbfgs_agrees_with_scipy(orc):
    from scipy.optimize import minimize
    rng = np.random.default_rng(10)
    n = 30
    c = rng.normal(size=n)

    def fg(x):  # smooth, strictly convex
        r = x - c
        return float(np.sum(np.sqrt(1 + r ** 2)) + 0.1 * x @ x), r / np.sqrt(1 + r ** 2) + 0.2 * x

    x, _ = orc.lbfgs(fg, np.zeros(n), max_iter=300)
    ref = minimize(fg, np.zeros(n), jac=True, method="L-BFGS-B", options=dict(gtol=1e-12, ftol=1e-15))
    np.testing.assert_allclose(x, ref.x, atol=1e-6)


# ---------------------------------------------------------------------------
# merge

def test_merge_identity_and_density(orc):
    rng = np.random.default_rng(12)
    sx = rng.uniform(size=(9, 9, 6))
    sy = rng.uniform(size=(9, 9, 6))
    D = np.zeros((2, 9, 9, 3))
    m, _, rho, wt = orc.merge(sx, sy, D)
    np.testing.assert_allclose(rho, 1.0, atol=1e-15)
    np.testing.assert_allclose(wt, 0.5, atol=1e-15)
    np.testing.assert_allclose(m, 0.5 * (sx + sy), atol=1e-15)
    m, _, _, _ = orc.merge(sx, sx, D)
    np.testing.assert_allclose(m, sx, atol=1e-15)
    # X-fast A-scans of row 4 all sample row 3: row 3 is sampled twice as
    # often, row 4 not at all; the weights favour Y there
    D[0, 4, :, 1] = -1.0
    m, _, rho, wt = orc.merge(sx, sy, D)
    assert rho[0, 3, 4] == pytest.approx(2.0)
    assert rho[0, 4, 4] == pytest.approx(2.0)
    assert wt[0, 4, 4] == pytest.approx(math.exp(-1) / (1 + math.exp(-1)))


def test_merge_octa_validity_gap(orc):
    rng = np.random.default_rng(13)
    sx, sy = rng.uniform(size=(2, 8, 8, 4))
    ox, oy = rng.uniform(size=(2, 8, 8, 4))
    vx = np.ones(8)
    vx[3] = 0.0
    vy = np.ones(8)
    vy[5] = 0.0
    m, mo, _, _ = orc.merge(sx, sy, np.zeros((2, 8, 8, 3)), ox, oy, vx, vy)
    np.testing.assert_allclose(mo[3, 2], oy[3, 2])   # X invalid in row 3 -> Y only
    np.testing.assert_allclose(mo[2, 5], ox[2, 5])   # Y invalid in column 5 -> X only
    np.testing.assert_array_equal(mo[3, 5], 0.0)     # both invalid: a black gap
    np.testing.assert_allclose(mo[1, 1], 0.5 * (ox[1, 1] + oy[1, 1]))


def test_substitute_invalid_and_enface(orc):
    vol = np.arange(5 * 5 * 2, dtype=float).reshape(5, 5, 2)
    out = orc.substitute_invalid(vol, np.array([1, 0, 0, 0, 1.0]), 0)
    np.testing.assert_array_equal(out[1], vol[0])
    np.testing.assert_array_equal(out[2], vol[0])   # tie -> lower index
    np.testing.assert_array_equal(out[3], vol[4])
    out = orc.substitute_invalid(vol, np.array([0, 1, 1, 1, 1.0]), 1)
    np.testing.assert_array_equal(out[:, 0], vol[:, 1])
    np.testing.assert_allclose(orc.enface_mean(vol), vol.mean(axis=2))


# ---------------------------------------------------------------------------
# end to end: synthetic recovery

def recovery_mask(pair):
    """A-scans away from the border and from B-scans that contain a saccade."""
    n = pair.meta["n"]
    fly = pair.meta["flyback"]
    m = np.ones((2, n, n), bool)
    tsX, tsY = pair.meta["saccade_times"]
    for t in tsX:
        b = t // (n + fly)
        m[:, max(0, b - 2):b + 3, :] = False
    for t in tsY:
        b = t // (n + fly)
        m[:, :, max(0, b - 2):b + 3] = False
    m[:, :3] = m[:, -3:] = False
    m[:, :, :3] = m[:, :, -3:] = False
    return m


@pytest.mark.slow
def test_synthetic_recovery_tiny(orc):
    pair = synth.make_pair("tiny")
    D, reps = orc.register(orc.level_from_pair(pair), orc.Params(levels=3))
    m = recovery_mask(pair)
    e = D - pair.d_gt.numpy()
    e -= e[m].mean(axis=0)
    rms = np.sqrt((e[m] ** 2).mean(axis=0))
    zero = pair.d_gt.numpy()[m]
    assert m.mean() > 0.4
    assert np.all(rms < 0.25), rms
    assert np.all(np.sqrt((zero ** 2).mean(axis=0)) > 1.0)  # the motion was real
    assert reps[-1]["f_end"] < reps[-1]["f_start"]


def test_round_storage_matches_library_conversions(orc):
    """Storage rounding against numpy's binary16 and torch's bfloat16
    conversions (both round to nearest, ties to even), on random values over
    many binades, exact ties, subnormals and overflow."""
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-30, 20, 20000))).astype(np.float32)
    halfway = np.float32(1.0 + 2.0 ** -8)   # exactly between two bfloat16 values
    halfway16 = np.float32(1.0 + 2.0 ** -11)  # exactly between two binary16 values
    extra = np.array([0.0, -0.0, 1.0, halfway, -halfway, halfway16, 3 * 2.0 ** -25, 2.0 ** -140, 65519.0, 65520.0,
                      1e6, -1e6, 3.0e38], np.float32)
    x = np.concatenate([x, extra])
    got16 = orc.round_storage(x, 2)
    with np.errstate(over="ignore"):
        ref16 = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(got16, ref16)
    gotbf = orc.round_storage(x, 1)
    refbf = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(gotbf, refbf)
    assert orc.round_storage(np.array([halfway]), 1)[0] == 1.0  # tie to even


def test_validity_hand_example(orc):
    """Sec. 2.2 input validity on a hand-worked case: 20 B-scans, 19 with mean
    decorrelation 0.1 and B-scan 7 with 1.0.  Mean 0.145, population standard
    deviation sqrt(0.038475) = 0.19615, threshold 0.7335: only B-scan 7 is
    flagged, and B-scans 5..9 are invalid."""
    rng = np.random.default_rng(3)
    h, w, d = 20, 6, 8
    vol = np.full((h, w, d), 0.1)
    # rows with the same mean but varying content
    noise = rng.uniform(-0.05, 0.05, (h, w, d))
    noise -= noise.mean(axis=(1, 2), keepdims=True)
    vol += noise
    vol[7] = 1.0
    v = orc.validity(vol, 0)
    expect = np.ones(h)
    expect[5:10] = 0.0
    assert np.array_equal(v, expect)
    # the Y-fast scan's B-scans are columns: the transposed volume gives the same
    assert np.array_equal(orc.validity(np.ascontiguousarray(vol.transpose(1, 0, 2)), 1), expect)


def test_validity_borders_and_constant(orc):
    h, w, d = 16, 4, 4
    vol = np.full((h, w, d), 0.2)
    assert np.array_equal(orc.validity(vol, 0), np.ones(h))  # sigma = 0: nothing above the mean
    vol[0] = 3.0
    vol[15] = 3.0
    v = orc.validity(vol, 0)
    # mean 0.55, sigma sqrt(0.8575) = 0.9260: threshold 3.328 > 3.0, so two outliers in 16 hide each other
    assert np.array_equal(v, np.ones(h))
    vol = np.full((40, w, d), 0.2)
    vol[0] = 3.0
    vol[39] = 3.0
    v = orc.validity(vol, 0)
    # 40 B-scans: mean 0.34, sigma sqrt(0.3724) = 0.6102, threshold 2.171: both flagged
    expect = np.ones(40)
    expect[:3] = 0.0
    expect[37:] = 0.0
    assert np.array_equal(v, expect)


def test_validity_recovers_synthetic_white_lines(orc):
    """The generator saturates the OCTA B-scan of every saccade and marks it and
    its two neighbours on each side invalid; the detection finds exactly those."""
    for p in range(3):
        pair = synth.make_pair("tiny", p, white_lines=True)
        assert (pair.vx == 0).any() or (pair.vy == 0).any()
        assert np.array_equal(orc.validity(pair.ox, 0), pair.vx.numpy())
        assert np.array_equal(orc.validity(pair.oy, 1), pair.vy.numpy())


# ---------------------------------------------------------------------------
# Segmentation-free en face projection (Sec. 2.3).

def _np_nearest_valid(img, valid, V):
    """Brute force: each invalid B-scan copies the valid one at the smallest
    distance, the lower index on a tie."""
    out = img.copy()
    nb = len(valid)
    ok = np.flatnonzero(valid > 0.5)
    if len(ok) == 0:
        return out
    for b in range(nb):
        if valid[b] > 0.5:
            continue
        src = ok[np.argmin(np.abs(ok - b) * 2 + (ok > b))]
        if V == 0:
            out[b] = img[src]
        else:
            out[:, b] = img[:, src]
    return out


def _scipy_projection(oct_vol, octa, V, valid):
    """The projection composed from library routines: scipy's median and rank
    filters (clamped borders), numpy's percentile, mean, standard deviation
    and median."""
    from scipy import ndimage
    m = ndimage.median_filter(octa, size=3, mode="nearest")
    fast, slow = ((1, 15, 1), (15, 1, 1)) if V == 0 else ((15, 1, 1), (1, 15, 1))
    r = ndimage.rank_filter(m, rank=2, size=fast, mode="nearest")
    r = ndimage.rank_filter(r, rank=2, size=slow, mode="nearest")
    sel = valid > 0.5 if (valid > 0.5).any() else np.ones_like(valid, bool)
    rv = r[sel] if V == 0 else r[:, sel]
    p5, p95 = np.percentile(rv, [5, 95])
    mask = r < p5 + 0.1 * (p95 - p5)
    d = octa.shape[2]
    nz = max(1, int(np.floor(0.05 * d + 0.5)))
    noise = oct_vol[:, :, :nz]
    mask &= oct_vol > noise.mean() + 2.0 * noise.std()
    cnt = mask.sum(axis=2)
    e = np.where(cnt > 0, (octa * mask).sum(axis=2) / np.maximum(cnt, 1), 0.0)
    e = e - (np.median(e, axis=1, keepdims=True) if V == 0 else np.median(e, axis=0, keepdims=True))
    return _np_nearest_valid(e, valid, V)


def test_median3_matches_scipy(orc):
    from scipy import ndimage
    for shape in [(9, 11, 7), (1, 5, 4), (6, 1, 1), (13, 10, 33)]:
        vol = RNG.standard_normal(shape)
        vol[vol > 1.0] = 1.0  # ties
        assert np.array_equal(orc.median3(vol), ndimage.median_filter(vol, size=3, mode="nearest")), shape


def test_rank_line_matches_scipy(orc):
    from scipy import ndimage
    for shape in [(20, 23, 6), (3, 40, 2), (31, 4, 5)]:
        vol = RNG.random(shape)
        vol[vol < 0.2] = 0.2
        for axis, size in ((0, (1, 15, 1)), (1, (15, 1, 1))):
            got = orc.rank_line(vol, axis, 7, 2)
            assert np.array_equal(got, ndimage.rank_filter(vol, rank=2, size=size, mode="nearest")), (shape, axis)
        # rank 0 of width 3 is the minimum filter
        assert np.array_equal(orc.rank_line(vol, 0, 1, 0), ndimage.minimum_filter(vol, size=(1, 3, 1), mode="nearest"))


def test_quantile_valid_matches_numpy(orc):
    vol = RNG.standard_normal((12, 9, 5))
    valid = np.ones(12)
    valid[[0, 4, 5]] = 0.0
    for q in (0.0, 0.05, 0.5, 0.95, 1.0):
        assert math.isclose(orc.quantile_valid(vol, 0, valid, q), np.percentile(vol[valid > 0.5], 100 * q),
                            rel_tol=1e-15, abs_tol=1e-15)
    vy = np.ones(9)
    vy[8] = 0.0
    assert math.isclose(orc.quantile_valid(vol, 1, vy, 0.05), np.percentile(vol[:, :8], 5), rel_tol=1e-15)
    # no valid B-scan: every voxel counts
    assert math.isclose(orc.quantile_valid(vol, 0, np.zeros(12), 0.95), np.percentile(vol, 95), rel_tol=1e-15)


@pytest.mark.parametrize("V", [0, 1])
def test_enface_projection_matches_library_composition(orc, V):
    h, w, d = 26, 23, 40
    rng = np.random.default_rng(11 + V)
    octa = rng.random((h, w, d))
    octa[:, :, 12:22] *= 0.15  # a low-decorrelation band, as the retina between vessels
    octv = rng.random((h, w, d)) * 0.2
    octv[:, :, 10:24] += 1.0
    nb = h if V == 0 else w
    valid = np.ones(nb)
    valid[[0, 7, 8, nb - 1]] = 0.0
    got = orc.enface_project(octv, octa, V, valid)
    ref = _scipy_projection(octv, octa, V, valid)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_enface_projection_layered_closed_form(orc):
    """A flat retina: decorrelation 0.1 in depths 10..19 and 1.0 elsewhere, one
    vessel one voxel wide (decorrelation 0.9) at x = 5, depth 13, running along
    y.  OCT is bright only in depths 10..15.  The median filter removes the
    vessel, the rank filters keep the layers, the percentile mask is exactly
    the band, the OCT mask keeps its upper six samples: the en face image is
    0.1 + 0.8 / 6 on the vessel column and 0.1 elsewhere, and after the B-scan
    median 0.8 / 6 and 0.  A mask of the high values would give 0 everywhere."""
    h, w, d = 12, 16, 40
    octa = np.ones((h, w, d))
    octa[:, :, 10:20] = 0.1
    octa[:, 5, 13] = 0.9
    octv = np.zeros((h, w, d))
    octv[:, :, 10:16] = 1.0
    e = orc.enface_project(octv, octa, 0)
    expect = np.zeros((h, w))
    expect[:, 5] = 0.8 / 6
    assert np.allclose(e, expect, atol=1e-14)
    # the Y-fast scan subtracts column medians: the vessel column is the whole B-scan, removed
    ey = orc.enface_project(octv, octa, 1)
    assert np.allclose(ey, 0.0, atol=1e-14)
    # an invalid B-scan takes its nearest valid neighbour's values
    vol2 = octa.copy()
    vol2[:, 9, 14] = 0.5  # a second vessel, seen by the X-fast image at x = 9
    vol2[4, 9, 14] = 0.1  # ... missing in B-scan 4
    valid = np.ones(h)
    valid[4] = 0.0
    e2 = orc.enface_project(octv, vol2, 0, valid)
    assert np.allclose(e2[:, 9], 0.4 / 6, atol=1e-14)
    e3 = orc.enface_project(octv, vol2, 0)
    assert math.isclose(e3[4, 9], 0.0, abs_tol=1e-14)


def test_enface_projection_fixed_mapping_and_details(orc):
    """With the fixed mapping equal to the measured percentiles the image is
    unchanged; the reported counts and thresholds are those of the closed
    form above (band of 6 OCT-bright samples, thresholds 0.19 and 0)."""
    h, w, d = 12, 16, 40
    octa = np.ones((h, w, d))
    octa[:, :, 10:20] = 0.1
    octv = np.zeros((h, w, d))
    octv[:, :, 10:16] = 1.0
    e, cnt, st = orc.enface_project(octv, octa, 0, details=True)
    assert np.array_equal(cnt, np.full((h, w), 6.0))
    assert math.isclose(st[0], 0.1, rel_tol=1e-15) and st[1] == 1.0
    assert math.isclose(st[2], 0.1 + 0.1 * 0.9, rel_tol=1e-15) and st[3] == 0.0
    rng = np.random.default_rng(5)
    octa = rng.random((h, w, d))
    octv = rng.random((h, w, d))
    e, cnt, st = orc.enface_project(octv, octa, 1, details=True)
    assert np.array_equal(orc.enface_project(octv, octa, 1, fixed=st[:2]), e)
    # a mapping whose threshold lies below every value keeps no voxel
    e0, cnt0, _ = orc.enface_project(octv, octa, 1, fixed=(-2.0, -1.0), details=True)
    assert not cnt0.any() and not e0.any()


# ---------------------------------------------------------------------------
# Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1).

def _layered_pair(h, w, d, mX, mY):
    return synth.layered_axial_pair(h, w, d, mX, mY)


def test_tilt_expand_closed_form_and_adjoint(orc):
    h, w = 5, 7
    th = RNG.standard_normal(2 * (w + h))
    D = orc.tilt_expand(th, w, h)
    assert not D[..., :2].any()
    # X-fast B-scan j = 3: z + t (i - 3); Y-fast B-scan i = 6: z + t (j - 2)
    assert np.allclose(D[0, 3, :, 2], th[6] + th[7] * (np.arange(w) - 3.0), rtol=0, atol=1e-15)
    assert np.allclose(D[1, :, 6, 2], th[2 * h + 12] + th[2 * h + 13] * (np.arange(h) - 2.0), rtol=0, atol=1e-15)
    G = RNG.standard_normal((2, h, w, 3))
    lhs = float((G * D).sum())
    rhs = float(orc.tilt_reduce(G) @ th)
    assert math.isclose(lhs, rhs, rel_tol=1e-13)


def test_prealign_objective_is_structural_objective_plus_T(orc):
    """At any theta the stage-1 objective is Eq. 1's structural objective at
    the expanded field (no angiographic term) plus T, whatever delta0 the
    parameters carry."""
    h, w, d = 10, 12, 20
    sx = RNG.random((h, w, d))
    sy = RNG.random((h, w, d))
    th = 0.3 * RNG.standard_normal(2 * (w + h))
    t, _ = orc.prealign_eval(sx, sy, th, orc.Params(delta0=0.5), 0.7)
    lv = orc.level_from(sx, sy, np.zeros((h, w)), np.zeros((h, w)))
    ref, _ = orc.evaluate(lv, orc.tilt_expand(th, w, h), orc.Params(delta0=0.0))
    assert math.isclose(t["F"], ref["F"], rel_tol=1e-13) and t["ang"] == 0.0
    T, _ = orc.tilt_term(th, w, h, d, 0.7)
    assert math.isclose(t["F1"], ref["F"] + T, rel_tol=1e-13)


def test_prealign_gradient_matches_finite_differences(orc):
    h, w, d = 9, 11, 24
    sx, sy = _layered_pair(h, w, d, np.zeros((h, w)), 0.4 * RNG.standard_normal((h, w)))
    th = 0.2 * RNG.standard_normal(2 * (w + h))
    _, g = orc.prealign_eval(sx, sy, th, orc.Params(), 1.0)
    eps = 1e-5
    for q in RNG.choice(th.size, 12, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[q] += eps
        tm[q] -= eps
        fd = (orc.prealign_eval(sx, sy, tp)[0]["F1"] - orc.prealign_eval(sx, sy, tm)[0]["F1"]) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-5 * max(1.0, abs(g[q])), (q, fd, g[q])


def _slope_projection_energy(D, V):
    """Squared norm of the part of scan V's axial field that is one common
    slope along the scan's fast axis (x for X-fast, y for Y-fast): the least
    squares fit of dz = tau (f - c) + (one offset per B-scan), by numpy's
    lstsq on the explicit design matrix."""
    dz = D[V, :, :, 2]
    h, w = dz.shape
    lines = dz if V == 0 else dz.T  # one B-scan per row, fast axis along it
    nb, nf = lines.shape
    rows, cols = np.meshgrid(np.arange(nb), np.arange(nf), indexing="ij")
    A = np.zeros((nb * nf, nb + 1))
    A[np.arange(nb * nf), rows.ravel()] = 1.0                # per-B-scan offsets
    A[:, nb] = cols.ravel() - cols.mean()                    # the common slope
    coef, *_ = np.linalg.lstsq(A, lines.ravel(), rcond=None)
    tau = coef[nb]
    return float(((tau * A[:, nb]) ** 2).sum())


def test_tilt_term_is_the_common_slope_energy(orc):
    """T is the tilt normalisation of Eq. 1 (its formula is in earlier work
    that is not available).  Its reading states three properties, each
    checked here without the oracle's own expression: T is gamma_t d / 2
    times the squared norm of each scan's common slope along its fast axis
    (least squares over the expanded field, so a wrong constant, a missing
    n_f or a sum of squared tilts instead of the squared sum fails);
    tilt patterns whose sum is zero cost nothing; the two scans add
    independently; and the quadratic form satisfies theta . grad T = 2 T."""
    for (h, w, d, g) in ((7, 9, 13, 1.0), (12, 5, 40, 0.35), (6, 6, 1, 2.0)):
        th = RNG.standard_normal(2 * (w + h))
        D = orc.tilt_expand(th, w, h)
        T, gT = orc.tilt_term(th, w, h, d, g)
        E = _slope_projection_energy(D, 0) + _slope_projection_energy(D, 1)
        assert math.isclose(T, 0.5 * g * d * E, rel_tol=1e-10), (h, w, T, 0.5 * g * d * E)
        # Euler's identity for a homogeneous quadratic
        assert math.isclose(float(th @ gT), 2.0 * T, rel_tol=1e-12)
        # the offsets z_b do not enter
        assert not gT[0::2].any()
        # the scans add independently
        thX, thY = th.copy(), th.copy()
        thX[2 * h:] = 0.0
        thY[:2 * h] = 0.0
        TX, _ = orc.tilt_term(thX, w, h, d, g)
        TY, _ = orc.tilt_term(thY, w, h, d, g)
        assert math.isclose(T, TX + TY, rel_tol=1e-13)
        # zero-sum tilt patterns (per scan) cost nothing, whatever the offsets
        tz = th.copy()
        tz[1:2 * h:2] -= tz[1:2 * h:2].mean()
        tz[2 * h + 1::2] -= tz[2 * h + 1::2].mean()
        T0, g0 = orc.tilt_term(tz, w, h, d, g)
        assert abs(T0) < 1e-24 * max(1.0, T) + 1e-28 and np.abs(g0).max() < 1e-12
        # a uniform tilt tau on one scan costs gamma_t d N_A var_f tau^2 / 2,
        # var_f the population variance of the fast-axis index
        tau = 0.37
        tu = np.zeros_like(th)
        tu[1:2 * h:2] = tau
        Tu, _ = orc.tilt_term(tu, w, h, d, g)
        assert math.isclose(Tu, 0.5 * g * d * (w * h) * np.var(np.arange(w)) * tau ** 2, rel_tol=1e-13)


def test_tilt_term_fixes_the_common_plane(orc):
    """The data term cannot see a plane a x + b y added to both scans'
    axial fields (pinned below); T is what fixes those two degrees of
    freedom: such a plane, written in each scan's B-scan parameters, costs
    gamma_t d / 2 times the plane's squared norm over both fields, and
    nothing only for a = b = 0."""
    h, w, d = 8, 11, 20
    a, b = 0.04, -0.025
    th = np.zeros(2 * (w + h))
    # X-fast B-scan j (fast axis x): z = a (w - 1) / 2 + b j, t = a
    th[0:2 * h:2] = a * (w - 1) / 2 + b * np.arange(h)
    th[1:2 * h:2] = a
    # Y-fast B-scan i (fast axis y): z = b (h - 1) / 2 + a i, t = b
    th[2 * h::2] = b * (h - 1) / 2 + a * np.arange(w)
    th[2 * h + 1::2] = b
    D = orc.tilt_expand(th, w, h)
    plane = a * np.arange(w)[None, :] + b * np.arange(h)[:, None]
    assert np.allclose(D[0, :, :, 2], plane, atol=1e-14) and np.allclose(D[1, :, :, 2], plane, atol=1e-14)
    T, _ = orc.tilt_term(th, w, h, d, 1.0)
    # the plane's part along x in the X-fast field and along y in the Y-fast one
    ex = ((a * (np.arange(w) - (w - 1) / 2)) ** 2).sum() * h
    ey = ((b * (np.arange(h) - (h - 1) / 2)) ** 2).sum() * w
    assert math.isclose(T, 0.5 * d * (ex + ey), rel_tol=1e-12)
    assert orc.tilt_term(np.zeros_like(th), w, h, d, 1.0)[0] == 0.0


def test_data_term_blind_to_a_common_plane(orc):
    """The two degrees of freedom T fixes: a plane a x + b y added to both
    scans' axial fields leaves the data term unchanged (interior voxels; the
    volume is extended in depth so no sample leaves it)."""
    h, w, d = 12, 12, 40
    sx, sy = _layered_pair(h, w, d, np.zeros((h, w)), np.zeros((h, w)))
    lv = orc.level_from(sx, sy, np.zeros((h, w)), np.zeros((h, w)))
    D = np.zeros((2, h, w, 3))
    plane = 0.05 * np.arange(w)[None, :] - 0.03 * np.arange(h)[:, None]
    D2 = D.copy()
    D2[:, :, :, 2] += plane
    p = orc.Params(delta0=0.0)
    a, _ = orc.evaluate(lv, D, p)
    b, _ = orc.evaluate(lv, D2, p)
    assert math.isclose(a["str"], b["str"], rel_tol=1e-12, abs_tol=1e-12)


def test_tilt_upsample_closed_forms(orc):
    # uniform offset z0 and tilt t0 over even sizes: tilt kept, offset doubled
    wc, hc = 6, 5
    th = np.zeros(2 * (wc + hc))
    th[0::2], th[1::2] = 0.7, 0.05
    f = orc.tilt_upsample(th, wc, hc, 12, 10)
    assert np.allclose(f[1::2], 0.05) and np.allclose(f[0::2], 1.4)
    # odd fine sizes: the fine field is twice the coarse field at (f - 0.5)/2
    f = orc.tilt_upsample(th, wc, hc, 11, 9)
    Dc = orc.tilt_expand(th, wc, hc)
    Df = orc.tilt_expand(f, 11, 9)
    for V, nf, nfc in ((0, 11, wc), (1, 9, hc)):
        line = Df[V, 4, :, 2] if V == 0 else Df[V, :, 4, 2]
        ff = np.arange(nf)
        expect = 2 * (0.7 + 0.05 * ((ff - 0.5) / 2 - (nfc - 1) / 2))
        assert np.allclose(line, expect, rtol=0, atol=1e-14)
    assert Dc.shape == (2, hc, wc, 3)


def test_resample_z_integer_shift_and_spline(orc):
    h, w, d = 3, 4, 30
    vol = RNG.random((h, w, d))
    dz = np.zeros((h, w))
    dz[1, 2] = 3.0
    out = orc.resample_z(vol, dz)
    assert np.array_equal(out[0], vol[0])
    assert np.array_equal(out[1, 2, :d - 3], vol[1, 2, 3:])
    assert np.all(out[1, 2, d - 3:] == vol[1, 2, d - 1])  # constant extension
    dz = RNG.uniform(-2.5, 2.5, (h, w))
    out = orc.resample_z(vol, dz)
    for j in range(h):
        for i in range(w):
            ref = _scipy_axis_interp(vol[j, i], 0, np.arange(d) + dz[j, i])
            assert np.allclose(out[j, i], ref, rtol=0, atol=1e-12)


def test_prealign_recovers_planted_axial_motion_and_tilt(orc):
    """Per-B-scan axial offsets (a random walk with a 2 px jump) and opposite
    tilts of the two scans, planted on analytic layered volumes, are recovered
    by the stage-1 solve: the difference of the two fields matches m^Y - m^X to
    0.1 px RMS (the motion itself is 0.8 px RMS)."""
    h = w = 24
    d = 48
    mX, mY = synth.planted_axial_motion(h, w)
    X, Y = _layered_pair(h, w, d, mX, mY)
    th, rep = orc.prealign(X, Y, orc.Params(levels=2), 1.0, 80)
    D = orc.tilt_expand(th, w, h)
    err = (D[0, :, :, 2] - D[1, :, :, 2]) - (mY - mX)
    assert np.sqrt((err ** 2).mean()) < 0.1
    assert rep[-1]["f_end"] < rep[-1]["f_start"]


# ---------------------------------------------------------------------------
# More than two volumes.

def _multi_inputs(orients, n=20, d=24, seed=0):
    sc = synth.make_scans("tiny", seed, tuple(orients), n=n, d=d, white_lines=True)
    return sc


def test_multi_two_volumes_equal_the_pair_functions(orc):
    """Two volumes of orientations (0, 1): objective, gradient, solve and merge
    are bit for bit the two-volume functions (which carry their own pins)."""
    p = synth.make_pair("tiny", 0, n=20, d=24, white_lines=True)
    vx, vy = p.vx.numpy().copy(), p.vy.numpy().copy()
    vy[4] = 0.4
    lv = orc.level_from(p.sx, p.sy, p.ax, p.ay, vx, vy)
    mv = orc.Multi([p.sx, p.sy], [0, 1], [p.ax, p.ay], [vx, vy])
    D = RNG.normal(0, 1.0, (2, 20, 20, 3))
    pp = orc.Params(alpha=0.7, mean_weight=1.3, levels=2, iters=15)
    t2, g2 = orc.evaluate(lv, D, pp, 1.3)
    tm, p05, gm = orc.evaluate_multi(mv, D, pp, [1.3])
    assert t2 == tm and np.array_equal(g2, gm)
    assert p05[0, 0] == t2["str05"] and p05[0, 1] == t2["ang05"]
    Dr, rep = orc.register(lv, pp)
    Dm, repm = orc.register_multi(mv, pp)
    assert np.array_equal(Dr, Dm)
    mo, ma, _, _ = orc.merge(p.sx, p.sy, Dr, p.ox, p.oy, vx, vy)
    mo2, ma2 = orc.merge_multi(mv, Dr, [p.ox, p.oy])
    assert np.array_equal(mo, mo2) and np.array_equal(ma, ma2)


def test_multi_objective_invariances(orc):
    sc = _multi_inputs((0, 1, 0))
    n, h, w = 3, 20, 20
    mv = orc.Multi(sc.S, sc.orient, sc.A, sc.V)
    D = RNG.normal(0, 0.8, (n, h, w, 3))
    eta = np.array([1.1, 0.9, 1.3])  # pairs (0,1), (0,2), (1,2)
    t, _, g = orc.evaluate_multi(mv, D, orc.Params(), eta)
    # relabelling the volumes (and with them the fields and the pairs' eta)
    perm = [2, 0, 1]
    mv2 = orc.Multi([sc.S[q] for q in perm], [sc.orient[q] for q in perm], [sc.A[q] for q in perm],
                    [sc.V[q] for q in perm])
    pairs = orc.pair_index(3)
    eta2 = [eta[pairs.index(tuple(sorted((perm[P], perm[Q]))))] for P, Q in pairs]
    t2, _, g2 = orc.evaluate_multi(mv2, D[perm], orc.Params(), eta2)
    for key in ("F", "data", "reg", "mean"):
        assert math.isclose(t[key], t2[key], rel_tol=1e-12), key
    assert np.allclose(g[perm], g2, rtol=1e-12, atol=1e-12)
    # identical volumes at zero displacement: no data term
    same = orc.Multi([sc.S[0]] * 3, [0, 1, 0], [sc.A[0]] * 3)
    t0, _, _ = orc.evaluate_multi(same, np.zeros((n, h, w, 3)))
    assert t0["data"] == 0.0


def test_multi_gradient_matches_finite_differences(orc):
    sc = _multi_inputs((0, 1, 1), n=12, d=16, seed=1)
    mv = orc.Multi(sc.S, sc.orient, sc.A, sc.V)
    D = RNG.normal(0, 0.7, (3, 12, 12, 3))
    eta = [1.2, 0.8, 1.0]
    _, _, g = orc.evaluate_multi(mv, D, orc.Params(), eta)
    eps = 1e-6
    for _ in range(12):
        idx = tuple(int(RNG.integers(0, s)) for s in D.shape)
        Dp, Dm = D.copy(), D.copy()
        Dp[idx] += eps
        Dm[idx] -= eps
        fd = (orc.evaluate_multi(mv, Dp, orc.Params(), eta, grad=False)[0]["F"] -
              orc.evaluate_multi(mv, Dm, orc.Params(), eta, grad=False)[0]["F"]) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-5 * max(1.0, abs(g[idx])), (idx, fd, g[idx])


def test_multi_merge_two_pairs_fill_white_line_gaps(orc):
    """Fig. 4(d): with one pair, the crossing of an invalid X-fast B-scan and
    an invalid Y-fast B-scan has no valid OCTA data (a gap, 0); a second,
    valid pair fills it with the mean of its two scans."""
    h = w = 16
    d = 8
    rng = np.random.default_rng(4)
    S = [rng.random((h, w, d)) for _ in range(4)]
    O = [rng.random((h, w, d)) + 0.5 for _ in range(4)]
    A = [np.zeros((h, w))] * 4
    j0, i0 = 7, 9
    vX1 = np.ones(h)
    vX1[j0] = 0.0
    vY1 = np.ones(w)
    vY1[i0] = 0.0
    D0 = np.zeros((4, h, w, 3))
    one = orc.Multi(S[:2], [0, 1], A[:2], [vX1, vY1])
    _, ma1 = orc.merge_multi(one, D0[:2], O[:2])
    assert np.all(ma1[j0, i0] == 0.0)
    two = orc.Multi(S, [0, 1, 0, 1], A, [vX1, vY1, np.ones(h), np.ones(w)])
    mo2, ma2 = orc.merge_multi(two, D0, O)
    assert np.allclose(ma2[j0, i0], 0.5 * (O[2][j0, i0] + O[3][j0, i0]), rtol=0, atol=1e-14)
    # away from the white lines all four scans count equally (identity fields: density 1)
    assert np.allclose(ma2[2, 3], 0.25 * sum(o[2, 3] for o in O), rtol=0, atol=1e-14)
    assert np.allclose(mo2[2, 3], 0.25 * sum(s[2, 3] for s in S), rtol=0, atol=1e-14)
