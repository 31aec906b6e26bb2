"""Segmentation-free en face projection (Sec. 2.3) on the GPU, through the C
ABI, against the FP64 oracle.

Integer decisions are compared exactly: the number of voxels averaged per
A-scan (which depends on every filter, both thresholds and both masks) and
the percentiles and threshold of the normalisation (the same FP64 arithmetic
on both sides, from exactly selected order statistics).  The en face values
are float32 results of FP64 means and medians: |gpu - oracle| <= 1e-6 (1 +
|oracle|).  At the full workload sizes, where the oracle's filters would take
minutes, A-scans are sampled: the oracle filters a crop of +-8 A-scans around
each (all a filtered value there depends on), and the percentile selection is
checked on a volume whose filtered values have a closed form."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log, rel

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _check(octmc, s, a, V, valid=None, fixed=None):
    """GPU projection of (s, a) against the oracle: counts and statistics
    exactly, values to TOL."""
    sv = s.cpu().numpy() if torch.is_tensor(s) else np.asarray(s)
    av = a.cpu().numpy() if torch.is_tensor(a) else np.asarray(a)
    vv = None if valid is None else (valid.cpu().numpy() if torch.is_tensor(valid) else np.asarray(valid))
    out, cnt, st = octmc.enface_project(torch.as_tensor(sv).cuda(), torch.as_tensor(av).cuda(), V,
                                        None if vv is None else torch.as_tensor(vv).cuda(), fixed=fixed, details=True)
    ref, rcnt, rst = oracle.enface_project(sv, av, V, vv, fixed=fixed, details=True)
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(cnt.cpu().numpy(), rcnt.astype(np.int32)), "voxel counts differ"
    assert st[0] == rst[0] and st[1] == rst[1] and st[2] == rst[2], (st, rst)
    assert rel(st[3], rst[3]) < 1e-12 or abs(st[3] - rst[3]) < 1e-15
    err = np.abs(got - ref) / (1.0 + np.abs(ref))
    assert err.max() <= TOL, err.max()
    return got, cnt.cpu().numpy(), st


@pytest.mark.parametrize("V", [0, 1])
def test_projection_parity_synthetic_with_white_lines(octmc, V):
    pair = synth.make_pair("tiny", 1, n=40, d=96, decorrelation=True, white_lines=True)
    valid = pair.vx if V == 0 else pair.vy
    log(f"projection parity tiny 40x40x96 scan {V}, {int((valid == 0).sum())} invalid B-scans")
    got, cnt, st = _check(octmc, pair.sx, pair.ox if V == 0 else pair.oy, V, valid)
    assert 0 < cnt.mean() < 96 and st[0] < st[1]


@pytest.mark.parametrize("shape", [(9, 47, 130), (33, 31, 65), (5, 3, 2), (1, 1, 1), (2, 70, 17), (64, 1, 40)])
def test_projection_parity_random_ragged(octmc, shape):
    h, w, d = shape
    rng = np.random.default_rng(h * 1000 + w * 10 + d)
    s = rng.random(shape, dtype=np.float32)
    a = rng.random(shape, dtype=np.float32)
    a[a < 0.1] = 0.1  # ties
    for V in (0, 1):
        nb = h if V == 0 else w
        valid = np.ones(nb, dtype=np.float32)
        valid[::4] = 0.0
        if nb == 1:
            valid[:] = 1.0
        log(f"projection parity random {shape} scan {V}")
        _check(octmc, s, a, V, valid)
        _check(octmc, s, a, V, None)
    log(f"projection parity random {shape}: no valid B-scan")
    _check(octmc, s, a, 0, np.zeros(h, dtype=np.float32))


def test_projection_fixed_mapping(octmc):
    pair = synth.make_pair("tiny", 2, n=36, d=80, decorrelation=True)
    _, _, st = oracle.enface_project(pair.sx, pair.oy, 1, details=True)
    log("projection with a fixed mapping")
    got, cnt, st2 = _check(octmc, pair.sx, pair.oy, 1, None, fixed=(st[0], st[1]))
    assert st2[0] == st[0] and st2[1] == st[1]
    ref = octmc.enface_project(pair.sx.cuda(), pair.oy.cuda(), 1)
    assert torch.equal(ref.cpu(), torch.from_numpy(got.astype(np.float32)))
    _, cnt0, _ = _check(octmc, pair.sx, pair.oy, 1, None, fixed=(-2.0, -1.0))
    assert not cnt0.any()


def test_projection_c_abi_host_inputs_and_workspace(octmc):
    pair = synth.make_pair("tiny", 0, n=24, d=64, decorrelation=True, white_lines=True)
    s = np.ascontiguousarray(pair.sx.numpy())
    a = np.ascontiguousarray(pair.ox.numpy())
    v = np.ascontiguousarray(pair.vx.numpy())
    h, w, d = a.shape
    ref = oracle.enface_project(s, a, 0, v)
    L = octmc.lib()
    shape = octmc.Shape(w, h, d, octmc.F32, octmc.MEM_HOST)
    out = torch.empty((h, w), dtype=torch.float32, device="cuda")
    vp = lambda x: x.ctypes.data_as(C.c_void_p)
    log("projection through the C ABI, host inputs, library workspace")
    rc = L.octmc_enface_project(octmc.context()._h, C.byref(shape), vp(s), vp(a), 0, vp(v), None,
                                C.c_void_p(out.data_ptr()), None, None, None, 0, None)
    assert rc == 0, octmc.last_error() if hasattr(octmc, "last_error") else rc
    assert np.abs(out.cpu().numpy() - ref).max() <= TOL * (1 + np.abs(ref).max())
    nbytes = octmc.enface_workspace_size(w, h, d)
    assert nbytes >= 8 * w * h * d
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out2 = torch.empty_like(out)
    log("projection through the C ABI, caller workspace (asynchronous)")
    octmc.enface_project(pair.sx.cuda(), pair.ox.cuda(), 0, pair.vx.cuda(), workspace=ws, out=out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    with pytest.raises(octmc.OctmcError):
        octmc.enface_project(pair.sx.cuda(), pair.ox.cuda(), 0, workspace=ws[: nbytes - 256])
    with pytest.raises(octmc.OctmcError):
        octmc.enface_project(pair.sx.cuda(), pair.ox.cuda(), 2)
    z = torch.zeros((1, 8193, 1), device="cuda")
    with pytest.raises(octmc.OctmcError):
        octmc.enface_project(z, z, 0)


def test_projection_parity_mid_size(octmc):
    """128 x 128 x 256: two median tiles deep plus a ragged one, five x
    segments, both scans (the oracle takes a few seconds)."""
    pair = synth.make_pair("tiny", 3, n=128, d=256, decorrelation=True, white_lines=True)
    for V in (0, 1):
        log(f"projection parity 128x128x256 scan {V}")
        _check(octmc, pair.sx, pair.ox if V == 0 else pair.oy, V, pair.vx if V == 0 else pair.vy)


def _crop_filtered(a, j, i, V):
    """Filtered value column R(i, j, :) from a +-8 crop, with the oracle."""
    h, w, _ = a.shape
    j0, j1, i0, i1 = max(0, j - 8), min(h, j + 9), max(0, i - 8), min(w, i + 9)
    c = np.ascontiguousarray(a[j0:j1, i0:i1], dtype=np.float64)
    m = oracle.median3(c)
    fast, slow = (0, 1) if V == 0 else (1, 0)
    r = oracle.rank_line(oracle.rank_line(m, fast), slow)
    return r[j - j0, i - i0]


@pytest.fixture(scope="module")
def clinical():
    log("generate clinical 300x300x640 with decorrelation background on cuda")
    return synth.make_pair("clinical", 0, decorrelation=True, white_lines=True, device="cuda")


@pytest.mark.parametrize("V", [0, 1])
def test_projection_full_size_sampled(octmc, clinical, V):
    pair = clinical
    s, a = pair.sx, (pair.ox if V == 0 else pair.oy)
    valid = pair.vx if V == 0 else pair.vy
    h, w, d = a.shape
    log(f"projection 300x300x640 scan {V}")
    out, cnt, st = octmc.enface_project(s, a, V, valid, details=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64)
    cnt = cnt.cpu().numpy()
    # OCT threshold from its definition
    nz = max(1, int(np.floor(0.05 * d + 0.5)))
    noise = s[:, :, :nz].double().cpu().numpy()
    assert rel(st[3], noise.mean() + 2.0 * noise.std()) < 1e-12
    # the same image with the measured mapping given as a fixed one
    again = octmc.enface_project(s, a, V, valid, fixed=(st[0], st[1]))
    assert np.array_equal(again.cpu().numpy().astype(np.float64), out)
    # sampled A-scans of valid B-scans: counts exactly, within-B-scan differences
    sn, an = s.cpu().numpy(), a.cpu().numpy()
    vn = valid.cpu().numpy()
    okb = np.flatnonzero(vn > 0.5)
    bs = [okb[0], okb[len(okb) // 2], okb[-1]]
    pos = [0, 1, 8, w // 2, w - 9, w - 1]
    for b in bs:
        E = []
        for p in pos:
            j, i = (b, p) if V == 0 else (p, b)
            r = _crop_filtered(an, j, i, V)
            m = (r < st[2]) & (sn[j, i].astype(np.float64) > st[3])
            assert int(m.sum()) == int(cnt[j, i]), (V, j, i)
            E.append(an[j, i][m].astype(np.float64).mean() if m.any() else 0.0)
            if len(E) > 1:
                jr, ir = (b, pos[0]) if V == 0 else (pos[0], b)
                diff = out[j, i] - out[jr, ir]
                assert abs(diff - (E[-1] - E[0])) <= TOL * (1 + abs(E[-1]) + abs(E[0])), (V, j, i)


def test_projection_full_size_percentiles(octmc):
    """A volume constant along x, A = f(k) + g(j): its filtered values are
    known without the 3-D filters (the median of 27 is the median of the 9
    distinct (j, k) samples, the x rank filter keeps the values), so the
    exact 5th and 95th percentiles over the valid B-scans follow from numpy's
    selection at the full 300 x 300 x 640 size."""
    h, w, d = 300, 300, 640
    rng = np.random.default_rng(17)
    f = rng.random(d).astype(np.float32)
    g = (2.0 * rng.random(h)).astype(np.float32)
    A2 = (g[:, None] + f[None, :]).astype(np.float32)
    jj = np.clip(np.arange(h)[:, None] + np.array([-1, 0, 1])[None, :], 0, h - 1)
    kk = np.clip(np.arange(d)[:, None] + np.array([-1, 0, 1])[None, :], 0, d - 1)
    M = np.median(A2[jj[:, None, :, None], kk[None, :, None, :]].reshape(h, d, 9), axis=2)  # [h][d]
    jw = np.clip(np.arange(h)[:, None] + np.arange(-7, 8)[None, :], 0, h - 1)
    R = np.sort(M[jw], axis=1)[:, 2, :]  # [h][d]
    vol = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(A2[:, None, :], (h, w, d)))).cuda()
    oct_vol = torch.rand((h, w, d), generator=torch.Generator().manual_seed(3)).cuda()
    for V in (0, 1):
        valid = np.ones(h if V == 0 else w, dtype=np.float32)
        valid[37:90] = 0.0
        log(f"projection percentiles on the x-constant volume, scan {V}")
        _, _, st = octmc.enface_project(oct_vol, vol, V, torch.from_numpy(valid).cuda(), details=True)
        vals = (R[valid > 0.5] if V == 0 else R).astype(np.float64).ravel()
        rep = w if V == 0 else int((valid > 0.5).sum())
        srt = np.sort(vals)
        n = srt.size * rep
        p = []
        for q in (0.05, 0.95):
            posq = q * float(n - 1)
            lo = int(np.floor(posq))
            lo = min(lo, n - 1)
            frac = posq - lo
            x0, x1 = srt[lo // rep], srt[min(lo + 1, n - 1) // rep]
            p.append(x0 + frac * (x1 - x0) if lo + 1 < n else x0)
        assert st[0] == p[0] and st[1] == p[1], (st, p)
        assert st[2] == p[0] + 0.1 * (p[1] - p[0])


def test_pair_with_projection_matches_oracle_objective(octmc):
    pair = synth.make_pair("tiny", 1, n=48, d=64, decorrelation=True, white_lines=True)
    log("pair with projected en face images vs oracle objective")
    P = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, vx=pair.vx, vy=pair.vy, levels=2, iters_per_level=20,
                   project_enface=True)
    ex = oracle.enface_project(pair.sx, pair.ox, 0, pair.vx)
    ey = oracle.enface_project(pair.sy, pair.oy, 1, pair.vy)
    lv = oracle.level_from(pair.sx, pair.sy, ex, ey, pair.vx.numpy(), pair.vy.numpy())
    D = synth.perturbed_field(pair.d_gt, 0.3, 4).float().cuda()
    t, g = P.eval(0, D, eta_mode=0)
    torch.cuda.synchronize()
    td = octmc.terms_dict(t)
    ref, gref = oracle.evaluate(lv, D.double().cpu().numpy(), oracle.Params(), td["eta"])
    assert rel(td["F"], ref["F"]) < 1e-4 and rel(td["ang"], ref["ang"]) < 1e-4
    # the plain depth mean gives a different angiographic term
    Pm = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, vx=pair.vx, vy=pair.vy, levels=2, iters_per_level=20)
    tm, _ = Pm.eval(0, D, eta_mode=0)
    assert rel(octmc.terms_dict(tm)["ang"], td["ang"]) > 1e-3
