"""Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1), on the GPU through
the C ABI against the FP64 oracle: the stage-1 objective and its gradient
with respect to the per-B-scan offsets and tilts (10^-4 relative, the
evaluation's bar), the stage-1 solve (expanded fields within 0.05 px RMS),
the axial resampling, recovery of planted motion, and a pair created with
OCTMC_PREALIGN."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import grad_err, grad_rel, log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _stage_pair(octmc, X, Y, levels=2, dtype="f32"):
    """A structural-only pair as stage 1 uses it: delta0 = 0, no en face data."""
    h, w, _ = X.shape
    z = torch.zeros((h, w))
    return octmc.Pair(torch.from_numpy(X).float(), torch.from_numpy(Y).float(), ax=z, ay=z, delta0=0.0,
                      levels=levels, dtype=dtype)


@pytest.fixture(scope="module")
def planted():
    h = w = 40
    d = 64
    mX, mY = synth.planted_axial_motion(h, w, seed=3)
    X, Y = synth.layered_axial_pair(h, w, d, mX, mY)
    return X.astype(np.float32), Y.astype(np.float32), mX, mY


@pytest.mark.parametrize("level", [0, 1])
def test_prealign_objective_and_gradient_parity(octmc, planted, level):
    X, Y, _, _ = planted
    P = _stage_pair(octmc, X, Y)
    w, h, d = P.level_shape(level)
    sx, sy = X.astype(np.float64), Y.astype(np.float64)
    for _ in range(level):
        sx, sy = oracle.pyr_down3(sx), oracle.pyr_down3(sy)
    rng = np.random.default_rng(level)
    for case, th in (("zero", np.zeros(2 * (w + h))), ("random", 0.4 * rng.standard_normal(2 * (w + h)))):
        log(f"stage-1 objective level {level} ({w}x{h}x{d}) theta {case}")
        t, T, g = P.prealign_eval(level, th, 0.8)
        ref, gref = oracle.prealign_eval(sx, sy, th, oracle.Params(delta0=0.0), 0.8)
        assert rel(t["F"] + T, ref["F1"]) < 1e-4, (t, T, ref)
        assert rel(T, ref["T"]) < 1e-12 or abs(T - ref["T"]) < 1e-12
        assert rel(t["reg"], ref["reg"]) < 1e-4 and t["ang"] == 0.0
        assert grad_err(g, gref) < 1e-4


def test_prealign_solve_parity_and_recovery(octmc, planted):
    X, Y, mX, mY = planted
    h, w, d = X.shape
    P = _stage_pair(octmc, X, Y)
    log("stage-1 solve on the GPU, 2 levels x 60 steps")
    th, rep = P.prealign(1.0, 60)
    log("stage-1 solve in the oracle")
    tho, repo = oracle.prealign(X.astype(np.float64), Y.astype(np.float64), oracle.Params(levels=2), 1.0, 60)
    Dg, Do = oracle.tilt_expand(th, w, h), oracle.tilt_expand(tho, w, h)
    rms = np.sqrt(((Dg - Do)[..., 2] ** 2).mean())
    assert rms < 0.05, rms
    for r, ro in zip(rep, repo):
        assert abs(r["f_end"] - ro["f_end"]) <= 0.05 * abs(ro["f_end"]), (r, ro)
    err = (Dg[0, ..., 2] - Dg[1, ..., 2]) - (mY - mX)
    assert np.sqrt((err ** 2).mean()) < 0.1


def test_resample_axial_parity(octmc):
    rng = np.random.default_rng(9)
    h, w, d = 13, 17, 70
    vol = rng.random((h, w, d), dtype=np.float32)
    dz = rng.uniform(-5, 5, (h, w)).astype(np.float32)
    dz[0, 0] = 1e6  # beyond the A-scan: constant extension
    dz[0, 1] = -3.0
    ref = oracle.resample_z(vol, dz)
    log("axial resampling, device inputs")
    got = octmc.resample_axial(torch.from_numpy(vol).cuda(), torch.from_numpy(dz).cuda())
    torch.cuda.synchronize()
    assert np.abs(got.cpu().numpy() - ref).max() < 2e-6
    assert torch.equal(got[0, 1, 3:].cpu(), torch.from_numpy(vol[0, 1, : d - 3]))  # integer shift: exact
    log("axial resampling, host inputs through the C ABI")
    out = torch.empty((h, w, d), device="cuda")
    shape = octmc.Shape(w, h, d, octmc.F32, octmc.MEM_HOST)
    rc = octmc.lib().octmc_resample_axial(octmc.context()._h, C.byref(shape), vol.ctypes.data_as(C.c_void_p),
                                          dz.ctypes.data_as(C.c_void_p), C.c_void_p(out.data_ptr()), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), got.cpu())


def test_pair_created_with_prealignment(octmc, planted):
    X, Y, mX, mY = planted
    h, w, d = X.shape
    ax = torch.rand((h, w), generator=torch.Generator().manual_seed(1))
    ay = torch.rand((h, w), generator=torch.Generator().manual_seed(2))
    log("pair with OCTMC_PREALIGN (2 levels x 60 stage-1 steps)")
    P = octmc.Pair(torch.from_numpy(X), torch.from_numpy(Y), ax=ax, ay=ay, levels=2, prealign=True,
                   prealign_iters=60)
    th, dz = P.prealignment()
    torch.cuda.synchronize()
    # the stage ran on the structural volumes alone, as a separate stage-1 pair does
    th1, _ = _stage_pair(octmc, X, Y).prealign(1.0, 60)
    assert np.array_equal(th, th1)
    D = oracle.tilt_expand(th, w, h)
    assert np.abs(dz.cpu().numpy() - D[..., 2]).max() < 1e-5
    # the pair holds the prealigned volumes: its objective equals the oracle's on them
    sx = oracle.resample_z(X, dz[0].cpu().numpy())
    sy = oracle.resample_z(Y, dz[1].cpu().numpy())
    lv = oracle.level_from(sx, sy, ax, ay)
    D0 = torch.zeros((2, h, w, 3), device="cuda")
    t, g = P.eval(0, D0, eta_mode=0)
    torch.cuda.synchronize()
    td = octmc.terms_dict(t)
    ref, gref = oracle.evaluate(lv, np.zeros((2, h, w, 3)), oracle.Params(), td["eta"])
    # norm-wise: the two sides evaluate different volumes here (the pair's are
    # resampled in float32, up to 2e-6 from the oracle's float64 resampling),
    # and at D = 0 after prealignment many residuals sit at the pseudo-Huber
    # kink, which magnifies such input differences entry by entry; the
    # evaluation itself is checked entry by entry on identical inputs above
    assert rel(td["F"], ref["F"]) < 1e-4 and grad_rel(g.double().cpu().numpy(), gref) < 1e-4
    # after prealignment the residual axial misalignment is small
    res = (D[0, ..., 2] - D[1, ..., 2]) - (mY - mX)
    assert np.sqrt((res ** 2).mean()) < 0.1
    with pytest.raises(octmc.OctmcError):
        _stage_pair(octmc, X, Y).prealignment()


def test_prealign_objective_parity_clinical_size(octmc):
    """One stage-1 evaluation at 300 x 300 x 640 (the clinical workload's
    size) against the oracle's full sum."""
    log("generate clinical 300x300x640 on cuda")
    pair = synth.make_pair("clinical", 0, octa_volumes=False, device="cuda")
    h, w, d = pair.sx.shape
    P = octmc.Pair(pair.sx, pair.sy, ax=torch.zeros((h, w)), ay=torch.zeros((h, w)), delta0=0.0, levels=4)
    th = 0.3 * np.random.default_rng(5).standard_normal(2 * (w + h))
    log("stage-1 objective 300x300x640 on the GPU")
    t, T, g = P.prealign_eval(0, th, 1.0)
    log("stage-1 objective 300x300x640 in the oracle")
    ref, gref = oracle.prealign_eval(pair.sx.cpu().numpy(), pair.sy.cpu().numpy(), th, oracle.Params(delta0=0.0),
                                     1.0)
    assert rel(t["F"] + T, ref["F1"]) < 1e-4
    assert grad_err(g, gref) < 1e-4


def test_full_pipeline_flags_equal_the_chained_entry_points(octmc):
    """Fig. 1 in one call (prealignment, saccade detection, projection,
    registration, merge) equals the same steps chained through the separate
    entry points, bit for bit."""
    pair = synth.make_pair("tiny", 1, n=48, d=64, white_lines=True, decorrelation=True)
    kw = dict(levels=2, iters_per_level=20, prealign_iters=30)
    log("pair with OCTMC_PREALIGN | OCTMC_DETECT_INVALID | OCTMC_ENFACE_PROJECT")
    P = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, prealign=True, detect_invalid=True,
                   project_enface=True, **kw)
    D1, mo1, ma1, _ = P.register(merged=True)
    th1, dz1 = P.prealignment()
    torch.cuda.synchronize()
    log("the same steps chained by hand")
    h, w, d = pair.sx.shape
    z = torch.zeros((h, w))
    S1 = octmc.Pair(pair.sx, pair.sy, ax=z, ay=z, delta0=0.0, **kw)
    th, _ = S1.prealign(1.0, 30)
    assert np.array_equal(th, th1)
    dz = dz1  # the field of th (checked against the oracle's expansion in another test)
    sx, sy = octmc.resample_axial(pair.sx.cuda(), dz[0]), octmc.resample_axial(pair.sy.cuda(), dz[1])
    ox, oy = octmc.resample_axial(pair.ox.cuda(), dz[0]), octmc.resample_axial(pair.oy.cuda(), dz[1])
    vx, vy = octmc.validity_from_octa(ox, 0), octmc.validity_from_octa(oy, 1)
    ax = octmc.enface_project(sx, ox, 0, vx)
    ay = octmc.enface_project(sy, oy, 1, vy)
    Q = octmc.Pair(sx, sy, ox=ox, oy=oy, ax=ax, ay=ay, vx=vx, vy=vy, **kw)
    D2, mo2, ma2, _ = Q.register(merged=True)
    torch.cuda.synchronize()
    assert torch.equal(D1, D2) and torch.equal(mo1, mo2) and torch.equal(ma1, ma2)
