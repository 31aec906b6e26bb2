"""More than two volumes on the GPU, through the C ABI, against the FP64
oracle: the n-volume objective and gradient (10^-4 relative), the joint
solve (0.05 px RMS), the merge (10^-4) including the filling of one pair's
white-line crossings by a second pair, and n = 2 against the pair path."""
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


@pytest.fixture(scope="module")
def scans():
    return synth.make_scans("tiny", 2, (0, 1, 0, 1), n=40, d=64, white_lines=True)


def _oracle_multi(sc, idx=None):
    idx = list(range(len(sc.S))) if idx is None else idx
    return oracle.Multi([sc.S[q] for q in idx], [sc.orient[q] for q in idx], [sc.A[q] for q in idx],
                        [sc.V[q] for q in idx])


def _gpu_multi(octmc, sc, idx=None, **kw):
    idx = list(range(len(sc.S))) if idx is None else idx
    return octmc.Multi([sc.S[q] for q in idx], [sc.orient[q] for q in idx], enface=[sc.A[q] for q in idx],
                       valid=[sc.V[q] for q in idx], **kw)


def test_multi_two_volumes_match_the_pair_path(octmc):
    p = synth.make_pair("tiny", 0, n=40, d=64, white_lines=True)
    D = synth.perturbed_field(p.d_gt, 0.3, 2).float().cuda()
    log("n = 2 multi vs pair, level 0")
    P = octmc.Pair(p.sx, p.sy, ax=p.ax, ay=p.ay, vx=p.vx, vy=p.vy, levels=2)
    M = octmc.Multi([p.sx, p.sy], [0, 1], enface=[p.ax, p.ay], valid=[p.vx, p.vy], levels=2)
    t1, g1 = P.eval(0, D, eta_mode=0)
    t2, g2 = M.eval(0, D, eta_mode=0)
    torch.cuda.synchronize()
    a, b = octmc.terms_dict(t1), octmc.terms_dict(t2)
    for key in ("F", "data", "str", "ang", "reg", "mean"):
        assert rel(b[key], a[key]) < 1e-12 or abs(b[key] - a[key]) < 1e-9, key
    assert grad_rel(g2.double().cpu().numpy(), g1.double().cpu().numpy()) < 1e-6


@pytest.mark.parametrize("level", [0, 1])
def test_multi_objective_parity(octmc, scans, level):
    sc = scans
    n = len(sc.S)
    M = _gpu_multi(octmc, sc, levels=2)
    w, h, d = M.level_shape(level)
    rng = np.random.default_rng(level)
    D = rng.normal(0, 0.8, (n, h, w, 3))
    # oracle inputs at this level: the pyramid of every volume
    S = [s.double().numpy() for s in sc.S]
    A = [a.double().numpy() for a in sc.A]
    V = [v.double().numpy() for v in sc.V]
    for _ in range(level):
        S = [oracle.pyr_down3(s) for s in S]
        A = [oracle.pyr_down2(a) for a in A]
        V = [oracle.pyr_down1(v) for v in V]
    om = oracle.Multi(S, sc.orient, A, V)
    t0, p05, _ = oracle.evaluate_multi(om, D, oracle.Params(), None, grad=False)
    eta = np.array([oracle.eta_from_terms(a, b) for a, b in p05])
    ref, _, gref = oracle.evaluate_multi(om, D, oracle.Params(), eta)
    log(f"n = 4 objective at level {level} ({w}x{h}x{d})")
    t, g = M.eval(level, torch.from_numpy(D).float().cuda(), eta_mode=0)
    torch.cuda.synchronize()
    td = octmc.terms_dict(t)
    for key in ("F", "data", "str", "ang", "reg", "mean"):
        assert rel(td[key], ref[key]) < 1e-4, (key, td[key], ref[key])
    assert grad_err(g.double().cpu().numpy(), gref) < 1e-4


def test_multi_register_parity(octmc, scans):
    sc = scans
    log("n = 4 joint solve, 2 levels x 40 steps, GPU")
    M = _gpu_multi(octmc, sc, levels=2, iters_per_level=40)
    Dg, _, _, rep = M.register()
    torch.cuda.synchronize()
    log("n = 4 joint solve in the oracle")
    Do, repo = oracle.register_multi(_oracle_multi(sc), oracle.Params(levels=2, iters=40))
    err = np.sqrt(((Dg.double().cpu().numpy() - Do) ** 2).mean())
    assert err < 0.05, err
    for r, ro in zip(rep, repo):
        assert abs(r["f_end"] - ro["f_end"]) <= 0.05 * abs(ro["f_end"]), (r, ro)
    assert rep[-1]["f_end"] < rep[-1]["f_start"]


def test_multi_merge_parity_and_gap_filling(octmc):
    """Identity fields (no solve steps), white lines in the first pair only:
    the merge equals the oracle's, and at the first pair's white-line
    crossings the second pair supplies the OCTA data."""
    sc = synth.make_scans("tiny", 3, (0, 1, 0, 1), n=36, d=48, white_lines=True)
    # white lines only in the first pair
    V = [sc.V[0], sc.V[1], torch.ones_like(sc.V[2]), torch.ones_like(sc.V[3])]
    O = [sc.O[0], sc.O[1], sc.O[2], sc.O[3]]
    log("n = 4 merge at identity fields")
    M = octmc.Multi(sc.S, sc.orient, octa=O, valid=V, levels=1, iters_per_level=0)
    D, mo, ma, _ = M.register(merged=True)
    torch.cuda.synchronize()
    assert not D.any()
    Osub = [oracle.substitute_invalid(O[q], V[q], sc.orient[q]) for q in range(4)]
    om = oracle.Multi(sc.S, sc.orient, [oracle.enface_mean(o) for o in Osub], V)
    rmo, rma = oracle.merge_multi(om, np.zeros((4, 36, 36, 3)), Osub)
    assert np.abs(mo.double().cpu().numpy() - rmo).max() <= 1e-4 * np.abs(rmo).max()
    assert np.abs(ma.double().cpu().numpy() - rma).max() <= 1e-4 * np.abs(rma).max()
    bx = np.flatnonzero(V[0].numpy() == 0)  # invalid rows of the X-fast scan of pair 1
    by = np.flatnonzero(V[1].numpy() == 0)  # invalid columns of its Y-fast scan
    assert bx.size and by.size
    cross = ma.cpu().numpy()[np.ix_(bx, by)]
    assert np.all(cross > 0.0)  # filled by the second pair
    log("the first pair alone leaves a gap there")
    M2 = octmc.Multi(sc.S[:2], sc.orient[:2], octa=O[:2], valid=V[:2], levels=1, iters_per_level=0)
    _, _, ma2, _ = M2.register(merged=True)
    torch.cuda.synchronize()
    assert np.all(ma2.cpu().numpy()[np.ix_(bx, by)] == 0.0)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_multi_merge_odd_depth_16bit(octmc, dtype):
    """The merge of four volumes of odd depth in 16-bit storage (stored with a
    padding sample per A-scan) at identity fields: element-wise the oracle's
    merge of the volumes rounded to the storage type."""
    sc = synth.make_scans("tiny", 5, (0, 1, 0, 1), n=30, d=37, white_lines=True)
    log(f"n = 4 merge at identity fields, 30x30x37 {dtype}")
    M = octmc.Multi(sc.S, sc.orient, octa=sc.O, valid=sc.V, levels=1, iters_per_level=0, dtype=dtype)
    D, mo, _, _ = M.register(merged=True)
    torch.cuda.synchronize()
    assert not D.any()
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16
    Sr = [t.to(tt).to(torch.float32) for t in sc.S]
    Osub = [oracle.substitute_invalid(sc.O[q], sc.V[q], sc.orient[q]) for q in range(4)]
    om = oracle.Multi(Sr, sc.orient, [oracle.enface_mean(o) for o in Osub], sc.V)
    rmo, _ = oracle.merge_multi(om, np.zeros((4, 30, 30, 3)), Osub)
    assert mo.shape == (30, 30, 37)
    assert np.abs(mo.double().cpu().numpy() - rmo).max() <= 1e-4 * np.abs(rmo).max()


def test_multi_rejects_bad_input(octmc, scans):
    sc = scans
    with pytest.raises(octmc.OctmcError):
        octmc.Multi(sc.S[:1], [0], enface=sc.A[:1])
    with pytest.raises(octmc.OctmcError):
        octmc.Multi([sc.S[0], sc.S[2]], [0, 0], enface=[sc.A[0], sc.A[2]])  # no orthogonal scan
    with pytest.raises(octmc.OctmcError):
        _gpu_multi(octmc, sc, prealign_iters=5, flags=octmc.PREALIGN)


_STORE = {"f32": 0, "bf16": 1, "f16": 2}


def _oracle_level_inputs(sc, level, idx, store=0):
    """The oracle's volumes, en face images and validity at `level`: the exact
    pyramid, each structural level rounded to the storage type as stored
    (16-bit storage: levels built in single precision, as the device builds
    them, so both sides take the same rounding decisions)."""
    S = [sc.S[q].double().numpy() for q in idx]
    A = [sc.A[q].double().numpy() for q in idx]
    V = [sc.V[q].double().numpy() for q in idx]
    down = oracle.pyr_down3_f32 if store else oracle.pyr_down3
    for _ in range(level):
        S = [down(s) for s in S]
        A = [oracle.pyr_down2(a) for a in A]
        V = [oracle.pyr_down1(v) for v in V]
    if store:
        S = [oracle.round_storage(s, store) for s in S]
    return S, A, V


@pytest.mark.parametrize("dtype,level,nvol,sigma", [("bf16", 0, 4, 0.8), ("bf16", 1, 4, 0.8), ("f16", 0, 4, 0.8),
                                                    ("bf16", 0, 3, 0.8), ("f16", 1, 3, 0.8), ("bf16", 0, 4, 12.0),
                                                    ("f32", 0, 4, 0.8), ("f32", 1, 3, 0.8), ("f32", 0, 4, 12.0)])
def test_multi_fused_objective_parity(octmc, scans, dtype, level, nvol, sigma):
    """n = 3 and 4 volumes: the fused structural pass (each volume resampled
    once per output A-scan; two samples per lane in 16-bit storage, one in
    float32) against the oracle on the volumes rounded as stored (10^-4
    relative), and against the pair-by-pair evaluation of the same library
    (float32 rounding apart).  sigma = 12 px puts many taps outside the
    volume (clamped) and above or below the A-scan."""
    sc = scans
    idx = list(range(nvol))
    M = _gpu_multi(octmc, sc, idx, levels=2, dtype=dtype)
    Mp = _gpu_multi(octmc, sc, idx, levels=2, dtype=dtype, pairwise=True)
    w, h, d = M.level_shape(level)
    assert dtype == "f32" or d % 2 == 0  # 16-bit storage: the fused pass serves even depths
    rng = np.random.default_rng(10 + level + nvol)
    D = rng.normal(0, sigma, (nvol, h, w, 3))
    S, A, V = _oracle_level_inputs(sc, level, idx, _STORE[dtype])
    om = oracle.Multi(S, [sc.orient[q] for q in idx], A, V)
    t0, p05, _ = oracle.evaluate_multi(om, D, oracle.Params(), None, grad=False)
    eta = np.array([oracle.eta_from_terms(a, b) for a, b in p05])
    ref, _, gref = oracle.evaluate_multi(om, D, oracle.Params(), eta)
    log(f"n = {nvol} fused objective, {dtype}, level {level} ({w}x{h}x{d})")
    Dg = torch.from_numpy(D).float().cuda()
    t, g = M.eval(level, Dg, eta_mode=0)
    tp, gp = Mp.eval(level, Dg, eta_mode=0)
    torch.cuda.synchronize()
    td, tpd = octmc.terms_dict(t), octmc.terms_dict(tp)
    for key in ("F", "data", "str", "ang", "reg", "mean"):
        assert rel(td[key], ref[key]) < 1e-4, (key, td[key], ref[key])
        assert rel(td[key], tpd[key]) < 1e-5 or abs(td[key] - tpd[key]) < 1e-9, (key, td[key], tpd[key])
    assert grad_err(g.double().cpu().numpy(), gref) < 1e-4
    assert grad_rel(g.double().cpu().numpy(), gp.double().cpu().numpy()) < 1e-5


@pytest.mark.parametrize("dtype,pairwise", [("bf16", False), ("bf16", True), ("f16", False), ("f32", False)])
def test_multi_odd_depth_level(octmc, dtype, pairwise):
    """A level of odd depth (66 -> 33): the 16-bit volumes are stored with a
    padding sample per A-scan (an even pitch), so the fused pass and the pair
    kernels both take two samples per lane; float32 storage takes the fused
    one-sample pass.  Every form meets the oracle's bar."""
    sc = synth.make_scans("tiny", 4, (0, 1, 0, 1), n=36, d=66)
    M = _gpu_multi(octmc, sc, levels=2, dtype=dtype, pairwise=pairwise)
    w, h, d = M.level_shape(1)
    assert d % 2 == 1
    D = np.random.default_rng(2).normal(0, 0.5, (4, h, w, 3))
    S, A, V = _oracle_level_inputs(sc, 1, range(4), _STORE[dtype])
    om = oracle.Multi(S, sc.orient, A, V)
    ref, _, gref = oracle.evaluate_multi(om, D, oracle.Params(), np.ones(6))
    log(f"n = 4 {dtype} pairwise={pairwise}, odd depth at level 1")
    t, g = M.eval(1, torch.from_numpy(D).float().cuda(), eta_mode=1)  # stored eta = 1
    torch.cuda.synchronize()
    td = octmc.terms_dict(t)
    for key in ("F", "data", "str", "reg"):
        assert rel(td[key], ref[key]) < 1e-4, (key, td[key], ref[key])
    assert grad_err(g.double().cpu().numpy(), gref) < 1e-4


def test_multi_fused_register_parity(octmc, scans):
    """The joint BF16 solve (fused structural pass at every level) against the
    oracle's solve on pyramid levels rounded as stored: 0.05 px RMS."""
    sc = scans
    log("n = 4 bf16 joint solve, 2 levels x 40 steps, GPU")
    M = _gpu_multi(octmc, sc, levels=2, iters_per_level=40, dtype="bf16")
    Dg, _, _, rep = M.register()
    torch.cuda.synchronize()
    log("the same solve in the oracle, levels rounded to bfloat16")
    Do, repo = oracle.register_multi(_oracle_multi(sc), oracle.Params(levels=2, iters=40, store=1))
    err = np.sqrt(((Dg.double().cpu().numpy() - Do) ** 2).mean())
    assert err < 0.05, err
    for r, ro in zip(rep, repo):
        assert abs(r["f_end"] - ro["f_end"]) <= 0.05 * abs(ro["f_end"]), (r, ro)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_multi_fused_full_size_matches_pairwise(octmc, dtype):
    """Four volumes of 300 x 300 A-scans x 640 samples, in the launch
    configuration the benchmark times: the fused structural pass against the
    pair-by-pair evaluation (each pair's structural kernel is pinned to the
    oracle by the pair tests, at full size included), float32 rounding
    apart, at levels 0 and 1."""
    log(f"four volumes 300x300x640 on cuda, {dtype}")
    sc = synth.make_scans("clinical", 0, (0, 1, 0, 1), device="cuda", white_lines=True)
    M = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, dtype=dtype)
    Mp = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, dtype=dtype, pairwise=True)
    gen = torch.Generator().manual_seed(4)
    for level in (0, 1):
        w, h, d = M.level_shape(level)
        D = (1.5 * torch.randn((4, h, w, 3), generator=gen)).float().cuda()
        log(f"fused vs pairwise, level {level} ({w}x{h}x{d})")
        t, g = M.eval(level, D, eta_mode=0)
        tp, gp = Mp.eval(level, D, eta_mode=0)
        torch.cuda.synchronize()
        td, tpd = octmc.terms_dict(t), octmc.terms_dict(tp)
        for key in ("F", "data", "str", "ang", "reg", "mean"):
            assert rel(td[key], tpd[key]) < 1e-5 or abs(td[key] - tpd[key]) < 1e-9, (level, key, td[key], tpd[key])
        assert grad_rel(g.double().cpu().numpy(), gp.double().cpu().numpy()) < 1e-5
    M.close()
    Mp.close()
