"""GPU parity of the full solve (pyramid, eta per level, L-BFGS, level
transitions) and of the merge against the FP64 oracle, through the C ABI.

Final displacements: <= 0.05 px RMS against the oracle's FP64 solve."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _orc_params(p):
    return oracle.Params(alpha=p.alpha, delta0=p.delta0, eps_h=p.eps_huber, eps_r=p.eps_reg,
                         flyback_frac=p.flyback_frac, mean_weight=p.mean_weight, levels=p.levels,
                         iters=p.iters_per_level, lbfgs_m=p.lbfgs_m, ls_max_evals=p.ls_max_evals, c1=p.c1, c2=p.c2,
                         merge_kappa=p.merge_kappa, merge_tau=p.merge_tau)


@pytest.mark.parametrize("iters", [100])
def test_register_matches_oracle_tiny(octmc, iters):
    pair = synth.make_pair("tiny")
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, levels=3,
                   iters_per_level=iters)
    log(f"register tiny iters={iters}")
    D, _, _, rep = P.register()
    torch.cuda.synchronize()
    Dg = D.double().cpu().numpy()
    Do, orep = oracle.register(oracle.level_from_pair(pair), _orc_params(P.params))
    diff = np.sqrt(((Dg - Do) ** 2).mean())
    print("levels gpu", rep, "oracle", orep, "rms diff", diff)
    assert len(rep) == 3
    assert abs(rep[0]["eta"] - orep[0]["eta"]) < 1e-6 * orep[0]["eta"]
    for r, o in zip(rep, orep):
        assert r["f_end"] < r["f_start"]
        assert abs(r["f_end"] - o["f_end"]) < 0.05 * o["f_end"]
    assert diff <= 0.05, diff


@pytest.mark.parametrize("n,d,dtype,levels", [(4, 4, "f32", 1), (6, 8, "bf16", 1), (9, 11, "f32", 2),
                                              (9, 11, "bf16", 2), (7, 5, "f16", 1)])
def test_register_minimal_shapes_vs_oracle(octmc, n, d, dtype, levels):
    """Whole solves of the smallest scans (every neighbourhood reaches past
    the volume; a 9 x 9 x 11 pair has a second level of 5 x 5 x 6; odd
    depths in 16-bit storage are stored with a padding sample): the final
    field within 0.05 px RMS of the oracle's solve on the volumes as
    stored."""
    pair = synth.make_pair("tiny", n=n, d=d)
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, levels=levels, dtype=dtype)
    log(f"register minimal {n}x{n}x{d} {dtype} levels={levels}")
    D, _, _, rep = P.register()
    torch.cuda.synchronize()
    prm = _orc_params(P.params)
    prm.store = {"f32": 0, "bf16": 1, "f16": 2}[dtype]
    Do, orep = oracle.register(oracle.level_from_pair(pair), prm)
    diff = np.sqrt(((D.double().cpu().numpy() - Do) ** 2).mean())
    print("levels gpu", rep, "oracle", orep, "rms diff", diff)
    assert len(rep) == levels
    assert diff <= 0.05, diff


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_register_storage_types_vs_oracle(octmc, dtype):
    """BF16 / FP16 storage: the displacement error against the FP64 oracle,
    twice.  Against the oracle whose pyramid levels are rounded to the same
    storage type it is compute error
    only and meets the FP32 bar (0.05 px RMS); against the oracle on the
    float32 volumes it is the effect of the rounding on the minimiser, stated
    and bounded by 0.25 px RMS (the recovery bar of the tiny workload)."""
    pair = synth.make_pair("tiny")
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, levels=3, dtype=dtype)
    log(f"register tiny storage={dtype}")
    D, _, _, rep = P.register()
    torch.cuda.synchronize()
    Dg = D.double().cpu().numpy()
    prm = _orc_params(P.params)
    lv = oracle.level_from_pair(pair)
    prm.store = {"bf16": 1, "f16": 2}[dtype]
    Dr, _ = oracle.register(lv, prm)  # every pyramid level rounded as stored
    prm.store = 0
    Df, _ = oracle.register(lv, prm)
    compute = np.sqrt(((Dg - Dr) ** 2).mean())
    storage = np.sqrt(((Dg - Df) ** 2).mean())
    print(f"{dtype}: RMS vs oracle on rounded volumes {compute:.4f} px, vs oracle on float32 volumes "
          f"{storage:.4f} px")
    assert compute <= 0.05, compute
    assert storage <= 0.25, storage


def test_module_register_equals_pair_register(octmc):
    """The one-call form (octmc.register: create, solve, merge, destroy) gives
    the field, merged volumes and report of the explicit pair, bit for bit,
    with en face images and with OCTA volumes (projected en face images)."""
    pair = synth.make_pair("tiny", n=48, d=64)
    log("module-level register against the explicit pair")
    D1, mo1, ma1, rep1 = octmc.register(pair.sx, pair.sy, enface_x=pair.ax, enface_y=pair.ay, valid_x=pair.vx,
                                        valid_y=pair.vy, levels=2)
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, levels=2)
    D2, mo2, ma2, rep2 = P.register(merged=True)
    torch.cuda.synchronize()
    P.close()
    assert rep1 == rep2
    assert torch.equal(D1, D2) and torch.equal(mo1, mo2)
    assert ma1 is None and ma2 is None
    D3, mo3, ma3, rep3 = octmc.register(pair.sx, pair.sy, pair.ox, pair.oy, levels=2, dtype="bf16",
                                        project_enface=True)
    Q = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, levels=2, dtype="bf16", project_enface=True)
    D4, mo4, ma4, rep4 = Q.register(merged=True)
    torch.cuda.synchronize()
    Q.close()
    assert rep3 == rep4
    assert torch.equal(D3, D4) and torch.equal(mo3, mo4) and torch.equal(ma3, ma4)


def test_register_recovers_motion(octmc):
    # pair 1 needs more than 100 steps per level to converge (so does the oracle)
    pair = synth.make_pair("tiny", pair=1)
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, levels=3, iters_per_level=300)
    D, _, _, _ = P.register()
    from test_oracle_pins import recovery_mask
    m = recovery_mask(pair)
    e = D.double().cpu().numpy() - pair.d_gt.numpy()
    e -= e[m].mean(axis=0)
    rms = np.sqrt((e[m] ** 2).mean(axis=0))
    assert np.all(rms < 0.3), rms


def test_merge_matches_oracle(octmc):
    pair = synth.make_pair("tiny", n=40, d=72, white_lines=True)
    P = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, vx=pair.vx, vy=pair.vy, levels=2)
    D = synth.perturbed_field(pair.d_gt, 0.2, 3).float()
    log("merge 40x40x72")
    mo, ma = P.merge(D.cuda(), octa=True)
    torch.cuda.synchronize()
    ox = oracle.substitute_invalid(pair.ox, pair.vx, 0)
    oy = oracle.substitute_invalid(pair.oy, pair.vy, 1)
    ro, ra, _, _ = oracle.merge(pair.sx, pair.sy, D.double(), ox, oy, pair.vx, pair.vy,
                                P.params.merge_kappa, P.params.merge_tau)
    assert np.abs(mo.double().cpu().numpy() - ro).max() < 1e-4 * max(1.0, np.abs(ro).max())
    assert np.abs(ma.double().cpu().numpy() - ra).max() < 1e-4 * max(1.0, np.abs(ra).max())


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_merge_matches_oracle_odd_depth_16bit(octmc, dtype):
    """The merge of an odd depth in 16-bit storage, whose volumes the library
    stores with one padding sample per A-scan: element-wise against the
    oracle's merge of the volumes rounded to the storage type."""
    pair = synth.make_pair("tiny", n=36, d=71, white_lines=True)
    P = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, vx=pair.vx, vy=pair.vy, levels=2, dtype=dtype)
    D = synth.perturbed_field(pair.d_gt, 0.4, 5).float()
    log(f"merge 36x36x71 {dtype}")
    mo, _ = P.merge(D.cuda(), octa=False)
    torch.cuda.synchronize()
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16
    sx, sy = pair.sx.to(tt).to(torch.float32), pair.sy.to(tt).to(torch.float32)
    ox = oracle.substitute_invalid(pair.ox, pair.vx, 0)
    oy = oracle.substitute_invalid(pair.oy, pair.vy, 1)
    ro, _, _, _ = oracle.merge(sx, sy, D.double(), ox, oy, pair.vx, pair.vy, P.params.merge_kappa,
                               P.params.merge_tau)
    assert mo.shape == (36, 36, 71)
    assert np.abs(mo.double().cpu().numpy() - ro).max() < 1e-4 * max(1.0, np.abs(ro).max())


def test_register_with_merge_and_enface_from_octa(octmc):
    pair = synth.make_pair("tiny", n=32, d=40)
    P = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, levels=2, iters_per_level=10)
    D, mo, ma, rep = P.register(merged=True)
    torch.cuda.synchronize()
    assert mo.shape == (32, 32, 40) and ma.shape == (32, 32, 40)
    assert torch.isfinite(mo).all() and torch.isfinite(ma).all()
    assert all(r["iters"] <= 10 for r in rep)


def test_automatic_levels_equal_the_explicit_count(octmc):
    """levels = 0 resolves to the fewest levels whose coarsest level is at
    most 16 A-scans wide (96 -> 48 -> 24 -> 12: 4 levels); the solve is then
    bit for bit the one with levels = 4, for a pair and for four volumes."""
    pair = synth.make_pair("tiny", 2, n=96, d=64)
    kw = dict(ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, iters_per_level=20)
    log("pair with levels = 0")
    P0 = octmc.Pair(pair.sx, pair.sy, levels=0, **kw)
    P4 = octmc.Pair(pair.sx, pair.sy, levels=4, **kw)
    assert P0.levels == 4 and P4.levels == 4
    D0, _, _, r0 = P0.register()
    D4, _, _, r4 = P4.register()
    torch.cuda.synchronize()
    assert len(r0) == 4 and torch.equal(D0, D4)
    log("four volumes with levels = 0")
    sc = synth.make_scans("tiny", 5, (0, 1, 0, 1), n=96, d=64)
    M0 = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=0, iters_per_level=10)
    M4 = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, iters_per_level=10)
    E0, _, _, q0 = M0.register()
    E4, _, _, q4 = M4.register()
    torch.cuda.synchronize()
    assert len(q0) == 4 and torch.equal(E0, E4)


# Stored FP64 oracle solves of the larger workloads (tests/golden, written by
# tests/golden/make_solve_golden.py from the oracle alone).  The solve is
# chaotic at these sizes: the oracle's own solution moves by 0.08-0.15 px RMS
# when its input volumes are perturbed by a relative 1e-7 or 1e-6 (measured at
# 300 x 300 x 640 with 4 and 6 levels; the distance does not shrink with the
# perturbation), so no float32 implementation can match it to 0.05 px there.
# Each golden of float32 inputs stores that distance, and the bar is
# GOLDEN_FACTOR times it (never below the 0.05 px of the tiny workload); the
# per-level objectives must agree to 5 % (as for the tiny workload; measured:
# within 1.1 %), and the GPU solve must be as far
# from the ground truth as the oracle's, to 0.05 px per component.
GOLDEN_FACTOR = 4.0
GOLDEN_CASES = [("clinical", 4, 0, "f32"), ("clinical", 4, 1, "bf16"), ("clinical", 6, 0, "f32"),
                ("dense", 4, 0, "bf16")]


@pytest.mark.slow
@pytest.mark.parametrize("workload,levels,store,dtype", GOLDEN_CASES)
def test_register_matches_stored_oracle_solve(octmc, workload, levels, store, dtype):
    """Full solves of the clinical (300 x 300 x 640) and dense (500 x 500 x
    800) pairs, generated on the GPU exactly as for the stored oracle solve
    (same input hash), at the workload's 4 levels and at the automatic depth,
    against the oracle's FP64 solve of the same inputs (rounded to the
    storage type for store = 1)."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_solve_golden as G
    g = G.load(workload, levels, store)
    if g is None:
        pytest.skip(f"no stored oracle solve of {workload} with {levels} levels, storage {store}")
    Do, meta = g
    sens = meta.get("perturbation", {}).get("rms_px")
    if sens is None:  # the sensitivity is a property of the inputs: take the float32-input golden's
        g0 = G.load(workload, levels, 0)
        sens = None if g0 is None else g0[1].get("perturbation", {}).get("rms_px")
    log(f"generate {workload} on cuda")
    pair = synth.make_pair(workload, meta["pair"], device="cuda", octa_volumes=False)
    assert G.input_hash(pair) == meta["input_sha256"], "the generator gave other inputs than the stored solve saw"
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=dtype,
                   levels=meta["params"]["levels"], iters_per_level=meta["params"]["iters"])
    log(f"register {workload} {dtype} levels {levels}")
    D, _, _, rep = P.register()
    torch.cuda.synchronize()
    Dg = D.double().cpu().numpy()
    rms = float(np.sqrt(((Dg - Do) ** 2).mean()))
    bar = max(0.05, GOLDEN_FACTOR * sens) if sens is not None else 0.05
    gt = pair.d_gt.numpy()
    e_gpu = np.sqrt(((Dg - gt) ** 2).reshape(-1, 3).mean(axis=0))
    e_orc = np.sqrt(((Do - gt) ** 2).reshape(-1, 3).mean(axis=0))
    print(f"{workload} {dtype} levels {levels}: {rms:.4f} px RMS from the oracle's solve "
          f"(its own sensitivity {sens} px, bar {bar:.3f} px); error against ground truth "
          f"{np.round(e_gpu, 3)} px, oracle's {np.round(e_orc, 3)} px")
    for r, o in zip(rep, meta["levels"]):
        assert abs(r["f_end"] - o["f_end"]) < 0.05 * o["f_end"], (r, o)
    assert np.all(np.abs(e_gpu - e_orc) <= 0.05), (e_gpu, e_orc)
    assert rms <= bar, (rms, bar)
