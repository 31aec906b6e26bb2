"""GPU parity of the hot path (one objective + gradient evaluation) against
the FP64 oracle, through the C ABI.

Tolerance: 1e-4 relative on the objective terms, and on the gradient 1e-4
both norm-wise and element-wise (|g - g_ref| <= 1e-4 (|g_ref| + 0.1
max |g_ref|), the floor set by the float32 rounding of the residual that the
pseudo-Huber kink magnifies; see gpu_util.ELEM_FLOOR), float32 kernels
against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import grad_err, grad_rel, log, make_field, rel, round_storage

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _gpu_pair(octmc, pair, dtype="f32", **kw):
    return octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=dtype, **kw)


def _orc_params(P):
    p = P.params
    return oracle.Params(alpha=p.alpha, delta0=p.delta0, eps_h=p.eps_huber, eps_r=p.eps_reg,
                         flyback_frac=p.flyback_frac, mean_weight=p.mean_weight)


def _compare(octmc, P, lv, level, D, tag, tol=TOL, eta_mode=0):
    log(f"eval {tag} level={level} shape={lv.whd}")
    Dg = D.to(device="cuda", dtype=torch.float32)
    terms, g = P.eval(level, Dg, eta_mode=eta_mode)
    torch.cuda.synchronize()
    assert torch.isfinite(terms).all() and torch.isfinite(g).all(), tag
    t = octmc.terms_dict(terms)
    prm = _orc_params(P)
    # the oracle sees exactly the float32 displacement the GPU saw
    D32 = Dg.double().cpu().numpy()
    eta = oracle.eta_at(lv, D32, prm) if eta_mode == 0 else t["eta"]
    assert rel(t["eta"], eta) < tol, (tag, t["eta"], eta)
    ref, gref = oracle.evaluate(lv, D32, prm, eta)
    for k in ("F", "data", "str", "ang", "reg", "str05", "ang05"):
        assert rel(t[k], ref[k]) < tol or abs(t[k] - ref[k]) < 1e-9 * max(1.0, abs(ref["F"])), (tag, k, t[k], ref[k])
    assert abs(t["mean"] - ref["mean"]) <= tol * max(abs(ref["mean"]), 1e-6 * abs(ref["F"])), (tag, t["mean"], ref["mean"])
    e = grad_err(g.double().cpu().numpy(), gref)
    assert e < tol, (tag, e)
    return t, g


@pytest.mark.parametrize("case", ["zero", "gt", "gt_noise", "smooth", "uniform"])
def test_eval_parity_tiny(octmc, case):
    pair = synth.make_pair("tiny")
    P = _gpu_pair(octmc, pair, levels=3)
    lv = oracle.level_from_pair(pair)
    _compare(octmc, P, lv, 0, make_field(pair, case, seed=3), f"tiny/{case}")


def test_eval_parity_ragged_all_levels(octmc):
    # 40 x 40 A-scans (several blocks, ragged last block), 150 samples
    # (two full depth chunks and a ragged tail); every pyramid level
    pair = synth.make_pair("tiny", n=40, d=150)
    P = _gpu_pair(octmc, pair, levels=3)
    pyr = oracle.pyramid(oracle.level_from_pair(pair), 3)
    for level in range(3):
        w, h, d = P.level_shape(level)
        assert (w, h, d) == pyr[level].whd
        D = synth.smooth_random_field(w, h, 1.5, seed=10 + level)
        _compare(octmc, P, pyr[level], level, D, f"ragged/L{level}")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_eval_parity_odd_depth(octmc, dtype):
    """Odd depth at the finest level (151, then 76): with float32 storage the
    last sample of an A-scan falls in a ragged depth step; 16-bit storage keeps
    one padding sample per A-scan and the two-samples-per-lane kernel.  Random
    fields give both parities of the first depth tap in both scans."""
    pair = synth.make_pair("tiny", n=36, d=151)
    # the library builds every level in float32 from the unrounded level above
    # and stores it rounded; the oracle's rounded pyramid takes the same
    # rounding decisions (oracle.pyramid with store = 1)
    pyr = oracle.pyramid(oracle.level_from_pair(pair), 2, store=0 if dtype == "f32" else 1)
    P = _gpu_pair(octmc, pair, dtype=dtype, levels=2)
    for level in range(2):
        w, h, d = P.level_shape(level)
        for case, seed in (("uniform", 1), ("smooth", 2)):
            D = synth.random_field(w, h, 3.0, seed) if case == "uniform" else synth.smooth_random_field(w, h, 2.5, seed)
            _compare(octmc, P, pyr[level], level, D, f"odd/{dtype}/{level}/{case}")


@pytest.mark.parametrize("n,d,dtype", [(4, 4, "f32"), (4, 4, "bf16"), (5, 5, "bf16"), (5, 6, "f16"), (6, 4, "f16"),
                                       (7, 9, "f32")])
def test_eval_parity_minimal_shapes(octmc, n, d, dtype):
    """The smallest scans the library takes (4 x 4 x 4) and a few other tiny
    shapes: every A-scan's 4 x 4 x 4 neighbourhood reaches past the volume on
    some side (random fields of up to 3 px, smooth ones of 2.5 px), an odd
    width leaves the 2 x 2 tiles of the last row and column partly outside
    the scan, and the depth is far below one depth step of the structural
    kernels (16-bit storage takes the two-samples-per-lane kernel at every
    depth, odd ones with a padding sample; float32 the one-sample kernel)."""
    pair = synth.make_pair("tiny", n=n, d=d)
    P = _gpu_pair(octmc, pair, dtype=dtype, levels=1)
    lv = oracle.level_from(round_storage(pair.sx, dtype), round_storage(pair.sy, dtype), pair.ax, pair.ay,
                           pair.vx, pair.vy)
    for case, seed in (("uniform", 1), ("smooth", 2)):
        D = synth.random_field(n, n, 3.0, seed) if case == "uniform" else synth.smooth_random_field(n, n, 2.5, seed)
        _compare(octmc, P, lv, 0, D, f"minimal/{n}x{n}x{d}/{dtype}/{case}")


def test_eval_parity_validity_and_white_lines(octmc):
    pair = synth.make_pair("tiny", n=48, d=64, white_lines=True)
    assert (pair.vx == 0).any() and (pair.vy == 0).any()
    P = _gpu_pair(octmc, pair, levels=2)
    lv = oracle.level_from_pair(pair)
    for case in ("gt", "gt_noise"):
        _compare(octmc, P, lv, 0, make_field(pair, case, seed=5), f"white/{case}")


def test_eval_parity_delta0_zero_and_params(octmc):
    pair = synth.make_pair("tiny", n=32, d=48)
    P = _gpu_pair(octmc, pair, levels=2, delta0=0.0, alpha=0.3, eps_reg=0.05, mean_weight=2.5)
    lv = oracle.level_from_pair(pair)
    t, _ = _compare(octmc, P, lv, 0, make_field(pair, "gt_noise", seed=2), "delta0=0")
    assert t["ang"] == 0.0


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_eval_parity_storage_types(octmc, dtype):
    pair = synth.make_pair("tiny")
    P = _gpu_pair(octmc, pair, dtype=dtype, levels=3)
    # compute error: the oracle reads the volumes rounded to the storage type
    lv = oracle.level_from(round_storage(pair.sx, dtype), round_storage(pair.sy, dtype), pair.ax, pair.ay,
                           pair.vx, pair.vy)
    _compare(octmc, P, lv, 0, make_field(pair, "gt_noise", seed=4), f"{dtype}/compute")


def test_eval_is_deterministic_and_eta_mode(octmc):
    pair = synth.make_pair("tiny", n=40, d=96)
    P = _gpu_pair(octmc, pair, levels=2)
    D = make_field(pair, "gt_noise", 1).float().cuda()
    t1, g1 = P.eval(0, D, eta_mode=0)
    t1, g1 = t1.clone(), g1.clone()
    t2, g2 = P.eval(0, D, eta_mode=1)
    torch.cuda.synchronize()
    assert torch.equal(t1, t2)
    assert torch.equal(g1, g2)
    # eta_mode 1 keeps the stored eta when the field changes
    D2 = make_field(pair, "smooth", 2).float().cuda()
    t3, _ = P.eval(0, D2, eta_mode=1)
    assert t3[octmc.TERM_ETA].item() == t1[octmc.TERM_ETA].item()


def test_eval_batched_matches_single(octmc):
    pairs = [synth.make_pair("batch", p, n=40, d=64) for p in range(3)]
    Ps = [_gpu_pair(octmc, q, levels=2) for q in pairs]
    D = torch.stack([make_field(q, "gt_noise", k) for k, q in enumerate(pairs)]).float().cuda()
    log("batched eval 3 pairs")
    tb, gb = octmc.eval_batched(Ps, 0, D, eta_mode=0)
    for k, P in enumerate(Ps):
        t, g = P.eval(0, D[k], eta_mode=0)
        torch.cuda.synchronize()
        assert torch.equal(t, tb[k])
        assert torch.equal(g, gb[k])
    lv = oracle.level_from_pair(pairs[1])
    _compare(octmc, Ps[1], lv, 0, D[1].double().cpu(), "batched/oracle")


@pytest.mark.slow
@pytest.mark.parametrize("workload,dtype,d", [("clinical", "f32", None), ("dense", "bf16", None), ("dense", "f16", None),
                                              ("dense", "f32", None), ("dense", "bf16", 465)])
def test_eval_parity_full_size_whole_objective(octmc, workload, dtype, d):
    """The clinical (300 x 300 x 640, float32) and the dense (500 x 500 x 800,
    BF16, FP16 and float32 storage) pairs, and the dense pair at the paper's
    depth of 465 samples (odd: BF16 stored with a padding sample), generated
    on the GPU, in the launch configuration the benchmark times, with the
    default alpha and mean term and eta computed at the field (Eq. 10): F,
    every term (both data terms, the regulariser, the mean term, eta) and every
    gradient entry of all A-scans against the oracle (Eqs. 1-10)."""
    log(f"generate {workload} (depth {d or 'as defined'}) on cuda, storage {dtype}")
    pair = synth.make_pair(workload, device="cuda", octa_volumes=False, d=d)
    P = _gpu_pair(octmc, pair, dtype=dtype, levels=4)
    sx, sy = round_storage(pair.sx, dtype), round_storage(pair.sy, dtype)
    lv = oracle.Level(*(oracle._f64(t) for t in (sx, sy, pair.ax, pair.ay, pair.vx, pair.vy)))
    del sx, sy
    _compare(octmc, P, lv, 0, make_field(pair, "gt_noise", seed=7), f"{workload}/{dtype}/whole objective")
    P.close()


@pytest.mark.slow
def test_eval_transposed_problem_full_size(octmc):
    """Transposing both scans (i <-> j), swapping the X-fast and Y-fast roles
    and the x and y components maps the objective onto itself, the symmetry
    the oracle is pinned to.  At the benchmark's size and storage (500 x 500
    x 800, BF16) the whole objective (eta at the field, both data terms,
    regulariser, mean term) and its gradient agree between the two problems;
    the two runs read the volumes in different orders, so this checks the
    X-fast and Y-fast paths of the kernels against each other at full size."""
    log("generate dense 500x500x800 on cuda (with its transpose)")
    pair = synth.make_pair("dense", device="cuda", octa_volumes=False)

    def T(v):
        return v.transpose(0, 1).contiguous()

    def swap(D):  # fields of the transposed problem <-> fields of the original
        return torch.stack([T(D[1])[..., [1, 0, 2]], T(D[0])[..., [1, 0, 2]]]).contiguous()

    P = _gpu_pair(octmc, pair, dtype="bf16", levels=4)
    Q = octmc.Pair(T(pair.sy), T(pair.sx), ax=T(pair.ay), ay=T(pair.ax), vx=pair.vy, vy=pair.vx, dtype="bf16",
                   levels=4)
    D = make_field(pair, "gt_noise", seed=11).float().cuda()
    log("eval original and transposed problems, level 0, eta at the field")
    t, g = P.eval(0, D, eta_mode=0)
    tq, gq = Q.eval(0, swap(D), eta_mode=0)
    torch.cuda.synchronize()
    a, b = octmc.terms_dict(t), octmc.terms_dict(tq)
    for k in ("eta", "F", "data", "str", "ang", "reg", "str05", "ang05"):
        assert rel(b[k], a[k]) < 1e-5, (k, a[k], b[k])
    assert abs(b["mean"] - a["mean"]) <= 1e-5 * max(abs(a["mean"]), 1e-6 * abs(a["F"])), (a["mean"], b["mean"])
    assert grad_rel(swap(gq).double().cpu().numpy(), g.double().cpu().numpy()) < 1e-5


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_eval_parity_max_size_sampled(octmc, dtype):
    """The largest accepted volume (800 x 800 A-scans x 838 samples: w h d
    float32 samples stay below 2^31 bytes): the data gradient of sampled
    A-scans, corners and edges included, against the oracle, in the storage
    types that use the one-sample and the two-sample structural kernel."""
    n, d = 800, 838
    log(f"generate {n}x{n}x{d} on cuda, storage {dtype}")
    pair = synth.make_pair("dense", 1, n=n, d=d, device="cuda", octa_volumes=False)
    P = _gpu_pair(octmc, pair, dtype=dtype, levels=4, alpha=0.0, mean_weight=0.0)
    D = make_field(pair, "gt_noise", seed=3)
    Dg = D.float().cuda()
    log(f"eval {n}x{n}x{d} level 0")
    terms, g = P.eval(0, Dg, eta_mode=1)
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    rng = np.random.default_rng(1)
    sample = np.concatenate([[0, n - 1, n * (n - 1), n * n - 1, n * (n // 2) + n // 2, n * 7, n * 7 + n - 1],
                             rng.integers(0, n * n, 121)])
    sx, sy = round_storage(pair.sx, dtype), round_storage(pair.sy, dtype)
    log("oracle on the sampled A-scans")
    lv = oracle.Level(*(oracle._f64(t) for t in (sx, sy, pair.ax, pair.ay, pair.vx, pair.vy)))
    del sx, sy
    _, gref = oracle.data_ascans(lv, Dg.double().cpu().numpy(), sample, _orc_params(P), 1.0)
    gg = g.double().cpu().numpy().reshape(2, -1, 3)
    got = np.concatenate([gg[0][sample], gg[1][sample]], axis=1)
    assert grad_err(got, gref) < TOL


def test_check_nan_rejects_non_finite_volumes(octmc):
    """OCTMC_CHECK_NAN: a NaN or an Inf in a structural volume makes pair
    creation fail with OCTMC_E_NAN (-6); the same volumes pass without the
    flag, and finite volumes pass with it."""
    pair = synth.make_pair("tiny", n=24, d=32)
    for bad in (float("nan"), float("inf")):
        sy = pair.sy.clone()
        sy[5, 7, 11] = bad
        log(f"pair creation with {bad} and OCTMC_CHECK_NAN")
        with pytest.raises(octmc.OctmcError) as e:
            octmc.Pair(pair.sx, sy, ax=pair.ax, ay=pair.ay, levels=2, flags=octmc.CHECK_NAN)
        assert e.value.code == -6
        octmc.Pair(pair.sx, sy, ax=pair.ax, ay=pair.ay, levels=2).close()
    octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, levels=2, flags=octmc.CHECK_NAN).close()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_degenerate_identical_and_constant_scans(octmc, dtype):
    """Degenerate inputs.  Identical scans at zero displacement: every
    resampled sample is the stored sample itself (the interpolation weights
    are 0, 1, 0, 0), so the structural term and its gradient are exactly
    zero.  Constant volumes at any displacement: the structural term matches
    the oracle (it is zero up to rounding) and so does the gradient.  Eq. 10
    leaves eta undefined when the structural term at delta0 vanishes; here it
    is zero only up to rounding (outside the exact-zero guard that sets
    eta = 1), so eta is given (stored eta = 1) rather than computed."""
    pair = synth.make_pair("tiny", n=32, d=48)
    h, w, _ = pair.sx.shape
    log(f"identical scans, zero displacement, {dtype}")
    P = octmc.Pair(pair.sx, pair.sx, ax=pair.ax, ay=pair.ax, levels=2, dtype=dtype, alpha=0.0, mean_weight=0.0)
    t, g = P.eval(0, torch.zeros((2, h, w, 3), device="cuda"), eta_mode=1)
    torch.cuda.synchronize()
    td = octmc.terms_dict(t)
    assert td["str"] == 0.0 and td["ang"] == 0.0 and td["F"] == 0.0
    assert not g.any()
    P.close()
    log(f"constant volumes, random displacement, {dtype}")
    c = torch.full_like(pair.sx, 0.375)  # exact in every storage type
    P = octmc.Pair(c, c, ax=pair.ax, ay=pair.ay, levels=2, dtype=dtype)
    lv = oracle.level_from(c, c, pair.ax, pair.ay)
    t, _ = _compare(octmc, P, lv, 0, make_field(pair, "uniform", seed=5), f"constant/{dtype}", eta_mode=1)
    assert abs(t["str"]) <= 1e-6 * abs(t["F"])
    P.close()
