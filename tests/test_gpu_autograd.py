"""The batched objective as a torch.autograd.Function (OctmcObjective),
through the C ABI's grouped evaluation: F and dF/dD of every pair against the
FP64 oracle (1e-4 relative, as the single-pair parity tests), the backward
pass scaling by the incoming gradient, and central finite differences of the
GPU forward against the GPU backward.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import grad_err, grad_rel, log, make_field, rel

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _orc_params(P):
    p = P.params
    return oracle.Params(alpha=p.alpha, delta0=p.delta0, eps_h=p.eps_huber, eps_r=p.eps_reg,
                         flyback_frac=p.flyback_frac, mean_weight=p.mean_weight)


def _pairs(octmc, n, d, count, levels, device="cpu"):
    pairs = [synth.make_pair("batch", p, n=n, d=d, device=device, octa_volumes=False) for p in range(count)]
    Ps = [octmc.Pair(q.sx, q.sy, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, levels=levels) for q in pairs]
    return pairs, Ps


def _check_against_oracle(octmc, pairs, Ps, level, D, F, grad, tag):
    for b, (q, P) in enumerate(zip(pairs, Ps)):
        lv = oracle.pyramid(oracle.level_from_pair(q), level + 1)[level]
        eta = octmc.terms_dict(P.eval(level, D[b].detach().contiguous(), grad=False)[0])["eta"]
        ref, gref = oracle.evaluate(lv, D[b].detach().double().cpu().numpy(), _orc_params(P), eta)
        assert rel(F[b].item(), ref["F"]) < TOL, (tag, b, F[b].item(), ref["F"])
        e = grad_err(grad[b].double().cpu().numpy(), gref)
        assert e < TOL, (tag, b, e)


@pytest.mark.parametrize("level", [0, 1])
def test_objective_matches_oracle(octmc, level):
    pairs, Ps = _pairs(octmc, 40, 64, 3, levels=2)
    w, h, _ = Ps[0].level_shape(level)
    if level == 0:
        D0 = torch.stack([make_field(q, "gt_noise", k) for k, q in enumerate(pairs)])
    else:
        D0 = torch.stack([synth.smooth_random_field(w, h, 1.0, k) for k in range(len(pairs))])
    D = D0.float().cuda()
    log(f"autograd level {level}: eta at D0")
    octmc.eval_batched(Ps, level, D, eta_mode=0)
    D = D.clone().requires_grad_(True)
    log(f"autograd level {level}: forward + backward of 3 pairs")
    F = octmc.objective(D, Ps, level)
    F.sum().backward()
    torch.cuda.synchronize()
    assert F.dtype == torch.float64 and F.shape == (3,)
    assert D.grad is not None and D.grad.shape == D.shape and torch.isfinite(D.grad).all()
    _check_against_oracle(octmc, pairs, Ps, level, D, F, D.grad, f"level{level}")


def test_objective_backward_scales_incoming_gradient(octmc):
    pairs, Ps = _pairs(octmc, 40, 64, 3, levels=2)
    D = torch.stack([make_field(q, "smooth", k) for k, q in enumerate(pairs)]).float().cuda()
    octmc.eval_batched(Ps, 0, D, eta_mode=0)
    log("autograd backward scaling")
    terms, g = octmc.eval_batched(Ps, 0, D)
    Dr = D.clone().requires_grad_(True)
    F = octmc.objective(Dr, Ps, 0)
    c = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (c * F).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(F, terms[:, octmc.TERM_F])
    for b in range(3):
        assert torch.equal(Dr.grad[b], g[b] * c[b].float()), b


def _fd_check(octmc, Ps, D, ncoord, hstep, seed, tag):
    """Central differences of the GPU forward at ncoord random coordinates
    against the GPU backward.  Per coordinate the error allowed is 2 % of the
    derivative plus a floor for the float32 rounding of the perturbed A-scan's
    depth sum (about one ulp per depth step of a sum of order d, divided by
    2h: 2e-4 d for h = 1e-3); the O(h^2) truncation of the cubic interpolant
    is far below both."""
    B, _, h, w, _ = D.shape
    d = Ps[0].level_shape(0)[2]
    Dr = D.clone().requires_grad_(True)
    octmc.objective(Dr, Ps, 0).sum().backward()
    torch.cuda.synchronize()
    g = Dr.grad.detach().double().cpu().numpy()
    rng = np.random.default_rng(seed)
    fd, an = [], []
    log(f"{tag}: finite differences, {ncoord} coordinates, h={hstep}")
    for _ in range(ncoord):
        idx = (int(rng.integers(B)), int(rng.integers(2)), int(rng.integers(h)), int(rng.integers(w)),
               int(rng.integers(3)))
        Dp = D.clone()
        Dm = D.clone()
        Dp[idx] += hstep
        Dm[idx] -= hstep
        with torch.no_grad():
            fp = octmc.objective(Dp, Ps, 0)[idx[0]].item()
            fm = octmc.objective(Dm, Ps, 0)[idx[0]].item()
        fd.append((fp - fm) / (2 * hstep))
        an.append(g[idx])
    fd, an = np.array(fd), np.array(an)
    err = np.abs(fd - an)
    log(f"{tag}: max err {err.max():.3e}, rel norm {np.linalg.norm(fd - an) / np.linalg.norm(an):.3e}")
    assert np.linalg.norm(fd - an) <= 1e-2 * np.linalg.norm(an)
    assert np.all(err <= 2e-2 * np.abs(an) + 2e-7 * d / hstep), (err.max(), d)


def test_objective_finite_differences(octmc):
    pairs, Ps = _pairs(octmc, 32, 48, 2, levels=1)
    D = torch.stack([synth.random_field(32, 32, 2.0, 5 + k) for k in range(2)]).float().cuda()
    octmc.eval_batched(Ps, 0, D, eta_mode=0)
    _fd_check(octmc, Ps, D, 256, 1e-3, 11, "small")


@pytest.mark.slow
def test_objective_batch_of_eight_full_size(octmc):
    """The batch workload at full size: 8 pairs of 200 x 200 A-scans x 512
    samples, generated on the GPU, one grouped forward + backward at the
    finest level; F and the gradient of every pair against the oracle, and
    central differences (h = 1e-3 px) at 256 random coordinates."""
    log("generate 8 pairs 200x200x512 on cuda")
    pairs, Ps = _pairs(octmc, 200, 512, 8, levels=3, device="cuda")
    D = torch.stack([make_field(q, "gt_noise", k) for k, q in enumerate(pairs)]).float().cuda()
    octmc.eval_batched(Ps, 0, D, eta_mode=0)
    Dr = D.clone().requires_grad_(True)
    log("batch forward + backward")
    F = octmc.objective(Dr, Ps, 0)
    F.sum().backward()
    torch.cuda.synchronize()
    log("oracle on 8 pairs")
    _check_against_oracle(octmc, pairs, Ps, 0, Dr, F, Dr.grad, "batch8")
    _fd_check(octmc, Ps, D, 256, 1e-3, 12, "batch8")
