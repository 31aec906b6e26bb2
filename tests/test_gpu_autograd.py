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
from gpu_util import grad_rel, log, make_field, rel

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
        e = grad_rel(grad[b].double().cpu().numpy(), gref)
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


def test_objective_finite_differences(octmc):
    """Central differences (h = 1e-2 px) of the GPU forward at 96 sampled
    coordinates against the GPU backward.  The tolerance covers the float32
    rounding of one A-scan's depth sum (about 1e-6 relative of a sum of order
    10, divided by 2h) and the O(h^2) truncation of the cubic interpolant."""
    pairs, Ps = _pairs(octmc, 32, 48, 2, levels=1)
    D = torch.stack([synth.random_field(32, 32, 2.0, 5 + k) for k in range(2)]).float().cuda()
    octmc.eval_batched(Ps, 0, D, eta_mode=0)
    Dr = D.clone().requires_grad_(True)
    octmc.objective(Dr, Ps, 0).sum().backward()
    torch.cuda.synchronize()
    g = Dr.grad.detach().double().cpu().numpy()
    rng = np.random.default_rng(11)
    hstep = 1e-2
    fd, an = [], []
    log("autograd finite differences, 96 coordinates")
    for _ in range(96):
        idx = (int(rng.integers(2)), int(rng.integers(2)), int(rng.integers(32)), int(rng.integers(32)),
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
    log(f"fd: max err {err.max():.3e}, rel norm {np.linalg.norm(fd - an) / np.linalg.norm(an):.3e}")
    assert np.linalg.norm(fd - an) <= 1e-2 * np.linalg.norm(an)
    assert np.all(err <= 2e-2 * np.abs(an) + 0.05)


@pytest.mark.slow
def test_objective_batch_of_eight_full_size(octmc):
    """The batch workload at full size: 8 pairs of 200 x 200 A-scans x 512
    samples, generated on the GPU, one grouped forward + backward at the
    finest level; F and the gradient of every pair against the oracle."""
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
