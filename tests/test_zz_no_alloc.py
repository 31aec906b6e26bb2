"""The allocation-free evaluation (octmc_eval_noalloc) through the C ABI:
two calls in a row, the second on a smaller pair, each bitwise equal to
octmc_eval on a pair created from the same level-0 data with the same eta
(eta set by the call itself, eta_mode 0, then read back, eta_mode 1), in
float32 and BF16 storage; an odd depth in BF16 (the caller's layout, so
the one-sample structural kernel) against the oracle; a pair larger than
the static scratch allows is refused."""
import pytest
import torch

import synth
from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _inputs(octmc, q, dtype):
    tt = {"f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    dev = torch.device("cuda")
    ins = [q.sx.to(dev).to(tt).contiguous(), q.sy.to(dev).to(tt).contiguous()]
    ins += [t.to(dev, torch.float32).contiguous() for t in (q.ax, q.ay, q.vx, q.vy)]
    return ins


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_equals_pair_eval(octmc, dtype):
    for k, (n, d) in enumerate([(48, 80), (28, 36)]):
        q = synth.make_pair("serving", 30 + k, n=n, d=d, octa_volumes=False, white_lines=False)
        P = octmc.Pair(q.sx, q.sy, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, dtype=dtype, levels=1)
        D = synth.perturbed_field(q.d_gt, 0.3, k).float().cuda()
        ins = _inputs(octmc, q, dtype)
        eta = torch.zeros(1, dtype=torch.float64, device="cuda")
        terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
        grad = torch.empty_like(D)
        log(f"eval_noalloc {dtype} {n}x{n}x{d}, eta_mode 0")
        octmc.eval_noalloc(*ins, D, eta, terms, grad, dtype=dtype, params=P.params, eta_mode=0)
        t_ref, g_ref = P.eval(0, D, eta_mode=0)
        torch.cuda.synchronize()
        assert torch.equal(terms, t_ref), (terms, t_ref)
        assert torch.equal(grad, g_ref)
        assert eta.item() == t_ref[octmc.TERM_ETA].item()
        # eta_mode 1 reads the stored eta; a displaced field, no gradient
        D2 = (D + 0.25).contiguous()
        log(f"eval_noalloc {dtype} {n}x{n}x{d}, eta_mode 1")
        octmc.eval_noalloc(*ins, D2, eta, terms, None, dtype=dtype, params=P.params, eta_mode=1)
        t2, _ = P.eval(0, D2, grad=False, eta_mode=1)
        torch.cuda.synchronize()
        assert torch.equal(terms, t2)
        P.close()


def test_noalloc_odd_depth_matches_oracle(octmc):
    """An odd depth in BF16 in the caller's layout (no padding sample, so the
    one-sample structural kernel): every term and the whole gradient against
    the oracle on the rounded volumes, at 1e-4; the pair path, which stores
    the depth padded and takes the two-sample kernel, agrees with it to
    float32 rounding."""
    import oracle
    from gpu_util import grad_err, grad_rel, rel, round_storage
    n, d = 24, 37
    q = synth.make_pair("tiny", n=n, d=d, octa_volumes=False)
    P = octmc.Pair(q.sx, q.sy, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, dtype="bf16", levels=1)
    ins = _inputs(octmc, q, "bf16")
    D = synth.random_field(n, n, 3.0, 4).float().cuda()
    eta = torch.zeros(1, dtype=torch.float64, device="cuda")
    terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(D)
    log(f"eval_noalloc bf16 {n}x{n}x{d} (odd depth), eta_mode 0")
    octmc.eval_noalloc(*ins, D, eta, terms, grad, dtype="bf16", params=P.params, eta_mode=0)
    torch.cuda.synchronize()
    t = octmc.terms_dict(terms)
    p = P.params
    prm = oracle.Params(alpha=p.alpha, delta0=p.delta0, eps_h=p.eps_huber, eps_r=p.eps_reg,
                        flyback_frac=p.flyback_frac, mean_weight=p.mean_weight)
    lv = oracle.level_from(round_storage(q.sx, "bf16"), round_storage(q.sy, "bf16"), q.ax, q.ay, q.vx, q.vy)
    D64 = D.double().cpu().numpy()
    eta_ref = oracle.eta_at(lv, D64, prm)
    ref, gref = oracle.evaluate(lv, D64, prm, eta_ref)
    assert rel(t["eta"], eta_ref) < 1e-4, (t["eta"], eta_ref)
    for k in ("F", "data", "str", "ang", "reg", "str05", "ang05"):
        assert rel(t[k], ref[k]) < 1e-4 or abs(t[k] - ref[k]) < 1e-9 * max(1.0, abs(ref["F"])), (k, t[k], ref[k])
    assert grad_err(grad.double().cpu().numpy(), gref) < 1e-4
    t2, g2 = P.eval(0, D, eta_mode=0)
    torch.cuda.synchronize()
    assert rel(octmc.terms_dict(t2)["F"], t["F"]) < 1e-5
    assert grad_rel(g2.double().cpu().numpy(), grad.double().cpu().numpy()) < 1e-5


def test_noalloc_refuses_more_than_its_scratch(octmc):
    n = 520  # 520^2 > 512^2 A-scans
    x = torch.zeros((n, n, 4), device="cuda")
    a = torch.zeros((n, n), device="cuda")
    v = torch.ones(n, device="cuda")
    D = torch.zeros((2, n, n, 3), device="cuda")
    eta = torch.ones(1, dtype=torch.float64, device="cuda")
    terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
    with pytest.raises(octmc.OctmcError) as e:
        octmc.eval_noalloc(x, x, a, a, v, v, D, eta, terms)
    assert e.value.code == -2
