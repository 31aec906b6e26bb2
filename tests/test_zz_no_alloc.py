"""The allocation-free evaluation (octmc_eval_noalloc) through the C ABI:
two calls in a row, the second on a smaller pair, each bitwise equal to
octmc_eval on a pair created from the same level-0 data with the same eta
(eta set by the call itself, eta_mode 0, then read back, eta_mode 1), in
float32 and BF16 storage; a pair larger than the static scratch allows is
refused."""
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
