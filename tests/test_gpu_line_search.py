"""The L-BFGS iteration with its decisions on the device against the same
iteration with its decisions on the host (OCTMC_HOST_LINE_SEARCH), through
the C ABI.

The two forms take the same float64 decisions in the same order of
operations, and the vector kernels form every product in the same order, so
the bar is equality bit for bit: of the displacement, of every level's step
and evaluation counts, line-search failure flag, eta and objective values.
The cases cover the paths of the device form: a history shorter than lbfgs_m
and one that drops its oldest pair every step (m = 1), line searches that
need more than one trial (the host then drives the rest), line searches that
fail (ls_max_evals = 1), a step limit that is not a multiple of the batch of
enqueued iterations, no step at all, and a gradient that is zero at the start.
"""
import numpy as np
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


def _solve(octmc, pair, dtype, host, **kw):
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=dtype,
                   host_line_search=host, **kw)
    D, _, _, rep = P.register()
    torch.cuda.synchronize()
    P.close()
    return D, rep


CASES = [
    # (workload, pair, dtype, parameters)
    ("tiny", 0, "f32", dict(levels=3)),
    ("tiny", 0, "bf16", dict(levels=3)),
    ("tiny", 1, "f16", dict(levels=3, lbfgs_m=1)),
    ("tiny", 1, "f32", dict(levels=2, lbfgs_m=6, iters_per_level=60)),
    ("tiny", 0, "f32", dict(levels=2, iters_per_level=7)),
    ("tiny", 0, "bf16", dict(levels=2, ls_max_evals=1)),
    ("tiny", 0, "f32", dict(levels=2, iters_per_level=0)),
    ("tiny", 2, "bf16", dict(levels=2, c2=0.1)),
    ("clinical", 0, "bf16", dict(levels=0)),
]


@pytest.mark.parametrize("workload,idx,dtype,kw", CASES,
                         ids=[f"{w}{i}-{d}-" + "-".join(f"{k}{v}" for k, v in kw.items()) for w, i, d, kw in CASES])
def test_device_decisions_equal_host_decisions(octmc, workload, idx, dtype, kw):
    pair = synth.make_pair(workload, idx)
    log(f"line search: {workload} pair {idx} {dtype} {kw} (device, then host decisions)")
    Dd, rd = _solve(octmc, pair, dtype, False, **kw)
    Dh, rh = _solve(octmc, pair, dtype, True, **kw)
    print("device", rd)
    print("host  ", rh)
    assert rd == rh
    assert torch.equal(Dd, Dh)
    if kw.get("iters_per_level", 100) == 0:
        assert all(r["iters"] == 0 and r["evals"] == 1 for r in rd)
    if kw.get("ls_max_evals") == 1:
        assert any(r["ls_fail"] for r in rd)  # the failure path ran
    if kw.get("iters_per_level", 100) >= 60:
        # line searches of more than one trial: the host-driven continuation ran
        assert any(r["evals"] > r["iters"] + 1 for r in rd)
    if kw.get("c2") == 0.1:
        # a strict curvature condition: many searches need further trials, far
        # more than the first iteration of each level accounts for, so the
        # pipelined iterations stalled and were resumed
        assert all(r["evals"] > r["iters"] + 10 for r in rd if r["iters"] > 0)


def test_zero_gradient_stops_at_once(octmc):
    """Identical scans: every term and its gradient vanish at the zero field,
    so each level stops before its first step, in both forms."""
    pair = synth.make_pair("tiny")
    pair.sy = pair.sx.clone()
    pair.ay = pair.ax.clone()
    pair.vy = pair.vx.clone()
    Dd, rd = _solve(octmc, pair, "f32", False, levels=2)
    Dh, rh = _solve(octmc, pair, "f32", True, levels=2)
    assert rd == rh
    assert torch.equal(Dd, Dh)
    assert all(r["iters"] == 0 for r in rd)
    assert float(Dd.abs().max()) == 0.0


@pytest.mark.parametrize("dtype,levels,iters", [("f32", 2, 60), ("bf16", 3, 40)])
def test_stage1_device_decisions_equal_host_decisions(octmc, dtype, levels, iters):
    """The stage-1 solve (per-B-scan offsets and tilts) runs the same
    iteration with the stage-1 evaluator: both forms give the same theta and
    report bit for bit."""
    h = w = 40
    d = 64
    mX, mY = synth.planted_axial_motion(h, w, seed=3)
    X, Y = synth.layered_axial_pair(h, w, d, mX, mY)
    z = torch.zeros((h, w))
    out = []
    for host in (False, True):
        P = octmc.Pair(torch.from_numpy(X).float(), torch.from_numpy(Y).float(), ax=z, ay=z, delta0=0.0,
                       levels=levels, dtype=dtype, host_line_search=host)
        log(f"stage 1 {dtype} levels {levels} ({'host' if host else 'device'} decisions)")
        out.append(P.prealign(1.0, iters))
        P.close()
    (thd, rd), (thh, rh) = out
    print("device", rd)
    print("host  ", rh)
    assert rd == rh
    assert np.array_equal(thd, thh)


@pytest.mark.parametrize("dtype,pairwise", [("f32", False), ("bf16", False), ("f32", True)])
def test_multi_device_decisions_equal_host_decisions(octmc, dtype, pairwise):
    """The joint solve of four volumes (two orthogonal pairs), fused or pair
    by pair: both forms of the iteration give the same fields and report."""
    sc = synth.make_scans("tiny", 2, (0, 1, 0, 1), n=40, d=64, white_lines=True)
    out = []
    for host in (False, True):
        M = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=2, iters_per_level=40, dtype=dtype,
                        pairwise=pairwise, host_line_search=host)
        log(f"four volumes {dtype} pairwise={pairwise} ({'host' if host else 'device'} decisions)")
        D, _, _, rep = M.register()
        torch.cuda.synchronize()
        out.append((D, rep))
        M.close()
    (Dd, rd), (Dh, rh) = out
    print("device", rd)
    print("host  ", rh)
    assert rd == rh
    assert torch.equal(Dd, Dh)
