"""Input validity of OCTA volumes (Sec. 2.2) on the GPU, through the C ABI:
exact agreement (0/1 per B-scan) with the FP64 oracle, and a pair created
with OCTMC_DETECT_INVALID behaving exactly like a pair given that validity."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import grad_err, grad_rel, log, make_field, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def octmc():
    import paper_2010_06931_amd as m
    m.lib()
    return m


def _planted(h, w, d, bad_rows, seed):
    rng = np.random.default_rng(seed)
    vol = rng.rayleigh(0.1, (h, w, d)).astype(np.float32)
    for b in bad_rows:
        vol[b] = 1.0 + 0.05 * rng.random((w, d), dtype=np.float32)
    return vol


@pytest.mark.parametrize("shape,bad", [((37, 41, 23), [0, 12, 36]), ((64, 64, 128), [30]), ((20, 20, 5), [])])
def test_validity_matches_oracle_planted(octmc, shape, bad):
    h, w, d = shape
    vol = _planted(h, w, d, bad, seed=h)
    for scan in (0, 1):
        v = vol if scan == 0 else np.ascontiguousarray(vol.transpose(1, 0, 2))  # Y-fast B-scans are columns
        log(f"validity planted {shape} scan {scan}")
        got = octmc.validity_from_octa(torch.from_numpy(v).cuda(), scan).cpu().numpy()
        ref = oracle.validity(v, scan)
        assert np.array_equal(got, ref.astype(np.float32)), (shape, scan, got, ref)
        if bad and scan == 0:
            assert (got == 0).sum() >= 3


def test_validity_host_input_and_white_lines(octmc):
    for p in range(3):
        pair = synth.make_pair("tiny", p, white_lines=True)
        log(f"validity white lines tiny pair {p}")
        gx = octmc.validity_from_octa(pair.ox, 0).cpu()        # host tensor: copied by the binding
        gy = octmc.validity_from_octa(pair.oy.cuda(), 1).cpu()
        assert torch.equal(gx, pair.vx) and torch.equal(gy, pair.vy)
    # host pointer straight through the C ABI
    import ctypes as C
    vol = np.ascontiguousarray(pair.ox.numpy())
    h, w, d = vol.shape
    out = torch.empty(h, dtype=torch.float32, device="cuda")
    shape = octmc.Shape(w, h, d, octmc.F32, octmc.MEM_HOST)
    rc = octmc.lib().octmc_validity_from_octa(octmc.context()._h, C.byref(shape), vol.ctypes.data_as(C.c_void_p), 0,
                                              C.c_void_p(out.data_ptr()), None)
    assert rc == 0
    assert torch.equal(out.cpu(), pair.vx)


def test_validity_clinical_size(octmc):
    log("generate clinical 300x300x640 with white lines on cuda")
    pair = synth.make_pair("clinical", white_lines=True, device="cuda")
    for scan, vol, truth in ((0, pair.ox, pair.vx), (1, pair.oy, pair.vy)):
        got = octmc.validity_from_octa(vol, scan).cpu().numpy()
        ref = oracle.validity(vol, scan)
        assert np.array_equal(got, ref.astype(np.float32))
        assert np.array_equal(got, truth.cpu().numpy())


def test_pair_detect_invalid_equals_given_validity(octmc):
    pair = synth.make_pair("tiny", 1, n=48, d=64, white_lines=True)
    vx, vy = oracle.validity(pair.ox, 0), oracle.validity(pair.oy, 1)
    assert (vx == 0).any() or (vy == 0).any()
    log("pair with detected validity vs given validity")
    Pd = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, levels=2, iters_per_level=20, detect_invalid=True)
    Pg = octmc.Pair(pair.sx, pair.sy, ox=pair.ox, oy=pair.oy, vx=torch.from_numpy(vx), vy=torch.from_numpy(vy),
                    levels=2, iters_per_level=20)
    D = make_field(pair, "gt_noise", 4).float().cuda()
    td, gd = Pd.eval(0, D, eta_mode=0)
    tg, gg = Pg.eval(0, D, eta_mode=0)
    torch.cuda.synchronize()
    assert torch.equal(td, tg) and torch.equal(gd, gg)
    # against the oracle with the oracle's validity
    lv = oracle.level_from(pair.sx, pair.sy, oracle.enface_mean(oracle.substitute_invalid(pair.ox, vx, 0)),
                           oracle.enface_mean(oracle.substitute_invalid(pair.oy, vy, 1)), vx, vy)
    t = octmc.terms_dict(td)
    ref, gref = oracle.evaluate(lv, D.double().cpu().numpy(), oracle.Params(), t["eta"])
    assert rel(t["F"], ref["F"]) < 1e-4
    assert grad_err(gd.double().cpu().numpy(), gref) < 1e-4
    Dd, _, _, _ = Pd.register()
    Dg, _, _, _ = Pg.register()
    torch.cuda.synchronize()
    assert torch.equal(Dd, Dg)
