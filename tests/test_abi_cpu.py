"""The C-ABI library loads on the CPU and exports every symbol its header
declares; argument checks that need no GPU return the documented codes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def m():
    import paper_2010_06931_amd as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2010_06931_amd import build
        build.build()
    mod.lib()
    return mod


def header_symbols():
    text = open(os.path.join(ROOT, "include", "octmc.h")).read()
    return sorted(set(re.findall(r"OCTMC_API\s+[\w\s\*]*?\b(octmc_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(m):
    syms = header_symbols()
    assert len(syms) >= 12
    L = C.CDLL(m.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(m.SYMBOLS) == syms


def test_version_and_defaults(m):
    assert "gfx950" in m.version()
    p = m.default_params()
    assert p.delta0 == 0.5 and p.eps_huber == 1e-3  # fixed by the paper
    assert p.levels == 3 and p.lbfgs_m == 5 and p.iters_per_level == 100


def test_invalid_arguments_are_reported(m):
    L = m.lib()
    rc = L.octmc_pair_create(None, None, None, *([None] * 8), None, None)
    assert rc == -1
    assert "NULL" in L.octmc_last_error().decode()
    assert L.octmc_eval(None, 0, None, None, None, 1, None) == -1
    assert L.octmc_params_default(None) == -1
    assert L.octmc_eval_batched(None, 0, 0, None, None, None, 1, None) == -1
    assert L.octmc_register(None, None, None, None, None, None) == -1


def test_structs_match_header(m):
    # octmc_params: 6 doubles, 4 int32, 4 doubles, 1 uint32 (+ padding)
    assert C.sizeof(m.Params) == 6 * 8 + 4 * 4 + 4 * 8 + 8
    assert C.sizeof(m.Shape) == 5 * 4
