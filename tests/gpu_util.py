"""Helpers shared by the GPU parity tests (inputs and comparisons only)."""
import sys

import numpy as np
import torch

import synth


def log(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def make_field(pair, case, seed=0):
    h, w, _ = pair.sx.shape
    gt = pair.d_gt
    if case == "zero":
        return torch.zeros((2, h, w, 3), dtype=torch.float64)
    if case == "gt":
        return gt.clone()
    if case == "gt_noise":
        return synth.perturbed_field(gt, 0.3, seed)
    if case == "smooth":
        return synth.smooth_random_field(w, h, 2.0, seed)
    if case == "uniform":
        # large, including sample positions outside the volume
        return synth.random_field(w, h, 3.5, seed)
    raise ValueError(case)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def grad_rel(g, ref):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


def round_storage(t: torch.Tensor, dtype: str) -> torch.Tensor:
    """The float32 volume rounded to the storage type (round to nearest even)
    and widened back, as the oracle sees it for BF16 / FP16 parity."""
    if dtype == "f32":
        return t
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16
    return t.to(tt).to(torch.float32)
