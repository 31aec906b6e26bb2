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
    """Norm-wise relative error."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


# Floor of the element-wise gradient check, as a fraction of max |ref|.  The
# float32 kernels round the residual r = I^X - I^Y to about 2^-24 of the
# intensities (order 1), and the pseudo-Huber derivative L'(r) has slope
# 1/eps = 10^3 at the kink, so each sample's L' carries an error of about
# 6e-5; over the d samples of an A-scan these add with random signs, about
# sqrt(d) 6e-5 |dI|, against a largest gradient entry of about d |dI|: some
# 2e-6 of max |ref| at d = 800 (measured: at most 3e-6 at 500 x 500 x 800).
# A floor of 0.1 max |ref| at the 1e-4 bar allows 1e-5 max |ref|, five times
# that; mistakes such as a dropped validity-derivative term next to a white
# line or a clamp slip at the border change entries by amounts of the order
# of the entries themselves.
ELEM_FLOOR = 0.1


def elem_err(g, ref, floor=ELEM_FLOOR):
    """Element-wise error max |g - ref| / (|ref| + floor max |ref|)."""
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    scale = np.abs(ref) + floor * max(float(np.abs(ref).max()), 1e-300)
    return float((np.abs(g - ref) / scale).max())


def grad_err(g, ref, floor=ELEM_FLOOR):
    """The larger of the norm-wise and the element-wise error of a gradient
    against the oracle's (both must meet the bar)."""
    return max(grad_rel(g, ref), elem_err(g, ref, floor))


def round_storage(t: torch.Tensor, dtype: str) -> torch.Tensor:
    """The float32 volume rounded to the storage type (round to nearest even)
    and widened back, as the oracle sees it for BF16 / FP16 parity."""
    if dtype == "f32":
        return t
    tt = torch.bfloat16 if dtype == "bf16" else torch.float16
    return t.to(tt).to(torch.float32)
