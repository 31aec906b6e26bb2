"""Write the FP64 oracle's solve of a synthetic workload pair to tests/golden/.

    python tests/golden/make_solve_golden.py clinical [--levels L] [--store 0|1|2] [--perturb REL] [--out-dir DIR]

Calls only the input generator (synth) and the oracle (oracle/): nothing here
comes from the HIP library.  The pair is generated with torch on the GPU,
whose kernels give the same bits on every device of one kind (torch on the
CPU does not: its results depend on the thread count and vector width), and
the SHA-256 of the float32 inputs is stored with the result, so a test that
regenerates the pair can check that it sees the same inputs.

The oracle solves the pair with the workload's pyramid depth (or --levels)
and 100 L-BFGS steps per level (Sec. 2.1, "optimization"), every other parameter at its
default, optionally with the volumes rounded to a 16-bit storage type
(--store).  With --perturb REL it solves a second time with every structural
sample multiplied by 1 + REL u, u uniform in [-1, 1] (seeded), and stores
the RMS distance between the two solutions: the sensitivity of the solve's
trajectory to input perturbations of about that relative size.

The displacement field is stored quantised to 2^-10 px (half a thousandth
of a pixel at most), delta-encoded along x and compressed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

QUANT = 2.0 ** -10


def golden_path(workload: str, levels: int, store: int, out_dir: str | None = None) -> str:
    return os.path.join(out_dir or os.path.dirname(os.path.abspath(__file__)),
                        f"solve_{workload}_L{levels}_store{store}.npz")


def input_hash(pair) -> str:
    h = hashlib.sha256()
    for t in (pair.sx, pair.sy, pair.ax, pair.ay, pair.vx, pair.vy):
        h.update(t.detach().float().contiguous().cpu().numpy().tobytes())
    return h.hexdigest()


def encode(D: np.ndarray) -> np.ndarray:
    q = np.rint(np.asarray(D, dtype=np.float64) / QUANT).astype(np.int64)
    assert np.abs(q).max() < 2**31
    return np.diff(q, axis=2, prepend=0).astype(np.int32)


def decode(enc: np.ndarray) -> np.ndarray:
    return np.cumsum(enc.astype(np.int64), axis=2).astype(np.float64) * QUANT


def load(workload: str, levels: int, store: int, out_dir: str | None = None):
    """(D [2][h][w][3] float64, meta dict) of a stored golden solve, or None."""
    p = golden_path(workload, levels, store, out_dir)
    if not os.path.exists(p):
        return None
    z = np.load(p, allow_pickle=False)
    return decode(z["D"]), json.loads(str(z["meta"]))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--pair", type=int, default=0)
    ap.add_argument("--store", type=int, default=0, choices=(0, 1, 2))
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--levels", type=int, default=0, help="pyramid levels (default: the workload's)")
    ap.add_argument("--perturb", type=float, default=0.0)
    ap.add_argument("--device", default="cuda")
    ap.add_argument("--out-dir", default=None, help="directory of the result (default: beside this script)")
    a = ap.parse_args()
    import torch

    cfg = synth.WORKLOADS[a.workload]
    t0 = time.time()
    pair = synth.make_pair(a.workload, a.pair, device=a.device, octa_volumes=False)
    sha = input_hash(pair)
    print(f"[golden] {a.workload} pair {a.pair} generated on {a.device} in {time.time() - t0:.1f} s, "
          f"inputs sha256 {sha[:16]}", flush=True)
    lv = oracle.level_from_pair(pair)
    prm = oracle.Params(levels=a.levels or cfg["levels"], iters=a.iters, store=a.store)
    threads = oracle.set_threads(0)
    oracle.set_progress(10)
    t0 = time.time()
    D, rep = oracle.register(lv, prm)
    el = time.time() - t0
    print(f"[golden] oracle solve {el:.1f} s on {threads} threads; levels {rep}", flush=True)
    meta = dict(workload=a.workload, pair=a.pair, n=cfg["n"], d=cfg["d"], seed=[synth.SEED_BASE + cfg["index"],
                a.pair], generated_on=a.device, torch=torch.__version__,
                device_name=torch.cuda.get_device_name(0) if a.device == "cuda" else "cpu",
                input_sha256=sha, params=dict(levels=prm.levels, iters=prm.iters, alpha=prm.alpha,
                                              delta0=prm.delta0, store=prm.store),
                levels=rep, oracle_seconds=round(el, 1), oracle_threads=threads, quantum_px=QUANT,
                command="python tests/golden/make_solve_golden.py " + " ".join(sys.argv[1:]))
    if a.perturb > 0:
        rng = np.random.default_rng(12345)
        lp = oracle.Level(lv.sx * (1 + a.perturb * rng.uniform(-1, 1, lv.sx.shape)),
                          lv.sy * (1 + a.perturb * rng.uniform(-1, 1, lv.sy.shape)), lv.ax, lv.ay, lv.vx, lv.vy)
        t0 = time.time()
        Dp, _ = oracle.register(lp, prm)
        sens = float(np.sqrt(((Dp - D) ** 2).mean()))
        print(f"[golden] perturbed solve ({a.perturb:g} relative) {time.time() - t0:.1f} s: "
              f"RMS distance {sens:.4f} px", flush=True)
        meta["perturbation"] = dict(relative=a.perturb, rms_px=sens)
    if a.out_dir:
        os.makedirs(a.out_dir, exist_ok=True)
    out = golden_path(a.workload, prm.levels, a.store, a.out_dir)
    np.savez_compressed(out, D=encode(D), meta=np.array(json.dumps(meta)))
    Dq, _ = load(a.workload, prm.levels, a.store, a.out_dir)
    assert np.abs(Dq - D).max() <= QUANT / 2 + 1e-12
    print(f"[golden] wrote {out} ({os.path.getsize(out)} bytes)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
