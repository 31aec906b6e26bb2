#!/usr/bin/env python3
"""Benchmark of the registration hot path on one MI355X.

A step is one evaluation of the full objective and its gradient (displacement
sum, structural resample + residual + depth reduction, en face / validity /
regulariser / mean terms and the float64 global sums) at the finest level of
the dense synthetic pair (500 x 500 A-scans x 800 samples per scan, X-fast +
Y-fast), with the inputs resident in HBM and the structural volumes stored
in BF16 (the second storage run, FP16, and FP32 storage are reported as
variants; all arithmetic is float32 with float64 global sums).  The line
printed last is one JSON object: evals/s, the roofline of the dominant kernel
(timed live with HIP events on the stream it runs on), the FP64 oracle's rate
on the host cores for a bounded sample of A-scans, and secondary figures (full
solve with its displacement error, storage variants, serving).

    python bench.py [--steps K] [--warmup W] [--dtype bf16|f16|f32]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "obj+grad evals/s & HBM GB/s (500²×800 pair); pairs/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# float32 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 flop per FMA (no packed FP32)
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# algorithmic work of the structural kernel per voxel pair: per scan 16 FMA
# lateral blend + 4 + 4 depth FIR (value, d/dz) + 4 adjoint FIR + 16 column
# dots + 1 (Gamma_z) = 45 FMA; two scans = 90 FMA = 180 flop; plus 12 single
# operations for residual, pseudo-Huber value and derivative and the sum
FLOP_PER_VOXEL_PAIR = 192
EXTRA_BYTES_PER_ASCAN = 2 * 12 + 32  # displacements in, partial sums out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def warm_clock(torch, step, seconds=None):
    """Untimed evaluations until `seconds` of device work have run: the
    device's clocks ramp up over the first tens of milliseconds of load after
    idle (20 evaluations of the dense pair right after idle ran at 1.18 ms
    each, later ones at 1.105 ms).  Returns the number of evaluations run."""
    seconds = WARM_SECONDS if seconds is None else seconds
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            step()
        torch.cuda.synchronize()
        n += 10
    return n


def source_sha():
    """Hash of the structural kernels' source (the part of kernels_eval.hip
    before the reduction helpers: stencils, k_struct, k_struct2), so that
    counter figures go stale only when those kernels change."""
    p = os.path.join(ROOT, "paper_2010_06931_amd", "csrc", "kernels_eval.hip")
    text = open(p, "rb").read()
    cut = text.find(b"// deterministic block reduction helpers")
    if cut < 0:
        raise RuntimeError("kernels_eval.hip: reduction helpers marker not found")
    return hashlib.sha256(text[:cut]).hexdigest()[:16]


def load_traffic(dtype):
    """HBM traffic of the structural kernel from the committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "k_struct_dense_counters.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
        r = rec.get(dtype)
        if not r or rec.get("source_sha") != source_sha():
            return None
        return r["bytes_per_launch"]
    except Exception:  # noqa: BLE001 - a malformed file means no figure
        return None


WARM_SECONDS = 0.2    # minimum untimed device work before the timed evaluations
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per copy
COPY_REPEATS = 3


def calibration_copies(torch):
    """Plain device-to-device copies of known size, run after the timed
    evaluations of a profile-only run so that the same counter pass sees them."""
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPY_REPEATS):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _counter_rows(path, counter):
    import csv
    rows = [r for r in csv.DictReader(open(path)) if r.get("Counter_Name", "").startswith(counter)]
    if not rows:
        raise SystemExit(f"{path}: no {counter} rows")
    return rows


def traffic_summary(fetch_csv, write_csv, dtype, out_path, command):
    """HBM bytes per launch of the structural kernel from two rocprofv3
    counter passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by
    the ratio of known bytes to counted bytes of the calibration copies."""
    res = {}
    for name, path, known in (("FETCH_SIZE", fetch_csv, COPY_BYTES), ("WRITE_SIZE", write_csv, COPY_BYTES)):
        rows = _counter_rows(path, name)
        ks = [float(r["Counter_Value"]) for r in rows if "k_struct" in r["Kernel_Name"]]
        # the calibration copies are the last copy dispatches of the run
        cp = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows
                    if "copyBuffer" in r["Kernel_Name"])
        cp = [v for _, v in cp[-COPY_REPEATS:]]
        if not ks or not cp:
            raise SystemExit(f"{path}: k_struct dispatches {len(ks)}, copy dispatches {len(cp)}")
        factor = known * COPY_REPEATS / (sum(cp) * 1024.0)
        res[name] = {"kib_per_dispatch": round(sum(ks) / len(ks), 1), "dispatches": len(ks),
                     "copy_kib_total": round(sum(cp), 1), "copy_factor": round(factor, 4),
                     "bytes_per_launch": sum(ks) / len(ks) * 1024.0 * factor}
    rec = {}
    if os.path.exists(out_path):
        rec = json.load(open(out_path))
        if rec.get("source_sha") != source_sha():
            rec = {}
    rec["source_sha"] = source_sha()
    rec[dtype] = {"bytes_per_launch": round(res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]),
                  "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"], "command": command}
    json.dump(rec, open(out_path, "w"), indent=1)
    print(json.dumps(rec[dtype]))


def cpu_baseline(pair, D, target_s=15.0):
    """The FP64 oracle (as it stands) on the host: the whole objective and
    its gradient (both data terms, regulariser, mean term; eta fixed) over
    the whole pair, repeated for about target_s seconds, as evaluations per
    second.  If one evaluation would take far longer than that, a bounded
    random sample of A-scans of the data term stands in, scaled to the pair."""
    import numpy as np

    import oracle
    lv = oracle.Level(*(oracle._f64(t) for t in (pair.sx, pair.sy, pair.ax, pair.ay, pair.vx, pair.vy)))
    Dn = D.double().cpu().numpy()
    w, h, d = lv.whd
    na = w * h
    rng = np.random.default_rng(0)
    prm = oracle.Params()
    probe = rng.choice(na, size=256, replace=False)
    t0 = time.perf_counter()
    oracle.data_ascans(lv, Dn, probe, prm, 1.0)
    t_probe = time.perf_counter() - t0
    cores = oracle.set_threads(0)  # the threads its parallel loops use
    est_full = t_probe * na / 256
    if est_full <= target_s / 2:
        t0 = time.perf_counter()
        reps = 0
        while reps < 1 or time.perf_counter() - t0 < target_s:
            oracle.evaluate(lv, Dn, prm, 1.0, grad=True)
            reps += 1
        dt = (time.perf_counter() - t0) / reps
        return {"value": 1.0 / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
                "sample": f"whole objective and gradient of the {w}x{h}x{d} pair (all {na} A-scans, both data "
                          f"terms, regulariser, mean term), {reps} evaluations, {dt:.2f} s each"}
    nsample = int(min(na, max(256, 256 * target_s / max(t_probe, 1e-3))))
    sample = rng.choice(na, size=nsample, replace=False)
    t0 = time.perf_counter()
    oracle.data_ascans(lv, Dn, sample, prm, 1.0)
    dt = time.perf_counter() - t0
    return {"value": (nsample / na) / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"data term of {nsample} random A-scans of the {w}x{h}x{d} pair, scaled by {na}/{nsample} "
                      f"({dt:.1f} s)"}


def cpu_baseline_small(torch):
    """The FP64 oracle's full objective and gradient (every term) on the tiny
    64^2 x 128 pair, on one host thread and on all of them: evaluations per
    second (a reported baseline beside the sampled one above)."""
    import oracle
    import synth
    pair = synth.make_pair("tiny", 0)
    lv = oracle.level_from_pair(pair)
    D = pair.d_gt.double().numpy()
    prm = oracle.Params()
    nall = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    res = {"workload": "tiny pair 64x64 A-scans x 128 samples, full objective and gradient, FP64 oracle"}
    for tag, nt in (("one_thread", 1), ("all_threads", nall)):
        used = oracle.set_threads(nt)
        oracle.evaluate(lv, D, prm, 1.0)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0:
            oracle.evaluate(lv, D, prm, 1.0)
            reps += 1
        res[tag] = {"evals_per_s": round(reps / (time.perf_counter() - t0), 3), "threads": used}
    oracle.set_threads(nall)
    return res


SERVE_SIZES = (300, 400, 500, 600)
SERVE_DEPTHS = (512, 640, 800)
UM_PER_PX = (12.0, 12.0, 3.0)  # transverse x, y and axial spacing of the dense / serving scans


def _interior_rms(D, gt, border=8):
    """Per-component RMS of D - gt over A-scans away from the border, after
    removing the common mean (the gauge the mean term fixes)."""
    import numpy as np
    e = D.double().cpu().numpy() - gt.double().cpu().numpy()
    h, w = e.shape[1:3]
    m = np.zeros(e.shape[:3], bool)
    m[:, border:h - border, border:w - border] = True
    e -= e[m].mean(axis=0)
    return np.sqrt((e[m] ** 2).mean(axis=0))


def _relative_rms(D, gt, border=8):
    """Per-component RMS of the error of the relative displacement
    d^X - d^Y (what the data term sees) over A-scans away from the border,
    after removing its mean.  A smooth warp common to both scans changes
    neither scan's agreement with the other, so it is left out of this
    figure but not out of _interior_rms."""
    import numpy as np
    e = (D[0] - D[1]).double().cpu().numpy() - (gt[0] - gt[1]).double().cpu().numpy()
    h, w = e.shape[:2]
    e = e[border:h - border, border:w - border].reshape(-1, 3)
    e -= e.mean(axis=0)
    return np.sqrt((e ** 2).mean(axis=0))


def serving(octmc, torch, nreq, budget_gib, max_active, log):
    """Mixed-size requests through the server (BF16 storage) against
    sequential FP32 solves of the same trace on the same GPU: with the
    workload's 4 levels (Poisson trace and two burst modes), then with the
    automatic pyramid depth (levels = 0, Poisson trace only)."""
    import numpy as np
    import synth
    classes = [(n, d) for n in SERVE_SIZES for d in SERVE_DEPTHS]
    log(f"serving: generating {len(classes)} size classes on cuda")
    pairs = [synth.make_pair("serving", c, n=n, d=d, device="cuda", octa_volumes=False)
             for c, (n, d) in enumerate(classes)]
    rng = np.random.default_rng(np.random.SeedSequence([20100693104, 999]))
    cls = rng.integers(0, len(classes), nreq)
    arrival = np.cumsum(rng.exponential(0.25, nreq))
    arrival -= arrival[0]
    torch.cuda.synchronize()

    def out_of(c):
        n = classes[c][0]
        return torch.empty((2, n, n, 3), dtype=torch.float32, device="cuda")

    def sequential(levels):
        """Plain FP32 solves, first-come first-served on the trace."""
        log(f"serving: {nreq} sequential FP32 solves, levels = {levels}")
        seq_t, seq_D = [], {}
        for r in range(nreq):
            q = pairs[cls[r]]
            t0 = time.perf_counter()
            P = octmc.Pair(q.sx, q.sy, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, dtype="f32", levels=levels)
            D, _, _, _ = P.register()
            torch.cuda.synchronize()
            P.close()
            seq_t.append(time.perf_counter() - t0)
            if cls[r] not in seq_D:
                seq_D[cls[r]] = D
        done = 0.0
        seq_lat = []
        for r in range(nreq):
            done = max(done, arrival[r]) + seq_t[r]
            seq_lat.append(done - arrival[r])
        return {"pairs_per_s_burst": round(nreq / sum(seq_t), 3),
                "pairs_per_s_trace": round(nreq / done, 3),
                "latency_p50_s": round(float(np.percentile(seq_lat, 50)), 3),
                "latency_p99_s": round(float(np.percentile(seq_lat, 99)), 3),
                "solve_s_mean": round(float(np.mean(seq_t)), 4)}, seq_D

    def served(mode, times, levels, budget):
        srv = octmc.Server(budget, max_active=max_active, mode=mode)
        outs = {}
        t0 = time.perf_counter()
        for r in range(nreq):
            wait = times[r] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            q = pairs[cls[r]]
            disp = out_of(cls[r])
            rid = srv.submit(q.sx, q.sy, disp, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, dtype="bf16", levels=levels,
                             tag=r)
            outs[rid] = (r, disp)
        comp = []
        while len(comp) < nreq:
            comp += srv.poll(nreq, wait_ms=120000)
        t_end = time.perf_counter() - t0
        srv.close()
        bad = [c for c in comp if c["status"] != 0]
        if bad:
            raise RuntimeError(f"served request failed: {bad[0]['error']}")
        lat = [c["t_done"] - c["t_submit"] for c in comp]
        res = {"pairs_per_s": round(nreq / t_end, 3),
               "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
               "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
               "max_reserved_GiB": round(max(c["bytes_reserved"] for c in comp) / (1 << 30), 3)}
        return res, {outs[c["id"]][0]: outs[c["id"]][1] for c in comp}

    def accuracy(got, seq_D):
        """Served BF16 against ground truth and against the FP32 solve of the same input."""
        acc_gt_bf16, acc_gt_f32, acc_vs_f32 = [], [], []
        for r, D in got.items():
            c = cls[r]
            gt = pairs[c].d_gt
            acc_gt_bf16.append(_interior_rms(D, gt))
            acc_gt_f32.append(_interior_rms(seq_D[c], gt))
            acc_vs_f32.append(np.sqrt(((D - seq_D[c]).double().cpu().numpy() ** 2).reshape(-1, 3).mean(axis=0)))
        med = lambda a: [round(float(x), 3) for x in np.median(np.array(a), axis=0)]
        return {"served_bf16_vs_ground_truth": med(acc_gt_bf16),
                "sequential_fp32_vs_ground_truth": med(acc_gt_f32),
                "served_bf16_vs_sequential_fp32": med(acc_vs_f32)}

    seq, seq_D = sequential(4)
    torch.cuda.empty_cache()  # return the generator's cached blocks to the device
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(budget_gib * (1 << 30), 0.6 * free))
    log(f"serving: memory budget {budget / 2**30:.1f} GiB")
    log("serving: Poisson trace, grouped launches")
    poisson, got = served(octmc.SERVE_GROUPED, arrival, 4, budget)
    log("serving: burst, grouped launches")
    burst, _ = served(octmc.SERVE_GROUPED, np.zeros(nreq), 4, budget)
    log("serving: burst, one stream per request")
    burst_streams, _ = served(octmc.SERVE_STREAMS, np.zeros(nreq), 4, budget)
    acc = accuracy(got, seq_D)
    del got, seq_D
    seq0, seq_D0 = sequential(0)
    log("serving: Poisson trace, grouped launches, levels = 0")
    poisson0, got0 = served(octmc.SERVE_GROUPED, arrival, 0, budget)
    log("serving: Poisson trace, one stream per request, levels = 0")
    poisson0s, _ = served(octmc.SERVE_STREAMS, arrival, 0, budget)
    log("serving: burst, grouped launches, levels = 0")
    burst0, _ = served(octmc.SERVE_GROUPED, np.zeros(nreq), 0, budget)
    log("serving: burst, one stream per request, levels = 0")
    burst0s, _ = served(octmc.SERVE_STREAMS, np.zeros(nreq), 0, budget)
    auto = {"levels": "0 (automatic: 6 levels at 300-500 A-scans, 7 at 600)",
            "served_poisson_grouped": poisson0, "served_poisson_streams": poisson0s,
            "served_burst_grouped": burst0, "served_burst_streams": burst0s, "sequential_fp32": seq0,
            "accuracy_median_rms_px": accuracy(got0, seq_D0)}
    return {"requests": nreq, "size_classes": [f"{n}x{n}x{d}" for n, d in classes],
            "arrivals": "Poisson, mean inter-arrival 0.25 s", "max_active": max_active, "storage": "bf16",
            "budget_GiB": round(budget / 2**30, 2),
            "grouped_mode": "evaluations of fewer than 128^2 A-scans grouped, larger ones on the request's stream",
            "levels": 4, "iters_per_level": 100,
            "served_poisson_grouped": poisson, "served_burst_grouped": burst,
            "served_burst_streams": burst_streams, "sequential_fp32": seq,
            "accuracy_median_rms_px": acc,
            "automatic_levels": auto}


def _golden(workload, levels, store, pair):
    """The oracle's stored solve of a workload pair (tests/golden, written by
    its script from the oracle alone), if it was made from the same inputs."""
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_solve_golden as G
    g = G.load(workload, levels, store)
    if g is None or g[1].get("input_sha256") != G.input_hash(pair):
        return None
    return g


def _rms_px(a, b):
    """Per-component RMS distance of two fields (numpy or torch)."""
    import numpy as np
    a = a.double().cpu().numpy() if hasattr(a, "cpu") else np.asarray(a, dtype=np.float64)
    b = b.double().cpu().numpy() if hasattr(b, "cpu") else np.asarray(b, dtype=np.float64)
    return [round(float(x), 4) for x in np.sqrt(((a - b) ** 2).reshape(-1, 3).mean(axis=0))]


def clinical_bench(octmc, torch, log, steps=200, warmup=20, cpu=True):
    """The clinical workload (300 x 300 A-scans x 640 samples, float32
    storage): evaluations per second of the full objective and gradient at
    the finest level, the structural kernel (k_struct<float>) against its
    roofs, and full solves at the workload's 4 levels and at the automatic
    depth: time, gauge-free error against ground truth, and distance to the
    FP64 oracle's solve of the same inputs (stored)."""
    import numpy as np
    import synth
    log("clinical 300x300x640: generating on cuda")
    pair = synth.make_pair("clinical", device="cuda", octa_volumes=False)
    h, w, d = pair.sx.shape
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype="f32", levels=4)
    rng = np.random.default_rng(1)
    D = (pair.d_gt + torch.from_numpy(rng.normal(0, 0.2, tuple(pair.d_gt.shape)))).float().cuda()
    terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(D)
    P.eval(0, D, grad=grad, terms=terms, eta_mode=0)
    for _ in range(warmup):
        P.eval(0, D, grad=grad, terms=terms)
    warm_clock(torch, lambda: P.eval(0, D, grad=grad, terms=terms))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        P.eval(0, D, grad=grad, terms=terms)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = np.array([P.eval_profile(0, D, grad=grad, terms=terms) for _ in range(40)]).mean(axis=0)
    alg = 2 * w * h * d * 4 + w * h * EXTRA_BYTES_PER_ASCAN
    t_struct = st[1] * 1e-3
    hbm = alg / t_struct / 1e9
    tfl = FLOP_PER_VOXEL_PAIR * w * h * d / t_struct / 1e12
    out = {"workload": f"clinical orthogonal pair {w}x{h} A-scans x {d} samples, finest level, storage f32",
           "evals_per_s": round(1000.0 / ms, 2), "ms_per_eval": round(ms, 5),
           "hbm_GBps_algorithmic_eval": round(alg / (ms * 1e-3) / 1e9, 1),
           "kernel_ms": {"sum": round(st[0], 5), "struct": round(st[1], 5), "combine": round(st[2], 5)},
           "roofline_struct": {"kernel": "k_struct<float>", "algorithmic_bytes": alg,
                               "hbm": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": round(hbm / HBM_PEAK_GBS, 4)},
                               "alu": {"achieved": round(tfl, 2), "peak": round(VALU_PEAK_TFLOPS, 1),
                                       "unit": "TFLOP/s", "frac": round(tfl / VALU_PEAK_TFLOPS, 4)}}}
    P.close()
    motion = _relative_rms(torch.zeros_like(pair.d_gt), pair.d_gt)
    out["relative_motion_rms_px"] = [round(float(x), 4) for x in motion]
    sol = {}
    for levels in (4, 0):
        for dt, store in (("f32", 0), ("bf16", 1)):
            Q = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=dt,
                           levels=levels)
            Q.register()  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Ds, _, _, rep = Q.register()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            L = Q.levels
            Q.close()
            r = {"levels": L, "seconds": round(el, 4), "evals_total": int(sum(x["evals"] for x in rep)),
                 "relative_rms_vs_ground_truth_px": [round(float(x), 4) for x in _relative_rms(Ds, pair.d_gt)]}
            for st_, tag in ((0, "fp32_inputs"), (store, "rounded_inputs")):
                if tag == "rounded_inputs" and store == 0:
                    continue
                g = _golden("clinical", L, st_, pair)
                if g is not None:
                    Do, meta = g
                    r[f"rms_vs_oracle_{tag}_px"] = _rms_px(Ds, Do)
                    pert = meta.get("perturbation")
                    if pert:
                        r[f"oracle_self_sensitivity_{tag}"] = pert
            sol[f"{dt}_levels{levels}"] = r
            log(f"clinical solve {dt} levels {L}: {el:.3f} s, {r}")
    out["solve"] = sol
    if cpu:
        log("clinical: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pair, D, target_s=6.0)
    del pair
    torch.cuda.empty_cache()
    return out


def enface_bench(octmc, torch, log, reps=20):
    """The segmentation-free en face projection (Sec. 2.3) of one OCTA volume,
    with its percentile normalisation and with a fixed mapping, at the
    paper's 500^2 x 465 volume size and at the dense 500^2 x 800 size.  The
    workspace and inputs are resident; each projection is one stream-ordered
    sequence of kernels, timed with events over `reps` back-to-back runs."""
    import synth
    res = {}
    for n, d in ((500, 465), (500, 800)):
        log(f"en face projection {n}x{n}x{d}: generating OCT and decorrelation OCTA")
        q = synth.make_pair("dense", 1, n=n, d=d, device="cuda", decorrelation=True, white_lines=True)
        s, a, v = q.sx, q.ox, q.vx
        del q
        torch.cuda.empty_cache()
        ws = torch.empty(octmc.enface_workspace_size(n, n, d), dtype=torch.uint8, device="cuda")
        out = torch.empty((n, n), dtype=torch.float32, device="cuda")
        _, _, st = octmc.enface_project(s, a, 0, v, details=True, workspace=ws)
        row = {}
        for mode, fixed in (("percentiles", None), ("fixed_mapping", (st[0], st[1]))):
            for _ in range(3):
                octmc.enface_project(s, a, 0, v, fixed=fixed, workspace=ws, out=out)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                octmc.enface_project(s, a, 0, v, fixed=fixed, workspace=ws, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row[mode] = {"ms_per_volume": round(ms, 4), "volumes_per_s": round(1000.0 / ms, 1)}
        nv = n * n * d
        # the projection must read the OCTA volume and the OCT volume at least once
        row["min_traffic_GBps"] = round(8 * nv / (row["percentiles"]["ms_per_volume"] * 1e-3) / 1e9, 1)
        row["workload"] = f"X-fast OCTA volume {n}x{n} A-scans x {d} samples, float32, white lines"
        log(f"  {row}")
        res[f"{n}x{n}x{d}"] = row
        del s, a, v, ws, out
        torch.cuda.empty_cache()
    res["paper_context"] = "about 209 ms per 500^2 x 465 volume, 66 ms with a fixed mapping (GTX 960)"
    return res


def prealign_bench(octmc, torch, pair, dtype, log, iters=100):
    """Stage-1 rough axial prealignment (per-B-scan offset and tilt) of the
    dense pair: a structural-only pair (delta0 = 0), 4 levels x `iters`
    L-BFGS steps, timed on the host clock around the solve."""
    h, w, _ = pair.sx.shape
    z = torch.zeros((h, w), device="cuda")
    Q = octmc.Pair(pair.sx, pair.sy, ax=z, ay=z, delta0=0.0, levels=4, dtype=dtype)
    log(f"stage-1 prealignment, 4 levels x {iters} steps")
    Q.prealign(1.0, 5)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, rep = Q.prealign(1.0, iters)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    Q.close()
    evals = int(sum(r["evals"] for r in rep))
    return {"seconds": round(sec, 4), "evals": evals, "ms_per_eval": round(1000 * sec / max(evals, 1), 4),
            "storage": dtype, "levels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                                         for r in rep],
            "paper_context": "26.7 s for the prealignment of a 500^2 x 465 pair (i7-6700K + GTX 960, CPU-heavy)"}


def multi_bench(octmc, torch, log, reps=50):
    """Four volumes (two orthogonal pairs of one phantom, white lines) at the
    clinical 300^2 x 640 size: evaluations of the four-volume objective (six
    pair terms) per second at the finest level and one joint solve (4 levels
    x 100 steps), BF16 storage; the evaluation also pair by pair (each volume
    resampled once per pair) beside the fused pass."""
    import synth
    log("four volumes 300x300x640: generating")
    sc = synth.make_scans("clinical", 0, (0, 1, 0, 1), device="cuda", white_lines=True)
    M = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, dtype="bf16")
    n, h, w = 4, sc.S[0].shape[0], sc.S[0].shape[1]
    D = (sc.d_gt + 0.2 * torch.randn(sc.d_gt.shape, generator=torch.Generator().manual_seed(1),
                                     dtype=torch.float64)).float().cuda()

    def time_evals(m):
        m.eval(0, D, eta_mode=0)
        for _ in range(5):
            m.eval(0, D)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            m.eval(0, D)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = time_evals(M)
    Mp = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, dtype="bf16", pairwise=True)
    ms_pairwise = time_evals(Mp)
    Mp.close()
    f32 = {}
    for pw in (False, True):
        Mf = octmc.Multi(sc.S, sc.orient, enface=sc.A, valid=sc.V, levels=4, dtype="f32", pairwise=pw)
        f32["ms_per_eval_pairwise" if pw else "ms_per_eval"] = round(time_evals(Mf), 4)
        Mf.close()
    log("four volumes: joint solve")
    t0 = time.perf_counter()
    Dsol, _, _, rep = M.register()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    err = [round(float(x), 4) for x in _interior_rms(Dsol, sc.d_gt)]
    M.close()
    return {"workload": "four volumes (X, Y, X, Y) 300x300 A-scans x 640 samples, BF16 storage",
            "ms_per_eval": round(ms, 4), "evals_per_s": round(1000.0 / ms, 1), "pair_terms_per_eval": 6,
            "ms_per_eval_pairwise": round(ms_pairwise, 4), "float32_storage": f32,
            "solve_seconds": round(sec, 3), "solve_evals": int(sum(r["evals"] for r in rep)),
            "solve_rms_vs_ground_truth_px": err}


def autograd_bench(octmc, torch, log, reps=50):
    """The differentiation variant: 8 independent pairs of 200^2 x 512 FP32
    as one batched objective (one grouped launch per kernel) behind
    torch.autograd (OctmcObjective): forward + backward per second, beside
    the grouped evaluation alone and 8 single-pair evaluations."""
    import synth
    B = 8
    log("autograd: generating 8 pairs 200x200x512")
    pairs = [synth.make_pair("batch", b, device="cuda", octa_volumes=False) for b in range(B)]
    Ps = [octmc.Pair(q.sx, q.sy, ax=q.ax, ay=q.ay, vx=q.vx, vy=q.vy, levels=3) for q in pairs]
    D = torch.stack([(q.d_gt + 0.2 * torch.randn(q.d_gt.shape, generator=torch.Generator().manual_seed(b),
                                                 dtype=torch.float64)).float() for b, q in enumerate(pairs)]).cuda()
    octmc.eval_batched(Ps, 0, D, eta_mode=0)  # each pair's eta at this level (Eq. 10)
    torch.cuda.synchronize()

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def fwd_bwd():
        Dv = D.detach().requires_grad_(True)
        octmc.objective(Dv, Ps, 0).sum().backward()

    ms_ad = timed(fwd_bwd)
    ms_grouped = timed(lambda: octmc.eval_batched(Ps, 0, D))
    ms_single = timed(lambda: [P.eval(0, D[b]) for b, P in enumerate(Ps)])
    for P in Ps:
        P.close()
    return {"workload": "8 pairs 200x200 A-scans x 512 samples, FP32 storage, finest level",
            "ms_per_forward_backward": round(ms_ad, 4), "pair_evals_per_s": round(B * 1000.0 / ms_ad, 1),
            "ms_per_grouped_eval": round(ms_grouped, 4), "ms_per_8_single_evals": round(ms_single, 4)}


def pipeline_bench(octmc, torch, log, runs=3):
    """The whole method of Fig. 1 on one pair at the paper's volume size
    (500^2 x 465; OCT and OCTA volumes resident on the device, BF16 storage):
    pair creation with stage-1 prealignment, saccade detection from the OCTA
    volumes and the en face projections, then the 4-level registration and
    the merge of both OCT and OCTA volumes.  Wall time per pair (median)."""
    import synth
    log("pipeline: generating a 500x500x465 pair with OCTA volumes")
    q = synth.make_pair("dense", 2, n=500, d=465, device="cuda", decorrelation=True, white_lines=True)
    out = {}
    times = []
    for r in range(runs + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = octmc.Pair(q.sx, q.sy, ox=q.ox, oy=q.oy, dtype="bf16", levels=4, prealign=True, detect_invalid=True,
                       project_enface=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        D, mo, ma, rep = P.register(merged=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        P.close()
        del D, mo, ma
        if r > 0:  # the first run warms up
            times.append((t1 - t0, t2 - t1))
    times.sort(key=lambda t: t[0] + t[1])
    c, g = times[len(times) // 2]
    out = {"workload": "pair 500x500 A-scans x 465 samples with OCTA volumes, BF16 storage, 4 levels x 100 steps",
           "create_s": round(c, 4), "register_and_merge_s": round(g, 4), "total_s": round(c + g, 4),
           "create_steps": "ingest, stage-1 prealignment, axial resampling, saccade detection, en face projections, "
                           "pyramid",
           "paper_context": "86.1 s in total for a 500^2 x 465 pair including saccade detection and merging "
                            "(i7-6700K + GTX 960), of which 11.5 s read/write"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f16", "f32"], help="storage of the volumes")
    ap.add_argument("--n", type=int, default=500)
    ap.add_argument("--d", type=int, default=800)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-enface", action="store_true", help="skip the en face projection timing")
    ap.add_argument("--no-prealign", action="store_true", help="skip the stage-1 prealignment timing")
    ap.add_argument("--no-multi", action="store_true", help="skip the four-volume timing")
    ap.add_argument("--no-autograd", action="store_true", help="skip the batched autograd timing")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the whole-pipeline timing at 500^2 x 465")
    ap.add_argument("--no-clinical", action="store_true", help="skip the 300^2 x 640 float32 evaluation and solves")
    ap.add_argument("--extras-only", action="store_true",
                    help="time only the stage-1 prealignment, the four-volume path, the batched autograd "
                         "objective and the projection")
    ap.add_argument("--enface-only", action="store_true", help="time only the en face projection")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=48.0)
    ap.add_argument("--serve-max-active", type=int, default=8)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the timed evaluations and the calibration copies (for rocprofv3)")
    ap.add_argument("--profile-workload", default="dense", choices=["dense", "clinical"],
                    help="with --profile-only: the dense pair (--dtype storage) or the clinical pair (float32)")
    ap.add_argument("--profile-solve", action="store_true",
                    help="only two full registrations of the dense pair (--dtype storage, automatic pyramid depth; "
                         "with --host-line-search the host-decision form), for rocprofv3")
    ap.add_argument("--host-line-search", action="store_true", help="with --profile-solve: OCTMC_HOST_LINE_SEARCH")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic of the structural kernel from two rocprofv3 counter passes")
    ap.add_argument("--summary-out", default=os.path.join(ROOT, "profiles", "k_struct_dense_counters.json"))
    ap.add_argument("--summary-command", default="")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.dtype, args.summary_out, args.summary_command)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (pairs are independent: a multi-GPU "
              f"deployment runs one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2010_06931_amd as octmc
    import synth

    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    free, total = torch.cuda.mem_get_info()
    log(f"device {props.name}: {props.multi_processor_count} CUs, {total / 2**30:.1f} GiB "
        f"({free / 2**30:.1f} GiB free)")
    if args.enface_only:
        print(json.dumps({"enface_projection": enface_bench(octmc, torch, log)}), flush=True)
        return
    if args.extras_only:
        log(f"generating the dense pair {args.n}x{args.n}x{args.d} on cuda (structural)")
        pair = synth.make_pair("dense", n=args.n, d=args.d, device="cuda", octa_volumes=False)
        extra = {"prealign": prealign_bench(octmc, torch, pair, args.dtype, log)}
        del pair
        torch.cuda.empty_cache()
        extra["multi_volume"] = multi_bench(octmc, torch, log)
        extra["autograd_batch"] = autograd_bench(octmc, torch, log)
        extra["pipeline"] = pipeline_bench(octmc, torch, log)
        extra["enface_projection"] = enface_bench(octmc, torch, log)
        print(json.dumps(extra), flush=True)
        return
    if args.profile_solve:
        log(f"generating the dense pair {args.n}x{args.n}x{args.d} on cuda")
        pair = synth.make_pair("dense", n=args.n, d=args.d, device="cuda", octa_volumes=False)
        P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=args.dtype, levels=0,
                       host_line_search=args.host_line_search)
        secs = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, rep = P.register()
            torch.cuda.synchronize()
            secs.append(round(time.perf_counter() - t0, 4))
        print(json.dumps({"workload": f"dense {args.n}x{args.n}x{args.d} {args.dtype}, automatic depth",
                          "decisions": "host" if args.host_line_search else "device", "seconds": secs,
                          "levels": len(rep), "evals": sum(r["evals"] for r in rep)}))
        return
    if args.profile_only and args.profile_workload == "clinical":
        # the clinical workload's finest-level evaluations alone (float32 storage), for rocprofv3
        log("generating the clinical pair 300x300x640 on cuda")
        pair = synth.make_pair("clinical", device="cuda", octa_volumes=False)
        P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype="f32", levels=4)
        D = (pair.d_gt + torch.from_numpy(np.random.default_rng(1).normal(0, 0.2, tuple(pair.d_gt.shape)))).float().cuda()
        terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
        grad = torch.empty_like(D)
        P.eval(0, D, grad=grad, terms=terms, eta_mode=0)
        for _ in range(args.warmup + args.steps):
            P.eval(0, D, grad=grad, terms=terms)
        torch.cuda.synchronize()
        st = np.array([P.eval_profile(0, D, grad=grad, terms=terms) for _ in range(args.steps)]).mean(axis=0)
        print(json.dumps({"workload": "clinical 300x300x640 f32", "struct_ms_events": round(float(st[1]), 5)}))
        return
    log(f"generating the dense pair {args.n}x{args.n}x{args.d} on cuda")
    pair = synth.make_pair("dense", n=args.n, d=args.d, device="cuda", octa_volumes=False)
    log("ingest")
    P = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=args.dtype, levels=4)
    rng = np.random.default_rng(1)
    D = (pair.d_gt + torch.from_numpy(rng.normal(0, 0.2, tuple(pair.d_gt.shape)))).float().cuda()
    terms = torch.empty(octmc.NTERMS, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(D)
    P.eval(0, D, grad=grad, terms=terms, eta_mode=0)  # eta of this level (Eq. 10)
    for _ in range(args.warmup):
        P.eval(0, D, grad=grad, terms=terms)
    torch.cuda.synchronize()
    # after the W warmup steps, evaluations continue untimed until
    # WARM_SECONDS of device work have run, so that the K timed steps see the
    # steady clock whatever W is (warm_clock)
    extra_warm = warm_clock(torch, lambda: P.eval(0, D, grad=grad, terms=terms))
    log(f"timing {args.steps} evaluations (after {args.warmup} + {extra_warm} warmup evaluations)")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        P.eval(0, D, grad=grad, terms=terms)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    evals_s = 1000.0 / ms
    log(f"{ms:.4f} ms/eval ({evals_s:.1f} evals/s), wall {wall:.2f} s")
    if args.profile_only:
        calibration_copies(torch)
        print(json.dumps({"ms_per_eval": ms}))
        return

    # achievable HBM rate on this device: a 1 GiB device-to-device copy (read + write)
    ca = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        cb.copy_(ca)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del ca, cb

    # spread of single evaluations: one event between consecutive evaluations
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record()
    for k in range(args.steps):
        P.eval(0, D, grad=grad, terms=terms)
        evs[k + 1].record()
    torch.cuda.synchronize()
    per_eval = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    pct = {f"p{q}": round(float(np.percentile(per_eval, q)), 5) for q in (10, 50, 90)}

    # dominant kernel timed live with HIP events on its stream
    stages = np.array([P.eval_profile(0, D, grad=grad, terms=terms) for _ in range(max(20, args.steps // 4))])
    st_ms = stages.mean(axis=0)
    w, h, d = args.n, args.n, args.d
    esz = 4 if args.dtype == "f32" else 2
    alg_bytes = 2 * w * h * d * esz + w * h * EXTRA_BYTES_PER_ASCAN
    t_struct = st_ms[1] * 1e-3
    hbm = alg_bytes / t_struct / 1e9
    flops = FLOP_PER_VOXEL_PAIR * w * h * d / t_struct / 1e12
    traffic = load_traffic(args.dtype)
    hbm_obj = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu_obj = {"bound": "alu", "achieved": round(flops, 2), "peak": round(VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
               "frac": round(flops / VALU_PEAK_TFLOPS, 4), "traffic": traffic}
    roof, other = (alu_obj, hbm_obj) if alu_obj["frac"] >= hbm_obj["frac"] else (hbm_obj, alu_obj)

    out = {"metric": METRIC, "value": round(evals_s, 2), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "warmup_extra_for_clock_ramp": extra_warm, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"dense orthogonal pair {w}x{h} A-scans x {d} samples, finest level, "
                                  f"storage {args.dtype}", "w": w, "h": h, "d": d, "level": 0,
                      "storage": args.dtype, "parallelism": "single GPU"},
           "roofline": roof, "roofline_other": other, "ms_per_eval_percentiles": pct,
           "kernel_ms": {"sum": round(st_ms[0], 5), "struct": round(st_ms[1], 5), "combine": round(st_ms[2], 5)},
           "hbm_GBps_algorithmic": round(hbm, 1), "hbm_copy_GBps": round(copy_gbs, 1)}

    if not args.no_variants:
        var = {}
        for dt in ("bf16", "f16", "f32"):
            if dt == args.dtype:
                continue
            log(f"variant storage {dt}")
            Q = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=dt, levels=4)
            Q.eval(0, D, grad=grad, terms=terms, eta_mode=0)
            for _ in range(args.warmup):
                Q.eval(0, D, grad=grad, terms=terms)
            warm_clock(torch, lambda: Q.eval(0, D, grad=grad, terms=terms))
            e0.record()
            for _ in range(args.steps):
                Q.eval(0, D, grad=grad, terms=terms)
            e1.record()
            torch.cuda.synchronize()
            vms = e0.elapsed_time(e1) / args.steps
            vst = np.array([Q.eval_profile(0, D, grad=grad, terms=terms) for _ in range(20)]).mean(axis=0)
            vb = 2 * w * h * d * (4 if dt == "f32" else 2) + w * h * EXTRA_BYTES_PER_ASCAN
            var[dt] = {"evals_per_s": round(1000 / vms, 2), "struct_ms": round(vst[1], 5),
                       "hbm_GBps_algorithmic": round(vb / (vst[1] * 1e-3) / 1e9, 1)}
            if not args.no_solve:
                t0 = time.perf_counter()
                Dq, _, _, _ = Q.register()
                torch.cuda.synchronize()
                var[dt]["solve_s"] = round(time.perf_counter() - t0, 4)
                var[dt]["solution"] = Dq
            Q.close()
            del Q
        out["storage_variants"] = var

    if not args.no_solve:
        log("full solve (4 levels x 100 L-BFGS steps)")
        P.register()  # warm
        torch.cuda.synchronize()
        lat = []
        for _ in range(3):
            t0 = time.perf_counter()
            Dsol, _, _, rep = P.register()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        rms_main = _interior_rms(Dsol, pair.d_gt)
        sols = {args.dtype: Dsol}
        for dt, v in out.get("storage_variants", {}).items():
            if v.get("solution") is not None:
                sols[dt] = v["solution"]
        ref32 = sols.get("f32")

        def vs32(D):
            return None if ref32 is None else [
                round(float(x), 4) for x in np.sqrt(((D - ref32).double().cpu().numpy() ** 2).reshape(-1, 3).mean(axis=0))]

        out["solve"] = {"storage": args.dtype, "seconds_median": round(float(np.median(lat)), 4),
                        "pairs_per_s": round(1 / float(np.median(lat)), 3),
                        "levels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()} for r in rep],
                        "evals_total": int(sum(r["evals"] for r in rep)),
                        "rms_vs_ground_truth_px": [round(float(x), 4) for x in rms_main],
                        "relative_rms_vs_ground_truth_px": [round(float(x), 4) for x in
                                                            _relative_rms(Dsol, pair.d_gt)],
                        "relative_motion_rms_px": [round(float(x), 4) for x in
                                                   _relative_rms(torch.zeros_like(pair.d_gt), pair.d_gt)],
                        "rms_vs_ground_truth_um": [round(float(x * s), 2) for x, s in zip(rms_main, UM_PER_PX)],
                        "rms_vs_fp32_storage_solve_px": vs32(Dsol)}
        # against the FP64 oracle's solve of the same inputs (stored; float32
        # inputs, so for 16-bit storage this is storage plus compute error)
        g = _golden("dense", 4, 0, pair)
        if g is not None:
            Do, meta = g
            for dt, Dq in sols.items():
                px = _rms_px(Dq, Do)
                rec = out["solve"] if dt == args.dtype else out["storage_variants"][dt]
                rec["rms_vs_oracle_px"] = px
                rec["rms_vs_oracle_um"] = [round(x * u, 3) for x, u in zip(px, UM_PER_PX)]
            if meta.get("perturbation"):
                out["solve"]["oracle_self_sensitivity"] = meta["perturbation"]
        # the same pair with the automatic pyramid depth (levels = 0)
        Pa = octmc.Pair(pair.sx, pair.sy, ax=pair.ax, ay=pair.ay, vx=pair.vx, vy=pair.vy, dtype=args.dtype, levels=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Da, _, _, _ = Pa.register()
        torch.cuda.synchronize()
        out["solve"]["automatic_levels"] = {
            "levels": Pa.levels, "seconds": round(time.perf_counter() - t0, 4),
            "rms_vs_ground_truth_px": [round(float(x), 4) for x in _interior_rms(Da, pair.d_gt)],
            "relative_rms_vs_ground_truth_px": [round(float(x), 4) for x in _relative_rms(Da, pair.d_gt)]}
        Pa.close()
        del Da
        for dt, v in out.get("storage_variants", {}).items():
            Dq = v.pop("solution", None)
            if Dq is None:
                continue
            r = _interior_rms(Dq, pair.d_gt)
            v["solve_rms_vs_ground_truth_px"] = [round(float(x), 4) for x in r]
            v["solve_rms_vs_ground_truth_um"] = [round(float(x * s), 2) for x, s in zip(r, UM_PER_PX)]
            if dt != "f32":
                v["solve_rms_vs_fp32_storage_solve_px"] = vs32(Dq)

    for v in out.get("storage_variants", {}).values():
        v.pop("solution", None)
    if not args.no_clinical:
        out["clinical"] = clinical_bench(octmc, torch, log, cpu=not args.no_cpu_baseline)
    if not args.no_prealign:
        out["prealign"] = prealign_bench(octmc, torch, pair, args.dtype, log)
    if not args.no_serve:
        out["serving"] = serving(octmc, torch, args.serve_requests, args.serve_budget_gib, args.serve_max_active, log)

    if not args.no_multi:
        out["multi_volume"] = multi_bench(octmc, torch, log)
    if not args.no_autograd:
        out["autograd_batch"] = autograd_bench(octmc, torch, log)
    if not args.no_pipeline:
        out["pipeline"] = pipeline_bench(octmc, torch, log)

    if not args.no_enface:
        del P
        torch.cuda.empty_cache()
        out["enface_projection"] = enface_bench(octmc, torch, log)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pair, D)
        out["cpu_baseline_small"] = cpu_baseline_small(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
