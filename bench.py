#!/usr/bin/env python3
"""Benchmark: complex double-double Newton steps per second.

Workload of the reported value: the dense n = 32 random system (32 monomials
per equation, each a product of 16 distinct variables with exponents uniform
in {1, 2, 3}, unit-circle coefficients) and B = 10240 distinct random
unit-modulus points.  One benchmark step applies one complete Newton step
(evaluation and differentiation by reverse mode, summation, modified
Gram-Schmidt solve, back substitution, update) to every point, starting each
step from the same points, so every step does the same work.  Inputs are
resident in device memory before the timed region.

Reported beside it, one object per workload:
* qd: the same in quad-double (2048 points);
* single: one Newton step of one point (latency);
* track8: single paths of random n = 8 systems tracked from t = 0 to 1
  (100 systems; status, steps, latency and paths/s), and of their
  finite-roots variants (every path ends at a finite root);
* sparse512: one Newton step of the sparse n = 512 system per MGS variant,
  with the bitwise comparison of the variants;
* batch64: 4096 paths of 64 random systems in one slot-table batch (Newton
  steps/s, paths/s of a finite-roots variant tracked to completion, and the
  time to a residual of 1e-28 of the plain and the mixed-precision corrector);
* serve: continuous batching of track_path requests at several arrival
  rates, with the one-at-a-time baseline on the same trace;
* cyclic: evaluation and differentiation of the cyclic n-roots system
  (n = 128, 352);
* double: complex double, reverse against tree-mode monomials.
Every GPU leg keeps a sample of its results; the CPU leg (the oracle, timed
on this host's cores) computes their errors against the oracle: forward
differences, normwise backward errors formed at 320 bits from the oracle's
quad-double Jacobian and residual, status and step counts of tracked paths.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import platform
import sys
import threading
import time

# The serving leg runs one stream per lane (6 lanes).  HIP maps streams onto
# GPU_MAX_HW_QUEUES hardware queues (4 by default), and streams that share a
# queue run in order, which would make small systems wait for large ones; the
# variable is read when the HIP runtime starts, so it is set before torch.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# HBM traffic per launch of the dense-DD kernels at 10240 points, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this leg (KiB per dispatch; the
# MGS per lane-group width and storage of [A | b], from the autotuner's
# launches), calibrated on the 10 MiB copy of the start points in the same
# runs (FETCH_SIZE reads 5131.5 KiB, WRITE_SIZE 10240 KiB for 10,485,760
# bytes).  The figures of a kernel hold for the sources whose digest is
# COUNTERS_DIGEST[kernel] (source_digest(kernel), over KERNEL_SOURCES[kernel]);
# other sources report traffic null.
HBM_COUNTERS_KIB = {
    "mgs": {(8, 0): (893249.1, 5304935.0), (8, 1): (274858.2, 205533.6), (8, 2): (274998.0, 205976.8),
            (8, 3): (437413.0, 542423.9), (16, 0): (889280.4, 4627086.8), (16, 1): (274869.4, 205816.3),
            (16, 2): (275004.8, 205733.9), (16, 3): (462631.3, 540749.1), (32, 0): (798724.1, 4027138.7),
            (32, 1): (274879.8, 206869.0), (32, 3): (556396.1, 538210.7)},
    "eval_monomials": (37741.6, 5570560.0), "eval_sums": (3653995.9, 393668.3)}
KERNEL_SOURCES = {
    "mgs": ("mgs.hip", "mgs_common.hpp", "mp.hpp", "internal.hpp", "tune.hip"),
    "eval_monomials": ("eval.hip", "eval_body.hpp", "mp.hpp", "internal.hpp"),
    "eval_sums": ("eval.hip", "eval_body.hpp", "mp.hpp", "internal.hpp"),
}
COUNTERS_DIGEST = {"mgs": "628da6c22ca3657c", "eval_monomials": "eb84ed1d7708358a",
                   "eval_sums": "eb84ed1d7708358a"}
MGS_PIN = None  # (lane group, storage) from --mgs-group / --mgs-storage, else autotuned
TUNE_REPS = 20  # Newton steps per MGS configuration the autotuner times (--tune-reps)


def set_tune_reps(reps: int) -> None:
    global TUNE_REPS
    TUNE_REPS = max(1, int(reps))
FETCH_CAL, WRITE_CAL = 10485760 / (5131.5 * 1024), 1.0
_T0 = time.time()
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "diverged", 3: "max_steps", 4: "step_too_small",
                5: "nan", -4: "singular"}


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.time() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def source_digest(kernel: str) -> str:
    """Digest of the sources a kernel is built from (its counter figures
    hold for one digest)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1501_06625_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel, ()):
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


B_DD = 10240
B_QD = 2048
# extrapolation degree of the tracked finite-roots paths (batch and serving)
PLANTED_ORDER = 4


def status_hist(codes) -> dict:
    hist = {}
    for c in codes:
        k = STATUS_NAMES.get(int(c), str(int(c)))
        hist[k] = hist.get(k, 0) + 1
    return hist


def limb_diff_max(a, b) -> float:
    """max over entries of |a - b| for limb arrays [..., 2, P] (leading limbs
    subtracted first)."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a[..., 0] - b[..., 0]
    for j in range(1, a.shape[-1]):
        d = d + (a[..., j] - b[..., j])
    return float(np.abs(d[..., 0] + 1j * d[..., 1]).max()) if d.size else 0.0


def lead_abs_max(a) -> float:
    import numpy as np
    a = np.asarray(a)
    return float(np.abs(a[..., 0, 0] + 1j * a[..., 1, 0]).max()) if a.size else 0.0


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def dense_leg(hcn, flops, S, dev, P: int, B: int, K: int, W: int, profile: bool, keep: int):
    import torch
    ps = S.dense32_system(0, P)
    pts = S.dense32_points(0, B, P)
    sysd = hcn.System(ps)
    x0 = torch.from_numpy(pts).to(dev)
    x = torch.empty_like(x0)
    if B > 1 and MGS_PIN is not None:
        hcn.tune_set(P, ps.N, MGS_PIN[0], MGS_PIN[1])
        tuned = (MGS_PIN[0], MGS_PIN[1], None)
    else:
        tuned = hcn.autotune(sysd, x0, reps=TUNE_REPS) if B > 1 else None
    ws = hcn.newton_ws(sysd, B)
    for _ in range(W):
        x.copy_(x0)
        hcn.newton_step(sysd, x, ws=ws)
    torch.cuda.synchronize()
    if profile:
        hcn.profile_reset()
        hcn.profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(K):
        x.copy_(x0)
        norms, status = hcn.newton_step(sysd, x, ws=ws)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    kern = {}
    if profile:
        hcn.profile_enable(False)
        for name in ("eval_monomials", "eval_sums", "mgs"):
            ms, cnt = hcn.profile_query(name)
            kern[name] = (ms, cnt)
        hcn.profile_reset()
    ok = int((status == 0).sum().item())
    fl = flops.newton_step(ps, P)
    # a sample of points spread over the batch for the oracle comparison
    idx = list(range(0, B, max(1, B // keep)))[:keep]
    sample = {"P": P, "x0": pts[idx], "x1": x[idx].cpu().numpy(), "index": idx}
    sysd.free()
    return dict(ms_per_step=ev_ms / K, wall_s=wall, B=B, ok=ok, flops=fl, kern=kern, tuned=tuned,
                sample=sample)


def track8_leg(hcn, S, dev, seeds: int = 100, mode_seeds: int = 8) -> dict:
    """Single paths: random n = 8 systems (8 monomials per equation of 3
    distinct variables, exponents 1..2), each path tracked from x = 1 at
    t = 0 to t = 1 (secant predictor, at most 3 Newton iterations a step,
    end-point refinement to 1e-28), one path at a time by the single-system
    tracker (100 systems; host wall time per path, the result on the host),
    and, for the first 8, also by a one-slot batch replaying its captured step
    and by a one-slot batch with one persistent workgroup (each of these
    first 8 is run twice and timed on the second run)."""
    import numpy as np
    import torch
    modes = ("tracker", "batch_graph", "batch_persistent")
    per = {m: [] for m in modes}
    sample = []
    for seed in range(seeds):
        ps = S.small_track_system(seed, 2)
        sd = hcn.System(ps)
        gam = S.random_unit_gamma(S.rng_for(0, 100 + seed), 2)
        x0 = torch.from_numpy(S.ones_point(ps.n, 2)).to(dev)
        for m in modes if seed < mode_seeds else modes[:1]:
            for rep in range(2 if seed < mode_seeds else 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if m == "tracker":
                    xo, r = hcn.track_paths(sd, gam, x0[None])
                    xo, r = xo[0], r[0]
                else:
                    bt = hcn.Batch(2, 1, ps.n, sd.info().nslots, persistent=(m == "batch_persistent"))
                    bt.add(0, sd, gam, x0)
                    bt.run(chunk=32)
                    xo, r = bt.result(0, ps.n)
                    bt.free()
                xh = xo.cpu().numpy()
                dt = time.perf_counter() - t0
            per[m].append((dt, int(r["steps"])))
            if m == "tracker":
                sample.append({"seed": seed, "gamma": gam, "x0": S.ones_point(ps.n, 2), "x1": xh,
                               "status": int(r["status"]), "steps": int(r["steps"])})
        sd.free()
    ms = np.array([d for d, _ in per["tracker"]]) * 1e3
    ok = sum(1 for s in sample if s["status"] == 0)
    res = {"paths": seeds, "ok": ok, "success_rate": ok / seeds,
           "status": status_hist([s["status"] for s in sample]),
           "steps_median": float(np.median([s["steps"] for s in sample])),
           "paths_per_s": seeds / (ms.sum() / 1e3),
           "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99))}
    for m in modes:
        res[m] = {"paths": len(per[m]),
                  "ms_per_path_median": float(np.median([d for d, _ in per[m]]) * 1e3),
                  "us_per_step": float(sum(d for d, _ in per[m]) / max(sum(k for _, k in per[m]), 1) * 1e6)}
    res["sample"] = sample
    # the finite-roots variant of the same systems (each equation gains a
    # pure power of its degree and a constant term, so no path goes to
    # infinity): the tracker with the degree-4 predictor, one path at a time
    progress("track8: finite-roots systems")
    fsample, fms = [], []
    for seed in range(seeds):
        ps = S.with_finite_roots(S.small_track_system(seed, 2), seed)
        sd = hcn.System(ps)
        gam = S.random_unit_gamma(S.rng_for(0, 100 + seed), 2)
        x0 = torch.from_numpy(S.ones_point(ps.n, 2)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xo, r = hcn.track_paths(sd, gam, x0[None], predictor_order=PLANTED_ORDER)
        xh = xo[0].cpu().numpy()
        fms.append((time.perf_counter() - t0) * 1e3)
        r = r[0]
        fsample.append({"seed": seed, "gamma": gam, "x0": S.ones_point(ps.n, 2), "x1": xh,
                        "status": int(r["status"]), "steps": int(r["steps"]), "end_status": int(r["end_status"])})
        sd.free()
    fms = np.array(fms)
    fok = sum(1 for q in fsample if q["status"] == 0)
    res["finite_roots"] = {
        "paths": seeds, "predictor_order": PLANTED_ORDER, "ok": fok, "success_rate": fok / seeds,
        "ok_and_refined_to_1e-28": int(sum(1 for q in fsample if q["status"] == 0 and q["end_status"] == 0)),
        "status": status_hist([q["status"] for q in fsample]),
        "steps_median": float(np.median([q["steps"] for q in fsample])),
        "paths_per_s": seeds / (fms.sum() / 1e3),
        "p50_ms": float(np.percentile(fms, 50)), "p99_ms": float(np.percentile(fms, 99)),
        "us_per_step": float(fms.sum() * 1e3 / max(sum(q["steps"] for q in fsample), 1))}
    res["sample_finite"] = fsample
    return res


SPARSE_RUNS = [(1, 16, "workgroup"), (2, 16, "right_looking"), (5, 16, "pipelined"),
               (4, 16, "tiled_T16"), (4, 8, "tiled_T8"), (4, 4, "tiled_T4")]


def sparse512_leg(hcn, flops, S, dev, reps: int = 10, variants=None) -> dict:
    """Sparse n = 512 system (4 monomials of 2 variables + a constant per
    equation): one Newton step of one point, timed per MGS variant (all, or
    the names in variants).  The solve dominates (17.2 GFLOP of MGS against
    1 MFLOP of evaluation).  The updated points of the variants are compared
    bit for bit with the right-looking one."""
    import numpy as np
    import torch
    ps = S.sparse512_system(0, 2)
    pts = S.random_unit_point(S.rng_for(2, 99), ps.n, 2)[None]
    sysd = hcn.System(ps)
    x0 = torch.from_numpy(pts).to(dev)
    x = torch.empty_like(x0)
    ws = hcn.newton_ws(sysd, 1)
    mgs_flops = flops.mgs_solve(ps.N, ps.n, 2)
    res = {}
    outs = {}
    for v, T, name in SPARSE_RUNS:
        if variants and name not in variants:
            continue
        hcn.set_mgs_variant(v)
        hcn.set_mgs_panel(T)
        x.copy_(x0)
        hcn.newton_step(sysd, x, ws=ws)
        torch.cuda.synchronize()
        hcn.profile_reset()
        hcn.profile_enable(True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            x.copy_(x0)
            hcn.newton_step(sysd, x, ws=ws)
        stop.record()
        torch.cuda.synchronize()
        hcn.profile_enable(False)
        ms_mgs, cnt = hcn.profile_query("mgs")
        hcn.profile_reset()
        step_ms = start.elapsed_time(stop) / reps
        mgs_ms = ms_mgs / max(cnt, 1)
        outs[name] = x[0].cpu().numpy()
        res[name] = {"newton_step_ms": step_ms, "mgs_ms": mgs_ms,
                     "mgs_tflops": mgs_flops / (mgs_ms / 1e3) / 1e12,
                     "mgs_frac_fp64_peak": mgs_flops / (mgs_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS}
    hcn.set_mgs_variant(0)
    hcn.set_mgs_panel(16)
    sysd.free()
    if "right_looking" in outs:
        ref = outs["right_looking"]
        for name, xo in outs.items():
            res[name]["bitwise_equal_right_looking"] = bool(np.array_equal(xo.view(np.uint64),
                                                                            ref.view(np.uint64)))
    res["mgs_gflop"] = mgs_flops / 1e9
    res["sample"] = {"x0": pts[0], "x1": outs}
    # two points of the system at once (paths of one system tracked
    # together): the two pipelined chains share the CUs (two workgroups per
    # CU; more would not fit the LDS with n = 512)
    if not variants or "pipelined" in variants:
        for B in (2,):
            ptsB = S.random_unit_point(S.rng_for(2, 100 + B), ps.n * B, 2).reshape(B, ps.n, 2, 2)
            sysd = hcn.System(ps)
            xB0 = torch.from_numpy(ptsB).to(dev)
            xB = torch.empty_like(xB0)
            wsB = hcn.newton_ws(sysd, B)
            hcn.set_mgs_variant(5)
            xB.copy_(xB0)
            hcn.newton_step(sysd, xB, ws=wsB)
            torch.cuda.synchronize()
            hcn.profile_reset()
            hcn.profile_enable(True)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                xB.copy_(xB0)
                hcn.newton_step(sysd, xB, ws=wsB)
            stop.record()
            torch.cuda.synchronize()
            hcn.profile_enable(False)
            ms_mgs, cnt = hcn.profile_query("mgs")
            hcn.profile_reset()
            hcn.set_mgs_variant(0)
            mgs_ms = ms_mgs / max(cnt, 1)
            res[f"pipelined_{B}_points"] = {
                "newton_step_ms": start.elapsed_time(stop) / reps, "mgs_ms": mgs_ms,
                "mgs_tflops": B * mgs_flops / (mgs_ms / 1e3) / 1e12,
                "mgs_frac_fp64_peak": B * mgs_flops / (mgs_ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS}
            sysd.free()
    return res


def batch_leg(hcn, flops, S, dev, nsys: int = 64, per: int = 64, steps: int = 10,
              split_n: int = 0, steps_only: bool = False) -> dict:
    """64 random systems (n in [16, 96], 16..64 monomials per equation, 4..12
    variables per monomial, exponents 1..3), 64 total-degree start solutions
    each: 4096 paths in one slot-table batch, in complex DD.
    * plain / mixed: a fixed number of predictor-corrector steps with the
      plain and with the mixed-precision corrector (Newton steps/s, FLOP/s);
      residual evaluations and solves counted per path on the device, flops
      per path from its own system.  These systems have no constant term, so
      most of their total-degree paths run to x = 0 or to infinity.
    * paths_finite: the finite-roots variant (per equation a pure power
      x_i^{d_i} and a constant term that makes x = (1, ..., 1) a root: no
      roots at infinity, so every total-degree path ends at a finite root),
      all 4096 paths tracked to completion with the predictor of degree 4
      (Section 4.2), end-point refinement to 1e-28 included: paths/s,
      status, steps.
    * newton_1e28: Newton's method from 1e-6 perturbations of the root
      x = 1 of the same variant (64 points per system), plain against mixed
      precision, until the residual is below 1e-28: time, iterations,
      distance to the root."""
    import numpy as np
    import torch
    systems = S.batch_systems(nsys, seed=0, P=2)
    loaded = [hcn.System(ps) for ps in systems]
    infos = [s.info() for s in loaded]
    max_n = max(ps.n for ps in systems)
    max_slots = max(i.nslots for i in infos)
    rng = S.rng_for(3, 777)
    starts, gammas = [], []
    for ps in systems:
        degs = S.degrees(ps)
        gammas.append(S.random_unit_gamma(rng, 2))
        starts.append(torch.from_numpy(np.stack([S.start_solution(rng, degs, 2)
                                                 for _ in range(per)])).to(dev))
    fl_plain = [flops.newton_step(ps, 2) for ps in systems]
    fl_mixed = [flops.mixed_step(ps, 2) for ps in systems]
    res = {"systems": nsys, "paths": nsys * per, "timed_steps": steps}
    # tune the MGS for every row-count bucket (a power of two) on one system
    # of the bucket at 256 of its start points; the batch reads the same table
    progress("batch: tuning the MGS per row-count bucket")
    tuned = {}
    for ps, sd, st in zip(systems, loaded, starts):
        bucket = 1 << max(3, (ps.N - 1).bit_length())
        if bucket not in tuned:
            tuned[bucket] = hcn.autotune(sd, st.repeat(4, 1, 1, 1).contiguous(), reps=3)[:2]
    res["mgs_tuned"] = {str(k): list(v) for k, v in sorted(tuned.items())}
    progress("batch: systems and start points ready")
    for mode in ("plain", "mixed"):
        progress(f"batch: {mode}, {steps} steps")
        bt = hcn.Batch(2, nsys * per, max_n, max_slots, max_systems=nsys, mixed=(mode == "mixed"),
                       split_n=split_n)
        for s in range(nsys):
            for q in range(per):
                bt.add(s * per + q, loaded[s], gammas[s], starts[s][q])
        bt.step(2)
        c0 = bt.counts()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        bt.step(steps)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        c1 = bt.counts()
        d = (c1 - c0).astype(np.int64)
        evals = int(d[:, 0].sum())
        solves = int(d[:, 1].sum())
        fl = 0.0
        for s in range(nsys):
            ev = d[s * per:(s + 1) * per, 0].sum()
            so = d[s * per:(s + 1) * per, 1].sum()
            if mode == "plain":
                f = fl_plain[s]
                fl += ev * (f["eval_monomials"] + f["eval_sums"]) + so * f["mgs"]
            else:
                f = fl_mixed[s]
                fl += ev * f["residual"] + so * (f["jacobian"] + f["mgs"] + f["update"])
        res[mode] = {"ms": ms, "evaluations": evals, "solves": solves,
                     "newton_steps_per_s": solves / (ms / 1e3),
                     "evaluations_per_s": evals / (ms / 1e3),
                     "tflops": fl / (ms / 1e3) / 1e12,
                     "pct_fp64_peak": 100.0 * fl / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                     "device_gb": bt.device_bytes() / 1e9}
        bt.free()
    for s in loaded:
        s.free()
    if steps_only:
        return res

    # finite-roots variant: paths to completion, and Newton to 1e-28
    progress("batch: finite-roots systems")
    planted = [S.with_finite_roots(ps, s) for s, ps in enumerate(systems)]
    ploaded = [hcn.System(ps) for ps in planted]
    pmax_slots = max(s.info().nslots for s in ploaded)
    res["paths_finite"] = {}
    sample = {"systems": planted, "gammas": gammas, "paths": []}
    for mode in ("plain", "mixed"):
        progress(f"batch: paths to completion, {mode}")
        bt = hcn.Batch(2, nsys * per, max_n, pmax_slots, max_systems=nsys, mixed=(mode == "mixed"),
                       split_n=split_n, predictor_order=PLANTED_ORDER)
        for s in range(nsys):
            for q in range(per):
                bt.add(s * per + q, ploaded[s], gammas[s], starts[s][q])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.run(chunk=16)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st, stp, ends = [], [], []
        for s in range(nsys):
            for q in range(per):
                xo, r = bt.result(s * per + q, systems[s].n)
                st.append(int(r["status"]))
                stp.append(int(r["steps"]))
                ends.append(int(r["end_status"]))
                if mode == "plain" and q == 0 and s % 8 == 0:
                    sample["paths"].append({"system": s, "x0": starts[s][q].cpu().numpy(),
                                            "x1": xo.cpu().numpy(), "status": int(r["status"]),
                                            "steps": int(r["steps"])})
        bt.free()
        ok = sum(1 for c in st if c == 0)
        res["paths_finite"][mode] = {
            "predictor_order": PLANTED_ORDER, "wall_s": wall, "paths_per_s": len(st) / wall, "ok": ok, "success_rate": ok / len(st),
            "status": status_hist(st), "steps_median": float(np.median(stp)),
            "ok_and_refined_to_1e-28": int(sum(1 for c, e in zip(st, ends) if c == 0 and e == 0))}
    progress("batch: Newton to 1e-28 from perturbed roots")
    rngp = S.rng_for(3, 4242)
    out = {}
    for mode in ("plain", "mixed"):
        total_ms, its, succ, dist, count = 0.0, [], 0, 0.0, 0
        for ps, sd in zip(planted, ploaded):
            x = np.zeros((per, ps.n, 2, 2))
            x[:, :, 0, 0] = 1.0
            x[:, :, :, 0] += 1e-6 * rngp.standard_normal((per, ps.n, 2))
            xd = torch.from_numpy(x).to(dev)
            kw = dict(max_iter=12 if mode == "plain" else 40, tol_res=1e-28, tol_dx=0.0,
                      max_eq_val=1e300, mixed=(mode == "mixed"))
            hcn.newton(sd, xd.clone(), **kw)  # warm-up
            torch.cuda.synchronize()
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record()
            status, iters, norms = hcn.newton(sd, xd, **kw)
            stop.record()
            torch.cuda.synchronize()
            total_ms += start.elapsed_time(stop)
            stt = status.cpu().numpy()
            its.extend(iters.cpu().numpy().tolist())
            succ += int((stt == 0).sum())
            xh = xd.cpu().numpy()
            one = np.zeros_like(xh)
            one[:, :, 0, 0] = 1.0
            if (stt == 0).any():
                dist = max(dist, limb_diff_max(xh[stt == 0], one[stt == 0]))
            count += per
        out[mode] = {"points": count, "ms_total": total_ms, "converged": succ,
                     "iterations_mean": float(np.mean(its)), "iterations_max": int(np.max(its)),
                     "max_distance_to_root": dist}
    out["time_ratio_plain_over_mixed"] = out["plain"]["ms_total"] / max(out["mixed"]["ms_total"], 1e-9)
    res["newton_1e28"] = out
    for s in ploaded:
        s.free()
    res["sample"] = sample
    return res


def serve_leg(hcn, S, dev, pool: int = 64, burst: int = 128, per_rate: int = 96,
              rates=(0.5, 0.8, 0.95), serial_sample: int = 12, literal_burst: int = 64,
              literal_max_steps: int = 400) -> dict:
    """Continuous batching of track_path requests.  Systems are drawn like the
    batch systems with n log-uniform in [8, 128]; each request picks one of
    `pool` systems, DD (p = 0.8) or QD, a random total-degree start solution
    and gamma.  Served systems are the finite-roots variants (per equation a
    pure power x_i^{d_i} and a constant making x = 1 a root), so every path
    ends at a finite root (tracked with the predictor of degree 4):
    capacity from a burst of simultaneous requests (the completion rate
    while the server is full: requests done by the time 80 % are done, over
    that time; the slowest few paths, QD with n near 128, would otherwise
    set it alone), then Poisson arrivals at 0.5, 0.8 and 0.95 times that
    capacity (p50/p99 of arrival to result, queueing and service apart), and
    the same server admitting one path at a time on the first requests of the
    0.8 trace, with their arrival times.  The literal systems (no constant
    term; paths run to x = 0 or infinity) are served once as a burst with a
    budget of 400 steps per request."""
    import numpy as np
    lit_dd = S.batch_systems(pool, seed=5, P=2, n_range=(8, 128), log_uniform_n=True)
    lit_qd = S.batch_systems(pool, seed=5, P=4, n_range=(8, 128), log_uniform_n=True)
    pl_dd = [S.with_finite_roots(ps, 100 + s) for s, ps in enumerate(lit_dd)]
    pl_qd = [S.with_finite_roots(ps, 100 + s) for s, ps in enumerate(lit_qd)]
    sets = {"finite": {2: pl_dd, 4: pl_qd}, "literal": {2: lit_dd, 4: lit_qd}}
    loaded = {k: {P: [hcn.System(ps) for ps in v[P]] for P in (2, 4)} for k, v in sets.items()}
    max_n = max(ps.n for ps in lit_dd)
    max_slots = max(s.info().nslots for k in loaded for s in loaded[k][4])
    rng = np.random.Generator(np.random.PCG64(4000))

    def make_requests(count):
        reqs = []
        for _ in range(count):
            si = int(rng.integers(0, pool))
            P = 4 if rng.random() < 0.2 else 2
            ps = lit_dd[si] if P == 2 else lit_qd[si]
            x0 = S.start_solution(rng, S.degrees(ps), P)
            gam = S.random_unit_gamma(rng, P)
            reqs.append((P, si, gam, x0))
        return reqs

    def run(kind, reqs, arrivals, serial=False, max_steps=1500):
        order = PLANTED_ORDER if kind == "finite" else 1
        srv = hcn.Server(int(8e9), max_n=max_n, max_nslots=max_slots, qd_share=0.2,
                         steps_per_round=8, serial=serial, max_steps=max_steps,
                         predictor_order=order)
        t0 = srv.now()
        last = [t0]
        nxt = 0
        got = {}
        while len(got) < len(reqs):
            now = srv.now() - t0
            while nxt < len(reqs) and arrivals[nxt] <= now:
                P, si, gam, x0 = reqs[nxt]
                srv.submit(nxt, loaded[kind][P][si], gam, x0, t0 + arrivals[nxt])
                nxt += 1
            srv.pump()
            while True:
                r = srv.fetch()
                if r is None:
                    break
                got[r[0]] = r
            if srv.now() - last[0] > 5.0:
                last[0] = srv.now()
                progress(f"serving: {len(got)}/{len(reqs)} done, {nxt} submitted")
        wall = srv.now() - t0
        cap = srv.capacity()
        srv.free()
        lat = np.array([got[i][5] - got[i][3] for i in range(len(reqs))])
        queue = np.array([got[i][4] - got[i][3] for i in range(len(reqs))])
        serv = np.array([got[i][5] - got[i][4] for i in range(len(reqs))])
        pct = lambda a, q: 1e3 * float(np.percentile(a, q))
        codes = [int(got[i][2]["status"]) for i in range(len(reqs))]
        ok = sum(1 for c in codes if c == 0)
        done_t = np.sort(np.array([got[i][5] for i in range(len(reqs))]) - t0)
        k80 = max(1, int(0.8 * len(reqs)))
        out = {"requests": len(reqs), "predictor_order": order, "wall_s": wall,
               "paths_per_s": len(reqs) / wall,
               "paths_per_s_to_80pct": k80 / max(float(done_t[k80 - 1]), 1e-9),
               "completed_ok": ok, "completion_rate": ok / len(reqs),
               "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
               "queue_p50_ms": pct(queue, 50), "queue_p99_ms": pct(queue, 99),
               "service_p50_ms": pct(serv, 50), "service_p99_ms": pct(serv, 99),
               "status": status_hist(codes), "slots": {"dd": cap[0], "qd": cap[1]}}
        return out, got

    res = {"pool_systems": pool, "systems": "finite-roots variants (pure powers and a constant term)"}
    progress("serving: systems loaded; burst")
    reqs = make_requests(burst)
    cap, _ = run("finite", reqs, np.zeros(burst))
    res["capacity_burst"] = cap
    trace08 = None
    sample = []
    for lam_f in rates:
        lam = lam_f * cap["paths_per_s_to_80pct"]
        rq = make_requests(per_rate)
        arr = np.cumsum(rng.exponential(1.0 / lam, size=per_rate))
        progress(f"serving: Poisson arrivals at {lam:.1f}/s ({lam_f} x capacity)")
        r, got = run("finite", rq, arr)
        r["rate_per_s"] = lam
        res[f"poisson_{lam_f}"] = r
        if lam_f == 0.8:
            trace08 = (rq, arr)
            n_dd = n_qd = 0
            for i in range(len(rq)):
                P, si, gam, x0 = rq[i]
                if (P == 2 and n_dd < 8) or (P == 4 and n_qd < 4):
                    n_dd += P == 2
                    n_qd += P == 4
                    sample.append({"P": P, "system": si, "gamma": gam, "x0": x0, "x1": got[i][1],
                                   "status": int(got[i][2]["status"]), "steps": int(got[i][2]["steps"])})
    progress("serving: one at a time on the same trace")
    rq, arr = trace08
    base, _ = run("finite", rq[:serial_sample], arr[:serial_sample], serial=True)
    res["one_at_a_time"] = base
    progress("serving: literal systems, burst")
    lit, _ = run("literal", make_requests(literal_burst), np.zeros(literal_burst),
                 max_steps=literal_max_steps)
    lit["max_steps"] = literal_max_steps
    res["literal_burst"] = lit
    for k in loaded.values():
        for v in k.values():
            for q in v:
                q.free()
    res["sample"] = {"systems": {2: pl_dd, 4: pl_qd}, "paths": sample}
    return res


def cyclic_leg(hcn, flops, S, dev, cases=((128, 32), (352, 4)), reps: int = 5) -> dict:
    """Evaluation and differentiation (hcn_eval_jac) of the cyclic n-roots
    system in complex DD at B points, n = 128 and 352 (its monomials have
    every number of variables 1..n).  The first point is the closed-form
    root (the residual there is the error of f), the others random
    unit-modulus points."""
    import numpy as np
    import torch
    out = {}
    for n, B in cases:
        ps = S.cyclic_system(n, 2)
        sd = hcn.System(ps)
        info = sd.info()
        rngc = S.rng_for(7, n)
        rnd = S.unit_complex(rngc.uniform(0, 2 * np.pi, (B - 1) * n), 2).reshape(B - 1, n, 2, 2)
        pts = np.concatenate([S.cyclic_root(n, 2)[None], rnd], axis=0)
        x = torch.from_numpy(pts).to(dev)
        f, J = hcn.eval_jac(sd, x)
        torch.cuda.synchronize()
        hcn.profile_reset()
        hcn.profile_enable(True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            f, J = hcn.eval_jac(sd, x)
        stop.record()
        torch.cuda.synchronize()
        hcn.profile_enable(False)
        kern = {k: hcn.profile_query(k) for k in ("eval_monomials", "eval_sums")}
        hcn.profile_reset()
        ms = start.elapsed_time(stop) / reps
        fm = flops.eval_monomials(ps, 2)
        fs = flops.eval_sums(ps, 2)
        mon_ms = kern["eval_monomials"][0] / max(kern["eval_monomials"][1], 1)
        sum_ms = kern["eval_sums"][0] / max(kern["eval_sums"][1], 1)
        scratch = info.nslots * 32.0 * B
        fr = f[0].cpu().numpy()
        del f, J
        # residual at the root relative to the sum of the magnitudes of the
        # terms of each equation (n terms of modulus 1 in equations 1..n-1)
        rel = lead_abs_max(fr[:-1]) / n
        achieved = fm * B / (mon_ms / 1e3) / 1e12
        out[str(n)] = {"points": B, "monomials": info.nmon, "scratch_slots_per_point": info.nslots,
                       "eval_jac_ms": ms, "points_per_s": B / (ms / 1e3),
                       "eval_monomials_ms": mon_ms, "eval_sums_ms": sum_ms,
                       "tflops": (fm + fs) * B / (ms / 1e3) / 1e12,
                       "roofline": {"bound": "alu", "kernel": "eval_monomials", "achieved": achieved,
                                    "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": achieved / FP64_PEAK_TFLOPS},
                       "scratch_gb_written_per_launch": scratch / 1e9,
                       "scratch_write_gbs": scratch / (mon_ms / 1e3) / 1e9,
                       "residual_at_closed_form_root_rel": rel,
                       "last_equation_residual": lead_abs_max(fr[-1:])}
        sd.free()
        torch.cuda.empty_cache()
    return out


def double_leg(hcn, flops, S, dev, B: int = 10240, reps: int = 10) -> dict:
    """Complex double (the paper's third precision) on the dense n = 32
    system at B points: evaluation and differentiation with the reverse
    mode (one lane per monomial) against the tree mode (a group of lanes per
    monomial, Section 3.2), and the whole Newton step."""
    import torch
    ps = S.dense32_system(0, 1)
    pts = S.dense32_points(0, B, 1)
    sd = hcn.System(ps)
    x0 = torch.from_numpy(pts).to(dev)
    out = {"points": B}
    fm, fs = flops.eval_monomials(ps, 1), flops.eval_sums(ps, 1)
    for mode in ("reverse", "tree"):
        hcn.set_mon_tree(mode == "tree")
        try:
            hcn.eval_jac(sd, x0)
            torch.cuda.synchronize()
            hcn.profile_reset()
            hcn.profile_enable(True)
            start = torch.cuda.Event(enable_timing=True)
            stop = torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                hcn.eval_jac(sd, x0)
            stop.record()
            torch.cuda.synchronize()
            hcn.profile_enable(False)
            mon_ms, cnt = hcn.profile_query("eval_monomials")
            hcn.profile_reset()
        finally:
            hcn.set_mon_tree(False)
        ms = start.elapsed_time(stop) / reps
        mon_ms /= max(cnt, 1)
        out[mode] = {"eval_jac_ms": ms, "eval_monomials_ms": mon_ms,
                     "monomials_tflops": fm * B / (mon_ms / 1e3) / 1e12,
                     "eval_tflops": (fm + fs) * B / (ms / 1e3) / 1e12}
    x = torch.empty_like(x0)
    ws = hcn.newton_ws(sd, B)
    x.copy_(x0)
    hcn.newton_step(sd, x, ws=ws)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        x.copy_(x0)
        hcn.newton_step(sd, x, ws=ws)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    fl = flops.newton_step(ps, 1)["total"]
    out["newton_step"] = {"ms": ms, "steps_per_s": B / (ms / 1e3),
                          "pct_fp64_peak": 100.0 * fl * B / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS}
    sd.free()
    return out


def run_gpu(steps: int, warmup: int, qd_steps: int, legs, sparse_variants=None,
            batch_steps_only: bool = False) -> dict:
    import torch
    from paper_1501_06625_amd import flops, hcn, systems as S

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    out = {}
    if "dd" in legs:
        progress("dense n=32 DD leg")
        out["dd"] = dense_leg(hcn, flops, S, dev, 2, B_DD, steps, warmup, profile=True, keep=8)
    if "qd" in legs:
        progress("dense n=32 QD leg")
        out["qd"] = dense_leg(hcn, flops, S, dev, 4, B_QD, qd_steps, 1, profile=False, keep=4)
    if "single" in legs:
        progress("single-path leg")
        out["single"] = dense_leg(hcn, flops, S, dev, 2, 1, 200, 5, profile=False, keep=1)
    def show(key):
        leg = {k: v for k, v in out[key].items() if k != "sample"}
        progress(f"{key}: " + json.dumps(leg, default=str)[:3000])

    if "track8" in legs:
        progress("single-path tracking leg (n = 8)")
        out["track8"] = track8_leg(hcn, S, dev)
        show("track8")
    if "sparse512" in legs:
        progress("sparse n=512 leg")
        out["sparse512"] = sparse512_leg(hcn, flops, S, dev, variants=sparse_variants)
        show("sparse512")
    if "batch64" in legs:
        progress("64-system batch leg")
        out["batch64"] = batch_leg(hcn, flops, S, dev, steps_only=batch_steps_only)
        show("batch64")
    if "cyclic" in legs:
        progress("cyclic n-roots leg")
        out["cyclic"] = cyclic_leg(hcn, flops, S, dev)
        show("cyclic")
    if "double" in legs:
        progress("complex double leg")
        out["double"] = double_leg(hcn, flops, S, dev)
        show("double")
    if "serve" in legs:
        progress("serving leg")
        out["serve"] = serve_leg(hcn, S, dev)
        show("serve")
    progress("GPU legs done")
    return out


# ---------------------------------------------------------------------------
# CPU leg: the oracle timed on this host, and the errors of the GPU samples
# ---------------------------------------------------------------------------

def host_info() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    smt = None
    try:
        with open("/sys/devices/system/cpu/smt/active") as fh:
            smt = fh.read().strip() == "1"
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "smt_active": smt, "nproc": os.cpu_count(),
            "affinity_cpus": affinity, "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_threads(info: dict) -> int:
    """Threads the oracle may use: the CPUs this process may run on, or the
    host's stated share (OMP_NUM_THREADS) when it is smaller."""
    n = info["affinity_cpus"]
    share = info["omp_num_threads"]
    if share and share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return max(1, n)


def _mpc(ctx, z):
    re = ctx.mpf(0)
    im = ctx.mpf(0)
    for v in z[0]:
        re += ctx.mpf(float(v))
    for v in z[1]:
        im += ctx.mpf(float(v))
    return ctx.mpc(re, im)


def backward_error(J, f, x0, x1) -> float:
    """eta = ||J dx + f|| / (||J|| ||dx|| + ||f||) (infinity norms) at 320
    bits, with J [n][N][2][P] and f [N][2][P] the oracle's quad-double
    Jacobian and residual at x0, dx = x1 - x0 (exact from the limbs).  A
    context of its own (mpmath's global precision is shared by threads)."""
    import mpmath
    import numpy as np
    ctx = mpmath.MPContext()
    ctx.prec = 320
    n, N = J.shape[0], J.shape[1]
    dx = [_mpc(ctx, x1[k]) - _mpc(ctx, x0[k]) for k in range(n)]
    nz = np.argwhere(np.abs(J[:, :, :, 0]).sum(axis=2) > 0)
    r = [_mpc(ctx, f[i]) for i in range(N)]
    rowJ = [ctx.mpf(0)] * N
    for k, i in nz:
        jk = _mpc(ctx, J[k, i])
        r[i] += jk * dx[k]
        rowJ[i] += abs(jk)
    num = max(abs(v) for v in r)
    den = max(rowJ) * max(abs(v) for v in dx) + max(abs(_mpc(ctx, f[i])) for i in range(N))
    return float(num / den) if den else float(num)


def _widen(ps, P_to: int):
    from paper_1501_06625_amd import systems as S
    if ps.P >= P_to:
        return ps
    return ps.with_precision(P_to, S.convert_precision(ps.coef, ps.P, P_to))


def _to_p(a, P_to):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    out = np.zeros(a.shape[:-1] + (P_to,))
    out[..., :a.shape[-1]] = a
    return out


def newton_errors(O, ps, x0s, x1s, threads: int) -> dict:
    """For each sample point: the oracle's Newton step from x0 against the
    GPU's x1 (forward difference relative to max(1, |x|)), and the backward
    error of the GPU's update from the oracle's quad-double J and f."""
    ps4 = _widen(ps, 4)
    ref4 = O.SysRef(ps4)
    ref = O.SysRef(ps)

    def one(q):
        t0 = time.perf_counter()
        rc, xo, _ = O.newton_step(ref, None, None, 1, 1.0, x0s[q])
        ms = (time.perf_counter() - t0) * 1e3
        fwd = limb_diff_max(x1s[q], xo) / max(1.0, lead_abs_max(xo))
        f4, J4 = O.eval_jac(ref4, _to_p(x0s[q], 4))
        eta = backward_error(J4, f4, x0s[q], x1s[q])
        return rc, fwd, eta, ms

    with cf.ThreadPoolExecutor(max(1, min(threads, len(x0s)))) as ex:
        rs = list(ex.map(one, range(len(x0s))))
    return {"points": len(x0s), "oracle_rc": sorted(set(r[0] for r in rs)),
            "max_forward_diff_vs_oracle": max(r[1] for r in rs),
            "max_backward_error": max(r[2] for r in rs),
            "oracle_ms_per_step": sum(r[3] for r in rs) / len(rs)}


def sparse_errors(O, ps, x0, x1s: dict) -> dict:
    """One oracle Newton step (its MGS spreads the columns over the host's
    threads) against the result of every MGS variant."""
    ps4 = _widen(ps, 4)
    t0 = time.perf_counter()
    rc, xo, _ = O.newton_step(ps, None, None, 1, 1.0, x0)
    ms = (time.perf_counter() - t0) * 1e3
    f4, J4 = O.eval_jac(ps4, _to_p(x0, 4))
    out = {"oracle_rc": rc, "oracle_ms_per_step": ms}
    for name, x1 in x1s.items():
        out[name] = {"forward_diff_vs_oracle": limb_diff_max(x1, xo) / max(1.0, lead_abs_max(xo)),
                     "backward_error": backward_error(J4, f4, x0, x1)}
    return out


def track_errors(O, items, threads: int, **track_kw) -> dict:
    """Oracle tracking of the same paths (one thread per path, with the
    GPU's tracking parameters track_kw): status and step count against the
    GPU's, end points against each other, and the quad-double residual of
    the GPU end point."""
    import numpy as np

    def one(it):
        ps, gam, x0, x1 = it["ps"], it["gamma"], it["x0"], it["x1"]
        t0 = time.perf_counter()
        xo, r = O.track(ps, O.total_degree_start(ps), gam, 1, x0, **track_kw)
        ms = (time.perf_counter() - t0) * 1e3
        same = (r.status == it["status"] and r.steps == it["steps"])
        both_ok = r.status == 0 and it["status"] == 0
        d = limb_diff_max(x1, xo) / max(1.0, lead_abs_max(xo)) if both_ok else None
        res = None
        if it["status"] == 0:
            f4, _ = O.eval_jac(_widen(ps, 4), _to_p(x1, 4))
            res = lead_abs_max(f4)
        return same, d, res, ms, r.status

    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        rs = list(ex.map(one, items))
    ds = [r[1] for r in rs if r[1] is not None]
    res = [r[2] for r in rs if r[2] is not None]
    ms = np.array([r[3] for r in rs])
    return {"paths": len(items), "same_status_and_steps": int(sum(1 for r in rs if r[0])),
            "oracle_ok": int(sum(1 for r in rs if r[4] == 0)),
            "max_endpoint_diff_vs_oracle": max(ds) if ds else None,
            "max_qd_residual_of_gpu_endpoint": max(res) if res else None,
            "oracle_ms_per_path_median": float(np.median(ms)),
            "oracle_ms_per_path_p99": float(np.percentile(ms, 99)),
            "oracle_threads": threads}


def endpoint_errors(O, items, threads: int) -> dict:
    """End points of tracked paths too long for the oracle to track again
    (n up to 128, hundreds of steps): for each end point that the GPU reports
    converged, the oracle's quad-double residual there and the size of one
    oracle Newton step in quad-double from it (its distance to the root the
    path reached, to first order)."""
    def one(it):
        if it["status"] != 0:
            return None
        ps4 = _widen(it["ps"], 4)
        x4 = _to_p(it["x1"], 4)
        f4, _ = O.eval_jac(ps4, x4)
        rc, xn, nr = O.newton_step(ps4, None, None, 1, 1.0, x4)
        return lead_abs_max(f4), (float(nr[1]) if rc == 0 else float("inf"))

    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        rs = [r for r in ex.map(one, items) if r is not None]
    return {"paths": len(items), "converged_checked": len(rs),
            "max_qd_residual": max((r[0] for r in rs), default=None),
            "max_qd_newton_step": max((r[1] for r in rs), default=None)}


def time_newton_steps(O, ps, pts, threads: int, target_s: float) -> dict:
    """The oracle's Newton step on distinct points, one thread per core (the
    oracle is C called through ctypes, which releases the GIL)."""
    ref = O.SysRef(ps)
    t0 = time.perf_counter()
    O.newton_step(ref, None, None, 1, 1.0, pts[0])
    one = time.perf_counter() - t0
    per_thread = max(1, min(2000, int(target_s / max(one, 1e-6))))
    done = [0] * threads

    def work(c):
        for _ in range(per_thread):
            O.newton_step(ref, None, None, 1, 1.0, pts[c % len(pts)])
            done[c] += 1

    ths = [threading.Thread(target=work, args=(c,)) for c in range(threads)]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    wall = time.perf_counter() - t0
    return {"steps": sum(done), "per_thread": per_thread, "wall_s": wall,
            "steps_per_s": sum(done) / wall}


def cpu_baseline(gpu: dict, target_s: float = 15.0):
    """The CPU oracle leg.  The headline baseline: the oracle's complex-DD
    Newton step on the dense n = 32 system, one thread per core for about
    target_s seconds (and the same in QD, shorter).  Then the errors of the
    GPU legs' samples against the oracle, and the oracle's own time on them."""
    from oracle import oracle as O
    from paper_1501_06625_amd import systems as S

    info = host_info()
    threads = cpu_threads(info)
    progress(f"CPU oracle baseline on {threads} threads")
    dd = time_newton_steps(O, S.dense32_system(0, 2), S.dense32_points(7, threads, 2), threads, target_s)
    qd = time_newton_steps(O, S.dense32_system(0, 4), S.dense32_points(7, threads, 4), threads,
                           target_s / 3)
    base = {"value": dd["steps_per_s"], "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{dd['steps']} complex-DD Newton steps of the dense n=32 system "
                      f"({dd['per_thread']} per thread on {threads} threads), {dd['wall_s']:.1f} s wall",
            "host": info,
            "qd": {"value": qd["steps_per_s"], "unit": "steps/s", "cores": threads,
                   "sample": f"{qd['steps']} complex-QD Newton steps, {qd['wall_s']:.1f} s wall"}}
    errs = {}
    for key in ("dd", "qd", "single"):
        leg = gpu.get(key)
        if leg:
            progress(f"oracle errors: dense {key}")
            smp = leg["sample"]
            errs[key] = newton_errors(O, S.dense32_system(0, smp["P"]), smp["x0"], smp["x1"], threads)
    if gpu.get("track8"):
        progress("oracle errors: tracked n = 8 paths")
        items = [dict(s, ps=S.small_track_system(s["seed"], 2)) for s in gpu["track8"]["sample"]]
        errs["track8"] = track_errors(O, items, threads)
        if gpu["track8"].get("sample_finite"):
            progress("oracle errors: tracked n = 8 paths, finite-roots systems")
            items = [dict(q, ps=S.with_finite_roots(S.small_track_system(q["seed"], 2), q["seed"]))
                     for q in gpu["track8"]["sample_finite"][:32]]
            errs["track8_finite"] = track_errors(O, items, threads, predictor_order=PLANTED_ORDER)
    if gpu.get("sparse512"):
        progress("oracle errors: sparse n = 512")
        smp = gpu["sparse512"]["sample"]
        ps = S.sparse512_system(0, 2)
        errs["sparse512"] = sparse_errors(O, ps, smp["x0"], smp["x1"])
    if gpu.get("batch64") and "sample" in gpu["batch64"]:
        progress("oracle errors: batch paths")
        smp = gpu["batch64"]["sample"]
        items = [dict(p, ps=smp["systems"][p["system"]]) for p in smp["paths"]]
        errs["batch64"] = endpoint_errors(O, items, threads)
    if gpu.get("serve"):
        progress("oracle errors: served paths")
        smp = gpu["serve"]["sample"]
        items = [dict(p, ps=smp["systems"][p["P"]][p["system"]]) for p in smp["paths"]]
        errs["serve"] = endpoint_errors(O, items, threads)
    progress("CPU leg done")
    return base, errs


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--qd-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--mgs-group", type=int, default=None,
                    help="pin the MGS lane-group width (8/16/32) instead of autotuning")
    ap.add_argument("--mgs-storage", type=int, default=0,
                    help="with --mgs-group: [A | b] in global memory (0), LDS (1) or registers (2)")
    ap.add_argument("--legs", default="dd,qd,single,track8,sparse512,batch64,serve,cyclic,double",
                    help="comma list of dd (the reported line), qd, single, track8, sparse512, "
                         "batch64, serve, cyclic, double")
    ap.add_argument("--sparse512-variants", default=None,
                    help="comma list of MGS variants for the sparse512 leg (" +
                         ", ".join(r[2] for r in SPARSE_RUNS) + "); default all")
    ap.add_argument("--tune-reps", type=int, default=TUNE_REPS,
                    help="Newton steps the autotuner times per MGS configuration of the dense legs")
    ap.add_argument("--batch-steps-only", action="store_true",
                    help="batch64: only the fixed-step timing (no paths to completion; for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(paths are independent: a multi-GPU run would give each GPU its own share of them)",
              file=sys.stderr)
        return 2
    global MGS_PIN
    set_tune_reps(args.tune_reps)
    if args.mgs_group is not None:
        MGS_PIN = (args.mgs_group, args.mgs_storage)
    rank = int(os.environ.get("RANK", "0"))
    legs = tuple(args.legs.split(","))
    if "dd" not in legs:
        legs = ("dd",) + legs
    sv = tuple(args.sparse512_variants.split(",")) if args.sparse512_variants else None
    r = run_gpu(args.steps, args.warmup, args.qd_steps, legs, sv, args.batch_steps_only)
    cpu, errs = (None, {})
    if rank == 0 and not args.no_cpu:
        cpu, errs = cpu_baseline(r)
    dd = r["dd"]
    ms = dd["ms_per_step"]
    value = dd["B"] / (ms / 1e3)
    # dominant kernel by measured time
    kern = dd["kern"]
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_cnt = kern[dom]
    avg_ms = dom_ms / max(dom_cnt, 1)
    flops_launch = dd["flops"][dom] * dd["B"]
    achieved = flops_launch / (avg_ms / 1e3) / 1e12
    traffic = None
    tuned_cfg = tuple(dd["tuned"][:2]) if dd["tuned"] else (16, 0)
    digest = source_digest(dom)
    counters = HBM_COUNTERS_KIB.get(dom) if digest == COUNTERS_DIGEST.get(dom) else None
    if isinstance(counters, dict):
        counters = counters.get(tuned_cfg)
    if counters is not None and dd["B"] == B_DD:
        traffic = counters[0] * 1024 * FETCH_CAL + counters[1] * 1024 * WRITE_CAL
    total_tflops = dd["flops"]["total"] * dd["B"] / (ms / 1e3) / 1e12
    qd = r.get("qd")
    single = r.get("single")

    def strip(leg):
        if leg is None:
            return None
        return {k: v for k, v in leg.items() if not k.startswith("sample")}

    def with_err(leg, key):
        d = strip(leg)
        if d is not None and key in errs:
            d["oracle"] = errs[key]
        if d is not None and key == "track8" and "finite_roots" in d and "track8_finite" in errs:
            d["finite_roots"]["oracle"] = errs["track8_finite"]
        return d

    line = {
        "metric": "complex-DD Newton steps/s",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "dense n=32 random system (32 monomials/equation, 16 distinct "
                        "variables/monomial, exponents 1..3, unit-circle coefficients); one "
                        f"complex-DD Newton step (eval_jac + mgs_solve + update) at each of "
                        f"{dd['B']} distinct unit-modulus points per step",
            "precision": "complex double-double",
            "points_per_step": dd["B"],
            "seed": 1000,
            "mgs_variant": {"lane_group": dd["tuned"][0], "lds": dd["tuned"][1]} if dd["tuned"] else None,
        },
        "roofline": {
            "bound": "alu",
            "kernel": dom,
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch",
            "traffic_source_digest": digest,
            "avg_launch_ms": avg_ms,
            "flops_per_launch": flops_launch,
        },
        "cpu_baseline": cpu,
        "pct_fp64_peak": 100.0 * total_tflops / FP64_PEAK_TFLOPS,
        "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kern.items()},
        "algorithmic_mflop_per_newton_step": dd["flops"]["total"] / 1e6,
        "converged_or_ok_points": dd["ok"],
        "oracle_error": errs.get("dd"),
        "qd": None if qd is None else {
            "steps_per_s": qd["B"] / (qd["ms_per_step"] / 1e3), "points": qd["B"],
            "ms_per_step": qd["ms_per_step"],
            "pct_fp64_peak": 100.0 * qd["flops"]["total"] * qd["B"] /
            (qd["ms_per_step"] / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "oracle": errs.get("qd")},
        "single": None if single is None else {
            "us_per_newton_step": single["ms_per_step"] * 1e3, "oracle": errs.get("single")},
        "track8": with_err(r.get("track8"), "track8"),
        "sparse512": with_err(r.get("sparse512"), "sparse512"),
        "batch64": with_err(r.get("batch64"), "batch64"),
        "serve": with_err(r.get("serve"), "serve"),
        "cyclic": strip(r.get("cyclic")),
        "double": strip(r.get("double")),
    }
    if rank == 0:
        print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
