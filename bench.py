#!/usr/bin/env python3
"""Benchmark: complex double-double Newton steps per second.

Workload: the dense n = 32 random system (32 monomials per equation, each
a product of 16 distinct variables with exponents uniform in {1, 2, 3},
unit-circle coefficients) and B = 10240 distinct random unit-modulus
points.  One benchmark step applies one complete Newton step (evaluation
and differentiation by reverse mode, summation, modified Gram-Schmidt
solve, back substitution, update) to every point, starting each step from
the same points, so every step does the same work.  Inputs are resident in
device memory before the timed region.

Reported beside it: the same in quad-double (2048 points), the latency of
one Newton step of a single path, the roofline position of the dominant
kernel (algorithmic FP64 operations of one launch over its mean HIP-event
duration, against the FP64 vector peak) and the CPU oracle timed on this
host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
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
# HBM traffic per launch of the dense-DD kernels at 10240 points, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this leg (KiB per dispatch; the
# MGS per lane-group width and storage of [A | b], from the autotuner's
# launches), calibrated on the 10 MiB copy of the start points in the same
# runs (FETCH_SIZE reads 5131.5 KiB, WRITE_SIZE 10240 KiB for 10,485,760
# bytes); valid for the kernels as they are now (summary and commands:
# profiles/newton_step_dense32_dd_b10240.md)
HBM_COUNTERS_KIB = {
    "mgs": {(8, 0): (914308.5, 5363301.7), (8, 1): (274850.0, 205529.5), (8, 2): (274997.6, 206119.3),
            (8, 3): (437086.8, 542545.7), (16, 0): (876101.0, 4627639.1), (16, 1): (274880.8, 205993.9),
            (16, 2): (275024.4, 205809.6), (16, 3): (451486.8, 540727.1), (32, 0): (793216.0, 3988355.4),
            (32, 1): (274887.6, 207304.7), (32, 3): (479989.7, 537147.9)},
    "eval_monomials": (38055.1, 5570560.0), "eval_sums": (3648677.0, 393871.9)}
MGS_PIN = None  # (lane group, storage) from --mgs-group / --mgs-storage, else autotuned
FETCH_CAL, WRITE_CAL = 10485760 / (5131.5 * 1024), 1.0
_T0 = time.time()


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result alone goes to stdout)."""
    print(f"[bench {time.time() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


B_DD = 10240
B_QD = 2048


def cpu_baseline(target_s: float = 15.0) -> dict:
    """The oracle's Newton step (plain evaluation + MGS, own DD arithmetic)
    on distinct points of the same system, one thread per core (the oracle
    is C called through ctypes, which releases the GIL)."""
    from oracle import oracle as O
    from paper_1501_06625_amd import systems as S

    ps = S.dense32_system(0, 2)
    ref = O.SysRef(ps)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    pts = S.dense32_points(7, cores, 2)
    t0 = time.perf_counter()
    O.newton_step(ref, None, None, 1, 1.0, pts[0])
    one = time.perf_counter() - t0
    per_thread = max(1, int(target_s / max(one, 1e-6) / 1.0))
    per_thread = min(per_thread, 2000)
    done = [0] * cores

    def work(c):
        for _ in range(per_thread):
            O.newton_step(ref, None, None, 1, 1.0, pts[c])
            done[c] += 1

    threads = [threading.Thread(target=work, args=(c,)) for c in range(cores)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    wall = time.perf_counter() - t0
    total = sum(done)
    return {"value": total / wall, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{total} complex-DD Newton steps of the dense n=32 system "
                      f"({per_thread} per thread on {cores} threads), {wall:.1f} s wall"}


def run_gpu(steps: int, warmup: int, qd_steps: int, legs=("dd", "qd", "single"),
            sparse_variants=None) -> dict:
    import numpy as np
    import torch
    from paper_1501_06625_amd import flops, hcn, systems as S

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    out = {}

    def leg(P: int, B: int, K: int, W: int, profile: bool):
        ps = S.dense32_system(0, P)
        pts = S.dense32_points(0, B, P)
        sysd = hcn.System(ps)
        x0 = torch.from_numpy(pts).to(dev)
        x = torch.empty_like(x0)
        if B > 1 and MGS_PIN is not None:
            hcn.tune_set(P, ps.N, MGS_PIN[0], MGS_PIN[1])
            tuned = (MGS_PIN[0], MGS_PIN[1], None)
        else:
            tuned = hcn.autotune(sysd, x0, reps=5) if B > 1 else None
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
        sysd.free()
        return dict(ms_per_step=ev_ms / K, wall_s=wall, B=B, ok=ok, flops=fl, kern=kern, tuned=tuned)

    if "dd" in legs:
        progress("dense n=32 DD leg")
        out["dd"] = leg(2, B_DD, steps, warmup, profile=True)
    if "qd" in legs:
        progress("dense n=32 QD leg")
        out["qd"] = leg(4, B_QD, qd_steps, 1, profile=False)
    if "single" in legs:
        # single-path latency: one Newton step of one point, stream-ordered
        progress("single-path leg")
        out["single"] = leg(2, 1, 200, 5, profile=False)
    if "track8" in legs:
        progress("single-path tracking leg (n = 8)")
        out["track8"] = track8_leg(hcn, S, dev)
    if "sparse512" in legs:
        progress("sparse n=512 leg")
        out["sparse512"] = sparse512_leg(hcn, flops, S, dev, variants=sparse_variants)
    if "batch64" in legs:
        progress("64-system batch leg")
        out["batch64"] = batch_leg(hcn, flops, S, dev)
    if "serve" in legs:
        progress("serving leg")
        out["serve"] = serve_leg(hcn, S, dev)
    progress("done")
    return out


def serve_leg(hcn, S, dev, pool: int = 32, burst: int = 384, poisson: int = 384,
              serial_sample: int = 12, max_steps: int = 400) -> dict:
    """Continuous batching of track_path requests: systems drawn like the
    batch systems but with n log-uniform in [8, 128]; each request picks a
    system, DD (p = 0.8) or QD, a random total-degree start solution and
    gamma.  Capacity: a burst of requests all arriving at once (paths/s).
    Latency: Poisson arrivals at 0.8 x that capacity (p50/p99 of arrival to
    result, queueing included).  Baseline: the same server admitting one
    path at a time, on a sample.  Paths stop after max_steps steps (a
    per-request budget: these random systems have no constant term, and
    their total-degree paths run to singular endpoints or to infinity,
    needing well over a thousand steps); the status histogram is reported."""
    import numpy as np
    dd_sys = S.batch_systems(pool, seed=5, P=2, n_range=(8, 128), log_uniform_n=True)
    qd_sys = S.batch_systems(pool, seed=5, P=4, n_range=(8, 128), log_uniform_n=True)
    loaded = {2: [hcn.System(ps) for ps in dd_sys], 4: [hcn.System(ps) for ps in qd_sys]}
    max_n = max(ps.n for ps in dd_sys)
    max_slots = max(s.info().nslots for s in loaded[4])
    rng = np.random.Generator(np.random.PCG64(4000))

    def make_requests(count):
        reqs = []
        for _ in range(count):
            si = int(rng.integers(0, pool))
            P = 4 if rng.random() < 0.2 else 2
            ps = (qd_sys if P == 4 else dd_sys)[si]
            x0 = S.start_solution(rng, S.degrees(ps), P)
            gam = S.random_unit_gamma(rng, P)
            reqs.append((P, si, gam, x0))
        return reqs

    def run(reqs, arrivals, serial=False):
        srv = hcn.Server(int(8e9), max_n=max_n, max_nslots=max_slots, qd_share=0.2,
                         steps_per_round=8, serial=serial, max_steps=max_steps)
        t0 = srv.now()
        last = [t0]
        nxt = 0
        got = {}
        while len(got) < len(reqs):
            now = srv.now() - t0
            while nxt < len(reqs) and arrivals[nxt] <= now:
                P, si, gam, x0 = reqs[nxt]
                srv.submit(nxt, loaded[P][si], gam, x0, t0 + arrivals[nxt])
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
        names = {0: "ok", 1: "not_converged", 2: "diverged", 3: "max_steps", 4: "step_too_small",
                 5: "nan", -4: "singular"}
        hist = {}
        for i in range(len(reqs)):
            key = names.get(int(got[i][2]["status"]), str(int(got[i][2]["status"])))
            hist[key] = hist.get(key, 0) + 1
        pct = lambda a, q: 1e3 * float(np.percentile(a, q))
        return {"requests": len(reqs), "wall_s": wall, "paths_per_s": len(reqs) / wall,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "queue_p50_ms": pct(queue, 50), "queue_p99_ms": pct(queue, 99),
                "service_p50_ms": pct(serv, 50), "service_p99_ms": pct(serv, 99),
                "status": hist, "slots": {"dd": cap[0], "qd": cap[1]}}

    progress("serving: systems loaded")
    reqs = make_requests(burst)
    progress("serving: burst")
    cap = run(reqs, np.zeros(burst))
    lam = 0.8 * cap["paths_per_s"]
    reqs2 = make_requests(poisson)
    arr = np.cumsum(rng.exponential(1.0 / lam, size=poisson))
    progress(f"serving: Poisson arrivals at {lam:.1f}/s")
    lat = run(reqs2, arr)
    lat["rate_per_s"] = lam
    progress("serving: one at a time")
    sample = reqs2[:serial_sample]
    base = run(sample, np.zeros(len(sample)), serial=True)
    for s in loaded.values():
        for q in s:
            q.free()
    return {"pool_systems": pool, "max_steps": max_steps, "capacity_burst": cap,
            "poisson_0.8": lat, "one_at_a_time": base}


def batch_leg(hcn, flops, S, dev, nsys: int = 64, per: int = 64, steps: int = 10,
              split_n: int = 0) -> dict:
    """64 random systems (n in [16, 96], 16..64 monomials per equation, 4..12
    variables per monomial, exponents 1..3), 64 total-degree start solutions
    each: 4096 paths in one slot-table batch, tracked in complex DD for a
    fixed number of predictor-corrector steps with the plain and with the
    mixed-precision corrector.  Counts residual evaluations and solves per
    path on the device; flops per path from its own system."""
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
        progress(f"batch: {mode}")
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
    return res


def track8_leg(hcn, S, dev, seeds: int = 8) -> dict:
    """One path at a time: random n = 8 systems (8 monomials per equation of
    3 distinct variables, exponents 1..2), each path tracked from x = 1 at
    t = 0 to t = 1 (secant predictor, at most 3 Newton iterations a step,
    end-point refinement) by the single-system tracker, by a one-slot batch
    replaying its captured step, and by a one-slot batch with one persistent
    workgroup; wall time per path from the host (the run ends with the
    result on the host)."""
    import numpy as np
    import torch
    modes = ("tracker", "batch_graph", "batch_persistent")
    per = {m: [] for m in modes}
    steps, ok = [], 0
    for seed in range(seeds):
        ps = S.small_track_system(seed, 2)
        sd = hcn.System(ps)
        gam = S.random_unit_gamma(S.rng_for(0, 100 + seed), 2)
        x0 = torch.from_numpy(S.ones_point(ps.n, 2)).to(dev)
        for m in modes:
            for rep in range(2):  # the first run of each mode warms up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if m == "tracker":
                    _, r = hcn.track_paths(sd, gam, x0[None])
                    r = r[0]
                else:
                    bt = hcn.Batch(2, 1, ps.n, sd.info().nslots, persistent=(m == "batch_persistent"))
                    bt.add(0, sd, gam, x0)
                    bt.run(chunk=32)
                    _, r = bt.result(0, ps.n)
                    bt.free()
                dt = time.perf_counter() - t0
            per[m].append((dt, int(r["steps"])))
        steps.append(int(r["steps"]))
        ok += int(r["status"] == 0)
        sd.free()
    res = {"paths": seeds, "ok": ok, "steps": steps}
    for m in modes:
        res[m] = {"ms_per_path_median": float(np.median([d for d, _ in per[m]]) * 1e3),
                  "us_per_step": float(sum(d for d, _ in per[m]) / max(sum(k for _, k in per[m]), 1) * 1e6)}
    return res


def sparse512_leg(hcn, flops, S, dev, reps: int = 10, variants=None) -> dict:
    """Sparse n = 512 system (4 monomials of 2 variables + a constant per
    equation): one Newton step of one point, timed per MGS variant (all, or
    the names in variants).  The solve dominates (17.2 GFLOP of MGS against
    1 MFLOP of evaluation)."""
    import torch
    ps = S.sparse512_system(0, 2)
    pts = S.random_unit_point(S.rng_for(2, 99), ps.n, 2)[None]
    sysd = hcn.System(ps)
    x0 = torch.from_numpy(pts).to(dev)
    x = torch.empty_like(x0)
    ws = hcn.newton_ws(sysd, 1)
    mgs_flops = flops.mgs_solve(ps.N, ps.n, 2)
    res = {}
    runs = [(1, 16, "workgroup"), (2, 16, "right_looking"), (3, 16, "column_resident"),
            (4, 16, "tiled_T16"), (4, 8, "tiled_T8"), (4, 4, "tiled_T4")]
    for v, T, name in runs:
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
        res[name] = {"newton_step_ms": step_ms, "mgs_ms": mgs_ms,
                     "mgs_tflops": mgs_flops / (mgs_ms / 1e3) / 1e12}
    hcn.set_mgs_variant(0)
    hcn.set_mgs_panel(16)
    sysd.free()
    res["mgs_gflop"] = mgs_flops / 1e9
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--qd-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--mgs-group", type=int, default=None,
                    help="pin the MGS lane-group width (8/16/32) instead of autotuning")
    ap.add_argument("--mgs-storage", type=int, default=0,
                    help="with --mgs-group: [A | b] in global memory (0), LDS (1) or registers (2)")
    ap.add_argument("--legs", default="dd,qd,single,track8,sparse512,batch64,serve",
                    help="comma list of dd (the reported line), qd, single, track8, sparse512, batch64, serve")
    ap.add_argument("--sparse512-variants", default=None,
                    help="comma list of MGS variants for the sparse512 leg (workgroup, right_looking, "
                         "column_resident, tiled_T16, tiled_T8, tiled_T4); default all")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(paths are independent: a multi-GPU run would give each GPU its own share of them)",
              file=sys.stderr)
        return 2
    global MGS_PIN
    if args.mgs_group is not None:
        MGS_PIN = (args.mgs_group, args.mgs_storage)
    rank = int(os.environ.get("RANK", "0"))
    cpu = None
    if rank == 0 and not args.no_cpu:
        # before the GPU is touched
        progress("CPU oracle baseline")
        cpu = cpu_baseline()
    legs = tuple(args.legs.split(","))
    if "dd" not in legs:
        legs = ("dd",) + legs
    sv = tuple(args.sparse512_variants.split(",")) if args.sparse512_variants else None
    r = run_gpu(args.steps, args.warmup, args.qd_steps, legs, sv)
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
    counters = HBM_COUNTERS_KIB.get(dom)
    if isinstance(counters, dict):
        counters = counters.get(tuned_cfg)
    if counters is not None and dd["B"] == 10240:
        traffic = counters[0] * 1024 * FETCH_CAL + counters[1] * 1024 * WRITE_CAL
    total_tflops = dd["flops"]["total"] * dd["B"] / (ms / 1e3) / 1e12
    qd = r.get("qd")
    single = r.get("single")
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
            "avg_launch_ms": avg_ms,
            "flops_per_launch": flops_launch,
        },
        "cpu_baseline": cpu,
        "pct_fp64_peak": 100.0 * total_tflops / FP64_PEAK_TFLOPS,
        "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kern.items()},
        "algorithmic_mflop_per_newton_step": dd["flops"]["total"] / 1e6,
        "converged_or_ok_points": dd["ok"],
        "qd": None if qd is None else {
            "steps_per_s": qd["B"] / (qd["ms_per_step"] / 1e3), "points": qd["B"],
            "ms_per_step": qd["ms_per_step"],
            "pct_fp64_peak": 100.0 * qd["flops"]["total"] * qd["B"] /
            (qd["ms_per_step"] / 1e3) / 1e12 / FP64_PEAK_TFLOPS},
        "single_path_us_per_newton_step": None if single is None else single["ms_per_step"] * 1e3,
        "track8": r.get("track8"),
        "sparse512": r.get("sparse512"),
        "batch64": r.get("batch64"),
        "serve": r.get("serve"),
    }
    if rank == 0:
        print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
