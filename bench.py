#!/usr/bin/env python3
"""Benchmark: Mpoints/s per defmm matvec on one MI355X.

Workload (default): 1,048,576 points uniform on the unit sphere (D = 2),
kappa*D = 256, L = 5, leaves <= 64 points, complex N(0,1) charges, at the
cheapest knob setting (eta, c_HF, E0) measured within 1e-4 of the FP64 direct
sum; the complex64 path is timed (value), the complex128 path beside it, and
the paper-literal setting (eta = 1, c_HF = 2, E0 = 0) after them.  A step is
one matvec (P2M .. P2P, L2P, scatter) with fresh charges already resident in
HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoints/s per FMM matvec at rel.err<=1e-4 (FP32 vs FP64 path); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
HBM_PASSES = {"setup", "p2m", "m2m", "m2f", "m2l", "f2l", "l2l", "p2p_reduce", "l2p", "scatter"}
MFMA_PASSES = {"m2l_dense"}
KERNEL_OF_PASS = {"m2l": "k_m2l_runs", "f2l": "k_f2l", "p2p": "k_p2p", "m2f": "k_m2f", "m2m": "k_m2m",
                  "l2l": "k_l2l", "p2m": "k_p2m", "l2p": "k_l2p", "m2l_dense": "k_m2l_dense"}
# the kernels of the pencil upward/downward passes (one thread per pencil of
# interpolation values, P2M once per leaf)
PENCIL_KERNEL_OF_PASS = {"m2m": "k_m2m_p", "l2l": "k_l2l_p", "p2m": "k_p2m_leaf"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere1m")
    ap.add_argument("--eta", type=float, default=None)
    ap.add_argument("--hf", type=float, default=None)
    ap.add_argument("--e0", type=int, default=None)
    ap.add_argument("--c128-steps", type=int, default=5)
    ap.add_argument("--check-targets", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accurate", action="store_true",
                    help="skip the second complex64 run at the paper-literal knobs")
    ap.add_argument("--cpu-sample", type=int, default=0, help="points in the oracle's sample (0: auto)")
    ap.add_argument("--cpu-single", type=int, default=4096,
                    help="points in the oracle's one-thread sample (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--c64-only", action="store_true", help="skip the complex128 path and the checks")
    ap.add_argument("--check", action="store_true",
                    help="with --c64-only: also the error against the FP64 direct sum on sampled targets")
    ap.add_argument("--force", default="",
                    help="with --c64-only: tuning fields set after the autotuner, e.g. m2l_variant=3,fourier_items=4")
    ap.add_argument("--compress", action="store_true",
                    help="one spectrum per symmetry class of offsets (DEFMM_COMPRESS_SPECTRA)")
    ap.add_argument("--serving", action="store_true",
                    help="serving configuration: Poisson-arriving requests with continuous batching")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--geometries", type=int, default=32)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of one-stream capacity")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--solves", type=int, default=32,
                    help="serving: GMRES solve requests run after the matvec requests (0: none)")
    ap.add_argument("--literal", action="store_true",
                    help="serving: paper-literal knobs instead of the per-order setting within 1e-4")
    ap.add_argument("--error-sample", type=int, default=8,
                    help="serving: requests whose first matvec is checked against the FP64 direct sum")
    return ap.parse_args()


# Knob settings (eta = MAC constant, hf_threshold = c_HF, dir_refine = E0).
PAPER_LITERAL = (1.0, 2.0, 0)
# Per workload, the cheapest setting found by a sweep on the device whose
# complex64 potentials are within 1e-4 of the FP64 direct sum: the headline is
# timed there.  None: no setting that fits one GPU reaches it, and the
# paper-literal setting is timed instead (the error is reported either way).
ACCURATE = {"sphere1m": (0.35, 0.75, 1), "ellipsoid2m": (0.35, 0.75, 1), "sphere1m_yukawa": (1.0, 2.0, 0),
            "sphere8k": (0.15, 0.75, 1), "cube8m": None}


def direct_sum_sampled(X, q, kappa, tau, targets, screened=False):
    """FP64 direct sum on sampled targets (torch on the device, chunked over sources),
    used only to report the method's error."""
    import torch
    Xt = torch.as_tensor(X, dtype=torch.float64, device="cuda")
    qt = torch.as_tensor(q, dtype=torch.complex128, device="cuda")
    xs = Xt[torch.as_tensor(targets, device="cuda")]
    out = torch.zeros(len(targets), dtype=torch.complex128, device="cuda")
    chunk = 1 << 12
    for j in range(0, Xt.shape[0], chunk):
        y = Xt[j:j + chunk]
        r = torch.sqrt(((xs[:, None, :] - y[None, :, :]) ** 2).sum(-1))
        mask = r > tau
        rr = torch.where(mask, r, torch.ones_like(r))
        k = torch.exp(-kappa * rr) + 0j if screened else torch.exp(1j * kappa * rr)
        g = torch.where(mask, k / (4 * np.pi * rr), torch.zeros_like(rr, dtype=torch.complex128))
        out += g @ qt[j:j + chunk]
    return out.cpu().numpy()


def kernel_source_hash(kernel):
    """Hash of the kernels.hip section (between two section rules) that defines
    `kernel`: the counters taken for it stay valid while that section is unchanged."""
    with open(os.path.join(ROOT, "paper_2202_04894_amd", "csrc", "kernels.hip")) as fh:
        text = fh.read()
    rule = "// " + "-" * 66
    at = text.find(f" void {kernel}(")
    if at < 0:
        return None
    a = text.rfind(rule, 0, at)
    b = text.find(rule, at)
    sec = text[max(a, 0):b if b >= 0 else len(text)]
    return hashlib.sha256(sec.encode()).hexdigest()[:16]


def load_traffic(kernel, workload, knobs):
    """HBM bytes per launch of `kernel` on `workload` at `knobs` from the committed
    counter summary, or None when there is none or the kernel's source section
    has changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}*.json"))):
        with open(path) as fh:
            t = json.load(fh)
        if t.get("workload") != workload or [float(v) for v in t.get("knobs", [])] != [float(v) for v in knobs]:
            continue
        if t.get("kernel_source_sha256_16") != kernel_source_hash(kernel):
            return None
        return t.get("bytes_per_launch")
    return None


def time_matvecs(ws, charges, steps, warmup, timing):
    import torch
    p = None
    for k in range(warmup):
        p = ws.matvec(charges[k % len(charges)], p)
    torch.cuda.synchronize()
    ws.set_timing(timing)
    if timing:
        ws.pass_times()  # reset
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        p = ws.matvec(charges[(warmup + k) % len(charges)], p)
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    passes = ws.pass_times() if timing else None
    ws.set_timing(False)
    return (t1 - t0) * 1e3 / steps, lat, passes


def _omp():
    import ctypes
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, X, kappa, knobs, perm, n_sample, n_single):
    """The FP64 oracle on bounded samples of the same workload: the first n_sample
    points in Morton order (a contiguous patch of the same surface at full
    density), same kappa/L/ncrit/knobs, on every host thread; then the first
    n_single points on one thread (a per-core figure).  The whole input at these
    knobs would take the oracle tens of minutes per matvec."""
    import oracle
    eta, hf, e0 = knobs
    kern = oracle.YUKAWA if wl.kernel == "yukawa" else oracle.HELMHOLTZ
    q_all = wl.charges(0)

    def run(n):
        idx = np.sort(perm[:n])
        F = oracle.FMM(X[idx], None, kappa, oracle.Params(L=wl.L, ncrit=wl.ncrit, eta=eta, hf_threshold=hf,
                                                          dir_refine=e0, kernel=kern))
        F.apply(q_all[idx])
        return F.last_seconds

    omp = _omp()
    threads = int(omp.omp_get_max_threads()) if omp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    secs = run(n_sample)
    single = None
    if omp and n_single:
        omp.omp_set_num_threads(1)
        try:
            s1 = run(n_single)
        finally:
            omp.omp_set_num_threads(threads)
        single = {"value": round(n_single / s1 / 1e6, 6), "unit": "Mpoints/s", "cores": 1,
                  "sample": f"first {n_single} points in Morton order, one FP64 matvec took {s1:.2f} s"}
    return {"value": round(n_sample / secs / 1e6, 6), "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": f"first {n_sample} of {wl.n} points in Morton order (a patch of the {wl.geometry} at "
                      f"full density), {wl.kernel} kernel, kappa*D={wl.kappa_d}, L={wl.L}, ncrit={wl.ncrit}, "
                      f"eta={eta}, c_HF={hf}, E0={e0}; one FP64 matvec (setup excluded) took {secs:.2f} s",
            "single_thread": single}


def run_serving(args):
    """Serving configuration: requests with N log-uniform in [1e4, 5e5] on
    spheres and cap-weighted ellipsoids (from a pool of geometries), kappa*D
    uniform in [16, 256], L in {4, 5}, leaves <= 64, 20 matvecs each with fresh
    complex64 charges drawn on the device from a per-request seed.

    Three runs over the same requests, each starting with an empty plan cache:
      * all requests queued at once, `slots` admitted at a time (continuous
        batching at full load): the capacity, requests/s (`value`);
      * the same, one request at a time: the one-stream capacity;
      * Poisson arrivals at `load` times the one-stream capacity: latencies.
    Then a sample of requests is run in a mix and alone: same bits."""
    import torch
    from paper_2202_04894_amd import serving as S
    from paper_2202_04894_amd import workloads as W
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)

    def requests(rate=None):
        return S.config_requests(n_requests=args.requests, n_geometries=args.geometries, seed=7, rate=rate,
                                 accurate=not args.literal)

    ex = S.DeviceExecutor()
    S.Scheduler(ex, budget, max_slots=2).run(requests()[:4])  # warm-up: kernels, allocator

    def run(reqs, slots):
        sch = S.Scheduler(ex, budget, max_slots=slots)
        t0 = time.perf_counter()
        out = sch.run(reqs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pts = sum(r.n_points * r.n_matvecs for r, o in zip(reqs, out) if o.ok)
        return dict(S.summarize(out, wall), Mpoints_per_s=round(pts / wall / 1e6, 3),
                    requests_per_s=round(sum(o.ok for o in out) / wall, 3), scheduler=sch.stats)

    def note(what, r):
        print(f"[serving] {what}: {r['requests_per_s']} requests/s over {r['wall_s']} s", file=sys.stderr, flush=True)

    full = run(requests(), args.slots)
    note("full load", full)
    one = run(requests(), 1)
    note("one at a time", one)
    rate = args.load * one["requests_per_s"]
    open_loop = run(requests(rate), args.slots)
    note("open loop", open_loop)
    # the same requests alone give the same bits (sampled)
    rng = np.random.default_rng(3)
    sample = sorted(rng.choice(args.requests, size=min(4, args.requests), replace=False).tolist())
    sub = [requests()[i] for i in sample]
    for r in sub:
        r.n_matvecs = 2
    exk = S.DeviceExecutor(keep_results=True)
    mix = S.Scheduler(exk, budget, max_slots=len(sub), keep_results=True).run(sub)
    same = True
    for r, m in zip(sub, mix):
        alone = S.Scheduler(exk, budget, max_slots=1, keep_results=True).run([r])[0]
        same = same and m.ok and alone.ok and all(np.array_equal(a, b) for a, b in zip(alone.results, m.results))
    # method error per request: the first matvec of a sample of requests against
    # the FP64 direct sum on 256 sampled targets (charges regenerated from the
    # request's seed, as the executor drew them)
    errors = []
    if args.error_sample:
        esample = sorted(rng.choice(args.requests, size=min(args.error_sample, args.requests),
                                    replace=False).tolist())
        esub = [requests()[i] for i in esample]
        for r in esub:
            r.n_matvecs = 1
        out_e = S.Scheduler(exk, budget, max_slots=args.slots, keep_results=True).run(esub)
        for r, o in zip(esub, out_e):
            if not o.ok:
                continue
            g = torch.Generator(device="cuda")
            g.manual_seed(1_000_003 * (r.rid + 1))
            q0 = torch.randn(r.n_points, dtype=torch.complex64, device="cuda", generator=g)
            X = np.ascontiguousarray(r.make_points(), dtype=np.float64)
            D = float((X.max(0) - X.min(0)).max())
            tg = W.sample_targets(r.n_points, 256, 3000 + r.rid)
            pd = direct_sum_sampled(X, q0.cpu().numpy().astype(np.complex128), r.kappa, 1e-12 * D, tg)
            p0 = o.results[0].astype(np.complex128)
            errors.append({"rid": r.rid, "n": r.n_points, "kappa_d": round(2 * r.kappa, 2), "L": r.order_L,
                           "rel_l2_vs_direct": float(np.linalg.norm(p0[tg] - pd) / np.linalg.norm(pd))})
    solves = None
    if args.solves:
        sreqs = S.solve_requests(n_requests=args.solves, n_geometries=args.geometries, seed=7,
                                 accurate=not args.literal)
        sch = S.Scheduler(ex, budget, max_slots=args.slots)
        t0 = time.perf_counter()
        out_s = sch.run(sreqs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(f"[serving] {len(out_s)} solves in {wall:.1f} s", file=sys.stderr, flush=True)
        ok = [o for o in out_s if o.ok]
        lat = np.array([o.latency for o in ok]) if ok else np.zeros(1)
        solves = {"solves": len(out_s), "completed": len(ok), "converged": sum(o.info.get("converged", False) for o in ok),
                  "solves_per_s": round(len(ok) / wall, 3), "wall_s": round(wall, 3),
                  "solve_p50_s": round(float(np.percentile(lat, 50)), 4),
                  "solve_p99_s": round(float(np.percentile(lat, 99)), 4),
                  "iterations_mean": round(float(np.mean([o.info["iterations"] for o in ok])), 2) if ok else None,
                  "matvecs_total": int(sum(o.info["matvecs"] for o in ok)),
                  "max_residual": max((o.info["residual"] for o in ok), default=None),
                  "system": "GMRES(30) on 0.5 x + G (w x) = b, equal-area weights w, complex N(0,1) b, tol 1e-4, "
                            "complex64, on the serving geometries",
                  "scheduler": sch.stats}
    line = {"metric": "serving: requests/s under continuous batching (full load); p50/p99 latency at "
                      f"{args.load:.0%} load",
            "value": full["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": "c64", "data": "synthetic",
            "config": {"workload": f"{args.requests} requests, N log-uniform in [1e4, 5e5] on spheres / "
                                   f"cap-weighted ellipsoids from a pool of {args.geometries} geometries, "
                                   "kappa*D in [16, 256], L in {4, 5}, leaf<=64, 20 complex64 matvecs each",
                       "knobs_by_L": {str(k): {f"kappa*D < {S.HIGH_KD:g}": v,
                                               f"kappa*D >= {S.HIGH_KD:g}": S.ACCURATE_KNOBS_HIGH_KD[k]}
                                      for k, v in S.ACCURATE_KNOBS.items()} if not args.literal
                       else {"4": S.LITERAL_KNOBS, "5": S.LITERAL_KNOBS},
                       "slots": args.slots, "budget_GiB": round(budget / 2 ** 30, 1)},
            "full_load": full, "one_at_a_time": one,
            "batching_speedup": round(full["requests_per_s"] / one["requests_per_s"], 3),
            "open_loop": dict(open_loop, arrival_rate_per_s=round(rate, 3), load=args.load),
            "alone_equals_mix_bitwise": bool(same), "alone_vs_mix_sample": sample,
            "direct_sum_errors": errors, "solves": solves}
    print(json.dumps(line), flush=True)


def roofline_of(names, per_step, bytes_, flops, tuned, wl_name, knobs):
    """Roofline of the pass that takes the most time, from per-pass HIP events
    (average launch duration over the timed matvecs)."""
    dom = int(np.argmax(per_step))
    dname = names[dom]
    t_launch = per_step[dom] / 1e3
    kern = KERNEL_OF_PASS.get(dname, dname)
    if dname == "m2l" and tuned["m2l_variant"] == 1:
        kern = "k_m2l_slice"
    if tuned.get("updown_variant", 0) == 1 and dname in PENCIL_KERNEL_OF_PASS:
        kern = PENCIL_KERNEL_OF_PASS[dname]
    if dname in MFMA_PASSES:
        ach = flops[dom] / t_launch / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_PEAK_TFLOPS, 4)}
    elif dname in HBM_PASSES:
        ach = bytes_[dom] / t_launch / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = flops[dom] / t_launch / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_PEAK_TFLOPS, 4)}
    roof["kernel"] = kern
    roof["avg_launch_ms"] = round(t_launch * 1e3, 4)
    roof["timing"] = "per-pass HIP events, passes in sequence on one stream (near field not overlapped)"
    roof["traffic"] = load_traffic(kern, wl_name, knobs)
    roof["algorithmic_bytes_per_launch"] = float(bytes_[dom])
    roof["flops_per_launch"] = float(flops[dom])
    t_floor = max(bytes_[dom] / (HBM_PEAK_GBS * 1e9), flops[dom] / (FP32_PEAK_TFLOPS * 1e12))
    roof["t_floor_ms"] = round(t_floor * 1e3, 4)
    roof["t_over_t_floor"] = round(t_launch / t_floor, 2) if t_floor > 0 else None
    if dname == "m2l":
        # what the caches serve: both operands of every pair, s_c (2L-1)^3 bytes each
        roof["effective_GBps"] = round(flops[dom] * 8 / 4 / t_launch / 1e9, 1)
    return roof


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the sharding by target "
              f"across GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        run_serving(args)
        return
    import torch
    from paper_2202_04894_amd import defmm
    from paper_2202_04894_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = W.WORKLOADS[args.workload]
    accurate = ACCURATE.get(args.workload)
    eta, hf, e0 = accurate if accurate else PAPER_LITERAL
    if args.eta is not None:
        eta = args.eta
    if args.hf is not None:
        hf = args.hf
    if args.e0 is not None:
        e0 = args.e0
    knobs = (eta, hf, e0)
    X = wl.points()
    kflag = defmm.YUKAWA if wl.kernel == "yukawa" else 0
    if args.compress:
        kflag |= defmm.COMPRESS_SPECTRA
    nsteps = max(args.steps, 1)
    nq = min(nsteps + args.warmup, 64)

    def make(prec, kn):
        t0 = time.perf_counter()
        plan = defmm.Plan(X, None, wl.kappa, defmm.Params(order_L=wl.L, ncrit=wl.ncrit, eta=kn[0],
                                                            hf_threshold=kn[1], dir_refine=kn[2], precision=prec,
                                                            m2l_mode=defmm.M2L_AUTO, flags=kflag))
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        return plan, defmm.Workspace(plan), setup

    plan64, ws64, setup64 = make(defmm.C64, knobs)
    charges64 = [torch.as_tensor(wl.charges(k, np.complex64), device="cuda") for k in range(nq)]
    # execution choices (M2L variant, dense levels, near-field overlap) tuned on this workspace
    tuned = ws64.autotune(charges64[0], reps=3)
    if args.force:
        tuned.update({k: int(v) for k, v in (kv.split("=") for kv in args.force.split(","))})
        ws64.set_tuning(**tuned)
    # production mode: tuned choices, no per-pass events
    ms64, lat64, _ = time_matvecs(ws64, charges64, nsteps, args.warmup, timing=False)
    # the same matvecs in sequence with per-pass HIP events: each kernel's own duration
    ws64.set_overlap(False)
    ms_seq, _, passes = time_matvecs(ws64, charges64, nsteps, 1, timing=True)
    ws64.set_tuning(**tuned)
    p64 = ws64.matvec(charges64[0]).cpu().numpy().astype(np.complex128)
    del charges64
    names = [defmm.pass_name(i) for i in range(defmm.NUM_PASSES)]
    ms_pass, _ = passes
    per_step = ms_pass / nsteps

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.c64_only:
        line = {"value": round(wl.n / (ms64 / 1e3) / 1e6, 3), "ms_per_step": round(ms64, 4),
                "p99_ms": round(float(np.percentile(lat64, 99)), 4),
                "knobs": knobs, "compress": bool(args.compress), "sequential_ms_per_step": round(ms_seq, 4),
                "tuning": tuned, "setup_s": round(setup64, 3),
                "passes_ms_per_step": {n: round(float(v), 4) for n, v in zip(names, per_step)},
                "stats": {k: v for k, v in plan64.stats().items() if k != "m2l_mode_per_level"}}
        if args.check:
            D, _ = plan64.geometry()
            tg = W.sample_targets(wl.n, args.check_targets, 3000 + wl.seed)
            pd = direct_sum_sampled(X, wl.charges(0), wl.kappa, 1e-12 * D, tg, screened=bool(wl.kernel == "yukawa"))
            line["rel_l2_vs_direct_c64"] = float(np.linalg.norm(p64[tg] - pd) / np.linalg.norm(pd))
        print(json.dumps(line), flush=True)
        return

    st = plan64.stats()
    bytes_, flops = ws64.pass_work()
    roof = roofline_of(names, per_step, bytes_, flops, tuned, wl.name, knobs)
    p2p_i = names.index("p2p")
    t_p2p = per_step[p2p_i] / 1e3
    p2p = {"kernel": "k_p2p", "point_pairs": int(st["p2p_point_pairs"]), "ms": round(t_p2p * 1e3, 4),
           "Gpairs_per_s": round(st["p2p_point_pairs"] / t_p2p / 1e9, 2),
           "TFLOPs_nominal": round(flops[p2p_i] / t_p2p / 1e12, 3),
           "frac_fp32_vector_peak": round(flops[p2p_i] / t_p2p / 1e12 / FP32_PEAK_TFLOPS, 4)}
    perm = plan64.tree(0)["perm"]
    D, _ = plan64.geometry()
    del plan64, ws64
    torch.cuda.empty_cache()

    # the plain FP64 (complex128) GPU path at the same knobs
    plan128, ws128, setup128 = make(defmm.C128, knobs)
    charges128 = [torch.as_tensor(wl.charges(k), device="cuda") for k in range(min(nq, 8))]
    ws128.autotune(charges128[0], reps=2)
    ms128, lat128, _ = time_matvecs(ws128, charges128, max(args.c128_steps, 1), 2, timing=False)
    p128 = ws128.matvec(charges128[0]).cpu().numpy()
    del charges128, plan128, ws128
    torch.cuda.empty_cache()
    rel_prec = float(np.linalg.norm(p64 - p128) / np.linalg.norm(p128))

    tg = W.sample_targets(wl.n, args.check_targets, 3000 + wl.seed)
    pd = direct_sum_sampled(X, wl.charges(0), wl.kappa, 1e-12 * D, tg, screened=bool(kflag))
    rel_direct = float(np.linalg.norm(p128[tg] - pd) / np.linalg.norm(pd))
    rel_direct64 = float(np.linalg.norm(p64[tg] - pd) / np.linalg.norm(pd))
    setting = ("cheapest setting measured within 1e-4 of the FP64 direct sum" if accurate and knobs == accurate
               else "paper-literal setting" if knobs == PAPER_LITERAL else "setting given on the command line")

    out = {
        "metric": METRIC,
        "value": round(wl.n / (ms64 / 1e3) / 1e6, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n} points uniform on the unit {wl.geometry}, "
                               + (f"screened kernel exp(-kappa r)/(4 pi r), " if kflag else "")
                               + f"kappa*D={wl.kappa_d}, L={wl.L}, leaf<={wl.ncrit}, complex N(0,1) charges",
                   "eta": eta, "hf_threshold": hf, "dir_refine": e0, "setting": setting},
        "p50_ms": round(float(np.percentile(lat64, 50)), 4),
        "p99_ms": round(float(np.percentile(lat64, 99)), 4),
        "rel_l2_c64_vs_c128": rel_prec,
        "rel_l2_vs_direct_c128": rel_direct,
        "rel_l2_vs_direct_c64": rel_direct64,
        "direct_check": f"FP64 direct sum on {len(tg)} sampled targets",
        "c128": {"value": round(wl.n / (ms128 / 1e3) / 1e6, 3), "unit": "Mpoints/s",
                 "ms_per_step": round(ms128, 4), "p50_ms": round(float(np.percentile(lat128, 50)), 4),
                 "p99_ms": round(float(np.percentile(lat128, 99)), 4)},
        "setup_s": {"c64": round(setup64, 3), "c128": round(setup128, 3)},
        "sequential_ms_per_step": round(ms_seq, 4),
        "tuning": tuned,
        "passes_ms_per_step": {n: round(float(v), 4) for n, v in zip(names, per_step)},
        # per pass: compulsory bytes / time against the HBM peak, flops / time
        "passes_roofline": {n: {"GBps": round(b / (t / 1e3) / 1e9, 1),
                                "frac_hbm": round(b / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                "TFLOPs": round(f / (t / 1e3) / 1e12, 3)}
                            for n, t, b, f in zip(names, per_step, bytes_, flops) if t > 0.005},
        "stats": st,
        "roofline": roof,
        "p2p": p2p,
    }

    if not args.no_accurate and knobs != PAPER_LITERAL:
        # the same workload at the paper-literal knobs, complex64: throughput and error
        pl, wsl, setup_l = make(defmm.C64, PAPER_LITERAL)
        ql = [torch.as_tensor(wl.charges(k, np.complex64), device="cuda") for k in range(nq)]
        tuned_l = wsl.autotune(ql[0], reps=2)
        ms_l, lat_l, _ = time_matvecs(wsl, ql, nsteps, args.warmup, timing=False)
        p_l = wsl.matvec(ql[0]).cpu().numpy().astype(np.complex128)
        stl = pl.stats()
        out["paper_literal"] = {
            "eta": PAPER_LITERAL[0], "hf_threshold": PAPER_LITERAL[1], "dir_refine": PAPER_LITERAL[2],
            "value": round(wl.n / (ms_l / 1e3) / 1e6, 3), "unit": "Mpoints/s", "ms_per_step": round(ms_l, 4),
            "p50_ms": round(float(np.percentile(lat_l, 50)), 4), "p99_ms": round(float(np.percentile(lat_l, 99)), 4),
            "rel_l2_vs_direct_c64": float(np.linalg.norm(p_l[tg] - pd) / np.linalg.norm(pd)),
            "setup_s": round(setup_l, 3), "m2l_pairs": stl["m2l_pairs"], "eff_expansions": stl["eff_expansions"],
            "tuning": tuned_l}
        del pl, wsl, ql
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, X, wl.kappa, knobs, perm, args.cpu_sample or min(wl.n, 32768),
                                           args.cpu_single or 0)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
