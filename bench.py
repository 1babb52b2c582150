"""Benchmark: voxel-iterations/s of the Fourier-Galerkin operator G.A inside the paper's solvers.

Default workload (one GPU): 3D, N = 135^3, two-phase Boolean model of overlapping spheres
(radius 8 voxels, volume fraction 0.30), A = I in the matrix and 100 I in the spheres,
E = (1, 0, 0), GaNi (trapezoidal rule on the N grid), FP64.  One step solves this cell with all
four solvers -- Richardson, conjugate gradients, Chebyshev on [1, 100], Eyre-Milton -- each to
1e-8 by its own stopping test, and evaluates A_H (the energy).  The metric counts one
voxel-iteration per grid point per operator application inside the solver loops.

Prints ONE JSON line.  Extra objects: "roofline" (dominant pass, measured with HIP events on the
plan's stream during the timed steps, against the 8 TB/s HBM peak) and "cpu_baseline" (the FP64
oracle timed on a bounded sample of the same workload on the host cores).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SOLVERS = ["richardson", "cg", "chebyshev", "eyre_milton"]
PASS_KERNELS = {"first": "k2_first", "axis_fwd": "k2_axis<forward>", "middle": "k2_middle<G>",
                "axis_inv": "k2_axis<inverse>", "last": "k2_last"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "middle_pass_135_fp64_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1508_02045_amd", "csrc", f) for f in
                  ("fgh_kernels.hip", "fgh_fft.hpp", "fgh_internal.hpp", "fgh_v2.hpp", "fgh_args.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pass_bytes(g, d, p_bytes):
    """Algorithmic HBM bytes per launch of the fixed-traffic passes (read + write of the
    half spectrum): the middle and strided-axis passes move d * s complex each way."""
    N = g
    H = (N[-1] + 1) // 2
    s1 = N[0] * N[1] * H if d == 3 else N[0] * H
    s2 = s1
    cplx = 2 * p_bytes
    npts = 1
    for v in N:
        npts *= v
    # first (plain apply, phase map): read x and one byte of phase per point, write the spectrum;
    # last (plain store): read the spectrum, write y
    return {"middle": 2 * d * s2 * cplx, "axis_fwd": d * (s1 + s2) * cplx, "axis_inv": d * (s1 + s2) * cplx,
            "first": d * npts * p_bytes + npts + d * s1 * cplx, "last": d * s1 * cplx + d * npts * p_bytes}


def c4_section(fgh, inputs, torch, np, n):
    """243^3 Boolean spheres (r = 12, f = 0.25), A = I / rho I, E = e1: CG in plain FP64 versus
    FP32 transforms inside FP64 defect correction, for rho = 1e3 and 1e4 (A_H relative difference
    against the FP64 CG solved to 1e-10), plus the FP32 operator's per-pass times and its
    algorithmic-bytes fraction of the HBM peak."""
    out = {"N": n}
    for rho in (1e3, 1e4):
        w = inputs.config4(rho, N=n)
        tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in w.tables])
        ph = torch.from_numpy(w.phase).cuda()
        rec = {"fraction": round(w.fraction, 4)}
        ref = None
        for name, prec, tol in (("fp64_reference", fgh.FGH_FP64, 1e-10), ("fp64_cg", fgh.FGH_FP64, 1e-8),
                                ("fp32_refined_cg", fgh.FGH_FP32_REFINED, 1e-8)):
            plan = fgh.Plan(w.N, precision=prec, phase=ph, phase_table=tab, c_A=1.0, C_A=rho)
            e = plan.field()
            if name != "fp64_reference":
                plan.solve("cg", w.E, tol, max_iter=20000, e=e)  # warm-up (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, stats = plan.solve("cg", w.E, tol, max_iter=20000, e=e)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            bil, _ = plan.effective(w.E, e)
            r = {"status": st, "iters": stats[0]["iters"], "outer": stats[0]["outer_iters"],
                 "fp64_applies": stats[0]["fp64_applies"], "seconds": round(dt, 4), "A_H_11": float(bil[0, 0]),
                 "rel_res_true": stats[0]["rel_res_true"]}
            if name == "fp64_reference":
                ref = float(bil[0, 0])
            else:
                r["A_H_rel_err_vs_fp64_1e-10"] = abs(float(bil[0, 0]) - ref) / ref
            rec[name] = r
            del plan, e
            log(f"[bench] c4 rho={rho:g} {name}: {r['iters']} it {dt:.3f} s")
        rec["speedup_fp32_refined_vs_fp64"] = round(rec["fp64_cg"]["seconds"] / rec["fp32_refined_cg"]["seconds"], 3)
        out[f"rho_{rho:g}"] = rec
    # FP32 operator per-pass times
    w = inputs.config4(1e3, N=n)
    tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in w.tables])
    plan = fgh.Plan(w.N, precision=fgh.FGH_FP32_REFINED, phase=torch.from_numpy(w.phase).cuda(), phase_table=tab)
    x = torch.randn((3,) + w.N, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        plan.apply(x, y)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    for _ in range(10):
        plan.apply(x, y)
    prof = plan.read_profile()
    plan.set_profiling(False)
    per = {k: round(v[0] * 1e3 / max(v[1], 1), 2) for k, v in prof.items()}
    tot_us = sum(per.values())
    b_alg = (5 * 2 * 3 * 4 * (1 + 1 / n) + 1) * n ** 3  # five passes of the half spectrum, phase map
    out["apply_fp32"] = {"per_pass_avg_us": per, "sum_us": round(tot_us, 1), "B_alg_bytes": b_alg,
                         "alg_GBs": round(b_alg / (tot_us * 1e-6) / 1e9, 1),
                         "frac_of_8TBs": round(b_alg / (tot_us * 1e-6) / 8e12, 4),
                         "voxel_iterations_per_s": round(n ** 3 / (tot_us * 1e-6))}
    return out


def kappa_section(fgh, inputs, np, torch, n=85, kappas=(10.0, 100.0, 1000.0, 10000.0)):
    """Iterations to 1e-6 versus the inclusion contrast kappa on the paper's square inclusion
    (Sec. 4.6): GaNi with the four solvers, Ga with Richardson, CG and Chebyshev; the log-log
    slope of each solver's counts (O(kappa) expected for Richardson, O(sqrt kappa) otherwise)."""
    N = (n, n)
    ph = torch.from_numpy(inputs.paper_square(N)).cuda()
    out = {"N": list(N), "kappas": list(kappas), "tol": 1e-6}
    for rule, name in ((fgh.FGH_GANI, "gani"), (fgh.FGH_GA, "ga")):
        sol = ["richardson", "cg", "chebyshev"] + (["eyre_milton"] if rule == fgh.FGH_GANI else [])
        rec = {}
        for s in sol:
            its, secs = [], []
            for k in kappas:
                tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in inputs.iso_tables(2, [1.0, k])])
                plan = fgh.Plan(N, rule=rule, phase=ph, phase_table=tab, c_A=1.0, C_A=k)
                _, st, stats = plan.solve(s, [1.0, 0.0], 1e-6, max_iter=500000)
                its.append(stats[0]["iters"])
                secs.append(round(stats[0]["seconds"], 4))
                plan.close()
            slope = float(np.polyfit(np.log10(kappas), np.log10(its), 1)[0])
            rec[s] = {"iters": its, "seconds": secs, "loglog_slope": round(slope, 3)}
        out[name] = rec
        log(f"[bench] kappa sweep {name}: " + ", ".join(f"{s} {r['iters']}" for s, r in rec.items()))
    return out


def monitor_section(fgh, inputs, np, torch, w, plan_main):
    """Cost of the per-iteration monitors on the bench workload (CG to 1e-8): no recording,
    residual + energy history, plus the non-conformity; and the GaNi guaranteed-bound monitor on
    the paper's 85^2 square (a Ga plan on 169^2 supplies A_{2N-1})."""
    out = {}
    e = plan_main.field()

    def timed(tag):
        plan_main.solve("cg", w.E, 1e-8, max_iter=5000, e=e)  # warm (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, stats = plan_main.solve("cg", w.E, 1e-8, max_iter=5000, e=e)
        torch.cuda.synchronize()
        out[tag] = {"seconds": round(time.perf_counter() - t0, 4), "iters": stats[0]["iters"]}

    timed("none")
    plan_main.set_history(512)
    timed("residual_energy")
    plan_main.set_history(512, conformity=True)
    timed("residual_energy_conformity")
    plan_main.set_history(0)
    N = (85, 85)
    tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in inputs.iso_tables(2, [1.0, 100.0])])
    ph = torch.from_numpy(inputs.paper_square(N)).cuda()
    gani = fgh.Plan(N, rule=fgh.FGH_GANI, phase=ph, phase_table=tab, c_A=1.0, C_A=100.0)
    ga = fgh.Plan(N, rule=fgh.FGH_GA, phase=ph, phase_table=tab, c_A=1.0, C_A=100.0)
    rec = {}
    for tag, bound in (("none", False), ("gani_bound_monitor", True)):
        if bound:
            h = gani.set_history(256, bound_plan=ga)
        gani.solve("cg", [1.0, 0.0], 1e-6)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e2, st, stats = gani.solve("cg", [1.0, 0.0], 1e-6)
        torch.cuda.synchronize()
        rec[tag] = {"seconds": round(time.perf_counter() - t0, 4), "iters": stats[0]["iters"]}
        if bound:
            en = h["energy"][0, : stats[0]["iters"] + 1].cpu().numpy()
            rec[tag]["bound_first_last"] = [float(en[0]), float(en[-1])]
            gani.set_history(0)
    out["square85_cg_1e-6"] = rec
    log(f"[bench] monitors: {out}")
    return out


def adaptive_section(fgh, inputs, np, torch, w_main, plan_main, m=40, margins=(0.9, 1.02)):
    """Adaptive spectral bounds: Lanczos estimates from m CG steps (fgh_estimate_bounds), set with
    margins (lo * 0.9, hi * 1.02), against the pointwise bounds c_A, C_A of the material, for
    Richardson, Chebyshev and Eyre-Milton to 1e-8 (CG for reference).  Workloads: the 63^3
    anisotropic field (pointwise eigenvalues in [1, 1e3]) and the 135^3 spheres of the main line."""
    w3 = inputs.config3()
    plan3 = fgh.Plan(w3.N, A=torch.from_numpy(inputs.sym_pack(w3.A_full)).cuda(), a_kind=fgh.FGH_A_SYM)
    out = {}
    for tag, w, plan in (("aniso63", w3, plan3), ("spheres135", w_main, plan_main)):
        e = plan.field()
        c0, C0 = plan.bounds()

        def run(s):
            plan.solve(s, w.E, 1e-8, max_iter=200000, e=e)  # warm (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, stats = plan.solve(s, w.E, 1e-8, max_iter=200000, e=e)
            torch.cuda.synchronize()
            return {"iters": stats[0]["iters"], "seconds": round(time.perf_counter() - t0, 4), "status": st}

        rec = {"pointwise_bounds": [c0, C0], "cg": run("cg")}
        for s in ("richardson", "chebyshev", "eyre_milton"):
            rec[s] = {"pointwise": run(s)}
        plan.estimate_bounds(w.E, m, e=e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est = plan.estimate_bounds(w.E, m, e=e)
        rec["estimate"] = {"steps": est["steps"], "seconds": round(time.perf_counter() - t0, 4),
                           "ritz_lo": est["lo"], "ritz_hi": est["hi"]}
        plan.set_bounds(margins[0] * est["lo"], margins[1] * est["hi"])
        for s in ("richardson", "chebyshev", "eyre_milton"):
            rec[s]["estimated"] = run(s)
        plan.set_bounds(c0, C0)
        out[tag] = rec
        log(f"[bench] adaptive {tag}: ritz [{est['lo']:.4g}, {est['hi']:.4g}] vs [{c0:.4g}, {C0:.4g}]; " +
            ", ".join(f"{s} {rec[s]['pointwise']['iters']} -> {rec[s]['estimated']['iters']}"
                      for s in ("richardson", "chebyshev", "eyre_milton")) + f"; cg {rec['cg']['iters']}")
    plan3.close()
    return out


def served_section(fgh, inputs, np, n_req, max_active=4, pool_gb=24):
    """Served stream (mixed d, N, rule, contrast, solver, tolerance; see inputs.serving_requests).
    Baseline: the same requests one at a time in plain FP64; its mean service time S sets the
    Poisson arrival rate 1/S (load 1 for the baseline).  Served: FP32 transforms with FP64
    defect correction, `max_active` concurrent slots, admission by HBM footprint."""
    reqs = inputs.serving_requests(n_req, inputs.config_rng(4))

    def pack(tables):
        return np.stack([inputs.sym_pack(t[None])[:, 0] for t in tables])

    def submit(srv, q, prec):
        r, keep = fgh.make_request(q["d"], q["N"], q["phase"], pack(q["tables"]), q["E"], q["solver"], q["tol"],
                                   rule=q["rule"], precision=prec)
        rid = srv.submit(r)
        del keep
        return rid

    # baseline: sequential plain FP64
    srv = fgh.Server(int(pool_gb * (1 << 30)), max_active=1)
    ids = [submit(srv, q, fgh.FGH_FP64) for q in reqs]
    res64 = [srv.wait(i) for i in ids]
    srv.close()
    service = np.array([r["t_done"] - r["t_admit"] for r in res64])
    s_mean = float(service.mean())
    log(f"[bench] served: sequential FP64 baseline {n_req} requests, mean service {s_mean * 1e3:.1f} ms")
    rng = np.random.default_rng(np.random.SeedSequence(inputs.ROOT_SEED + 5))
    gaps = rng.exponential(1.0, size=n_req)  # unit-mean gaps, scaled per load below

    def fifo_latencies(arrivals):
        # the baseline under the same arrivals: one FIFO server with the measured service times
        t_free, out = 0.0, []
        for a, sv in zip(arrivals, service):
            start = max(a, t_free)
            t_free = start + sv
            out.append(t_free - a)
        return np.array(out)

    def replay(arrivals):
        srv = fgh.Server(int(pool_gb * (1 << 30)), max_active=max_active)
        t0 = time.perf_counter()
        ids = []
        for a, q in zip(arrivals, reqs):
            dt = t0 + a - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids.append(submit(srv, q, fgh.FGH_FP32_REFINED))
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
        srv.close()
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        return res, st, {"throughput_solves_per_s": round(n_req / span, 3),
                         "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                         "p99_latency_s": round(float(np.percentile(lat, 99)), 4)}

    served, seq = {}, {}
    res = st = None
    for load in (1.0, 0.5):
        arrivals = np.cumsum(gaps * (s_mean / load))
        arrivals -= arrivals[0]
        r_, st_, rec = replay(arrivals)
        if load == 1.0:
            res, st = r_, st_
        served[f"at_load_{load:g}"] = rec
        lat64 = fifo_latencies(arrivals)
        seq[f"at_load_{load:g}"] = {"p50_latency_s": round(float(np.percentile(lat64, 50)), 4),
                                    "p99_latency_s": round(float(np.percentile(lat64, 99)), 4)}
        log(f"[bench] served at load {load:g}: {rec}")
    # capacity: the whole stream submitted at once
    srv = fgh.Server(int(pool_gb * (1 << 30)), max_active=max_active)
    cids = [submit(srv, q, fgh.FGH_FP32_REFINED) for q in reqs]
    cres = [srv.wait(i) for i in cids]
    cap_span = max(r["t_done"] for r in cres) - min(r["t_submit"] for r in cres)
    srv.close()
    cap = n_req / cap_span
    rel = np.array([abs(r["energy"] - b["energy"]) / abs(b["energy"]) for r, b in zip(res, res64)])
    ok = sum(1 for r in res if r["status"] == 0)
    ok64 = sum(1 for r in res64 if r["status"] == 0)
    return {"requests": n_req, "max_active": max_active, "pool_GB": pool_gb,
            "arrival_rate_at_load_1_per_s": round(1.0 / s_mean, 3),
            "served_fp32_refined": {"capacity_solves_per_s": round(cap, 3), **served, "status_ok": ok,
                                    "peak_active": st["peak_active"],
                                    "peak_pool_GB": round(st["peak_pool_bytes"] / 2 ** 30, 2)},
            "sequential_fp64": {"capacity_solves_per_s": round(1.0 / s_mean, 3), **seq, "status_ok": ok64,
                                "latency_model": "single FIFO server, measured service times"},
            "capacity_ratio_served_vs_sequential": round(cap * s_mean, 3),
            "energy_rel_diff_served_vs_fp64": {"max": float(rel.max()), "median": float(np.median(rel))},
            "mix": {"d3": sum(q["d"] == 3 for q in reqs), "ga": sum(q["rule"] == 1 for q in reqs),
                    "eyre_milton": sum(q["solver"] == "eyre_milton" for q in reqs)}}


COPY_BYTES = 512 * 1024 * 1024


def applies_only(args, fgh, inputs, torch, np):
    """K plain applications y = G A x of the bench workload with per-pass timing, then a plain
    device copy of COPY_BYTES (read COPY_BYTES, write COPY_BYTES) that calibrates the HBM byte
    counters of a profiler run."""
    w = inputs.config2(N=args.n) if args.workload == "spheres135" else inputs.config4(1e3, N=243)
    tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in w.tables])
    prec = fgh.FGH_FP64 if args.precision == "fp64" else fgh.FGH_FP32_REFINED
    plan = fgh.Plan(w.N, precision=prec, phase=torch.from_numpy(w.phase).cuda(), phase_table=tab, c_A=1.0,
                    C_A=w.contrast)
    dt = torch.float64 if prec == fgh.FGH_FP64 else torch.float32
    x = torch.randn((3,) + w.N, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        plan.apply(x, y)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    for i in range(args.applies_only):
        plan.apply(x, y)
    prof = plan.read_profile()
    plan.set_profiling(False)
    torch.cuda.synchronize()
    log(f"[bench] {args.applies_only} applies done")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    pb = pass_bytes(w.N, 3, 8 if prec == fgh.FGH_FP64 else 4)
    per = {k: round(v[0] * 1e3 / max(v[1], 1), 2) for k, v in prof.items()}
    print(json.dumps({"workload": w.name, "precision": args.precision, "applies": args.applies_only,
                      "per_pass_avg_us": per, "algorithmic_bytes_per_launch": pb,
                      "copy_bytes_each_way": COPY_BYTES}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=135)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=16)
    ap.add_argument("--no-c4", action="store_true", help="skip the 243^3 FP32-refinement section")
    ap.add_argument("--no-served", action="store_true", help="skip the served-stream section")
    ap.add_argument("--no-kappa", action="store_true", help="skip the iterations-versus-contrast section")
    ap.add_argument("--no-monitors", action="store_true", help="skip the monitor-cost section")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive-bounds section")
    ap.add_argument("--served-n", type=int, default=64)
    ap.add_argument("--c4-n", type=int, default=243)
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the per-pass HIP events (solver loops then replay HIP graphs)")
    ap.add_argument("--applies-only", type=int, default=0, metavar="K",
                    help="counter runs: K plain operator applications of the workload (and a copy of known "
                         "size for calibration), a summary line, nothing else")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64", help="with --applies-only")
    ap.add_argument("--workload", choices=["spheres135", "spheres243"], default="spheres135",
                    help="with --applies-only: the 135^3 r=8 f=0.30 or the 243^3 r=12 f=0.25 Boolean spheres")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              f"path: a solve runs on one device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1508_02045_amd import fgh, inputs

    torch.cuda.set_device(0)
    if args.applies_only > 0:
        applies_only(args, fgh, inputs, torch, np)
        return
    n = args.n
    log(f"[bench] generating Boolean spheres {n}^3 r=8 f=0.30")
    w = inputs.config2(N=n)
    tab = np.stack([inputs.sym_pack(t[None])[:, 0] for t in w.tables])
    phase_dev = torch.from_numpy(w.phase).cuda()
    plan = fgh.Plan(w.N, phase=phase_dev, phase_table=tab, c_A=1.0, C_A=w.contrast)
    d = 3
    npts = plan.npts
    tol = 1e-8
    e = plan.field()

    def step():
        out = {}
        for s in SOLVERS:
            e_, st, stats = plan.solve(s, w.E, tol, max_iter=5000, e=e)
            if st != fgh.FGH_OK:
                raise RuntimeError(f"{s}: status {st} {stats}")
            bil, flux = plan.effective(w.E, e)
            out[s] = {"iters": stats[0]["iters"], "seconds": stats[0]["seconds"], "A_H_11": float(bil[0, 0]),
                      "flux": [float(v) for v in flux[0]], "rel_res_true": stats[0]["rel_res_true"]}
        return out

    for i in range(args.warmup):
        log(f"[bench] warmup step {i + 1}/{args.warmup}")
        step()
    # untimed: per-pass breakdown of one step, to name the dominant fixed-traffic pass
    plan.set_profiling(True)
    step()
    prof_all = plan.read_profile()
    plan.set_profiling(False)
    pb = pass_bytes(w.N, d, 8)
    dom = max(("middle", "axis_fwd", "axis_inv"), key=lambda k: prof_all[k][0])

    torch.cuda.synchronize()
    if not args.no_profile:
        plan.set_profiling(True, passes=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_iters = 0
    res = None
    for i in range(args.steps):
        res = step()
        total_iters += sum(r["iters"] for r in res.values())
        log(f"[bench] step {i + 1}/{args.steps}: " + ", ".join(f"{k} {v['iters']}" for k, v in res.items()))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.read_profile()
    plan.set_profiling(False)
    elapsed = t1 - t0
    value = total_iters * npts / elapsed

    # roofline of the dominant fixed-traffic pass, timed with HIP events inside the timed steps
    ms_tot, launches = prof[dom]
    avg_s = ms_tot / 1e3 / max(launches, 1) if launches else float("nan")
    achieved = pb[dom] / avg_s / 1e9 if launches else None
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("pass") == dom:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "kernel": PASS_KERNELS[dom], "achieved": None if achieved is None else round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": pb[dom], "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
                "per_pass_avg_us_untimed_step": {k: round(v[0] * 1e3 / max(v[1], 1), 2) for k, v in prof_all.items()},
                "per_pass_share_untimed_step": {k: round(v[0] / max(sum(x[0] for x in prof_all.values()), 1e-30), 3)
                                                for k, v in prof_all.items()}}
    extra = None if args.no_c4 else c4_section(fgh, inputs, torch, np, args.c4_n)
    served = None if args.no_served else served_section(fgh, inputs, np, args.served_n)
    kappa = None if args.no_kappa else kappa_section(fgh, inputs, np, torch)
    monitors = None if args.no_monitors else monitor_section(fgh, inputs, np, torch, w, plan)
    adaptive = None if args.no_adaptive else adaptive_section(fgh, inputs, np, torch, w, plan)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import orc
        A_full = w.full()
        log(f"[bench] cpu baseline: oracle CG, {args.cpu_iters} fixed iterations at {n}^3 "
            f"on {orc.num_threads()} threads")
        tc = time.perf_counter()
        r = orc.solve(w.N, orc.GANI, A_full, w.E, "cg", 1.0, w.contrast, tol, fixed_iters=args.cpu_iters)
        tcpu = time.perf_counter() - tc
        cpu = {"value": args.cpu_iters * npts / tcpu, "unit": "voxel-iterations/s", "cores": orc.num_threads(),
               "kind": "oracle",
               "sample": f"FP64 oracle (naive DFT) CG with {args.cpu_iters} fixed iterations on the same {n}^3 "
                         f"input, wall {tcpu:.1f} s including its right-hand side and exit-residual applies"}
        del r

    line = {
        "metric": "voxel-iterations/s of G.A",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D Boolean spheres {n}^3 r=8 f={w.fraction:.4f} contrast 100, GaNi, FP64, "
                               f"Richardson+CG+Chebyshev+Eyre-Milton to 1e-8, E=e1",
                   "N": list(w.N), "solvers": SOLVERS, "tol": tol, "voxel_iterations_per_step": total_iters // args.steps * npts},
        "solvers": res,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "c4_fp32_refined_243": extra,
        "served": served,
        "kappa_sweep": kappa,
        "monitors": monitors,
        "adaptive_bounds": adaptive,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
