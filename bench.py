"""Benchmark: voxel-iterations/s of the Fourier-Galerkin operator G.A inside the paper's solvers.

Default workload (one GPU): 3D, N = 243^3, two-phase Boolean model of overlapping spheres (radius
12 voxels, volume fraction 0.25), A = I in the matrix and rho I in the spheres for rho = 1e3 and
1e4, E = (1, 0, 0), GaNi (trapezoidal rule on the N grid), plain FP64 conjugate gradients
(Algorithm 2) to 1e-8.  One step solves the cell for both contrasts and evaluates A_H (the
energy).  The metric counts one voxel-iteration per grid point per loop body (one operator
application each).  The timed steps run the library as it ships: loop bodies replayed from HIP
graphs, no profiling.

Prints ONE JSON line.  Extra objects:
  roofline      the kernel with the largest share of GPU time in a step like the timed ones (every
                launch timed with HIP events attached to its dispatch, on the stream it runs on,
                in one profiled step after the timed ones), its algorithmic bytes per launch over
                its average duration, against the 8 TB/s HBM peak; `traffic` from the committed
                rocprofv3 counter summary when it was taken on the current kernel sources;
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample of the same workload;
  apply_243     the operator alone: median of 5 runs of 100 back-to-back applications (FP64, FP32);
  c4_fp32_refined  FP32 transforms inside FP64 defect correction against plain FP64 CG;
  c2_spheres135 the 135^3 spheres with all four solvers; c3_aniso63: exact integration on 125^3;
  served, kappa_sweep, monitors, adaptive_bounds: see their functions.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--quick]
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SOLVERS = ["richardson", "cg", "chebyshev", "eyre_milton"]
KINDS = ["first", "axis_fwd", "middle", "axis_inv", "last", "cg_update", "reduce"]
# kernels of one CG body on a specialised 3D grid, by launch kind
CG_KERNELS = {"first": "k2_first<double,3> (x += alpha p, p = r + beta p, A p, r2c of the last axis)",
              "axis_fwd": "k2_axis<double,forward>", "middle": "k2_middle<double,3,G>",
              "axis_inv": "k2_axis<double,inverse>", "last": "k2_last<double,3,EPI_CG> (c2r, q = C p, (q, p))",
              "cg_update": "k_cg_update<double> (r -= alpha q, (r, r))", "reduce": "k_reduce"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_243.json")
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


def geometry(N, p_bytes):
    """Field bytes F = d |grid| p and half-spectrum bytes S = d rows (n_last + 1)/2 2p of a GaNi grid."""
    d = len(N)
    npts = 1
    for v in N:
        npts *= v
    H = (N[-1] + 1) // 2
    s1 = npts // N[-1] * H
    return d, npts, d * npts * p_bytes, d * s1 * 2 * p_bytes


def apply_bytes(N, p_bytes, a_bytes=1):
    """Algorithmic HBM bytes of one application y = G A x (five passes in 3D, three in 2D): the
    first pass reads x and the coefficients (a bytes per point) and writes the half spectrum, each
    strided / middle pass reads and writes it, the last pass reads it and writes y."""
    d, npts, F, S = geometry(N, p_bytes)
    inner = 2 * d - 3  # passes between the first and the last (3D: axis 1, axis 0, axis 1), each S in and out
    return 2 * F + a_bytes * npts + 2 * S + inner * 2 * S


LAST_LEVEL_CACHE_BYTES = 256 * 1024 * 1024


def cg_defers(N, p_bytes):
    """Whether the library's CG leaves x += alpha p to the next body's first pass: when its four
    vectors exceed the device's 256 MiB last-level cache (the library's rule)."""
    d, npts, F, S = geometry(N, p_bytes)
    return 4 * F > LAST_LEVEL_CACHE_BYTES


def cg_kind_bytes(N, p_bytes, a_bytes=1):
    """Algorithmic bytes per launch of each kernel of one CG body (Algorithm 2) with a phase map.
    With the deferred iterate update (cg_defers): first: x, r, p in, x, p out, phase, spectrum out;
    update: r, q in, r out.  Otherwise: first: r, p in, p out, phase, spectrum out; update: x, p,
    r, q in, x, r out.  Strided / middle: spectrum in and out; last: spectrum and p in, q out;
    reduce: the partial sums."""
    d, npts, F, S = geometry(N, p_bytes)
    defer = cg_defers(N, p_bytes)
    return {"first": (5 if defer else 3) * F + a_bytes * npts + S, "axis_fwd": 2 * S, "middle": 2 * S,
            "axis_inv": 2 * S, "last": S + 2 * F, "cg_update": (3 if defer else 6) * F, "reduce": 1024 * 8}


def phase_table(inputs, np, tables):
    return np.stack([inputs.sym_pack(t[None])[:, 0] for t in tables])


def time_applies(torch, plan, x, y, reps=100, runs=5):
    """Median over `runs` of the mean time of `reps` back-to-back applications (ms), from torch
    events on the current stream, which is the plan's stream."""
    for _ in range(3):
        plan.apply(x, y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.apply(x, y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / reps)
    return statistics.median(ts), ts


def apply_section(fgh, inputs, torch, np, n, plan64):
    """The operator alone at n^3: FP64 on the timed workload's plan and FP32 on a refined plan of
    the same input; median of 5 runs of 100 back-to-back applications against the algorithmic
    bytes of the five passes."""
    out = {"N": n, "timing": "median of 5 runs of 100 back-to-back applications, torch events on the plan's stream"}
    w = inputs.config4(1e3, N=n)
    plan32 = fgh.Plan(w.N, precision=fgh.FGH_FP32_REFINED, phase=torch.from_numpy(w.phase).cuda(),
                      phase_table=phase_table(inputs, np, w.tables), c_A=1.0, C_A=1e3)
    for tag, plan, dt, p in (("fp64", plan64, torch.float64, 8), ("fp32", plan32, torch.float32, 4)):
        x = torch.randn((3,) + w.N, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        ms, runs = time_applies(torch, plan, x, y)
        b = apply_bytes(w.N, p)
        out[tag] = {"ms_per_apply": round(ms, 4), "runs_ms": [round(t, 4) for t in runs], "B_alg_bytes": b,
                    "alg_GBs": round(b / (ms * 1e-3) / 1e9, 1), "frac_of_8TBs": round(b / (ms * 1e-3) / 8e12, 4),
                    "voxel_applications_per_s": round(n ** 3 / (ms * 1e-3))}
        log(f"[bench] apply {tag} {n}^3: {ms * 1e3:.1f} us, {out[tag]['frac_of_8TBs']:.3f} of 8 TB/s")
        del x, y
    plan32.close()
    return out


def refined_section(fgh, inputs, torch, np, n, fp64_seconds):
    """C4 variant (ii): FP32 transforms, projection and A multiply inside FP64 defect correction,
    CG to 1e-8, for rho = 1e3 and 1e4; A_H error against plain FP64 CG solved to 1e-10 and the
    speedup over the plain FP64 CG of the timed steps (fp64_seconds, per contrast)."""
    out = {"N": n}
    for rho in (1e3, 1e4):
        w = inputs.config4(rho, N=n)
        ph = torch.from_numpy(w.phase).cuda()
        tab = phase_table(inputs, np, w.tables)
        rec = {}
        ref = None
        for name, prec, tol in (("fp64_reference_1e-10", fgh.FGH_FP64, 1e-10),
                                ("fp32_refined_cg", fgh.FGH_FP32_REFINED, 1e-8)):
            plan = fgh.Plan(w.N, precision=prec, phase=ph, phase_table=tab, c_A=1.0, C_A=rho)
            e = plan.field()
            if prec == fgh.FGH_FP32_REFINED:
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
            if ref is None:
                ref = float(bil[0, 0])
            else:
                r["A_H_rel_err_vs_fp64_1e-10"] = abs(float(bil[0, 0]) - ref) / ref
            rec[name] = r
            plan.close()
            del e
            log(f"[bench] c4 rho={rho:g} {name}: {r['iters']} it {dt:.3f} s")
        rec["fp64_cg_1e-8_seconds"] = round(fp64_seconds[rho], 4)
        rec["speedup_fp32_refined_vs_fp64"] = round(fp64_seconds[rho] / rec["fp32_refined_cg"]["seconds"], 3)
        out[f"rho_{rho:g}"] = rec
    return out


def c2_section(fgh, inputs, torch, np, n=135):
    """135^3 Boolean spheres (r = 8, f = 0.30), A = I / 100 I, E = e1: the four solvers to 1e-8,
    time to tolerance and A_H each (one warm-up solve each first)."""
    w = inputs.config2(N=n)
    plan = fgh.Plan(w.N, phase=torch.from_numpy(w.phase).cuda(), phase_table=phase_table(inputs, np, w.tables),
                    c_A=1.0, C_A=w.contrast)
    e = plan.field()
    out = {"N": n, "fraction": round(w.fraction, 4)}
    total_vox, total_s = 0, 0.0
    for s in SOLVERS:
        plan.solve(s, w.E, 1e-8, max_iter=5000, e=e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, stats = plan.solve(s, w.E, 1e-8, max_iter=5000, e=e)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bil, _ = plan.effective(w.E, e)
        out[s] = {"iters": stats[0]["iters"], "seconds": round(dt, 4), "A_H_11": float(bil[0, 0]),
                  "rel_res_true": stats[0]["rel_res_true"]}
        total_vox += stats[0]["iters"] * plan.npts
        total_s += dt
    out["voxel_iterations_per_s"] = round(total_vox / total_s)
    plan.close()
    log(f"[bench] c2 135^3: " + ", ".join(f"{s} {out[s]['iters']}" for s in SOLVERS))
    return out


def c3_section(fgh, inputs, torch, np):
    """Anisotropic 63^3 (per-voxel R^T diag(lambda) R, lambda in [1, 1e3]): loads e1, e2, e3 by CG
    to 1e-9 with exact integration on the double grid 125^3 and with GaNi on 63^3; the full A_H."""
    w = inputs.config3()
    A = torch.from_numpy(inputs.sym_pack(w.A_full)).cuda()
    out = {"N": list(w.N)}
    for rule, tag in ((fgh.FGH_GA, "ga_125"), (fgh.FGH_GANI, "gani_63")):
        t0 = time.perf_counter()
        plan = fgh.Plan(w.N, rule=rule, A=A, a_kind=fgh.FGH_A_SYM)
        t_plan = time.perf_counter() - t0
        E = np.eye(3)
        e = plan.field(3)
        plan.solve("cg", E, 1e-9, max_iter=5000, e=e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, stats = plan.solve("cg", E, 1e-9, max_iter=5000, e=e)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bil, _ = plan.effective(E, e)
        out[tag] = {"grid": list(plan.grid), "plan_seconds": round(t_plan, 3), "seconds_3_loads": round(dt, 4),
                    "iters": [s["iters"] for s in stats], "A_H": [[float(v) for v in row] for row in bil]}
        plan.close()
        log(f"[bench] c3 {tag}: iters {out[tag]['iters']}, {dt:.3f} s")
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
    defect correction, `max_active` worker slots, admission by HBM footprint, requests of one size
    class solved together in shared launches.  Capacities (whole stream submitted at once) are
    also given with shared launches switched off and for plain FP64 in the slots, to separate
    the gains of batching, of FP32 and of overlap."""
    import os
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
        for k, (a, q) in enumerate(zip(arrivals, reqs)):
            dt = t0 + a - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids.append(submit(srv, q, fgh.FGH_FP32_REFINED))
            if (k + 1) % 500 == 0:
                log(f"[bench] served: {k + 1} of {n_req} requests submitted")
        res = [srv.wait(i) for i in ids]
        st = srv.stats()
        srv.close()
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        return res, st, {"throughput_solves_per_s": round(n_req / span, 3),
                         "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                         "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                         "peak_batch": st["peak_batch"], "groups": st["batches"]}

    def capacity(prec, batching=True):
        if not batching:
            os.environ["FGH_BATCH"] = "0"
        try:
            srv = fgh.Server(int(pool_gb * (1 << 30)), max_active=max_active)
            cids = [submit(srv, q, prec) for q in reqs]
            n_req_here = len(cids)
            cres = [srv.wait(i) for i in cids]
            st = srv.stats()
            srv.close()
        finally:
            os.environ.pop("FGH_BATCH", None)
        span = max(r["t_done"] for r in cres) - min(r["t_submit"] for r in cres)
        return n_req_here / span, cres, st

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
    cap, cres, cst = capacity(fgh.FGH_FP32_REFINED)
    cap_nb, _, _ = capacity(fgh.FGH_FP32_REFINED, batching=False)
    cap64, _, _ = capacity(fgh.FGH_FP64)
    # where shared launches pay: streams of one size class (mixed contrast and tolerance), whole
    # stream at once, with and without shared launches; the larger classes on long runs only
    small = {}
    classes = [((45, 45, 45), "cg", 64), ((81, 81), "eyre_milton", 64)]
    if n_req >= 1000:
        classes += [((243, 243), "cg", 32), ((81, 81, 81), "cg", 32), ((135, 135, 135), "cg", 16)]
    for N, solver, count in classes:
        srng = np.random.default_rng(np.random.SeedSequence(inputs.ROOT_SEED + 6))
        sreqs = []
        for k in range(count):
            ph, _, _ = inputs.boolean_spheres(N, max(2, round(N[0] / 20)), float(srng.uniform(0.1, 0.4)), srng)
            E = np.zeros(len(N))
            E[0] = 1.0
            sreqs.append({"d": len(N), "N": N, "phase": ph, "rule": 0, "solver": solver, "E": E,
                          "tol": [1e-6, 1e-8][k % 2],
                          "tables": inputs.iso_tables(len(N), [1.0, float(10 ** srng.uniform(1, 4))])})
        saved = reqs[:]
        reqs[:] = sreqs
        try:
            capacity(fgh.FGH_FP32_REFINED)  # warm-up: tile tuning of the shape
            on, _, sst = capacity(fgh.FGH_FP32_REFINED)
            off, _, _ = capacity(fgh.FGH_FP32_REFINED, batching=False)
        finally:
            reqs[:] = saved
        small[f"{count}x" + "x".join(map(str, N)) + "_" + solver] = {"shared_launches_solves_per_s": round(on, 1),
                                                      "separate_solves_per_s": round(off, 1),
                                                      "peak_batch": sst["peak_batch"], "groups": sst["batches"]}
    log(f"[bench] served small classes: {small}")
    log(f"[bench] served capacity: FP32 refined {cap:.2f}/s (peak batch {cst['peak_batch']}, {cst['batches']} groups), "
        f"without shared launches {cap_nb:.2f}/s, FP64 in the slots {cap64:.2f}/s, sequential FP64 {1 / s_mean:.2f}/s")
    rel = np.array([abs(r["energy"] - b["energy"]) / abs(b["energy"]) for r, b in zip(res, res64)])
    ok = sum(1 for r in res if r["status"] == 0)
    ok64 = sum(1 for r in res64 if r["status"] == 0)
    return {"requests": n_req, "max_active": max_active, "pool_GB": pool_gb,
            "arrival_rate_at_load_1_per_s": round(1.0 / s_mean, 3),
            "served_fp32_refined": {"capacity_solves_per_s": round(cap, 3), **served, "status_ok": ok,
                                    "peak_active": st["peak_active"],
                                    "peak_pool_GB": round(st["peak_pool_bytes"] / 2 ** 30, 2),
                                    "capacity_peak_batch": cst["peak_batch"], "capacity_groups": cst["batches"]},
            "served_fp32_refined_without_shared_launches": {"capacity_solves_per_s": round(cap_nb, 3)},
            "single_small_class_streams": small,
            "served_fp64_in_slots": {"capacity_solves_per_s": round(cap64, 3)},
            "sequential_fp64": {"capacity_solves_per_s": round(1.0 / s_mean, 3), **seq, "status_ok": ok64,
                                "latency_model": "single FIFO server, measured service times"},
            "capacity_ratio_served_vs_sequential": round(cap * s_mean, 3),
            "energy_rel_diff_served_vs_fp64": {"max": float(rel.max()), "median": float(np.median(rel))},
            "mix": {"d3": sum(q["d"] == 3 for q in reqs), "ga": sum(q["rule"] == 1 for q in reqs),
                    "eyre_milton": sum(q["solver"] == "eyre_milton" for q in reqs)}}


COPY_BYTES = 512 * 1024 * 1024


def counters_mode(args, fgh, inputs, torch, np):
    """Runs for rocprofv3 counter collection (243^3 unless --n): `cg64` runs K fixed FP64 CG bodies
    of the timed workload (rho = 1e3), `rich64` K fixed FP64 Richardson bodies (the fused last +
    first pass), `apply64` / `apply32` K plain applications; then a plain device copy of
    COPY_BYTES each way that calibrates the byte counters."""
    n = args.n
    w = inputs.config4(1e3, N=n)
    prec = fgh.FGH_FP32_REFINED if args.counters == "apply32" else fgh.FGH_FP64
    plan = fgh.Plan(w.N, precision=prec, phase=torch.from_numpy(w.phase).cuda(),
                    phase_table=phase_table(inputs, np, w.tables), c_A=1.0, C_A=1e3)
    if args.counters == "cg64":
        e = plan.field()
        _, st, stats = plan.solve_fixed("cg", w.E, args.counter_reps, e=e)
        kb = cg_kind_bytes(w.N, 8)
    elif args.counters == "rich64":
        e = plan.field()
        _, st, stats = plan.solve_fixed("richardson", w.E, args.counter_reps, e=e)
        d, npts, F, S = geometry(w.N, 8)
        # fused last + first: spectrum, x, phase in; x, next spectrum out
        kb = {"fused": 2 * S + 2 * F + npts, "axis_fwd": 2 * S, "middle": 2 * S, "axis_inv": 2 * S}
    else:
        dt = torch.float64 if prec == fgh.FGH_FP64 else torch.float32
        x = torch.randn((3,) + w.N, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.counter_reps):
            plan.apply(x, y)
        d, npts, F, S = geometry(w.N, 8 if prec == fgh.FGH_FP64 else 4)
        kb = {"first": F + npts + S, "axis_fwd": 2 * S, "middle": 2 * S, "axis_inv": 2 * S, "last": S + F}
    torch.cuda.synchronize()
    log(f"[bench] counters {args.counters}: {args.counter_reps} done")
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": w.name, "mode": args.counters, "reps": args.counter_reps,
                      "algorithmic_bytes_per_launch": kb, "copy_bytes_each_way": COPY_BYTES,
                      "kernel_source_hash": kernel_source_hash()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=243, help="grid size of the timed workload (243: C4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-applies", type=int, default=2, help="oracle applications in the CPU baseline sample")
    ap.add_argument("--quick", action="store_true", help="the headline line only (no extra sections)")
    for name in ("apply", "refined", "c2", "c3", "served", "kappa", "monitors", "adaptive"):
        ap.add_argument(f"--no-{name}", action="store_true", help=f"skip the {name} section")
    ap.add_argument("--served-n", type=int, default=64)
    ap.add_argument("--counters", choices=["cg64", "rich64", "apply64", "apply32"], default=None,
                    help="counter runs for rocprofv3 --pmc: K CG bodies or K applications at 243^3 and a copy "
                         "of known size for calibration, a summary line, nothing else")
    ap.add_argument("--counter-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              f"path: a solve runs on one device", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1508_02045_amd import fgh, inputs

    torch.cuda.set_device(0)
    if args.counters:
        counters_mode(args, fgh, inputs, torch, np)
        return
    n = args.n
    tol = 1e-8
    rhos = (1e3, 1e4)
    log(f"[bench] generating Boolean spheres {n}^3 r=12 f=0.25")
    w = inputs.config4(1e3, N=n)
    ph = torch.from_numpy(w.phase).cuda()
    plans, fields = {}, {}
    t0 = time.perf_counter()
    for rho in rhos:
        plans[rho] = fgh.Plan(w.N, phase=ph, phase_table=phase_table(inputs, np, inputs.iso_tables(3, [1.0, rho])),
                              c_A=1.0, C_A=rho)
        fields[rho] = plans[rho].field()
    plan_seconds = (time.perf_counter() - t0) / len(rhos)
    npts = plans[rhos[0]].npts

    def step():
        out = {}
        for rho in rhos:
            ts = time.perf_counter()
            _, st, stats = plans[rho].solve("cg", w.E, tol, max_iter=20000, e=fields[rho])
            if st != fgh.FGH_OK:
                raise RuntimeError(f"rho {rho}: status {st} {stats}")
            bil, flux = plans[rho].effective(w.E, fields[rho])
            torch.cuda.synchronize()
            out[rho] = {"iters": stats[0]["iters"], "seconds": round(time.perf_counter() - ts, 4),
                        "A_H_11": float(bil[0, 0]), "flux": [float(v) for v in flux[0]],
                        "rel_res_true": stats[0]["rel_res_true"]}
        return out

    for i in range(args.warmup):
        log(f"[bench] warmup step {i + 1}/{args.warmup}")
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_iters = 0
    res = None
    seconds = {rho: [] for rho in rhos}
    for i in range(args.steps):
        res = step()
        total_iters += sum(r["iters"] for r in res.values())
        for rho in rhos:
            seconds[rho].append(res[rho]["seconds"])
        log(f"[bench] step {i + 1}/{args.steps}: " + ", ".join(f"rho {k:g}: {v['iters']} it {v['seconds']:.3f} s"
                                                              for k, v in res.items()))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = total_iters * npts / elapsed

    # one more step with every launch timed (HIP events attached to the dispatches, on the stream
    # they run on; loop bodies are then launched one by one instead of replayed from graphs)
    for rho in rhos:
        plans[rho].set_profiling(True)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    step()
    torch.cuda.synchronize()
    profiled_ms = (time.perf_counter() - tp) * 1e3
    kinds = {k: [0.0, 0] for k in KINDS}
    for rho in rhos:
        for k, (ms, cnt) in plans[rho].read_profile().items():
            kinds[k][0] += ms
            kinds[k][1] += cnt
        plans[rho].set_profiling(False)
    kb = cg_kind_bytes(w.N, 8)
    gpu_ms = sum(v[0] for v in kinds.values())
    table = {}
    for k, (ms, cnt) in kinds.items():
        if cnt == 0:
            continue
        avg = ms / cnt * 1e-3
        table[k] = {"kernel": CG_KERNELS[k], "launches": cnt, "avg_us": round(avg * 1e6, 2),
                    "share": round(ms / gpu_ms, 4), "alg_bytes_per_launch": kb[k],
                    "alg_GBs": round(kb[k] / avg / 1e9, 1), "frac": round(kb[k] / avg / 8e12, 4)}
    dom = max(table, key=lambda k: table[k]["share"])
    traffic = None
    traffic_src = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_hash") == kernel_source_hash() and dom in tr.get("cg64", {}):
            traffic = tr["cg64"][dom]["bytes_per_launch"]
            traffic_src = os.path.relpath(TRAFFIC_FILE, ROOT)
    dom_avg = table[dom]["avg_us"] * 1e-6
    roofline = {"bound": "hbm", "kernel": CG_KERNELS[dom], "kind": dom, "achieved": table[dom]["alg_GBs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": table[dom]["frac"], "traffic": traffic,
                "traffic_source": traffic_src, "algorithmic_bytes_per_launch": kb[dom],
                "avg_launch_us": round(dom_avg * 1e6, 2), "launches": table[dom]["launches"],
                "timing": "HIP events on each dispatch in one profiled step after the timed steps",
                "profiled_step_ms": round(profiled_ms, 1), "kernel_ms_in_profiled_step": round(gpu_ms, 1),
                "kernels": table}
    log(f"[bench] dominant kernel {dom}: {table[dom]['avg_us']} us, {table[dom]['frac']:.3f} of 8 TB/s")
    # what streaming reaches on this device at the same working-set size: a device copy of one
    # 243^3 FP64 vector field (344 MB each way), median of 5 runs of 20 copies
    src = torch.empty((3,) + w.N, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    cts = []
    for _ in range(5):
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(20):
            dst.copy_(src)
        c1.record()
        c1.synchronize()
        cts.append(c0.elapsed_time(c1) / 20 * 1e-3)
    copy_gbs = 2 * src.numel() * 8 / statistics.median(cts) / 1e9
    del src, dst
    roofline["copy_GBs_same_size"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(table[dom]["alg_GBs"] / copy_gbs, 4)
    log(f"[bench] device copy of a 344 MB field: {copy_gbs:.0f} GB/s ({copy_gbs / 8000:.3f} of 8 TB/s)")

    extra = {}
    fp64_seconds = {rho: statistics.median(seconds[rho]) for rho in rhos}
    if not args.quick and not args.no_apply:
        extra["apply_243"] = apply_section(fgh, inputs, torch, np, n, plans[1e3])
    for rho in rhos:
        plans[rho].close()
    plans.clear()
    fields.clear()
    torch.cuda.empty_cache()
    if not args.quick and not args.no_refined:
        extra["c4_fp32_refined"] = refined_section(fgh, inputs, torch, np, n, fp64_seconds)
    if not args.quick and not args.no_c2:
        extra["c2_spheres135"] = c2_section(fgh, inputs, torch, np)
    if not args.quick and not args.no_c3:
        extra["c3_aniso63"] = c3_section(fgh, inputs, torch, np)
    if not args.quick and not args.no_served:
        extra["served"] = served_section(fgh, inputs, np, args.served_n)
    if not args.quick and not args.no_kappa:
        extra["kappa_sweep"] = kappa_section(fgh, inputs, np, torch)
    if not args.quick and (not args.no_monitors or not args.no_adaptive):
        w2 = inputs.config2()
        plan2 = fgh.Plan(w2.N, phase=torch.from_numpy(w2.phase).cuda(), phase_table=phase_table(inputs, np, w2.tables),
                         c_A=1.0, C_A=w2.contrast)
        if not args.no_monitors:
            extra["monitors"] = monitor_section(fgh, inputs, np, torch, w2, plan2)
        if not args.no_adaptive:
            extra["adaptive_bounds"] = adaptive_section(fgh, inputs, np, torch, w2, plan2)
        plan2.close()

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import orc
        A_full = w.full()
        x = np.random.default_rng(0).standard_normal((3,) + w.N)
        k = args.cpu_applies
        log(f"[bench] cpu baseline: {k} oracle applications of G.A at {n}^3 on {orc.num_threads()} threads")
        tc = time.perf_counter()
        for _ in range(k):
            orc.apply(w.N, orc.GANI, A_full, x)
        tcpu = time.perf_counter() - tc
        cpu = {"value": k * npts / tcpu, "unit": "voxel-iterations/s", "cores": orc.num_threads(), "kind": "oracle",
               "sample": f"{k} applications of G.A by the FP64 oracle (naive DFT) on the same {n}^3 input, "
                         f"one CG body's operator work each, wall {tcpu:.1f} s"}
        del A_full

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
        "config": {"workload": f"C4: 3D Boolean spheres {n}^3 r=12 f={w.fraction:.4f}, A = I / rho I with rho 1e3 "
                               f"and 1e4, E=e1, GaNi, plain FP64 CG to 1e-8 (one solve per contrast per step)",
                   "N": list(w.N), "rho": list(rhos), "solver": "cg", "tol": tol,
                   "voxel_iterations_per_step": total_iters // args.steps * npts},
        "solves": {f"rho_{k:g}": v for k, v in res.items()},
        "time_to_tolerance_s": {f"rho_{k:g}": round(v, 4) for k, v in fp64_seconds.items()},
        "plan_seconds": round(plan_seconds, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
