"""Benchmark: formal-solution throughput of the line radiative transfer path on
one MI355X.

Workload (default): the large-velocity-gradient clumpy cloud, 200,000
points in a sphere with k = 16 neighbour lists, log-normal density,
rotation plus turbulence with Doppler shifts up to 20 line widths between
neighbours, 20-level linear rotor (19 lines), 48 HEALPix rays, 39 bins per
line; formal solution in FP32 with FP64 statistical equilibrium and
classical Ng of order 4.  The 3D outflow (50,000 points) and a short
serving run are reported as extra keys.

A step is one Lambda-iteration over the whole model: line coefficients ->
formal solution (every origin x ray x line x bin) -> statistical
equilibrium -> convergence measure (-> Ng every 4th iterate).  The ray trace
is static geometry, done once per model before the timed region (its time is
reported as trace_ms).  value = N * R * nlines * nbins / (seconds per step),
i.e. point.ray.frequency updates per second for the whole job.

Also reported: the dominant kernel's roofline (per-launch duration from HIP
events inside the library, on the stream the kernel runs on), the
converged-model time of the FP32-bulk/FP64-solve form and of the plain FP64
form from LTE, and the CPU oracle timed on a bounded sample of origins.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("formal-solve point·ray·freq updates/s, converged-model time vs FP64 form")

# Algorithmic work of the formal solution, per element (one point of one
# ray pair for one (line, bin) lane), counted from the arithmetic the method
# needs (FMA = 2 FLOP; exp2 and reciprocal count 1 each):
#   offset x (fma + mul) 3, profile (square, exp2) 2, opacity 1, chi'*b 1,
#   trapezoid (add, 2 mul) 3, Feautrier step (2 + 1 + fma 2 + rcp 1 + 1 +
#   fma 2 + 1) 10  ->  20 FLOP
# A semi-analytic segment adds: 2 offsets (4), divided difference (sub, 2
# mul, div 4), 2 erfc (~2 x 12), opacity average (fma 2, 3 mul)  ->  ~38 FLOP.
# The origin row per (pair, lane) adds 8.
# In a model with one Doppler width everywhere an erfc value at a point is
# shared by the semi-analytic segments on both sides of it, so such a model is
# credited one erfc per semi-analytic segment (a lower bound of its unique
# work: a run of k such segments needs k + 1).
FLOP_PER_ELEMENT = 20.0
FLOP_PER_SEMI = 38.0
FLOP_PER_SEMI_ONE_WIDTH = 26.0
FLOP_PER_ORIGIN_ROW = 8.0
# A second, coarser count of the same work: one operation each for ~17
# simple vector operations, the profile exponential and two reciprocals per
# element (20), and one per erf/erfc evaluation, two per semi-analytic
# segment.
OPS_PER_ELEMENT_COARSE = 20.0
OPS_PER_SEMI_COARSE = 2.0
# Peaks: MI355X's published vector figures, FP32 157.3 TFLOP/s (256 CUs x
# 128 FP32 FMA lanes per clock x 2 FLOP x 2.4 GHz) and FP64 78.6 TFLOP/s.
# The FP32 figure is the ceiling of this build too, although it emits no
# packed FP32 instructions: its counters show wave64 FP32 VALU instructions
# retiring at more than one per four clocks per SIMD (the 39.3 T lane-op/s
# a 16-lane SIMD would allow), so the plain instructions reach the published
# rate.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", choices=["outflow", "clumpy", "shells", "batch", "serve"],
                   default="clumpy")
    p.add_argument("--no-extras", action="store_true",
                   help="default workload only: skip the outflow and serving extra keys")
    p.add_argument("--extra-serve-seconds", type=float, default=8.0)
    p.add_argument("--serve-seconds", type=float, default=20.0,
                   help="serve workload: length of the request stream")
    p.add_argument("--serve-models", type=int, default=8)
    p.add_argument("--batch-models", type=int, default=256,
                   help="models in the batch workload (the recipe's first K)")
    p.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    p.add_argument("--no-converge", action="store_true", help="skip converged-model timing")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--max-iter", type=int, default=200)
    p.add_argument("--tol", type=float, default=1e-6,
                   help="converged-model legs: relative-change tolerance of every leg")
    p.add_argument("--converge-seconds", type=float, default=240.0,
                   help="stop a converged-model leg after this long (reported)")
    p.add_argument("--ng-study", action="store_true",
                   help="classical vs adaptive Ng iteration counts on the spherical shells")
    p.add_argument("--profile-steps", action="store_true",
                   help="only warmup + timed steps (for rocprofv3 runs)")
    return p.parse_args()


def make_model(name):
    from paper_2411_03040_amd import synth
    if name == "outflow":
        m = synth.config(1)
        desc = ("3D outflow: 50000 points in r in [1,20], k=16 NN, 10-level rotor (9 lines), "
                "48 rays, 31 bins/line, v=15 km/s (1-1/r)^0.5, T=2000 r^-0.7 K")
    elif name == "clumpy":
        m = synth.config(2)
        desc = ("clumpy cloud: 200000 points, log-normal density, rotation+turbulence with "
                "shifts up to 20 widths, 20-level rotor (19 lines), 48 rays, 39 bins/line")
    else:
        m = synth.config(0)
        desc = "1D spherical shells: 64 shells, two-level species, 12 rays, 31 bins"
    return m, desc


def alu_roofline(ctx, m, ms_per_launch, precision):
    c = ctx.counters()
    lanes = m.nlines * m.nbins
    npairs = m.nrays // 2
    elements = lanes * c["total_records"]
    one_width = bool(np.ptp(m.T) == 0 and np.ptp(m.vturb2) == 0)
    per_semi = FLOP_PER_SEMI_ONE_WIDTH if one_width else FLOP_PER_SEMI
    flop = (elements * FLOP_PER_ELEMENT + lanes * c["semi_segments"] * per_semi +
            lanes * m.npoints * npairs * FLOP_PER_ORIGIN_ROW)
    ops_coarse = elements * OPS_PER_ELEMENT_COARSE + lanes * c["semi_segments"] * OPS_PER_SEMI_COARSE
    sec = ms_per_launch * 1e-3
    achieved = flop / sec / 1e12
    peak = PEAK_FP32_TFLOPS if precision == "fp32" else PEAK_FP64_TFLOPS
    # algorithmic HBM bytes of one launch: the packed trace once, the trace
    # offsets, the per-point line table (chi', S' in the solve precision)
    # and per-point widths once, J-bar and Lambda* written once (FP64)
    tsz = 4 if precision == "fp32" else 8
    rec_bytes = 24 if precision == "fp32" else 48
    alg_bytes = (c["total_records"] * rec_bytes + (m.npoints * m.nrays + 1) * 8 +
                 m.npoints * m.nlines * 2 * tsz + m.npoints * 2 * tsz +
                 m.npoints * m.nlines * 2 * 8)
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": None,
           "kernel": "k_formal_solve<%s>" % ("float" if precision == "fp32" else "double"),
           "flop_per_launch": flop, "elements_per_launch": elements,
           "semi_segments": c["semi_segments"], "one_width": one_width,
           "flop_count": "per element 20 FLOP, per semi-analytic segment and lane %d, per "
                         "origin row 8 (FMA = 2)" % per_semi,
           "coarse_count": {"ops_per_launch": ops_coarse,
                            "rule": "20 per element, 2 (the two erf/erfc) per semi-analytic "
                                    "segment and lane",
                            "achieved": round(ops_coarse / sec / 1e12, 3),
                            "frac": round(ops_coarse / sec / 1e12 / peak, 4)},
           "ms_per_launch": round(ms_per_launch, 4),
           "algorithmic_bytes_per_launch": alg_bytes,
           "hbm_GBps_algorithmic": round(alg_bytes / sec / 1e9, 1),
           "hbm_frac_algorithmic": round(alg_bytes / sec / 8e12, 5)}
    return out


def committed_traffic(workload):
    """HBM bytes per formal-solve launch from the committed rocprofv3 counter
    summary, or None when the kernel code changed since it was taken."""
    import re
    name = {"outflow": "outflow_50k", "clumpy": "clumpy_200k"}.get(workload)
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", f"formal_solve_{name}.md")
    src = os.path.join(ROOT, "paper_2411_03040_amd", "csrc", "formal_solve.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m1 = re.search(r"^code_sha256: (\w+)", text, re.M)
    m2 = re.search(r"^traffic_bytes_per_launch: ([0-9.e+-]+)", text, re.M)
    if not (m1 and m2):
        return None
    if code_sha256(src) != m1.group(1):
        return None
    return float(m2.group(1))


def code_sha256(path):
    """SHA-256 of a C/HIP source with comments removed and whitespace runs
    collapsed: a profile stays valid across comment edits, not code edits."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def converge(mgx, torch, m, precision, tol, max_iter, time_limit, ng_mode=None, ng_param=4):
    """Converged-model time from LTE, trace included: the Lambda-iteration
    with Ng (classical order 4 by default), driven step by step through the C
    ABI (the same sequence mgx_iterate runs) so progress is visible."""
    ng_mode = mgx.NG_CLASSICAL if ng_mode is None else ng_mode
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cx = mgx.Context(device=0, precision=precision)
    cx.load_model(m)
    cx.trace_rays()
    cx.set_lte_populations()
    classical = (ng_mode & 0xF) == mgx.NG_CLASSICAL
    cx.ng_reset(ng_param + 1 if classical else ng_param)
    it, ch, ok, applied = 0, float("inf"), False, 0
    while it < max_iter:
        it += 1
        cx.formal_solve(copy=False)
        ch = cx.update_populations()
        if ch <= tol:
            ok = True
            break
        applied += cx.ng_accelerate(ng_mode, ng_param)
        log(f"  converge {'fp32' if precision == mgx.FP32 else 'fp64'} ng {ng_mode}/{ng_param} "
            f"iter {it} change {ch:.3e}")
        if time.perf_counter() - t0 > time_limit:
            break
    pops = cx.get_populations()
    masing = cx.counters()["masing"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del cx
    return {"seconds": dt, "iterations": it, "final_change": ch, "converged": ok, "tol": tol,
            "seconds_per_iteration": dt / it, "ng": {"mode": int(ng_mode), "param": ng_param,
                                                   "predictions_used": applied},
            "masing_clamps_last_iteration": masing,
            "cut_at_seconds": None if ok or it >= max_iter else time_limit, "pops": pops}


def cpu_baseline(m, seconds, gpu_J=None, converged=None, tol=1e-10):
    """The oracle (all host cores) on a seeded sample of origins of the same
    model from LTE populations, as updates/s.  With the GPU's J-bar from the
    same LTE populations (gpu_J), also its largest relative error on the
    sample; with converged populations ({name: (pops, iterations)}), the
    oracle's own Lambda-iteration step from them at sampled points (how far
    they are from the oracle's fixed point) and, for the FP64 form, the
    oracle's converged-model time extrapolated from the sampled rate."""
    import oracle
    from paper_2411_03040_amd import synth
    orc = oracle.Oracle(m)
    pops = orc.lte()
    lanes = m.nlines * m.nbins
    n = 16
    t = 0.0
    while True:
        origins = synth.origin_sample(m.npoints, n, seed=99)
        t0 = time.perf_counter()
        J, _ = orc.solve_origins(pops, origins)
        t = time.perf_counter() - t0
        if t > 0.25 * seconds or n >= m.npoints:
            break
        n = min(m.npoints, int(n * max(2.0, 0.3 * seconds / max(t, 1e-3))))
    rate = n * m.nrays * lanes / t
    cores = oracle.num_threads()
    out = {"value": rate, "unit": "updates/s", "cores": cores, "kind": "oracle",
           "sample": f"formal solution (line coefficients + all rays, lines, bins) of {n} "
                     f"seeded origins of the same model from LTE populations, {t:.1f} s"}
    # the same origins' first few on one thread: the single-core rate
    n1 = max(1, min(n, int(n * 0.1 * seconds / max(t * cores, 1e-3))))
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        orc.solve_origins(pops, origins[:n1])
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    out["single_thread_value"] = n1 * m.nrays * lanes / t1
    out["single_thread_sample"] = f"the first {n1} of those origins on one thread, {t1:.1f} s"
    if gpu_J is not None:
        g = np.asarray(gpu_J)[origins]
        out["gpu_Jbar_max_rel_err"] = float(np.max(np.abs(g - J) / np.abs(J)))
    for name, (p, iters, done) in (converged or {}).items():
        sub = synth.origin_sample(m.npoints, 48, seed=98)
        Jc, Lc = orc.solve_origins(p, sub)
        _, _, Sc, _ = orc.line_coeffs(p)
        res = 0.0
        for k, o in enumerate(sub):
            _, new = orc.stateq_point(int(o), Jc[k], Lc[k], Sc[o])
            res = max(res, float(np.max(np.abs(new - p[o]) / np.maximum(p[o], 1e-12))))
        out[f"{name}_pops_oracle_step_max_rel"] = res
        out[f"{name}_pops_oracle_step_points"] = int(sub.size)
        if name == "fp64":
            per_iter = m.npoints * m.nrays * lanes / rate
            if per_iter * iters < 0.5 * seconds:
                # small enough: the oracle converges the model itself (same
                # tolerance and Ng schedule as the FP64 GPU form)
                t0 = time.perf_counter()
                r = orc.iterate(tol=tol, max_iter=2000, ng_mode=1, ng_param=4)
                out["oracle_converged_seconds"] = time.perf_counter() - t0
                out["oracle_converged_iterations"] = r["iters"]
                out["fp64_pops_max_rel_vs_oracle"] = float(
                    np.max(np.abs(p - r["pops"]) / np.maximum(r["pops"], 1e-12)))
            else:
                out["oracle_converged_seconds_extrapolated"] = per_iter * iters
                out["oracle_converged_note"] = (
                    f"{iters} iterations (those of the FP64 GPU form) x {per_iter:.1f} s per "
                    "iteration at the sampled rate" + (
                        "" if done else "; a lower bound: the FP64 GPU form had not converged "
                        "within the benchmark's time cap"))
    return out


def ng_study(mgx, torch):
    """Iterations to converge with no Ng, classical Ng of N_steps and adaptive
    Ng with N_max, each also with the restart reading in which a prediction
    starts the history afresh (NG_FRESH): on the two spherical variants
    (moderate and high optical depth; FP64 to 1e-10) and on the clumpy cloud
    (FP32-bulk to 1e-6; its plain iteration does not converge): the
    comparison of the paper's Ng section."""
    from paper_2411_03040_amd import synth
    res = {}
    modes = ([("none", mgx.NG_NONE, 0)] +
             [(f"classical_{n}", mgx.NG_CLASSICAL, n) for n in (2, 3, 4, 8)] +
             [(f"adaptive_{n}", mgx.NG_ADAPTIVE, n) for n in (4, 8, 16, 32)] +
             [("classical_4_fresh", mgx.NG_CLASSICAL | mgx.NG_FRESH, 4)] +
             [(f"adaptive_{n}_fresh", mgx.NG_ADAPTIVE | mgx.NG_FRESH, n) for n in (8, 32)])
    cases = [(f"shells_{v}", synth.spherical_shells(v), mgx.FP64, 1e-10, 2000, modes) for v in ("a", "b")]
    cases.append(("clumpy_fp32_bulk", synth.config(2), mgx.FP32, 1e-6, 300,
                  [m for m in modes if m[0] in ("classical_4", "adaptive_8", "adaptive_32",
                                                 "classical_4_fresh", "adaptive_8_fresh",
                                                 "adaptive_32_fresh")]))
    for name, m, prec, tol, max_iter, case_modes in cases:
        row = {}
        for label, mode, param in case_modes:
            cx = mgx.Context(device=0, precision=prec)
            cx.load_model(m)
            cx.trace_rays()
            cx.set_lte_populations()
            t0 = time.perf_counter()
            it, ch, ok = cx.iterate(tol=tol, max_iter=max_iter, ng_mode=mode,
                                    ng_param=param if mode else 4, raise_on_noconv=False)
            dt = time.perf_counter() - t0
            c = cx.counters()
            row[label] = {"iterations": it, "converged": ok, "ng_applied": c["ng_applied"],
                          "seconds": dt}
            log(f"  ng-study {name} {label}: {it} iterations, {dt:.2f} s")
            del cx
        res[name] = {"tol": tol, "precision": "fp64" if prec == mgx.FP64 else "fp32 bulk",
                     "modes": row}
    return res


def bench_batch(args, mgx, torch):
    """Many uneven models iterated together: a step is one iteration of every
    model (three graph replays: line coefficients, formal solution, statistical
    equilibrium), all models active; then the whole batch converged from LTE."""
    from paper_2411_03040_amd import synth
    t0 = time.perf_counter()
    spec = synth.batch_spec(args.batch_models)
    prec = mgx.FP32 if args.precision == "fp32" else mgx.FP64
    b = mgx.Batch(device=0, precision=prec)
    for i, kw in enumerate(spec):
        b.add_model(synth.outflow_3d(**kw))
        if i % 32 == 31:
            log(f"bench batch: {i + 1} models generated and loaded")
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b.prepare()
    prep_s = time.perf_counter() - t0
    log(f"bench batch: traced and prepared in {prep_s:.1f} s")
    b.set_lte_populations()
    b.iterate(tol=0.0, max_iter=max(1, args.warmup), raise_on_noconv=False)
    log("bench batch: tuned, captured, warmed up")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.iterate(tol=0.0, max_iter=args.steps, raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = b.stats()
    ms_step = dt / args.steps * 1e3
    fs_ms = st["fs_ms_total"] / max(st["fs_launches"], 1)
    upd = st["updates_per_iteration"]
    value = upd / (ms_step * 1e-3)
    flop = (st["lane_records"] * FLOP_PER_ELEMENT + st["lane_semi"] * FLOP_PER_SEMI +
            st["lane_origin_pairs"] * FLOP_PER_ORIGIN_ROW)
    peak = PEAK_FP32_TFLOPS if prec == mgx.FP32 else PEAK_FP64_TFLOPS
    achieved = flop / (fs_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "kernel": "k_formal_solve_batch (all lane classes of one iteration)",
            "flop_per_launch": flop, "ms_per_launch": round(fs_ms, 4)}
    log(f"bench batch: {ms_step:.1f} ms/step, formal solution {fs_ms:.1f} ms")
    # converged from LTE (FP32-bulk formal solution, FP64 statistical
    # equilibrium, classical Ng of order 4), each model stopping on its own
    b.set_lte_populations()
    tol = 1e-6 if prec == mgx.FP32 else 1e-10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, chg, nconv = b.iterate(tol=tol, max_iter=args.max_iter, ng_order=4,
                                raise_on_noconv=False)
    torch.cuda.synchronize()
    conv_s = time.perf_counter() - t0
    log(f"bench batch: converged {nconv}/{len(spec)} in {conv_s:.1f} s")
    stuck = [{"model": i, "npoints": spec[i]["npoints"], "levels": spec[i]["nlev"],
              "rays": 12 if spec[i]["nside"] == 1 else 48, "last_change": float(chg[i])}
             for i in range(len(spec)) if not chg[i] <= tol]
    npts = [kw["npoints"] for kw in spec]
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == mgx.FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(spec)} outflow models: points log-uniform "
                               f"1e3-1e5 (total {sum(npts)}), 2-20 levels, 12 or 48 rays, "
                               "31 bins/line",
                   "models": len(spec), "total_points": int(sum(npts)),
                   "formal_solve": args.precision, "stateq": "f64", "ng": "classical order 4"},
        "formal_solve_ms": fs_ms, "updates_per_step": upd,
        "schedule": {"lane_classes": st["lane_classes"], "work_items": st["work_items"],
                     "tune_seconds": st["tune_seconds"],
                     "classes": [{"threads": st["class_threads"][k],
                                  "items": st["class_items"][k],
                                  "chunk": st["class_chunk"][k],
                                  "order": ("by model and Morton origin" if st["class_order"][k]
                                            else "longest first")}
                                 for k in range(16) if st["class_items"][k]]},
        "generate_seconds": gen_s, "prepare_seconds": prep_s,
        "converged": {"seconds": conv_s, "models_converged": nconv, "tol": tol,
                      "seconds_to_last_converged": b.stats()["last_converged_seconds"],
                      "replays": int(its.max()), "iterations_median": float(np.median(its)),
                      "iterations_max": int(its.max()), "not_converged": stuck},
        "roofline": roof,
    }
    if not args.no_cpu:
        # the oracle on a sample of origins of one mid-sized model of the batch
        j = int(np.argsort(npts)[len(npts) // 2])
        log(f"bench batch: CPU oracle baseline on model {j}")
        out["cpu_baseline"] = cpu_baseline(synth.outflow_3d(**spec[j]), args.cpu_seconds)
        out["cpu_baseline"]["sample"] += f" (batch model {j}, {npts[j]} points)"
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_serve(args, mgx, torch, models=None, seconds=None, emit=True):
    """A Poisson stream of requests (mean 50/s) on resident models: 98 %
    renders (256 x 256 pixels x 63 bins around a line, random model and
    inclination), 2 % converges from LTE (random model, FP32 formal solution,
    tol 1e-6, Ng order 4).  Reports latency percentiles per kind and the
    formal-solution updates/s the server sustained."""
    from paper_2411_03040_amd import synth
    spec = synth.serve_spec(args.serve_models if models is None else models)
    srv = mgx.Server(device=0, precision=mgx.FP32, render_slots=2)
    t0 = time.perf_counter()
    models = []
    for i, kw in enumerate(spec):
        m = synth.outflow_3d(**kw)
        srv.add_model(m)
        models.append(m)
        log(f"bench serve: model {i} ({m.npoints} points, {m.nlev} levels) loaded")
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    srv.start()
    start_s = time.perf_counter() - t0
    st0 = srv.stats()
    log(f"bench serve: started in {start_s:.1f} s, resident {st0['hbm_resident'] / 1e9:.1f} GB")
    rng = np.random.default_rng(11)
    rate, T = 50.0, args.serve_seconds if seconds is None else seconds
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * T * 2)))
    arrivals = arrivals[arrivals < T]
    kinds = np.where(rng.random(arrivals.size) < 0.02, 0, 1)
    which = rng.integers(0, len(models), arrivals.size)
    th = np.arccos(rng.uniform(-1, 1, arrivals.size))
    ph = rng.uniform(0, 2 * np.pi, arrivals.size)
    ids = []
    c0 = srv.clock()
    w0 = time.perf_counter()
    for k, ta in enumerate(arrivals):
        dt = ta - (time.perf_counter() - w0)
        if dt > 0:
            time.sleep(dt)
        j = int(which[k])
        m = models[j]
        if kinds[k] == 0:
            ids.append(srv.submit_converge(j, tol=1e-6, max_iter=200, ng_order=4))
        else:
            nu = m.nu[min(1, m.nlines - 1)]
            d = (np.sin(th[k]) * np.cos(ph[k]), np.sin(th[k]) * np.sin(ph[k]), np.cos(th[k]))
            ids.append(srv.submit_render(j, d, 256, 256, nu * (1 - 5e-5), nu * (1 + 5e-5), 63))
        if k % 200 == 199:
            log(f"bench serve: {k + 1} requests submitted")
    infos = []
    for rid in ids:
        infos.append(srv.wait(rid, timeout=600, raise_on_error=False))
        infos[-1].pop("image", None)
    wall = srv.clock() - c0
    st = srv.stats()
    log(f"bench serve: {len(infos)} requests done in {wall:.1f} s")

    def pct(v, q):
        return float(np.percentile(v, q)) if len(v) else None

    res = {}
    for name, kind in (("converge", 0), ("render", 1)):
        lat = [i["t_done"] - i["t_submit"] for i in infos if i["kind"] == kind and i["status"] == 0]
        svc = [i["t_done"] - i["t_start"] for i in infos if i["kind"] == kind and i["status"] == 0]
        res[name] = {"requests": int(sum(1 for i in infos if i["kind"] == kind)),
                     "ok": len(lat), "latency_p50_s": pct(lat, 50), "latency_p99_s": pct(lat, 99),
                     "service_p50_s": pct(svc, 50), "service_p99_s": pct(svc, 99)}
    res["converge"]["iterations_median"] = float(np.median(
        [i["iterations"] for i in infos if i["kind"] == 0] or [0]))
    upd = st["updates"] - st0["updates"]
    out = {
        "metric": METRIC, "value": upd / wall, "unit": "updates/s", "n_gpus": 1,
        "steps": len(infos), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving: Poisson 50 req/s for {T:.0f} s on {len(models)} resident "
                               "outflow models (points log-uniform 1e4-1e6, 5-20 levels, 12 rays, "
                               "31 bins); 98% renders 256x256x63, 2% converges from LTE",
                   "models": [{"npoints": m.npoints, "levels": m.nlev} for m in models]},
        "requests": len(infos), "request_rate_per_s": len(infos) / wall, "wall_s": wall,
        "latency": res, "replays": st["replays"] - st0["replays"],
        "iterate_busy_s": st["iterate_busy_s"], "render_busy_s": st["render_busy_s"],
        "hbm": {"budget": st["hbm_budget"], "resident": st["hbm_resident"],
                "render_peak": st["hbm_render_peak"]},
        "generate_seconds": gen_s, "start_seconds": start_s,
        "roofline": None, "cpu_baseline": None,
    }
    srv.close()
    if not emit:
        return {k: out[k] for k in ("value", "config", "requests", "request_rate_per_s", "wall_s",
                                    "latency", "replays", "iterate_busy_s", "render_busy_s",
                                    "hbm", "start_seconds")}
    print(json.dumps(out), flush=True)


def bench_single(args, mgx, torch, workload, steps, warmup, converge_legs, cpu, render):
    """One model: a step is one Lambda-iteration (line coefficients, formal
    solution, statistical equilibrium, convergence measure, Ng decision)."""
    m, desc = make_model(workload)
    prec = mgx.FP32 if args.precision == "fp32" else mgx.FP64
    ctx = mgx.Context(device=0, precision=prec)
    ctx.load_model(m)
    log(f"bench: model {m.name} loaded")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.trace_rays()
    torch.cuda.synchronize()
    trace_ms = (time.perf_counter() - t0) * 1e3
    ctx.set_lte_populations()
    ng_order = 4
    ctx.ng_reset(ng_order + 1)

    def step():
        ctx.formal_solve(copy=False)
        ctx.update_populations()
        ctx.ng_accelerate(mgx.NG_CLASSICAL, ng_order)

    for _ in range(warmup):
        step()
    log(f"bench: {workload} warmup done")
    ctx.reset_timers()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / steps * 1e3
    c = ctx.counters()
    fs_ms = c["fs_ms_total"] / max(c["fs_launches"], 1)
    updates = m.npoints * m.nrays * m.nlines * m.nbins
    value = updates / (ms_step * 1e-3)
    log(f"bench: {workload} {ms_step:.2f} ms/step, formal solution {fs_ms:.2f} ms")
    # the formal solution alone (line coefficients excluded, trace cached):
    # median of per-launch event times over 10 more steps, outside the timing
    fs_each = []
    for _ in range(10):
        step()
        fs_each.append(ctx.counters()["fs_ms_last"])
    fs_median = float(np.median(fs_each))
    if args.profile_steps:
        # calibration for hardware byte counters: a plain elementwise kernel
        # that reads 256 MiB and writes 256 MiB (larger than every cache level
        # up to the L2s; run right after a fill of a different buffer)
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        flush = torch.zeros(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del flush
        return {"ms_per_step": ms_step, "fs_ms": fs_ms, "value": value,
                "copy_calibration_bytes": src.numel() * 4}
    rend = None
    if render and m.dim == 3:
        # synthetic image as the serving workload asks for it: 256 x 256
        # pixels x 63 bins around the second line at a seeded inclination
        rng = np.random.default_rng(7)
        th = rng.uniform(0, np.pi)
        view = [np.sin(th), 0.0, np.cos(th)]
        nu_r = m.nu[min(1, m.nlines - 1)]
        ctx.render_image(view, 256, 256, nu_r * (1 - 5e-5), nu_r * (1 + 5e-5), 63)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nrep = 3
        for _ in range(nrep):
            ctx.render_image(view, 256, 256, nu_r * (1 - 5e-5), nu_r * (1 + 5e-5), 63)
        torch.cuda.synchronize()
        render_ms = (time.perf_counter() - t0) / nrep * 1e3
        rend = {"pixels": 256 * 256, "bins": 63, "ms": render_ms,
                "pixel_bins_per_s": 256 * 256 * 63 / (render_ms * 1e-3),
                "includes": "line coefficients, pixel entry search, walks, integration, "
                            "copy of the float image to the host"}
    roof = alu_roofline(ctx, m, fs_ms, args.precision)
    if args.precision == "fp32":
        roof["traffic"] = committed_traffic(workload)
        if roof["traffic"]:
            roof["hbm_GBps_measured"] = round(roof["traffic"] / (fs_ms * 1e-3) / 1e9, 1)
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == mgx.FP32 else "f64", "data": "synthetic",
        "config": {"workload": desc, "npoints": m.npoints, "rays": m.nrays,
                   "lines": m.nlines, "bins": m.nbins, "levels": m.nlev,
                   "formal_solve": args.precision, "stateq": "f64", "ng": "classical order 4"},
        "formal_solve_ms": fs_ms, "trace_ms": trace_ms,
        "render": rend,
        "ray_pair_solves_per_s": value / 2.0,
        "formal_solve_only": {"ms_median": fs_median,
                              "updates_per_s": updates / (fs_median * 1e-3),
                              "ray_pair_solves_per_s": updates / (fs_median * 1e-3) / 2.0},
        "roofline": roof,
    }
    del ctx
    conv_pops = None
    if converge_legs:
        conv = {}
        legs = [("fp32_bulk", mgx.FP32, mgx.NG_CLASSICAL, 4), ("fp64", mgx.FP64, mgx.NG_CLASSICAL, 4)]
        if workload == "clumpy":
            legs.insert(1, ("fp32_bulk_adaptive", mgx.FP32, mgx.NG_ADAPTIVE | mgx.NG_FRESH, 8))
        # every leg to the same tolerance (the FP32-bulk form's), so the
        # converged-model times compare like for like
        for name, p, mode, param in legs:
            tol = args.tol
            r = converge(mgx, torch, m, p, tol, max_iter=args.max_iter,
                         time_limit=args.converge_seconds, ng_mode=mode, ng_param=param)
            conv[name] = r
        pops = {k: v.pop("pops") for k, v in conv.items()}
        a, b = pops["fp32_bulk"], pops["fp64"]
        conv_pops = {k: (pops[k], conv[k]["iterations"], conv[k]["converged"])
                     for k in ("fp32_bulk", "fp64")}
        conv["fp32_vs_fp64_pops_max_rel"] = float(np.max(np.abs(a - b) / np.maximum(b, 1e-12)))
        conv["fp32_vs_fp64_compares"] = ("two converged states" if conv["fp64"]["converged"]
                                         else "FP64 state cut before convergence")
        conv["speedup_fp32_bulk_over_fp64_per_iteration"] = (
            conv["fp64"]["seconds_per_iteration"] / conv["fp32_bulk"]["seconds_per_iteration"])
        conv["speedup_fp32_bulk_over_fp64_converged"] = (
            conv["fp64"]["seconds"] / conv["fp32_bulk"]["seconds"])
        out["converged"] = conv
    if cpu:
        log(f"bench: {workload} CPU oracle baseline")
        cx = mgx.Context(device=0, precision=prec)
        cx.load_model(m)
        cx.trace_rays()
        cx.set_lte_populations()
        gpu_J, _ = cx.formal_solve()
        del cx
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_seconds, gpu_J=gpu_J, converged=conv_pops,
                                           tol=args.tol)
    else:
        out["cpu_baseline"] = None
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2411_03040_amd import mgx

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.ng_study:
        print(json.dumps({"ng_study": ng_study(mgx, torch)}), flush=True)
        return
    if args.workload == "batch":
        bench_batch(args, mgx, torch)
        return
    if args.workload == "serve":
        bench_serve(args, mgx, torch)
        return
    out = bench_single(args, mgx, torch, args.workload, args.steps, args.warmup,
                       converge_legs=not args.no_converge, cpu=not args.no_cpu,
                       render=True)
    if args.profile_steps:
        print(json.dumps(out), flush=True)
        return
    if args.workload == "clumpy" and not args.no_extras:
        # the 3D outflow: timed steps and the kernel roofline only
        o = bench_single(args, mgx, torch, "outflow", args.steps, args.warmup,
                         converge_legs=False, cpu=False, render=False)
        out["outflow"] = {k: o[k] for k in ("value", "ms_per_step", "formal_solve_ms",
                                            "config", "roofline", "trace_ms",
                                            "formal_solve_only")}
        # a short serving run: p50/p99 latency of converge and render requests
        out["serving"] = bench_serve(args, mgx, torch, models=3,
                                     seconds=args.extra_serve_seconds, emit=False)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
