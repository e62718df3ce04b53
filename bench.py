"""Benchmark of the flood GaBP hot path on one MI355X.

Workload: the variable-coefficient upwind convection-diffusion operator on a 2048 x 2048
interior grid (4,194,304 unknowns, 20,963,328 nonzeros, 16,769,024 directed message edges),
k = exp(g) with g a 16-mode random field, rotating velocity 20(-(y-1/2), x-1/2),
b ~ U(-1,1), seeded synthetic data.

One *step* = one block of the solver's main loop: ``check_every`` (16) flood sweeps of
Algorithm 1 in FP64 (joint Lt and m update, read-off on the last one) followed by the
residual check r = b - A x with its norms. ``value`` = directed edge-message updates per
second over the timed steps (inputs resident in HBM).

Also reported on the same JSON line:
  * roofline of the dominant kernel (the joint sweep kernel; by default the tiled layout,
    two sweeps per launch, `--no-tiles` for one): algorithmic bytes per launch (one pass
    over the message state) over its average launch time from HIP events on the launch
    stream, the counted HBM bytes from the committed counter record, and the streaming
    equivalent (the bytes one-sweep launches would move for the same sweeps);
  * FP32 mean-only sweep rate (the inner kernel of FP32-message iterative refinement) and
    FP64 mean-only sweep rate with precomputed Lt;
  * time to relative residual 1e-8 on the same 2048 x 2048 operator through gabp_solve:
    by default FP32 messages + FP64 refinement with a manufactured solution (b := A x*), so
    the error of x is reported too; the FP64 variants and the workload's own b with
    --ttr-only --ttr-variants ... --ttr-rhs uniform (each takes minutes);
  * the CPU oracle timed on a bounded sample of sweeps on this host (a baseline only).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-ttr]
       python bench.py --ttr-only --ttr-variants fp64_joint,fp64_precomp,fp32_ir
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def sweep_bytes_joint64(slots, n, rb=4):
    # per slot: Lt_in, m_in, coefficient (8 B each), reverse index (rb B), Lt_out, m_out
    # (8 B each); per row: diagonal and b (8 B each)
    return (40 + rb) * slots + 16 * n


def sweep_bytes_mean32(slots, n, rb=4):
    # per slot: m_in, Lt* (FP32), reverse index (rb B), m_out; per row: FP32 rhs
    return (12 + rb) * slots + 4 * n


def sweep_bytes_mean64(slots, n, rb=4):
    # per slot: m_in, Lt* (8 B), reverse index (rb B), m_out (8 B); per row: b (8 B)
    return (24 + rb) * slots + 8 * n


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (its name with template arguments) from the committed
    counter summary, or None when that kernel was not counted or the kernel source has
    changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        entry = rec["kernels"][kernel]
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_prefix"):
        return None
    return entry["hbm_bytes_per_launch"]


def _events_time(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    fn(reps)
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=2048)
    ap.add_argument("--no-ttr", action="store_true")
    ap.add_argument("--ttr-variants", default="fp32_ir",
                    help="comma list of fp64_joint, fp64_precomp, fp32_ir (time to rel.res)")
    ap.add_argument("--ttr-rhs", default="manufactured", choices=["manufactured", "uniform"])
    ap.add_argument("--ttr-tol", type=float, default=1e-8)
    ap.add_argument("--ttr-only", action="store_true",
                    help="only the time-to-residual legs on the --grid workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tiles", action="store_true",
                    help="plain one-sweep-per-launch flood kernels instead of the tiled "
                         "two-sweep kernels")
    ap.add_argument("--cpu-sweeps", type=int, default=60)
    ap.add_argument("--profile", action="store_true",
                    help="short run for the profiler: few launches of each kernel")
    ap.add_argument("--suite", action="store_true",
                    help="also measure the multigrid, batching and adjoint configurations")
    ap.add_argument("--suite-only", action="store_true")
    ap.add_argument("--suite-part", default="all",
                    choices=["all", "small", "batch", "batch_full", "mg", "mg_c4", "mg_profile",
                             "sweeps_large",
                             "adjoint", "adjoint_full", "lines", "sec5", "colours"],
                    help="with --suite-only: run one part of the suite")
    ap.add_argument("--line-sweeps", type=int, default=50,
                    help="timed sweeps per variant in the line-sweep part")
    args = ap.parse_args()
    ttr_variants = tuple(v for v in args.ttr_variants.split(",") if v)
    if any(v not in TTR_VARIANTS for v in ttr_variants):
        ap.error(f"--ttr-variants: choose from {sorted(TTR_VARIANTS)}")
    if args.ttr_only:
        import torch  # noqa: F401
        lg = lambda *a: print(*a, file=sys.stderr, flush=True)
        print(json.dumps(time_to_residual(args.grid, lg, ttr_variants, args.ttr_rhs,
                                          args.ttr_tol, tiles=not args.no_tiles)), flush=True)
        return
    if args.suite_only:
        import torch  # noqa: F401
        print(json.dumps(suite(lambda *a: print(*a, file=sys.stderr, flush=True),
                               part=args.suite_part, line_sweeps=args.line_sweeps)),
              flush=True)
        return
    if args.profile:
        args.steps, args.warmup, args.no_ttr, args.no_cpu = 5, 1, True, True
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has "
              "no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W

    torch.cuda.set_device(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    n = args.grid
    t0 = time.time()
    a, b = W.precision_at_scale(n)
    log(f"[bench] generated {n}x{n} operator: N={a.n} nnz={a.nnz} ({time.time()-t0:.1f}s)")
    edges = a.nnz - a.n
    CE = 16
    t0 = time.time()
    tiles = not args.no_tiles
    tkw = dict(tiles=True, grid=(n, n)) if tiles else {}
    sj = gabp.Solver.from_csr(a, mode="joint", check_every=CE, **tkw)
    lay = sj.layout_info()
    log(f"[bench] setup {time.time()-t0:.1f}s layout {lay}")
    # streaming hints by measurement (the library's autotuner, as a user would call it)
    tuned = sj.autotune()
    log(f"[bench] autotuned {tuned}")
    bt = torch.as_tensor(b).cuda()
    x = torch.zeros(a.n, dtype=torch.float64, device="cuda")

    def step(k):
        for _ in range(k):
            sj.sweeps(bt, CE, reset=False, x=x)
            sj.residual(bt, x, want_r=False)

    sj.sweeps(bt, 1, reset=True, x=x)
    step(args.warmup)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    t_gpu = _events_time(step, args.steps)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - tw
    ms_step = 1e3 * t_gpu / args.steps
    value = edges * CE * args.steps / t_gpu
    log(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step, {value/1e9:.2f} G edge-upd/s")

    # attainable bandwidth: plain 16-byte-vector copy of 1 GiB
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    gabp.copy_probe(src, dst)
    NC = 3 if args.profile else 10
    # best of three rounds: the attainable ceiling, not a clock-ramp sample
    t_cp = min(_events_time(lambda k: [gabp.copy_probe(src, dst) for _ in range(k)], NC) / NC
               for _ in range(1 if args.profile else 3))
    copy_gbs = 2 * src.numel() * 8 / t_cp / 1e9
    del src, dst
    log(f"[bench] copy probe: {copy_gbs:.0f} GB/s (read + write of 1 GiB)")

    # dominant kernel: the joint FP64 sweep kernel, back-to-back launches on the launch
    # stream; tiled, one launch does two sweeps and moves the message state once, so its
    # algorithmic bytes are one pass over the state (int32 reverse index)
    NS = 20 if args.profile else 200
    sweeps_only = lambda k: sj.sweeps(bt, k, reset=False, x=x)
    sweeps_only(20)
    t_all = _events_time(sweeps_only, NS)
    per_launch = 2 if tiles else 1
    t_launch = t_all / (NS // per_launch)
    t_sw = t_all / NS
    rb = 4 if tiles else lay["rev_bytes"]
    ab = sweep_bytes_joint64(lay["slots"], a.n, rb)
    achieved = ab / t_launch / 1e9
    nt = "true" if tuned["stream_hints"] else "false"
    kname = (f"k_joint2<0, {tuned['stream_hints']}, false>" if tiles
             else f"k_joint<4, 0, {nt}, {'true' if rb == 2 else 'false'}, false>")
    log(f"[bench] joint sweep kernel {t_launch*1e6:.1f} us per launch ({per_launch} sweeps), "
        f"{achieved:.0f} GB/s algorithmic")

    # residual kernel and its norm reduction, without the host readback: 20 calls recorded
    # in a graph and replayed, so that host launch gaps between the calls are not timed
    sj.residual(bt, x, want_r=False, want_norms=False)
    torch.cuda.synchronize()
    res_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(res_graph):
        for _ in range(20):
            sj.residual(bt, x, want_r=False, want_norms=False)
    res_graph.replay()
    t_res = _events_time(lambda k: [res_graph.replay() for _ in range(k)], 5) / 100

    # FP32 mean-only sweep and FP64 mean-only sweep with precomputed Lt
    s32 = gabp.Solver.from_csr(a, mode="precomp", precision="f32_ir", check_every=CE,
                               tol_lambda=1e-7, **tkw)
    lsw = s32.precompute_lambda()
    sp = gabp.Solver.from_csr(a, mode="precomp", check_every=CE, tol_lambda=1e-12, **tkw)
    lsw64 = sp.precompute_lambda()
    s32.autotune()
    sp.autotune()
    sp.sweeps(bt, 1, reset=True, x=x)
    t_m64 = _events_time(lambda k: sp.sweeps(bt, k, reset=False, x=x), NS) / NS
    # FP32 mean-only sweeps (the inner kernel of iterative refinement): the call also casts
    # b and widens x once, removed by differencing two sweep counts
    x32 = torch.zeros_like(x)
    s32.sweeps(bt, 2, reset=True, x=x32)
    t_a = _events_time(lambda k: s32.sweeps(bt, NS + 1, reset=False, x=x32), 1)
    t_b = _events_time(lambda k: s32.sweeps(bt, 1, reset=False, x=x32), 1)
    t_m32 = (t_a - t_b) / NS
    log(f"[bench] mean sweeps: FP64 {t_m64*1e6:.1f} us, FP32 {t_m32*1e6:.1f} us "
        f"(Lt phase {lsw} / {lsw64} sweeps)")

    out = {
        "metric": "edge-msg updates/s, HBM GB/s; time to rel.res 1e-8: FP32+refine vs FP64",
        "value": value,
        "unit": "edge-msg updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"upwind convection-diffusion {n}x{n}, variable k=exp(g), "
                               "rotating v, FP64 joint flood GaBP, 16 sweeps + residual check per step"
                               + (" (two sweeps per launch over 13x64 tiles)" if tiles else ""),
                   "unknowns": a.n, "nnz": a.nnz, "directed_edges": edges,
                   "sweeps_per_step": CE, "tiles": tiles,
                   "stream_hints": tuned["stream_hints"]},
        "roofline": {"bound": "hbm",
                     "kernel": kname + (" (two FP64 joint flood sweeps per launch, tiled)"
                                        if tiles else " (FP64 joint flood sweep)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(kname),
                     "frac_of_copy": achieved / copy_gbs,
                     "algorithmic_bytes_per_launch": ab, "launch_us": t_launch * 1e6,
                     "sweeps_per_launch": per_launch, "reverse_index_bytes": rb,
                     # the bytes one-sweep launches would stream for this launch's work
                     # (2-byte reverse deltas), over this launch's time: above 1 of the
                     # peak means the launch did more work than streaming allows
                     "streaming_equivalent_GBs": per_launch * sweep_bytes_joint64(
                         lay["slots"], a.n, 2) / t_launch / 1e9},
        "wall_s_timed": t_wall,
        "kernels": {
            "joint_f64_sweep_us": t_sw * 1e6,
            "joint_f64_edge_updates_per_s": edges / t_sw,
            "mean_f64_sweep_us": t_m64 * 1e6,
            "mean_f64_edge_updates_per_s": edges / t_m64,
            "mean_f64_GBs": sweep_bytes_mean64(lay["slots"], a.n, rb) / (per_launch * t_m64) / 1e9,
            "mean_f32_sweep_us": t_m32 * 1e6,
            "mean_f32_edge_updates_per_s": edges / t_m32,
            "mean_f32_GBs": sweep_bytes_mean32(lay["slots"], a.n, rb) / (per_launch * t_m32) / 1e9,
            "sweeps_per_launch": per_launch,
            "GBs_note": "algorithmic bytes of one pass over the message state per launch "
                        "(a launch does sweeps_per_launch sweeps)",
            "residual_us": t_res * 1e6,
            "residual_GBs": (12 * lay["slots"] + 32 * a.n) / t_res / 1e9,
            "residual_note": "one residual check: k_residual and the single-block norm "
                             "reduction k_finalize_norms, replayed from a graph; GB/s are "
                             "k_residual's bytes over both",
            "copy_probe_GBs": copy_gbs,
            "lambda_phase_sweeps_f32": lsw, "lambda_phase_sweeps_f64": lsw64,
        },
    }
    del s32, sp

    if not args.no_ttr:
        out["time_to_rel_res"] = time_to_residual(n, log, ttr_variants, args.ttr_rhs,
                                                  args.ttr_tol, ab=(a, b), tiles=tiles)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a, b, args.cpu_sweeps, log)
    if args.suite:
        out["suite"] = suite(log)
    print(json.dumps(out), flush=True)


TTR_VARIANTS = {"fp64_joint": dict(mode="joint"),
                "fp64_precomp": dict(mode="precomp", tol_lambda=1e-12),
                "fp32_ir": dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)}


def time_to_residual(n, log, variants=("fp32_ir",), rhs="manufactured", tol=1e-8, ab=None,
                     tiles=True):
    """Time to ||b - A x||_2 / ||b||_2 <= tol on the n x n workload, each variant one
    gabp_solve call (Lt phase included in the time; autotuning before it is not).

    rhs "manufactured": b := A x* with a smooth manufactured x* (the workload's operator,
    x* a 16-mode random field), so the error of x is reported; rhs "uniform": the
    workload's own b ~ U(-1,1) (no reference solution at this size, no x error)."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    a, b = W.precision_at_scale(n) if ab is None else ab
    xstar = None
    if rhs == "manufactured":
        xstar, b = W.manufactured_solution(a, n)
    bt = torch.as_tensor(b).cuda()
    res = {"grid": n, "unknowns": a.n, "tol": tol, "rhs": rhs, "tiles": tiles,
           "entry_point": "gabp_solve (one call per variant)"}
    for name in variants:
        kw = TTR_VARIANTS[name]
        s = gabp.Solver.from_csr(a, progress_s=30.0,
                                 **(dict(tiles=True, grid=(n, n)) if tiles else {}), **kw)
        tuned = s.autotune()             # hints and check interval by measurement
        torch.cuda.synchronize()
        log(f"[ttr] {name} {n}x{n} rhs={rhs} tol={tol:g}: solving ({tuned})")
        t0 = time.perf_counter()
        lsw = s.precompute_lambda() if kw["mode"] == "precomp" else 0   # timed: Lt phase
        x, info = s.solve(bt, tol, 2_000_000_000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        entry = {"seconds": dt, "sweeps": info.sweeps, "lambda_sweeps": lsw,
                 "outer_iters": info.outer_iters, "rel_res2": info.rel_res2,
                 "res_inf": info.res_inf, "status": info.status, "autotuned": tuned}
        if xstar is not None:
            xe = x.cpu().numpy()
            entry["x_rel_err"] = float(np.linalg.norm(xe - xstar) / np.linalg.norm(xstar))
            entry["x_max_rel_err"] = float(np.abs(xe - xstar).max() / np.abs(xstar).max())
        res[name] = entry
        log(f"[ttr] {name}: {json.dumps(entry)}")
        del s
    if "fp64_joint" in res and "fp32_ir" in res:
        res["speedup_fp32_ir_vs_fp64_joint"] = res["fp64_joint"]["seconds"] / res["fp32_ir"]["seconds"]
    if "fp64_precomp" in res and "fp32_ir" in res:
        res["speedup_fp32_ir_vs_fp64_precomp"] = (res["fp64_precomp"]["seconds"] /
                                                  res["fp32_ir"]["seconds"])
    return res


def cpu_baseline(a, b, sweeps, log):
    """The FP64 oracle, as it stands, on this host: ``sweeps`` flood sweeps of the full grid."""
    from oracle import gabp as G
    t0 = time.perf_counter()
    g = G.Graph.from_csr(a)
    t_build = time.perf_counter() - t0
    Lt = np.zeros(g.E)
    m = np.zeros(g.E)
    t0 = time.perf_counter()
    for _ in range(sweeps):
        _, Lt, m, _, _ = G.sweep(g, b, Lt, m)
    t = time.perf_counter() - t0
    rate = g.E * sweeps / t
    log(f"[bench] cpu oracle: {t/sweeps:.3f} s/sweep, {rate/1e6:.1f} M edge-upd/s")
    return {"value": rate, "unit": "edge-msg updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} FP64 joint flood sweeps of the full {int(np.sqrt(a.n))}^2 grid "
                      f"(numpy, single-threaded; graph build {t_build:.1f}s excluded)",
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def suite(log, part="all", line_sweeps=50):
    """Measurements of the other configurations (sizes stated in each entry)."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    res = {}
    if part != "all":
        fn = {"small": lambda: suite_small(log), "batch": lambda: suite_batch(log),
              "batch_full": lambda: suite_batch(log, full_only=True),
              "mg": lambda: suite_mg(log),
              "mg_c4": lambda: suite_mg(log, problems=("anisotropic_peclet4",),
                                        smoothers=("redblack_gabp_f32_seq_lambda_2_2",
                                                   "redblack_gabp_f64_seq_lambda_2_2"),
                                        cap=100),
              "adjoint": lambda: suite_adjoint(log),
              "adjoint_full": lambda: suite_adjoint_full(log),
              "mg_profile": lambda: suite_mg_profile(log),
              "sweeps_large": lambda: suite_sweeps_large(log),
              "lines": lambda: suite_lines(log, sweeps=line_sweeps),
              "sec5": lambda: suite_sec5(log), "colours": lambda: suite_colours(log)}[part]
        res[part] = fn()
        return res
    res["small_32x32_fp64"] = suite_small(log)
    res["batch"] = suite_batch(log)
    res["multigrid"] = suite_mg(log)
    res["lines"] = suite_lines(log, sweeps=line_sweeps)
    res["sec5"] = suite_sec5(log)
    res["colours"] = suite_colours(log)
    res["adjoint"] = suite_adjoint(log)
    return res


def _sec5_printed():
    """V-cycle counts printed in the paper's Sec. 5 tables (tests/golden/sec5_iterations.txt)."""
    out = []
    for line in open(os.path.join(ROOT, "tests", "golden", "sec5_iterations.txt")):
        f = line.split("#")[0].split()
        if not f:
            continue
        kw = {k: float(v) if ("." in v or "e" in v) else int(v)
              for k, v in (p.split("=") for p in f[1].split(","))}
        nu = (2, 2) if f[3] == "any" else (int(f[3]), int(f[4]))
        out.append((f[0], kw, f[1], f[2], nu, None if f[-2] == "div" else int(f[-2])))
    return out


def suite_sec5(log, cap=100):
    """The paper's Sec. 5 multigrid problems on the 63 x 63 grid: V-cycles (down to one point)
    until ||r||_inf <= 2e-4, next to the counts the paper prints."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    smoothers = {"redblack_gabp": ("gabp", dict(mode="joint", schedule="redblack")),
                 "colour4_gabp": ("gabp", dict(mode="joint", schedule="redblack")),
                 "line_gabp": ("gabp", dict(mode="joint", schedule="lines_alt")),
                 "redblack_gs": ("rbgs", dict())}
    rows = []
    for prob, kw, pname, smoother, nu, printed in _sec5_printed():
        levels, b = W.sec5_hierarchy(prob, 6, 1, **kw)
        sides = [int(round(np.sqrt(a.n))) for a in levels]
        sm, skw = smoothers[smoother]
        lines = skw.get("schedule", "").startswith("lines")
        colouring = W.grid_colouring4 if smoother == "colour4_gabp" else W.grid_colouring
        solvers = [gabp.Solver.from_csr(a, colour=None if lines else colouring(sd),
                                        grid=(sd, sd) if lines else None, **skw)
                   for a, sd in zip(levels, sides)]
        mg = gabp.Multigrid(solvers, sides, smoother=sm, nu1=nu[0], nu2=nu[1])
        bt = torch.as_tensor(b).cuda()
        x = torch.zeros(levels[0].n, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        ours, rinf = None, float("nan")
        for k in range(1, cap + 1):
            mg.vcycle(bt, x)
            _, (_, rinf, _) = solvers[0].residual(bt, x, want_r=False)
            if not np.isfinite(rinf) or rinf > 1e30:
                break
            if rinf <= 2e-4:
                ours = k
                break
        dt = time.perf_counter() - t0
        rec = {"problem": prob, "params": pname, "smoother": smoother, "pre_post": list(nu),
               "paper_cycles": printed if printed is not None else "diverges",
               "cycles": ours if ours is not None else "diverges" if not rinf <= 1e30 else f"cap {cap}",
               "seconds": dt, "cpu_baseline": cpu_baseline_sec5(levels, b, smoother, nu, cap)}
        rows.append(rec)
        log(f"[suite] sec5 {rec}")
        del mg, solvers
    return rows


def suite_small(log):
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    # small plain case: 32 x 32 upwind operator, FP64 joint GaBP to rel.res 1e-10
    a, b = W.small_upwind(32)
    s = gabp.Solver.from_csr(a, mode="joint")
    ce = s.autotune()["check_every"]
    bt = torch.as_tensor(b).cuda()
    x = torch.zeros(a.n, dtype=torch.float64, device="cuda")
    for _ in range(3):      # recordings of the check blocks, clocks up
        s.solve(bt, 1e-10, 10000, x=x)
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(bt, 1e-10, 10000, x=x)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    xs = np.linalg.solve(W.csr_to_dense(a), b)
    out = {"seconds": float(np.median(times)), "sweeps": info.sweeps,
           "rel_res2": info.rel_res2,
           "x_rel_err_vs_dense": float(np.abs(x.cpu().numpy() - xs).max() / np.abs(xs).max())}
    # CPU baseline: the oracle's whole solve with the same check interval (measured, not
    # extrapolated: it converges in about a second)
    from oracle import gabp as G
    g = G.Graph.from_csr(a)
    t0 = time.perf_counter()
    _, oinfo, _, _ = G.solve(g, b, 1e-10, 10000, check_every=ce)
    out["cpu_baseline"] = {"seconds": time.perf_counter() - t0, "sweeps": oinfo.sweeps,
                           "cores": 1, "kind": "oracle",
                           "sample": "the whole solve, same check interval"}
    log(f"[suite] small: {out}")
    return out


# algorithmic bytes per grid node of one line sweep (both orientations): the line update
# reads diag, lo, hi, b and the other orientation's two messages and writes two messages
# (64 B per orientation in FP64 joint mode); each orientation's messages are then
# transposed into the other layout (read + write); mean-only sweeps move alpha, beta, b,
# one incoming and one outgoing mean (40 B / 20 B per orientation) plus one transposed mean
LINE_BYTES_PER_NODE = {"joint_f64": 2 * 64 + 2 * 32, "mean_f64": 2 * 40 + 2 * 16,
                       "mean_f32": 2 * 20 + 2 * 8}


def suite_lines(log, n=4095, sweeps=50):
    """Line GaBP sweep rates on the anisotropic convection-diffusion fine grid."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    t0 = time.perf_counter()
    a = W.anisotropic_mg(n, kx=1.0, ky=0.01, peclet=4.0, scaled=False)
    b = torch.as_tensor(W.rng(4, 2).uniform(-1, 1, a.n)).cuda()
    out = {"grid": f"{n}x{n}", "nodes": a.n, "generate_s": time.perf_counter() - t0,
           "bytes_per_node": LINE_BYTES_PER_NODE}
    # the plain copy kernel on 1 GiB: the attainable-bandwidth reference of this run, and
    # the calibration kernel of the HBM byte counters
    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    gabp.copy_probe(src, dst)
    t_cp = _events_time(lambda k: [gabp.copy_probe(src, dst) for _ in range(k)], 4) / 4
    out["copy_probe_GBps"] = 2 * src.numel() * 8 / t_cp / 1e9
    del src, dst
    variants = (("joint_f64", dict(mode="joint")),
                ("mean_f64", dict(mode="precomp", tol_lambda=1e-12)),
                ("mean_f32", dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)))
    for sched in ("lines", "lines_alt"):
        for name, kw in variants:
            s = gabp.Solver.from_csr(a, schedule=sched, grid=(n, n), **kw)
            lsw = s.precompute_lambda() if kw["mode"] == "precomp" else 0
            x = torch.zeros(a.n, dtype=torch.float64, device="cuda")
            s.sweeps(b, 2, x=x)
            torch.cuda.synchronize()
            dt = _events_time(lambda k: s.sweeps(b, sweeps, reset=False, x=x), 1) / sweeps
            bpn = LINE_BYTES_PER_NODE[name]
            rec = {"sweep_us": dt * 1e6, "lambda_sweeps": lsw,
                   "algorithmic_GBps": bpn * a.n / dt / 1e9,
                   "frac_of_hbm_peak": bpn * a.n / dt / 1e9 / HBM_PEAK_GBS,
                   "frac_of_copy": bpn * a.n / dt / 1e9 / out["copy_probe_GBps"]}
            out[f"{sched}_{name}"] = rec
            log(f"[suite] lines {sched} {name}: {rec}")
            del s
    out["cpu_baseline"] = cpu_baseline_lines(log)
    return out


def suite_colours(log, n=2048, sweeps=40):
    """Sweep rates of the coloured schedules at n x n: red-black on the benchmark's 5-point
    upwind operator next to its flood sweep, and the 4-colour schedule on a dominant random
    9-point operator next to its flood sweep. A coloured sweep updates every directed slot
    once (one launch per colour class, in place), so its algorithmic bytes are the flood
    kernel's: joint (40 + rb) B per slot + 16 B per row, frozen-Lt FP64 (24 + rb) + 8, FP32
    (12 + rb) + 4 (rb = bytes of the reverse index)."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    t0 = time.perf_counter()
    a5, b5 = W.precision_at_scale(n)
    a9 = W.random_grid_9pt(n, n, W.rng(6, 0))
    b9 = W.rng(6, 1).uniform(-1, 1, a9.n)
    out = {"grid": f"{n}x{n}", "generate_s": time.perf_counter() - t0}
    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    gabp.copy_probe(src, dst)
    t_cp = _events_time(lambda k: [gabp.copy_probe(src, dst) for _ in range(k)], 4) / 4
    out["copy_probe_GBps"] = 2 * src.numel() * 8 / t_cp / 1e9
    del src, dst
    rb5, c4 = W.grid_colouring(n), W.grid_colouring4(n)
    joint, m64 = dict(mode="joint"), dict(mode="precomp", tol_lambda=1e-12)
    m32 = dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)
    variants = (("upwind5", "flood", "joint_f64", joint, None),
                ("upwind5", "redblack", "joint_f64", joint, rb5),
                ("upwind5", "redblack", "mean_f64", m64, rb5),
                ("upwind5", "flood", "mean_f32", m32, None),
                ("upwind5", "redblack", "mean_f32", m32, rb5),
                ("grid9", "flood", "joint_f64", joint, None),
                ("grid9", "colour4", "joint_f64", joint, c4),
                ("grid9", "colour4", "mean_f32", m32, c4))
    for op, sched, var, kw, colour in variants:
        a, b = (a5, b5) if op == "upwind5" else (a9, b9)
        s = gabp.Solver.from_csr(a, colour=colour,
                                 schedule="flood" if colour is None else "redblack", **kw)
        if kw["mode"] == "precomp":
            s.precompute_lambda()
        li = s.layout_info()
        slots, nn, rb = li["slots"], li["n"], li["rev_bytes"]
        per = {"joint_f64": (40 + rb) * slots + 16 * nn, "mean_f64": (24 + rb) * slots + 8 * nn,
               "mean_f32": (12 + rb) * slots + 4 * nn}[var]
        bt = torch.as_tensor(b).cuda()
        x = torch.zeros(a.n, dtype=torch.float64, device="cuda")
        s.sweeps(bt, 2, x=x)
        torch.cuda.synchronize()
        dt = _events_time(lambda k: s.sweeps(bt, sweeps, reset=False, x=x), 1) / sweeps
        rec = {"sweep_us": dt * 1e6, "colours": 1 if colour is None else int(colour.max()) + 1,
               "slots": slots, "algorithmic_MB": per / 1e6,
               "algorithmic_GBps": per / dt / 1e9, "frac_of_hbm_peak": per / dt / 1e9 / HBM_PEAK_GBS,
               "frac_of_copy": per / dt / 1e9 / out["copy_probe_GBps"],
               "edge_updates_per_s": slots / dt}
        out[f"{op}_{sched}_{var}"] = rec
        log(f"[suite] colours {op} {sched} {var}: {rec}")
        del s
    return out


def cpu_baseline_sec5(levels, b, smoother, nu, cap):
    """The oracle's multigrid (numpy, one thread) on the same problem: cycles and seconds."""
    from oracle import mg as MG
    okw = {"redblack_gabp": dict(smoother="gabp", gabp_mode="joint", schedule="redblack"),
           "colour4_gabp": dict(smoother="gabp", gabp_mode="joint", schedule="colour4"),
           "line_gabp": dict(smoother="gabp", gabp_mode="joint", schedule="lines_alt"),
           "redblack_gs": dict(smoother="rbgs")}[smoother]
    t0 = time.perf_counter()
    h = MG.Hierarchy(levels, nu1=nu[0], nu2=nu[1], **okw)
    g = h.graphs[0]
    x = np.zeros(g.n)
    cycles = None
    for k in range(1, cap + 1):
        x = h.vcycle(b, x)
        r = float(np.abs(g.residual(b, x)).max())
        if not np.isfinite(r) or r > 1e30:
            cycles = "diverges"
            break
        if r <= 2e-4:
            cycles = k
            break
    return {"cycles": cycles if cycles is not None else f"cap {cap}", "cores": 1,
            "seconds": time.perf_counter() - t0, "kind": "oracle"}


def cpu_baseline_lines(log, n=256, sweeps=3):
    """The region oracle (dense LU per line, numpy, one thread) against the HIP flood line
    sweep on the same n x n anisotropic operator."""
    import torch
    from oracle import regions as RG
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    a = W.anisotropic_mg(n, kx=1.0, ky=0.01, peclet=4.0, scaled=False)
    b = W.rng(4, 2).uniform(-1, 1, a.n)
    t0 = time.perf_counter()
    rg = RG.RegionGraph(a, RG.grid_lines(n, n))
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    RG.run(rg, b, sweeps)
    t_cpu = (time.perf_counter() - t0) / sweeps
    s = gabp.Solver.from_csr(a, schedule="lines", grid=(n, n))
    bt = torch.as_tensor(b).cuda()
    x = torch.zeros_like(bt)
    s.sweeps(bt, 2, x=x)
    t_gpu = _events_time(lambda k: s.sweeps(bt, k, reset=False, x=x), 200) / 200
    rec = {"grid": f"{n}x{n}", "cpu_sweep_s": t_cpu, "cpu_build_s": t_build, "cores": 1,
           "gpu_sweep_us": t_gpu * 1e6, "gpu_over_cpu": t_cpu / t_gpu,
           "sample": f"{sweeps} joint flood line sweeps, region oracle (dense LU per line)"}
    log(f"[suite] lines cpu baseline (oracle): {rec}")
    return rec


def suite_batch(log, full_only=False):
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    out = {}
    # full shape: 512 systems, sides 48..384, 4 right-hand sides: batched FP32 sweep rate
    t0 = time.perf_counter()
    fam = W.batch_family(nsys=512, nrhs=4)
    systems = [x for x, _ in fam]
    rhs = np.stack([np.concatenate([bb[q] for _, bb in fam]) for q in range(4)])
    del fam
    gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    bs = gabp.BatchSolver(systems, nrhs=4, mode="precomp", precision="f32_ir", tol_lambda=1e-7)
    setup = time.perf_counter() - t0
    edges = sum(int(x.nnz - x.n) for x in systems)
    Bt = torch.as_tensor(rhs).cuda()
    # fixed work: 2 x 64 sweeps inside the refinement loop, tolerance unreachable
    bs.solve(Bt, 1e-30, 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, infos = bs.solve(Bt, 1e-30, 256)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sw = infos[0].sweeps
    out["full_shape"] = {"systems": 512, "sides": "48..384", "nrhs": 4,
                         "unknowns": int(sum(x.n for x in systems)), "directed_edges": edges,
                         "sweeps": sw, "seconds": dt,
                         "edge_rhs_updates_per_s": edges * 4 * sw / dt,
                         "generate_s": gen, "setup_s": setup}
    log(f"[suite] batch full shape: {out['full_shape']}")
    del bs, X, Bt
    if full_only:   # the full shape alone (for a kernel profile of the batched sweep)
        return out
    # reduced batch to rel.res 1e-8: 64 systems, sides 48..96, 4 rhs; batched vs loop
    fam = W.batch_family(nsys=64, nrhs=4, side_lo=48, side_hi=96, seed=3)
    systems = [x for x, _ in fam]
    rhs_l = [bb for _, bb in fam]
    rhs = np.stack([np.concatenate([r[q] for r in rhs_l]) for q in range(4)])
    Bt = torch.as_tensor(rhs).cuda()
    bs = gabp.BatchSolver(systems, nrhs=4, mode="precomp", precision="f32_ir", tol_lambda=1e-7)
    bs.autotune()
    bs.solve(Bt, 1e-8, 2_000_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, infos = bs.solve(Bt, 1e-8, 2_000_000)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    ok = all(i.status == 0 for i in infos)
    singles = [gabp.Solver.from_csr(x, mode="precomp", precision="f32_ir", tol_lambda=1e-7)
               for x in systems]
    for sgl in singles:
        sgl.autotune()
    rb = [[torch.as_tensor(r[q]).cuda() for q in range(4)] for r in rhs_l]
    for sgl, r in zip(singles, rb):
        sgl.solve(r[0], 1e-8, 2_000_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for sgl, r in zip(singles, rb):
        for q in range(4):
            _, inf = sgl.solve(r[q], 1e-8, 2_000_000)
            worst = max(worst, inf.rel_res2)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    out["reduced_to_1e-8"] = {"systems": 64, "sides": "48..96", "nrhs": 4,
                              "batched_seconds": t_batch, "loop_of_single_solves_seconds": t_loop,
                              "speedup": t_loop / t_batch, "all_converged": ok,
                              "max_sweeps": max(i.sweeps for i in infos),
                              "min_sweeps": min(i.sweeps for i in infos),
                              "loop_worst_rel_res2": worst}
    log(f"[suite] batch reduced: {out['reduced_to_1e-8']}")
    out["cpu_baseline"] = cpu_baseline_batch(systems, rhs_l, t_batch, log)
    return out


def cpu_baseline_batch(systems, rhs_l, t_batch, log):
    """The oracle's FP32-message refinement (numpy, one thread) on the smallest system of the
    reduced batch, one right-hand side, against the batch's time per (system, rhs) pair."""
    from oracle import gabp as G
    k = int(np.argmin([x.n for x in systems]))
    g = G.Graph.from_csr(systems[k])
    t0 = time.perf_counter()
    Lt, S, _ = G.lambda_phase(g, 1e-7, 10000)
    x, info = G.ir_solve(g, rhs_l[k][0], 1e-8,
                         (Lt.astype(np.float32), (1.0 / S).astype(np.float32)), check_every=256)
    dt = time.perf_counter() - t0
    per_pair_gpu = t_batch / (len(systems) * len(rhs_l[0]))
    rec = {"unknowns": g.n, "sweeps": info.sweeps, "seconds": dt, "cores": 1, "kind": "oracle",
           "gpu_batch_seconds_per_pair": per_pair_gpu, "ratio": dt / per_pair_gpu,
           "sample": "one (system, rhs) pair, the smallest system of the reduced batch"}
    log(f"[suite] batch cpu baseline (oracle): {rec}")
    return rec


def suite_mg(log, J=12, problems=None, smoothers=None, cap=60):
    """V(2,2) multigrid to rel.res 1e-8 (at most ``cap`` cycles) per problem and smoother;
    ``problems`` / ``smoothers``: names to run (None: all)."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    out = {}
    for name, JJ, kw in (("anisotropic_peclet4", J, dict(kx=1.0, ky=0.01, peclet=4.0)),
                         ("poisson", J, dict(kx=1.0, ky=1.0, peclet=0.0)),
                         ("anisotropic_peclet4_63x63", 6, dict(kx=1.0, ky=0.01, peclet=4.0))):
        if problems is not None and name not in problems:
            continue
        t0 = time.perf_counter()
        levels = W.mg_hierarchy(JJ, coarsest=3, **kw)
        sides = [int(round(np.sqrt(x.n))) for x in levels]
        gen = time.perf_counter() - t0
        b = W.rng(4, 1).uniform(-1, 1, levels[0].n)
        bt = torch.as_tensor(b).cuda()
        entry = {"grid": f"{sides[0]}x{sides[0]}", "levels": len(levels), "generate_s": gen,
                 "cycle_cap": cap}
        for sm_name, smoother, kwg in (
                ("rbgs_2_2", "rbgs", {}),
                ("redblack_gabp_f32_seq_lambda_2_2", "gabp",
                 dict(mode="seq", precision="f32_ir", schedule="redblack")),
                ("redblack_gabp_f64_seq_lambda_2_2", "gabp", dict(mode="seq", schedule="redblack")),
                ("redblack_gabp_f64_joint_2_2", "gabp", dict(mode="joint", schedule="redblack")),
                ("redblack_gabp_f32_frozen_lambda_2_2", "gabp",
                 dict(mode="precomp", precision="f32_ir", schedule="redblack", tol_lambda=1e-7)),
                ("flood_gabp_f32_seq_lambda_2_2", "gabp", dict(mode="seq", precision="f32_ir")),
                ("flood_gabp_f32_frozen_lambda_2_2", "gabp",
                 dict(mode="precomp", precision="f32_ir", tol_lambda=1e-7)),
                ("lines_alt_gabp_f32_frozen_lambda_2_2", "gabp",
                 dict(mode="precomp", precision="f32_ir", schedule="lines_alt", tol_lambda=1e-7)),
                ("lines_alt_gabp_f64_joint_2_2", "gabp", dict(mode="joint", schedule="lines_alt"))):
            if smoothers is not None and sm_name not in smoothers:
                continue
            t0 = time.perf_counter()
            lines = kwg.get("schedule", "").startswith("lines")
            solvers = [gabp.Solver.from_csr(x, colour=None if lines else W.grid_colouring(sd),
                                            grid=(sd, sd) if lines else None, **kwg)
                       for x, sd in zip(levels, sides)]
            mg = gabp.Multigrid(solvers, sides, smoother=smoother, nu1=2, nu2=2)
            x = torch.zeros(levels[0].n, dtype=torch.float64, device="cuda")
            mg.vcycle(bt, x)       # first cycle: Lt phases and recordings
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            t0 = time.perf_counter()
            x, info = mg.solve(bt, 1e-8, cap)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            entry[sm_name] = {"status": info["status"], "cycles": info["cycles"],
                              "rel_res2": info["rel_res2"], "seconds": dt,
                              "ms_per_cycle": 1e3 * dt / max(info["cycles"], 1),
                              "setup_s": setup}
            log(f"[suite] mg {name} {sm_name}: {entry[sm_name]}")
            del mg, solvers
        if JJ <= 6:
            entry["cpu_baseline"] = cpu_baseline_mg(levels, b, log)
        out[name] = entry
    return out


def suite_sweeps_large(log, n=4095, sweeps=40):
    """Sweep kernels on the 4095 x 4095 operator of the benchmark's family (16.8M rows,
    67M directed slots): every message array is far larger than the 256 MB last-level
    cache, so the rates are HBM rates. Plain (one sweep per launch) and tiled (two per
    launch) joint FP64, frozen-Lt FP64 and FP32 mean-only sweeps."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    t0 = time.perf_counter()
    a, b = W.precision_at_scale(n)
    bt = torch.as_tensor(b).cuda()
    out = {"grid": f"{n}x{n}", "unknowns": a.n, "generate_s": time.perf_counter() - t0}
    src = torch.empty(2 ** 28, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    gabp.copy_probe(src, dst)
    t_cp = _events_time(lambda k: [gabp.copy_probe(src, dst) for _ in range(k)], 4) / 4
    out["copy_probe_GBps"] = 2 * src.numel() * 8 / t_cp / 1e9
    del src, dst
    for tiles in (False, True):
        tkw = dict(tiles=True, grid=(n, n)) if tiles else {}
        for name, kw, bytes_fn in (("joint_f64", dict(mode="joint"), sweep_bytes_joint64),
                                   ("mean_f64", dict(mode="precomp", tol_lambda=1e-12),
                                    sweep_bytes_mean64),
                                   ("mean_f32", dict(mode="precomp", precision="f32_ir",
                                                     tol_lambda=1e-7), sweep_bytes_mean32)):
            s = gabp.Solver.from_csr(a, **kw, **tkw)
            lay = s.layout_info()
            if kw["mode"] == "precomp":
                s.precompute_lambda()
            tuned = s.autotune()
            x = torch.zeros(a.n, dtype=torch.float64, device="cuda")
            s.sweeps(bt, 2, x=x)
            torch.cuda.synchronize()
            # FP32: differencing removes the cast of b and the widening of x per call
            t1 = _events_time(lambda k: s.sweeps(bt, sweeps + 1, reset=False, x=x), 1)
            t0_ = _events_time(lambda k: s.sweeps(bt, 1, reset=False, x=x), 1)
            dt = (t1 - t0_) / sweeps
            per = 2 if tiles else 1
            rb = 4 if tiles else lay["rev_bytes"]
            ab = bytes_fn(lay["slots"], a.n, rb)
            rec = {"sweep_us": dt * 1e6, "launch_us": per * dt * 1e6, "sweeps_per_launch": per,
                   "algorithmic_bytes_per_launch": ab,
                   "GBps_per_launch": ab / (per * dt) / 1e9,
                   "frac_of_hbm_peak": ab / (per * dt) / 1e9 / HBM_PEAK_GBS,
                   "edge_updates_per_s": (a.nnz - a.n) / dt,
                   "stream_hints": tuned["stream_hints"]}
            out[("tiled_" if tiles else "plain_") + name] = rec
            log(f"[suite] sweeps {n}x{n} tiles={tiles} {name}: {rec}")
            del s
    return out


MG_PROFILE_SMOOTHERS = (
    ("redblack_gabp_f32_seq_lambda_2_2", "gabp",
     dict(mode="seq", precision="f32_ir", schedule="redblack")),
    ("redblack_gabp_f64_seq_lambda_2_2", "gabp", dict(mode="seq", schedule="redblack")),
    ("redblack_gabp_f64_joint_2_2", "gabp", dict(mode="joint", schedule="redblack")),
    ("rbgs_2_2", "rbgs", {}))


def suite_mg_profile(log, J=12, cycles=4):
    """A few V(2,2) cycles per smoother on the 4095 x 4095 anisotropic hierarchy, for a
    kernel trace: one eager cycle (Lt phases, recording), then ``cycles`` replays of the
    recorded cycle, each timed with HIP events on the caller's stream."""
    import torch
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    levels = W.mg_hierarchy(J, coarsest=3, kx=1.0, ky=0.01, peclet=4.0)
    sides = [int(round(np.sqrt(x.n))) for x in levels]
    bt = torch.as_tensor(W.rng(4, 1).uniform(-1, 1, levels[0].n)).cuda()
    out = {"grid": f"{sides[0]}x{sides[0]}", "levels": len(levels), "sides": sides}
    for sm_name, smoother, kwg in MG_PROFILE_SMOOTHERS:
        solvers = [gabp.Solver.from_csr(x, colour=W.grid_colouring(sd), **kwg)
                   for x, sd in zip(levels, sides)]
        mg = gabp.Multigrid(solvers, sides, smoother=smoother, nu1=2, nu2=2)
        x = torch.zeros(levels[0].n, dtype=torch.float64, device="cuda")
        mg.vcycle(bt, x)
        mg.vcycle(bt, x)          # recorded here
        torch.cuda.synchronize()
        ts = [1e3 * _events_time(lambda k: mg.vcycle(bt, x), 1) for _ in range(cycles)]
        out[sm_name] = {"ms_per_cycle": ts, "median_ms": float(np.median(ts))}
        log(f"[suite] mg profile {sm_name}: {out[sm_name]}")
        del mg, solvers
    return out


def cpu_baseline_mg(levels, b, log):
    """The oracle's V(2,2) cycles (numpy, one thread) on the same hierarchy, to rel.res 1e-8
    (cap 60): cycle counts to compare with the GPU's and seconds per cycle."""
    from oracle import mg as MG
    rec = {}
    for name, kw in (("rbgs_2_2", dict(smoother="rbgs")),
                     ("redblack_gabp_f64_joint_2_2",
                      dict(smoother="gabp", gabp_mode="joint", schedule="redblack")),
                     ("redblack_gabp_f64_seq_lambda_2_2",
                      dict(smoother="gabp", gabp_mode="seq", schedule="redblack")),
                     ("lines_alt_gabp_f64_joint_2_2",
                      dict(smoother="gabp", gabp_mode="joint", schedule="lines_alt"))):
        t0 = time.perf_counter()
        h = MG.Hierarchy(levels, nu1=2, nu2=2, **kw)
        _, hist = h.solve(b, 1e-8, 60)
        dt = time.perf_counter() - t0
        rec[name] = {"cycles": len(hist), "rel_res2": hist[-1], "seconds": dt,
                     "ms_per_cycle": 1e3 * dt / max(len(hist), 1), "cores": 1, "kind": "oracle"}
        log(f"[suite] mg cpu baseline (oracle) {name}: {rec[name]}")
    return rec


def suite_adjoint(log, n_full=1024, n_small=128, batch=8):
    import torch
    from paper_1904_04093_amd import autograd as AG
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    out = {}
    for n in (n_small, n_full):
        field = AG.ThetaField(n)
        solver = gabp.Solver.from_csr(field.pattern, mode="precomp", precision="f32_ir",
                                      tol_lambda=1e-7)
        solver.autotune()
        b = torch.as_tensor(W.rng(5, 101).uniform(-1, 1, n * n)).cuda()
        xt = torch.as_tensor(W.rng(5, 100).uniform(-1, 1, n * n)).cuda()
        if n == n_full:
            # per-sweep rate of forward and adjoint FP32 sweeps on the full grid
            th = torch.as_tensor(W.theta_problem(n, 0)).cuda()
            solver.update_values(field.values(th).detach().contiguous())
            solver.precompute_lambda()
            solver.precompute_lambda(transposed=True)
            xx = torch.zeros_like(b)
            solver.sweeps(b, 2, x=xx)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.sweeps(b, 401, reset=False, x=xx)
            solver.sweeps(b, 401, reset=False, transposed=True, x=xx)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 802
            e = field.pattern.nnz - field.pattern.n
            out[f"full_{n}x{n}"] = {"fp32_sweep_us": dt * 1e6, "edge_updates_per_s": e / dt,
                                    "note": "gradient to 1e-8 at this size needs ~1.4M sweeps per solve"}
            log(f"[suite] adjoint full: {out[f'full_{n}x{n}']}")
            continue
        t0 = time.perf_counter()
        losses = []
        for t in range(batch):
            th = torch.tensor(W.theta_problem(n, t), device="cuda", requires_grad=True)
            x = AG.gabp_solve(field.values(th), b, solver, tol=1e-8)
            loss = 0.5 * ((x - xt) ** 2).sum()
            loss.backward()
            losses.append(float(loss))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"gradients_{n}x{n}_batch{batch}"] = {"seconds": dt, "per_theta_s": dt / batch,
                                                 "loss_mean": float(np.mean(losses))}
        log(f"[suite] adjoint {n}: {out[f'gradients_{n}x{n}_batch{batch}']}")
    out["cpu_baseline"] = cpu_baseline_adjoint(log)
    return out


def suite_adjoint_full(log, n=1024, batch=8, tol=1e-8, tiles=True):
    """The differentiation configuration at its full size: 8 theta fields on the 1024 x 1024
    grid, L = 0.5 ||x(theta) - x_target||^2, FP32 messages inside FP64 refinement to rel.res
    1e-8 for the forward and the transposed (adjoint) solve, gradient reduced onto theta;
    timed per theta end to end (operator assembly, both solves with their Lt phases, the
    scatter and the chain rule)."""
    import torch
    from paper_1904_04093_amd import autograd as AG
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    field = AG.ThetaField(n)
    solver = gabp.Solver.from_csr(field.pattern, mode="precomp", precision="f32_ir",
                                  tol_lambda=1e-7, progress_s=30.0,
                                  **(dict(tiles=True, grid=(n, n)) if tiles else {}))
    tuned = solver.autotune()
    b = torch.as_tensor(W.rng(5, 101).uniform(-1, 1, n * n)).cuda()
    xt = torch.as_tensor(W.rng(5, 100).uniform(-1, 1, n * n)).cuda()
    per = []
    t_all = time.perf_counter()
    for t in range(batch):
        th = torch.tensor(W.theta_problem(n, t), device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = AG.gabp_solve(field.values(th), b, solver, tol=tol, max_sweeps=2_000_000_000)
        loss = 0.5 * ((x - xt) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fi, bi = solver.last_forward_info, solver.last_backward_info
        rec = {"theta": t, "loss": float(loss), "grad_norm": float(th.grad.norm()),
               "forward": {"seconds": t1 - t0, "sweeps": fi.sweeps, "outer": fi.outer_iters,
                           "rel_res2": fi.rel_res2, "status": fi.status},
               "adjoint": {"seconds": t2 - t1, "sweeps": bi.sweeps, "outer": bi.outer_iters,
                           "rel_res2": bi.rel_res2, "status": bi.status},
               "seconds": t2 - t0}
        per.append(rec)
        log(f"[suite] adjoint {n}x{n} theta {t}: {json.dumps(rec)}")
    total = time.perf_counter() - t_all
    e = field.pattern.nnz - field.pattern.n
    sweeps = sum(r["forward"]["sweeps"] + r["adjoint"]["sweeps"] for r in per)
    return {"grid": f"{n}x{n}", "batch": batch, "tol": tol, "autotuned": tuned, "tiles": tiles,
            "seconds": total, "per_theta_s": total / batch, "per_theta": per,
            "fp32_edge_updates_per_s": e * sweeps / total,
            "cpu_baseline": cpu_baseline_adjoint(log)}


def cpu_baseline_adjoint(log, n=64):
    """One theta-gradient on an n x n grid: the oracle (FP64 flood GaBP forward and
    transposed solves to 1e-8 and the scatter, numpy, one thread) against the HIP path
    (FP32 messages, FP64 refinement, autograd) on the same problem."""
    import torch
    from oracle import adjoint as OA
    from oracle import gabp as G
    from paper_1904_04093_amd import autograd as AG
    from paper_1904_04093_amd import gabp
    from paper_1904_04093_amd import workloads as W
    th = W.theta_problem(n, 0)
    b = W.rng(5, 101).uniform(-1, 1, n * n)
    xt = W.rng(5, 100).uniform(-1, 1, n * n)
    a = W.theta_operator(n, th)
    t0 = time.perf_counter()
    res = OA.gabp_adjoint(G.Graph.from_csr(a), b, xt, 1e-8, 2_000_000, check_every=16)
    t_cpu = time.perf_counter() - t0
    field = AG.ThetaField(n)
    solver = gabp.Solver.from_csr(field.pattern, mode="precomp", precision="f32_ir",
                                  tol_lambda=1e-7)
    bt, xtt = torch.as_tensor(b).cuda(), torch.as_tensor(xt).cuda()

    def grad_once():
        tt = torch.tensor(th, device="cuda", requires_grad=True)
        x = AG.gabp_solve(field.values(tt), bt, solver, tol=1e-8)
        (0.5 * ((x - xtt) ** 2).sum()).backward()
    grad_once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad_once()
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    rec = {"grid": f"{n}x{n}", "cpu_seconds": t_cpu, "gpu_seconds": t_gpu, "cores": 1,
           "kind": "oracle", "cpu_sweeps": [res["info"][0].sweeps, res["info"][1].sweeps],
           "sample": "one theta-gradient (forward + transposed solve to 1e-8, scatter)"}
    log(f"[suite] adjoint cpu baseline (oracle): {rec}")
    return rec


if __name__ == "__main__":
    main()
