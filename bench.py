#!/usr/bin/env python3
"""Benchmark of the matching-based AMG + flexible CG path on one MI355X.

One step = bcm_setup (hierarchy build) + bcm_solve from x0 = 0 to true relative
residual 1e-8 + bcm_free, on the 3-D Poisson 7-point 100^3 workload (n = 1e6),
inputs resident in HBM before the timed region.  The headline value is the
FP32-cycle form (float32 hierarchy and V-cycle inside float64 flexible CG); the
plain float64 path is timed the same way and reported beside it.

value = n / (mean seconds per step) / 1e6  [Mdof/s]

roofline: the single kernel with the largest event time per step over the
whole step (setup kernels included), timed with HIP events taken by that
kernel's own dispatch on the library's stream during a third timed leg (the
FP32 form, eager launches); achieved GB/s = its algorithmic bytes / its event
time.  The two headline legs run without events.
setup_roofline: the setup's algorithmic bytes (sum over its pairwise sweeps of
72 z + 80 m) over its time, with the event-timed setup classes beside it.
roofline_hbm_160: the finest-level solve kernels on the 160^3 heterogeneous
diffusion workload, whose matrix and vectors (about 0.8 GB) do not fit the
256 MB Infinity Cache: an HBM-bound point, timed the same way.
cpu_baseline: the serial oracle (one thread) running full setups + solves of
the same workload.
"""
import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "setup+solve s to rel-res 1e-8 (Mdof/s, HBM %), FP32-cycle vs FP64 AMG-FCG"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1810_04221_amd", "csrc")
# the sources of each profiled kernel: recorded counter traffic applies while
# they hash to the value stored with it
TRAFFIC_SOURCES = {"down0": ("sell_kernels.h", "device.h"), "up0": ("sell_kernels.h", "device.h"),
                   "spmv_dots": ("sell_kernels.h", "device.h"), "update": ("sell_kernels.h", "device.h"),
                   "setup_suitor": ("setup.hip", "device.h")}


def sources_sha256(cls):
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES.get(cls.replace("_160", ""), ()):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


SOLVE_CLASSES = ["down0", "up0", "spmv_dots", "update", "coarse", "mid"]
SETUP_CLASSES = ["setup_match", "setup_suitor", "setup_galerkin"]
CLASSES = SOLVE_CLASSES + SETUP_CLASSES
# classes that are one kernel launch per bracket
SINGLE_KERNEL = ["down0", "up0", "spmv_dots", "update", "coarse", "setup_suitor"]
KERNEL_OF_CLASS = {"down0": "k_down_res_sell_ad (finest level: p * (b - (A D) b), the down leg's residual, on the values of A D)",
                   "up0": "k_smooth_sell (finest level: post-smoothing of the prolonged iterate)",
                   "spmv_dots": "k_spmv_dots_sell (v = A w and three dot products, finest level, FP64)",
                   "update": "k_update (the step scalars from the product's partials, four vector updates and ||r||^2)",
                   "coarse": "coarsest-level solve (k_coarse_dense on the folded levels, k_tail or k_coarse, the "
                             "k_star_* recurrence on a star level, else k_jacobi_sweep)",
                   "setup_suitor": "k_suitor (Suitor matching, proposals raised by 64-bit atomicMax)"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="G2")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--min-ratio", type=float, default=0.0,
                    help="also stop coarsening at the first level formed with n_(k-1)/n_k below this "
                         "(a rule of this library, not the paper's; 0 = Section 5's rule alone)")
    ap.add_argument("--no-hbm-point", action="store_true",
                    help="skip the 160^3 roofline point (HBM-bound finest-level kernels)")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (reference for HBM counters)")
    ap.add_argument("--ablation", choices=sorted(ABLATIONS), default=None,
                    help="instead of the benchmark line: time setup + solve under each setting of one "
                         "knob (lane width, cycle type, sweeps per level, smooth vector) and print one "
                         "JSON line")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path; run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1810_04221_amd import bcm, problems

    torch.cuda.set_device(0)
    c = problems.config(args.workload, args.scale)
    n, tol = c["n"], c["tol"]
    log(f"workload {c['name']} n={n} nnz={len(c['col'])}")
    dev = torch.device("cuda", 0)
    rp = torch.as_tensor(c["rowptr"], device=dev)
    ci = torch.as_tensor(c["col"], device=dev)
    va = torch.as_tensor(c["val"], device=dev)
    w = torch.as_tensor(c["w"], device=dev)
    b = torch.as_tensor(c["b"], device=dev)
    torch.cuda.synchronize()
    if args.calibration_copy_mb:
        src = torch.empty(args.calibration_copy_mb << 17, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibration_copy_mb} MiB read + written")
        del src, dst

    def step(precision, mask, wvec=None, **kw):
        kw.setdefault("min_ratio", args.min_ratio)
        h = bcm.Hierarchy(rp, ci, va, w if wvec is None else wvec, max_coarse=c["max_coarse"],
                          precision=precision, profile=mask, **kw)
        h.solve(b, tol=tol)
        info = h.info()
        prof = {k: h.profile(k) for k in CLASSES if mask & bcm.PROF[k]}
        h.close()
        return info, prof

    if args.ablation:
        ablation(args, c, step)
        return

    all_mask = sum(bcm.PROF.values())
    # warm-up, and the single kernel with the largest event time per step
    # (setup and solve kernels alike)
    share = {k: 0.0 for k in CLASSES}
    setup_cls = {k: [0, 0.0, 0.0] for k in SETUP_CLASSES}
    nwarm = max(1, args.warmup)
    for it in range(nwarm):
        for prec in ("fp32", "fp64"):
            info, prof = step(prec, all_mask)
            if prec == "fp32":
                for k, (nl_, ms, by) in prof.items():
                    share[k] += ms / nwarm
                    if k in setup_cls:
                        setup_cls[k][0] += nl_ / nwarm
                        setup_cls[k][1] += ms / nwarm
                        setup_cls[k][2] += by / nwarm
    dom = max(SINGLE_KERNEL, key=share.get)
    # the dominant solve kernel (the bandwidth-bound part), timed in a leg of its
    # own when the step's dominant kernel is a setup kernel
    dom_solve = max([k for k in SINGLE_KERNEL if k in SOLVE_CLASSES], key=share.get)
    log("event time per step by class (fp32 cycle, ms): "
        + ", ".join(f"{k} {v:.3f}" for k, v in sorted(share.items(), key=lambda kv: -kv[1])) + f"; dominant {dom}")

    # timed legs: FP32 cycle (the headline) and FP64, no profiling; then a third
    # timed leg of the FP32 form with the dominant kernel bracketed by HIP
    # events on the library's stream, for the roofline (all legs launch every
    # kernel eagerly: faster here than replaying the iteration from a graph)
    results = {}
    legs = ("fp32", "fp64", "roofline") + (("roofline_solve",) if dom_solve != dom else ())
    for leg in legs:
        prec = "fp64" if leg == "fp64" else "fp32"
        cls = dom_solve if leg == "roofline_solve" else dom
        mask = bcm.PROF[cls] if leg.startswith("roofline") else 0
        kw = dict(graph=False) if leg.startswith("roofline") else {}
        tot_l, tot_ms, tot_b = 0, 0.0, 0.0
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info, prof = step(prec, mask, **kw)
            infos.append(info)
            if cls in prof:
                l_, ms, by = prof[cls]
                tot_l += l_; tot_ms += ms; tot_b += by
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_step = (t1 - t0) * 1e3 / args.steps
        inf = infos[-1]
        results[leg] = dict(ms_per_step=ms_step, mdofs=n / (ms_step * 1e-3) / 1e6, iters=inf["iters"],
                            relres=inf["relres"], t_setup_ms=float(np.mean([i["t_setup_ms"] for i in infos])),
                            t_solve_ms=float(np.mean([i["t_solve_ms"] for i in infos])), levels=inf["n"],
                            vcmplx=inf["vcmplx"], iter_bytes=inf["iter_bytes"], setup_bytes=inf["setup_bytes"],
                            sweeps=inf["sweeps_run"], prof=(tot_l, tot_ms, tot_b))
        r = results[leg]
        r["solve_hbm_frac"] = r["iter_bytes"] * r["iters"] / (r["t_solve_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
        log(f"{leg}: {ms_step:.2f} ms/step ({r['t_setup_ms']:.2f} setup + {r['t_solve_ms']:.2f} solve), "
            f"{r['mdofs']:.1f} Mdof/s, iters {r['iters']}, relres {r['relres']:.2e}, levels {r['levels']}")

    f32 = results["fp32"]
    l_, ms, by = results["roofline"]["prof"]
    roofline = {"bound": "hbm", "kernel": KERNEL_OF_CLASS[dom]}
    # the counter traffic on record is the default 100^3 workload's
    recorded = args.workload == "G2" and args.scale == 1.0 and args.min_ratio <= 1.0
    roofline.update(class_roofline(dom, l_, ms, by, recorded))
    roofline.update({"timed_leg": "FP32 cycle, eager launches, HIP events taken by the kernel's own dispatch",
                     "timed_leg_ms_per_step": results["roofline"]["ms_per_step"]})
    if dom == "setup_suitor":
        roofline["note"] = ("latency-bound: each proposal that displaces another suitor continues that "
                            "vertex's list, so the kernel's time is its longest chain of dependent steps (an "
                            "atomicMax, then a candidate load) times their latency, not its bytes over the "
                            "bandwidth; the algorithmic bytes count one candidate and one proposal word per vertex")
    roofline_solve = None
    if "roofline_solve" in results:
        l_, ms, by = results["roofline_solve"]["prof"]
        roofline_solve = {"bound": "hbm", "kernel": KERNEL_OF_CLASS[dom_solve]}
        roofline_solve.update(class_roofline(dom_solve, l_, ms, by, recorded))
        roofline_solve.update({"timed_leg": "FP32 cycle, eager launches, HIP events taken by the kernel's own "
                                            "dispatch", "timed_leg_ms_per_step": results["roofline_solve"]["ms_per_step"]})

    # the setup against its byte model
    sb = f32["setup_bytes"]
    setup_roofline = {"bound": "hbm", "achieved": sb / (f32["t_setup_ms"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": sb / (f32["t_setup_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9),
                      "algorithmic_bytes": sb, "sweeps": f32["sweeps"],
                      "model": "sum over the pairwise sweeps on (m rows, z entries) of 72 z + 80 m",
                      "setup_ms": f32["t_setup_ms"], "setup_fraction_of_step": f32["t_setup_ms"] / f32["ms_per_step"],
                      "classes": {k: {"brackets": v[0], "ms": v[1], "algorithmic_bytes": v[2],
                                      "GBs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] else None,
                                      "frac": (v[2] / (v[1] * 1e-3) / (HBM_PEAK_GBS * 1e9)) if v[1] else None}
                                  for k, v in setup_cls.items()},
                      "timed": f"classes: HIP events per sweep over {nwarm} warm-up setup(s), FP32 form"}

    hbm160 = None if args.no_hbm_point else hbm_point(args)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        log("cpu baseline: serial oracle, full setup + solve of the same workload, repeated for ~10 s")
        times = []
        while len(times) < 8 and sum(times) < 10.0:
            t0 = time.perf_counter()
            ho = oracle.Hierarchy(c["rowptr"], c["col"], c["val"], c["w"], max_coarse=c["max_coarse"])
            xo, io = ho.solve(c["b"], tol=tol)
            times.append(time.perf_counter() - t0)
            del ho
        ts = sum(times) / len(times)
        cpu = {"value": n / ts / 1e6, "unit": "Mdof/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(times)} full setups + solves of {c['name']} (n={n}, {io['iters']} iterations each), "
                         f"{sum(times):.1f} s on one host thread, mean {ts:.2f} s per setup + solve",
               "host": host_cpu()}
        log(f"cpu baseline {cpu['value']:.3f} Mdof/s ({len(times)} runs, mean {ts:.2f} s) on {cpu['host']}")

    grad = gradient_leg(args, c, rp, ci, va, w, b, tol) if "xstar" in c else None

    f64 = results["fp64"]
    out = {
        "metric": METRIC, "value": f32["mdofs"], "unit": "Mdof/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f32["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 cycle + f64 outer CG", "data": "synthetic",
        "config": {"workload": f"3-D Poisson 7-point {c['name']}, n={n}, nnz={len(c['col'])}, b~U[-1,1) seed 1, "
                               f"w=1, coarsest<{c['max_coarse'] + 1} rows, tol {tol:g}, FP32 V-cycle in FP64 FCG"
                   if args.workload == "G2" else c["name"] + (f", coarsening also stopped at n_(k-1)/n_k < {args.min_ratio:g}"
                                                               if args.min_ratio > 1 else "")},
        "setup_ms": f32["t_setup_ms"], "solve_ms": f32["t_solve_ms"], "iters": f32["iters"],
        "relres": f32["relres"], "levels": f32["levels"], "vcmplx": f32["vcmplx"],
        "solve_hbm_frac": f32["solve_hbm_frac"],
        "fp64": {"value": f64["mdofs"], "ms_per_step": f64["ms_per_step"], "setup_ms": f64["t_setup_ms"],
                 "solve_ms": f64["t_solve_ms"], "iters": f64["iters"], "relres": f64["relres"],
                 "solve_hbm_frac": f64["solve_hbm_frac"]},
        "fp32_over_fp64": f32["mdofs"] / f64["mdofs"],
        "fp32_over_fp64_solve": f64["t_solve_ms"] / f32["t_solve_ms"],
        # a solve bound by bandwidth alone would gain the ratio of the algorithmic bytes per iteration
        "fp32_over_fp64_solve_byte_model": (f64["iter_bytes"] * f64["iters"]) / (f32["iter_bytes"] * f32["iters"]),
        "roofline": roofline, "setup_roofline": setup_roofline, "cpu_baseline": cpu,
    }
    if roofline_solve is not None:
        out["roofline_solve"] = roofline_solve
    if hbm160 is not None:
        out["roofline_hbm_160"] = hbm160
    if grad is not None:
        out["gradient"] = grad
    print(json.dumps(out), flush=True)


def class_roofline(cls, launches, ms, nbytes, recorded=True):
    """achieved / peak of one event-timed class, with the counter traffic
    recorded for it when its sources still hash to the recorded value and the
    run is the recorded workload (recorded=False: another workload, no traffic)."""
    achieved = (nbytes / launches) / ((ms / launches) * 1e-3) / 1e9 if launches else None
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath)).get("per_class", {}).get(cls)
        if recorded and t and t.get("sources_sha256") == sources_sha256(cls):
            traffic = t["hbm_bytes"]
    return {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "algorithmic_bytes_per_launch": (nbytes / launches) if launches else None,
            "avg_launch_us": (ms / launches * 1e3) if launches else None, "launches": launches}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return f"{model}; {avail} host threads available (nproc), 1 used"


def hbm_point(args):
    """The finest-level solve kernels on the 160^3 heterogeneous diffusion
    workload (beyond the Infinity Cache), FP32 cycle, one setup + solve with
    HIP events on three classes."""
    import torch
    from paper_1810_04221_amd import bcm, problems
    c = problems.config("G3", 1.0)
    dev = torch.device("cuda", 0)
    t = {k: torch.as_tensor(c[k], device=dev) for k in ("rowptr", "col", "val", "w", "b")}
    mask = bcm.PROF["down0"] | bcm.PROF["spmv_dots"] | bcm.PROF["update"] | bcm.PROF["up0"]
    h = bcm.Hierarchy(t["rowptr"], t["col"], t["val"], t["w"], max_coarse=c["max_coarse"], precision="fp32",
                      profile=mask, graph=False)
    h.solve(t["b"], tol=c["tol"])
    inf = h.info()
    ks = {}
    for cls, name in (("spmv_dots", "k_spmv_dots_sell"), ("down0", "k_down_res_sell"), ("up0", "k_smooth_sell"),
                      ("update", "k_update")):
        l_, ms, by = h.profile(cls)
        ks[name] = class_roofline(cls + "_160", l_, ms, by)
    h.close()
    log("160^3 HBM point: " + ", ".join(f"{k} {v['frac'] * 100:.1f}%" for k, v in ks.items() if v["frac"]))
    return {"workload": f"{c['name']} (n={c['n']}, nnz={len(c['col'])}), FP32 cycle, {inf['iters']} iterations",
            "bound": "hbm", "kernels": ks,
            "timed": "HIP events taken by each kernel's own dispatch, one setup + solve"}


def gradient_leg(args, c, rp, ci, va, w, b, tol):
    """Backward pass of the differentiable workload (loss 1/2 ||x - x*||^2): the
    adjoint solve A lambda = x - x* on the forward hierarchy (dL/db = lambda) and
    the sampled outer product dL/da_ij = -lambda_i x_j on A's pattern.  The
    adjoint solve is timed per call (synchronised); the outer product by events
    around `reps` back-to-back launches on the library's stream."""
    import numpy as np
    import torch

    from paper_1810_04221_amd import bcm

    n, z = c["n"], len(c["col"])
    xs = torch.as_tensor(c["xstar"], device=b.device)
    h = bcm.Hierarchy(rp, ci, va, w, max_coarse=c["max_coarse"], precision="fp32", adjoint_tol=tol)
    x = h.solve(b, tol=tol)
    g = x - xs
    lam = h.solve_adjoint(g)
    h.sampled_outer(lam, x)
    torch.cuda.synchronize()
    t_adj = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        lam = h.solve_adjoint(g)
        torch.cuda.synchronize()
        t_adj.append((time.perf_counter() - t0) * 1e3)
    inf = h.info()
    reps = 20
    out = torch.empty(z, dtype=torch.float64, device=b.device)
    lib = bcm.load_library()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    args_ = (h.h, C.c_void_p(lam.data_ptr()), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
    e0.record()
    rcs = [lib.bcm_sampled_outer(*args_) for _ in range(reps)]
    e1.record()
    e1.synchronize()
    if any(rcs):
        raise RuntimeError(f"bcm_sampled_outer failed: {lib.bcm_last_error().decode()}")
    us = e0.elapsed_time(e1) * 1e3 / reps
    # row pointers, columns, lambda and x once (x gathered), the output written
    alg = 4.0 * (n + 1) + 12.0 * z + 16.0 * n
    h.close()
    r = {"adjoint_ms": float(np.mean(t_adj)), "adjoint_iters": inf["iters"], "adjoint_relres": inf["relres"],
         "sampled_outer_us": us, "sampled_outer_bytes": alg, "sampled_outer_GBs": alg / (us * 1e-6) / 1e9,
         "sampled_outer_hbm_frac": alg / (us * 1e-6) / (HBM_PEAK_GBS * 1e9),
         "timing": f"adjoint: mean of {args.steps} synchronised calls; outer product: events around {reps} launches"}
    log(f"gradient: adjoint {r['adjoint_ms']:.2f} ms ({r['adjoint_iters']} iterations, relres "
        f"{r['adjoint_relres']:.2e}); sampled outer product {us:.1f} us, {r['sampled_outer_GBs']:.0f} GB/s "
        f"({100 * r['sampled_outer_hbm_frac']:.1f}% of 8 TB/s)")
    return r


ABLATIONS = {
    # lane width of the CSR row kernels (the paper's miniwarp), with and without
    # the sliced-ELL copies of the finest and large levels
    "miniwarp": [("rule (4..64 from nnz/row) + SELL", "fp64", dict(group=0, sell=True)),
                 ("rule, CSR only", "fp64", dict(group=0, sell=False)),
                 ("4 lanes, CSR only", "fp64", dict(group=4, sell=False)),
                 ("8 lanes, CSR only", "fp64", dict(group=8, sell=False)),
                 ("16 lanes, CSR only", "fp64", dict(group=16, sell=False)),
                 ("32 lanes, CSR only", "fp64", dict(group=32, sell=False)),
                 ("64 lanes (one wavefront per row), CSR only", "fp64", dict(group=64, sell=False)),
                 ("timed per level, CSR only", "fp64", dict(group=-1, sell=False)),
                 ("timed per level + SELL", "fp64", dict(group=-1, sell=True))],
    "cycles": [(f"{cy}{'' if kl == 0 else f' (K on {kl} levels)'} {pr}", pr, dict(cycle=cy, kcycle_levels=kl))
               for pr in ("fp64", "fp32") for cy, kl in (("V", 0), ("W", 0), ("K", 0), ("K", 1))],
    # pairwise sweeps composed per level (aggregates of up to 2^sweeps rows)
    "coarsening": [(f"{sw} sweep{'s' if sw > 1 else ''} per level {pr}", pr, dict(sweeps=sw))
                   for pr in ("fp64", "fp32") for sw in (1, 2, 3, 4)],
    # one flexible-CG iteration replayed from a HIP graph, or every kernel launched
    "graph": [(f"{cy} {pr} {'graph replay' if g else 'eager launches'}", pr, dict(cycle=cy, graph=g))
              for cy in ("V", "W") for pr in ("fp64", "fp32") for g in (True, False)],
    # V-cycle levels from the first with at most 2048 rows applied as one dense
    # operator formed at setup, or level by level
    "fold": [(f"V {pr} {'folded small levels' if f else 'level by level'}", pr, dict(fold=f))
             for pr in ("fp64", "fp32") for f in (True, False)],
    # the smooth vector w the matching weights and prolongator are built from
    "smoothvec": [(f"w = {wk} {pr}", pr, dict(wvec=wk)) for pr in ("fp64", "fp32")
                  for wk in ("ones", "uniform[0.5,1.5)", "grid sine (lowest Laplacian mode)")],
}


def ablation(args, c, step):
    import numpy as np
    import torch
    from paper_1810_04221_amd import problems
    rows = []
    for label, prec, kw in ABLATIONS[args.ablation]:
        kw = dict(kw)
        if "wvec" in kw:
            wk = kw.pop("wvec")
            if wk == "ones":
                wv = np.ones(c["n"])
            elif wk.startswith("uniform"):
                wv = np.random.default_rng(17).uniform(0.5, 1.5, c["n"])
            else:
                nx = int(round(c["n"] ** (1.0 / 3.0)))
                if nx ** 3 != c["n"] or not c["name"].startswith("poisson3d"):
                    log(f"skipping '{label}': needs a cubic 3-D Poisson grid")
                    continue
                wv = problems.grid_sine_vector(nx)
            kw["wvec"] = torch.as_tensor(wv, device="cuda")
        for _ in range(max(1, args.warmup)):
            step(prec, 0, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [step(prec, 0, **kw)[0] for _ in range(args.steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        inf = infos[-1]
        row = {"setting": label, "precision": prec, "ms_per_step": ms, "mdofs": c["n"] / (ms * 1e-3) / 1e6,
               "setup_ms": sum(i["t_setup_ms"] for i in infos) / len(infos),
               "solve_ms": sum(i["t_solve_ms"] for i in infos) / len(infos), "iters": inf["iters"],
               "relres": inf["relres"], "levels": len(inf["n"])}
        rows.append(row)
        log(f"{label:48s} {ms:8.2f} ms/step  setup {row['setup_ms']:7.2f}  solve {row['solve_ms']:7.2f}  "
            f"iters {row['iters']:4d}  relres {row['relres']:.2e}")
    print(json.dumps({"ablation": args.ablation, "workload": c["name"], "n": c["n"], "steps": args.steps,
                      "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
