#!/usr/bin/env python3
"""Benchmark of the H^2 matrix-vector product on one MI355X.

Workload (default): Laplace single layer on the unit icosphere refined 8 times
(1,310,720 triangles), tensor Chebyshev interpolation of order 4 (k = 64),
leaf size 64, admissibility max(diam) <= dist (eta = 1/2), near field by the
7-point rule with Sauter-Schwab order 4 for touching pairs, coupling, transfer,
leaf and near-field data stored in FP32 with FP32 accumulation; x ~ N(0,1),
seed 3.  A step is one full product y <- y + G~ x (forward transformation,
coupling, backward transformation, near field) with x and y resident in HBM.

Prints one JSON line with the throughput, the roofline of the dominant kernel
(the coupling phase, HIP events on the launch stream), the same product in FP64
storage for comparison, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (mesh kind, level, order, leaf, storage, seed)
    "sphere1310k_m4_f32": ("sphere", 8, 4, 64, "f32", 3),
    "sphere1310k_m4_f64": ("sphere", 8, 4, 64, "f64", 3),
    "sphere327k_m4_f64": ("sphere", 7, 4, 64, "f64", 2),
    "cube786k_m4_f32": ("cube", 256, 4, 64, "f32", 4),
    "sphere5120_m4_f64": ("sphere", 4, 4, 64, "f64", 2),
}
# the same products with the coupling matrices evaluated during the product
OTF_WORKLOADS = {"sphere1310k_m4_f32_otf": "sphere1310k_m4_f32", "sphere1310k_m4_f64_otf": "sphere1310k_m4_f64"}
# Peak rate of the on-the-fly coupling kernel in coupling entries per second:
# each entry takes two FP32 FMAs (64 lanes per CU per clock; packed FP32 is not
# used) and one v_rsq_f32, which issues at half that rate on gfx950 (32 lanes per
# CU per clock, measured with a throughput probe), so 2/64 + 1/32 CU clocks per
# entry on 256 CUs at 2.4 GHz.
OTF_F32_PEAK_TENTRY = 256 * 2.4e9 / (2.0 / 64 + 1.0 / 32) / 1e12
# many right-hand sides: (mesh kind, level, order, leaf, storage, seed, nrhs)
MULTI = {"cube786k_m4_r64": ("cube", 256, 4, 64, "f32", 4, 64)}
MFMA_F32_PEAK_TFS = 157.3
# Helmholtz products: (mesh kind, level, order, leaf, storage, seed, kappa)
HELMHOLTZ = {"sphere327k_helmholtz_k4": ("sphere", 7, 4, 64, "f32", 2, 4.0),
             "sphere1310k_helmholtz_k4": ("sphere", 8, 4, 64, "f32", 3, 4.0)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure(A, x, y, steps, warmup, torch, h2):
    for _ in range(warmup):
        A.matvec(x, y)
    torch.cuda.synchronize()
    h2.h2_profile(A.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        A.matvec(x, y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = h2.h2_profile_read(A.h)
    h2.h2_profile(A.h, False)
    return el, prof


def graph_timing(A, x, y, torch, reps=20, warmup=5):
    """Median and p90 of single products replayed from a captured HIP graph,
    each timed with HIP events on the replay stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        A.matvec(x, y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matvec(x, y)
    for _ in range(warmup):
        g.replay()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del g
    ms.sort()
    return {"replays": reps, "median_ms": ms[len(ms) // 2], "p90_ms": ms[int(0.9 * (len(ms) - 1))],
            "matvec_per_s_median": 1e3 / ms[len(ms) // 2]}


_ORACLE = {}


def _oracle_setup(kind, level, order, leaf, seed):
    """The oracle's trees for the workload (built once, shared by forked workers)."""
    import h2_inputs as I
    from oracle.h2 import H2Oracle
    from oracle.kernels import Kernel

    V, T = I.mesh_for(kind, level)
    H = H2Oracle(V, T, Kernel(), m=order, leaf=leaf, eta=0.5, build_blocks=False)
    x = I.random_vector(H.mesh.n, seed, "normal")
    subs = [H.tree.root]
    while subs[0].level < 5 and all(c.children for c in subs):
        subs = [ch for c in subs for ch in c.children]
    _ORACLE.update(H=H, x=x, subs=subs, seed=seed)


def _oracle_sample(worker, budget_s):
    """Oracle (FP64, Algorithms 1-3 as written) timed on a sample of the product.

    Forward/backward transformation: Algorithms 1 and 2 on one subtree at depth
    5 (about 1/32 of the clusters; worker w takes subtree w).  Interaction phase:
    Algorithm 3 on the admissible and inadmissible leaves of the block rows of
    random leaf clusters (matrices assembled first, then applied and timed)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    H, x, subs = _ORACLE["H"], _ORACLE["x"], _ORACLE["subs"]
    with threadpool_limits(limits=1):
        ncl = len(H.tree.clusters)
        sub = subs[worker % len(subs)]
        nsub = sum(1 for _ in _walk(sub))
        xhat = [None] * ncl
        t0 = time.perf_counter()
        H.forward(sub, x, xhat)
        t_fwd = time.perf_counter() - t0
        yhat = [np.zeros(H.k) if v is None else v.copy() for v in xhat]
        y = np.zeros(H.mesh.n)
        t0 = time.perf_counter()
        H.backward(sub, yhat, y)
        t_bwd = time.perf_counter() - t0
        rng = np.random.default_rng(_ORACLE["seed"] + 1000 * worker)
        adm, near = [], []
        t_start = time.perf_counter()
        for lid in rng.permutation(len(H.tree.leaves)):
            a, nn = H.row_blocks(H.tree.leaves[lid])
            adm += a
            near += nn
            for t_, s_ in a:
                H.S(t_, s_)
                if xhat[s_.id] is None:
                    xhat[s_.id] = np.zeros(H.k)
            for t_, s_ in nn:
                H.N(t_, s_)
            if time.perf_counter() - t_start > 0.6 * budget_s:
                break
        yh = np.zeros(H.k)
        t0 = time.perf_counter()
        for t_, s_ in adm:
            yh = yh + H.S(t_, s_) @ xhat[s_.id]
        t_adm = time.perf_counter() - t0
        t0 = time.perf_counter()
        for t_, s_ in near:
            y[t_.idx] += H.N(t_, s_) @ x[s_.idx]
        t_near = time.perf_counter() - t0
    return dict(t_fwd=t_fwd, t_bwd=t_bwd, nsub=nsub, ncl=ncl, t_adm=t_adm, nadm=len(adm), t_near=t_near,
                nnear=len(near))


def cpu_baseline_child(args):
    """Child process of the CPU baseline: the oracle on `workers` host cores, each
    core timing its own sample (its own subtree and block rows); no GPU use."""
    import multiprocessing as mp

    kind, level, order, leaf, storage, seed = WORKLOADS[args.workload]
    W = args.cpu_baseline_child
    _oracle_setup(kind, level, order, leaf, seed)
    budget = args.cpu_budget_s
    if W == 1:
        parts = [_oracle_sample(0, budget)]
    else:
        with mp.get_context("fork").Pool(W) as pool:
            parts = pool.starmap(_oracle_sample, [(w, budget) for w in range(W)])
    est = []
    for p in parts:
        est.append((p["t_fwd"] + p["t_bwd"]) * p["ncl"] / p["nsub"] + p["t_adm"] * args.n_adm / max(1, p["nadm"])
                   + p["t_near"] * args.n_near / max(1, p["nnear"]))
    # each core computes its share of the product at its own measured rate
    rate = sum(1.0 / e for e in est)
    sample = ("oracle Algorithms 1-2 on a depth-5 subtree (about 1/%d of the clusters) and Algorithm 3 on "
              "%d admissible + %d inadmissible blocks (block rows of random leaves) per core, FP64, matrices "
              "pre-assembled, one BLAS thread per process; scaled to the whole product, the cores' rates added"
              % (len(_ORACLE["subs"]), sum(p["nadm"] for p in parts) // W, sum(p["nnear"] for p in parts) // W))
    print(json.dumps({"value": rate, "unit": "H2 matvecs/s", "cores": W, "kind": "oracle", "sample": sample,
                      "est_seconds_per_matvec_per_core": est}), flush=True)


def cpu_baseline(args, kind_workload, n_adm, n_near, workers, budget_s):
    """Runs the oracle baseline in a child process (fresh interpreter, no GPU)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", str(workers), "--workload",
           kind_workload, "--n-adm", str(n_adm), "--n-near", str(n_near), "--cpu-budget-s", str(budget_s)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"value": None, "error": r.stderr[-2000:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def read_ceiling(torch, h2, gib=4.0, reps=10):
    """HBM read rate of the library's read-only streaming kernel (16-byte
    non-temporal loads, as the product kernels issue them) over `gib` GiB, far
    beyond the caches, with 4, 8 and 16 loads in flight per thread; HIP events on
    the launch stream, mean over `reps`; the best of the three is the ceiling."""
    nbytes = int(gib * (1 << 30))
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(4096, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    rates = {}
    for loads in (4, 8, 16):
        for _ in range(2):
            h2.h2_stream_read(buf, sink, loads, stream=s.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            h2.h2_stream_read(buf, sink, loads, stream=s.cuda_stream)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rates[loads] = {"avg_launch_ms": ms, "GBs": nbytes / (ms * 1e-3) / 1e9}
    del buf, sink
    torch.cuda.empty_cache()
    best = max(rates, key=lambda k: rates[k]["GBs"])
    return {"kernel": "stream_read", "bytes_per_launch": nbytes, "loads_in_flight": best,
            "avg_launch_ms": rates[best]["avg_launch_ms"], "GBs": rates[best]["GBs"],
            "by_loads_in_flight": rates}


def copy_probe(torch, gib=2.0, reps=5):
    """Device-to-device copy of a known size: measured HBM rate (read + write bytes)."""
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * 4 * n, "GBs": 2 * 4 * n * reps / el / 1e9}


def recorded_traffic(workload, kernel="coupling64", source="matvec.hip"):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    profiles/<kernel>_<workload>_pmc.md, or None if the kernel's source file
    changed since the counters were taken (or none were taken)."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", "%s_%s_pmc.md" % (kernel, workload))
    src = os.path.join(ROOT, "paper_2203_05665_amd", "csrc", source)
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    mt = re.search(r"traffic_bytes_per_launch %s: (\d+)" % re.escape(kernel), text)
    mh = re.search(r"%s sha256 prefix: ([0-9a-f]+)" % re.escape(source), text)
    if not (mt and mh):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != mh.group(1):
        return None
    return float(mt.group(1))


def otf_roofline(info, coup_avg_ms, storage):
    """Roofline of the on-the-fly coupling kernel: bound by vector ALU issue
    (FP32: the peak derived above; FP64: no peak figure is claimed)."""
    entries = float(info["n_adm"]) * info["k"] ** 2
    achieved = entries / (coup_avg_ms * 1e-3) / 1e12
    peak = OTF_F32_PEAK_TENTRY if storage == "f32" else None
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tentry/s",
            "frac": achieved / peak if peak else None, "traffic": None, "kernel": "coupling64_otf",
            "entries_per_launch": entries, "avg_launch_ms": coup_avg_ms}


def variant_roofline(info, ph, storage, kw, leaf=64):
    """Roofline of the dominant kernel of a variant: the on-the-fly coupling
    (ALU) when it is the longest phase, else the phase that streams stored data
    from HBM (symmetric coupling: the kept S blocks; near field: the kept panels
    and V)."""
    sb = {"f64": 8, "f32": 4}[storage]
    if kw.get("coupling_otf") and ph["coupling"] >= ph["near"]:
        return otf_roofline(info, ph["coupling"], storage)
    if not kw.get("coupling_otf") and ph["coupling"] >= ph["near"]:
        nbytes, kern = float(info["s_blocks_stored"]) * info["k"] ** 2 * sb, "coupling64_sym"
        ms = ph["coupling"]
    else:
        nbytes = float(info["near_entries_stored"] + info["n"] * info["k"]) * sb
        kern = "near_backward_sym" if kw.get("symmetric") else ("near_backward64" if leaf <= 64 else "near_backward")
        ms = ph["near"]
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": kern, "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": ms}


def _walk(c):
    yield c
    for ch in c.children:
        yield from _walk(ch)


def bench_helmholtz(args):
    """Helmholtz e^{i kappa r}/(4 pi r) products (complex vectors, FP32 storage): one
    column and 16 columns, coupling stored and evaluated during the product."""
    import numpy as np
    import torch

    import h2_inputs as I
    from paper_2203_05665_amd import h2

    kind, level, order, leaf, storage, seed, kappa = HELMHOLTZ[args.workload]
    V, T = I.mesh_for(kind, level)
    n = T.shape[0]
    log("bench: %s n=%d m=%d leaf=%d storage=%s kappa=%g" % (args.workload, n, order, leaf, storage, kappa))
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((16, n)) + 1j * rng.standard_normal((16, n))
    Xd = torch.tensor(X, device="cuda").t()            # n x 16, column-major
    x1 = Xd[:, 0].contiguous()
    res = {}
    for otf in (False, True):
        A = h2.H2Matrix(V, T, kernel="helmholtz", kappa=kappa, order=order, leaf=leaf, eta=0.5, storage=storage,
                        coupling_otf=otf)
        torch.cuda.synchronize()
        for cols, xx in ((1, x1), (16, Xd)):
            yy = torch.zeros_like(xx)
            el, prof = measure(A, xx, yy, args.steps, args.warmup, torch, h2)
            ph = {k: v[0] / max(1, v[1]) for k, v in prof.items()}
            key = "%s_%dcol" % ("on_the_fly" if otf else "stored", cols)
            res[key] = {"ms_per_product": 1e3 * el / args.steps, "rhs_products_per_s": cols * args.steps / el,
                        "phase_ms": ph, "device_bytes": A.info["bytes_total"], "n_adm": A.info["n_adm"]}
        A.close()
        del A
        torch.cuda.empty_cache()
    st = res["stored_1col"]
    sbytes = float(st["n_adm"]) * 64 * 64 * 8             # complex FP32 S of every admissible block
    ach = sbytes / (st["phase_ms"]["coupling"] * 1e-3) / 1e9
    out = {
        "metric": "complex H2 matvecs/s", "value": 1e3 / st["ms_per_product"], "unit": "matvec/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": st["ms_per_product"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "mesh": "%s level %d" % (kind, level), "triangles": n,
                   "order_m": order, "k": order ** 3, "leaf": leaf, "eta": 0.5, "storage": storage,
                   "kernel": "helmholtz", "kappa": kappa},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "coupling64c",
                     "algorithmic_bytes_per_launch": sbytes, "avg_launch_ms": st["phase_ms"]["coupling"]},
        "results": res,
    }
    print(json.dumps(out), flush=True)


def bench_multi(args):
    """Many right-hand sides in one call (matrix-core path): one JSON line."""
    print(json.dumps(run_multi(args, args.workload, full=True)), flush=True)


def run_multi(args, workload, full=True):
    """The many-right-hand-side product on its workload; with full, also the
    variant with the coupling evaluated during the product and the columns one
    at a time."""
    import torch

    import h2_inputs as I
    from paper_2203_05665_amd import h2

    kind, level, order, leaf, storage, seed, R = MULTI[workload]
    V, T = I.mesh_for(kind, level)
    n = T.shape[0]
    log("bench: %s n=%d m=%d leaf=%d storage=%s nrhs=%d" % (workload, n, order, leaf, storage, R))
    t0 = time.perf_counter()
    A = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = A.info
    X = torch.tensor(I.random_vector(n, seed, "normal", nrhs=R), dtype=torch.float64, device="cuda")
    X = X.t().contiguous().t()
    Y = torch.zeros_like(X)
    if getattr(args, "copy_probe", False):
        copy = copy_probe(torch)  # a copy of known size, for the counter calibration
    tuning = A.tune(R, "f64", reps=5)  # tile shapes for R columns, before the timed region
    tuning_order = A.tune(R, "f64", reps=5, knob="row_order")
    log("bench: tuning %s %s" % (tuning, tuning_order))
    el, prof = measure(A, X, Y, args.steps, args.warmup, torch, h2)
    try:
        graph = graph_timing(A, X, Y, torch)  # the whole pass captured once, replayed
        graph["rhs_matvec_per_s_median"] = R * graph["matvec_per_s_median"]
    except Exception as e:  # reported, not fatal
        graph = {"error": repr(e)}
    k = info["k"]
    # the coupling kernel the tuned schedule runs (row groups on 64-column passes)
    coup_kernel = "mcoupling_grp" if tuning_order.get("chosen") == 3 and tuning.get("chosen") == 64 else "mcoupling"
    # every step as a dense contraction over R columns: V twice, E twice (dense on
    # this path), S, near field
    flops_total = 2.0 * R * (2.0 * n * k + 2.0 * k * k * (info["nclusters"] - 1) + k * k * info["n_adm"]
                             + info["near_entries"])
    coup_flops = 2.0 * k * k * info["n_adm"] * R
    coup_ms = prof["coupling"][0] / max(1, prof["coupling"][1])
    achieved = coup_flops / (coup_ms * 1e-3) / 1e12
    out = {
        "metric": "RHS x H2 matvecs/s", "value": R * args.steps / el, "unit": "rhs-matvec/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "mesh": "%s level %d" % (kind, level), "triangles": n,
                   "order_m": order, "k": k, "leaf": leaf, "eta": 0.5, "storage": storage, "rhs": R},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_F32_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_F32_PEAK_TFS,
                     "traffic": recorded_traffic(workload, coup_kernel, "matvec_multi.hip"), "kernel": coup_kernel,
                     "algorithmic_flops_per_launch": coup_flops, "avg_launch_ms": coup_ms},
        "path": {"flops": flops_total, "TFLOPs": flops_total / (el / args.steps) / 1e12,
                 "phase_ms": {kk: v[0] / max(1, v[1]) for kk, v in prof.items()}, "build_s": build_s,
                 "device_bytes": info["bytes_total"]},
        "tuning": tuning, "tuning_row_order": tuning_order, "graph_replay": graph,
    }
    if getattr(args, "copy_probe", False):
        out["copy_probe"] = copy
    A.close()
    del A
    torch.cuda.empty_cache()
    if not full:
        return out
    if not args.no_otf:
        log("bench: many right-hand sides with the coupling evaluated during the product")
        C = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage, coupling_otf=True)
        Yc = torch.zeros_like(X)
        tuning_c = C.tune(R, "f64", reps=5)
        elc, profc = measure(C, X, Yc, args.steps, args.warmup, torch, h2)
        cms = profc["coupling"][0] / max(1, profc["coupling"][1])
        out["otf_variant"] = {
            "value": R * args.steps / elc, "unit": "rhs-matvec/s", "ms_per_step": 1e3 * elc / args.steps,
            "phase_ms": {kk: v[0] / max(1, v[1]) for kk, v in profc.items()},
            "device_bytes": C.info["bytes_total"], "tuning": tuning_c,
            "roofline": {"bound": "mfma", "achieved": coup_flops / (cms * 1e-3) / 1e12, "peak": MFMA_F32_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": coup_flops / (cms * 1e-3) / 1e12 / MFMA_F32_PEAK_TFS,
                         "traffic": None, "kernel": "mcoupling_otf", "algorithmic_flops_per_launch": coup_flops,
                         "avg_launch_ms": cms}}
        C.close()
    # the same columns one at a time, for comparison
    B = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage)
    x1 = X[:, 0].contiguous()
    y1 = torch.zeros_like(x1)
    el1, _ = measure(B, x1, y1, max(3, args.steps), 1, torch, h2)
    out["single_rhs_compare"] = {"value": max(3, args.steps) / el1, "unit": "matvec/s",
                                 "speedup_per_rhs": (R * args.steps / el) / (max(3, args.steps) / el1)}
    B.close()
    return out


def bench_serve(args):
    """Poisson stream of solve requests served with continuous batching: one JSON line."""
    st = run_serve(args, args.serve_requests, args.serve_rate, args.serve_deadline_s)
    span = st["serving"]["span_s"]
    out = {
        "metric": "served solves/s", "value": st["serving"]["done"] / span, "unit": "solves/s", "n_gpus": 1,
        "steps": args.serve_requests, "warmup": 0, "ms_per_step": 1e3 * span / max(1, st["serving"]["done"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64-refinement",
        "data": "synthetic", "config": st["config"], "serving": st["serving"],
    }
    print(json.dumps(out), flush=True)


def run_serve(args, nreq, rate, deadline_s):
    """Poisson stream of `nreq` solve requests at `rate` per second on the seven
    meshes and three kernels of the serving workload, served with continuous
    batching; returns the configuration and the service statistics."""
    import numpy as np
    import torch

    import h2_inputs as I
    from paper_2203_05665_amd.serve import GPUBackend, H2Server

    meshes = {"sphere%d" % r: I.icosphere(r) for r in (4, 5, 6, 7)}
    meshes.update({"cube%d" % N: I.cube_surface(N) for N in (32, 64, 128)})
    kernels = [("laplace", 0.0), ("helmholtz", 2.0), ("helmholtz", 4.0)]
    S = H2Server(GPUBackend(order=4, leaf=64, eta=0.5, storage="f32", coupling_otf=not args.no_otf),
                 mem_budget=args.serve_budget_gb * 1e9, max_active=args.serve_slots,
                 vec_budget=args.serve_vec_gb * 1e9)
    for name, (V, T) in meshes.items():
        S.register_mesh(name, V, T)
    t0 = time.perf_counter()
    for name in meshes:                       # structures are built once and stay resident
        for kern, kap in kernels:
            S._make_resident((name, kern, float(kap)))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log("serve: %d structures resident, %.1f GB, built in %.1f s" % (len(S.resident), S.used_bytes() / 1e9, build_s))
    rng = np.random.default_rng(5)
    names = sorted(meshes)
    gaps = rng.exponential(1.0 / rate, nreq)
    arrivals = np.cumsum(gaps)
    reqs_spec = []
    for i in range(nreq):
        name = names[rng.integers(len(names))]
        kern, kap = kernels[rng.integers(3)]
        r = int(rng.integers(1, 17))
        V, T = meshes[name]
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        B = rng.standard_normal((T.shape[0], r))
        if kern == "helmholtz":
            B = B + 1j * rng.standard_normal((T.shape[0], r))
        B[:, 0] = area
        reqs_spec.append((name, kern, kap, B))
    start = S.clock() + 0.05
    for (name, kern, kap, B), a in zip(reqs_spec, arrivals):
        S.submit(name, B, kernel=kern, kappa=kap, rtol=1e-8, arrival=start + a)
    S.run(progress=lambda d: log("serve progress:", json.dumps(d)), progress_every=10.0,
          deadline=start + deadline_s)
    torch.cuda.synchronize()
    st = S.stats()
    span = max(q.finish for q in S.finished) - start
    done = [q for q in S.finished if q.status == "done"]
    res = {
        "config": {"workload": "serve_mix", "meshes": {k: int(v[1].shape[0]) for k, v in meshes.items()},
                   "kernels": ["laplace", "helmholtz k=2", "helmholtz k=4"], "rhs": "U{1..16}",
                   "requests": nreq, "arrival_rate_per_s": rate, "rtol": 1e-8, "slots": args.serve_slots,
                   "storage": "f32 (FP64 iterative refinement)",
                   "coupling": "stored" if args.no_otf else "evaluated during the product"},
        "serving": dict(st, build_s=build_s, span_s=span, resident_GB=S.used_bytes() / 1e9,
                        solves_per_s=len(done) / span if span > 0 else None,
                        rhs_per_s=sum(q.nrhs for q in done) / span if span > 0 else None,
                        failures=S.failures()[:20],
                        iterations_mean=float(np.mean([q.iterations for q in S.finished])),
                        iterations_by_kernel={k: float(np.mean([q.iterations for q in S.finished if q.kernel == k]))
                                              for k in ("laplace", "helmholtz")},
                        latency_p50_by_kernel={k: float(np.percentile([q.latency for q in done if q.kernel == k], 50))
                                               for k in ("laplace", "helmholtz")
                                               if any(q.kernel == k for q in done)}),
    }
    for res_ in S.resident.values():
        S.be.free(res_.obj)
    del S
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere1310k_m4_f32",
                    choices=sorted(WORKLOADS) + sorted(OTF_WORKLOADS) + sorted(MULTI) + sorted(HELMHOLTZ)
                    + ["serve_mix"])
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="mean arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-budget-gb", type=float, default=220.0)
    ap.add_argument("--serve-vec-gb", type=float, default=40.0, help="request vector arena of the service")
    ap.add_argument("--serve-deadline-s", type=float, default=150.0, help="cancel what is unfinished after this")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--n-adm", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--n-near", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-budget-s", type=float, default=20.0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-cores", type=int, default=0, help="host cores for the all-core oracle baseline "
                    "(default: all this process may use, at most 16)")
    ap.add_argument("--recompress", type=float, default=1e-5, metavar="EPS",
                    help="tolerance of the algebraically recompressed variant (default 1e-5)")
    ap.add_argument("--no-recompress", dest="recompress", action="store_const", const=None,
                    help="skip the recompressed variant")
    ap.add_argument("--recompress-full-near", dest="recompress_sym_near", action="store_false",
                    help="recompressed variant with the near field stored in full (default: one block per pair)")
    ap.add_argument("--no-solve", "--no-fp64", dest="no_solve", action="store_true",
                    help="skip the solve comparison (FP64 vs mixed precision vs BF16 coupling)")
    ap.add_argument("--copy-probe", action="store_true", help="also time a device copy of known size")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the read-only streaming kernel")
    ap.add_argument("--no-multi", action="store_true", help="skip the 64-column leg of the default run")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg of the default run")
    ap.add_argument("--bench-serve-requests", type=int, default=100)
    ap.add_argument("--bench-serve-rate", type=float, default=2.0)
    ap.add_argument("--bench-serve-deadline-s", type=float, default=100.0)
    ap.add_argument("--no-otf", action="store_true",
                    help="skip the variant with coupling matrices evaluated during the product")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        return cpu_baseline_child(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the H^2 product here runs on a single MI355X "
              "(multi-GPU sharding is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import h2_inputs as I
    from paper_2203_05665_amd import h2

    if args.workload in MULTI:
        return bench_multi(args)
    if args.workload in HELMHOLTZ:
        return bench_helmholtz(args)
    if args.workload == "serve_mix":
        return bench_serve(args)
    otf = args.workload in OTF_WORKLOADS
    kind, level, order, leaf, storage, seed = WORKLOADS[OTF_WORKLOADS.get(args.workload, args.workload)]
    V, T = I.mesh_for(kind, level)
    n = T.shape[0]
    log("bench: %s n=%d m=%d leaf=%d storage=%s%s" % (args.workload, n, order, leaf, storage,
                                                      " coupling on the fly" if otf else ""))
    t0 = time.perf_counter()
    A = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage, coupling_otf=otf)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = A.info
    log("bench: built in %.2f s, %.2f GB on device, %d admissible / %d near blocks" %
        (build_s, info["bytes_total"] / 1e9, info["n_adm"], info["n_near"]))
    x = torch.tensor(I.random_vector(n, seed, "normal"), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    el, prof = measure(A, x, y, args.steps, args.warmup, torch, h2)
    ms_step = 1e3 * el / args.steps
    sbytes = {"f64": 8, "f32": 4, "f32_sbf16": 2}[storage]
    coup_bytes = float(info["n_adm"]) * info["k"] ** 2 * sbytes
    coup_ms, coup_calls = prof["coupling"]
    coup_avg_ms = coup_ms / max(1, coup_calls)
    achieved = coup_bytes / (coup_avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(args.workload),
            "kernel": "coupling64", "algorithmic_bytes_per_launch": coup_bytes, "avg_launch_ms": coup_avg_ms}
    if otf:
        roof = otf_roofline(info, coup_avg_ms, storage)
    log("bench: %.3f ms/matvec; phases %s" % (ms_step, {k: round(v[0] / max(1, v[1]), 4) for k, v in prof.items()}))
    out = {
        "metric": "H2 matvecs/s", "value": args.steps / el, "unit": "matvec/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"f64": "f64", "f32": "f32", "f32_sbf16": "bf16+f32"}[storage],
        "data": "synthetic",
        "config": {"workload": args.workload, "mesh": "%s level %d" % (kind, level), "triangles": n,
                   "order_m": order, "k": order ** 3, "leaf": leaf, "eta": 0.5, "storage": storage,
                   "accumulate": "f64" if storage == "f64" else "f32", "rhs": 1,
                   "coupling": "evaluated during the product" if otf else "stored"},
        "roofline": roof,
        "path": {"algorithmic_bytes": info["matvec_bytes"],
                 "achieved_GBs": info["matvec_bytes"] / (el / args.steps) / 1e9,
                 "frac_hbm_peak": info["matvec_bytes"] / (el / args.steps) / 1e9 / HBM_PEAK_GBS,
                 "phase_ms": {k: v[0] / max(1, v[1]) for k, v in prof.items()},
                 "build_s": build_s, "device_bytes": info["bytes_total"],
                 "n_adm": info["n_adm"], "n_near": info["n_near"], "near_entries": info["near_entries"],
                 "nclusters": info["nclusters"]},
    }
    try:
        out["graph_replay"] = graph_timing(A, x, y, torch)
    except Exception as e:  # a report, never a reason to lose the line
        out["graph_replay"] = {"error": repr(e)}
    A.close()
    del A
    torch.cuda.empty_cache()
    if not otf and not args.no_otf and storage in ("f32", "f64"):
        # the same product from byte-reducing representations of the same G~
        out["variants"] = {}
        for vname, kw in (("coupling_on_the_fly", dict(coupling_otf=True)), ("symmetric", dict(symmetric=True)),
                          ("coupling_on_the_fly+symmetric", dict(coupling_otf=True, symmetric=True))):
            log("bench: variant %s" % vname)
            B = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage, **kw)
            yb = torch.zeros_like(x)
            elb, profb = measure(B, x, yb, args.steps, args.warmup, torch, h2)
            ph = {k: v[0] / max(1, v[1]) for k, v in profb.items()}
            out["variants"][vname] = {"value": args.steps / elb, "unit": "matvec/s", "ms_per_step": 1e3 * elb / args.steps,
                                      "device_bytes": B.info["bytes_total"],
                                      "algorithmic_bytes": B.info["matvec_bytes"], "phase_ms": ph,
                                      "roofline": variant_roofline(B.info, ph, storage, kw, leaf)}
            B.close()
            del B
            torch.cuda.empty_cache()
    if args.recompress is not None and not otf and storage in ("f32", "f64"):
        # algebraic recompression of the stored representation (smaller uniform rank k')
        log("bench: recompressed variant, eps %g" % args.recompress)
        B = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=storage,
                        symmetric_near=args.recompress_sym_near)
        y0 = torch.zeros_like(x)
        B.matvec(x, y0)
        rc = B.recompress(args.recompress)
        yb = torch.zeros_like(x)
        B.matvec(x, yb)
        torch.cuda.synchronize()
        change = float(np.linalg.norm((yb - y0).cpu().numpy()))
        bound = float(np.sqrt(2.0 * rc["discarded"]) * np.linalg.norm(x.cpu().numpy()))
        tuning_b = B.tune(1, "f64", reps=5)  # slot width of the small-rank coupling
        log("bench: tuning %s" % tuning_b)
        elb, profb = measure(B, x, yb, args.steps, args.warmup, torch, h2)
        ph = {k: v[0] / max(1, v[1]) for k, v in profb.items()}
        sb = {"f64": 8, "f32": 4}[storage]
        inf = B.info
        if ph["coupling"] >= ph["near"]:
            kern = "coupling_small" if inf["k"] <= 32 else "coupling_any"
            nbytes, ms = float(inf["s_blocks_stored"]) * inf["k"] ** 2 * sb, ph["coupling"]
        else:
            kern = "near_backward_sym" if args.recompress_sym_near else (
                "near_backward64" if leaf <= 64 else "near_backward")
            nbytes, ms = float(inf["near_entries_stored"] + inf["n"] * inf["k"]) * sb, ph["near"]
        ach = nbytes / (ms * 1e-3) / 1e9
        out.setdefault("variants", {})["recompressed"] = {
            "value": args.steps / elb, "unit": "matvec/s", "ms_per_step": 1e3 * elb / args.steps,
            "eps": args.recompress, "rank": rc["rank"], "recompress_s": rc["seconds"],
            "near_field": "symmetric (one block per pair)" if args.recompress_sym_near else "full",
            "rel_change_vs_stored": change / float(np.linalg.norm(y0.cpu().numpy())),
            "bytes_V_E_S": [rc["bytes_before"], rc["bytes_after"]], "device_bytes": inf["bytes_total"],
            "algorithmic_bytes": inf["matvec_bytes"], "phase_ms": ph,
            "change_vs_stored": change, "frobenius_bound": bound, "tuning": tuning_b,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": kern,
                         "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": ms}}
        B.close()
        del B
        torch.cuda.empty_cache()
    if not args.no_solve:
        # time to a 1e-8 solve, b_i = |T_i| (z ~ 1 on the unit sphere), CG
        P = V[T]
        area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
        bd = torch.tensor(area, dtype=torch.float64, device="cuda")
        solves = {}
        for st_name in (["f64", storage] if storage != "f64" else ["f64"]) + (["f32_sbf16"] if storage == "f32" else []):
            log("bench: solve with %s storage" % st_name)
            M = h2.H2Matrix(V, T, kernel="laplace", order=order, leaf=leaf, eta=0.5, storage=st_name)
            yy = torch.zeros_like(x)
            elv, _ = measure(M, x, yy, max(3, args.steps // 2), 1, torch, h2)
            mv = max(3, args.steps // 2) / elv
            # a few untimed steps first: the solver's workspace and kernels are set up
            # on the handle's first solve (about 0.1 s once per process and handle)
            z = torch.zeros_like(bd)
            h2.h2_solve(M.h, bd, z, method="cg", rtol=1e-8, maxit=3, refine=st_name != "f64", inner_rtol=1e-4,
                        check=False)
            z = torch.zeros_like(bd)
            torch.cuda.synchronize()
            info_s = h2.h2_solve(M.h, bd, z, method="cg", rtol=1e-8, maxit=2000, refine=st_name != "f64",
                                 inner_rtol=1e-4, check=False)
            torch.cuda.synchronize()
            zz = z.cpu().numpy()
            solves[st_name] = dict(info_s, matvec_per_s=mv, matvec_bytes=M.info["matvec_bytes"],
                                   frac_hbm_peak=M.info["matvec_bytes"] * mv / 1e9 / HBM_PEAK_GBS,
                                   z_minus_1_rms=float(np.sqrt(np.mean((zz - 1.0) ** 2))))
            if st_name == "f64":
                z64 = zz
            else:
                solves[st_name]["rel_diff_to_f64_solution"] = float(np.linalg.norm(zz - z64) / np.linalg.norm(z64))
            M.close()
            del M
            torch.cuda.empty_cache()
        out["solve_compare"] = solves
        if "f64" in solves and storage in solves and storage != "f64":
            out["fp64_compare"] = {"value": solves["f64"]["matvec_per_s"], "unit": "matvec/s",
                                   "speedup_f32_over_f64": solves[storage]["matvec_per_s"] / solves["f64"]["matvec_per_s"],
                                   "time_to_1e-8_f64_s": solves["f64"]["seconds"],
                                   "time_to_1e-8_mixed_s": solves[storage]["seconds"]}
    if args.copy_probe:
        out["copy_probe"] = copy_probe(torch)
    if not args.no_ceiling:
        log("bench: read ceiling")
        ceil = read_ceiling(torch, h2)
        roof = out["roofline"]
        roof["measured_ceiling"] = ceil["GBs"] if roof["unit"] == "GB/s" else None
        roof["frac_of_measured_ceiling"] = roof["achieved"] / ceil["GBs"] if roof["unit"] == "GB/s" else None
        out["read_ceiling"] = ceil
    headline = args.workload == "sphere1310k_m4_f32"
    if headline and not args.no_multi:
        log("bench: many right-hand sides (cube786k, 64 columns)")
        mr = run_multi(args, "cube786k_m4_r64", full=False)
        out["multi_rhs"] = {k: mr[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "roofline", "path",
                                               "tuning", "tuning_row_order", "graph_replay")}
    if headline and not args.no_serve:
        log("bench: serving leg (%d requests at %.1f/s)" % (args.bench_serve_requests, args.bench_serve_rate))
        out["serving"] = run_serve(args, args.bench_serve_requests, args.bench_serve_rate, args.bench_serve_deadline_s)
    if not args.no_cpu_baseline:
        wl = OTF_WORKLOADS.get(args.workload, args.workload)
        cores = args.cpu_cores or min(16, host_cores())
        try:
            log("bench: CPU oracle sample, %d cores" % cores)
            allc = cpu_baseline(args, wl, info["n_adm"], info["n_near"], cores, 12.0)
            log("bench: CPU oracle sample, 1 core")
            one = cpu_baseline(args, wl, info["n_adm"], info["n_near"], 1, 20.0)
            allc["one_core"] = one
            out["cpu_baseline"] = allc
        except Exception as e:  # the baseline is a report, never a reason to lose the line
            out["cpu_baseline"] = {"value": None, "error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
