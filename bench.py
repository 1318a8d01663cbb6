#!/usr/bin/env python3
"""Throughput of the block-sparse contractions of symmetric CTM on one MI355X.

Default (no flags): the batched workload, 64 independent U(1) enlarged
corners C.T.T.a with D drawn from {4..8} and chi from {32..160}: a step is
the three contraction steps of all 64 corners, each step one grouped
bf16x3 GEMM launch (with its gather), replayed from a HIP graph, on
resident synthetic tensors.  `value` = useful flops (sum over matched block
pairs of 2 m n k, a split product counted once) per second.  Beside it: the
same corners as per-contraction FP32 launches (the speedup), the dominant
GEMM's fraction of the bf16x3 MFMA ceiling (BF16 peak / 3), the FP64 oracle
timed on a bounded sample of the corners (`cpu_baseline`), and the full CTM
left move of the D = 6, chi = 64 workload in FP32 (`move_D6_chi64_f32`).

`--config N` times one workload on its own: 1, 2, 4, 6 a full left move
(the four corners, halves, FP64 projectors with truncation to chi,
renormalised and normalised C1', T4', C4'), 3 the SU(2) move, 5 the batched
corners.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "bf16x3": 2516.6 / 3, "bf16x6": 2516.6 / 6}
HEADLINE_METRIC = "useful GFLOP/s per CTM move + % MFMA peak; bf16x3 batched vs FP32 per-block"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6   # FP64 vector (non-MFMA) peak: 256 CUs x 4 SIMDs x 16 FMA lanes x 2 x 2.4 GHz


def build_workload(cfgd, seed, dtype, st, draw, TENSOR_INDEX):
    """Device tensors of the workload filled with the seeded draws."""
    phys, virt, chi, flux = cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"]
    g = cfgd["group"].lower()
    T = {"A": st.Tensor.create([(phys, 1), (virt, 1), (virt, 1), (virt, -1), (virt, -1)], flux, dtype, group=g)}
    T["A"].upload(draw((seed, TENSOR_INDEX["A"]), T["A"].nnz))
    T["a"] = st.double_layer(T["A"])
    dd = T["a"].legs()[0][0]
    legs = {"C1": [(chi, 1), (chi, -1)], "T1": [(chi, 1), (dd, -1), (chi, -1)],
            "T2": [(chi, 1), (dd, 1), (chi, -1)], "T3": [(chi, 1), (dd, 1), (chi, -1)],
            "T4": [(chi, 1), (dd, -1), (chi, -1)]}
    for c in ("C2", "C3", "C4"):
        legs[c] = legs["C1"]
    for n, l in legs.items():
        T[n] = st.Tensor.create(l, 0, dtype, group=g)
        T[n].upload(draw((seed, TENSOR_INDEX[n]), T[n].nnz))
    return T


def sources_sha256():
    """Hash of the library sources (kernels, planner, ABI)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1808_10804_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def traffic_for(kernel_name, workload):
    """HBM bytes per launch of `kernel_name` on `workload` from the committed
    counter summary, if it was taken on the current library sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != sources_sha256() or rec.get("workload") != workload:
        return None
    # batched launches carry a ",batched" suffix in libsymten's own timing
    k = rec.get("kernels", {}).get(kernel_name.replace(",batched", ""))
    return None if k is None else k.get("bytes_per_launch")


def profile_name(rocprof_name):
    """libsymten's profile name of a kernel from its demangled name."""
    import re
    m = re.search(r"symten::(gemm_f32_kernel|gemm_f64_kernel|gemm_bf16_kernel|copy_kernel)<([^()]*)>\(", rocprof_name)
    if not m:
        return None
    fam, args = m.group(1), m.group(2)
    t = re.search(r"TileShape<(\d+), (\d+), (\d+)>", args)
    last = args.rsplit(",", 1)[-1].strip()
    if fam == "gemm_f64_kernel":
        return "gemm_f64_kernel<%sx%sx%s>" % t.groups()
    if fam == "gemm_f32_kernel":
        return "gemm_f32_kernel<%sx%sx%s,f32>" % t.groups()
    if fam == "gemm_bf16_kernel":
        # template arguments after the tile: the number of bf16 planes, then
        # whether the epilogue scatters into the next contraction's panels
        tail = [x.strip() for x in args[args.index(t.group(0)) + len(t.group(0)):].split(",") if x.strip()]
        kind = {"1": "bf16", "2": "bf16x3", "3": "bf16x6"}.get(tail[0], tail[0]) if tail else "?"
        scatter = ",scatter" if len(tail) > 1 and tail[1] == "true" else ""
        return "gemm_bf16_kernel<%sx%sx%s,%s%s>" % (t.groups() + (kind, scatter))
    src = "f64" if "double" in args else "f32"
    dst = {"0": "f32", "1": "f64", "2": "bf16", "3": "bf16x2", "4": "acc", "5": "bf16x3"}.get(last, last)
    return "copy_kernel<%s,%s>" % (src, dst)


def write_traffic(base, workload, command, out=None):
    """profiles/traffic.json (or `out`) from the FETCH_SIZE / WRITE_SIZE
    summaries under `base` (bench and calibration copy), scaled by the
    calibration copy."""
    load = lambda n: json.load(open(os.path.join(base, n + ".summary.json")))
    cal = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        rows = [r for r in load("pmc_copy_" + c) if "copyBuffer" in r["kernel"] and r["counter"] == c]
        cal[c] = rows[0]["avg_per_dispatch"] * 1024.0 / (256 << 20)
    kern = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        for r in load("pmc_" + c):
            name = profile_name(r["kernel"])
            if name is None or r["counter"] != c:
                continue
            k = kern.setdefault(name, {})
            k[c.lower() + "_kib_per_dispatch"] = r["avg_per_dispatch"]
            k[c.lower() + "_dispatches"] = r["dispatches"]
            k[("fetch" if c == "FETCH_SIZE" else "write") + "_bytes_per_launch"] = r["avg_per_dispatch"] * 1024.0 / cal[c]
    for k in kern.values():
        if "fetch_bytes_per_launch" in k and "write_bytes_per_launch" in k:
            k["bytes_per_launch"] = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    rec = {"sources_sha256": sources_sha256(), "workload": workload, "command": command,
           "calibration": {"copy_bytes_each_way": 256 << 20, "fetch_counter_per_byte": cal["FETCH_SIZE"],
                           "write_counter_per_byte": cal["WRITE_SIZE"]},
           "kernels": kern}
    json.dump(rec, open(out or os.path.join(ROOT, "profiles", "traffic.json"), "w"), indent=1)
    return rec


CPU_SAMPLE_SECONDS = 10.0    # the oracle's moves are repeated until this much CPU work
CPU_SAMPLE_MAX_MOVES = 20


def cpu_baseline(cfgd, gpu_flops=None):
    """The FP64 dense oracle timed on the host on full moves of the same
    workload (the oracle as it stands, BLAS threads = host cores), repeated
    until about CPU_SAMPLE_SECONDS of work or CPU_SAMPLE_MAX_MOVES moves."""
    from oracle import u1
    from synth import draw, TENSOR_INDEX, SITE_AND_ENV
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    if cfgd["group"] == "Z2":
        return cpu_baseline_z2(cfgd, threads, gpu_flops)
    w = u1.Workload(cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"])
    vals = {n: draw((cfgd["seed"], TENSOR_INDEX[n]), w.nnz_of(n)) for n in SITE_AND_ENV}
    dt, moves, fl = 0.0, 0, 0
    while moves < CPU_SAMPLE_MAX_MOVES and (moves == 0 or dt < CPU_SAMPLE_SECONDS):
        t0 = time.perf_counter()
        T = w.dense_tensors(vals)
        a, _ = u1.double_layer(T["A"], w.A_legs)
        mv = u1.ctm_left_move(w, T, a, cfgd["chi_target"])
        dt += time.perf_counter() - t0
        moves += 1
        fl += u1.move_gemm_flops(w, mv["proj"]["kept"])["total"]
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{moves} full left move(s) of the same workload (dense FP64, {dt:.1f} s in all)",
            "seconds": dt, "moves": moves}


def cpu_baseline_z2(cfgd, threads, gpu_flops=None):
    """The whole-environment dense FP64 oracle timed on one left move of the
    Z2 workload (inputs embedded on the host from the same seeded draws)."""
    from oracle import u1, ctm
    from synth import draw, TENSOR_INDEX
    L = lambda s, d: u1.Leg(s, d)
    phys, virt, chi = cfgd["phys"], cfgd["virt"], cfgd["chi"]
    A_legs = [L(phys, 1), L(virt, 1), L(virt, 1), L(virt, -1), L(virt, -1)]
    t0 = time.perf_counter()
    A = u1.embed(A_legs, cfgd["flux"], draw((cfgd["seed"], TENSOR_INDEX["A"]), u1.nnz(A_legs, cfgd["flux"], 2)), 2)
    a, a_legs = u1.double_layer(A, A_legs, modulus=2)
    dd = a_legs[0].sectors()
    legs = {"C1": [L(chi, 1), L(chi, -1)], "T1": [L(chi, 1), L(dd, -1), L(chi, -1)],
            "T2": [L(chi, 1), L(dd, 1), L(chi, -1)], "T3": [L(chi, 1), L(dd, 1), L(chi, -1)],
            "T4": [L(chi, 1), L(dd, -1), L(chi, -1)]}
    for c in ("C2", "C3", "C4"):
        legs[c] = legs["C1"]
    D = {n: u1.embed(l, 0, draw((cfgd["seed"], TENSOR_INDEX[n]), u1.nnz(l, 0, 2)), 2) for n, l in legs.items()}
    ctm.left_move([D["C1"], D["C2"], D["C3"], D["C4"]], [D["T1"], D["T2"], D["T3"], D["T4"]], a,
                  cfgd["chi_target"])
    dt = time.perf_counter() - t0
    moves = 1
    while moves < CPU_SAMPLE_MAX_MOVES and dt < CPU_SAMPLE_SECONDS:
        t0 = time.perf_counter()
        ctm.left_move([D["C1"], D["C2"], D["C3"], D["C4"]], [D["T1"], D["T2"], D["T3"], D["T4"]], a,
                      cfgd["chi_target"])
        dt += time.perf_counter() - t0
        moves += 1
    return {"value": None if gpu_flops is None else moves * gpu_flops / dt / 1e9, "unit": "GFLOP/s",
            "cores": int(threads), "kind": "oracle", "seconds": dt, "moves": moves,
            "sample": f"{moves} full left move(s) of the same workload (dense FP64 whole-environment oracle, "
                      f"{dt:.1f} s in all); useful flops counted as on the GPU side"}


def build_corner_inputs(cfgd, key, dtype, st, draw, TENSOR_INDEX):
    """C1, T1, T4, a of one corner-1 contraction with seeded draws."""
    phys, virt, chi, flux = cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"]
    A = st.Tensor.create([(phys, 1), (virt, 1), (virt, 1), (virt, -1), (virt, -1)], flux, dtype)
    A.upload(draw(key + (TENSOR_INDEX["A"],), A.nnz))
    a = st.double_layer(A)
    dd = a.legs()[0][0]
    T = {"a": a}
    legs = {"C1": [(chi, 1), (chi, -1)], "T1": [(chi, 1), (dd, -1), (chi, -1)], "T4": [(chi, 1), (dd, -1), (chi, -1)]}
    for n, l in legs.items():
        T[n] = st.Tensor.create(l, 0, dtype)
        T[n].upload(draw(key + (TENSOR_INDEX[n],), T[n].nnz))
    return T


def cpu_baseline_corners(c5, draws):
    """The FP64 dense oracle timed on the host on the corners of the batched
    workload (the oracle as it stands, BLAS threads = host cores): corners in
    draw order until about CPU_SAMPLE_SECONDS of work.  The oracle builds all
    four enlarged corners of a draw, so the sample counts the useful flops of
    all four."""
    from oracle import u1
    from synth import draw, TENSOR_INDEX, SITE_AND_ENV
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    dt, fl, done = 0.0, 0, []
    for b, d in enumerate(draws):
        if dt >= CPU_SAMPLE_SECONDS:
            break
        w = u1.Workload(c5["phys"], d["virt"], d["chi"], c5["flux"])
        vals = {n: draw((c5["seed"], b, TENSOR_INDEX[n]), w.nnz_of(n)) for n in SITE_AND_ENV}
        t0 = time.perf_counter()
        T = w.dense_tensors(vals)
        a, _ = u1.double_layer(T["A"], w.A_legs)
        u1.enlarged_corners(w, T, a)
        dt += time.perf_counter() - t0
        fl += sum(s["flops"] for k in (1, 2, 3, 4) for s in u1.corner_tables(w, k))
        done.append((d["D"], d["chi_total"]))
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"the four enlarged corners of the first {len(done)} draws of the batched workload "
                      f"(D, chi) = {done} (dense FP64, {dt:.1f} s in all)",
            "seconds": dt, "draws": len(done)}


def roofline_of(k, steps, prec=None, workload=None):
    """Roofline entry of one kernel's libsymten timing record: a GEMM against
    its precision's MFMA peak (useful flops), a gather against HBM
    (algorithmic bytes), both per launch over the launch's average time."""
    avg = k["ms"] / k["launches"]
    if k["name"].startswith("eigh"):
        # the projector stage's FP64 eigensolver: plain FP64 vector arithmetic
        # (no MFMA), its algorithmic flops against the FP64 vector peak
        ach = k["useful_flops"] / k["launches"] / (avg * 1e-3) / 1e12
        r = {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
             "frac": ach / FP64_VECTOR_TFLOPS}
    elif k["name"].startswith("gemm"):
        kp = prec or next(x for x in ("bf16x6", "bf16x3", "bf16", "f64", "f32") if x in k["name"])
        ach = k["useful_flops"] / k["launches"] / (avg * 1e-3) / 1e12
        r = {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[kp], "unit": "TFLOP/s",
             "frac": ach / PEAK_TFLOPS[kp]}
    else:
        ach = k["bytes"] / k["launches"] / (avg * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    r.update({"traffic": traffic_for(k["name"], workload) if workload else None, "kernel": k["name"],
              "avg_launch_ms": avg, "launches_per_step": k["launches"] / steps,
              "algorithmic_bytes_per_launch": k["bytes"] / k["launches"],
              "useful_flops_per_launch": k["useful_flops"] / k["launches"]})
    return r


def bench_batched(args):
    """64 independent corner contractions: one grouped launch per step in
    bf16x3 (HIP graph) against per-contraction FP32 launches."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, batched_draws, TENSOR_INDEX

    c5 = config(5)
    prec = args.prec or "bf16x3"
    use_recorded_tiles(c5["name"])
    draws = batched_draws(c5["seed"], c5["batch"], c5["D_choices"], c5["chi_range"])
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    ins = [build_corner_inputs(dict(phys=c5["phys"], flux=c5["flux"], virt=d["virt"], chi=d["chi"]),
                               (c5["seed"], b), "f32", st, draw, TENSOR_INDEX) for b, d in enumerate(draws)]
    Cs, T1s, T4s, As = ([x[k] for x in ins] for k in ("C1", "T1", "T4", "a"))

    def run_batched():
        return st.enlarged_corners_batched(Cs, T1s, T4s, As, prec=prec, use_graph=True, stream=stream)

    def run_single():
        fl = 0
        for x in ins:
            _, info = st.enlarged_corner(1, x["C1"], x["T1"], x["T4"], x["a"], prec="f32", stream=stream)
            fl += info["useful_flops"]
        return fl

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, r

    ms_b, (outs, info) = timed(run_batched, args.steps)
    del outs
    ms_s, fl_s = timed(run_single, max(1, args.steps // 2))
    flops = info["useful_flops"]
    # per-kernel durations: the same batched launches run eagerly, each
    # bracketed by HIP events on its stream (a graph replay carries no
    # per-launch events)
    st.profile_begin()
    for _ in range(args.steps):
        st.enlarged_corners_batched(Cs, T1s, T4s, As, prec=prec, use_graph=False, stream=stream)
    torch.cuda.synchronize()
    kst = st.profile_end()
    gemms = [k for k in kst if k["name"].startswith("gemm")]
    gathers = [k for k in kst if k["name"].startswith("copy")]
    dom = max(gemms, key=lambda k: k["ms"]) if gemms else None
    value = flops / (ms_b * 1e-3) / 1e9
    out = {
        "metric": HEADLINE_METRIC,
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic (seeded Gaussian blocks)",
        "config": {"workload": c5["name"], "what": c5["what"] + ": three grouped steps, HIP graph",
                   "batch": c5["batch"], "D": [d["D"] for d in draws], "chi": [d["chi_total"] for d in draws]},
        "roofline": roofline_of(dom, args.steps, prec, c5["name"]) if dom else None,
        "step_mfma_frac": value / 1e3 / PEAK_TFLOPS[prec],
        "useful_flops": flops,
        "per_contraction_f32": {"ms": ms_s, "gflops": fl_s / (ms_s * 1e-3) / 1e9,
                                "step_mfma_frac": fl_s / (ms_s * 1e-3) / 1e12 / PEAK_TFLOPS["f32"]},
        "speedup_vs_per_contraction_f32": ms_s / ms_b,
        "gather": roofline_of(max(gathers, key=lambda k: k["ms"]), args.steps, None, c5["name"]) if gathers else None,
        "kernels": sorted(kst, key=lambda k: -k["ms"])[:6],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_corners(c5, draws)
    return out


def bench_su2(args):
    """SU(2) workload: one full left move on reduced tensors (recoupling
    scalars in the gathers, projectors per total spin), against the same move
    on the U(1)-expanded (S^z) tensors through the same kernels, truncated to
    the same number of states.  a = A A* is the double layer of a seeded
    SU(2) site tensor (physical spin 1/2)."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX

    c = config(3)
    chi, dd = c["chi"], c["dd"]
    prec = args.prec or "f32"
    dtype = "f64" if prec == "f64" else "f32"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    legs = {"T1": [(chi, 1), (dd, -1), (chi, -1)], "T2": [(chi, 1), (dd, 1), (chi, -1)],
            "T3": [(chi, 1), (dd, 1), (chi, -1)], "T4": [(chi, 1), (dd, -1), (chi, -1)]}
    for n in ("C1", "C2", "C3", "C4"):
        legs[n] = [(chi, 1), (chi, -1)]
    R = {}
    for n, l in legs.items():
        R[n] = st.Tensor.create(l, dtype=dtype, group="su2", stream=stream)
        R[n].upload(draw((c["seed"], TENSOR_INDEX[n]), R[n].nnz), stream=stream)
    v = c["virt"]
    A = st.Tensor.create([(c["phys"], 1), (v, 1), (v, 1), (v, -1), (v, -1)], dtype=dtype, group="su2", stream=stream)
    A.upload(draw((c["seed"], TENSOR_INDEX["A"]), A.nnz), stream=stream)
    R["a"] = st.double_layer(A, stream=stream)
    U = {n: t.to_u1(stream=stream) for n, t in R.items()}

    def runner(T, chi_states):
        env = st.CtmEnv([T[k] for k in ("C1", "C2", "C3", "C4")], [T[k] for k in ("T1", "T2", "T3", "T4")])

        def step(stats=False):
            env.set(0, T["C1"])
            env.set(3, T["C4"])
            env.set(7, T["T4"])
            return env.move(T["a"], chi_states, prec=prec, stats=stats, stream=stream)
        return step

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    step_r = runner(R, c["chi_target"])
    ms_r = timed(step_r)
    sr = step_r(stats=True)
    kept_states = sum((tj + 1) * k for tj, k in sr["kept"].items())
    step_u = runner(U, kept_states)
    ms_u = timed(step_u)
    su = step_u(stats=True)
    fl = lambda x: x["flops_corners"] + x["flops_halves"] + x["flops_renorm"]
    st.profile_begin()
    for _ in range(args.steps):
        step_r()
    torch.cuda.synchronize()
    kst = st.profile_end()
    dom = max(kst, key=lambda k: k["ms"])
    roof = roofline_of(dom, args.steps, None, c["name"])
    gemms = [k for k in kst if k["name"].startswith("gemm")]
    gemm_roof = roofline_of(max(gemms, key=lambda k: k["ms"]), args.steps, None, c["name"]) if gemms else None
    phases = ("ms_corners", "ms_halves", "ms_proj", "ms_renorm", "ms_total")
    out = {
        "metric": "useful GFLOP/s per CTM move (SU(2) reduced left move, sector GEMMs on MFMA)",
        "value": fl(sr) / (ms_r * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_r, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic (seeded Gaussian reduced blocks)",
        "config": {"workload": c["name"], "virtual": c["virt"], "chi_multiplets": chi, "dd_multiplets": dd,
                   "chi_states": c["chi_target"], "parallelism": "single GPU"},
        "roofline": roof, "gemm_roofline": gemm_roof,
        "reduced": {"ms": ms_r, "useful_flops": fl(sr), "phase_ms": {k: sr[k] for k in phases},
                    "kept_multiplets": sr["kept"], "kept_states": kept_states},
        "u1_expanded": {"ms": ms_u, "useful_flops": fl(su), "gflops": fl(su) / (ms_u * 1e-3) / 1e9,
                        "phase_ms": {k: su[k] for k in phases}},
        "speedup_vs_u1_expanded": ms_u / ms_r, "flop_ratio_expanded_over_reduced": fl(su) / fl(sr),
        "kernels": sorted(kst, key=lambda k: -k["ms"])[:6],
    }
    print(json.dumps(out))


def bench_corners(args):
    """The four enlarged corners of a workload through the single-layer route
    (A and A* absorbed separately) against the double-layer route (a = A A*
    built once, as in a CTM run), one corner call at a time on one stream."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX
    cfgd = config(move_config(args.config))
    prec = args.prec or {"sweep": "f32"}.get(cfgd["prec"], cfgd["prec"])
    dtype = "f64" if prec == "f64" else "f32"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    T = build_workload(cfgd, cfgd["seed"], dtype, st, draw, TENSOR_INDEX)
    names = {1: ("C1", "T1", "T4"), 2: ("C2", "T1", "T2"), 3: ("C3", "T3", "T2"), 4: ("C4", "T3", "T4")}

    def single():
        fl = 0
        for w, n in names.items():
            _, inf = st.enlarged_corner_single_layer(w, T[n[0]], T[n[1]], T[n[2]], T["A"], prec=prec, stream=stream)
            fl += inf["useful_flops"]
        return fl

    def double():
        fl = 0
        for w, n in names.items():
            _, inf = st.enlarged_corner(w, T[n[0]], T[n[1]], T[n[2]], T["a"], prec=prec, stream=stream)
            fl += inf["useful_flops"]
        return fl

    res = {}
    for name, fn in (("single", single), ("double", double)):
        for _ in range(args.warmup):
            fl = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        res[name] = ((time.perf_counter() - t0) * 1e3 / args.steps, fl)
    out = {
        "metric": "ms per four enlarged corners, single-layer route (A and A* absorbed separately)",
        "value": res["single"][0], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["single"][0], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic (seeded Gaussian blocks)",
        "config": {"workload": cfgd["name"], "what": "the four enlarged corners of the move", "D_virtual": cfgd["virt"],
                   "chi_sectors": cfgd["chi"], "parallelism": "single GPU"},
        "double_layer_ms": res["double"][0], "speedup_vs_double_layer": res["double"][0] / res["single"][0],
        "useful_flops_single": res["single"][1], "useful_flops_double": res["double"][1],
    }
    print(json.dumps(out))


def bench_cell(args):
    """A 2 x 2 unit cell of the workload's site (four independent draws of
    the site and its environment): one left move of the cell = four cuts,
    each from the enlarged corners of its 2 x 2 block, and eight
    renormalised tensors per column."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX
    cfgd = config(move_config(args.config))
    prec = args.prec or {"sweep": "f32"}.get(cfgd["prec"], cfgd["prec"])
    dtype = "f64" if prec == "f64" else "f32"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    env_names = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")
    sites = [[build_workload(cfgd, cfgd["seed"] + 100 * (2 * x + y), dtype, st, draw, TENSOR_INDEX) for y in range(2)]
             for x in range(2)]

    def fresh():
        return st.CtmCell([[([s[k] for k in env_names[:4]], [s[k] for k in env_names[4:]]) for s in col]
                           for col in sites])
    a = [[s["a"] for s in col] for col in sites]
    cell = fresh()
    for _ in range(args.warmup):
        cell = fresh()
        cell.move(a, cfgd["chi_target"], prec=prec, stream=stream)
    torch.cuda.synchronize()
    cells = [fresh() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for c in cells:
        c.move(a, cfgd["chi_target"], prec=prec, stream=stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    out = {
        "metric": "ms per left move of a 2 x 2 unit cell (four cuts, one projector pair each)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic (seeded Gaussian blocks, four draws)",
        "config": {"workload": cfgd["name"] + "_cell2x2", "D_virtual": cfgd["virt"], "chi": cfgd["chi_target"],
                   "chi_sectors": cfgd["chi"], "parallelism": "single GPU"},
        "ms_per_cut": ms / 4,
    }
    print(json.dumps(out))


def bench_unit(args):
    """The CTM part of the paper's timed optimisation unit (Sec. 4): a 2 x 2
    unit cell re-converged with 8 steps, each one move toward every side
    (left, top, right, bottom), at bond dimension 3 and chi = 10 (3 + 1) = 40
    in FP64 -- the geometry of the paper's U(1) timing at d = 3 -- with
    seeded Gaussian site tensors
    (four draws) and environments in place of an optimised state.  A timed
    step is one whole re-initialisation (32 cell moves) from a fresh cell."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX, binomial_sectors
    cfgd = config(1)
    prec = args.prec or "f64"
    cfgd.update(name="u1_ctm_unit_D3_chi40_" + prec, virt={-2: 1, 0: 1, 2: 1}, chi=binomial_sectors(40, 5),
                chi_target=40)
    dtype = "f64" if prec == "f64" else "f32"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    env_names = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")
    sites = [[build_workload(cfgd, cfgd["seed"] + 100 * (2 * x + y), dtype, st, draw, TENSOR_INDEX) for y in range(2)]
             for x in range(2)]
    a = [[s["a"] for s in col] for col in sites]

    def fresh():
        return st.CtmCell([[([s[k] for k in env_names[:4]], [s[k] for k in env_names[4:]]) for s in col]
                           for col in sites])

    def unit(cell):
        for _ in range(8):
            for direction in range(4):
                cell.move(a, cfgd["chi_target"], prec=prec, direction=direction, stream=stream)

    for _ in range(args.warmup):
        unit(fresh())
    torch.cuda.synchronize()
    cells = [fresh() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for c in cells:
        unit(c)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kept = len(cells[-1].singular_values())
    out = {
        "metric": "ms per CTM re-initialisation of a 2 x 2 unit cell (8 steps of one move toward each side)",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic (seeded Gaussian blocks, four draws)",
        "config": {"workload": cfgd["name"] + "_cell2x2", "D_virtual": cfgd["virt"], "chi": cfgd["chi_target"],
                   "chi_sectors": cfgd["chi"], "moves": 32, "parallelism": "single GPU"},
        "ms_per_cell_move": ms / 32,
        "kept_values_last_move": kept,
    }
    print(json.dumps(out))


def use_recorded_tiles(workload):
    """GEMM tile choices recorded with the committed counter runs: when
    profiles/tune_<workload>.txt exists (and SYMTEN_TUNE_CACHE is not set),
    the autotuner starts from a private copy of it, so that the launches are
    the ones whose HBM traffic was counted."""
    import shutil
    import tempfile
    path = os.path.join(ROOT, "profiles", "tune_%s.txt" % workload)
    if os.environ.get("SYMTEN_TUNE_CACHE") or not os.path.exists(path):
        return
    fd, tmp = tempfile.mkstemp(prefix="symten_tune_", suffix=".txt")
    os.close(fd)
    shutil.copy(path, tmp)
    os.environ["SYMTEN_TUNE_CACHE"] = tmp


def calibrate_copy():
    """A plain device copy of known size, for scaling the HBM traffic
    counters (FETCH_SIZE / WRITE_SIZE) of the profiled kernels."""
    import torch
    n = 64 << 20                                   # 64 Mi float32 = 256 MiB each way
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes_read": 4 * n, "calibration_copy_bytes_written": 4 * n,
                      "dispatches": 5}))


def pmc_summary(path):
    """Average per dispatch of every counter in the rocprofv3 counter CSVs
    under `path`, per kernel name (KiB for FETCH_SIZE / WRITE_SIZE)."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(path, "**", "*counter_collection*.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            key = (row.get("Kernel_Name", "?"), row.get("Counter_Name", "?"))
            disp = row.get("Dispatch_Id", row.get("Correlation_Id", "?"))
            d = acc.setdefault(key, {})
            d[disp] = d.get(disp, 0.0) + float(row.get("Counter_Value", 0.0))
    out = []
    for (kern, ctr), d in sorted(acc.items()):
        out.append({"kernel": kern, "counter": ctr, "dispatches": len(d), "avg_per_dispatch": sum(d.values()) / len(d)})
    return out


def main():
    if "--calibrate-copy" in sys.argv:
        calibrate_copy()
        return
    if "--pmc-summary" in sys.argv:
        print(json.dumps(pmc_summary(sys.argv[sys.argv.index("--pmc-summary") + 1]), indent=1))
        return
    if "--write-traffic" in sys.argv:
        i = sys.argv.index("--write-traffic")
        print(json.dumps(write_traffic(sys.argv[i + 1], sys.argv[i + 2], " ".join(sys.argv[i + 3:])), indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--prec", default=None, choices=[None, "f64", "f32", "bf16", "bf16x3", "bf16x6"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-move", action="store_true",
                    help="config 5: leave out the D = 6, chi = 64 left move reported beside the batched corners")
    ap.add_argument("--cell", action="store_true", help="time the left move of a 2 x 2 unit cell")
    ap.add_argument("--unit", action="store_true",
                    help="time a CTM re-initialisation of a 2 x 2 cell (8 steps per direction, D=3, chi=40)")
    ap.add_argument("--corners", action="store_true",
                    help="time the four enlarged corners, single-layer against double-layer route")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the move runs on one GPU (asked for {args.gpus}); "
              "its multi-GPU sharding is a design, not an implementation.", file=sys.stderr)
        sys.exit(2)
    if args.corners:
        bench_corners(args)
        return
    if args.cell:
        bench_cell(args)
        return
    if args.unit:
        bench_unit(args)
        return
    if args.config == 3:
        bench_su2(args)
        return

    if args.config == 5:
        out = bench_batched(args)
        if not args.no_move:
            mv = bench_move(args, 2, "f32", min(args.steps, 10), min(args.warmup, 2), with_cpu=False)
            out["move_D6_chi64_f32"] = {k: mv[k] for k in ("value", "unit", "ms_per_step", "steps", "config",
                                                          "roofline", "gemm_roofline", "useful_flops_per_move", "gemm_phase_gflops",
                                                          "phase_ms", "kept", "trunc_err", "consecutive_moves")}
        print(json.dumps(out))
        return
    print(json.dumps(bench_move(args, args.config, args.prec, args.steps, args.warmup,
                                with_cpu=not args.no_cpu_baseline)))


EVOLVING_MOVES = 6


def move_config(config_no):
    """The move workload of --cell and --corners: config 5 (the default) is
    the batched-corner workload, which has no single site; it stands for the
    D = 6, chi = 64 move (config 2) there."""
    return 2 if config_no == 5 else config_no


def bench_move(args, config_no, prec, steps, warmup, with_cpu):
    """One full left move of workload `config_no` per step (the environment
    reset to the same C1, C4, T4 before every move, so that every step does
    the same work), then EVOLVING_MOVES consecutive moves without resets."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX

    cfgd = config(config_no)
    prec = prec or {"sweep": "f32"}.get(cfgd["prec"], cfgd["prec"])
    use_recorded_tiles(cfgd["name"])
    dtype = "f64" if prec == "f64" else "f32"
    chi = cfgd["chi_target"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream

    T = build_workload(cfgd, cfgd["seed"], dtype, st, draw, TENSOR_INDEX)
    env = st.CtmEnv([T[k] for k in ("C1", "C2", "C3", "C4")], [T[k] for k in ("T1", "T2", "T3", "T4")])

    def step(stats=False):
        env.set(0, T["C1"])
        env.set(3, T["C4"])
        env.set(7, T["T4"])
        return env.move(T["a"], chi, prec=prec, stats=stats, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps

    # per-kernel durations: the same steps again with HIP events around
    # every launch on the launch stream
    st.profile_begin()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kstats = st.profile_end()

    stats = step(stats=True)

    # A run of consecutive left moves from the same start, without resets:
    # each move works on the environment the previous one left, and a new
    # chi-leg structure is planned on the host (and its GEMM tiles chosen)
    # the first time it appears, as in a real CTM run.
    run_env = st.CtmEnv([T[k] for k in ("C1", "C2", "C3", "C4")], [T[k] for k in ("T1", "T2", "T3", "T4")])
    run_ms, run_kept = [], []
    for _ in range(EVOLVING_MOVES):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = run_env.move(T["a"], chi, prec=prec, stats=True, stream=stream)
        torch.cuda.synchronize()
        run_ms.append((time.perf_counter() - t0) * 1e3)
        run_kept.append(s["kept"])

    flops = stats["flops_corners"] + stats["flops_halves"] + stats["flops_renorm"]
    value = flops / (ms_per_step * 1e-3) / 1e9
    gemm_ms = stats["ms_corners"] + stats["ms_halves"] + stats["ms_renorm"]
    dom = max(kstats, key=lambda k: k["ms"]) if kstats else None
    gemms = [k for k in kstats if k["name"].startswith("gemm")]
    out = {
        "metric": f"useful GFLOP/s per CTM move ({cfgd['group'].replace('U1', 'U(1)')} left move, sector GEMMs on MFMA)",
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic (seeded Gaussian blocks)",
        "config": {"workload": cfgd["name"], "what": cfgd["what"], "D_virtual": cfgd["virt"],
                   "chi": chi, "chi_sectors": cfgd["chi"], "parallelism": "single GPU"},
        "roofline": roofline_of(dom, steps, None, cfgd["name"]) if dom else None,
        "gemm_roofline": roofline_of(max(gemms, key=lambda k: k["ms"]), steps, None, cfgd["name"]) if gemms else None,
        "useful_flops_per_move": flops,
        "gemm_phase_gflops": flops / (gemm_ms * 1e-3) / 1e9 if gemm_ms > 0 else None,
        "phase_ms": {k: stats[k] for k in ("ms_corners", "ms_halves", "ms_proj", "ms_renorm", "ms_total")},
        "kept": stats["kept"], "trunc_err": stats["trunc_err"],
        "kernels": sorted(kstats, key=lambda k: -k["ms"])[:6],
        "consecutive_moves": {"what": "left moves from the same start without resets (new chi legs "
                                      "planned when first seen)", "ms": run_ms, "kept": run_kept},
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(cfgd, flops)
    return out


if __name__ == "__main__":
    main()
