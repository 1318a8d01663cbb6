#!/usr/bin/env python3
"""Throughput of one U(1)-symmetric CTM left move on one MI355X.

A step is one whole move on resident synthetic tensors: the four enlarged
corners C.T.T.a, the halves, the FP64 QR/SVD projectors with truncation to
chi, the renormalised C1', T4', C4' and their FP64 normalisation.  Default
workload: D = 6 (virtual charges {-2:1, 0:4, +2:1}), chi = 64 (charges
{-4:4,-2:16,0:24,2:16,4:4}), sector GEMMs in FP32.

Prints one JSON line.  `value` = useful GEMM flops of the move (sum over
matched block pairs of 2 m n k in the corners, halves and renormalisation)
divided by the wall time of the whole move.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6, "bf16x3": 2516.6 / 3}
HBM_PEAK_GBS = 8000.0


def build_workload(cfgd, seed, dtype, st, draw, TENSOR_INDEX):
    """Device tensors of the workload filled with the seeded draws."""
    phys, virt, chi, flux = cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"]
    T = {"A": st.Tensor.create([(phys, 1), (virt, 1), (virt, 1), (virt, -1), (virt, -1)], flux, dtype)}
    T["A"].upload(draw((seed, TENSOR_INDEX["A"]), T["A"].nnz))
    T["a"] = st.double_layer(T["A"])
    dd = T["a"].legs()[0][0]
    legs = {"C1": [(chi, 1), (chi, -1)], "T1": [(chi, 1), (dd, -1), (chi, -1)],
            "T2": [(chi, 1), (dd, 1), (chi, -1)], "T3": [(chi, 1), (dd, 1), (chi, -1)],
            "T4": [(chi, 1), (dd, -1), (chi, -1)]}
    for c in ("C2", "C3", "C4"):
        legs[c] = legs["C1"]
    for n, l in legs.items():
        T[n] = st.Tensor.create(l, 0, dtype)
        T[n].upload(draw((seed, TENSOR_INDEX[n]), T[n].nnz))
    return T


def traffic_for(kernel_name):
    """HBM bytes per launch of `kernel_name` from the committed counter
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1808_10804_amd", "csrc", "kernels.hip"), "rb").read()
    if rec.get("kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(cfgd):
    """The FP64 dense oracle timed on the host on one full move of the same
    workload (the oracle as it stands, BLAS threads = host cores)."""
    from oracle import u1
    from synth import draw, TENSOR_INDEX
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    w = u1.Workload(cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"])
    vals = {n: draw((cfgd["seed"], TENSOR_INDEX[n]), w.nnz_of(n)) for n in TENSOR_INDEX}
    t0 = time.perf_counter()
    T = w.dense_tensors(vals)
    a, _ = u1.double_layer(T["A"], w.A_legs)
    mv = u1.ctm_left_move(w, T, a, cfgd["chi_target"])
    dt = time.perf_counter() - t0
    fl = u1.move_gemm_flops(w, mv["proj"]["kept"])["total"]
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one full left move of the same workload (dense FP64, {dt:.1f} s)",
            "seconds": dt}


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


def bench_batched(args):
    """64 independent corner contractions: one grouped launch per step in
    bf16x3 (HIP graph) against per-contraction FP32 launches."""
    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, batched_draws, TENSOR_INDEX

    c5 = config(5)
    draws = batched_draws(c5["seed"], c5["batch"], c5["D_choices"], c5["chi_range"])
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    ins = [build_corner_inputs(dict(phys=c5["phys"], flux=c5["flux"], virt=d["virt"], chi=d["chi"]),
                               (c5["seed"], b), "f32", st, draw, TENSOR_INDEX) for b, d in enumerate(draws)]
    Cs, T1s, T4s, As = ([x[k] for x in ins] for k in ("C1", "T1", "T4", "a"))

    def run_batched():
        return st.enlarged_corners_batched(Cs, T1s, T4s, As, prec=args.prec or "bf16x3", use_graph=True,
                                           stream=stream)

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
    ms_s, fl_s = timed(run_single, max(1, args.steps // 2))
    flops = info["useful_flops"]
    st.profile_begin()
    for _ in range(args.steps):
        run_batched()
    torch.cuda.synchronize()
    kst = st.profile_end()
    out = {
        "metric": "useful GFLOP/s of 64 batched enlarged corners (bf16x3, one grouped launch per step, HIP graph)",
        "value": flops / (ms_b * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec or "bf16x3", "data": "synthetic (seeded Gaussian blocks)",
        "config": {"workload": c5["name"], "batch": c5["batch"], "D": [d["D"] for d in draws],
                   "chi": [d["chi_total"] for d in draws]},
        "useful_flops": flops, "per_contraction_f32": {"ms": ms_s, "gflops": fl_s / (ms_s * 1e-3) / 1e9},
        "speedup_vs_per_contraction_f32": ms_s / ms_b,
        "kernels": sorted(kst, key=lambda k: -k["ms"])[:6],
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 4, 5])
    ap.add_argument("--prec", default=None, choices=[None, "f64", "f32", "bf16", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); "
              "the move's multi-GPU sharding is described, not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.config == 5:
        bench_batched(args)
        return

    import torch
    import paper_1808_10804_amd as st
    from synth import config, draw, TENSOR_INDEX

    cfgd = config(args.config)
    prec = args.prec or {"sweep": "f32"}.get(cfgd["prec"], cfgd["prec"])
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # per-kernel durations: the same steps again with HIP events around
    # every launch on the launch stream
    st.profile_begin()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kstats = st.profile_end()

    stats = step(stats=True)
    flops = stats["flops_corners"] + stats["flops_halves"] + stats["flops_renorm"]
    value = flops / (ms_per_step * 1e-3) / 1e9
    gemm_ms = stats["ms_corners"] + stats["ms_halves"] + stats["ms_renorm"]

    dom = max(kstats, key=lambda k: k["ms"]) if kstats else None
    roof = None
    if dom:
        avg_ms = dom["ms"] / dom["launches"]
        is_gemm = dom["name"].startswith("gemm")
        if is_gemm:
            kprec = "f64" if "f64" in dom["name"] else ("bf16x3" if "bf16x3" in dom["name"]
                                                       else ("bf16" if "bf16" in dom["name"] else "f32"))
            achieved = dom["useful_flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
            peak = PEAK_TFLOPS[kprec]
            roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak}
        else:
            achieved = dom["bytes"] / dom["launches"] / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS}
        tb = traffic_for(dom["name"])
        roof["traffic"] = tb
        roof["kernel"] = dom["name"]
        roof["launches_per_step"] = dom["launches"] / args.steps
        roof["avg_launch_ms"] = avg_ms
        roof["algorithmic_bytes_per_launch"] = dom["bytes"] / dom["launches"]
        roof["useful_flops_per_launch"] = dom["useful_flops"] / dom["launches"]

    out = {
        "metric": "useful GFLOP/s per CTM move (U(1) left move, sector GEMMs on MFMA)",
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic (seeded Gaussian blocks)",
        "config": {"workload": cfgd["name"], "what": cfgd["what"], "D_virtual": cfgd["virt"],
                   "chi": chi, "chi_sectors": cfgd["chi"], "parallelism": "single GPU"},
        "roofline": roof,
        "useful_flops_per_move": flops,
        "gemm_phase_gflops": flops / (gemm_ms * 1e-3) / 1e9 if gemm_ms > 0 else None,
        "phase_ms": {k: stats[k] for k in ("ms_corners", "ms_halves", "ms_proj", "ms_renorm", "ms_total")},
        "kept": stats["kept"], "trunc_err": stats["trunc_err"],
        "kernels": sorted(kstats, key=lambda k: -k["ms"])[:6],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfgd)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
