"""Throughput of the sliced single-amplitude contraction on one MI355X.

Workload: a seeded 5x5 grid, depth-20 Rules 1-3 circuit, 64 uniformly random
output bitstrings, k = 6 variables sliced by the host planner, i.e. 64 x 2^6
= 4096 slice contractions per step.  One step = one call of the all-device
entry point: prologue (tables, constant steps), the per-item contraction
chain over all 4096 (bitstring, slice) items, and the FP64 compensated slice
reduction.  Inputs are resident in device memory before timing starts.

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X published vector FP32 peak
N, DEPTH, SEED, N_BS, K = 5, 20, 0, 64, 6


def cpu_baseline(text, bits, sliced, budget_s=12.0):
    """The FP64 oracle (variable elimination, one einsum per variable) on a
    bounded sample of the same (bitstring, slice) items."""
    import oracle
    from oracle.network import build_network
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)  # the oracle runs on one host core
    net = build_network(text)
    done = 0
    t0 = time.perf_counter()
    n_bs = 0
    for x in bits:
        oracle.ve_slice_values(text, x, sliced=sliced, net=net)
        done += 1 << len(sliced)
        n_bs += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    threads = 1
    return {"value": done / dt, "unit": "slice contractions/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_bs} bitstrings x 2^{len(sliced)} slices of the same workload ({done} slices, "
                      f"{dt:.1f} s), numpy einsum per eliminated variable, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the slice axis would shard across GPUs "
                                   "by contiguous slice ranges (see qgm_amplitudes_range)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1805_01450_amd as q
    from workload import generate_circuit, random_bitstrings

    torch.cuda.set_device(0)
    text = generate_circuit(N, DEPTH, SEED)
    bits = random_bitstrings(N * N, N_BS, SEED + 1000)
    circ = q.Circuit(text)
    sliced, order = circ.plan_slices(k_req=K, time_budget_s=1.0, seed=SEED)
    n_items = N_BS << K
    d_bits = torch.from_numpy(bits).cuda()
    d_part = torch.empty((N_BS, 4), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    results = {}
    for name, prec, engine in (("c64", q.QGM_C64, q.QGM_ENGINE_AUTO), ("c128", q.QGM_C128, q.QGM_ENGINE_AUTO),
                               ("c64_interp", q.QGM_C64, q.QGM_ENGINE_INTERPRETER)):
        plan = q.Plan(circ, sliced, order, prec=prec, profile=True, engine=engine)
        ws = plan.workspace(N_BS)
        for _ in range(args.warmup):
            q.qgm_amplitudes_device(plan.h, d_bits, None, 0, 1 << K, ws, d_part, stream)
        torch.cuda.synchronize()
        q.qgm_plan_timing(plan.h, reset=True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            q.qgm_amplitudes_device(plan.h, d_bits, None, 0, 1 << K, ws, d_part, stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        (ms_pro, ms_chain, ms_red), n_runs = q.qgm_plan_timing(plan.h, reset=True)
        part = d_part.cpu().numpy()
        amps = part[:, 0] + part[:, 2] + 1j * (part[:, 1] + part[:, 3])
        results[name] = dict(plan=plan, wall=wall, ms_chain=ms_chain, ms_pro=ms_pro, ms_red=ms_red, amps=amps,
                             n_runs=n_runs)

    import oracle
    ref = np.array([oracle.ve_amplitude(text, x) for x in bits])
    nerr = lambda a: float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 2.0 ** (-N * N / 2))))

    st = results["c64"]["plan"].stats()
    r = results["c64"]
    ms_step = 1e3 * r["wall"] / args.steps
    value = n_items / (r["wall"] / args.steps)
    flops_launch = st["flops_item"] * n_items
    achieved = flops_launch / (r["ms_chain"] * 1e-3) / 1e12
    line = {
        "metric": "slice contractions/sec",
        "value": value,
        "unit": "slice contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (fp32 complex arithmetic, fp64 slice reduction)",
        "data": "synthetic",
        "config": {"workload": f"{N}x{N} grid depth {DEPTH} Rules 1-3 circuit seed {SEED}, {N_BS} random "
                               f"bitstrings, k={K} planner-sliced variables: {n_items} slice contractions per step",
                   "sliced_vars": sliced, "max_rank": st["max_rank"], "item_elems": st["item_elems"],
                   "flops_per_slice": st["flops_item"], "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "kernel": "qgm_chain (generated)" if st["engine"] == 2 else "chain_kernel<float>",
                     "kernel_ms": r["ms_chain"]},
        "amplitude_error_c64": nerr(r["amps"]),
        "amplitude_error_c128": nerr(results["c128"]["amps"]),
        "c128_value": n_items / (results["c128"]["wall"] / args.steps),
        "engine": {1: "interpreter", 2: "generated"}[st["engine"]],
        "interpreter_c64_value": n_items / (results["c64_interp"]["wall"] / args.steps),
        "interpreter_c64_error": nerr(results["c64_interp"]["amps"]),
        "mfma_frac": 0.0,
        "kernel_ms": {"prologue": r["ms_pro"], "chain": r["ms_chain"], "reduce": r["ms_red"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(text, bits, sliced)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
