"""Throughput of the sliced single-amplitude contraction on one MI355X.

Default workload: the whole amplitude <x|C|0^64> of a seeded 8x8 grid,
depth-40 Rules 1-3 circuit for one uniformly random bitstring, with the
stored k = 8 plan (8 sliced variables, 256 slices).  One step = one call of
the all-device entry point over all 256 slices: constant steps, the per-slice
contraction chain (level kernels, matrix cores for the large two-operand
contractions) and the FP64 compensated slice sum.  Inputs are resident in
device memory before timing starts.

The headline is complex64 (FP32 arithmetic, FP64 slice sum); BF16x3 and
complex128 legs of the same workload ride along with their own rates, their
matrix-core fraction of peak, and the error of each against the FP64 oracle's
values of single slices (stored by tests/golden/make_stored_plan_slices.py)
and against the complex128 whole amplitude.  A 5x5x20 batch (64 bitstrings x
2^6 slices) is reported as extra keys.

Prints one JSON line.
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

METRIC = "slice contractions/sec + % MFMA peak (c64 vs BF16x3) at stated amplitude rel. error"
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X published vector FP32 peak (packed dual issue)
PEAK_FP32_VECTOR_NONPACKED_TFLOPS = 78.6  # the same without packed FP32, which the kernels here are compiled without
PEAK_FP32_MATRIX_TFLOPS = 157.3  # MI355X published dense FP32 matrix-core peak
PEAK_BF16_MATRIX_TFLOPS = 2500.0  # MI355X published dense BF16 matrix-core peak
PEAK_FP64_MATRIX_TFLOPS = 78.6  # MI355X published dense FP64 matrix-core peak
PEAK_FP64_VECTOR_TFLOPS = 78.6  # MI355X published vector FP64 peak
PEAK_HBM_GBS = 8000.0  # MI355X published HBM3E bandwidth
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")  # rocprofv3 HBM byte counters, summarised
GOLDEN_SLICES = os.path.join(ROOT, "tests", "golden", "stored_plan_slices.json")
# matrix-core tile table written by paper_1805_01450_amd/plans/make_tiles.py
# (qgm_plan_tune_tiles on this GPU model)
TILE_TABLE = os.path.join(ROOT, "paper_1805_01450_amd", "plans", "tiles_mi355x.txt")

# name: (grid n, depth, circuit seed, bitstrings, k, slices timed per bitstring (None = all 2^k),
#        stored plan name or None (planned here), default steps, default warm-up runs)
WORKLOADS = {
    "8x8x40-k8-full": (8, 40, 0, 1, 8, None, "8x8x40-k8", 20, 5),
    "8x8x40-k9-full": (8, 40, 0, 1, 9, None, "8x8x40-k9", 20, 5),
    "8x8x40-k10-full": (8, 40, 0, 1, 10, None, "8x8x40-k10", 20, 5),
    "8x8x40-k11-full": (8, 40, 0, 1, 11, None, "8x8x40-k11", 20, 5),
    "8x8x40-k12-full": (8, 40, 0, 1, 12, None, "8x8x40-k12", 20, 5),
    "8x8x40-full": (8, 40, 0, 1, 13, None, "8x8x40", 10, 3),
    "8x8x40": (8, 40, 0, 1, 13, 64, "8x8x40", 50, 10),
    "7x7x30": (7, 30, 0, 1, 6, None, "7x7x30", 50, 10),
    "6x6x25": (6, 25, 0, 1024, 10, None, None, 50, 10),
    "5x5x20": (5, 20, 0, 64, 6, None, None, 200, 50),
    "4x4x10": (4, 10, 0, 1, 0, None, None, 200, 50),
}
DEFAULT_WORKLOAD = "8x8x40-k8-full"
# Planner objective of the workloads planned here (qgm_plan_slices_ex flags,
# always with QGM_PLAN_DETERMINISTIC so every host gets the same plan): 4096
# items are too few to fill the GPU, so the 5x5x20 batch is planned for the
# latency of one item on four wavefronts; 6x6x25 keeps the sum of 2^deg(v).
PLAN_FLAGS = {"5x5x20": 4}
PLAN_BUDGET = 1.0


def host_cpu() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def _oracle_pieces(job):
    """Worker: FP64 oracle values of sub-slices `pieces` (one process, one
    BLAS thread).  Returns (values, CPU seconds)."""
    text, x, sliced, order, pieces = job
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    import oracle
    from oracle.network import build_network
    t0 = time.process_time()
    vals = oracle.ve_slice_values(text, x, sliced=sliced, order=order, slices=pieces, net=build_network(text))
    return [complex(v) for v in vals], time.process_time() - t0


def cpu_baseline(text, x, sliced, order, max_width=24, max_workers=16):
    """The FP64 oracle (variable elimination, one einsum per variable) on a
    bounded sample of the same workload.  Slice s = 0 of the plan is split
    into 2^j pieces by fixing j more variables (the oracle's own greedy
    choice, so that no tensor exceeds 2^max_width entries); one piece runs on
    each of the host's cores (at most max_workers processes, one BLAS thread
    each), and the rate is extrapolated to whole slices: 1 slice per 2^j
    pieces.  Runs before the GPU is touched; workers are spawned processes."""
    import multiprocessing as mp

    from oracle.elimination import _graph_of, greedy_extra_slices, order_cost
    from oracle.network import build_network, project

    net = build_network(text)
    base, _ = project(net, x)
    g = _graph_of(base, net.free_vars)
    for v in sliced:
        g.fix(v)
    verts = sorted(g.vertices)
    _, width = order_cost(verts, g.edges, order)
    extra, rest, j = [], list(order), 0
    while width > max_width:
        j += 1
        extra, rest, _, width = greedy_extra_slices(verts, g.edges, order, j)
    k = len(sliced)
    workers = max(1, min(max_workers, os.cpu_count() or 1, 1 << j))
    jobs = [(text, x, list(sliced) + extra, rest, [t << k]) for t in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(_oracle_pieces, jobs)
    wall = time.perf_counter() - t0
    cpu_s = sum(o[1] for o in out)
    return {"value": workers / (wall * (1 << j)), "unit": "slice contractions/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{workers} of the 2^{j} pieces of slice 0 of the same plan (k={k}, split by {j} more "
                      f"fixed variables, max tensor rank {width}), one per process x 1 thread; {wall:.1f} s wall, "
                      f"{cpu_s:.1f} s CPU; rate extrapolated to whole slices (2^{j} pieces each); numpy einsum "
                      f"per eliminated variable, FP64",
            "single_core_value": workers / (cpu_s * (1 << j)), "host": host_cpu()}


def stored_plan(name):
    """Sliced variables and order stored by paper_1805_01450_amd/plans/make_plans.py."""
    path = os.path.join(ROOT, "paper_1805_01450_amd", "plans", name + ".json")
    with open(path) as f:
        rec = json.load(f)
    return rec, f"stored plan {name}.json (search budget {rec['budget_s']} s)"


def source_digest() -> str:
    """sha256 over what the timed kernels are built and generated from: the
    library sources, the stored plans and the circuit generator."""
    import hashlib
    pkg = os.path.join(ROOT, "paper_1805_01450_amd")
    paths = []
    for d in (os.path.join(pkg, "csrc"), os.path.join(pkg, "plans"), os.path.join(ROOT, "workload")):
        paths += [os.path.join(d, name) for name in sorted(os.listdir(d))]
    h = hashlib.sha256()
    for path in paths:
        if os.path.isfile(path) and not path.endswith(".pyc"):
            h.update(os.path.relpath(path, ROOT).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str, waves: int, prec: str = "c64"):
    """HBM bytes per launch of `kernel`, from rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs of this workload, each scaled by what the counter reads
    for a plain copy of known size.  The counters cannot be read from inside
    the process, so they are stored with a digest of the sources they were
    taken on; None once the sources have changed or when no run matches."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    for e in rec["entries"]:
        if (e["workload"] == workload and e["kernel"] == kernel and e["waves"] == waves
                and e.get("prec", "c64") == prec):
            return e["bytes_per_launch"]
    return None


def timed(q, torch, plan, d_bits, d_part, n_s, steps, warmup, stream):
    """W direct warm-up runs (HIP events around each kernel of the second and
    later ones give the per-kernel durations), then the timed region: one
    replay of a HIP graph holding exactly `steps` captured runs, bracketed by
    synchronisation on both sides and by HIP events on the launch stream."""
    ws = plan.workspace(d_bits.shape[0], n_s)
    q.qgm_plan_timing(plan.h, reset=True)
    wide = plan.stats()["engine"] == q.QGM_ENGINE_WIDE
    for w in range(warmup):
        q.qgm_amplitudes_device(plan.h, d_bits, None, 0, n_s, ws, d_part, stream)
        if w == 0 and warmup > 1 and wide:
            # the first run touches the fresh workspace first: its kernels
            # are left out of the per-kernel durations
            torch.cuda.synchronize()
            q.qgm_plan_level_timing(plan.h, reset=True)
    torch.cuda.synchronize()
    levels = None
    if wide:
        levels = q.qgm_plan_level_timing(plan.h, reset=False)  # per level kernel: ms, flops/slice, mfma steps
    (ms_pro, ms_chain, ms_red), n_runs = q.qgm_plan_timing(plan.h, reset=True)
    g = q.qgm_graph_create(plan.h, d_bits, None, 0, n_s, ws, d_part, repeat=steps)
    q.qgm_graph_launch(g, stream)  # first replay outside the timed region
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    q.qgm_graph_launch(g, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    q.qgm_graph_free(g)
    part = d_part.cpu().numpy()
    amps = part[:, 0] + part[:, 2] + 1j * (part[:, 1] + part[:, 3])
    return dict(wall=wall, gpu_ms_step=gpu_ms / steps, ms_chain=ms_chain, ms_pro=ms_pro, ms_red=ms_red, amps=amps,
                n_runs=n_runs, levels=levels)


def level_roofline(levels, workload, prec_name):
    """Roofline of the dominant level kernel (longest HIP-event duration) and
    of the eight longest: the ceiling each is closest to (matrix cores,
    vector ALUs or HBM) and that fraction."""
    # the first pass of items is timed; flops and bytes count a step shared
    # between the pass's groups once per pass
    ms_l, fl_l, mf_l, _, items_l, by_l, _ = levels
    i = max(range(len(ms_l)), key=lambda j: ms_l[j])
    k_flops = fl_l[i] * items_l
    k_tf = k_flops / (ms_l[i] * 1e-3) / 1e12
    k_gbs = by_l[i] * items_l / (ms_l[i] * 1e-3) / 1e9
    # matrix-core peak in useful (complex) flops: FP64, FP32, or for BF16x3
    # the bfloat16 peak over the three bfloat16 products per real product
    mpeak = {"c128": PEAK_FP64_MATRIX_TFLOPS, "bf16x3": PEAK_BF16_MATRIX_TFLOPS / 3}.get(prec_name,
                                                                                       PEAK_FP32_MATRIX_TFLOPS)
    vpeak = PEAK_FP64_VECTOR_TFLOPS if prec_name == "c128" else PEAK_FP32_VECTOR_TFLOPS
    peak = mpeak if mf_l[i] else vpeak
    traffic = measured_traffic(workload, f"wl{i}", 1, prec_name)
    # the ceiling the kernel is closest to: its arithmetic (matrix cores or
    # vector ALUs) or HBM
    if k_gbs / PEAK_HBM_GBS > k_tf / peak:
        roof = {"bound": "hbm", "achieved": k_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": k_gbs / PEAK_HBM_GBS,
                "achieved_tflops": k_tf, "frac_of_arith_peak": k_tf / peak}
    else:
        roof = {"bound": "mfma" if mf_l[i] else "alu", "achieved": k_tf, "peak": peak, "unit": "TFLOP/s",
                "frac": k_tf / peak}
    roof.update({"traffic": traffic, "kernel": f"wl{i} (generated level kernel, {prec_name})",
                 "kernel_ms": ms_l[i], "flops_per_launch": k_flops, "algorithmic_bytes_per_launch": by_l[i] * items_l,
                 "matrix_core_steps": mf_l[i], "slices_per_launch": items_l})
    per_level = []
    for j in sorted(range(len(ms_l)), key=lambda x: -ms_l[x])[:8]:
        tf = fl_l[j] * items_l / (ms_l[j] * 1e-3) / 1e12
        gb = by_l[j] * items_l / (ms_l[j] * 1e-3) / 1e9
        pk = mpeak if mf_l[j] else vpeak
        fr_f, fr_b = tf / pk, gb / PEAK_HBM_GBS
        per_level.append({"kernel": f"wl{j}", "ms": ms_l[j], "tflops": tf, "hbm_gbs": gb,
                          "bound": ("mfma" if mf_l[j] else "alu") if fr_f >= fr_b else "hbm",
                          "frac": max(fr_f, fr_b)})
    roof["levels"] = per_level
    mk = [j for j in range(len(ms_l)) if mf_l[j]]
    if mk:
        roof["matrix_core_kernels_ms"] = sum(ms_l[j] for j in mk)
        roof["matrix_core_kernels_tflops"] = (sum(fl_l[j] for j in mk) * items_l
                                              / (sum(ms_l[j] for j in mk) * 1e-3) / 1e12)
    return roof


def golden_slices(plan_name):
    """{slice: oracle value} of this plan, or {} (tests/golden/stored_plan_slices.json,
    written by a script that calls only the oracle)."""
    try:
        with open(GOLDEN_SLICES) as f:
            rec = json.load(f).get(plan_name)
    except OSError:
        return {}
    if not rec:
        return {}
    return {int(s): complex(v[0], v[1]) for s, v in rec["slices"].items()}


def slice_errors(plan, x, ref):
    """max over the stored slices of |alpha_s - oracle| / |oracle|."""
    worst = 0.0
    for s, want in ref.items():
        part = plan.amplitudes_range([x], None, s, s + 1)[0]
        got = part[0] + part[2] + 1j * (part[1] + part[3])
        worst = max(worst, abs(got - want) / abs(want))
    return worst


def extra_5x5x20(q, torch, stream):
    """The 5x5x20 batch (64 bitstrings x 2^6 slices, generated register
    kernel, c64): rate and the chain kernel against the vector FP32 peaks."""
    from workload import generate_circuit, random_bitstrings
    n, depth, seed, n_bs, k, _, _, steps, warmup = WORKLOADS["5x5x20"]
    text = generate_circuit(n, depth, seed)
    bits = random_bitstrings(n * n, n_bs, seed + 1000)
    circ = q.Circuit(text)
    sliced, order = circ.plan_slices(k_req=k, time_budget_s=PLAN_BUDGET, seed=seed,
                                     flags=PLAN_FLAGS["5x5x20"] | q.QGM_PLAN_DETERMINISTIC)
    plan = q.Plan(circ, sliced, order, prec=q.QGM_C64, profile=True)
    waves = plan.autotune(n_bs, 1 << k)
    d_bits = torch.from_numpy(bits).cuda()
    d_part = torch.empty((n_bs, 4), dtype=torch.float64, device="cuda")
    r = timed(q, torch, plan, d_bits, d_part, 1 << k, steps, warmup, stream)
    st = plan.stats()
    n_items = n_bs << k
    k_ms = min(r["ms_chain"], r["gpu_ms_step"])
    tf = st["flops_item"] * n_items / (k_ms * 1e-3) / 1e12
    # the same batch with 4 output variables left open: 16 amplitudes per
    # (bitstring, slice) contraction
    open_q = [0, 6, 12, 18]
    po = q.Plan(circ, sliced, order, prec=q.QGM_C64, profile=True, open_qubits=open_q)
    po.autotune(n_bs, 1 << k)
    d_part_o = torch.empty((n_bs << len(open_q), 4), dtype=torch.float64, device="cuda")
    ro = timed(q, torch, po, d_bits, d_part_o, 1 << k, steps, warmup, stream)
    amps_closed = n_bs / (r["wall"] / steps)
    amps_open = (n_bs << len(open_q)) / (ro["wall"] / steps)
    return {"workload": f"5x5 grid depth 20 seed 0, 64 random bitstrings x 2^6 slices = {n_items} slice "
                        f"contractions per step (deterministic latency plan)",
            "amplitudes_per_s": amps_closed,
            "open_outputs": {"open_qubits": open_q, "amplitudes_per_step": n_bs << len(open_q),
                             "amplitudes_per_s": amps_open, "ms_per_step": 1e3 * ro["wall"] / steps,
                             "engine": {1: "interpreter", 2: "generated", 3: "wide"}[po.stats()["engine"]],
                             "speedup_per_amplitude": amps_open / amps_closed},
            "value": n_items / (r["wall"] / steps), "unit": "slice contractions/s", "steps": steps,
            "ms_per_step": 1e3 * r["wall"] / steps, "engine": "generated", "waves_per_block": waves,
            "kernel": "qgm_chain (generated)", "kernel_ms": k_ms, "achieved_tflops_algorithmic": tf,
            "frac_vector_fp32_peak": tf / PEAK_FP32_VECTOR_TFLOPS,
            "frac_vector_fp32_nonpacked": tf / PEAK_FP32_VECTOR_NONPACKED_TFLOPS,
            "traffic": measured_traffic("5x5x20", "qgm_chain", waves)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed runs (default: per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="warm-up runs (default: per workload)")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--engine", default="auto", choices=["auto", "interpreter", "generated"])
    ap.add_argument("--vector-only", action="store_true",
                    help="wide engine: keep every step on the vector ALUs (no matrix cores)")
    ap.add_argument("--workspace-gib", type=float, default=128.0,
                    help="wide engine: item memory per pass in GiB (0 = the library default, 96 GiB; 128 holds "
                         "all 256 slices of the 8x8x40 k=8 plan in complex64 and BF16x3 in one pass)")
    ap.add_argument("--precisions", default="c64,bf16x3,c128",
                    help="comma-separated legs; the first is the headline")
    ap.add_argument("--tiles", default=None,
                    help="matrix-core tile table (default: the stored tuned table when present; 'none' = built-in)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 5x5x20 extra keys")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; the slice axis would shard across GPUs "
                                   "by contiguous slice ranges (qgm_amplitudes_range)"}))
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        torch.cuda.set_device(0)
        n = 1 << 28
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_dispatch": 4 * n, "copy_bytes_written_per_dispatch": 4 * n,
                          "dispatches": 5}), flush=True)
        return

    import numpy as np

    from workload import generate_circuit, random_bitstrings

    n, depth, seed, n_bs, k, n_run, plan_name, d_steps, d_warm = WORKLOADS[args.workload]
    steps = d_steps if args.steps is None else args.steps
    warmup = d_warm if args.warmup is None else args.warmup
    text = generate_circuit(n, depth, seed)
    bits = random_bitstrings(n * n, n_bs, seed + 1000)
    n_s = (1 << k) if n_run is None else n_run
    n_items = n_bs * n_s

    import paper_1805_01450_amd as q
    circ = q.Circuit(text)
    t_plan = time.perf_counter()
    if plan_name is not None:
        rec, plan_source = stored_plan(plan_name)
        sliced, order = rec["sliced"], rec["order"]
        assert rec["circuit"] == {"n": n, "depth": depth, "seed": seed} and rec["k"] == k
    else:
        flags = PLAN_FLAGS.get(args.workload, 0) | q.QGM_PLAN_DETERMINISTIC
        sliced, order = circ.plan_slices(k_req=k, time_budget_s=PLAN_BUDGET, seed=seed, flags=flags)
        plan_source = f"planned here (flags {flags}, deterministic budget {PLAN_BUDGET})"
    t_plan = time.perf_counter() - t_plan
    print(f"[bench] {args.workload}: {plan_source} (k={len(sliced)})", file=sys.stderr, flush=True)

    # The oracle's baseline runs first, on the host cores, before the GPU is used.
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        if n_bs == 1:
            cpu = cpu_baseline(text, bits[0], sliced, order)
        else:
            cpu = cpu_baseline_items(text, bits, sliced)
        print(f"[bench] cpu baseline: {cpu['value']:.4g} slices/s on {cpu['cores']} cores "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)

    import torch
    torch.cuda.set_device(0)
    d_bits = torch.from_numpy(bits).cuda()
    d_part = torch.empty((n_bs, 4), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    eng = {"auto": q.QGM_ENGINE_AUTO, "interpreter": q.QGM_ENGINE_INTERPRETER,
           "generated": q.QGM_ENGINE_GENERATED}[args.engine]
    precs = {"c64": q.QGM_C64, "bf16x3": q.QGM_BF16X3, "c128": q.QGM_C128}
    legs = [p for p in args.precisions.split(",") if p]
    tiles = args.tiles if args.tiles is not None else (TILE_TABLE if os.path.exists(TILE_TABLE) else "none")
    tile_path = None if tiles == "none" else tiles
    ref_slices = golden_slices(plan_name) if (plan_name and n_bs == 1) else {}
    results = {}
    for name in legs:
        plan = q.Plan(circ, sliced, order, prec=precs[name], profile=True, engine=eng,
                      vector_only=args.vector_only, workspace_cap=int(args.workspace_gib * (1 << 30)),
                      tile_table_path=tile_path)
        st = plan.stats()
        waves = plan.autotune(n_bs, n_s) if st["engine"] == q.QGM_ENGINE_GENERATED else 1
        r = timed(q, torch, plan, d_bits, d_part, n_s, steps, warmup, stream)
        r["stats"] = plan.stats()
        r["waves"] = waves
        r["slice_err"] = slice_errors(plan, bits[0], ref_slices) if ref_slices else None
        plan.release_workspace()  # the next precision's plan may need the memory
        del plan
        torch.cuda.empty_cache()
        results[name] = r
        print(f"[bench] {args.workload} {name}: {r['gpu_ms_step']:.4f} ms per step, compile "
              f"{r['stats']['compile_s']:.1f} s", file=sys.stderr, flush=True)

    head = legs[0]
    r = results[head]
    st = r["stats"]
    wide = st["engine"] == q.QGM_ENGINE_WIDE
    ms_step = 1e3 * r["wall"] / steps
    value = n_items / (r["wall"] / steps)
    flops_launch = st["flops_item"] * n_items
    if wide and r["levels"] and r["levels"][0]:
        roofline = level_roofline(r["levels"], args.workload, head)
    else:
        # The chain kernel is the run's only long kernel.  HIP events around a
        # direct launch add a few microseconds of their own, so the kernel
        # time is the smaller of that and the graph replay time per run.
        k_ms = min(r["ms_chain"], r["gpu_ms_step"])
        k_tf = flops_launch / (k_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": k_tf, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                    "frac": k_tf / PEAK_FP32_VECTOR_TFLOPS,
                    "frac_nonpacked": k_tf / PEAK_FP32_VECTOR_NONPACKED_TFLOPS,
                    "traffic": measured_traffic(args.workload, "qgm_chain", r["waves"])
                    if st["engine"] == q.QGM_ENGINE_GENERATED else None,
                    "kernel": {1: "chain_kernel", 2: "qgm_chain (generated)"}.get(st["engine"], "?"),
                    "kernel_ms": k_ms, "flops_per_launch": flops_launch}
    # work per slice as run: steps shared between the groups of a pass
    # count once per pass (the timed first pass; the whole run is one pass
    # when the workspace holds it)
    lv = r["levels"] if wide and r["levels"] and r["levels"][0] else None
    flops_run = sum(lv[1]) if lv else st["flops_item"]
    bytes_run = sum(lv[5]) if lv else st["bytes_item"]
    roof_run = lv[6] if lv else st["roof_s_item"]
    roofline["chain_ms"] = r["ms_chain"]
    roofline["chain_tflops"] = flops_run * n_items / (r["ms_chain"] * 1e-3) / 1e12
    roofline["chain_hbm_gbs"] = bytes_run * n_items / (r["ms_chain"] * 1e-3) / 1e9

    a128 = complex(results["c128"]["amps"][0]) if "c128" in results else None

    def rel_vs_c128(amps):
        if a128 is None:
            return None
        return abs(complex(amps[0]) - a128) / max(abs(a128), 2.0 ** (-n * n / 2))

    dtype = {"c64": "c64 (fp32 complex arithmetic, fp64 slice sum)",
             "bf16x3": "bf16x3 (three bf16 products per real product, fp32 accumulation, fp64 slice sum)",
             "c128": "c128 (fp64 complex arithmetic)"}[head]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "slice contractions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": (f"{n}x{n} grid depth {depth} Rules 1-3 circuit seed {seed}, {n_bs} random "
                                f"bitstring{'s' if n_bs > 1 else ''}, k={k} sliced variables, "
                                + (f"the whole amplitude: all {n_s} slices per step" if n_run is None else
                                   f"{n_s} of the {1 << k} slices per step")),
                   "plan": plan_source, "plan_s": round(t_plan, 2), "sliced_vars": sliced,
                   "matrix_core_tiles": os.path.relpath(tile_path, ROOT) if tile_path else "built-in",
                   "compile_s": round(st["compile_s"], 1), "max_rank": st["max_rank"],
                   "flops_per_slice": st["flops_item"], "bytes_per_slice": st["bytes_item"],
                   "flops_per_slice_run": flops_run, "bytes_per_slice_run": bytes_run,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "engine": {1: "interpreter", 2: "generated", 3: "wide"}[st["engine"]],
        "timing": "timed region = one HIP graph replay of `steps` captured runs (events on the launch stream); "
                  "kernel_ms = HIP events around each kernel over the warm-up runs",
        "gpu_ms_per_step": r["gpu_ms_step"],
        "mfma_flops_share": st["flops_mfma"] / st["flops_item"],
        "mfma_steps": st["mfma_steps"],
        "launches_per_pass": st["launches"],
        "roofline_time_frac": roof_run * n_items / (ms_step * 1e-3) if wide else None,
    }
    if n_run is None and n_bs == 1:
        line["amplitude"] = [complex(r["amps"][0]).real, complex(r["amps"][0]).imag]
        line["seconds_per_amplitude"] = ms_step * 1e-3
    if n_run is not None:
        per_slice_ms = r["gpu_ms_step"] / n_items
        line["per_slice_ms"] = per_slice_ms
        line["projected_full_sum_s"] = per_slice_ms * 1e-3 * (1 << k) * n_bs
    # every leg: rate, matrix-core fraction of its own peak, errors
    for name, rr in results.items():
        leg = {"value": n_items / (rr["wall"] / steps), "ms_per_step": 1e3 * rr["wall"] / steps,
               "compile_s": round(rr["stats"]["compile_s"], 1),
               "slice_rel_error_vs_oracle": rr["slice_err"],
               "amplitude_rel_error_vs_c128": rel_vs_c128(rr["amps"]) if name != "c128" else 0.0}
        if rr["levels"] and rr["levels"][0]:
            lr = level_roofline(rr["levels"], args.workload, name)
            leg["dominant_kernel"] = {x: lr[x] for x in ("kernel", "kernel_ms", "achieved", "frac", "bound")}
            if "matrix_core_kernels_tflops" in lr:
                tf = lr["matrix_core_kernels_tflops"]
                leg["matrix_core_kernels_tflops"] = tf
                if name == "c64":
                    line["c64_mfma_frac_fp32_peak"] = tf / PEAK_FP32_MATRIX_TFLOPS
                elif name == "bf16x3":
                    # three bfloat16 products per real product
                    line["bf16x3_mfma_frac_bf16_peak"] = 3 * tf / PEAK_BF16_MATRIX_TFLOPS
                else:
                    line["c128_mfma_frac_fp64_peak"] = tf / PEAK_FP64_MATRIX_TFLOPS
        line[name] = leg
    if ref_slices:
        line["oracle_slices_checked"] = sorted(ref_slices)
    if not args.no_extra and args.workload != "5x5x20":
        line["extra_5x5x20"] = extra_5x5x20(q, torch, stream)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def _oracle_items(job):
    text, rows, sliced = job
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    import oracle
    from oracle.network import build_network
    net = build_network(text)
    t0 = time.process_time()
    for x in rows:
        oracle.ve_slice_values(text, x, sliced=sliced, net=net)
    return time.process_time() - t0


def cpu_baseline_items(text, bits, sliced, max_workers=16, per_worker=1):
    """Batches of bitstrings: the oracle on `per_worker` whole bitstrings (all
    2^k slices each) per process, on up to max_workers host cores."""
    import multiprocessing as mp
    workers = max(1, min(max_workers, os.cpu_count() or 1, len(bits)))
    jobs = [(text, bits[w * per_worker:(w + 1) * per_worker], list(sliced)) for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        cpu_s = sum(pool.map(_oracle_items, jobs))
    wall = time.perf_counter() - t0
    done = workers * per_worker << len(sliced)
    return {"value": done / wall, "unit": "slice contractions/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers * per_worker} bitstrings x 2^{len(sliced)} slices of the same workload, "
                      f"{workers} processes x 1 thread; {wall:.1f} s wall, {cpu_s:.1f} s CPU",
            "single_core_value": done / cpu_s, "host": host_cpu()}


if __name__ == "__main__":
    main()
