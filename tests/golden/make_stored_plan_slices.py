"""Write tests/golden/stored_plan_slices.json: FP64 oracle values of single
slices of the stored benchmark plans, for the GPU parity tests.

Only the oracle computes here.  The inputs are the seeded circuit generator
(``workload``) and the stored plans (``paper_1805_01450_amd/plans/*.json``,
read as plain data: sliced variables and elimination order, inputs of the
method like any caller's order).

* 8x8x40 (Rules 1-3, seed 0), the bitstring of seed 1000, every stored plan
  k = 8 ... 13: alpha_{x,s} for a few slices s.  A slice whose elimination
  would hold a tensor of more than 2^27 entries is itself split by fixing j
  more variables (the oracle's own greedy choice) and its 2^j pieces are
  summed exactly (``math.fsum``): fixing a variable changes only how the sum
  is split (Section "Parallelization by fixing the values of variables").
* 7x7x30 with every T replaced by RZ(theta), theta of seed 2000, bitstring
  of seed 1000, stored plan 7x7x30 (k = 6; RZ and T are both diagonal, so
  the graph and the plan are the same): two slices and, for slice 0, the
  slice identity d alpha_s / d theta_j of a seeded subset of 16 angles.

    python tests/golden/make_stored_plan_slices.py [--only NAME ...]
    python tests/golden/make_stored_plan_slices.py --whole 8x8x40-k8 --workers 6 --state FILE

Values are stored as JSON floats (repr, exact round trip).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle.elimination import _graph_of, greedy_extra_slices, order_cost  # noqa: E402
from oracle.gradient import ve_slice_gradients  # noqa: E402
from oracle.network import build_network, project  # noqa: E402
from workload import generate_circuit, parse_header, random_bitstrings, random_thetas  # noqa: E402

OUT = os.path.join(HERE, "stored_plan_slices.json")
PLANS = os.path.join(ROOT, "paper_1805_01450_amd", "plans")
MAX_WIDTH = 27  # largest tensor rank the oracle builds here (2^27 complex128 = 2 GiB)

# stored plan -> slices checked
SLICES = {
    "8x8x40": [0, 1, 4095, 8191],
    "8x8x40-k12": [0, 4095],
    "8x8x40-k11": [0, 2047],
    "8x8x40-k10": [0, 777],
    "8x8x40-k9": [0, 511],
    "8x8x40-k8": [0, 255],
}


def load_plan(name):
    with open(os.path.join(PLANS, name + ".json")) as f:
        rec = json.load(f)
    return rec


def slice_value(text, x, net, sliced, order, s, params=None):
    """alpha_{x,s}; split into 2^j exactly summed pieces when the plan's
    width exceeds MAX_WIDTH."""
    base, _ = project(net, x)
    g = _graph_of(base, net.free_vars)
    for v in sliced:
        g.fix(v)
    verts = sorted(g.vertices)
    _, width = order_cost(verts, g.edges, order)
    extra, rest, j = [], list(order), 0
    while width > MAX_WIDTH:
        j += 1
        extra, rest, _, width = greedy_extra_slices(verts, g.edges, order, j)
    k = len(sliced)
    pieces = [int(s) | (t << k) for t in range(1 << j)]
    vals = oracle.ve_slice_values(text, x, sliced=list(sliced) + extra, order=rest, params=params,
                                  slices=pieces, net=net)
    v = complex(math.fsum(vals.real), math.fsum(vals.imag))
    return v, {"extra_fixed": extra, "pieces": len(pieces), "width": width}


def grid_entry(name, log):
    rec = load_plan(name)
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, c["seed"] + 1000)[0]
    net = build_network(text)
    out = {"circuit": c, "bitstring_seed": c["seed"] + 1000, "k": rec["k"], "slices": {}}
    for s in SLICES[name]:
        t0 = time.time()
        v, how = slice_value(text, x, net, rec["sliced"], rec["order"], s)
        out["slices"][str(s)] = [v.real, v.imag]
        log(f"{name} slice {s}: {v!r} ({how}, {time.time() - t0:.1f} s)")
    return out


def config4_entry(log):
    rec = load_plan("7x7x30")
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"], rz=True)
    _, npar = parse_header(text)
    th = random_thetas(npar, c["seed"] + 2000)
    x = random_bitstrings(c["n"] ** 2, 1, c["seed"] + 1000)[0]
    net = build_network(text, th)
    out = {"circuit": dict(c, rz=True), "bitstring_seed": c["seed"] + 1000, "theta_seed": c["seed"] + 2000,
           "k": rec["k"], "slices": {}}
    for s in (0, 37):
        t0 = time.time()
        v, how = slice_value(text, x, net, rec["sliced"], rec["order"], s, params=th)
        out["slices"][str(s)] = [v.real, v.imag]
        log(f"7x7x30-rz slice {s}: {v!r} ({how}, {time.time() - t0:.1f} s)")
    # 16 angles: seeded, plus the first angle whose variable is fixed (an
    # output or a sliced variable) and a pair of angles on one variable
    rng = np.random.default_rng(0)
    which = set(int(j) for j in rng.choice(npar, 13, replace=False))
    fixed = [j for j in range(npar) if net.param_var[j] in set(rec["sliced"])
             or (net.param_var[j] >= 0 and net.variables[net.param_var[j]].is_output)]
    if fixed:
        which.add(fixed[0])
    by_var = {}
    for j in range(npar):
        by_var.setdefault(net.param_var[j], []).append(j)
    pair = next((v for v in by_var.values() if len(v) >= 2), [])
    which.update(pair[:2])
    which = sorted(which)
    while len(which) < 16:
        extra = int(rng.integers(npar))
        if extra not in which:
            which = sorted(which + [extra])
    t0 = time.time()
    g = ve_slice_gradients(text, x, th, rec["sliced"], rec["order"], 0, which=which, net=net)
    out["grad_slice"] = 0
    out["grad_which"] = which
    out["grad"] = [[v.real, v.imag] for v in g]
    log(f"7x7x30-rz d alpha_0 / d theta for {which} ({time.time() - t0:.1f} s)")
    # the whole amplitude and its gradient for the same angles: every slice,
    # summed exactly
    t0 = time.time()
    n_s = 1 << rec["k"]
    vals = oracle.ve_slice_values(text, x, sliced=rec["sliced"], order=rec["order"], params=th, net=net)
    out["alpha"] = [math.fsum(vals.real), math.fsum(vals.imag)]
    gs = np.array([ve_slice_gradients(text, x, th, rec["sliced"], rec["order"], s, which=which, net=net)
                   for s in range(n_s)])
    out["grad_full"] = [[math.fsum(gs[:, i].real), math.fsum(gs[:, i].imag)] for i in range(len(which))]
    log(f"7x7x30-rz alpha {complex(*out['alpha'])!r} and its gradient ({time.time() - t0:.1f} s)")
    return out


def _whole_slice(job):
    name, s, max_width = job
    global MAX_WIDTH
    MAX_WIDTH = max_width
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    rec = load_plan(name)
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, c["seed"] + 1000)[0]
    v, _ = slice_value(text, x, build_network(text), rec["sliced"], rec["order"], s)
    return s, [v.real, v.imag]


def whole_entry(name, log, workers, state_path, max_width=26):
    """The whole amplitude of a stored plan: every slice (each split so no
    tensor exceeds 2^max_width entries), summed exactly.  Slice values are
    kept in state_path as they finish, so an interrupted run resumes."""
    import multiprocessing as mp
    rec = load_plan(name)
    done = {}
    if state_path and os.path.exists(state_path):
        with open(state_path) as f:
            done = {int(k): v for k, v in json.load(f).items()}
    todo = [s for s in range(1 << rec["k"]) if s not in done]
    t0 = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        for s, v in pool.imap_unordered(_whole_slice, [(name, s, max_width) for s in todo]):
            done[s] = v
            if state_path:
                with open(state_path, "w") as f:
                    json.dump(done, f)
            log(f"{name} whole: slice {s} done, {len(done)} of {1 << rec['k']} ({time.time() - t0:.0f} s)")
    vals = [done[s] for s in range(1 << rec["k"])]
    alpha = [math.fsum(v[0] for v in vals), math.fsum(v[1] for v in vals)]
    c = rec["circuit"]
    return {"circuit": c, "bitstring_seed": c["seed"] + 1000, "k": rec["k"], "alpha": alpha,
            "slices": {str(s): done[s] for s in (0, (1 << rec["k"]) - 1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None, help="entries to (re)compute; others are kept")
    ap.add_argument("--whole", default=None, help="stored plan whose whole amplitude is computed (all slices)")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--state", default=None, help="file keeping finished slices of --whole (resumable)")
    args = ap.parse_args()
    if args.whole:
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as f:
                data = json.load(f)
        data[args.whole + "-whole"] = whole_entry(args.whole, lambda m: print(m, flush=True), args.workers,
                                                  args.state)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)
        return
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["about"] = ("FP64 oracle slice values of the stored plans (tests/golden/make_stored_plan_slices.py); "
                     "slice s fixes sliced[j] to bit j of s")
    names = list(SLICES) + ["7x7x30-rz"]
    todo = names if args.only is None else args.only

    def log(msg):
        print(msg, flush=True)

    for name in todo:
        data[name] = config4_entry(log) if name == "7x7x30-rz" else grid_entry(name, log)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
