"""Precompute the elimination plans (sliced variables and ordering) of the
large benchmark circuits with a long planner search, so that runs do not
spend minutes planning.  The planner is the library's own
(qgm_plan_slices_ex with QGM_PLAN_SEARCH | QGM_PLAN_WIDE_TIME); a stored
plan is an input like any caller-supplied order, validated by
qgm_plan_create.

    python -m paper_1805_01450_amd.plans.make_plans [--budget SECONDS] [--out DIR] [name ...]
    python -m paper_1805_01450_amd.plans.make_plans --regroup name ...

The planner returns its sliced variables in the order for group sharing
(qgm_sliced_order_for_groups).  --regroup rewrites the sliced order of
existing plan files that way, without a new search: the set of sliced
variables, the elimination order and the amplitude stay the same; slice
indices other than all-zeros and all-ones then denote other assignments.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
# name: (grid n, depth, circuit seed, sliced variables k)
CIRCUITS = {"7x7x30": (7, 30, 0, 6), "8x8x40": (8, 40, 0, 13), "8x8x40-k12": (8, 40, 0, 12),
            "8x8x40-k14": (8, 40, 0, 14), "8x8x40-k11": (8, 40, 0, 11), "8x8x40-k10": (8, 40, 0, 10),
            "8x8x40-k9": (8, 40, 0, 9), "8x8x40-k8": (8, 40, 0, 8)}


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    import paper_1805_01450_amd as q
    from workload import generate_circuit
    ap = argparse.ArgumentParser()
    ap.add_argument("--budget", type=float, default=600.0)
    ap.add_argument("--out", default=HERE, help="directory for the plan files")
    ap.add_argument("--regroup", action="store_true", help="reorder the sliced variables of existing plan files")
    ap.add_argument("names", nargs="*", default=["7x7x30", "8x8x40"])
    args = ap.parse_args()
    if args.regroup:
        for name in args.names:
            path = os.path.join(args.out, f"{name}.json")
            with open(path) as f:
                rec = json.load(f)
            c = rec["circuit"]
            circ = q.Circuit(generate_circuit(c["n"], c["depth"], c["seed"]))
            sliced, frac = q.qgm_sliced_order_for_groups(circ.h, rec["sliced"], rec["order"])
            assert sorted(sliced) == sorted(rec["sliced"])
            rec["sliced"] = sliced
            rec["sliced_order"] = "groups"
            with open(path, "w") as f:
                json.dump(rec, f)
            print(name, "sliced", sliced, "work independent of slice bits 6 and 7: %.3f" % frac, flush=True)
        return
    flags = q.QGM_PLAN_SEARCH | q.QGM_PLAN_WIDE_TIME
    for name in args.names:
        n, d, seed, k = CIRCUITS[name]
        circ = q.Circuit(generate_circuit(n, d, seed))
        t0 = time.time()
        sliced, order = circ.plan_slices(k_req=k, time_budget_s=args.budget, seed=seed, flags=flags)
        st = q.Plan(circ, sliced, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE).stats()
        rec = {"circuit": {"n": n, "depth": d, "seed": seed}, "k": k, "flags": flags, "budget_s": args.budget,
               "plan_s": round(time.time() - t0, 1), "sliced": sliced, "sliced_order": "groups", "order": order,
               "flops_item": st["flops_item"], "bytes_item": st["bytes_item"], "max_rank": st["max_rank"]}
        with open(os.path.join(args.out, f"{name}.json"), "w") as f:
            json.dump(rec, f)
        print(name, {x: rec[x] for x in ("plan_s", "flops_item", "bytes_item", "max_rank")}, flush=True)


if __name__ == "__main__":
    main()
