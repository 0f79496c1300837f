"""Tune the matrix-core tiles of the benchmark plans on the device
(qgm_plan_tune_tiles) and write the table the benchmark uses.

    python paper_1805_01450_amd/plans/make_tiles.py [--out PATH] [name ...]

Needs a GPU.  The table holds one line per (precision, row bits, column
bits, summed bits) shape; shapes already in an existing table at PATH are
kept unless tuned again.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    import paper_1805_01450_amd as q
    from workload import generate_circuit
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tiles_mi355x.txt"))
    ap.add_argument("names", nargs="*", default=["8x8x40-k8", "8x8x40"])
    args = ap.parse_args()
    for name in args.names:
        with open(os.path.join(HERE, name + ".json")) as f:
            rec = json.load(f)
        c = rec["circuit"]
        circ = q.Circuit(generate_circuit(c["n"], c["depth"], c["seed"]))
        for prec in (q.QGM_C64, q.QGM_BF16X3):
            t0 = time.time()
            p = q.Plan(circ, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE)
            n = q.qgm_plan_tune_tiles(p.h, args.out)
            print(f"{name} prec {prec}: {n} shapes tuned in {time.time() - t0:.1f} s", flush=True)
            del p
    print(open(args.out).read(), flush=True)


if __name__ == "__main__":
    main()
