"""Tune the matrix-core tiles of the benchmark plans on the device
(qgm_plan_tune_tiles) and write the table the benchmark uses.

    python paper_1805_01450_amd/plans/make_tiles.py [--out PATH] [--no-confirm] [name ...]

Needs a GPU.  The table holds one line per (precision, row bits, column
bits, summed bits) shape; shapes already in an existing table at PATH are
kept unless tuned again.  The tuner times each shape alone, which does not
see the operand strides and cache state of the plan's own levels; so each
entry is then settled inside the plan: the plan's level kernels are timed
with the tuned entry, without it (the library's built-in tile for the
shape), with the per-item form at its default tile (complex64: four
items per block; BF16x3: eight) and, for a complex64 per-item entry, with
the same tile in the three-multiplication form (layout + 32), and the
fastest is kept unless it beats the tuned entry by less than 0.5 %.
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
    ap.add_argument("--no-confirm", action="store_true", help="skip the in-plan confirmation")
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
            if not args.no_confirm:
                confirm(q, circ, rec, prec, args.out)
    with open(args.out) as f:
        body = [ln for ln in f if not ln.startswith("# written by")]
    with open(args.out, "w") as f:
        f.write(f"# written by: python paper_1805_01450_amd/plans/make_tiles.py {' '.join(args.names)} "
                f"(qgm_plan_tune_tiles on one MI355X{'' if args.no_confirm else ', entries settled in the plan'})\n")
        f.writelines(body)
    print(open(args.out).read(), flush=True)


def plan_ms(q, torch, circ, rec, prec, table, d_bits, d_part, n_s, runs=3):
    """Sum of the plan's level-kernel times (HIP events, mean of `runs`
    runs after one untimed run) for n_s slices with the given tile table."""
    p = q.Plan(circ, rec["sliced"], rec["order"], prec=prec, profile=True, engine=q.QGM_ENGINE_WIDE,
               tile_table_path=table)
    ws = p.workspace(d_bits.shape[0], n_s)
    for w in range(runs + 1):
        q.qgm_amplitudes_device(p.h, d_bits, None, 0, n_s, ws, d_part)
        if w == 0:
            torch.cuda.synchronize()
            q.qgm_plan_level_timing(p.h, reset=True)
    torch.cuda.synchronize()
    ms = sum(q.qgm_plan_level_timing(p.h, reset=False)[0])
    p.release_workspace()
    del p
    return ms


def confirm(q, circ, rec, prec, table, margin=0.005):
    """Settle each entry of precision `prec` inside the plan: the tuned
    entry, no entry (the built-in tile) or the per-item form's default tile,
    whichever runs the plan fastest (by more than `margin` against the tuned
    entry)."""
    import torch
    from workload import random_bitstrings
    c = rec["circuit"]
    d_bits = torch.from_numpy(random_bitstrings(c["n"] * c["n"], 1, c["seed"] + 1000)).cuda()
    d_part = torch.empty((1, 4), dtype=torch.float64, device="cuda")
    n_s = min(1 << rec["k"], 128)
    tmp = table + ".candidate"
    per_item = "2 65536 0 16" if prec == q.QGM_C64 else "2 131072 0 8"
    with open(table) as f:
        lines = f.readlines()
    entries = [ln for ln in lines if ln.strip() and not ln.startswith("#") and int(ln.split()[0]) == prec]
    for ln in entries:
        with open(table) as f:
            cur = f.readlines()
        base = plan_ms(q, torch, circ, rec, prec, table, d_bits, d_part, n_s)
        shape = " ".join(ln.split()[:4])
        per, budget, band, layout = (int(v) for v in ln.split()[4:8])
        alt = {"built-in": [x for x in cur if x != ln],
               "per-item": [x if x != ln else f"{shape} {per_item}\n" for x in cur]}
        if " ".join(ln.split()[4:]) == per_item:
            del alt["per-item"]
        if prec == q.QGM_C64 and layout & 16 and not layout & 32:
            # the same per-item tile with three FP32 products per complex product
            alt["per-item, 3 products"] = [x if x != ln else f"{shape} {per} {budget} {band} {layout | 32}\n"
                                           for x in cur]
        best, best_ms = None, base * (1.0 - margin)
        times = []
        for name, body in alt.items():
            with open(tmp, "w") as f:
                f.writelines(body)
            t = plan_ms(q, torch, circ, rec, prec, tmp, d_bits, d_part, n_s)
            times.append(f"{t:.2f} ms {name}")
            if t < best_ms:
                best, best_ms = name, t
        print(f"  confirm {ln.strip()}: {base:.2f} ms tuned, " + ", ".join(times) +
              f" -> {best or 'tuned'}", flush=True)
        if best:
            with open(table, "w") as f:
                f.writelines(alt[best])
        if best == "per-item" and prec == q.QGM_C64:
            # the chosen per-item tile in the three-product form as well
            line3 = f"{shape} {per_item[:-2]}{int(per_item.split()[-1]) | 32}\n"
            body = [x if x.split()[:4] != ln.split()[:4] else line3 for x in alt[best]]
            with open(tmp, "w") as f:
                f.writelines(body)
            t3 = plan_ms(q, torch, circ, rec, prec, tmp, d_bits, d_part, n_s)
            keep = t3 < best_ms * (1.0 - margin)
            print(f"    three products: {t3:.2f} ms -> {'taken' if keep else 'not taken'}", flush=True)
            if keep:
                with open(table, "w") as f:
                    f.writelines(body)
    if os.path.exists(tmp):
        os.remove(tmp)


if __name__ == "__main__":
    main()
