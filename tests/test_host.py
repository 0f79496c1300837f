"""CPU tests of the C-ABI library: loading, exported symbols, parser, graph
model, planner and plan validation.  No device code runs here."""
import math
import re

import numpy as np
import pytest

import oracle
import paper_1805_01450_amd as q
from oracle.elimination import order_cost as oracle_order_cost
from oracle.network import build_network
from tests.conftest import ROOT
from workload import generate_circuit


def test_header_symbols_are_exported():
    import subprocess
    hdr = open(f"{ROOT}/include/qgm.h").read()
    declared = set(re.findall(r"\b(qgm_\w+)\s*\(", hdr))
    assert declared == set(q.DECLARED)
    out = subprocess.run(["nm", "-D", "--defined-only", q.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (qgm_\w+)", out))
    assert declared <= exported


@pytest.mark.parametrize("text,needle", [
    ("0 H 0\n", "qubits"),
    ("qubits 2\n0 X 0\n", "unknown gate"),
    ("qubits 2\n0 H 2\n", "out of range"),
    ("qubits 2\n0 CZ 1 1\n", "single qubit"),
    ("qubits 2\n0 H 0\n0 T 0\n", "two gates"),
    ("qubits 2\n0 RZ 0\n", "fields"),
    ("qubits 65\n", "qubits"),
])
def test_parse_errors(text, needle):
    with pytest.raises(q.QgmError) as e:
        q.qgm_circuit_parse(text)
    assert e.value.status == -2 and needle in str(e.value)


@pytest.mark.parametrize("n,d,seed,rz", [(4, 10, 0, False), (5, 20, 1, True), (6, 25, 2, False)])
def test_variables_and_graph_match_oracle(n, d, seed, rz):
    text = generate_circuit(n, d, seed, rz=rz)
    c = q.Circuit(text)
    net = build_network(text, np.zeros(c.n_params))
    assert c.n_vars == len(net.variables) and c.n_qubits == n * n
    ours = c.vars()
    theirs = [(v.id, v.qubit, v.cycle, int(v.is_output)) for v in net.variables]
    assert ours == theirs
    outs = [v.id for v in net.variables if v.is_output]
    assert set(c.graph()) == net.graph_edges(exclude=outs)


def test_fig2_graph(fig2_text):
    c = q.Circuit(fig2_text)
    # Fig. 3: 10 free vertices and 12 edges; the letters map to ids 0..9
    # in creation order a b c d e f g h i j
    letters = "abcdefghij"
    edges = {"".join(sorted(letters[a] + letters[b])) for a, b in c.graph()}
    assert edges == set("ab ae ah be bg ce df ef fg gj hi ij".split())


def _plan(n, d, seed, k):
    c = q.Circuit(generate_circuit(n, d, seed))
    sl, order = c.plan_slices(k_req=k, time_budget_s=1.0, seed=seed)
    return c, sl, order


def test_planner_output_is_valid_and_cost_matches_oracle():
    c, sl, order = _plan(5, 20, 0, 6)
    free = [v for v, _, _, out in c.vars() if not out]
    assert len(sl) == 6 and len(set(sl)) == 6 and set(sl) <= set(free)
    assert sorted(order) == sorted(set(free) - set(sl))
    cost, width = q.qgm_order_cost(c.h, sl, order)
    # same cost from the oracle's graph operations on the oracle's graph
    text = generate_circuit(5, 20, 0)
    net = build_network(text)
    outs = [v.id for v in net.variables if v.is_output]
    edges = {e for e in net.graph_edges(exclude=outs + sl)}
    rest = [v for v in net.free_vars if v not in sl]
    ocost, owidth = oracle_order_cost(rest, edges, order)
    assert (cost, width) == (ocost, owidth)
    # slicing lowers the cost of the unsliced min-fill ordering
    sl0, order0 = c.plan_slices(k_req=0, time_budget_s=0.0)
    cost0, width0 = q.qgm_order_cost(c.h, sl0, order0)
    assert cost < cost0 and width <= width0


def test_planner_target_rank():
    c = q.Circuit(generate_circuit(6, 25, 0))
    sl, order = c.plan_slices(k_req=-1, target_rank=8, time_budget_s=0.5)
    _, width = q.qgm_order_cost(c.h, sl, order)
    assert width <= 8


def test_plan_validation_errors():
    c, sl, order = _plan(4, 10, 0, 2)
    free = [v for v, _, _, out in c.vars() if not out]
    outv = [v for v, _, _, out in c.vars() if out]
    cases = [
        (sl, order[:-1], -3),                       # order misses a variable
        (sl, order + [order[0]], -3),               # repeated
        (sl, order + [sl[0]], -3),                  # sliced variable in order
        (sl, order + [outv[0]], -3),                # output variable in order
        ([sl[0], sl[0]], order, -4),                # repeated slice
        ([outv[0]], [v for v in free], -4),          # output variable sliced
        (list(range(41)), order, -4),                # k > 40
    ]
    for s_, o_, code in cases:
        with pytest.raises(q.QgmError) as e:
            q.qgm_plan_create(c.h, s_, o_)
        assert e.value.status == code, (s_, o_)
    with pytest.raises(q.QgmError) as e:
        q.qgm_plan_create(c.h, sl, order, prec=9)
    assert e.value.status == -7
    with pytest.raises(q.QgmError) as e:
        q.qgm_plan_create(c.h, sl, order, workspace_cap=64)
    assert e.value.status == -5


def test_plan_stats():
    c, sl, order = _plan(5, 20, 0, 6)
    p = q.Plan(c, sl, order, prec=q.QGM_C64)
    st = p.stats()
    cost, width = q.qgm_order_cost(c.h, sl, order)
    assert st["k"] == 6 and st["cost"] == cost
    assert st["max_rank"] <= width + 1
    assert st["flops_item"] > 0 and st["item_elems"] >= 1


def test_large_rank_plan_runs_on_wide_engine_only(monkeypatch):
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")  # structure only: skip compiling the step kernels
    c = q.Circuit(generate_circuit(7, 30, 0))
    sl, order = c.plan_slices(k_req=4, time_budget_s=1.0, seed=0, flags=q.QGM_PLAN_DETERMINISTIC)
    st = q.Plan(c, sl, order).stats()
    assert st["engine"] == q.QGM_ENGINE_WIDE and st["max_rank"] >= 16
    for eng in (q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED):
        with pytest.raises(q.QgmError) as e:
            q.Plan(c, sl, order, engine=eng)
        assert e.value.status == -7


def test_gradient_plans_split_large_sums(monkeypatch):
    """Reverse steps that sum many variables are split (no step sums > 8)."""
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")
    text = generate_circuit(7, 30, 0, rz=True)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=1.0)
    p = q.Plan(c, sl, order, gradient=True)
    assert p.stats()["engine"] == q.QGM_ENGINE_WIDE
    assert p.stats()["n_steps"] > q.Plan(c, sl, order).stats()["n_steps"]


@pytest.mark.parametrize("k", [13, 20])
def test_8x8x40_plans_compile(k, monkeypatch):
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")
    c = q.Circuit(generate_circuit(8, 40, 0))
    sl, order = c.plan_slices(k_req=k, time_budget_s=2.0)
    for grad in (False,):
        st = q.Plan(c, sl, order, prec=q.QGM_C64, gradient=grad).stats()
        assert st["engine"] == q.QGM_ENGINE_WIDE and st["k"] == k


def test_generated_wide_kernels_compile_for_gfx950():
    """hiprtc builds the per-step wide kernels of a 7x7x30 plan."""
    c, sl, order = _plan(7, 30, 0, 6)
    st = q.Plan(c, sl, order, prec=q.QGM_C64).stats()
    assert st["engine"] == q.QGM_ENGINE_WIDE and st["compile_s"] > 0


def test_planner_reorder_flag_gives_valid_plans():
    c = q.Circuit(generate_circuit(6, 25, 0))
    free = [v for v, _, _, out in c.vars() if not out]
    for flags in (0, q.QGM_PLAN_REORDER, q.QGM_PLAN_BYTES, q.QGM_PLAN_REORDER | q.QGM_PLAN_BYTES):
        sl, order = c.plan_slices(k_req=8, time_budget_s=0.5, flags=flags)
        assert len(sl) == 8 and sorted(order) == sorted(set(free) - set(sl))
        cost, width = q.qgm_order_cost(c.h, sl, order)
        assert width <= 8


def test_multiwave_schedules_exist():
    """List schedules of the 5x5x20 item tree on 2, 4 and 8 wavefronts pass
    the plan-time simulation of their waits and fit in LDS (complex64)."""
    c = q.Circuit(generate_circuit(5, 20, 0))
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=q.QGM_PLAN_LATENCY)
    for w in (1, 2, 4, 8):
        st = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, waves=w).stats()
        assert st["waves"] == w


def test_generated_source_shapes():
    """The generated kernel of a small plan is cut across wavefronts only for
    amplitude programs (gradient programs are not trees)."""
    text = generate_circuit(5, 20, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2)
    amp = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED).stats()
    assert amp["engine"] == q.QGM_ENGINE_GENERATED and amp["waves"] in (1, 2, 4, 8)
    rz = generate_circuit(4, 10, 3, rz=True)
    c2 = q.Circuit(rz)
    sl2, order2 = c2.plan_slices(k_req=2, time_budget_s=0.2)
    g = q.Plan(c2, sl2, order2, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, gradient=True).stats()
    assert g["waves"] == 1


def test_stored_plans_are_valid(monkeypatch):
    """Plans precomputed for the large benchmark circuits name distinct free
    variables and order every remaining one (checked by plan creation)."""
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")  # structure only: no kernel build
    import json
    import os
    import glob
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_01450_amd", "plans")
    paths = sorted(glob.glob(os.path.join(here, "*.json")))
    for path in paths:
        rec = json.load(open(path))
        cz = rec["circuit"]
        c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
        assert len(rec["sliced"]) == rec["k"] == len(set(rec["sliced"]))
        free = [v for v, _, _, out in c.vars() if not out]
        assert sorted(rec["order"]) == sorted(set(free) - set(rec["sliced"]))
        q.qgm_order_cost(c.h, rec["sliced"], rec["order"])  # the library validates the plan
        if os.path.basename(path) in ("7x7x30.json", "8x8x40.json"):  # compiled in full for the main two
            # the recorded rank is the program's when the plan was searched;
            # the program transforms merge steps and never raise it
            st = q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE).stats()
            assert 0 < st["max_rank"] <= rec["max_rank"]


def test_matrix_core_step_selection():
    """The wide engine puts the two-operand contractions of a 7x7x30 plan on
    the matrix cores for complex64 and BF16x3 (the same steps), never for
    complex128 or with vector_only; vector_only takes 0 or 1."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_01450_amd", "plans",
                        "7x7x30.json")
    rec = json.load(open(path))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    sl, order = rec["sliced"], rec["order"]
    s64 = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE).stats()
    sbf = q.Plan(c, sl, order, prec=q.QGM_BF16X3, engine=q.QGM_ENGINE_WIDE).stats()
    svo = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, vector_only=True).stats()
    s128 = q.Plan(c, sl, order, prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE).stats()
    assert s64["mfma_steps"] >= 1 and 0 < s64["flops_mfma"] < s64["flops_item"]
    assert sbf["mfma_steps"] == s64["mfma_steps"] and sbf["flops_mfma"] == s64["flops_mfma"]
    assert svo["mfma_steps"] == 0 and s128["mfma_steps"] == 0
    # the chain roofline time is at least the flops time and the bytes time
    assert s64["roof_s_item"] >= max(s64["flops_item"] / 157.3e12, s64["bytes_item"] / 8e12) * (1 - 1e-12)
    with pytest.raises(q.QgmError):
        opts = q.PlanOpts()
        opts.prec = q.QGM_C64
        opts.engine = q.QGM_ENGINE_WIDE
        opts.vector_only = 2
        h = q.C.c_void_p()
        q.check(q.lib.qgm_plan_create(c.h, q._i32(sl), len(sl), q._i32(order), len(order), q.C.byref(opts),
                                      q.C.byref(h)))


def test_planner_choose_k():
    """QGM_PLAN_CHOOSE_K tries k_req down to k_req - 6 and returns a valid
    plan for one of them (the least predicted whole-amplitude time)."""
    c = q.Circuit(generate_circuit(6, 25, 0))
    free = [v for v, _, _, out in c.vars() if not out]
    flags = q.QGM_PLAN_SEARCH | q.QGM_PLAN_WIDE_TIME | q.QGM_PLAN_CHOOSE_K
    sl, order = c.plan_slices(k_req=8, time_budget_s=3.5, seed=0, flags=flags)
    assert 2 <= len(sl) <= 8 and len(set(sl)) == len(sl)
    assert sorted(order) == sorted(set(free) - set(sl))
    q.qgm_order_cost(c.h, sl, order)  # validated by the library


def test_workspace_cap_applies_to_the_wide_program(monkeypatch):
    """The cap is checked against the program the wide engine runs: at
    8x8x40, k = 8 one 64-slice group needs about 28 GiB after the constant
    regrouping and the step merges (far more before them), so a cap at that
    need, rounded up to a GiB, is accepted and one a GiB below it is
    refused."""
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")  # structure only: no kernel build
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_01450_amd", "plans",
                        "8x8x40-k8.json")
    rec = json.load(open(path))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    st = q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE,
                workspace_cap=48 << 30).stats()
    need = st["item_elems"] * 64 * 8
    assert 16 << 30 < need < 40 << 30
    cap = -(-need // (1 << 30)) << 30
    q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, workspace_cap=cap)
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, workspace_cap=cap - (1 << 30))
    assert e.value.status == -5


def test_bench_traffic_lookup(monkeypatch):
    """bench.py reports stored HBM counter bytes only for the sources they
    were taken on: a changed source digest gives None."""
    import importlib.util
    import os
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    rec = json.load(open(b.TRAFFIC_FILE))
    e = rec["entries"][0]
    monkeypatch.setattr(b, "source_digest", lambda: rec["source_sha256"])
    assert b.measured_traffic(e["workload"], e["kernel"], e["waves"]) == e["bytes_per_launch"]
    assert b.measured_traffic(e["workload"], e["kernel"], 3) is None
    monkeypatch.setattr(b, "source_digest", lambda: "0" * 64)
    assert b.measured_traffic(e["workload"], e["kernel"], e["waves"]) is None


@pytest.mark.parametrize("flags", [0, q.QGM_PLAN_LATENCY, q.QGM_PLAN_SEARCH | q.QGM_PLAN_REORDER])
def test_deterministic_planning_repeats(flags):
    """QGM_PLAN_DETERMINISTIC counts work instead of time: the same arguments
    give the same plan, however long each restart takes (a slow host thread
    is simulated by a concurrent busy loop), and the plan is valid."""
    import threading
    text = generate_circuit(5, 20, 3)
    c = q.Circuit(text)
    f = flags | q.QGM_PLAN_DETERMINISTIC
    a = c.plan_slices(k_req=5, time_budget_s=0.4, seed=7, flags=f)
    stop = []

    def spin():
        x = 0
        while not stop:
            x += 1

    ts = [threading.Thread(target=spin) for _ in range(4)]
    for t in ts:
        t.start()
    try:
        b = c.plan_slices(k_req=5, time_budget_s=0.4, seed=7, flags=f)
    finally:
        stop.append(1)
        for t in ts:
            t.join()
    assert a == b
    sl, order = a
    assert len(sl) == 5
    net = build_network(text)
    assert sorted(order + sl) == sorted(net.free_vars)


def test_persistent_generated_kernels_compile():
    """opts.persistent = 1: the generated kernel's work-queue form compiles
    for every wavefront cut, with and without RZ tables; bad values are
    refused."""
    for rz in (False, True):
        text = generate_circuit(5, 20, 0, rz=rz)
        c = q.Circuit(text)
        sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=q.QGM_PLAN_DETERMINISTIC)
        for w in (1, 4):
            p = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, waves=w, persistent=True,
                       gradient=rz)
            assert p.stats()["engine"] == q.QGM_ENGINE_GENERATED
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, sl, order, persistent=2)
    assert e.value.status == -1


def test_tile_table_round_trip_and_errors(tmp_path, monkeypatch):
    """A plan reads the tile table named by opts.tile_table_path; entries
    change the generated matrix-core steps; a malformed table is refused."""
    import glob
    import json
    import os
    rec = json.load(open(os.path.join(ROOT, "paper_1805_01450_amd", "plans", "7x7x30.json")))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path / "a"))
    os.makedirs(tmp_path / "a")
    q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE)
    default = open(glob.glob(str(tmp_path / "a" / "qgm_wide_*.hip"))[0]).read()
    shapes = set(re.findall(r"\(matrix cores\) b \d+ i (\d+) j (\d+) k (\d+)", default))
    assert shapes
    table = tmp_path / "tiles.txt"
    lines = ["# test table"] + [f"1 {i} {j} {k} 4 81920 1 1" for i, j, k in sorted(shapes)]
    table.write_text("\n".join(lines) + "\n")
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path / "b"))
    os.makedirs(tmp_path / "b")
    p = q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, tile_table_path=str(table))
    tuned = open(glob.glob(str(tmp_path / "b" / "qgm_wide_*.hip"))[0]).read()
    assert tuned != default and p.stats()["mfma_steps"] >= 1
    assert "const int wi = 0, wj = 0, wq = w4;" in tuned  # layout 1: four item groups
    bad = tmp_path / "bad.txt"
    bad.write_text("1 5 5 3 3 81920 1 1\n")  # 3 k per stage is not a power of two
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, tile_table_path=str(bad))
    assert e.value.status == -1 and "line 1" in str(e.value)
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE,
               tile_table_path=str(tmp_path / "missing.txt"))
    assert e.value.status == -1


def test_checkpointed_gradient_plans():
    """checkpoint_every = n: the 7x7x30 RZ gradient plan holds fewer item
    tensors at its peak, recomputes at most one more forward pass, and still
    has one GRAD step per angle; the 8x8x40 RZ gradient plan (whose reverse
    pass once tripped over a moved tensor list) compiles and shrinks too."""
    import json
    import os
    rec = json.load(open(os.path.join(ROOT, "paper_1805_01450_amd", "plans", "7x7x30.json")))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"], rz=True))
    fwd = q.Plan(c, rec["sliced"], rec["order"], engine=q.QGM_ENGINE_WIDE).stats()
    full = q.Plan(c, rec["sliced"], rec["order"], gradient=True, engine=q.QGM_ENGINE_WIDE).stats()
    ck = q.Plan(c, rec["sliced"], rec["order"], gradient=True, checkpoint_every=4, engine=q.QGM_ENGINE_WIDE).stats()
    assert ck["item_elems"] <= 0.6 * full["item_elems"]
    assert full["flops_item"] < ck["flops_item"] <= full["flops_item"] + 2 * fwd["flops_item"]
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, rec["sliced"], rec["order"], checkpoint_every=4)  # not a gradient plan
    assert e.value.status == -1
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, rec["sliced"], rec["order"], gradient=True, checkpoint_every=-1)
    assert e.value.status == -1


def test_8x8x40_gradient_plan_compiles(monkeypatch):
    import json
    import os
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")  # skip generating kernels: the program is what is checked
    rec = json.load(open(os.path.join(ROOT, "paper_1805_01450_amd", "plans", "8x8x40.json")))
    c = q.Circuit(generate_circuit(8, 40, 0, rz=True))
    full = q.Plan(c, rec["sliced"], rec["order"], gradient=True, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE).stats()
    ck = q.Plan(c, rec["sliced"], rec["order"], gradient=True, prec=q.QGM_C64, checkpoint_every=8,
                engine=q.QGM_ENGINE_WIDE).stats()
    assert ck["item_elems"] <= 0.5 * full["item_elems"]


def test_open_output_plans_compile():
    """opts.open_qubits: plans keep those outputs open on every engine, the
    final step has rank j, and 2^j amplitudes cost less than 2^j runs."""
    text = generate_circuit(5, 20, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=q.QGM_PLAN_DETERMINISTIC)
    closed = q.Plan(c, sl, order, engine=q.QGM_ENGINE_INTERPRETER).stats()
    for eng in (q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED, q.QGM_ENGINE_WIDE):
        st = q.Plan(c, sl, order, prec=q.QGM_C64, engine=eng, open_qubits=[3, 7, 12]).stats()
        assert st["n_open"] == 3 and st["engine"] == eng
    op = q.Plan(c, sl, order, engine=q.QGM_ENGINE_INTERPRETER, open_qubits=[3, 7, 12]).stats()
    assert closed["flops_item"] < op["flops_item"] < 8 * closed["flops_item"]


def _small_circuit(seed, n_sx=9):
    """3 qubits: H layer, then CZ and SX / SY gates at random, enough to give
    about n_sx free variables."""
    rng = np.random.default_rng(seed)
    lines = ["qubits 3"] + [f"0 H {qb}" for qb in range(3)]
    cyc = 1
    placed = 0
    while placed < n_sx:
        a, b = rng.choice(3, 2, replace=False)
        lines.append(f"{cyc} CZ {a} {b}")
        cyc += 1
        qb = int(rng.integers(3))
        lines.append(f"{cyc} {'SX' if rng.integers(2) else 'SY'} {qb}")
        cyc += 1
        placed += 1
    return "\n".join(lines)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_order_search_is_exact_on_small_graphs(seed):
    """qgm_order_search with all children tried and a complete search gives
    the best (width, sum 2^deg) over every ordering, found here by brute
    force with the oracle's own cost function."""
    import itertools
    text = _small_circuit(seed)
    c = q.Circuit(text)
    net = build_network(text)
    outs = [v.id for v in net.variables if v.is_output]
    edges = net.graph_edges(exclude=outs)
    free = net.free_vars
    assert 6 <= len(free) <= 9
    best = None
    for perm in itertools.permutations(free):
        cost, width = oracle_order_cost(free, edges, list(perm))
        if best is None or (width, cost) < best:
            best = (width, cost)
    init = list(reversed(free))  # a poor first incumbent
    order, cost, width, complete = q.qgm_order_search(c.h, [], init, 10 ** 7, beam=0)
    assert complete and sorted(order) == sorted(free)
    assert (width, cost) == best
    assert oracle_order_cost(free, edges, order) == (cost, width)


def test_order_search_anytime_and_planner_flag():
    """On a large graph the search is anytime: never worse than its
    incumbent, and the QGM_PLAN_BNB plans are valid and deterministic."""
    text = generate_circuit(6, 25, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=4, time_budget_s=0.2, flags=q.QGM_PLAN_DETERMINISTIC)
    c0, w0 = q.qgm_order_cost(c.h, sl, order)
    o2, c2, w2, complete = q.qgm_order_search(c.h, sl, order, 300, beam=3)
    assert not complete and (w2, c2) <= (w0, c0)
    assert q.qgm_order_cost(c.h, sl, o2) == (c2, w2)
    f = q.QGM_PLAN_BNB | q.QGM_PLAN_DETERMINISTIC
    a = c.plan_slices(k_req=4, time_budget_s=1.0, flags=f)
    b = c.plan_slices(k_req=4, time_budget_s=1.0, flags=f)
    assert a == b
    net = build_network(text)
    assert sorted(a[1] + a[0]) == sorted(net.free_vars)


def _two_qubit_circuit(seed, n=9, cycles=14):
    """H layer, then random CX / ISWAP / SQISW / CZ pairs and one-qubit gates."""
    rng = np.random.default_rng(seed)
    lines = [f"qubits {n}"] + [f"0 H {q}" for q in range(n)]
    for cyc in range(1, cycles + 1):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        lines.append(f"{2 * cyc - 1} {['CX', 'ISWAP', 'SQISW', 'CZ'][int(rng.integers(4))]} {a} {b}")
        q = int(rng.integers(n))
        lines.append(f"{2 * cyc} {['SX', 'SY', 'T'][int(rng.integers(3))]} {q}")
    # a gate on an untouched qubit: its old index is still the input 0
    lines.append(f"{2 * cycles + 1} CX 0 1")
    return "\n".join(lines)


@pytest.mark.parametrize("seed", [0, 1])
def test_two_qubit_gates_variables_and_graph_match_oracle(seed):
    text = _two_qubit_circuit(seed)
    c = q.Circuit(text)
    net = build_network(text)
    assert c.vars() == [(v.id, v.qubit, v.cycle, int(v.is_output)) for v in net.variables]
    outs = [v.id for v in net.variables if v.is_output]
    assert set(c.graph()) == net.graph_edges(exclude=outs)
    sl, order = c.plan_slices(k_req=2, time_budget_s=0.1, flags=q.QGM_PLAN_DETERMINISTIC)
    for eng in (q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED, q.QGM_ENGINE_WIDE):
        assert q.Plan(c, sl, order, engine=eng).stats()["engine"] == eng
    with pytest.raises(q.QgmError) as e:
        q.Circuit("qubits 2\n0 CX 1 1\n")
    assert e.value.status == -2 and "single qubit" in str(e.value)


def test_sliced_order_for_groups(monkeypatch):
    """qgm_sliced_order_for_groups returns the same sliced variables, keeps
    plans with k <= 6 as they are, leaves the stored k = 8 plan (already in
    that order) unchanged with a third of its item work independent of the
    variables at slice bits 6 and 7, and is what the planner returns."""
    monkeypatch.setenv("QGM_WIDE_PREBUILT", "1")
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_01450_amd", "plans")
    rec = json.load(open(os.path.join(here, "8x8x40-k8.json")))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    out, frac = q.qgm_sliced_order_for_groups(c.h, rec["sliced"], rec["order"])
    assert out == rec["sliced"] and 0.3 < frac < 0.4
    rev = rec["sliced"][::-1]
    out2, frac2 = q.qgm_sliced_order_for_groups(c.h, rev, rec["order"])
    assert sorted(out2) == sorted(rev) and abs(frac2 - frac) < 1e-12
    assert set(out2[6:]) == set(out[6:])  # the same two variables go to the group bits
    rec7 = json.load(open(os.path.join(here, "7x7x30.json")))
    c7 = q.Circuit(generate_circuit(7, 30, 0))
    assert q.qgm_sliced_order_for_groups(c7.h, rec7["sliced"], rec7["order"]) == (rec7["sliced"], 0.0)
    c5 = q.Circuit(generate_circuit(5, 20, 0))
    sl, order = c5.plan_slices(k_req=8, time_budget_s=0.3, flags=q.QGM_PLAN_DETERMINISTIC)
    assert q.qgm_sliced_order_for_groups(c5.h, sl, order)[0] == sl
