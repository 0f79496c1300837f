"""Constants contracted once per plan: for plans without RZ angles the
sub-networks that depend on neither the bitstring nor the slice (the
constant steps) run at upload into plan-owned memory, and every run reads
them; the results equal the per-run contraction's bit for bit."""
import json
import os

import numpy as np
import pytest

import paper_1805_01450_amd as q
from workload import generate_circuit, random_bitstrings

pytestmark = pytest.mark.gpu


def _plans(monkeypatch, text, sl, order, **kw):
    c = q.Circuit(text)
    cached = q.Plan(c, sl, order, **kw)
    monkeypatch.setenv("QGM_NO_CONST_CACHE", "1")
    fresh = q.Plan(c, sl, order, **kw)
    return cached, fresh


@pytest.mark.parametrize("engine,prec", [(q.QGM_ENGINE_WIDE, q.QGM_C64), (q.QGM_ENGINE_WIDE, q.QGM_C128),
                                         (q.QGM_ENGINE_INTERPRETER, q.QGM_C64)])
def test_cached_constants_match_per_run_constants(monkeypatch, engine, prec):
    rec = json.load(open(os.path.join(os.path.dirname(q.__file__), "plans", "7x7x30.json")))
    cz = rec["circuit"]
    text = generate_circuit(cz["n"], cz["depth"], cz["seed"])
    if engine == q.QGM_ENGINE_INTERPRETER:
        text = generate_circuit(5, 20, 0)
        c = q.Circuit(text)
        sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=q.QGM_PLAN_DETERMINISTIC)
        bits = random_bitstrings(25, 8, 5)
    else:
        sl, order = rec["sliced"], rec["order"]
        bits = random_bitstrings(49, 2, 5)
    cached, fresh = _plans(monkeypatch, text, sl, order, prec=prec, engine=engine)
    for rep in range(2):  # the cache is read again by later calls
        a = cached.amplitudes_range(bits, None, 0, 1 << len(sl))
        b = fresh.amplitudes_range(bits, None, 0, 1 << len(sl))
        assert np.array_equal(a, b)
