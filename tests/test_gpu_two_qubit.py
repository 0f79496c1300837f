"""Circuits with two-qubit gates that are not diagonal (CX, ISWAP, SQISW:
the K4 gadget of Fig. "tensornodes", four-variable factors) on every engine
and precision, against the FP64 state vector."""
import numpy as np
import pytest

import oracle
import paper_1805_01450_amd as q
from tests.test_host import _two_qubit_circuit

pytestmark = pytest.mark.gpu
ENGINES = [q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED, q.QGM_ENGINE_WIDE]


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec,tol", [(q.QGM_C128, 1e-12), (q.QGM_C64, 2e-4)])
@pytest.mark.parametrize("k", [0, 3])
def test_two_qubit_gates_all_outputs(seed, engine, prec, tol, k):
    text = _two_qubit_circuit(seed)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=k, time_budget_s=0.1, flags=q.QGM_PLAN_DETERMINISTIC)
    p = q.Plan(c, sl, order, prec=prec, engine=engine)
    xs = np.array([[(i >> j) & 1 for j in range(9)] for i in range(512)], np.uint8)
    got = p.amplitudes(xs)
    psi = oracle.sv_state(text)
    err = np.abs(got - psi) / np.maximum(np.abs(psi), 2.0 ** -4.5)
    print("[gpu-2q] seed", seed, "engine", engine, "prec", prec, "k", k, "max err", err.max(), flush=True)
    assert err.max() <= tol
