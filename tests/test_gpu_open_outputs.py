"""Open outputs: j output variables left open give 2^j amplitudes per
contraction (the paper's Discussion, a large slice of amplitudes from one
evaluation), on every engine, against the FP64 state vector."""
import numpy as np
import pytest

import oracle
import paper_1805_01450_amd as q
from workload import generate_circuit, random_bitstrings

pytestmark = pytest.mark.gpu
DET = q.QGM_PLAN_DETERMINISTIC
ENGINES = [q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED, q.QGM_ENGINE_WIDE]


def note(*args):
    print("[gpu-open]", *args, flush=True)


@pytest.fixture(scope="module")
def case():
    text = generate_circuit(5, 20, 0)
    psi = oracle.sv_state(text)
    bits = random_bitstrings(25, 16, 1000)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.5, flags=DET)
    return text, psi, bits, c, sl, order


def expected(psi, bits, open_q):
    """amplitude e of bitstring b: x = b with x[open_q[i]] = bit i of e."""
    out = []
    for x in bits:
        for e in range(1 << len(open_q)):
            y = np.array(x, dtype=np.int64)
            for i, qb in enumerate(open_q):
                y[qb] = (e >> i) & 1
            out.append(psi[int(np.sum(y << np.arange(len(y))))])
    return np.array(out)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec,tol", [(q.QGM_C128, 1e-12), (q.QGM_C64, 2e-4)])
@pytest.mark.parametrize("open_q", [[3, 7, 12], [24, 0], [5]])
def test_open_outputs_vs_state_vector(case, engine, prec, tol, open_q):
    text, psi, bits, c, sl, order = case
    p = q.Plan(c, sl, order, prec=prec, engine=engine, open_qubits=open_q)
    st = p.stats()
    assert st["engine"] == engine and st["n_open"] == len(open_q)
    got = p.amplitudes(bits)
    want = expected(psi, bits, open_q)
    assert got.shape == want.shape == (16 << len(open_q),)
    e = np.abs(got - want) / np.maximum(np.abs(want), 2.0 ** -12.5)
    note("engine", engine, "prec", prec, "open", open_q, "max err", e.max())
    assert e.max() <= tol


def test_open_outputs_ranges_device_entry_and_persistent(case):
    """Slice ranges combine to the whole sum; the all-device entry and the
    persistent generated kernel give the host entry's partials bit for bit."""
    import torch
    text, psi, bits, c, sl, order = case
    open_q = [2, 9, 17, 21]
    p = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, open_qubits=open_q)
    pp = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, open_qubits=open_q, persistent=True)
    full = p.amplitudes_range(bits, None, 0, 64)
    assert full.shape == (16 << 4, 4)
    a = p.amplitudes_range(bits, None, 0, 29)
    b = p.amplitudes_range(bits, None, 29, 64)
    tot = (a[:, 0] + b[:, 0]) + (a[:, 2] + b[:, 2]) + 1j * ((a[:, 1] + b[:, 1]) + (a[:, 3] + b[:, 3]))
    want = expected(psi, bits, open_q)
    assert np.max(np.abs(tot - want) / np.maximum(np.abs(want), 2.0 ** -12.5)) <= 2e-4
    d_bits = torch.from_numpy(bits).cuda()
    d_part = torch.empty((16 << 4, 4), dtype=torch.float64, device="cuda")
    q.qgm_amplitudes_device(p.h, d_bits, None, 0, 64, p.workspace(16), d_part)
    assert np.array_equal(d_part.cpu().numpy(), full)
    assert np.array_equal(pp.amplitudes_range(bits, None, 0, 64), full)


def test_open_outputs_errors(case):
    text, psi, bits, c, sl, order = case
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, sl, order, open_qubits=[3, 3])
    assert e.value.status == -1
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, sl, order, open_qubits=[25])
    assert e.value.status == -1
    with pytest.raises(q.QgmError) as e:
        q.Plan(c, sl, order, open_qubits=[1], gradient=True)
    assert e.value.status == -7
