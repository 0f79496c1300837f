"""The generated register kernel in its persistent form (opts.persistent = 1:
a resident grid pulling 64-item chunks from a device work queue) against the
one-block-per-chunk form: every item runs the same code, so the slice sums
are bit-identical; and against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import paper_1805_01450_amd as q
from workload import generate_circuit, parse_header, random_bitstrings, random_thetas

pytestmark = pytest.mark.gpu
DET = q.QGM_PLAN_DETERMINISTIC


def note(*args):
    print("[gpu-persistent]", *args, flush=True)


@pytest.fixture(scope="module")
def case5():
    text = generate_circuit(5, 20, 0)
    bits = random_bitstrings(25, 64, 1000)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.5, flags=q.QGM_PLAN_LATENCY | DET)
    ref = np.array([oracle.ve_amplitude(text, x) for x in bits[:8]])
    return c, sl, order, bits, ref


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("prec", [q.QGM_C64, q.QGM_C128, q.QGM_BF16X3])
def test_persistent_equals_one_block_per_chunk(case5, waves, prec):
    c, sl, order, bits, ref = case5
    a = q.Plan(c, sl, order, prec=prec, engine=q.QGM_ENGINE_GENERATED, waves=waves)
    b = q.Plan(c, sl, order, prec=prec, engine=q.QGM_ENGINE_GENERATED, waves=waves, persistent=True)
    assert a.stats()["waves"] == b.stats()["waves"]
    note("5x5x20 waves", waves, "prec", prec)
    for n_bs, s0, s1 in ((64, 0, 64), (63, 0, 64), (5, 3, 61)):  # fused, ragged, unfused
        pa = a.amplitudes_range(bits[:n_bs], None, s0, s1)
        pb = b.amplitudes_range(bits[:n_bs], None, s0, s1)
        assert np.array_equal(pa, pb)
    got = b.amplitudes(bits[:8])
    # the parity tolerances of tests/test_gpu_parity.py
    tol = {q.QGM_C128: 1e-12, q.QGM_C64: 2e-4,
           q.QGM_BF16X3: np.sqrt(b.stats()["n_steps"]) * 3 * 2.0 ** -16}[prec]
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 2.0 ** -12.5)) <= tol


def test_persistent_many_chunks_and_graph_replays():
    """6x6x25, 1024 bitstrings x 2^10 slices = 16384 chunks on a resident
    grid; a captured graph replayed three times (the queue counter is reset
    by a fill kernel each run) gives the direct result every time."""
    import torch
    text = generate_circuit(6, 25, 0)
    bits = random_bitstrings(36, 1024, 1000)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=10, time_budget_s=1.0, flags=DET)
    a = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED)
    b = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED, persistent=True)
    d_bits = torch.from_numpy(bits).cuda()
    pa = torch.empty((1024, 4), dtype=torch.float64, device="cuda")
    pb = torch.full((1024, 4), float("nan"), dtype=torch.float64, device="cuda")
    q.qgm_amplitudes_device(a.h, d_bits, None, 0, 1024, a.workspace(1024), pa)
    ws = b.workspace(1024)
    q.qgm_amplitudes_device(b.h, d_bits, None, 0, 1024, ws, pb)
    torch.cuda.synchronize()
    direct = pa.cpu().numpy()
    assert np.array_equal(pb.cpu().numpy(), direct)
    g = q.qgm_graph_create(b.h, d_bits, None, 0, 1024, ws, pb, repeat=2)
    try:
        for rep in range(3):
            pb.fill_(float("nan"))
            torch.cuda.synchronize()
            q.qgm_graph_launch(g)
            torch.cuda.synchronize()
            note("graph replay", rep)
            assert np.array_equal(pb.cpu().numpy(), direct)
    finally:
        q.qgm_graph_free(g)
    amp = direct[:, 0] + direct[:, 2] + 1j * (direct[:, 1] + direct[:, 3])
    sub = list(range(0, 1024, 256))
    ref = np.array([oracle.ve_amplitude(text, bits[i]) for i in sub])
    assert np.max(np.abs(amp[sub] - ref) / np.maximum(np.abs(ref), 2.0 ** -18)) <= 2e-4


def test_persistent_gradient_plan():
    text = generate_circuit(4, 12, 7, rz=True)
    _, npar = parse_header(text)
    th = random_thetas(npar, 2007)
    bits = random_bitstrings(16, 1, 1007)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=3, time_budget_s=0.2, flags=DET)
    a = q.Plan(c, sl, order, engine=q.QGM_ENGINE_GENERATED, gradient=True)
    b = q.Plan(c, sl, order, engine=q.QGM_ENGINE_GENERATED, gradient=True, persistent=True)
    amp_a, g_a = a.amplitude_grad(bits[0], th)
    amp_b, g_b = b.amplitude_grad(bits[0], th)
    assert amp_a == amp_b and np.array_equal(g_a, g_b)
    shift = oracle.sv_gradient_shift(text, bits[0], th)
    assert np.max(np.abs(g_b - shift)) <= 1e-11 * max(abs(amp_b), 2.0 ** -8)
