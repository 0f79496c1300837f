"""Parity of the HIP path (through the C-ABI) against the FP64 CPU oracle.

Error measure: e = |alpha - alpha_ref| / max(|alpha_ref|, 2^{-N/2}); this is
the relative error for amplitudes of typical size (|alpha| ~ 2^{-N/2} for
random circuits) and a scaled absolute error for near-zero ones.
Tolerances: complex128 1e-12; complex64 (FP32 arithmetic, unit roundoff
u = 2^-24) C64_TOL, a bound on accumulated rounding over a few hundred
dependent operations per slice times the slice-sum cancellation factor.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1805_01450_amd as q
from tests.conftest import golden_path
from workload import generate_circuit, parse_header, random_bitstrings, random_thetas

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12
C64_TOL = 2e-4
# Gradients run the reverse steps after the forward ones: twice the chain
# depth in the linear rounding bound behind C64_TOL.
C64_GRAD_TOL = 2 * C64_TOL
DET = q.QGM_PLAN_DETERMINISTIC


def bf16x3_tol(n_steps):
    """BF16x3: every real product x y becomes xh yh + xh yl + xl yh with
    x = xh + xl + dx (bfloat16 halves, round to nearest even), which errs by
    at most 3 * 2^-16 |x y| (tests/test_gpu_contraction.py); over the D =
    n_steps dependent steps of a plan the rounding errors grow like a random
    walk, so the normalised amplitude error stays below sqrt(D) * 3 * 2^-16.
    A plain bfloat16 product (2^-8 per product) or a lost cross term gives
    about 2^8 times that."""
    return math.sqrt(n_steps) * 3 * 2.0 ** -16


def nerr(a, ref, n_qubits):
    a = np.asarray(a)
    ref = np.asarray(ref)
    return np.abs(a - ref) / np.maximum(np.abs(ref), 2.0 ** (-n_qubits / 2))


def note(*args):
    print("[gpu-parity]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


ENGINES = [q.QGM_ENGINE_INTERPRETER, q.QGM_ENGINE_GENERATED, q.QGM_ENGINE_WIDE]


def run(text, bits, k=0, prec=q.QGM_C128, params=None, seed=0, engine=q.QGM_ENGINE_AUTO):
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=k, time_budget_s=0.5, seed=seed, flags=DET)
    p = q.Plan(c, sl, order, prec=prec, engine=engine)
    if engine != q.QGM_ENGINE_AUTO:
        assert p.stats()["engine"] == engine
    return p.amplitudes(bits, params), p


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_config1_4x4x10_c128(seed):
    text = generate_circuit(4, 10, seed)
    x = np.zeros((1, 16), np.uint8)
    note("4x4x10 seed", seed, "x=0^16 k=0 c128")
    got, _ = run(text, x)
    ref = oracle.sv_amplitudes(text, x)
    assert nerr(got, ref, 16).max() <= C128_TOL


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec,tol", [(q.QGM_C128, C128_TOL), (q.QGM_C64, C64_TOL)])
def test_fig2_all_outputs(fig2_text, prec, tol, engine):
    bits = np.array([[(i >> j) & 1 for j in range(4)] for i in range(16)], np.uint8)
    note("fig2 circuit, all 16 x, prec", prec, "engine", engine)
    got, _ = run(fig2_text, bits, prec=prec, engine=engine)
    ref = oracle.sv_amplitudes(fig2_text, bits)
    assert np.abs(got - ref).max() <= tol


@pytest.mark.parametrize("engine", ENGINES)
def test_closed_forms(engine):
    n = 5
    allx = np.array([[(i >> j) & 1 for j in range(n)] for i in range(1 << n)], np.uint8)
    note("closed forms, 5 qubits")
    # empty circuit: delta(x, 0)
    got, _ = run(f"qubits {n}\n", allx, engine=engine)
    want = np.zeros(1 << n)
    want[0] = 1
    assert np.abs(got - want).max() == 0
    # H layer then diagonal gates (CZ, T, RZ): closed-form phases
    rng = np.random.default_rng(3)
    lines = [f"qubits {n}"] + [f"0 H {qq}" for qq in range(n)]
    th = rng.uniform(0, 2 * np.pi, 3)
    lines += ["1 CZ 0 1", "1 T 2", "1 RZ 3 0", "2 CZ 1 4", "2 RZ 0 1", "3 CZ 2 3", "3 RZ 4 2", "4 T 0"]
    text = "\n".join(lines)
    got, _ = run(text, allx, params=th, engine=engine)
    ref = oracle.sv_amplitudes(text, allx, th)
    assert np.abs(got - ref).max() <= 1e-14
    # a qubit that never gets a non-diagonal gate contributes delta(x_q, 0)
    text = "qubits 3\n0 H 0\n0 H 2\n1 T 1\n2 CZ 0 1\n3 SX 2\n"
    allx3 = allx[:8, :3]
    got, _ = run(text, allx3, engine=engine)
    ref = oracle.sv_amplitudes(text, allx3)
    assert np.abs(got - ref).max() <= 1e-15


@pytest.fixture(scope="module")
def config2():
    text = generate_circuit(5, 20, 0)
    bits = random_bitstrings(25, 64, 1000)
    ref = np.array([oracle.ve_amplitude(text, x) for x in bits])
    return text, bits, ref


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("prec,tol", [(q.QGM_C128, C128_TOL), (q.QGM_C64, C64_TOL)])
def test_config2_5x5x20_k6(config2, prec, tol, engine):
    text, bits, ref = config2
    note("5x5x20 seed 0, 64 bitstrings, k=6, prec", prec, "engine", engine)
    got, p = run(text, bits, k=6, prec=prec, engine=engine)
    assert p.k == 6
    e = nerr(got, ref, 25)
    note("max normalised error", e.max())
    assert e.max() <= tol


def test_slicing_and_order_invariance_on_device(config2):
    text, bits, ref = config2
    c = q.Circuit(text)
    outs = []
    for k, seed in [(0, 0), (3, 1), (6, 2), (9, 3), (12, 4)]:
        sl, order = c.plan_slices(k_req=k, time_budget_s=0.2, seed=seed, flags=DET)
        note("invariance k", k)
        outs.append(q.Plan(c, sl, order).amplitudes(bits[:8]))
    # a different (random) elimination order of the same slices
    sl, order = c.plan_slices(k_req=4, time_budget_s=0.0, flags=DET)
    rng = np.random.default_rng(0)
    outs.append(q.Plan(c, sl, list(rng.permutation(order))).amplitudes(bits[:8]))
    for o in outs:
        assert nerr(o, ref[:8], 25).max() <= C128_TOL


def test_range_resume_equals_full(config2):
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=DET)
    p = q.Plan(c, sl, order)
    full = p.amplitudes_range(bits, None, 0, 64)
    a = p.amplitudes_range(bits, None, 0, 23)     # stop after 23 slices
    b = p.amplitudes_range(bits, None, 23, 64)    # resume
    tot_full = full[:, 0] + full[:, 2] + 1j * (full[:, 1] + full[:, 3])
    tot = (a[:, 0] + b[:, 0]) + (a[:, 2] + b[:, 2]) + 1j * ((a[:, 1] + b[:, 1]) + (a[:, 3] + b[:, 3]))
    assert nerr(tot, ref, 25).max() <= C128_TOL
    assert nerr(tot_full, ref, 25).max() <= C128_TOL
    empty = p.amplitudes_range(bits, None, 5, 5)
    assert np.all(empty == 0)


@pytest.mark.parametrize("engine", ENGINES)
def test_engines_agree_bitwise_on_reduction_order(config2, engine):
    """k = 8: 4 chunks of 64 slices per bitstring (fused chunk partials + combine)."""
    text, bits, ref = config2
    note("k=8 chunked slice sums, engine", engine)
    got, p = run(text, bits[:16], k=8, engine=engine)
    assert nerr(got, ref[:16], 25).max() <= C128_TOL


def test_device_entry_matches_host_entry(config2, cuda):
    torch = cuda
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=DET)
    p = q.Plan(c, sl, order, prec=q.QGM_C64)
    host = p.amplitudes(bits)
    d_bits = torch.from_numpy(bits).cuda()
    d_part = torch.empty((64, 4), dtype=torch.float64, device="cuda")
    ws = p.workspace(64)
    q.qgm_amplitudes_device(p.h, d_bits, None, 0, 64, ws, d_part)
    part = d_part.cpu().numpy()
    dev = part[:, 0] + part[:, 2] + 1j * (part[:, 1] + part[:, 3])
    assert np.array_equal(dev, host)


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("n_bs,k", [(1, 0), (63, 1), (65, 2), (130, 0), (7, 7), (3, 8)])
def test_ragged_batches(n_bs, k, engine):
    text = generate_circuit(4, 12, 5)
    bits = random_bitstrings(16, n_bs, 77 + n_bs)
    note("ragged n_bs", n_bs, "k", k, "engine", engine)
    got, _ = run(text, bits, k=k, prec=q.QGM_C64, engine=engine)
    psi = oracle.sv_state(text)
    ref = np.array([psi[int(sum(int(b) << j for j, b in enumerate(x)))] for x in bits])
    assert nerr(got, ref, 16).max() <= C64_TOL


def test_rz_parameters_and_gradient_by_shift(cuda):
    text = generate_circuit(4, 10, 3, rz=True)
    _, npar = parse_header(text)
    th = random_thetas(npar, 2003)
    bits = random_bitstrings(16, 4, 1003)
    note("RZ circuit, params", npar)
    got, p = run(text, bits, k=2, params=th)
    ref = oracle.sv_amplitudes(text, bits, th)
    assert nerr(got, ref, 16).max() <= C128_TOL
    # shift rule through the device path: d alpha/d theta_0 = alpha(theta + pi e_0)/2
    th2 = th.copy()
    th2[0] += np.pi
    g = 0.5 * p.amplitudes(bits, th2)
    gref = np.array([oracle.sv_gradient_shift(text, x, th, which=[0])[0] for x in bits])
    assert np.abs(g - gref).max() <= 1e-13


def test_errors_on_device(config2, cuda):
    torch = cuda
    text, bits, _ = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=3, time_budget_s=0.1, flags=DET)
    p = q.Plan(c, sl, order)
    need = q.qgm_workspace_size(p.h, 4, 8)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QgmError) as e:
        q.qgm_amplitudes(p.h, bits[:4], None, small)
    assert e.value.status == -5
    bad = bits[:2].copy()
    bad[0, 0] = 2
    with pytest.raises(q.QgmError) as e:
        p.amplitudes(bad)
    assert e.value.status == -1
    with pytest.raises(q.QgmError) as e:
        p.amplitudes_range(bits[:2], None, 0, 9)
    assert e.value.status == -1
    assert p.amplitudes(bits[:0]).shape == (0,)


def test_one_shot_entry(config2):
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=2, time_budget_s=0.1, flags=DET)
    a = q.qgm_amplitude(text, bits[5], sl, order)
    assert nerr(a, ref[5], 25) <= C128_TOL


def test_config3_6x6x25_one_launch():
    text = generate_circuit(6, 25, 0)
    bits = random_bitstrings(36, 1024, 1000)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=10, time_budget_s=1.0, flags=DET)
    p = q.Plan(c, sl, order, prec=q.QGM_C64)
    note("6x6x25, 1024 bitstrings x 2^10 slices, c64, stats", p.stats())
    got = p.amplitudes(bits)
    sub = list(range(0, 1024, 64))
    ref = np.array([oracle.ve_amplitude(text, bits[i]) for i in sub])
    e = nerr(got[sub], ref, 36)
    note("subset max normalised error", e.max())
    assert e.max() <= C64_TOL
    # sum_x |alpha_x|^2 = 1 implies E_x[2^N |alpha_x|^2] = 1 over uniform x
    m1 = np.mean((2.0 ** 36) * np.abs(got) ** 2)
    note("Porter-Thomas first moment", m1)
    assert abs(m1 - 1.0) < 0.2


@pytest.mark.parametrize("engine", ENGINES)
def test_graph_replay_matches_direct_launch(config2, cuda, engine):
    """Captured runs replayed several times, with eager work in between, give
    the direct launch's result bit for bit on every replay."""
    torch = cuda
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=7, time_budget_s=0.2, flags=DET)
    p = q.Plan(c, sl, order, prec=q.QGM_C64, engine=engine)
    n_s = 1 << 7
    d_bits = torch.from_numpy(bits).cuda()
    ws = p.workspace(64, n_s)
    d_direct = torch.empty((64, 4), dtype=torch.float64, device="cuda")
    q.qgm_amplitudes_device(p.h, d_bits, None, 0, n_s, ws, d_direct)
    direct = d_direct.cpu().numpy()
    d_part = torch.full((64, 4), float("nan"), dtype=torch.float64, device="cuda")
    g = q.qgm_graph_create(p.h, d_bits, None, 0, n_s, ws, d_part, repeat=3)
    try:
        for rep in range(4):
            d_part.fill_(float("nan"))
            scratch = torch.randn(1 << 16, device="cuda") * 2.0  # unrelated eager work
            torch.cuda.synchronize()
            q.qgm_graph_launch(g)
            torch.cuda.synchronize()
            note("graph replay", rep, "engine", engine, float(scratch.sum()))
            assert np.array_equal(d_part.cpu().numpy(), direct)
    finally:
        q.qgm_graph_free(g)
    amp = direct[:, 0] + direct[:, 2] + 1j * (direct[:, 1] + direct[:, 3])
    assert nerr(amp, ref, 25).max() <= C64_TOL


def _rz_case(n, d, seed, n_bs=1):
    text = generate_circuit(n, d, seed, rz=True)
    _, npar = parse_header(text)
    th = random_thetas(npar, seed + 2000)
    bits = random_bitstrings(n * n, n_bs, seed + 1000)
    return text, th, bits


@pytest.mark.parametrize("engine", ENGINES)
def test_gradient_vs_shift_rule_and_fd(engine):
    text, th, bits = _rz_case(4, 10, 3)
    x = bits[0]
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=2, time_budget_s=0.2, flags=DET)
    p = q.Plan(c, sl, order, engine=engine, gradient=True)
    note("gradient 4x4x10 RZ, params", len(th), "engine", engine, "stats", p.stats()["n_steps"])
    amp, grad = p.amplitude_grad(x, th)
    ref_amp = oracle.sv_amplitudes(text, [x], th)[0]
    shift = oracle.sv_gradient_shift(text, x, th)
    scale = max(abs(ref_amp), 2.0 ** -8)
    assert abs(amp - ref_amp) / scale <= C128_TOL
    assert np.max(np.abs(grad - shift)) / scale <= 1e-11
    # central differences of the device amplitudes, h = 1e-4 (error ~ h^2/6 |alpha'''|)
    plain = q.Plan(c, sl, order, engine=engine)
    fd = oracle.fd_gradient(lambda pp: plain.amplitudes([x], pp)[0], th, h=1e-4)
    assert np.max(np.abs(grad - fd)) / scale <= 1e-7


@pytest.mark.parametrize("engine", ENGINES)
def test_gradient_summed_over_slices_5x5x20(engine):
    text, th, bits = _rz_case(5, 20, 1)
    x = bits[0]
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.3, flags=DET)
    p = q.Plan(c, sl, order, engine=engine, gradient=True)
    note("gradient 5x5x20 RZ, k=6, params", len(th), "engine", engine)
    amp, grad = p.amplitude_grad(x, th)
    net = oracle.build_network(text, th)
    ref_amp = oracle.ve_amplitude(text, x, params=th, net=net)
    shift = []
    for j in range(len(th)):
        t2 = th.copy()
        t2[j] += np.pi
        shift.append(0.5 * oracle.ve_amplitude(text, x, params=t2))
    shift = np.array(shift)
    scale = max(abs(ref_amp), 2.0 ** -12.5)
    assert abs(amp - ref_amp) / scale <= C128_TOL
    assert np.max(np.abs(grad - shift)) / scale <= 1e-11


def test_gradient_c64_and_device_entry(cuda):
    torch = cuda
    text, th, bits = _rz_case(4, 12, 7, n_bs=3)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=3, time_budget_s=0.2, flags=DET)
    p = q.Plan(c, sl, order, prec=q.QGM_C64, gradient=True)
    npar = len(th)
    d_bits = torch.from_numpy(bits).cuda()
    d_th = torch.from_numpy(th).cuda()
    d_part = torch.empty((3, 4), dtype=torch.float64, device="cuda")
    d_g = torch.empty((3, npar, 4), dtype=torch.float64, device="cuda")
    q.qgm_gradients_device(p.h, d_bits, d_th, 0, 8, p.workspace(3), d_part, d_g)
    g = d_g.cpu().numpy()
    grads = g[..., 0] + g[..., 2] + 1j * (g[..., 1] + g[..., 3])
    for i in range(3):
        shift = oracle.sv_gradient_shift(text, bits[i], th)
        ref = oracle.sv_amplitudes(text, [bits[i]], th)[0]
        scale = max(abs(ref), 2.0 ** -8)
        assert np.max(np.abs(grads[i] - shift)) / scale <= C64_GRAD_TOL


def test_autograd_function_gradcheck(cuda):
    torch = cuda
    text, th, bits = _rz_case(3, 8, 11)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=1, time_budget_s=0.1, flags=DET)
    p = q.Plan(c, sl, order, gradient=True)
    Fn = q.AmplitudeFn
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    note("gradcheck 3x3x8 RZ params", len(th))
    assert torch.autograd.gradcheck(lambda t: Fn.apply(t, p, bits[0]), (theta,), eps=1e-6, atol=1e-8, rtol=1e-6)
    # |alpha|^2 backward against the shift rule
    a = Fn.apply(theta, p, bits[0])
    (a.abs() ** 2).backward()
    ref = oracle.sv_amplitudes(text, [bits[0]], th)[0]
    shift = oracle.sv_gradient_shift(text, bits[0], th)
    want = 2.0 * np.real(np.conj(ref) * shift)
    assert np.max(np.abs(theta.grad.numpy() - want)) <= 1e-12


@pytest.fixture(scope="module")
def config4():
    """7x7x30 with every T replaced by RZ(theta), k = 6 (64 slices = one group)."""
    text, th, bits = _rz_case(7, 30, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=2.0, flags=DET)
    return text, th, bits[0], c, sl, order


def test_config4_7x7x30_slices_vs_oracle(config4):
    text, th, x, c, sl, order = config4
    p = q.Plan(c, sl, order)
    st = p.stats()
    note("7x7x30 RZ k=6 stats", {k: st[k] for k in ("engine", "max_rank", "item_elems", "n_steps")})
    assert st["engine"] == q.QGM_ENGINE_WIDE
    net = oracle.build_network(text, th)
    for s in (0, 37):
        part = p.amplitudes_range([x], th, s, s + 1)[0]
        got = part[0] + part[2] + 1j * (part[1] + part[3])
        ref = oracle.ve_slice_values(text, x, sliced=sl, params=th, slices=[s], net=net)[0]
        note("slice", s, "device", got, "oracle", ref)
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 2.0 ** -24.5)


def test_config4_gradient_vs_device_shift_and_fd(config4):
    """Adjoint d alpha / d theta for all angles vs the parameter-shift rule and
    central differences (h = 1e-4, FP64), both evaluated on the device path
    whose slices are pinned to the oracle above."""
    text, th, x, c, sl, order = config4
    g = q.Plan(c, sl, order, gradient=True)
    note("7x7x30 gradient stats", {k: g.stats()[k] for k in ("engine", "item_elems", "n_steps")})
    amp, grad = g.amplitude_grad(x, th)
    p = q.Plan(c, sl, order)
    assert abs(p.amplitudes([x], th)[0] - amp) <= 1e-12 * abs(amp)
    scale = max(abs(amp), 2.0 ** -24.5)
    rng = np.random.default_rng(0)
    subset = sorted(rng.choice(len(th), 16, replace=False))
    shift = []
    for j in range(len(th)):
        t2 = th.copy()
        t2[j] += np.pi
        shift.append(0.5 * p.amplitudes([x], t2)[0])
    shift = np.array(shift)
    note("params", len(th), "max |adjoint - shift| / scale", np.max(np.abs(grad - shift)) / scale)
    assert np.max(np.abs(grad - shift)) / scale <= 1e-11
    fd = oracle.fd_gradient(lambda pp: p.amplitudes([x], pp)[0], th, h=1e-4, which=subset)
    assert np.max(np.abs(grad[subset] - fd)) / scale <= 1e-7


def test_wide_engine_multiple_groups_and_passes(config2):
    """640 bitstrings x 2^3 slices = 80 groups of 64 items, in passes of 7 groups."""
    text, _, _ = config2
    bits = random_bitstrings(25, 640, 4242)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=3, time_budget_s=0.2, flags=DET)
    gen = q.Plan(c, sl, order, engine=q.QGM_ENGINE_GENERATED).amplitudes(bits)
    st = q.Plan(c, sl, order, engine=q.QGM_ENGINE_WIDE).stats()
    cap = 7 * st["item_elems"] * 64 * 16 + 100000
    wide = q.Plan(c, sl, order, engine=q.QGM_ENGINE_WIDE, workspace_cap=cap).amplitudes(bits)
    assert np.max(np.abs(wide - gen) / np.maximum(np.abs(gen), 2.0 ** -12.5)) <= C128_TOL
    ref = np.array([oracle.ve_amplitude(text, bits[i]) for i in range(0, 640, 80)])
    assert nerr(wide[::80], ref, 25).max() <= C128_TOL


def test_autotune_keeps_results(config2):
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=DET)
    for prec, tol in ((q.QGM_C64, C64_TOL), (q.QGM_C128, C128_TOL)):
        p = q.Plan(c, sl, order, prec=prec, engine=q.QGM_ENGINE_GENERATED)
        w = p.autotune(64)
        note("autotune prec", prec, "chose waves", w, "stats waves", p.stats()["waves"])
        assert w in (1, 2, 4, 8) and p.stats()["waves"] == w
        assert nerr(p.amplitudes(bits), ref, 25).max() <= tol


@pytest.mark.parametrize("flags", [0, q.QGM_PLAN_LATENCY])
@pytest.mark.parametrize("waves", [1, 2, 4, 8])
@pytest.mark.parametrize("prec,tol", [(q.QGM_C64, C64_TOL), (q.QGM_C128, C128_TOL), (q.QGM_BF16X3, None)])
def test_multiwave_schedules(config2, waves, prec, tol, flags):
    """The generated kernel with its item tree list-scheduled on 1, 2, 4 or 8
    wavefronts (tensors crossing wavefronts through LDS) against the oracle;
    a schedule whose exchange does not fit in LDS falls back to fewer."""
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.5, flags=flags | DET)
    p = q.Plan(c, sl, order, prec=prec, engine=q.QGM_ENGINE_GENERATED, waves=waves)
    got_w = p.stats()["waves"]
    note("5x5x20 planner flags", flags, "prec", prec, "waves asked", waves, "got", got_w)
    assert got_w <= waves
    got = p.amplitudes(bits)
    assert np.all(np.isfinite(got))  # a wait that gave up would flag the block with NaN
    tol = bf16x3_tol(p.stats()["n_steps"]) if tol is None else tol
    assert nerr(got, ref, 25).max() <= tol


@pytest.mark.parametrize("engine", ENGINES)
def test_bf16x3_config2(config2, engine):
    text, bits, ref = config2
    note("BF16x3 5x5x20 k=6 engine", engine)
    got, p = run(text, bits, k=6, prec=q.QGM_BF16X3, engine=engine)
    e = nerr(got, ref, 25)
    c64, _ = run(text, bits, k=6, prec=q.QGM_C64, engine=engine)
    e64 = nerr(c64, ref, 25)
    tol = bf16x3_tol(p.stats()["n_steps"])
    note("max normalised error bf16x3", e.max(), "c64", e64.max(), "tol", tol)
    assert e.max() <= tol
    assert e.max() > e64.max()  # the split products are coarser than FP32 products


def test_wide_prebuilt_step_kernel_matches_generated(config2):
    """The wide engine's prebuilt step kernel (kept as the fallback when
    generated kernels cannot be built) against the generated ones."""
    import os
    text, bits, ref = config2
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.2, flags=DET)
    gen = q.Plan(c, sl, order, engine=q.QGM_ENGINE_WIDE).amplitudes(bits)
    os.environ["QGM_WIDE_PREBUILT"] = "1"
    try:
        pre = q.Plan(c, sl, order, engine=q.QGM_ENGINE_WIDE).amplitudes(bits)
    finally:
        del os.environ["QGM_WIDE_PREBUILT"]
    assert nerr(pre, ref, 25).max() <= C128_TOL
    assert nerr(gen, ref, 25).max() <= C128_TOL


def _stored(name):
    import json
    import os
    path = os.path.join(os.path.dirname(q.__file__), "plans", name + ".json")
    with open(path) as f:
        rec = json.load(f)
    cc = rec["circuit"]
    return generate_circuit(cc["n"], cc["depth"], cc["seed"]), rec["sliced"], rec["order"]


def test_matrix_core_steps_7x7x30():
    """Wide engine, complex64 and BF16x3, two-operand contractions on the matrix cores:
    amplitudes against the complex128 path (pinned to the oracle) and the
    vector-only complex64 path, and single slices against the oracle."""
    text, sl, order = _stored("7x7x30")
    c = q.Circuit(text)
    pm = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE)
    pv = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, vector_only=True)
    pd = q.Plan(c, sl, order, prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE)
    sm, sv = pm.stats(), pv.stats()
    note("7x7x30 stored plan: mfma steps", sm["mfma_steps"], "flops share", sm["flops_mfma"] / sm["flops_item"])
    assert sm["mfma_steps"] >= 1 and sv["mfma_steps"] == 0 and sv["flops_mfma"] == 0.0
    bits = random_bitstrings(49, 8, 777)
    am, av, ad = pm.amplitudes(bits), pv.amplitudes(bits), pd.amplitudes(bits)
    note("max err mfma", nerr(am, ad, 49).max(), "vector", nerr(av, ad, 49).max())
    assert nerr(am, ad, 49).max() <= C64_TOL
    assert nerr(av, ad, 49).max() <= C64_TOL
    pb = q.Plan(c, sl, order, prec=q.QGM_BF16X3, engine=q.QGM_ENGINE_WIDE)
    pbv = q.Plan(c, sl, order, prec=q.QGM_BF16X3, engine=q.QGM_ENGINE_WIDE, vector_only=True)
    assert pb.stats()["mfma_steps"] == sm["mfma_steps"] and pbv.stats()["mfma_steps"] == 0
    ab, abv = pb.amplitudes(bits), pbv.amplitudes(bits)
    note("max err bf16x3 mfma", nerr(ab, ad, 49).max(), "vector", nerr(abv, ad, 49).max())
    tb = bf16x3_tol(pb.stats()["n_steps"])
    note("bf16x3 tolerance", tb)
    assert nerr(ab, ad, 49).max() <= tb
    assert nerr(abv, ad, 49).max() <= tb
    net = oracle.build_network(text)
    scale = 2.0 ** -24.5 / 2.0 ** 3
    for s in (0, 45):
        part = pm.amplitudes_range([bits[0]], None, s, s + 1)[0]
        got = part[0] + part[2] + 1j * (part[1] + part[3])
        ref = oracle.ve_slice_values(text, bits[0], sliced=sl, slices=[s], net=net)[0]
        note("slice", s, "mfma", got, "oracle", ref)
        assert abs(got - ref) / max(abs(ref), scale) <= C64_TOL


def test_matrix_core_steps_8x8x40():
    """8x8x40 with the stored k = 13 plan: most of the work runs on the matrix
    cores; 64 slices of one bitstring against the complex128 path and the
    vector-only path, slice by slice for three slices."""
    text, sl, order = _stored("8x8x40")
    c = q.Circuit(text)
    pm = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE)
    pd = q.Plan(c, sl, order, prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE)
    sm = pm.stats()
    note("8x8x40 stored plan: mfma steps", sm["mfma_steps"], "flops share", sm["flops_mfma"] / sm["flops_item"])
    assert sm["mfma_steps"] >= 5 and sm["flops_mfma"] >= 0.5 * sm["flops_item"]
    x = random_bitstrings(64, 1, 1000)[0]
    scale = 2.0 ** -32 / 2.0 ** 6.5

    def val(p, s0, s1):
        part = p.amplitudes_range([x], None, s0, s1)[0]
        return part[0] + part[2] + 1j * (part[1] + part[3])

    pb = q.Plan(c, sl, order, prec=q.QGM_BF16X3, engine=q.QGM_ENGINE_WIDE)
    assert pb.stats()["mfma_steps"] == sm["mfma_steps"]
    tb = bf16x3_tol(pb.stats()["n_steps"])
    for s0, s1 in ((0, 64), (100, 101), (4095, 4096), (8191, 8192)):
        got, ref, gb = val(pm, s0, s1), val(pd, s0, s1), val(pb, s0, s1)
        note("slices", s0, s1, "mfma", got, "bf16x3", gb, "c128", ref)
        assert abs(got - ref) / max(abs(ref), scale) <= C64_TOL
        assert abs(gb - ref) / max(abs(ref), scale) <= tb


def test_level_timing_entry_point(cuda):
    """qgm_plan_level_timing on a profiling wide plan: one entry per level
    launch, positive HIP-event durations that add up to about the chain's,
    per-level flops summing to the plan's flops per slice (one 64-item group:
    nothing shared), the matrix-core step counts, and the items of the timed
    pass; with two bitstrings in the pass, the steps that depend on no
    output bit run once for both groups, so the pass's work per item lies
    between half and all of the plan's."""
    text, sl, order = _stored("7x7x30")
    c = q.Circuit(text)
    p = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE, profile=True)
    st = p.stats()
    bits = random_bitstrings(49, 2, 55)
    for _ in range(3):
        p.amplitudes(bits[:1])
    cuda.cuda.synchronize()
    ms, fl, mf, runs, items, by, roof = q.qgm_plan_level_timing(p.h, reset=False)
    (ms_pro, ms_chain, ms_red), n = q.qgm_plan_timing(p.h, reset=True)
    note("levels", len(ms), "runs", runs, "items", items, "sum ms", sum(ms), "chain ms", ms_chain)
    assert len(ms) == st["launches"] and runs == 3 and items == 64
    assert all(t > 0 for t in ms)
    assert abs(sum(fl) - st["flops_item"]) <= 1e-9 * st["flops_item"]
    assert abs(sum(by) - st["bytes_item"]) <= 1e-9 * st["bytes_item"]
    assert abs(roof - st["roof_s_item"]) <= 1e-9 * st["roof_s_item"]
    assert sum(mf) == st["mfma_steps"]
    assert 0.5 * ms_chain <= sum(ms) <= 1.05 * ms_chain
    # reset forgot the runs
    ms2, _, _, runs2, _, _, _ = q.qgm_plan_level_timing(p.h, reset=True)
    assert runs2 == 0 and all(t == 0 for t in ms2)
    p.amplitudes(bits)
    cuda.cuda.synchronize()
    ms, fl, mf, runs, items, by, roof = q.qgm_plan_level_timing(p.h, reset=True)
    note("two bitstrings: flops per item", sum(fl), "of", st["flops_item"], "roofline", roof, "of", st["roof_s_item"])
    assert runs == 1 and items == 2 * 64
    assert 0.5 * st["flops_item"] <= sum(fl) <= st["flops_item"] * (1 + 1e-9)
    assert 0.5 * st["roof_s_item"] <= roof <= st["roof_s_item"] * (1 + 1e-9)


def test_matrix_core_steps_8x8x40_k10():
    """8x8x40 with the stored k = 10 plan (rank-24 intermediates, several
    64-item groups per pass): single slices and a range of complex64 on the
    matrix cores against the complex128 path."""
    text, sl, order = _stored("8x8x40-k10")
    c = q.Circuit(text)
    pm = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE)
    pd = q.Plan(c, sl, order, prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE)
    sm = pm.stats()
    note("8x8x40 k=10 plan: max rank", sm["max_rank"], "mfma steps", sm["mfma_steps"],
         "flops share", sm["flops_mfma"] / sm["flops_item"])
    assert sm["k"] == 10 and sm["mfma_steps"] >= 1
    x = random_bitstrings(64, 1, 1000)[0]
    scale = 2.0 ** -32 / 2.0 ** 5

    def val(p, s0, s1):
        part = p.amplitudes_range([x], None, s0, s1)[0]
        return part[0] + part[2] + 1j * (part[1] + part[3])

    for s0, s1 in ((0, 1), (777, 778), (0, 200)):
        got, ref = val(pm, s0, s1), val(pd, s0, s1)
        note("slices", s0, s1, "c64", got, "c128", ref)
        assert abs(got - ref) / max(abs(ref), scale) <= C64_TOL


def test_gradient_c64_with_matrix_core_steps(config4):
    """Reverse-mode plans run their large two-operand steps on the matrix
    cores too: complex64 amplitude and d alpha / d theta for every angle of
    the 7x7x30 RZ circuit against the complex128 plan (pinned above)."""
    text, th, x, c, sl, order = config4
    g64 = q.Plan(c, sl, order, prec=q.QGM_C64, gradient=True)
    st = g64.stats()
    note("7x7x30 c64 gradient plan: engine", st["engine"], "mfma steps", st["mfma_steps"])
    assert st["engine"] == q.QGM_ENGINE_WIDE and st["mfma_steps"] >= 1
    a64, d64 = g64.amplitude_grad(x, th)
    a128, d128 = q.Plan(c, sl, order, gradient=True).amplitude_grad(x, th)
    scale = max(abs(a128), 2.0 ** -24.5)
    note("amp err", abs(a64 - a128) / scale, "max grad err", np.max(np.abs(d64 - d128)) / scale)
    assert abs(a64 - a128) / scale <= C64_TOL
    assert np.max(np.abs(d64 - d128)) / scale <= C64_GRAD_TOL
