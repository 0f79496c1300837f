"""The stored plans the benchmark times, against the FP64 oracle.

tests/golden/stored_plan_slices.json holds the oracle's values of single
slices of every stored 8x8x40 plan (k = 8 ... 13; k = 8 is the benchmark's
whole-amplitude workload) and of the 7x7x30 plan with RZ angles (slices,
the whole amplitude and 16 derivatives d alpha / d theta).  They are written
by tests/golden/make_stored_plan_slices.py, which calls only the oracle.

Tolerances (per slice, relative to the oracle's slice value):
* complex128: 1e-12;
* complex64: C64_TOL of the other parity tests (2e-4);
* BF16x3: sqrt(D) * 3 * 2^-16 with D the number of item steps of the
  plan: the per-product bound of the three-term split (3 * 2^-16, see
  tests/test_gpu_contraction.py) grown like a random walk over D dependent
  steps.  A plain bfloat16 product (2^-8) gives about 256x that.
"""
import json
import math
import os

import numpy as np
import pytest

import paper_1805_01450_amd as q
from tests.conftest import golden_path
from workload import generate_circuit, parse_header, random_bitstrings, random_thetas

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12
C64_TOL = 2e-4

with open(golden_path("stored_plan_slices.json")) as _f:
    GOLD = json.load(_f)


def note(*args):
    print("[gpu-stored]", *args, flush=True)


@pytest.fixture(autouse=True)
def _release_device_memory():
    """Plans of these circuits take tens of GiB of workspace: hand the cached
    blocks back after each test so the next plan's sizes fit."""
    yield
    import gc

    import torch
    gc.collect()
    torch.cuda.empty_cache()


def bf16x3_tol(n_steps):
    return math.sqrt(n_steps) * 3 * 2.0 ** -16


def _plan_rec(name):
    with open(os.path.join(os.path.dirname(q.__file__), "plans", name + ".json")) as f:
        return json.load(f)


def _slice(p, x, s, params=None):
    part = p.amplitudes_range([x], params, s, s + 1)[0]
    return part[0] + part[2] + 1j * (part[1] + part[3])


@pytest.mark.parametrize("name", ["8x8x40-k8", "8x8x40"])
@pytest.mark.parametrize("prec", [q.QGM_C128, q.QGM_C64, q.QGM_BF16X3])
def test_benched_plans_slices_vs_oracle(name, prec):
    """Slices of the benchmark's k = 8 plan and of the k = 13 plan, every
    precision, the matrix-core steps included."""
    rec = _plan_rec(name)
    gold = GOLD[name]
    c = rec["circuit"]
    assert gold["circuit"] == c and gold["k"] == rec["k"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, gold["bitstring_seed"])[0]
    circ = q.Circuit(text)
    p = q.Plan(circ, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE)
    st = p.stats()
    if prec != q.QGM_C128:
        assert st["mfma_steps"] >= 5
    tol = {q.QGM_C128: C128_TOL, q.QGM_C64: C64_TOL, q.QGM_BF16X3: bf16x3_tol(st["n_steps"])}[prec]
    for s, v in gold["slices"].items():
        ref = complex(v[0], v[1])
        got = _slice(p, x, int(s))
        err = abs(got - ref) / abs(ref)
        note(name, "prec", prec, "slice", s, "rel err", err, "tol", tol)
        assert err <= tol


@pytest.mark.parametrize("name", ["8x8x40-k9", "8x8x40-k10", "8x8x40-k11", "8x8x40-k12"])
def test_other_stored_plans_slices_vs_oracle(name):
    """The remaining stored plans: complex128 and complex64 slices."""
    rec = _plan_rec(name)
    gold = GOLD[name]
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, gold["bitstring_seed"])[0]
    circ = q.Circuit(text)
    for prec, tol in ((q.QGM_C128, C128_TOL), (q.QGM_C64, C64_TOL)):
        p = q.Plan(circ, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE)
        for s, v in gold["slices"].items():
            ref = complex(v[0], v[1])
            err = abs(_slice(p, x, int(s)) - ref) / abs(ref)
            note(name, "prec", prec, "slice", s, "rel err", err)
            assert err <= tol
        del p


@pytest.fixture(scope="module")
def whole_k13():
    rec = _plan_rec("8x8x40")
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, c["seed"] + 1000)[0]
    circ = q.Circuit(text)
    p = q.Plan(circ, rec["sliced"], rec["order"], prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE)
    a = p.amplitudes([x])[0]
    note("8x8x40 whole amplitude, k=13 plan, c128:", a)
    return circ, x, a


@pytest.mark.parametrize("name", ["8x8x40-k8", "8x8x40-k9", "8x8x40-k10", "8x8x40-k11", "8x8x40-k12"])
def test_whole_amplitude_same_for_every_stored_plan(whole_k13, name):
    """Fixing variables changes only how the sum is split (Section
    "Parallelization by fixing the values of variables"): the complex128
    whole amplitude of every stored plan equals the k = 13 plan's."""
    circ, x, a13 = whole_k13
    rec = _plan_rec(name)
    p = q.Plan(circ, rec["sliced"], rec["order"], prec=q.QGM_C128, engine=q.QGM_ENGINE_WIDE)
    a = p.amplitudes([x])[0]
    note(name, "c128 whole amplitude", a, "rel diff to k=13", abs(a - a13) / abs(a13))
    assert abs(a - a13) <= C128_TOL * abs(a13)


@pytest.fixture(scope="module")
def config4_rz():
    gold = GOLD["7x7x30-rz"]
    rec = _plan_rec("7x7x30")
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"], rz=True)
    _, npar = parse_header(text)
    th = random_thetas(npar, gold["theta_seed"])
    x = random_bitstrings(c["n"] ** 2, 1, gold["bitstring_seed"])[0]
    return gold, rec, q.Circuit(text), th, x


@pytest.mark.parametrize("prec,tol", [(q.QGM_C128, C128_TOL), (q.QGM_C64, C64_TOL)])
def test_config4_amplitude_and_slices_vs_oracle(config4_rz, prec, tol):
    gold, rec, circ, th, x = config4_rz
    p = q.Plan(circ, rec["sliced"], rec["order"], prec=prec)
    for s, v in gold["slices"].items():
        ref = complex(v[0], v[1])
        err = abs(_slice(p, x, int(s), th) - ref) / abs(ref)
        note("7x7x30 RZ slice", s, "prec", prec, "rel err", err)
        assert err <= tol
    a = p.amplitudes([x], th)[0]
    ref = complex(*gold["alpha"])
    note("7x7x30 RZ amplitude", a, "oracle", ref)
    assert abs(a - ref) <= tol * abs(ref)


def test_config4_slice_gradient_vs_oracle(config4_rz):
    """The adjoint over one slice, qgm_gradients_device on [s, s + 1), against
    the oracle's slice identity d alpha_s / d theta_j = (i/2)(alpha_s|u=1 -
    alpha_s|u=0) (u = theta_j's variable) for 16 angles, among them two on
    one variable and one on a fixed variable."""
    import torch
    gold, rec, circ, th, x = config4_rz
    g = q.Plan(circ, rec["sliced"], rec["order"], gradient=True)
    s = gold["grad_slice"]
    npar = len(th)
    d_bits = torch.from_numpy(np.asarray([x], dtype=np.uint8)).cuda()
    d_th = torch.from_numpy(th).cuda()
    d_part = torch.empty((1, 4), dtype=torch.float64, device="cuda")
    d_g = torch.empty((1, npar, 4), dtype=torch.float64, device="cuda")
    q.qgm_gradients_device(g.h, d_bits, d_th, s, s + 1, g.workspace(1, 1), d_part, d_g)
    gg = d_g.cpu().numpy()[0]
    grad = gg[:, 0] + gg[:, 2] + 1j * (gg[:, 1] + gg[:, 3])
    part = d_part.cpu().numpy()[0]
    alpha_s = part[0] + part[2] + 1j * (part[1] + part[3])
    ref_s = complex(*gold["slices"][str(s)])
    assert abs(alpha_s - ref_s) <= C128_TOL * abs(ref_s)
    which = gold["grad_which"]
    want = np.array([complex(*v) for v in gold["grad"]])
    scale = abs(ref_s)
    err = np.abs(grad[which] - want) / scale
    note("slice", s, "max |adjoint - oracle| / |alpha_s|", err.max())
    assert err.max() <= 1e-11


def test_config4_whole_gradient_vs_oracle(config4_rz):
    """d alpha / d theta over all slices, complex128 and complex64, against
    the oracle's slice identity summed over every slice, for the same 16
    angles.  complex64 tolerance: 2 x C64_TOL (the reverse pass doubles the
    chain depth in the linear rounding bound)."""
    gold, rec, circ, th, x = config4_rz
    which = gold["grad_which"]
    want = np.array([complex(*v) for v in gold["grad_full"]])
    alpha = complex(*gold["alpha"])
    scale = max(abs(alpha), 2.0 ** -24.5)
    for prec, tol in ((q.QGM_C128, 1e-11), (q.QGM_C64, 2 * C64_TOL)):
        g = q.Plan(circ, rec["sliced"], rec["order"], prec=prec, gradient=True)
        amp, grad = g.amplitude_grad(x, th)
        err = np.abs(grad[which] - want) / scale
        note("7x7x30 whole gradient prec", prec, "max err", err.max(), "amp err", abs(amp - alpha) / abs(alpha))
        assert abs(amp - alpha) <= (C128_TOL if prec == q.QGM_C128 else C64_TOL) * abs(alpha)
        assert err.max() <= tol


@pytest.mark.parametrize("ck", [2, 4, 8])
def test_config4_checkpointed_gradient_vs_oracle(config4_rz, ck):
    """checkpoint_every = n keeps only the forward tensors consumed in another
    segment of n eliminations and recomputes the rest by the same steps: the
    gradient equals the fully stored one (same operations on the same values)
    and the oracle's, with about half the peak item memory."""
    gold, rec, circ, th, x = config4_rz
    which = gold["grad_which"]
    want = np.array([complex(*v) for v in gold["grad_full"]])
    alpha = complex(*gold["alpha"])
    g0 = q.Plan(circ, rec["sliced"], rec["order"], gradient=True)
    g = q.Plan(circ, rec["sliced"], rec["order"], gradient=True, checkpoint_every=ck)
    note("checkpoint_every", ck, "item elems", g.stats()["item_elems"], "vs", g0.stats()["item_elems"])
    assert g.stats()["item_elems"] < g0.stats()["item_elems"]
    a0, d0 = g0.amplitude_grad(x, th)
    a, d = g.amplitude_grad(x, th)
    scale = abs(alpha)
    note("max |checkpointed - stored| / |alpha|", np.max(np.abs(d - d0)) / scale)
    assert a == a0
    assert np.max(np.abs(d - d0)) <= 1e-14 * scale
    assert np.max(np.abs(d[which] - want)) <= 1e-11 * scale


@pytest.mark.parametrize("prec", [q.QGM_C128, q.QGM_C64, q.QGM_BF16X3])
def test_benchmark_whole_amplitude_vs_oracle(prec):
    """The benchmark's result itself: the whole 8x8x40 amplitude (all 256
    slices of the stored k = 8 plan, the matrix-core steps and the stored
    tile table as bench.py runs them) against the FP64 oracle's sum of every
    slice (tests/golden/make_stored_plan_slices.py --whole)."""
    gold = GOLD["8x8x40-k8-whole"]
    rec = _plan_rec("8x8x40-k8")
    c = rec["circuit"]
    assert gold["circuit"] == c and gold["k"] == rec["k"] == 8
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    x = random_bitstrings(c["n"] ** 2, 1, gold["bitstring_seed"])[0]
    tiles = os.path.join(os.path.dirname(q.__file__), "plans", "tiles_mi355x.txt")
    p = q.Plan(q.Circuit(text), rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE,
               tile_table_path=tiles if prec != q.QGM_C128 else None)
    got = p.amplitudes([x])[0]
    ref = complex(gold["alpha"][0], gold["alpha"][1])
    tol = {q.QGM_C128: C128_TOL, q.QGM_C64: C64_TOL, q.QGM_BF16X3: bf16x3_tol(p.stats()["n_steps"])}[prec]
    err = abs(got - ref) / abs(ref)
    note("8x8x40-k8 whole amplitude prec", prec, got, "oracle", ref, "rel err", err, "tol", tol)
    assert err <= tol


def test_group_sharing_matches_unshared_passes():
    """Steps that depend on none of the slice bits (or bitstrings) that differ
    between the 64-item groups of a pass run in group 0 only and the other
    groups read their results (the stored k = 8 plan's sliced order puts the
    variables the least work depends on at slice bits 6 and 7).  Every slice
    value is the same whether or not a step is shared, so a pass of four
    groups (sharing over bits 6 and 7), of two bitstrings x two groups (bit 6
    and the bitstring), and a range that starts inside a group (no sharing)
    must give the amplitudes of one-group passes (nothing to share) up to the
    FP64 reduction order."""
    rec = _plan_rec("8x8x40-k8")
    c = rec["circuit"]
    text = generate_circuit(c["n"], c["depth"], c["seed"])
    xs = random_bitstrings(c["n"] ** 2, 2, 1000)
    circ = q.Circuit(text)
    tiles = os.path.join(os.path.dirname(q.__file__), "plans", "tiles_mi355x.txt")
    p4 = q.Plan(circ, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE,
                tile_table_path=tiles, workspace_cap=128 << 30)
    p1 = q.Plan(circ, rec["sliced"], rec["order"], prec=q.QGM_C64, engine=q.QGM_ENGINE_WIDE,
                tile_table_path=tiles, workspace_cap=30 << 30)
    assert p4.stats()["item_elems"] * 64 * 8 <= 30 << 30  # one group fits the small cap

    def amp(p, bits, s0, s1):
        part = p.amplitudes_range(bits, None, s0, s1)
        return part[:, 0] + part[:, 2] + 1j * (part[:, 1] + part[:, 3])

    for bits, s0, s1 in (([xs[0]], 0, 256), (list(xs), 0, 128), ([xs[0]], 32, 160)):
        a4, a1 = amp(p4, bits, s0, s1), amp(p1, bits, s0, s1)
        err = np.abs(a4 - a1) / np.abs(a1)
        note("group sharing", len(bits), "bitstrings, slices", s0, s1, a4, a1, "rel diff", err)
        assert np.all(err <= 1e-12)
