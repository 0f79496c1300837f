"""Pins of the FP64 oracle against the paper and against mathematics.

Nothing here retypes the oracle's formulas: each check comes from the
paper's worked example, a closed form, an algebraic identity of the gates,
or an agreement between the oracle's three independent routes (state
vector, variable elimination, brute-force labelling sum).
"""
import cmath
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle.elimination import exact_sum, min_fill_order
from oracle.gates import gate_matrix
from oracle.graph import Graph
from oracle.network import build_network, project
from tests.conftest import golden_path
from workload import generate_circuit, random_bitstrings, random_thetas

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)
I2 = np.eye(2, dtype=complex)


# --------------------------------------------------------------- gate tables
def test_gate_identities():
    sx, sy, t, h = (gate_matrix(g) for g in ("SX", "SY", "T", "H"))
    assert np.allclose(sx @ sx, X, atol=1e-15)
    assert np.allclose(sy @ sy, Y, atol=1e-15)
    assert np.allclose(h @ h, I2, atol=1e-15)
    assert np.allclose(t @ t, np.diag([1, 1j]), atol=1e-15)
    assert np.allclose(np.linalg.matrix_power(t, 8), I2, atol=1e-15)
    for m in (sx, sy, t, h, gate_matrix("RZ", 0.7)):
        assert np.allclose(m.conj().T @ m, I2, atol=1e-15)
    # T = e^{i pi/8} RZ(pi/4)
    assert np.allclose(t, cmath.exp(1j * math.pi / 8) * gate_matrix("RZ", math.pi / 4), atol=1e-15)
    # d RZ / d theta = (1/2) RZ(theta + pi)
    th, h_ = 0.37, 1e-6
    num = (gate_matrix("RZ", th + h_) - gate_matrix("RZ", th - h_)) / (2 * h_)
    assert np.allclose(num, 0.5 * gate_matrix("RZ", th + math.pi), atol=1e-9)


def test_cz_pair_identity():
    # CZ_12 CZ_13 = |0><0| (x) I_23 + |1><1| (x) Z_2 Z_3 (Discussion section)
    cz = gate_matrix("CZ")
    cz12 = np.kron(cz, I2)
    cz13 = np.zeros((8, 8), dtype=complex)
    for i in range(8):
        b1, b2, b3 = (i >> 2) & 1, (i >> 1) & 1, i & 1
        cz13[i, i] = -1 if (b1 and b3) else 1
    p0 = np.diag([1, 0]).astype(complex)
    p1 = np.diag([0, 1]).astype(complex)
    rhs = np.kron(p0, np.kron(I2, I2)) + np.kron(p1, np.kron(Z, Z))
    assert np.allclose(cz12 @ cz13, rhs)


# ------------------------------------------------------- worked example
def _read_fig3():
    sec = {}
    cur = None
    with open(golden_path("fig3_graph.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                sec[cur] = []
            else:
                sec[cur].append(line)
    return sec


def _edges(line):
    return {tuple(sorted(e)) for e in line.split()[1:]}


def _letter_map(net):
    """letter -> variable id, from the labelling i_1..i_7 of the example."""
    sec = _read_fig3()
    mapping = {}
    for line in sec["labelling"]:
        t, letters = line.split()
        cycle = int(t) - 1  # paper cycle C_t is cycle t-1 here
        for q, ch in enumerate(letters):
            cands = [v.id for v in net.variables if v.qubit == q and v.cycle <= cycle]
            vid = max(cands)
            assert mapping.setdefault(ch, vid) == vid, f"letter {ch} maps to two variables"
    assert len(set(mapping.values())) == len(mapping), "two letters share a variable"
    return mapping


def test_fig2_network_is_fig3_graph(fig2_text):
    net = build_network(fig2_text)
    sec = _read_fig3()
    m = _letter_map(net)
    inv = {v: k for k, v in m.items()}
    free = net.free_vars
    assert sorted(inv[v] for v in free) == sorted(sec["graph"][0].split()[1])
    outs = [v.id for v in net.variables if v.is_output]
    ours = {tuple(sorted(inv[a] + inv[b])) for a, b in net.graph_edges(exclude=outs)}
    assert ours == _edges(sec["graph"][1])
    # 2^28 terms before merging, 2^10 after (seven 4-bit strings -> 10 vars)
    before, after = map(int, sec["terms"][0].split())
    assert 7 * 4 == before and len(free) == after


@pytest.mark.parametrize("op,v", [("fix", "c"), ("fix", "e"), ("eliminate", "c"), ("eliminate", "e")])
def test_fig5_fig6_graph_operations(op, v):
    sec = _read_fig3()
    verts = set(sec["graph"][0].split()[1])
    g = Graph(verts, _edges(sec["graph"][1]))
    rank = getattr(g, op)(v)
    want = sec[f"{op} {v}"]
    assert g.vertices == set(want[0].split()[1])
    assert {tuple(sorted(e)) for e in g.edges} == _edges(want[1])
    if len(want) > 2:
        assert rank == int(want[2].split()[1])


# ---------------------------------------------------------- closed forms
def _all_x(n):
    return [tuple(b) for b in itertools.product([0, 1], repeat=n)]


def test_empty_circuit_is_delta():
    text = "qubits 3\n"
    for x in _all_x(3):
        want = 1.0 if x == (0, 0, 0) else 0.0
        assert oracle.sv_amplitudes(text, [x])[0] == want
        assert oracle.ve_amplitude(text, x) == want
        assert oracle.brute_amplitude(text, x) == want


def test_h_then_diagonal_closed_form():
    rng = np.random.default_rng(5)
    n = 5
    lines = [f"qubits {n}"] + [f"0 H {q}" for q in range(n)]
    czs, ts, rzs = [], [], []
    thetas = rng.uniform(0, 2 * np.pi, 4)
    for cyc in range(1, 7):
        a, b = rng.choice(n, 2, replace=False)
        lines.append(f"{cyc} CZ {a} {b}")
        czs.append((a, b))
        used = {a, b}
        q = int(rng.choice([q for q in range(n) if q not in used]))
        if cyc <= 4:
            lines.append(f"{cyc} RZ {q} {cyc - 1}")
            rzs.append((q, thetas[cyc - 1]))
        else:
            lines.append(f"{cyc} T {q}")
            ts.append(q)
    text = "\n".join(lines)
    for x in _all_x(n):
        want = 2 ** (-n / 2)
        for a, b in czs:
            want *= (-1) ** (x[a] * x[b])
        for q in ts:
            want *= cmath.exp(1j * math.pi * x[q] / 4)
        for q, th in rzs:
            want *= cmath.exp(1j * th * (2 * x[q] - 1) / 2)
        for got in (oracle.sv_amplitudes(text, [x], thetas)[0], oracle.ve_amplitude(text, x, params=thetas),
                    oracle.brute_amplitude(text, x, params=thetas)):
            assert abs(got - want) < 1e-14


def test_double_hadamard_and_t8():
    n = 4
    hh = "\n".join([f"qubits {n}"] + [f"{c} H {q}" for c in (0, 1) for q in range(n)])
    t8 = "\n".join([f"qubits {n}"] + [f"0 H {q}" for q in range(n)]
                   + [f"{c} T {q}" for c in range(1, 9) for q in range(n)]
                   + [f"9 H {q}" for q in range(n)])
    for text in (hh, t8):
        for x in _all_x(n):
            want = 1.0 if sum(x) == 0 else 0.0
            assert abs(oracle.sv_amplitudes(text, [x])[0] - want) < 1e-14
            assert abs(oracle.ve_amplitude(text, x) - want) < 1e-14


def test_bit_order_is_qubit_index():
    # SX SX = X on qubit 0 only: all amplitude on x = (1, 0, 0)
    text = "qubits 3\n0 SX 0\n1 SX 0\n"
    for x in _all_x(3):
        want = 1.0 if x == (1, 0, 0) else 0.0
        assert abs(oracle.sv_amplitudes(text, [x])[0] - want) < 1e-15
        assert abs(oracle.ve_amplitude(text, x) - want) < 1e-15
    assert oracle.sv_state(text)[1] != 0  # index 1 = bit 0 set


def test_qubit_without_nondiagonal_gate():
    text = "qubits 2\n0 H 0\n1 T 1\n2 CZ 0 1\n"
    for x in _all_x(2):
        want = 2 ** -0.5 if x[1] == 0 else 0.0
        assert abs(oracle.ve_amplitude(text, x) - want) < 1e-15
        assert abs(oracle.sv_amplitudes(text, [x])[0] - want) < 1e-15


# ------------------------------------------------- three routes agree
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sv_ve_brute_agree_4x4x10(seed):
    text = generate_circuit(4, 10, seed)
    for x in random_bitstrings(16, 4, seed + 1000):
        a = oracle.sv_amplitudes(text, [x])[0]
        b = oracle.ve_amplitude(text, x)
        c = oracle.brute_amplitude(text, x)
        assert abs(a - b) < 1e-13 and abs(a - c) < 1e-13


def test_fig2_all_outputs(fig2_text):
    for x in _all_x(4):
        a = oracle.sv_amplitudes(fig2_text, [x])[0]
        assert abs(a - oracle.ve_amplitude(fig2_text, x)) < 1e-14
        assert abs(a - oracle.brute_amplitude(fig2_text, x)) < 1e-14


def test_unitarity_sum_over_x():
    text = generate_circuit(3, 16, 4)
    vals = [oracle.ve_amplitude(text, x) for x in _all_x(9)]
    assert abs(sum(abs(v) ** 2 for v in vals) - 1.0) < 1e-13
    psi = oracle.sv_state(text)
    assert abs(np.vdot(psi, psi) - 1.0) < 1e-13


def test_slicing_and_order_invariance():
    text = generate_circuit(4, 12, 9, rz=True)
    th = random_thetas(40, 2009)
    x = random_bitstrings(16, 1, 1009)[0]
    net = build_network(text, th)
    ref = oracle.sv_amplitudes(text, [x], th)[0]
    rng = np.random.default_rng(0)
    free = net.free_vars
    for k in (0, 1, 3, 5):
        sl = [int(v) for v in rng.choice(free, k, replace=False)]
        rest = [v for v in free if v not in sl]
        for order in (None, list(rng.permutation(rest))):
            order = None if order is None else [int(v) for v in order]
            got = oracle.ve_amplitude(text, x, sliced=sl, order=order, params=th, net=net)
            assert abs(got - ref) < 1e-13


def test_ve_rejects_bad_order():
    text = generate_circuit(4, 10, 0)
    net = build_network(text)
    with pytest.raises(ValueError):
        oracle.ve_amplitude(text, [0] * 16, order=net.free_vars[:-1])


# -------------------------------------------------------------- gradients
def test_gradient_shift_fd_and_slice_identity():
    text = generate_circuit(4, 10, 2, rz=True)
    nq = 16
    from workload import parse_header
    _, npar = parse_header(text)
    th = random_thetas(npar, 2002)
    x = random_bitstrings(nq, 1, 1002)[0]
    shift = oracle.sv_gradient_shift(text, x, th)
    fd = oracle.fd_gradient(lambda p: oracle.sv_amplitudes(text, [x], p)[0], th)
    assert np.max(np.abs(shift - fd)) < 1e-8
    # d alpha / d theta_j = (i/2) (alpha|_{u=1} - alpha|_{u=0}), u = RZ's variable
    net = build_network(text, th)
    from oracle.circuit import parse_circuit
    circ = parse_circuit(text)
    cur = {}
    var_at = {}
    for g in sorted(circ.gates, key=lambda g: (g.cycle, min(g.qubits))):
        if g.name in ("H", "SX", "SY"):
            cur[g.qubits[0]] = max(v.id for v in net.variables
                                   if v.qubit == g.qubits[0] and v.cycle == g.cycle)
        if g.name == "RZ":
            var_at[g.param] = cur.get(g.qubits[0])
    for j in range(npar):
        u = var_at[j]
        if u is None or net.variables[u].is_output:
            continue
        vals = oracle.ve_slice_values(text, x, sliced=[u], params=th, net=net)
        assert abs(0.5j * (vals[1] - vals[0]) - shift[j]) < 1e-13


def test_exact_sum_is_exactly_rounded():
    vals = np.array([1e16, 1.0, -1e16, 1.0j], dtype=complex)
    assert exact_sum(vals) == complex(1.0, 1.0)


def test_min_fill_order_small_width():
    text = generate_circuit(5, 20, 0)
    net = build_network(text)
    factors, _ = project(net, [0] * 25)
    edges = set()
    for vs, _ in factors:
        for i in range(len(vs)):
            for j in range(i + 1, len(vs)):
                edges.add(tuple(sorted((vs[i], vs[j]))))
    order = min_fill_order(net.free_vars, edges)
    cost, width = oracle.order_cost(net.free_vars, edges, order)
    assert sorted(order) == sorted(net.free_vars)
    assert width <= 12 and cost < 1 << 16


# ------------------------------------------------ cost model of an ordering
def test_order_cost_on_fig3_graph():
    """Sum of 2^deg(v) on the Fig. 3 graph, worked by hand for the order
    d, c, h, i, j, a, b, e, f, g: degrees 1, 1, 2, 2, 2, 3, 2, 2, 1, 0 at
    their eliminations (h adds a-i, i adds a-j, j adds a-g, a adds e-g), so
    the cost is 2+2+4+4+4+8+4+4+2+1 = 35 and the width 3.  Eliminating e
    first costs 2^4 (the rank-4 tensor of Fig. 6); c first costs 2^1."""
    sec = _read_fig3()
    verts = sorted(sec["graph"][0].split()[1])
    edges = _edges(sec["graph"][1])
    assert oracle.order_cost(verts, edges, list("dchijabefg")) == (35, 3)
    assert oracle.order_cost(verts, edges, ["e"]) == (16, 4)
    assert oracle.order_cost(verts, edges, ["c", "e"]) == (2 + 8, 3)


def test_greedy_extra_slices_keep_the_sum():
    """Fixing more variables only splits the sum: the extra pieces chosen by
    the greedy removal add up to the unsliced slice, and the cost per piece
    does not grow."""
    from oracle.elimination import _graph_of, greedy_extra_slices
    text = generate_circuit(4, 12, 1)
    x = random_bitstrings(16, 1, 1001)[0]
    net = build_network(text)
    base, _ = project(net, x)
    g = _graph_of(base, net.free_vars)
    verts = sorted(g.vertices)
    order = min_fill_order(verts, g.edges)
    cost0, width0 = oracle.order_cost(verts, g.edges, order)
    extra, rest, cost, width = greedy_extra_slices(verts, g.edges, order, 3)
    assert len(set(extra)) == 3 and sorted(rest + extra) == sorted(order)
    assert cost <= cost0 and width <= width0
    whole = oracle.ve_amplitude(text, x, order=order, net=net)
    pieces = oracle.ve_slice_values(text, x, sliced=extra, order=rest, net=net)
    assert len(pieces) == 8
    assert abs(exact_sum(pieces) - whole) < 1e-15
    assert abs(whole - oracle.sv_amplitudes(text, [x])[0]) < 1e-14


# ------------------------------------------------------- gradient identities
def _rz_circuit_with_repeats():
    """H layer, RZ angles on post-H variables, on a variable that is sliced
    below, twice on one variable (no non-diagonal gate between), and on
    output variables (after the last SX/SY of their qubit)."""
    lines = ["qubits 4"] + [f"0 H {q}" for q in range(4)]
    lines += ["1 RZ 0 0", "1 CZ 1 2", "2 RZ 0 1", "2 SX 1", "3 CZ 0 1", "3 SY 2", "4 RZ 1 2",
              "4 CZ 2 3", "5 SX 0", "5 RZ 3 3", "6 CZ 0 3", "6 RZ 2 4", "7 SY 3", "7 RZ 0 5", "8 RZ 3 6"]
    return "\n".join(lines)


def test_network_param_var_is_the_qubits_current_variable():
    text = _rz_circuit_with_repeats()
    th = random_thetas(7, 7)
    net = build_network(text, th)
    # post-H variables are 0..3; SX on 1 at cycle 2 -> 4; SY on 2 at cycle 3 -> 5;
    # SX on 0 at cycle 5 -> 6; SY on 3 at cycle 7 -> 7
    assert net.param_var == {0: 0, 1: 0, 2: 4, 3: 3, 4: 5, 5: 6, 6: 7}
    outs = sorted(v.id for v in net.variables if v.is_output)
    assert outs == [4, 5, 6, 7]


def test_slice_gradients_sum_to_the_shift_rule():
    """Per-slice derivatives (slice identity) summed over all slices equal the
    parameter-shift derivative of the state vector; angles on one variable
    have equal derivatives; an angle on an output variable u = x_q gives
    (i/2)(2 x_q - 1) alpha."""
    from oracle.gradient import ve_slice_gradients
    text = _rz_circuit_with_repeats()
    th = random_thetas(7, 8)
    net = build_network(text, th)
    for x in ([0, 1, 1, 0], [1, 0, 0, 1]):
        shift = oracle.sv_gradient_shift(text, x, th)
        alpha = oracle.sv_amplitudes(text, [x], th)[0]
        # angles 0 and 1 sit on variable 0; 5 and 6 on outputs 6 (qubit 0) and 7 (qubit 3)
        assert abs(shift[0] - shift[1]) < 1e-15
        assert abs(shift[5] - 0.5j * (2 * x[0] - 1) * alpha) < 1e-15
        assert abs(shift[6] - 0.5j * (2 * x[3] - 1) * alpha) < 1e-15
        free = net.free_vars
        for sliced in ([], [0], [3, 1], [0, 1, 2, 3]):
            rest = [v for v in free if v not in sliced]
            tot = np.zeros(7, complex)
            per = []
            for s in range(1 << len(sliced)):
                per.append(ve_slice_gradients(text, x, th, sliced, rest, s, net=net))
            per = np.array(per)
            tot = np.array([exact_sum(per[:, j]) for j in range(7)])
            assert np.max(np.abs(tot - shift)) < 1e-15


def test_porter_thomas_second_moment():
    """A deep random 4x4 circuit: over all 2^16 outputs, p = 2^N |alpha_x|^2
    has mean exactly 1 (unitarity) and second moment close to 2, the
    exponential (Porter-Thomas) value the paper's Rules 1-3 circuits
    approach (Section "Numerical Results")."""
    text = generate_circuit(4, 40, 0)
    psi = oracle.sv_state(text)
    p = (2.0 ** 16) * np.abs(psi) ** 2
    assert abs(p.mean() - 1.0) < 1e-12
    assert abs((p ** 2).mean() - 2.0) < 0.1


# ---------------------------------------------- two-qubit non-diagonal gates
def _random_2q_circuit(seed, n=4, cycles=10, gate="CX"):
    rng = np.random.default_rng(seed)
    lines = [f"qubits {n}"] + [f"0 H {q}" for q in range(n)]
    for cyc in range(1, cycles + 1):
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        lines.append(f"{2 * cyc - 1} {gate} {a} {b}")
        q = int(rng.integers(n))
        lines.append(f"{2 * cyc} {['SX', 'SY', 'T'][int(rng.integers(3))]} {q}")
    return "\n".join(lines)


def _expand(text, rule):
    """Replace each two-qubit gate line by the lines rule(a, b) returns, the
    cycles renumbered so every replacement gate gets a cycle of its own."""
    out, cyc = [], 0
    for line in text.splitlines():
        tok = line.split()
        if tok[0] == "qubits":
            out.append(line)
            continue
        if len(tok) == 4 and tok[1] in ("CX", "ISWAP"):
            for g in rule(int(tok[2]), int(tok[3])):
                cyc += 1
                out.append(f"{cyc} {g}")
        else:
            cyc += 1
            out.append(f"{cyc} " + " ".join(tok[1:]))
    return "\n".join(out)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cx_is_h_cz_h(seed):
    """CX(a -> b) = (H on b) CZ(a, b) (H on b): the gadget of a non-diagonal
    two-qubit gate against one-qubit gadgets and the diagonal CZ."""
    text = _random_2q_circuit(seed, cycles=6, gate="CX")
    ref = _expand(text, lambda a, b: [f"H {b}", f"CZ {a} {b}", f"H {b}"])
    xs = [tuple((i >> q) & 1 for q in range(4)) for i in range(16)]
    want = oracle.sv_amplitudes(ref, xs)
    assert np.max(np.abs(oracle.sv_amplitudes(text, xs) - want)) < 1e-14
    for x in xs[:4]:
        assert abs(oracle.ve_amplitude(text, x) - want[xs.index(x)]) < 1e-14
        assert abs(oracle.brute_amplitude(text, x) - want[xs.index(x)]) < 1e-14


@pytest.mark.parametrize("seed", [3, 4])
def test_iswap_is_sqisw_twice(seed):
    text = _random_2q_circuit(seed, gate="ISWAP")
    ref = _expand(text, lambda a, b: [f"SQISW {a} {b}", f"SQISW {a} {b}"])
    xs = [tuple((i >> q) & 1 for q in range(4)) for i in range(16)]
    assert np.max(np.abs(oracle.sv_amplitudes(text, xs) - oracle.sv_amplitudes(ref, xs))) < 1e-14
    for x in xs[::5]:
        assert abs(oracle.ve_amplitude(text, x) - oracle.ve_amplitude(ref, x)) < 1e-14


def test_two_qubit_gates_closed_forms():
    """Worked by hand: SX SX = X on qubit 0, then CX(0 -> 1) gives |11>;
    ISWAP on |q0 = 1, q1 = 0> gives i |q0 = 0, q1 = 1>; SQISW on |00> keeps
    it."""
    xs = [(a, b) for b in (0, 1) for a in (0, 1)]  # (x0, x1)
    for route in ("sv", "ve", "brute"):
        def amp(text, x):
            if route == "sv":
                return oracle.sv_amplitudes(text, [x])[0]
            return (oracle.ve_amplitude if route == "ve" else oracle.brute_amplitude)(text, x)
        t1 = "qubits 2\n0 SX 0\n1 SX 0\n2 CX 0 1\n"
        assert [amp(t1, x) for x in xs] == pytest.approx([0, 0, 0, 1], abs=1e-15)
        t2 = "qubits 2\n0 SX 0\n1 SX 0\n2 ISWAP 0 1\n"
        assert [amp(t2, x) for x in xs] == pytest.approx([0, 0, 1j, 0], abs=1e-15)
        t3 = "qubits 2\n0 SQISW 0 1\n"
        assert [amp(t3, x) for x in xs] == pytest.approx([1, 0, 0, 0], abs=1e-15)


def test_two_qubit_gadget_is_k4():
    """A two-qubit gate that is not diagonal creates a variable on each of its
    qubits and one factor over the new and the old variables: in the graph
    the four form a clique (Fig. "tensornodes")."""
    text = "qubits 2\n0 H 0\n0 H 1\n1 ISWAP 0 1\n2 SX 0\n3 SX 1\n"
    net = build_network(text)
    # H: 0, 1; ISWAP: 2 (qubit 0), 3 (qubit 1); SX: 4, 5 (outputs)
    assert [(v.id, v.qubit) for v in net.variables] == [(0, 0), (1, 1), (2, 0), (3, 1), (4, 0), (5, 1)]
    edges = net.graph_edges()
    assert {(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)} <= edges
    assert (2, 4) in edges and (3, 5) in edges and (0, 4) not in edges
