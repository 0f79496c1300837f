"""Undirected graphical model of a circuit (Section "Undirected Graphical Model").

Every distinct index value i_k^(j) of Eq. (1) is a binary variable.  A
diagonal gate forces its input and output index to be equal, so it creates
no variable; a non-diagonal one-qubit gate creates a new variable on its
qubit (gadgets of Fig. "tensornodes").  The initial index i_0 = 0...0 is a
constant, so the first variable of each qubit carries the unary factor
U[v, 0] of the gate that created it.

Variable numbering: variables are numbered in order of creation, gates
taken by ascending cycle and, inside a cycle, by ascending qubit.  For Rules
1-3 circuits, ids 0..N-1 are the variables after the initial H layer.  The
output variable of qubit q is its last variable; it is fixed to x_q
("removed for free", Section "Parallelization by fixing the values of
variables").  A qubit that no non-diagonal gate touches keeps the input
constant 0 as its output, which contributes delta(x_q, 0).

Factors are (vars, table) pairs: ``table`` is a complex128 array with one
length-2 axis per variable in ``vars`` (axis order = ``vars`` order).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuit import Circuit, parse_circuit
from .gates import TWO_QUBIT_NONDIAG, gate_matrix

INPUT = -1  # marker for the constant input index i_0 = 0


@dataclass
class Variable:
    id: int
    qubit: int
    cycle: int
    is_output: bool = False


@dataclass
class Network:
    n_qubits: int
    variables: list = field(default_factory=list)
    factors: list = field(default_factory=list)  # list of (tuple vars, ndarray)
    output_var: list = field(default_factory=list)  # per qubit: var id or INPUT
    n_params: int = 0
    # per RZ parameter index: the variable its diagonal factor sits on (the
    # qubit's current variable when the gate acts), or INPUT
    param_var: dict = field(default_factory=dict)

    @property
    def free_vars(self):
        """Variables that are neither outputs nor the input constant."""
        return [v.id for v in self.variables if not v.is_output]

    def graph_edges(self, exclude=()):
        """Edges (u < w) between distinct non-excluded variables sharing a factor."""
        ex = set(exclude)
        edges = set()
        for vs, _ in self.factors:
            live = sorted({v for v in vs if v not in ex})
            for i in range(len(live)):
                for j in range(i + 1, len(live)):
                    edges.add((live[i], live[j]))
        return edges


def _restrict(vars_, table, fixed: dict):
    """Index ``table`` at the fixed variables' values; returns (vars, table)."""
    keep = []
    idx = []
    for v in vars_:
        if v in fixed:
            idx.append(int(fixed[v]))
        else:
            idx.append(slice(None))
            keep.append(v)
    return tuple(keep), np.asarray(table[tuple(idx)], dtype=np.complex128)


def build_network(circuit, params=None) -> Network:
    c = parse_circuit(circuit) if isinstance(circuit, str) else circuit
    assert isinstance(c, Circuit)
    n = c.n_qubits
    net = Network(n_qubits=n, n_params=c.n_params)
    cur = [INPUT] * n
    fixed_input = {INPUT: 0}
    # creation order: by cycle, then by qubit inside the cycle
    order = sorted(range(len(c.gates)), key=lambda i: (c.gates[i].cycle, min(c.gates[i].qubits)))
    for gi in order:
        g = c.gates[gi]
        if g.name == "CZ":
            a, b = g.qubits
            table = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128)
            u, w = cur[a], cur[b]
            if u == w:  # cannot happen for distinct qubits
                raise AssertionError
            vs, t = _restrict((u, w), table, fixed_input)
            net.factors.append((vs, t))
        elif g.name in ("T", "I", "RZ"):
            theta = None if g.param < 0 else float(params[g.param])
            d = np.diag(gate_matrix(g.name, theta)).copy()
            q = g.qubits[0]
            if g.param >= 0:
                net.param_var[g.param] = cur[q]
            vs, t = _restrict((cur[q],), d, fixed_input)
            net.factors.append((vs, t))
        elif g.name in TWO_QUBIT_NONDIAG:
            # a two-qubit gate that is not diagonal: a new variable on each
            # qubit (the lower qubit's first) and one factor over the two new
            # and the two old variables (the K4 gadget of Fig. "tensornodes")
            a, b = g.qubits
            new = {}
            for q in sorted((a, b)):
                v = len(net.variables)
                net.variables.append(Variable(v, q, g.cycle))
                new[q] = v
            u = gate_matrix(g.name).reshape(2, 2, 2, 2)  # [out b, out a, in b, in a]
            table = np.transpose(u, (1, 0, 3, 2))  # [out a, out b, in a, in b]
            vs, t = _restrict((new[a], new[b], cur[a], cur[b]), table, fixed_input)
            net.factors.append((vs, t))
            cur[a], cur[b] = new[a], new[b]
        else:  # H, SX, SY: new variable
            q = g.qubits[0]
            v = len(net.variables)
            net.variables.append(Variable(v, q, g.cycle))
            u = gate_matrix(g.name)
            vs, t = _restrict((v, cur[q]), u, fixed_input)
            net.factors.append((vs, t))
            cur[q] = v
    for q in range(n):
        net.output_var.append(cur[q])
        if cur[q] != INPUT:
            net.variables[cur[q]].is_output = True
    return net


def project(net: Network, x, fixed_extra: dict | None = None):
    """Factors with outputs fixed to ``x`` and ``fixed_extra`` vars fixed.

    Returns (factors, scalar) where ``scalar`` collects the constant
    factors (rank 0 after fixing), including delta(x_q, 0) for a qubit whose
    output is the input constant.
    """
    fixed = {}
    scalar = 1.0 + 0.0j
    for q, v in enumerate(net.output_var):
        if v == INPUT:
            if int(x[q]) != 0:
                scalar = 0.0 + 0.0j
        else:
            fixed[v] = int(x[q])
    if fixed_extra:
        fixed.update({int(k): int(b) for k, b in fixed_extra.items()})
    out = []
    for vs, t in net.factors:
        kv, kt = _restrict(vs, t, fixed)
        if len(kv) == 0:
            scalar = scalar * complex(kt)
        else:
            out.append((kv, kt))
    return out, scalar
