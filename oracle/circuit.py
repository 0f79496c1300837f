"""Circuit text parser (format v1), independent of the GPU library's parser.

A circuit is a sequence of clock cycles C_1 ... C_d, each a tensor product
of one- and two-qubit gates (Eq. (1)).  Text format, one gate per line::

    qubits N
    grid R C                       (optional, informational)
    <cycle> <GATE> <q0> [<q1>] [<param_index>]

GATE in {H, CZ, T, SX, SY, RZ, I, CX, ISWAP, SQISW}; CZ, CX, ISWAP and
SQISW have two qubits (q0 first), RZ one qubit and a parameter index.  Gates are applied in ascending cycle, and within a cycle
in the order written (they act on distinct qubits, so they commute).
"""
from __future__ import annotations

from dataclasses import dataclass, field

ONE_QUBIT = {"H", "T", "SX", "SY", "I"}
TWO_QUBIT = {"CZ", "CX", "ISWAP", "SQISW"}


@dataclass
class Gate:
    cycle: int
    name: str
    qubits: tuple
    param: int = -1


@dataclass
class Circuit:
    n_qubits: int
    gates: list = field(default_factory=list)
    n_params: int = 0


def parse_circuit(text: str) -> Circuit:
    nq = None
    gates = []
    n_params = 0
    for lineno, raw in enumerate(text.splitlines(), 1):
        tok = raw.split("#", 1)[0].split()
        if not tok:
            continue
        if tok[0] == "qubits":
            nq = int(tok[1])
            continue
        if tok[0] == "grid":
            continue
        cyc = int(tok[0])
        name = tok[1]
        if name in TWO_QUBIT:
            if len(tok) != 4:
                raise ValueError(f"line {lineno}: {name} needs two qubits")
            qs = (int(tok[2]), int(tok[3]))
            if qs[0] == qs[1]:
                raise ValueError(f"line {lineno}: {name} on one qubit")
            g = Gate(cyc, name, qs)
        elif name == "RZ":
            if len(tok) != 4:
                raise ValueError(f"line {lineno}: RZ needs qubit and parameter index")
            g = Gate(cyc, name, (int(tok[2]),), int(tok[3]))
            n_params = max(n_params, g.param + 1)
        elif name in ONE_QUBIT:
            if len(tok) != 3:
                raise ValueError(f"line {lineno}: {name} needs one qubit")
            g = Gate(cyc, name, (int(tok[2]),))
        else:
            raise ValueError(f"line {lineno}: unknown gate {name!r}")
        gates.append(g)
    if nq is None:
        raise ValueError("missing 'qubits N' header")
    for g in gates:
        for q in g.qubits:
            if not 0 <= q < nq:
                raise ValueError(f"qubit {q} out of range")
    # stable sort by cycle keeps the written order inside a cycle
    gates.sort(key=lambda g: g.cycle)
    return Circuit(nq, gates, n_params)
