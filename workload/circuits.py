"""Rules 1-3 random grid circuits ("Numerical Results" section), as text.

Circuit text format v1 (one gate per line, '#' starts a comment)::

    qubits N
    grid R C                     # optional
    <cycle> <GATE> <q0> [<q1>] [<param_index>]

GATE is one of H, CZ, T, SX, SY, RZ, I.  CZ takes two qubits, RZ one qubit
and one parameter index (the angle itself is passed separately), every
other gate one qubit.  Gates of one cycle act on distinct qubits.

Readings of the rules (the paper states them only in words and draws the
CZ layouts for an 8x7 lattice):

* Rule 1: cycle 0 holds an H on every qubit.
* Rule 2: the depth d counts the CZ cycles after the H cycle; cycle
  t = 1..d uses CZ configuration ((t-1) mod 8) + 1.  The layouts of Fig. 4
  reduce to a closed form on row r (top to bottom) and column c:
  horizontal pair (r,c)-(r,c+1) is present iff (c + 2r) mod 4 equals the
  configuration's residue, vertical pair (r,c)-(r+1,c) iff (r + 2c) mod 4
  does.  Qubit q = r*ncols + c.
* Rule 3: at cycle t >= 2 a qubit receives a single-qubit gate iff it was
  in a CZ at cycle t-1 and is not in one at cycle t (3.A).  Its first such
  gate is T (3.B); later ones are drawn uniformly from {SX, SY, T},
  independently.  There is no final layer after cycle d.
* With ``rz=True`` every T becomes RZ with its own parameter index
  0, 1, 2, ... in the order the gates are written.
"""
from __future__ import annotations

import numpy as np

# configuration -> (orientation, residue); 'h' = horizontal, 'v' = vertical.
CZ_CONFIGS = {
    1: ("h", 2),
    2: ("h", 0),
    3: ("v", 3),
    4: ("v", 1),
    5: ("h", 3),
    6: ("h", 1),
    7: ("v", 0),
    8: ("v", 2),
}


def cz_pairs(config: int, nrows: int, ncols: int):
    """CZ qubit pairs (q0 < q1) of one configuration on an nrows x ncols grid."""
    orient, res = CZ_CONFIGS[config]
    pairs = []
    for r in range(nrows):
        for c in range(ncols):
            q = r * ncols + c
            if orient == "h" and c + 1 < ncols and (c + 2 * r) % 4 == res:
                pairs.append((q, q + 1))
            if orient == "v" and r + 1 < nrows and (r + 2 * c) % 4 == res:
                pairs.append((q, q + ncols))
    return sorted(pairs)


def generate_circuit(n: int, d: int, seed: int, rz: bool = False, m: int | None = None) -> str:
    """Text of one seeded Rules 1-3 circuit on an m x n grid (m defaults to n)."""
    nrows = n if m is None else m
    ncols = n
    nq = nrows * ncols
    rng = np.random.Generator(np.random.PCG64(seed))
    lines = [f"qubits {nq}", f"grid {nrows} {ncols}"]
    for q in range(nq):
        lines.append(f"0 H {q}")
    had_1q = [False] * nq
    prev_cz = set()
    n_param = 0
    for t in range(1, d + 1):
        pairs = cz_pairs((t - 1) % 8 + 1, nrows, ncols)
        in_cz = set()
        for a, b in pairs:
            in_cz.add(a)
            in_cz.add(b)
        gates = []
        for a, b in pairs:
            gates.append((a, f"{t} CZ {a} {b}"))
        if t >= 2:
            for q in range(nq):
                if q in prev_cz and q not in in_cz:
                    if not had_1q[q]:
                        g = "T"
                        had_1q[q] = True
                    else:
                        g = ("SX", "SY", "T")[int(rng.integers(0, 3))]
                    if g == "T" and rz:
                        gates.append((q, f"{t} RZ {q} {n_param}"))
                        n_param += 1
                    else:
                        gates.append((q, f"{t} {g} {q}"))
        gates.sort(key=lambda g: g[0])
        lines.extend(s for _, s in gates)
        prev_cz = in_cz
    return "\n".join(lines) + "\n"


def parse_header(text: str):
    """(n_qubits, n_params) from circuit text, without interpreting gates."""
    nq = None
    n_param = 0
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].split()
        if not line:
            continue
        if line[0] == "qubits":
            nq = int(line[1])
        elif len(line) >= 4 and line[1] == "RZ":
            n_param = max(n_param, int(line[3]) + 1)
    return nq, n_param


def random_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """(count, n_qubits) uint8 array of uniform 0/1 values from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2, size=(count, n_qubits), dtype=np.uint8)


def random_thetas(count: int, seed: int) -> np.ndarray:
    """count float64 angles, uniform on [0, 2*pi), from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 2.0 * np.pi, size=count)
