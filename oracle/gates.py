"""Gate matrices in FP64 (the paper names the gates but prints no matrix).

Readings (gates named in Fig. 2 and in Rule 3):
* H  = (1/sqrt 2) [[1, 1], [1, -1]]
* SX = principal square root of X = 1/2 [[1+i, 1-i], [1-i, 1+i]]
* SY = principal square root of Y = 1/2 [[1+i, -1-i], [1+i, 1+i]]
* T  = diag(1, e^{i pi/4});  I = identity;  CZ = diag(1, 1, 1, -1)
* RZ(theta) = exp(-i theta Z / 2) = diag(e^{-i theta/2}, e^{i theta/2})
Matrices are indexed [out, in].

Two-qubit non-diagonal gates (the "arbitrary circuit" gadget: a gate that is
not diagonal creates a new variable on both of its qubits, Fig.
"tensornodes"), 4 x 4 with index bit(q0) + 2 bit(q1), [out, in]:
* CX: control q0, target q1, |c t> -> |c, t xor c>
* ISWAP: |01> -> i|10>, |10> -> i|01>, |00> and |11> unchanged
* SQISW: the square root of ISWAP with the 2 x 2 block
  (1/sqrt 2)[[1, i], [i, 1]] on {|01>, |10>}
"""
from __future__ import annotations

import numpy as np

DIAGONAL = {"T", "RZ", "I", "CZ"}
TWO_QUBIT_NONDIAG = {"CX", "ISWAP", "SQISW"}


def gate_matrix(name: str, theta: float | None = None) -> np.ndarray:
    if name == "H":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    if name == "SX":
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
    if name == "SY":
        return 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)
    if name == "T":
        return np.diag([1.0, np.exp(1j * np.pi / 4)]).astype(np.complex128)
    if name == "I":
        return np.eye(2, dtype=np.complex128)
    if name == "RZ":
        return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)
    if name == "CZ":
        return np.diag([1.0, 1.0, 1.0, -1.0]).astype(np.complex128)
    if name == "CX":
        u = np.zeros((4, 4), dtype=np.complex128)
        for c in (0, 1):
            for t in (0, 1):
                u[c + 2 * (t ^ c), c + 2 * t] = 1.0
        return u
    if name == "ISWAP":
        u = np.eye(4, dtype=np.complex128)
        u[1, 1] = u[2, 2] = 0.0
        u[2, 1] = u[1, 2] = 1j
        return u
    if name == "SQISW":
        r = 1.0 / np.sqrt(2.0)
        u = np.eye(4, dtype=np.complex128)
        u[1, 1] = u[2, 2] = r
        u[2, 1] = u[1, 2] = 1j * r
        return u
    raise ValueError(name)


def diagonal_entries(name: str, theta: float | None = None) -> np.ndarray:
    """Diagonal of a one-qubit diagonal gate (T, RZ, I)."""
    return np.diag(gate_matrix(name, theta)).copy()
