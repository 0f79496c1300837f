"""O1: state-vector evaluation of Eq. (1), the plain definition.

psi <- |0...0>; apply every gate of C_1, ..., C_d in order; alpha_x is the
entry of psi at index sum_q x_q 2^q (qubit q is bit q of the index).
"""
from __future__ import annotations

import numpy as np

from .circuit import Circuit, parse_circuit
from .gates import TWO_QUBIT_NONDIAG, gate_matrix


def _apply_1q(psi: np.ndarray, n: int, q: int, u: np.ndarray) -> np.ndarray:
    v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    out = np.empty_like(v)
    a0 = v[:, 0, :]
    a1 = v[:, 1, :]
    out[:, 0, :] = u[0, 0] * a0 + u[0, 1] * a1
    out[:, 1, :] = u[1, 0] * a0 + u[1, 1] * a1
    return out.reshape(-1)


def _apply_diag(psi: np.ndarray, n: int, q: int, d: np.ndarray) -> None:
    v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    if d[0] != 1.0:
        v[:, 0, :] *= d[0]
    if d[1] != 1.0:
        v[:, 1, :] *= d[1]


def _apply_cz(psi: np.ndarray, n: int, a: int, b: int) -> None:
    lo, hi = min(a, b), max(a, b)
    v = psi.reshape(1 << (n - hi - 1), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    v[:, 1, :, 1, :] *= -1.0


def _apply_2q(psi: np.ndarray, n: int, a: int, b: int, u: np.ndarray) -> np.ndarray:
    """u is 4 x 4 over index bit(a) + 2 bit(b), [out, in]."""
    t = psi.reshape([2] * n)  # axis n - 1 - q is qubit q
    ax_a, ax_b = n - 1 - a, n - 1 - b
    t = np.moveaxis(t, (ax_a, ax_b), (-2, -1))  # [..., bit a, bit b]
    shp = t.shape
    v = t.reshape(-1, 2, 2)
    # flat index bit(a) + 2 bit(b) -> [bit b][bit a]
    u4 = u.reshape(2, 2, 2, 2)  # [out b, out a, in b, in a]
    w = np.einsum("yxvu,nuv->nxy", u4, v)  # v[n, a, b]; result [n, out a, out b]
    t = w.reshape(shp)
    t = np.moveaxis(t, (-2, -1), (ax_a, ax_b))
    return np.ascontiguousarray(t).reshape(-1)


def sv_state(circuit, params=None) -> np.ndarray:
    """Full output state C|0...0> as a complex128 vector of length 2^N."""
    c = parse_circuit(circuit) if isinstance(circuit, str) else circuit
    assert isinstance(c, Circuit)
    n = c.n_qubits
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for g in c.gates:
        if g.name == "CZ":
            _apply_cz(psi, n, g.qubits[0], g.qubits[1])
        elif g.name in TWO_QUBIT_NONDIAG:
            psi = _apply_2q(psi, n, g.qubits[0], g.qubits[1], gate_matrix(g.name))
        elif g.name in ("T", "I", "RZ"):
            theta = None if g.param < 0 else float(params[g.param])
            m = gate_matrix(g.name, theta)
            _apply_diag(psi, n, g.qubits[0], np.diag(m))
        else:
            psi = _apply_1q(psi, n, g.qubits[0], gate_matrix(g.name))
    return psi


def bit_index(bits) -> int:
    return int(sum(int(b) << q for q, b in enumerate(bits)))


def sv_amplitudes(circuit, bitstrings, params=None) -> np.ndarray:
    """alpha_x for each row x of ``bitstrings`` (shape (B, N), entries 0/1)."""
    psi = sv_state(circuit, params)
    bs = np.atleast_2d(np.asarray(bitstrings))
    return np.array([psi[bit_index(x)] for x in bs], dtype=np.complex128)
