"""Gradients of alpha with respect to RZ angles.

RZ(theta) = diag(e^{-i theta/2}, e^{i theta/2}) satisfies
d RZ / d theta = (1/2) RZ(theta + pi); alpha is linear in each gate matrix
and each angle belongs to one gate, so d alpha / d theta_j =
(1/2) alpha(theta + pi e_j) exactly (parameter-shift identity).
"""
from __future__ import annotations

import numpy as np

from .statevector import sv_amplitudes


def sv_gradient_shift(circuit, x, params, which=None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    which = range(len(params)) if which is None else which
    out = []
    for j in which:
        p = params.copy()
        p[j] += np.pi
        out.append(0.5 * sv_amplitudes(circuit, [x], p)[0])
    return np.array(out, dtype=np.complex128)


def fd_gradient(amp_fn, params, h=1e-4, which=None) -> np.ndarray:
    """Central finite differences of amp_fn(params) -> complex."""
    params = np.asarray(params, dtype=np.float64)
    which = range(len(params)) if which is None else which
    out = []
    for j in which:
        p = params.copy()
        p[j] += h
        fp = amp_fn(p)
        p[j] -= 2 * h
        fm = amp_fn(p)
        out.append((fp - fm) / (2 * h))
    return np.array(out, dtype=np.complex128)
