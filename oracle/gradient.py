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


def ve_slice_gradients(circuit, x, params, sliced, order, s, which=None, net=None) -> np.ndarray:
    """d alpha_{x,s} / d theta_j of one slice s of the slicing ``sliced``.

    RZ(theta_j) puts the diagonal factor f(u) = e^{i theta_j (2u - 1)/2} on
    the variable u of its qubit, and df/dtheta_j = (i/2)(2u - 1) f(u).  Since
    alpha_s is linear in f, its derivative is the slice with u's sum split
    by value:
      u summed:           (i/2) (alpha_s|_{u=1} - alpha_s|_{u=0}),
      u fixed to b        (i/2) (2b - 1) alpha_s
    where alpha_s|_{u=b} fixes u to b on top of the slice (Section
    "Parallelization by fixing the values of variables": fixing adds no
    tensor).  u is fixed when it is an output (b = x_q), a sliced variable
    (b = its bit of s) or the input constant (b = 0).  Angles on one
    variable have equal derivatives.  Each split slice is evaluated once.
    """
    from .elimination import ve_slice_values
    from .network import INPUT, build_network

    params = np.asarray(params, dtype=np.float64)
    if net is None:
        net = build_network(circuit, params)
    which = range(len(params)) if which is None else which
    sliced = [int(v) for v in sliced]
    k = len(sliced)
    order = [int(v) for v in order]
    alpha_s = None
    split = {}
    out = []
    for j in which:
        u = net.param_var[int(j)]
        if u == INPUT or net.variables[u].is_output or u in sliced:
            if u == INPUT:
                b = 0
            elif u in sliced:
                b = (int(s) >> sliced.index(u)) & 1
            else:
                b = int(x[net.variables[u].qubit])
            if alpha_s is None:
                alpha_s = ve_slice_values(circuit, x, sliced, order, params, slices=[s], net=net)[0]
            out.append(0.5j * (2 * b - 1) * alpha_s)
            continue
        if u not in split:
            rest = [v for v in order if v != u]
            vals = ve_slice_values(circuit, x, sliced + [u], rest, params,
                                   slices=[int(s), int(s) | (1 << k)], net=net)
            split[u] = 0.5j * (vals[1] - vals[0])
        out.append(split[u])
    return np.array(out, dtype=np.complex128)
