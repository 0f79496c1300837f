"""O3: brute-force sum over all 0/1 labellings of the graphical model.

Each term of the Feynman sum corresponds to one labelling of the free
vertices; its value is the product of all factor values at that labelling
(Section "Undirected Graphical Model").  Exponential in the number of free
variables; used for small circuits only.
"""
from __future__ import annotations

import numpy as np

from .network import build_network, project


def brute_amplitude(circuit, x, params=None, max_vars: int = 24) -> complex:
    net = build_network(circuit, params)
    factors, scalar = project(net, x)
    free = sorted({v for vs, _ in factors for v in vs})
    nv = len(free)
    if nv > max_vars:
        raise ValueError(f"{nv} free variables is too many for brute force")
    pos = {v: i for i, v in enumerate(free)}
    total = 0.0 + 0.0j
    chunk = 1 << min(nv, 16)
    for start in range(0, 1 << nv, chunk):
        lab = np.arange(start, min(start + chunk, 1 << nv), dtype=np.int64)
        term = np.full(lab.shape, scalar, dtype=np.complex128)
        for vs, t in factors:
            idx = tuple((lab >> pos[v]) & 1 for v in vs)
            term *= t[idx]
        total += term.sum()
    return complex(total)
