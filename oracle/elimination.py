"""O2: variable elimination with slicing (Section "Our Algorithm").

To eliminate v: collect T_v (tensors containing v) and V_v (their
variables), multiply the tensors of T_v into sigma over V_v, sum sigma over
v, and put sigma' back in place of T_v.  Steps 2 and 3 are one
``numpy.einsum`` call, which pairs the small input tensors first (the
paper's note on einsum).  When every variable is eliminated the remaining
tensors are scalars whose product is the amplitude.

Slicing (Section "Parallelization by fixing the values of variables"):
fixing the k variables ``sliced`` to the bits of s in [0, 2^k) (bit j of s
is the value of ``sliced[j]``) gives 2^k independent sums whose total is the
amplitude.  The slice values are combined with ``math.fsum`` on real and
imaginary parts (exactly rounded).

The elimination order defaults to this module's own min-fill heuristic.
"""
from __future__ import annotations

import math

import numpy as np

from .graph import Graph
from .network import Network, build_network, project


def _graph_of(factors, vertices) -> Graph:
    g = Graph(vertices)
    for vs, _ in factors:
        for i in range(len(vs)):
            for j in range(i + 1, len(vs)):
                g.add_edge(vs[i], vs[j])
    return g


def min_fill_order(vertices, edges, seed_order=None) -> list:
    """Greedy min-fill ordering; ties broken by degree, then by vertex id."""
    g = Graph(vertices, edges)
    order = []
    while g.adj:
        v = min(g.adj, key=lambda u: (g.fill_in(u), g.degree(u), u))
        order.append(v)
        g.eliminate(v)
    return order


def order_cost(vertices, edges, order):
    """(sum over steps of 2^deg(v), max deg) of eliminating in ``order``."""
    g = Graph(vertices, edges)
    total = 0
    width = 0
    for v in order:
        d = g.eliminate(v)
        total += 1 << d
        width = max(width, d)
    return total, width


def _eliminate_all(factors, order):
    tensors = list(factors)
    letters = {}
    for v in order:
        tv = [t for t in tensors if v in t[0]]
        rest = [t for t in tensors if v not in t[0]]
        if not tv:
            # no tensor mentions v: the sum over v of 1 is 2
            rest.append(((), np.array(2.0 + 0.0j)))
            tensors = rest
            continue
        vv = []
        for vs, _ in tv:
            for u in vs:
                if u not in vv:
                    vv.append(u)
        out_vars = tuple(u for u in vv if u != v)
        letters = {u: i for i, u in enumerate(vv)}
        args = []
        for vs, t in tv:
            args.append(t)
            args.append([letters[u] for u in vs])
        args.append([letters[u] for u in out_vars])
        sigma_p = np.einsum(*args, optimize="greedy")
        rest.append((out_vars, np.asarray(sigma_p, dtype=np.complex128)))
        tensors = rest
    value = 1.0 + 0.0j
    for vs, t in tensors:
        if len(vs) != 0:
            raise ValueError(f"variables {vs} were never eliminated")
        value *= complex(t)
    return value


def _check_order(net: Network, sliced, order):
    free = set(net.free_vars) - set(sliced)
    if sorted(order) != sorted(free):
        raise ValueError("order must list every free, non-sliced variable once")


def ve_slice_values(circuit, x, sliced=(), order=None, params=None, slices=None, net=None):
    """alpha_{x,s} for each slice s (default: all 2^k in ascending order)."""
    if net is None:
        net = build_network(circuit, params)
    sliced = [int(v) for v in sliced]
    free = [v for v in net.free_vars if v not in set(sliced)]
    if order is None:
        base, _ = project(net, x)
        g = _graph_of(base, net.free_vars)
        for v in sliced:
            g.fix(v)
        order = min_fill_order(sorted(free), g.edges)
    _check_order(net, sliced, order)
    k = len(sliced)
    if slices is None:
        slices = range(1 << k)
    vals = []
    for s in slices:
        fix = {sliced[j]: (int(s) >> j) & 1 for j in range(k)}
        factors, scalar = project(net, x, fix)
        if scalar == 0:
            vals.append(0j)
            continue
        vals.append(scalar * _eliminate_all(factors, order))
    return np.array(vals, dtype=np.complex128)


def exact_sum(values) -> complex:
    return complex(math.fsum(v.real for v in values), math.fsum(v.imag for v in values))


def ve_amplitude(circuit, x, sliced=(), order=None, params=None, net=None) -> complex:
    """alpha_x = sum over all 2^k slices, combined exactly (fsum)."""
    return exact_sum(ve_slice_values(circuit, x, sliced, order, params, net=net))


def greedy_extra_slices(vertices, edges, order, j, n_candidates=40):
    """Fix j more vertices, one at a time, each the one whose removal gives
    the least cost sum 2^deg(v) of eliminating the rest of ``order`` (the
    paper's greedy key-vertex removal under a fixed ordering, Section "The
    variable elimination ordering").  Candidates at each pick are the
    ``n_candidates`` vertices of largest degree at their elimination; ties
    go to the smaller vertex id.  Returns (picked, remaining order, cost,
    width)."""
    picked = []
    rest = [int(v) for v in order]
    live = set(int(v) for v in vertices)
    edges = [(int(a), int(b)) for a, b in edges]
    for _ in range(j):
        g = Graph(sorted(live), [(a, b) for a, b in edges if a in live and b in live])
        deg = {}
        for v in rest:
            deg[v] = g.eliminate(v)
        cands = sorted(rest, key=lambda v: (-deg[v], v))[:n_candidates]
        best = None
        for c in cands:
            live_c = live - {c}
            cost, width = order_cost(sorted(live_c), [(a, b) for a, b in edges if a in live_c and b in live_c],
                                     [v for v in rest if v != c])
            if best is None or (cost, width, c) < best:
                best = (cost, width, c)
        picked.append(best[2])
        live.discard(best[2])
        rest = [v for v in rest if v != best[2]]
    live_edges = [(a, b) for a, b in edges if a in live and b in live]
    cost, width = order_cost(sorted(live), live_edges, rest)
    return picked, rest, cost, width
