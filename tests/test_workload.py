"""Pins of the seeded Rules 1-3 generator against the paper.

* CZ layouts: the closed form must reproduce every pair drawn in the CZ
  layout figure (Fig. 4, 8x7 lattice, configurations 1-8).
* Gate counts: the paper's g_2 estimate is exact when 8 divides d, and its
  g_1 estimate is exact for even n when 8 divides d (Section "Application to
  Random Circuit Sampling").
* Rule 3 placement and the forced first T.
"""
import numpy as np
import pytest

from tests.conftest import golden_path
from workload import cz_pairs, generate_circuit, random_bitstrings, random_thetas, parse_header


def load_fig4():
    cfg = {c: set() for c in range(1, 9)}
    with open(golden_path("fig4_cz_layouts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c, a, b = map(int, line.split())
            cfg[c].add((min(a, b), max(a, b)))
    return cfg


def test_fig4_layouts_match_closed_form():
    drawn = load_fig4()
    assert sum(len(v) for v in drawn.values()) == 97
    for c in range(1, 9):
        # label L = 7 r + c + 1 -> qubit q = 7 r + c on an 8 x 7 grid
        ours = {(a + 1, b + 1) for a, b in cz_pairs(c, 8, 7)}
        assert ours == drawn[c], f"configuration {c}"


def test_every_lattice_edge_once_per_8_cycles():
    for nr, nc in [(8, 7), (5, 5), (6, 6), (4, 4)]:
        seen = []
        for c in range(1, 9):
            seen.extend(cz_pairs(c, nr, nc))
        assert len(seen) == len(set(seen)) == nr * (nc - 1) + (nr - 1) * nc


def _gates(text):
    out = []
    for line in text.splitlines()[2:]:
        t = line.split()
        out.append((int(t[0]), t[1], tuple(int(v) for v in t[2:])))
    return out


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8, 9, 10])
@pytest.mark.parametrize("d", [8, 16, 24, 40])
def test_gate_count_formulas(n, d):
    g = _gates(generate_circuit(n, d, seed=1))
    g2 = sum(1 for _, name, _ in g if name == "CZ")
    g1 = sum(1 for _, name, _ in g if name in ("T", "SX", "SY"))
    assert g2 == d // 8 * (2 * n * (n - 1))
    N = n * n
    if n % 2 == 0:
        assert g1 == d // 8 * (3 * N - (2 * n + 1)) - N // 4


def test_rule3_placement_and_first_t():
    n, d = 5, 20
    g = _gates(generate_circuit(n, d, seed=3))
    in_cz = {t: set() for t in range(d + 1)}
    one_q = {}
    for t, name, qs in g:
        if name == "CZ":
            in_cz[t].update(qs)
        elif name != "H":
            one_q[(t, qs[0])] = name
    seen = set()
    for t in range(1, d + 1):
        for q in range(n * n):
            expect = t >= 2 and q in in_cz[t - 1] and q not in in_cz[t]
            assert ((t, q) in one_q) == expect
            if (t, q) in one_q:
                if q not in seen:
                    assert one_q[(t, q)] == "T"
                seen.add(q)


def test_rz_variant_and_seeds():
    a = generate_circuit(4, 10, seed=7)
    b = generate_circuit(4, 10, seed=7, rz=True)
    na = sum(1 for _, name, _ in _gates(a) if name == "T")
    nq, npar = parse_header(b)
    assert nq == 16 and npar == na
    assert "T" not in {name for _, name, _ in _gates(b)}
    assert generate_circuit(5, 20, 0) == generate_circuit(5, 20, 0)
    assert generate_circuit(5, 20, 0) != generate_circuit(5, 20, 1)
    bs = random_bitstrings(25, 64, 1000)
    assert bs.shape == (64, 25) and set(np.unique(bs)) <= {0, 1}
    th = random_thetas(10, 2000)
    assert np.all((th >= 0) & (th < 2 * np.pi))
