"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only generates inputs (circuit text, output bitstrings, Rz
angles).  It contains none of the amplitude arithmetic: no gate matrices, no
graphical model and no contraction.
"""
from .circuits import (  # noqa: F401
    CZ_CONFIGS,
    cz_pairs,
    generate_circuit,
    random_bitstrings,
    random_thetas,
    parse_header,
)
