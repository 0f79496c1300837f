"""FP64 CPU oracle for single output amplitudes <x|C|0^N> of grid circuits.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the package
entry and the CPU-baseline leg of the benchmark may import this package.
It shares no code with the GPU library: it has its own circuit parser, its
own gate tables, its own graphical-model builder and its own contraction.

Three independent ways to the same number (the method is exact; slicing,
ordering and contraction tree change cost and rounding only):

* ``statevector``  -- the plain definition, Eq. (1): apply C_1 ... C_d to
  |0...0> and read entry x.
* ``elimination``  -- variable elimination on the undirected graphical
  model (Section "Variable elimination"), one ``numpy.einsum`` per
  eliminated variable, with slicing by fixed variables (Section
  "Parallelization by fixing the values of variables") summed exactly.
* ``brute``        -- the sum over all 0/1 labellings of the graphical
  model's free vertices (Section "Undirected Graphical Model").

Every function is pinned by the CPU tests (worked example of Figs. 2/3/5/6,
closed forms, invariants, cross-checks between the three routes).
"""
from .circuit import Circuit, parse_circuit  # noqa: F401
from .gates import gate_matrix  # noqa: F401
from .statevector import sv_amplitudes, sv_state  # noqa: F401
from .network import Network, build_network  # noqa: F401
from .graph import Graph  # noqa: F401
from .elimination import (  # noqa: F401
    ve_amplitude,
    ve_slice_values,
    min_fill_order,
    order_cost,
)
from .brute import brute_amplitude  # noqa: F401
from .gradient import sv_gradient_shift, fd_gradient  # noqa: F401
