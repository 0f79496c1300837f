"""qgm: single amplitudes <x|C|0^N> by sliced variable elimination on MI355X.

Thin Python binding of the C-ABI in include/qgm.h.  The functions below have
the C names and only marshal arguments; every step of the computation runs
in libqgm.so (host planner/compiler in C++, contraction in HIP kernels).
PyTorch supplies device memory and the HIP stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import DECLARED, LIB_PATH, PlanOpts, QgmError, Stats, Tile, VarInfo, check, lib  # noqa: F401

QGM_C128 = 0
QGM_C64 = 1
QGM_BF16X3 = 2
QGM_ENGINE_AUTO = 0
QGM_ENGINE_INTERPRETER = 1
QGM_ENGINE_GENERATED = 2
QGM_ENGINE_WIDE = 3


def _i32(seq):
    arr = (C.c_int32 * max(1, len(seq)))(*[int(v) for v in seq])
    return arr


def qgm_circuit_parse(text: str) -> C.c_void_p:
    raw = text.encode()
    h = C.c_void_p()
    check(lib.qgm_circuit_parse(raw, len(raw), C.byref(h)))
    return h


def qgm_circuit_info(c):
    nq, nv, npar = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib.qgm_circuit_info(c, C.byref(nq), C.byref(nv), C.byref(npar)))
    return nq.value, nv.value, npar.value


def qgm_circuit_vars(c):
    _, nv, _ = qgm_circuit_info(c)
    buf = (VarInfo * max(1, nv))()
    check(lib.qgm_circuit_vars(c, buf, nv))
    return [(v.id, v.qubit, v.cycle_created, v.is_output) for v in buf[:nv]]


def qgm_circuit_graph(c):
    n = C.c_int32()
    check(lib.qgm_circuit_graph(c, None, 0, C.byref(n)))
    buf = (C.c_int32 * max(2, 2 * n.value))()
    check(lib.qgm_circuit_graph(c, buf, n.value, C.byref(n)))
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n.value)]


def qgm_circuit_free(c) -> None:
    lib.qgm_circuit_free(c)


QGM_PLAN_REORDER = 1
QGM_PLAN_BYTES = 2
QGM_PLAN_LATENCY = 4
QGM_PLAN_SEARCH = 8
QGM_PLAN_WIDE_TIME = 16
QGM_PLAN_CHOOSE_K = 32
QGM_PLAN_DETERMINISTIC = 64


def qgm_plan_slices(c, k_req: int = -1, target_rank: int = 0, time_budget_s: float = 1.0, seed: int = 0,
                    flags: int = 0):
    _, nv, _ = qgm_circuit_info(c)
    sl = (C.c_int32 * 40)()
    order = (C.c_int32 * max(1, nv))()
    k, n = C.c_int32(), C.c_int32()
    check(lib.qgm_plan_slices_ex(c, k_req, target_rank, float(time_budget_s), seed, flags, sl, C.byref(k), order,
                                 C.byref(n)))
    return list(sl[: k.value]), list(order[: n.value])


QGM_PLAN_BNB = 128


def qgm_order_search(c, sliced, init_order, max_nodes: int, beam: int = 0):
    """Branch and bound over orderings: (order, cost, width, complete)."""
    out = (C.c_int32 * max(1, len(init_order)))()
    cost, width, complete = C.c_double(), C.c_int32(), C.c_int32()
    check(lib.qgm_order_search(c, _i32(sliced), len(sliced), _i32(init_order), len(init_order), max_nodes, beam, out,
                               C.byref(cost), C.byref(width), C.byref(complete)))
    return list(out[:len(init_order)]), cost.value, width.value, bool(complete.value)


def qgm_sliced_order_for_groups(c, sliced, order):
    """The same sliced variables ordered for group sharing, and the fraction
    of the item work independent of those at slice bits 6 and 7."""
    out, frac = (C.c_int32 * max(1, len(sliced)))(), C.c_double()
    check(lib.qgm_sliced_order_for_groups(c, _i32(sliced), len(sliced), _i32(order), len(order), out,
                                          C.byref(frac)))
    return list(out[:len(sliced)]), frac.value


def qgm_order_cost(c, sliced, order):
    cost, width = C.c_double(), C.c_int32()
    check(lib.qgm_order_cost(c, _i32(sliced), len(sliced), _i32(order), len(order), C.byref(cost), C.byref(width)))
    return cost.value, width.value


def qgm_plan_create(c, sliced, order, prec: int = QGM_C128, workspace_cap: int = 0, profile: bool = False,
                    engine: int = QGM_ENGINE_AUTO, gradient: bool = False, waves: int = 0,
                    vector_only: bool = False, checkpoint_every: int = 0, persistent: bool = False,
                    deterministic: bool = False, tile_table_path: str | None = None, open_qubits=()):
    opts = PlanOpts()
    oq = _i32(open_qubits)
    opts.n_open = len(open_qubits)
    opts.open_qubits = C.cast(oq, C.POINTER(C.c_int32)) if len(open_qubits) else None
    opts.checkpoint_every = checkpoint_every
    opts.persistent = int(persistent)
    opts.deterministic = int(deterministic)
    opts.tile_table_path = None if tile_table_path is None else tile_table_path.encode()
    opts.prec = prec
    opts.profile = 1 if profile else 0
    opts.engine = engine
    opts.gradient = 1 if gradient else 0
    opts.waves = waves
    opts.vector_only = int(vector_only)
    opts.workspace_cap = workspace_cap
    h = C.c_void_p()
    check(lib.qgm_plan_create(c, _i32(sliced), len(sliced), _i32(order), len(order), C.byref(opts), C.byref(h)))
    return h


def qgm_plan_stats(p) -> dict:
    s = Stats()
    check(lib.qgm_plan_stats(p, C.byref(s)))
    return {name: getattr(s, name) for name, _ in Stats._fields_}


def qgm_workspace_size(p, n_bs: int, n_slices: int) -> int:
    out = C.c_size_t()
    check(lib.qgm_workspace_size(p, n_bs, n_slices, C.byref(out)))
    return out.value


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _host_inputs(bitstrings, params):
    bs = np.ascontiguousarray(np.atleast_2d(np.asarray(bitstrings, dtype=np.uint8)))
    par = None if params is None else np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    return bs, par


def _n_amp(p) -> int:
    return 1 << qgm_plan_stats(p)["n_open"]


def qgm_amplitudes(p, bitstrings, params, workspace, stream=None) -> np.ndarray:
    """Host arrays in, complex128 numpy array out (n_bs x 2^n_open entries,
    bitstring-major); workspace is a CUDA uint8 tensor."""
    bs, par = _host_inputs(bitstrings, params)
    out = np.empty(2 * bs.shape[0] * _n_amp(p), dtype=np.float64)
    check(lib.qgm_amplitudes(p, bs.ctypes.data_as(C.POINTER(C.c_uint8)), bs.shape[0],
                             None if par is None else par.ctypes.data_as(C.POINTER(C.c_double)),
                             _ptr(workspace), workspace.numel(), _stream(stream),
                             out.ctypes.data_as(C.POINTER(C.c_double))))
    return out[0::2] + 1j * out[1::2]


def qgm_amplitudes_range(p, bitstrings, params, s_begin: int, s_end: int, workspace, stream=None) -> np.ndarray:
    """(n_bs x 2^n_open, 4) float64: sum re, sum im, compensation re, compensation im."""
    bs, par = _host_inputs(bitstrings, params)
    out = np.empty(4 * bs.shape[0] * _n_amp(p), dtype=np.float64)
    check(lib.qgm_amplitudes_range(p, bs.ctypes.data_as(C.POINTER(C.c_uint8)), bs.shape[0],
                                   None if par is None else par.ctypes.data_as(C.POINTER(C.c_double)),
                                   s_begin, s_end, _ptr(workspace), workspace.numel(), _stream(stream),
                                   out.ctypes.data_as(C.POINTER(C.c_double))))
    return out.reshape(-1, 4)


def qgm_amplitudes_device(p, d_bits, d_params, s_begin: int, s_end: int, workspace, d_partial, stream=None) -> None:
    """All-device form: d_bits uint8 (n_bs, n_qubits), d_params float64, d_partial float64 (n_bs, 4)."""
    check(lib.qgm_amplitudes_device(p, _ptr(d_bits), d_bits.shape[0], _ptr(d_params), s_begin, s_end,
                                    _ptr(workspace), workspace.numel(), _stream(stream), _ptr(d_partial)))


QGM_NOALLOC_SCRATCH_BYTES = 64 << 20


def qgm_amplitudes_device_noalloc(p, d_bits, d_params, s_begin: int, s_end: int, d_partial, stream=None) -> None:
    """qgm_amplitudes_device with the library's fixed device workspace (no allocation)."""
    check(lib.qgm_amplitudes_device_noalloc(p, _ptr(d_bits), d_bits.shape[0], _ptr(d_params), s_begin, s_end,
                                            _stream(stream), _ptr(d_partial)))


def qgm_gradients_device(p, d_bits, d_params, s_begin: int, s_end: int, workspace, d_partial, d_grad_partial,
                         stream=None) -> None:
    """All-device amplitudes and d alpha / d theta: d_grad_partial float64 (n_bs, n_params, 4)."""
    check(lib.qgm_gradients_device(p, _ptr(d_bits), d_bits.shape[0], _ptr(d_params), s_begin, s_end,
                                   _ptr(workspace), workspace.numel(), _stream(stream), _ptr(d_partial),
                                   _ptr(d_grad_partial)))


def qgm_amplitude_grad(p, bitstring, params, workspace, n_params: int, stream=None):
    """(alpha, d alpha / d theta as a complex128 array) for one bitstring."""
    x = np.ascontiguousarray(np.asarray(bitstring, dtype=np.uint8))
    par = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    amp = np.empty(2, dtype=np.float64)
    grad = np.empty(max(1, 2 * n_params), dtype=np.float64)
    check(lib.qgm_amplitude_grad(p, x.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 par.ctypes.data_as(C.POINTER(C.c_double)), _ptr(workspace), workspace.numel(),
                                 _stream(stream), amp.ctypes.data_as(C.POINTER(C.c_double)),
                                 grad.ctypes.data_as(C.POINTER(C.c_double))))
    return complex(amp[0], amp[1]), grad[0:2 * n_params:2] + 1j * grad[1:2 * n_params:2]


def qgm_graph_create(p, d_bits, d_params, s_begin: int, s_end: int, workspace, d_partial, repeat: int = 1):
    """HIP graph of `repeat` runs of qgm_amplitudes_device with these device tensors."""
    g = C.c_void_p()
    check(lib.qgm_graph_create(p, _ptr(d_bits), d_bits.shape[0], _ptr(d_params), s_begin, s_end, _ptr(workspace),
                               workspace.numel(), _ptr(d_partial), repeat, C.byref(g)))
    return g


def qgm_graph_launch(g, stream=None) -> None:
    check(lib.qgm_graph_launch(g, _stream(stream)))


def qgm_graph_free(g) -> None:
    lib.qgm_graph_free(g)


def qgm_plan_timing(p, reset: bool = True):
    """(prologue ms, chain ms, reduction ms) averaged over the profiled runs, and the run count."""
    ms = (C.c_double * 3)()
    n = C.c_int32()
    check(lib.qgm_plan_timing(p, 1 if reset else 0, ms, C.byref(n)))
    return (ms[0], ms[1], ms[2]), n.value


def qgm_plan_level_timing(p, reset: bool = True):
    """Per level kernel of a WIDE plan: (ms, flops_item, mfma_steps) lists, the
    number of runs averaged, the items of the timed (first) pass, the
    bytes_item list and that pass's roofline seconds per item (work of steps
    shared between the pass's groups counted once per pass)."""
    nl, nr, it, roof = C.c_int32(), C.c_int32(), C.c_uint64(), C.c_double()
    check(lib.qgm_plan_level_timing(p, 0, None, None, None, None, 0, C.byref(nl), C.byref(nr), C.byref(it), None))
    n = nl.value
    ms = (C.c_double * max(1, n))()
    fl = (C.c_double * max(1, n))()
    by = (C.c_double * max(1, n))()
    mf = (C.c_int32 * max(1, n))()
    check(lib.qgm_plan_level_timing(p, 1 if reset else 0, ms, fl, by, mf, n, C.byref(nl), C.byref(nr),
                                    C.byref(it), C.byref(roof)))
    return list(ms[:n]), list(fl[:n]), list(mf[:n]), nr.value, it.value, list(by[:n]), roof.value


def qgm_plan_autotune(p, n_bs: int, n_slices: int, workspace, stream=None) -> int:
    """Time the generated kernel's wavefront cuts on the device; keeps the fastest. Returns the wave count."""
    w = C.c_int32()
    check(lib.qgm_plan_autotune(p, n_bs, n_slices, _ptr(workspace), workspace.numel(), _stream(stream), C.byref(w)))
    return w.value


def qgm_plan_free(p) -> None:
    lib.qgm_plan_free(p)


def qgm_last_error() -> str:
    m = lib.qgm_last_error()
    return m.decode() if m else ""


def qgm_amplitude(text: str, bitstring, sliced=(), order=None, params=None) -> complex:
    raw = text.encode()
    x = np.ascontiguousarray(np.asarray(bitstring, dtype=np.uint8))
    par = None if params is None else np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    out = (C.c_double * 2)()
    order = [] if order is None else order
    check(lib.qgm_amplitude(raw, len(raw), x.ctypes.data_as(C.POINTER(C.c_uint8)), _i32(sliced), len(sliced),
                            _i32(order), len(order),
                            None if par is None else par.ctypes.data_as(C.POINTER(C.c_double)), out))
    return complex(out[0], out[1])


def qgm_contraction_create(prec: int, nb: int, ni: int, nj: int, nk: int, vector_only: bool = False, tile=None):
    """tile: None or (per, lds_budget, jband, layout)."""
    h = C.c_void_p()
    t = None if tile is None else C.byref(Tile(*tile))
    check(lib.qgm_contraction_create(prec, nb, ni, nj, nk, 1 if vector_only else 0, t, C.byref(h)))
    return h


def qgm_plan_tune_tiles(p, table_path: str, stream=None) -> int:
    """Tune the matrix-core tiles of a WIDE plan on the device; writes the table. Returns the shapes tuned."""
    n = C.c_int32()
    check(lib.qgm_plan_tune_tiles(p, table_path.encode(), _stream(stream), C.byref(n)))
    return n.value


def qgm_contraction_info(h):
    """(runs on the matrix cores, elements per item, useful flops per item)."""
    mc, el, fl = C.c_int32(), C.c_uint64(), C.c_double()
    check(lib.qgm_contraction_info(h, C.byref(mc), C.byref(el), C.byref(fl)))
    return bool(mc.value), el.value, fl.value


def qgm_contraction_run(h, d_mem, n_groups: int, stream=None) -> None:
    check(lib.qgm_contraction_run(h, _ptr(d_mem), n_groups, _stream(stream)))


def qgm_contraction_free(h) -> None:
    lib.qgm_contraction_free(h)


class Contraction:
    """Owning wrapper of one two-operand contraction step (qgm_contraction_*)."""

    def __init__(self, prec: int, nb: int, ni: int, nj: int, nk: int, vector_only: bool = False, tile=None):
        self.prec, self.nb, self.ni, self.nj, self.nk = prec, nb, ni, nj, nk
        self.h = qgm_contraction_create(prec, nb, ni, nj, nk, vector_only, tile)
        self.matrix_cores, self.elems, self.flops = qgm_contraction_info(self.h)

    def run(self, d_mem, n_groups: int, stream=None) -> None:
        qgm_contraction_run(self.h, d_mem, n_groups, stream)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and lib is not None:
            try:
                lib.qgm_contraction_free(h)
            except Exception:  # interpreter shutdown
                pass


class Circuit:
    """Owning wrapper of a qgm_circuit handle."""

    def __init__(self, text: str):
        self.h = qgm_circuit_parse(text)
        self.n_qubits, self.n_vars, self.n_params = qgm_circuit_info(self.h)

    def vars(self):
        return qgm_circuit_vars(self.h)

    def graph(self):
        return qgm_circuit_graph(self.h)

    def plan_slices(self, k_req=-1, target_rank=0, time_budget_s=1.0, seed=0, flags=0):
        return qgm_plan_slices(self.h, k_req, target_rank, time_budget_s, seed, flags)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and lib is not None:
            try:
                lib.qgm_circuit_free(h)
            except Exception:  # interpreter shutdown
                pass


class Plan:
    """Owning wrapper of a qgm_plan handle plus a cached device workspace."""

    def __init__(self, circuit: Circuit, sliced, order, prec: int = QGM_C128, workspace_cap: int = 0,
                 profile: bool = False, engine: int = QGM_ENGINE_AUTO, gradient: bool = False, waves: int = 0,
                 vector_only: bool = False, checkpoint_every: int = 0, persistent: bool = False,
                 deterministic: bool = False, tile_table_path: str | None = None, open_qubits=()):
        self.circuit = circuit
        self.open_qubits = [int(x) for x in open_qubits]
        self.sliced = list(sliced)
        self.order = list(order)
        self.prec = prec
        self.gradient = gradient
        self.h = qgm_plan_create(circuit.h, self.sliced, self.order, prec, workspace_cap, profile, engine,
                                 gradient, waves, vector_only, checkpoint_every, persistent, deterministic,
                                 tile_table_path, self.open_qubits)
        self._ws = None

    @property
    def k(self):
        return len(self.sliced)

    def stats(self):
        return qgm_plan_stats(self.h)

    def workspace(self, n_bs: int, n_slices: int | None = None):
        import torch
        n_slices = (1 << self.k) if n_slices is None else n_slices
        need = qgm_workspace_size(self.h, n_bs, n_slices)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def release_workspace(self):
        """Drop the cached workspace (the next call allocates a new one)."""
        self._ws = None

    def amplitudes(self, bitstrings, params=None, stream=None):
        bs = np.atleast_2d(np.asarray(bitstrings, dtype=np.uint8))
        return qgm_amplitudes(self.h, bs, params, self.workspace(bs.shape[0]), stream)

    def amplitudes_range(self, bitstrings, params, s_begin, s_end, stream=None):
        bs = np.atleast_2d(np.asarray(bitstrings, dtype=np.uint8))
        ws = self.workspace(bs.shape[0], s_end - s_begin)
        return qgm_amplitudes_range(self.h, bs, params, s_begin, s_end, ws, stream)

    def autotune(self, n_bs: int, n_slices: int | None = None, stream=None) -> int:
        n_slices = (1 << self.k) if n_slices is None else n_slices
        return qgm_plan_autotune(self.h, n_bs, n_slices, self.workspace(n_bs, n_slices), stream)

    def amplitude_grad(self, bitstring, params, stream=None):
        """(alpha, d alpha / d theta) for one bitstring; needs gradient=True."""
        return qgm_amplitude_grad(self.h, bitstring, params, self.workspace(1), self.circuit.n_params, stream)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and lib is not None:
            try:
                lib.qgm_plan_free(h)
            except Exception:  # interpreter shutdown
                pass


def _amplitude_fn():
    import torch

    class AmplitudeFn(torch.autograd.Function):
        """alpha_x(theta) as a differentiable function of the RZ angles.

        forward(theta, plan, bitstring) -> complex128 scalar tensor.  The
        backward returns Re(conj(grad_out) * d alpha / d theta), PyTorch's
        convention for a real input and a complex output; d alpha / d theta
        comes from the library's reverse-mode pass run together with alpha.
        """

        @staticmethod
        def forward(ctx, theta, plan, bitstring):
            th = theta.detach().to("cpu", torch.float64).numpy()
            amp, grad = plan.amplitude_grad(bitstring, th)
            ctx.save_for_backward(torch.from_numpy(grad).to(theta.device))
            return torch.tensor(amp, dtype=torch.complex128, device=theta.device)

        @staticmethod
        def backward(ctx, grad_out):
            (grad,) = ctx.saved_tensors
            g = (grad_out.conj() * grad).real.to(torch.float64)
            return g, None, None

    return AmplitudeFn


def __getattr__(name):
    if name == "AmplitudeFn":
        return _amplitude_fn()
    raise AttributeError(name)
