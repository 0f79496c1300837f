"""qgm_amplitudes_device_noalloc (fixed device workspace, no allocation)
against qgm_amplitudes_device on the same inputs: the same kernels in the
same order, so the partial sums are bit-identical.  Two calls in a row, the
second with a smaller batch, for each engine that small plans use; a batch
whose workspace exceeds the fixed array is refused before any device work.
"""
import numpy as np
import pytest

import paper_1805_01450_amd as q
from workload import generate_circuit, random_bitstrings

pytestmark = pytest.mark.gpu


def note(*args):
    print("[gpu-noalloc]", *args, flush=True)


@pytest.mark.parametrize("engine,prec", [(q.QGM_ENGINE_GENERATED, q.QGM_C64), (q.QGM_ENGINE_GENERATED, q.QGM_C128),
                                         (q.QGM_ENGINE_INTERPRETER, q.QGM_C64), (q.QGM_ENGINE_WIDE, q.QGM_C64)])
def test_noalloc_matches_device_entry(engine, prec):
    import torch
    text = generate_circuit(5, 20, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.5, flags=q.QGM_PLAN_DETERMINISTIC)
    p = q.Plan(c, sl, order, prec=prec, engine=engine)
    assert p.stats()["engine"] == engine
    bits = random_bitstrings(25, 64, 1000)
    for n_bs, s0, s1 in ((64, 0, 64), (16, 5, 37)):
        d_bits = torch.from_numpy(bits[:n_bs]).cuda()
        want = torch.full((n_bs, 4), float("nan"), dtype=torch.float64, device="cuda")
        got = torch.full((n_bs, 4), float("nan"), dtype=torch.float64, device="cuda")
        ws = p.workspace(n_bs, s1 - s0)  # uploads the plan's tables to the device
        assert ws.numel() <= q.QGM_NOALLOC_SCRATCH_BYTES
        note("engine", engine, "prec", prec, "bitstrings", n_bs, "slices", s0, s1)
        q.qgm_amplitudes_device(p.h, d_bits, None, s0, s1, ws, want)
        q.qgm_amplitudes_device_noalloc(p.h, d_bits, None, s0, s1, got)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())
        assert np.all(np.isfinite(got.cpu().numpy()))


def test_noalloc_refuses_oversize_and_unloaded_plans():
    import torch
    text = generate_circuit(5, 20, 0)
    c = q.Circuit(text)
    sl, order = c.plan_slices(k_req=6, time_budget_s=0.5, flags=q.QGM_PLAN_DETERMINISTIC)
    p = q.Plan(c, sl, order, prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED)
    bits = torch.from_numpy(random_bitstrings(25, 4, 1000)).cuda()
    part = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QgmError) as e:  # tables not uploaded yet
        q.qgm_amplitudes_device_noalloc(p.h, bits, None, 0, 64, part)
    assert e.value.status == -1
    # 2^20 items per bitstring x 64 bitstrings: the per-item results alone
    # exceed the fixed array
    wide = q.Plan(c, sl + [v for v in order[:14]], order[14:], prec=q.QGM_C64, engine=q.QGM_ENGINE_GENERATED)
    big = torch.from_numpy(random_bitstrings(25, 64, 1001)).cuda()
    part = torch.empty((64, 4), dtype=torch.float64, device="cuda")
    need = q.qgm_workspace_size(wide.h, 64, 1 << 20)
    assert need > q.QGM_NOALLOC_SCRATCH_BYTES
    with pytest.raises(q.QgmError) as e:
        q.qgm_amplitudes_device_noalloc(wide.h, big, None, 0, 1 << 20, part)
    assert e.value.status == -5
