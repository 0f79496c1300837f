"""One two-operand contraction step (qgm_contraction_*) against its FP64
product, element by element, with a rigorous first-order bound for each
precision.

For an output element c = sum_{k<K} a_k b_k (complex), the computed value
differs from the exact product of the stored operands by at most

    eps_prec * sum_k |a_k| |b_k|

because each real part sums 2K real products (|ar br| + |ai bi| <= |a||b|):
* complex128: eps = (2K + 2) 2^-53 (one rounding per multiply-add);
* complex64: eps = (2K + 2) 2^-24;
* complex64 in the three-multiplication form (per-item tiles, layout + 32:
  P1 = sum ar br, P2 = sum ai bi, P3 = sum (ar + ai)(br + bi), Re = P1 -
  P2, Im = P3 - (P1 + P2)): P1 and P2 err by (K + 1) u times their sums of
  |products|, P3 by (K + 3) u sum |ar + ai||br + bi| <= 2 (K + 3) u sum
  |a||b| (the two operand sums round once each), and P1 + P2 and the two
  subtractions add one rounding each, so to first order eps = (3K + 9)
  2^-24 (u = 2^-24, |ar br| + |ai bi| <= |a||b|);
* BF16x3: every real product x y becomes xh yh + xh yl + xl yh with
  x = xh + xl + dx, xh = bf16(x), xl = bf16(x - xh) (round to nearest even,
  8 significant bits): |x - xh| <= 2^-8 |x| and |dx| <= 2^-8 |x - xh| <=
  2^-16 |x|, so the dropped xl yl and the two split residuals cost at most
  3 * 2^-16 |x y| per product, plus the FP32 accumulation of complex64:
  eps = 3 * 2^-16 + (2K + 2) 2^-24.
A plain bfloat16 product (or a lost cross term xh yl) errs by about 2^-8 per
product, far above the BF16x3 bound for these sizes, so either mistake
fails here.
"""
import numpy as np
import pytest

import paper_1805_01450_amd as q

pytestmark = pytest.mark.gpu


def note(*args):
    print("[gpu-contract]", *args, flush=True)


def _eps(prec, K, three_m=False):
    if prec == q.QGM_C128:
        return (2 * K + 2) * 2.0 ** -53
    if prec == q.QGM_C64:
        return ((3 * K + 9) if three_m else (2 * K + 2)) * 2.0 ** -24
    return 3 * 2.0 ** -16 + (2 * K + 2) * 2.0 ** -24


def _run(prec, nb, ni, nj, nk, n_groups, vector_only, seed):
    import torch
    c = q.Contraction(prec, nb, ni, nj, nk, vector_only=vector_only)
    ea, eb = 1 << (nb + ni + nk), 1 << (nb + nk + nj)
    ec = 1 << (nb + ni + nj)
    assert c.elems == ea + eb + ec
    items = 64 * n_groups
    rng = np.random.default_rng(seed)
    cdt = np.complex128 if prec == q.QGM_C128 else np.complex64
    # A[item, b, k, i], B[item, b, j, k]: the element orders of the layout
    A = (rng.standard_normal((items, 1 << nb, 1 << nk, 1 << ni))
         + 1j * rng.standard_normal((items, 1 << nb, 1 << nk, 1 << ni))).astype(cdt)
    B = (rng.standard_normal((items, 1 << nb, 1 << nj, 1 << nk))
         + 1j * rng.standard_normal((items, 1 << nb, 1 << nj, 1 << nk))).astype(cdt)
    mem = np.zeros((n_groups, c.elems, 64), dtype=cdt)
    mem[:, :ea, :] = A.reshape(n_groups, 64, ea).transpose(0, 2, 1)
    mem[:, ea:ea + eb, :] = B.reshape(n_groups, 64, eb).transpose(0, 2, 1)
    tdt = torch.complex128 if prec == q.QGM_C128 else torch.complex64
    d_mem = torch.from_numpy(mem).to("cuda")
    assert d_mem.dtype == tdt and d_mem.is_contiguous()
    note("prec", prec, "nb ni nj nk", (nb, ni, nj, nk), "groups", n_groups, "vector_only", vector_only,
         "matrix cores", c.matrix_cores)
    c.run(d_mem, n_groups)
    torch.cuda.synchronize()
    got = d_mem.cpu().numpy()[:, ea + eb:, :].transpose(0, 2, 1).reshape(items, 1 << nb, 1 << nj, 1 << ni)
    # untouched operands
    assert np.array_equal(d_mem.cpu().numpy()[:, :ea + eb, :], mem[:, :ea + eb, :])
    A64, B64 = A.astype(np.complex128), B.astype(np.complex128)
    want = np.matmul(B64, A64)  # [item, b, j, i] = sum_k B[.., j, k] A[.., k, i]
    mag = np.matmul(np.abs(B64), np.abs(A64))
    return c, got, want, mag


SHAPES = [
    (2, 5, 5, 3),  # 2 x 2 wavefront tiles of one 16-item group
    (1, 4, 4, 1),  # 4 i and 4 j bits: four item groups per block
    (2, 5, 4, 2),  # 5 i bits, 4 j bits: wavefronts split i and items
    (2, 4, 5, 2),  # 4 i bits, 5 j bits: wavefronts split j and items
    (1, 6, 7, 8),  # K = 256, several tiles per item
    (0, 3, 3, 2),  # too narrow for the matrix cores: vector ALUs
    (1, 6, 6, 2),  # BF16x3 per item: 64 x 64 tiles, one K step
    (0, 7, 6, 5),  # two row tiles, eight K steps
    (2, 4, 6, 3),  # 16 x 64 tiles, eight complex k per stage
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [q.QGM_C64, q.QGM_BF16X3])
@pytest.mark.parametrize("vector_only", [False, True])
def test_contraction_within_bound(shape, prec, vector_only):
    nb, ni, nj, nk = shape
    c, got, want, mag = _run(prec, nb, ni, nj, nk, 2, vector_only, seed=hash(shape) % 1000)
    on_mc = not vector_only and ni >= 4 and nj >= 4 and nk >= 1
    assert c.matrix_cores == on_mc
    K = 1 << nk
    ratio = np.abs(got - want) / mag
    note("max |err| / sum|a||b|", ratio.max(), "bound", _eps(prec, K))
    assert np.all(np.isfinite(got))
    assert ratio.max() <= _eps(prec, K)
    if prec == q.QGM_BF16X3:
        # the split products are coarser than FP32 ones, and far finer than bf16
        assert ratio.max() > 2.0 ** -24
        assert ratio.max() < 2.0 ** -12


@pytest.mark.parametrize("shape", [(2, 5, 5, 3), (0, 3, 3, 2)])
def test_contraction_c128(shape):
    nb, ni, nj, nk = shape
    c, got, want, mag = _run(q.QGM_C128, nb, ni, nj, nk, 1, False, seed=5)
    assert not c.matrix_cores
    assert (np.abs(got - want) / mag).max() <= _eps(q.QGM_C128, 1 << nk)


def test_contraction_rejects_bad_shapes():
    with pytest.raises(q.QgmError) as e:
        q.Contraction(q.QGM_C64, 20, 10, 10, 1)
    assert e.value.status == -1
    with pytest.raises(q.QgmError) as e:
        q.Contraction(7, 1, 4, 4, 1)
    assert e.value.status == -7


TILES = [(1, 53248, 2, 0), (4, 53248, 2, 0), (2, 81920, 0, 0), (2, 114688, 3, 0), (4, 81920, 1, 1),
         (1, 53248, 2, 2), (4, 114688, 2, 3), (2, 53248, 3, 1),
         (1, 98304, 0, 4), (2, 49152, 0, 5), (1, 32768, 0, 6),
         (2, 131072, 0, 8), (1, 131072, 1, 8), (2, 98304, 0, 13),
         # the per-item form for either precision (complex64: FP32 16 x 16 x 4)
         (2, 65536, 0, 16), (1, 131072, 0, 24), (2, 98304, 0, 21),
         # complex64: the three-multiplication product in the per-item form
         (2, 65536, 0, 48), (1, 131072, 0, 56)]


def _per_item(prec, layout):
    if prec == q.QGM_BF16X3:
        return bool(layout & 16) or (layout & 7) in (0, 4, 5, 6)
    return bool(layout & 16)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("prec", [q.QGM_C64, q.QGM_BF16X3])
def test_tile_variants_match_builtin_tile(tile, prec):
    """Every tile parameter set keeps the k order of each output's sum, so the
    result equals the built-in tile's bit for bit (and meets the bound).
    Each precision has two families, the per-item forms (BF16x3 16 x 16 x
    32, built in for this K = 32 shape: layouts 0 and 4 to 6, or + 16;
    complex64 16 x 16 x 4: layouts + 16; + 8 for eight items per block) and
    the 16-item forms (layouts 1 to 3; complex64's built-in): across
    families the same terms are summed in another order and meet the
    bound."""
    import torch
    if prec == q.QGM_BF16X3 and tile[0] == 1 and tile[3] in (1, 2, 3):
        tile = (2,) + tile[1:]
    shape = (1, 6, 7, 5)
    c0, got0, want, mag = _run(prec, *shape, 2, False, seed=11)
    c1 = q.Contraction(prec, *shape, tile=tile)
    assert c1.matrix_cores
    # same operands through the variant
    nb, ni, nj, nk = shape
    ea, eb = 1 << (nb + ni + nk), 1 << (nb + nk + nj)
    cdt = np.complex64
    rng = np.random.default_rng(11)
    items = 128
    A = (rng.standard_normal((items, 1 << nb, 1 << nk, 1 << ni))
         + 1j * rng.standard_normal((items, 1 << nb, 1 << nk, 1 << ni))).astype(cdt)
    B = (rng.standard_normal((items, 1 << nb, 1 << nj, 1 << nk))
         + 1j * rng.standard_normal((items, 1 << nb, 1 << nj, 1 << nk))).astype(cdt)
    mem = np.zeros((2, c1.elems, 64), dtype=cdt)
    mem[:, :ea, :] = A.reshape(2, 64, ea).transpose(0, 2, 1)
    mem[:, ea:ea + eb, :] = B.reshape(2, 64, eb).transpose(0, 2, 1)
    d_mem = torch.from_numpy(mem).to("cuda")
    note("tile", tile, "prec", prec)
    c1.run(d_mem, 2)
    torch.cuda.synchronize()
    got1 = d_mem.cpu().numpy()[:, ea + eb:, :].transpose(0, 2, 1).reshape(items, 1 << nb, 1 << nj, 1 << ni)
    builtin_per_item = prec == q.QGM_BF16X3  # for this K = 32 shape
    if _per_item(prec, tile[3]) != builtin_per_item:
        three_m = prec == q.QGM_C64 and bool(tile[3] & 32)
        err = (np.abs(got1 - want) / mag).max()
        note("tile", tile, "max |err| / sum|a||b|", err, "bound", _eps(prec, 1 << nk, three_m))
        assert err <= _eps(prec, 1 << nk, three_m)
    else:
        assert np.array_equal(got1, got0)


def test_plan_tile_tuner_and_table(tmp_path):
    """qgm_plan_tune_tiles on the 7x7x30 plan writes a table; a plan created
    with it gives the default plan's amplitudes within the precision's
    bound: tiles of one form family keep the k order of every sum, but the
    tuner may pick the other family for a shape (the same products summed
    in another order)."""
    import json
    import os
    from workload import generate_circuit, random_bitstrings
    rec = json.load(open(os.path.join(os.path.dirname(q.__file__), "plans", "7x7x30.json")))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    bits = random_bitstrings(49, 2, 77)
    for prec in (q.QGM_C64, q.QGM_BF16X3):
        p = q.Plan(c, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE)
        table = str(tmp_path / "tiles.txt")
        n = q.qgm_plan_tune_tiles(p.h, table)
        note("tuned shapes", n, open(table).read())
        assert n >= 1
        t = q.Plan(c, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE, tile_table_path=table)
        got, want = t.amplitudes(bits), p.amplitudes(bits)
        tol = 2e-4 if prec == q.QGM_C64 else np.sqrt(p.stats()["n_steps"]) * 3 * 2.0 ** -16
        note("tuned against built-in tiles, max rel diff", np.max(np.abs(got - want) / np.abs(want)))
        assert np.max(np.abs(got - want) / np.abs(want)) <= tol
