"""Host-side model of the generated matrix-core steps (no GPU).

The wide engine emits each matrix-core step as straight-line HIP whose index
arithmetic is fixed at plan time.  This test evaluates that arithmetic for
every block and thread of every matrix-core step of the stored 7x7x30 plan
(complex64 and BF16x3), of blocks at both ends of every matrix-core step of
the benchmark's 8x8x40 plan, and of single contractions that take each of the
four block shapes, and replays the LDS ring in program order:
  - every HBM copy stays inside the group's item memory and every LDS copy
    target and operand read inside the kernel's LDS array;
  - every operand read finds a slot written by a copy of the same unit,
    holding the item the lane owns (lane l: item 16 wq + l / 4);
  - over the K loop each operand lane reads each summed row exactly once;
  - the result stores cover distinct elements.
The barrier protocol itself (which copies a wave may issue after which wait)
is exercised on the device by the parity tests."""
import glob
import json
import os
import re

import numpy as np
import pytest

import paper_1805_01450_amd as q
from workload import generate_circuit


def _py_expr(e):
    """A C integer expression of the generated code as a numpy expression."""
    for cast in ("(long long)", "(int)", "(unsigned long long)", "(unsigned)"):
        e = e.replace(cast, "")
    e = re.sub(r"(\d+)ull", r"\1", e)
    e = re.sub(r"(\d+)ll", r"\1", e)
    e = re.sub(r"(\d+)u\b", r"\1", e)
    e = e.replace("/", "//")
    while True:  # "(name ? a : b)" with nested parentheses
        m = re.search(r"\((\w+) \? ", e)
        if not m:
            break
        i, depth, j, colon = m.start(), 0, m.start(), None
        while True:
            if e[j] == "(":
                depth += 1
            elif e[j] == ")":
                depth -= 1
                if depth == 0:
                    break
            elif e.startswith(" : ", j) and depth == 1 and colon is None:
                colon = j
            j += 1
        e = e[:i] + f"np.where({m.group(1)}, {e[m.end():colon]}, {e[colon + 3:j]})" + e[j + 1:]
    if " ? " in e:
        c, rest = e.split(" ? ", 1)
        a, b = rest.rsplit(" : ", 1)
        e = f"np.where({c}, {a}, {b})"
    return e.replace("threadIdx.x", "threadIdx_x")


# (the A rows of a step come from operand 0's base gq0, the B rows from gq1)
COPY = re.compile(r"__builtin_amdgcn_global_load_lds\(\(const void\*\)\(\(isa(\d+) \? gq0 : gq1\) \+ e \* 64ll \+ itb \+ "
                  r"2 \* pq\1\), "
                  r"\(__attribute__\(\(address_space\(3\)\)\) void\*\)\(lds \+ \((.*?)\) \* (\d+) \+ lds(\d+)\), 16, 0, 0\);")
E_LINE = re.compile(r"const (?:long long|unsigned) e = (.*);$")


def check_step(body, S, E, lds_size, group_c2, max_blocks=None):
    """max_blocks: evaluate only the first and last max_blocks / 2 blocks of
    the step's range (large steps)."""
    lines = [l.strip() for l in body.split("\n")]
    blocks = np.arange(S, E, dtype=np.int64)
    if max_blocks is not None and E - S > max_blocks:
        blocks = np.concatenate([blocks[:max_blocks // 2], blocks[-(max_blocks // 2):]])
    blk = np.repeat(blocks, 256)
    th = np.tile(np.arange(256, dtype=np.int64), len(blocks))
    env = {"np": np, "blk": blk, "threadIdx_x": th, "wv": th >> 6}

    def ev(e):
        return np.asarray(eval(_py_expr(e), env))

    i_loop = next(i for i, l in enumerate(lines) if l.startswith("for (int u = 0;"))
    for l in lines[:i_loop]:  # per-thread set-up values
        m = re.match(r"const (?:unsigned long long|long long|unsigned|int|bool) (.*);$", l)
        if m and not E_LINE.match(l):
            for part in re.split(r", (?=[a-z]\w* = )", m.group(1)):
                name, e = part.split(" = ", 1)
                env[name.strip()] = ev(e)
    nu = int(re.search(r"for \(int u = 0; u < (\d+); \+\+u\)", body).group(1))
    m = re.search(r"const char\* sb = lds \+ \(u % (\d+)\) \* (\d+);", body)
    P, stage = int(m.group(1)), int(m.group(2))
    ring = {}

    def copy(line, e_expr, st, unit):
        m = COPY.match(line)
        g = ev(e_expr) * 64 + env["itb"] + 2 * env["pq" + m.group(1)]
        lo = st * int(m.group(3)) + env["lds" + m.group(4)] + 16 * env["lid"]
        assert lo.min() >= 0 and lo.max() + 16 <= lds_size
        assert g.min() >= 0 and g.max() + 1 < group_c2
        ring.setdefault(st, []).append((unit, g, lo))

    e_expr = None
    for l in lines[:i_loop]:  # prologue copies: literal unit and stage
        if E_LINE.match(l):
            e_expr = E_LINE.match(l).group(1)
        m = COPY.match(l)
        if m:
            mu = re.search(r"\(\(\((\d+)\)\) >> 0\)|\(\(\(\d \* \((\d+)\) \+ h\d+\)\) >> 0\)", e_expr)
            env["u"] = 0
            copy(l, e_expr, int(m.group(2)), int(mu.group(1) or mu.group(2)))
    loop = lines[i_loop:]
    copies = [l for l in loop if E_LINE.match(l) or l.startswith("__builtin_amdgcn_global_load_lds")]
    reads = [l for l in loop if re.match(r"const C2 [ab]\d_\d = ", l)]
    rows = {}
    for u in range(nu):
        env["u"] = u
        env["un"] = min(u + P - 1, nu - 1)
        st = u % P
        slot = {}
        for (un, g, lo) in ring.get(st, []):
            if un == u:
                for c in range(2):
                    slot.update(zip(zip(blk.tolist(), (lo + 8 * c).tolist()), (g + c).tolist()))
        want_item = env["itb"] + 16 * env["wq"] + (env["lid"] >> 2)
        for l in reads:
            m = re.match(r"const C2 ([ab])\d_(\d) = \*\(const C2\*\)\(sb \+ (.*)\);$", l)
            off = ev(m.group(3)) + st * stage
            assert off.min() >= 0 and off.max() + 8 <= lds_size
            got = np.array([slot.get(k, -1) for k in zip(blk.tolist(), off.tolist())])
            assert (got >= 0).all(), "operand read of a slot this unit did not fill"
            assert ((got % 64) == want_item).all(), "operand read of another item"
            rows.setdefault((m.group(1), m.group(2)), []).append(got // 64)
        st2 = (u + P - 1) % P
        ring[st2] = []
        for l in copies:
            if E_LINE.match(l):
                e_expr = E_LINE.match(l).group(1)
            else:
                copy(l, e_expr, st2, env["un"])
    for r in rows.values():
        r = np.stack(r, 0)
        assert all(len(np.unique(r[:, c])) == r.shape[0] for c in range(0, r.shape[1], 61)), \
            "a summed row read twice or not at all"
    st_lines = [l for l in lines if l.startswith("gm[(lo + ")]
    stores = np.concatenate([ev(re.match(r"gm\[\((lo \+ \d+ll)\) \* 64ll \+ it\]", l).group(1)) * 64 + env["it"]
                             for l in st_lines])
    assert len(np.unique(stores)) == len(stores) and stores.min() >= 0 and stores.max() < group_c2
    scaled = [re.search(r", cst\[scl \+ (\d+)ll\]\);$", l) for l in st_lines]
    if any(scaled):
        assert all(scaled), "some results of a scaled step stored unscaled"
        sidx = np.concatenate([env["scl"] + int(m.group(1)) for m in scaled])
        check_scale_linear(stores // 64, sidx)
    return nu


def check_scale_linear(elem, sidx):
    """A step with a constant scale operand multiplies output element e by the
    scale's entry at e's values of the scale's variables: the entry index is
    base + sum_j bit_j(e) * w_j for fixed weights w_j.  Checks that the
    generated index has that form on the elements evaluated (a least-squares
    fit over their bits must reproduce every index exactly)."""
    elem = np.asarray(elem, dtype=np.int64)
    sidx = np.asarray(sidx, dtype=np.int64)
    rel = elem - elem.min()
    nbits = max(1, int(rel.max()).bit_length())
    bits = ((rel[:, None] >> np.arange(nbits)[None, :]) & 1).astype(np.float64)
    X = np.concatenate([np.ones((len(rel), 1)), bits], 1)
    w, *_ = np.linalg.lstsq(X, sidx.astype(np.float64), rcond=None)
    assert np.array_equal(np.rint(X @ w).astype(np.int64), sidx), "scale index not linear in the output bits"


COPY16 = re.compile(r"__builtin_amdgcn_global_load_lds\(\(const void\*\)\(\(isa(\d+) \? gq0 : gq1\) \+ "
                    r"\(eo\1 \+ \(isa\1 \? ka : kb\)\) \* 64ll \+ src\d+\), \(__attribute__\(\(address_space\(3\)\)\) void\*\)\(lds \+ \((.*?)\) \* (\d+) \+ "
                    r"(\d+) \+ 1024 \* w4\), 16, 0, 0\);")
K_LINE = re.compile(r"const long long (ka|kb) = (.*);$")
READ16 = re.compile(r"const C2 ([ab])(\d+)_(\d+) = \*\(const C2\*\)\(sb \+ (rda|rdb) \+ (\d+)\);$")


def check_step16(body, S, E, lds_size, group_c2, max_blocks=None, threads=256):
    """The per-item form (one item per wavefront, 16 x 16 x 32 operands):
    replays the ring and checks that lane l of wavefront w reads, for K step
    t and row tile f (column tile g), the slot a copy of the same unit filled
    with item itb + w, row 16 f + l % 16 (column 16 g + l % 16) and local k
    4 t + l / 16, in both operands; copies and reads stay in bounds; every
    (row, column) of the tile is stored once per item."""
    lines = [l.strip() for l in body.split("\n")]
    blocks = np.arange(S, E, dtype=np.int64)
    if max_blocks is not None and E - S > max_blocks:
        blocks = np.concatenate([blocks[:max_blocks // 2], blocks[-(max_blocks // 2):]])
    blk = np.repeat(blocks, threads)
    th = np.tile(np.arange(threads, dtype=np.int64), len(blocks))
    env = {"np": np, "blk": blk, "threadIdx_x": th, "wv": th >> 6}

    def ev(e):
        return np.asarray(eval(_py_expr(e), env)) + np.zeros_like(blk)

    i_loop = next(i for i, l in enumerate(lines) if l.startswith("for (int u = 0;"))
    for l in lines[:i_loop]:
        m = re.match(r"const (?:unsigned long long|long long|unsigned|int|bool) (.*);$", l)
        if m and not K_LINE.match(l):
            for part in re.split(r", (?=[a-z]\w* = )", m.group(1)):
                name, e = part.split(" = ", 1)
                env[name.strip()] = ev(e)
    nu = int(re.search(r"for \(int u = 0; u < (\d+); \+\+u\)", body).group(1))
    m = re.search(r"const char\* sb = lds \+ \(u % (\d+)\) \* (\d+);", body)
    P, stage = int(m.group(1)), int(m.group(2))
    lid, w4 = env["lid"], env["w4"]
    ring = {}
    kk = {}

    def copy(line, st, unit):
        m = COPY16.match(line)
        q_ = m.group(1)
        isa = env["isa" + q_].astype(bool)
        g = (env["eo" + q_] + np.where(isa, kk["ka"], kk["kb"])) * 64 + env["src" + q_]
        lo = st * int(m.group(3)) + int(m.group(4)) + 1024 * w4 + 16 * lid
        assert lo.min() >= 0 and lo.max() + 16 <= lds_size
        assert g.min() >= 0 and g.max() + 1 < group_c2
        meta = np.stack([isa.astype(np.int64), env["kl" + q_], env["rw" + q_]], 1)
        ring.setdefault(st, []).append((unit, g, lo, meta))

    loop = lines[i_loop:]
    for l in lines[:i_loop]:  # prologue: literal unit and stage
        mk = K_LINE.match(l)
        if mk:
            kk[mk.group(1)] = ev(mk.group(2))
            unit = int(re.search(r"\(\(\((\d+)\) >> \d+\) & 1\)", mk.group(2)).group(1)) if "(((" in mk.group(2) else 0
        if COPY16.match(l):
            copy(l, int(COPY16.match(l).group(2)), unit)
    body_copies = [l for l in loop if K_LINE.match(l) or l.startswith("__builtin_amdgcn_global_load_lds")]
    reads = [l for l in loop if READ16.match(l)]
    item = env["itb"] + w4
    seen_k = {}
    for u in range(nu):
        env["u"] = u
        env["un"] = min(u + P - 1, nu - 1)
        st = u % P
        slot = {}
        for (un, g, lo, meta) in ring.get(st, []):
            if un == u:
                for c in range(2):
                    for key, gg, mm in zip(zip(blk.tolist(), (lo + 8 * c).tolist()), (g + c).tolist(), meta.tolist()):
                        slot[key] = (gg, mm)
        for l in reads:
            m = READ16.match(l)
            ab, t, fg = m.group(1), int(m.group(2)), int(m.group(3))
            off = env[m.group(4)] + int(m.group(5)) + st * stage
            assert off.min() >= 0 and off.max() + 8 <= lds_size
            got = [slot.get(k_, None) for k_ in zip(blk.tolist(), off.tolist())]
            assert all(x is not None for x in got), "operand read of a slot this unit did not fill"
            gidx = np.array([x[0] for x in got])
            meta = np.array([x[1] for x in got])
            assert ((gidx % 64) == item).all(), "operand read of another item"
            assert (meta[:, 0] == (1 if ab == "a" else 0)).all(), "operand read of the other operand"
            assert (meta[:, 1] == 4 * t + (lid >> 4)).all(), "k slot of another lane group"
            assert (meta[:, 2] == 16 * fg + (lid & 15)).all(), "row or column of another lane"
            seen_k.setdefault((ab, fg), []).append(gidx // 64)
        st2 = (u + P - 1) % P
        ring[st2] = []
        for l in body_copies:
            mk = K_LINE.match(l)
            if mk:
                kk[mk.group(1)] = ev(mk.group(2))
            else:
                copy(l, st2, env["un"])
    for r in seen_k.values():
        r = np.stack(r, 0)
        assert all(len(np.unique(r[:, c])) == r.shape[0] for c in range(0, r.shape[1], 61)), \
            "a summed row read twice or not at all"
    if not any(l.startswith("gm[(so + ") for l in lines):
        return nu  # results through LDS: check_epilogue16
    for l in lines:  # the result offsets, set after the loop
        m = re.match(r"const long long (so|sit) = (.*);$", l)
        if m:
            env[m.group(1)] = ev(m.group(2))
    stores = np.concatenate([ev(re.match(r"gm\[\((so \+ \d+ll)\) \* 64ll \+ sit\]", l).group(1)) * 64 + env["sit"]
                             for l in lines if l.startswith("gm[(so + ")])
    assert len(np.unique(stores)) == len(stores) and stores.min() >= 0 and stores.max() < group_c2
    return nu


RES = r"(?:cm\()?C2\{cr(?P<c>\d+_\d+)\[(?P<e>\d)\], ci(?P=c)\[(?P=e)\]\}(?:, cst\[scl \+ (?P<s>\d+)ll\]\))?"


def _result_map(body, S, n_blocks, lds_size=None, threads=256, scales=None):
    """Where each accumulator register (block, thread, tile, register) of a
    per-item step lands in the group's memory, evaluated from the generated
    result code: direct stores, or the LDS staging (writes, barrier, 16-byte
    reads and stores), replayed chunk by chunk."""
    lines = [l.strip() for l in body.split("\n")]
    blocks = np.arange(S, S + n_blocks, dtype=np.int64)
    blk = np.repeat(blocks, threads)
    th = np.tile(np.arange(threads, dtype=np.int64), len(blocks))
    env = {"np": np, "blk": blk, "threadIdx_x": th, "wv": th >> 6}

    def ev(e):
        return np.asarray(eval(_py_expr(e), env)) + np.zeros_like(blk)

    for l in lines:
        m = re.match(r"const (?:unsigned long long|long long|unsigned|int|bool) (.*);$", l)
        if m and not K_LINE.match(l) and "=" in m.group(1) and "*(const" not in l:
            for part in re.split(r", (?=[a-z]\w* = )", m.group(1)):
                name, e = part.split(" = ", 1)
                try:
                    env[name.strip()] = ev(e)
                except NameError:
                    pass  # loop-local names (u, un, ...)
    out = {}
    direct = [l for l in lines if l.startswith("gm[(so + ")]
    if direct:
        for l in direct:
            m = re.match(r"gm\[\((so \+ \d+ll)\) \* 64ll \+ sit\] = " + RES + ";$", l)
            g = ev(m.group(1)) * 64 + env["sit"]
            for b_, t_, gg in zip(blk.tolist(), th.tolist(), g.tolist()):
                key = (b_, t_, m.group("c"), int(m.group("e")))
                assert key not in out
                out[key] = gg
            if m.group("s") is not None and scales is not None:
                for b_, t_, sc in zip(blk.tolist(), th.tolist(), (env["scl"] + int(m.group("s"))).tolist()):
                    scales[(b_, t_, m.group("c"), int(m.group("e")))] = sc
        return out
    i_epi = next(i for i, l in enumerate(lines) if l.startswith("const int wre"))
    lds = {}
    for l in lines[i_epi:]:
        if l == "__syncthreads();":
            continue
        m = re.match(r"\*\(C2\*\)\(lds \+ (.*)\) = " + RES + ";$", l)
        if m:
            a = ev(m.group(1))
            if m.group("s") is not None and scales is not None:
                for b_, t_, sc in zip(blk.tolist(), th.tolist(), (env["scl"] + int(m.group("s"))).tolist()):
                    scales[(b_, t_, m.group("c"), int(m.group("e")))] = sc
            assert a.min() >= 0 and (lds_size is None or a.max() + 8 <= lds_size)
            for b_, t_, aa in zip(blk.tolist(), th.tolist(), a.tolist()):
                assert (b_, aa) not in lds or lds[(b_, aa)][0] == "read", "LDS slot written twice in one chunk"
                lds[(b_, aa)] = ("acc", (b_, t_, m.group("c"), int(m.group("e"))))
            continue
        m = re.match(r"const f32x4 v = \*\(const f32x4\*\)\(lds \+ (\d+) \+ 16 \* tt\);$", l)
        if m:
            a = int(m.group(1)) + 16 * env["tt"]
            cur = []
            for b_, aa in zip(blk.tolist(), a.tolist()):
                lo8, hi8 = lds.get((b_, aa)), lds.get((b_, aa + 8))
                assert lo8 and hi8 and lo8[0] == "acc" and hi8[0] == "acc", "read of an LDS slot not written"
                cur.append((lo8[1], hi8[1]))
                lds[(b_, aa)] = ("read", None)
                lds[(b_, aa + 8)] = ("read", None)
            continue
        m = re.match(r"\*\(f32x4\*\)\(gm \+ \((seo \+ \d+ll)\) \* 64ll \+ sit\) = (?:sws \? .* : )?v;$", l)
        if m:
            g = ev(m.group(1)) * 64 + env["sit"]
            sws = env["sws"].astype(bool) if "sws" in env else np.zeros_like(blk, dtype=bool)
            for (lo8, hi8), gg, sw in zip(cur, g.tolist(), sws.tolist()):
                for key, dst in ((hi8, gg), (lo8, gg + 1)) if sw else ((lo8, gg), (hi8, gg + 1)):
                    assert key not in out
                    out[key] = dst
    return out


def check_epilogue16(src_lds, src_direct, n_blocks=4):
    """The LDS-staged results of a per-item step go where the direct stores
    put them, every accumulator register exactly once."""
    m1, m2 = STEP.search(src_lds), STEP.search(src_direct)
    assert m1.group(4) and m2.group(4) and m1.group(1) == m2.group(1)
    lds_size = int(re.search(r"char lds\[(\d+)\]", src_lds).group(1))
    threads = _threads(src_lds, m1.start())
    assert threads == _threads(src_direct, m2.start())
    got = _result_map(m1.group(5), int(m1.group(1)), n_blocks, lds_size, threads)
    want = _result_map(m2.group(5), int(m2.group(1)), n_blocks, threads=threads)
    assert len(want) == n_blocks * threads * 4 * len({k[2] for k in want})
    assert got == want


STEP = re.compile(r"  if \(blk >= (\d+)ull && blk < (\d+)ull\) \{\n  // step (\d+) \(matrix cores(, per item)?\)[^\n]*\n"
                  r"(.*?)\n  return;\n  \}", re.S)


def _threads(src, at):
    """Threads per block of the kernel whose body holds position `at`."""
    return int(list(re.finditer(r"__launch_bounds__\((\d+)\)", src[:at]))[-1].group(1))


def check_source(src, group_elems, max_blocks=None):
    steps = list(STEP.finditer(src))
    shapes = set()
    for m in steps:
        lds_size = int(list(re.finditer(r"char lds\[(\d+)\]", src[:m.start()]))[-1].group(1))
        if m.group(4):
            threads = _threads(src, m.start())
            nu = check_step16(m.group(5), int(m.group(1)), int(m.group(2)), lds_size, group_elems * 64, max_blocks,
                              threads)
            shapes.add("per item" if threads == 256 else "per item x8")
            if "cst[scl + " in m.group(5):
                scales = {}
                res = _result_map(m.group(5), int(m.group(1)), min(4, int(m.group(2)) - int(m.group(1))), lds_size,
                                  threads, scales)
                assert set(scales) == set(res), "some results of a scaled step stored unscaled"
                keys = sorted(res)
                check_scale_linear([res[k_] // 64 for k_ in keys], [scales[k_] for k_ in keys])
        else:
            nu = check_step(m.group(5), int(m.group(1)), int(m.group(2)), lds_size, group_elems * 64, max_blocks)
            shapes.add(re.search(r"const int wi = (.*?), wj = (.*?), wq = (.*?);", m.group(5)).groups())
        assert nu >= 1
    return len(steps), shapes


# (wi, wj, wq) of the four block shapes: 2 x 2 tiles, 2 i tiles x 2 item
# groups, 2 j tiles x 2 item groups, 4 item groups
SHAPE_212 = ("w4 & 1", "0", "w4 >> 1")


@pytest.mark.parametrize("plan,max_blocks,prec,table", [("7x7x30", None, q.QGM_C64, False),
                                                        ("7x7x30", None, q.QGM_BF16X3, False),
                                                        ("8x8x40-k8", 4, q.QGM_C64, True),
                                                        ("8x8x40-k8", 4, q.QGM_BF16X3, True)])
def test_matrix_core_step_indexing_stored_plans(plan, max_blocks, prec, table, tmp_path, monkeypatch):
    """Every matrix-core step of the stored plans (of the benchmark's 8x8x40
    k = 8 plan: the first and last blocks of each step, with the stored tile
    table the benchmark uses)."""
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_01450_amd", "plans")
    rec = json.load(open(os.path.join(here, plan + ".json")))
    cz = rec["circuit"]
    c = q.Circuit(generate_circuit(cz["n"], cz["depth"], cz["seed"]))
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    tiles = os.path.join(here, "tiles_mi355x.txt") if table else None
    st = q.Plan(c, rec["sliced"], rec["order"], prec=prec, engine=q.QGM_ENGINE_WIDE, tile_table_path=tiles).stats()
    src = open(glob.glob(str(tmp_path / "qgm_wide_*.hip"))[0]).read()
    n, _ = check_source(src, st["item_elems"], max_blocks)
    assert n == st["mfma_steps"] >= 1


@pytest.mark.parametrize("shape", [(2, 5, 5, 3), (2, 5, 4, 2), (2, 4, 5, 2), (1, 4, 4, 1), (0, 4, 6, 4), (1, 6, 6, 5)])
@pytest.mark.parametrize("prec", [q.QGM_C64, q.QGM_BF16X3])
def test_matrix_core_step_indexing_block_shapes(shape, prec, tmp_path, monkeypatch):
    """Single contractions (qgm_contraction_create) that take every block
    shape, among them 5 i bits with 4 j bits, which no stored plan uses."""
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    con = q.Contraction(prec, *shape)
    assert con.matrix_cores
    src = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
    n, shapes = check_source(src, con.elems)
    assert n == 1
    if shape == (2, 5, 4, 2) and prec == q.QGM_C64:
        assert shapes == {SHAPE_212}
    if prec == q.QGM_BF16X3 and shape[3] >= 5:  # built in: the per-item form for sums of 5 or more bits
        assert shapes == {"per item"}
        # the same step with the results stored straight from registers
        for f in glob.glob(str(tmp_path / "qgm_contract_*.hip")):
            os.remove(f)
        q.Contraction(prec, *shape, tile=(2, 65536, 1, 0))
        direct = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
        assert "gm[(so + " in direct and "gm[(so + " not in src
        check_epilogue16(src, direct)


TILES = [(1, 53248, 2, 0), (4, 53248, 2, 0), (2, 81920, 0, 0), (2, 114688, 3, 0), (4, 81920, 1, 1),
         (1, 53248, 2, 2), (4, 114688, 2, 3), (2, 53248, 3, 1),
         # BF16x3 per-item form: narrower row / column tiles (layouts 4 to 6)
         (1, 98304, 0, 4), (2, 49152, 0, 5), (1, 32768, 0, 6)]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape", [(2, 5, 5, 3), (1, 6, 7, 4), (3, 4, 6, 2)])
@pytest.mark.parametrize("prec", [q.QGM_C64, q.QGM_BF16X3])
def test_matrix_core_step_indexing_tile_variants(tile, shape, prec, tmp_path, monkeypatch):
    """Every tile parameter set the autotuner may choose (k steps per stage,
    ring budget, band, block layout) keeps copies and reads in bounds, each
    lane on its own item and each summed row read once."""
    if prec == q.QGM_BF16X3 and tile[0] == 1:
        tile = (2,) + tile[1:]
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    con = q.Contraction(prec, *shape, tile=tile)
    assert con.matrix_cores
    src = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
    n, _ = check_source(src, con.elems, max_blocks=16)
    assert n == 1


PER_ITEM_TILES = [(2, 65536, 0, 0), (4, 65536, 1, 0), (2, 98304, 0, 4), (4, 32768, 0, 5), (1, 49152, 1, 6),
                  # eight items per block (layout + 8)
                  (2, 131072, 0, 8), (1, 131072, 1, 8), (2, 65536, 0, 12), (2, 98304, 0, 13), (1, 65536, 1, 14)]


@pytest.mark.parametrize("tile", PER_ITEM_TILES)
@pytest.mark.parametrize("shape", [(2, 6, 7, 2), (1, 5, 6, 3), (0, 6, 6, 5)])
def test_per_item_form_variants(tile, shape, tmp_path, monkeypatch):
    """BF16x3 per-item form: every K steps per stage (more than the sum
    holds, too), ring budget, result path (jband 1: direct stores) and row /
    column tile compiles, keeps copies and reads in bounds, and puts the
    results where the direct stores do."""
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    con = q.Contraction(q.QGM_BF16X3, *shape, tile=tile)
    assert con.matrix_cores
    src = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
    n, shapes = check_source(src, con.elems, max_blocks=16)
    assert n == 1 and shapes == {"per item x8" if tile[3] & 8 else "per item"}
    if tile[2] != 1:
        for f in glob.glob(str(tmp_path / "qgm_contract_*.hip")):
            os.remove(f)
        q.Contraction(q.QGM_BF16X3, *shape, tile=(tile[0], tile[1], 1, tile[3]))
        direct = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
        check_epilogue16(src, direct)


@pytest.mark.parametrize("tile", [(2, 65536, 0, 16), (1, 131072, 0, 24), (2, 65536, 0, 21), (1, 49152, 1, 22),
                                  (2, 65536, 0, 48), (1, 131072, 1, 56)])
@pytest.mark.parametrize("shape", [(1, 6, 7, 5), (0, 6, 6, 3)])
def test_per_item_form_complex64(tile, shape, tmp_path, monkeypatch):
    """complex64 in the per-item form (FP32 16 x 16 x 4): the same copies,
    operand reads and result placement as the BF16x3 form."""
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    con = q.Contraction(q.QGM_C64, *shape, tile=tile)
    assert con.matrix_cores
    src = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
    assert "__builtin_amdgcn_mfma_f32_16x16x4f32" in src
    n, shapes = check_source(src, con.elems, max_blocks=16)
    assert n == 1 and shapes == {"per item x8" if tile[3] & 8 else "per item"}
    if tile[2] != 1:
        for f in glob.glob(str(tmp_path / "qgm_contract_*.hip")):
            os.remove(f)
        q.Contraction(q.QGM_C64, *shape, tile=(tile[0], tile[1], 1, tile[3]))
        direct = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
        check_epilogue16(src, direct)


@pytest.mark.parametrize("prec,tile", [(q.QGM_C64, (2, 65536, 0, 16)), (q.QGM_C64, (1, 131072, 0, 24)),
                                       (q.QGM_C64, (2, 65536, 0, 48)),
                                       (q.QGM_C64, (2, 65536, 1, 21)), (q.QGM_BF16X3, (2, 65536, 0, 0)),
                                       (q.QGM_BF16X3, (2, 131072, 0, 8)), (q.QGM_BF16X3, (2, 65536, 1, 4))])
@pytest.mark.parametrize("shape", [(0, 6, 6, 3), (1, 6, 7, 5), (1, 7, 6, 2)])
def test_per_item_results_cover_the_output(prec, tile, shape, tmp_path, monkeypatch):
    """Over all blocks of a per-item step, the results of every item and
    output element are written exactly once: the tile index covers each
    (item group, row tile, column tile, batch) combination once."""
    monkeypatch.setenv("QGM_DUMP_DIR", str(tmp_path))
    con = q.Contraction(prec, *shape, tile=tile)
    assert con.matrix_cores
    src = open(glob.glob(str(tmp_path / "qgm_contract_*.hip"))[0]).read()
    m = STEP.search(src)
    assert m.group(4)
    S, E = int(m.group(1)), int(m.group(2))
    lds_size = int(list(re.finditer(r"char lds\[(\d+)\]", src[:m.start()]))[-1].group(1))
    res = _result_map(m.group(5), S, E - S, lds_size, _threads(src, m.start()))
    dst = np.array(list(res.values()), dtype=np.int64)
    nb, ni, nj, _ = shape
    assert len(dst) == 64 << (nb + ni + nj)
    assert len(np.unique(dst)) == len(dst)
    assert dst.min() >= 0 and dst.max() < con.elems * 64
