"""Pin: every emitted operation is the FIRST applicable one in the order
R_p, R_x, R_y, R_z, P_0, P_delta, P_a (Sec. 3.4), with the operation
semantics of Sec. 3.2, re-derived here by brute force on small bricks."""
import numpy as np
import pytest

import synth
from brute import morton_coords, pyramid_dense

ORDER = ["Rp", "Rx", "Ry", "Rz", "P0", "Pd", "Pa"]


def morton_index(x, y, z, bits):
    m = 0
    for b in range(bits):
        m |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return m


def applicable(levels, l, C, parent, L, pal):
    """All operations that would assign label L to the child at coords C on
    level l-1, plus the smallest usable delta."""
    N = len(levels) - 1
    g = 1 << (N - (l - 1))
    bits = N - (l - 1)
    ok = {}
    ok["Rp"] = parent == L
    for a, name in enumerate(["Rx", "Ry", "Rz"]):
        # the neighbour lies outside the 2^3 sibling block along axis a
        d = -1 if (C[a] & 1) == 0 else +1
        n = list(C)
        n[a] += d
        if not (0 <= n[a] < g):
            ok[name] = False  # neighbours in other bricks are never referenced
            continue
        if morton_index(*n, bits) < morton_index(*C, bits):
            v = levels[l - 1][n[2], n[1], n[0]]  # already decoded
        else:
            v = levels[l][n[2] >> 1, n[1] >> 1, n[0] >> 1]  # later: take its parent
        ok[name] = v == L
    ok["P0"] = pal[-1] == L
    delta = None
    for d in range(16):
        i = len(pal) - 1 - d - 1
        if i < 0:
            break
        if pal[i] == L:
            delta = d
            break
    ok["Pd"] = delta is not None
    ok["Pa"] = True
    return ok, delta


def check_brick(orc, brick):
    b = brick.shape[0]
    N = b.bit_length() - 1
    sym, cum, palette = orc.brick_symbols(brick)
    levels, consts = pyramid_dense(brick)
    pal = [levels[N][0, 0, 0]]
    seg_start = 0
    for l in range(N, 0, -1):
        m_lvl = l - 1
        seg_end = int(cum[m_lvl])
        nodes = [morton_coords(m, N - l) for m in range(8 ** (N - l))]
        expanded = [c for c in nodes if not consts[l][c[2], c[1], c[0]]]
        nd = seg_end - seg_start - 8 * len(expanded)  # deltas come first
        assert nd >= 0
        dc, opc = seg_start, seg_start + nd
        for (X, Y, Z) in expanded:
            parent = levels[l][Z, Y, X]
            for k in range(8):
                C = (2 * X + (k & 1), 2 * Y + ((k >> 1) & 1), 2 * Z + (k >> 2))
                L = levels[m_lvl][C[2], C[1], C[0]]
                nib = int(sym[opc]); opc += 1
                op, stop = nib & 7, nib >> 3
                want_stop = int(consts[m_lvl][C[2], C[1], C[0]]) if m_lvl >= 1 else 0
                assert stop == want_stop
                ok, delta = applicable(levels, l, C, parent, L, pal)
                first = next(i for i, name in enumerate(ORDER) if ok[name])
                assert op == first, (l, C, op, first)
                if ORDER[op] == "Pd":
                    assert int(sym[dc]) == delta
                    dc += 1
                if ORDER[op] == "Pa":
                    pal.append(L)
        assert opc == seg_end
        assert dc == seg_start + nd
        seg_start = seg_end
    assert [int(v) for v in palette] == [int(v) for v in pal]


@pytest.mark.parametrize("seed", range(24))
def test_first_applicable_op_4cubed(orc, seed):
    nl = 2 + seed % 4
    check_brick(orc, synth.random_brick(4, nl, seed, smooth=seed % 3))


@pytest.mark.parametrize("seed", range(6))
def test_first_applicable_op_8cubed(orc, seed):
    check_brick(orc, synth.random_brick(8, 3 + seed, 100 + seed, smooth=2 + seed % 3))


def test_first_applicable_op_palette_duplicates(orc):
    # many labels in a small brick forces P_delta and palette duplicates
    rng = np.random.default_rng(7)
    brick = rng.integers(1, 20, size=(8, 8, 8)).astype(np.uint32)
    check_brick(orc, brick)
    sym, cum, pal = orc.brick_symbols(brick)
    assert len(pal) > len(np.unique(brick))  # duplicates occurred


def test_first_applicable_op_real_brick(orc):
    v = synth.voronoi_bg()
    check_brick(orc, np.ascontiguousarray(v[:16, 16:32, 32:48]))
