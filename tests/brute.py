"""Brute-force references written straight from the paper's definitions,
used to pin the oracle (pure numpy / Python, tiny inputs only)."""
import numpy as np


def morton_coords(m: int, bits: int):
    """Coordinates of Morton index m: bit 0 of each 3-bit group is x."""
    x = y = z = 0
    for b in range(bits):
        x |= ((m >> (3 * b)) & 1) << b
        y |= ((m >> (3 * b + 1)) & 1) << b
        z |= ((m >> (3 * b + 2)) & 1) << b
    return x, y, z


def morton_to_dense(arr, g: int) -> np.ndarray:
    bits = g.bit_length() - 1
    out = np.zeros((g, g, g), dtype=arr.dtype)
    for m in range(g ** 3):
        x, y, z = morton_coords(m, bits)
        out[z, y, x] = arr[m]
    return out


def pyramid_dense(brick: np.ndarray):
    """Levels L_0..L_N as dense [z][y][x] arrays: a node is the most frequent
    of its 8 children, a tie going to the child that comes first in child
    order k = cx + 2 cy + 4 cz (Sec. 3.1, Sec. 3.4).  Also the flags
    'whole subtree holds one label'."""
    levels = [brick.astype(np.uint32)]
    consts = [np.ones(brick.shape, dtype=bool)]
    while levels[-1].shape[0] > 1:
        a, c = levels[-1], consts[-1]
        ch = np.stack([a[cz::2, cy::2, cx::2] for cz in (0, 1) for cy in (0, 1) for cx in (0, 1)])
        cc = np.stack([c[cz::2, cy::2, cx::2] for cz in (0, 1) for cy in (0, 1) for cx in (0, 1)])
        # ch[k] is child k with k = cx + 2cy + 4cz (loop order above: cz outer, cx inner)
        counts = np.stack([(ch == ch[k]).sum(axis=0) for k in range(8)])
        best = np.argmax(counts, axis=0)  # first maximum = first occurrence
        levels.append(np.take_along_axis(ch, best[None], axis=0)[0])
        consts.append(cc.all(axis=0) & (ch == ch[0]).all(axis=0))
    return levels, consts


def subtree_constant(brick: np.ndarray, level: int):
    """Direct definition: every voxel under the node has the same label."""
    s = 1 << level
    g = brick.shape[0] // s
    out = np.zeros((g, g, g), dtype=bool)
    for z in range(g):
        for y in range(g):
            for x in range(g):
                blk = brick[z * s:(z + 1) * s, y * s:(y + 1) * s, x * s:(x + 1) * s]
                out[z, y, x] = (blk == blk.flat[0]).all()
    return out
