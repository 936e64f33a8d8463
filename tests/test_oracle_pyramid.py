"""Pins for the oracle's resolution pyramid (Sec. 3.1, Sec. 3.4 tie rule)."""
import numpy as np
import pytest

import synth
from brute import morton_to_dense, pyramid_dense, subtree_constant


@pytest.mark.parametrize("b,nl,smooth,seed", [(2, 3, 0, 1), (4, 2, 0, 2), (4, 5, 1, 3), (8, 3, 2, 4), (8, 9, 0, 5),
                                              (16, 4, 3, 6)])
def test_pyramid_matches_definition(orc, b, nl, smooth, seed):
    brick = synth.random_brick(b, nl, seed, smooth)
    levels, consts = orc.pyramid(brick)
    ref, refc = pyramid_dense(brick)
    for l in range(len(levels)):
        g = b >> l
        np.testing.assert_array_equal(morton_to_dense(levels[l], g), ref[l])
        np.testing.assert_array_equal(morton_to_dense(consts[l], g), refc[l])


def test_constant_flag_is_subtree_uniformity(orc):
    brick = synth.random_brick(8, 2, 11, smooth=4)
    _, consts = orc.pyramid(brick)
    for l in range(4):
        np.testing.assert_array_equal(morton_to_dense(consts[l], 8 >> l), subtree_constant(brick, l))


def test_tie_goes_to_first_child(orc):
    # children (Morton order) B A A B B A C C: A and B both 3 times, B first
    ch = [4, 17, 17, 4, 4, 17, 9, 9]
    brick = np.zeros((2, 2, 2), np.uint32)
    for k, v in enumerate(ch):
        brick[k >> 2, (k >> 1) & 1, k & 1] = v
    levels, consts = orc.pyramid(brick)
    assert levels[1][0] == 4
    assert not consts[1][0]
