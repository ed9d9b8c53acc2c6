"""CPU check of the traversal stack bound (no GPU).

The build splits a sorted key range where neighbouring keys differ in their
highest bit (the key XOR of neighbours; equal keys fall back to the position
XOR, ranked below every code difference).  The short stack's spill area is
sized from the claim that no root-to-leaf path repeats the highest bit of a
split, so a tree is at most 63 code-bit + 31 position-bit levels + the leaf
edge = 95 deep, and a four-wide walk (three deferred entries per two binary
levels) holds at most 3 * ceil(95 / 2) entries.  This file models the split
structure on the CPU for uniform, duplicate-heavy and comb-shaped inputs and
checks the claim, the height bound and the spill-area constants in the
traversal header.
"""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def morton3(pts):
    """21 bits per dimension, bit-loop interleave (x highest), on the unit cube."""
    cell = np.clip(np.floor(pts.astype(np.float64) * (1 << 21)), 0, (1 << 21) - 1).astype(np.uint64)
    code = np.zeros(len(pts), dtype=np.uint64)
    for b in range(20, -1, -1):
        for d in range(3):
            code = (code << np.uint64(1)) | ((cell[:, d] >> np.uint64(b)) & np.uint64(1))
    return code


def split_keys(codes):
    """Split key between sorted positions i and i + 1: code XOR above bit 31, else position XOR."""
    c = [int(x) for x in np.sort(codes)]
    return [((c[i] ^ c[i + 1]) << 31) if c[i] != c[i + 1] else (i ^ (i + 1)) for i in range(len(c) - 1)]


def walk_tree(keys):
    """Binary radix tree over n = len(keys) + 1 sorted leaves, split where the split key is
    largest.  Returns the height in edges and checks that highest bits strictly decrease."""
    n = len(keys) + 1
    height = 0
    stack = [(0, n - 1, 1 << 200, 0)]  # range [l, r], parent's split highest-bit bound, depth
    while stack:
        l, r, parent_bit, depth = stack.pop()
        if l == r:
            height = max(height, depth)
            continue
        seg = keys[l:r]
        s = l + max(range(len(seg)), key=lambda j: seg[j])
        bit = keys[s].bit_length() - 1
        assert bit < parent_bit, "a path repeats the highest bit of a split"
        # the split is unique in its range: no other key of the range has the same highest bit
        assert sum(1 for k in seg if k.bit_length() - 1 == bit) == 1
        stack.append((l, s, bit, depth + 1))
        stack.append((s + 1, r, bit, depth + 1))
    return height


def header_constants():
    src = open(os.path.join(ROOT, "paper_2507_23700_amd", "csrc", "traverse.hpp")).read()
    h = int(re.search(r"constexpr int kMaxTreeHeight = (\d+);", src).group(1))
    s = int(re.search(r"constexpr int kSpill = (\d+);", src).group(1))
    return h, s


def test_spill_area_covers_the_four_wide_bound():
    h, s = header_constants()
    assert h == 63 + 31 + 1
    assert s >= 3 * ((h + 1) // 2)


def test_uniform_points():
    g = np.random.default_rng(1)
    assert walk_tree(split_keys(morton3(g.random((3000, 3))))) <= header_constants()[0]


def test_equal_points_split_by_position():
    h = walk_tree(split_keys(np.zeros(1000, dtype=np.uint64)))
    assert h == 10  # position splits alone make a balanced tree of ceil(log2 1000) levels


def test_comb_close_to_the_deepest_tree():
    # one split at every code bit (cell 2^j in one dimension) above 2^10 copies of the origin
    pts = [np.zeros(3)] * (1 << 10) + [np.full(3, 1 - 2.0 ** -22)]
    for d in range(3):
        for j in range(21):
            p = np.zeros(3)
            p[d] = 2.0 ** (j - 21)
            pts.append(p)
    h = walk_tree(split_keys(morton3(np.array(pts))))
    assert 63 <= h <= header_constants()[0]
    # the deepest binary path defers at most one subtree per level, a four-wide walk three per two levels
    assert 3 * ((h + 1) // 2) <= header_constants()[1]


def test_planted_repeat_is_caught():
    # a planted mistake in the model (two splits with the same highest bit on one path) trips the check
    try:
        walk_tree([4, 5, 1])  # 5 (bit 2) above 4 (bit 2) on the left path
    except AssertionError:
        return
    raise AssertionError("the repeated highest bit went unnoticed")
