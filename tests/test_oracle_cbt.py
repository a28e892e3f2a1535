"""Pins of the CPU reference's CBT primitives: the paper's CBT figure
(Section 3.1) and its decode examples (Section 3.2), and brute force."""
import numpy as np
import pytest

from oracle import cbt_reduce, one_to_bit, zero_to_bit
from tests.helpers import read_golden


def _heap_from_bits(bits, D):
    h = np.zeros(2 << D, np.uint32)
    h[1 << D:] = bits
    return cbt_reduce(h, D)


def test_figure_tree_values():
    g = read_golden("we2_cbt.txt")
    D = int(g["D"])
    bits = [int(x) for x in g["bitfield"].split()]
    h = _heap_from_bits(bits, D)
    assert h[1] == int(g["root"])
    assert h[2:4].tolist() == [int(x) for x in g["level1"].split()]
    assert h[4:8].tolist() == [int(x) for x in g["level2"].split()]
    assert h[8:16].tolist() == [int(x) for x in g["level3"].split()]
    assert h[16:32].tolist() == bits
    assert h[1] == sum(bits)  # the root counts the set bits


def test_figure_decode_examples():
    g = read_golden("we2_cbt.txt")
    D = int(g["D"])
    h = _heap_from_bits([int(x) for x in g["bitfield"].split()], D)
    for pair in g["one_to_bit"].split():
        i, want = (int(x) for x in pair.split(":"))
        assert one_to_bit(h, D, i) == want


def test_figure_decode_all_by_scan():
    g = read_golden("we2_cbt.txt")
    D = int(g["D"])
    bits = [int(x) for x in g["bitfield"].split()]
    h = _heap_from_bits(bits, D)
    ones = [i for i, b in enumerate(bits) if b]
    zeros = [i for i, b in enumerate(bits) if not b]
    assert [one_to_bit(h, D, i) for i in range(len(ones))] == ones == [0, 3, 10, 11, 12, 13, 14]
    assert [zero_to_bit(h, D, i) for i in range(len(zeros))] == zeros == [1, 2, 4, 5, 6, 7, 8, 9, 15]


@pytest.mark.parametrize("D", [1, 2, 3, 5, 8, 12])
def test_decode_brute_force(D):
    rng = np.random.default_rng(100 + D)
    for trial in range(6):
        p = [0.0, 1.0, 0.5, rng.random()][trial % 4]
        bits = (rng.random(1 << D) < p).astype(np.uint32)
        h = _heap_from_bits(bits, D)
        ones = np.nonzero(bits)[0]
        zeros = np.nonzero(bits == 0)[0]
        assert h[1] == ones.size
        # every inner node is the number of set bits below it
        for node in range(1, 1 << D):
            lvl = node.bit_length() - 1
            span = 1 << (D - lvl)
            lo = (node - (1 << lvl)) * span
            assert h[node] == bits[lo:lo + span].sum()
        got1 = [one_to_bit(h, D, i) for i in range(ones.size)]
        got0 = [zero_to_bit(h, D, i) for i in range(zeros.size)]
        assert got1 == ones.tolist()
        assert got0 == zeros.tolist()
