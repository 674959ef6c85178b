"""Host checks of the comparator network that orders a lane's nine stencil
rows by length in the pair walk (csrc/pc_device.h, sort9_desc).  By the 0-1
principle a comparator network sorts every input iff it sorts every input
of zeros and ones, so all 2^9 of them are tried."""
import itertools
import re
from pathlib import Path

import numpy as np

HEADER = Path(__file__).resolve().parents[1] / "paper_1805_11007_amd" / "csrc" / "pc_device.h"


def _network():
    src = HEADER.read_text()
    m = re.search(r"constexpr int kNet\[(\d+)\]\[2\] = \{(.*?)\};", src, re.S)
    assert m, "sort9_desc's network not found"
    pairs = [tuple(map(int, p)) for p in re.findall(r"\{(\d+),\s*(\d+)\}", m.group(2))]
    assert len(pairs) == int(m.group(1))
    return pairs


def _apply(net, v):
    v = list(v)
    for a, b in net:
        # the kernel keeps the larger key at the lower index
        hi, lo = max(v[a], v[b]), min(v[a], v[b])
        v[a], v[b] = hi, lo
    return v


def test_nine_key_network_sorts_every_zero_one_input():
    net = _network()
    assert all(0 <= a < b < 9 for a, b in net)
    for bits in itertools.product((0, 1), repeat=9):
        assert _apply(net, bits) == sorted(bits, reverse=True), bits


def test_nine_key_network_sorts_random_keys_with_distinct_rows():
    # keys as the kernel forms them: length << 5 | row, all distinct
    net = _network()
    rng = np.random.default_rng(3)
    for _ in range(2000):
        lens = rng.integers(0, 2048, 9)
        keys = [int(l) << 5 | r for r, l in enumerate(lens)]
        assert _apply(net, keys) == sorted(keys, reverse=True)
