"""Compact storage of the CPML memory variables (host-side check of the
layout the layer kernels address, csrc/wfd_cpml.hip).

A memory variable of one axis is nonzero only on that axis' layer, the B
border cells at each end of the N padded cells.  It is stored as two slabs of
W = B + 8 cells ([0, W) and [N - W, N), the whole axis when they would
meet).  The kernels read a variable only at points within reach (4 cells) of
the layer and at most 4 cells from such a point, and address the read as
"stored index of the point + offset": that is valid only if the whole read
lies in the point's own slab.  Checked by brute force on every cell of axes
from tiny (slabs meeting) to large.
"""

import pytest

REACH = 4


def slab(N, B):
    half = N if 2 * (B + 8) >= N else B + 8
    length = N if 2 * (B + 8) >= N else 2 * (B + 8)
    return half, length


def cidx(i, half, length, N):
    return i if i < half else i - (N - length)


def stored(i, half, length, N):
    return i < half or i >= N - (length - half)


@pytest.mark.parametrize("n,B", [(1, 1), (2, 3), (5, 4), (16, 8), (30, 4), (64, 16),
                                 (200, 20), (512, 32), (7, 0)])
def test_every_layer_read_lands_in_its_slab(n, B):
    N = n + 2 * B
    half, length = slab(N, B)
    assert 0 < length <= N
    layer = [i < B or i >= N - B for i in range(N)]
    reach = [any(layer[j] for j in range(max(0, i - REACH), min(N, i + REACH + 1)))
             for i in range(N)]
    for i in range(N):
        if layer[i]:
            assert stored(i, half, length, N)
            assert 0 <= cidx(i, half, length, N) < length
        if not reach[i]:
            continue
        base = cidx(i, half, length, N)
        for j in range(-REACH, REACH + 1):
            k = i + j
            if k < 0 or k >= N:
                continue          # outside the grid: read as zero
            # stored, and addressed as the point's index plus the offset
            assert stored(k, half, length, N)
            assert cidx(k, half, length, N) == base + j
            assert 0 <= base + j < length
    # distinct cells of the layer map to distinct stored cells
    idx = [cidx(i, half, length, N) for i in range(N) if layer[i]]
    assert len(set(idx)) == len(idx)
