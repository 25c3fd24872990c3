"""Index sets I_k for IBMI -- oracle side (test infrastructure only).

The paper partitions {1..p} into K contiguous sets that may overlap (section "The
Multi-Block, Overlapping Case" and its figures of the four-block partitions).  Its cost
section fixes the shape: with core size m and overlap h, the two end sets have m+h rows
and the interior ones m+2h rows, i.e. every set is a core extended into its neighbours.
The paper never states how "overlap" is measured, so this module takes this reading:

* ``overlap`` is the number of rows shared by two consecutive sets;
* core stride m = block_rows - overlap; K = ceil(p / m), and K = 1 when p <= block_rows;
* core k = [k m, min((k+1) m, p)); set k = core k extended by floor(overlap/2) rows to
  the left and ceil(overlap/2) rows to the right, clipped to [0, p);
* a last core shorter than ``overlap`` is merged into the one before it.

With p=4096, block_rows=576, overlap=64 this gives 8 sets (544, 576 x 6, 544) that share
64 rows pairwise; with p=16384 it gives 32 sets.  Pinned by tests of covering, of set
sizes at every benchmark workload, and of pairwise overlap.
"""
from __future__ import annotations

import numpy as np


def partition(p: int, block_rows: int, overlap: int = 0) -> list:
    """Half-open ranges [(s_0, e_0), ...] for the reading stated in the module docstring."""
    if p < 1 or block_rows < 1 or overlap < 0 or overlap >= block_rows:
        raise ValueError("need p >= 1, block_rows >= 1 and 0 <= overlap < block_rows")
    if p <= block_rows:
        return [(0, p)]
    m = block_rows - overlap
    k_sets = -(-p // m)
    cores = [[k * m, min((k + 1) * m, p)] for k in range(k_sets)]
    if len(cores) > 1 and cores[-1][1] - cores[-1][0] < overlap:
        cores[-2][1] = cores[-1][1]
        cores.pop()
    h_left, h_right = overlap // 2, overlap - overlap // 2
    return [(max(0, s - h_left), min(p, e + h_right)) for s, e in cores]


def validate_blocks(p: int, blocks) -> None:
    """Ranges must be non-empty, sorted by start, inside [0, p) and cover every index."""
    covered = np.zeros(p, dtype=bool)
    last_start = -1
    for s, e in blocks:
        if not (0 <= s < e <= p) or s < last_start:
            raise ValueError(f"bad block [{s},{e}) for p={p}")
        last_start = s
        covered[s:e] = True
    if not covered.all():
        raise ValueError("blocks do not cover [0, p)")


def complement(p: int, idx: np.ndarray) -> np.ndarray:
    """I^c = {0..p-1} minus I, in increasing order."""
    mask = np.ones(p, dtype=bool)
    mask[idx] = False
    return np.nonzero(mask)[0]
