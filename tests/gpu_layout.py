"""Test-side comparator between the oracle's particle order and the GPU
library's storage layout.

The oracle re-sorts as the paper stores particles (Sections 3 and 4.3): a
stable sort by (supercell, cell), so every cell's particles sit together in
their previous order.  The GPU library stores the same per-cell lists
interleaved in rounds inside each supercell: round r holds the r-th particle
of every cell that has more than r, cells in x-fastest order.  The
interleave is pure layout (no arithmetic of the step depends on it), so it is
applied here, to the oracle's output, before orders are compared.

``round_interleave(keys, S3)`` computes that layout from keys that are
already in per-cell order, as a stable sort on the composite key
(supercell, rank of the particle in its cell, cell).  ``LayoutOracle`` is an
``oracle.OracleSim`` whose re-sorts are followed by that permutation, for
tests that follow the oracle over several re-sorts next to the GPU.
"""
from __future__ import annotations

import numpy as np

import oracle


def sort_keys(n, S, x, y, z, absorb_x=False):
    """Sort key (supercell * S^3 + cell in supercell, both x-fastest) of
    every position; removed particles (absorbing x, x < 0) get n0 n1 n2."""
    n = [int(v) for v in n]
    c = [np.floor(np.asarray(a, dtype=np.float64)).astype(np.int64) for a in (x, y, z)]
    ns0, ns1 = n[0] // S, n[1] // S
    sc = c[0] // S + ns0 * (c[1] // S + ns1 * (c[2] // S))
    loc = c[0] % S + S * (c[1] % S + S * (c[2] % S))
    key = sc * S ** 3 + loc
    if absorb_x:
        key = np.where(np.asarray(x) < 0.0, n[0] * n[1] * n[2], key)
    return key


def round_interleave(keys, S3):
    """Permutation (new index -> index in the input) that turns particles in
    per-cell order (keys non-decreasing) into the round-interleaved layout.
    Keys beyond the last cell (removed particles) keep their place at the
    end."""
    keys = np.asarray(keys, dtype=np.int64)
    n = len(keys)
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    assert np.all(np.diff(keys) >= 0), "input is not in per-cell order"
    idx = np.arange(n, dtype=np.int64)
    first = np.searchsorted(keys, keys, side="left")   # first slot of each particle's key
    rank = idx - first                                  # rank of the particle in its cell
    sc = keys // S3
    cell = keys % S3
    return np.lexsort((cell, rank, sc))                 # by supercell, then rank, then cell


class LayoutOracle(oracle.OracleSim):
    """The oracle, with the GPU library's round-interleaved layout applied
    after every re-sort (including the sort at load)."""

    def _sort(self, s):
        super()._sort(s)
        P = self.P[s]
        keys = sort_keys(self.n, self.S, P[0], P[1], P[2], self.absorb_x)
        perm = round_interleave(keys, self.S ** 3)
        self.P[s] = [np.ascontiguousarray(a[perm]) for a in P]
