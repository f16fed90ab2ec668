"""Oracle of the paper's warp-based sequence blocks (Sec. 3.2, Alg. 1):
which container (column) each sequence joins, the block heights and the
padding-to-real ratio (PRR) of Table 2.

Test infrastructure only (see the package docstring).

Reading of Alg. 1 and Sec. 3.2 implemented here:
* sequences are taken longest first (ties in input order); each occupies
  its residues plus one ending residue, so its footprint is L + 1 rows;
* ``lines = N * S`` containers; container x starts with the x-th sequence;
* ``maxLen`` starts as the longest container; a search pointer starts at
  ``lines`` and, for every later sequence, moves down one container at a
  time (continuing from where the previous sequence was placed) until a
  container whose length plus the sequence's footprint is at most
  ``maxLen``; if it runs below container 0 the sequence is forced onto the
  last container and the pointer starts over from ``lines``; after each
  placement ``maxLen`` grows to the placed container's length if that is
  longer;
* containers x = i S .. i S + S - 1 form block i; its height M_i is its
  longest container; padding is S M_i minus the block's container lengths;
* PRR = padding / real residues (ending residues are counted apart).
"""
from __future__ import annotations

import numpy as np


def pack(lengths, nblocks: int, width: int):
    """Returns dict(container [n] int64 (per sequence, input order),
    heights [nblocks], padding, real, ending, prr)."""
    lengths = [int(v) for v in lengths]
    n = len(lengths)
    lines = nblocks * width
    order = sorted(range(n), key=lambda i: -lengths[i])      # stable: ties in input order
    cont_len = [0] * lines
    container = [-1] * n
    for x in range(min(lines, n)):
        s = order[x]
        container[s] = x
        cont_len[x] = lengths[s] + 1
    max_len = max(cont_len) if n else 0
    ptr = lines
    for y in range(lines, n):
        s = order[y]
        need = lengths[s] + 1
        while True:
            ptr -= 1
            if ptr < 0:
                ptr = lines
                target = lines - 1
                break
            if need + cont_len[ptr] <= max_len:
                target = ptr
                break
        container[s] = target
        cont_len[target] += need
        if cont_len[target] > max_len:
            max_len = cont_len[target]
    heights = [max(cont_len[i * width:(i + 1) * width]) for i in range(nblocks)]
    padding = sum(width * heights[i] - sum(cont_len[i * width:(i + 1) * width])
                  for i in range(nblocks))
    real = sum(lengths)
    return {"container": np.array(container, dtype=np.int64),
            "heights": np.array(heights, dtype=np.int64),
            "padding": padding, "real": real, "ending": n,
            "prr": padding / real if real else 0.0}
