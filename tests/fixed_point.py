"""The quantum of the tiled spread's fixed-point sums (Sec. II.C spreading, deterministic form), as a
bar term for element-by-element checks.

A (component, tile) list of cnt entries, 2^(lc - 1) <= cnt < 2^lc, whose forces satisfy |F| < 2^em,
adds each contribution phi F as an integer number of units 2^-sc with sc = min(48 - em, 60 - em - lc)
(every contribution below 2^50, every sum below 2^62); float64 keeps the remainder below one unit in a
32-bit word at a further 2^-sl, sl = 30 - lc.  Each contribution is thus rounded to half a unit of
2^-sc (float32) or 2^-(sc + sl) (float64), and a cell that n_J contributions reach is off by at most
n_J such half units beyond the arithmetic of phi F itself.  Any fixed-point sum has such a floor, which
a bar relative to the cell's own magnitude sum |phi||F| cannot express for cells far out in the weights'
tails; both are stated here.
"""
import math

import numpy as np


def unit(max_abs_f: float, cnt_bound: int, fp64: bool) -> float:
    """Upper bound of the rounding unit of any list with at most cnt_bound entries and |F| <= max_abs_f."""
    if max_abs_f == 0.0:
        return 0.0
    em = math.frexp(max_abs_f)[1]  # |F| < 2^em
    lc = int(cnt_bound).bit_length()  # cnt < 2^lc
    sc = min(48 - em, 60 - em - lc)
    return math.ldexp(1.0, -(sc + (30 - lc if fp64 else 0)))


def list_bound(sc, tile) -> int:
    """Upper bound of the length of any spread list of scene sc with the given tile shape: a list holds
    nodes whose nearest lattice node lies in the tile or one cell outside it along x, all of them in
    the tile's 3 x 3 x 3 neighbourhood of tiles by the cell that contains them."""
    bop = sc.box[sc.node_particle()]
    best = 0
    for b, B in enumerate(sc.boxes):
        sel = bop == b
        if not sel.any():
            continue
        n = np.array(B.n)
        nt = -(-n // np.array(tile))
        c = np.floor((sc.x64[:, sel].T - np.array(B.origin)) / B.h).astype(np.int64) % n
        t = c // np.array(tile)
        cnt = np.zeros(nt, dtype=np.int64)
        np.add.at(cnt, (t[:, 0], t[:, 1], t[:, 2]), 1)
        nb = np.zeros_like(cnt)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    nb += np.roll(cnt, (dx, dy, dz), axis=(0, 1, 2))
        best = max(best, int(nb.max()))
    return best
