"""Lattices and coupling lists.

Sites are numbered from 0.  A cylinder of width W (periodic) and length Lx (open)
numbers site (x, y) as x*W + y: column by column, y fastest.  This is the MPO
site order.  Couplings are dicts {(i, j): value} with i < j.
"""


def merge_bonds(*dicts):
    out = {}
    for d in dicts:
        for (i, j), v in d.items():
            key = (min(i, j), max(i, j))
            out[key] = out.get(key, 0.0) + v
    return out


def chain_bonds(n, J=1.0):
    """Nearest-neighbour bonds of an open chain of n sites."""
    return {(i, i + 1): J for i in range(n - 1)}


def _cyl(x, y, W):
    return x * W + (y % W)


def cylinder_j1_bonds(W, Lx, J=1.0):
    """Directly adjacent pairs on a W x Lx cylinder (periodic in y, open in x).

    A pair that the periodic wrap would produce twice (W == 2) is kept once.
    """
    pairs = set()
    for x in range(Lx):
        for y in range(W):
            if W > 1:
                a, b = _cyl(x, y, W), _cyl(x, y + 1, W)
                if a != b:
                    pairs.add((min(a, b), max(a, b)))
            if x + 1 < Lx:
                a, b = _cyl(x, y, W), _cyl(x + 1, y, W)
                pairs.add((min(a, b), max(a, b)))
    return {p: J for p in sorted(pairs)}


def cylinder_j2_bonds(W, Lx, J=1.0):
    """Diagonally adjacent pairs: both diagonals of every plaquette, including
    the plaquettes that straddle the periodic seam."""
    pairs = set()
    for x in range(Lx - 1):
        for y in range(W):
            for dy in (1, -1):
                a, b = _cyl(x, y, W), _cyl(x + 1, y + dy, W)
                if a != b:
                    pairs.add((min(a, b), max(a, b)))
    return {p: J for p in sorted(pairs)}
