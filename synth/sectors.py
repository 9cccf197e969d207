"""Bond-leg sector models.

A leg is a list [(charge tuple, dim), ...] sorted strictly ascending by charge.

The isolated-bond workloads use the block-size model of the paper's complexity
table (Table 2): the l-th block has dimension b_l = floor((m/q) r^l), with
q = 4, r = 0.6 for spins and r = 0.65 for electrons.  Spins: one sector at the
centre charge and two (+-l) for each l >= 1, since (1/4)(1 + 2*0.6/0.4) = 1
makes the infinite sum exactly m; the leftover of the floors goes to the centre.
Electrons: a 2-D charge lattice (d_up, d_dn) around the centre with
b = floor(P r^(|d_up| + |d_dn|)), P = m / (1 + 4 r / (1 - r)^2) so that the
infinite sum is m; again the leftover goes to the centre.
"""
import itertools
import math


def spin_bond_leg(m, q=4.0, r=0.6, center=0):
    dims = {}
    l = 0
    while True:
        b = int(math.floor((m / q) * r ** l))
        if b <= 0:
            break
        if l == 0:
            dims[center] = b
        else:
            dims[center + 2 * l] = b
            dims[center - 2 * l] = b
        l += 1
    dims[center] = dims.get(center, 0) + m - sum(dims.values())   # m < q: the centre sector only
    return [((c,), dims[c]) for c in sorted(dims)]


def electron_bond_leg(m, r=0.65, center=(0, 0)):
    P = m / (1.0 + 4.0 * r / (1.0 - r) ** 2)
    dims = {}
    L = 0
    while P * r ** L >= 1.0:
        L += 1
    for du in range(-L, L + 1):
        for dd in range(-L, L + 1):
            b = int(math.floor(P * r ** (abs(du) + abs(dd))))
            if b > 0:
                key = (center[0] + du + dd, center[1] + du - dd)
                dims[key] = dims.get(key, 0) + b
    dims[tuple(center)] += m - sum(dims.values())
    return [(c, dims[c]) for c in sorted(dims)]


def mps_bond_legs(n_sites, phys, target, m0):
    """Bond legs (n_sites + 1 of them) for a random initial MPS in the sector of
    total charge ``target``.  Bond j (to the left of site j) holds the charges
    reachable from the left with j sites that can still reach ``target`` with
    the remaining sites; each sector gets min(#left states, #right states,
    m0 // #sectors, at least 1) states.  Bond 0 = [(0, 1)], bond n = [(target, 1)].
    """
    r = len(phys[0][0])
    zero = tuple([0] * r)
    charges = [q for q, _ in phys]

    def counts(nsteps):
        out = [{zero: 1}]
        for _ in range(nsteps):
            nxt = {}
            for q, c in out[-1].items():
                for s in charges:
                    qq = tuple(a + b for a, b in zip(q, s))
                    nxt[qq] = nxt.get(qq, 0) + c
            out.append(nxt)
        return out

    left = counts(n_sites)
    right = counts(n_sites)
    legs = []
    for j in range(n_sites + 1):
        secs = []
        for q, nl in left[j].items():
            rest = tuple(t - a for t, a in zip(target, q))
            nr = right[n_sites - j].get(rest, 0)
            if nr > 0:
                secs.append((q, nl, nr))
        secs.sort()
        per = max(1, m0 // max(1, len(secs)))
        legs.append([(q, int(min(nl, nr, per))) for q, nl, nr in secs])
    return legs


def all_products(n):
    return itertools.product(*[range(k) for k in n])
