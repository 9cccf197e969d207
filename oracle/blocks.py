"""Legs, canonical layout, block tensors and the block contraction (Alg. 2).

Quantum-number block form (Sec. II-D): an order-r tensor is a list of dense
blocks, one per tuple of sector labels whose charges are allowed.  Here a leg
is a list [(charge tuple, dim)] sorted strictly ascending, a tensor carries one
sign per leg, and a block (tuple of sector indices) is allowed iff
sum_i sign_i * charge_i == 0 componentwise.

Canonical layout (the byte-exact contract with the GPU library):
  * blocks = all allowed sector-index tuples in lexicographic order;
  * each block is dense and row-major over its legs in leg order;
  * offsets[0] = 0, offsets[b+1] = offsets[b] + round_up(size_b, 32) elements;
    the padding is zero.
"""
import functools
import itertools

import numpy as np

ALIGN = 32


def ein(spec, *ops):
    """einsum with an unconstrained-memory contraction order (NumPy's default
    path search caps intermediates at the largest input, which forces a naive
    order for multi-operand contractions)."""
    path = np.einsum_path(spec, *ops, optimize=("optimal", 1e9))[0]
    return np.einsum(spec, *ops, optimize=path)


def check_leg(leg):
    qs = [tuple(q) for q, _ in leg]
    for a, b in zip(qs, qs[1:]):
        if not a < b:
            raise ValueError("leg charges must be strictly ascending")
    for _, d in leg:
        if d < 1:
            raise ValueError("sector dimensions must be >= 1")


def leg_dim(leg):
    return sum(d for _, d in leg)


def leg_starts(leg):
    out, s = [], 0
    for _, d in leg:
        out.append(s)
        s += d
    return out


def allowed(legs, signs, key):
    r = len(legs[0][0][0])
    tot = [0] * r
    for leg, sg, i in zip(legs, signs, key):
        q = leg[i][0]
        for c in range(r):
            tot[c] += sg * q[c]
    return all(t == 0 for t in tot)


def allowed_keys(legs, signs):
    """All allowed sector-index tuples, lexicographic order (brute force)."""
    return [key for key in itertools.product(*[range(len(l)) for l in legs])
            if allowed(legs, signs, key)]


def block_shape(legs, key):
    return tuple(leg[i][1] for leg, i in zip(legs, key))


def round_up(x, a=ALIGN):
    return (x + a - 1) // a * a


def _freeze(legs, signs):
    return (tuple(tuple((tuple(q), int(d)) for q, d in l) for l in legs), tuple(signs))


@functools.lru_cache(maxsize=4096)
def _layout_cached(frozen):
    legs, signs = frozen
    for l in legs:
        check_leg(l)
    keys = allowed_keys(legs, signs)
    offsets = [0]
    for k in keys:
        offsets.append(offsets[-1] + round_up(int(np.prod(block_shape(legs, k)))))
    return tuple(keys), tuple(offsets)


def canonical_layout(legs, signs):
    """(keys, offsets) of the canonical layout; len(offsets) == len(keys) + 1."""
    keys, offs = _layout_cached(_freeze(legs, signs))
    return list(keys), list(offs)


class BlockTensor:
    """Dict of dense blocks keyed by sector-index tuples."""

    def __init__(self, legs, signs, blocks=None):
        self.legs = [list(l) for l in legs]
        self.signs = list(signs) if signs is not None else None
        self.blocks = dict(blocks or {})

    # -- construction ------------------------------------------------------
    @classmethod
    def from_fn(cls, legs, signs, fn):
        """Fill every allowed block with fn(key) (shape must match)."""
        bt = cls(legs, signs)
        for k in canonical_layout(legs, signs)[0]:
            v = np.asarray(fn(k), dtype=np.float64).reshape(block_shape(legs, k))
            bt.blocks[k] = v.copy()
        return bt

    @classmethod
    def zeros(cls, legs, signs):
        return cls.from_fn(legs, signs, lambda k: np.zeros(block_shape(legs, k)))

    def copy(self):
        return BlockTensor(self.legs, self.signs, {k: v.copy() for k, v in self.blocks.items()})

    # -- dense embedding (the "sparse-dense" format of Sec. IV-A) ------------
    def to_dense(self):
        shape = tuple(leg_dim(l) for l in self.legs)
        out = np.zeros(shape)
        starts = [leg_starts(l) for l in self.legs]
        for k, v in self.blocks.items():
            sl = tuple(slice(starts[i][k[i]], starts[i][k[i]] + self.legs[i][k[i]][1])
                       for i in range(len(k)))
            out[sl] = v
        return out

    @classmethod
    def from_dense(cls, dense, legs, signs, check_zero=True, atol=0.0):
        """Extract allowed blocks; optionally assert zeros everywhere else."""
        bt = cls(legs, signs)
        starts = [leg_starts(l) for l in legs]
        mask = np.zeros(dense.shape, dtype=bool)
        for k in canonical_layout(legs, signs)[0]:
            sl = tuple(slice(starts[i][k[i]], starts[i][k[i]] + legs[i][k[i]][1])
                       for i in range(len(k)))
            bt.blocks[k] = dense[sl].copy()
            mask[sl] = True
        if check_zero:
            outside = np.abs(dense[~mask]).max() if (~mask).any() else 0.0
            if outside > atol:
                raise AssertionError(f"charge conservation violated: |outside| = {outside}")
        return bt

    # -- canonical flat layout ---------------------------------------------
    def pack(self):
        keys, offs = canonical_layout(self.legs, self.signs)
        out = np.zeros(offs[-1])
        for k, o in zip(keys, offs):
            if k in self.blocks:
                v = self.blocks[k].ravel()
                out[o:o + v.size] = v
        return out

    @classmethod
    def unpack(cls, flat, legs, signs):
        keys, offs = canonical_layout(legs, signs)
        bt = cls(legs, signs)
        for k, o in zip(keys, offs):
            shp = block_shape(legs, k)
            n = int(np.prod(shp))
            bt.blocks[k] = np.array(flat[o:o + n], dtype=np.float64).reshape(shp)
        return bt

    # -- small helpers -----------------------------------------------------
    def norm(self):
        return float(np.sqrt(sum(float(np.sum(v * v)) for v in self.blocks.values())))

    def dot(self, other):
        return float(sum(float(np.sum(v * other.blocks[k]))
                         for k, v in self.blocks.items() if k in other.blocks))

    def scale(self, a):
        return BlockTensor(self.legs, self.signs, {k: a * v for k, v in self.blocks.items()})

    def axpy(self, a, other):
        out = self.copy()
        for k, v in other.blocks.items():
            out.blocks[k] = out.blocks.get(k, 0.0) + a * v
        return out


def contract(A, B, axes_a, axes_b, out_signs=None):
    """Block contraction of A and B over axes_a / axes_b (Alg. 2).

    Every pair (A block, B block) whose sector labels agree on all contracted
    legs (the legs are identical, so equal label means equal charge) is
    contracted with one dense tensordot; the result is keyed by the remaining
    labels, A's remaining legs first, and pairs are accumulated in
    lexicographic (A key, B key) order.  Returns (C, flops) with
    flops = sum over pairs of 2 * (product of all distinct index extents).
    """
    for ia, ib in zip(axes_a, axes_b):
        if [tuple(q) for q, _ in A.legs[ia]] != [tuple(q) for q, _ in B.legs[ib]] or \
           [d for _, d in A.legs[ia]] != [d for _, d in B.legs[ib]]:
            raise ValueError("contracted legs differ")
    rem_a = [i for i in range(len(A.legs)) if i not in axes_a]
    rem_b = [i for i in range(len(B.legs)) if i not in axes_b]
    legs_c = [A.legs[i] for i in rem_a] + [B.legs[i] for i in rem_b]
    C = BlockTensor(legs_c, out_signs)
    flops = 0
    for ka in sorted(A.blocks):
        va = A.blocks[ka]
        for kb in sorted(B.blocks):
            if any(ka[ia] != kb[ib] for ia, ib in zip(axes_a, axes_b)):
                continue
            vb = B.blocks[kb]
            kc = tuple(ka[i] for i in rem_a) + tuple(kb[i] for i in rem_b)
            prod = np.tensordot(va, vb, axes=(list(axes_a), list(axes_b)))
            flops += 2 * int(np.prod(va.shape)) * int(np.prod([vb.shape[i] for i in rem_b]))
            if kc in C.blocks:
                C.blocks[kc] = C.blocks[kc] + prod
            else:
                C.blocks[kc] = prod
    return C, flops
