"""Host-side marshalling of problem inputs into the canonical block layout.

The block table (sector tuples and offsets) always comes from the library's
own layout routine; this module only copies input values into place.
"""
import numpy as np

from . import lib


def leg_starts(leg):
    out, s = [], 0
    for _, d in leg:
        out.append(s)
        s += d
    return out


def pack_fn(legs, signs, block_fn):
    """Flat FP64 array: block_fn(key tuple) for every allowed block."""
    keys, offs = lib.layout(legs, signs)
    out = np.zeros(int(offs[-1]))
    for b, k in enumerate(keys):
        v = np.asarray(block_fn(tuple(int(x) for x in k)), dtype=np.float64).ravel()
        out[offs[b]:offs[b] + v.size] = v
    return out


def pack_dense(dense, legs, signs):
    """Flat FP64 array of the allowed blocks of a dense array."""
    starts = [leg_starts(l) for l in legs]

    def blk(k):
        sl = tuple(slice(starts[i][k[i]], starts[i][k[i]] + legs[i][k[i]][1]) for i in range(len(k)))
        return dense[sl]
    return pack_fn(legs, signs, blk)


def bond_problem(spec):
    """Plan dict and packed host operands of an isolated-bond problem."""
    wl = spec.w_leg()
    s = spec.s_leg
    prob = {"a": spec.a_leg, "s1": s, "s2": s, "c": spec.c_leg, "wl": wl, "wm": wl, "wr": wl,
            "w1": pack_dense(spec.W1, [wl, s, s, wl], lib.W_SIGNS),
            "w2": pack_dense(spec.W2, [wl, s, s, wl], lib.W_SIGNS)}
    ops = {
        "L": pack_fn([spec.a_leg, wl, spec.a_leg], lib.ENV_SIGNS, spec.L_block),
        "R": pack_fn([spec.c_leg, wl, spec.c_leg], lib.ENV_SIGNS, spec.R_block),
        "psi": pack_fn([spec.a_leg, s, s, spec.c_leg], lib.PSI_SIGNS, spec.psi_block),
        "W1": prob["w1"], "W2": prob["w2"],
    }
    return prob, ops


def concat(plan, ops_list):
    """Concatenate per-problem packed operands at the plan's offsets."""
    info = plan.info()
    sizes = {"psi": info["psi_elems"], "L": info["L_elems"], "R": info["R_elems"],
             "W1": info["W1_elems"], "W2": info["W2_elems"]}
    out = {k: np.zeros(int(v)) for k, v in sizes.items()}
    for p, ops in enumerate(ops_list):
        off = plan.offsets(p)
        for k in out:
            out[k][off[k]:off[k] + ops[k].size] = ops[k]
    return out


def initial_mps(mpo, target, m0, seed):
    """Seeded random initial MPS in the sector of total charge ``target`` as
    (legs, packed FP64 array) per site: bond legs from the sector model of
    synth.mps_bond_legs, block values from synth.blocks.mps_block."""
    from synth.sectors import mps_bond_legs
    from synth.blocks import mps_block
    n = len(mpo.W)
    legs = mps_bond_legs(n, mpo.phys, tuple(target), m0)
    out = []
    for j in range(n):
        lj = [legs[j], mpo.phys, legs[j + 1]]

        def blk(k, j=j, lj=lj):
            shape = tuple(lj[i][k[i]][1] for i in range(3))
            return mps_block(seed, j, k, shape)
        out.append((lj, pack_fn(lj, lib.MPS_SIGNS, blk)))
    return out


def unpack_dense(flat, legs, signs):
    """Dense array of a tensor in canonical layout (zeros outside the allowed
    blocks): the inverse of pack_dense."""
    keys, offs = lib.layout(legs, signs)
    starts = [leg_starts(l) for l in legs]
    dense = np.zeros(tuple(sum(d for _, d in l) for l in legs))
    for b, k in enumerate(keys):
        shape = tuple(legs[i][k[i]][1] for i in range(len(legs)))
        sl = tuple(slice(starts[i][k[i]], starts[i][k[i]] + shape[i]) for i in range(len(legs)))
        dense[sl] = np.asarray(flat[offs[b]:offs[b] + int(np.prod(shape))]).reshape(shape)
    return dense
