"""Seeded random block values and isolated-bond problem descriptions.

``gaussian_block(seed, tag, key, shape)`` is a pure function of its arguments
(NumPy's SeedSequence over [seed, tag, *key]); ``key`` holds non-negative
integers (sector indices, channel indices).  A consumer asks for the blocks it
needs in any order and always receives the same values.

Environment blocks follow the (bra, MPO channel, ket) index order of the left
environment in Sec. II-C.  For an isolated bond the environments are random but
*Hermitian-structured*, so that the effective Hamiltonian is symmetric: the
block of a negative-flux channel is the transpose of the block of its conjugate
positive-flux channel, flux-0 channels are symmetric matrices, and the boundary
channel (``start`` for L, ``done`` for R) is exactly the identity.
"""
import numpy as np

from .mpo import synthetic_heisenberg_bond, synthetic_hubbard_bond, SPIN_PHYS
from .sectors import spin_bond_leg, electron_bond_leg

TAG_L, TAG_R, TAG_PSI, TAG_MPS = 11, 12, 13, 14


def gaussian_block(seed, tag, key, shape):
    ss = np.random.SeedSequence([int(seed), int(tag)] + [int(x) for x in key])
    return np.random.default_rng(ss).standard_normal(shape)


def _channel_ranges(mpo):
    out, c0 = [], 0
    for _, n in mpo.w_leg():
        out.append((c0, n))
        c0 += n
    return out


def env_block(kind, mpo, bond_leg, seed, key):
    """Block (bra sector ib, channel sector iw, ket sector ik) of a synthetic
    Hermitian-structured environment, shape (b_bra, n_channels, b_ket).

    kind = 'L' (identity on the ``start`` channel) or 'R' (identity on ``done``).
    """
    ib, iw, ik = key
    tag = TAG_L if kind == "L" else TAG_R
    ident = mpo.start if kind == "L" else mpo.done
    c0, n = _channel_ranges(mpo)[iw]
    bb, bk = bond_leg[ib][1], bond_leg[ik][1]
    out = np.zeros((bb, n, bk))
    for t in range(n):
        g = c0 + t
        f = mpo.flux[g]
        if g == ident:
            assert ib == ik
            out[:, t, :] = np.eye(bb)
        elif all(x == 0 for x in f):
            assert ib == ik
            G = gaussian_block(seed, tag, (ib, g, ik), (bb, bk))
            out[:, t, :] = (G + G.T) / np.sqrt(2.0 * bk)
        elif f > tuple([0] * len(f)):
            out[:, t, :] = gaussian_block(seed, tag, (ib, g, ik), (bb, bk)) / np.sqrt(bk)
        else:
            prim = gaussian_block(seed, tag, (ik, mpo.conj[g], ib), (bk, bb)) / np.sqrt(bb)
            out[:, t, :] = prim.T
    return out


class BondSpec:
    """An isolated two-site problem: legs, two MPO sites, seeds.

    psi legs (a, s1, s2, c); L legs (a, w_left, a); R legs (c, w_right, c);
    W_i = mpo.W[0], W_{i+1} = mpo.W[1] (dense, channels sector-major).
    """

    def __init__(self, a_leg, c_leg, mpo, seed, name=""):
        self.a_leg, self.c_leg, self.mpo, self.seed, self.name = a_leg, c_leg, mpo, seed, name
        self.s_leg = mpo.phys

    @property
    def W1(self):
        return self.mpo.W[0]

    @property
    def W2(self):
        return self.mpo.W[1]

    def w_leg(self):
        return self.mpo.w_leg()

    def L_block(self, key):
        return env_block("L", self.mpo, self.a_leg, self.seed, key)

    def R_block(self, key):
        return env_block("R", self.mpo, self.c_leg, self.seed + 1, key)

    def psi_block(self, key):
        ia, i1, i2, ic = key
        shape = (self.a_leg[ia][1], self.s_leg[i1][1], self.s_leg[i2][1], self.c_leg[ic][1])
        return gaussian_block(self.seed + 2, TAG_PSI, key, shape)


def c2_bond(m=1024, k=14, seed=1):
    """Mid-chain bond of a Heisenberg cylinder: spin sector model at bond
    dimension m on both bond legs (centre 2Sz = 0), Heisenberg-type MPO with k
    channels and U(0.5, 1.5) couplings."""
    leg = spin_bond_leg(m)
    mpo = synthetic_heisenberg_bond(k, seed)
    return BondSpec(leg, leg, mpo, seed, name=f"heisenberg-bond m={m} k={k}")


def c4_bond(m=4096, k=22, seed=1):
    """Mid-chain bond of a Hubbard cylinder at half filling: electron sector
    model at bond dimension m on both bond legs (left leg centred at charge
    (N, 2Sz) = (0, 0), right leg at (2, 0): two sites add two electrons),
    Hubbard-type MPO with k channels, U = 8 and U(0.5, 1.5) hoppings."""
    a = electron_bond_leg(m, center=(0, 0))
    c = electron_bond_leg(m, center=(2, 0))
    mpo = synthetic_hubbard_bond(k, seed)
    return BondSpec(a, c, mpo, seed, name=f"hubbard-bond m={m} k={k}")


def c3_batch(n=64, seed0=100, ms=(256, 512, 1024, 2048), ks=(10, 14, 18)):
    """Batch of independent isolated bonds; problem i draws its width class
    (k) and m uniformly with seed seed0 + i."""
    out = []
    for i in range(n):
        rng = np.random.default_rng([seed0 + i, 5])
        k = int(ks[rng.integers(len(ks))])
        m = int(ms[rng.integers(len(ms))])
        out.append(c2_bond(m=m, k=k, seed=seed0 + i))
    return out


def mps_block(seed, site, key, shape):
    """Random block of the initial MPS tensor at ``site``."""
    return gaussian_block(seed, TAG_MPS, (site,) + tuple(key), shape)


__all__ = ["gaussian_block", "env_block", "BondSpec", "c2_bond", "c3_batch", "mps_block",
           "SPIN_PHYS"]
