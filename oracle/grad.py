"""Reference gradients of the two-site energy functional.

E(psi, L, W_i, W_{i+1}, R) = psi^T H_eff psi with H_eff the two-site form of
the effective operator of Sec. II-C (real tensors).  E is linear in each of L,
W_i, W_{i+1} and R, so every partial derivative is the same full contraction
with that operand left out; dE/dpsi = (H_eff + H_eff^T) psi.  Written with
einsum on the dense-embedded (sparse-dense, Sec. IV-A) arrays, then read back
on the allowed blocks.  Index letters: x=a', p=s1', q=s2', y=c', w, u=w',
v=w'', a, s=s1, t=s2, c.
"""
import numpy as np

from .blocks import BlockTensor, ein as _ein
from .heff import PSI_SIGNS, ENV_SIGNS, W_SIGNS

_E = "xpqy,xwa,wpsu,uqtv,yvc,astc->"


def energy(L, W1, W2, R, psi):
    P, Ld, W1d, W2d, Rd = psi.to_dense(), L.to_dense(), W1.to_dense(), W2.to_dense(), R.to_dense()
    return float(_ein(_E, P, Ld, W1d, W2d, Rd, P))


def gradients(L, W1, W2, R, psi):
    """dict of BlockTensors: psi, L, W1, W2, R (dE/d each)."""
    P, Ld, W1d, W2d, Rd = psi.to_dense(), L.to_dense(), W1.to_dense(), W2.to_dense(), R.to_dense()
    g_bra = _ein("xwa,wpsu,uqtv,yvc,astc->xpqy", Ld, W1d, W2d, Rd, P)
    g_ket = _ein("xpqy,xwa,wpsu,uqtv,yvc->astc", P, Ld, W1d, W2d, Rd)
    gL = _ein("xpqy,wpsu,uqtv,yvc,astc->xwa", P, W1d, W2d, Rd, P)
    gW1 = _ein("xpqy,xwa,uqtv,yvc,astc->wpsu", P, Ld, W2d, Rd, P)
    gW2 = _ein("xpqy,xwa,wpsu,yvc,astc->uqtv", P, Ld, W1d, Rd, P)
    gR = _ein("xpqy,xwa,wpsu,uqtv,astc->yvc", P, Ld, W1d, W2d, P)
    full = lambda d, legs, signs: BlockTensor.from_dense(d, legs, signs, check_zero=False)
    return {
        "psi": full(g_bra + g_ket, psi.legs, PSI_SIGNS),
        "L": full(gL, L.legs, ENV_SIGNS),
        "W1": full(gW1, W1.legs, W_SIGNS),
        "W2": full(gW2, W2.legs, W_SIGNS),
        "R": full(gR, R.legs, ENV_SIGNS),
    }
