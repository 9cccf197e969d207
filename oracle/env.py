"""Environment extension and two-site merge (Sec. II-C).

Left environment over the bond to the right of a left-canonical site A:
  L'(b', w', b) = sum A(a',s',b') L(a',w,a) W(w,s',s,w') A(a,s,b)
Right environment over the bond to the left of a right-canonical site B:
  R'(b', w, b)  = sum B(b',s',c') W(w,s',s,w') R(c',w',c) B(b,s,c)
(the left environment A_{i k l} of Sec. II-C with bra, MPO, ket order; the
tensors are real so the conjugate is the plain tensor).  Boundaries have unit
dimension (the footnote on the first and last MPS sites): the left one selects
the MPO's ``start`` channel, the right one its ``done`` channel.
Two-site tensor x^(j,j+1) = sum_b T^(j)(a,s1,b) T^(j+1)(b,s2,c) (Sec. II-C).
"""
import numpy as np

from .blocks import BlockTensor, contract, ein
from .heff import ENV_SIGNS, PSI_SIGNS


def left_boundary(w_leg, start, r):
    leg0 = [(tuple([0] * r), 1)]
    dense = np.zeros((1, sum(n for _, n in w_leg), 1))
    dense[0, start, 0] = 1.0
    return BlockTensor.from_dense(dense, [leg0, w_leg, leg0], ENV_SIGNS)


def right_boundary(w_leg, done, target):
    legN = [(tuple(target), 1)]
    dense = np.zeros((1, sum(n for _, n in w_leg), 1))
    dense[0, done, 0] = 1.0
    return BlockTensor.from_dense(dense, [legN, w_leg, legN], ENV_SIGNS)


def left_update_dense(L, A, W):
    """O1 form: dense einsum of the left extension."""
    Ld, Ad, Wd = L.to_dense(), A.to_dense(), W.to_dense()
    out = ein("xpy,xwa,wpsv,asb->yvb", Ad, Ld, Wd, Ad)
    return BlockTensor.from_dense(out, [A.legs[2], W.legs[3], A.legs[2]], ENV_SIGNS)


def right_update_dense(R, B, W):
    Rd, Bd, Wd = R.to_dense(), B.to_dense(), W.to_dense()
    out = ein("ypx,wpsv,xva,bsa->ywb", Bd, Wd, Rd, Bd)
    return BlockTensor.from_dense(out, [B.legs[0], W.legs[0], B.legs[0]], ENV_SIGNS)


def _full(bt, legs):
    z = BlockTensor.zeros(legs, ENV_SIGNS)
    for k in z.blocks:
        if k in bt.blocks:
            z.blocks[k] = bt.blocks[k]
    return z


def left_update_blocks(L, A, W):
    """O2 form: the same extension as three Alg. 2 contractions."""
    X1, _ = contract(L, A, [2], [0])              # a' w s b
    X2, _ = contract(X1, W, [1, 2], [0, 2])       # a' b s' w'
    Y, _ = contract(A, X2, [0, 1], [0, 2])        # b' b w'
    out = BlockTensor(Y.legs, None, {(k[0], k[2], k[1]): v.transpose(0, 2, 1)
                                     for k, v in Y.blocks.items()})
    return _full(out, [A.legs[2], W.legs[3], A.legs[2]])


def right_update_blocks(R, B, W):
    X1, _ = contract(B, R, [2], [2])              # b s c' w'
    X2, _ = contract(X1, W, [1, 3], [2, 3])       # b c' w s'
    Y, _ = contract(B, X2, [1, 2], [3, 1])        # b' b w
    out = BlockTensor(Y.legs, None, {(k[0], k[2], k[1]): v.transpose(0, 2, 1)
                                     for k, v in Y.blocks.items()})
    return _full(out, [B.legs[0], W.legs[0], B.legs[0]])


def merge(A, B):
    """theta(a, s1, s2, c) = sum_b A(a,s1,b) B(b,s2,c), all allowed blocks."""
    T, _ = contract(A, B, [2], [0])
    full = BlockTensor.zeros([A.legs[0], A.legs[1], B.legs[1], B.legs[2]], PSI_SIGNS)
    for k in full.blocks:
        if k in T.blocks:
            full.blocks[k] = T.blocks[k]
    return full
