"""Contraction of an MPO into the dense matrix it represents (Sec. II-B: the
MPO factorises H_{sigma_1..sigma_N nu_1..nu_N} into a product of order-4
tensors summed over the bond indices), with the left boundary on the
``start`` channel and the right boundary on the ``done`` channel.  Used only
to check MPO inputs against the textbook Hamiltonians."""
import numpy as np


def mpo_to_dense(mpo):
    W = mpo.W
    d = mpo.d
    cur = W[0][mpo.start]                         # (s', s, w')
    cur = cur.reshape(d, d, -1)
    for Wj in W[1:]:
        # cur: (bra..., ket..., w) flattened as (D, D, w)
        D = cur.shape[0]
        nxt = np.einsum("abw,wpsv->apbsv", cur, Wj)  # (D, d, D, d, w')
        cur = nxt.reshape(D * d, D * d, -1)
    return cur[:, :, mpo.done]
