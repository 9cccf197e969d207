"""MPOs with a bond leg per bond, and their lossless SVD compression (the
paper compresses its MPOs by SVD with a 1e-13 cutoff, Sec. VI-B).

An MPO site W_j(w, s', s, w') (bra before ket) conserves flux:
f_w + q_s' - q_s - f_w' = 0.  Fusing (s', s) into one leg p with charge
q_s' - q_s turns the MPO into a chain of order-3 tensors M_j(w, p, w') with the
sign rule of an MPS site, so the compression is two sweeps of the library's
own sweep operations on that chain (bsdmrg_merge, bsdmrg_truncate):
  1. left to right, theta = M_j M_{j+1} split with A = U (left-orthonormal)
     and B = S V^T, dropping only the numerical null space (1e-14 of the norm);
  2. right to left, theta = M_{j-1} M_j split with A = U S and B = V^T,
     dropping the singular values below cutoff times the norm (the sites to
     the left are orthonormal, so these are the operator's Schmidt values
     across the bond and the norm is the operator's Frobenius norm).
The boundary channels (start on the first bond, done on the last) are
absorbed first, so both end bonds carry one channel.  Fusing and unfusing the
physical pair is a permutation of the tiny site tensors on the host; every
contraction and SVD runs in the library.
"""
import numpy as np

from . import lib, problems


class BondMPO:
    """MPO with its own leg on every bond: W[j] dense (k_j, d, d, k_{j+1}),
    legs[j] the flux sectors [(flux, n)] of bond j (N + 1 of them), the left
    boundary on channel ``start`` of bond 0 and the right one on ``done`` of
    bond N."""

    def __init__(self, W, legs, phys, start, done):
        self.W, self.legs, self.phys, self.start, self.done = W, legs, phys, start, done

    @classmethod
    def uniform(cls, mpo):
        """The finite-state-machine MPO with the same channel leg on every bond."""
        return cls(list(mpo.W), [mpo.w_leg()] * (len(mpo.W) + 1), mpo.phys, mpo.start, mpo.done)

    def bond_dims(self):
        return [sum(n for _, n in leg) for leg in self.legs]


def _pair_leg(phys):
    """Fused (s', s) leg: sectors of charge q_s' - q_s ascending, the pairs of
    a sector in lexicographic order.  Returns (leg, index of every pair)."""
    q = [tuple(c) for c, _ in phys]
    d = len(q)
    by_charge = {}
    for sp in range(d):
        for s in range(d):
            by_charge.setdefault(tuple(a - b for a, b in zip(q[sp], q[s])), []).append((sp, s))
    leg, index, pos = [], {}, 0
    for ch in sorted(by_charge):
        leg.append((ch, len(by_charge[ch])))
        for pr in by_charge[ch]:
            index[pr] = pos
            pos += 1
    return leg, index


def _flux_list(leg):
    out = []
    for f, n in leg:
        out += [tuple(f)] * n
    return out


def compress(mpo, cutoff=1e-13, device="cuda"):
    """Compressed BondMPO of an MPO (FSM MPO or BondMPO) with the library's
    merge and truncation on the fused chain (see the module docstring)."""
    import torch
    src = mpo if isinstance(mpo, BondMPO) else BondMPO.uniform(mpo)
    N = len(src.W)
    d = len(src.phys)
    P, pidx = _pair_leg(src.phys)
    perm = np.zeros(d * d, dtype=np.int64)
    for (sp, s), i in pidx.items():
        perm[i] = sp * d + s
    legs = list(src.legs)
    W = [np.asarray(w, dtype=np.float64) for w in src.W]
    # absorb the boundary channels
    f0, fN = _flux_list(legs[0])[src.start], _flux_list(legs[N])[src.done]
    W[0] = W[0][src.start:src.start + 1]
    W[N - 1] = W[N - 1][..., src.done:src.done + 1]
    legs[0], legs[N] = [(f0, 1)], [(fN, 1)]

    def fuse(w, l, r):
        kl, kr = w.shape[0], w.shape[3]
        m = w.reshape(kl, d * d, kr)[:, perm, :]
        return torch.from_numpy(problems.pack_dense(m, [l, P, r], lib.MPS_SIGNS)).to(device)

    M = [fuse(W[j], legs[j], legs[j + 1]) for j in range(N)]

    def step(j, direction, cut):
        op = lib.merge_plan(legs[j], P, legs[j + 1], P, legs[j + 2])
        theta = torch.zeros(max(1, op.query()["out_elems"]), dtype=torch.float64, device=device)
        lib.merge(op, M[j], M[j + 1], theta)
        A, B, leg, sv, disc = lib.truncate([legs[j], P, P, legs[j + 2]], theta, direction, cutoff=cut,
                                           cutoff_mode=0)
        op.destroy()
        M[j], M[j + 1] = A, B
        legs[j + 1] = leg

    for j in range(N - 1):
        step(j, 0, 1e-14)
    for j in range(N - 2, -1, -1):
        step(j, 1, cutoff)
    out = []
    for j in range(N):
        m = problems.unpack_dense(M[j].cpu().numpy(), [legs[j], P, legs[j + 1]], lib.MPS_SIGNS)
        w = np.zeros((m.shape[0], d * d, m.shape[2]))
        w[:, perm, :] = m
        out.append(w.reshape(m.shape[0], d, d, m.shape[2]))
    return BondMPO(out, legs, src.phys, 0, 0)
