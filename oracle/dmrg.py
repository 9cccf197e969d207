"""Two-site DMRG sweeps (Sec. II-C, Fig. 1; Alg. 1 of Sec. II-C for the eigensolver).

Bond j sits to the left of site j (j = 0 .. N); MPS tensor T_j has legs
(bond j, s_j, bond j+1).  Starting from a right-canonical MPS, a sweep visits
the pairs (j, j+1) left to right and then right to left: merge the two sites,
find the lowest eigenpair of the two-site effective Hamiltonian with the
Davidson routine started from the merged tensor, split with the truncated SVD
absorbing S in the sweep direction, and extend the environment.

Readings: the energy of a bond is the Ritz value returned by the eigensolver;
the initial MPS is random (Gaussian blocks on the allowed sectors of the
target charge) and is right-canonicalised by splits without truncation.
"""
import numpy as np

from .blocks import BlockTensor, canonical_layout, block_shape
from .eig import davidson
from .env import (left_boundary, right_boundary, left_update_dense, right_update_dense,
                  left_update_blocks, right_update_blocks, merge)
from .heff import MPS_SIGNS, PSI_SIGNS, DenseHeff, heff1_dense, heff_blocks, w_tensor
from .truncate import truncate


def random_mps(mpo, n_sites, target, m0, seed, block_fn):
    """Random MPS from the bond model and a block generator (inputs)."""
    from synth.sectors import mps_bond_legs
    legs = mps_bond_legs(n_sites, mpo.phys, target, m0)
    out = []
    for j in range(n_sites):
        L = [legs[j], mpo.phys, legs[j + 1]]
        out.append(BlockTensor.from_fn(L, MPS_SIGNS,
                                       lambda k, j=j, L=L: block_fn(seed, j, k, block_shape(L, k))))
    return out


def mask_of(legs, signs):
    keys, offs = canonical_layout(legs, signs)
    n = offs[-1]
    m = np.zeros(n, dtype=bool)
    for k, o in zip(keys, offs):
        m[o:o + int(np.prod(block_shape(legs, k)))] = True
    return m


CANON_CUTOFF = 1e-14


def right_canonicalize(mps):
    """Right-canonical form by splits from the right (S absorbed to the left).
    Singular values below 1e-14 of the norm are numerically zero: they carry
    no weight and their singular vectors are not unique, so they are dropped."""
    mps = [t.copy() for t in mps]
    for j in range(len(mps) - 1, 0, -1):
        theta = merge(mps[j - 1], mps[j])
        A, B, _, _, _ = truncate(theta, "left", cutoff=CANON_CUTOFF, m_max=1 << 60)
        mps[j - 1], mps[j] = A, B
    return mps


def solve_bond(Lenv, W1, W2, Renv, theta, dav, heff="dense", seed=0, record=None):
    legs = theta.legs
    if heff == "dense":
        op = DenseHeff(Lenv, W1, W2, Renv)
    else:
        op = lambda x: heff_blocks(Lenv, W1, W2, Renv, x)

    def mv(v):
        return op(BlockTensor.unpack(v, legs, PSI_SIGNS)).pack()

    lam, x, st = davidson(mv, theta.pack(), dav.get("max_iter", 40), dav.get("tol", 1e-12),
                          restart_mask=mask_of(legs, PSI_SIGNS), seed=seed, record=record)
    return lam, BlockTensor.unpack(x, legs, PSI_SIGNS), st


def dmrg(mpo, mps, n_sweeps, m_max, cutoff=1e-10, cutoff_mode="sv", dav=None,
         heff="dense", target=None, log=None):
    """Two-site sweeps.  ``m_max`` is an int or a per-sweep list.  Returns
    (energies per visited bond, MPS, per-sweep last energy, discarded weights)."""
    dav = dav or {"max_iter": 40, "tol": 1e-12}
    N = len(mps)
    r = len(mpo.phys[0][0])
    target = target if target is not None else mps[-1].legs[2][0][0]
    wl = mpo.w_leg()
    Ws = [w_tensor(W, wl, mpo.phys, wl) for W in mpo.W]
    lu = left_update_dense if heff == "dense" else left_update_blocks
    ru = right_update_dense if heff == "dense" else right_update_blocks
    mps = right_canonicalize(mps)
    Lenv = [None] * (N + 1)
    Renv = [None] * (N + 1)
    Lenv[0] = left_boundary(wl, mpo.start, r)
    Renv[N] = right_boundary(wl, mpo.done, target)
    for j in range(N - 1, 1, -1):
        Renv[j] = ru(Renv[j + 1], mps[j], Ws[j])
    energies, sweep_e, disc = [], [], []
    mlist = m_max if isinstance(m_max, (list, tuple)) else [m_max] * n_sweeps
    step = 0
    for sw in range(n_sweeps):
        order = [(j, "right") for j in range(N - 1)] + [(j, "left") for j in range(N - 2, -1, -1)]
        for j, d in order:
            theta = merge(mps[j], mps[j + 1])
            lam, x, st = solve_bond(Lenv[j], Ws[j], Ws[j + 1], Renv[j + 2], theta, dav, heff,
                                    seed=step)
            A, B, _, _, dw = truncate(x, d, cutoff=cutoff, cutoff_mode=cutoff_mode,
                                      m_max=mlist[sw])
            mps[j], mps[j + 1] = A, B
            if d == "right":
                Lenv[j + 1] = lu(Lenv[j], A, Ws[j])
            else:
                Renv[j + 1] = ru(Renv[j + 2], B, Ws[j + 1])
            energies.append(lam)
            disc.append(dw)
            if log is not None:
                log.append({"sweep": sw, "bond": j, "dir": d, "E": lam, "iters": st["iters"],
                            "res": st["residual"], "disc": dw})
            step += 1
        sweep_e.append(energies[-1])
    return energies, mps, sweep_e, disc


def _with_dummy(t, pos):
    """The one-site tensor (a, s, c) as a two-site tensor with a one-state
    zero-charge leg inserted at position pos (2: (a, s, 1, c); 1: (a, 1, s, c));
    blocks and their order are unchanged."""
    a, s, c = t.legs
    zero = tuple([0] * len(a[0][0]))
    one = [(zero, 1)]
    legs = [a, s, one, c] if pos == 2 else [a, one, s, c]
    out = BlockTensor(legs, PSI_SIGNS)
    for (ia, i_s, ic), v in t.blocks.items():
        key = (ia, i_s, 0, ic) if pos == 2 else (ia, 0, i_s, ic)
        out.blocks[key] = v.reshape(v.shape[0], v.shape[1], 1, v.shape[2]) if pos == 2 else \
            v.reshape(v.shape[0], 1, v.shape[1], v.shape[2])
    return out


def _drop_dummy(t, pos):
    legs = [l for i, l in enumerate(t.legs) if i != pos]
    out = BlockTensor(legs, MPS_SIGNS)
    for k, v in t.blocks.items():
        key = tuple(x for i, x in enumerate(k) if i != pos)
        out.blocks[key] = v.reshape([n for i, n in enumerate(v.shape) if i != pos])
    return out


def dmrg1(mpo, mps, n_sweeps, dav=None, target=None, log=None):
    """Single-site sweeps (the single-site form of Sec. II-C: the projected
    operator L W_j R acts on one site tensor).  From the given MPS (any
    gauge; it is right-canonicalised first), a sweep solves site j for
    j = 0 .. N-2 moving right (the solution split by SVD into a
    left-orthonormal site and S V^T carried into site j+1) and j = N-1 .. 1
    moving left (U S carried into site j-1).  The bond dimensions never grow;
    the split drops only numerically zero singular values.  Returns (energy
    of every solve, MPS, last energy of every sweep)."""
    dav = dav or {"max_iter": 40, "tol": 1e-12}
    N = len(mps)
    r = len(mpo.phys[0][0])
    target = target if target is not None else mps[-1].legs[2][0][0]
    wl = mpo.w_leg()
    Ws = [w_tensor(W, wl, mpo.phys, wl) for W in mpo.W]
    mps = right_canonicalize(mps)
    Lenv = [None] * (N + 1)
    Renv = [None] * (N + 1)
    Lenv[0] = left_boundary(wl, mpo.start, r)
    Renv[N] = right_boundary(wl, mpo.done, target)
    for j in range(N - 1, 0, -1):
        Renv[j] = right_update_dense(Renv[j + 1], mps[j], Ws[j])
    energies, sweep_e = [], []
    step = 0
    for sw in range(n_sweeps):
        order = [(j, "right") for j in range(N - 1)] + [(j, "left") for j in range(N - 1, 0, -1)]
        for j, d in order:
            psi = mps[j]
            legs = psi.legs

            def mv(v, j=j, legs=legs):
                return heff1_dense(Lenv[j], Ws[j], Renv[j + 1], BlockTensor.unpack(v, legs, MPS_SIGNS)).pack()
            lam, xv, st = davidson(mv, psi.pack(), dav.get("max_iter", 40), dav.get("tol", 1e-12),
                                   restart_mask=mask_of(legs, MPS_SIGNS), seed=step)
            x = BlockTensor.unpack(xv, legs, MPS_SIGNS)
            if d == "right":
                # x(a, s, 1, c) = A(a, s, b) [S V^T](b, 1, c); S V^T goes into site j+1
                A, SV, _, _, _ = truncate(_with_dummy(x, 2), "right", cutoff=CANON_CUTOFF, m_max=1 << 60)
                mps[j] = A
                mps[j + 1] = _drop_dummy(merge(SV, mps[j + 1]), 1)
                Lenv[j + 1] = left_update_dense(Lenv[j], mps[j], Ws[j])
            else:
                # x(a, 1, s, c) = [U S](a, 1, b) B(b, s, c); U S goes into site j-1
                US, B, _, _, _ = truncate(_with_dummy(x, 1), "left", cutoff=CANON_CUTOFF, m_max=1 << 60)
                mps[j] = B
                mps[j - 1] = _drop_dummy(merge(mps[j - 1], US), 2)
                Renv[j] = right_update_dense(Renv[j + 1], mps[j], Ws[j])
            energies.append(lam)
            if log is not None:
                log.append({"sweep": sw, "site": j, "dir": d, "E": lam, "iters": st["iters"]})
            step += 1
        sweep_e.append(energies[-1])
    return energies, mps, sweep_e

