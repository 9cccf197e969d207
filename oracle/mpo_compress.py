"""Lossless SVD compression of an MPO (the paper compresses its MPOs by SVD
with a cutoff of 1e-13, Sec. VI-B; the electron MPO then has k = 26).

The MPO is treated as a chain of order-4 tensors W_j(w, s', s, w') whose bond
legs carry flux sectors (a channel's flux is the charge change already
applied to its left; W_j conserves it: f_w + q_s' - q_s - f_w' = 0).  Every
step below is a dense linear-algebra call on one flux sector at a time, so
the block structure is kept:

  0. the boundary channels are absorbed: W_0 keeps only its ``start`` row,
     W_{N-1} only its ``done`` column (both end bonds become one channel);
  1. left-to-right orthogonalisation: W_j as a matrix with rows (w, s', s)
     and columns w', per flux sector of w': X = U S V^T, W_j <- U (the
     columns with s > 1e-14 ||X|| of the sector matrix, the numerical null
     space dropped), W_{j+1} <- (S V^T) W_{j+1};
  2. right-to-left truncation: W_j as a matrix with rows w and columns
     (s', s, w'), per flux sector of w: X = U S V^T; the singular values of
     all sectors of the bond are pooled and those below cutoff * ||W_j||_F
     are dropped (after step 1 the sites left of j are orthonormal, so
     ||W_j||_F is the norm of the whole operator and these are its Schmidt
     values across the bond); W_j <- V^T, W_{j-1} <- W_{j-1} U S.

Readings (the paper gives only the cutoff): the cutoff is relative to the
Frobenius norm of the operator, in the same sense as the "sv" cutoff of the
state truncation; the orthogonalisation sweep drops the exact null space
(1e-14 relative), which changes nothing within rounding.

Checked against the dense matrix of the operator (mpo_to_dense_bonds) on
small lattices and by ED energies.
"""
import numpy as np


def _flux_of(leg):
    """Per-channel flux tuples of a leg [(flux, n), ...]."""
    out = []
    for f, n in leg:
        out += [tuple(f)] * n
    return out


def _leg_of(fluxes):
    """[(flux, n)] of a sector-major list of per-channel fluxes."""
    out = []
    for f in fluxes:
        if out and out[-1][0] == f:
            out[-1] = (f, out[-1][1] + 1)
        else:
            out.append((f, 1))
    return out


def _sub(a, b):
    return tuple(x - y for x, y in zip(a, b))


def _add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def compress_mpo(Ws, legs, phys, start, done, cutoff=1e-13):
    """Compress an MPO whose bond j has the channel leg legs[j] (N + 1 legs;
    a single leg [(flux, n), ...] means the same leg on every bond).

    Returns dict(W=[dense (k_j, d, d, k_{j+1})], legs=[N + 1 bond legs],
    start=0, done=0) with one channel on both end bonds."""
    N = len(Ws)
    pq = [tuple(q) for q, _ in phys]
    d = len(pq)
    if not isinstance(legs[0], list):      # one leg [(flux, n), ...] for every bond
        legs = [legs] * (N + 1)
    W = [np.array(w, dtype=np.float64) for w in Ws]
    bond_flux = [_flux_of(l) for l in legs]
    W[0] = W[0][start:start + 1]
    bond_flux[0] = [bond_flux[0][start]]
    W[N - 1] = W[N - 1][..., done:done + 1]
    bond_flux[N] = [bond_flux[N][done]]

    # 1. left-to-right orthogonalisation
    for j in range(N - 1):
        kl, kr = W[j].shape[0], W[j].shape[3]
        X = W[j].reshape(kl * d * d, kr)
        row_flux = [_sub(_add(bond_flux[j][w], pq[sp]), pq[s]) for w in range(kl) for sp in range(d)
                    for s in range(d)]
        new_cols, new_flux, R_rows = [], [], []
        for f in sorted(set(bond_flux[j + 1])):
            cols = [c for c in range(kr) if bond_flux[j + 1][c] == f]
            rows = [r for r in range(kl * d * d) if row_flux[r] == f]
            if not rows:
                continue
            Xf = X[np.ix_(rows, cols)]
            U, S, Vt = np.linalg.svd(Xf, full_matrices=False)
            keep = S > 1e-14 * max(np.linalg.norm(X), 1e-300)
            if not keep.any():
                continue
            Q = np.zeros((kl * d * d, int(keep.sum())))
            Q[rows, :] = U[:, keep]
            new_cols.append(Q)
            Rf = np.zeros((int(keep.sum()), kr))
            Rf[:, cols] = S[keep, None] * Vt[keep]
            R_rows.append(Rf)
            new_flux += [f] * int(keep.sum())
        Q = np.concatenate(new_cols, axis=1)
        R = np.concatenate(R_rows, axis=0)
        W[j] = Q.reshape(kl, d, d, -1)
        W[j + 1] = np.einsum("ab,bpsv->apsv", R, W[j + 1])
        bond_flux[j + 1] = new_flux

    # 2. right-to-left truncation
    for j in range(N - 1, 0, -1):
        kl, kr = W[j].shape[0], W[j].shape[3]
        X = W[j].reshape(kl, d * d * kr)
        col_flux = [_add(_sub(bond_flux[j + 1][w], pq[sp]), pq[s]) for sp in range(d) for s in range(d)
                    for w in range(kr)]
        norm = np.linalg.norm(X)
        new_rows, new_flux, US_cols = [], [], []
        for f in sorted(set(bond_flux[j])):
            rows = [r for r in range(kl) if bond_flux[j][r] == f]
            cols = [c for c in range(d * d * kr) if col_flux[c] == f]
            if not cols:
                continue
            Xf = X[np.ix_(rows, cols)]
            U, S, Vt = np.linalg.svd(Xf, full_matrices=False)
            keep = S >= cutoff * norm
            if not keep.any():
                continue
            Vk = np.zeros((int(keep.sum()), d * d * kr))
            Vk[:, cols] = Vt[keep]
            new_rows.append(Vk)
            USf = np.zeros((kl, int(keep.sum())))
            USf[rows, :] = U[:, keep] * S[keep][None, :]
            US_cols.append(USf)
            new_flux += [f] * int(keep.sum())
        Vt_all = np.concatenate(new_rows, axis=0)
        US = np.concatenate(US_cols, axis=1)
        W[j] = Vt_all.reshape(-1, d, d, kr)
        W[j - 1] = np.einsum("apsv,vb->apsb", W[j - 1], US)
        bond_flux[j] = new_flux
    return {"W": W, "legs": [_leg_of(f) for f in bond_flux], "start": 0, "done": 0}


def mpo_to_dense_bonds(W, start, done):
    """Dense matrix of an MPO given as site tensors with any bond dimensions
    (left boundary channel ``start`` on bond 0, right ``done`` on bond N)."""
    d = W[0].shape[1]
    cur = W[0][start].reshape(d, d, -1)
    for Wj in W[1:]:
        D = cur.shape[0]
        cur = np.einsum("abw,wpsv->apbsv", cur, Wj).reshape(D * d, D * d, -1)
    return cur[:, :, done]
