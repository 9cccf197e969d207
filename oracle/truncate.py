"""SVD split of the two-site tensor (Sec. II-C, Fig. 1e; Sec. IV-A).

The order-4 tensor theta(a, s1, s2, c) is "wrapped" into one matrix per charge
q of the new bond: rows are the (a, s1) pairs with q_a + q_s1 = q, columns the
(s2, c) pairs with q_c - q_s2 = q, each in lexicographic order of their sector
indices and then row-major inside the block.  Each matrix is decomposed with a
plain SVD; the singular values of all charges are pooled and truncated; the
singular values are absorbed in the direction of the sweep.

Readings where the paper is silent or loose:
  * cutoff_mode 'sv' (default; "removes all singular values below 1e-12"):
    discard s < cutoff * ||theta||;  'weight': discard the smallest values
    whose squares sum to at most cutoff * ||theta||^2;
  * then keep at most m_max, largest first; ties in the global order are
    broken by (charge index, index within the charge);
  * degenerate groups: if the first discarded value s_d and a kept value v
    satisfy v - s_d <= degen_rtol * v, v is discarded too (so a cut never
    splits a multiplet); if that would discard everything, the plain cut is
    kept;
  * sign gauge: in every kept singular pair the entry of u with the largest
    magnitude (the first, in row order, among entries within 1e-10 relative of
    the maximum) is made positive, v flips with it;
  * discarded weight = sum of the squares of the discarded values.
"""
import numpy as np

from .blocks import BlockTensor
from .heff import MPS_SIGNS


def _sectors(theta):
    a, s1, s2, c = theta.legs
    r = len(a[0][0])
    add = lambda x, y: tuple(x[i] + y[i] for i in range(r))
    sub = lambda x, y: tuple(x[i] - y[i] for i in range(r))
    rows, cols = {}, {}
    for ia in range(len(a)):
        for i1 in range(len(s1)):
            rows.setdefault(add(a[ia][0], s1[i1][0]), []).append((ia, i1))
    for i2 in range(len(s2)):
        for ic in range(len(c)):
            cols.setdefault(sub(c[ic][0], s2[i2][0]), []).append((i2, ic))
    qs = sorted(q for q in rows if q in cols)
    return [(q, rows[q], cols[q]) for q in qs]


def wrap(theta):
    """[(q, row_keys, col_keys, matrix)] per charge, ascending q."""
    a, s1, s2, c = theta.legs
    out = []
    for q, rk, ck in _sectors(theta):
        rdim = [a[ia][1] * s1[i1][1] for ia, i1 in rk]
        cdim = [s2[i2][1] * c[ic][1] for i2, ic in ck]
        Mq = np.zeros((sum(rdim), sum(cdim)))
        r0 = 0
        for (ia, i1), rd in zip(rk, rdim):
            c0 = 0
            for (i2, ic), cd in zip(ck, cdim):
                blk = theta.blocks.get((ia, i1, i2, ic))
                if blk is not None:
                    Mq[r0:r0 + rd, c0:c0 + cd] = blk.reshape(rd, cd)
                c0 += cd
            r0 += rd
        out.append((q, rk, ck, Mq))
    return out


def select(svals_per_sector, cutoff, cutoff_mode, m_max, degen_rtol):
    """Global kept set -> list of kept counts per sector; discarded weight."""
    pool = []
    for si, s in enumerate(svals_per_sector):
        for j, v in enumerate(s):
            pool.append((-float(v), si, j))
    pool.sort()
    vals = np.array([-p[0] for p in pool])
    total2 = float(np.sum(vals ** 2))
    norm = np.sqrt(total2)
    if cutoff_mode == "sv":
        n_keep = int(np.sum(vals >= cutoff * norm)) if vals.size else 0
    elif cutoff_mode == "weight":
        n_keep = vals.size
        acc = 0.0
        while n_keep > 0 and acc + vals[n_keep - 1] ** 2 <= cutoff * total2:
            acc += vals[n_keep - 1] ** 2
            n_keep -= 1
    else:
        raise ValueError("cutoff_mode must be 'sv' or 'weight'")
    n_keep = min(n_keep, int(m_max))
    if 0 < n_keep < vals.size:
        sd = vals[n_keep]
        n2 = n_keep
        while n2 > 0 and vals[n2 - 1] - sd <= degen_rtol * vals[n2 - 1]:
            n2 -= 1
        if n2 > 0:
            n_keep = n2
    counts = [0] * len(svals_per_sector)
    for _, si, _j in pool[:n_keep]:
        counts[si] += 1
    discarded = float(np.sum(vals[n_keep:] ** 2))
    return counts, discarded, vals[:n_keep]


def fix_gauge(U, Vt):
    U, Vt = U.copy(), Vt.copy()
    for j in range(U.shape[1]):
        col = np.abs(U[:, j])
        mx = col.max()
        i = int(np.nonzero(col >= mx * (1.0 - 1e-10))[0][0])
        if U[i, j] < 0:
            U[:, j] *= -1.0
            Vt[j, :] *= -1.0
    return U, Vt


def truncate(theta, direction="right", cutoff=0.0, cutoff_mode="sv", m_max=1 << 60,
             degen_rtol=1e-10):
    """Split theta(a,s1,s2,c) into A(a,s1,b) B(b,s2,c).

    direction 'right': A = U, B = S V^T (sweeping right); 'left': A = U S, B = V^T.
    Returns (A, B, new_leg, kept singular values (descending), discarded weight).
    """
    sec = wrap(theta)
    decs = []
    for q, rk, ck, Mq in sec:
        U, S, Vt = np.linalg.svd(Mq, full_matrices=False)
        decs.append((U, S, Vt))
    counts, disc, kept = select([d[1] for d in decs], cutoff, cutoff_mode, m_max, degen_rtol)
    a, s1, s2, c = theta.legs
    new_leg = [(q, n) for (q, _, _, _), n in zip(sec, counts) if n > 0]
    A = BlockTensor([a, s1, new_leg], MPS_SIGNS)
    B = BlockTensor([new_leg, s2, c], MPS_SIGNS)
    ib = 0
    for (q, rk, ck, _), (U, S, Vt), n in zip(sec, decs, counts):
        if n == 0:
            continue
        U, Vt = fix_gauge(U[:, :n], Vt[:n, :])
        S = S[:n]
        if direction == "right":
            Vt = S[:, None] * Vt
        else:
            U = U * S[None, :]
        r0 = 0
        for ia, i1 in rk:
            rd = a[ia][1] * s1[i1][1]
            A.blocks[(ia, i1, ib)] = U[r0:r0 + rd, :].reshape(a[ia][1], s1[i1][1], n)
            r0 += rd
        c0 = 0
        for i2, ic in ck:
            cd = s2[i2][1] * c[ic][1]
            B.blocks[(ib, i2, ic)] = Vt[:, c0:c0 + cd].reshape(n, s2[i2][1], c[ic][1])
            c0 += cd
        ib += 1
    return A, B, new_leg, kept, disc
