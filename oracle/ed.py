"""Exact diagonalisation references (textbook constructions, independent of the
MPO builders).

Spin-1/2 Heisenberg H = sum J_ij S_i . S_j (Sec. V) and the Hubbard model
H = -sum t_ij (c+_is c_js + h.c.) + U sum n_iu n_id (Sec. V).

Full-space matrices use the product basis with site 0 most significant and
the local orders: spin 0 = down, 1 = up; electron local index 2 n_up + n_dn.
Fermion operators are Jordan-Wigner strings over the mode order
(0 up, 0 down, 1 up, ...): c_p = Z x ... x Z x b x I x ... x I on 2N two-level
modes, b = |0><1|, Z = diag(1, -1).  Sector Hamiltonians are built on
occupation bit strings with the fermionic sign (-1)^(occupied modes before p).
"""
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _kron_all(mats):
    out = np.array([[1.0]])
    for m in mats:
        out = np.kron(out, m)
    return out


def heisenberg_full(n, bonds):
    sz = np.diag([-0.5, 0.5])
    splus = np.array([[0.0, 0.0], [1.0, 0.0]])
    sminus = splus.T
    I = np.eye(2)
    H = np.zeros((2 ** n, 2 ** n))

    def op(i, m):
        return _kron_all([m if k == i else I for k in range(n)])

    for (i, j), J in bonds.items():
        H += J * (op(i, sz) @ op(j, sz) + 0.5 * (op(i, splus) @ op(j, sminus) +
                                                   op(i, sminus) @ op(j, splus)))
    return H


def heisenberg_sector(n, bonds, n_up):
    """Sparse H in the sector with n_up up spins (2Sz = 2 n_up - n)."""
    states = [s for s in range(2 ** n) if bin(s).count("1") == n_up]
    index = {s: i for i, s in enumerate(states)}
    rows, cols, vals = [], [], []
    bit = lambda s, i: (s >> (n - 1 - i)) & 1      # site 0 = most significant
    for a, s in enumerate(states):
        diag = 0.0
        for (i, j), J in bonds.items():
            bi, bj = bit(s, i), bit(s, j)
            diag += J * (bi - 0.5) * (bj - 0.5)
            if bi != bj:
                t = s ^ (1 << (n - 1 - i)) ^ (1 << (n - 1 - j))
                rows.append(index[t]); cols.append(a); vals.append(0.5 * J)
        rows.append(a); cols.append(a); vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(states), len(states)))


def fermion_ops(n_modes):
    b = np.array([[0.0, 1.0], [0.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    I = np.eye(2)
    return [_kron_all([Z] * p + [b] + [I] * (n_modes - p - 1)) for p in range(n_modes)]


def hubbard_full(n, hops, U):
    c = fermion_ops(2 * n)
    dim = 4 ** n
    H = np.zeros((dim, dim))
    for (i, j), t in hops.items():
        for s in (0, 1):
            p, q = 2 * i + s, 2 * j + s
            H += -t * (c[p].T @ c[q] + c[q].T @ c[p])
    for i in range(n):
        nu = c[2 * i].T @ c[2 * i]
        nd = c[2 * i + 1].T @ c[2 * i + 1]
        H += U * (nu @ nd)
    return H


def hubbard_sector(n, hops, U, n_up, n_dn):
    nm = 2 * n
    up_modes = [2 * i for i in range(n)]
    dn_modes = [2 * i + 1 for i in range(n)]
    states = []
    for ups in itertools.combinations(up_modes, n_up):
        for dns in itertools.combinations(dn_modes, n_dn):
            s = 0
            for p in ups + dns:
                s |= 1 << (nm - 1 - p)
            states.append(s)
    states.sort()
    index = {s: i for i, s in enumerate(states)}
    occ = lambda s, p: (s >> (nm - 1 - p)) & 1
    rows, cols, vals = [], [], []
    for a, s in enumerate(states):
        diag = sum(U for i in range(n) if occ(s, 2 * i) and occ(s, 2 * i + 1))
        rows.append(a); cols.append(a); vals.append(diag)
        for (i, j), t in hops.items():
            for sg in (0, 1):
                for p, q in ((2 * i + sg, 2 * j + sg), (2 * j + sg, 2 * i + sg)):
                    # c+_p c_q |s>
                    if not occ(s, q) or (occ(s, p) and p != q):
                        continue
                    sign = (-1) ** sum(occ(s, r) for r in range(q))
                    s1 = s ^ (1 << (nm - 1 - q))
                    sign *= (-1) ** sum(occ(s1, r) for r in range(p))
                    s2 = s1 | (1 << (nm - 1 - p))
                    rows.append(index[s2]); cols.append(a); vals.append(-t * sign)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(states), len(states)))


def lowest(H):
    if H.shape[0] <= 4000:
        Hd = H.toarray() if sp.issparse(H) else H
        return float(np.linalg.eigvalsh(Hd)[0])
    v0 = np.ones(H.shape[0]) / np.sqrt(H.shape[0])
    return float(spla.eigsh(H, k=1, which="SA", v0=v0, tol=1e-14)[0][0])
