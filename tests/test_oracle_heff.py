"""Pins of the oracle's effective Hamiltonian, eigensolver, truncation,
environments and gradients against mathematics and exact diagonalisation."""
import numpy as np
import pytest

import synth
from synth.blocks import mps_block
from oracle import ed, grad
from oracle.blocks import BlockTensor, canonical_layout, block_shape
from oracle.dmrg import random_mps, right_canonicalize, mask_of
from oracle.eig import davidson, lanczos
from oracle.env import (left_boundary, right_boundary, left_update_dense, right_update_dense,
                        left_update_blocks, right_update_blocks, merge)
from oracle.heff import (bond_operands, heff_dense, heff_blocks, heff_diagonal, w_tensor, PSI_SIGNS,
                         ENV_SIGNS, useful_flops)
from oracle.truncate import truncate


def small_bond(m=48, k=14, seed=5):
    return bond_operands(synth.c2_bond(m=m, k=k, seed=seed))


def rand_like(bt, seed):
    r = np.random.default_rng(seed)
    out = bt.copy()
    for k in out.blocks:
        out.blocks[k] = r.standard_normal(out.blocks[k].shape)
    return out


# ------------------------------------------------------------- H_eff ---------
def test_o1_equals_o2():
    L, W1, W2, R, psi = small_bond()
    a, b = heff_dense(L, W1, W2, R, psi), heff_blocks(L, W1, W2, R, psi)
    scale = max(np.abs(v).max() for v in a.blocks.values())
    assert max(np.abs(a.blocks[k] - b.blocks[k]).max() for k in a.blocks) < 1e-13 * scale


def test_heff_symmetric_for_hermitian_structured_environments():
    L, W1, W2, R, psi = small_bond(seed=9)
    x, y = rand_like(psi, 1), rand_like(psi, 2)
    lhs = y.dot(heff_blocks(L, W1, W2, R, x))
    rhs = x.dot(heff_blocks(L, W1, W2, R, y))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_heff_linear():
    L, W1, W2, R, psi = small_bond(m=32)
    x, y = rand_like(psi, 3), rand_like(psi, 4)
    h = lambda t: heff_blocks(L, W1, W2, R, t)
    lhs = h(x.scale(2.0).axpy(-3.0, y))
    rhs = h(x).scale(2.0).axpy(-3.0, h(y))
    assert max(np.abs(lhs.blocks[k] - rhs.blocks[k]).max() for k in lhs.blocks) < 1e-12


def test_identity_operator_returns_psi_exactly():
    leg = synth.spin_bond_leg(40)
    wl = [((0,), 1)]
    phys = synth.SPIN_PHYS
    Ld = np.zeros((40, 1, 40)); Ld[:, 0, :] = np.eye(40)
    L = BlockTensor.from_dense(Ld, [leg, wl, leg], ENV_SIGNS)
    W = w_tensor(np.eye(2).reshape(1, 2, 2, 1), wl, phys, wl)
    psi = BlockTensor.from_fn([leg, phys, phys, leg], PSI_SIGNS,
                              lambda k: synth.gaussian_block(1, 2, k, block_shape(
                                  [leg, phys, phys, leg], k)))
    out = heff_blocks(L, W, W, L, psi)
    assert all(np.array_equal(out.blocks[k], psi.blocks[k]) for k in psi.blocks)


def test_sz_only_operator_is_diagonal():
    # H = Sz_1 Sz_2 on the two sites, identity environments: diagonal, eigen-
    # values (2Sz1)(2Sz2)/4 per element
    leg = synth.spin_bond_leg(24)
    wl = [((0,), 3)]                        # start, Sz strand, done
    Id = np.eye(2); sz = np.diag([-0.5, 0.5])
    W1 = np.zeros((3, 2, 2, 3)); W1[0, :, :, 1] = sz; W1[2, :, :, 2] = Id
    W2 = np.zeros((3, 2, 2, 3)); W2[1, :, :, 2] = sz
    Ld = np.zeros((24, 3, 24)); Ld[:, 0, :] = np.eye(24)
    Rd = np.zeros((24, 3, 24)); Rd[:, 2, :] = np.eye(24)
    phys = synth.SPIN_PHYS
    L = BlockTensor.from_dense(Ld, [leg, wl, leg], ENV_SIGNS)
    R = BlockTensor.from_dense(Rd, [leg, wl, leg], ENV_SIGNS)
    psi = BlockTensor.from_fn([leg, phys, phys, leg], PSI_SIGNS,
                              lambda k: synth.gaussian_block(4, 2, k, block_shape(
                                  [leg, phys, phys, leg], k)))
    out = heff_blocks(L, w_tensor(W1, wl, phys, wl), w_tensor(W2, wl, phys, wl), R, psi)
    for (ia, i1, i2, ic), v in psi.blocks.items():
        z = (phys[i1][0][0] * phys[i2][0][0]) / 4.0
        assert np.allclose(out.blocks[(ia, i1, i2, ic)], z * v, atol=1e-15, rtol=0)


def _center_chain(n, j, m0=8, seed=0):
    """MPS of an n-site chain with orthogonality centre on sites (j, j+1)."""
    b = synth.chain_bonds(n, 1.0)
    mpo = synth.heisenberg_mpo(n, b)
    mps = right_canonicalize(random_mps(mpo, n, (0,), m0, seed, mps_block))
    for s in range(j):
        A, B, _, _, _ = truncate(merge(mps[s], mps[s + 1]), "right")
        mps[s], mps[s + 1] = A, B
    return b, mpo, mps


def test_heff_equals_projected_hamiltonian():
    """K = Q^T H Q (Sec. II-C) with Q built from the canonical MPS and H from
    exact diagonalisation; pins H_eff, the environments, the boundaries and
    the MPO together."""
    n, j = 6, 2
    b, mpo, mps = _center_chain(n, j)
    wl = mpo.w_leg()
    Ws = [w_tensor(W, wl, mpo.phys, wl) for W in mpo.W]
    Lenv = left_boundary(wl, mpo.start, 1)
    for s in range(j):
        Lenv = left_update_dense(Lenv, mps[s], Ws[s])
    Renv = right_boundary(wl, mpo.done, (0,))
    for s in range(n - 1, j + 1, -1):
        Renv = right_update_dense(Renv, mps[s], Ws[s])
    # left basis Lb[sigma_0 .. sigma_{j-1}, a], right basis Rb[c, sigma_{j+2} ..]
    Lb = mps[0].to_dense()[0]
    for s in range(1, j):
        Lb = np.einsum("...b,bsc->...sc", Lb, mps[s].to_dense())
    Rb = mps[n - 1].to_dense()[:, :, 0]
    for s in range(n - 2, j + 1, -1):
        Rb = np.einsum("bsc,c...->bs...", mps[s].to_dense(), Rb)
    theta = merge(mps[j], mps[j + 1])
    x = rand_like(theta, 11)
    X = x.to_dense()                                           # (a, s, s, c)
    Lf = Lb.reshape(-1, Lb.shape[-1])                          # (2^j, a)
    Rf = Rb.reshape(Rb.shape[0], -1)                           # (c, 2^(n-j-2))
    vec = np.einsum("la,astc,cr->lstr", Lf, X, Rf).reshape(-1)
    H = ed.heisenberg_full(n, b)
    Hv = (H @ vec).reshape(Lf.shape[0], 2, 2, Rf.shape[1])
    K_x = np.einsum("la,lstr,cr->astc", Lf, Hv, Rf)
    got = heff_dense(Lenv, Ws[j], Ws[j + 1], Renv, x).to_dense()
    assert np.abs(got - K_x).max() < 1e-13 * max(1.0, np.abs(K_x).max())


def test_useful_flops_of_the_mid_chain_bond_model():
    # the flop count is a property of the block structure alone
    L, W1, W2, R, psi = bond_operands(synth.c2_bond(m=128, k=14, seed=1))
    f = useful_flops(L, W1, W2, R, psi)
    # independent count from the sector model: S1 = sum over psi blocks and L
    # blocks sharing the ket sector, S3 the same over R (symmetric legs here)
    leg, wl = L.legs[0], L.legs[1]
    s1 = 0
    for (ia, i1, i2, ic) in psi.blocks:
        for iw, (fw, nw) in enumerate(wl):
            q = leg[ia][0][0] + fw[0]
            if any(c[0] == q for c, _ in leg):
                ib = [c[0] for c, _ in leg].index(q)
                s1 += 2 * leg[ib][1] * nw * leg[ia][1] * leg[ic][1]
    assert f >= s1          # S3 >= 0 on top of S1
    assert f == 2 * s1      # the problem is left/right symmetric


# -------------------------------------------------------- eigensolvers ------
def _explicit(L, W1, W2, R, psi):
    legs = psi.legs
    mask = mask_of(legs, PSI_SIGNS)
    idx = np.nonzero(mask)[0]
    n = mask.size

    def mv(v):
        return heff_blocks(L, W1, W2, R, BlockTensor.unpack(v, legs, PSI_SIGNS)).pack()
    H = np.zeros((idx.size, idx.size))
    for c, i in enumerate(idx):
        e = np.zeros(n); e[i] = 1.0
        H[:, c] = mv(e)[idx]
    return H, mv, mask


def test_davidson_matches_dense_eigh():
    L, W1, W2, R, psi = small_bond(m=16, k=5)
    H, mv, mask = _explicit(L, W1, W2, R, psi)
    assert np.abs(H - H.T).max() < 1e-12
    lam, x, st = davidson(mv, psi.pack(), max_iter=H.shape[0], tol=1e-10, restart_mask=mask)
    e = np.linalg.eigvalsh(H)[0]
    assert st["converged"] and abs(lam - e) < 1e-10 * abs(e)
    r = mv(x) - lam * x
    assert np.linalg.norm(r) < 1e-9


def test_davidson_ritz_values_equal_lanczos_krylov():
    L, W1, W2, R, psi = small_bond(m=64, k=14)

    def mv(v):
        return heff_blocks(L, W1, W2, R, BlockTensor.unpack(v, psi.legs, PSI_SIGNS)).pack()
    rec = []
    davidson(mv, psi.pack(), max_iter=12, tol=0.0, record=rec)
    lz = lanczos(mv, psi.pack(), 12)
    assert np.allclose(rec, lz, rtol=1e-10, atol=0)
    assert all(b <= a + 1e-12 for a, b in zip(rec, rec[1:]))      # monotone Ritz values


def test_davidson_breakdown_triggers_seeded_restart():
    # identity operator: q = 0 after the first step, so the routine must draw
    # the seeded random vector instead of dividing by zero
    n = 64
    mask = np.ones(n, dtype=bool); mask[50:] = False
    x0 = np.zeros(n); x0[:50] = 1.0
    lam, x, st = davidson(lambda v: 2.5 * v, x0, max_iter=3, tol=-1.0, restart_mask=mask, seed=4)
    assert st["restarts"] >= 1 and abs(lam - 2.5) < 1e-14
    # an exact eigenvector of a non-trivial operator restarts and still ends right
    D = np.diag(np.arange(1.0, n + 1.0))
    e0 = np.zeros(n); e0[0] = 1.0
    lam, x, st = davidson(lambda v: D @ v, e0, max_iter=4, tol=-1.0, seed=1)
    assert st["restarts"] >= 1 and abs(lam - 1.0) < 1e-14 and abs(abs(x[0]) - 1) < 1e-14


def test_davidson_stops_when_basis_spans_the_space():
    """A basis as large as the allowed space gives the exact eigenpair: with
    max_iter above the dimension and an unreachable tolerance the routine
    stops after dim products, without restarts, at the dense lowest pair."""
    L, W1, W2, R, psi = small_bond(m=4, k=5)
    H, mv, mask = _explicit(L, W1, W2, R, psi)
    dim = H.shape[0]
    assert dim < 64
    lam, x, st = davidson(mv, psi.pack(), max_iter=64, tol=-1.0, restart_mask=mask)
    w, U = np.linalg.eigh(H)
    assert st["iters"] == dim and st["restarts"] == 0
    assert abs(lam - w[0]) < 1e-12 * abs(w[0])
    assert abs(abs(float(x[mask] @ U[:, 0])) - 1.0) < 1e-10


def test_heff_diagonal_equals_explicit_matrix_diagonal():
    """The diagonal used by the preconditioner is the diagonal of the explicit
    matrix (brute force column by column), for a spin and an electron bond,
    and zero on the padding."""
    L, W1, W2, R, psi = bond_operands(synth.c2_bond(m=16, k=5, seed=5))
    H, mv, mask = _explicit(L, W1, W2, R, psi)
    d = heff_diagonal(L, W1, W2, R, psi.legs)
    assert np.abs(d[mask] - np.diag(H)).max() < 1e-13 * np.abs(H).max()
    assert np.all(d[~mask] == 0.0)
    # electron bond: sampled entries <e_i|H e_i> through the block-loop product
    L, W1, W2, R, psi = bond_operands(synth.c4_bond(m=40, k=10, seed=2))
    mask = mask_of(psi.legs, PSI_SIGNS)
    d = heff_diagonal(L, W1, W2, R, psi.legs)
    assert np.all(d[~mask] == 0.0)
    idx = np.random.default_rng(1).choice(np.nonzero(mask)[0], 24, replace=False)
    for i in idx:
        e = np.zeros(mask.size)
        e[i] = 1.0
        hi = heff_blocks(L, W1, W2, R, BlockTensor.unpack(e, psi.legs, PSI_SIGNS)).pack()[i]
        assert abs(hi - d[i]) <= 1e-13 * max(1.0, abs(hi))


def test_restarted_davidson_converges_to_dense_lowest():
    """Bounded basis (6 vectors, thick restart to 2 + 1): the restarts happen,
    the Ritz values never increase (the current Ritz vector is always kept),
    and the solve ends at the dense lowest eigenpair."""
    L, W1, W2, R, psi = small_bond(m=24, k=14, seed=3)
    H, mv, mask = _explicit(L, W1, W2, R, psi)
    rec = []
    lam, x, st = davidson(mv, psi.pack(), max_iter=400, tol=1e-10, restart_mask=mask, basis=6, keep=2,
                          record=rec)
    w, U = np.linalg.eigh(H)
    assert st["converged"] and st["thick_restarts"] >= 3
    assert abs(lam - w[0]) < 1e-10 * abs(w[0])
    assert abs(abs(float(x[mask] @ U[:, 0])) - 1.0) < 1e-10
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(rec, rec[1:]))
    # keeping more vectors never needs more products on this problem
    _, _, st_wide = davidson(mv, psi.pack(), max_iter=400, tol=1e-10, restart_mask=mask, basis=12, keep=4)
    assert st_wide["iters"] <= st["iters"]


def test_restart_with_smallest_basis_reaches_lowest_value():
    """keep + 2 == basis (a restart after every product) on a diagonal
    operator started from a vector with weight on every state: the solve
    still reaches the exact lowest value (the kept pair spans the current and
    the previous Ritz vector, or the newest direction when they coincide)."""
    D = np.diag([1.0, 2.0, 3.0, 10.0])
    x0 = np.array([1.0, 1.0, 1.0, 1.0])
    lam, x, st = davidson(lambda v: D @ v, x0, max_iter=40, tol=1e-12, basis=3, keep=1)
    assert st["converged"] and abs(lam - 1.0) < 1e-12


def test_preconditioned_davidson_converges_and_helps_on_diagonal_dominance():
    """Davidson's diagonal preconditioner: on the effective Hamiltonian it
    still ends at the dense lowest pair; on a strongly diagonally dominant
    symmetric matrix (where the diagonal is a good approximation of the
    operator) it needs far fewer products than the unpreconditioned routine."""
    L, W1, W2, R, psi = small_bond(m=24, k=14, seed=3)
    H, mv, mask = _explicit(L, W1, W2, R, psi)
    d = heff_diagonal(L, W1, W2, R, psi.legs)
    lam, x, st = davidson(mv, psi.pack(), max_iter=400, tol=1e-10, restart_mask=mask, precond=d)
    w = np.linalg.eigvalsh(H)
    assert st["converged"] and abs(lam - w[0]) < 1e-10 * abs(w[0])
    lam2, _, st2 = davidson(mv, psi.pack(), max_iter=400, tol=1e-10, restart_mask=mask, precond=d, basis=8,
                            keep=3)
    assert st2["converged"] and abs(lam2 - w[0]) < 1e-10 * abs(w[0])
    r = np.random.default_rng(7)
    n = 300
    A = r.standard_normal((n, n)) * 0.01
    A = A + A.T + np.diag(np.arange(n, dtype=float))
    wA = np.linalg.eigvalsh(A)[0]
    x0 = np.full(n, 1e-3)       # near the lowest diagonal state
    x0[0] = 1.0
    lp, _, sp = davidson(lambda v: A @ v, x0, max_iter=200, tol=1e-10, precond=np.diag(A).copy())
    lu, _, su = davidson(lambda v: A @ v, x0, max_iter=200, tol=1e-10)
    assert sp["converged"] and abs(lp - wA) < 1e-10 * max(1.0, abs(wA))
    assert sp["iters"] * 3 < su["iters"] or not su["converged"]


# ---------------------------------------------------------- truncation -------
def _theta(m=40, seed=3):
    leg = synth.spin_bond_leg(m)
    phys = synth.SPIN_PHYS
    legs = [leg, phys, phys, leg]
    return BlockTensor.from_fn(legs, PSI_SIGNS, lambda k: synth.gaussian_block(
        seed, 9, k, block_shape(legs, k)))


def _dense_matrix(theta):
    d = theta.to_dense()
    return d.reshape(d.shape[0] * d.shape[1], -1)


def test_truncation_singular_values_equal_dense_svd():
    th = _theta()
    A, B, leg, kept, disc = truncate(th, "right", cutoff=0.0)
    s = np.linalg.svd(_dense_matrix(th), compute_uv=False)
    s = s[s > 1e-12 * s[0]]
    assert np.allclose(np.sort(kept)[::-1], s[:kept.size], rtol=1e-12)
    assert kept.size == s.size


@pytest.mark.parametrize("direction", ["right", "left"])
def test_truncation_eckart_young_and_orthogonality(direction):
    th = _theta(seed=5)
    A, B, leg, kept, disc = truncate(th, direction, m_max=25)
    approx = merge(A, B)
    err = sum(float(np.sum((th.blocks[k] - approx.blocks[k]) ** 2)) for k in th.blocks)
    assert abs(err - disc) < 1e-10 * max(disc, 1e-300) + 1e-13
    s = np.linalg.svd(_dense_matrix(th), compute_uv=False)
    assert abs(disc - np.sum(s[kept.size:] ** 2)) < 1e-10 * disc
    if direction == "right":
        Ad = A.to_dense(); G = np.einsum("asb,asc->bc", Ad, Ad)
    else:
        Bd = B.to_dense(); G = np.einsum("bsc,dsc->bd", Bd, Bd)
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12


def test_truncation_degenerate_group_and_cutoff_modes():
    from oracle.truncate import select
    # values 3, 2, 2(1+1e-13), 1 with m_max = 2: the cut would split the pair
    counts, disc, kept = select([np.array([3.0, 2.0]), np.array([2.0 * (1 + 1e-13), 1.0])],
                                0.0, "sv", 2, 1e-10)
    assert counts == [1, 0] and abs(disc - (4.0 + 4.0 * (1 + 1e-13) ** 2 + 1.0)) < 1e-12
    # sv cutoff is relative to ||theta||
    counts, _, _ = select([np.array([1.0, 1e-3, 1e-9])], 1e-6, "sv", 100, 1e-10)
    assert counts == [2]
    counts, disc, _ = select([np.array([1.0, 1e-3, 1e-9])], 1e-5, "weight", 100, 1e-10)
    assert counts == [1] and abs(disc - (1e-6 + 1e-18)) < 1e-20


def test_truncation_sign_gauge():
    th = _theta(seed=8)
    A, B, _, _, _ = truncate(th, "right")
    Ad = {}
    for (ia, i1, ib), v in A.blocks.items():
        Ad.setdefault(ib, []).append(v.reshape(-1, v.shape[-1]))
    for ib, parts in Ad.items():
        U = np.concatenate(parts, axis=0)
        for j in range(U.shape[1]):
            i = int(np.argmax(np.abs(U[:, j])))
            assert U[i, j] > 0


# ---------------------------------------------------------- environments ----
def test_environment_updates_dense_equals_blocks():
    b, mpo, mps = _center_chain(8, 4, m0=12, seed=2)
    wl = mpo.w_leg()
    Ws = [w_tensor(W, wl, mpo.phys, wl) for W in mpo.W]
    L = left_boundary(wl, mpo.start, 1)
    R = right_boundary(wl, mpo.done, (0,))
    for s in range(3):
        L1, L2 = left_update_dense(L, mps[s], Ws[s]), left_update_blocks(L, mps[s], Ws[s])
        assert max(np.abs(L1.blocks[k] - L2.blocks[k]).max() for k in L1.blocks) < 1e-13
        L = L1
    for s in range(7, 5, -1):
        R1, R2 = right_update_dense(R, mps[s], Ws[s]), right_update_blocks(R, mps[s], Ws[s])
        assert max(np.abs(R1.blocks[k] - R2.blocks[k]).max() for k in R1.blocks) < 1e-13
        R = R1


# ------------------------------------------------------------- gradients ----
def test_gradient_euler_identities_and_fd():
    L, W1, W2, R, psi = small_bond(m=24, k=8, seed=2)
    E = grad.energy(L, W1, W2, R, psi)
    assert abs(E - psi.dot(heff_blocks(L, W1, W2, R, psi))) < 1e-12 * abs(E)
    g = grad.gradients(L, W1, W2, R, psi)
    for name, X in (("L", L), ("W1", W1), ("W2", W2), ("R", R)):
        assert abs(g[name].dot(X) - E) < 1e-11 * abs(E), name
    assert abs(g["psi"].dot(psi) - 2 * E) < 1e-11 * abs(E)
    # central finite difference along a random direction of L
    dL = rand_like(L, 7)
    h = 1e-6
    Ep = grad.energy(L.axpy(h, dL), W1, W2, R, psi)
    Em = grad.energy(L.axpy(-h, dL), W1, W2, R, psi)
    assert abs((Ep - Em) / (2 * h) - g["L"].dot(dL)) < 1e-6 * abs(g["L"].dot(dL))
    dp = rand_like(psi, 8)
    Ep = grad.energy(L, W1, W2, R, psi.axpy(h, dp))
    Em = grad.energy(L, W1, W2, R, psi.axpy(-h, dp))
    assert abs((Ep - Em) / (2 * h) - g["psi"].dot(dp)) < 1e-6 * abs(g["psi"].dot(dp))


def test_gradient_at_eigenvector_is_2_lambda_psi():
    L, W1, W2, R, psi = small_bond(m=16, k=5, seed=4)
    _, mv, mask = _explicit(L, W1, W2, R, psi)
    lam, x, st = davidson(mv, psi.pack(), max_iter=200, tol=1e-11, restart_mask=mask)
    X = BlockTensor.unpack(x, psi.legs, PSI_SIGNS)
    g = grad.gradients(L, W1, W2, R, X)["psi"]
    assert max(np.abs(g.blocks[k] - 2 * lam * X.blocks[k]).max() for k in g.blocks) < 1e-9
