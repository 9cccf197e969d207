"""Two-site DMRG sweeps of the oracle against exact diagonalisation and closed
forms (the paper prints no energies, so every pin is ED or mathematics)."""
import numpy as np

import synth
from synth.blocks import mps_block
from oracle import ed
from oracle.dmrg import random_mps, dmrg, dmrg1

DAV = {"max_iter": 40, "tol": 1e-12}


def run(mpo, n, target, m, sweeps, m0=16, seed=0, heff="dense", cutoff=1e-10):
    mps = random_mps(mpo, n, target, m0, seed, mps_block)
    log = []
    E, _, swe, disc = dmrg(mpo, mps, sweeps, m, cutoff=cutoff, dav=DAV, heff=heff, log=log)
    return E, swe, disc, log


def test_closed_form_two_and_three_site_chains():
    _, swe, _, _ = run(synth.heisenberg_mpo(2, synth.chain_bonds(2)), 2, (0,), 8, 2)
    assert abs(swe[-1] + 0.75) < 1e-13
    _, swe, _, _ = run(synth.heisenberg_mpo(3, synth.chain_bonds(3)), 3, (1,), 8, 2)
    assert abs(swe[-1] + 1.0) < 1e-13


def test_two_site_hubbard_closed_form():
    U = 8.0
    _, swe, _, _ = run(synth.hubbard_mpo(2, synth.chain_bonds(2), U), 2, (2, 0), 8, 2)
    assert abs(swe[-1] - (U - np.sqrt(U * U + 16.0)) / 2.0) < 1e-13


def test_chain_l12_m64_is_exact():
    n = 12
    b = synth.chain_bonds(n)
    _, swe, _, _ = run(synth.heisenberg_mpo(n, b), n, (0,), 64, 2)
    e0 = ed.lowest(ed.heisenberg_sector(n, b, n // 2))
    assert abs(swe[-1] - e0) < 1e-10 * abs(e0)


def test_chain_l16_m64_four_sweeps_against_ed():
    """The first isolated workload: L=16 open chain, k=5, m=64, cutoff 1e-10,
    4 sweeps, Davidson tol 1e-12, FP64."""
    n = 16
    b = synth.chain_bonds(n)
    mpo = synth.heisenberg_mpo(n, b)
    assert mpo.k == 5
    E, swe, disc, _ = run(mpo, n, (0,), 64, 4)
    e0 = ed.lowest(ed.heisenberg_sector(n, b, n // 2))
    assert swe[-1] >= e0 - 1e-12 * abs(e0)                   # variational bound
    assert (swe[-1] - e0) / abs(e0) < 1e-9
    for a, c in zip(swe, swe[1:]):                           # non-increasing sweeps
        assert c <= a + 1e-12 * abs(a)


def test_block_loop_sweeps_equal_dense_sweeps():
    n = 10
    mpo = synth.heisenberg_mpo(n, synth.chain_bonds(n))
    E1, _, _, _ = run(mpo, n, (0,), 16, 2, heff="dense")
    E2, _, _, _ = run(mpo, n, (0,), 16, 2, heff="blocks")
    assert np.allclose(E1, E2, rtol=1e-10, atol=0)


def test_free_fermions_pin_jordan_wigner_signs():
    W, Lx = 2, 3
    hops = synth.cylinder_j1_bonds(W, Lx)
    n = W * Lx
    T = np.zeros((n, n))
    for (i, j), t in hops.items():
        T[i, j] = T[j, i] = -t
    e_free = 2.0 * np.sort(np.linalg.eigvalsh(T))[:n // 2].sum()
    _, swe, _, _ = run(synth.hubbard_mpo(n, hops, 0.0), n, (n, 0), 64, 3, m0=32)
    assert abs(swe[-1] - e_free) < 1e-9 * abs(e_free)


def test_hubbard_cylinder_against_ed():
    W, Lx, U = 2, 3, 8.0
    hops = synth.cylinder_j1_bonds(W, Lx)
    n = W * Lx
    e0 = ed.lowest(ed.hubbard_sector(n, hops, U, n // 2, n // 2))
    _, swe, _, _ = run(synth.hubbard_mpo(n, hops, U), n, (n, 0), 64, 3, m0=32)
    assert abs(swe[-1] - e0) < 1e-9 * abs(e0)


def test_j1_j2_cylinder_against_ed():
    W, Lx, J2 = 3, 3, 0.5
    bonds = synth.merge_bonds(synth.cylinder_j1_bonds(W, Lx), synth.cylinder_j2_bonds(W, Lx, J2))
    n = W * Lx
    e0 = ed.lowest(ed.heisenberg_sector(n, bonds, (n + 1) // 2))
    _, swe, _, _ = run(synth.heisenberg_mpo(n, bonds), n, (1,), 32, 3)
    assert abs(swe[-1] - e0) < 1e-9 * abs(e0)


def test_single_site_operator_equals_two_site_with_identity_site():
    """The single-site operator L W R (Sec. II-C) equals the two-site operator
    whose second site is the identity on a one-state zero-charge leg, acting
    on the site tensor with that leg inserted (the two-site form is pinned to
    Q^T H Q by exact diagonalisation)."""
    from oracle.blocks import BlockTensor, block_shape
    from oracle.heff import heff1_dense, heff_blocks, w_tensor, MPS_SIGNS, ENV_SIGNS, PSI_SIGNS
    base = synth.c2_bond(m=40, k=14, seed=4)
    # a single site adds one spin: the right bond leg has odd charges
    spec = synth.BondSpec(base.a_leg, synth.spin_bond_leg(40, center=1), base.mpo, 4)
    wl, s = spec.w_leg(), spec.s_leg
    a, c = spec.a_leg, spec.c_leg
    L = BlockTensor.from_fn([a, wl, a], ENV_SIGNS, spec.L_block)
    R = BlockTensor.from_fn([c, wl, c], ENV_SIGNS, spec.R_block)
    W = w_tensor(spec.W1, wl, s, wl)
    psi = BlockTensor.from_fn([a, s, c], MPS_SIGNS, lambda k: synth.gaussian_block(2, 7, k, block_shape([a, s, c], k)))
    one = [((0,), 1)]
    k = sum(n for _, n in wl)
    Wid = w_tensor(np.eye(k).reshape(k, 1, 1, k), wl, one, wl)
    psi2 = BlockTensor([a, s, one, c], PSI_SIGNS,
                       {(ia, i_s, 0, ic): v.reshape(v.shape[0], v.shape[1], 1, v.shape[2])
                        for (ia, i_s, ic), v in psi.blocks.items()})
    got = heff1_dense(L, W, R, psi).pack()
    ref = heff_blocks(L, W, Wid, R, psi2).pack()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_single_site_sweeps_reach_ed_and_never_rise():
    """Single-site sweeps from a random MPS whose bonds already hold the whole
    space (L = 8, every sector of every bond at its full size): the energy of
    every solve is non-increasing and the last equals exact diagonalisation."""
    n = 8
    b = synth.chain_bonds(n)
    mpo = synth.heisenberg_mpo(n, b)
    mps = random_mps(mpo, n, (0,), 256, 2, mps_block)
    E, _, swe = dmrg1(mpo, mps, 3)
    e0 = ed.lowest(ed.heisenberg_sector(n, b, n // 2))
    assert abs(swe[-1] - e0) < 1e-10 * abs(e0)
    for x, y in zip(E, E[1:]):
        assert y <= x + 1e-11 * abs(x)
