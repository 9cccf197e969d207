"""Two-site DMRG sweeps of the oracle against exact diagonalisation and closed
forms (the paper prints no energies, so every pin is ED or mathematics)."""
import numpy as np

import synth
from synth.blocks import mps_block
from oracle import ed
from oracle.dmrg import random_mps, dmrg

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
