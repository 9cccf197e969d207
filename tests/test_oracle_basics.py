"""Pins of the oracle's building blocks: RNG, layout, MPO inputs, contraction."""
import os

import numpy as np
import pytest

from oracle import rng, ed, mpo_dense
from oracle.blocks import BlockTensor, canonical_layout, contract, allowed_keys
from oracle.heff import w_tensor
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- RNG -------
def test_splitmix64_published_vectors():
    for line in open(os.path.join(GOLD, "splitmix64.txt")):
        if line.startswith("#") or not line.strip():
            continue
        vals = [int(x) for x in line.split()]
        assert rng.splitmix64_stream(vals[0], len(vals) - 1) == vals[1:]


def test_gaussian_stream_moments_and_counter_property():
    key = rng.restart_key(7, 3, 1)
    z = rng.gaussian_at(key, np.arange(200000))
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    # counter-based: any subset of indices gives the same values
    idx = np.array([5, 17, 199999, 0])
    assert np.array_equal(rng.gaussian_at(key, idx), z[idx])
    # element e uses outputs 2e, 2e+1 of the SplitMix64 stream
    s = rng.splitmix64_stream(key, 4)
    u1, u2 = (s[2] >> 11) * 2.0 ** -53, (s[3] >> 11) * 2.0 ** -53
    assert z[1] == np.sqrt(-2 * np.log(1 - u1)) * np.cos(2 * np.pi * u2)


# ------------------------------------------------------------- layout -------
LEG_A = [((-1,), 2), ((1,), 3)]
LEG_S = [((-1,), 1), ((1,), 1)]
LEG_C = [((-2,), 1), ((0,), 4), ((2,), 2)]


def test_canonical_layout_hand_example():
    # rule q_a + q_s - q_c = 0; worked out by hand:
    #  (0,0,0): -1-1=-2 -> 2*1*1 = 2   -> slot 32
    #  (0,1,1): -1+1= 0 -> 2*1*4 = 8   -> slot 32
    #  (1,0,1):  1-1= 0 -> 3*1*4 = 12  -> slot 32
    #  (1,1,2):  1+1= 2 -> 3*1*2 = 6   -> slot 32
    keys, offs = canonical_layout([LEG_A, LEG_S, LEG_C], (1, 1, -1))
    assert keys == [(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 2)]
    assert offs == [0, 32, 64, 96, 128]


def test_canonical_layout_large_block_padding():
    a = [((0,), 33)]
    keys, offs = canonical_layout([a, a], (1, -1))
    assert keys == [(0, 0)] and offs == [0, 33 * 33 + (32 - (33 * 33) % 32)]
    assert offs[1] % 32 == 0 and offs[1] >= 33 * 33


def test_layout_rejects_unsorted_leg():
    with pytest.raises(ValueError):
        canonical_layout([[((1,), 1), ((0,), 1)]], (1,))


def test_pack_unpack_roundtrip_and_zero_padding():
    legs = [LEG_A, LEG_S, LEG_C]
    r = np.random.default_rng(1)
    bt = BlockTensor.from_fn(legs, (1, 1, -1), lambda k: r.standard_normal(
        tuple(l[i][1] for l, i in zip(legs, k))))
    flat = bt.pack()
    keys, offs = canonical_layout(legs, (1, 1, -1))
    for k, o, o2 in zip(keys, offs, offs[1:]):
        n = bt.blocks[k].size
        assert np.array_equal(flat[o:o + n], bt.blocks[k].ravel())
        assert np.all(flat[o + n:o2] == 0.0)
    back = BlockTensor.unpack(flat, legs, (1, 1, -1))
    assert all(np.array_equal(back.blocks[k], bt.blocks[k]) for k in keys)


def test_dense_embedding_detects_charge_violation():
    legs = [LEG_A, LEG_S, LEG_C]
    d = np.zeros((5, 2, 7))
    d[0, 0, 0] = 1.0            # allowed: (a=-1, s=-1, c=-2)
    BlockTensor.from_dense(d, legs, (1, 1, -1))
    d[0, 0, 2] = 1.0            # a=-1, s=-1, c=0: not allowed
    with pytest.raises(AssertionError):
        BlockTensor.from_dense(d, legs, (1, 1, -1))


# ------------------------------------------------------- Alg. 2 contract ----
def test_block_contraction_equals_dense_matmul():
    r = np.random.default_rng(2)
    legs_a = [LEG_A, LEG_S, LEG_C]
    A = BlockTensor.from_fn(legs_a, (1, 1, -1), lambda k: r.standard_normal(
        tuple(l[i][1] for l, i in zip(legs_a, k))))
    legs_b = [LEG_C, LEG_S, [((-3,), 2), ((-1,), 1), ((1,), 3), ((3,), 1)]]
    B = BlockTensor.from_fn(legs_b, (1, 1, -1), lambda k: r.standard_normal(
        tuple(l[i][1] for l, i in zip(legs_b, k))))
    C, flops = contract(A, B, [2], [0])
    dense = np.tensordot(A.to_dense(), B.to_dense(), axes=([2], [0]))
    got = BlockTensor(C.legs, None, C.blocks).to_dense()
    assert np.allclose(got, dense, atol=1e-14, rtol=0)
    # brute-force pair count: every (A, B) pair with equal label on the bond
    brute = 0
    for ka in allowed_keys(legs_a, (1, 1, -1)):
        for kb in allowed_keys(legs_b, (1, 1, -1)):
            if ka[2] == kb[0]:
                brute += 2 * LEG_A[ka[0]][1] * LEG_C[ka[2]][1] * legs_b[2][kb[2]][1]
    assert flops == brute


# ------------------------------------------------------------- MPOs ---------
def test_heisenberg_mpo_equals_kronecker_hamiltonian():
    b = synth.chain_bonds(6, 1.0)
    m = synth.heisenberg_mpo(6, b)
    assert m.k == 5
    assert np.abs(mpo_dense.mpo_to_dense(m) - ed.heisenberg_full(6, b)).max() < 1e-14
    j1 = synth.cylinder_j1_bonds(3, 2)
    j2 = synth.cylinder_j2_bonds(3, 2, 0.5)
    bb = synth.merge_bonds(j1, j2)
    m = synth.heisenberg_mpo(6, bb)
    assert np.abs(mpo_dense.mpo_to_dense(m) - ed.heisenberg_full(6, bb)).max() < 1e-14


def test_hubbard_mpo_equals_jordan_wigner_hamiltonian():
    for n, hops in [(3, synth.chain_bonds(3, 1.0)), (4, synth.cylinder_j1_bonds(2, 2, 0.7))]:
        m = synth.hubbard_mpo(n, hops, 8.0)
        H = ed.hubbard_full(n, hops, 8.0)
        assert np.abs(mpo_dense.mpo_to_dense(m) - H).max() < 1e-13


def test_mpo_sites_conserve_charge():
    mpos = [synth.heisenberg_mpo(4, synth.chain_bonds(4)),
            synth.hubbard_mpo(4, synth.cylinder_j1_bonds(2, 2), 4.0),
            synth.synthetic_heisenberg_bond(14, 3), synth.synthetic_heisenberg_bond(10, 3)]
    for m in mpos:
        wl = m.w_leg()
        for W in m.W:
            w_tensor(W, wl, m.phys, wl)      # raises if a forbidden entry is non-zero
    assert synth.synthetic_heisenberg_bond(10, 1).k == 10
    assert synth.synthetic_heisenberg_bond(18, 1).k == 18


def test_sector_ed_matches_full_space_projection():
    n, hops, U = 4, synth.cylinder_j1_bonds(2, 2), 8.0
    Hf = ed.hubbard_full(n, hops, U)
    # basis index = sum over sites of local (2 n_up + n_dn) * 4^(n-1-site)
    idx = []
    for s in range(4 ** n):
        digs = [(s // 4 ** (n - 1 - i)) % 4 for i in range(n)]
        if sum(d >> 1 for d in digs) == 2 and sum(d & 1 for d in digs) == 2:
            idx.append(s)
    e_full = np.linalg.eigvalsh(Hf[np.ix_(idx, idx)])[0]
    e_sec = ed.lowest(ed.hubbard_sector(n, hops, U, 2, 2))
    assert abs(e_full - e_sec) < 1e-12
    b = synth.chain_bonds(6)
    Hs = ed.heisenberg_full(6, b)
    idx = [s for s in range(64) if bin(s).count("1") == 3]
    assert abs(np.linalg.eigvalsh(Hs[np.ix_(idx, idx)])[0] -
               ed.lowest(ed.heisenberg_sector(6, b, 3))) < 1e-12


def test_closed_forms_of_ed():
    assert abs(ed.lowest(ed.heisenberg_sector(2, synth.chain_bonds(2), 1)) + 0.75) < 1e-14
    assert abs(ed.lowest(ed.heisenberg_sector(3, synth.chain_bonds(3), 1)) + 1.0) < 1e-14
    U = 8.0
    e = ed.lowest(ed.hubbard_sector(2, synth.chain_bonds(2), U, 1, 1))
    assert abs(e - (U - np.sqrt(U * U + 16.0)) / 2.0) < 1e-13
    # U = 0: free fermions, E = 2 * sum of the lowest N/2 hopping eigenvalues
    hops = synth.cylinder_j1_bonds(3, 2)
    T = np.zeros((6, 6))
    for (i, j), t in hops.items():
        T[i, j] = T[j, i] = -t
    e0 = 2.0 * np.sort(np.linalg.eigvalsh(T))[:3].sum()
    assert abs(ed.lowest(ed.hubbard_sector(6, hops, 0.0, 3, 3)) - e0) < 1e-12


def test_sector_models():
    leg = synth.spin_bond_leg(1024)
    assert sum(d for _, d in leg) == 1024 and len(leg) == 21
    assert max(d for _, d in leg) == 270
    leg = synth.electron_bond_leg(4096, center=(32, 0))
    assert sum(d for _, d in leg) == 4096
    assert 100 <= len(leg) <= 400
