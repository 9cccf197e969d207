"""GPU parity of the MPO compression (merge and truncation on the chain of
fused (s', s) legs) and of the merge / truncation with physical sectors of
dimension above 1, against the oracle.

Tolerances: the operator compressed on the device equals the dense
Hamiltonian to 1e-12 relative (FP64 SVDs of small matrices); bond legs equal
the oracle's exactly (singular values are gauge independent; the kept ones
are O(1) of the norm and the dropped ones at the rounding level, far from the
1e-13 cut); DMRG energies with the compressed operator equal exact
diagonalisation to 1e-10 relative."""
import numpy as np
import pytest

import synth
from oracle import ed, mpo_dense
from oracle.blocks import BlockTensor, block_shape
from oracle.env import merge as o_merge
from oracle.heff import PSI_SIGNS, MPS_SIGNS
from oracle.mpo_compress import compress_mpo, mpo_to_dense_bonds
from oracle.truncate import truncate as o_truncate

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _j1j2(W, Lx, J2=0.5):
    j1, j2 = synth.cylinder_j1_bonds(W, Lx), synth.cylinder_j2_bonds(W, Lx)
    return synth.heisenberg_j2_derivative(W * Lx, j1, j2, J2)[0]


PAIR = [((-2,), 1), ((0,), 2), ((2,), 1)]          # (s', s) pairs of spin-1/2 by charge


def test_merge_and_truncate_with_multi_state_physical_sectors(gpu_lib):
    lib = gpu_lib
    a = [((-2,), 7), ((0,), 9), ((2,), 6)]
    b = [((-2,), 5), ((0,), 8), ((2,), 5)]
    c = [((-2,), 6), ((0,), 10), ((2,), 7)]
    A = BlockTensor.from_fn([a, PAIR, b], MPS_SIGNS, lambda k: synth.gaussian_block(3, 21, k, block_shape([a, PAIR, b], k)))
    B = BlockTensor.from_fn([b, PAIR, c], MPS_SIGNS, lambda k: synth.gaussian_block(3, 22, k, block_shape([b, PAIR, c], k)))
    theta_o = o_merge(A, B)
    op = lib.merge_plan(a, PAIR, b, PAIR, c)
    theta = torch.zeros(op.query()["out_elems"], dtype=torch.float64, device="cuda")
    lib.merge(op, dev(A.pack()), dev(B.pack()), theta)
    torch.cuda.synchronize()
    assert rel(theta.cpu().numpy(), theta_o.pack()) < 1e-13
    for direction in (0, 1):
        gA, gB, leg, sv, disc = lib.truncate(theta_o.legs, dev(theta_o.pack()), direction, cutoff=1e-12, max_m=12)
        oA, oB, oleg, osv, odisc = o_truncate(theta_o, "right" if direction == 0 else "left", cutoff=1e-12,
                                              m_max=12)
        assert leg == oleg
        assert np.allclose(sv, osv, rtol=1e-12, atol=1e-14 * osv[0])
        assert rel(gA.cpu().numpy(), oA.pack()) < 1e-11
        assert rel(gB.cpu().numpy(), oB.pack()) < 1e-11


@pytest.mark.parametrize("case", ["j1j2_3x3", "hub_2x2", "j1j2_6x6", "hub_4x16"])
def test_device_compression_matches_oracle(gpu_lib, case):
    from paper_2007_05540_amd import mpo as gmpo
    if case == "j1j2_3x3":
        m = _j1j2(3, 3)
    elif case == "hub_2x2":
        m = synth.hubbard_mpo(4, synth.cylinder_j1_bonds(2, 2), 8.0)
    elif case == "j1j2_6x6":
        m = _j1j2(6, 6)
    else:
        m = synth.hubbard_mpo(64, synth.cylinder_j1_bonds(4, 16), 8.0)
    c = gmpo.compress(m)
    o = compress_mpo(m.W, m.w_leg(), m.phys, m.start, m.done)
    print(f"{case}: k {m.k} -> {max(c.bond_dims())}", flush=True)
    assert c.legs == o["legs"]
    if len(m.W) <= 9:
        H = mpo_dense.mpo_to_dense(m)
        Hc = mpo_to_dense_bonds(c.W, c.start, c.done)
        assert np.abs(Hc - H).max() <= 1e-12 * np.abs(H).max()


@pytest.mark.parametrize("case", ["j1j2_3x3", "hub_2x3"])
def test_dmrg_with_compressed_mpo_equals_ed(gpu_lib, case):
    """Two-site sweeps with the compressed operator (its own leg on every
    bond, one channel at both ends) reach the exact ground energy, as the
    uncompressed operator does."""
    from paper_2007_05540_amd import mpo as gmpo, problems, dmrg as gdmrg
    if case == "j1j2_3x3":
        m = _j1j2(3, 3)
        j1, j2 = synth.cylinder_j1_bonds(3, 3), synth.cylinder_j2_bonds(3, 3)
        bonds = synth.merge_bonds(j1, {p: 0.5 * v for p, v in j2.items()})
        e0 = ed.lowest(ed.heisenberg_sector(9, bonds, 5))
        target, m_max = (1,), 32
    else:
        hops = synth.cylinder_j1_bonds(2, 3)
        m = synth.hubbard_mpo(6, hops, 8.0)
        e0 = ed.lowest(ed.hubbard_sector(6, hops, 8.0, 3, 3))
        target, m_max = (6, 0), 128
    c = gmpo.compress(m)
    energies = {}
    for name, op in (("uncompressed", m), ("compressed", c)):
        g = gdmrg.GpuDMRG(op, problems.initial_mps(op, target, 16, 3), target)
        _, swe = g.run(4, m_max, cutoff=1e-12, max_iter=40, tol=1e-11)
        energies[name] = swe[-1]
    assert abs(energies["compressed"] - e0) <= 1e-10 * abs(e0)
    assert abs(energies["uncompressed"] - e0) <= 1e-10 * abs(e0)
