"""Pins of the oracle's MPO compression: the compressed operator equals the
dense Hamiltonian, and its bond dimensions equal the operator Schmidt ranks,
which follow from the coupling matrices alone."""
import numpy as np
import pytest

import synth
from oracle import ed, mpo_dense
from oracle.mpo_compress import compress_mpo, mpo_to_dense_bonds


def _compress(mpo):
    return compress_mpo(mpo.W, mpo.w_leg(), mpo.phys, mpo.start, mpo.done)


def _j1j2(W, Lx, J2=0.5):
    j1, j2 = synth.cylinder_j1_bonds(W, Lx), synth.cylinder_j2_bonds(W, Lx)
    mpo = synth.heisenberg_j2_derivative(W * Lx, j1, j2, J2)[0]
    return mpo, synth.merge_bonds(j1, {p: J2 * v for p, v in j2.items()})


@pytest.mark.parametrize("case", ["chain8", "j1j2_3x3", "hub_2x2", "hub_chain4"])
def test_compressed_mpo_equals_dense_hamiltonian(case):
    if case == "chain8":
        mpo = synth.heisenberg_mpo(8, synth.chain_bonds(8))
        H = ed.heisenberg_full(8, synth.chain_bonds(8))
    elif case == "j1j2_3x3":
        mpo, _ = _j1j2(3, 3)
        H = mpo_dense.mpo_to_dense(mpo)
    elif case == "hub_2x2":
        mpo = synth.hubbard_mpo(4, synth.cylinder_j1_bonds(2, 2), 8.0)
        H = mpo_dense.mpo_to_dense(mpo)
    else:
        mpo = synth.hubbard_mpo(4, synth.chain_bonds(4), 4.0)
        H = mpo_dense.mpo_to_dense(mpo)
    c = _compress(mpo)
    Hc = mpo_to_dense_bonds(c["W"], c["start"], c["done"])
    assert np.abs(Hc - H).max() <= 1e-12 * np.abs(H).max()
    dims = [sum(n for _, n in leg) for leg in c["legs"]]
    assert dims[0] == dims[-1] == 1 and max(dims) <= mpo.k


def _schmidt_dims(n, couplings, per_pair, local):
    """Operator Schmidt rank of H = sum_{i<j} c_ij O_i . O_j (+ on-site
    terms) across every bond: the crossing terms contribute per_pair times the
    rank of the coupling block between the two sides, and H_A (x) I, I (x) H_B
    one each when non-zero."""
    C = np.zeros((n, n))
    for (i, j), v in couplings.items():
        C[i, j] = C[j, i] = v
    dims = [1]
    for b in range(1, n):
        A, B = range(b), range(b, n)
        rank = np.linalg.matrix_rank(C[np.ix_(list(A), list(B))]) if couplings else 0
        h_a = local or any(i < b and j < b for (i, j) in couplings)
        h_b = local or any(i >= b and j >= b for (i, j) in couplings)
        dims.append(int(h_a) + int(h_b) + per_pair * int(rank))
    return dims + [1]


@pytest.mark.parametrize("case", ["j1j2_3x3", "j1j2_6x6", "hub_4x16"])
def test_compressed_bond_dims_equal_operator_schmidt_ranks(case):
    if case == "j1j2_3x3":
        mpo, J = _j1j2(3, 3)
        want = _schmidt_dims(9, J, 3, False)
    elif case == "j1j2_6x6":
        mpo, J = _j1j2(6, 6)
        want = _schmidt_dims(36, J, 3, False)
    else:
        hops = synth.cylinder_j1_bonds(4, 16)
        mpo = synth.hubbard_mpo(64, hops, 8.0)
        want = _schmidt_dims(64, hops, 4, True)
    c = _compress(mpo)
    assert [sum(n for _, n in leg) for leg in c["legs"]] == want


def test_compression_is_idempotent():
    """Compressing the compressed operator again keeps every bond leg and the
    operator itself (3 x 3 lattice: the dense 512 x 512 operator is compared)."""
    mpo, _ = _j1j2(3, 3)
    c1 = _compress(mpo)
    c2 = compress_mpo(c1["W"], c1["legs"], mpo.phys, c1["start"], c1["done"])
    assert c2["legs"] == c1["legs"]
    H1 = mpo_to_dense_bonds(c1["W"], 0, 0)
    H2 = mpo_to_dense_bonds(c2["W"], 0, 0)
    assert np.abs(H2 - H1).max() <= 1e-12 * np.abs(H1).max()
