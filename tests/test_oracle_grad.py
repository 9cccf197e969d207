"""Pins of the oracle's environment-extension cotangents and of the
MPO-parameter derivative dE/dJ2 against mathematics and exact diagonalisation.

- Euler identities: the extension is linear in its environment and in W, so
  <dEnv, Env> = <dW, W> = <D, out> for any output cotangent D.
- Central differences along random directions (exact for a linear map up to
  rounding).
- Hellmann-Feynman: for the ground state of H(J2) = H_J1 + J2 H_J2,
  dE/dJ2 = <psi0|H_J2|psi0>; the exact value comes from a sparse ED of the
  sector (itself checked by a finite difference of ED energies), and the
  oracle's reverse-mode value (two-site gradients carried outwards through
  the environment cotangents, chain rule over dW_s/dJ2) must agree with it
  for a converged, untruncated MPS.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from synth.blocks import mps_block
from oracle import ed, grad
from oracle.blocks import BlockTensor
from oracle.dmrg import random_mps, right_canonicalize, dmrg
from oracle.env import left_update_dense, right_update_dense
from oracle.heff import w_tensor, ENV_SIGNS


def rand_like(bt, seed):
    r = np.random.default_rng(seed)
    out = bt.copy()
    for k in out.blocks:
        out.blocks[k] = r.standard_normal(out.blocks[k].shape)
    return out


def env_case(side, seed=4):
    n = 10
    mpo = synth.heisenberg_mpo(n, synth.merge_bonds(synth.chain_bonds(n), {(i, i + 2): 0.4 for i in range(n - 2)}))
    mps = random_mps(mpo, n, (0,), 24, seed, mps_block)
    wl = mpo.w_leg()
    W = w_tensor(mpo.W[4], wl, mpo.phys, wl)
    site = mps[4]
    x = site.legs[0] if side == 0 else site.legs[2]
    env = BlockTensor.from_fn([x, wl, x], ENV_SIGNS, lambda k: synth.gaussian_block(
        seed, 30 + side, k, (x[k[0]][1], wl[k[1]][1], x[k[2]][1])))
    upd = left_update_dense if side == 0 else right_update_dense
    out = upd(env, site, W)
    D = rand_like(out, seed + 1)
    return env, site, W, D, out, upd


@pytest.mark.parametrize("side", [0, 1])
def test_env_cotangents_euler_identities(side):
    env, site, W, D, out, upd = env_case(side)
    g = grad.env_gradients(env, site, W, D, side)
    ref = D.dot(out)
    assert abs(g["env"].dot(env) - ref) < 1e-11 * abs(ref)
    assert abs(g["W"].dot(W) - ref) < 1e-11 * abs(ref)


@pytest.mark.parametrize("side", [0, 1])
def test_env_cotangents_directional_derivatives(side):
    env, site, W, D, out, upd = env_case(side, seed=6)
    g = grad.env_gradients(env, site, W, D, side)
    h = 1e-3
    dE, dW = rand_like(env, 11), rand_like(W, 12)
    fd_env = (D.dot(upd(env.axpy(h, dE), site, W)) - D.dot(upd(env.axpy(-h, dE), site, W))) / (2 * h)
    fd_w = (D.dot(upd(env, site, W.axpy(h, dW))) - D.dot(upd(env, site, W.axpy(-h, dW)))) / (2 * h)
    assert abs(fd_env - g["env"].dot(dE)) < 1e-9 * abs(fd_env)
    assert abs(fd_w - g["W"].dot(dW)) < 1e-9 * abs(fd_w)


@pytest.mark.parametrize("side", [0, 1])
def test_env_cotangent_of_env_is_opposite_extension(side):
    """The environment's cotangent is the opposite-side extension of D with
    the same site tensor (the identity the device path relies on)."""
    env, site, W, D, out, upd = env_case(side, seed=8)
    g = grad.env_gradients(env, site, W, D, side)
    other = right_update_dense if side == 0 else left_update_dense
    o = other(D, site, W)
    assert max(np.abs(o.blocks[k] - g["env"].blocks[k]).max() for k in o.blocks) < 1e-12 * max(
        np.abs(v).max() for v in o.blocks.values())


def test_expectation_equals_dense_vector_expectation():
    n = 8
    bonds = synth.chain_bonds(n)
    mpo = synth.heisenberg_mpo(n, bonds)
    mps = random_mps(mpo, n, (0,), 8, 2, mps_block)
    # dense state vector (site 0 most significant, local index 0 = down)
    v = np.ones((1, 1))
    for A in mps:
        Ad = A.to_dense()
        v = np.einsum("ia,asb->isb", v, Ad).reshape(-1, Ad.shape[2])
    v = v[:, 0]
    H = ed.heisenberg_full(n, bonds)
    ref = float(v @ H @ v / (v @ v))
    assert abs(grad.expectation(mps, mpo.W, mpo.start, mpo.done) - ref) < 1e-12 * abs(ref)


@pytest.fixture(scope="module")
def j1j2_3x4():
    W, Lx, J2 = 3, 4, 0.5
    n = W * Lx
    j1, j2 = synth.cylinder_j1_bonds(W, Lx), synth.cylinder_j2_bonds(W, Lx)
    H = lambda x: ed.heisenberg_sector(n, synth.merge_bonds(j1, {p: x * v for p, v in j2.items()}), n // 2)
    w, v = spla.eigsh(H(J2), k=1, which="SA", tol=1e-14)
    v = v[:, 0]
    hf = float(v @ (ed.heisenberg_sector(n, j2, n // 2) @ v))
    return {"n": n, "j1": j1, "j2": j2, "J2": J2, "E": float(w[0]), "hf": hf, "H": H}


def test_ed_hellmann_feynman_equals_finite_difference(j1j2_3x4):
    c = j1j2_3x4
    h = 1e-4
    ep = spla.eigsh(c["H"](c["J2"] + h), k=1, which="SA", tol=1e-14)[0][0]
    em = spla.eigsh(c["H"](c["J2"] - h), k=1, which="SA", tol=1e-14)[0][0]
    assert abs((ep - em) / (2 * h) - c["hf"]) < 1e-6


def test_adjoint_de_dj2_equals_hellmann_feynman(j1j2_3x4):
    """Untruncated two-site DMRG (m = 64 = 2^6 is exact for 12 sites): the
    reverse-mode dE/dJ2 and the expectation of the J2-only MPO both equal the
    ED value."""
    c = j1j2_3x4
    n = c["n"]
    mpo, dWs = synth.heisenberg_j2_derivative(n, c["j1"], c["j2"], c["J2"])
    mps = random_mps(mpo, n, (0,), 16, 3, mps_block)
    _, mps, swe, _ = dmrg(mpo, mps, 3, 64, cutoff=1e-12)
    assert abs(swe[-1] - c["E"]) < 1e-10 * abs(c["E"])
    wl = mpo.w_leg()
    Ws = [w_tensor(x, wl, mpo.phys, wl) for x in mpo.W]
    dWb = [w_tensor(x, wl, mpo.phys, wl) for x in dWs]
    E, dW = grad.mpo_gradients(mps, Ws, wl, mpo.start, mpo.done, (0,), 0)
    assert abs(E - c["E"]) < 1e-10 * abs(c["E"])
    assert abs(grad.parameter_derivative(dW, dWb) - c["hf"]) < 1e-9 * abs(c["hf"])
    mj = synth.heisenberg_mpo(n, c["j2"])
    assert abs(grad.expectation(mps, mj.W, mj.start, mj.done) - c["hf"]) < 1e-9 * abs(c["hf"])
    # a planted mistake is seen: dropping one site's contribution changes the value
    partial = grad.parameter_derivative(dW[:-3] + [d.scale(0.0) for d in dW[-3:]], dWb)
    assert abs(partial - c["hf"]) > 1e-3


def test_mpo_gradients_euler_identity_per_site():
    """E = <Psi|H|Psi> is linear in every W_s: <dE/dW_s, W_s> = E for each
    site, and the bond energy equals the MPO expectation value."""
    n = 8
    mpo = synth.heisenberg_mpo(n, synth.merge_bonds(synth.chain_bonds(n), {(i, i + 2): 0.4 for i in range(n - 2)}))
    mps = right_canonicalize(random_mps(mpo, n, (0,), 12, 9, mps_block))
    wl = mpo.w_leg()
    Ws = [w_tensor(x, wl, mpo.phys, wl) for x in mpo.W]
    E, dW = grad.mpo_gradients(mps, Ws, wl, mpo.start, mpo.done, (0,), 0)
    nrm = sum(float(np.sum(v * v)) for v in mps[0].blocks.values())
    assert abs(E / nrm - grad.expectation(mps, mpo.W, mpo.start, mpo.done)) < 1e-12 * abs(E / nrm)
    for j in range(n):
        assert abs(dW[j].dot(Ws[j]) - E) < 1e-12 * abs(E), j
