"""GPU parity of the environment-extension adjoint and of dE/dJ2 by reverse
mode (EnvUpdate x sites -> HeffEnergy -> backward) against the oracle and
exact diagonalisation.

Tolerances: single extensions 1e-12 norm-wise relative (FP64 GEMMs and
fixed-order dots against dense einsums).  Per-site MPO gradients along a
chain of extensions 1e-10 (errors of up to ~10 chained FP64 contractions).
dE/dJ2 of an untruncated, converged state against the ED Hellmann-Feynman
value 1e-9 relative (the eigensolver tolerance 1e-12 on the residual bounds
the state error; dE/dJ2 is first order in it only through the
non-stationary part, so the bound is loose).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from synth.blocks import mps_block
from oracle import ed, grad
from oracle.blocks import BlockTensor
from oracle.dmrg import random_mps, right_canonicalize
from oracle.env import left_update_dense, right_update_dense
from oracle.heff import w_tensor, MPS_SIGNS, ENV_SIGNS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods(gpu_lib):
    from paper_2007_05540_amd import problems, dmrg as gdmrg
    return gpu_lib, problems, gdmrg


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def j1j2_chain(n, j2=0.4):
    return synth.merge_bonds(synth.chain_bonds(n), {(i, i + 2): j2 for i in range(n - 2)})


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("hub", [False, True])
def test_env_backward_matches_oracle(mods, side, hub):
    lib, problems, _ = mods
    n = 8
    if hub:
        mpo = synth.hubbard_mpo(n, synth.chain_bonds(n), 4.0)
        target = (n, 0)
    else:
        mpo = synth.heisenberg_mpo(n, j1j2_chain(n))
        target = (0,)
    mps = random_mps(mpo, n, target, 24, 5, mps_block)
    wl, s = mpo.w_leg(), mpo.phys
    W = w_tensor(mpo.W[3], wl, s, wl)
    W_host = problems.pack_dense(mpo.W[3], [wl, s, s, wl], lib.W_SIGNS)
    site = mps[3]
    x = site.legs[0] if side == 0 else site.legs[2]
    y = site.legs[2] if side == 0 else site.legs[0]
    env = BlockTensor.from_fn([x, wl, x], ENV_SIGNS, lambda k: synth.gaussian_block(
        17, side, k, (x[k[0]][1], wl[k[1]][1], x[k[2]][1])))
    out = (left_update_dense if side == 0 else right_update_dense)(env, site, W)
    D = BlockTensor.from_fn(out.legs, ENV_SIGNS, lambda k: synth.gaussian_block(
        18, side, k, tuple(out.legs[i][k[i]][1] for i in range(3))))
    ref = grad.env_gradients(env, site, W, D, side)
    op = lib.env_plan(x, s, y, wl, wl, W_host, side)
    adj = lib.env_plan(y, s, x, wl, wl, W_host, 1 - side)
    dW = torch.full((W_host.size,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.empty(lib.env_backward_workspace(op), dtype=torch.uint8, device="cuda")
    d_site, d_env_in, d_out = dev(site.pack()), dev(env.pack()), dev(D.pack())
    lib.env_backward(op, d_env_in, d_site, d_out, dW, ws)
    d_env = torch.zeros(adj.query()["out_elems"], dtype=torch.float64, device="cuda")
    ws2 = torch.empty(max(1, adj.query()["workspace_bytes"]), dtype=torch.uint8, device="cuda")
    lib.env_update(adj, d_out, d_site, dev(W_host), d_env, ws2)
    torch.cuda.synchronize()
    got_w = dW.cpu().numpy()
    assert np.all(np.isfinite(got_w))
    assert rel(got_w, ref["W"].pack()) < 1e-12
    assert rel(d_env.cpu().numpy(), ref["env"].pack()) < 1e-12


def host_mps(problems, mps):
    return [(t.legs, problems.pack_fn(t.legs, MPS_SIGNS, lambda k, t=t: t.blocks[k])) for t in mps]


def test_mpo_gradients_match_oracle_per_site(mods):
    """Random MPS brought to mixed-canonical form around bond 0 (numerically
    zero singular values dropped only): every per-site dE/dW_s, divided by
    E (both are quadratic in the state, so the ratio does not depend on its
    norm or gauge), equals the oracle's reverse-mode value."""
    lib, problems, gdmrg = mods
    n = 8
    mpo = synth.heisenberg_mpo(n, j1j2_chain(n))
    mps = random_mps(mpo, n, (0,), 12, 9, mps_block)
    g = gdmrg.GpuDMRG(mpo, host_mps(problems, mps), (0,))
    g.right_canonicalize()
    E, grads = g.energy_and_mpo_gradients(0)
    wl, s = mpo.w_leg(), mpo.phys
    Ws = [w_tensor(x, wl, s, wl) for x in mpo.W]
    Eo, dWo = grad.mpo_gradients(right_canonicalize(mps), Ws, wl, mpo.start, mpo.done, (0,), 0)
    keys, offs = lib.layout([wl, s, s, wl], lib.W_SIGNS)
    for j in range(n):
        got = grads[j].cpu().numpy() / E
        ref = dWo[j].pack() / Eo
        if j in (0, 1):   # the two-site adjoint covers the non-zero W blocks
            wh = problems.pack_dense(mpo.W[j], [wl, s, s, wl], lib.W_SIGNS)
            m = np.zeros(wh.size, dtype=bool)
            for b in range(len(keys)):
                if np.any(wh[offs[b]:offs[b + 1]] != 0):
                    m[offs[b]:offs[b + 1]] = True
            got, ref = got[m], ref[m]
        assert rel(got, ref) < 1e-10, j


def test_de_dj2_matches_exact_hellmann_feynman(mods):
    """3 x 4 J1-J2 cylinder (J2/J1 = 0.5), untruncated two-site sweeps on the
    GPU (m = 64 is exact for 12 sites), then dE/dJ2 by reverse mode and the
    chain rule over the MPO builder's dW/dJ2, against ED."""
    lib, problems, gdmrg = mods
    Wd, Lx, J2 = 3, 4, 0.5
    n = Wd * Lx
    j1, j2 = synth.cylinder_j1_bonds(Wd, Lx), synth.cylinder_j2_bonds(Wd, Lx)
    mpo, dWs = synth.heisenberg_j2_derivative(n, j1, j2, J2)
    mps = random_mps(mpo, n, (0,), 16, 3, mps_block)
    g = gdmrg.GpuDMRG(mpo, host_mps(problems, mps), (0,))
    _, swe = g.run(3, 64, cutoff=1e-12, max_iter=40, tol=1e-12)
    H = ed.heisenberg_sector(n, synth.merge_bonds(j1, {p: J2 * v for p, v in j2.items()}), n // 2)
    w, v = spla.eigsh(H, k=1, which="SA", tol=1e-14)
    v = v[:, 0]
    hf = float(v @ (ed.heisenberg_sector(n, j2, n // 2) @ v))
    assert abs(swe[-1] - w[0]) < 1e-10 * abs(w[0])
    E, grads = g.energy_and_mpo_gradients(0)
    assert abs(E - w[0]) < 1e-10 * abs(w[0])
    dE = g.parameter_derivative(grads, dWs)
    assert abs(dE - hf) < 1e-9 * abs(hf)


def test_param_derivative_entry_point(gpu_lib):
    """bsdmrg_param_derivative against a host dot product of the same
    vectors: 70 sites (three launch groups), one of them empty, sizes up to
    a few 10^4; per-site terms to 1e-14 relative, the ordered sum to
    1e-13, bit-identical on a second call."""
    lib = gpu_lib
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(1, 40000, size=70)]
    sizes[17] = 0
    xs = [rng.standard_normal(n) for n in sizes]
    ys = [rng.standard_normal(n) for n in sizes]
    gx = [torch.from_numpy(x).to("cuda") for x in xs]
    gy = [torch.from_numpy(y).to("cuda") for y in ys]
    terms = torch.full((len(sizes) + 1,), float("nan"), dtype=torch.float64, device="cuda")
    total = lib.param_derivative(gx, gy, terms)
    want = np.array([float(np.dot(x, y)) for x, y in zip(xs, ys)])
    got = terms.cpu().numpy()
    scale = np.array([np.linalg.norm(x) * np.linalg.norm(y) for x, y in zip(xs, ys)])
    assert np.all(np.abs(got[:-1] - want) <= 1e-14 * np.maximum(scale, 1e-300))
    assert got[17] == 0.0
    assert abs(total - want.sum()) <= 1e-13 * scale.sum()
    assert got[-1] == total
    assert lib.param_derivative(gx, gy, terms) == total
    with pytest.raises(ValueError):
        lib.param_derivative(gx[:3], gy[:2], terms)
