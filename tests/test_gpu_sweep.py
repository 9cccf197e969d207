"""GPU parity of the sweep operations (merge, environment extension,
truncated SVD split) and of full two-site sweeps against the CPU oracle and
exact diagonalisation."""
import numpy as np
import pytest

import synth
from synth.blocks import mps_block
from oracle import ed
from oracle.blocks import BlockTensor
from oracle.dmrg import random_mps, dmrg, dmrg1
from oracle.env import left_update_blocks, right_update_blocks, merge
from oracle.heff import w_tensor, MPS_SIGNS, ENV_SIGNS, PSI_SIGNS
from oracle.truncate import truncate as o_truncate

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


def random_sites(n=8, m0=24, seed=3, hub=False):
    if hub:
        mpo = synth.hubbard_mpo(n, synth.chain_bonds(n), 4.0)
        target = (n, 0)
    else:
        mpo = synth.heisenberg_mpo(n, synth.chain_bonds(n))
        target = (0,)
    return mpo, random_mps(mpo, n, target, m0, seed, mps_block), target


@pytest.mark.parametrize("hub", [False, True])
def test_merge_matches_oracle(mods, hub):
    lib, problems, _ = mods
    mpo, mps, _ = random_sites(hub=hub)
    A, B = mps[3], mps[4]
    op = lib.merge_plan(A.legs[0], A.legs[1], A.legs[2], B.legs[1], B.legs[2])
    theta = torch.zeros(op.query()["out_elems"], dtype=torch.float64, device="cuda")
    lib.merge(op, dev(A.pack()), dev(B.pack()), theta)
    torch.cuda.synchronize()
    assert rel(theta.cpu().numpy(), merge(A, B).pack()) < 1e-13


@pytest.mark.parametrize("hub", [False, True])
def test_environment_extension_matches_oracle(mods, hub):
    lib, problems, _ = mods
    mpo, mps, target = random_sites(hub=hub)
    wl = mpo.w_leg()
    Wb = w_tensor(mpo.W[3], wl, mpo.phys, wl)
    W_host = problems.pack_dense(mpo.W[3], [wl, mpo.phys, mpo.phys, wl], lib.W_SIGNS)
    site = mps[3]
    # a random environment on the site's left / right bond
    for side in (0, 1):
        x = site.legs[0] if side == 0 else site.legs[2]
        env = BlockTensor.from_fn([x, wl, x], ENV_SIGNS, lambda k: synth.gaussian_block(
            7, side, k, (x[k[0]][1], wl[k[1]][1], x[k[2]][1])))
        if side == 0:
            ref = left_update_blocks(env, site, Wb)
            op = lib.env_plan(site.legs[0], mpo.phys, site.legs[2], wl, wl, W_host, 0)
        else:
            ref = right_update_blocks(env, site, Wb)
            op = lib.env_plan(site.legs[2], mpo.phys, site.legs[0], wl, wl, W_host, 1)
        info = op.query()
        out = torch.zeros(info["out_elems"], dtype=torch.float64, device="cuda")
        ws = torch.empty(max(1, info["workspace_bytes"]), dtype=torch.uint8, device="cuda")
        lib.env_update(op, dev(env.pack()), dev(site.pack()), dev(W_host), out, ws)
        torch.cuda.synchronize()
        assert rel(out.cpu().numpy(), ref.pack()) < 1e-13, side


@pytest.mark.parametrize("direction,max_m", [(0, 1 << 40), (1, 1 << 40), (0, 20), (1, 13)])
def test_truncation_matches_oracle(mods, direction, max_m):
    lib, problems, _ = mods
    mpo, mps, _ = random_sites(m0=32, seed=5)
    theta = merge(mps[3], mps[4])
    A, B, leg, sv, disc = lib.truncate(theta.legs, dev(theta.pack()), direction, cutoff=1e-12, max_m=max_m)
    oA, oB, oleg, osv, odisc = o_truncate(theta, "right" if direction == 0 else "left", cutoff=1e-12,
                                          m_max=max_m)
    assert leg == oleg
    assert np.allclose(sv, osv, rtol=1e-12, atol=1e-14)
    assert abs(disc - odisc) <= 1e-12 * max(odisc, 1e-300) + 1e-28
    # random Gaussian blocks: no degenerate singular values, so the gauge
    # fixes A and B uniquely
    assert rel(A.cpu().numpy(), oA.pack()) < 1e-11
    assert rel(B.cpu().numpy(), oB.pack()) < 1e-11


def _big_theta(seed, low_rank, huge=False):
    """theta with charge sectors of up to 250 x 270 (huge: 390 x 390, which the
    truncation factorises with the multi-workgroup QR), so the block Jacobi
    runs many block pairs per step; low_rank builds it as the merge of two
    random sites over an inner bond of at most 60 states per sector
    (rank-deficient sectors, as in a sweep)."""
    from oracle.blocks import block_shape
    a = [((-2,), 90), ((0,), 300 if huge else 160), ((2,), 90)]
    c = [((-2,), 70), ((0,), 320 if huge else 200), ((2,), 70)]
    s = synth.SPIN_PHYS
    if not low_rank:
        legs = [a, s, s, c]
        return BlockTensor.from_fn(legs, PSI_SIGNS, lambda k: synth.gaussian_block(seed, 9, k, block_shape(legs, k)))
    b = [((-3,), 20), ((-1,), 60), ((1,), 60), ((3,), 20)]
    A = BlockTensor.from_fn([a, s, b], MPS_SIGNS, lambda k: synth.gaussian_block(seed, 10, k, block_shape([a, s, b], k)))
    B = BlockTensor.from_fn([b, s, c], MPS_SIGNS, lambda k: synth.gaussian_block(seed, 11, k, block_shape([b, s, c], k)))
    return merge(A, B)


@pytest.mark.parametrize("low_rank,direction,max_m,huge", [(False, 0, 1 << 40, False), (False, 1, 300, False),
                                                           (True, 0, 1 << 40, False), (True, 1, 100, False),
                                                           (False, 0, 1 << 40, True), (True, 1, 1 << 40, True)])
def test_truncation_large_sectors_matches_oracle(mods, low_rank, direction, max_m, huge):
    lib, problems, _ = mods
    theta = _big_theta(21, low_rank, huge)
    A, B, leg, sv, disc = lib.truncate(theta.legs, dev(theta.pack()), direction, cutoff=1e-12, max_m=max_m)
    oA, oB, oleg, osv, odisc = o_truncate(theta, "right" if direction == 0 else "left", cutoff=1e-12, m_max=max_m)
    assert leg == oleg
    assert np.allclose(sv, osv, rtol=1e-12, atol=1e-14 * osv[0])
    # singular values at the rounding level of the SVD (below sqrt(m) eps
    # ||theta||) are reported as 0, so the discarded weight agrees up to that
    # level squared
    norm2 = float(np.sum(theta.pack() ** 2))
    assert abs(disc - odisc) <= 1e-12 * max(odisc, 1e-300) + 1e-20 * norm2
    assert rel(A.cpu().numpy(), oA.pack()) < 1e-10
    assert rel(B.cpu().numpy(), oB.pack()) < 1e-10


def test_truncation_of_zero_theta_is_an_error(mods):
    """theta = 0 has no singular vector to keep: ESOLVER, not a zero-width
    bond."""
    lib, problems, _ = mods
    mpo, mps, _ = random_sites()
    theta = merge(mps[3], mps[4])
    z = torch.zeros(theta.pack().size, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.BsdmrgError) as e:
        lib.truncate(theta.legs, z, 0, cutoff=1e-12)
    assert e.value.status == lib.ESOLVER


def test_truncation_rejects_small_workspace(mods):
    lib, problems, _ = mods
    mpo, mps, _ = random_sites()
    theta = merge(mps[3], mps[4])
    import ctypes
    L = lib.load()
    bufs = [lib._LegBuf(l) for l in theta.legs]
    arr = (lib.Leg * 4)(*[b.leg for b in bufs])
    o = lib.TruncOpts(0, 0, 0.0, 10, 1e-10)
    z = ctypes.c_int64(0)
    n = ctypes.c_int32(0)
    dd = ctypes.c_double(0)
    st = L.bsdmrg_truncate(arr, lib._ptr(dev(theta.pack())), ctypes.byref(o), ctypes.byref(n), None, None, 0,
                           None, 0, ctypes.byref(z), None, 0, ctypes.byref(z), None, 0, ctypes.byref(z),
                           ctypes.byref(dd), None, 0, None)
    assert st == lib.EINVAL


def host_mps(problems, lib, mps):
    return [(t.legs, problems.pack_fn(t.legs, MPS_SIGNS, lambda k, t=t: t.blocks[k])) for t in mps]


def test_heisenberg_chain_l16_m64_sweeps(mods):
    """L=16 open Heisenberg chain, k=5, m=64, cutoff 1e-10, 4 sweeps, Davidson
    tol 1e-12 (cap 40), FP64: energies against the oracle and ED."""
    lib, problems, gdmrg = mods
    n = 16
    b = synth.chain_bonds(n)
    mpo = synth.heisenberg_mpo(n, b)
    mps = random_mps(mpo, n, (0,), 16, 0, mps_block)
    g = gdmrg.GpuDMRG(mpo, host_mps(problems, lib, mps), (0,))
    E, swe = g.run(4, 64, cutoff=1e-10, max_iter=40, tol=1e-12, progress=True)
    oE, _, oswe, _ = dmrg(mpo, mps, 4, 64, cutoff=1e-10, dav={"max_iter": 40, "tol": 1e-12})
    e0 = ed.lowest(ed.heisenberg_sector(n, b, n // 2))
    assert abs(swe[-1] - e0) < 1e-9 * abs(e0)
    assert abs(swe[-1] - oswe[-1]) < 1e-9 * abs(e0)
    for a, c in zip(swe, swe[1:]):
        assert c <= a + 1e-12 * abs(a)


def test_hubbard_cylinder_sweeps_against_ed(mods):
    lib, problems, gdmrg = mods
    W, Lx, U = 2, 3, 8.0
    hops = synth.cylinder_j1_bonds(W, Lx)
    n = W * Lx
    mpo = synth.hubbard_mpo(n, hops, U)
    mps = random_mps(mpo, n, (n, 0), 32, 1, mps_block)
    g = gdmrg.GpuDMRG(mpo, host_mps(problems, lib, mps), (n, 0))
    E, swe = g.run(3, 64, cutoff=1e-10, max_iter=40, tol=1e-12)
    e0 = ed.lowest(ed.hubbard_sector(n, hops, U, n // 2, n // 2))
    assert abs(swe[-1] - e0) < 1e-9 * abs(e0)


def test_hubbard_4x16_sweep_products_match_oracle_on_sampled_bonds(mods):
    """Two-site sweeps of the 4x16 Hubbard cylinder (U(1)xU(1), k = 18, m up
    to 256, the plan and op cache in use), then at two mid-chain bonds the
    environments are rebuilt from the current site tensors on the device and
    the library's FP64 product on those operands is compared with the
    oracle's block loop (Alg. 2) on the same operands: 1e-12 norm-wise and
    1e-10 per block."""
    lib, problems, gdmrg = mods
    from oracle.heff import heff_blocks, W_SIGNS
    Wd, Lx = 4, 16
    n = Wd * Lx
    mpo = synth.hubbard_mpo(n, synth.cylinder_j1_bonds(Wd, Lx), 8.0)
    target = (n, 0)
    g = gdmrg.GpuDMRG(mpo, problems.initial_mps(mpo, target, 16, 0), target)
    g.run(3, [64, 128, 256], cutoff=1e-10, max_iter=20, tol=1e-8)
    assert g.cache_hits > 0
    for j in (21, 40):
        L = g.L[0]
        for i in range(j):
            L = g._env(L, g.T[i], i, 0)
        R = g.R[n]
        for i in range(n - 1, j + 1, -1):
            R = g._env(R, g.T[i], i, 1)
        theta = g._merge(g.T[j], g.T[j + 1])
        a, s1, s2, c = theta.legs
        plan = lib.Plan([{"a": a, "s1": s1, "s2": s2, "c": c, "wl": g.legs[j], "wm": g.legs[j + 1],
                          "wr": g.legs[j + 2], "w1": g.W_host[j], "w2": g.W_host[j + 1]}])
        out = torch.full_like(theta.data, float("nan"))
        ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
        lib.heff_apply(plan, lib.F64, L.data, g.W[j], g.W[j + 1], R.data, theta.data, out, ws)
        torch.cuda.synchronize()
        s = g.s
        oL = BlockTensor.unpack(L.data.cpu().numpy(), L.legs, ENV_SIGNS)
        oR = BlockTensor.unpack(R.data.cpu().numpy(), R.legs, ENV_SIGNS)
        oW1 = BlockTensor.unpack(g.W_host[j], [g.legs[j], s, s, g.legs[j + 1]], W_SIGNS)
        oW2 = BlockTensor.unpack(g.W_host[j + 1], [g.legs[j + 1], s, s, g.legs[j + 2]], W_SIGNS)
        opsi = BlockTensor.unpack(theta.data.cpu().numpy(), theta.legs, PSI_SIGNS)
        ref = heff_blocks(oL, oW1, oW2, oR, opsi)
        got = BlockTensor.unpack(out.cpu().numpy(), theta.legs, PSI_SIGNS)
        print(f"bond {j}: m = {sum(d for _, d in a)} x {sum(d for _, d in c)}, {len(ref.blocks)} blocks", flush=True)
        assert rel(got.pack(), ref.pack()) < 1e-12
        scale = max(np.abs(v).max() for v in ref.blocks.values())
        for k, v in ref.blocks.items():
            assert np.abs(got.blocks[k] - v).max() <= 1e-10 * max(np.abs(v).max(), 1e-3 * scale)
        plan.destroy()


def test_single_site_operator_matches_oracle(mods):
    """The single-site operator L W R through the two-site plan with an
    identity second site on a one-state leg, against the oracle's direct
    single-site contraction."""
    lib, problems, _ = mods
    from oracle.blocks import block_shape
    from oracle.heff import heff1_dense
    base = synth.c2_bond(m=256, k=14, seed=8)
    # a single site adds one spin: the right bond leg has odd charges
    spec = synth.BondSpec(base.a_leg, synth.spin_bond_leg(256, center=1), base.mpo, 8)
    wl, s = spec.w_leg(), spec.s_leg
    a, c = spec.a_leg, spec.c_leg
    one = [((0,), 1)]
    k = sum(n for _, n in wl)
    W = problems.pack_dense(spec.W1, [wl, s, s, wl], lib.W_SIGNS)
    Wid = problems.pack_dense(np.eye(k).reshape(k, 1, 1, k), [wl, one, one, wl], lib.W_SIGNS)
    prob = {"a": a, "s1": s, "s2": one, "c": c, "wl": wl, "wm": wl, "wr": wl, "w1": W, "w2": Wid}
    plan = lib.Plan([prob])
    L = problems.pack_fn([a, wl, a], lib.ENV_SIGNS, spec.L_block)
    R = problems.pack_fn([c, wl, c], lib.ENV_SIGNS, spec.R_block)
    psi = BlockTensor.from_fn([a, s, c], MPS_SIGNS, lambda kk: synth.gaussian_block(2, 7, kk, block_shape([a, s, c], kk)))
    out = torch.zeros(plan.info()["psi_elems"], dtype=torch.float64, device="cuda")
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, dev(L), dev(W), dev(Wid), dev(R), dev(psi.pack()), out, ws)
    torch.cuda.synchronize()
    Lo = BlockTensor.unpack(L, [a, wl, a], ENV_SIGNS)
    Ro = BlockTensor.unpack(R, [c, wl, c], ENV_SIGNS)
    ref = heff1_dense(Lo, w_tensor(spec.W1, wl, s, wl), Ro, psi).pack()
    assert rel(out.cpu().numpy(), ref) < 1e-12


def test_single_site_sweeps_match_oracle_and_ed(mods):
    """Single-site sweeps of the 12-site chain from the same random MPS with
    every bond sector at its full size: the energy of every solve equals the
    oracle's single-site sweeps, and the last one exact diagonalisation."""
    lib, problems, gdmrg = mods
    n = 12
    b = synth.chain_bonds(n)
    mpo = synth.heisenberg_mpo(n, b)
    mps = random_mps(mpo, n, (0,), 4096, 4, mps_block)
    g = gdmrg.GpuDMRG(mpo, host_mps(problems, lib, mps), (0,))
    E, swe = g.run_single_site(3, max_iter=40, tol=1e-12)
    oE, _, oswe = dmrg1(mpo, mps, 3)
    e0 = ed.lowest(ed.heisenberg_sector(n, b, n // 2))
    assert len(E) == len(oE)
    assert max(abs(x - y) for x, y in zip(E, oE)) < 1e-9 * abs(e0)
    assert abs(swe[-1] - e0) < 1e-10 * abs(e0)
