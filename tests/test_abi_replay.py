"""CPU replay of a full two-site sweep: at every step the library builds (host
only) the plans a GPU sweep would run -- merge, H_eff product, environment
extension -- and checks on the host that every index table stays inside its
buffers.  The shapes come from the oracle's own sweep, which takes the same
truncation decisions."""
import numpy as np
import pytest

import synth
from synth.blocks import mps_block
from oracle.dmrg import random_mps, right_canonicalize, solve_bond
from oracle.env import (left_boundary, right_boundary, left_update_dense, right_update_dense, merge)
from oracle.heff import w_tensor
from oracle.truncate import truncate


@pytest.fixture(scope="module")
def lib():
    from paper_2007_05540_amd import lib as L
    import os
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libbsdmrg.so not built")
    L.load()
    return L


def check_env(op):
    """An environment op and the tables of its adjoint (built and checked on
    the host by the workspace query)."""
    from paper_2007_05540_amd import lib
    assert lib.env_backward_workspace(op) > 0
    op.destroy()


def replay(lib, mpo, n, target, m0, m_max, sweeps, dav):
    from paper_2007_05540_amd import problems
    wl = mpo.w_leg()
    s = mpo.phys
    Wh = [problems.pack_dense(W, [wl, s, s, wl], lib.W_SIGNS) for W in mpo.W]
    Ws = [w_tensor(W, wl, s, wl) for W in mpo.W]
    mps = random_mps(mpo, n, target, m0, 0, mps_block)
    # right canonicalisation shapes (merge plans of every pair)
    for j in range(n - 1, 0, -1):
        A, B = mps[j - 1], mps[j]
        lib.merge_plan(A.legs[0], A.legs[1], A.legs[2], B.legs[1], B.legs[2], host_only=True).destroy()
    mps = right_canonicalize(mps)
    r = len(s[0][0])
    L = [None] * (n + 1)
    R = [None] * (n + 1)
    L[0] = left_boundary(wl, mpo.start, r)
    R[n] = right_boundary(wl, mpo.done, target)
    for j in range(n - 1, 1, -1):
        B = mps[j]
        lib.env_plan(B.legs[2], s, B.legs[0], wl, wl, Wh[j], 1, host_only=True).destroy()
        R[j] = right_update_dense(R[j + 1], B, Ws[j])
    count = 0
    for sw in range(sweeps):
        order = [(j, "right") for j in range(n - 1)] + [(j, "left") for j in range(n - 2, -1, -1)]
        for j, d in order:
            A0, B0 = mps[j], mps[j + 1]
            lib.merge_plan(A0.legs[0], A0.legs[1], A0.legs[2], B0.legs[1], B0.legs[2], host_only=True).destroy()
            theta = merge(A0, B0)
            a, s1, s2, c = theta.legs
            prob = {"a": a, "s1": s1, "s2": s2, "c": c, "wl": wl, "wm": wl, "wr": wl, "w1": Wh[j], "w2": Wh[j + 1]}
            p = lib.Plan([prob], host_only=True)
            assert p.info()["psi_elems"] == theta.pack().size
            assert lib.heff_backward_workspace(p) > 0      # adjoint tables built and checked
            p.destroy()
            lam, x, st = solve_bond(L[j], Ws[j], Ws[j + 1], R[j + 2], theta, dav, "dense", seed=count)
            A, B, _, _, _ = truncate(x, d, cutoff=1e-10, m_max=m_max)
            mps[j], mps[j + 1] = A, B
            if d == "right":
                check_env(lib.env_plan(A.legs[0], s, A.legs[2], wl, wl, Wh[j], 0, host_only=True))
                L[j + 1] = left_update_dense(L[j], A, Ws[j])
            else:
                check_env(lib.env_plan(B.legs[2], s, B.legs[0], wl, wl, Wh[j + 1], 1, host_only=True))
                R[j + 1] = right_update_dense(R[j + 2], B, Ws[j + 1])
            count += 1
    return count


def test_replay_heisenberg_chain_sweep_tables(lib):
    n = 16
    mpo = synth.heisenberg_mpo(n, synth.chain_bonds(n))
    assert replay(lib, mpo, n, (0,), 16, 64, 2, {"max_iter": 40, "tol": 1e-12}) == 2 * 2 * (n - 1)


def test_replay_hubbard_cylinder_sweep_tables(lib):
    W, Lx = 2, 3
    n = W * Lx
    mpo = synth.hubbard_mpo(n, synth.cylinder_j1_bonds(W, Lx), 8.0)
    replay(lib, mpo, n, (n, 0), 32, 64, 1, {"max_iter": 40, "tol": 1e-12})
