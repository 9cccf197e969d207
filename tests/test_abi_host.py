"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and its layout and planner agree with the
oracle bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.blocks import canonical_layout, allowed_keys, block_shape
from oracle.heff import bond_operands, useful_flops, PSI_SIGNS, ENV_SIGNS, W_SIGNS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2007_05540_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libbsdmrg.so not built")
    L.load()
    return L


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "bsdmrg.h")).read()
    return sorted(set(re.findall(r"\b(bsdmrg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    names = declared_symbols()
    assert "bsdmrg_heff_apply" in names and "bsdmrg_eigensolve" in names
    for n in names:
        assert hasattr(so, n), n


@pytest.mark.parametrize("legs,signs", [
    ([synth.spin_bond_leg(200), synth.SPIN_PHYS, synth.SPIN_PHYS, synth.spin_bond_leg(200)], PSI_SIGNS),
    ([synth.spin_bond_leg(300), [((-2,), 4), ((0,), 6), ((2,), 4)], synth.spin_bond_leg(300)], ENV_SIGNS),
    ([[((-2,), 4), ((0,), 6), ((2,), 4)], synth.SPIN_PHYS, synth.SPIN_PHYS, [((-2,), 4), ((0,), 6), ((2,), 4)]],
     W_SIGNS),
    ([synth.electron_bond_leg(512, center=(8, 0)), synth.HUB_PHYS, synth.HUB_PHYS,
      synth.electron_bond_leg(512, center=(10, 0))], PSI_SIGNS),
])
def test_layout_bit_exact_with_oracle(lib, legs, signs):
    keys, offs = lib.layout(legs, signs)
    ok, oo = canonical_layout(legs, signs)
    assert np.array_equal(keys, np.array(ok, dtype=np.int32).reshape(-1, len(legs)))
    assert np.array_equal(offs, np.array(oo, dtype=np.int64))
    assert keys.tobytes() == np.array(ok, dtype=np.int32).reshape(-1, len(legs)).tobytes()


def test_layout_rejects_unsorted_leg(lib):
    with pytest.raises(lib.BsdmrgError) as e:
        lib.layout([[((1,), 1), ((0,), 1)], [((0,), 1)]], (1, -1))
    assert e.value.status == lib.EQN


@pytest.mark.parametrize("m,k,seed", [(128, 14, 1), (256, 10, 2), (200, 18, 3), (512, 20, 4)])
def test_planner_flops_equal_oracle_block_pairs(lib, m, k, seed):
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=m, k=k, seed=seed)
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob], host_only=True)
    info = plan.info()
    ops_o = bond_operands(spec)
    assert info["flops_s1"] + info["flops_s3"] == useful_flops(*ops_o)
    # packed operands equal the oracle's canonical packing
    L, W1, W2, R, psi = ops_o
    assert np.array_equal(ops["psi"], psi.pack()) and np.array_equal(ops["L"], L.pack())


@pytest.mark.parametrize("m,k,seed", [(128, 10, 1), (512, 22, 2)])
def test_planner_flops_equal_oracle_block_pairs_electron_bond(lib, m, k, seed):
    """U(1)xU(1) charges (N, 2Sz), four physical sectors, fermionic MPO."""
    from paper_2007_05540_amd import problems
    spec = synth.c4_bond(m=m, k=k, seed=seed)
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob], host_only=True)
    info = plan.info()
    ops_o = bond_operands(spec)
    assert info["flops_s1"] + info["flops_s3"] == useful_flops(*ops_o)
    L, W1, W2, R, psi = ops_o
    assert np.array_equal(ops["psi"], psi.pack()) and np.array_equal(ops["L"], L.pack())
    assert np.array_equal(ops["W1"], W1.pack())


def test_planner_task_set_equals_brute_force_enumeration(lib):
    """S1 tasks = every (psi block, channel sector) whose bra sector exists,
    found here by brute force over all sector triples."""
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=96, k=14, seed=5)
    prob, _ = problems.bond_problem(spec)
    plan = lib.Plan([prob], host_only=True)
    t1 = plan.tasks(1)
    a, wl = spec.a_leg, spec.w_leg()
    psi_legs = [a, spec.s_leg, spec.s_leg, spec.c_leg]
    brute = []
    for kp in allowed_keys(psi_legs, PSI_SIGNS):
        for f in range(len(wl)):
            for iap in range(len(a)):
                if (iap, f, kp[0]) in set(map(tuple, allowed_keys([a, wl, a], ENV_SIGNS))):
                    brute.append((a[iap][1] * wl[f][1], spec.c_leg[kp[3]][1], a[kp[0]][1], 1))
    assert sorted(map(tuple, t1.tolist())) == sorted(brute)


def test_plan_rejects_physical_dim_above_one(lib):
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=32, k=5, seed=1)
    prob, _ = problems.bond_problem(spec)
    prob = dict(prob)
    prob["s1"] = [((-1,), 2), ((1,), 1)]
    with pytest.raises(lib.BsdmrgError):
        lib.Plan([prob], host_only=True)


@pytest.mark.parametrize("m,k,seed", [(64, 5, 1), (256, 14, 2), (1024, 14, 1)])
def test_adjoint_tables_build_and_pass_host_checks(lib, m, k, seed):
    """The adjoint's tables are built (and every index table checked on the
    host) by the first query; its workspace holds the product's and more."""
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=m, k=k, seed=seed)
    prob, _ = problems.bond_problem(spec)
    plan = lib.Plan([prob, prob], host_only=True)
    info = plan.info()
    assert info["backward_workspace_bytes"] == 0          # tables not built yet
    need = lib.heff_backward_workspace(plan)
    assert need > info["apply_workspace_bytes"] + 8 * (info["t1_elems"] + info["t2_elems"])
    assert plan.info()["backward_workspace_bytes"] == need
    assert lib.heff_backward_workspace(plan) == need


def test_truncate_rejects_charge_matrix_above_4096_columns(lib):
    """The truncation SVD holds a pair of column blocks of a charge matrix in
    the 128 KB of LDS of one workgroup: charge matrices above 4096 columns
    are refused on the host (EINVAL) before any launch."""
    big = [((0,), 4100)]
    legs = [big, synth.SPIN_PHYS, synth.SPIN_PHYS, big]
    with pytest.raises(lib.BsdmrgError) as e:
        lib.truncate_workspace(legs)
    assert e.value.status == lib.EINVAL
    ok = [((0,), 4000)]
    assert lib.truncate_workspace([ok, synth.SPIN_PHYS, synth.SPIN_PHYS, ok]) > 0


def test_plan_rejects_bond_sector_above_4096(lib):
    """A bond sector above 4096 states exceeds one mixing work item: refused
    on the host (EINVAL)."""
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=64, k=5, seed=1)
    wl, s = spec.w_leg(), spec.s_leg
    prob = {"a": [((0,), 8)], "s1": s, "s2": s, "c": [((0,), 5000)], "wl": wl, "wm": wl, "wr": wl,
            "w1": problems.pack_dense(spec.W1, [wl, s, s, wl], lib.W_SIGNS),
            "w2": problems.pack_dense(spec.W2, [wl, s, s, wl], lib.W_SIGNS)}
    with pytest.raises(lib.BsdmrgError) as e:
        lib.Plan([prob], host_only=True)
    assert e.value.status == lib.EINVAL


@pytest.mark.parametrize("name,spec_fn,expect", [
    ("spin m=128", lambda: synth.c2_bond(m=128, k=14, seed=3), 512),
    ("spin m=1024", lambda: synth.c2_bond(m=1024, k=14, seed=1), 512),
    ("spin m=2048", lambda: synth.c2_bond(m=2048, k=14, seed=1), 1024),
    ("electron m=4096", lambda: synth.c4_bond(m=4096, k=22, seed=1), 0),
])
def test_s3_split_width_rule(lib, name, spec_fn, expect):
    """S3 split-K width: the widest of none, 4096, 2048, 1024 that keeps at
    least 3072 S3 tiles, else 512."""
    from paper_2007_05540_amd import problems
    prob, _ = problems.bond_problem(spec_fn())
    plan = lib.Plan([prob], host_only=True)
    info = plan.info()
    plan.destroy()
    assert info["s3_split_k"] in (0, 4096, 2048, 1024, 512)
    assert info["s3_split_k"] == expect, name
    if info["s3_split_k"] != 512:
        assert info["n_s3_tiles"] >= 3072


def test_dense_plan_host_only(lib):
    """The sparse-dense op: flops of its three stages equal the dense GEMM
    counts, out_elems = ma d^2 mc, and the workspace covers T1, T2 (ma k d^2
    mc each) and WW in FP64; out-of-range shapes are rejected."""
    from paper_2007_05540_amd import dense
    ma, mc, k, d = 150, 130, 14, 2
    op = lib.dense_plan(ma, mc, k, d, host_only=True)
    q = op.query()
    f1, f2, f3 = dense.dense_flops(ma, mc, k, d)
    assert q["flops"] == pytest.approx(f1 + f2 + f3, rel=1e-12)
    assert q["out_elems"] == ma * d * d * mc
    assert q["workspace_bytes"] >= 8 * (2 * ma * k * d * d * mc + (d * d * k) ** 2)
    op.destroy()
    for bad in ((0, 4, 2, 2), (4, 4, 0, 2), (4, 4, 2, 9), (1 << 20, 1 << 20, 14, 2)):
        with pytest.raises(lib.BsdmrgError):
            lib.dense_plan(*bad, host_only=True)
