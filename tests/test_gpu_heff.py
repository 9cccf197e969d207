"""GPU parity of the two-site product and the Davidson eigensolver against the
CPU oracle (same seeded inputs, compared element by element).

Tolerances
  FP64 product: norm-wise relative 1e-12 (the required agreement).
  FP32 product: block GEMMs accumulate K <= 14 * 270 products in FP32; the
    worst-case relative error of one output is ~K * 2^-24 ~ 2e-4 and the
    typical (random-sign) one sqrt(K) * 2^-24 ~ 4e-6; the test bounds the
    norm-wise relative error by 5e-5.
  Ritz values (fixed iteration count): relative 1e-11 (FP64 basis built in a
    different summation order; the Krylov sequence is stable for these steps).
"""
import numpy as np
import pytest

import synth
from oracle.blocks import BlockTensor
from oracle.eig import davidson
from oracle.dmrg import mask_of
from oracle.heff import bond_operands, heff_blocks, PSI_SIGNS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def setup(specs, lib, problems):
    pairs = [problems.bond_problem(s) for s in specs]
    plan = lib.Plan([p for p, _ in pairs])
    ops = problems.concat(plan, [o for _, o in pairs])
    d = {k: dev(v) for k, v in ops.items()}
    return plan, ops, d


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def blockwise_max_rel(lib, got, ref, legs):
    """Largest ||got_b - ref_b|| / ||ref_b|| over the blocks of the canonical
    layout with a non-zero reference block (the small edge sectors count as
    much as the large ones)."""
    keys, offs = lib.layout(legs, PSI_SIGNS)
    worst = 0.0
    for b in range(len(keys)):
        r = ref[offs[b]:offs[b + 1]]
        nr = np.linalg.norm(r)
        if nr > 0.0:
            worst = max(worst, float(np.linalg.norm(got[offs[b]:offs[b + 1]] - r) / nr))
    return worst


def oracle_apply(spec, psi_flat=None):
    L, W1, W2, R, psi = bond_operands(spec)
    if psi_flat is not None:
        psi = BlockTensor.unpack(psi_flat, psi.legs, PSI_SIGNS)
    return heff_blocks(L, W1, W2, R, psi).pack()


@pytest.fixture(scope="module")
def mods(gpu_lib):
    from paper_2007_05540_amd import problems
    return gpu_lib, problems


CASES = [(64, 5, 1), (96, 14, 2), (256, 14, 3), (256, 10, 4), (200, 18, 5)]


@pytest.mark.parametrize("m,k,seed", CASES)
def test_apply_f64_matches_oracle(mods, m, k, seed):
    lib, problems = mods
    spec = synth.c2_bond(m=m, k=k, seed=seed)
    plan, ops, d = setup([spec], lib, problems)
    info = plan.info()
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(info["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle_apply(spec)
    assert rel(got, ref) < 1e-12
    # padding of out is left untouched (zero here)
    mask = mask_of([spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg], PSI_SIGNS)
    assert np.all(got[~mask] == 0.0)


def test_smallest_bond_apply_and_eigensolve(mods):
    """m = 2: one sector per bond leg, two 2 x 2 psi blocks (dimension 8):
    product against the oracle, and a solve capped by the dimension that
    returns the dense lowest eigenvalue."""
    lib, problems = mods
    spec = synth.c2_bond(m=2, k=5, seed=2)
    assert len(spec.a_leg) == 1
    plan, ops, d = setup([spec], lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), oracle_apply(spec)) < 1e-12
    lam, _, ost, _ = oracle_davidson(spec, 40, tol=-1.0)
    e, st, _ = run_eig(lib, plan, d, lib.eig_opts(max_iter=40, tol=1e-14))
    assert abs(e[0] - lam) < 1e-12 * abs(lam) and st[0]["iters"] <= 8


def test_apply_f64_full_size_mid_chain_bond(mods):
    """m = 1024, k = 14: the full-size isolated bond, whole output compared."""
    lib, problems = mods
    spec = synth.c2_bond()
    plan, ops, d = setup([spec], lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    got, ref = out.cpu().numpy(), oracle_apply(spec)
    assert rel(got, ref) < 1e-12
    assert blockwise_max_rel(lib, got, ref, [spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg]) < 1e-12


ELECTRON_CASES = [(96, 10, 1), (256, 22, 2), (1024, 22, 3)]


@pytest.mark.parametrize("m,k,seed", ELECTRON_CASES)
def test_apply_f64_electron_bond_matches_oracle(mods, m, k, seed):
    """U(1)xU(1) (N, 2Sz) bonds of the electron sector model with a
    Hubbard-type MPO (fermionic strands, four physical sectors)."""
    lib, problems = mods
    spec = synth.c4_bond(m=m, k=k, seed=seed)
    plan, ops, d = setup([spec], lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert rel(got, oracle_apply(spec)) < 1e-12
    mask = mask_of([spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg], PSI_SIGNS)
    assert np.all(got[~mask] == 0.0)


def test_apply_hubbard_bond_full_size(mods):
    """m = 4096, k = 22 (313 sectors, 22476 S1 tasks): the full-size bond in
    the bench's launch configuration; FP64 output compared element by element
    with the oracle, FP32 output within the FP32 bound."""
    lib, problems = mods
    spec = synth.c4_bond(m=4096, k=22, seed=1)
    plan, ops, d = setup([spec], lib, problems)
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    outs = {}
    for prec in (lib.F64, lib.F32):
        out = torch.zeros_like(d["psi"])
        lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
        torch.cuda.synchronize()
        outs[prec] = out.cpu().numpy()
    del ws, d
    ref = oracle_apply(spec)
    assert rel(outs[lib.F64], ref) < 1e-12
    assert blockwise_max_rel(lib, outs[lib.F64], ref, [spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg]) < 1e-12
    assert 1e-9 < rel(outs[lib.F32], ref) < 5e-5


@pytest.mark.parametrize("spec_fn,width", [(lambda: synth.c2_bond(m=1024, k=14, seed=1), 512),
                                            (lambda: synth.c2_bond(m=2048, k=14, seed=1), 1024)])
def test_apply_split_k_widths_match_oracle(mods, spec_fn, width):
    """The plan's S3 split-K width (512 at m=1024, 1024 at m=2048; the m=4096
    electron bond is unsplit): FP64 output element by element against the
    oracle, FP32 within the FP32 bound."""
    lib, problems = mods
    spec = spec_fn()
    plan, ops, d = setup([spec], lib, problems)
    info = plan.info()
    assert info["s3_split_k"] == width
    ws = torch.empty(info["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    outs = {}
    for prec in (lib.F64, lib.F32):
        out = torch.zeros_like(d["psi"])
        lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
        torch.cuda.synchronize()
        outs[prec] = out.cpu().numpy()
    del ws, d
    ref = oracle_apply(spec)
    assert rel(outs[lib.F64], ref) < 1e-12
    assert 1e-9 < rel(outs[lib.F32], ref) < 5e-5


def test_apply_f32_within_fp32_bound(mods):
    lib, problems = mods
    spec = synth.c2_bond(m=512, k=14, seed=7)
    plan, ops, d = setup([spec], lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F32, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    err = rel(out.cpu().numpy(), oracle_apply(spec))
    assert 1e-9 < err < 5e-5        # really FP32 (not silently FP64), within the bound


def test_apply_deterministic(mods):
    lib, problems = mods
    spec = synth.c2_bond(m=256, k=14, seed=9)
    plan, ops, d = setup([spec], lib, problems)
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    outs = []
    for prec in (lib.F64, lib.F64, lib.F32, lib.F32):
        out = torch.zeros_like(d["psi"])
        lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
        outs.append(out.cpu())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[2], outs[3])


def test_stage_timing_of_the_solve_stages(mods):
    """bsdmrg_stage_timing with F32_REFINE times the stages as the FP32 phase
    of a mixed eigensolve runs them (FP32 products: S3 and its split-K sum
    write FP32 results) and leaves out holding the FP32 product, equal bit for
    bit to bsdmrg_heff_apply's, as the F32 timing does; an unknown precision
    is rejected."""
    lib, problems = mods
    spec = synth.c2_bond(m=1024, k=14, seed=1)
    plan, ops, d = setup([spec], lib, problems)
    info = plan.info()
    assert info["s3_split_k"] > 0   # the split-K sum is among the timed stages
    ws = torch.empty(info["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    ref = torch.zeros_like(d["psi"])
    lib.heff_apply(plan, lib.F32, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ref, ws)
    for prec in (lib.F32, lib.F32_REFINE):
        out = torch.zeros_like(d["psi"])
        ms = lib.stage_timing(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws, reps=2)
        assert all(ms[k] > 0.0 for k in ("s1", "s2", "s3", "s3_sum"))
        assert torch.equal(out.cpu(), ref.cpu())
    with pytest.raises(lib.BsdmrgError):
        lib.stage_timing(plan, 7, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ref, ws, reps=1)


def test_apply_batch_equals_single(mods):
    lib, problems = mods
    specs = [synth.c2_bond(m=m, k=k, seed=s) for m, k, s in [(64, 10, 1), (128, 14, 2), (96, 18, 3)]]
    plan, ops, d = setup(specs, lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for p, spec in enumerate(specs):
        o = plan.offsets(p)["psi"]
        ref = oracle_apply(spec)
        assert rel(got[o:o + ref.size], ref) < 1e-12


def test_apply_rejects_bad_arguments(mods):
    lib, problems = mods
    spec = synth.c2_bond(m=64, k=5, seed=1)
    plan, ops, d = setup([spec], lib, problems)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros_like(d["psi"])
    with pytest.raises(lib.BsdmrgError) as e:
        lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    assert e.value.status == lib.EINVAL
    with pytest.raises(lib.BsdmrgError):
        lib.heff_apply(plan, 7, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)


@pytest.mark.parametrize("spec_fn", [lambda: synth.c2_bond(m=512, k=14, seed=31),
                                     lambda: synth.c4_bond(m=512, k=22, seed=32)])
def test_tile_shape_classes_bit_identical_and_autotune(mods, spec_fn):
    """128 x 128 tiles for large tasks (forced with a low threshold, and as
    chosen by the autotuner) give the same products bit for bit as 64 x 64
    tiles only, in both precisions; FP64 matches the oracle."""
    lib, problems = mods
    spec = spec_fn()
    plan, ops, d = setup([spec], lib, problems)
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")

    def products():
        res = {}
        for prec in (lib.F64, lib.F32):
            out = torch.zeros_like(d["psi"])
            lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
            torch.cuda.synchronize()
            res[prec] = out.cpu().numpy()
        return res
    assert plan.info()["s1_big_min"] == lib.NO_BIG_TILES
    base = products()
    lib.plan_set_tiles(plan, 0, 0)                 # persistent launch of both stages
    assert plan.info()["s1_big_min"] == 0 and plan.info()["s3_big_min"] == 0
    persistent = products()
    lib.plan_set_tiles(plan, 64, 64)
    info = plan.info()
    assert info["s1_big_min"] == 64 and info["s3_big_min"] == 64
    forced = products()
    out = torch.zeros_like(d["psi"])
    got = lib.plan_autotune(plan, lib.F32, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws, reps=3)
    classes = (lib.NO_BIG_TILES, 0, 384, 256, 160, 96)
    assert got["s1"] in classes and got["s3"] in classes
    assert plan.info()["s3_big_min"] == got["s3"]
    assert np.array_equal(out.cpu().numpy(), base[lib.F32])
    tuned = products()
    for prec in (lib.F64, lib.F32):
        assert np.array_equal(persistent[prec], base[prec])
        assert np.array_equal(forced[prec], base[prec])
        assert np.array_equal(tuned[prec], base[prec])
    assert rel(base[lib.F64], oracle_apply(spec)) < 1e-12
    # a captured solve after a re-schedule uses the new tables
    o = lib.eig_opts(max_iter=4, fixed_iters=1, use_graph=1)
    e1, _, _ = run_eig(lib, plan, d, o)
    lib.plan_set_tiles(plan, lib.NO_BIG_TILES, lib.NO_BIG_TILES)
    e2, _, _ = run_eig(lib, plan, d, o)
    assert e1[0] == e2[0]


def test_sector_wider_than_2048_matches_oracle(mods):
    """A right bond leg with one 2100-wide sector: the S2 and split-K-sum
    launches then take 16 outputs per thread (items of up to 4096) instead of
    8; the product equals the oracle in FP64 (1e-12) and FP32 (1e-5)."""
    lib, problems = mods
    from synth.blocks import BondSpec, synthetic_heisenberg_bond
    a = [((-2,), 5), ((0,), 6), ((2,), 5)]
    c = [((0,), 2100)]
    spec = BondSpec(a, c, synthetic_heisenberg_bond(14, 5), 5, name="wide sector")
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    d = {k: dev(v) for k, v in ops.items()}
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    ref = oracle_apply(spec)
    for precision, tol in ((lib.F64, 1e-12), (lib.F32, 1e-5)):
        out = torch.zeros_like(d["psi"])   # the product does not write the padding
        lib.heff_apply(plan, precision, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
        torch.cuda.synchronize()
        assert rel(out.cpu().numpy(), ref) < tol
    plan.destroy()


@pytest.mark.parametrize("m", [96, 150])
def test_dense_format_ablation_matches_oracle(mods, m):
    """The sparse-dense format (every operand one dense array, the product
    run by the library's three grouped-GEMM stages on them) computes the
    same product: FP64 within 1e-12 of the oracle, FP32 within 1e-5 (FP32
    MFMA sums over up to k m terms), and exactly zero outside the allowed
    blocks in FP64.  m = 150 leaves ragged 64 x 64 tiles in every stage."""
    lib, problems = mods
    from paper_2007_05540_amd import dense
    spec = synth.c2_bond(m=m, k=14, seed=41)
    prob, ops = problems.bond_problem(spec)
    wl, s = spec.w_leg(), spec.s_leg
    legs_psi = [spec.a_leg, s, s, spec.c_leg]
    Ld = dev(problems.unpack_dense(ops["L"], [spec.a_leg, wl, spec.a_leg], lib.ENV_SIGNS))
    Rd = dev(problems.unpack_dense(ops["R"], [spec.c_leg, wl, spec.c_leg], lib.ENV_SIGNS))
    pd = dev(problems.unpack_dense(ops["psi"], legs_psi, lib.PSI_SIGNS))
    ma, k, _ = Ld.shape
    dp = dense.DenseProduct(ma, Rd.shape[0], k, pd.shape[1])
    ref = oracle_apply(spec)
    for precision, tol in ((lib.F64, 1e-12), (lib.F32, 1e-5)):
        out = torch.full_like(pd, float("nan"))
        dp.apply(precision, Ld, dev(spec.W1), dev(spec.W2), Rd, pd, out)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        got = problems.pack_dense(out, legs_psi, lib.PSI_SIGNS)
        assert rel(got, ref) < tol
        if precision == lib.F64:
            assert np.array_equal(problems.unpack_dense(got, legs_psi, lib.PSI_SIGNS), out)
    f1, f2, f3 = dense.dense_flops(ma, Rd.shape[0], k, pd.shape[1])
    assert dp.flops == pytest.approx(f1 + f2 + f3, rel=1e-12)
    dp.destroy()


# ------------------------------------------------------------ eigensolver ---
def oracle_davidson(spec, n_iter, tol=0.0, seed=0):
    L, W1, W2, R, psi = bond_operands(spec)

    def mv(v):
        return heff_blocks(L, W1, W2, R, BlockTensor.unpack(v, psi.legs, PSI_SIGNS)).pack()
    rec = []
    lam, x, st = davidson(mv, psi.pack(), n_iter, tol, restart_mask=mask_of(psi.legs, PSI_SIGNS),
                          seed=seed, record=rec)
    return lam, x, st, rec


def run_eig(lib, plan, d, opts, stream=None):
    ws = torch.empty(lib.eig_workspace(plan, opts), dtype=torch.uint8, device="cuda")
    psi = d["psi"].clone()
    e, st = lib.eigensolve(plan, d["L"], d["W1"], d["W2"], d["R"], psi, opts, ws, stream=stream)
    return e, st, psi


@pytest.mark.parametrize("m,k,n_iter", [(64, 5, 8), (256, 14, 10)])
def test_eigensolve_fixed_iterations_match_oracle(mods, m, k, n_iter):
    lib, problems = mods
    spec = synth.c2_bond(m=m, k=k, seed=11)
    plan, ops, d = setup([spec], lib, problems)
    opts = lib.eig_opts(max_iter=n_iter, fixed_iters=1)
    e, st, psi = run_eig(lib, plan, d, opts)
    lam, x, ost, rec = oracle_davidson(spec, n_iter)
    assert abs(e[0] - lam) < 1e-11 * abs(lam)
    assert st[0]["iters"] == n_iter
    ov = abs(float(np.dot(psi.cpu().numpy(), x)))
    assert abs(ov - 1.0) < 1e-9


def test_eigensolve_converges_to_dense_lowest(mods):
    lib, problems = mods
    spec = synth.c2_bond(m=24, k=5, seed=4)
    plan, ops, d = setup([spec], lib, problems)
    opts = lib.eig_opts(max_iter=64, tol=1e-10)
    e, st, psi = run_eig(lib, plan, d, opts)
    lam, x, ost, _ = oracle_davidson(spec, 64, tol=1e-10)
    assert st[0]["converged"] == 1
    assert abs(e[0] - lam) < 1e-10 * abs(lam)
    # residual of the returned vector through the GPU product
    out = torch.zeros_like(psi)
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], psi, out, ws)
    r = out.cpu().numpy() - e[0] * psi.cpu().numpy()
    assert np.linalg.norm(r) < 1e-8


def test_eigensolve_mixed_precision_energy(mods):
    """FP32 products, then FP64 refinement restarted from the FP32 Ritz vector:
    the final energy agrees with the converged FP64 oracle to 1e-9."""
    lib, problems = mods
    spec = synth.c2_bond(m=24, k=5, seed=4)
    plan, ops, d = setup([spec], lib, problems)
    lam, x, ost, _ = oracle_davidson(spec, 64, tol=1e-10)
    assert ost["converged"]
    o = lib.eig_opts(max_iter=64, precision=lib.F32_REFINE, refine_max_iter=64, tol=1e-10, tol_f32=1e-5)
    e32, st32, psi = run_eig(lib, plan, d, o)
    assert st32[0]["iters_f32"] >= 1 and st32[0]["iters"] >= 1
    assert abs(e32[0] - lam) < 1e-9 * abs(lam)
    # eigenvector error 1 - |<psi, psi_oracle>| (both normalised): a residual
    # of 1e-10 bounds it by ~(1e-10 / gap)^2
    assert 1.0 - abs(float(np.dot(psi.cpu().numpy(), x))) < 1e-12


def test_eigensolve_mixed_precision_energy_electron_bond(mods):
    lib, problems = mods
    spec = synth.c4_bond(m=40, k=10, seed=6)
    plan, ops, d = setup([spec], lib, problems)
    lam, _, ost, _ = oracle_davidson(spec, 64, tol=1e-10)
    assert ost["converged"]
    o = lib.eig_opts(max_iter=64, precision=lib.F32_REFINE, refine_max_iter=64, tol=1e-10, tol_f32=1e-5)
    e32, st32, _ = run_eig(lib, plan, d, o)
    assert st32[0]["iters_f32"] >= 1 and st32[0]["iters"] >= 1
    assert abs(e32[0] - lam) < 1e-9 * abs(lam)


def test_eigensolve_stops_when_basis_spans_the_space(mods):
    """dim(psi) < max_iter and a tolerance the FP32 phase cannot reach: both
    paths stop once the basis spans the space (no restart failure) and give
    the dense lowest eigenvalue."""
    lib, problems = mods
    spec = synth.c2_bond(m=4, k=5, seed=8)
    plan, ops, d = setup([spec], lib, problems)
    mask = mask_of([spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg], PSI_SIGNS)
    dim = int(mask.sum())
    assert dim < 64
    lam, _, ost, _ = oracle_davidson(spec, 64, tol=-1.0)
    assert ost["iters"] == dim
    for o in (lib.eig_opts(max_iter=64, tol=1e-14),
              lib.eig_opts(max_iter=64, precision=lib.F32_REFINE, refine_max_iter=64, tol=1e-14, tol_f32=1e-14)):
        e, st, _ = run_eig(lib, plan, d, o)
        assert st[0]["restarts"] == 0
        assert abs(e[0] - lam) < 1e-11 * abs(lam)
        assert st[0]["iters"] <= dim and st[0]["iters_f32"] <= dim


def test_eigensolve_graph_replay_equals_eager(mods):
    lib, problems = mods
    spec = synth.c2_bond(m=128, k=14, seed=12)
    plan, ops, d = setup([spec], lib, problems)
    s = torch.cuda.Stream()
    eager = lib.eig_opts(max_iter=6, fixed_iters=1, use_graph=0)
    graph = lib.eig_opts(max_iter=6, fixed_iters=1, use_graph=1)
    e0, _, p0 = run_eig(lib, plan, d, eager, stream=s)
    ws = torch.empty(lib.eig_workspace(plan, graph), dtype=torch.uint8, device="cuda")
    for rep in range(3):
        psi = d["psi"].clone()
        torch.cuda.synchronize()
        e1, _ = lib.eigensolve(plan, d["L"], d["W1"], d["W2"], d["R"], psi, graph, ws, stream=s)
        torch.cuda.synchronize()
        assert e1[0] == e0[0]
        assert torch.equal(psi.cpu(), p0.cpu())
        # eager work between replays
        lib.eigensolve(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"].clone(), eager,
                       torch.empty(lib.eig_workspace(plan, eager), dtype=torch.uint8, device="cuda"),
                       stream=s)


def test_eigensolve_batch_matches_single(mods):
    lib, problems = mods
    specs = [synth.c2_bond(m=m, k=k, seed=s) for m, k, s in [(64, 10, 21), (128, 14, 22), (96, 18, 23)]]
    plan, ops, d = setup(specs, lib, problems)
    opts = lib.eig_opts(max_iter=8, fixed_iters=1)
    e, st, psi = run_eig(lib, plan, d, opts)
    for p, spec in enumerate(specs):
        lam, x, _, _ = oracle_davidson(spec, 8)
        assert abs(e[p] - lam) < 1e-11 * abs(lam)


def test_eigensolve_restart_on_breakdown(mods):
    """H_eff = identity (unit environments and MPO): q = 0 after the first
    step, so the seeded random restart must be taken; the Ritz values and the
    restarted basis follow the oracle's identical counter-based stream."""
    lib, problems = mods
    leg = synth.spin_bond_leg(40)
    s = synth.SPIN_PHYS
    wl = [((0,), 1)]
    W = np.eye(2).reshape(1, 2, 2, 1)
    prob = {"a": leg, "s1": s, "s2": s, "c": leg, "wl": wl, "wm": wl, "wr": wl,
            "w1": problems.pack_dense(W, [wl, s, s, wl], lib.W_SIGNS),
            "w2": problems.pack_dense(W, [wl, s, s, wl], lib.W_SIGNS)}
    eye = lambda k: np.eye(leg[k[0]][1]).reshape(leg[k[0]][1], 1, leg[k[0]][1])
    L = problems.pack_fn([leg, wl, leg], lib.ENV_SIGNS, eye)
    psi = problems.pack_fn([leg, s, s, leg], lib.PSI_SIGNS,
                           lambda k: synth.gaussian_block(3, 4, k, (leg[k[0]][1], 1, 1, leg[k[3]][1])))
    plan = lib.Plan([prob])
    d = {"L": dev(L), "R": dev(L), "W1": dev(prob["w1"]), "W2": dev(prob["w2"]), "psi": dev(psi)}
    opts = lib.eig_opts(max_iter=3, fixed_iters=1, seed=5)
    e, st, out = run_eig(lib, plan, d, opts)
    assert st[0]["restarts"] >= 1 and abs(e[0] - 1.0) < 1e-14


def test_batch_c3_shape_with_the_largest_bond(mods):
    """A batch of the shape of the 64-bond workload including its largest
    bond (m = 2048, k = 18, 25 sectors) beside an m = 1024, k = 10 and an
    m = 256, k = 14 bond: the batched FP64 product of every problem against
    the oracle (norm-wise and block by block), and a batched fixed 6-step
    eigensolve against the oracle's Davidson per problem."""
    lib, problems = mods
    specs = [synth.c2_bond(m=2048, k=18, seed=101), synth.c2_bond(m=1024, k=10, seed=102),
             synth.c2_bond(m=256, k=14, seed=103)]
    plan, ops, d = setup(specs, lib, problems)
    out = torch.zeros_like(d["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    del ws, out
    for p, spec in enumerate(specs):
        o = plan.offsets(p)["psi"]
        ref = oracle_apply(spec)
        piece = got[o:o + ref.size]
        print(f"batch problem {p}: rel {rel(piece, ref):.2e}", flush=True)
        assert rel(piece, ref) < 1e-12
        assert blockwise_max_rel(lib, piece, ref, [spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg]) < 1e-12
    opts = lib.eig_opts(max_iter=6, fixed_iters=1)
    e, st, _ = run_eig(lib, plan, d, opts)
    for p, spec in enumerate(specs):
        lam, _, _, _ = oracle_davidson(spec, 6)
        assert abs(e[p] - lam) < 1e-11 * abs(lam)


@pytest.mark.parametrize("spec_fn", [lambda: synth.c2_bond(m=1024, k=14, seed=1),
                                     lambda: synth.c2_bond(m=2048, k=18, seed=2),
                                     lambda: synth.c4_bond(m=4096, k=22, seed=1)])
def test_persistent_launch_bit_identical_at_full_size(mods, spec_fn):
    """The persistent launch of both GEMM stages (one workgroup per resident
    slot, tiles dealt on the host) gives the same products bit for bit as one
    workgroup per tile, in both precisions, on the full-size bonds (split-K
    S3 at m = 1024 and 2048, 313 electron sectors at m = 4096)."""
    lib, problems = mods
    spec = spec_fn()
    plan, ops, d = setup([spec], lib, problems)
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    res = {}
    for mode in (lib.NO_BIG_TILES, 0):
        lib.plan_set_tiles(plan, mode, mode)
        for prec in (lib.F64, lib.F32):
            out = torch.full_like(d["psi"], 0.0)
            lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], out, ws)
            torch.cuda.synchronize()
            res[(mode, prec)] = out.cpu().numpy()
    for prec in (lib.F64, lib.F32):
        assert np.array_equal(res[(0, prec)], res[(lib.NO_BIG_TILES, prec)])
