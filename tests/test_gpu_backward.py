"""GPU parity of the adjoint of the two-site energy (bsdmrg_heff_backward) and
of the energy entry point against the oracle's reference gradients (each the
full dense contraction with one operand left out), on the same seeded inputs.

Tolerance: norm-wise relative 1e-12 for every gradient (FP64 block GEMMs and
fixed-order reductions against a dense FP64 einsum; the sums have at most a
few thousand terms of random sign).  W gradients are compared on the blocks
that are non-zero in the planned W; the other blocks must be exactly 0.
"""
import numpy as np
import pytest

import synth
from oracle.grad import energy as o_energy, gradients as o_gradients
from oracle.heff import bond_operands, W_SIGNS

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods(gpu_lib):
    from paper_2007_05540_amd import problems, autograd
    return gpu_lib, problems, autograd


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def setup(specs, lib, problems):
    pairs = [problems.bond_problem(s) for s in specs]
    plan = lib.Plan([p for p, _ in pairs])
    ops = problems.concat(plan, [o for _, o in pairs])
    return plan, ops, {k: dev(v) for k, v in ops.items()}


def nz_mask(lib, legs, packed):
    keys, offs = lib.layout(legs, W_SIGNS)
    m = np.zeros(packed.size, dtype=bool)
    for b in range(len(keys)):
        if np.any(packed[offs[b]:offs[b + 1]] != 0.0):
            m[offs[b]:offs[b + 1]] = True
    return m


def run_backward(lib, plan, d, g, want=("psi", "L", "W1", "W2", "R")):
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    out = {k: (torch.full_like(d[k], float("nan")) if k in want else None) for k in ("psi", "L", "W1", "W2", "R")}
    lib.heff_backward(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], g, out["psi"], out["L"], out["W1"],
                      out["W2"], out["R"], ws)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def oracle_grads(spec):
    L, W1, W2, R, psi = bond_operands(spec)
    g = o_gradients(L, W1, W2, R, psi)
    return {k: v.pack() for k, v in g.items()}, o_energy(L, W1, W2, R, psi)


def compare(lib, spec, got, ref, scale=1.0, ops=None):
    wleg = spec.w_leg()
    for k in got:
        r = scale * ref[k]
        if k in ("W1", "W2"):
            m = nz_mask(lib, [wleg, spec.s_leg, spec.s_leg, wleg], ops[k])
            assert np.all(got[k][~m] == 0.0), k
            assert rel(got[k][m], r[m]) < 1e-12, k
        else:
            assert rel(got[k], r) < 1e-12, k
        assert np.all(np.isfinite(got[k])), k


@pytest.mark.parametrize("m,k,seed", [(64, 5, 1), (96, 14, 2), (160, 10, 3), (512, 20, 5)])
def test_backward_matches_oracle(mods, m, k, seed):
    """Up to the m = 512, k = 20 bond of the differentiable J1-J2 workload."""
    lib, problems, _ = mods
    spec = synth.c2_bond(m=m, k=k, seed=seed)
    plan, ops, d = setup([spec], lib, problems)
    got = run_backward(lib, plan, d, 1.0)
    ref, e_ref = oracle_grads(spec)
    compare(lib, spec, got, ref, ops=ops)
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    e = lib.heff_energy(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ws)
    assert abs(e[0] - e_ref) <= 1e-12 * abs(e_ref)


def test_backward_scaled_partial_outputs(mods):
    lib, problems, _ = mods
    spec = synth.c2_bond(m=96, k=14, seed=4)
    plan, ops, d = setup([spec], lib, problems)
    full = run_backward(lib, plan, d, 1.0)
    part = run_backward(lib, plan, d, -0.375, want=("W1", "R"))
    assert set(part) == {"W1", "R"}
    for k in part:   # a power-of-two scale is exact
        assert np.array_equal(part[k], -0.375 * full[k])


def test_backward_batch_per_problem_cotangent(mods):
    lib, problems, _ = mods
    specs = [synth.c2_bond(m=m, k=k, seed=s) for m, k, s in [(64, 10, 11), (96, 14, 12), (80, 18, 13)]]
    gs = [1.0, -2.0, 0.5]
    plan, ops, d = setup(specs, lib, problems)
    got = run_backward(lib, plan, d, gs)
    info = plan.info()
    sizes = {"psi": info["psi_elems"], "L": info["L_elems"], "R": info["R_elems"], "W1": info["W1_elems"],
             "W2": info["W2_elems"]}
    for p, spec in enumerate(specs):
        off = plan.offsets(p)
        nxt = plan.offsets(p + 1) if p + 1 < len(specs) else sizes
        ref, _ = oracle_grads(spec)
        _, o1 = problems.bond_problem(spec)
        piece = {k: got[k][off[k]:nxt[k]] for k in got}
        compare(lib, spec, piece, ref, scale=gs[p], ops=o1)
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    e = lib.heff_energy(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ws)
    for p, spec in enumerate(specs):
        _, e_ref = oracle_grads(spec)
        assert abs(e[p] - e_ref) <= 1e-12 * abs(e_ref)


def test_backward_deterministic_and_euler_identities_full_size(mods):
    """m = 1024, k = 14: two calls are bitwise equal; E is linear in L, W1, W2,
    R (<dE/dX, X> = E) and quadratic in psi (<dE/dpsi, psi> = 2E)."""
    lib, problems, _ = mods
    spec = synth.c2_bond()
    plan, ops, d = setup([spec], lib, problems)
    a = run_backward(lib, plan, d, 1.0)
    b = run_backward(lib, plan, d, 1.0)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    e = lib.heff_energy(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ws)[0]
    for k in ("L", "W1", "W2", "R"):
        assert abs(float(np.dot(a[k], ops[k])) - e) <= 1e-11 * abs(e), k
    assert abs(float(np.dot(a["psi"], ops["psi"])) - 2 * e) <= 1e-11 * abs(e)


def test_backward_rejects_bad_arguments(mods):
    lib, problems, _ = mods
    spec = synth.c2_bond(m=64, k=5, seed=1)
    plan, ops, d = setup([spec], lib, problems)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(d["L"])
    with pytest.raises(lib.BsdmrgError) as e:
        lib.heff_backward(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], 1.0, None, out, None, None, None, small)
    assert e.value.status == lib.EINVAL
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.BsdmrgError):   # output aliases an input
        lib.heff_backward(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], 1.0, None, d["L"], None, None, None, ws)
    with pytest.raises(lib.BsdmrgError):
        lib.heff_backward(plan, d["L"], d["W1"], d["W2"], d["R"], d["psi"], float("nan"), None, out, None, None,
                          None, ws)


def test_autograd_function_and_directional_derivatives(mods):
    """HeffEnergy through torch.autograd: gradients equal the library's
    adjoint, and central differences along random directions agree with
    <grad, direction> (exact for the linear operands, up to rounding)."""
    lib, problems, ag = mods
    spec = synth.c2_bond(m=96, k=14, seed=21)
    plan, ops, d = setup([spec], lib, problems)
    x = {k: v.clone().requires_grad_(True) for k, v in d.items()}
    E = ag.HeffEnergy.apply(plan, x["L"], x["W1"], x["W2"], x["R"], x["psi"])
    (2.5 * E.sum()).backward()
    ref = run_backward(lib, plan, d, 2.5)
    for k in ref:
        assert np.array_equal(x[k].grad.cpu().numpy(), ref[k]), k
    rng = np.random.default_rng(5)
    ws = torch.empty(lib.heff_backward_workspace(plan), dtype=torch.uint8, device="cuda")
    grads = run_backward(lib, plan, d, 1.0)
    for k in ("L", "R", "W1", "psi"):
        dirn = rng.standard_normal(ops[k].size) * (ops[k] != 0)
        h = 1e-3
        ep = dict(d)
        em = dict(d)
        ep[k] = dev(ops[k] + h * dirn)
        em[k] = dev(ops[k] - h * dirn)
        fp = lib.heff_energy(plan, ep["L"], ep["W1"], ep["W2"], ep["R"], ep["psi"], ws)[0]
        fm = lib.heff_energy(plan, em["L"], em["W1"], em["W2"], em["R"], em["psi"], ws)[0]
        fd = (fp - fm) / (2 * h)
        an = float(np.dot(grads[k], dirn))
        assert abs(fd - an) <= 1e-9 * max(abs(an), 1.0), k
