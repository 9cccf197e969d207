"""The product entry point that allocates nothing (bsdmrg_heff_apply_noalloc)
against the workspace entry point (bsdmrg_heff_apply): same kernels, so the
outputs agree bit for bit, on two calls in a row that share the library's
scratch array, the second with a smaller problem; FP64 also within 1e-12 of
the oracle.  A plan larger than the scratch array is refused on the host."""
import numpy as np
import pytest

import synth
from oracle.heff import bond_operands, heff_blocks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _setup(lib, problems, spec):
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    d = {k: torch.from_numpy(v).to("cuda") for k, v in ops.items()}
    return plan, d


def _both(lib, plan, d, prec):
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    ref = torch.full_like(d["psi"], 0.0)
    lib.heff_apply(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], ref, ws)
    got = torch.full_like(d["psi"], 0.0)
    lib.heff_apply_noalloc(plan, prec, d["L"], d["W1"], d["W2"], d["R"], d["psi"], got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_workspace_entry_two_calls(gpu_lib):
    lib = gpu_lib
    from paper_2007_05540_amd import problems
    # first call: the m = 1024, k = 14 bond (FP64 needs 144 MB of the 160 MiB);
    # second call: a smaller bond whose product reuses the same scratch
    for m, k, seed in ((1024, 14, 1), (256, 10, 4)):
        spec = synth.c2_bond(m=m, k=k, seed=seed)
        print(f"noalloc m={m} k={k} seed={seed}", flush=True)
        plan, d = _setup(lib, problems, spec)
        got = {}
        for prec in (lib.F64, lib.F32):
            ref, got[prec] = _both(lib, plan, d, prec)
            assert np.array_equal(ref, got[prec]), (m, prec)
        if m <= 256:
            L, W1, W2, R, psi = bond_operands(spec)
            want = heff_blocks(L, W1, W2, R, psi).pack()
            assert np.linalg.norm(got[lib.F64] - want) <= 1e-12 * np.linalg.norm(want)
        plan.destroy()


def test_noalloc_rejects_plan_above_the_scratch_size(gpu_lib):
    lib = gpu_lib
    from paper_2007_05540_amd import problems
    spec = synth.c2_bond(m=2048, k=14, seed=1)
    prob, _ = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    psi = torch.zeros(plan.info()["psi_elems"], dtype=torch.float64, device="cuda")
    out = torch.zeros_like(psi)
    with pytest.raises(lib.BsdmrgError) as e:
        # the size check happens before any operand is read
        lib.heff_apply_noalloc(plan, lib.F64, psi, psi, psi, psi, psi, out)
    assert e.value.status == lib.EINVAL and "maximum" in str(e.value)
    plan.destroy()
