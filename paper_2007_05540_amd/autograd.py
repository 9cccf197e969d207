"""torch.autograd wrappers of the library's two-site energy and its adjoint.

``HeffEnergy.apply(plan, L, W1, W2, R, psi)`` returns the energies
E_p = psi_p^T H_eff,p psi_p of every problem of the plan (a float64 tensor of
n_probs entries on the device of psi).  Its backward calls the hand-written
adjoint of the library (``bsdmrg_heff_backward``): gradients for L, W1, W2, R
and psi, each in the canonical block layout of its operand, scaled per
problem by the incoming cotangent.  torch only owns the buffers and the
stream; the energy and every gradient are computed by the library's kernels.
"""
import torch

from . import lib


def _check(x, name):
    if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 device tensor")


class HeffEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, L, W1, W2, R, psi):
        for x, n in ((L, "L"), (W1, "W1"), (W2, "W2"), (R, "R"), (psi, "psi")):
            _check(x, n)
        ws = torch.empty(max(1, lib.heff_backward_workspace(plan)), dtype=torch.uint8, device=psi.device)
        e = lib.heff_energy(plan, L, W1, W2, R, psi, ws)
        ctx.plan = plan
        ctx.save_for_backward(L, W1, W2, R, psi)
        return torch.tensor(e, dtype=torch.float64, device=psi.device)

    @staticmethod
    def backward(ctx, g_e):
        L, W1, W2, R, psi = ctx.saved_tensors
        need = ctx.needs_input_grad[1:]
        outs = [torch.empty_like(x) if n else None for x, n in zip((L, W1, W2, R, psi), need)]
        if not any(n for n in need):
            return (None,) * 6
        ws = torch.empty(max(1, lib.heff_backward_workspace(ctx.plan)), dtype=torch.uint8, device=psi.device)
        g = g_e.detach().to("cpu", torch.float64).numpy()
        lib.heff_backward(ctx.plan, L, W1, W2, R, psi, g, outs[4], outs[0], outs[1], outs[2], outs[3], ws)
        return (None, *outs)


class EnvUpdate(torch.autograd.Function):
    """env_out = extension of env through one site (an environment op of the
    library).  ``op_adj`` is the op of the opposite side over the same site
    (old and new bond swapped): it maps the output cotangent to the cotangent
    of env.  The cotangent of W comes from the library's adjoint of the op;
    the site tensor is held fixed (no gradient)."""

    @staticmethod
    def forward(ctx, op, op_adj, env, site, W):
        for x, n in ((env, "env"), (site, "site"), (W, "W")):
            _check(x, n)
        info = op.query()
        out = torch.zeros(max(1, info["out_elems"]), dtype=torch.float64, device=env.device)
        ws = torch.empty(max(1, info["workspace_bytes"]), dtype=torch.uint8, device=env.device)
        lib.env_update(op, env, site, W, out, ws)
        ctx.op, ctx.op_adj = op, op_adj
        ctx.save_for_backward(env, site, W)
        return out

    @staticmethod
    def backward(ctx, d_out):
        env, site, W = ctx.saved_tensors
        if ctx.needs_input_grad[3]:
            raise NotImplementedError("EnvUpdate: the site tensor has no gradient (the MPS is held fixed)")
        d_out = d_out.contiguous()
        d_env = d_w = None
        if ctx.needs_input_grad[2]:
            info = ctx.op_adj.query()
            d_env = torch.zeros_like(env)
            ws = torch.empty(max(1, info["workspace_bytes"]), dtype=torch.uint8, device=env.device)
            lib.env_update(ctx.op_adj, d_out, site, W, d_env, ws)
        if ctx.needs_input_grad[4]:
            d_w = torch.empty_like(W)
            ws = torch.empty(max(1, lib.env_backward_workspace(ctx.op)), dtype=torch.uint8, device=env.device)
            lib.env_backward(ctx.op, env, site, d_out, d_w, ws)
        return None, None, d_env, None, d_w
