"""The sparse-dense format of Sec. IV-A on the GPU, as an ablation of the
block-sparse list path: every operand of the two-site product embedded in one
dense array (the forbidden blocks are zeros) and the product run by the
library's grouped GEMM stages on those arrays (bsdmrg_dense_plan /
bsdmrg_dense_apply).  It computes the same product with all the work that the
block structure avoids; its only use is to measure that work.

Index names as in the block-sparse path: L (a', w, a), W_i (w, s1', s1, v),
W_{i+1} (v, s2', s2, w''), R (c', w'', c), psi (a, s1, s2, c).
"""
from . import lib


def dense_flops(m_a, m_c, k, d):
    """Flops of the three dense GEMMs (S1, the MPO mixing, S3)."""
    s1 = 2.0 * (m_a * k) * m_a * (d * d * m_c)
    s2 = 2.0 * (m_a * m_c) * (k * d * d) * (d * d * k)
    s3 = 2.0 * (m_a * d * d) * (k * m_c) * m_c
    return s1, s2, s3


class DenseProduct:
    """H_eff psi in the dense format for fixed (m_a, m_c, k, d): the op and
    its workspace are made once; apply() runs the three library stages."""

    def __init__(self, m_a, m_c, k, d, device="cuda"):
        import torch
        self.op = lib.dense_plan(m_a, m_c, k, d)
        q = self.op.query()
        self.shape = (m_a, d, d, m_c)
        self.ws = torch.empty(max(1, q["workspace_bytes"]), dtype=torch.uint8, device=device)
        self.flops = q["flops"]

    def apply(self, precision, L, W1, W2, R, psi, out, stream=None):
        """out (m_a, d, d, m_c) = H_eff psi; dense FP64 device tensors."""
        for t in (L, W1, W2, R, psi, out):
            if not t.is_contiguous() or t.dtype.itemsize != 8:
                raise ValueError("dense operands must be contiguous FP64 tensors")
        if tuple(psi.shape) != self.shape or tuple(out.shape) != self.shape:
            raise ValueError("psi / out shape does not match the plan")
        lib.dense_apply(self.op, precision, L, W1, W2, R, psi, out, self.ws, stream)

    def destroy(self):
        self.op.destroy()
        self.ws = None
