"""The sparse-dense format of Sec. IV-A on the GPU, as an ablation of the
block-sparse list path: every operand of the two-site product embedded in one
dense tensor (the forbidden blocks are zeros), and each stage one dense
library GEMM (torch.matmul on the device).  It computes the same product with
all the work that the block structure avoids; its only use is to measure that
work.

Index names as in the block-sparse path: L (a', w, a), W_i (w, s1', s1, v),
W_{i+1} (v, s2', s2, w''), R (c', w'', c), psi (a, s1, s2, c).
"""


def dense_flops(m_a, m_c, k, d):
    """Flops of the three dense GEMMs (S1, the MPO mixing, S3)."""
    s1 = 2.0 * (m_a * k) * m_a * (d * d * m_c)
    s2 = 2.0 * (m_a * m_c) * (k * d * d) * (d * d * k)
    s3 = 2.0 * (m_a * d * d) * (k * m_c) * m_c
    return s1, s2, s3


def heff_dense(L, W1, W2, R, psi):
    """out = H_eff psi with dense device tensors of one dtype."""
    ma, k, _ = L.shape
    mc = R.shape[0]
    d = psi.shape[1]
    T1 = (L.reshape(ma * k, ma) @ psi.reshape(ma, d * d * mc)).reshape(ma, k, d, d, mc)
    WW = (W1.reshape(k * d * d, k) @ W2.reshape(k, d * d * k)).reshape(k, d, d, d, d, k)   # w s1' s1 s2' s2 w''
    A = T1.permute(0, 4, 1, 2, 3).reshape(ma * mc, k * d * d)                                 # (a' c) (w s1 s2)
    B = WW.permute(0, 2, 4, 1, 3, 5).reshape(k * d * d, d * d * k)                            # (w s1 s2) (s1' s2' w'')
    T2 = (A @ B).reshape(ma, mc, d, d, k).permute(0, 2, 3, 4, 1).reshape(ma * d * d, k * mc)  # (a' s1' s2') (w'' c)
    out = T2 @ R.reshape(mc, k * mc).t().contiguous()
    return out.reshape(ma, d, d, mc)
