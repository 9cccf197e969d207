"""The two-site effective Hamiltonian applied to a two-site tensor.

Sec. II-C gives the single-site projected operator K = A . H^(j) . B through
the left environment A (indices bra, MPO, ket), the MPO site and the right
environment B, applied implicitly (Fig. 1d).  For the two-site tensor
x_{i sigma sigma' i''} = sum T^(j) T^(j+1) the same construction with two MPO
sites in the middle gives

  out(a',s1',s2',c') = sum L(a',w,a) W_i(w,s1',s1,w') W_{i+1}(w',s2',s2,w'')
                           R(c',w'',c) psi(a,s1,s2,c).

Signs (allowed-block rules, charges of a bond = total charge to its left):
  psi, out (a, s1, s2, c): q_a + q_s1 + q_s2 - q_c = 0
  L (a', w, a):            -q_a' + f_w + q_a = 0      (bra, channel, ket)
  R (c', w, c):            -q_c' + f_w + q_c = 0
  W (w, s', s, w'):        f_w + q_s' - q_s - f_w' = 0
"""
import numpy as np

from .blocks import BlockTensor, contract

PSI_SIGNS = (1, 1, 1, -1)
ENV_SIGNS = (-1, 1, 1)
W_SIGNS = (1, 1, -1, -1)
MPS_SIGNS = (1, 1, -1)


def w_tensor(W, w_left, phys, w_right, drop_zero=True):
    """Block form of a dense MPO site; raises if W breaks charge conservation.
    Blocks that are exactly zero are dropped (treated as structurally absent)."""
    bt = BlockTensor.from_dense(np.asarray(W, dtype=np.float64),
                                [w_left, phys, phys, w_right], W_SIGNS, check_zero=True)
    if drop_zero:
        bt.blocks = {k: v for k, v in bt.blocks.items() if np.any(v != 0.0)}
    return bt


def bond_operands(spec):
    """(L, W1, W2, R, psi) block tensors of an isolated-bond problem."""
    wl = spec.w_leg()
    L = BlockTensor.from_fn([spec.a_leg, wl, spec.a_leg], ENV_SIGNS, spec.L_block)
    R = BlockTensor.from_fn([spec.c_leg, wl, spec.c_leg], ENV_SIGNS, spec.R_block)
    W1 = w_tensor(spec.W1, wl, spec.s_leg, wl)
    W2 = w_tensor(spec.W2, wl, spec.s_leg, wl)
    psi = BlockTensor.from_fn([spec.a_leg, spec.s_leg, spec.s_leg, spec.c_leg], PSI_SIGNS,
                              spec.psi_block)
    return L, W1, W2, R, psi


def heff_dense(L, W1, W2, R, psi):
    """O1: embed every block into dense arrays at its sector's index range (the
    sparse-dense format of Sec. IV-A) and contract in the order L.psi, then the
    two MPO sites, then R.  Asserts exact zeros outside allowed blocks."""
    Ld, W1d, W2d, Rd, pd = (t.to_dense() for t in (L, W1, W2, R, psi))
    T1 = np.tensordot(Ld, pd, axes=([2], [0]))                      # a' w s1 s2 c
    WW = np.tensordot(W1d, W2d, axes=([3], [0]))                    # w s1' s1 s2' s2 w''
    T2 = np.tensordot(T1, WW, axes=([1, 2, 3], [0, 2, 4]))          # a' c s1' s2' w''
    out = np.tensordot(T2, Rd, axes=([1, 4], [2, 1]))               # a' s1' s2' c'
    return BlockTensor.from_dense(out, psi.legs, PSI_SIGNS, check_zero=True)


class DenseHeff:
    """O1 with the operand embeddings (and W_i W_{i+1}) formed once, for
    repeated application inside an eigensolver; the same arithmetic as
    ``heff_dense``."""

    def __init__(self, L, W1, W2, R):
        self.Ld, self.Rd = L.to_dense(), R.to_dense()
        self.WW = np.tensordot(W1.to_dense(), W2.to_dense(), axes=([3], [0]))

    def __call__(self, psi):
        T1 = np.tensordot(self.Ld, psi.to_dense(), axes=([2], [0]))
        T2 = np.tensordot(T1, self.WW, axes=([1, 2, 3], [0, 2, 4]))
        out = np.tensordot(T2, self.Rd, axes=([1, 4], [2, 1]))
        return BlockTensor.from_dense(out, psi.legs, PSI_SIGNS, check_zero=True)


def heff_blocks(L, W1, W2, R, psi, return_flops=False):
    """O2: the same contraction done block by block with Alg. 2 at every step
    (one dense tensordot per compatible block pair).  Flops of the two large
    steps (L.psi and T2.R) are the "useful" count used for every rate."""
    T1, f1 = contract(L, psi, [2], [0])                              # a' w s1 s2 c
    WW, _ = contract(W1, W2, [3], [0])                               # w s1' s1 s2' s2 w''
    T2, f2 = contract(T1, WW, [1, 2, 3], [0, 2, 4])                  # a' c s1' s2' w''
    out, f3 = contract(T2, R, [1, 4], [2, 1], out_signs=PSI_SIGNS)   # a' s1' s2' c'
    full = BlockTensor.zeros(psi.legs, PSI_SIGNS)
    for k in full.blocks:
        if k in out.blocks:
            full.blocks[k] = out.blocks[k]
    if return_flops:
        return full, {"s1": f1, "s2_dense_blocks": f2, "s3": f3}
    return full


def useful_flops(L, W1, W2, R, psi):
    """Useful flop count (S1 + S3) of one application, from the block-pair
    structure alone (the same definition as the flop counts of Sec. VI, which
    are measured on the list method)."""
    _, f = heff_blocks(L, W1, W2, R, psi, return_flops=True)
    return f["s1"] + f["s3"]


def heff1_dense(L, W, R, psi):
    """Single-site projected operator of Sec. II-C applied to the one-site
    tensor psi(a, s, c) (bond, physical, bond; MPS signs):
      out(a',s',c') = sum L(a',w,a) W(w,s',s,w') R(c',w',c) psi(a,s,c),
    on the dense embeddings, read back on the allowed blocks."""
    Ld, Wd, Rd, pd = (t.to_dense() for t in (L, W, R, psi))
    t = np.einsum("xwa,asc->xwsc", Ld, pd)            # sum over a
    t = np.einsum("xwsc,wpsv->xpvc", t, Wd)           # sum over w, s
    out = np.einsum("xpvc,yvc->xpy", t, Rd)           # sum over v (w'), c
    return BlockTensor.from_dense(out, psi.legs, MPS_SIGNS, check_zero=True)


def heff_diagonal(L, W1, W2, R, psi_legs):
    """Diagonal of H_eff on the packed canonical vector: the matrix element
    <e|H_eff|e> of every basis tensor e, i.e. the two-site formula with the
    bra indices equal to the ket indices,
      D(a,s1,s2,c) = sum L(a,w,a) W_i(w,s1,s1,w') W_{i+1}(w',s2,s2,w'') R(c,w'',c),
    evaluated on the dense embeddings (padding entries 0)."""
    Ld, W1d, W2d, Rd = (t.to_dense() for t in (L, W1, W2, R))
    ldg = np.einsum("awa->aw", Ld)
    rdg = np.einsum("cwc->cw", Rd)
    w1 = np.einsum("wssv->wsv", W1d)
    w2 = np.einsum("vttz->vtz", W2d)
    D = np.einsum("aw,wsv,vtz,cz->astc", ldg, w1, w2, rdg)
    return BlockTensor.from_dense(D, psi_legs, PSI_SIGNS, check_zero=False).pack()


def heff_dense_matrix(L, W1, W2, R, psi_legs):
    """Explicit matrix of H_eff on the packed canonical vector (tiny cases)."""
    z = BlockTensor.zeros(psi_legs, PSI_SIGNS)
    n = z.pack().size
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        x = BlockTensor.unpack(e, psi_legs, PSI_SIGNS)
        cols.append(heff_dense(L, W1, W2, R, x).pack())
    return np.stack(cols, axis=1)
