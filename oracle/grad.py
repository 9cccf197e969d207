"""Reference gradients of the two-site energy functional.

E(psi, L, W_i, W_{i+1}, R) = psi^T H_eff psi with H_eff the two-site form of
the effective operator of Sec. II-C (real tensors).  E is linear in each of L,
W_i, W_{i+1} and R, so every partial derivative is the same full contraction
with that operand left out; dE/dpsi = (H_eff + H_eff^T) psi.  Written with
einsum on the dense-embedded (sparse-dense, Sec. IV-A) arrays, then read back
on the allowed blocks.  Index letters: x=a', p=s1', q=s2', y=c', w, u=w',
v=w'', a, s=s1, t=s2, c.
"""
import numpy as np

from .blocks import BlockTensor, ein as _ein
from .heff import PSI_SIGNS, ENV_SIGNS, W_SIGNS

_E = "xpqy,xwa,wpsu,uqtv,yvc,astc->"


def energy(L, W1, W2, R, psi):
    P, Ld, W1d, W2d, Rd = psi.to_dense(), L.to_dense(), W1.to_dense(), W2.to_dense(), R.to_dense()
    return float(_ein(_E, P, Ld, W1d, W2d, Rd, P))


def gradients(L, W1, W2, R, psi):
    """dict of BlockTensors: psi, L, W1, W2, R (dE/d each)."""
    P, Ld, W1d, W2d, Rd = psi.to_dense(), L.to_dense(), W1.to_dense(), W2.to_dense(), R.to_dense()
    g_bra = _ein("xwa,wpsu,uqtv,yvc,astc->xpqy", Ld, W1d, W2d, Rd, P)
    g_ket = _ein("xpqy,xwa,wpsu,uqtv,yvc->astc", P, Ld, W1d, W2d, Rd)
    gL = _ein("xpqy,wpsu,uqtv,yvc,astc->xwa", P, W1d, W2d, Rd, P)
    gW1 = _ein("xpqy,xwa,uqtv,yvc,astc->wpsu", P, Ld, W2d, Rd, P)
    gW2 = _ein("xpqy,xwa,wpsu,yvc,astc->uqtv", P, Ld, W1d, Rd, P)
    gR = _ein("xpqy,xwa,wpsu,uqtv,astc->yvc", P, Ld, W1d, W2d, P)
    full = lambda d, legs, signs: BlockTensor.from_dense(d, legs, signs, check_zero=False)
    return {
        "psi": full(g_bra + g_ket, psi.legs, PSI_SIGNS),
        "L": full(gL, L.legs, ENV_SIGNS),
        "W1": full(gW1, W1.legs, W_SIGNS),
        "W2": full(gW2, W2.legs, W_SIGNS),
        "R": full(gR, R.legs, ENV_SIGNS),
    }


# ---------------------------------------------------- environment extension --
# Left:  L'(b',w',b) = sum A(a',s',b') L(a',w,a) W(w,s',s,w') A(a,s,b)
# Right: R'(b',w,b)  = sum B(b',s',c') W(w,s',s,w') R(c',w',c) B(b,s,c)
# Both are linear in the environment and in W; the cotangents for an output
# cotangent D are the same contractions with that operand left out.
# Letters: x=a' (c'), p=s', y=b', w, v=w', a (c), s, b.

def env_gradients(env, site, W, d_out, side):
    """dict(env=..., W=...) for the left (side 0) or right (side 1) extension;
    the W cotangent covers every allowed W block."""
    E, S, Wd, D = env.to_dense(), site.to_dense(), W.to_dense(), d_out.to_dense()
    if side == 0:
        gE = _ein("xpy,wpsv,asb,yvb->xwa", S, Wd, S, D)
        gW = _ein("xpy,xwa,asb,yvb->wpsv", S, E, S, D)
    else:
        gE = _ein("ypx,wpsv,bsa,ywb->xva", S, Wd, S, D)
        gW = _ein("ypx,xva,bsa,ywb->wpsv", S, E, S, D)
    full = lambda d, legs, signs: BlockTensor.from_dense(d, legs, signs, check_zero=False)
    return {"env": full(gE, env.legs, ENV_SIGNS), "W": full(gW, W.legs, W_SIGNS)}


# ------------------------------------------------------- expectation values --
def expectation(mps, Ws, w_start, w_done):
    """<Psi|O|Psi> / <Psi|Psi> for an MPS (list of BlockTensors (a, s, b)) and
    an MPO given by dense site tensors Ws[j] (w, s', s, w') with boundary
    channels w_start and w_done: the left environment is extended through
    every site (dense einsums), then closed on the done channel."""
    env = np.zeros((1, Ws[0].shape[0], 1))
    env[0, w_start, 0] = 1.0
    nrm = np.ones((1, 1))
    for A, W in zip(mps, Ws):
        Ad = A.to_dense()
        env = _ein("xpy,xwa,wpsv,asb->yvb", Ad, env, W, Ad)
        nrm = _ein("xpy,xa,apb->yb", Ad, nrm, Ad)
    return float(env[0, w_done, 0] / nrm[0, 0])


# ------------------------------------------------- MPO-parameter derivatives --
def mpo_gradients(mps, Ws, wl, start, done, target, bond):
    """E = psi^T H_eff psi at bond (bond, bond+1) and dE/dW_s for every site s.

    The MPS must be in mixed-canonical form around the bond (sites left of it
    left-canonical, right of it right-canonical) and normalised, so E equals
    <Psi|H|Psi>.  Ws: W BlockTensors per site.  Reverse mode: the two-site
    gradients give dE/dW at the bond and dE/dL, dE/dR; the environment
    cotangents are carried outwards through the extensions (each linear in
    its environment and in W), collecting dE/dW_s on the way."""
    from .env import left_boundary, right_boundary, left_update_dense, right_update_dense, merge
    N = len(mps)
    r = len(wl[0][0])
    L = [left_boundary(wl, start, r)]
    for j in range(bond):
        L.append(left_update_dense(L[j], mps[j], Ws[j]))
    R = {N: right_boundary(wl, done, target)}
    for j in range(N - 1, bond + 1, -1):
        R[j] = right_update_dense(R[j + 1], mps[j], Ws[j])
    theta = merge(mps[bond], mps[bond + 1])
    g = gradients(L[bond], Ws[bond], Ws[bond + 1], R[bond + 2], theta)
    E = energy(L[bond], Ws[bond], Ws[bond + 1], R[bond + 2], theta)
    dW = [None] * N
    dW[bond], dW[bond + 1] = g["W1"], g["W2"]
    d = g["L"]
    for j in range(bond - 1, -1, -1):
        eg = env_gradients(L[j], mps[j], Ws[j], d, 0)
        dW[j], d = eg["W"], eg["env"]
    d = g["R"]
    for j in range(bond + 2, N):
        eg = env_gradients(R[j + 1], mps[j], Ws[j], d, 1)
        dW[j], d = eg["W"], eg["env"]
    return E, dW


def parameter_derivative(dW, dW_dp):
    """Chain rule over the sites: sum_s <dE/dW_s, dW_s/dp>."""
    return float(sum(a.dot(b) for a, b in zip(dW, dW_dp)))
