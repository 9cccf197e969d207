"""Eigensolvers for the lowest eigenpair of the implicit effective Hamiltonian.

``davidson`` follows Alg. 1 (Sec. III): no preconditioning, Gram row from the
stored products, smallest Ritz pair of the projected matrix, residual, modified
Gram-Schmidt, randomisation when reorthogonalisation fails.  Readings where the
listing is silent or slightly off:
  * the start vector and every new basis vector are normalised;
  * at iteration i the projected matrix is (i+1) x (i+1) (the block the
    listing diagonalises is one row and column short of that: it must
    contain the newest vector);
  * m_ij = m_ji = (v^A_j)^T v_i for j <= i;
  * convergence when ||q||_2 <= tol (after q = sum s_j v^A_j - lambda x);
  * modified Gram-Schmidt is applied twice (robustness; ~1e-15 effect);
  * if ||q|| after orthogonalisation < restart_rtol * ||q|| before it (or the
    iteration limit of the basis would otherwise stall), q is replaced by a
    seeded Gaussian vector restricted to the allowed elements and
    orthogonalised again, at most 3 attempts;
  * ``max_iter`` is the largest basis size, i.e. the number of products with A;
    once the basis spans the whole allowed space (its size equals the number
    of allowed elements) the Ritz pair is exact and the iteration stops.
``lanczos`` (full reorthogonalisation) is the independent Krylov reference:
without preconditioning the Davidson basis spans the same Krylov space, so the
Ritz values agree iteration by iteration.
"""
import numpy as np

from . import rng


def lanczos(matvec, x0, n_iter):
    """Ritz values (lowest) after 1..n_iter Lanczos steps, full reorth."""
    q = x0 / np.linalg.norm(x0)
    Q = [q]
    alphas, betas, ritz = [], [], []
    for i in range(n_iter):
        w = matvec(Q[-1])
        a = float(Q[-1] @ w)
        alphas.append(a)
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        ritz.append(float(np.linalg.eigvalsh(T)[0]))
        w = w - a * Q[-1] - (betas[-1] * Q[-2] if betas else 0.0)
        for _ in range(2):
            for v in Q:
                w = w - (v @ w) * v
        b = float(np.linalg.norm(w))
        if b < 1e-14 or i == n_iter - 1:
            break
        betas.append(b)
        Q.append(w / b)
    return ritz


def davidson(matvec, x0, max_iter, tol=0.0, restart_mask=None, seed=0,
             restart_rtol=1e-10, max_attempts=3, record=None):
    """Alg. 1.  Returns (lambda, x normalised, stats dict).

    matvec        function: flat vector -> flat vector (the implicit H_eff)
    x0            start vector (any norm)
    restart_mask  boolean array of allowed elements for random restarts
                  (padding of the block layout stays zero); None = all
    record        optional list receiving the Ritz value of every iteration
    """
    n = x0.size
    mask = np.ones(n, dtype=bool) if restart_mask is None else restart_mask
    dim = int(mask.sum())       # a basis of this size spans the whole space
    V = [x0 / np.linalg.norm(x0)]
    VA = [matvec(V[0])]
    M = np.zeros((max_iter, max_iter))
    restarts = 0
    lam, x, qn = 0.0, V[0], np.inf
    for i in range(max_iter):
        for j in range(i + 1):
            M[i, j] = M[j, i] = float(VA[j] @ V[i])
        evals, evecs = np.linalg.eigh(M[:i + 1, :i + 1])
        lam = float(evals[0])
        s = evecs[:, 0]
        x = sum(s[j] * V[j] for j in range(i + 1))
        q = sum(s[j] * VA[j] for j in range(i + 1)) - lam * x
        qn = float(np.linalg.norm(q))
        if record is not None:
            record.append(lam)
        if qn <= tol or i == max_iter - 1 or i + 1 >= dim:
            break
        before = qn
        q = _mgs2(q, V)
        after = float(np.linalg.norm(q))
        attempt = 0
        while after < restart_rtol * before or after == 0.0:
            if attempt >= max_attempts:
                raise RuntimeError("Davidson: reorthogonalisation failed after restarts")
            key = rng.restart_key(seed, i, attempt)
            r = np.zeros(n)
            idx = np.nonzero(mask)[0]
            r[idx] = rng.gaussian_at(key, idx)
            before = float(np.linalg.norm(r))
            q = _mgs2(r, V)
            after = float(np.linalg.norm(q))
            attempt += 1
            restarts += 1
        V.append(q / after)
        VA.append(matvec(V[-1]))
    xn = x / np.linalg.norm(x)
    return lam, xn, {"iters": i + 1, "residual": qn, "restarts": restarts,
                     "converged": bool(qn <= tol)}


def _mgs2(q, V):
    for _ in range(2):
        for v in V:
            q = q - float(v @ q) * v
    return q
