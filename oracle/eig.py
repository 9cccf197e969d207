"""Eigensolvers for the lowest eigenpair of the implicit effective Hamiltonian.

``davidson`` follows Alg. 1 (Sec. II-C): no preconditioning, Gram row from the
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

Two extensions for long solves (the paper keeps the subspace at 2 vectors and
leaves preconditioning out for its cost on CPUs; both are silent on details):
  * bounded basis with thick restart: when the basis holds ``basis`` vectors
    and the solve goes on, it is replaced by the ``keep`` lowest Ritz vectors
    plus the previous step's Ritz vector orthogonalised against them (twice;
    when less than 1e-8 of it remains, the newest basis vector orthogonalised
    the same way is taken instead);
    the products of the new basis are the same combinations of the stored
    products, so a restart costs no product and keeps the current Ritz pair;
  * diagonal preconditioning (Davidson's correction): the new direction is
    t = q / max(D - lambda, delta), D the diagonal of H_eff and
    delta = 1e-3 max(|lambda|, 1): a positive preconditioner whose
    amplification is bounded by 1 / delta (with the plain D - lambda, a
    Ritz value above some diagonal entries meets near-zero denominators and
    the iteration becomes chaotic: rounding-level differences change the
    trajectory); t is then orthogonalised like q.
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
             restart_rtol=1e-10, max_attempts=3, record=None, basis=None, keep=0,
             precond=None):
    """Alg. 1.  Returns (lambda, x normalised, stats dict).

    matvec        function: flat vector -> flat vector (the implicit H_eff)
    x0            start vector (any norm)
    max_iter      number of products with A (the basis size when there is no
                  restart)
    restart_mask  boolean array of allowed elements for random restarts
                  (padding of the block layout stays zero); None = all
    record        optional list receiving the Ritz value of every iteration
    basis, keep   bounded basis: at most ``basis`` vectors, thick restart to
                  keep + 1 vectors (keep >= 1, keep + 2 <= basis)
    precond       the diagonal D of the operator (flat, same layout) for the
                  preconditioned correction, or None (Alg. 1 as printed)
    """
    n = x0.size
    mask = np.ones(n, dtype=bool) if restart_mask is None else restart_mask
    dim = int(mask.sum())       # a basis of this size spans the whole space
    B = max_iter if basis is None else int(basis)
    if basis is not None and not (1 <= keep and keep + 2 <= B):
        raise ValueError("thick restart needs 1 <= keep <= basis - 2")
    V = [x0 / np.linalg.norm(x0)]
    VA = [matvec(V[0])]
    products, restarts, thick = 1, 0, 0
    sprev = None                # previous Ritz vector, coordinates of the current basis
    M = np.zeros((0, 0))
    while True:
        j = len(V)
        # projected matrix m_rc = (v^A_c)^T v_r: the new row (all rows after a restart)
        Mn = np.zeros((j, j))
        k0 = M.shape[0]
        Mn[:k0, :k0] = M
        for r in range(k0, j):
            for c in range(r + 1):
                Mn[r, c] = Mn[c, r] = float(VA[c] @ V[r])
        M = Mn
        evals, evecs = np.linalg.eigh(M)
        lam = float(evals[0])
        s = evecs[:, 0]
        x = sum(s[c] * V[c] for c in range(j))
        q = sum(s[c] * VA[c] for c in range(j)) - lam * x
        qn = float(np.linalg.norm(q))
        if record is not None:
            record.append(lam)
        if qn <= tol or products >= max_iter or j >= dim:
            break
        if j == B:
            # thick restart: keep lowest Ritz vectors + the previous Ritz vector
            S = evecs[:, :keep]
            p = np.zeros(j) if sprev is None else np.concatenate([sprev, np.zeros(j - sprev.size)])
            for _ in range(2):
                p = p - S @ (S.T @ p)
            pn = float(np.linalg.norm(p))
            if not pn > 1e-8:
                p = np.zeros(j)
                p[j - 1] = 1.0
                for _ in range(2):
                    p = p - S @ (S.T @ p)
                pn = float(np.linalg.norm(p))
            extra = p / pn
            S = np.column_stack([S, extra])
            V = [sum(S[c, t] * V[c] for c in range(j)) for t in range(S.shape[1])]
            VA = [sum(S[c, t] * VA[c] for c in range(j)) for t in range(S.shape[1])]
            M = np.zeros((0, 0))
            thick += 1
            sprev = np.zeros(len(V))
            sprev[0] = 1.0          # the current Ritz vector is the first kept one
        else:
            sprev = s.copy()
        if precond is None:
            t = q
        else:
            den = np.maximum(precond - lam, 1e-3 * max(abs(lam), 1.0))
            t = q / den
        before = float(np.linalg.norm(t))
        t = _mgs2(t, V)
        after = float(np.linalg.norm(t))
        attempt = 0
        while after < restart_rtol * before or after == 0.0:
            if attempt >= max_attempts:
                raise RuntimeError("Davidson: reorthogonalisation failed after restarts")
            key = rng.restart_key(seed, products - 1, attempt)
            r = np.zeros(n)
            idx = np.nonzero(mask)[0]
            r[idx] = rng.gaussian_at(key, idx)
            before = float(np.linalg.norm(r))
            t = _mgs2(r, V)
            after = float(np.linalg.norm(t))
            attempt += 1
            restarts += 1
        V.append(t / after)
        VA.append(matvec(V[-1]))
        products += 1
    xn = x / np.linalg.norm(x)
    return lam, xn, {"iters": products, "residual": qn, "restarts": restarts,
                     "thick_restarts": thick, "converged": bool(qn <= tol)}


def _mgs2(q, V):
    for _ in range(2):
        for v in V:
            q = q - float(v @ q) * v
    return q
