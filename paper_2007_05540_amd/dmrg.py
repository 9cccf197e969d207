"""Two-site DMRG sweeps on one GPU (Sec. II-C, Fig. 1).

Bond j sits to the left of site j; MPS site j has legs (bond j, s, bond j+1).
Starting from a right-canonical MPS, a sweep visits the pairs (j, j+1) left
to right and back: merge the two sites, find the lowest eigenpair of the
two-site effective Hamiltonian with the Davidson routine started from the
merged tensor, split it with the truncated SVD (singular values absorbed in
the sweep direction) and extend the environment.  This module only orders the
calls and keeps leg tables; every contraction, eigensolve and SVD runs in the
library through its C ABI.
"""
from collections import OrderedDict

import numpy as np

from . import lib, problems


class Tensor:
    """Device tensor in canonical block layout plus its legs."""

    def __init__(self, legs, data):
        self.legs, self.data = legs, data


def _lk(leg):
    """Hashable form of a leg [(charge, dim), ...]."""
    return tuple((tuple(q), int(d)) for q, d in leg)


class GpuDMRG:
    def __init__(self, mpo, mps_host, target, device="cuda", precision=lib.F64, refine_max_iter=8,
                 tol_f32=1e-6):
        """mpo: a uniform-channel MPO (W[j] dense (k, d, d, k), channels
        sector-major) or a BondMPO (a leg per bond, e.g. after compression);
        mps_host: list of (legs, packed FP64 array); target: total charge of
        the state."""
        import torch
        from .mpo import BondMPO
        self.torch = torch
        self.device = device
        self.mpo = mpo
        bm = mpo if isinstance(mpo, BondMPO) else BondMPO.uniform(mpo)
        self.N = len(bm.W)
        self.legs = bm.legs            # channel leg of every bond (N + 1)
        s = bm.phys
        self.s = s
        self.W_host = [problems.pack_dense(W, [self.legs[j], s, s, self.legs[j + 1]], lib.W_SIGNS)
                       for j, W in enumerate(bm.W)]
        self.W = [torch.from_numpy(w).to(device) for w in self.W_host]
        self.T = [Tensor(l, torch.from_numpy(np.ascontiguousarray(a)).to(device)) for l, a in mps_host]
        self.target = tuple(target)
        self.precision = precision
        self.refine_max_iter = refine_max_iter
        self.tol_f32 = tol_f32
        r = len(s[0][0])
        zero = tuple([0] * r)
        self.L = [None] * (self.N + 1)
        self.R = [None] * (self.N + 1)
        self.L[0] = self._boundary(zero, bm.start, self.legs[0])
        self.R[self.N] = self._boundary(self.target, bm.done, self.legs[self.N])
        self.log = []
        # plans and ops keyed by what they are built from (site, side and the
        # legs of the operands): sweeps at a saturated bond dimension meet the
        # same sector structure again and reuse them
        self._cache = OrderedDict()
        self._cache_max = 6 * self.N + 8
        self.cache_hits = self.cache_misses = 0

    def _cached(self, key, build):
        obj = self._cache.get(key)
        if obj is not None:
            self._cache.move_to_end(key)
            self.cache_hits += 1
            return obj
        self.cache_misses += 1
        obj = build()
        self._cache[key] = obj
        if len(self._cache) > self._cache_max:
            _, old = self._cache.popitem(last=False)
            old.destroy()
        return obj

    # -- helpers -------------------------------------------------------------
    def _boundary(self, q, channel, wleg):
        leg = [(tuple(q), 1)]
        k = sum(n for _, n in wleg)
        dense = np.zeros((1, k, 1))
        dense[0, channel, 0] = 1.0
        data = problems.pack_dense(dense, [leg, wleg, leg], lib.ENV_SIGNS)
        return Tensor([leg, wleg, leg], self.torch.from_numpy(data).to(self.device))

    def _merge(self, A, B):
        a, s1, b = A.legs
        _, s2, c = B.legs
        op = self._cached(("merge", _lk(a), _lk(s1), _lk(b), _lk(s2), _lk(c)),
                          lambda: lib.merge_plan(a, s1, b, s2, c))
        theta = self.torch.zeros(max(1, op.query()["out_elems"]), dtype=self.torch.float64, device=self.device)
        lib.merge(op, A.data, B.data, theta)
        return Tensor([a, s1, s2, c], theta)

    def _split(self, theta, direction, cutoff, cutoff_mode, max_m):
        A, B, leg, sv, disc = lib.truncate(theta.legs, theta.data, direction, cutoff, cutoff_mode, max_m)
        a, s1, s2, c = theta.legs
        return Tensor([a, s1, leg], A), Tensor([leg, s2, c], B), disc

    def _env(self, env, site, j, side):
        """side 0: left extension through site j (A); side 1: right (B)."""
        if side == 0:
            x, s, y = site.legs
        else:
            y, s, x = site.legs
        op = self._cached(("env", j, side, _lk(x), _lk(s), _lk(y)),
                          lambda: lib.env_plan(x, s, y, self.legs[j], self.legs[j + 1], self.W_host[j], side))
        info = op.query()
        out = self.torch.zeros(max(1, info["out_elems"]), dtype=self.torch.float64, device=self.device)
        ws = self.torch.empty(max(1, info["workspace_bytes"]), dtype=self.torch.uint8, device=self.device)
        lib.env_update(op, env.data, site.data, self.W[j], out, ws)
        return Tensor([y, self.legs[j + 1] if side == 0 else self.legs[j], y], out)

    # -- algorithm -----------------------------------------------------------
    def right_canonicalize(self, cutoff=1e-14, progress=False):
        """Splits from the right with S absorbed to the left; singular values
        below 1e-14 of the norm (numerically zero, with non-unique vectors)
        are dropped."""
        for j in range(self.N - 1, 0, -1):
            if progress:
                print(f"  canonicalize {j}", flush=True)
            theta = self._merge(self.T[j - 1], self.T[j])
            self.T[j - 1], self.T[j], _ = self._split(theta, 1, cutoff, 0, 1 << 62)
        for j in range(self.N - 1, 1, -1):
            self.R[j] = self._env(self.R[j + 1], self.T[j], j, 1)

    def solve_bond(self, j, theta, max_iter, tol, seed):
        a, s1, s2, c = theta.legs
        prob = {"a": a, "s1": s1, "s2": s2, "c": c, "wl": self.legs[j], "wm": self.legs[j + 1],
                "wr": self.legs[j + 2], "w1": self.W_host[j], "w2": self.W_host[j + 1]}
        plan = self._cached(("heff", j, _lk(a), _lk(s1), _lk(s2), _lk(c)), lambda: lib.Plan([prob]))
        if self.precision == lib.F64:
            opts = lib.eig_opts(max_iter=max_iter, tol=tol, seed=seed)
        else:
            opts = lib.eig_opts(max_iter=max_iter, precision=lib.F32_REFINE, refine_max_iter=self.refine_max_iter,
                                tol=tol, tol_f32=self.tol_f32, seed=seed)
        ws = self.torch.empty(lib.eig_workspace(plan, opts), dtype=self.torch.uint8, device=self.device)
        e, st = lib.eigensolve(plan, self.L[j].data, self.W[j], self.W[j + 1], self.R[j + 2].data, theta.data,
                               opts, ws)
        info = plan.info()
        return e[0], st[0], info["flops_s1"] + info["flops_s3"]

    def energy_and_mpo_gradients(self, bond=0):
        """E = psi^T H_eff psi at (bond, bond + 1) and dE/dW_s for every site
        s, by reverse mode through the autograd graph EnvUpdate x sites ->
        HeffEnergy.  The MPS must be mixed-canonical around the bond and
        normalised (as after run(), for bond 0), so that E = <Psi|H|Psi>.
        Returns (E, [dE/dW_s device tensors in canonical W layout])."""
        from . import autograd
        torch = self.torch
        N, lg = self.N, self.legs
        Wg = [w.detach().clone().requires_grad_(True) for w in self.W]
        keep = []
        L = self.L[0].data
        for j in range(bond):
            x, s, y = self.T[j].legs
            op = lib.env_plan(x, s, y, lg[j], lg[j + 1], self.W_host[j], 0)
            adj = lib.env_plan(y, s, x, lg[j], lg[j + 1], self.W_host[j], 1)
            keep += [op, adj]
            L = autograd.EnvUpdate.apply(op, adj, L, self.T[j].data, Wg[j])
        R = self.R[N].data
        for j in range(N - 1, bond + 1, -1):
            y, s, x = self.T[j].legs
            op = lib.env_plan(x, s, y, lg[j], lg[j + 1], self.W_host[j], 1)
            adj = lib.env_plan(y, s, x, lg[j], lg[j + 1], self.W_host[j], 0)
            keep += [op, adj]
            R = autograd.EnvUpdate.apply(op, adj, R, self.T[j].data, Wg[j])
        theta = self._merge(self.T[bond], self.T[bond + 1])
        a, s1, s2, c = theta.legs
        plan = lib.Plan([{"a": a, "s1": s1, "s2": s2, "c": c, "wl": lg[bond], "wm": lg[bond + 1],
                          "wr": lg[bond + 2], "w1": self.W_host[bond], "w2": self.W_host[bond + 1]}])
        E = autograd.HeffEnergy.apply(plan, L, Wg[bond], Wg[bond + 1], R, theta.data)
        E.sum().backward()
        torch.cuda.synchronize()
        grads = [w.grad if w.grad is not None else torch.zeros_like(w) for w in Wg]
        plan.destroy()
        for o in keep:
            o.destroy()
        return float(E[0].item()), grads

    def parameter_derivative(self, grads, dW_dp):
        """Chain rule over the sites, sum_s <dE/dW_s, dW_s/dp>, for an MPO
        parameter p with dense per-site derivatives dW_dp[s] (w, s', s, w') from
        the MPO builder: the derivatives are packed in the canonical W layout
        and the inner products and their sum run in the library."""
        torch = self.torch
        dps = [torch.from_numpy(problems.pack_dense(d, [self.legs[j], self.s, self.s, self.legs[j + 1]],
                                                    lib.W_SIGNS)).to(self.device)
               for j, d in enumerate(dW_dp)]
        terms = torch.empty(len(grads) + 1, dtype=torch.float64, device=self.device)
        return lib.param_derivative([g.detach().contiguous() for g in grads], dps, terms)

    def run(self, n_sweeps, m_max, cutoff=1e-10, cutoff_mode=0, max_iter=40, tol=1e-12, progress=False,
            on_sweep=None):
        """Two-site sweeps; m_max is an int or a per-sweep list; on_sweep(sweep,
        energy, seconds) is called after every sweep.  Returns (energies per
        visited bond, last energy of every sweep)."""
        import time
        self.right_canonicalize(progress=progress)
        mlist = m_max if isinstance(m_max, (list, tuple)) else [m_max] * n_sweeps
        energies, sweep_e = [], []
        self.sweep_seconds = []
        step = 0
        N = self.N
        for sw in range(n_sweeps):
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            order = [(j, 0) for j in range(N - 1)] + [(j, 1) for j in range(N - 2, -1, -1)]
            for j, d in order:
                theta = self._merge(self.T[j], self.T[j + 1])
                if progress:
                    print(f"  sweep {sw} bond {j} dir {d}: solve", flush=True)
                E, st, flops = self.solve_bond(j, theta, max_iter, tol, step)
                if not np.isfinite(E):
                    raise FloatingPointError(f"non-finite energy at sweep {sw} bond {j}")
                A, B, disc = self._split(theta, d, cutoff, cutoff_mode, mlist[sw])
                self.T[j], self.T[j + 1] = A, B
                if d == 0:
                    self.L[j + 1] = self._env(self.L[j], A, j, 0)
                else:
                    self.R[j + 1] = self._env(self.R[j + 2], B, j + 1, 1)
                energies.append(E)
                self.log.append({"sweep": sw, "bond": j, "dir": d, "E": E, "iters": st["iters"],
                                 "iters_f32": st["iters_f32"], "res": st["residual"], "disc": disc,
                                 "m": sum(dd for _, dd in A.legs[2]), "flops_per_product": flops})
                step += 1
            sweep_e.append(energies[-1])
            self.torch.cuda.synchronize()
            self.sweep_seconds.append(time.perf_counter() - t0)
            if on_sweep is not None:
                on_sweep(sw, sweep_e[-1], self.sweep_seconds[-1])
        return energies, sweep_e

    # -- single-site sweeps -----------------------------------------------
    def _identity_site(self, j):
        """W(w, 1, 1, w') = delta on the channel leg of bond j with a one-state
        zero-charge physical leg: the second site of the two-site plan that
        turns it into the single-site operator L W_j R."""
        if not hasattr(self, "_ids"):
            self._ids = {}
        if j not in self._ids:
            leg = self.legs[j]
            k = sum(n for _, n in leg)
            one = self._one_leg()
            dense = np.eye(k).reshape(k, 1, 1, k)
            host = problems.pack_dense(dense, [leg, one, one, leg], lib.W_SIGNS)
            self._ids[j] = (host, self.torch.from_numpy(host).to(self.device))
        return self._ids[j]

    def _one_leg(self):
        return [(tuple([0] * len(self.s[0][0])), 1)]

    def solve_site(self, j, max_iter, tol, seed):
        """Lowest eigenpair of the single-site operator L_j W_j R_{j+1} (Sec.
        II-C) on site tensor j, through a two-site plan whose second site is
        the identity on a one-state leg (the site tensor (a, s, c) is the
        two-site tensor (a, s, 1, c): same blocks, same layout).  The solution
        overwrites the site tensor."""
        a, s, c = self.T[j].legs
        one = self._one_leg()
        wid_host, wid = self._identity_site(j + 1)
        prob = {"a": a, "s1": s, "s2": one, "c": c, "wl": self.legs[j], "wm": self.legs[j + 1],
                "wr": self.legs[j + 1], "w1": self.W_host[j], "w2": wid_host}
        plan = self._cached(("site", j, _lk(a), _lk(s), _lk(c)), lambda: lib.Plan([prob]))
        if self.precision == lib.F64:
            opts = lib.eig_opts(max_iter=max_iter, tol=tol, seed=seed)
        else:
            opts = lib.eig_opts(max_iter=max_iter, precision=lib.F32_REFINE, refine_max_iter=self.refine_max_iter,
                                tol=tol, tol_f32=self.tol_f32, seed=seed)
        ws = self.torch.empty(lib.eig_workspace(plan, opts), dtype=self.torch.uint8, device=self.device)
        e, st = lib.eigensolve(plan, self.L[j].data, self.W[j], wid, self.R[j + 1].data, self.T[j].data, opts, ws)
        return e[0], st[0]

    def run_single_site(self, n_sweeps, max_iter=40, tol=1e-12, on_sweep=None):
        """Single-site sweeps from the current MPS (the bond dimensions stay
        fixed: start from a two-site result or an MPS of the wanted size).  A
        sweep solves site j = 0 .. N-2 moving right (the solution split by the
        library's SVD into a left-orthonormal site and S V^T merged into site
        j+1, dropping only singular values below 1e-14 of the norm) and
        j = N-1 .. 1 moving left (U S merged into site j-1).  Returns (energy
        of every solve, last energy of every sweep)."""
        import time
        N = self.N
        one = self._one_leg()
        self.right_canonicalize()
        self.R[1] = self._env(self.R[2], self.T[1], 1, 1)
        energies, sweep_e = [], []
        self.sweep_seconds = []
        step = 0
        for sw in range(n_sweeps):
            self.torch.cuda.synchronize()
            t0 = time.perf_counter()
            order = [(j, 0) for j in range(N - 1)] + [(j, 1) for j in range(N - 1, 0, -1)]
            for j, d in order:
                E, st = self.solve_site(j, max_iter, tol, step)
                a, s, c = self.T[j].legs
                if d == 0:
                    theta = Tensor([a, s, one, c], self.T[j].data)
                    A, SV, _ = self._split(theta, 0, 1e-14, 0, 1 << 62)
                    self.T[j] = A
                    nxt = self._merge(SV, self.T[j + 1])      # (b, 1, s', d)
                    self.T[j + 1] = Tensor([nxt.legs[0], nxt.legs[2], nxt.legs[3]], nxt.data)
                    self.L[j + 1] = self._env(self.L[j], self.T[j], j, 0)
                else:
                    theta = Tensor([a, one, s, c], self.T[j].data)
                    US, B, _ = self._split(theta, 1, 1e-14, 0, 1 << 62)
                    self.T[j] = B
                    prv = self._merge(self.T[j - 1], US)      # (x, s', 1, b)
                    self.T[j - 1] = Tensor([prv.legs[0], prv.legs[1], prv.legs[3]], prv.data)
                    self.R[j] = self._env(self.R[j + 1], self.T[j], j, 1)
                energies.append(E)
                self.log.append({"sweep": sw, "site": j, "dir": d, "E": E, "iters": st["iters"],
                                 "iters_f32": st["iters_f32"], "res": st["residual"]})
                step += 1
            sweep_e.append(energies[-1])
            self.torch.cuda.synchronize()
            self.sweep_seconds.append(time.perf_counter() - t0)
            if on_sweep is not None:
                on_sweep(sw, sweep_e[-1], self.sweep_seconds[-1])
        return energies, sweep_e

    def host_mps(self):
        """The current MPS as (legs, packed FP64 array) pairs (a warm start)."""
        return [(t.legs, t.data.detach().cpu().numpy()) for t in self.T]
