"""Matrix product operators built as finite-state machines (FSM).

An MPO site tensor is W[w, s', s, w'] (Sec. II-B: H^(j) with bra index before ket
index): w is the channel on the left bond, w' on the right bond, s' the output
(bra) and s the input (ket) physical index.  Each channel carries a *flux*: the
charge change that the operators already placed to its left have applied.  The
channel leg is ordered sector-major: channels sorted by flux (ascending,
lexicographic for tuples), ties by creation order, so every flux sector is a
contiguous range.  With uniform channels on every bond, the left boundary picks
the ``start`` channel and the right boundary the ``done`` channel.

Physical bases (index = ascending charge order):
  spin-1/2, charge (2Sz,):   0 = down (-1), 1 = up (+1)
  electron, charge (N, 2Sz): 0 = empty (0,0), 1 = down (1,-1), 2 = up (1,+1),
                             3 = up+down (2,0) = c_up^+ c_dn^+ |0>
Fermion modes are ordered (site 0 up, site 0 down, site 1 up, ...); the
Jordan-Wigner string between two sites is F = (-1)^(n_up + n_dn) per site.
"""
import numpy as np

SPIN_PHYS = [((-1,), 1), ((1,), 1)]
HUB_PHYS = [((0, 0), 1), ((1, -1), 1), ((1, 1), 1), ((2, 0), 1)]


def spin_ops():
    sz = np.diag([-0.5, 0.5])
    sp = np.zeros((2, 2))
    sp[1, 0] = 1.0          # |up><down|
    sm = sp.T.copy()
    return {"I": np.eye(2), "Sz": sz, "S+": sp, "S-": sm}


def hub_ops():
    """Local electron operators in the basis above (matrices [bra, ket])."""
    b_up = np.zeros((4, 4)); b_up[0, 2] = 1.0; b_up[1, 3] = 1.0
    b_dn = np.zeros((4, 4)); b_dn[0, 1] = 1.0; b_dn[2, 3] = 1.0
    z_up = np.diag([1.0, 1.0, -1.0, -1.0])
    F = np.diag([1.0, -1.0, -1.0, 1.0])
    c_up = b_up                      # no mode precedes 'up' on its own site
    c_dn = z_up @ b_dn               # 'up' precedes 'down' on the same site
    n_up = np.diag([0.0, 0.0, 1.0, 1.0])
    n_dn = np.diag([0.0, 1.0, 0.0, 1.0])
    return {"I": np.eye(4), "F": F, "cu": c_up, "cd": c_dn,
            "cu+": c_up.T.copy(), "cd+": c_dn.T.copy(), "nu": n_up, "nd": n_dn}


class MPO:
    """Uniform-channel MPO: ``W[j]`` has shape (k, d, d, k) for every site j.

    Attributes
    ----------
    W        list of site tensors (channels in sector-major order)
    flux     list of k flux tuples
    names    list of k channel names
    phys     physical leg [(charge, 1), ...]
    start, done   channel indices selected by the left / right boundary
    conj     channel index of the Hermitian-conjugate channel (for synthetic
             environments): S+ strand <-> S- strand, flux-0 channels map to
             themselves
    """

    def __init__(self, W, flux, names, phys, start, done, conj):
        self.W, self.flux, self.names, self.phys = W, flux, names, phys
        self.start, self.done, self.conj = start, done, conj

    @property
    def k(self):
        return len(self.flux)

    @property
    def d(self):
        return len(self.phys)

    def w_leg(self):
        """Channel leg as [(flux, n_channels)] in ascending flux order."""
        out = []
        for f in self.flux:
            if out and out[-1][0] == f:
                out[-1] = (f, out[-1][1] + 1)
            else:
                out.append((f, 1))
        return out


def _assemble(channels, site_transitions, d, phys, conj_names):
    """channels: list of (name, flux) in creation order.
    site_transitions: per site, list of (from_name, to_name, op[d, d]).
    """
    k = len(channels)
    order = sorted(range(k), key=lambda i: (channels[i][1], i))
    pos = {channels[old][0]: new for new, old in enumerate(order)}
    names = [channels[old][0] for old in order]
    flux = [tuple(channels[old][1]) for old in order]
    Ws = []
    for trans in site_transitions:
        W = np.zeros((k, d, d, k))
        for a, b, op in trans:
            W[pos[a], :, :, pos[b]] += op
        Ws.append(W)
    conj = [pos[conj_names.get(n, n)] for n in names]
    return MPO(Ws, flux, names, phys, pos["start"], pos["done"], conj)


def _spin_flux(op):
    return {"S+": (2,), "S-": (-2,), "Sz": (0,)}[op]


_SPIN_COMP = {"S+": ("S-", 0.5), "S-": ("S+", 0.5), "Sz": ("Sz", 1.0)}


def heisenberg_mpo(n_sites, bonds):
    """H = sum_{(i,j)} J_ij S_i . S_j (Sec. V, J1-J2 model) as a distance FSM.

    Channel (op, r) means: ``op`` was placed r sites to the left and waits for
    its partner.  k = 2 + 3 R with R the largest |i - j| in ``bonds``.
    """
    ops = spin_ops()
    R = max((j - i for (i, j) in bonds), default=1)
    chans = [("start", (0,))]
    for op in ("S+", "S-", "Sz"):
        for r in range(1, R + 1):
            chans.append((f"{op}@{r}", _spin_flux(op)))
    chans.append(("done", (0,)))
    conj = {}
    for r in range(1, R + 1):
        conj[f"S+@{r}"] = f"S-@{r}"
        conj[f"S-@{r}"] = f"S+@{r}"
    sites = []
    for j in range(n_sites):
        t = [("start", "start", ops["I"]), ("done", "done", ops["I"])]
        for op in ("S+", "S-", "Sz"):
            t.append(("start", f"{op}@1", ops[op]))
            for r in range(1, R):
                t.append((f"{op}@{r}", f"{op}@{r + 1}", ops["I"]))
            comp, fac = _SPIN_COMP[op]
            for r in range(1, R + 1):
                J = bonds.get((j - r, j), 0.0)
                if J != 0.0:
                    t.append((f"{op}@{r}", "done", fac * J * ops[comp]))
        sites.append(t)
    return _assemble(chans, sites, 2, SPIN_PHYS, conj)


def heisenberg_j2_derivative(n_sites, j1_bonds, j2_bonds, J2):
    """Return (MPO at J2, [dW/dJ2 per site]).  Couplings enter W only through
    the strand-completing transitions, so W is affine in J2 and the derivative
    is W(J2 = 1) - W(J2 = 0) on the same channel set (zero-valued couplings
    still count towards the FSM range)."""
    def build(scale):
        b = dict(j1_bonds)
        for p, v in j2_bonds.items():
            b[p] = b.get(p, 0.0) + scale * v
        return heisenberg_mpo(n_sites, b)
    full, w0, w1 = build(J2), build(0.0), build(1.0)
    assert w0.names == w1.names == full.names
    return full, [b - a for a, b in zip(w0.W, w1.W)]


_HUB_FLUX = {"cu+": (1, 1), "cu": (-1, -1), "cd+": (1, -1), "cd": (-1, 1)}


def hubbard_mpo(n_sites, hops, U):
    """H = -sum_{(i,j),s} t_ij (c+_is c_js + h.c.) + U sum_i n_iu n_id (Sec. V).

    For i < j:  c+_is c_js = (c~+_s F)_i F_{i+1..j-1} (c~_s)_j  and
                c+_js c_is = (F c~_s)_i  F_{i+1..j-1} (c~+_s)_j,
    with c~_up = b_up, c~_dn = Z_up b_dn the on-site mode operators.  A strand
    carries F between its two ends.
    """
    o = hub_ops()
    R = max((j - i for (i, j) in hops), default=1)
    left_op = {"cu+": o["cu+"] @ o["F"], "cd+": o["cd+"] @ o["F"],
               "cu": o["F"] @ o["cu"], "cd": o["F"] @ o["cd"]}
    comp = {"cu+": o["cu"], "cd+": o["cd"], "cu": o["cu+"], "cd": o["cd+"]}
    chans = [("start", (0, 0))]
    for op in ("cu+", "cu", "cd+", "cd"):
        for r in range(1, R + 1):
            chans.append((f"{op}@{r}", _HUB_FLUX[op]))
    chans.append(("done", (0, 0)))
    conj = {}
    for r in range(1, R + 1):
        conj[f"cu+@{r}"] = f"cu@{r}"; conj[f"cu@{r}"] = f"cu+@{r}"
        conj[f"cd+@{r}"] = f"cd@{r}"; conj[f"cd@{r}"] = f"cd+@{r}"
    sites = []
    for j in range(n_sites):
        t = [("start", "start", o["I"]), ("done", "done", o["I"])]
        if U != 0.0:
            t.append(("start", "done", U * (o["nu"] @ o["nd"])))
        for op in ("cu+", "cu", "cd+", "cd"):
            t.append(("start", f"{op}@1", left_op[op]))
            for r in range(1, R):
                t.append((f"{op}@{r}", f"{op}@{r + 1}", o["F"]))
            for r in range(1, R + 1):
                tij = hops.get((j - r, j), 0.0)
                if tij != 0.0:
                    t.append((f"{op}@{r}", "done", -tij * comp[op]))
        sites.append(t)
    return _assemble(chans, sites, 4, HUB_PHYS, conj)


def synthetic_heisenberg_bond(k, seed):
    """Two MPO sites (W_i, W_{i+1}) of a Heisenberg-type FSM with exactly k
    channels, for isolated-bond workloads.

    n = (k - 2) // 3 strands of (S+, S-, Sz); the remaining (k - 2) % 3 channels
    are extra flux-0 Ising strands (Sz ... Sz).  Couplings are drawn from
    U(0.5, 1.5) with the given seed.
    """
    ops = spin_ops()
    n = (k - 2) // 3
    pad = (k - 2) - 3 * n
    assert n >= 1
    rng = np.random.default_rng([int(seed), 77])
    chans = [("start", (0,))]
    for op in ("S+", "S-", "Sz"):
        for r in range(1, n + 1):
            chans.append((f"{op}@{r}", _spin_flux(op)))
    for p in range(pad):
        chans.append((f"pad{p}", (0,)))
    chans.append(("done", (0,)))
    conj = {}
    for r in range(1, n + 1):
        conj[f"S+@{r}"] = f"S-@{r}"
        conj[f"S-@{r}"] = f"S+@{r}"
    sites = []
    for _site in range(2):
        J = rng.uniform(0.5, 1.5, size=n)
        Jpad = rng.uniform(0.5, 1.5, size=pad)
        t = [("start", "start", ops["I"]), ("done", "done", ops["I"])]
        for op in ("S+", "S-", "Sz"):
            t.append(("start", f"{op}@1", ops[op]))
            for r in range(1, n):
                t.append((f"{op}@{r}", f"{op}@{r + 1}", ops["I"]))
            c, fac = _SPIN_COMP[op]
            for r in range(1, n + 1):
                t.append((f"{op}@{r}", "done", fac * J[r - 1] * ops[c]))
        for p in range(pad):
            t.append(("start", f"pad{p}", ops["Sz"]))
            t.append((f"pad{p}", "done", Jpad[p] * ops["Sz"]))
        sites.append(t)
    return _assemble(chans, sites, 2, SPIN_PHYS, conj)


def synthetic_hubbard_bond(k, seed, U=8.0):
    """Two MPO sites of a Hubbard-type FSM with exactly k channels, for
    isolated-bond workloads of the electron model.

    n = (k - 2) // 4 hopping strands per spin and direction (c+_up, c_up,
    c+_dn, c_dn with Jordan-Wigner strings, as in ``hubbard_mpo`` with hops of
    range 1..n); the remaining (k - 2) % 4 channels are flux-0 density strands
    (n_tot ... n_tot).  Hoppings t_r and densities are drawn from U(0.5, 1.5)
    with the given seed; the on-site term is U n_up n_dn.
    """
    o = hub_ops()
    n = (k - 2) // 4
    pad = (k - 2) - 4 * n
    assert n >= 1
    rng = np.random.default_rng([int(seed), 78])
    left_op = {"cu+": o["cu+"] @ o["F"], "cd+": o["cd+"] @ o["F"],
               "cu": o["F"] @ o["cu"], "cd": o["F"] @ o["cd"]}
    comp = {"cu+": o["cu"], "cd+": o["cd"], "cu": o["cu+"], "cd": o["cd+"]}
    ntot = o["nu"] + o["nd"]
    chans = [("start", (0, 0))]
    for op in ("cu+", "cu", "cd+", "cd"):
        for r in range(1, n + 1):
            chans.append((f"{op}@{r}", _HUB_FLUX[op]))
    for p in range(pad):
        chans.append((f"pad{p}", (0, 0)))
    chans.append(("done", (0, 0)))
    conj = {}
    for r in range(1, n + 1):
        conj[f"cu+@{r}"] = f"cu@{r}"; conj[f"cu@{r}"] = f"cu+@{r}"
        conj[f"cd+@{r}"] = f"cd@{r}"; conj[f"cd@{r}"] = f"cd+@{r}"
    sites = []
    for _site in range(2):
        t_hop = rng.uniform(0.5, 1.5, size=n)
        Jpad = rng.uniform(0.5, 1.5, size=pad)
        t = [("start", "start", o["I"]), ("done", "done", o["I"]),
             ("start", "done", U * (o["nu"] @ o["nd"]))]
        for op in ("cu+", "cu", "cd+", "cd"):
            t.append(("start", f"{op}@1", left_op[op]))
            for r in range(1, n):
                t.append((f"{op}@{r}", f"{op}@{r + 1}", o["F"]))
            for r in range(1, n + 1):
                t.append((f"{op}@{r}", "done", -t_hop[r - 1] * comp[op]))
        for p in range(pad):
            t.append(("start", f"pad{p}", ntot))
            t.append((f"pad{p}", "done", Jpad[p] * ntot))
        sites.append(t)
    return _assemble(chans, sites, 4, HUB_PHYS, conj)
