"""ctypes binding of libbsdmrg.so (argument marshalling only).

Names follow the C ABI in include/bsdmrg.h.  Device buffers are passed as
torch CUDA tensors (FP64, canonical block layout); torch provides device
memory and streams, every step of the computation runs in the library's
kernels.  Loading fails loudly when the shared library is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsdmrg.so")

OK, EINVAL, EQN, ENOMEM, EHIP, ESOLVER, ECAPACITY = range(7)
F64, F32, F32_REFINE = 0, 1, 2
PLAN_HOST_ONLY = 1

PSI_SIGNS = (1, 1, 1, -1)
ENV_SIGNS = (-1, 1, 1)
W_SIGNS = (1, 1, -1, -1)
MPS_SIGNS = (1, 1, -1)


class BsdmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bsdmrg status {status}: {msg}")
        self.status = status


class Leg(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("n_charges", ctypes.c_int32),
                ("charges", ctypes.POINTER(ctypes.c_int32)), ("dims", ctypes.POINTER(ctypes.c_int64))]


class Problem(ctypes.Structure):
    _fields_ = [("a", Leg), ("s1", Leg), ("s2", Leg), ("c", Leg), ("wl", Leg), ("wm", Leg), ("wr", Leg),
                ("w1_host", ctypes.POINTER(ctypes.c_double)), ("w2_host", ctypes.POINTER(ctypes.c_double))]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_probs", "psi_elems", "L_elems", "R_elems", "W1_elems",
                                               "W2_elems", "t1_elems", "t2_elems",
                                               "apply_workspace_bytes", "backward_workspace_bytes")] + \
               [(n, ctypes.c_double) for n in ("flops_s1", "flops_s2", "flops_s3")] + \
               [(n, ctypes.c_int64) for n in ("n_s1_tasks", "n_s3_tasks", "n_s1_tiles", "n_s3_tiles",
                                               "n_mix_terms", "n_coefs", "s1_big_min", "s3_big_min",
                                               "s3_split_k")]


class EigOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("refine_max_iter", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("restart_keep", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("tol", ctypes.c_double), ("tol_f32", ctypes.c_double), ("restart_rtol", ctypes.c_double),
                ("basis", ctypes.c_int32), ("precond", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class EigStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("iters_f32", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("residual", ctypes.c_double), ("thick_restarts", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class TruncOpts(ctypes.Structure):
    _fields_ = [("direction", ctypes.c_int32), ("cutoff_mode", ctypes.c_int32), ("cutoff", ctypes.c_double),
                ("max_m", ctypes.c_int64), ("degen_rtol", ctypes.c_double)]


class EnvProblem(ctypes.Structure):
    _fields_ = [("x", Leg), ("s", Leg), ("y", Leg), ("wl", Leg), ("wr", Leg),
                ("w_host", ctypes.POINTER(ctypes.c_double))]


_lib = None

EXPORTS = ["bsdmrg_layout", "bsdmrg_plan", "bsdmrg_plan_query", "bsdmrg_plan_offsets", "bsdmrg_plan_tasks",
           "bsdmrg_plan_destroy", "bsdmrg_heff_apply", "bsdmrg_heff_apply_noalloc", "bsdmrg_eig_workspace",
           "bsdmrg_eigensolve", "bsdmrg_heff_diagonal",
           "bsdmrg_heff_backward", "bsdmrg_heff_backward_workspace", "bsdmrg_heff_energy", "bsdmrg_stage_timing",
           "bsdmrg_plan_autotune", "bsdmrg_plan_set_tiles", "bsdmrg_truncate_workspace", "bsdmrg_truncate",
           "bsdmrg_env_plan", "bsdmrg_merge_plan", "bsdmrg_op_query", "bsdmrg_op_destroy", "bsdmrg_env_update",
           "bsdmrg_env_backward_workspace", "bsdmrg_env_backward", "bsdmrg_param_derivative",
           "bsdmrg_merge", "bsdmrg_dense_plan", "bsdmrg_dense_apply", "bsdmrg_last_error"]


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2007_05540_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.bsdmrg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "bsdmrg_last_error":
            getattr(lib, name).restype = ctypes.c_int32
    lib.bsdmrg_layout.argtypes = [ctypes.POINTER(Leg), i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                  ctypes.POINTER(i32), ctypes.POINTER(i64), i64]
    lib.bsdmrg_plan.argtypes = [ctypes.POINTER(Problem), i32, i32, ctypes.POINTER(vp)]
    lib.bsdmrg_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.bsdmrg_plan_offsets.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.bsdmrg_plan_tasks.argtypes = [vp, i32, ctypes.POINTER(i64), i64, ctypes.POINTER(i64)]
    lib.bsdmrg_plan_destroy.argtypes = [vp]
    lib.bsdmrg_heff_apply.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    lib.bsdmrg_heff_apply_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.bsdmrg_eig_workspace.argtypes = [vp, ctypes.POINTER(EigOpts), ctypes.POINTER(i64)]
    lib.bsdmrg_heff_diagonal.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.bsdmrg_eigensolve.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(EigOpts),
                                      ctypes.POINTER(dp), ctypes.POINTER(EigStats), vp, i64, vp]
    lib.bsdmrg_heff_backward.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dp), vp, vp, vp, vp, vp, vp,
                                         i64, vp]
    lib.bsdmrg_heff_backward_workspace.argtypes = [vp, ctypes.POINTER(i64)]
    lib.bsdmrg_heff_energy.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(dp), vp, i64, vp]
    lib.bsdmrg_stage_timing.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, i32,
                                        ctypes.POINTER(ctypes.c_float), vp]
    P = ctypes.POINTER
    lib.bsdmrg_plan_autotune.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, i32, P(i32), vp]
    lib.bsdmrg_plan_set_tiles.argtypes = [vp, i32, i32]
    lib.bsdmrg_truncate_workspace.argtypes = [P(Leg), P(i64)]
    lib.bsdmrg_truncate.argtypes = [P(Leg), vp, P(TruncOpts), P(i32), P(i32), P(i64), i32, vp, i64, P(i64), vp,
                                    i64, P(i64), P(dp), i64, P(i64), P(dp), vp, i64, vp]
    lib.bsdmrg_env_plan.argtypes = [P(EnvProblem), i32, i32, P(vp)]
    lib.bsdmrg_merge_plan.argtypes = [P(Leg), i32, P(vp)]
    lib.bsdmrg_op_query.argtypes = [vp, P(i64), P(i64), P(dp)]
    lib.bsdmrg_op_destroy.argtypes = [vp]
    lib.bsdmrg_env_update.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
    lib.bsdmrg_merge.argtypes = [vp, vp, vp, vp, vp]
    lib.bsdmrg_env_backward_workspace.argtypes = [vp, P(i64)]
    lib.bsdmrg_env_backward.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp]
    lib.bsdmrg_param_derivative.argtypes = [i32, P(vp), P(vp), P(i64), vp, P(ctypes.c_double), vp]
    lib.bsdmrg_dense_plan.argtypes = [i64, i64, i32, i32, i32, P(vp)]
    lib.bsdmrg_dense_apply.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    _lib = lib
    return lib


def check(status):
    if status != OK:
        raise BsdmrgError(status, load().bsdmrg_last_error().decode())


# ------------------------------------------------------------- marshalling --
class _LegBuf:
    """Keeps the ctypes arrays of a leg alive."""

    def __init__(self, leg):
        nc = len(leg[0][0])
        self.q = (ctypes.c_int32 * (len(leg) * nc))(*[int(x) for c, _ in leg for x in c])
        self.d = (ctypes.c_int64 * len(leg))(*[int(d) for _, d in leg])
        self.leg = Leg(len(leg), nc, self.q, self.d)


def layout(legs, signs):
    """(block sector tuples [n, order], offsets [n + 1]) of the canonical layout."""
    lib = load()
    bufs = [_LegBuf(l) for l in legs]
    arr = (Leg * len(legs))(*[b.leg for b in bufs])
    sg = (ctypes.c_int32 * len(legs))(*signs)
    n = ctypes.c_int64(0)
    st = lib.bsdmrg_layout(arr, len(legs), sg, ctypes.byref(n), None, None, 0)
    if st not in (OK, ECAPACITY):
        check(st)
    keys = np.zeros(max(1, n.value) * len(legs), dtype=np.int32)
    offs = np.zeros(n.value + 1, dtype=np.int64)
    check(lib.bsdmrg_layout(arr, len(legs), sg, ctypes.byref(n),
                            keys.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n.value))
    return keys[:n.value * len(legs)].reshape(n.value, len(legs)), offs


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A contraction plan over one or more isolated two-site problems.

    problems: list of dicts with keys a, s1, s2, c, wl, wm, wr (legs as
    [(charge tuple, dim)]) and w1, w2 (host FP64 arrays in canonical layout).
    """

    def __init__(self, problems, host_only=False):
        lib = load()
        self._keep = []
        arr = (Problem * len(problems))()
        for i, p in enumerate(problems):
            legs = {k: _LegBuf(p[k]) for k in ("a", "s1", "s2", "c", "wl", "wm", "wr")}
            w1 = np.ascontiguousarray(p["w1"], dtype=np.float64)
            w2 = np.ascontiguousarray(p["w2"], dtype=np.float64)
            self._keep += [legs, w1, w2]
            arr[i] = Problem(*[legs[k].leg for k in ("a", "s1", "s2", "c", "wl", "wm", "wr")],
                             w1.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             w2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        check(lib.bsdmrg_plan(arr, len(problems), PLAN_HOST_ONLY if host_only else 0, ctypes.byref(h)))
        self.handle = h
        self.n_probs = len(problems)
        self._keep = None

    def info(self):
        inf = PlanInfo()
        check(load().bsdmrg_plan_query(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def offsets(self, p):
        o = (ctypes.c_int64 * 5)()
        check(load().bsdmrg_plan_offsets(self.handle, p, o))
        return dict(zip(("psi", "L", "R", "W1", "W2"), list(o)))

    def tasks(self, stage):
        n = ctypes.c_int64(0)
        st = load().bsdmrg_plan_tasks(self.handle, stage, None, 0, ctypes.byref(n))
        if st not in (OK, ECAPACITY):
            check(st)
        buf = np.zeros(4 * max(1, n.value), dtype=np.int64)
        check(load().bsdmrg_plan_tasks(self.handle, stage, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       n.value, ctypes.byref(n)))
        return buf[:4 * n.value].reshape(n.value, 4)

    def destroy(self):
        if self.handle:
            check(load().bsdmrg_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def heff_apply(plan, precision, L, W1, W2, R, psi, out, workspace, stream=None):
    check(load().bsdmrg_heff_apply(plan.handle, precision, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi),
                                   _ptr(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                   _stream(stream)))


NOALLOC_SCRATCH_BYTES = 160 << 20


def heff_apply_noalloc(plan, precision, L, W1, W2, R, psi, out, stream=None):
    """out = H_eff psi with the library's own per-GPU scratch array (no
    workspace argument, nothing allocated by the call)."""
    check(load().bsdmrg_heff_apply_noalloc(plan.handle, precision, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R),
                                           _ptr(psi), _ptr(out), _stream(stream)))


def eig_opts(max_iter=10, precision=F64, refine_max_iter=4, fixed_iters=0, use_graph=0, seed=0, tol=1e-12,
             tol_f32=1e-5, restart_rtol=1e-10, restart_keep=0, basis=0, precond=0, check_every=1):
    """Options of eigensolve (bsdmrg_eig_opts): max_iter products in the first
    phase; with restart_keep = 1 the basis holds at most `basis` vectors
    (0: 64) and is restarted when full; precond = 1 uses the diagonal; in tol
    mode the residual is checked after every check_every-th product."""
    return EigOpts(max_iter, precision, refine_max_iter, fixed_iters, use_graph, restart_keep, seed, tol, tol_f32,
                   restart_rtol, basis, precond, check_every, 0)


def heff_diagonal(plan, L, W1, W2, R, D, stream=None):
    """D = diagonal of H_eff in psi's layout (padding 0)."""
    check(load().bsdmrg_heff_diagonal(plan.handle, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(D),
                                      _stream(stream)))


def eig_workspace(plan, opts):
    n = ctypes.c_int64(0)
    check(load().bsdmrg_eig_workspace(plan.handle, ctypes.byref(opts), ctypes.byref(n)))
    return n.value


def eigensolve(plan, L, W1, W2, R, psi, opts, workspace, stream=None):
    """Returns (energies [n_probs], stats list of dicts); psi is overwritten."""
    np_ = plan.n_probs
    e = (ctypes.c_double * np_)()
    st = (EigStats * np_)()
    check(load().bsdmrg_eigensolve(plan.handle, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi),
                                   ctypes.byref(opts), e, st, _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream)))
    stats = [{f: getattr(s, f) for f, _ in EigStats._fields_} for s in st]
    return list(e), stats


def heff_backward_workspace(plan):
    """Workspace bytes of heff_backward / heff_energy (builds the adjoint tables once)."""
    n = ctypes.c_int64(0)
    check(load().bsdmrg_heff_backward_workspace(plan.handle, ctypes.byref(n)))
    return n.value


def heff_backward(plan, L, W1, W2, R, psi, g_E, d_psi, d_L, d_W1, d_W2, d_R, workspace, stream=None):
    """g_E: one cotangent per problem (a scalar is broadcast).  Outputs may be None."""
    g = np.broadcast_to(np.asarray(g_E, dtype=np.float64), (plan.n_probs,))
    garr = (ctypes.c_double * plan.n_probs)(*[float(x) for x in g])
    check(load().bsdmrg_heff_backward(plan.handle, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi), garr,
                                      _ptr(d_psi), _ptr(d_L), _ptr(d_W1), _ptr(d_W2), _ptr(d_R), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _stream(stream)))


def heff_energy(plan, L, W1, W2, R, psi, workspace, stream=None):
    """[psi_p^T H_eff,p psi_p for every problem p] (FP64)."""
    e = (ctypes.c_double * plan.n_probs)()
    check(load().bsdmrg_heff_energy(plan.handle, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi), e,
                                    _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream(stream)))
    return list(e)


def stage_timing(plan, precision, L, W1, W2, R, psi, out, workspace, reps=20, stream=None):
    """Average ms per launch of {coef, S1, S2, S3 GEMM, S3 split-K sum}, timed
    with HIP events on the stream."""
    ms = (ctypes.c_float * 5)()
    check(load().bsdmrg_stage_timing(plan.handle, precision, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi),
                                     _ptr(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     reps, ms, _stream(stream)))
    return dict(zip(("coef", "s1", "s2", "s3", "s3_sum"), list(ms)))


NO_BIG_TILES = 1 << 30


def plan_autotune(plan, precision, L, W1, W2, R, psi, out, workspace, reps=10, stream=None):
    """Pick the tile shape classes of the S1 and S3 launches by timing (see
    bsdmrg_plan_autotune); returns {"s1": big_min, "s3": big_min}."""
    bm = (ctypes.c_int32 * 2)()
    check(load().bsdmrg_plan_autotune(plan.handle, precision, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi),
                                      _ptr(out), _ptr(workspace), workspace.numel() * workspace.element_size(),
                                      reps, bm, _stream(stream)))
    return {"s1": int(bm[0]), "s3": int(bm[1])}


def plan_set_tiles(plan, s1_big_min, s3_big_min):
    """Install tile shape classes (tasks with M and N >= big_min use 128 x 128
    tiles; NO_BIG_TILES: 64 x 64 tiles only)."""
    check(load().bsdmrg_plan_set_tiles(plan.handle, int(s1_big_min), int(s3_big_min)))


# ------------------------------------------------------------ sweep ops ----
class Op:
    """An environment-extension or merge op (plan tables on the device)."""

    def __init__(self, handle):
        self.handle = handle

    def query(self):
        ws, n = ctypes.c_int64(0), ctypes.c_int64(0)
        f = ctypes.c_double(0)
        check(load().bsdmrg_op_query(self.handle, ctypes.byref(ws), ctypes.byref(n), ctypes.byref(f)))
        return {"workspace_bytes": ws.value, "out_elems": n.value, "flops": f.value}

    def destroy(self):
        if self.handle:
            check(load().bsdmrg_op_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def env_plan(x, s, y, wl, wr, w_host, side, host_only=False):
    """side 0: left extension (env (x,wl,x), A (x,s,y) -> (y,wr,y));
    side 1: right extension (env (x,wr,x), B (y,s,x) -> (y,wl,y))."""
    bufs = [_LegBuf(l) for l in (x, s, y, wl, wr)]
    w = np.ascontiguousarray(w_host, dtype=np.float64)
    prob = EnvProblem(*[b.leg for b in bufs], w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    check(load().bsdmrg_env_plan(ctypes.byref(prob), side, PLAN_HOST_ONLY if host_only else 0, ctypes.byref(h)))
    return Op(h)


def merge_plan(a, s1, b, s2, c, host_only=False):
    bufs = [_LegBuf(l) for l in (a, s1, b, s2, c)]
    arr = (Leg * 5)(*[x.leg for x in bufs])
    h = ctypes.c_void_p()
    check(load().bsdmrg_merge_plan(arr, PLAN_HOST_ONLY if host_only else 0, ctypes.byref(h)))
    return Op(h)


def env_update(op, env, mps, W, env_out, workspace, stream=None):
    nb = 0 if workspace is None else workspace.numel() * workspace.element_size()
    check(load().bsdmrg_env_update(op.handle, _ptr(env), _ptr(mps), _ptr(W), _ptr(env_out), _ptr(workspace), nb,
                                   _stream(stream)))


def env_backward_workspace(op):
    n = ctypes.c_int64(0)
    check(load().bsdmrg_env_backward_workspace(op.handle, ctypes.byref(n)))
    return n.value


def param_derivative(grads, dW_dp, terms, stream=None):
    """sum_s <grads[s], dW_dp[s]> on the device (see the header); grads and
    dW_dp are lists of device tensors in canonical W layout, terms a device
    tensor of len(grads) + 1 doubles.  Returns the sum."""
    n = len(grads)
    if len(dW_dp) != n:
        raise ValueError("param_derivative: one derivative tensor per site")
    for g, d in zip(grads, dW_dp):
        if g.numel() != d.numel():
            raise ValueError("param_derivative: gradient and derivative sizes differ")
    x = (ctypes.c_void_p * n)(*[_ptr(g) for g in grads])
    y = (ctypes.c_void_p * n)(*[_ptr(d) for d in dW_dp])
    cnt = (ctypes.c_int64 * n)(*[g.numel() for g in grads])
    out = ctypes.c_double(0.0)
    check(load().bsdmrg_param_derivative(n, x, y, cnt, _ptr(terms), ctypes.byref(out), _stream(stream)))
    return out.value


def env_backward(op, env, mps, d_out, d_W, workspace, stream=None):
    """d_W = cotangent of W of an environment op (see the header)."""
    check(load().bsdmrg_env_backward(op.handle, _ptr(env), _ptr(mps), _ptr(d_out), _ptr(d_W), _ptr(workspace),
                                     workspace.numel() * workspace.element_size(), _stream(stream)))


def dense_plan(ma, mc, k, d, host_only=False):
    """Op of the two-site product in the sparse-dense format (see the header)."""
    h = ctypes.c_void_p()
    check(load().bsdmrg_dense_plan(int(ma), int(mc), int(k), int(d), PLAN_HOST_ONLY if host_only else 0,
                                   ctypes.byref(h)))
    return Op(h)


def dense_apply(op, precision, L, W1, W2, R, psi, out, workspace, stream=None):
    """out = H_eff psi with dense FP64 device operands (see the header)."""
    check(load().bsdmrg_dense_apply(op.handle, precision, _ptr(L), _ptr(W1), _ptr(W2), _ptr(R), _ptr(psi), _ptr(out),
                                    _ptr(workspace), workspace.numel() * workspace.element_size(),
                                    _stream(stream)))


def merge(op, A, B, theta, stream=None):
    check(load().bsdmrg_merge(op.handle, _ptr(A), _ptr(B), _ptr(theta), _stream(stream)))


def truncate_workspace(theta_legs):
    bufs = [_LegBuf(l) for l in theta_legs]
    arr = (Leg * 4)(*[b.leg for b in bufs])
    n = ctypes.c_int64(0)
    check(load().bsdmrg_truncate_workspace(arr, ctypes.byref(n)))
    return n.value


def truncate(theta_legs, theta, direction, cutoff=0.0, cutoff_mode=0, max_m=1 << 62, degen_rtol=1e-10,
             stream=None):
    """Returns (A, B, new_leg, kept singular values, discarded weight);
    A and B are new FP64 device tensors in canonical layout."""
    import torch
    lib = load()
    bufs = [_LegBuf(l) for l in theta_legs]
    arr = (Leg * 4)(*[b.leg for b in bufs])
    ws = torch.empty(truncate_workspace(theta_legs), dtype=torch.uint8, device=theta.device)
    o = TruncOpts(direction, cutoff_mode, cutoff, max_m, degen_rtol)
    nc = len(theta_legs[0][0][0])
    a, s1, s2, c = theta_legs
    # exact capacity bounds from the per-charge matrix sizes (kept <= min(rows, cols, max_m))
    rows, cols = {}, {}
    for qa, da in a:
        for qs, ds in s1:
            rows.setdefault(tuple(x + y for x, y in zip(qa, qs)), []).append(da * ds)
    for qs, ds in s2:
        for qc, dc in c:
            cols.setdefault(tuple(x - y for x, y in zip(qc, qs)), []).append(ds * dc)
    rup = lambda x: (x + 31) // 32 * 32
    cap_leg, cap_sv, cap_A, cap_B = 1, 1, 1, 1
    for qq, rl in rows.items():
        if qq not in cols:
            continue
        k = min(sum(rl), sum(cols[qq]), max_m)
        cap_leg += 1
        cap_sv += k
        cap_A += sum(rup(r * k) for r in rl)
        cap_B += sum(rup(k * cc) for cc in cols[qq])
    new_n = ctypes.c_int32(0)
    q = (ctypes.c_int32 * (cap_leg * nc))()
    d = (ctypes.c_int64 * cap_leg)()
    an, bn, nk = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    disc = ctypes.c_double(0)
    A = torch.empty(cap_A, dtype=torch.float64, device=theta.device)
    B = torch.empty(cap_B, dtype=torch.float64, device=theta.device)
    sv = (ctypes.c_double * cap_sv)()
    check(lib.bsdmrg_truncate(arr, _ptr(theta), ctypes.byref(o), ctypes.byref(new_n), q, d, cap_leg, _ptr(A),
                              cap_A, ctypes.byref(an), _ptr(B), cap_B, ctypes.byref(bn), sv, cap_sv,
                              ctypes.byref(nk), ctypes.byref(disc), _ptr(ws), ws.numel(), _stream(stream)))
    leg = [(tuple(q[i * nc + k] for k in range(nc)), int(d[i])) for i in range(new_n.value)]
    return A[:an.value].clone(), B[:bn.value].clone(), leg, list(sv)[:nk.value], disc.value
