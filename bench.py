"""Benchmark of the block-sparse two-site H_eff product inside the Davidson
eigensolver on one MI355X.

Workload (default): the isolated mid-chain bond of a 6x6 Heisenberg cylinder,
m = 1024 on both bond legs (21 spin sectors, largest block 270, sector model of
the paper's Table 2), MPO k = 14, random Hermitian-structured environments,
random start vector; synthetic seeded inputs.

One step = one converged bsdmrg_eigensolve call (bounded basis with thick
restart), from the same start vector, until the FP64 residual ||q|| <= --tol:
  mixed path (the reported value): FP32-MFMA products until the FP32 phase's
      residual reaches --tol-f32, then FP64 products from the two kept basis
      vectors; all orthogonalisation, Rayleigh quotients and the energy FP64;
  f64 path: FP64 products throughout.
Both reach the same accuracy (their energies agree to ~1e-11 here; the line
reports the difference and the eigenvector error between them).
value = useful GFLOP/s = (products per solve x useful flops per product) /
time per solve, useful flops being the block-pair flops of the two GEMM
stages (the flop definition of the paper's list method), Davidson overhead
included in the time.

The JSON line also carries the per-stage times and MFMA rooflines of one
product in both precisions (m = 1024 and m = 2048, k = 18), the roofline of the
dominant FP32 grouped GEMM, the same product in the sparse-dense format (the
work the blocks avoid), the 64-bond batch (one launch per stage for all
bonds, fixed 10-step solves), the m = 4096 Hubbard-type bond (U(1)xU(1),
k = 22), sweeps of the 6x6 J1-J2 cylinder at m = 256 (s/sweep of the FP64 and
the mixed path at equal accuracy) and of the 16-site chain, and the oracle's
CPU rate (cpu_baseline).  Other workloads: --workload j1j2-6x6 (adds dE/dJ2 by
the adjoint and by finite differences), chain16, hubbard-4x16.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3}      # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                       # GB/s
# HBM bytes per launch of the FP32 S1 / S3 grouped GEMM on the m=1024, k=14
# bond as the mixed eigensolve launches them (S3 with FP32 output), from
# rocprofv3 FETCH_SIZE and WRITE_SIZE counters of the current kernels
# (FETCH_SIZE scaled by 1.997 and WRITE_SIZE by 1.000, the ratios of the
# known bytes of the FP32 cast of L, a plain elementwise kernel, to what the
# counters read for it)
HBM_TRAFFIC = {"s1": 74163245, "s3": 77817309}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-f32", type=int, default=10)
    ap.add_argument("--n-f64", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-bond batch measurement")
    ap.add_argument("--no-hubbard", action="store_true", help="skip the m=4096 Hubbard bond measurement")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the 6x6 J1-J2 cylinder at m=512 (sweeps, dE/dJ2 by the adjoint and by finite "
                         "differences, FP64 vs mixed s/sweep) and the 16-site chain sweeps")
    ap.add_argument("--workload", default="bond", choices=["bond", "j1j2-6x6", "chain16", "hubbard-4x16", "bond-m2048", "bond-m1024-stages"],
                    help="bond: the isolated-bond product bench (default); j1j2-6x6: DMRG sweeps on the "
                         "6x6 J1-J2 cylinder, dE/dJ2 by the adjoint and by finite differences; chain16: "
                         "sweeps of the 16-site Heisenberg chain; hubbard-4x16: sweeps of the 4x16 Hubbard "
                         "cylinder at half filling; bond-m2048 / bond-m1024-stages: per-stage rooflines of the "
                         "m=2048, k=18 bond / of the headline m=1024, k=14 bond only")
    ap.add_argument("--m-max", type=int, default=512)
    ap.add_argument("--tol", type=float, default=1e-5, help="FP64 residual of a converged solve")
    ap.add_argument("--tol-f32", type=float, default=1e-5, help="residual that ends the FP32 phase")
    ap.add_argument("--basis", type=int, default=16, help="Davidson basis (thick restart to 2 vectors)")
    ap.add_argument("--max-products", type=int, default=1000)
    ap.add_argument("--check-every", type=int, default=4,
                    help="read the residual back after every this many products (tol-driven solves)")
    ap.add_argument("--no-large", action="store_true", help="skip the m=2048, k=18 bond stage rooflines")
    return ap.parse_args()


def cpu_baseline(spec, flops, budget_s):
    """The oracle's block-loop product (one NumPy matmul per block pair),
    timed on the host cores on a bounded number of products: with the host
    BLAS threads on all cores (the reported value) and on one core."""
    from oracle.heff import bond_operands, heff_blocks
    blas, cores, limit = "unknown", os.cpu_count(), None
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        info = threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
        blas = ", ".join(sorted({f"{i.get('internal_api', '?')} {i.get('version', '')}".strip() for i in info}))
        limit = threadpool_limits
    except Exception:
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        pass
    L, W1, W2, R, psi = bond_operands(spec)

    def rate(budget):
        heff_blocks(L, W1, W2, R, psi)          # warm-up
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget or n == 0:
            heff_blocks(L, W1, W2, R, psi)
            n += 1
        return n, (time.perf_counter() - t0) / n
    n, dt = rate(budget_s)
    out = {"value": round(flops / dt / 1e9, 3), "unit": "useful GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{n} FP64 block-loop H_eff products of the m=1024 k=14 bond ({dt:.3f} s each)",
           "cpu_model": model, "nproc": os.cpu_count(), "blas": blas}
    if limit is not None:
        with limit(limits=1):
            n1, dt1 = rate(budget_s / 3)
        out["value_1_core"] = round(flops / dt1 / 1e9, 3)
        out["sample_1_core"] = f"{n1} products ({dt1:.3f} s each)"
    return out


def batch_bench(args):
    """64 independent bonds (widths 4/6/8 -> k = 10/14/18, m drawn from
    256..2048) planned as one batch: every stage of a product runs as one
    grouped launch over all 64 problems, and the fixed-step Davidson solve is
    captured once as a hipGraph.  Returns ms per batched Davidson step and
    useful GFLOP/s for the FP64 and the mixed schedule."""
    import torch
    import synth
    from paper_2007_05540_amd import lib, problems

    t0 = time.perf_counter()
    specs = synth.c3_batch()
    pairs = [problems.bond_problem(s) for s in specs]
    probs = [p for p, _ in pairs]
    plan = lib.Plan(probs)
    ops = problems.concat(plan, [o for _, o in pairs])
    del pairs
    info = plan.info()
    flops = info["flops_s1"] + info["flops_s3"]
    dev = {k: torch.from_numpy(v).to("cuda") for k, v in ops.items()}
    del ops
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    out = {"problems": len(specs), "useful_gflop_per_batched_product": round(flops / 1e9, 3),
           "setup_s": round(setup_s, 1), "tiles": autotune(plan, info, dev, stream)}
    energies = {}
    for path in ("f64", "mixed"):
        if path == "mixed":
            o = lib.eig_opts(max_iter=args.n_f32, precision=lib.F32_REFINE, refine_max_iter=args.n_f64,
                             fixed_iters=1, use_graph=1)
        else:
            o = lib.eig_opts(max_iter=args.n_f32 + args.n_f64, fixed_iters=1, use_graph=1)
        ws = torch.empty(lib.eig_workspace(plan, o), dtype=torch.uint8, device="cuda")
        psi = torch.empty_like(dev["psi"])
        with torch.cuda.stream(stream):
            for _ in range(2):
                psi.copy_(dev["psi"])
                lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws, stream=stream)
            torch.cuda.synchronize()
            reps = max(2, args.steps // 4)
            t1 = time.perf_counter()
            for _ in range(reps):
                psi.copy_(dev["psi"])
                e, st = lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws,
                                       stream=stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / reps
        products = args.n_f32 + args.n_f64
        energies[path] = list(e)
        out[path] = {"ms_per_davidson_step": round(dt * 1e3, 3),
                     "useful_gflops": round(products * flops / dt / 1e9, 1)}
        del ws, psi
    out["speedup_mixed_vs_f64"] = round(out["f64"]["ms_per_davidson_step"] / out["mixed"]["ms_per_davidson_step"], 3)

    # the plain FP64 path: one plan and one FP64 solve per bond (the same
    # fixed schedule), called one after another, on views of the same operands
    plans = [lib.Plan([p]) for p in probs]
    o = lib.eig_opts(max_iter=args.n_f32 + args.n_f64, fixed_iters=1, use_graph=1)
    ws = torch.empty(max(lib.eig_workspace(pl, o) for pl in plans), dtype=torch.uint8, device="cuda")
    psi = torch.empty_like(dev["psi"])
    views = []
    for i, pl in enumerate(plans):
        off, pi = plan.offsets(i), pl.info()
        size = {"psi": pi["psi_elems"], "L": pi["L_elems"], "R": pi["R_elems"], "W1": pi["W1_elems"],
                "W2": pi["W2_elems"]}
        views.append({k: (dev[k] if k != "psi" else psi)[off[k]:off[k] + size[k]] for k in size})

    def plain_pass():
        e_all = []
        for pl, v in zip(plans, views):
            e, _ = lib.eigensolve(pl, v["L"], v["W1"], v["W2"], v["R"], v["psi"], o, ws, stream=stream)
            e_all.append(e[0])
        return e_all

    with torch.cuda.stream(stream):
        psi.copy_(dev["psi"])
        plain_pass()
        torch.cuda.synchronize()
        reps = max(2, args.steps // 4)
        t1 = time.perf_counter()
        for _ in range(reps):
            psi.copy_(dev["psi"])
            e_plain = plain_pass()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
    products = args.n_f32 + args.n_f64
    out["plain_f64"] = {"ms_per_davidson_step": round(dt * 1e3, 3),
                        "useful_gflops": round(products * flops / dt / 1e9, 1),
                        "max_energy_diff_vs_batched_f64": float(max(abs(a - b) for a, b in
                                                                    zip(e_plain, energies["f64"])))}
    out["speedup_mixed_batched_vs_plain_f64"] = round(dt * 1e3 / out["mixed"]["ms_per_davidson_step"], 3)
    out["speedup_f64_batched_vs_plain_f64"] = round(dt * 1e3 / out["f64"]["ms_per_davidson_step"], 3)
    # the fixed schedule is not a converged solve: the mixed energies differ
    # from the FP64 ones by the FP32 error of an unconverged Krylov space
    out["max_rel_energy_diff_mixed_vs_f64"] = float(max(abs(a - b) / abs(b) for a, b in
                                                        zip(energies["mixed"], energies["f64"])))
    for pl in plans:
        pl.destroy()
    del ws, psi, views
    plan.destroy()
    return out


def j1j2_bench(args, with_fd=True):
    """Two-site DMRG on the 6x6 J1-J2 Heisenberg cylinder (J2/J1 = 0.5,
    width 6 periodic, length 6 open), U(1) Sz, m up to --m-max, from a seeded
    random MPS; then dE/dJ2 by reverse mode (EnvUpdate x sites -> HeffEnergy ->
    adjoint, chain rule over the MPO builder's dW/dJ2) and by central finite
    differences of warm-started DMRG energies at J2 +- 1e-4; and one sweep
    from the converged state in FP64 and in mixed precision (s/sweep at
    equal accuracy)."""
    import torch
    import synth
    from paper_2007_05540_amd import lib, problems, dmrg as gdmrg, mpo as gmpo

    Wd, Lx, J2, h = 6, 6, 0.5, 1e-4
    n = Wd * Lx
    j1, j2 = synth.cylinder_j1_bonds(Wd, Lx), synth.cylinder_j2_bonds(Wd, Lx)
    # the sweeps run with the SVD-compressed operator (cutoff 1e-13 of its
    # norm); the adjoint differentiates the builder's own operator, whose
    # site tensors are affine in J2, at the same converged state
    full, dWs = synth.heisenberg_j2_derivative(n, j1, j2, J2)
    k_full = sum(d for _, d in full.w_leg())
    mpo = gmpo.compress(full)
    k = max(mpo.bond_dims())
    m = args.m_max
    sched = [min(m, x) for x in (64, 128, 256)] + [m] * 3
    opts = dict(cutoff=1e-10, max_iter=30, tol=1e-10)
    def log(tag):
        return lambda sw, e, t: print(f"{tag} sweep {sw}: E = {e:.12f} ({t:.2f} s)", file=sys.stderr, flush=True)

    g = gdmrg.GpuDMRG(mpo, problems.initial_mps(mpo, (0,), 16, 5), (0,))
    _, swe = g.run(len(sched), sched, on_sweep=log("dmrg"), **opts)
    warm = g.host_mps()
    sweep = {}
    for name, prec in (("f64", lib.F64), ("mixed", lib.F32_REFINE)):
        gg = gdmrg.GpuDMRG(mpo, warm, (0,), precision=prec, refine_max_iter=10, tol_f32=1e-6)
        _, e = gg.run(1, m, on_sweep=log(name), **opts)
        sweep[name] = {"s_per_sweep": round(gg.sweep_seconds[0], 3), "energy": e[-1]}
    sweep["energy_rel_diff"] = abs(sweep["mixed"]["energy"] - sweep["f64"]["energy"]) / abs(sweep["f64"]["energy"])
    sweep["speedup_mixed_vs_f64"] = round(sweep["f64"]["s_per_sweep"] / sweep["mixed"]["s_per_sweep"], 3)
    if not with_fd:
        return {"workload": f"6x6 J1-J2 Heisenberg cylinder, J2/J1=0.5, U(1) Sz, m={m}", "mpo_k": k,
                "mpo_k_uncompressed": k_full,
                "m_schedule": sched, "sweep_energies": swe, "sweep_seconds": [round(t, 3) for t in g.sweep_seconds],
                "one_sweep_from_converged": sweep}
    t0 = time.perf_counter()
    ga = gdmrg.GpuDMRG(full, warm, (0,))
    E_bond, grads = ga.energy_and_mpo_gradients(0)
    dE_adj = ga.parameter_derivative(grads, dWs)
    t_adj = time.perf_counter() - t0
    ef = {}
    for sgn in (1, -1):
        mp, _ = synth.heisenberg_j2_derivative(n, j1, j2, J2 + sgn * h)
        gg = gdmrg.GpuDMRG(gmpo.compress(mp), warm, (0,))
        _, e = gg.run(2, m, on_sweep=log(f"J2{sgn * h:+g}"), **opts)
        ef[sgn] = e[-1]
    dE_fd = (ef[1] - ef[-1]) / (2 * h)
    return {"metric": "6x6 J1-J2 cylinder: DMRG energy and dE/dJ2 (adjoint vs finite differences)",
            "config": {"workload": "6x6 J1-J2 Heisenberg cylinder, J2/J1=0.5, U(1) Sz", "mpo_k": k,
                       "mpo_k_uncompressed": k_full,
                       "m_schedule": sched, "cutoff": opts["cutoff"], "davidson_tol": opts["tol"]},
            "sweep_energies": swe, "sweep_seconds": [round(t, 3) for t in g.sweep_seconds],
            "energy_per_site": swe[-1] / n, "bond_energy": E_bond,
            "dE_dJ2_adjoint": dE_adj, "adjoint_seconds": round(t_adj, 3),
            "dE_dJ2_finite_difference": dE_fd, "fd_step": h,
            "rel_diff_adjoint_vs_fd": abs(dE_adj - dE_fd) / abs(dE_fd),
            "one_sweep_from_converged": sweep, "data": "synthetic (seeded random initial MPS)"}


def sweeps_bench(args):
    """Two-site DMRG sweeps, FP64 path against the mixed path (FP32 products,
    FP64 refinement) from the same seeded initial MPS: seconds per sweep and
    the energy of every sweep.
      chain16: 16-site Heisenberg chain, U(1) Sz = 0, m = 64 (4 sweeps),
               cutoff 1e-10, Davidson tol 1e-12;
      hubbard-4x16: 4 x 16 Hubbard cylinder (t = 1, U = 8, periodic width 4),
               half filling N = 64, 2Sz = 0, U(1)xU(1), m growing to --m-max
               (two sweeps at each of 256, 512, ..., m_max), cutoff 1e-10,
               Davidson tol 1e-10."""
    import torch
    import synth
    from paper_2007_05540_amd import lib, problems
    from paper_2007_05540_amd import dmrg as gdmrg

    if args.workload == "chain16":
        n = 16
        mpo = synth.heisenberg_mpo(n, synth.chain_bonds(n))
        target, sched, opts = (0,), [64] * 4, dict(cutoff=1e-10, max_iter=40, tol=1e-12)
        desc = "16-site Heisenberg chain, U(1) Sz=0, m=64"
    else:
        Wd, Lx = 4, 16
        n = Wd * Lx
        mpo = synth.hubbard_mpo(n, synth.cylinder_j1_bonds(Wd, Lx), 8.0)
        target = (n, 0)
        sched, m = [], 256
        while m < args.m_max:
            sched += [m, m]
            m *= 2
        sched += [args.m_max, args.m_max]
        opts = dict(cutoff=1e-10, max_iter=40, tol=1e-10)
        desc = f"4x16 Hubbard cylinder, t=1, U=8, half filling, U(1)xU(1), m up to {args.m_max}"
    k = sum(d for _, d in mpo.w_leg())
    out = {"metric": "two-site DMRG seconds per sweep: FP64 vs mixed (FP32 products + FP64 refinement)",
           "config": {"workload": desc, "mpo_k": k, "m_schedule": sched, **opts},
           "data": "synthetic (seeded random initial MPS)"}
    mps0 = problems.initial_mps(mpo, target, 16, 0)
    for name, prec in (("f64", lib.F64), ("mixed", lib.F32_REFINE)):
        def log(sw, e, t):
            print(f"{name} sweep {sw}: E = {e:.12f} ({t:.2f} s)", file=sys.stderr, flush=True)
        g = gdmrg.GpuDMRG(mpo, mps0, target, precision=prec, refine_max_iter=10, tol_f32=1e-6)
        _, swe = g.run(len(sched), sched, on_sweep=log, **opts)
        out[name] = {"sweep_energies": swe, "sweep_seconds": [round(t, 3) for t in g.sweep_seconds],
                     "final_m": max(r["m"] for r in g.log[-(n - 1):]),
                     "davidson_products": sum(r["iters"] + r["iters_f32"] for r in g.log)}
        del g
        torch.cuda.empty_cache()
    ef, em = out["f64"]["sweep_energies"][-1], out["mixed"]["sweep_energies"][-1]
    out["final_energy_rel_diff"] = abs(em - ef) / abs(ef)
    out["speedup_mixed_vs_f64_total"] = round(sum(out["f64"]["sweep_seconds"]) / sum(out["mixed"]["sweep_seconds"]), 3)
    return out


def dense_ablation(spec, plan, dev, reps=5):
    """The same product in the sparse-dense format (all operands dense, one
    library GEMM per stage; the work the block structure avoids is done):
    ms per product in FP64 and FP32 and its agreement with the block-sparse
    product."""
    import torch
    from paper_2007_05540_amd import lib, problems, dense
    wl, s = spec.w_leg(), spec.s_leg
    legs_psi = [spec.a_leg, s, s, spec.c_leg]
    host = {"L": problems.unpack_dense(dev["L"].cpu().numpy(), [spec.a_leg, wl, spec.a_leg], lib.ENV_SIGNS),
            "R": problems.unpack_dense(dev["R"].cpu().numpy(), [spec.c_leg, wl, spec.c_leg], lib.ENV_SIGNS),
            "psi": problems.unpack_dense(dev["psi"].cpu().numpy(), legs_psi, lib.PSI_SIGNS),
            "W1": spec.W1, "W2": spec.W2}
    ma, k, _ = host["L"].shape
    mc, d = host["R"].shape[0], host["psi"].shape[1]
    f1, f2, f3 = dense.dense_flops(ma, mc, k, d)
    out = {"dense_gflop_per_product": round((f1 + f2 + f3) / 1e9, 2)}
    ref = torch.zeros_like(dev["psi"])
    ws = torch.empty(plan.info()["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    lib.heff_apply(plan, lib.F64, dev["L"], dev["W1"], dev["W2"], dev["R"], dev["psi"], ref, ws)
    ref = ref.cpu().numpy()
    del ws
    t = {kk: torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for kk, v in host.items()}
    dp = dense.DenseProduct(ma, mc, k, d)
    y = torch.zeros_like(t["psi"])
    for name, prec in (("f64", lib.F64), ("f32", lib.F32)):
        dp.apply(prec, t["L"], t["W1"], t["W2"], t["R"], t["psi"], y)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            dp.apply(prec, t["L"], t["W1"], t["W2"], t["R"], t["psi"], y)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        got = problems.pack_dense(y.cpu().numpy(), legs_psi, lib.PSI_SIGNS)
        out[name] = {"ms_per_product": round(ms, 3), "dense_tflops": round((f1 + f2 + f3) / ms / 1e9, 1),
                     "rel_diff_vs_block_sparse_f64": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
    dp.destroy()
    del t, y
    torch.cuda.empty_cache()
    return out


def autotune(plan, info, dev, stream):
    """Tile shape classes of the S1/S3 launches chosen by the library's
    autotuner (timed in FP32, the precision of most products), and the S3
    split-K width the plan chose."""
    import torch
    from paper_2007_05540_amd import lib
    ws = torch.empty(info["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    out = torch.empty_like(dev["psi"])
    got = lib.plan_autotune(plan, lib.F32, dev["L"], dev["W1"], dev["W2"], dev["R"], dev["psi"], out, ws,
                            reps=10, stream=stream)
    del ws, out
    res = {k: ("64x64 only" if v >= lib.NO_BIG_TILES else f"128x128 for M,N>={v}") for k, v in got.items()}
    res["s3_split_k"] = info["s3_split_k"] if info["s3_split_k"] > 0 else "none"
    return res


def bond_measure(spec, args):
    """Plan one isolated bond, upload its operands and time the FP64 and the
    mixed fixed-step Davidson solves (graph replay).  Returns the plan, its
    info, the useful flops per product, the device operands and the results."""
    import torch
    from paper_2007_05540_amd import lib, problems

    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    info = plan.info()
    flops = info["flops_s1"] + info["flops_s3"]
    dev = {k: torch.from_numpy(v).to("cuda") for k, v in ops.items()}
    del ops
    stream = torch.cuda.Stream()
    psi0 = dev["psi"]
    results = {"tiles": autotune(plan, info, dev, stream)}
    for path in ("f64", "mixed"):
        if path == "mixed":
            o = lib.eig_opts(max_iter=args.n_f32, precision=lib.F32_REFINE, refine_max_iter=args.n_f64,
                             fixed_iters=1, use_graph=1)
        else:
            o = lib.eig_opts(max_iter=args.n_f32 + args.n_f64, fixed_iters=1, use_graph=1)
        ws = torch.empty(lib.eig_workspace(plan, o), dtype=torch.uint8, device="cuda")
        psi = torch.empty_like(psi0)
        energy = None
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                psi.copy_(psi0)
                energy, st = lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws,
                                            stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                psi.copy_(psi0)
                energy, st = lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws,
                                            stream=stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
        products = args.n_f32 + args.n_f64
        results[path] = {"ms_per_step": dt * 1e3, "gflops": products * flops / dt / 1e9,
                         "energy": energy[0], "residual": st[0]["residual"], "products": products}
        del ws, psi
    return plan, info, flops, dev, results


def hubbard_bond_bench(args):
    """The isolated mid-chain bond of the 4x16 Hubbard cylinder at half
    filling: electron sector model at m = 4096 (313 U(1)xU(1) sectors, largest
    block 468), Hubbard-type MPO with k = 22, the same fixed-step solves."""
    import torch
    import synth

    spec = synth.c4_bond(m=4096, k=22, seed=1)
    t0 = time.perf_counter()
    plan, info, flops, dev, res = bond_measure(spec, args)
    out = {"workload": "isolated mid-chain two-site bond, 4x16 Hubbard cylinder, m=4096, k=22, "
                       "313 U(1)xU(1) sectors",
           "useful_gflop_per_product": round(flops / 1e9, 3), "s1_tasks": info["n_s1_tasks"],
           "s3_tasks": info["n_s3_tasks"], "tiles": res.pop("tiles")}
    for path in ("f64", "mixed"):
        out[path] = {"ms_per_davidson_step": round(res[path]["ms_per_step"], 3),
                     "useful_gflops": round(res[path]["gflops"], 1), "energy": res[path]["energy"]}
    out["speedup_mixed_vs_f64"] = round(res["f64"]["ms_per_step"] / res["mixed"]["ms_per_step"], 3)
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    del dev
    plan.destroy()
    torch.cuda.empty_cache()
    return out


def converged_solves(plan, info, dev, args, stream):
    """Time-to-solution of the FP64 path and of the mixed path on one bond,
    both run until the FP64 residual ||q|| <= args.tol (the mixed path: FP32
    products until its own residual reaches args.tol_f32, then FP64 products
    from the kept basis), from the same start vector.  Returns per path the
    ms per converged solve (mean of --steps solves after --warmup), the
    products of each precision, the energy and the residual."""
    import torch
    from paper_2007_05540_amd import lib
    flops = info["flops_s1"] + info["flops_s3"]
    common = dict(restart_keep=1, basis=args.basis, tol=args.tol, max_iter=args.max_products,
                  check_every=args.check_every)
    opts = {"f64": lib.eig_opts(**common),
            "mixed": lib.eig_opts(precision=lib.F32_REFINE, refine_max_iter=args.max_products, tol_f32=args.tol_f32,
                                  **common)}
    out = {}
    for path, o in opts.items():
        ws = torch.empty(lib.eig_workspace(plan, o), dtype=torch.uint8, device="cuda")
        psi = torch.empty_like(dev["psi"])
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                psi.copy_(dev["psi"])
                lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                psi.copy_(dev["psi"])
                e, st = lib.eigensolve(plan, dev["L"], dev["W1"], dev["W2"], dev["R"], psi, o, ws, stream=stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
        products = st[0]["iters"] + st[0]["iters_f32"]
        out[path] = {"ms_per_solve": dt * 1e3, "products_f32": st[0]["iters_f32"], "products_f64": st[0]["iters"],
                     "energy": e[0], "residual": st[0]["residual"], "converged": bool(st[0]["converged"]),
                     "thick_restarts": st[0]["thick_restarts"], "gflops": products * flops / dt / 1e9,
                     "psi": psi.clone()}
        del ws
    return out


def stage_roofline(plan, info, dev, stream, reps=20):
    """Per-stage ms of one product in both precisions (HIP events on the
    launch stream) and the MFMA roofline of the two grouped-GEMM stages."""
    import torch
    from paper_2007_05540_amd import lib
    out = torch.zeros_like(dev["psi"])
    wsa = torch.empty(info["apply_workspace_bytes"], dtype=torch.uint8, device="cuda")
    stage, roof = {}, {}
    # f32: the FP32 product of bsdmrg_heff_apply (FP64 output); f32_solve: the
    # same stages as the FP32 phase of the mixed eigensolve runs them (S3 and
    # its split-K sum write FP32 products)
    for prec, name, peak in ((lib.F32, "f32", "f32"), (lib.F32_REFINE, "f32_solve", "f32"), (lib.F64, "f64", "f64")):
        ms = lib.stage_timing(plan, prec, dev["L"], dev["W1"], dev["W2"], dev["R"], dev["psi"], out, wsa, reps=reps,
                              stream=stream)
        stage[name] = {k: round(v, 5) for k, v in ms.items()}
        for st in ("s1", "s3"):
            tf = info["flops_" + st] / (ms[st] * 1e-3) / 1e12
            roof[f"{st}_{name}"] = {"tflops": round(tf, 2), "frac": round(tf / PEAK[peak], 4)}
    del out, wsa
    return stage, roof


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)
    if args.workload == "j1j2-6x6":
        print(json.dumps(j1j2_bench(args)))
        return
    if args.workload in ("chain16", "hubbard-4x16"):
        print(json.dumps(sweeps_bench(args)))
        return
    if args.workload == "bond-m2048":
        print(json.dumps(large_bond_bench(args)))
        return
    if args.workload == "bond-m1024-stages":
        print(json.dumps(large_bond_bench(args, m=1024, k=14)))
        return
    import torch
    import synth
    from paper_2007_05540_amd import lib, problems

    spec = synth.c2_bond(m=1024, k=14, seed=1)
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    info = plan.info()
    flops = info["flops_s1"] + info["flops_s3"]
    dev = {k: torch.from_numpy(v).to("cuda") for k, v in ops.items()}
    del ops
    stream = torch.cuda.Stream()
    tiles = autotune(plan, info, dev, stream)
    solves = converged_solves(plan, info, dev, args, stream)
    mixed, f64 = solves["mixed"], solves["f64"]
    overlap = abs(float(torch.dot(mixed.pop("psi"), f64.pop("psi"))))
    rel_de = abs(mixed["energy"] - f64["energy"]) / abs(f64["energy"])

    # live per-kernel timing of one product (HIP events on the launch stream)
    stage, roofs = stage_roofline(plan, info, dev, stream)
    s32 = stage["f32_solve"]   # the FP32 kernels of the timed mixed solve
    dom = "s1" if s32["s1"] >= s32["s3"] else "s3"
    dom_flops = info["flops_" + dom]
    achieved = dom_flops / (s32[dom] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": f"ggemm {dom.upper()} FP32", "achieved": round(achieved, 3),
                "peak": PEAK["f32"], "unit": "TFLOP/s", "frac": round(achieved / PEAK["f32"], 4),
                "traffic": HBM_TRAFFIC[dom], "traffic_unit": "bytes per launch",
                "ms_per_launch": round(s32[dom], 5), "flops_per_launch": dom_flops}
    s64 = stage["f64"]
    dom64 = "s1" if s64["s1"] >= s64["s3"] else "s3"
    a64 = info["flops_" + dom64] / (s64[dom64] * 1e-3) / 1e12
    roofline_f64 = {"bound": "mfma", "kernel": f"ggemm {dom64.upper()} FP64", "achieved": round(a64, 3),
                    "peak": PEAK["f64"], "unit": "TFLOP/s", "frac": round(a64 / PEAK["f64"], 4),
                    "ms_per_launch": round(s64[dom64], 5), "flops_per_launch": info["flops_" + dom64]}

    ablation = dense_ablation(spec, plan, dev)
    line = {
        "metric": "block-sparse H_eff·ψ useful GFLOP/s & s/sweep: FP64 vs mixed+batched at 1e-9 dE",
        "value": round(mixed["gflops"], 3), "unit": "useful GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mixed["ms_per_solve"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-mfma products + f64 refinement",
        "data": "synthetic (seeded Heisenberg-type bond, Hermitian-structured random environments)",
        "config": {"workload": "isolated mid-chain two-site bond, 6x6 Heisenberg cylinder, m=1024, k=14, "
                               "21 U(1) sectors; one step = one Davidson solve to ||q|| <= %g" % args.tol,
                   "davidson": f"basis {args.basis}, thick restart to 2, FP32 phase to ||q|| <= {args.tol_f32:g}, "
                               f"residual checked every {args.check_every} products",
                   "useful_gflop_per_product": round(flops / 1e9, 4), "tiles": tiles},
        "f64_path": {"value": round(f64["gflops"], 3), "ms_per_step": round(f64["ms_per_solve"], 4),
                     "products": f64["products_f64"], "energy": f64["energy"], "residual": f64["residual"],
                     "converged": f64["converged"]},
        "mixed_path": {"products_f32": mixed["products_f32"], "products_f64": mixed["products_f64"],
                       "energy": mixed["energy"], "residual": mixed["residual"], "converged": mixed["converged"]},
        "equal_accuracy": {"energy_rel_diff": rel_de, "within_1e-9": bool(rel_de <= 1e-9),
                           "psi_error": 1.0 - overlap},
        "speedup_mixed_vs_f64": round(f64["ms_per_solve"] / mixed["ms_per_solve"], 3),
        "stage_ms": stage, "stage_roofline": roofs,
        "dense_format_ablation": ablation,
        "roofline": roofline, "roofline_f64": roofline_f64,
    }
    del dev
    plan.destroy()
    torch.cuda.empty_cache()
    if not args.no_large:
        line["bond_m2048_k18"] = large_bond_bench(args)
    if not args.no_batch:
        line["batch_64_bonds"] = batch_bench(args)
    if not args.no_hubbard:
        line["hubbard_bond_m4096"] = hubbard_bond_bench(args)
    if not args.no_sweeps:
        a2 = argparse.Namespace(**vars(args))
        a2.m_max = 512
        line["j1j2_6x6_m512_dE_dJ2"] = j1j2_bench(a2, with_fd=True)
        a3 = argparse.Namespace(**vars(args))
        a3.workload = "chain16"
        line["sweeps_chain16"] = sweeps_bench(a3)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec, flops, args.cpu_seconds)
    print(json.dumps(line))


def large_bond_bench(args, m=2048, k=18):
    """An isolated spin bond (by default m = 2048, k = 18: 25 sectors, the
    largest of the batch): per-stage times and MFMA rooflines of one product
    in both precisions."""
    import torch
    import synth
    from paper_2007_05540_amd import lib, problems
    spec = synth.c2_bond(m=m, k=k, seed=1)
    prob, ops = problems.bond_problem(spec)
    plan = lib.Plan([prob])
    info = plan.info()
    dev = {kk: torch.from_numpy(v).to("cuda") for kk, v in ops.items()}
    del ops
    stream = torch.cuda.Stream()
    stage, roofs = stage_roofline(plan, info, dev, stream)
    out = {"workload": f"isolated two-site bond, m={m}, k={k}, {len(spec.a_leg)} U(1) sectors",
           "useful_gflop_per_product": round((info["flops_s1"] + info["flops_s3"]) / 1e9, 3),
           "s3_split_k": info["s3_split_k"], "stage_ms": stage, "stage_roofline": roofs}
    del dev
    plan.destroy()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
