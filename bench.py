#!/usr/bin/env python3
"""Benchmark of the statically condensed GL-DGSEM implicit-step solve on one GPU.

One step = the whole hot path over one synthetic Newton system A dQ = B that is
already resident in device memory: batched inversion of the interior blocks,
X_e = A_ii^-1 A_ib and the element Schur blocks, condensed right-hand side,
GMRES(30) with point-Jacobi on the condensed system, back-substitution, and the
FP64 full-system residual that certifies ||B - A dQ|| / ||B|| <= 1e-8.

Workload (default): 8^3 periodic hex elements of order 5 (552 960 DOFs), a
Taylor-Green-like state at Ma 0.1, Re 1600, dt 5e-3, BR1 + local Lax-Friedrichs,
generated on the device by the seeded generator in workload/.

Prints ONE JSON line.  Per-kernel device times come from HIP events recorded
by the library on its stream during the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "hbm_gbs": 8000.0}


def progress(msg: str) -> None:
    """A progress line on stderr (never inside a timed region)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_work(case, plan_prec: str, n_rem: int) -> dict:
    """Algorithmic flops / bytes per launch of each kernel (unpadded element blocks).

    The condensed product S x streams the element blocks T_e once, the A_bb
    remainder blocks (values + column index) once, and reads x / writes y."""
    import numpy as np
    e = case.n_elem
    ni = np.broadcast_to(np.asarray(case.n_i, dtype=np.int64), (e,)).astype(np.float64)
    nc = np.broadcast_to(np.asarray(case.n_c, dtype=np.int64), (e,)).astype(np.float64)
    esz = 8 if plan_prec == "fp64" else 4
    nnzb = int(case.bb_rowptr[-1])
    n1, n2, ndof = case.n1, case.n2, case.n_dof
    bb_bytes = nnzb * 25 * 8 + nnzb * 4 + (case.n_bnodes + 1) * 8
    t = lambda a: float(np.sum(a))
    return {
        "inverse": {"flops": t(2 * ni ** 3), "bytes": t(ni * ni) * esz * 2},
        "gemm_x": {"flops": t(2 * ni * ni * nc), "bytes": t(ni * ni + 2 * ni * nc) * esz},
        "gemm_s": {"flops": t(2 * nc * nc * ni), "bytes": t(2 * ni * nc + nc * nc) * esz},
        "schur_apply": {"flops": t(2 * nc * nc) + n_rem * 50,
                        "bytes": t(nc * nc) * esz + n_rem * (25 * 8 + 4) + 2 * n1 * 8},
        "rhs": {"flops": t(2 * ni * ni + 2 * nc * ni),
                "bytes": t(ni * ni + nc * ni) * esz + (ndof + n1) * 8},
        "backsolve": {"flops": t(2 * ni * ni + 2 * ni * nc),
                      "bytes": t(ni * ni + ni * nc) * esz + (2 * ndof + n1) * 8},
        "residual": {"flops": t(2 * (ni * ni + 2 * ni * nc)) + nnzb * 50,
                     "bytes": t(ni * ni + 2 * ni * nc) * 8 + bb_bytes + 3 * ndof * 8},
    }


def assembled_s_node_blocks(case) -> int:
    """Node-block nonzeros of the assembled condensed matrix S: the union of the
    A_bb pattern and of every C_e x C_e block (the pattern S = A_bb -
    sum_e P_e A_bi A_ii^-1 A_ib P_e^T fills)."""
    import numpy as np
    nb = int(case.n_bnodes)
    keys = [np.repeat(np.arange(nb, dtype=np.int64), np.diff(case.bb_rowptr)) * nb + case.bb_col]
    for e in range(case.n_elem):
        c = case.c_node[case.c_ptr[e]:case.c_ptr[e + 1]].astype(np.int64)
        keys.append((c[:, None] * nb + c[None, :]).reshape(-1))
    return int(np.unique(np.concatenate(keys)).size)


def roofline_entry(name, work, phase, prec):
    if phase["count"] == 0 or phase["ms"] <= 0:
        return None
    per_launch_s = phase["ms"] / phase["count"] / 1e3
    if name in ("gemm_x", "gemm_s", "inverse"):
        peak = PEAK["fp64_mfma_tflops"] if prec == "fp64" else PEAK["fp32_mfma_tflops"]
        achieved = work["flops"] / per_launch_s / 1e12
        return {"kernel": name, "bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_ms": round(per_launch_s * 1e3, 4), "launches": phase["count"],
                "algorithmic_flops_per_launch": work["flops"]}
    achieved = work["bytes"] / per_launch_s / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK["hbm_gbs"],
            "unit": "GB/s", "frac": round(achieved / PEAK["hbm_gbs"], 4), "traffic": None,
            "avg_launch_ms": round(per_launch_s * 1e3, 4), "launches": phase["count"],
            "algorithmic_bytes_per_launch": work["bytes"]}


def dg_operator_timing(case, plan=None, calls: int = 20) -> dict:
    """Event-timed device residual R(Q) and Newton-matrix product A v
    (scdg_dg_residual, scdg_dg_jacobian_apply: lifts, the volume sums and the
    face fluxes once per face, on dual numbers for the product) at the state of
    the step, with a seeded direction.  Counters (rocprofv3, same workload)
    place them at neither roofline: ~1 TB/s of HBM traffic and the vector ALU
    active for about a third of the busy cycles, at two waves per SIMD (one
    512- or 256-thread workgroup per element, 512 elements): short kernels
    bound by latency at low occupancy.  The bytes below count one read of each
    input, one write of each output and the gradient workspace written once
    and read once."""
    import torch
    from paper_1911_02366_amd import DgResidual
    mesh, prm = case.mesh, case.prm
    q = case.q_state.to("cuda").reshape(-1).contiguous()
    gen = torch.Generator(device="cuda").manual_seed(7)
    v = torch.randn(q.shape, dtype=torch.float64, device="cuda", generator=gen)
    out = torch.empty_like(q)
    dg = DgResidual(mesh.k_elem, mesh.order, mach=prm.mach, reynolds=prm.reynolds)

    def timed(fn):
        for _ in range(3):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(calls):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / calls

    ms_r = timed(lambda: dg.residual(q, q, 1.0 / case.dt, out=out))
    ms_a = timed(lambda: dg.jacobian_apply(q, v, 1.0 / case.dt, out=out))
    blocks = None
    if plan is not None and getattr(case, "xyz", None) is None:
        # the element blocks of the Newton matrix formed by the library itself
        # (scdg_dg_jacobian_blocks; asynchronous after its first call with a
        # plan, host-timed up to a device synchronisation)
        import time
        dg.jacobian_blocks(plan, q, 1.0 / case.dt)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            blk = dg.jacobian_blocks(plan, q, 1.0 / case.dt)
        torch.cuda.synchronize()
        ms_b = (time.perf_counter() - t0) / reps * 1e3
        out_bytes = 8 * sum(blk[k].numel() for k in ("aii", "aib", "abi", "bb_val"))
        same = max(float((blk[k] - getattr(case, k).reshape(-1)).abs().max() /
                         getattr(case, k).abs().max()) for k in ("aii", "aib", "abi", "bb_val"))
        del blk
        blocks = {"ms": round(ms_b, 3), "output_gb": round(out_bytes / 1e9, 3),
                  "written_gbs": round(out_bytes / (ms_b / 1e3) / 1e9, 1),
                  "max_rel_diff_vs_generator": same}
    dg.close()
    nodes = q.numel() // 5
    bytes_r = nodes * 8 * (5 + 15 + 15 + 5 + 5 + 5)          # q (lift), g w/r, q, q_s, r
    bytes_a = nodes * 8 * (10 + 30 + 30 + 10 + 5)            # q, v (lifts), g and gd w/r, q, v, out
    return {"calls": calls, "residual_ms": round(ms_r, 4), "jacobian_apply_ms": round(ms_a, 4),
            "jacobian_apply_over_residual": round(ms_a / ms_r, 3),
            "residual_dof_s": round(q.numel() / (ms_r / 1e3), 1),
            "jacobian_apply_dof_s": round(q.numel() / (ms_a / 1e3), 1),
            "bound": "latency",
            "hbm_gbs": {"residual": round(bytes_r / (ms_r / 1e3) / 1e9, 1),
                        "jacobian_apply": round(bytes_a / (ms_a / 1e3) / 1e9, 1)},
            "jacobian_blocks": blocks}


def cpu_baseline(case, tol: float, max_seconds: float) -> dict:
    """The FP64 oracle, timed on the host on the step's own inputs (the blocks of
    the benchmark's system, copied from the device), with the paper's phase split
    (Tables Advantages / Advantages2):

      * condensed route, all host threads (`value`): once = LAPACK LU of every
        A_ii + element Schur blocks A_bi A_ii^-1 A_ib + diag(S)
        (oracle.condense_cpu); per step = condensed right-hand side + GMRES(30)
        with point Jacobi on S to the step's tolerance + back-substitution
        (oracle.condensed_gmres_solve) + the full FP64 residual from the blocks;
        value = DOFs / (once + per step);
      * the same on one thread, from a sample: the once-phase of the first
        elements and two Schur products, scaled to all elements and to the
        iteration count of the all-thread run;
      * uncondensed route, all threads: GMRES(30) on the global matrix with
        element-block Jacobi (oracle.solve_gmres_element_jacobi) to the same
        tolerance, iterations capped so that it stays within max_seconds; the
        global matrix's assembly from the blocks is reported, not counted."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = len(os.sched_getaffinity(0))
    t = lambda x: x.detach().cpu().numpy()
    args = (case.order, case.c_ptr, case.c_node, case.bb_rowptr, case.bb_col, t(case.bb_val),
            t(case.aii), t(case.aib), t(case.abi))
    b = t(case.rhs)
    bnorm = float(np.linalg.norm(b))
    progress(f"cpu baseline: condensed oracle route on {case.n_dof} DOFs, {threads} threads")
    t0 = time.perf_counter()
    cond = oracle.condense_cpu(*args)
    t1 = time.perf_counter()
    dq, iters, _ = oracle.condensed_gmres_solve(cond, b, tol=tol)
    r = oracle.full_residual_blocks(*args, b, dq)
    t2 = time.perf_counter()
    rel = float(np.linalg.norm(r) / bnorm)
    once, per_step = t1 - t0, t2 - t1
    value = case.n_dof / (once + per_step)
    legs = {"condensed_all_threads": {"once_s": round(once, 3), "per_step_s": round(per_step, 3),
                                      "gmres_iters": int(iters), "rel_res_full": rel,
                                      "dof_s": round(value, 1)}}
    if threadpool_limits is not None:
        with threadpool_limits(1):
            import scipy.linalg as sla
            n_s = min(case.n_elem, 16)
            aii, aib, abi = args[6], args[7], args[8]
            s0 = time.perf_counter()
            for e in range(n_s):
                lu = sla.lu_factor(aii[e])
                _ = abi[e] @ sla.lu_solve(lu, aib[e])
            once1 = (time.perf_counter() - s0) * case.n_elem / n_s
            x = np.random.default_rng(0).standard_normal(case.n1)
            s0 = time.perf_counter()
            for _ in range(2):
                oracle.schur_matvec_cpu(cond, x)
            mv1 = (time.perf_counter() - s0) / 2
        step1 = once1 + iters * mv1
        legs["condensed_1_thread_sampled"] = {
            "once_s": round(once1, 3), "schur_product_s": round(mv1, 4),
            "per_step_s_estimate": round(iters * mv1, 3), "dof_s": round(case.n_dof / step1, 1),
            "sample": f"once-phase of {n_s} of {case.n_elem} elements scaled, 2 Schur products x "
                      f"{iters} iterations (Gram-Schmidt, right-hand side and back-substitution left out)"}
    del cond
    progress("cpu baseline: uncondensed oracle route (GMRES on A, element-block Jacobi)")
    s0 = time.perf_counter()
    a = oracle.assemble_global(*args)
    asm = time.perf_counter() - s0
    s0 = time.perf_counter()
    _ = a @ b
    mv = time.perf_counter() - s0
    cap = max(5, int(max_seconds / max(3.0 * mv, 1e-3)))
    s0 = time.perf_counter()
    xa, it_a, rel_a = oracle.solve_gmres_element_jacobi(a, b, case.order, tol=tol, max_iter=cap)
    unc = time.perf_counter() - s0
    legs["uncondensed_all_threads"] = {
        "seconds": round(unc, 3), "gmres_iters": int(it_a), "iteration_cap": cap,
        "rel_res_A": float(rel_a), "converged": bool(rel_a <= tol),
        "dof_s": round(case.n_dof / unc, 1) if rel_a <= tol else None,
        "assembly_of_A_s_not_counted": round(asm, 3),
        "speedup_condensed_over_uncondensed": round(unc / (once + per_step), 3) if rel_a <= tol else None}
    del a
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(value, 1), "unit": "DOF/s", "cores": int(threads), "kind": "oracle",
            "sample": f"the whole step on the benchmark's own system ({case.n_dof} DOFs): oracle condensed "
                      f"route, once {once:.2f} s + per step {per_step:.2f} s ({iters} GMRES iterations "
                      f"to {tol:g} on S, full residual {rel:.1e})",
            "legs": legs, "cpu_model": model}


def learned_guess_experiment(args) -> dict:
    """Backward-Euler run with the learned initial guess (the Taylor-Green state of
    the workload, 16^3 elements of order 4 by default): steps 1..train collect
    (state, previous increment, increment) samples, the network is trained by the
    library's kernels, and every later step is solved three times from the same
    state -- zero guess, previous increment, network prediction -- to the same
    Newton tolerance; the run advances with the network's solution."""
    import numpy as np
    import torch
    from paper_1911_02366_amd.newton import ImplicitStepper, LearnedGuess
    from workload.cases import WORKLOADS, build_case, jacobian_blocks

    cfg = dict(WORKLOADS[args.lg_workload])
    if args.lg_k:
        cfg["k_elem"] = args.lg_k
    case = build_case(device="cuda", **cfg)
    mesh, prm, dt = case.mesh, case.prm, case.dt
    st = ImplicitStepper(case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt,
                         lambda q: jacobian_blocks(q, mesh, prm, dt), lin_tol=args.lg_lin_tol,
                         newton_tol=args.lg_newton_tol)
    st32 = ImplicitStepper(case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt,
                           lambda q: jacobian_blocks(q, mesh, prm, dt), lin_tol=args.lg_lin_tol,
                           newton_tol=args.lg_newton_tol, precision="fp32", graph=True)
    n_elem, dpe = mesh.n_elem, 5 * mesh.p ** 3
    lg = LearnedGuess(n_elem, dpe, capacity=args.lg_train, seed=args.lg_seed, batch=args.lg_batch)
    # the same network with the step's right-hand side R(Q_s) as a third input block
    lgr = LearnedGuess(n_elem, dpe, capacity=args.lg_train, seed=args.lg_seed, batch=args.lg_batch,
                       use_residual=True)
    # the same network trained on the step's first Newton correction (the solution
    # of the first linear system, which the GMRES x0 seeds) instead of the step increment
    lg1 = LearnedGuess(n_elem, dpe, capacity=args.lg_train, seed=args.lg_seed, batch=args.lg_batch)
    rc_prev1 = None
    inv_dt = 1.0 / dt
    q = case.q_state.reshape(-1).contiguous()
    dq_prev = torch.zeros_like(q)
    rc_prev = None
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    t_collect = time.perf_counter()
    for step in range(1, args.lg_train + 1):
        st.prepare(q)
        r_s = st.dg.residual(q, q, inv_dt)
        q1, info = st.solve_step(q, guess=dq_prev if step > 1 else None, keep_first=True)
        if not info["converged"]:
            raise RuntimeError(f"step {step} did not converge: {info}")
        dq = q1 - q
        if step > 1:
            lg.record(q, dq_prev, dq)
            lgr.record(q, dq_prev, dq, r_s)
            lg1.record(q, dq_prev, info["first_dq"])
            rc_prev = lg.correction_rms(q, dq_prev, dq)
            rc_prev1 = lg1.correction_rms(q, dq_prev, info["first_dq"])
        q, dq_prev = q1, dq
        log(f"train-phase step {step}: newton {info['newton']} gmres {info['gmres']}")
    t_collect = time.perf_counter() - t_collect
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history, hold = lg.train(epochs=args.lg_epochs, lr=args.lg_lr, holdout_rows=n_elem)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    hold_zero = lg.loss_on(lg.count - n_elem, lg.count, zero=True)
    # the same network trained with bfloat16 matrix products on the same samples
    lg16 = LearnedGuess(n_elem, dpe, capacity=args.lg_train, seed=args.lg_seed, batch=args.lg_batch,
                        compute="bf16")
    lg16.copy_samples(lg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history16, hold16 = lg16.train(epochs=args.lg_epochs, lr=args.lg_lr, holdout_rows=n_elem)
    torch.cuda.synchronize()
    t_train16 = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history_r, hold_r = lgr.train(epochs=args.lg_epochs, lr=args.lg_lr, holdout_rows=n_elem)
    torch.cuda.synchronize()
    t_train_r = time.perf_counter() - t0
    log(f"residual-input network: loss {history_r[0]:.3e} -> {history_r[-1]:.3e}, hold-out {hold_r:.3e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history_1, hold_1 = lg1.train(epochs=args.lg_epochs, lr=args.lg_lr, holdout_rows=n_elem)
    torch.cuda.synchronize()
    t_train_1 = time.perf_counter() - t0
    log(f"first-correction network: loss {history_1[0]:.3e} -> {history_1[-1]:.3e}, hold-out {hold_1:.3e} "
        f"(alpha {lg1.alpha:.3f})")
    # the same network trained on the condensed residual its guess leaves (S of the
    # last training step weighting every stored step), on the same samples
    lgs = LearnedGuess(n_elem, dpe, capacity=args.lg_train, seed=args.lg_seed, batch=args.lg_batch)
    lgs.copy_samples(lg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    history_s, hold_s = lgs.train_condensed(st.plan, epochs=args.lg_condensed_epochs, lr=args.lg_lr)
    torch.cuda.synchronize()
    t_train_s = time.perf_counter() - t0
    last = lg.count // n_elem - 1
    hold_s_mse = lg.condensed_loss_on(st.plan, last)
    log(f"condensed-loss network: loss {history_s[0]:.3e} -> {history_s[-1]:.3e}, hold-out {hold_s:.3e} "
        f"(alpha {lgs.alpha:.3f}); mean-squared network on that measure {hold_s_mse:.3e}")
    log(f"trained {args.lg_epochs} epochs in {t_train:.1f} s: loss {history[0]:.3e} -> {history[-1]:.3e}, "
        f"hold-out {hold:.3e} (previous increment: {hold_zero:.3e})")
    variants = [("zero", "gmres"), ("previous", "gmres"), ("learned", "gmres"), ("learned_s", "gmres"),
                ("learned_first", "gmres"),
                ("previous_newton_start", "newton"), ("learned_newton_start", "newton"),
                ("learned_bf16_newton_start", "newton"), ("learned_r_newton_start", "newton"),
                ("fp32_ir_zero", "gmres"), ("fp32_ir_previous_newton_start", "newton"),
                ("fp32_ir_learned_newton_start", "newton"),
                ("fp32_graph_previous_newton_start", "newton"), ("fp32_graph_learned_newton_start", "newton"),
                ("fp32_graph_learned_r_newton_start", "newton")]
    names = [v for v, _ in variants]
    rec = {k: {"first": [], "total": [], "newton": [], "seconds": [], "guess_res": [], "rejected": []}
           for k in names}
    infer_ms, infer16_ms, infer_r_ms, infer_s_ms, infer_1_ms = [], [], [], [], []
    prep = {"fp64": [], "fp32": []}
    for step in range(args.lg_train + 1, args.lg_steps + 1):
        prep["fp64"].append(st.prepare(q))
        prep["fp32"].append(st32.prepare(q, blocks=st._blocks))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pred = lg.predict(q, dq_prev, rc_prev)
        torch.cuda.synchronize()
        infer_ms.append((time.perf_counter() - t1) * 1e3)
        t1 = time.perf_counter()
        pred16 = lg16.predict(q, dq_prev, rc_prev)
        torch.cuda.synchronize()
        infer16_ms.append((time.perf_counter() - t1) * 1e3)
        t1 = time.perf_counter()
        pred_r = lgr.predict(q, dq_prev, rc_prev, st.dg.residual(q, q, inv_dt))
        torch.cuda.synchronize()
        infer_r_ms.append((time.perf_counter() - t1) * 1e3)
        t1 = time.perf_counter()
        pred_s = lgs.predict(q, dq_prev, rc_prev)
        torch.cuda.synchronize()
        infer_s_ms.append((time.perf_counter() - t1) * 1e3)
        t1 = time.perf_counter()
        pred_1 = lg1.predict(q, dq_prev, rc_prev1)
        torch.cuda.synchronize()
        infer_1_ms.append((time.perf_counter() - t1) * 1e3)
        out = {}
        first_zero = None
        for name, mode in variants:
            g = None if name.endswith("zero") else (dq_prev if "previous" in name else
                                                    (pred16 if "bf16" in name else
                                                     (pred_r if "learned_r" in name else
                                                      (pred_s if name == "learned_s" else
                                                       (pred_1 if name == "learned_first" else pred)))))
            q1, info = (st32 if name.startswith("fp32") else st).solve_step(q, guess=g, mode=mode,
                                                                            graph="graph" in name,
                                                                            keep_first=name == "zero")
            if name == "zero":
                first_zero = info["first_dq"]
            if not info["converged"]:
                raise RuntimeError(f"step {step} ({name}) did not converge: {info}")
            r = rec[name]
            r["first"].append(info["first_gmres"])
            r["total"].append(info["gmres"])
            r["newton"].append(info["newton"])
            infer = (infer16_ms[-1] if "bf16" in name else
                     (infer_r_ms[-1] if "learned_r" in name else
                      (infer_s_ms[-1] if name == "learned_s" else
                       (infer_1_ms[-1] if name == "learned_first" else infer_ms[-1]))))
            r["seconds"].append(info["seconds"] + (infer * 1e-3 if "learned" in name else 0.0))
            r["guess_res"].append(info["guess_res"])
            r["rejected"].append(info["guess_rejected"])
            out[name] = q1
        log(f"step {step}: GMRES per step " + " ".join(f"{k} {rec[k]['total'][-1]}" for k in names))
        dq = out["zero"] - q
        rc_prev = lg.correction_rms(q, dq_prev, dq)
        rc_prev1 = lg1.correction_rms(q, dq_prev, first_zero)
        dq_prev = dq
        q = out["zero"]
    mean = lambda v: float(np.mean(v))
    result = {
        "experiment": "learned_initial_guess", "workload": args.lg_workload, "k_elem": mesh.k_elem,
        "order": mesh.order, "dofs": mesh.n_dof,
        "steps": args.lg_steps, "train_steps": f"2-{args.lg_train}",
        "test_steps": f"{args.lg_train + 1}-{args.lg_steps}",
        "newton_tol": args.lg_newton_tol, "gmres_tol": args.lg_lin_tol,
        "network": f"{2 * dpe}-256-256-{dpe} tanh, FP32, {lg.net.n_params} parameters",
        "train": {"samples": lg.count - n_elem, "epochs": args.lg_epochs, "batch": args.lg_batch,
                  "lr": args.lg_lr, "seconds": t_train, "loss_first_epoch": history[0],
                  "loss_last_epoch": history[-1], "holdout_loss": hold,
                  "holdout_loss_previous_increment": hold_zero, "alpha": lg.alpha,
                  "collect_seconds": t_collect},
        "train_bf16": {"seconds": t_train16, "loss_first_epoch": history16[0], "loss_last_epoch": history16[-1],
                       "holdout_loss": hold16, "alpha": lg16.alpha},
        "inference_ms_mean": mean(infer_ms),
        "inference_bf16_ms_mean": mean(infer16_ms),
        "train_residual_input": {"seconds": t_train_r, "loss_first_epoch": history_r[0],
                                 "loss_last_epoch": history_r[-1], "holdout_loss": hold_r, "alpha": lgr.alpha,
                                 "network": f"{3 * dpe}-256-256-{dpe} tanh, FP32, {lgr.net.n_params} parameters"},
        "inference_residual_input_ms_mean": mean(infer_r_ms),
        "train_condensed": {"seconds": t_train_s, "epochs": args.lg_condensed_epochs,
                            "batch": f"one step ({n_elem} elements)", "lr": args.lg_lr,
                            "loss_first_epoch": history_s[0], "loss_last_epoch": history_s[-1],
                            "holdout_condensed_loss": hold_s, "alpha": lgs.alpha,
                            "holdout_condensed_loss_mse_network": hold_s_mse,
                            "holdout_condensed_loss_previous_increment": 1.0,
                            "weighting": "S of the last training step for every stored step"},
        "inference_condensed_ms_mean": mean(infer_s_ms),
        "train_first_correction": {"seconds": t_train_1, "loss_first_epoch": history_1[0],
                                   "loss_last_epoch": history_1[-1], "holdout_loss": hold_1, "alpha": lg1.alpha,
                                   "target": "first Newton correction of the step (first linear solve's solution)"},
        "inference_first_correction_ms_mean": mean(infer_1_ms),
        "guess_rejected": {k: int(np.sum(rec[k]["rejected"])) for k in names},
        "forcing": "GMRES tol per Newton iteration = clip(0.5 newton_tol |R0| / |R|, gmres_tol, 0.1)",
    }
    for key, field in (("first_solve_gmres_mean", "first"), ("gmres_per_step_mean", "total"),
                       ("newton_per_step_mean", "newton"), ("solve_seconds_per_step_mean", "seconds"),
                       ("guess_rel_residual_median", "guess_res")):
        agg = np.median if field == "guess_res" else np.mean
        result[key] = {k: float(agg(rec[k][field])) for k in names}
    # an implicit step = factor + condense (at the step's Jacobian) + the Newton solve
    pm = {p: float(np.mean(v[1:] if len(v) > 1 else v)) for p, v in prep.items()}   # first call autotunes
    result["factor_condense_seconds_per_step"] = pm
    result["step_seconds_mean"] = {k: result["solve_seconds_per_step_mean"][k] +
                                   pm["fp32" if k.startswith("fp32") else "fp64"] for k in names}
    z = result["step_seconds_mean"]["zero"]
    result["time_to_solution_vs_plain_fp64"] = {k: z / result["step_seconds_mean"][k] for k in names}
    lg.close()
    lg16.close()
    lgr.close()
    lgs.close()
    lg1.close()
    st.close()
    st32.close()
    return result


def time_stepping_experiment(args) -> dict:
    """Backward-Euler steps of the Taylor-Green workload with the Newton loop
    driven from the host (one library call per linear solve, norms read back)
    and with every Newton iteration replayed from the library's captured graph
    (scdg_newton_step), in FP64 and with FP32 factors.  Every variant solves
    each step from the same state, with the previous increment as the Newton
    starting state, to the same Newton tolerance; the run advances with the
    host FP64 solution."""
    import numpy as np
    import torch
    from paper_1911_02366_amd.newton import ImplicitStepper
    from workload.cases import WORKLOADS, build_case, jacobian_blocks

    case = build_case(device="cuda", **WORKLOADS[args.ts_workload])
    mesh, prm, dt = case.mesh, case.prm, case.dt
    mk = lambda prec, sm="assembled": ImplicitStepper(
        case.structure(), mesh.k_elem, mesh.order, prm.mach, prm.reynolds, dt,
        lambda q: jacobian_blocks(q, mesh, prm, dt), lin_tol=args.lg_lin_tol, newton_tol=args.lg_newton_tol,
        precision=prec, graph=True, schur_mode=sm)
    # the *_mf steppers apply S through X_e, A_bi and A_bb (T_e never formed), the *_mfs
    # steppers through the nonzero blocks of A_ib and A_bi and A_ii^-1
    steppers = {"fp64": mk("fp64"), "fp32": mk("fp32"), "fp64_mf": mk("fp64", "matrix_free"),
                "fp32_mf": mk("fp32", "matrix_free"), "fp64_mfs": mk("fp64", "matrix_free_sparse"),
                "fp32_mfs": mk("fp32", "matrix_free_sparse")}
    variants = [("host_fp64", "fp64", False), ("graph_fp64", "fp64", True),
                ("host_fp32", "fp32", False), ("graph_fp32", "fp32", True),
                ("graph_fp64_mf", "fp64_mf", True), ("graph_fp32_mf", "fp32_mf", True),
                ("graph_fp64_mfs", "fp64_mfs", True), ("graph_fp32_mfs", "fp32_mfs", True)]
    rec = {v: {"seconds": [], "newton": [], "gmres": [], "lin_unconverged": []} for v, _, _ in variants}
    prep = {k: [] for k in steppers}
    diff = {v: [] for v, _, _ in variants if v != "host_fp64"}
    q = case.q_state.reshape(-1).contiguous()
    dq_prev = None
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    for step in range(1, args.ts_steps + 1):
        prep["fp64"].append(steppers["fp64"].prepare(q))
        for k in ("fp32", "fp64_mf", "fp32_mf", "fp64_mfs", "fp32_mfs"):
            prep[k].append(steppers[k].prepare(q, blocks=steppers["fp64"]._blocks))
        out = {}
        for name, prec, graph in variants:
            q1, info = steppers[prec].solve_step(q, guess=dq_prev, mode="newton", graph=graph)
            if not info["converged"]:
                raise RuntimeError(f"step {step} ({name}) did not converge: {info}")
            r = rec[name]
            r["seconds"].append(info["seconds"])
            r["newton"].append(info["newton"])
            r["gmres"].append(info["gmres"])
            r["lin_unconverged"].append(info.get("lin_unconverged", 0))
            out[name] = q1
        ref = out["host_fp64"] - q
        for k in diff:
            diff[k].append(float((out[k] - q - ref).norm() / ref.norm()))
        log(f"step {step}: " + " ".join(f"{k} {rec[k]['seconds'][-1] * 1e3:.1f} ms/{rec[k]['gmres'][-1]} it"
                                        for k in rec))
        dq_prev = ref
        q = out["host_fp64"]
    mean = lambda v: float(np.mean(v[1:] if len(v) > 1 else v))    # the first step captures / autotunes
    names = [v for v, _, _ in variants]
    pm = {p: mean(v) for p, v in prep.items()}
    result = {
        "experiment": "newton_graph_time_stepping", "workload": args.ts_workload, "k_elem": mesh.k_elem,
        "order": mesh.order, "dofs": mesh.n_dof, "steps": args.ts_steps, "newton_tol": args.lg_newton_tol,
        "gmres_tol": args.lg_lin_tol, "graph_cycles": steppers["fp64"].graph_cycles,
        "newton_start": "previous increment (zero at step 1)",
        "factor_condense_seconds_per_step": pm,
        "solve_seconds_per_step_mean": {k: mean(rec[k]["seconds"]) for k in names},
        "newton_per_step_mean": {k: float(np.mean(rec[k]["newton"])) for k in names},
        "gmres_per_step_mean": {k: float(np.mean(rec[k]["gmres"])) for k in names},
        "lin_unconverged_total": {k: int(np.sum(rec[k]["lin_unconverged"])) for k in names},
        "max_rel_diff_vs_host_fp64_increment": {k: float(np.max(v)) for k, v in diff.items()},
    }
    which = {v: st for v, st, _ in variants}
    result["step_seconds_mean"] = {k: result["solve_seconds_per_step_mean"][k] + pm[which[k]] for k in names}
    z = result["step_seconds_mean"]["host_fp64"]
    result["speedup_vs_host_fp64"] = {k: z / result["step_seconds_mean"][k] for k in names}
    for s_ in steppers.values():
        s_.close()
    return result


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tgv_n5_k8")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=30, help="GMRES restart length (1..63)")
    ap.add_argument("--krylov-mode", choices=["host", "device", "graph"], default="host",
                    help="where the GMRES cycle runs (the phase timers do not see kernels inside a graph)")
    ap.add_argument("--precond", type=int, default=1, choices=[0, 1, 2],
                    help="GMRES right preconditioner: 0 none, 1 point Jacobi, 2 5x5 node-block Jacobi")
    ap.add_argument("--cpu-seconds", type=float, default=60.0,
                    help="time cap of the oracle's uncondensed GMRES leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the measured MFMA / HBM ceilings")
    ap.add_argument("--no-dg-timing", action="store_true",
                    help="skip the timing of the device residual and Newton-matrix product")
    ap.add_argument("--fp32-inner-tol", type=float, default=1e-4,
                    help="GMRES tolerance inside each refinement sweep of the FP32 variant")
    ap.add_argument("--fp32-sweep", type=float, nargs="*", default=[],
                    help="extra inner tolerances to time for the FP32 variant")
    ap.add_argument("--no-fp32-variant", action="store_true")
    ap.add_argument("--no-matrix-free-variant", action="store_true",
                    help="skip the FP64 variant with matrix-free Schur products")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 2 GiB FP64 buffer three times (HBM counter calibration)")
    ap.add_argument("--inverse-mode", choices=["auto", "single", "blocked", "resident"], default="auto",
                    help="form of the batched inverse (auto: resident panel up to n_i = 352, blocked above 320 "
                         "otherwise)")
    ap.add_argument("--learned-guess", action="store_true",
                    help="run the learned-initial-guess time-stepping experiment instead")
    ap.add_argument("--lg-workload", default="tgv_n4_k16")
    ap.add_argument("--lg-k", type=int, default=0, help="override the elements per direction")
    ap.add_argument("--lg-steps", type=int, default=200)
    ap.add_argument("--lg-train", type=int, default=50)
    ap.add_argument("--lg-epochs", type=int, default=20)
    ap.add_argument("--lg-condensed-epochs", type=int, default=40,
                    help="epochs of the network trained on the condensed residual (one step per batch)")
    ap.add_argument("--lg-batch", type=int, default=1024)
    ap.add_argument("--lg-lr", type=float, default=1e-3)
    ap.add_argument("--lg-seed", type=int, default=0)
    ap.add_argument("--lg-lin-tol", type=float, default=1e-10)
    ap.add_argument("--lg-newton-tol", type=float, default=1e-8)
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON file of tile choices per problem signature (default: $SCDG_AUTOTUNE_CACHE)")
    ap.add_argument("--wall-batch", type=int, default=96,
                    help="complex-step directions per residual evaluation when generating a wall workload")
    ap.add_argument("--time-stepping", action="store_true",
                    help="host-driven vs graph-replayed Newton iterations over implicit steps")
    ap.add_argument("--ts-workload", default="tgv_n4_k16")
    ap.add_argument("--ts-steps", type=int, default=8)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(one plan per GPU, element-partitioned); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.learned_guess:
        print(json.dumps(learned_guess_experiment(args)), flush=True)
        return 0
    if args.time_stepping:
        print(json.dumps(time_stepping_experiment(args)), flush=True)
        return 0
    if args.calibrate_copy:
        n = (2 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))
        return 0

    from paper_1911_02366_amd import Plan
    from workload.cases import WORKLOADS, named_case
    from workload.mixed import MIXED_WORKLOADS, mixed_order_case

    from workload.walls import WALL_WORKLOADS, build_wall_case

    dev = "cuda"
    wall = args.workload in WALL_WORKLOADS
    if wall:
        wcfg = WALL_WORKLOADS[args.workload]
        t_gen = time.perf_counter()
        case = build_wall_case(device=dev, seed=0, max_batch=args.wall_batch,
                               progress=lambda c, n: progress(f"wall Jacobian: colour {c + 1} of {n}")
                               if c % 4 == 0 else None, **wcfg)
        torch.cuda.synchronize()
        progress(f"wall workload generated in {time.perf_counter() - t_gen:.1f} s")
        k_w, n_w = wcfg["k_elem"], wcfg["order"]
        cfg = dict(wcfg)
        cfg["walls"] = ("isothermal no-slip walls on the two faces normal to z (Section 2.1.1 outer state), "
                        "wall-face DOFs in Q_i")
        cfg["condensed_ratio"] = round(case.n1 / case.n_dof, 6)
        cfg["condensed_ratio_without_walls"] = round(((n_w + 1) ** 3 - (n_w - 1) ** 3) / (n_w + 1) ** 3, 6)
    elif args.workload in MIXED_WORKLOADS:
        k_m, lo_m, hi_m, seed_m = MIXED_WORKLOADS[args.workload]
        case = mixed_order_case(k_m, lo_m, hi_m, seed_m, device=dev)
        cfg = {"order": f"{lo_m}..{hi_m} (seeded per element)", "reynolds": None, "dt": None,
               "values": "synthetic, strictly diagonally dominant"}
    else:
        case = named_case(args.workload, device=dev)
        cfg = dict(WORKLOADS[args.workload])
    torch.cuda.synchronize()
    b = case.rhs
    plan = Plan.from_structure(case.structure())
    plan.set_inverse_mode(args.inverse_mode)
    plan.set_krylov_mode(args.krylov_mode)
    plan.assemble(case.aii, case.aib, case.abi, case.bb_val)
    dq = torch.empty(case.n_dof, dtype=torch.float64, device=dev)

    def measure(precision, tol, steps, warmup):
        opts = dict(solver="gmres", restart=args.restart, tol=tol, ir_tol=1e-8, ir_max=10, precond=args.precond)

        def step():
            plan.factor(precision)
            plan.condense()
            _, info = plan.solve(b, dq, **opts)
            return info

        plan.factor(precision)
        tuning = plan.autotune(cache=args.autotune_cache)
        progress(f"{precision}: tiles x {tuning['x']} s {tuning['s']}"
                 f"{' (from cache)' if tuning['cached'] else ''}")
        for i in range(warmup):
            step()
            torch.cuda.synchronize()
            progress(f"{precision}: warm-up step {i + 1} of {warmup}")
        torch.cuda.synchronize()
        plan.enable_timing(True)
        plan.phase_times()
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(step())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        progress(f"{precision}: {steps} timed steps, {(t1 - t0) / steps * 1e3:.2f} ms each")
        phases = plan.phase_times()
        plan.enable_timing(False)
        return (t1 - t0) / steps * 1e3, infos, phases, tuning, opts

    fp32_tol = args.fp32_inner_tol
    ms_per_step, infos, phases, tuning, opts = measure(
        args.precision, args.tol if args.precision == "fp64" else fp32_tol, args.steps, args.warmup)
    variants = {}
    if args.precision == "fp64" and not args.no_fp32_variant:
        for tol in sorted(set([fp32_tol] + args.fp32_sweep)):
            ms32, inf32, ph32, tun32, _ = measure("fp32", tol, args.steps, args.warmup)
            variants[f"fp32_ir_inner_tol_{tol:g}"] = {
                "ms_per_step": round(ms32, 3), "value_dof_s": round(case.n_dof / (ms32 / 1e3), 1),
                "speedup_vs_fp64": round(ms_per_step / ms32, 3),
                "rel_res_full_max": max(i["rel_res_full"] for i in inf32),
                "gmres_iters_per_step": sum(i["iters"] for i in inf32) / len(inf32),
                "ir_sweeps_per_step": sum(i["ir_sweeps"] for i in inf32) / len(inf32),
                "phase_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in ph32.items()},
                "gemm_tiles": {"x": tun32["x"], "s": tun32["s"]}}
    if args.precision == "fp64" and not args.no_matrix_free_variant:
        # Schur products without T_e: through X_e, A_bi and the full A_bb (matrix_free), or
        # through the nonzero 5x5 blocks of A_ib and A_bi and A_ii^-1 (matrix_free_sparse)
        import numpy as np
        nb_e = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), (case.n_elem,))
        nix = float(np.sum(nb_e(case.n_i) * nb_e(case.n_c)))
        nii = float(np.sum(nb_e(case.n_i) ** 2))
        nnzb = int(case.bb_rowptr[-1])
        nz_blocks = None
        if case.aib.dim() == 3:                  # uniform order: count the nonzero blocks
            ne_, ni_, nc_ = case.aib.shape
            nzb = lambda m, r, c: int((m.reshape(ne_, r // 5, 5, c // 5, 5).abs().amax(dim=(2, 4)) > 0).sum())
            nz_blocks = nzb(case.aib, ni_, nc_) + nzb(case.abi, nc_, ni_)
        vec_bytes = 2 * case.n1 * 8 + 2 * (case.n2 + 5 * case.n_bnodes) * 8
        for smode in ("matrix_free", "matrix_free_sparse"):
            plan.set_schur_mode(smode)
            for prec, tol in (("fp64", args.tol), ("fp32", fp32_tol)):
                esz = 8 if prec == "fp64" else 4
                ms_mf, inf_mf, ph_mf, _, _ = measure(prec, tol, args.steps, args.warmup)
                sa = ph_mf.get("schur_apply", {"ms": 0.0, "count": 0})
                per_launch = sa["ms"] / max(sa["count"], 1)
                if smode == "matrix_free":
                    # X_e and A_bi(e) dense in the factor precision, all of A_bb, vectors
                    mf_bytes = 2 * nix * esz + nnzb * (25 * 8 + 4) + vec_bytes
                elif nz_blocks is not None:
                    # nonzero blocks of A_ib and A_bi (values + node index), A_ii^-1, A_bb, vectors
                    mf_bytes = nz_blocks * (25 * esz + 4) + nii * esz + nnzb * (25 * 8 + 4) + vec_bytes
                else:
                    mf_bytes = None
                variants[f"{smode}_{prec}" + ("" if prec == "fp64" else f"_ir_inner_tol_{tol:g}")] = {
                    "ms_per_step": round(ms_mf, 3), "value_dof_s": round(case.n_dof / (ms_mf / 1e3), 1),
                    "speedup_vs_assembled_fp64": round(ms_per_step / ms_mf, 3),
                    "rel_res_full_max": max(i["rel_res_full"] for i in inf_mf),
                    "gmres_iters_per_step": sum(i["iters"] for i in inf_mf) / len(inf_mf),
                    "ir_sweeps_per_step": sum(i["ir_sweeps"] for i in inf_mf) / len(inf_mf),
                    "schur_apply_ms_per_launch": round(per_launch, 4),
                    "schur_apply_algorithmic_bytes": mf_bytes,
                    "schur_apply_gbs": round(mf_bytes / (per_launch / 1e3) / 1e9, 1)
                    if per_launch > 0 and mf_bytes else None,
                    "phase_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in ph_mf.items()}}
        plan.set_schur_mode("assembled")
    value = case.n_dof / (ms_per_step / 1e3)
    work = algorithmic_work(case, args.precision, plan.n_remainder)
    kernels = {k: v for k, v in phases.items() if k in work}
    dominant = max(kernels, key=lambda k: kernels[k]["ms"])
    entries = {k: roofline_entry(k, work[k], kernels[k], args.precision) for k in kernels}
    if entries.get("schur_apply") is not None:
        # Algorithmic bytes of one product S x: the values of the assembled S (its
        # node-block nonzeros x 25 in the factor precision), the minimum any storage
        # of the operator reads.  The library's element-block storage (T_e plus the
        # A_bb remainder, vectors) reads more where coupling sets overlap; its
        # count and rate are kept beside.
        e = entries["schur_apply"]
        s_bytes = float(assembled_s_node_blocks(case) * 25 * (8 if args.precision == "fp64" else 4))
        per_launch_s = e["avg_launch_ms"] / 1e3
        e["element_block_bytes_per_launch"] = e.pop("algorithmic_bytes_per_launch")
        e["element_block_achieved"] = e["achieved"]
        e["element_block_frac"] = e["frac"]
        e["algorithmic_bytes_per_launch"] = s_bytes
        e["algorithmic_bytes"] = "values of the assembled S: node-block nonzeros x 25 x element size"
        e["achieved"] = round(s_bytes / per_launch_s / 1e9, 1)
        e["frac"] = round(e["achieved"] / PEAK["hbm_gbs"], 4)
    # the three factor/condense kernels together, against the FP64 (or FP32) matrix-core peak:
    # LU-equivalent flops (2/3) n_i^3 + 2 n_i^2 n_c + 2 n_c^2 n_i per element over their summed time
    fc_keys = ("inverse", "gemm_x", "gemm_s")
    if all(entries.get(k) for k in fc_keys):
        fc_ms = sum(entries[k]["avg_launch_ms"] for k in fc_keys)
        fc_flops = work["inverse"]["flops"] / 3.0 + work["gemm_x"]["flops"] + work["gemm_s"]["flops"]
        peak = PEAK["fp64_mfma_tflops"] if args.precision == "fp64" else PEAK["fp32_mfma_tflops"]
        ach = fc_flops / (fc_ms / 1e3) / 1e12
        entries["factor_condense"] = {"kernel": "factor_condense (inverse + gemm_x + gemm_s)", "bound": "mfma",
                                      "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                                      "frac": round(ach / peak, 4), "traffic": None, "avg_launch_ms": round(fc_ms, 4),
                                      "launches": entries["inverse"]["launches"],
                                      "algorithmic_flops_per_launch": fc_flops,
                                      "flop_count": "LU-equivalent: (2/3) n_i^3 + 2 n_i^2 n_c + 2 n_c^2 n_i per element"}
    from paper_1911_02366_amd.profiling import load_traffic
    csrc = os.path.join(ROOT, "paper_1911_02366_amd", "csrc")
    for k, srcs in (("schur_apply", ["k_vec.hip"]), ("gemm_s", ["k_gemm.hip"]), ("gemm_x", ["k_gemm.hip"]),
                    ("inverse", ["k_inverse.hip"])):
        rec = load_traffic(os.path.join(ROOT, "profiles", f"traffic_{k}_{args.workload}_{args.precision}.json"),
                           [os.path.join(csrc, f) for f in srcs])
        if entries.get(k) is not None and rec is not None:
            entries[k]["traffic"] = rec["traffic_bytes_per_launch"]
    measured = None
    if not args.no_probe:
        # measured ceilings beside the vendor peaks (context; `frac` stays against the vendor figure)
        from paper_1911_02366_amd import probe
        measured = {"fp64_mfma_tflops": round(probe.mfma_tflops("fp64"), 2),
                    "fp32_mfma_tflops": round(probe.mfma_tflops("fp32"), 2),
                    "hbm_read_gbs": round(probe.hbm_read_gbs(4 << 30), 1),
                    "how": "scdg_probe_mfma: back-to-back 16x16x4 MFMAs on register operands, "
                           "8 workgroups of 4 waves per CU; scdg_probe_hbm_read: 16-byte nontemporal "
                           "streaming read of a 4 GiB buffer; best of 3 / 5 launches"}
        progress(f"measured ceilings: {measured['fp64_mfma_tflops']} TF/s FP64 MFMA, "
                 f"{measured['fp32_mfma_tflops']} TF/s FP32 MFMA, {measured['hbm_read_gbs']} GB/s read")
        for e in entries.values():
            if e is None:
                continue
            if e["bound"] == "mfma":
                m = measured["fp64_mfma_tflops" if args.precision == "fp64" else "fp32_mfma_tflops"]
            else:
                m = measured["hbm_read_gbs"]
            e["peak_measured"] = m
            e["frac_of_measured"] = round(e["achieved"] / m, 4)
    worst = max(i["rel_res_full"] for i in infos)
    out = {
        "metric": "condensed implicit-step DOF/s at 1e-8 residual",
        "value": round(value, 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "elements": case.n_elem, "order": cfg["order"],
                   "dofs": case.n_dof, "n1_condensed": case.n1, "n2_interior": case.n2,
                   "reynolds": cfg["reynolds"], "mach": 0.1 if cfg["reynolds"] else None, "dt": cfg["dt"],
                   "solver": f"gmres({args.restart})+" + ["none", "point-jacobi", "block-jacobi-5x5"][args.precond],
                   "gmres_tol": opts["tol"],
                   "precision": args.precision, "krylov_mode": args.krylov_mode,
                   **({k: cfg[k] for k in ("walls", "condensed_ratio", "condensed_ratio_without_walls")}
                      if wall else {})},
        "roofline": entries[dominant],
        "roofline_all": entries,
        "measured_peaks": measured,
        "phase_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in phases.items()},
        "rel_res_full_max": worst,
        "variants": variants,
        "gemm_tiles": {"x": tuning["x"], "s": tuning["s"], "from_cache": tuning["cached"],
                       "autotune_ms_s": {k: round(v, 3) for k, v in tuning.get("ms_s", {}).items()},
                       "autotune_ms_x": {k: round(v, 3) for k, v in tuning.get("ms_x", {}).items()}},
        "gmres_iters_per_step": sum(i["iters"] for i in infos) / len(infos),
        "a_bb_blocks": {"folded": plan.n_folded, "remainder": plan.n_remainder},
        "inverse_form": plan.inverse_mode_used(),
        "ir_sweeps_per_step": sum(i["ir_sweeps"] for i in infos) / len(infos),
    }
    if worst > 1e-8:
        out["warning"] = "full-system residual above 1e-8"
    if not args.no_dg_timing and args.workload not in MIXED_WORKLOADS and not wall:
        out["dg_operators"] = dg_operator_timing(case, plan)
    if not args.no_cpu_baseline and case.aii.dim() == 3:      # one order per mesh
        out["cpu_baseline"] = cpu_baseline(case, args.tol, args.cpu_seconds)
    plan.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
