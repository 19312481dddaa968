#!/usr/bin/env python3
"""Benchmark: DOFs/s of the matrix-free exact Jacobian-vector product of the
3D compressible Navier-Stokes DG discretisation (P3, 32^3 periodic hexes,
Taylor-Green-like synthetic field), plus wall time to a 1e-8 FGMRES solve of
one backward-Euler system (P4, 24^3 hexes, CFL 100, block-Jacobi).

One step = one Jv (gradient, face and volume kernels) on data resident in HBM.
Prints one JSON line (see the keys below).  --gpus > 1 is not supported:
the library runs on a single GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOFs/s for matrix-free DG Jv (p=3, 3D hex); wall time to 1e-8 FGMRES solve"
PEAK_FP64 = 78.6  # TFLOP/s, MI355X dense FP64 matrix (MFMA) peak
PEAK_HBM = 8000.0  # GB/s
PEAK_FP32 = 157.3  # TFLOP/s, MI355X dense FP32 matrix peak


def pointwise_counts(d=3, flux="roe"):
    """Pointwise flops per volume point and per face point (residual and Jv):
    the instrumented count of the oracle's physics, stored by
    tests/golden/make_pointwise_flops.py (read here as data)."""
    path = os.path.join(ROOT, "tests", "golden", "pointwise_flops.json")
    with open(path) as fh:
        return json.load(fh)["counts"][flux][str(d)]


def jv_kernel_flops(ne, nb, nq, nfq, d, pointwise=True):
    """Algorithmic flops of the exact Jv per launch, by kernel.

    Contractions per element: volume part 2*[2 Nq Nb n (1+3d)] (interpolation
    of U and grad U, lifting at the volume points, projection; value and
    tangent); face part 2*[d * 2 Nfq Nb n (2d+8)] (traces of both sides, local
    liftings, face projection).  Placement in these kernels: the d lifting
    units are the gradient kernel's (modal corrected gradients), the face
    projection (2 of the 2d+8 face units) is done by the volume kernel.
    Pointwise (value and tangent, instrumented count): Nq volume-flux
    evaluations per element in the volume kernel, d*Nfq face-flux
    evaluations per element (its d owned faces) in the face kernel.
    """
    n = d + 2
    unit = 2 * (2 * nq * nb * n)
    face = 2 * (d * 2 * nfq * nb * n * (2 * d + 8))
    face_proj = face * 2 / (2 * d + 8)
    out = {"vol_jvp": (unit * (1 + 2 * d) + face_proj) * ne, "grad_jvp": unit * d * ne,
           "face_jvp": (face - face_proj) * ne}
    if pointwise:
        pc = pointwise_counts(d)
        out["vol_jvp"] += nq * pc["vol_jvp"] * ne
        out["face_jvp"] += d * nfq * pc["face_jvp"] * ne
    return out


KERNEL_SOURCES = ("dg_mfma.h", "dg_mfma_f64.hip", "dg_device.h", "host_setup.cpp", "dg_internal.h")
KERNELS = ("grad_jvp", "face_jvp", "vol_jvp")


def kernel_source_sha():
    """sha256[:16] over the code of the timed Jv kernels' sources (concatenated;
    line comments, indentation and blank lines left out, so an edit of a comment
    does not orphan counters taken on the same code)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1809_00866_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH/WRITE summary, or
    None when the kernel sources changed since the counters were taken."""
    prof = os.path.join(ROOT, "profiles", "jv_p3_32cube_hbm_counters.txt")
    try:
        text = open(prof).read()
        sha = kernel_source_sha()
    except OSError:
        return None
    if f": {sha}" not in text:
        return None
    for line in text.splitlines():
        parts = line.split()
        if "traffic_bytes" in parts and parts[-2] == kernel:
            return float(parts[-1].replace(",", ""))
    return None


_CPU_STATE = {}


def _oracle_rows(elems):
    """Exact Jv rows of the given elements with the oracle prepared in
    _CPU_STATE (worker processes inherit it through fork); returns seconds."""
    o, U, V = _CPU_STATE["o"], _CPU_STATE["U"], _CPU_STATE["V"]
    t = time.perf_counter()
    J = o.jvp(U, V, elems=elems)
    assert np.all(np.isfinite(J))
    return time.perf_counter() - t


def cpu_baseline(sample_elems=8192, reps=3):
    """Oracle Jv (complex step, FP64, numpy) on a bounded sample of the P3 32^3
    workload, timed on the host before the GPU is initialised: single-threaded
    (BLAS pools limited to one thread) on an eighth of the sample, and on all
    host cores as a pool of forked worker processes, one BLAS thread each,
    over disjoint slices of the sample; median of reps runs each."""
    import multiprocessing as mp
    import synth
    from oracle import DGOracle, NavierStokes
    from threadpoolctl import threadpool_limits
    cfg, mesh, fld = synth.preset("cfg2")
    o = DGOracle(mesh, cfg["order"], cfg["space"], cfg["nq1d"], NavierStokes(3, mu=cfg["mu"], flux="roe"))
    # a slab of whole lattice planes (every element row costs the same; the
    # slab keeps the untimed projection of the sample's neighbours small)
    sample = np.arange(min(sample_elems, o.ne))
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    workers = max(1, min(16, visible))
    with threadpool_limits(1):
        # the sample's rows need the sample and its face neighbours
        need = np.unique(np.concatenate([sample, o.nbr[sample].reshape(-1)]))
        U = np.zeros((o.ne, o.nvar, o.nb))
        U[need] = o.project(fld, elems=need)
        V = np.zeros_like(U)
        V[need] = np.random.default_rng(866).standard_normal((len(need), o.nvar, o.nb))
        _CPU_STATE.update(o=o, U=U, V=V)
        sub = sample[: max(1, sample_elems // 8)]
        single = sorted(len(sub) * o.nvar * o.nb / _oracle_rows(sub) for _ in range(reps))[reps // 2]
        chunks = np.array_split(sample, workers)
        ctx = mp.get_context("fork")
        walls = []
        with ctx.Pool(workers) as pool:
            for _ in range(reps):
                t = time.perf_counter()
                pool.map(_oracle_rows, chunks)
                walls.append(time.perf_counter() - t)
    wall = sorted(walls)[reps // 2]
    dofs = sample_elems * o.nvar * o.nb
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": dofs / wall, "unit": "DOFs/s", "cores": workers, "kind": "oracle",
            "sample": f"exact Jv rows of the first {sample_elems} elements (whole z-planes) of the P3 32^3 workload "
                      f"({dofs} DOFs), "
                      f"complex-step numpy oracle, {workers} forked worker processes with one BLAS thread each on "
                      f"disjoint slices, median of {reps} runs ({wall:.2f} s); single_thread_value: the first "
                      f"eighth of those elements in one thread, median of {reps}",
            "single_thread_value": single, "host": {"cpu_model": model, "cpus_visible": visible}}


SMALL_SOLVE = dict(preset="cfg3", N=4, order=3)


def _small_system_name():
    return ("backward Euler, P3 on a 4^3 periodic lattice of the P4 24^3 workload's domain and field, CFL 100, "
            "FGMRES(30) + FP64 EWBJ to 1e-8 (6,400 DOFs)")


def oracle_time_to_tolerance():
    """The oracle solving a small backward-Euler system end to end (its block
    diagonal by coloured complex-step probing, dense block inverses, its
    FGMRES(30) with CGS2), timed on the host; the GPU solves the same system
    in gpu_small_time_to_tolerance."""
    import synth
    from oracle import DGOracle, NavierStokes, fgmres, backward_euler_dt
    cfg, mesh, fld = synth.preset(SMALL_SOLVE["preset"], N=SMALL_SOLVE["N"], order=SMALL_SOLVE["order"])
    k = cfg["order"]
    t0 = time.perf_counter()
    o = DGOracle(mesh, k, cfg["space"], cfg["nq1d"], NavierStokes(3, mu=cfg["mu"], flux="roe"))
    U = o.project(fld)
    et = o.elem_tables(np.arange(o.ne))
    smax = o.phys.max_wave_speed(np.einsum("eqb,ecb->eqc", et["phi"], U)).max()
    shift = 1.0 / backward_euler_dt(smax, float(np.min(mesh["h"])), k, cfg["cfl"])
    b = -o.to_flat(o.residual(U))
    t1 = time.perf_counter()
    Dinv = np.linalg.inv(o.block_diagonal(U, shift=shift))
    t2 = time.perf_counter()
    A = lambda x: o.to_flat(o.operator(U, o.from_flat(x), shift))
    M = lambda v: o.to_flat((Dinv @ o.from_flat(v).reshape(o.ne, -1, 1)).reshape(U.shape))
    x, info = fgmres(A, b, M, restart=30, rtol=cfg["rtol"], max_iter=3000)
    t3 = time.perf_counter()
    return {"workload": _small_system_name(), "seconds": t3 - t1, "setup_s": t2 - t1, "solve_s": t3 - t2,
            "prepare_s": t1 - t0, "iters": info["iters"], "converged": bool(info["converged"]),
            "rel_res_true": info["rel_res_true"], "shift": shift, "ndof": int(b.size)}


def gpu_small_time_to_tolerance():
    """The same small system as oracle_time_to_tolerance through the library
    (FP64 block setup, FGMRES(30) with EWBJ)."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    cfg, mesh, fld = synth.preset(SMALL_SOLVE["preset"], N=SMALL_SOLVE["N"], order=SMALL_SOLVE["order"])
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    w = g.project_field(fld)
    smax = g.max_wave_speed(w)
    shift = 1.0 / (cfg["cfl"] * float(np.min(mesh["h"])) / ((2 * cfg["order"] + 1) * smax))
    b = -g.residual(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.block_setup(w, shift, storage="fp64")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, st = g.fgmres(w, shift, b, restart=30, max_iter=3000, rtol=cfg["rtol"], precond="bj")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.close()
    return {"workload": _small_system_name(), "seconds": t2 - t0, "setup_s": t1 - t0, "solve_s": t2 - t1,
            "iters": st["iters"], "converged": bool(st["converged"]), "rel_res_true": st["rel_res_true"],
            "shift": shift}


PHASES = ("grad_jvp", "face_jvp", "vol_jvp", "grad_jvp_f32", "face_jvp_f32", "vol_jvp_f32", "grad_jvp_bf16",
          "face_jvp_bf16", "vol_jvp_bf16", "block_probe", "block_invert", "block_apply", "arnoldi", "mg_vcycle",
          "mg_probe", "mg_coarse_invert", "mlp_apply", "grad_probe", "face_probe", "vol_probe", "grad_probe_f32",
          "face_probe_f32", "vol_probe_f32", "grad_probe_bf16", "face_probe_bf16", "vol_probe_bf16")
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2}


def solve_phases(g, w, shift, b, cfg, precond, storage, curved, mg_setup=None):
    """Per-phase breakdown of one solve: the setup (block Jacobi, or the
    hierarchy through mg_setup()) and the solve again with HIP events around
    each phase (the timed run above carries no events).  Each phase: total ms,
    calls, ms per call; the Jv phases with their contraction flops against the
    FP64 (or FP32) matrix peak on affine meshes, the block apply with its bytes
    against HBM.  mg_probe is the whole hierarchy probing and includes the
    fine block probing and inversion."""
    import torch
    g.set_profiling(True)
    for k in PHASES:
        g.kernel_time(k)  # reset
    if precond != "mg":
        g.block_setup(w, shift, storage=storage)
    elif mg_setup is not None:
        mg_setup()
    g.fgmres(w, shift, b, restart=cfg["restart"], max_iter=3000, rtol=cfg["rtol"], precond=precond)
    torch.cuda.synchronize()
    g.set_profiling(False)
    out = {}
    for k in PHASES:
        ms, n = g.kernel_time(k)
        if n:
            out[k] = {"ms_total": round(ms, 3), "calls": n, "ms_per_call": round(ms / n, 4)}
    nfq = cfg["nq1d"] ** 2
    fl = jv_kernel_flops(g.ne, g.nb, g.nq, nfq, 3)
    for suf, peak in (("", PEAK_FP64), ("_f32", PEAK_FP32), ("_bf16", PEAK_FP32)):
        ks = [k + suf for k in KERNELS]
        fused = "grad_jvp" + suf not in out  # corrected gradients formed in the volume kernel
        if curved or not all(k in out for k in ks if not (fused and k.startswith("grad"))):
            continue
        ms = sum(out[k]["ms_per_call"] for k in ks if k in out)
        tf = sum(fl.values()) / (ms * 1e-3) / 1e12
        out["jv" + suf] = {"ms_per_call": round(ms, 4), "achieved_tflops": round(tf, 2), "peak": peak,
                           "frac": round(tf / peak, 3)}
    if "block_apply" in out:
        m = g.nv * g.nb
        by = g.ne * m * m * STORAGE_BYTES[storage] + 2 * g.ndof * 8
        gbs = by / (out["block_apply"]["ms_per_call"] * 1e-3) / 1e9
        out["block_apply"].update({"bytes_per_call": by, "achieved_gbs": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM, 3)})
    return out


def time_to_tolerance(storage="fp64", precond="bj", fine_precision="fp64", rescale=False, coarse_ilu=False,
                      preset="cfg3"):
    """Backward-Euler system of the P4 24^3 workload solved by FGMRES(30) to 1e-8,
    preconditioned by block Jacobi or by the P4/P2/P1 p-multigrid V-cycle
    (GMRES[EWBJ] smoothers 8/8/40, one captured graph per cycle)."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    cfg, mesh, fld = synth.preset(preset)
    tc = time.perf_counter()
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    t_create = time.perf_counter() - tc
    w = g.project_field(fld)
    smax = g.max_wave_speed(w)
    h = float(np.min(mesh["h"]))
    dt = cfg["cfl"] * h / ((2 * cfg["order"] + 1) * smax)
    shift = 1.0 / dt
    b = -g.residual(w)
    for _ in range(3):
        g.jvp(w, b, shift=shift)
    torch.cuda.synchronize()
    tj = time.perf_counter()
    for _ in range(10):
        g.jvp(w, b, shift=shift)
    torch.cuda.synchronize()
    jv_ms = (time.perf_counter() - tj) * 100.0
    def setup_mg():
        g.mg_setup(w, shift, cfg["mg_orders"], cfg["mg_smooth"], storage=storage, use_graph=True,
                   fine_precision=fine_precision, rescale=rescale, coarse_ilu=coarse_ilu)

    def setup():
        if precond == "mg":
            setup_mg()
        else:
            g.block_setup(w, shift, storage=storage)
        torch.cuda.synchronize()

    # a first, untimed setup: the autotuner times its candidate launch shapes
    # once per problem shape and process (the choices are cached), so the
    # timed setup is what every later solve of this shape pays
    tf = time.perf_counter()
    setup()
    first_setup_s = time.perf_counter() - tf
    t0 = time.perf_counter()
    setup()
    t1 = time.perf_counter()
    x, st = g.fgmres(w, shift, b, restart=cfg["restart"], max_iter=3000, rtol=cfg["rtol"], precond=precond)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    extra = {"phases": solve_phases(g, w, shift, b, cfg, precond, storage, curved=preset != "cfg3",
                                    mg_setup=setup_mg)}
    if precond == "mg":  # one preconditioner application (the captured V-cycle), outside the solve
        z = g.empty()
        g.mg_apply(b, out=z)
        torch.cuda.synchronize()
        tv = time.perf_counter()
        for _ in range(5):
            g.mg_apply(b, out=z)
        torch.cuda.synchronize()
        extra["vcycle_ms"] = (time.perf_counter() - tv) * 200.0
        del z
    g.close()
    name = (f"p-multigrid V-cycle P4/P2/P1{' rescaled-inherited' if rescale else ''}, GMRES[EWBJ] smoothers "
            f"8/8/40{' (coarsest: GMRES[block ILU(0)])' if coarse_ilu else ''}, {fine_precision} fine operator, "
            if precond == "mg" else "block Jacobi ") + storage
    mesh_name = "P4 24^3 hexes" if preset == "cfg3" else "P4 24^3 curved hexes (vertices moved by +-0.1h)"
    return {"workload": f"backward Euler, {mesh_name}, CFL 100, FGMRES(30), " + name, "create_s": t_create,
            "jv_ms": jv_ms,
            "seconds": t2 - t0, "setup_s": t1 - t0, "first_setup_s": first_setup_s, "solve_s": t2 - t1,
            "iters": st["iters"],
            "converged": bool(st["converged"]), "rel_res_true": st["rel_res_true"], "dt": dt, **extra}


def vcycle_tuning(storage="fp32", fine_precision="fp32", n_cycles=20):
    """The P4/P2/P1 V-cycle of the P4 24^3 backward-Euler system (the fastest
    solve configuration: FP32 fine operator and factors) with the built-in
    launch shapes and with the autotuned ones: ms per captured cycle, set-up
    seconds (the first tuned set-up of a shape includes its timing runs; later
    ones reuse the process-wide choices), the FGMRES solve, and the chosen
    shapes."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    cfg, mesh, fld = synth.preset("cfg3")
    out = {"workload": "P4 24^3 hexes, CFL 100 backward-Euler operator, V-cycle P4/P2/P1 GMRES[EWBJ] 8/8/40, "
                       f"{fine_precision} fine operator, {storage} factors"}
    for mode in ("fixed", "auto"):
        g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
        g.set_tuning(mode)
        w = g.project_field(fld)
        smax = g.max_wave_speed(w)
        dt = cfg["cfl"] * float(np.min(mesh["h"])) / ((2 * cfg["order"] + 1) * smax)
        shift = 1.0 / dt
        b = -g.residual(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "auto":
            g.autotune(w)
        g.mg_setup(w, shift, cfg["mg_orders"], cfg["mg_smooth"], storage=storage, use_graph=True,
                   fine_precision=fine_precision)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        z = g.empty()
        for _ in range(2):
            g.mg_apply(b, out=z)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(3):
            tv = time.perf_counter()
            for _ in range(n_cycles):
                g.mg_apply(b, out=z)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - tv) * 1e3 / n_cycles)
        t1 = time.perf_counter()
        x, st = g.fgmres(w, shift, b, restart=cfg["restart"], max_iter=3000, rtol=cfg["rtol"], precond="mg")
        torch.cuda.synchronize()
        out[mode] = {"vcycle_ms": best, "setup_s": setup_s, "solve_s": time.perf_counter() - t1,
                     "iters": st["iters"], "converged": bool(st["converged"]), "rel_res_true": st["rel_res_true"],
                     "shapes": g.tuning_report().splitlines()}
        g.close()
        del w, b, z, x
        torch.cuda.empty_cache()
    out["vcycle_speedup"] = out["fixed"]["vcycle_ms"] / out["auto"]["vcycle_ms"]
    return out


def mg_trajectory(n_steps=4, lag=1, cycle="v", scheme="be"):
    """Backward-Euler steps of the P4 24^3 workload (CFL 100), each solved by
    FGMRES(30) to 1e-8 with the P4/P2/P1 p-multigrid preconditioner (FP32 fine
    smoothing and factors).  lag > 1: the hierarchy is built every lag steps and
    in between only its fine level follows the current state and time step
    (coarse operators frozen, fine block Jacobi refreshed).  scheme "ros2": each
    step is a two-stage ROS2 Rosenbrock step (Alg. ros), one solve per stage
    with the hierarchy of the step's initial state."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    cfg, mesh, fld = synth.preset("cfg3")
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    w = g.project_field(fld)
    h = float(np.min(mesh["h"]))
    iters, t_setup, t_solve = [], 0.0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    from paper_1809_00866_amd import schemes
    for k in range(n_steps):
        dt = cfg["cfl"] * h / ((2 * cfg["order"] + 1) * g.max_wave_speed(w))
        shift = 1.0 / dt if scheme == "be" else 1.0 / (schemes.ROS2["gamma"] * dt)
        ta = time.perf_counter()
        if k % lag == 0:
            g.mg_setup(w, shift, cfg["mg_orders"], cfg["mg_smooth"], storage="fp32", use_graph=True,
                       fine_precision="fp32", cycle=cycle)
        else:
            g.mg_update_fine(w, shift, refresh_blocks=True)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        if scheme == "be":
            dw, st = g.fgmres(w, shift, -g.residual(w), restart=cfg["restart"], max_iter=600, rtol=cfg["rtol"],
                              precond="mg")
            w_next = w + dw
        else:
            w_next, st = g.rosenbrock_step(w, dt, schemes.ROS2, restart=cfg["restart"], max_iter=600,
                                           rtol=cfg["rtol"], precond="mg")
        torch.cuda.synchronize()
        tc = time.perf_counter()
        t_setup += tb - ta
        t_solve += tc - tb
        if not st["converged"]:
            raise RuntimeError(f"step {k} did not converge: {st}")
        iters.append(st["iters"])
        w = w_next
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    g.close()
    kind = "backward-Euler steps" if scheme == "be" else "ROS2 Rosenbrock steps (2 solves each)"
    return {"workload": f"{n_steps} {kind}, P4 24^3 hexes, CFL 100, FGMRES(30) to 1e-8, p-multigrid "
                        f"{'full' if cycle == 'full' else 'V'} cycle P4/P2/P1 8/8/40, fp32 smoothing, "
                        f"hierarchy rebuilt every {lag} step(s)",
            "seconds": total, "setup_s": t_setup, "solve_s": t_solve, "iters_per_step": iters}


def learned_preconditioner(train_steps=3000, max_iter=1000):
    """The learned element-local preconditioner on the P3 32^3 workload, as a
    correction to block Jacobi (z_K = D_K^-1 r_K + s_K MLP(x_K); a zero last
    layer is block Jacobi exactly): pairs from backward-Euler snapshots 0, 2, 4
    (inputs r = R(w) and three terms of the block-Jacobi-preconditioned Krylov
    sequence, targets the solutions of G z = r to 1e-6), 1e5 pairs sampled,
    Adam with batch 1024; the held-out snapshot 6 system solved to 1e-8 with
    block Jacobi, the trained correction (with and without its judge), the
    untrained correction, no preconditioner and the p-multigrid V-cycle."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd import learned as LR
    cfg, mesh, fld = synth.preset("cfg5")
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    h = float(np.min(mesh["h"]))
    t0 = time.perf_counter()
    states = LR.trajectory(g, g.project_field(fld), 6, cfg["cfl"], cfg["order"], h)
    shifts = [LR.time_step(g, s, cfg["cfl"], cfg["order"], h) for s in states]
    g.mlp_set_mode("correct_bj")
    XT = [LR.pairs(g, states[k], shifts[k], n_krylov=3) for k in (0, 2, 4)]
    X = torch.cat([a for a, _ in XT])
    T = torch.cat([b for _, b in XT])
    Xv, Tv = LR.pairs(g, states[6], shifts[6], n_krylov=3)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_in, n_out = g.mlp_sizes
    theta0 = synth.mlp_init_weights(n_in, n_out, seed=1809)
    theta0[-(n_out * 256 + n_out):] = 0.0          # W3, b3: the untrained correction is zero
    theta0 = torch.from_numpy(theta0)
    g.mlp_set_weights(theta0)
    sub = torch.randperm(X.shape[0], generator=torch.Generator().manual_seed(0))[:100000].cuda()
    Xt, Tt = X[sub].contiguous(), T[sub].contiguous()
    val0 = LR.validation_loss(g, Xv, Tv)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = LR.train(g, Xt, Tt, train_steps, batch=1024, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    val1 = LR.validation_loss(g, Xv, Tv)
    theta1 = g.mlp_get_weights()
    w6, sh6 = states[6], shifts[6]
    b = -g.residual(w6)
    g.block_setup(w6, sh6)
    held = {}

    def run(name, **kw):
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, st = g.fgmres(w6, sh6, b, rtol=1e-8, max_iter=max_iter, **kw)
        torch.cuda.synchronize()
        held[name] = {"iters": st["iters"], "converged": bool(st["converged"]), "rel_res_true": st["rel_res_true"],
                      "rho": st["rho"], "fallbacks": st["fallbacks"], "seconds": time.perf_counter() - a}

    run("block_jacobi", precond="bj")
    run("none", precond="none")
    run("learned_correction", precond="mlp")
    run("learned_correction_with_judge", precond="mlp", rho_ref=held["block_jacobi"]["rho"])
    g.mlp_set_weights(theta0)
    run("untrained_correction", precond="mlp")
    g.mlp_set_weights(theta1)
    orders, its = LR.mg_levels(cfg["order"])
    torch.cuda.synchronize()
    a = time.perf_counter()
    g.mg_setup(w6, sh6, orders, its)
    torch.cuda.synchronize()
    mg_setup_s = time.perf_counter() - a
    run("p_multigrid", precond="mg")
    held["p_multigrid"]["setup_s"] = mg_setup_s
    g.close()
    return {"workload": f"P3 32^3, backward-Euler snapshots 0/2/4 (train) and 6 (held out), CFL {cfg['cfl']:g}; "
                        "network = correction to block Jacobi",
            "pairs_available": int(X.shape[0]), "pairs_train": int(Xt.shape[0]), "pairs_val": int(Xv.shape[0]),
            "train_steps": train_steps, "batch": 1024, "data_s": t_data, "train_s": t_train,
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]), "val_loss_untrained": val0,
            "val_loss_trained": val1, "held_out_solve_to_1e-8": held}


def poisson_assessment(sizes=(32, 64, 128), shift=1.0, rtol=1e-8):
    """The Poisson assessment of App. B (Table Poisson3L's three-level setting)
    on the BR2 Laplacian at k = 6: FGMRES(30) to rtol preconditioned by the
    V-cycle 6/3/1 with one smoothing step on the two finer levels and 40 on the
    coarsest (GMRES preconditioned by block Jacobi, and by block ILU(0) on the
    coarsest level), with inherited and with rescaled-inherited coarse
    operators (App. A).  Periodic unit square with N^2 uniform quadrilaterals,
    and distorted ones (every vertex moved by a seeded U(-0.1h, 0.1h): the
    curved-element kernels), with the operator shift*I + L (one backward-Euler
    step of the heat equation, diffusion-dominated): the periodic meshes carry
    no Dirichlet boundary."""
    import torch
    import synth
    from paper_1809_00866_amd import DG
    rows = []
    for N, perturb in [(N, p) for p in (0.0, 0.1) for N in sizes]:
        mesh = synth.lattice_mesh((N, N), L=1.0, perturb=perturb, seed=1396 if perturb else None)
        g = DG(mesh, 6, nq1d=8, mu=1.0, physics="diffusion")
        w = g.empty().zero_()
        b = g.project_field(lambda x: np.exp(-25.0 * ((x[..., 0] - 0.75) ** 2 + (x[..., 1] - 0.75) ** 2))[..., None])
        for rescale in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.mg_setup(w, shift, (6, 3, 1), (1, 1, 40), storage="fp64", use_graph=True, rescale=rescale,
                       coarse_ilu=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, st = g.fgmres(w, shift, b, restart=30, rtol=rtol, max_iter=500, precond="mg")
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rows.append({"N": N, "mesh": "distorted" if perturb else "uniform", "dofs": g.ndof,
                         "scaling": "on" if rescale else "off", "iters": st["iters"],
                         "rho": st["rho"], "converged": bool(st["converged"]), "setup_s": t1 - t0,
                         "solve_s": t2 - t1})
        g.close()
    return {"workload": f"BR2 Laplacian k=6, periodic N^2 quads (uniform; vertices moved by +-0.1h), operator "
                        f"{shift:g}*I + L, FGMRES(30) to {rtol:g}, "
                        "V-cycle 6/3/1, smoothing 1/1/40 (coarsest: GMRES[block ILU(0)])", "rows": rows}


def _progress(msg, t0=[time.perf_counter()]):
    """One line per finished leg on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg} ({time.perf_counter() - t0[0]:.1f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner experiment")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain streaming kernel of known size (c = a - b over 256 MiB vectors: "
                         "512 MiB read, 256 MiB written), the reference for the HBM counters")
    ap.add_argument("--tuning", choices=("auto", "fixed"), default="auto",
                    help="launch shapes of the Jv legs: autotuned (default) or the built-in ones only "
                         "(counter runs: no tuning launches beside the timed kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the library runs on one GPU "
              "(elements would shard into slabs with one halo exchange per Jv; not built)", file=sys.stderr)
        sys.exit(2)

    # the oracle's CPU baseline runs first, before anything touches the GPU
    # (its worker processes are forked)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_sample)
    if cpu is not None:
        _progress("oracle CPU baseline")
        cpu["time_to_tol_small"] = {"oracle": oracle_time_to_tolerance()}
        _progress("oracle time to tolerance (small system)")

    import torch
    import synth
    from paper_1809_00866_amd import DG

    torch.cuda.set_device(0)
    cfg, mesh, fld = synth.preset("cfg2")
    g = DG(mesh, cfg["order"], basis=cfg["space"], nq1d=cfg["nq1d"], flux="roe", mu=cfg["mu"])
    w = g.project_field(fld)
    v = torch.tensor(synth.random_vector(g.ndof, cfg["v_seed"]), device="cuda")
    out = g.empty()

    def timed_pass():
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            g.jvp(w, v, out=out)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    # the built-in launch shapes, then the autotuned ones (the metric), each
    # timed over K steps after the same warm-up
    g.set_tuning("fixed")
    for _ in range(args.warmup):
        g.jvp(w, v, out=out)
    wall_fixed = timed_pass()
    if args.tuning == "auto":
        g.set_tuning("auto")
        g.autotune(w)
        for _ in range(args.warmup):
            g.jvp(w, v, out=out)
        wall = timed_pass()
    else:
        wall = wall_fixed
    shapes = g.tuning_report().splitlines()
    # the survey's protocol beside the contract's single pass: 5 passes of 100
    # Jv calls (after 10 warm-up calls), HIP events around each pass, median
    proto = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(10):
        g.jvp(w, v, out=out)
    for _ in range(5):
        ev0.record()
        for _ in range(100):
            g.jvp(w, v, out=out)
        ev1.record()
        ev1.synchronize()
        proto.append(ev0.elapsed_time(ev1) / 100)
    proto.sort()
    jv_protocol = {"passes": 5, "calls_per_pass": 100, "median_ms": proto[2], "min_ms": proto[0], "max_ms": proto[-1],
                   "median_value": g.ndof / (proto[2] * 1e-3), "unit": "DOFs/s"}
    # per-kernel HIP events (on the stream of each launch) over a second pass
    # of the same K steps: the event records themselves cost ~0.02 ms per Jv,
    # so the throughput above is taken without them
    g.set_profiling(True)
    for k in KERNELS:
        g.kernel_time(k)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.jvp(w, v, out=out)
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t0
    g.set_profiling(False)
    kt = {k: g.kernel_time(k) for k in KERNELS}
    assert torch.isfinite(out).all()
    # the reduced-precision operator (FP32 contractions and fluxes) on the same
    # workload, reported beside the FP64 metric (it serves preconditioners only)
    out32 = g.empty()
    for _ in range(args.warmup):
        g.jvp(w, v, out=out32, mode="exact_fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.jvp(w, v, out=out32, mode="exact_fp32")
    torch.cuda.synchronize()
    wall32 = time.perf_counter() - t0
    jv_fp32 = {"value": g.ndof / (wall32 / args.steps), "unit": "DOFs/s", "ms_per_step": wall32 * 1e3 / args.steps,
               "rel_diff_vs_fp64": float((out32 - out).norm() / out.norm())}
    # the BF16-contraction operator (BF16 operands, FP32 accumulation, FP32
    # pointwise fluxes) on the same workload
    for _ in range(args.warmup):
        g.jvp(w, v, out=out32, mode="exact_bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.jvp(w, v, out=out32, mode="exact_bf16")
    torch.cuda.synchronize()
    wall16 = time.perf_counter() - t0
    jv_bf16 = {"value": g.ndof / (wall16 / args.steps), "unit": "DOFs/s", "ms_per_step": wall16 * 1e3 / args.steps,
               "rel_diff_vs_fp64": float((out32 - out).norm() / out.norm())}
    del out32
    _progress("Jv legs (FP64, FP32, BF16)")
    ms_per_step = wall * 1e3 / args.steps
    value = g.ndof / (wall / args.steps)

    nfq = cfg["nq1d"] ** 2
    flops = jv_kernel_flops(g.ne, g.nb, g.nq, nfq, 3)
    flops_c = jv_kernel_flops(g.ne, g.nb, g.nq, nfq, 3, pointwise=False)
    if kt["grad_jvp"][1] == 0:  # the volume kernel forms the corrected gradients itself
        for fl in (flops, flops_c):
            fl["vol_jvp"] += fl.pop("grad_jvp")
        kt.pop("grad_jvp")
    avg = {k: kt[k][0] / max(kt[k][1], 1) for k in kt}
    dom = max(avg, key=avg.get)
    achieved = flops[dom] / (avg[dom] * 1e-3) / 1e12
    per_dof = sum(flops.values()) / g.ndof
    # FP64 MFMA and FP64 vector FMA share one 78.6 TFLOP/s issue budget, so the
    # contractions (MFMA) and the counted pointwise flops (vector ALU) are priced
    # against the same peak
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": measured_traffic(dom), "traffic_unit": "bytes/launch",
                "flops_per_launch": {k: flops[k] for k in flops},
                "contraction_only": {"flops_per_launch": flops_c[dom],
                                     "frac": flops_c[dom] / (avg[dom] * 1e-3) / 1e12 / PEAK_FP64},
                "kernel_ms": {k: round(avg[k], 4) for k in avg},
                "kernel_frac": {k: round(flops[k] / (avg[k] * 1e-3) / 1e12 / PEAK_FP64, 3) for k in avg},
                "ms_per_step_with_kernel_events": wall_prof * 1e3 / args.steps,
                # the whole Jv against the algorithmic count (contractions plus the
                # instrumented pointwise value-and-tangent flops)
                "whole_jv": {"flop_per_dof": per_dof, "achieved": value * per_dof / 1e12, "peak": PEAK_FP64,
                             "unit": "TFLOP/s", "frac": value * per_dof / 1e12 / PEAK_FP64}}
    g_ndof = g.ndof
    g.close()
    del w, v, out
    if args.calib_copy:
        a = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        b = torch.ones_like(a)
        c = torch.empty_like(a)
        for _ in range(3):
            torch.sub(a, b, out=c)
        torch.cuda.synchronize()
        del a, b, c
    torch.cuda.empty_cache()

    res = {"metric": METRIC, "value": value, "unit": "DOFs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "exact Jv, 3D compressible NS, P3 (Nb=20), 32^3 periodic hexes, 4^3/4^2 Gauss, "
                                  "Roe + BR2, Taylor-Green-like field Mach 0.1 Re 1600",
                      "n_elem": int(32 ** 3), "ndof": int(32 ** 3 * 100), "dofs_per_variable": int(32 ** 3 * 20)},
           "roofline": roofline, "jv_fp32": jv_fp32, "jv_bf16": jv_bf16,
           "launch_shapes": shapes, "jv_protocol": jv_protocol,
           "jv_fixed_shapes": {"ms_per_step": wall_fixed * 1e3 / args.steps,
                               "value": g_ndof / (wall_fixed / args.steps), "unit": "DOFs/s"}}
    if not args.no_solve:
        res["time_to_tol"] = time_to_tolerance("fp64")
        _progress("time_to_tol")
        res["time_to_tol_fp32_blocks"] = time_to_tolerance("fp32")
        _progress("time_to_tol_fp32_blocks")
        res["time_to_tol_bf16_blocks"] = time_to_tolerance("bf16")
        _progress("time_to_tol_bf16_blocks")
        res["time_to_tol_pmg"] = time_to_tolerance("fp64", precond="mg")
        _progress("time_to_tol_pmg")
        res["time_to_tol_pmg_fp32_smoothing"] = time_to_tolerance("fp32", precond="mg", fine_precision="fp32")
        _progress("time_to_tol_pmg_fp32_smoothing")
        res["vcycle_tuning"] = vcycle_tuning()
        _progress("vcycle_tuning")
        res["time_to_tol_pmg_bf16_factors"] = time_to_tolerance("bf16", precond="mg", fine_precision="fp32")
        _progress("time_to_tol_pmg_bf16_factors")
        res["time_to_tol_pmg_bf16_operator"] = time_to_tolerance("bf16", precond="mg", fine_precision="bf16")
        _progress("time_to_tol_pmg_bf16_operator")
        res["time_to_tol_pmg_fp32_rescaled"] = time_to_tolerance("fp32", precond="mg", fine_precision="fp32",
                                                                 rescale=True)
        res["time_to_tol_pmg_fp32_coarse_ilu"] = time_to_tolerance("fp32", precond="mg", fine_precision="fp32",
                                                                   coarse_ilu=True)
        res["time_to_tol_pmg_curved"] = time_to_tolerance("fp32", precond="mg", fine_precision="fp64", preset="cfg4")
        _progress("time_to_tol_pmg_curved")
        res["time_to_tol_pmg_curved_fp32_smoothing"] = time_to_tolerance("fp32", precond="mg", fine_precision="fp32",
                                                                         preset="cfg4")
        res["time_to_tol_pmg_curved_bf16_factors"] = time_to_tolerance("bf16", precond="mg", fine_precision="fp32",
                                                                       preset="cfg4")
        res["time_to_tol_bj_curved"] = time_to_tolerance("fp32", preset="cfg4")
        _progress("time_to_tol_bj_curved")
        res["time_to_tol_bj_curved_fp64"] = time_to_tolerance("fp64", preset="cfg4")
        _progress("time_to_tol_bj_curved_fp64")
        res["trajectory_pmg"] = mg_trajectory(4, lag=1)
        _progress("trajectory_pmg")
        res["trajectory_pmg_lag3"] = mg_trajectory(4, lag=3)
        _progress("trajectory_pmg_lag3")
        res["trajectory_pmg_full_cycle"] = mg_trajectory(4, lag=1, cycle="full")
        _progress("trajectory_pmg_full_cycle")
        res["trajectory_pmg_ros2"] = mg_trajectory(4, lag=1, scheme="ros2")
        _progress("trajectory_pmg_ros2")
    if not args.no_learned:
        res["learned_precond"] = learned_preconditioner()
        _progress("learned_precond")
    if not args.no_solve:
        res["poisson_pmg"] = poisson_assessment()
        _progress("poisson_pmg")
    if cpu is not None:
        small = cpu["time_to_tol_small"]
        small["gpu"] = gpu_small_time_to_tolerance()
        small["speedup"] = small["oracle"]["seconds"] / small["gpu"]["seconds"]
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
