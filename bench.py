#!/usr/bin/env python3
"""Throughput of the batched space-time solves on one MI355X.

One step = one pass of the whole path over one batch of synthetic input: the
configured estimator end to end (sample points, KL synthesis, Crank-Nicolson /
Newton / GMRES solves on every level and the coarse partner level, QoIs,
level differences, estimator).  The KL basis and level set-up are one-time
set-up outside the timed region; sample points and normals are produced or
resident in HBM before timing starts.

Default workload: the batched uneven MLQMC estimator (c4, 9^3..129^3, 16 shifts) in
mixed precision, with its FP64 companion run on the same sample plan: the line
reports both passes' time to the same RMSE (one pass gives the estimate and its
shift-based RMSE) and their ratio.

Prints one JSON line.  Metric: space-time DOF x inner iterations per second =
sum over samples, steps and Newton iterations of n_l * (GMRES iterations), over
wall time, for the headline precision.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time DOF·iters/s per GPU + MLQMC time-to-RMSE, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
APPLY_SOURCE = os.path.join(ROOT, "paper_2105_02007_amd", "csrc", "mlq_stencil3.hip")
TET_APPLY_SOURCE = os.path.join(ROOT, "paper_2105_02007_amd", "csrc", "mlq_tet.hip")
COPY_ELEMS = 1 << 27  # 1 GiB of FP64 for the counter calibration copy


def counter_traffic(config, prec, tet=False):
    """HBM bytes per algorithmic byte of the apply, from the committed rocprofv3 counter summary.

    The summary records FETCH_SIZE and WRITE_SIZE summed over the apply dispatches
    of one estimator pass, each scaled by what the same counter reads for a copy
    of known size, and the SHA-256 of the kernel source it was taken with.  A
    summary for a different source (the kernel changed since) gives None.
    """
    import hashlib
    kernel, source = ("k_tet_apply", TET_APPLY_SOURCE) if tet else ("k_wave3", APPLY_SOURCE)
    path = os.path.join(ROOT, "profiles", f"apply_{kernel}_{config}_{prec}_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for ln in open(path):
        if ln.startswith("record:"):
            for kv in ln.split()[1:]:
                k, v = kv.split("=")
                rec[k] = v
    if rec.get("source_sha256") != hashlib.sha256(open(source, "rb").read()).hexdigest():
        return None
    return float(rec["hbm_bytes_per_alg_byte"])

# probe points of the action potential (--fields), in the unit box: near the stimulus, the
# centre, a face, the far corner
FIELD_PROBES = [[0.05, 0.05, 0.05], [0.5, 0.5, 0.5], [1.0, 0.5, 0.25], [1.0, 1.0, 1.0]]

def field_probes(cfg, runner):
    """Probe points of --fields: FIELD_PROBES in the unit box, or on a shell four vertices of the
    finest mesh spread over its vertex order (from the inner apex region outwards)."""
    import numpy as np
    if runner.tet:
        xyz = runner.meshes[-1]["xyz"]
        return xyz[[0, len(xyz) // 3, (2 * len(xyz)) // 3, len(xyz) - 1]]
    return np.array(FIELD_PROBES)[:, :cfg["dim"]]


WORKLOAD_TEXT = {
    "c1": "2D unit square Q1 33x33, 64 steps, 16-mode KL (l=0.2, s=0.3 rad), 16 MC samples, mean u(T), FP64",
    "c2": "3D unit cube Q1 9^3..65^3 nested, 32..256 steps, 64-mode KL (l=0.1, s=0.3 rad) on 65^3, "
          "MLMC 2048/512/128/32 samples, mean activation time, FP64",
    "c3": "3D unit cube Q1 129^3, 512 steps, 128-mode KL, 64 rank-1 lattice points x 1 shift, "
          "mean activation time, FP32 inner + FP64 Newton residual",
    "c4": "3D unit cube Q1 9^3..129^3 nested, 32..512 steps, 128-mode KL, MLQMC 16 shifts x 256/64/16/4/1, "
          "mean activation time",
    "c2i": "the paper's cube model: isotropic G = max(v, 0.1 E[V]) I, v = E[V] + W, E[V] = 3.325e-3, W a "
           "squared-exponential KL field (0.3 E[V], sigma_KL = 0.25) with 66 uniform coordinates, 3D unit cube "
           "Q1 9^3..65^3 nested, 32..256 steps, MLMC 2048/512/128/32 samples, mean activation time, FP64",
    "c4i": "the paper's cube model (as c2i) with the paper's QMC rule: MLQMC with Halton points (indices 1..N_l, "
           "16 random shifts mod 1), 3D unit cube Q1 9^3..129^3 nested, 32..512 steps, 256/64/16/4/1 points, "
           "mean activation time",
    "c5": "non-nested prolate-ellipsoidal shell, P1 tetrahedra 25k/199k/1.6M vertices, 512 steps, 256-mode KL "
          "(l = 0.1 long axis), rule-based +60/-60 deg fibres, combination estimator 16/64/256 nested MC points, "
          "mean activation time",
    "c5i": "the c5 shells with the paper's idealised-ventricle model: isotropic G = max(v, 0.1 E[V]) I, "
           "v = E[V] + W, W a squared-exponential KL field (0.3 E[V], sigma_KL = 0.5) with 87 uniform "
           "coordinates, combination estimator 16/64/256 nested MC points, mean activation time",
    "c5v": "the c5 shells with the paper's heart model: eq. (AdmV) with a random vector field V = sigma_l f0 + W, "
           "W three independent squared-exponential KL fields (0.3 sigma_l, sigma_KL = 0.64), 3 x 45 uniform "
           "coordinates, combination estimator 16/64/256 nested MC points, mean activation time",
}


CPU_STEPS = 16  # time steps per sample of the CPU baseline (the first steps of every solve)


def _cpu_job(args):
    """One oracle solve for the CPU baseline (a worker of the process pool, one BLAS thread): the
    sample's field is a seeded perturbation in place of the KL field (the KL set-up is not part of
    the timed solve).  Returns (vertices, steps, oracle iterations, seconds)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import fem, run, stepper
    name, l, i = args
    cfg = W.config(name)
    lv, ph = cfg["levels"][l], cfg["physics"]
    steps = min(CPU_STEPS, lv["n_steps"])
    with threadpool_limits(1):
        if lv.get("kind") == "tet":
            from oracle.tetfem import TetMesh
            m = W.tet_mesh(lv)
            mesh = TetMesh(m["xyz"], m["tets"])
            r = W.random_nodal(cfg["seed"] + 1000 * l + i, 3, mesh.n_elems)
            if cfg.get("model") == "vector":
                f0 = np.cos(m["theta0"])[:, None] * m["e_circ"] + np.sin(m["theta0"])[:, None] * m["e_long"]
                G = fem.conductivity(ph["sigma_l"] * (f0 + 0.3 * r.T), ph["sigma_t"])
            elif cfg.get("model") == "iso":
                G = fem.conductivity_iso(cfg["kl"]["mean"] * (1.0 + 0.3 * r[0]), 3, ph["sigma_t"])
            else:
                G = mesh.conductivity(m["theta0"] + 0.3 * r[0], m["e_circ"], m["e_long"], ph["sigma_l"],
                                      ph["sigma_t"])
            t0 = time.perf_counter()
            out = stepper.solve(mesh, G, ph, lv["n_steps"], tol=1e-13, stop_after=steps)
            el = time.perf_counter() - t0
        else:
            mesh = run.level_meshes(cfg)[l]
            th = 0.3 * W.random_nodal(cfg["seed"] + 1000 * l + i, 1, mesh.n_elems)[0]
            if cfg.get("model") == "iso":
                th = cfg["kl"]["mean"] * (1.0 + th)
            t0 = time.perf_counter()
            out = run.solve_theta(mesh, th, ph, lv["n_steps"], stop_after=steps, model=cfg.get("model"))
            el = time.perf_counter() - t0
    return mesh.n_nodes, steps, out["lin_iters"], el


def cpu_baseline(name, cfg, budget_s):
    """The oracle timed on the host's cores, sample-parallel: one process per core (at most 16, the
    GPU machine's share), one BLAS thread each, every worker solving seeded samples of the workload's
    levels (coarsest first, as many levels as the budget allows; the first CPU_STEPS steps of each
    solve).  Runs before the GPU is touched, so the pool can fork.  The oracle's iteration count is
    its own: Krylov iterations on meshes above its direct-solver size, one per Newton step where it
    factorises (so DOF·iters/s is not comparable with the GPU's; the space-time DOF rate is)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    levels = list(range(len(cfg["levels"])))
    done, per_level = [], {}
    t_all = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        for l in levels:
            # estimate the level's cost from the previous one before committing the pool to it
            if per_level and time.perf_counter() - t_all > 0.5 * budget_s:
                break
            t0 = time.perf_counter()
            res = pool.map(_cpu_job, [(name, l, i) for i in range(cores)], chunksize=1)
            el = time.perf_counter() - t0
            done += res
            n, steps = res[0][0], res[0][1]
            per_level[l] = dict(vertices=n, steps=steps, samples=len(res), wall_s=round(el, 2),
                                s_per_sample_step=round(sum(r[3] for r in res) / (len(res) * steps), 4))
            if time.perf_counter() - t_all + 5.0 * el > budget_s:  # the next level costs about 5x
                break
        pool.close()
        pool.join()  # every worker has exited before the GPU is touched
    wall = sum(v["wall_s"] for v in per_level.values())
    dof_iters = sum(r[0] * r[2] for r in done)
    st_dof = sum(r[0] * r[1] for r in done)
    desc = "; ".join(f"level {l}: {v['samples']} samples x first {v['steps']} steps, {v['vertices']} nodes"
                     for l, v in per_level.items())
    return dict(value=dof_iters / wall, unit="DOF·iters/s", cores=cores, kind="oracle",
                sample=f"{desc}; one process per core, one BLAS thread each; seeded fields in place of the KL "
                       f"field; {wall:.1f} s",
                st_dof_per_s=st_dof / wall, seconds=round(wall, 2), levels=per_level,
                iterations="the oracle's own: Krylov iterations above its direct-solver size, one per Newton "
                           "step where it factorises")


def kl_synthesis(runner, cfg, dev, reps=5):
    """Time the KL synthesis (MFMA contraction) of the finest level's batch: HIP events
    on the stream the binding launches on (torch's current stream)."""
    import torch

    import workloads as W
    l = len(runner.levels) - 1
    L = runner.levels[l]
    M = runner.n_modes
    samp = cfg["sampling"]
    if samp["kind"] == "combination":  # the finest level sees the points of Q_0
        B = samp["n_per_level"][0]
    else:
        B = samp["n_per_level"][l] * samp.get("n_shifts", 1)
    Y = torch.as_tensor(W.mc_normals(cfg["seed"], l, B, M), device=dev)
    theta = L.sample_fields(Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        L.sample_fields(Y, theta)
    e1.record()
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    P = L.n_elems
    wb = 4 if L.mixed else 8
    flops = 2.0 * P * M * B
    peak = 157.3 if L.mixed else 78.6  # dense MFMA TFLOP/s for the synthesis dtype
    gb = (P * M * wb + P * B * wb) / 1e9
    return dict(kernel="k_kl_mfma", dtype="f32" if L.mixed else "f64", shape=dict(elements=P, modes=M, samples=B),
                us=round(us, 2), tflops=round(flops / us / 1e6, 2), peak_tflops=peak,
                frac_mfma=round(flops / us / 1e6 / peak, 4), hbm_gbs=round(gb / us * 1e6, 1),
                frac_hbm=round(gb / us * 1e6 / HBM_PEAK_GBS, 4))


def make_step(cfg, runner, args, dev):
    """The estimator pass of the workload and its inputs (resident on the device)."""
    import torch

    import workloads as W
    samp = cfg["sampling"]
    M = runner.n_modes
    kind = samp["kind"]
    draw = W.mc_uniforms if cfg["kl"].get("variables") == "uniform" else W.mc_normals
    n_dims = M * int(cfg["kl"].get("components", 1))
    if kind == "combination":
        Yc = torch.as_tensor(draw(cfg["seed"], 0, max(samp["n_per_level"]), n_dims), device=dev)
        if args.fields:
            probes = field_probes(cfg, runner)
            return lambda: runner.run_combination_fields(Yc, probes=probes)
        return lambda: runner.run_combination(Yc)
    if kind in ("mc", "mlmc"):
        Ys = [torch.as_tensor(draw(cfg["seed"], l, n, n_dims), device=dev) for l, n in enumerate(samp["n_per_level"])]
        if kind == "mc":
            return lambda: runner.run_mc(Ys[0])
        if args.fields:
            probes = field_probes(cfg, runner)
            return lambda: runner.run_mlmc_fields(Ys, probes=probes)
        return lambda: runner.run_mlmc(Ys)
    S = samp.get("n_shifts", 1)
    shifts = [W.lattice_shifts(cfg["seed"], l, S, n_dims) for l in range(len(cfg["levels"]))]
    return lambda: runner.run_mlqmc(shifts)


def timed_passes(step, runner, steps, warmup, log, tag):
    """warmup untimed passes, then `steps` timed ones between two device synchronisations; the
    finest levels' apply launches are timed by HIP events on their streams meanwhile."""
    import torch
    for i in range(warmup):
        step()
        log(f"{tag}: warmup {i} done")
    for L in runner.levels:
        L.timing_enable(("apply",))
        L.timing_read(reset=True)
    runner.reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for i in range(steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"{tag}: {steps} timed passes, {el / steps:.3f} s each")
    per_level = []
    for l, L in enumerate(runner.levels):
        t = L.timing_read(reset=True)["apply"]
        per_level.append(dict(level=l, nodes=L.n_nodes, apply_ms=round(t["ms"], 3), apply_launches=t["launches"],
                              alg_bytes=round(t["bytes"]), kernel_bytes=round(t["kernel_bytes"]), units=t["units"]))
        L.timing_enable(())
    return el, res, per_level


def roofline_of(cfg, runner, config_name, prec, per_level):
    """The finest level's Jacobian apply, the kernel that carries most of the bytes: algorithmic
    bytes (every operand once: 16 B per node-sample in FP32 plus the fused projections' basis reads)
    over the summed HIP-event time of its launches."""
    import workloads as W
    top = per_level[-1]
    ms, launches = top["apply_ms"], max(top["apply_launches"], 1)
    alg, kb = float(top["alg_bytes"]), float(top["kernel_bytes"])
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    ratio = counter_traffic(config_name, "fp64" if prec == W.PREC_FP64 else "mixed", tet=runner.tet)
    lvl = cfg["levels"][-1]
    shape = (f"{lvl['cells'][0]}x{lvl['cells'][1]}x{lvl['cells'][2]} shell" if runner.tet
             else "x".join(map(str, lvl["n"])))
    kernel = ("k_tet_apply (Jacobian apply on the padded slot-major P1 pattern)" if runner.tet else
              "k_wave3 (preconditioned Jacobian apply + fused projections)" if cfg["dim"] == 3 else
              "k_apply_pk (2D preconditioned Jacobian apply)")
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=None if ratio is None else round(ratio * kb / launches),
                kernel=f"{kernel}, finest level ({shape})",
                alg_bytes_per_launch=round(alg / launches), alg_bytes_per_unit=round(alg / max(top["units"], 1.0), 2),
                kernel_bytes_per_launch=round(kb / launches),
                frac_kernel_bytes=round(kb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms > 0 else 0.0,
                avg_launch_us=round(1e3 * ms / launches, 2), launches=top["apply_launches"])


def level_stats(runner, steps):
    """Per level: its solves' DOF x iterations over their host wall time (the coarser levels run
    concurrently, so their rates are while sharing the GPU), Newton and GMRES iterations per step
    (per time block in the all-at-once mode)."""
    out = []
    for l, L in enumerate(runner.levels):
        mb = min(runner.steps_per_block, int(L.desc.n_steps)) if runner.steps_per_block else 1
        units = max(runner.level_sample_steps[l] / mb, 1.0)
        out.append(dict(level=l, dof_iters_per_s=(runner.level_dof_iters[l] / runner.level_seconds[l]
                                                  if runner.level_seconds[l] > 0 else None),
                        seconds=round(runner.level_seconds[l] / max(steps, 1), 4),
                        **{("newton_per_block" if mb > 1 else "newton_per_step"):
                           round(runner.level_newton[l] / units, 3),
                           ("gmres_per_block" if mb > 1 else "gmres_per_step"): round(runner.level_inner[l] / units, 2)}))
    return out


def compare_runs(cfg, a, b):
    """Mixed-precision estimator a against the FP64 one b on the same sample plan: relative
    differences of the estimate, the level means and every per-sample QoI, also relative to the
    informative part T - QoI of the censored mean activation time."""
    import numpy as np
    T = cfg["physics"]["t_end"]
    est_a, est_b = a["estimate"], b["estimate"]
    out = dict(estimate_mixed=est_a, estimate_fp64=est_b, estimate_rel_diff=abs(est_a - est_b) / abs(est_b))
    if cfg["qoi"] == 1:
        out["estimate_diff_rel_to_T_minus_qoi"] = abs(est_a - est_b) / abs(T - est_b)
    lm = [abs(x - y) / abs(y) for x, y in zip(a["level_mean"], b["level_mean"]) if y != 0.0]
    out["level_mean_max_rel_diff"] = max(lm) if lm else 0.0
    # the level means of the finer levels are differences F_l - F_(l-1), small against the estimate
    la = [abs(x - y) for x, y in zip(a["level_mean"], b["level_mean"])]
    out["level_mean_max_abs_diff"] = max(la) if la else 0.0
    out["level_mean_max_diff_rel_to_estimate"] = (max(la) / abs(est_b)) if la and est_b != 0.0 else 0.0
    diffs, scale = [], []
    for fa, fb in [(a["f_fine"], b["f_fine"]), (a.get("f_coarse") or [], b.get("f_coarse") or [])]:
        for x, y in zip(fa, fb):
            if x is None or y is None:
                continue
            x, y = np.asarray(x), np.asarray(y)
            diffs.append(np.abs(x - y).max())
            scale.append(np.abs(y).min())
    out["per_sample_max_abs_diff"] = float(max(diffs)) if diffs else 0.0
    out["per_sample_max_rel_diff"] = float(max(d / s for d, s in zip(diffs, scale))) if diffs else 0.0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--prec", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--companion-steps", type=int, default=3,
                    help="timed passes of the FP64 companion of a mixed-precision run (0: no companion)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown", action="store_true", help="extra untimed pass timing every kernel class")
    ap.add_argument("--newton-guess", choices=["previous", "extrapolate", "reference", "reference-local"],
                    default="extrapolate",
                    help="Newton initial guess of each step: u_k, 2 u_k - u_(k-1), or from the unperturbed "
                         "reference solution (global r_(k+1), or local u_k + r_(k+1) - r_k)")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative residual at which GMRES stops (default 1e-4; mixed boxes 1e-3)")
    ap.add_argument("--fields", action="store_true",
                    help="MLMC workloads: also estimate the field quantities of interest (mean space-time "
                         "potential on the finest grid, mean activation map, mean action potential at 4 points)")
    ap.add_argument("--steps-per-block", type=int, default=0,
                    help="all-at-once solves in time blocks of this many steps (0: time stepping)")
    ap.add_argument("--block-guess", choices=["previous", "reference", "reference-local"], default="previous",
                    help="Newton start of a time block: the previous block's final state (multiple time blocks), "
                         "the reference solution (global) or its increment (local)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch autotuner (lane layout by grid width, one GMRES launch sequence per "
                         "iteration, whole batches)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB FP64 copy (torch.neg) before warm-up, as a counter reference")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(samples would shard across GPUs with one all-reduce of the estimator sums).", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    cfg = W.config(args.config)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:  # before any GPU call: the worker pool forks
        log("timing the CPU oracle")
        cpu = cpu_baseline(args.config, cfg, args.cpu_seconds)
        log(f"CPU oracle: {cpu['sample']}")

    import torch

    from paper_2105_02007_amd import mlq
    from paper_2105_02007_amd.driver import ConfigRunner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda:0"
    prec = cfg["prec"] if args.prec is None else (W.PREC_FP64 if args.prec == "fp64" else W.PREC_MIXED)
    guess = {"previous": mlq.MLQ_GUESS_PREVIOUS, "extrapolate": mlq.MLQ_GUESS_EXTRAPOLATE,
             "reference": mlq.MLQ_GUESS_REFERENCE, "reference-local": mlq.MLQ_GUESS_REFERENCE_LOCAL}[args.newton_guess]
    t_setup = time.perf_counter()
    bguess = {"previous": mlq.MLQ_GUESS_PREVIOUS, "reference": mlq.MLQ_GUESS_REFERENCE,
              "reference-local": mlq.MLQ_GUESS_REFERENCE_LOCAL}[args.block_guess]
    if args.steps_per_block > 0:
        args.no_tune = True
        args.companion_steps = 0
    runner = ConfigRunner(cfg, prec=prec, device=dev, log=log, newton_guess=guess, inner_tol=args.inner_tol,
                          tune_launch=not args.no_tune, steps_per_block=args.steps_per_block, block_guess=bguess)
    t_setup = time.perf_counter() - t_setup
    log(f"set-up done in {t_setup:.1f} s (KL {runner.kl_method}, rank {runner.kl_rank})")
    runner.log = log
    samp = cfg["sampling"]
    step = make_step(cfg, runner, args, dev)
    if args.fields:
        runner.prepare_fields(field_probes(cfg, runner))
        log("field transfer set-up done")
    if args.copy_calibration:
        src = torch.ones(COPY_ELEMS, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    el, res, per_level = timed_passes(step, runner, args.steps, args.warmup, log, "main")
    dof_iters, st_dof = runner.dof_iters, runner.st_dof
    roofline = roofline_of(cfg, runner, args.config, prec, per_level)
    for p_ in per_level:
        p_.pop("units")
    levels = level_stats(runner, args.steps)

    breakdown = None
    if args.breakdown:
        for L in runner.levels:
            L.timing_enable(tuple(mlq.KERNEL_CLASSES))
        torch.cuda.synchronize()
        tb = time.perf_counter()
        step()
        torch.cuda.synchronize()
        tb = time.perf_counter() - tb
        tot = {}
        for L in runner.levels:
            for c, v in L.timing_read(reset=True).items():
                tot[c] = tot.get(c, 0.0) + v["ms"]
            L.timing_enable(())
        breakdown = dict(wall_ms=round(tb * 1e3, 1), kernel_ms={c: round(v, 2) for c, v in tot.items()})

    launch_tuning = None
    if not args.no_tune:
        # the same pass once more with every level at the untuned configuration
        from paper_2105_02007_amd import tune
        tuned = [dict(L.tuning) for L in runner.levels]
        for L in runner.levels:
            box3 = L.desc.mesh_kind == mlq.MLQ_MESH_Q1_BOX and L.desc.dim == 3
            tune.apply_config(L, dict(lanes_x=(16 if L.desc.n[0] >= 48 else 8) if box3 else 0, gmres_block=0,
                                      chunk=int(L.desc.max_batch)))
        torch.cuda.synchronize()
        tu = time.perf_counter()
        step()
        torch.cuda.synchronize()
        tu = time.perf_counter() - tu
        for L, t in zip(runner.levels, tuned):
            tune.apply_config(L, t)
        launch_tuning = dict(
            tuned_pass_s=round(el / args.steps, 4), untuned_pass_s=round(tu, 4),
            levels=[dict(level=l, lanes_x=t["lanes_x"], gmres_block=t["gmres_block"], chunk=t["chunk"],
                         cached=t.get("cached", False), trials_ms=t.get("trials_ms"))
                    for l, t in enumerate(tuned)])
        log(f"untuned pass {tu:.3f} s, tuned {el / args.steps:.3f} s")

    has_rmse = not (samp["kind"] == "combination" or (samp["kind"] in ("qmc", "mlqmc") and samp.get("n_shifts", 1) < 2))
    line = {
        "metric": METRIC, "value": dof_iters / el, "unit": "DOF·iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == W.PREC_FP64 else "f32+f64",
        "data": "synthetic (seeded KL random fields; MC normal or uniform coordinates, shifted rank-1 "
                "lattice or Halton points)",
        "config": {"workload": f"{args.config}: {WORKLOAD_TEXT[args.config]}", "levels": len(cfg["levels"]),
                   "samples_per_level": samp["n_per_level"], "n_shifts": samp.get("n_shifts", 1),
                   "precision": "mixed: FP32 KL synthesis, operator and Krylov; FP64 residual, Newton update, QoIs "
                                "and estimator" if prec == W.PREC_MIXED else "FP64 throughout",
                   "parallelism": "single GPU, samples batched per level"},
        "st_dof_per_s": st_dof / el,
        "estimate": res["estimate"],
        # no error estimate: the combination form over nested point sets, or a QMC rule with one shift
        "rmse_est": res["rmse"] if has_rmse else None,
        "level_means": res["level_mean"],
        "kl": {"method": runner.kl_method, "rank": runner.kl_rank,
               ("eig_resid" if runner.kl_method == "exact" else "trace_resid"): runner.kl_resid},
        "setup_s": round(t_setup, 2),
        "roofline": roofline,
        "apply_per_level": per_level,
        "levels": levels,
        "newton_guess": args.newton_guess,
        "time_blocks": ({"steps_per_block": args.steps_per_block, "block_guess": args.block_guess}
                        if args.steps_per_block > 0 else None),
        "lanes_x": [getattr(L, "lanes_x", None) for L in runner.levels],
        "inner_tol": runner.levels[-1].desc.inner_tol,
    }
    if launch_tuning:
        line["launch_tuning"] = launch_tuning
    if args.fields:
        line["fields"] = fields_summary(cfg, runner, res, dev)
    if breakdown:
        line["breakdown"] = breakdown
    line["kl_synthesis"] = kl_synthesis(runner, cfg, dev)
    runner.log = None
    if prec == W.PREC_MIXED and args.companion_steps > 0:
        # the FP64 GPU path on the same sample plan: the same estimator to the same RMSE
        del runner, step
        torch.cuda.empty_cache()
        t64 = time.perf_counter()
        r64 = ConfigRunner(cfg, prec=W.PREC_FP64, device=dev, log=log, newton_guess=guess,
                           tune_launch=not args.no_tune)
        t64 = time.perf_counter() - t64
        step64 = make_step(cfg, r64, args, dev)
        el64, res64, pl64 = timed_passes(step64, r64, args.companion_steps, 1, log, "fp64 companion")
        cmp_ = compare_runs(cfg, res, res64)
        mixed_s, fp64_s = el / args.steps, el64 / args.companion_steps
        line["time_to_rmse"] = dict(
            rmse_mixed=res["rmse"] if has_rmse else None, rmse_fp64=res64["rmse"] if has_rmse else None,
            mixed_s=round(mixed_s, 4), fp64_s=round(fp64_s, 4), fp64_over_mixed=round(fp64_s / mixed_s, 3),
            fp64_passes=args.companion_steps, fp64_value=r64.dof_iters / el64, fp64_setup_s=round(t64, 2),
            fp64_apply_frac=roofline_of(cfg, r64, args.config, W.PREC_FP64, pl64)["frac"],
            **cmp_)
        del r64, step64
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def fields_summary(cfg, runner, res, dev):
    """Field quantities of interest of --fields: grid sizes, the mean action potential at the probes,
    and on boxes the domain mean of the activation map against the scalar estimate."""
    import torch
    eu, ep = res["mean_u"], res["mean_probe"]
    out = {"u_grid": list(eu.shape), "u_bytes": eu.numel() * 8,
           "mean_action_potential": {f"{f:g}T": [float(x) for x in ep[:, int(round(f * (ep.shape[1] - 1)))].cpu()]
                                     for f in (0.25, 0.5, 1.0)}}
    if runner.tet:
        out["probes"] = [list(map(float, p)) for p in field_probes(cfg, runner)]
        return out
    # the domain mean of the estimated activation map equals the scalar estimate (the transfer is
    # the Q1 interpolant, which the lumped node weights integrate exactly)
    fl = cfg["levels"][-1]
    w1 = []
    for a in range(cfg["dim"]):
        h = (fl["hi"][a] - fl["lo"][a]) / (fl["n"][a] - 1)
        v = torch.full((fl["n"][a],), h, dtype=torch.float64, device=dev)
        v[0] = v[-1] = 0.5 * h
        w1.append(v)
    wts = w1[0]
    for v in w1[1:]:
        wts = (v[:, None] * wts[None, :]).reshape(-1)
    act_mean = float((wts * res["mean_act_map"]).sum() / wts.sum())
    out.update(act_map_domain_mean=act_mean, act_map_mean_minus_estimate=act_mean - res["estimate"],
               level_term_norms_l2_h1=res["level_term_norms"], probes=FIELD_PROBES)
    return out


if __name__ == "__main__":
    main()
