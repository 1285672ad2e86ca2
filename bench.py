#!/usr/bin/env python3
"""Throughput of the batched space-time solves on one MI355X.

One step = one pass of the whole path over one batch of synthetic input: the
configured estimator end to end (sample points, KL synthesis, Crank-Nicolson /
Newton / GMRES solves on every level and the coarse partner level, QoIs,
level differences, estimator).  The KL basis and level set-up are one-time
set-up outside the timed region; Monte Carlo normals are inputs and are
resident in HBM before timing starts.

Prints one JSON line (rank 0).  Metric: space-time DOF x inner iterations per
second = sum over samples, steps and Newton iterations of n_l * (GMRES
iterations), over wall time.
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
# algorithmic bytes per node-sample of the preconditioned Jacobian apply
# w = v_j / eta_j + dt/2 K z: z, v_j and the two element coefficients (one
# element per node) read, w written, in the inner precision
APPLY_BYTES = {0: 5 * 8, 1: 5 * 4}
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
    "c5": "non-nested prolate-ellipsoidal shell, P1 tetrahedra 26k/187k/1.4M vertices, 512 steps, 256-mode KL "
          "(l = 0.1 long axis), rule-based +60/-60 deg fibres, combination estimator 16/64/256 nested MC points, "
          "mean activation time",
    "c5i": "the c5 shells with the paper's idealised-ventricle model: isotropic G = max(v, 0.1 E[V]) I, "
           "v = E[V] + W, W a squared-exponential KL field (0.3 E[V], sigma_KL = 0.5) with 87 uniform "
           "coordinates, combination estimator 16/64/256 nested MC points, mean activation time",
    "c5v": "the c5 shells with the paper's heart model: eq. (AdmV) with a random vector field V = sigma_l f0 + W, "
           "W three independent squared-exponential KL fields (0.3 sigma_l, sigma_KL = 0.64), 3 x 45 uniform "
           "coordinates, combination estimator 16/64/256 nested MC points, mean activation time",
}


def cpu_baseline_tet(cfg, budget_s):
    """The oracle on the coarsest shell: one sample (rule-based angle or mean vector field plus
    a seeded random perturbation in place of the KL field), as many steps as the budget allows."""
    import numpy as np

    import workloads as W
    from oracle import stepper
    from oracle.tetfem import TetMesh
    lv = cfg["levels"][0]
    m = W.tet_mesh(lv)
    mesh = TetMesh(m["xyz"], m["tets"])
    ph = cfg["physics"]
    if cfg.get("model") == "vector":  # E[V] plus a seeded perturbation of each component
        from oracle import fem
        f0 = np.cos(m["theta0"])[:, None] * m["e_circ"] + np.sin(m["theta0"])[:, None] * m["e_long"]
        V = ph["sigma_l"] * (f0 + 0.3 * W.random_nodal(cfg["seed"], 3, mesh.n_elems).T)
        G = fem.conductivity(V, ph["sigma_t"])
    elif cfg.get("model") == "iso":  # E[V] times a seeded perturbation, bounded below
        from oracle import fem
        v = cfg["kl"]["mean"] * (1.0 + 0.3 * W.random_nodal(cfg["seed"], 1, mesh.n_elems)[0])
        G = fem.conductivity_iso(v, 3, ph["sigma_t"])
    else:
        th = m["theta0"] + 0.3 * W.random_nodal(cfg["seed"], 1, mesh.n_elems)[0]
        G = mesh.conductivity(th, m["e_circ"], m["e_long"], ph["sigma_l"], ph["sigma_t"])
    t0 = time.perf_counter()
    steps = 2
    while True:  # grow the step count until the budget is used (each run starts from u = 0)
        t1 = time.perf_counter()
        out = stepper.solve(mesh, G, ph, lv["n_steps"], tol=1e-13, stop_after=steps)
        el = time.perf_counter() - t1
        if time.perf_counter() - t0 + 2.5 * el > budget_s or steps >= lv["n_steps"]:
            break
        steps *= 2
    n = mesh.n_nodes
    return dict(value=n * out["lin_iters"] / el, unit="DOF·iters/s", cores=1, kind="oracle",
                sample=f"1 sample of level 0 ({n} vertices, first {steps} of {lv['n_steps']} steps); single process; "
                       f"GMRES iterations; KL set-up excluded (seeded perturbation of the rule-based angle); {el:.1f} s",
                st_dof_per_s=n * steps / el, seconds=el)


def cpu_baseline(cfg, budget_s):
    """The oracle on a bounded sample of the same workload (level 0 and 1 samples of its first two levels)."""
    import numpy as np

    import workloads as W
    from oracle import run
    if cfg["levels"][0].get("kind") == "tet":
        return cpu_baseline_tet(cfg, budget_s)
    meshes = run.level_meshes(cfg)
    B = run.kl_basis(cfg, meshes, max_rank=2 * cfg["kl"]["n_modes"])
    M = cfg["kl"]["n_modes"]
    phys = cfg["physics"]
    dof_iters, st_dof, n_solves = 0.0, 0.0, 0
    t0 = time.perf_counter()
    # level 0 and level 1 samples, interleaved so that a cut at the budget keeps both
    plan = [(0, i) for i in range(8)]
    if len(meshes) > 1:
        for i in range(8):
            plan += [(1, i), (0, 8 + i)]
    done = []
    draw = W.mc_uniforms if cfg["kl"].get("variables") == "uniform" else W.mc_normals
    for l, i in plan:
        if time.perf_counter() - t0 > budget_s:
            break
        Y = draw(cfg["seed"], l, i + 1, M)[:, i:i + 1]
        th = run.sample_theta(B["phi"][l], B["sqrt_lam"], Y, run.level_theta0(cfg, meshes[l]))[0]
        out = run.solve_theta(meshes[l], th, phys, cfg["levels"][l]["n_steps"], model=cfg.get("model"))
        n = meshes[l].n_nodes
        dof_iters += n * out["lin_iters"]
        st_dof += n * cfg["levels"][l]["n_steps"]
        n_solves += 1
        done.append(l)
    el = time.perf_counter() - t0
    counts = {l: done.count(l) for l in sorted(set(done))}
    desc = ", ".join(f"{c} sample(s) of level {l} ({'x'.join(map(str, cfg['levels'][l]['n']))} nodes, "
                     f"{cfg['levels'][l]['n_steps']} steps)" for l, c in counts.items())
    return dict(value=dof_iters / el, unit="DOF·iters/s", cores=1, kind="oracle",
                sample=f"{desc}; single process; a direct sparse solve counts as one iteration, "
                       f"GMRES iterations otherwise; KL set-up excluded; {el:.1f} s",
                st_dof_per_s=st_dof / el, seconds=el)


def qoi_vs_fp64(cfg, runner, res, dev, log, Ys=None, Yc=None, shifts=None, nq=4):
    """The first nq samples of the finest level re-solved by the FP64 path (the same KL
    set-up and the same points), against the mixed run's QoIs of those samples.  The FP64
    path itself is pinned to the oracle (1e-10 per QoI) by the parity tests."""
    import numpy as np
    import torch

    from paper_2105_02007_amd import mlq
    from paper_2105_02007_amd.driver import ConfigRunner
    L = len(cfg["levels"]) - 1
    samp = cfg["sampling"]
    if samp["kind"] == "combination":
        Y = Yc
    elif samp["kind"] in ("mc", "mlmc"):
        Y = Ys[L]
    else:
        Y = runner.qmc_points(L, shifts[L])
    nq = min(nq, Y.shape[1])
    Y = Y[:, :nq].contiguous()
    mixed_q = np.asarray(res["f_fine"][L][:nq])
    log(f"FP64 re-solve of {nq} finest-level samples")
    t0 = time.perf_counter()
    r64 = ConfigRunner(cfg, prec=mlq.MLQ_FP64, device=dev, concurrent=False)
    q64 = r64.solve(L, Y).cpu().numpy()
    el = time.perf_counter() - t0
    del r64
    torch.cuda.empty_cache()
    rel = np.abs(mixed_q - q64) / np.abs(q64)
    return dict(level=L, samples=nq, max_rel_diff=float(rel.max()), mean_rel_diff=float(rel.mean()),
                fp64_seconds=round(el, 1),
                reference="FP64 GPU solve of the same samples (the FP64 path is pinned to the oracle at 1e-10)")


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--prec", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown", action="store_true", help="extra untimed pass timing every kernel class")
    ap.add_argument("--no-qoi-check", action="store_true",
                    help="skip the FP64 re-solve of a few finest-level samples after a mixed-precision run")
    ap.add_argument("--newton-guess", choices=["previous", "extrapolate", "reference", "reference-local"],
                    default="extrapolate",
                    help="Newton initial guess of each step: u_k, 2 u_k - u_(k-1), or from the unperturbed "
                         "reference solution (global r_(k+1), or local u_k + r_(k+1) - r_k)")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="relative residual at which GMRES stops (default 1e-4; mixed boxes 1e-3)")
    ap.add_argument("--fields", action="store_true",
                    help="MLMC workloads: also estimate the field quantities of interest (mean space-time "
                         "potential on the finest grid, mean activation map, mean action potential at 4 points)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB FP64 copy (torch.neg) before warm-up, as a counter reference")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(samples would shard across GPUs with one all-reduce of the estimator sums).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2105_02007_amd import mlq
    from paper_2105_02007_amd.driver import ConfigRunner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda:0"
    cfg = W.config(args.config)
    prec = cfg["prec"] if args.prec is None else (W.PREC_FP64 if args.prec == "fp64" else W.PREC_MIXED)
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    t_setup = time.perf_counter()
    guess = {"previous": mlq.MLQ_GUESS_PREVIOUS, "extrapolate": mlq.MLQ_GUESS_EXTRAPOLATE,
             "reference": mlq.MLQ_GUESS_REFERENCE, "reference-local": mlq.MLQ_GUESS_REFERENCE_LOCAL}[args.newton_guess]
    runner = ConfigRunner(cfg, prec=prec, device=dev, log=log, newton_guess=guess, inner_tol=args.inner_tol)
    t_setup = time.perf_counter() - t_setup
    log(f"set-up done in {t_setup:.1f} s (KL rank {runner.kl_rank})")
    runner.log = log
    samp = cfg["sampling"]
    M = runner.n_modes
    kind = samp["kind"]
    Ys = Yc = shifts = None
    draw = W.mc_uniforms if cfg["kl"].get("variables") == "uniform" else W.mc_normals
    n_dims = M * int(cfg["kl"].get("components", 1))
    if kind == "combination":
        Yc = torch.as_tensor(draw(cfg["seed"], 0, max(samp["n_per_level"]), n_dims), device=dev)
        if args.fields:
            probes = field_probes(cfg, runner)
            step = lambda: runner.run_combination_fields(Yc, probes=probes)
        else:
            step = lambda: runner.run_combination(Yc)
    elif kind in ("mc", "mlmc"):
        Ys = [torch.as_tensor(draw(cfg["seed"], l, n, n_dims), device=dev)
              for l, n in enumerate(samp["n_per_level"])]
        if kind == "mc":
            step = lambda: runner.run_mc(Ys[0])
        elif args.fields:
            probes = field_probes(cfg, runner)
            step = lambda: runner.run_mlmc_fields(Ys, probes=probes)
        else:
            step = lambda: runner.run_mlmc(Ys)
    else:
        S = samp.get("n_shifts", 1)
        shifts = [W.lattice_shifts(cfg["seed"], l, S, n_dims) for l in range(len(cfg["levels"]))]
        step = lambda: runner.run_mlqmc(shifts)

    if args.fields:
        runner.prepare_fields(field_probes(cfg, runner))
        log("field transfer set-up done")
    if args.copy_calibration:
        src = torch.ones(COPY_ELEMS, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        step()
        log(f"warmup {i} done")
    for L in runner.levels:
        L.timing_enable(("apply",))
        L.timing_read(reset=True)
    runner.reset_counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dof_iters, st_dof = runner.dof_iters, runner.st_dof

    # dominant kernel: the Jacobian apply of the finest level (most of the bytes; its solves
    # run with the GPU to themselves, the coarser levels' solves share it with each other)
    per_level = []
    for l, L in enumerate(runner.levels):
        t = L.timing_read(reset=True)["apply"]
        per_level.append(dict(level=l, nodes=L.n_nodes, apply_ms=round(t["ms"], 3), apply_launches=t["launches"],
                              alg_bytes=round(t["bytes"]), units=t["units"]))
        L.timing_enable(())
    top = per_level[-1]
    apply_ms, apply_bytes, apply_units, apply_launches = (top["apply_ms"], float(top["alg_bytes"]), top["units"],
                                                          top["apply_launches"])
    # the library reports the algorithmic bytes of every apply launch (with the
    # Gram-Schmidt projections fused in, the basis vectors they read count too)
    alg_bytes = apply_bytes if apply_bytes > 0 else apply_units * APPLY_BYTES[prec]
    per_launch = alg_bytes / max(apply_launches, 1)
    achieved = alg_bytes / (apply_ms * 1e-3) / 1e9 if apply_ms > 0 else 0.0
    ratio = counter_traffic(args.config, "fp64" if prec == W.PREC_FP64 else "mixed", tet=runner.tet)
    lvl = cfg["levels"][-1]
    shape = (f"{lvl['cells'][0]}x{lvl['cells'][1]}x{lvl['cells'][2]} shell" if runner.tet
             else "x".join(map(str, lvl["n"])))
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if ratio is None else round(ratio * per_launch),
                    kernel=("k_tet_apply (Jacobian apply on the padded slot-major P1 pattern)"
                            if runner.tet else
                            "k_wave3 (preconditioned Jacobian apply + fused projections)"
                            if cfg["dim"] == 3 else
                            "k_apply_pk (2D preconditioned Jacobian apply)") + f", finest level ({shape})",
                    bytes_per_node_sample=round(alg_bytes / max(apply_units, 1.0), 2),
                    alg_bytes_per_launch=round(per_launch),
                    alg_bytes_total=round(alg_bytes),
                    avg_launch_us=round(1e3 * apply_ms / max(apply_launches, 1), 2),
                    launches=apply_launches)
    for p_ in per_level:
        p_.pop("units")

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

    line = {
        "metric": METRIC, "value": dof_iters / el, "unit": "DOF·iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == W.PREC_FP64 else "f32+f64",
        "data": "synthetic (seeded KL random fields; MC normal or uniform coordinates, shifted rank-1 "
                "lattice or Halton points)",
        "config": {"workload": f"{args.config}: {WORKLOAD_TEXT[args.config]}", "levels": len(cfg["levels"]),
                   "samples_per_level": samp["n_per_level"], "n_shifts": samp.get("n_shifts", 1),
                   "parallelism": "single GPU, samples batched per level"},
        "st_dof_per_s": st_dof / el,
        # no error estimate: the combination form over nested point sets, or a QMC rule
        # with a single random shift
        "estimate": res["estimate"],
        "rmse_est": None if samp["kind"] == "combination" or (samp["kind"] in ("qmc", "mlqmc")
                                                            and samp.get("n_shifts", 1) < 2) else res["rmse"],
        "level_means": res["level_mean"],
        "kl": {"rank": runner.kl_rank, "trace_resid": runner.kl_resid},
        "setup_s": round(t_setup, 2),
        "roofline": roofline,
        "apply_per_level": per_level,
    }
    if args.fields and runner.tet:
        eu, ep = res["mean_u"], res["mean_probe"]
        line["fields"] = {
            "u_grid": list(eu.shape), "u_bytes": eu.numel() * 8,
            "probes": [list(map(float, p)) for p in field_probes(cfg, runner)],
            "mean_action_potential": {f"{f:g}T": [float(x) for x in ep[:, int(round(f * (ep.shape[1] - 1)))].cpu()]
                                      for f in (0.25, 0.5, 1.0)},
        }
    elif args.fields:
        # the domain mean of the estimated activation map equals the scalar estimate (the
        # transfer is the Q1 interpolant, which the lumped node weights integrate exactly)
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
        ea, eu, ep = res["mean_act_map"], res["mean_u"], res["mean_probe"]
        act_mean = float((wts * ea).sum() / wts.sum())
        line["fields"] = {
            "u_grid": list(eu.shape), "u_bytes": eu.numel() * 8,
            "act_map_domain_mean": act_mean,
            # per level: ||mean_0|| and ||mean_l - T mean_(l-1)|| in L^2((0,T); L^2), L^2((0,T); H^1)
            "level_term_norms_l2_h1": res["level_term_norms"],
            "act_map_mean_minus_estimate": act_mean - res["estimate"],
            "probes": FIELD_PROBES,
            # the mean action potential at the probes at a quarter, half and all of [0, T]
            "mean_action_potential": {f"{f:g}T": [float(x) for x in ep[:, int(round(f * (ep.shape[1] - 1)))].cpu()]
                                      for f in (0.25, 0.5, 1.0)},
        }
    # per level: its solves' DOF x iterations over their host wall time (the coarser levels
    # run concurrently, so their rates are while sharing the GPU)
    line["levels"] = [dict(level=l, dof_iters_per_s=(runner.level_dof_iters[l] / runner.level_seconds[l]
                                                     if runner.level_seconds[l] > 0 else None),
                           seconds=round(runner.level_seconds[l] / max(args.steps, 1), 4),
                           newton_per_step=round(runner.level_newton[l] / runner.level_sample_steps[l], 3),
                           gmres_per_step=round(runner.level_inner[l] / runner.level_sample_steps[l], 2))
                      for l in range(len(runner.levels))]
    line["newton_guess"] = args.newton_guess
    line["lanes_x"] = [getattr(L, "lanes_x", None) for L in runner.levels]
    line["inner_tol"] = runner.levels[-1].desc.inner_tol
    if breakdown:
        line["breakdown"] = breakdown
    line["kl_synthesis"] = kl_synthesis(runner, cfg, dev)
    if prec == W.PREC_MIXED and not args.no_qoi_check and not runner.tet:
        line["qoi_vs_fp64"] = qoi_vs_fp64(cfg, runner, res, dev, log, Ys, Yc, shifts)
    runner.log = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
