"""Workload driver: sets a configuration up and runs its estimator through the C ABI.

Host orchestration only (which level, which batch, in which order); the KL
basis, field synthesis, solves, lattice points, level differences and
estimators all run in libmlq (HIP kernels, or its host C++ for the estimator
sums).  Random numbers of Monte Carlo sampling (standard normals) and the
random shifts of lattice rules are inputs, passed in by the caller.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

import workloads as W

from . import mlq, tune

EST_OF = {"mc": mlq.MLQ_EST_MC, "qmc": mlq.MLQ_EST_MLQMC, "mlmc": mlq.MLQ_EST_MLMC, "mlqmc": mlq.MLQ_EST_MLQMC}


class ConfigRunner:
    """Levels of one workload with their KL bases (Section 2.3) on one device."""

    def __init__(self, cfg: dict, prec: int | None = None, device="cuda", newton_tol=None, inner_tol=None,
                 max_inner=30, kl_rank_factor=2, kl_eps=1e-2, kl_method=None, kl_tol=1e-8, log=None,
                 concurrent=True,
                 newton_guess=mlq.MLQ_GUESS_EXTRAPOLATE, tune_layout=True, tune_launch=True, steps_per_block=0,
                 block_guess=mlq.MLQ_GUESS_PREVIOUS):
        say = log if log is not None else (lambda m: None)
        self.cfg = cfg
        self.device = device
        self.prec = cfg["prec"] if prec is None else prec
        self.phys = cfg["physics"]
        kcfg = cfg["kl"]
        M = kcfg["n_modes"]
        kl_level = cfg["levels"][kcfg["grid_level"]]
        self.tet = kl_level.get("kind") == "tet"
        # the paper's vector model: `components` independent fields with the same KL basis
        # (block-diagonal covariance), uniform coordinates (modes scaled by sqrt(3 lambda))
        self.vector = cfg.get("model") == "vector"
        self.components = int(kcfg.get("components", 1))
        self.uniform = kcfg.get("variables") == "uniform"
        cov = mlq.MLQ_COV_SQEXP if kcfg.get("kernel") == "sqexp" else mlq.MLQ_COV_EXP
        self.iso = cfg.get("model") == "iso"
        # the KL standard deviation is relative to sigma_l (vector model) or E[V] (isotropic)
        std = kcfg["std"] * (self.phys["sigma_l"] if self.vector else kcfg["mean"] if self.iso else 1.0)
        # the KL route: "cholesky" (pivoted Cholesky, eq. (redEig)) or "exact" (the top M
        # eigenpairs of eq. (algEig) to the relative residual kl_tol; Q1 boxes only)
        method = kl_method if kl_method is not None else kcfg.get("method", "cholesky")
        if method not in ("cholesky", "exact") or (method == "exact" and self.tet):
            raise ValueError(f"KL method {method!r} is not available for this workload")
        def make_kd(m, max_rank, route="cholesky"):
            if self.tet:
                return mlq.kl_desc_tet(self.meshes[kcfg["grid_level"]], std, kcfg["corr_len"], m,
                                       max_rank=max_rank, eps=kl_eps, cov_kernel=cov)
            exact = route == "exact"
            return mlq.kl_desc(cfg["dim"], kl_level["n"], kl_level["lo"], kl_level["hi"], std,
                               kcfg["corr_len"], m, max_rank=max_rank, eps=kl_tol if exact else kl_eps,
                               cov_kernel=cov, method=mlq.MLQ_KL_EXACT if exact else mlq.MLQ_KL_CHOLESKY)
        if self.tet:
            # tetrahedral levels: the seeded shells of the workload (non-nested), the KL on
            # the vertices of the finest one, the transfer by point location
            self.meshes = [W.tet_mesh(lv) for lv in cfg["levels"]]
        if M == 0:
            # the stochastic dimension from the truncation tolerance (Section 5.1)
            n_kl = self.meshes[kcfg["grid_level"]]["xyz"].shape[0] if self.tet else int(np.prod(kl_level["n"]))
            M, resid = mlq.kl_dimension(make_kd(0, min(256, n_kl)), device=device)
            if resid > kl_eps:
                raise ValueError(f"the truncation tolerance {kl_eps} needs more than {M} modes")
            say(f"stochastic dimension M = {M} (trace residual {resid:.4f})")
        self.n_modes = M
        # all-at-once solves in time blocks of steps_per_block steps (0: time stepping); the block
        # GMRES needs about that many more iterations than one step
        self.steps_per_block = int(steps_per_block)
        self.block_guess = block_guess
        if self.steps_per_block > 0:
            max_inner = min(64, max_inner + self.steps_per_block)
            tune_launch = False
        self.kl_method = method
        self.kd = make_kd(M, kl_rank_factor * M, method)
        say(f"KL set-up ({method})")
        # kl_resid: the trace residual of the Cholesky factor, or the largest relative
        # eigen-residual of the exact modes
        lam, psi, self.kl_rank, self.kl_resid = mlq.kl_modes(self.kd, device=device)
        say(f"KL modes done (rank {self.kl_rank})")
        self.lam = lam
        sl = torch.as_tensor(mlq.kl_weights(lam, uniform=self.uniform), dtype=torch.float64, device=device)
        self.levels = []
        samp = cfg["sampling"]
        n_shifts = samp.get("n_shifts", 1)
        top = len(cfg["levels"]) - 1
        for l, lv in enumerate(cfg["levels"]):
            if samp["kind"] == "combination":
                # level j is evaluated on the points of Q_{L-j}
                nb = samp["n_per_level"][top - l]
            else:
                # the batch a level sees: its own samples and, as the coarse side, level l+1's,
                # solved together (solve_all merges the jobs of one level)
                nb = samp["n_per_level"][l] * n_shifts
                if l + 1 < len(cfg["levels"]):
                    nb += samp["n_per_level"][l + 1] * n_shifts
            theta0 = v_mean = None
            if self.tet:
                mesh = self.meshes[l]
                lv = dict(lv, mesh=mesh)
                phi = mlq.kl_transfer_tet(self.kd, psi, mesh, device=device)
                if self.vector:  # E[V] = sigma_l f0 with the rule-based fibre f0
                    v_mean = mlq.fibre_field(mesh["theta0"], mesh["e_circ"], mesh["e_long"], self.phys["sigma_l"])
                elif self.iso:  # the field is v = E[V] + W
                    theta0 = torch.full((mesh["tets"].shape[0],), float(kcfg["mean"]), dtype=torch.float64,
                                        device=device)
                else:
                    theta0 = torch.as_tensor(mesh["theta0"], dtype=torch.float64, device=device)
            else:
                phi = mlq.kl_transfer(self.kd, psi, lv, device=device)
                if self.iso:  # the field is v = E[V] + W
                    n_el = int(np.prod([n - 1 for n in lv["n"]]))
                    theta0 = torch.full((n_el,), float(kcfg["mean"]), dtype=torch.float64, device=device)
            desc, keep = mlq.make_desc(
                lv, self.phys, n_modes=M, phi=phi, sqrt_lambda=sl, theta0=theta0, prec=self.prec, qoi=cfg["qoi"],
                newton_tol=newton_tol if newton_tol is not None else (1e-13 if self.prec == mlq.MLQ_FP64 else 1e-10),
                inner_tol=inner_tol if inner_tol is not None else self.default_inner_tol(),
                max_inner=max_inner, max_batch=nb, newton_guess=newton_guess,
                diffusion=(mlq.MLQ_DIFF_VECTOR if self.vector else mlq.MLQ_DIFF_ISO if self.iso
                           else mlq.MLQ_DIFF_FIBRE), v_mean=v_mean)
            L = mlq.Level(desc, keep, device=device)
            L._keep = None  # arrays were copied into the level blob
            L.chunk = nb
            if tune_launch:
                # launch configuration (lane layout, GMRES graph blocks, batch chunk) from short
                # trial solves of seeded samples; the finest level's launches are large and keep
                # one launch per GMRES iteration (their apply is the kernel timed per launch)
                draw = W.mc_uniforms if self.uniform else W.mc_normals
                Yt = torch.as_tensor(draw(987654, l, nb, M * self.components), device=device)
                th = self._fields(L, Yt)
                L.tuning = tune.tune(L, th, graphs=l < top, log=say)
                del th, Yt
            elif tune_layout and not self.tet and cfg["dim"] == 3:
                # the faster lane layout of the 3D kernels for this grid and batch, by timing
                t = L.tune_lane_layout()
                say(f"level {l}: lane layout {L.lanes_x} (apply ms: 8 lanes {t[8]:.3f}, 16 lanes {t[16]:.3f})")
            if newton_guess in (mlq.MLQ_GUESS_REFERENCE, mlq.MLQ_GUESS_REFERENCE_LOCAL) or (
                    self.steps_per_block > 0 and block_guess != mlq.MLQ_GUESS_PREVIOUS):
                # the unperturbed reference solution (all coordinates zero: theta = its mean)
                Y0 = torch.zeros((M * self.components, 1), dtype=torch.float64, device=device)
                if self.vector:
                    th0 = torch.stack([L.sample_fields(Y0[c * M:(c + 1) * M].contiguous())
                                       for c in range(self.components)])
                else:
                    th0 = L.sample_fields(Y0)
                ref = torch.zeros((L.desc.n_steps + 1, L.n_nodes), dtype=torch.float64, device=device)
                r = L.solve_fields(th0, u_sum=ref)
                if r["code"] != mlq.MLQ_OK:
                    raise mlq.MlqError(r["code"], f"reference solve failed on level {l}")
                L.set_reference(ref)
            self.levels.append(L)
            say(f"level {l} created ({L.n_nodes} nodes, {L.n_elems} elements)")
            del phi
        del psi
        torch.cuda.synchronize()
        self.dof_iters = 0.0
        self.st_dof = 0.0
        self.log = None  # optional callable(str) for progress lines
        # levels solve concurrently, each from a host thread of its own on a stream of its
        # own (default priority); the solves of one level run in order on its stream
        self.concurrent = concurrent
        self.streams = [torch.cuda.Stream(device=device) for _ in self.levels]
        self._lock = threading.Lock()
        self.reset_counters()

    def reset_counters(self):
        self.dof_iters = 0.0
        self.st_dof = 0.0
        n = len(self.levels)
        self.level_dof_iters = [0.0] * n
        self.level_seconds = [0.0] * n
        self.level_newton = [0.0] * n       # Newton iterations (summed over samples and steps)
        self.level_inner = [0.0] * n        # GMRES iterations
        self.level_sample_steps = [0.0] * n

    def _fields(self, L, Y):
        """KL synthesis of the samples Y on level L: (B, P), or (components, B, P) for the vector model."""
        if self.vector:  # Y stacks the coordinates of the components: (components x M, B)
            M = self.kd.n_modes
            return torch.stack([L.sample_fields(Y[c * M:(c + 1) * M].contiguous()) for c in range(self.components)])
        return L.sample_fields(Y)

    def solve(self, l: int, Y: torch.Tensor, fields=None):
        """QoIs (device FP64) of the samples Y (M x B, device FP64) on level l; with `fields`
        (keyword arguments of Level.solve_fields) the field outputs are streamed as well.  A level
        tuned to a smaller batch chunk solves the samples in consecutive chunks."""
        L = self.levels[l]
        t0 = time.perf_counter()
        B = Y.shape[1]
        c = getattr(L, "chunk", B) if fields is None else B
        outs = []
        for i in range(0, B, c):
            theta = self._fields(L, Y[:, i:i + c] if c < B else Y)
            if self.steps_per_block > 0 and fields is None:
                out = L.solve_blocks(theta, min(self.steps_per_block, int(L.desc.n_steps)), self.block_guess)
            else:
                out = L.solve(theta) if fields is None else L.solve_fields(theta, per_sample_probes=False, **fields)
            if out["code"] != mlq.MLQ_OK:
                st = out["status"].cpu().numpy()
                raise mlq.MlqError(out["code"], f"{int((st != 0).sum())} samples failed on level {l}")
            outs.append(out)
        if len(outs) > 1:
            out = dict(qoi=torch.cat([o["qoi"] for o in outs]), iters=torch.cat([o["iters"] for o in outs]))
        it = out["iters"]
        sums = it.sum(dim=0).cpu()  # waits for the solve on this stream
        newton, inner = float(sums[0]), float(sums[1])
        el = time.perf_counter() - t0
        # a block GMRES iteration applies the operator to every time level of the block
        per_it = float(L.n_nodes) * (min(self.steps_per_block, int(L.desc.n_steps)) if self.steps_per_block else 1)
        with self._lock:
            self.dof_iters += per_it * inner
            self.st_dof += float(L.n_nodes) * float(L.desc.n_steps) * B
            self.level_dof_iters[l] += per_it * inner
            self.level_seconds[l] += el
            self.level_newton[l] += newton
            self.level_inner[l] += inner
            self.level_sample_steps[l] += float(B) * float(L.desc.n_steps)
        if self.log is not None:
            self.log(f"level {l}: {B} samples x {L.n_nodes} nodes x {L.desc.n_steps} steps solved")
        return out["qoi"]

    def solve_all(self, jobs):
        """QoIs of the jobs [(level, Y)] or [(level, Y, fields)], in order.  The finest level's solves run first on
        their own (so that its kernels, which dominate the cost, have the GPU to
        themselves), then all other levels at the same time (co-scheduled on one GPU: the
        small levels' latency-bound launches fill each other's gaps).  The results do not
        depend on the schedule: every solve is independent and the estimators sum on the
        host in sample order."""
        levels = sorted({job[0] for job in jobs}, reverse=True)
        out = [None] * len(jobs)

        def run_level(l):
            # the jobs of one level without field outputs (a level's own samples and its finer
            # neighbour's coarse side) form one batch: one solve per grid, with fuller launches
            plain = [i for i, job in enumerate(jobs) if job[0] == l and len(job) == 2]
            if len(plain) > 1:
                q = self.solve(l, torch.cat([jobs[i][1] for i in plain], dim=1))
                k = 0
                for i in plain:
                    n = jobs[i][1].shape[1]
                    out[i] = q[k:k + n]
                    k += n
            for i, job in enumerate(jobs):
                if job[0] == l and out[i] is None:
                    out[i] = self.solve(*job)

        if not self.concurrent or len(levels) < 3:
            for l in levels:
                run_level(l)
            return out
        main = torch.cuda.current_stream()

        def work(l):
            s = self.streams[l]
            s.wait_stream(main)  # the inputs were written on the caller's stream
            with torch.cuda.stream(s):
                run_level(l)
                s.synchronize()

        work(levels[0])
        with ThreadPoolExecutor(max_workers=len(levels) - 1) as ex:
            for f in [ex.submit(work, l) for l in levels[1:]]:
                f.result()
        return out

    # ---- estimators -----------------------------------------------------
    def run_mlmc(self, Ys):
        """eq. (StandardML) with independent MC sets: Ys[l] = (M x N_l) device normals."""
        jobs = []
        for l, Y in enumerate(Ys):
            jobs.append((l, Y))
            if l > 0:
                jobs.append((l - 1, Y))
        res = self.solve_all(jobs)
        ff, fc, k = [], [], 0
        for l in range(len(Ys)):
            ff.append(res[k])
            k += 1
            if l > 0:
                fc.append(res[k])
                k += 1
            else:
                fc.append(None)
        return self._estimate(mlq.MLQ_EST_MLMC, ff, fc, [Y.shape[1] for Y in Ys], 1)

    # ---- field quantities of interest ------------------------------------
    def _tet_weights(self, j):
        """P1 interpolation of level j's shell at the finest shell's vertices: (node, w) device
        tensors (n_L x 4), cached."""
        if not hasattr(self, "_wcache"):
            self._wcache = {}
        if j not in self._wcache:
            node, w = mlq.tet_locate(self.meshes[j], self.meshes[-1]["xyz"])
            self._wcache[j] = (torch.as_tensor(node, device=self.device), torch.as_tensor(w, device=self.device))
        return self._wcache[j]

    def default_inner_tol(self):
        """GMRES stopping tolerance of the workloads (an inexact-Newton forcing term; the discrete
        solution is fixed by the Newton stopping test).  Chosen by measured time per estimator
        pass: 1e-4 in FP64; in mixed precision 1e-3 on boxes and 1e-4 on shells, whose diagonal
        preconditioner leaves more Newton iterations at the looser value."""
        if self.prec == mlq.MLQ_FP64:
            return 1e-4
        return 1e-4 if self.tet else 1e-3

    def prepare_fields(self, probes=None):
        """Set-up of the field estimators outside any timed region: on shells, the location of
        the finest vertices in every coarser shell and of the probe points in every shell (host
        work, seconds on the 1.4M-vertex shell)."""
        if self.tet:
            for j in range(len(self.levels) - 1):
                self._tet_weights(j)
        if probes is not None:
            for j in range(len(self.levels)):
                self._probe_weights(j, probes)

    def _to_finest(self, j, src, dst, alpha, space=True, time=True, rows=1):
        """dst (finest grid) += alpha * T_j src (level j's grid): Q1 interpolation between nested
        boxes, P1 interpolation at the finest vertices between non-nested shells, linear in time."""
        lv, fin = self.levels[j], self.levels[-1]
        if self.tet and space:
            if j == len(self.levels) - 1:  # the finest shell itself: elementwise
                mlq.transfer_add(lv, fin, src, dst, alpha=alpha, space=False, time=False, rows=src.numel())
            else:
                node, w = self._tet_weights(j)
                mlq.transfer_add_weighted(lv, fin, node, w, src, dst, alpha=alpha, time=time, rows=rows)
        else:
            mlq.transfer_add(lv, fin, src, dst, alpha=alpha, space=space, time=time, rows=rows)

    def _probe_weights(self, j, probes):
        """(node, w) host arrays (P x 8) interpolating level j at the probe points (cached)."""
        if not hasattr(self, "_pcache"):
            self._pcache = {}
        key = (j, np.ascontiguousarray(probes, dtype=np.float64).tobytes())
        if key not in self._pcache:
            if not self.tet:
                self._pcache[key] = self.levels[j].probe_weights(probes)
            else:
                node4, w4 = mlq.tet_locate(self.meshes[j], probes)
                node = np.zeros((len(node4), mlq.PROBE_NODES), dtype=np.int64)
                w = np.zeros((len(node4), mlq.PROBE_NODES))
                node[:, :4], w[:, :4] = node4, w4
                self._pcache[key] = (node, w)
        return self._pcache[key]

    def _field_buffers(self, j, npr, pw):
        lv = self.levels[j]
        z = lambda *shape: torch.zeros(shape, dtype=torch.float64, device=self.device)
        f = dict(u_sum=z(lv.desc.n_steps + 1, lv.n_nodes), act_sum=z(lv.n_nodes))
        if npr:
            f.update(probe_node=pw[j][0], probe_w=pw[j][1], probe_sum=z(npr, lv.desc.n_steps + 1))
        return f

    def _field_estimate(self, terms, npr):
        """sum of alpha T_j S over terms [(j, alpha, buffers)] on the finest grids."""
        fin = self.levels[-1]
        z = lambda *shape: torch.zeros(shape, dtype=torch.float64, device=self.device)
        est_u, est_a = z(fin.desc.n_steps + 1, fin.n_nodes), z(fin.n_nodes)
        est_p = z(npr, fin.desc.n_steps + 1) if npr else None
        for j, alpha, f in terms:
            self._to_finest(j, f["u_sum"], est_u, alpha)
            self._to_finest(j, f["act_sum"], est_a, alpha, time=False)
            if npr:  # each probe's series: time transfer only
                mlq.transfer_add(self.levels[j], fin, f["probe_sum"], est_p, alpha=alpha, space=False, rows=npr)
        return est_u, est_a, est_p

    def run_combination_fields(self, Y, probes=None):
        """eq. (PimpedML) for the field quantities of interest (Section 2.4) with nested point
        sets: level j = L - l is solved at the points of Q_l in two batches, the points of
        Q_(l-1) and the rest, so that its term mean_Ql - mean_Q(l-1) is
            T_j ((1/N_l - 1/N_(l-1)) S_A + (1/N_l) S_B)
        with S_A, S_B the two batches' streamed sums; the fields are moved to the finest grids
        (non-nested shells: P1 interpolation at the finest vertices).  Also the scalar estimate."""
        npl = self.cfg["sampling"]["n_per_level"]
        L = len(self.levels) - 1
        npr = 0 if probes is None else len(probes)
        pw = [self._probe_weights(j, probes) for j in range(L + 1)] if npr else None
        jobs, terms, parts = [], [], []
        for l in range(L + 1):
            j, n_l, n_p = L - l, npl[l], (npl[l - 1] if l > 0 else 0)
            if n_p > 0:
                fa = self._field_buffers(j, npr, pw)
                jobs.append((j, Y[:, :n_p].contiguous(), fa))
                terms.append((j, 1.0 / n_l - 1.0 / n_p, fa))
            fb = self._field_buffers(j, npr, pw)
            jobs.append((j, Y[:, n_p:n_l].contiguous(), fb))
            terms.append((j, 1.0 / n_l, fb))
            parts.append((j, 2 if n_p > 0 else 1))
        res = self.solve_all(jobs)
        f = [None] * (L + 1)
        k = 0
        for j, cnt in parts:
            f[j] = torch.cat(res[k:k + cnt])
            k += cnt
        est_u, est_a, est_p = self._field_estimate(terms, npr)
        out = self._estimate(mlq.MLQ_EST_COMBINATION, f, None, list(npl), 1)
        out.update(mean_u=est_u, mean_act_map=est_a, mean_probe=est_p)
        return out

    def run_mlmc_fields(self, Ys, probes=None):
        """eq. (StandardML) for the field quantities of interest of Section 2.4, with independent
        MC sets Ys[l]: the mean transmembrane potential E[u] on the finest
        level's space-time grid ((m_L + 1) x n_L), the mean activation map on its nodes, and the
        mean action potential at the probe points (P x 3) on its time grid.  Each solve streams
        its sums on its own level's grid; the level terms are moved to the finest grid by the
        space-time transfer, so that the estimate is
            sum_l (1/N_l) (T_l S_fine(l) - T_(l-1) S_coarse(l)),
        with S the sums over the level's samples (non-nested shells: P1 interpolation at the
        finest vertices; the level-term norms are computed on boxes).  Also returns the scalar
        estimate."""
        dev = self.device
        npr = 0 if probes is None else len(probes)
        pw = [self._probe_weights(j, probes) for j in range(len(self.levels))] if npr else None

        def zeros(*shape):
            return torch.zeros(shape, dtype=torch.float64, device=dev)
        jobs, terms = [], []
        for l, Y in enumerate(Ys):
            for j, sign in [(l, 1.0)] + ([(l - 1, -1.0)] if l > 0 else []):
                f = self._field_buffers(j, npr, pw)
                jobs.append((j, Y, f))
                terms.append((j, sign / Y.shape[1], f))
        res = self.solve_all(jobs)
        est_u, est_a, est_p = self._field_estimate(terms, npr)
        # norms of the level terms on their own grids: mean_0 and, for l > 0, the mean level
        # difference mean_l - T mean_(l-1) (the quantities whose decay the level hierarchy
        # relies on), in L^2((0,T); L^2) and L^2((0,T); H^1)
        corr = [] if not self.tet else None
        k = 0
        for l, Y in enumerate(Ys if not self.tet else []):
            lv = self.levels[l]
            D = zeros(lv.desc.n_steps + 1, lv.n_nodes)
            mlq.transfer_add(lv, lv, jobs[k][2]["u_sum"], D, alpha=1.0 / Y.shape[1])
            k += 1
            if l > 0:
                mlq.transfer_add(self.levels[l - 1], lv, jobs[k][2]["u_sum"], D, alpha=-1.0 / Y.shape[1])
                k += 1
            corr.append([float(x) ** 0.5 for x in (mlq.field_norm2(lv, D, q=0).item(),
                                                      mlq.field_norm2(lv, D, q=1).item())])
            del D
        ff, fc, k = [], [], 0
        for l in range(len(Ys)):
            ff.append(res[k])
            k += 1
            if l > 0:
                fc.append(res[k])
                k += 1
            else:
                fc.append(None)
        out = self._estimate(mlq.MLQ_EST_MLMC, ff, fc, [Y.shape[1] for Y in Ys], 1)
        out.update(mean_u=est_u, mean_act_map=est_a, mean_probe=est_p, level_term_norms=corr)
        return out

    def run_mc(self, Y, level=0):
        f = self.solve(level, Y)
        return self._estimate(mlq.MLQ_EST_MC, [f], None, [Y.shape[1]], 1)

    def qmc_points(self, l, shifts):
        """Randomly shifted QMC points for level l: (M x S*N_l) device tensor, shift-major.
        Rank-1 lattices (CBC generating vector, Gaussian coordinates) or the paper's Halton
        points (indices 1..N_l, uniform or Gaussian coordinates as the workload draws them)."""
        samp = self.cfg["sampling"]
        N = samp["n_per_level"][l]
        M = shifts.shape[1]
        if samp.get("rule", "lattice") == "halton":
            cols = [mlq.halton(M, 1, N, shifts[s], uniform=self.uniform, device=self.device)
                    for s in range(shifts.shape[0])]
            return torch.cat(cols, dim=1)
        # product weights from the KL eigenvalues, repeated for every component of a vector field
        gamma = mlq.lattice_weights(self.lam, M // len(self.lam))
        z = mlq.cbc(N, M, gamma)
        cols = [mlq.lattice_points(z, shifts[s], N, 0, N, uniform=self.uniform, device=self.device)
                for s in range(shifts.shape[0])]
        return torch.cat(cols, dim=1)

    def run_mlqmc(self, shifts_per_level, levels=None):
        """eq. (StandardML) with randomly shifted QMC rules (shift-major sample order)."""
        levels = range(len(self.levels)) if levels is None else levels
        npl = []
        S = shifts_per_level[0].shape[0]
        jobs = []
        for l in levels:
            Y = self.qmc_points(l, shifts_per_level[l])
            jobs.append((l, Y))
            if l > 0:
                jobs.append((l - 1, Y))
            npl.append(Y.shape[1] // S)
        res = self.solve_all(jobs)
        ff, fc, k = [], [], 0
        for l in levels:
            ff.append(res[k])
            k += 1
            if l > 0:
                fc.append(res[k])
                k += 1
            else:
                fc.append(None)
        return self._estimate(mlq.MLQ_EST_MLQMC, ff, fc, npl, S)

    def run_combination(self, Y):
        """eq. (PimpedML) with nested Monte Carlo points: Y (M x N_max) device normals; level j
        is solved at the first N_{L-j} points (Q_{L-j})."""
        npl = self.cfg["sampling"]["n_per_level"]
        L = len(self.levels) - 1
        f = self.solve_all([(j, Y[:, :npl[L - j]].contiguous()) for j in range(L + 1)])
        return self._estimate(mlq.MLQ_EST_COMBINATION, f, None, list(npl), 1)

    def _estimate(self, kind, ff, fc, npl, S):
        ffh = [f.cpu().numpy() for f in ff]
        fch = [c.cpu().numpy() if c is not None else None for c in (fc or [None] * len(ff))]
        res = mlq.estimate(kind, ffh, fch, n_per_level=npl, n_shifts=S)
        res["f_fine"], res["f_coarse"] = ffh, fch
        return res
