"""Autotuner of the per-level launch configuration of the batched solves.

For one level and one batch size it times short trial solves (the first steps of the
space-time problem of real samples) over the candidate configurations and keeps the fastest:

* lane layout of the 3D box kernels (waves of 8 x 8 or 16 x 4 lanes; tile shape in x-y);
* GMRES schedule: iterations launched one at a time with a host read each, or blocks of J
  iterations replayed from captured HIP graphs with one read per block;
* batch chunk: the level's samples solved in one call or in two consecutive halves.

Every configuration gives the same results (the operators are the same in both layouts, and
the graph blocks replay the same launches); only the time differs.  Winners are cached in a
JSON file keyed by (mesh shape, batch, precision) so that later runs skip the trials; the file is
MLQ_TUNE_CACHE, else ~/.cache/mlq/tune.json (MLQ_TUNE_CACHE=off disables the cache).
Configuration only: the solves themselves run in the library.
"""
from __future__ import annotations

import json
import os
import time

from . import mlq

GMRES_BLOCKS = (0, 1, 2, 4)


def cache_path():
    p = os.environ.get("MLQ_TUNE_CACHE")
    if p == "off":
        return None
    return p or os.path.join(os.path.expanduser("~"), ".cache", "mlq", "tune.json")


def _load():
    p = cache_path()
    if p is None or not os.path.exists(p):
        return {}
    try:
        with open(p) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    p = cache_path()
    if p is None:
        return
    data = _load()
    data[key] = value
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def level_key(level, batch):
    d = level.desc
    if d.mesh_kind == mlq.MLQ_MESH_P1_TET:
        shape = f"tet{int(d.n_vert)}x{int(d.n_tet)}"
    else:
        shape = "box" + "x".join(str(int(d.n[a])) for a in range(int(d.dim)))
    return f"{shape}|steps{int(d.n_steps)}|batch{int(batch)}|{'mixed' if level.mixed else 'fp64'}|diff{int(d.diffusion)}"


def apply_config(level, cfg):
    if level.desc.mesh_kind == mlq.MLQ_MESH_Q1_BOX and level.desc.dim == 3:
        level.set_lane_layout(cfg["lanes_x"])
    level.set_gmres_block(cfg["gmres_block"])
    level.chunk = cfg["chunk"]


def candidates(level, batch, graphs=True):
    box3 = level.desc.mesh_kind == mlq.MLQ_MESH_Q1_BOX and level.desc.dim == 3
    lanes = (8, 16) if box3 else (0,)
    blocks = GMRES_BLOCKS if graphs else (0,)
    chunks = [batch] + ([(batch + 1) // 2] if batch >= 256 else [])
    return [dict(lanes_x=lx, gmres_block=J, chunk=c) for lx in lanes for J in blocks for c in chunks]


def tune(level, theta, steps=12, graphs=True, use_cache=True, log=None):
    """Fastest configuration of `level` for the batch of fields theta ((B, P) or (3, B, P) device
    tensor; its solves are the trials).  Applies it to the level and returns it with the trial
    times (ms per solve of `steps` steps of the whole batch)."""
    import torch
    B = int(theta.shape[-2])
    key = level_key(level, B) + ("" if graphs else "|nographs")
    if use_cache:
        hit = _load().get(key)
        if hit is not None:
            apply_config(level, hit)
            return dict(hit, cached=True)
    steps = min(int(steps), int(level.desc.n_steps))
    trials = {}
    for cfg in candidates(level, B, graphs):
        apply_config(level, cfg)
        c = cfg["chunk"]
        parts = [theta[..., i:i + c, :] for i in range(0, B, c)]

        def run():
            for th in parts:
                out = level.solve(th.contiguous(), n_steps=steps)
                if out["code"] != mlq.MLQ_OK:
                    raise mlq.MlqError(out["code"], "trial solve failed")
        run()  # warm-up: workspace, graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        trials[f"lanes{cfg['lanes_x']}_block{cfg['gmres_block']}_chunk{c}"] = round(ms, 3)
        cfg["ms"] = ms
    default = next(c for c in candidates(level, B, graphs)
                   if c["gmres_block"] == 0 and c["chunk"] == B
                   and c["lanes_x"] in (0, 16 if level.desc.n[0] >= 48 else 8))
    best = min(candidates(level, B, graphs), key=lambda c: trials[
        f"lanes{c['lanes_x']}_block{c['gmres_block']}_chunk{c['chunk']}"])
    ms_best = trials[f"lanes{best['lanes_x']}_block{best['gmres_block']}_chunk{best['chunk']}"]
    ms_def = trials[f"lanes{default['lanes_x']}_block{default['gmres_block']}_chunk{default['chunk']}"]
    if ms_best > 0.97 * ms_def:  # near ties keep the default, so that noise does not flip choices
        best = default
    out = dict(lanes_x=best["lanes_x"], gmres_block=best["gmres_block"], chunk=best["chunk"], steps=steps,
               trials_ms=trials)
    apply_config(level, out)
    if use_cache:
        _store(key, out)
    if log is not None:
        log(f"tuned {key}: lanes {out['lanes_x']}, gmres block {out['gmres_block']}, chunk {out['chunk']}")
    return dict(out, cached=False)
