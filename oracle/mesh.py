"""Uniform tensor-product Q1 meshes (test infrastructure; see ``oracle/__init__``).

The paper uses nested shape-regular meshes with h_l ~ 2^-l (Section 3.1).  The
cube workloads here use axis-aligned boxes split into 2^d-node bricks.

Numbering: node (i_0, .., i_{d-1}) has index i_0 + n_0 (i_1 + n_1 i_2); element
(e_0, ..) likewise with n_a - 1 per axis.  The local node a of an element has
bit k of a equal to its offset along axis k.
"""
from __future__ import annotations

import itertools
import numpy as np


class BoxMesh:
    def __init__(self, n, lo=None, hi=None):
        self.n = [int(v) for v in n]
        self.d = len(self.n)
        self.lo = np.array(lo if lo is not None else [0.0] * self.d, dtype=np.float64)
        self.hi = np.array(hi if hi is not None else [1.0] * self.d, dtype=np.float64)
        self.h = (self.hi - self.lo) / (np.array(self.n) - 1)
        self.n_nodes = int(np.prod(self.n))
        self.ne = [v - 1 for v in self.n]
        self.n_elems = int(np.prod(self.ne))

        # node coordinates, axis 0 fastest
        grids = [self.lo[a] + self.h[a] * np.arange(self.n[a]) for a in range(self.d)]
        mesh = np.meshgrid(*grids, indexing="ij")
        self.nodes = np.stack([m.transpose(*reversed(range(self.d))).ravel() for m in mesh], axis=1)

        # element connectivity
        eidx = np.stack(np.meshgrid(*[np.arange(v) for v in self.ne], indexing="ij"), axis=-1)
        eidx = eidx.transpose(*reversed(range(self.d)), self.d).reshape(-1, self.d)  # (E, d), axis 0 fastest
        self.elem_index = eidx
        conn = np.zeros((self.n_elems, 2 ** self.d), dtype=np.int64)
        for a in range(2 ** self.d):
            off = [(a >> k) & 1 for k in range(self.d)]
            conn[:, a] = self.node_id(eidx + np.array(off))
        self.elems = conn
        self.centres = self.lo + (eidx + 0.5) * self.h

    def node_id(self, ijk):
        ijk = np.asarray(ijk)
        idx = ijk[..., 0].astype(np.int64)
        stride = 1
        for a in range(1, self.d):
            stride *= self.n[a - 1]
            idx = idx + stride * ijk[..., a]
        return idx

    @property
    def volume(self) -> float:
        return float(np.prod(self.hi - self.lo))

    def locate(self, pts):
        """Element multi-index containing each point and its reference coordinates in [0,1]^d.

        Points on an interior element face belong to the element on the upper side,
        points on the upper domain boundary to the last element.
        """
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        rel = (pts - self.lo) / self.h
        e = np.floor(rel).astype(np.int64)
        e = np.clip(e, 0, np.array(self.ne) - 1)
        xi = rel - e
        return e, xi


def local_offsets(d):
    return [tuple((a >> k) & 1 for k in range(d)) for a in range(2 ** d)]


def all_offsets(d):
    return list(itertools.product((0, 1), repeat=d))
