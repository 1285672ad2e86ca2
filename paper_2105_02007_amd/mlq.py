"""Thin ctypes binding of libmlq.so (include/mlq.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  Device buffers are torch tensors on the current HIP device;
torch provides memory and streams.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlq.so")

MLQ_OK, MLQ_EINVAL, MLQ_EHIP, MLQ_ENOCONV, MLQ_ESIZE, MLQ_ESTATE = 0, -1, -2, -3, -4, -5
MLQ_FP64, MLQ_MIXED = 0, 1
MLQ_QOI_MEAN_U_FINAL, MLQ_QOI_MEAN_ACT_TIME = 0, 1
MLQ_SAMPLE_OK, MLQ_SAMPLE_NOCONV, MLQ_SAMPLE_NAN = 0, 1, 2
MLQ_EST_MC, MLQ_EST_MLMC, MLQ_EST_MLQMC, MLQ_EST_COMBINATION = 0, 1, 2, 3
MLQ_MESH_Q1_BOX, MLQ_MESH_P1_TET = 0, 1

EXPORTED = [
    "mlq_level_bytes", "mlq_create_level", "mlq_destroy_level", "mlq_level_sizes", "mlq_workspace_bytes",
    "mlq_sample_fields", "mlq_solve_batch", "mlq_solve_batch_ex", "mlq_apply", "mlq_check",
    "mlq_lattice_normals", "mlq_halton", "mlq_cbc", "mlq_accumulate", "mlq_estimate", "mlq_last_error",
    "mlq_kl_workspace_bytes", "mlq_kl_modes", "mlq_kl_transfer", "mlq_timing_enable", "mlq_timing_read",
    "mlq_kl_transfer_tet_bytes", "mlq_kl_transfer_tet", "mlq_solve_batch_fields", "mlq_probe_weights",
    "mlq_transfer_add", "mlq_field_norm2", "mlq_set_reference", "mlq_tet_locate", "mlq_transfer_add_weighted",
    "mlq_set_lane_layout", "mlq_lattice_points", "mlq_solve_batch_static",
    "mlq_kl_weights", "mlq_lattice_weights", "mlq_fibre_field", "mlq_set_gmres_block", "mlq_set_persistent",
    "mlq_workspace_bytes_blocks", "mlq_solve_batch_blocks",
]
STATIC_WS_BYTES = 64 << 20
MLQ_GUESS_PREVIOUS, MLQ_GUESS_EXTRAPOLATE, MLQ_GUESS_REFERENCE, MLQ_GUESS_REFERENCE_LOCAL = 0, 1, 2, 3
MLQ_DIFF_FIBRE, MLQ_DIFF_ISO, MLQ_DIFF_VECTOR = 0, 1, 2
MLQ_COV_EXP, MLQ_COV_SQEXP = 0, 1
MLQ_MAP_NORMAL, MLQ_MAP_UNIFORM = 0, 1
MLQ_KL_CHOLESKY, MLQ_KL_EXACT = 0, 1
KERNEL_CLASSES = ["apply", "residual", "rhs", "precond", "dots", "orth", "small", "update", "qoi", "persistent"]


class MlqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mlq error {code}: {msg}")
        self.code = code


class LevelDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("mesh_kind", C.c_int32),
        ("n", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("n_steps", C.c_int32), ("t_end", C.c_double),
        ("alpha", C.c_double), ("u_rest", C.c_double), ("u_th", C.c_double), ("u_peak", C.c_double),
        ("sigma_l", C.c_double), ("sigma_t", C.c_double),
        ("stim_lo", C.c_double * 3), ("stim_hi", C.c_double * 3),
        ("stim_t_on", C.c_double), ("stim_t_off", C.c_double), ("stim_amp", C.c_double),
        ("n_modes", C.c_int32),
        ("phi", C.POINTER(C.c_double)), ("sqrt_lambda", C.POINTER(C.c_double)), ("theta0", C.POINTER(C.c_double)),
        ("prec", C.c_int32), ("qoi", C.c_int32),
        ("newton_tol", C.c_double), ("inner_tol", C.c_double),
        ("max_newton", C.c_int32), ("max_inner", C.c_int32), ("max_batch", C.c_int32),
        ("arrays_on_device", C.c_int32),
        ("n_vert", C.c_int64), ("n_tet", C.c_int64),
        ("xyz", C.POINTER(C.c_double)), ("tets", C.POINTER(C.c_int32)),
        ("e_circ", C.POINTER(C.c_double)), ("e_long", C.POINTER(C.c_double)),
        ("stim_center", C.c_double * 3), ("stim_radius", C.c_double),
        ("newton_guess", C.c_int32), ("diffusion", C.c_int32), ("v_mean", C.POINTER(C.c_double)),
    ]


class KlDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("std_dev", C.c_double), ("corr_len", C.c_double),
        ("n_modes", C.c_int32), ("max_rank", C.c_int32), ("eps", C.c_double),
        ("mesh_kind", C.c_int32), ("n_vert", C.c_int64), ("n_tet", C.c_int64),
        ("xyz", C.POINTER(C.c_double)), ("tets", C.POINTER(C.c_int32)),
        ("cov_kernel", C.c_int32), ("method", C.c_int32),
    ]


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * 16), ("launches", C.c_int64 * 16), ("units", C.c_double * 16),
                ("bytes", C.c_double * 16), ("kernel_bytes", C.c_double * 16)]


class EstimateOut(C.Structure):
    _fields_ = [("estimate", C.c_double), ("rmse", C.c_double), ("n_levels", C.c_int32),
                ("level_mean", C.c_double * 16), ("level_var", C.c_double * 16)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python paper_2105_02007_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "mlq_level_bytes": [C.POINTER(LevelDesc), C.POINTER(C.c_size_t)],
        "mlq_create_level": [C.POINTER(LevelDesc), VP, C.c_size_t, VP, C.POINTER(VP)],
        "mlq_level_sizes": [VP, C.POINTER(I64), C.POINTER(I64)],
        "mlq_workspace_bytes": [VP, I32, C.POINTER(C.c_size_t)],
        "mlq_sample_fields": [VP, VP, I32, VP, VP],
        "mlq_solve_batch": [VP, VP, I32, VP, C.c_size_t, VP, VP, VP, VP],
        "mlq_solve_batch_ex": [VP, VP, I32, I32, VP, C.c_size_t, VP, VP, VP, VP, VP, VP],
        "mlq_solve_batch_static": [VP, VP, I32, VP, VP, VP, VP],
        "mlq_apply": [VP, VP, I32, VP, VP, VP, VP, C.c_size_t, VP],
        "mlq_check": [VP, I32],
        "mlq_lattice_normals": [VP, VP, I32, I64, I64, I32, VP, VP],
        "mlq_halton": [I32, I64, I32, VP, I32, VP, VP],
        "mlq_solve_batch_fields": [VP, VP, I32, VP, C.c_size_t, VP, VP, VP, VP, VP],
        "mlq_probe_weights": [VP, VP, I32, VP, VP],
        "mlq_transfer_add": [VP, VP, I32, I32, I64, C.c_double, VP, VP, VP],
        "mlq_field_norm2": [VP, I32, I32, I64, VP, VP, VP, VP],
        "mlq_set_reference": [VP, VP],
        "mlq_set_lane_layout": [VP, I32],
        "mlq_set_gmres_block": [VP, I32],
        "mlq_set_persistent": [VP, I32],
        "mlq_workspace_bytes_blocks": [VP, I32, I32, C.POINTER(C.c_size_t)],
        "mlq_solve_batch_blocks": [VP, VP, I32, I32, I32, VP, C.c_size_t, VP, VP, VP, VP, VP],
        "mlq_lattice_points": [VP, VP, I32, I64, I64, I32, I32, VP, VP],
        "mlq_tet_locate": [VP, I64, VP, I64, VP, I64, VP, VP],
        "mlq_transfer_add_weighted": [VP, VP, I32, I64, I32, VP, VP, C.c_double, VP, VP, VP],
        "mlq_cbc": [I64, I32, VP, VP],
        "mlq_kl_weights": [VP, I32, I32, VP],
        "mlq_lattice_weights": [VP, I32, I32, VP],
        "mlq_fibre_field": [I64, VP, VP, VP, C.c_double, VP],
        "mlq_accumulate": [VP, VP, I32, VP, VP],
        "mlq_estimate": [I32, I32, I32, VP, VP, VP, C.POINTER(EstimateOut)],
        "mlq_kl_workspace_bytes": [C.POINTER(KlDesc), C.POINTER(C.c_size_t)],
        "mlq_kl_modes": [C.POINTER(KlDesc), VP, C.c_size_t, VP, VP, VP, VP, VP],
        "mlq_kl_transfer": [C.POINTER(KlDesc), VP, VP, VP, VP, VP, VP],
        "mlq_kl_transfer_tet_bytes": [I64, C.POINTER(C.c_size_t)],
        "mlq_kl_transfer_tet": [C.POINTER(KlDesc), VP, I64, VP, I64, VP, VP, C.c_size_t, VP, VP],
        "mlq_timing_enable": [VP, C.c_uint32],
        "mlq_timing_read": [VP, C.POINTER(Timing), I32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.mlq_destroy_level.argtypes = [VP]
    lib.mlq_destroy_level.restype = None
    lib.mlq_last_error.argtypes = []
    lib.mlq_last_error.restype = C.c_char_p
    return lib


lib = _load()


def check(code):
    if code != MLQ_OK:
        raise MlqError(code, lib.mlq_last_error().decode())
    return code


def check_status(status):
    """mlq_check on host per-sample status words: MLQ_OK, or MLQ_ENOCONV if any sample failed."""
    import numpy as np
    st = np.ascontiguousarray(np.asarray(status, dtype=np.int32))
    return lib.mlq_check(st.ctypes.data_as(C.c_void_p), int(st.size))


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class FieldOut(C.Structure):
    _fields_ = [("u_sum", C.c_void_p), ("act_sum", C.c_void_p), ("probe", C.c_void_p), ("n_probe", C.c_int32),
                ("probe_node", C.c_void_p), ("probe_w", C.c_void_p), ("probe_sum", C.c_void_p)]


PROBE_NODES = 8


def make_desc(level: dict, phys: dict, *, n_modes=0, phi=None, sqrt_lambda=None, theta0=None,
              prec=MLQ_FP64, qoi=MLQ_QOI_MEAN_U_FINAL, newton_tol=1e-13, inner_tol=1e-6,
              max_newton=20, max_inner=30, max_batch=1, newton_guess=MLQ_GUESS_PREVIOUS,
              diffusion=MLQ_DIFF_FIBRE, v_mean=None):
    """Fills an mlq_level_desc from a workload level and physics dict.  Returns (desc, keepalive)."""
    d = LevelDesc()
    dim = level["dim"]
    keep = []
    if level.get("kind") == "tet":
        # P1 tetrahedra: level["mesh"] holds xyz (V, 3), tets (T, 4), e_circ / e_long (T, 3)
        m = level["mesh"]
        xyz = np.ascontiguousarray(m["xyz"], dtype=np.float64)
        tets = np.ascontiguousarray(m["tets"], dtype=np.int32)
        ec = np.ascontiguousarray(m["e_circ"], dtype=np.float64)
        el = np.ascontiguousarray(m["e_long"], dtype=np.float64)
        keep += [xyz, tets, ec, el]
        d.dim, d.mesh_kind = 3, MLQ_MESH_P1_TET
        d.n_vert, d.n_tet = xyz.shape[0], tets.shape[0]
        d.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
        d.tets = tets.ctypes.data_as(C.POINTER(C.c_int32))
        d.e_circ = ec.ctypes.data_as(C.POINTER(C.c_double))
        d.e_long = el.ctypes.data_as(C.POINTER(C.c_double))
        for a in range(3):
            d.stim_center[a] = float(phys["stim_center"][a])
        d.stim_radius = float(phys["stim_radius"])
    else:
        d.dim, d.mesh_kind = dim, MLQ_MESH_Q1_BOX
        for a in range(3):
            d.n[a] = level["n"][a] if a < dim else 1
            d.lo[a] = level["lo"][a] if a < dim else 0.0
            d.hi[a] = level["hi"][a] if a < dim else 1.0
            d.stim_lo[a] = phys["stim_lo"][a] if a < dim else 0.0
            d.stim_hi[a] = phys["stim_hi"][a] if a < dim else 1.0
    d.n_steps, d.t_end = int(level["n_steps"]), float(phys["t_end"])
    for k in ("alpha", "u_rest", "u_th", "u_peak", "sigma_l", "sigma_t", "stim_t_on", "stim_t_off", "stim_amp"):
        setattr(d, k, float(phys[k]))
    d.n_modes = int(n_modes)
    on_dev = n_modes > 0 and hasattr(phi, "data_ptr")
    d.arrays_on_device = 1 if on_dev else 0
    if on_dev:  # torch device tensors
        keep += [phi, sqrt_lambda, theta0]
        d.phi = C.cast(C.c_void_p(phi.data_ptr()), C.POINTER(C.c_double))
        d.sqrt_lambda = C.cast(C.c_void_p(sqrt_lambda.data_ptr()), C.POINTER(C.c_double))
        if theta0 is not None:
            d.theta0 = C.cast(C.c_void_p(theta0.data_ptr()), C.POINTER(C.c_double))
    else:
        if n_modes > 0:
            phi = np.ascontiguousarray(phi, dtype=np.float64)
            sl = np.ascontiguousarray(sqrt_lambda, dtype=np.float64)
            keep += [phi, sl]
            d.phi = phi.ctypes.data_as(C.POINTER(C.c_double))
            d.sqrt_lambda = sl.ctypes.data_as(C.POINTER(C.c_double))
        if theta0 is not None:
            t0 = np.ascontiguousarray(theta0, dtype=np.float64)
            keep.append(t0)
            d.theta0 = t0.ctypes.data_as(C.POINTER(C.c_double))
    d.prec, d.qoi = int(prec), int(qoi)
    d.newton_tol, d.inner_tol = float(newton_tol), float(inner_tol)
    d.max_newton, d.max_inner, d.max_batch = int(max_newton), int(max_inner), int(max_batch)
    d.newton_guess = int(newton_guess)
    d.diffusion = int(diffusion)
    if v_mean is not None:  # vector model: E[V] per element (n_tet, 3)
        vm = np.ascontiguousarray(v_mean, dtype=np.float64)
        keep.append(vm)
        d.v_mean = vm.ctypes.data_as(C.POINTER(C.c_double))
    return d, keep


class Level:
    """One level: descriptor, device blob, level handle.  Device memory comes from torch."""

    def __init__(self, desc: LevelDesc, keep=None, device="cuda"):
        import torch
        self.desc, self._keep = desc, keep
        nbytes = C.c_size_t()
        check(lib.mlq_level_bytes(C.byref(desc), C.byref(nbytes)))
        self.blob = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(lib.mlq_create_level(C.byref(desc), _ptr(self.blob), nbytes.value, _stream(), C.byref(h)))
        self.handle = h
        nn, ne = C.c_int64(), C.c_int64()
        check(lib.mlq_level_sizes(self.handle, C.byref(nn), C.byref(ne)))
        self.n_nodes, self.n_elems = int(nn.value), int(ne.value)
        self.mixed = desc.prec == MLQ_MIXED
        self.device = device
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:  # lib is None during interpreter shutdown
            lib.mlq_destroy_level(h)
            self.handle = None

    @property
    def theta_dtype(self):
        import torch
        return torch.float32 if self.mixed else torch.float64

    def workspace(self, batch):
        import torch
        nbytes = C.c_size_t()
        check(lib.mlq_workspace_bytes(self.handle, int(batch), C.byref(nbytes)))
        if self._ws is None or self._ws.numel() < nbytes.value:
            self._ws = None
            self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        return self._ws, int(nbytes.value)

    def sample_fields(self, Y, theta=None):
        """Y: (M, B) FP64 device tensor, column b = sample b (stored as B x M row-major)."""
        import torch
        B = Y.shape[1]
        Yc = Y.t().contiguous()  # column-major M x B == row-major B x M
        if theta is None:
            theta = torch.empty((B, self.n_elems), dtype=self.theta_dtype, device=self.device)
        check(lib.mlq_sample_fields(self.handle, _ptr(Yc), int(B), _ptr(theta), _stream()))
        return theta

    def solve(self, theta, n_steps=None, want_state=False):
        """theta: (B, P) field, or (3, B, P) components of the vector model."""
        import torch
        B = theta.shape[-2]
        ws, nbytes = self.workspace(B)
        qoi = torch.empty(B, dtype=torch.float64, device=self.device)
        status = torch.empty(B, dtype=torch.int32, device=self.device)
        iters = torch.empty((B, 2), dtype=torch.int64, device=self.device)
        u = act = None
        if want_state:
            u = torch.empty((B, self.n_nodes), dtype=torch.float64, device=self.device)
            act = torch.empty((B, self.n_nodes), dtype=torch.float64, device=self.device)
        steps = self.desc.n_steps if n_steps is None else int(n_steps)
        code = lib.mlq_solve_batch_ex(self.handle, _ptr(theta), int(B), steps, _ptr(ws), nbytes, _ptr(qoi),
                                      _ptr(status), _ptr(iters), _ptr(u), _ptr(act), _stream())
        if code not in (MLQ_OK, MLQ_ENOCONV):
            check(code)
        return dict(qoi=qoi, status=status, iters=iters, u=u, act=act, code=code)

    def solve_blocks(self, theta, steps_per_block, guess=MLQ_GUESS_PREVIOUS, want_state=False):
        """All-at-once solve in time blocks of steps_per_block steps (mlq_solve_batch_blocks)."""
        import torch
        B = theta.shape[-2]
        nbytes = C.c_size_t()
        check(lib.mlq_workspace_bytes_blocks(self.handle, int(B), int(steps_per_block), C.byref(nbytes)))
        if self._ws is None or self._ws.numel() < nbytes.value:
            self._ws = None
            self._ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        qoi = torch.empty(B, dtype=torch.float64, device=self.device)
        status = torch.empty(B, dtype=torch.int32, device=self.device)
        iters = torch.empty((B, 2), dtype=torch.int64, device=self.device)
        u = torch.empty((B, self.n_nodes), dtype=torch.float64, device=self.device) if want_state else None
        code = lib.mlq_solve_batch_blocks(self.handle, _ptr(theta), int(B), int(steps_per_block), int(guess),
                                          _ptr(self._ws), nbytes.value, _ptr(qoi), _ptr(status), _ptr(iters), _ptr(u),
                                          _stream())
        if code not in (MLQ_OK, MLQ_ENOCONV):
            check(code)
        return dict(qoi=qoi, status=status, iters=iters, u=u, code=code)

    def solve_static(self, theta):
        """mlq_solve_batch_static: the solve with the library's static device workspace (no
        workspace from torch).  Returns the same dict as solve (without states)."""
        import torch
        B = theta.shape[-2]
        qoi = torch.empty(B, dtype=torch.float64, device=self.device)
        status = torch.empty(B, dtype=torch.int32, device=self.device)
        iters = torch.empty((B, 2), dtype=torch.int64, device=self.device)
        code = lib.mlq_solve_batch_static(self.handle, _ptr(theta), int(B), _ptr(qoi), _ptr(status), _ptr(iters),
                                          _stream())
        if code not in (MLQ_OK, MLQ_ENOCONV):
            check(code)
        return dict(qoi=qoi, status=status, iters=iters, code=code)

    def solve_fields(self, theta, u_sum=None, act_sum=None, probe_node=None, probe_w=None, probe_sum=None,
                     per_sample_probes=True):
        """Solve with field outputs: u_sum ((n_steps + 1) x n), act_sum (n) and probe_sum
        (n_probe x (n_steps + 1)) device FP64 tensors are added into; probe_node / probe_w
        (n_probe x 8 host arrays) select probe points, whose per-sample series come back as
        out["probe"] (B x n_probe x (n_steps + 1)) unless per_sample_probes is False."""
        import torch
        B = theta.shape[-2]
        ws, nbytes = self.workspace(B)
        qoi = torch.empty(B, dtype=torch.float64, device=self.device)
        status = torch.empty(B, dtype=torch.int32, device=self.device)
        iters = torch.empty((B, 2), dtype=torch.int64, device=self.device)
        f = FieldOut()
        keep = []
        probe = None
        if u_sum is not None:
            f.u_sum = u_sum.data_ptr()
        if act_sum is not None:
            f.act_sum = act_sum.data_ptr()
        if probe_node is not None:
            pn = np.ascontiguousarray(probe_node, dtype=np.int64).reshape(-1, PROBE_NODES)
            pw = np.ascontiguousarray(probe_w, dtype=np.float64).reshape(-1, PROBE_NODES)
            keep += [pn, pw]
            if per_sample_probes:
                probe = torch.empty((B, pn.shape[0], self.desc.n_steps + 1), dtype=torch.float64,
                                    device=self.device)
                f.probe = probe.data_ptr()
            if probe_sum is not None:
                f.probe_sum = probe_sum.data_ptr()
            f.n_probe = pn.shape[0]
            f.probe_node, f.probe_w = pn.ctypes.data, pw.ctypes.data
        code = lib.mlq_solve_batch_fields(self.handle, _ptr(theta), int(B), _ptr(ws), nbytes, _ptr(qoi),
                                          _ptr(status), _ptr(iters), C.byref(f), _stream())
        if code not in (MLQ_OK, MLQ_ENOCONV):
            check(code)
        return dict(qoi=qoi, status=status, iters=iters, probe=probe, code=code)

    def set_lane_layout(self, lanes_x):
        """Lanes along x of the 3D box kernels' waves: 8, 16, or 0 (by grid width)."""
        check(lib.mlq_set_lane_layout(self.handle, int(lanes_x)))
        self.lanes_x = int(lanes_x)

    def set_gmres_block(self, iterations):
        """GMRES iterations per captured graph (0: one launch sequence and host read per iteration)."""
        check(lib.mlq_set_gmres_block(self.handle, int(iterations)))
        self.gmres_block = int(iterations)

    def set_persistent(self, on):
        """Persistent per-sample solves (small 3D box levels): one launch per solve, enqueue only;
        failures then show in the returned status, not in the return code."""
        check(lib.mlq_set_persistent(self.handle, 1 if on else 0))
        self.persistent = bool(on)

    def tune_lane_layout(self, batch=None, reps=5, margin=0.05):
        """Times the operator apply of this level at `batch` samples (default: the level's
        largest batch) in both lane layouts and keeps the other layout than the default (by grid
        width) only if it is faster by more than `margin`, so that near ties do not flip between
        runs.  Returns {lanes_x: ms}."""
        import torch
        B = int(batch or self.desc.max_batch)
        tdt = torch.float32 if self.mixed else torch.float64
        theta = torch.zeros((B, self.n_elems), dtype=tdt, device=self.device)
        x = torch.ones((B, self.n_nodes), dtype=tdt, device=self.device)
        d = torch.zeros_like(x)
        y = torch.empty_like(x)
        times = {}
        for lx in (8, 16):
            self.set_lane_layout(lx)
            self.apply(theta, x, d, y)  # warm-up (and workspace size for this layout)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                self.apply(theta, x, d, y)
            e1.record()
            torch.cuda.synchronize()
            times[lx] = e0.elapsed_time(e1) / reps
        default = 16 if self.desc.n[0] >= 48 else 8
        other = 8 if default == 16 else 16
        self.set_lane_layout(other if times[other] < (1.0 - margin) * times[default] else default)
        return times

    def set_reference(self, ref):
        """Reference space-time solution ((n_steps + 1) x n device FP64) for the reference
        Newton guesses; the level keeps a reference to the tensor."""
        self._ref = ref
        check(lib.mlq_set_reference(self.handle, None if ref is None else _ptr(ref)))

    def probe_weights(self, points):
        """(node, weight) host arrays (P x 8) of the Q1 interpolant at points (P x 3) of a box level."""
        pts = np.zeros((len(points), 3))
        p = np.asarray(points, dtype=np.float64)
        pts[:, :p.shape[1]] = p
        node = np.zeros((len(pts), PROBE_NODES), dtype=np.int64)
        w = np.zeros((len(pts), PROBE_NODES))
        check(lib.mlq_probe_weights(self.handle, pts.ctypes.data, int(len(pts)), node.ctypes.data, w.ctypes.data))
        return node, w

    def timing_enable(self, classes=("apply",)):
        mask = 0
        for c in classes:
            mask |= 1 << KERNEL_CLASSES.index(c)
        check(lib.mlq_timing_enable(self.handle, mask))

    def timing_read(self, reset=True):
        t = Timing()
        check(lib.mlq_timing_read(self.handle, C.byref(t), 1 if reset else 0))
        return {c: dict(ms=t.ms[i], launches=int(t.launches[i]), units=t.units[i], bytes=t.bytes[i],
                        kernel_bytes=t.kernel_bytes[i])
                for i, c in enumerate(KERNEL_CLASSES)}

    def apply(self, theta, x, d, y=None):
        import torch
        B = theta.shape[-2]
        ws, nbytes = self.workspace(B)
        if y is None:
            y = torch.empty_like(x)
        check(lib.mlq_apply(self.handle, _ptr(theta), int(B), _ptr(x), _ptr(d), _ptr(y), _ptr(ws), nbytes,
                            _stream()))
        return y


def transfer_add(src_level, dst_level, src, dst, alpha=1.0, space=True, time=True, rows=1):
    """dst += alpha * (time x space interpolation) src between the grids of two levels."""
    check(lib.mlq_transfer_add(src_level.handle, dst_level.handle, 1 if space else 0, 1 if time else 0, int(rows),
                               float(alpha), _ptr(src), _ptr(dst), _stream()))
    return dst


def tet_locate(mesh: dict, pts):
    """(node (P x 4) int64, weight (P x 4)) host arrays: P1 interpolation of the tetrahedral mesh
    (mesh["xyz"], mesh["tets"]) at the points (P x 3)."""
    xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
    tets = np.ascontiguousarray(mesh["tets"], dtype=np.int32)
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    node = np.zeros((p.shape[0], 4), dtype=np.int64)
    w = np.zeros((p.shape[0], 4))
    check(lib.mlq_tet_locate(xyz.ctypes.data, xyz.shape[0], tets.ctypes.data, tets.shape[0], p.ctypes.data,
                             p.shape[0], node.ctypes.data, w.ctypes.data))
    return node, w


def transfer_add_weighted(src_level, dst_level, node, w, src, dst, alpha=1.0, time=True, rows=1):
    """dst += alpha * (time x weighted space interpolation) src; node, w: device tensors (n_to x K)."""
    K = node.shape[1]
    check(lib.mlq_transfer_add_weighted(src_level.handle, dst_level.handle, 1 if time else 0, int(rows), int(K),
                                        _ptr(node), _ptr(w), float(alpha), _ptr(src), _ptr(dst), _stream()))
    return dst


def field_norm2(level, f, q=0, space=True, rows=1):
    """Squared L^2((0,T); H^q) norms of rows of space-time fields (space=True), or squared
    H^q(0,T) norms of rows of time series (space=False): (rows,) FP64 device tensor."""
    import torch
    out = torch.empty(rows, dtype=torch.float64, device=f.device)
    part = torch.empty((rows, 1024), dtype=torch.float64, device=f.device) if space else None
    check(lib.mlq_field_norm2(level.handle, 1 if space else 0, int(q), int(rows), _ptr(f),
                              None if part is None else _ptr(part), _ptr(out), _stream()))
    return out


def lattice_normals(z, shift, N, first, count, device="cuda"):
    """(s, count) FP64 device tensor of shifted-lattice normals."""
    import torch
    zd = torch.as_tensor(np.asarray(z, dtype=np.int64), device=device)
    sd = torch.as_tensor(np.asarray(shift, dtype=np.float64), device=device)
    s = zd.numel()
    Y = torch.empty((count, s), dtype=torch.float64, device=device)  # column-major s x count
    check(lib.mlq_lattice_normals(_ptr(zd), _ptr(sd), int(s), int(N), int(first), int(count), _ptr(Y), _stream()))
    return Y.t()


def lattice_points(z, shift, N, first, count, uniform=True, device="cuda"):
    """(s, count) FP64 device tensor of shifted-lattice coordinates, uniform on [-1, 1] or Gaussian."""
    import torch
    zd = torch.as_tensor(np.asarray(z, dtype=np.int64), device=device)
    sd = torch.as_tensor(np.asarray(shift, dtype=np.float64), device=device)
    s = zd.numel()
    Y = torch.empty((count, s), dtype=torch.float64, device=device)  # column-major s x count
    check(lib.mlq_lattice_points(_ptr(zd), _ptr(sd), int(s), int(N), int(first), int(count),
                                 MLQ_MAP_UNIFORM if uniform else MLQ_MAP_NORMAL, _ptr(Y), _stream()))
    return Y.t()


def halton(s, first, count, shift=None, uniform=True, device="cuda"):
    """(s, count) FP64 device tensor of Halton coordinates (uniform on [-1, 1] or Gaussian),
    optionally shifted mod 1."""
    import torch
    sd = None if shift is None else torch.as_tensor(np.asarray(shift, dtype=np.float64), device=device)
    Y = torch.empty((count, s), dtype=torch.float64, device=device)  # column-major s x count
    check(lib.mlq_halton(int(s), int(first), int(count), None if sd is None else _ptr(sd),
                         MLQ_MAP_UNIFORM if uniform else MLQ_MAP_NORMAL, _ptr(Y), _stream()))
    return Y.t()


def cbc(N, s, gamma):
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    z = np.zeros(s, dtype=np.int64)
    check(lib.mlq_cbc(int(N), int(s), g.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p)))
    return z


def kl_weights(lam, uniform=False):
    """sqrt(lambda) (normal coordinates) or sqrt(3 lambda) (uniform on [-1, 1]), host array."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros_like(lam)
    check(lib.mlq_kl_weights(lam.ctypes.data_as(C.c_void_p), int(lam.size), MLQ_MAP_UNIFORM if uniform else MLQ_MAP_NORMAL,
                             out.ctypes.data_as(C.c_void_p)))
    return out


def lattice_weights(lam, components=1):
    """Product weights lambda_k / lambda_0, repeated for each component (host array)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.zeros(lam.size * int(components))
    check(lib.mlq_lattice_weights(lam.ctypes.data_as(C.c_void_p), int(lam.size), int(components),
                                  out.ctypes.data_as(C.c_void_p)))
    return out


def fibre_field(theta0, e_circ, e_long, scale):
    """scale (cos theta0 e_circ + sin theta0 e_long) per element (host arrays, n x 3)."""
    th = np.ascontiguousarray(theta0, dtype=np.float64)
    ec = np.ascontiguousarray(e_circ, dtype=np.float64)
    el = np.ascontiguousarray(e_long, dtype=np.float64)
    out = np.zeros((th.size, 3))
    check(lib.mlq_fibre_field(int(th.size), th.ctypes.data_as(C.c_void_p), ec.ctypes.data_as(C.c_void_p),
                              el.ctypes.data_as(C.c_void_p), float(scale), out.ctypes.data_as(C.c_void_p)))
    return out


def accumulate(f_fine, f_coarse, acc):
    n = f_fine.numel()
    check(lib.mlq_accumulate(_ptr(f_fine), _ptr(f_coarse), int(n), _ptr(acc), _stream()))
    return acc


def estimate(kind, f_fine, f_coarse=None, n_per_level=None, n_shifts=1):
    """Host estimator over lists of numpy arrays (per level)."""
    L = len(f_fine)
    ff = [np.ascontiguousarray(a, dtype=np.float64) for a in f_fine]
    fc = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
          for a in (f_coarse or [None] * L)]
    if n_per_level is None:
        n_per_level = [a.size // n_shifts for a in ff]
    npl = np.ascontiguousarray(n_per_level, dtype=np.int64)
    pf = (C.c_void_p * L)(*[a.ctypes.data for a in ff])
    pc = (C.c_void_p * L)(*[(a.ctypes.data if a is not None else None) for a in fc])
    out = EstimateOut()
    check(lib.mlq_estimate(int(kind), L, int(n_shifts), npl.ctypes.data_as(C.c_void_p), C.cast(pf, C.c_void_p),
                           C.cast(pc, C.c_void_p), C.byref(out)))
    return dict(estimate=out.estimate, rmse=out.rmse, level_mean=list(out.level_mean[:L]),
                level_var=list(out.level_var[:L]))


def kl_desc(dim, n, lo, hi, std_dev, corr_len, n_modes, max_rank=None, eps=1e-2, cov_kernel=MLQ_COV_EXP,
            method=MLQ_KL_CHOLESKY):
    """KL descriptor on a Q1 box; method MLQ_KL_EXACT: the exact top eigenpairs to the relative
    residual eps (subspace iteration), else the pivoted Cholesky route (eps: trace criterion)."""
    d = KlDesc()
    d.cov_kernel = int(cov_kernel)
    d.method = int(method)
    d.dim = int(dim)
    for a in range(3):
        d.n[a] = int(n[a]) if a < dim else 1
        d.lo[a] = float(lo[a]) if a < dim else 0.0
        d.hi[a] = float(hi[a]) if a < dim else 1.0
    d.std_dev, d.corr_len = float(std_dev), float(corr_len)
    d.n_modes = int(n_modes)
    d.max_rank = int(max_rank if max_rank is not None else 2 * n_modes)
    d.eps = float(eps)
    return d


def kl_desc_tet(mesh: dict, std_dev, corr_len, n_modes, max_rank=None, eps=1e-2, cov_kernel=MLQ_COV_EXP):
    """KL descriptor on the vertices of a tetrahedral mesh (mesh["xyz"], mesh["tets"])."""
    d = KlDesc()
    d.cov_kernel = int(cov_kernel)
    xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
    tets = np.ascontiguousarray(mesh["tets"], dtype=np.int32)
    d.dim, d.mesh_kind = 3, MLQ_MESH_P1_TET
    d.n_vert, d.n_tet = xyz.shape[0], tets.shape[0]
    d.xyz = xyz.ctypes.data_as(C.POINTER(C.c_double))
    d.tets = tets.ctypes.data_as(C.POINTER(C.c_int32))
    d._keep = (xyz, tets)
    d.std_dev, d.corr_len = float(std_dev), float(corr_len)
    d.n_modes = int(n_modes)
    d.max_rank = int(max_rank if max_rank is not None else 2 * n_modes)
    d.eps = float(eps)
    return d


def kl_transfer_tet(kd: KlDesc, psi, mesh: dict, device="cuda"):
    """Phi_l (n_tet x M, device FP64) at the centroids of a tetrahedral level (non-nested)."""
    import torch
    xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
    tets = np.ascontiguousarray(mesh["tets"], dtype=np.int32)
    P = tets.shape[0]
    nbytes = C.c_size_t()
    check(lib.mlq_kl_transfer_tet_bytes(P, C.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    phi = torch.empty((P, kd.n_modes), dtype=torch.float64, device=device)
    check(lib.mlq_kl_transfer_tet(C.byref(kd), _ptr(psi), xyz.shape[0], xyz.ctypes.data_as(C.c_void_p), P,
                                  tets.ctypes.data_as(C.c_void_p), _ptr(ws), nbytes.value, _ptr(phi), _stream()))
    return phi


def kl_modes(kd: KlDesc, device="cuda"):
    """Returns (lambda (M,) numpy, psi (M, n) device tensor [row k = mode k], rank, relative residual)."""
    import torch
    nbytes = C.c_size_t()
    check(lib.mlq_kl_workspace_bytes(C.byref(kd), C.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    n = 1
    for a in range(kd.dim):
        n *= kd.n[a]
    if kd.mesh_kind == MLQ_MESH_P1_TET:
        n = kd.n_vert
    psi = torch.empty((kd.n_modes, n), dtype=torch.float64, device=device)  # column-major n x M
    lam = np.zeros(kd.n_modes)
    rank, resid = C.c_int32(), C.c_double()
    check(lib.mlq_kl_modes(C.byref(kd), _ptr(ws), nbytes.value, lam.ctypes.data_as(C.c_void_p), _ptr(psi),
                           C.byref(rank), C.byref(resid), _stream()))
    del ws
    return lam, psi, int(rank.value), float(resid.value)


def kl_dimension(kd: KlDesc, device="cuda"):
    """The stochastic dimension M fixed by the truncation tolerance kd.eps (the pivoted Cholesky
    rank at which trace(C - L L^T) <= eps trace(C)), and the relative residual there."""
    m = kd.n_modes
    kd.n_modes = 0
    try:
        _, _, rank, resid = kl_modes(kd, device=device)
    finally:
        kd.n_modes = m
    return rank, resid


def kl_transfer(kd: KlDesc, psi, level: dict, device="cuda"):
    """Phi_l (P x M, device FP64) at the element centres of a Q1 box level."""
    import torch
    dim = kd.dim
    n = np.array([level["n"][a] if a < dim else 2 for a in range(3)], dtype=np.int64)
    lo = np.array([level["lo"][a] if a < dim else 0.0 for a in range(3)], dtype=np.float64)
    hi = np.array([level["hi"][a] if a < dim else 1.0 for a in range(3)], dtype=np.float64)
    P = int(np.prod(n[:dim] - 1))
    phi = torch.empty((P, kd.n_modes), dtype=torch.float64, device=device)
    check(lib.mlq_kl_transfer(C.byref(kd), _ptr(psi), n.ctypes.data_as(C.c_void_p), lo.ctypes.data_as(C.c_void_p),
                              hi.ctypes.data_as(C.c_void_p), _ptr(phi), _stream()))
    return phi
