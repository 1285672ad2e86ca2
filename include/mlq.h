/*
 * mlq.h -- C ABI of the MI355X (gfx950) library for the batched per-sample
 * space-time solves of the parametric monodomain equation and the single- and
 * multilevel quadrature estimators built on them.
 *
 * Method (Ben Bader, Harbrecht, Krause, Multerer, Quaglino, Schmidlin,
 * "Space-time multilevel quadrature methods and their application for cardiac
 * electrophysiology"):
 *   - conductivity per element, eq. (AdmV):  G = s_t I + (s_l - s_t) f f^T,
 *     f = (cos theta, sin theta[, 0]), theta the fibre angle of the element;
 *   - fibre angle field, eq. (KLlowrank) with the element-midpoint transfer of
 *     Section 4:  theta = theta0 + Phi diag(sqrt(lambda)) y;
 *   - Crank-Nicolson space-time system eq. (st-system) with the reaction term of
 *     eq. (mono_disc), I_ion of eq. (ionic_term); the block lower-bidiagonal
 *     system eq. (system_C) is solved by forward substitution in time, each time
 *     level by Newton's method with the Jacobian of Section 3.2 and a batched
 *     GMRES (Section 3.3);
 *   - quantities of interest of Section 2.4 (mean potential at the end time,
 *     mean activation time);
 *   - estimators eqs. (SL), (StandardML), (PimpedML) of Section 4.
 *
 * Conventions
 *   Ownership: the library never allocates device memory at run time.  Every
 *     device buffer (level blob, fields, workspace, outputs) is passed in by the
 *     caller and stays owned by the caller; the one exception is the static
 *     workspace array of mlq_solve_batch_static, part of the library's code
 *     object on each GPU, and the twiddle tables hipFFT keeps while the plans
 *     of an MLQ_KL_EXACT mlq_kl_modes call exist (created and destroyed inside
 *     that call).  Host arrays given to mlq_create_level are
 *     copied during the call.  Each level object owns a few bytes of pinned host
 *     memory for convergence flags.
 *   Layouts: a batch of B samples on a level with n nodes and P elements stores
 *     nodal vectors sample-major, [B][n]; element fields [B][P].  Nodes and
 *     elements of a Q1 box are numbered with axis 0 fastest.
 *   Streams: every call takes a hipStream_t (passed as void*; NULL = the null
 *     stream).  mlq_sample_fields, mlq_apply, mlq_lattice_normals and
 *     mlq_accumulate only enqueue work.  mlq_solve_batch steers Newton and GMRES
 *     from the host and returns after the work on the stream has finished.
 *   Errors: every entry point returns an mlq_status; nothing throws across the
 *     ABI.  mlq_last_error() returns a thread-local message for the last error.
 *   Determinism: all reductions have a fixed order, so FP64 results are bitwise
 *     reproducible for a fixed batch.
 */
#ifndef MLQ_H
#define MLQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLQ_OK = 0,
  MLQ_EINVAL = -1,  /* invalid argument or descriptor */
  MLQ_EHIP = -2,    /* a HIP runtime call failed */
  MLQ_ENOCONV = -3, /* at least one sample did not converge (see status array) */
  MLQ_ESIZE = -4,   /* a caller-provided buffer is too small */
  MLQ_ESTATE = -5   /* object used in a wrong state */
} mlq_status;

typedef enum { MLQ_FP64 = 0, MLQ_MIXED = 1 } mlq_precision;
typedef enum { MLQ_QOI_MEAN_U_FINAL = 0, MLQ_QOI_MEAN_ACT_TIME = 1 } mlq_qoi;
typedef enum { MLQ_MESH_Q1_BOX = 0, MLQ_MESH_P1_TET = 1 } mlq_mesh_kind;
typedef enum {
  MLQ_GUESS_PREVIOUS = 0,
  MLQ_GUESS_EXTRAPOLATE = 1,
  MLQ_GUESS_REFERENCE = 2,       /* r_(k+1): the unperturbed reference solution (mlq_set_reference) */
  MLQ_GUESS_REFERENCE_LOCAL = 3  /* u_k + r_(k+1) - r_k: the reference's increment on the sample's state */
} mlq_newton_guess;
typedef enum { MLQ_DIFF_FIBRE = 0, MLQ_DIFF_ISO = 1, MLQ_DIFF_VECTOR = 2 } mlq_diffusion;
typedef enum { MLQ_COV_EXP = 0, MLQ_COV_SQEXP = 1 } mlq_cov_kernel;

/* per-sample status codes written by mlq_solve_batch */
enum { MLQ_SAMPLE_OK = 0, MLQ_SAMPLE_NOCONV = 1, MLQ_SAMPLE_NAN = 2 };

/* Description of one level (Section 3.1: mesh, time grid; Section 5.1: model
 * constants).  The arrays are read during mlq_create_level; they are host
 * pointers unless arrays_on_device is 1. */
typedef struct {
  int32_t dim;        /* 2 or 3 (3 for tetrahedra) */
  int32_t mesh_kind;  /* MLQ_MESH_Q1_BOX or MLQ_MESH_P1_TET */
  int64_t n[3];       /* box: nodes per axis (>= 2 each; unused axes ignored; at most 2^27 nodes in total) */
  double lo[3], hi[3];/* box corners */
  int32_t n_steps;    /* time steps on [0, t_end]; dt = t_end / n_steps */
  double t_end;
  double alpha, u_rest, u_th, u_peak; /* eq. (ionic_term) */
  double sigma_l, sigma_t;            /* along / across the fibre */
  double stim_lo[3], stim_hi[3];      /* stimulus box (indicator in space) */
  double stim_t_on, stim_t_off;       /* stimulus active on [t_on, t_off) */
  double stim_amp;                    /* stimulus rate */
  int32_t n_modes;                    /* M: KL modes (<= 1024) */
  const double* phi;                  /* P x M row-major: modes at element centres */
  const double* sqrt_lambda;          /* M */
  const double* theta0;               /* P, or NULL for theta0 = 0 */
  int32_t prec;                       /* mlq_precision */
  int32_t qoi;                        /* mlq_qoi */
  double newton_tol;                  /* normwise backward error of each step */
  double inner_tol;                   /* relative residual of each GMRES solve */
  int32_t max_newton;                 /* Newton iterations per step */
  int32_t max_inner;                  /* GMRES iterations per Newton step (<= 64) */
  int32_t max_batch;                  /* largest batch used with this level (<= 65535) */
  int32_t arrays_on_device;           /* 1: phi, sqrt_lambda, theta0 are device pointers */
  /* P1 tetrahedra (mesh_kind = MLQ_MESH_P1_TET; Section 3.1 with the P1 space of a
   * shape-regular tetrahedral mesh).  Host arrays, always; copied at creation.
   * The elements of the level are the tetrahedra (P = n_tet); the fibre of
   * element e is f = cos(theta_e) e_circ[e] + sin(theta_e) e_long[e], eq. (AdmV)
   * with V = sigma_l f.  The stimulus is the ball (stim_center, stim_radius):
   * load F = M chi with chi the indicator of the vertices inside it.  The
   * Krylov preconditioner is the diagonal of the Jacobian. */
  int64_t n_vert, n_tet;              /* vertices (<= 2^27), tetrahedra (<= 2^27) */
  const double* xyz;                  /* n_vert x 3 */
  const int32_t* tets;                /* n_tet x 4 vertex indices, positively oriented */
  const double* e_circ;               /* n_tet x 3 unit vectors */
  const double* e_long;               /* n_tet x 3 unit vectors orthogonal to e_circ */
  double stim_center[3], stim_radius;
  /* Newton initial guess of step k + 1 (the discrete solution does not depend on it
   * beyond the stopping test): 0 = u_k, the previous time level (the multiple-time-block
   * strategy of Section 3.3 with one step per block); 1 = 2 u_k - u_{k-1}, linear
   * extrapolation from the two previous time levels (u_k at the first step); 2 and 3 start from
   * an unperturbed reference solution r (Section 3.3, the sample-based Newton initial guess,
   * read for time stepping): 2 = r_(k+1) (the global guess), 3 = u_k + (r_(k+1) - r_k) (the
   * local one); r is set with mlq_set_reference. */
  int32_t newton_guess;               /* mlq_newton_guess */
  /* Conductivity model of the elements: MLQ_DIFF_FIBRE: the field is the fibre angle theta,
   * G = sigma_t I + (sigma_l - sigma_t) f f^T with f = (cos theta, sin theta[, 0]) on boxes and
   * f = cos theta e_circ + sin theta e_long on tetrahedra, eq. (AdmV) with V = sigma_l f;
   * MLQ_DIFF_ISO: the field is a scalar conductivity v, G = max(v, sigma_t) I (isotropic
   * diffusion, the paper's cube and idealised-ventricle experiments of Section 5.2; sigma_t is
   * the lower bound b_min that keeps G positive definite, sigma_l is unused);
   * MLQ_DIFF_VECTOR (tetrahedra only): eq. (AdmV) itself with a random vector field,
   * G = g I + (|V| - g) V V^T / V^T V, g = sigma_t, V = v_mean + the field, whose three
   * components the solve and apply calls take component-major ([3][B][P]: component c of
   * sample b at (c B + b) P + e). */
  int32_t diffusion;
  const double* v_mean;               /* MLQ_DIFF_VECTOR: n_tet x 3 host array, E[V] per element */
} mlq_level_desc;

typedef struct mlq_level mlq_level; /* opaque */

/* Device bytes the level blob needs (Phi in FP64 and FP32, theta0, load vector,
 * node weights).  Returns MLQ_EINVAL for an invalid descriptor. */
mlq_status mlq_level_bytes(const mlq_level_desc* desc, size_t* level_bytes);

/* Validates desc, copies its arrays into level_mem_dev (>= mlq_level_bytes,
 * 256-byte aligned), waits for the copies on stream, returns the level in *out.
 * Rejects (MLQ_EINVAL) a descriptor with dt * |min I_ion'| >= 1, where the step
 * equation may have several roots. */
mlq_status mlq_create_level(const mlq_level_desc* desc, void* level_mem_dev, size_t level_bytes,
                            void* hip_stream, mlq_level** out);

void mlq_destroy_level(mlq_level* level);

/* Level geometry: nodes n and elements P per sample. */
mlq_status mlq_level_sizes(const mlq_level* level, int64_t* n_nodes, int64_t* n_elems);

/* Workspace bytes for one mlq_solve_batch call with `batch` samples: per sample and
 * node four FP64 state vectors, and in the inner precision the GMRES basis (max_inner + 1
 * vectors), on boxes the preconditioned basis (max_inner vectors), and three more. */
mlq_status mlq_workspace_bytes(const mlq_level* level, int32_t batch, size_t* ws_bytes);

/* KL synthesis, eq. (KLlowrank) at the level's element centres:
 *   theta[b][p] = theta0[p] + sum_k phi[p][k] sqrt_lambda[k] Y[k + M b].
 * Y_dev: M x batch column-major FP64 (column b = sample b).
 * theta_dev: batch x P, FP32 when the level is MLQ_MIXED, else FP64.
 * Enqueues only. */
mlq_status mlq_sample_fields(mlq_level* level, const double* Y_dev, int32_t batch, void* theta_dev,
                             void* hip_stream);

/* Solves the space-time problem of every sample of the batch (fibre angles
 * theta_dev as produced by mlq_sample_fields) and writes the quantity of
 * interest qoi_dev[b] (FP64), a status word status_dev[b] (MLQ_SAMPLE_*) and
 * iters_dev[2 b] = Newton iterations, iters_dev[2 b + 1] = GMRES iterations
 * (operator applications) summed over all steps.  ws_dev: >= mlq_workspace_bytes,
 * 256-byte aligned.  Returns after the stream has finished; MLQ_ENOCONV if any
 * sample failed (its QoI is still written). */
mlq_status mlq_solve_batch(mlq_level* level, const void* theta_dev, int32_t batch, void* ws_dev,
                           size_t ws_bytes, double* qoi_dev, int32_t* status_dev, int64_t* iters_dev,
                           void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mlq_solve_batch with the library's own static
 * workspace instead of a caller's buffer.  Same arguments (minus the workspace), results and
 * errors as mlq_solve_batch; allocates nothing.  The workspace is a device array of
 * MLQ_STATIC_WS_BYTES (64 MiB) that every GPU the library runs on holds once, from the first
 * use of the library on it until the process ends.  MLQ_ESIZE when the batch needs more
 * (mlq_workspace_bytes tells); MLQ_EINVAL when the current device is not the level's.  All calls
 * on one GPU share its array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and give undefined results.  The array keeps the last call's contents; the solve
 * initialises everything it reads, so nothing has to be cleared between calls. */
#define MLQ_STATIC_WS_BYTES (64u << 20)
mlq_status mlq_solve_batch_static(mlq_level* level, const void* theta_dev, int32_t batch, double* qoi_dev,
                                  int32_t* status_dev, int64_t* iters_dev, void* hip_stream);

/* Same as mlq_solve_batch but stops after `n_steps` steps (<= the level's) and
 * also copies the final nodal state (batch x n, FP64) to u_out_dev (may be
 * NULL) and the per-node activation times (batch x n, FP64, -1 = not
 * activated) to act_out_dev (may be NULL). QoIs refer to t = n_steps * dt. */
mlq_status mlq_solve_batch_ex(mlq_level* level, const void* theta_dev, int32_t batch, int32_t n_steps,
                              void* ws_dev, size_t ws_bytes, double* qoi_dev, int32_t* status_dev,
                              int64_t* iters_dev, double* u_out_dev, double* act_out_dev,
                              void* hip_stream);

/* All-at-once solve in time blocks (Section 3.3, the multiple-time-blocks strategy; eq. (system_C)
 * with the reaction term of eq. (mono_disc)), 3D box levels: [0, T] is cut into K = n_steps /
 * steps_per_block blocks of m' = steps_per_block steps, solved one after the other, each by Newton's
 * method on all m' unknown time levels at once (the block's first level couples to the previous
 * block's final state), every Newton system by GMRES on the whole block with the block-Jacobi
 * preconditioner (per time level M (I + D), as in the time-stepping solve).  m' = n_steps is the
 * direct method over the whole interval.  Newton's first iterate of a block, `guess`:
 *   MLQ_GUESS_PREVIOUS          the previous block's final state at every time level (the
 *                               multiple-time-blocks start);
 *   MLQ_GUESS_REFERENCE         the reference solution r (mlq_set_reference) at the block's time
 *                               levels (the global sample-based guess);
 *   MLQ_GUESS_REFERENCE_LOCAL   the previous block's final state plus the reference's increment
 *                               since the block's start (the local sample-based guess).
 * The discrete solution is the time-stepping one (the block system is block lower triangular), so
 * qoi_dev, status_dev and iters_dev mean what they mean for mlq_solve_batch; iters_dev[2 b] counts
 * block Newton iterations, iters_dev[2 b + 1] block GMRES iterations (each applies the operator to
 * m' time levels).  u_out_dev (may be NULL): the final state, batch x n.  The level's max_inner
 * bounds the GMRES iterations per Newton step (the block-Jacobi-preconditioned block operator needs
 * about m' more than one step does).  ws_dev >= mlq_workspace_bytes_blocks, 256-byte aligned.
 * MLQ_EINVAL unless steps_per_block divides n_steps, the level is a 3D box and batch (m' + 1) <=
 * 65535; MLQ_ESTATE for a reference guess without a reference.  Returns after the stream has
 * finished. */
mlq_status mlq_workspace_bytes_blocks(const mlq_level* level, int32_t batch, int32_t steps_per_block,
                                      size_t* ws_bytes);
mlq_status mlq_solve_batch_blocks(mlq_level* level, const void* theta_dev, int32_t batch, int32_t steps_per_block,
                                  int32_t guess, void* ws_dev, size_t ws_bytes, double* qoi_dev, int32_t* status_dev,
                                  int64_t* iters_dev, double* u_out_dev, void* hip_stream);

/* Field quantities of interest (Section 2.4: the transmembrane potential u itself, the
 * activation map, the action potential u(x0, t) at a point), streamed while a batch is
 * solved.  Each output pointer may be NULL (that output is skipped).  Device arrays, FP64:
 *   u_sum    (n_steps + 1) x n, ACCUMULATED: u_sum[k n + i] += sum_b u_b(x_i, t_k) for
 *            k = 0 .. n_steps (row 0 holds the initial state), the space-time field summed
 *            over the batch's samples;
 *   act_sum  n, ACCUMULATED: act_sum[i] += sum_b a_b(x_i), the activation times with nodes
 *            that never reach u_th counted at the stop time (as for MLQ_QOI_MEAN_ACT_TIME);
 *   probe    batch x n_probe x (n_steps + 1), WRITTEN: probe[(b n_probe + p)(n_steps + 1) + k]
 *            = sum_j probe_w[8 p + j] u_b(node probe_node[8 p + j], t_k);
 *   probe_sum n_probe x (n_steps + 1), ACCUMULATED: probe_sum[p (n_steps + 1) + k] += the sum
 *            over the batch of the same values (the action potential summed over samples).
 * Accumulated outputs let several batches add into one sum; the caller clears them first.
 * probe_node and probe_w are HOST arrays of n_probe x 8 entries (unused slots: weight 0 and
 * any valid node), e.g. from mlq_probe_weights; 1 <= n_probe <= 16 when probe or probe_sum
 * is not NULL.
 * MLQ_EINVAL for a node outside the level or a weight that is not finite. */
typedef struct {
  double* u_sum;
  double* act_sum;
  double* probe;
  int32_t n_probe;
  const int64_t* probe_node;
  const double* probe_w;
  double* probe_sum;
} mlq_field_out;

/* Lane layout of the 3D box kernels (a tuning knob): lanes_x = 8 (waves of 8 x 8 lanes, each
 * owning 7 x 7 nodes per plane) or 16 (16 x 4 lanes, 15 x 3 nodes, full 128-byte rows in FP64),
 * 0 = chosen by the grid width (16 from 48 nodes along x).  The operators give the same
 * results in every layout; the Gram-Schmidt projections fused into the apply are summed over
 * other partitions, so solves agree within rounding.  The workspace size depends on it: query
 * mlq_workspace_bytes after a change.  MLQ_EINVAL for other values or levels. */
mlq_status mlq_set_lane_layout(mlq_level* level, int32_t lanes_x);

/* GMRES launch schedule of the level's solves (a tuning knob, Section 3.3's Krylov iteration):
 * iterations = 0 launches the GMRES iterations one at a time and reads each iteration's count of
 * still-active samples on the host (one read per iteration, one iteration behind the launches);
 * iterations = J (1..64) runs them in blocks of J captured once into a HIP graph (per workspace,
 * field array, batch and block) and replayed, with one count read per block, one block behind.
 * Samples that have converged skip the work of every later iteration in either schedule, so the
 * results are the same bit for bit; a block costs up to J - 1 iterations of launches that find no
 * active sample.  Captured launches are not timed (mlq_timing_enable).  MLQ_EINVAL for other
 * values. */
mlq_status mlq_set_gmres_block(mlq_level* level, int32_t iterations);

/* Persistent per-sample solves of a small 3D box level (a launch knob for the latency-bound
 * coarse levels of a multilevel estimator; Section 3.3's time stepping with Newton-GMRES, the
 * same method and stopping tests as the batched path).  on = 1: mlq_solve_batch and
 * mlq_solve_batch_ex run each sample's whole time loop inside one workgroup of a single
 * launch (workgroups walk the batch), with no host round trip: the call only enqueues work on
 * the stream and returns MLQ_OK; per-sample failures are reported in status_dev (check with
 * mlq_check after synchronising), and the iteration counts in iters_dev.  Applies when the
 * level's nodal vector fits 64 KiB (n_nodes x 8 bytes in FP64, x 4 in mixed precision) and the
 * call asks for no field outputs and no reference Newton guess; other calls keep the batched
 * path.  Results agree with the batched path within the stopping tests (a different summation
 * order).  on = 0: the batched path (default).  MLQ_EINVAL for a tetrahedral, 2D or too large
 * level when on = 1. */
mlq_status mlq_set_persistent(mlq_level* level, int32_t on);

/* Reference space-time solution for the Newton guesses MLQ_GUESS_REFERENCE(_LOCAL): ref_dev
 * is (n_steps + 1) x n FP64 on the device, e.g. the u_sum of a one-sample solve of the
 * unperturbed field; the level keeps the pointer (the caller keeps the memory alive while it
 * solves; NULL clears it).  Without a reference these guesses start from u_k, as
 * MLQ_GUESS_PREVIOUS (which is how the reference itself is computed). */
mlq_status mlq_set_reference(mlq_level* level, const double* ref_dev);

/* mlq_solve_batch with field outputs (see mlq_field_out); same arguments, results and
 * errors otherwise. */
mlq_status mlq_solve_batch_fields(mlq_level* level, const void* theta_dev, int32_t batch, void* ws_dev,
                                  size_t ws_bytes, double* qoi_dev, int32_t* status_dev, int64_t* iters_dev,
                                  const mlq_field_out* fields, void* hip_stream);

/* Interpolation weights of points for probe outputs, host only: for point p (xyz_host[3 p ..],
 * the unused coordinate of a 2D box ignored) the nodes of the box cell that contains it and
 * their Q1 weights, node_out[8 p + j] and w_out[8 p + j] (2D: 4 used, the rest weight 0).
 * MLQ_EINVAL for a point outside the box or a tetrahedral level (on tetrahedra, probe a
 * vertex: node v with weight 1). */
mlq_status mlq_probe_weights(const mlq_level* level, const double* xyz_host, int32_t n_points, int64_t* node_out,
                             double* w_out);

/* Transfer of fields between the grids of two levels (Section 5, the error measures: the
 * tensor product of the space and the time interpolation), accumulated:
 *   dst += alpha * (T x S) src.
 * space = 1: S is the Q1 interpolation from the nodes of `from` to those of `to` (box levels
 * over the same box, (n_to - 1) a multiple of (n_from - 1) on every axis), else the identity
 * on a single column;  time = 1: T is the linear interpolation from the time nodes of `from`
 * to those of `to` (the same end time, n_steps of `to` a multiple of that of `from`), else the
 * identity on a single time node.  Layout, row-major: src rows x T_f x S_f, dst rows x T_t x
 * S_t with T = n_steps + 1 or 1 and S = n_nodes or 1, e.g. u_sum (rows = 1, space and time),
 * act_sum (rows = 1, space only), probe series (rows = batch n_probe, time only).  Device
 * arrays of those sizes; from == to gives the identity.  Enqueues only. */
mlq_status mlq_transfer_add(const mlq_level* from, const mlq_level* to, int32_t space, int32_t time, int64_t rows,
                            double alpha, const double* src_dev, double* dst_dev, void* hip_stream);

/* P1 interpolation weights of points in a tetrahedral mesh (host only): for point p the four
 * vertices node_out[4 p ..] of the tetrahedron found for it and the weights w_out[4 p ..], its
 * barycentric coordinates.  The tetrahedron is the one with the largest smallest barycentric
 * coordinate (lowest index on ties within 1e-12), searched in a uniform bucket grid; a point
 * outside the mesh (the boundary of a finer non-nested mesh) takes the best tetrahedron of the
 * neighbouring cells, its negative coordinates clipped to 0 and the rest renormalised (§4, the
 * transfer between non-nested meshes).  xyz: n_vert x 3, tets: n_tet x 4, pts: n_pts x 3, host.
 * MLQ_EINVAL for a vertex index out of range or a failed search. */
mlq_status mlq_tet_locate(const double* xyz, int64_t n_vert, const int32_t* tets, int64_t n_tet, const double* pts,
                          int64_t n_pts, int64_t* node_out, double* w_out);

/* Transfer between the grids of two levels with explicit interpolation weights in space (for
 * non-nested meshes, e.g. from mlq_tet_locate at the target level's vertices), accumulated:
 *   dst[r][k'][i'] += alpha * sum_k T[k'][k] sum_{j < K} w_dev[i' K + j] src[r][k][node_dev[i' K + j]],
 * with T the linear time interpolation from `from`'s time nodes to `to`'s (time = 1, nested time
 * grids with the same end time) or the identity on one time node (time = 0).  node_dev, w_dev:
 * device arrays of n_to x K (1 <= K <= 8); node indices are clamped to [0, n_from).  src: rows x
 * T_f x n_from, dst: rows x T_t x n_to (T = n_steps + 1 or 1), device.  Enqueues only. */
mlq_status mlq_transfer_add_weighted(const mlq_level* from, const mlq_level* to, int32_t time, int64_t rows,
                                     int32_t K, const int64_t* node_dev, const double* w_dev, double alpha,
                                     const double* src_dev, double* dst_dev, void* hip_stream);

/* Squared error norms of fields on a level's grids (eq. (space-time-error), eq. (point-error)):
 *   space = 1: f_dev is rows x (n_steps + 1) x n (space-time fields of a box level);
 *     out_dev[r] = ||f_r||^2 in L^2((0, T); H^q(D)) of the interpolant that is Q1 in space and
 *     linear in time, integrated exactly (q = 1: the full H^1 norm, L^2 part included);
 *     part_dev: rows x 1024 FP64 device scratch for partial sums;
 *   space = 0: f_dev is rows x (n_steps + 1) (time series, e.g. probe outputs);
 *     out_dev[r] = ||f_r||^2 in H^q(0, T) of the linear interpolant; part_dev unused.
 * q is 0 or 1, 1 <= rows <= 65535; out_dev: rows FP64 on the device.  The sums run in a fixed
 * order (results do not vary between runs).  Enqueues only. */
mlq_status mlq_field_norm2(const mlq_level* level, int32_t space, int32_t q, int64_t rows, const double* f_dev,
                           double* part_dev, double* out_dev, void* hip_stream);

/* Jacobian of one step (Section 3.2) applied matrix-free to a batch:
 *   y = M ((1 + d) x) + dt/2 K_G x,
 * with G per element from theta (level precision).  x, d, y: batch x n in the
 * level's inner precision (FP32 when MLQ_MIXED, else FP64).  Enqueues only. */
mlq_status mlq_apply(mlq_level* level, const void* theta_dev, int32_t batch, const void* x_dev,
                     const void* d_dev, void* y_dev, void* ws_dev, size_t ws_bytes, void* hip_stream);

/* Check after a synchronisation: MLQ_ENOCONV if any status is not MLQ_SAMPLE_OK. */
mlq_status mlq_check(const int32_t* status_host, int32_t batch);

/* Randomly shifted rank-1 lattice points mapped to N(0,1) coordinates:
 *   Y[k + s (i - first)] = Phi^-1( frac( ((i z_k) mod N) / N + shift_k ) ),
 * i = first .. first + count - 1, k < s, x clamped to [2^-53, 1 - 2^-53].
 * z_dev (s integers, 0 < z_k < N) and shift_dev (s values in [0, 1)) are device
 * arrays; Y_dev is s x count column-major FP64.  Enqueues only. */
mlq_status mlq_lattice_normals(const int64_t* z_dev, const double* shift_dev, int32_t s, int64_t N,
                               int64_t first, int32_t count, double* Y_dev, void* hip_stream);

/* Halton points, the paper's quasi-Monte Carlo rule (Section 5.1, quadrature methods):
 *   x_k(i) = phi_{p_k}(i), p_k the (k+1)-th prime, phi_p(i) = sum_j d_j p^(-j-1) for the base-p
 *   digits i = sum_j d_j p^j, rounded once from the exact rational; with shift_dev (s values in
 *   [0, 1), device) x_k = x_k + shift_k, minus 1 if that reached 1 (randomised QMC);
 *   map MLQ_MAP_UNIFORM: Y = 2x - 1, the coordinates y in [-1, 1] of Section 4;
 *   map MLQ_MAP_NORMAL:  Y = Phi^-1(x), x clamped to [2^-53, 1 - 2^-53].
 * Y[k + s (i - first)] for i = first .. first + count - 1, column-major s x count FP64 on the
 * device (may be NULL when count = 0).  shift_dev may be NULL (no shift).  1 <= s <= 1024,
 * first >= 0, first + count <= 2^32; MLQ_EINVAL otherwise.  Point 0 is the origin; samplers usually
 * start at first = 1.  Enqueues only. */
typedef enum { MLQ_MAP_NORMAL = 0, MLQ_MAP_UNIFORM = 1 } mlq_coordinate_map;
mlq_status mlq_halton(int32_t s, int64_t first, int32_t count, const double* shift_dev, int32_t map, double* Y_dev,
                      void* hip_stream);

/* The same shifted lattice points in either coordinate map (mlq_coordinate_map, declared with
 * mlq_halton): MLQ_MAP_NORMAL as mlq_lattice_normals, MLQ_MAP_UNIFORM y = 2x - 1, the uniform
 * coordinates on [-1, 1] of the paper's parametrisation (Section 4).  Same arguments, layout and
 * errors as mlq_lattice_normals otherwise.  Enqueues only. */
mlq_status mlq_lattice_points(const int64_t* z_dev, const double* shift_dev, int32_t s, int64_t N, int64_t first,
                              int32_t count, int32_t map, double* Y_dev, void* hip_stream);

/* Mode weights of eq. (KLlowrank) for the distribution of the coordinates (host only):
 *   out[k] = sqrt(lambda[k])      map = MLQ_MAP_NORMAL  (standard normal y_k, E[y^2] = 1),
 *   out[k] = sqrt(3 lambda[k])    map = MLQ_MAP_UNIFORM (y_k uniform on [-1, 1], E[y^2] = 1/3;
 *                                  the paper's parametrisation, Section 5.1),
 * so that the field sum_k out[k] psi_k y_k has the covariance sum_k lambda_k psi_k psi_k^T in
 * either case; out is the sqrt_lambda array of mlq_level_desc.  lambda, out: M host values.
 * MLQ_EINVAL for a negative or non-finite eigenvalue or an unknown map. */
mlq_status mlq_kl_weights(const double* lambda, int32_t M, int32_t map, double* out);

/* Product weights of the lattice construction (mlq_cbc) from the KL eigenvalues (host only):
 * gamma_out[c M + k] = lambda[k] / lambda[0] for each of `components` independent fields with
 * the same basis (the coordinates of component c follow those of component c - 1).
 * lambda: M host values, descending, lambda[0] > 0; gamma_out: components x M host values. */
mlq_status mlq_lattice_weights(const double* lambda, int32_t M, int32_t components, double* gamma_out);

/* Mean field of the vector conductivity model (host only): the rule-based fibre of angle theta0
 * in the element frame, scaled, eq. (AdmV) with V = scale f:
 *   v_out[3 e + a] = scale (cos theta0[e] e_circ[3 e + a] + sin theta0[e] e_long[3 e + a]),
 * e < n; with scale = sigma_l this is the v_mean array of mlq_level_desc for MLQ_DIFF_VECTOR. */
mlq_status mlq_fibre_field(int64_t n, const double* theta0, const double* e_circ, const double* e_long, double scale,
                           double* v_out);

/* Component-by-component generating vector of an N-point rank-1 lattice in s
 * dimensions, product weights gamma (s), minimising the shift-averaged
 * worst-case error of the unanchored Sobolev space.  Host only. */
mlq_status mlq_cbc(int64_t N, int32_t s, const double* gamma, int64_t* z_out);

/* Level difference and accumulation in FP64 on the device:
 *   Y_i = f_fine[i] - f_coarse[i] (f_coarse may be NULL: Y_i = f_fine[i]),
 *   acc[0] += count, acc[1] += sum Y_i, acc[2] += sum Y_i^2   (fixed order). */
mlq_status mlq_accumulate(const double* f_fine_dev, const double* f_coarse_dev, int32_t count,
                          double* acc_dev, void* hip_stream);

typedef enum {
  MLQ_EST_MC = 0,          /* eq. (SL), Monte Carlo */
  MLQ_EST_MLMC = 1,        /* eq. (StandardML), independent MC sets per level */
  MLQ_EST_MLQMC = 2,       /* eq. (StandardML), randomly shifted lattice rules */
  MLQ_EST_COMBINATION = 3  /* eq. (PimpedML), nested point sets */
} mlq_estimator;

typedef struct {
  double estimate;
  double rmse;              /* estimated root mean square error */
  int32_t n_levels;
  double level_mean[16];
  double level_var[16];     /* sample variance of the level differences (MC kinds) */
} mlq_estimate_out;

/* Host FP64 estimators, plain sums in sample order.
 *  MLQ_EST_MC:    n_levels = 1, f_fine[0] has n_per_level[0] values.
 *  MLQ_EST_MLMC:  f_fine[l], f_coarse[l] (ignored for l = 0) have n_per_level[l] values.
 *  MLQ_EST_MLQMC: f_fine[l], f_coarse[l] have n_shifts * n_per_level[l] values, shift-major.
 *  MLQ_EST_COMBINATION: n_per_level[l] = points of Q_l (nested, increasing);
 *     f_fine[j] = F_j at the first n_per_level[L - j] points. */
mlq_status mlq_estimate(int32_t kind, int32_t n_levels, int32_t n_shifts, const int64_t* n_per_level,
                        const double* const* f_fine, const double* const* f_coarse,
                        mlq_estimate_out* out);

/* ---- KL basis set-up (Section 2.3; element-midpoint transfer of Section 4) ----
 * Covariance C(x, x') = std_dev^2 exp(-|x - x'|_2 / corr_len) (or the squared-exponential
 * kernel, cov_kernel) on the nodes of a uniform Q1 box or of a tetrahedral mesh (normally
 * the finest level).  eq. (algEig) is reduced by a
 * pivoted Cholesky factor C ~ L L^T (largest remaining diagonal first, lowest
 * index on ties; stops at rank max_rank, or once the rank is >= n_modes and
 * trace(C - L L^T) <= eps trace(C)) to eq. (redEig), L^T M L v~ = lambda v~. */
typedef struct {
  int32_t dim;          /* 2 or 3 */
  int64_t n[3];         /* nodes per axis of the KL grid */
  double lo[3], hi[3];
  double std_dev;       /* s */
  double corr_len;      /* l */
  int32_t n_modes;      /* M <= 1024; 0 asks for the stochastic dimension (see mlq_kl_modes) */
  int32_t max_rank;     /* max(n_modes, 1) <= max_rank <= min(4096, nodes) */
  double eps;           /* relative trace tolerance of the pivoted Cholesky */
  /* mesh_kind = MLQ_MESH_P1_TET: the KL lives on the vertices of a tetrahedral
   * mesh (host arrays, dim = 3, n/lo/hi ignored) with its P1 mass matrix */
  int32_t mesh_kind;
  int64_t n_vert, n_tet;
  const double* xyz;    /* n_vert x 3 */
  const int32_t* tets;  /* n_tet x 4, positively oriented */
  /* covariance kernel: MLQ_COV_EXP, std_dev^2 exp(-|x - x'|_2 / corr_len) (the default), or
   * MLQ_COV_SQEXP, std_dev^2 exp(-|x - x'|_2^2 / corr_len) (the paper's kernel of Section 5.1,
   * with corr_len = sigma_KL) */
  int32_t cov_kernel;
  /* eigenpairs: MLQ_KL_CHOLESKY, the pivoted Cholesky route above (any mesh); MLQ_KL_EXACT (Q1
   * boxes), the n_modes largest eigenpairs of eq. (algEig) itself, by subspace iteration on
   * 2 n_modes (at least n_modes + 16) columns with Rayleigh-Ritz, the covariance applied through
   * the FFT of its circulant embedding (2 (n_a - 1) points per axis; exact, since the covariance of
   * a uniform grid depends on index offsets only), until every returned pair has
   * |C M psi - lambda psi|_M <= eps lambda (eps > 0; max_rank is not used; 2 n_modes <= nodes) */
  int32_t method;
} mlq_kl_desc;
typedef enum { MLQ_KL_CHOLESKY = 0, MLQ_KL_EXACT = 1 } mlq_kl_method;

/* Device workspace bytes of mlq_kl_modes (dominated by two n x max_rank FP64 arrays). */
mlq_status mlq_kl_workspace_bytes(const mlq_kl_desc* kd, size_t* ws_bytes);

/* Largest n_modes eigenpairs: lambda_host (M, descending) and the M-orthonormal
 * modes psi_dev (n x M column-major FP64 device array, psi_k^T M psi_k = 1, entry of
 * largest magnitude positive).  rank_out: Cholesky rank used (MLQ_KL_EXACT: the subspace
 * columns); resid_out: trace(C - L L^T) / trace(C) (MLQ_KL_EXACT: the largest relative residual
 * of the returned pairs; MLQ_ENOCONV if it stayed above eps).  Synchronises the stream.
 * MLQ_KL_EXACT creates hipFFT plans for the duration of the call (their work area lies in ws_dev;
 * the FFT library keeps its own twiddle tables while a plan exists).
 * n_modes = 0: the paper's way of fixing M (Section 5.1): the factorisation runs until
 * trace(C - L L^T) <= eps trace(C) (or max_rank) and only rank_out (that rank, the stochastic
 * dimension M) and resid_out are written; lambda_host and psi_dev may be NULL. */
mlq_status mlq_kl_modes(const mlq_kl_desc* kd, void* ws_dev, size_t ws_bytes, double* lambda_host,
                        double* psi_dev, int32_t* rank_out, double* resid_out, void* hip_stream);

/* Element-midpoint transfer: phi_dev (P x M row-major FP64, device) = the Q1
 * interpolant of the KL-grid modes at the element centres of the Q1 box level
 * (level_n nodes per axis on [level_lo, level_hi]).  Enqueues only. */
mlq_status mlq_kl_transfer(const mlq_kl_desc* kd, const double* psi_dev, const int64_t* level_n,
                           const double* level_lo, const double* level_hi, double* phi_dev, void* hip_stream);

/* Non-nested transfer to a tetrahedral level (Section 4, with the reading for
 * non-nested meshes): phi_dev (n_tet x M row-major FP64, device) = the P1
 * interpolant of the KL modes (kd a tetrahedral KL mesh) at the centroids of the
 * level's tetrahedra (host arrays xyz, tets).  Each centroid takes the KL
 * tetrahedron with the largest smallest barycentric coordinate (lowest index on
 * ties within 1e-12; a point outside the KL mesh takes the best nearby one) and
 * its barycentric weights clipped at 0 and renormalised.  ws_dev (>=
 * mlq_kl_transfer_tet_bytes) holds the located weights; enqueues the
 * interpolation and returns after it finished. */
mlq_status mlq_kl_transfer_tet_bytes(int64_t n_tet, size_t* ws_bytes);
mlq_status mlq_kl_transfer_tet(const mlq_kl_desc* kd, const double* psi_dev, int64_t n_vert, const double* xyz,
                               int64_t n_tet, const int32_t* tets, void* ws_dev, size_t ws_bytes,
                               double* phi_dev, void* hip_stream);

/* ---- kernel timing (HIP events on the solve's stream) ----
 * Kernel classes of mlq_solve_batch; `units` counts node-samples processed. */
enum {
  MLQ_K_APPLY = 0,    /* Jacobian apply inside GMRES */
  MLQ_K_RESIDUAL = 1, /* nonlinear residual + ionic terms */
  MLQ_K_RHS = 2,      /* right-hand side of a step */
  MLQ_K_PRECOND = 3,  /* preconditioner */
  MLQ_K_DOTS = 4,     /* Gram-Schmidt projections (+ their final sums) */
  MLQ_K_ORTH = 5,     /* Gram-Schmidt update + norm */
  MLQ_K_SMALL = 6,    /* per-sample scalar kernels (checks, Givens, counts) */
  MLQ_K_UPDATE = 7,   /* Newton update */
  MLQ_K_QOI = 8,      /* activation tracking and QoI reductions */
  MLQ_K_PERSISTENT = 9, /* persistent per-sample solves (mlq_set_persistent): the whole launch */
  MLQ_K_CLASSES = 10
};

typedef struct {
  double ms[16];        /* summed kernel time per class */
  int64_t launches[16]; /* launches per class */
  double units[16];     /* node-samples processed per class */
  double bytes[16];     /* algorithmic bytes per class (MLQ_K_APPLY only; 0 elsewhere): every
                           operand read or written once per launch -- boxes: x, y, d (or v_j) and
                           the element's field value per node-sample, plus the basis vectors of
                           the fused projections; tetrahedra: x, y, d per vertex-sample and the
                           field value per tetrahedron-sample */
  double kernel_bytes[16]; /* the bytes the kernels' own data layout reads and writes once
                           (MLQ_K_APPLY only): e.g. assembled stiffness values in place of the
                           field on tetrahedra */
} mlq_timing;

/* Times the kernel classes whose bit is set in kernel_mask (0 turns timing off)
 * during later mlq_solve_batch calls on this level.  Each timed launch is
 * bracketed by two events on the solve's stream. */
mlq_status mlq_timing_enable(mlq_level* level, uint32_t kernel_mask);

/* Reads (and with reset != 0 clears) the accumulated timings of the level. */
mlq_status mlq_timing_read(mlq_level* level, mlq_timing* out, int32_t reset);

/* Thread-local message describing the last error. */
const char* mlq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLQ_H */
