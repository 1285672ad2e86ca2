// Internal declarations shared by the host library (mlq_api.cpp) and the HIP
// kernels (mlq_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlq.h"

namespace mlq {

// Geometry of a uniform Q1 box level, passed by value to the stencil kernels.
// Element matrices of a brick with edges hx, hy, hz factor into 1D pieces; the
// H* scalars are the edge-length factors of the mass, the three second-derivative
// terms and the x-y cross term (Section 3.1, eq. (semi-disc)).
struct Geo {
  int32_t dim;
  int32_t nx, ny, nz;  // nodes per axis (nz = 1 in 2D)
  int64_t nn;          // nodes per sample
  int64_t P;           // elements per sample
  double Hm, Hxx, Hyy, Hzz, Hxy;
  double Hx, Hy, Hz;   // edge lengths
  // Box elements carry per-sample coefficients (p, q); the conductivity of an element is
  //   G_xx = cx0 + cx1 p,  G_yy = cy0 + cy1 p,  G_zz = cz0 + cz1 p,  G_xy = q.
  // Fibre angle model: p, q = (s_l - s_t)/2 (cos 2t, sin 2t), cx0 = cy0 = (s_l + s_t)/2,
  // cx1 = 1, cy1 = -1, cz0 = s_t, cz1 = 0.  Isotropic scalar model: p = v, q = 0,
  // cx0 = cy0 = cz0 = 0, cx1 = cy1 = cz1 = 1 (G = v I).
  double cx0, cx1, cy0, cy1, cz0, cz1;
  int32_t tet;         // 1: P1 tetrahedra (TetDev holds the mesh), 0: Q1 box
  int64_t nnz;         // tetrahedra: stored (padded, slot-major) entries of the vertex adjacency
  int32_t lx;          // 3D boxes: lanes along x of a wave (8 or 16), 0 = chosen by the grid width
  // The field value behind (p, q), for kernels that form the coefficients from it: iso = 1: p =
  // max(v, cfa), q = 0 (cfa the floor); iso = 0: p, q = cfa (cos 2t, sin 2t) (cfa = (s_l - s_t)/2).
  int32_t iso;
  double cfa;
  // All-at-once time blocks (3D boxes): the stencil kernels see every time level of a block as a
  // virtual sample, group = time levels per block + 1 consecutive virtual samples per sample (slot
  // 0 holds the block's initial state and is skipped); 0 or 1 = ordinary solves.  Per-sample data
  // (coefficients, flags, Krylov scalars) is indexed by virtual sample / group.
  int32_t group;
};

// P1 tetrahedral level data on the device (inside the level blob).  The sparsity
// of M and K is the vertex adjacency (CSR); each nonzero lists the element
// matrix entries that add into it, in increasing element order.
struct TetDev {
  int64_t nv, nt, nell, nc;
  int32_t width;           // slots per row: the longest row of the P1 pattern
  // the pattern stored slot-major: entry (s, i) at s * nv + i (consecutive rows are
  // consecutive in memory for every slot); padded slots point at row i with value 0
  const int32_t* ecol;     // nell: column
  const int32_t* ediag;    // nv: slot of the diagonal entry of each row
  const double* em;        // nell: consistent P1 mass
  const float* em32;       // nell
  const double* mdiag;     // nv: diagonal of M
  const float* mdiag32;    // nv
  const int32_t* ecptr;    // nell + 1
  const int32_t* ecdat;    // nc: (tet << 4) | (4 a + b), a = local row vertex, b = local column vertex
  const double* geo;       // nt x kTetGeo: grad phi_0..3 (12), e_circ (3), e_long (3), volume
  int32_t model;           // conductivity model (MLQ_DIFF_*; vector: the field is V - vmean, 3 components)
  const double* vmean;     // nt x 3: E[V] per element (vector model), else unused
};
constexpr int kTetGeo = 19;

// Host-side preparation of a tetrahedral level (mlq_tetmesh.cpp).
struct TetHost {
  int64_t nv = 0, nt = 0, nnz = 0, nc = 0, nell = 0;
  int32_t width = 0;
  std::vector<int32_t> rowptr, col, cptr, cdat;   // CSR (rows sorted)
  std::vector<int32_t> ecol, ecptr, ecdat, ediag; // the same, slot-major padded (TetDev)
  std::vector<double> mval, em, mdiag, geo, wts, fload;
  double vol = 0.0;
};
// Validates the tetrahedral fields of desc and builds the CSR structure (and, with
// values = true, the mass, contributions, geometry, weights and stimulus load).
// Returns an empty string on success, else the reason.
std::string tet_build(const mlq_level_desc* d, TetHost& h, bool values);

// Physics constants of eq. (ionic_term) and the time step.
struct Ionic {
  double alpha, u_rest, u_th, u_peak;
  double dt;
};

constexpr int kBlock = 256;      // threads per block of the nodal kernels
constexpr int kRedChunk = 2048;  // nodes per block of the Krylov reduction kernels
constexpr int kMaxInner = 64;    // upper bound on GMRES iterations per solve

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Pointers of one solve's workspace (carved from the caller's buffer).
struct Work {
  // FP64 per-node state, [B][n]
  double* uk;    // u_k, state at the current time level
  double* ukm1;  // u_{k-1} (extrapolated Newton guess)
  double* u;     // Newton iterate for u_{k+1}
  double* b;     // right-hand side of the step
  double* act;   // activation times (-1: not yet activated)
  // inner precision per-node vectors, [B][n]
  void* d;       // dt * I_ion'(u)
  void* z;       // preconditioned basis z_j = P^-1 v_j inv_eta_j, kmax vectors of [B][n]
  void* w;       // operator output
  void* V;       // GMRES basis, (kmax + 1) vectors of [B][n]
  // per element coefficients [B][P][2] (inner precision)
  void* coef;
  // the element field of the solve ([B][P], inner precision); mixed-precision 3D box kernels
  // form the coefficients from it in registers instead of reading coef
  const void* theta;
  // per-sample small arrays
  double* part;      // reduction partials (residual norms, Gram-Schmidt norms)
  double* dpart;     // Gram-Schmidt projection partials [B][kmax+1][nred]
  double* H;         // [B][kmax+1][kmax] Hessenberg
  double* cs;        // [B][kmax]
  double* sn;        // [B][kmax]
  double* g;         // [B][kmax+1]
  double* y;         // [B][kmax]: y_i * inv_eta_i of the final combination
  double* hc;        // [B][kmax+1]: h_ij * inv_eta_i of the current Gram-Schmidt step
  double* inv_eta;   // [B][kmax+1]: V_true[i] = V_stored[i] * inv_eta[i]
  double* beta;      // [B]
  int32_t* newton_active;  // [B]
  int32_t* inner_active;   // [B]
  int32_t* inner_k;        // [B] iterations taken in the current solve
  int32_t* status;         // [B] (internal copy)
  int64_t* iters;          // [B][2]
  int32_t* counter;        // [4]
  int kmax;                // GMRES iterations per solve (basis holds kmax + 1 vectors)
  int32_t nblk;            // blocks per sample of the nodal kernels
  int32_t nred;            // blocks per sample of the reduction kernels
  int32_t nres;            // blocks per sample of the residual kernel (partial norms)
  int32_t nwav;            // workgroups per sample of the 3D stencil kernels (projection partials when fused)
  size_t bytes;
};

// Carves the workspace for a batch.  With base == nullptr only computes bytes.  res_groups: the
// residual kernel's workgroups per sample are res_groups times those of g (time blocks).
Work carve_workspace(void* base, const Geo& g, int32_t batch, int kmax, bool mixed, int res_groups = 1);

// ---- kernel launchers (mlq_kernels.hip) --------------------------------------
void launch_coefs(const void* theta, void* coef, int64_t P, int32_t B, double half_dsig, bool iso, bool mixed,
                  hipStream_t s);
void launch_init(const Work& w, int64_t nn, int32_t B, double u_th, hipStream_t s);
// Newton initial guess u = 2 u_k - u_{k-1}
void launch_extrapolate(const Work& w, int64_t nn, int32_t B, hipStream_t s);
void launch_guess_reference(const Work& w, const double* ref_k, const double* ref_k1, int64_t nn, int32_t B,
                            bool local, hipStream_t s);
void launch_rhs(const Geo& g, const Work& w, const double* fbox, double load_coef, double dt, int32_t B,
                bool mixed, hipStream_t s);
void launch_residual(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s);
void launch_newton_check(const Geo& g, const Work& w, int32_t B, double tol, hipStream_t s);
void launch_count(const int32_t* flags, int32_t B, int32_t* out, int32_t* zero, hipStream_t s);
void launch_dots(const Geo& g, const Work& w, int j, int32_t B, bool mixed, hipStream_t s);
// Above kHsumMinReads partial reads per sample (blocks x partials) the projection coefficients are
// summed once per sample by a kernel of their own before the orthogonalisation.
constexpr int64_t kHsumMinReads = 1 << 14;
void launch_orth(const Geo& g, const Work& w, int j, int32_t B, bool mixed, hipStream_t s, int32_t npart);
// Givens rotation of column j; also counts the samples still active into counter[1 + (j & 1)]
// and clears counter[1 + ((j + 1) & 1)] for the next iteration.
void launch_givens(const Geo& g, const Work& w, int j, int32_t B, double tol, hipStream_t s, int32_t nparts);
void launch_solve_y(const Work& w, int32_t B, bool scaled, hipStream_t s);
void launch_activation(const Work& w, int64_t nn, int32_t B, double u_th, double t_k, double dt,
                       hipStream_t s);
void launch_qoi(const Work& w, const double* wts, int64_t nn, int32_t B, int qoi, double t_stop,
                double vol, double* qoi_out, hipStream_t s);
void launch_apply_public(const Geo& g, const void* coef, const void* x, const void* d, void* y,
                         double ck, int32_t B, bool mixed, hipStream_t s);
void launch_kl(const double* phi64T, const float* phi32T, const double* sqrt_lambda, const double* theta0,
               const double* Y, int64_t P, int32_t M, int32_t B, void* theta, bool mixed, hipStream_t s);
void launch_transpose_f64(const double* src, double* dst, int64_t rows, int64_t cols, hipStream_t s);
void launch_lattice(const int64_t* z, const double* shift, int32_t sdim, int64_t N, int64_t first, int32_t count,
                    bool uniform, double* Y, hipStream_t s);
// Field quantities of interest: probe table (passed by value as a kernel argument) and the
// geometry of a space-time transfer (spatial node counts per axis, time node counts, steps).
constexpr int kMaxProbes = 16;
constexpr int kProbeNodes = 8;
struct ProbeTab {
  int64_t node[kMaxProbes * kProbeNodes];
  double w[kMaxProbes * kProbeNodes];
  int32_t n;
};
struct XferGeo {
  int64_t sn_f[3], sn_t[3];  // spatial nodes per axis, from / to (1 on unused axes or no space transfer)
  int64_t tn_f, tn_t;        // time nodes, from / to (1 when no time transfer)
  int64_t m_f, m_t;          // steps, from / to
};
void launch_field_sum(const double* u, int32_t B, int64_t n, double* dst, hipStream_t s);
void launch_act_sum(const double* act, int32_t B, int64_t n, double t_stop, double* dst, hipStream_t s);
void launch_probe(const double* u, int32_t B, int64_t n, const ProbeTab& tab, int32_t k, int32_t ld, double* out,
                  hipStream_t s);
void launch_probe_sum(const double* u, int32_t B, int64_t n, const ProbeTab& tab, int32_t k, int32_t ld, double* sum,
                      hipStream_t s);
void launch_transfer(const XferGeo& g, int64_t rows, double alpha, const double* src, double* dst, hipStream_t s);
void launch_transfer_weighted(const XferGeo& g, int64_t rows, int64_t n_from, int64_t n_to, int K,
                              const int64_t* node, const double* w, double alpha, const double* src, double* dst,
                              hipStream_t s);
constexpr int kNormBlocks = 1024;  // partial sums per row of a space-time norm
struct NormGeo {
  int64_t n[3];  // nodes per axis (1 on unused axes)
  double h[3];   // spacing per axis
  int dim;
  int64_t m;     // time steps
  double dt;
  int q;         // 0: L^2 in space, 1: H^1
};
void launch_st_norm(const NormGeo& g, int64_t rows, const double* f, double* part, double* out, hipStream_t s);
void launch_time_norm(const double* f, int64_t rows, int64_t m, double dt, int q, double* out, hipStream_t s);

constexpr int kHaltonMaxDims = 1024;
void launch_halton(int32_t sdim, int64_t first, int32_t count, const double* shift, bool uniform, double* Y,
                   hipStream_t s);
void launch_newton_reset(const Work& w, int32_t B, hipStream_t s);
void launch_mark_failed(const Work& w, int32_t B, hipStream_t s);
void launch_accumulate(const double* ff, const double* fc, int32_t count, double* acc, hipStream_t s);

// KL set-up (mlq_kl.hip)
mlq_status kl_validate(const mlq_kl_desc* kd);
size_t kl_workspace_bytes(const mlq_kl_desc* kd);
mlq_status kl_modes(const mlq_kl_desc* kd, void* ws, double* lambda_host, double* psi_dev, int32_t* rank_out,
                    double* resid_out, hipStream_t s, std::string& err);
mlq_status kl_transfer(const mlq_kl_desc* kd, const double* psi_dev, const int64_t* level_n, const double* level_lo,
                       const double* level_hi, double* phi_dev, hipStream_t s);
size_t kl_transfer_tet_bytes(int64_t n_tet);
mlq_status locate_points_tet(const mlq_kl_desc* kd, const double* pts, int64_t np, std::vector<int32_t>& vid,
                             std::vector<double>& wts, std::string& err);
mlq_status kl_transfer_tet(const mlq_kl_desc* kd, const double* psi_dev, int64_t nv, const double* xyz, int64_t nt,
                           const int32_t* tets, void* ws, double* phi_dev, hipStream_t s, std::string& err);
void launch_minv_basis(const Geo& g, const Work& w, const void* tri, int nmax, int j, int32_t B, bool mixed,
                       hipStream_t s);
void launch_apply_pk(const Geo& g, const Work& w, int j, double ck, int32_t B, bool mixed, hipStream_t s);
void launch_update_zbasis(const Geo& g, const Work& w, int32_t B, bool mixed, hipStream_t s);
hipError_t prepare_minv_kernels(size_t bytes);
int32_t stencil3_blocks(const Geo& g);
// jb > 0: also accumulate the Gram-Schmidt projections w . v_i (i <= j < jb) into dpart,
// one partial per workgroup (Work::nwav per sample)
void launch_apply_pk3(const Geo& g, const Work& w, int j, double ck, int32_t B, bool mixed, hipStream_t s, int jb);
// coef: the (p, q) pairs in FP64, or in mixed precision the element field itself
void launch_apply_full3(const Geo& g, const void* coef, const void* x, const void* d, void* y, double ck, int32_t B,
                        bool mixed, hipStream_t s);
void launch_residual3(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s);
// 3D boxes: b = (M - dt/2 K) u_k + load F_box and the Newton start u := u_k; with uprev
// (u_{k-1}, may be NULL) also the extrapolated start 2 u_k - u_{k-1} (extrap) and the activation
// times of the step from t_prev = t_{k-1} to t_k (first crossing of u_th) into w.act.
void launch_rhs3(const Geo& g, const Work& w, const double* fbox, double load_coef, double dt, int32_t B, bool mixed,
                 hipStream_t s, const double* uprev = nullptr, bool extrap = false, double u_th = 0.0,
                 double t_prev = 0.0);
// 3D boxes: the step equation's residual without a separate right-hand side,
//   F = M ((u - u_k) + dt I_ion(u)) + dt/2 K (u + u_k) - load F_box,
// with -F and d = dt I_ion'(u) written and the partial norms |F|^2, |w u|^2, |w u_k + load F_box|^2
// (w the lumped mass) per workgroup.  start: the Newton iterate is w.u (0), u_k (1) or the
// extrapolation 2 u_k - u_(k-1) (2), written to w.u when start > 0; uprev (u_(k-1), may be NULL):
// also records the activation times of the step from t_prev to t_prev + dt.
void launch_residual3f(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s, int start,
                       const double* uprev, const double* fbox, double load, double u_th, double t_prev);
void launch_activation_between(const double* uold, const double* unew, double* act, int64_t nn, int32_t B,
                               double u_th, double t_k, double dt, hipStream_t s);
void launch_cast_f32(const double* src, float* dst, int64_t n, hipStream_t s);
// All-at-once time blocks (g.group > 1, virtual samples as above).  Right-hand sides of every
// time level of the block from the level before it, b_q = (M - dt/2 K) U_(q-1) + load(k0 + q) F,
// with the stimulus rate of [t_on, t_off) at the time nodes (the step's trapezoid); U and b
// [B][group][n].
void launch_rhs3_block(const Geo& g, const double* U, double* b, const void* coef, const double* fbox, int k0,
                       double dt, double t_on, double t_off, double amp, int32_t Bv, bool mixed, hipStream_t s);
// w += (-M + dt/2 K) x_(q-1) for every time level q >= 1 of a block (the sub-diagonal block of
// eq. (system_C)), x and w [B][group][n] in the inner precision; inactive samples skipped.
void launch_block_guess(double* U, int G, int64_t nn, int32_t B, const double* ref, int k0, int mode, hipStream_t s);
void launch_block_close(double* U, int G, int64_t nn, int32_t B, double* act, double u_th, int k0, double dt,
                        hipStream_t s);
void launch_coupling3(const Geo& g, const void* x, void* wv, const void* coef_or_theta, double ck, int32_t Bv,
                      const int32_t* active, bool mixed, hipStream_t s);

// Persistent per-sample solver of small 3D box levels (mlq_small.hip): one workgroup runs the
// whole time loop (Newton, GMRES, preconditioner, activation, QoI) of one sample at a time,
// the same method as the batched path.  The level's vector must fit kSmallMaxLds bytes of LDS.
constexpr int kSmallThreads = 256;
constexpr size_t kSmallMaxLds = 65536;
struct SmallArgs {
  Geo g;
  Ionic io;
  int32_t B, n_steps, kmax, max_newton, extrap, qoi;
  double newton_tol, inner_tol;
  double t_on, t_off, amp;  // stimulus rate amp on [t_on, t_off)
  const double* fbox;       // stimulus load vector
  const double* wts;        // node weights (M 1)
  double vol;
  const void* tri;          // 1 / pivots per axis, [3][nmax], inner precision
  int32_t nmax;
  Work w;                   // the batched workspace; w.coef holds the element coefficient pairs
  double* qoi_out;
  int32_t* status_out;
  int64_t* iters_out;
  double* u_out;            // final states and activation times (may be NULL)
  double* act_out;
};
bool small_solver_fits(const Geo& g, bool mixed);
hipError_t launch_solve_small(const SmallArgs& a, bool mixed, hipStream_t s);

// P1 tetrahedra (mlq_tet.hip).  kval: per-sample stiffness values [B][nell] (slot-major
// padded pattern of TetDev), inner precision.
void launch_tet_assemble(const TetDev& t, const void* theta, void* kval, int32_t B, double sigma_t, double dsig,
                         bool mixed, hipStream_t s);
void launch_tet_apply(const TetDev& t, const void* kval, const void* x, const void* d, void* y, double ck, int32_t B,
                      const int32_t* active, bool mixed, hipStream_t s);
void launch_tet_residual(const TetDev& t, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s);
void launch_tet_rhs(const TetDev& t, const Work& w, const double* fload, double load, double dt, int32_t B,
                    bool mixed, hipStream_t s, const double* uprev = nullptr, bool extrap = false,
                    double u_th = 0.0, double t_prev = 0.0);
// z_j = v_j inv_eta_j / diag(J) into the preconditioned basis, ck = dt / 2.
void launch_tet_jacobi_basis(const TetDev& t, const Work& w, int j, double ck, int32_t B, bool mixed,
                             hipStream_t s);

}  // namespace mlq
