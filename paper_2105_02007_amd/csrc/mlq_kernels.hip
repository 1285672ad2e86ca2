// HIP kernels for gfx950 (CDNA4, wave64): matrix-free Q1 operators of the
// Crank-Nicolson / Newton space-time solve, batched GMRES, ionic pointwise
// terms, quantities of interest, KL synthesis and lattice sampling.
//
// Batch layout: nodal vectors are [B][n] (sample-major, node index with axis 0
// fastest), element data [B][P][...].  Grids use blockIdx.y for the sample so a
// block never straddles two samples; per-sample masks let whole blocks exit.
#include "mlq_internal.h"
#include "mlq_q1.h"

#include <cmath>

namespace mlq {

// ---------------------------------------------------------------------------
// Per-element coefficients.  Fibre angles: p = (s_l - s_t)/2 cos 2t, q = (s_l - s_t)/2 sin 2t
// (a = (s_l - s_t)/2).  Isotropic scalar field (iso): p = max(v, a), q = 0 (a = the floor).
template <typename TT, typename TC>
__global__ void k_coefs(const TT* __restrict__ theta, TC* __restrict__ coef, int64_t total, double half_dsig,
                        int iso) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  if (iso) {
    const double v = (double)theta[i];
    coef[2 * i] = (TC)(v > half_dsig ? v : half_dsig);
    coef[2 * i + 1] = (TC)0;
  } else if constexpr (sizeof(TC) == 4) {
    const float t2 = 2.0f * (float)theta[i];
    float sv, cv;
    sincosf(t2, &sv, &cv);
    coef[2 * i] = (float)half_dsig * cv;
    coef[2 * i + 1] = (float)half_dsig * sv;
  } else {
    const double t2 = 2.0 * (double)theta[i];
    double sv, cv;
    sincos(t2, &sv, &cv);
    coef[2 * i] = half_dsig * cv;
    coef[2 * i + 1] = half_dsig * sv;
  }
}

void launch_coefs(const void* theta, void* coef, int64_t P, int32_t B, double half_dsig, bool iso, bool mixed,
                  hipStream_t s) {
  const int64_t total = P * (int64_t)B;
  const dim3 grid((unsigned)cdiv(total, kBlock));
  if (mixed)
    hipLaunchKernelGGL((k_coefs<float, float>), grid, dim3(kBlock), 0, s, (const float*)theta, (float*)coef,
                       total, half_dsig, iso ? 1 : 0);
  else
    hipLaunchKernelGGL((k_coefs<double, double>), grid, dim3(kBlock), 0, s, (const double*)theta,
                       (double*)coef, total, half_dsig, iso ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Initial state u_0 = 0, activation flags, per-sample counters.
__global__ void k_init(double* uk, double* act, int64_t nn, double u_th, int32_t* status, int64_t* iters,
                       int32_t B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = nn * B;
  if (i < total) {
    uk[i] = 0.0;
    act[i] = (0.0 >= u_th) ? 0.0 : -1.0;
  }
  if (i < B) {
    status[i] = MLQ_SAMPLE_OK;
    iters[2 * i] = 0;
    iters[2 * i + 1] = 0;
  }
}

void launch_init(const Work& w, int64_t nn, int32_t B, double u_th, hipStream_t s) {
  const int64_t total = nn * B > B ? nn * B : B;
  hipLaunchKernelGGL(k_init, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, w.uk, w.act, nn, u_th,
                     w.status, w.iters, B);
}

__global__ void k_extrapolate(double* __restrict__ u, const double* __restrict__ uk, const double* __restrict__ ukm1,
                              int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) u[i] = 2.0 * uk[i] - ukm1[i];
}

void launch_extrapolate(const Work& w, int64_t nn, int32_t B, hipStream_t s) {
  const int64_t total = nn * B;
  hipLaunchKernelGGL(k_extrapolate, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, w.u, w.uk, w.ukm1,
                     total);
}

// Newton start from an unperturbed reference solution r_k (one space-time field shared by the
// batch): u = r_(k+1) (global guess), or u = u_k + (r_(k+1) - r_k) (its increment added to the
// sample's own state, local guess).
__global__ void k_guess_reference(double* __restrict__ u, const double* __restrict__ uk,
                                  const double* __restrict__ r0, const double* __restrict__ r1, int64_t nn,
                                  int64_t total, int local) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t j = i % nn;
  u[i] = local ? uk[i] + (r1[j] - r0[j]) : r1[j];
}

void launch_guess_reference(const Work& w, const double* ref_k, const double* ref_k1, int64_t nn, int32_t B,
                            bool local, hipStream_t s) {
  const int64_t total = nn * B;
  hipLaunchKernelGGL(k_guess_reference, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, w.u, w.uk, ref_k,
                     ref_k1, nn, total, local ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Right-hand side of step k (eq. (st-system)):  b = (M - dt/2 K) u_k + c_k F_box,
// c_k = dt/2 (s(t_{k+1}) + s(t_k)).  Also starts Newton from u = u_k.
template <int DIM, typename TC>
__global__ __launch_bounds__(kBlock) void k_rhs(Geo g, const double* __restrict__ uk, const TC* __restrict__ coef,
                                                const double* __restrict__ fbox, double load_coef, double half_dt,
                                                double* __restrict__ bvec, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sb = blockIdx.y;
  if (i >= g.nn) return;
  const double* us = uk + (int64_t)sb * g.nn;
  const TC* cf = coef + (int64_t)sb * g.P * 2;
  int ix, iy, iz;
  node_xyz(i, g, ix, iy, iz);
  double xm[27], xk[27];
  load_nbhd<DIM, double>(ix, iy, iz, g, [&](int64_t j, double& a, double& b) { a = b = us[j]; }, xm, xk);
  double SM, SK;
  gather<DIM, double, TC>(ix, iy, iz, g, cf, xm, xk, SM, SK);
  const int64_t o = (int64_t)sb * g.nn + i;
  bvec[o] = g.Hm * SM - half_dt * SK + load_coef * fbox[i];
  u[o] = us[i];
}

void launch_rhs(const Geo& g, const Work& w, const double* fbox, double load_coef, double dt, int32_t B, bool mixed,
                hipStream_t s) {
  const dim3 grid((unsigned)cdiv(g.nn, kBlock), B);
  if (g.dim == 3) {
    if (mixed)
      hipLaunchKernelGGL((k_rhs<3, float>), grid, dim3(kBlock), 0, s, g, w.uk, (const float*)w.coef, fbox, load_coef,
                         0.5 * dt, w.b, w.u);
    else
      hipLaunchKernelGGL((k_rhs<3, double>), grid, dim3(kBlock), 0, s, g, w.uk, (const double*)w.coef, fbox,
                         load_coef, 0.5 * dt, w.b, w.u);
  } else {
    if (mixed)
      hipLaunchKernelGGL((k_rhs<2, float>), grid, dim3(kBlock), 0, s, g, w.uk, (const float*)w.coef, fbox, load_coef,
                         0.5 * dt, w.b, w.u);
    else
      hipLaunchKernelGGL((k_rhs<2, double>), grid, dim3(kBlock), 0, s, g, w.uk, (const double*)w.coef, fbox,
                         load_coef, 0.5 * dt, w.b, w.u);
  }
}

// ---------------------------------------------------------------------------
// Nonlinear residual of a step (eq. (mono_disc)), FP64:
//   G(u) = M (u + dt I_ion(u)) + dt/2 K u,   F = G(u) - b.
// Writes r0 = -F (inner precision: GMRES right-hand side), d = dt I_ion'(u),
// and per-block partial sums of |F|^2, |G|^2, |b|^2.
template <int DIM, typename TC, typename TI>
__global__ __launch_bounds__(kBlock) void k_residual(Geo g, Ionic io, const double* __restrict__ u,
                                                     const double* __restrict__ bvec, const TC* __restrict__ coef,
                                                     TI* __restrict__ r0, TI* __restrict__ dvec,
                                                     double* __restrict__ part, const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  __shared__ double sh[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double f2 = 0.0, g2 = 0.0, b2 = 0.0;
  if (i < g.nn) {
    const double* us = u + (int64_t)sb * g.nn;
    const TC* cf = coef + (int64_t)sb * g.P * 2;
    int ix, iy, iz;
    node_xyz(i, g, ix, iy, iz);
    double xm[27], xk[27];
    load_nbhd<DIM, double>(
        ix, iy, iz, g,
        [&](int64_t j, double& a, double& b) {
          const double v = us[j];
          a = v + io.dt * iion(v, io);
          b = v;
        },
        xm, xk);
    double SM, SK;
    gather<DIM, double, TC>(ix, iy, iz, g, cf, xm, xk, SM, SK);
    const int64_t o = (int64_t)sb * g.nn + i;
    const double G = g.Hm * SM + 0.5 * io.dt * SK;
    const double bb = bvec[o];
    const double F = G - bb;
    r0[o] = (TI)(-F);
    dvec[o] = (TI)(io.dt * diion(us[i], io));
    f2 = F * F;
    g2 = G * G;
    b2 = bb * bb;
  }
  const double s0 = block_sum<kBlock>(f2, sh);
  const double s1 = block_sum<kBlock>(g2, sh);
  const double s2 = block_sum<kBlock>(b2, sh);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)sb * gridDim.x + blockIdx.x) * 3;
    p[0] = s0;
    p[1] = s1;
    p[2] = s2;
  }
}

void launch_residual(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(g.nn, kBlock), B);
#define MLQ_RES(D, TC, TI)                                                                                        \
  hipLaunchKernelGGL((k_residual<D, TC, TI>), grid, dim3(kBlock), 0, s, g, io, w.u, w.b, (const TC*)w.coef,       \
                     (TI*)w.V, (TI*)w.d, w.part, w.newton_active)
  if (g.dim == 3) {
    if (mixed) MLQ_RES(3, float, float); else MLQ_RES(3, double, double);
  } else {
    if (mixed) MLQ_RES(2, float, float); else MLQ_RES(2, double, double);
  }
#undef MLQ_RES
}

// Per-sample Newton test: backward error |F| / (|G| + |b|) <= tol.  Also starts
// GMRES: beta = |r0|, g = (beta, 0, ..), inv_eta[0] = 1/beta.
__global__ __launch_bounds__(kBlock) void k_newton_check(const double* __restrict__ part, int32_t nblk, double tol,
                                                         int32_t* newton_active, int32_t* inner_active,
                                                         int32_t* inner_k, int32_t* status, double* beta, double* gv,
                                                         double* inv_eta, int kmax) {
  const int sb = blockIdx.x;
  if (newton_active[sb] == 0) return;
  __shared__ double sh[kBlock / 64];
  double a0 = 0, a1 = 0, a2 = 0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) {
    const double* p = part + ((int64_t)sb * nblk + i) * 3;
    a0 += p[0];
    a1 += p[1];
    a2 += p[2];
  }
  const double F2 = block_sum<kBlock>(a0, sh);
  const double G2 = block_sum<kBlock>(a1, sh);
  const double B2 = block_sum<kBlock>(a2, sh);
  if (threadIdx.x == 0) {
    const double nf = sqrt(F2), den = sqrt(G2) + sqrt(B2);
    const double err = den == 0.0 ? 0.0 : nf / den;
    inner_k[sb] = 0;
    if (!(err == err) || !isfinite(nf)) {
      status[sb] = MLQ_SAMPLE_NAN;
      newton_active[sb] = 0;
      inner_active[sb] = 0;
    } else if (err <= tol || nf == 0.0) {
      newton_active[sb] = 0;
      inner_active[sb] = 0;
    } else {
      inner_active[sb] = 1;
      beta[sb] = nf;
      inv_eta[(int64_t)sb * (kmax + 1)] = 1.0 / nf;
      double* gs = gv + (int64_t)sb * (kmax + 1);
      gs[0] = nf;
      for (int j = 1; j <= kmax; ++j) gs[j] = 0.0;
    }
  }
}


void launch_newton_check(const Geo& g, const Work& w, int32_t B, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_newton_check, dim3(B), dim3(kBlock), 0, s, w.part, w.nres, tol, w.newton_active,
                     w.inner_active, w.inner_k, w.status, w.beta, w.g, w.inv_eta, w.kmax);
}

// Number of set flags into out[0]; also clears `zero` (may be NULL), the counter the next
// Givens launch accumulates into.
__global__ void k_count(const int32_t* __restrict__ flags, int32_t B, int32_t* out, int32_t* zero) {
  __shared__ double sh[kBlock / 64];
  double c = 0;
  for (int i = threadIdx.x; i < B; i += kBlock) c += flags[i] != 0 ? 1.0 : 0.0;
  c = block_sum<kBlock>(c, sh);
  if (threadIdx.x == 0) {
    out[0] = (int32_t)c;
    if (zero != nullptr) zero[0] = 0;
  }
}

void launch_count(const int32_t* flags, int32_t B, int32_t* out, int32_t* zero, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(kBlock), 0, s, flags, B, out, zero);
}

// ---------------------------------------------------------------------------
// Jacobian apply (Section 3.2): y = M ((1 + d) x) + ck K_G x, ck = dt/2.
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_apply(Geo g, const T* __restrict__ x, const T* __restrict__ d,
                                                  const T* __restrict__ coef, T* __restrict__ y, T ck,
                                                  const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active != nullptr && active[sb] == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nn) return;
  const T* xs = x + (int64_t)sb * g.nn;
  const T* ds = d + (int64_t)sb * g.nn;
  const T* cf = coef + (int64_t)sb * g.P * 2;
  int ix, iy, iz;
  node_xyz(i, g, ix, iy, iz);
  T xm[27], xk[27];
  load_nbhd<DIM, T>(
      ix, iy, iz, g,
      [&](int64_t j, T& a, T& b) {
        const T v = xs[j];
        a = v + ds[j] * v;
        b = v;
      },
      xm, xk);
  T SM, SK;
  gather<DIM, T, T>(ix, iy, iz, g, cf, xm, xk, SM, SK);
  y[(int64_t)sb * g.nn + i] = (T)g.Hm * SM + ck * SK;
}

template <typename T>
static void apply_dispatch(const Geo& g, const T* coef, const T* x, const T* d, T* y, double ck, int32_t B,
                           const int32_t* active, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(g.nn, kBlock), B);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_apply<3, T>), grid, dim3(kBlock), 0, s, g, x, d, coef, y, (T)ck, active);
  else
    hipLaunchKernelGGL((k_apply<2, T>), grid, dim3(kBlock), 0, s, g, x, d, coef, y, (T)ck, active);
}

void launch_apply_public(const Geo& g, const void* coef, const void* x, const void* d, void* y, double ck,
                         int32_t B, bool mixed, hipStream_t s) {
  if (mixed)
    apply_dispatch<float>(g, (const float*)coef, (const float*)x, (const float*)d, (float*)y, ck, B, nullptr, s);
  else
    apply_dispatch<double>(g, (const double*)coef, (const double*)x, (const double*)d, (double*)y, ck, B, nullptr,
                           s);
}

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt, step j of GMRES, per sample:
//   part[b][i][blk] = sum_chunk w . Vs_i  (i <= j)
// One pass: w is read once and all j + 1 projections accumulate in registers
// (JB >= j + 1 accumulators); each is summed in a fixed order.
template <typename T, int JB>
__global__ __launch_bounds__(kBlock) void k_dots(int64_t nn, const T* __restrict__ w, const T* __restrict__ V,
                                                 size_t vs, int j, int kmax, double* __restrict__ part,
                                                 const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  __shared__ double sh[JB][kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  const int64_t end = base + kRedChunk < nn ? base + kRedChunk : nn;
  const T* ws = w + (int64_t)sb * nn;
  const T* vs0 = V + (int64_t)sb * nn;
  double acc[JB];
#pragma unroll
  for (int i = 0; i < JB; ++i) acc[i] = 0.0;
  for (int64_t t = base + threadIdx.x; t < end; t += kBlock) {
    const double wv = (double)ws[t];
#pragma unroll
    for (int i = 0; i < JB; ++i)
      if (i <= j) acc[i] += wv * (double)vs0[i * vs + t];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < JB; ++i)
    if (i <= j) {
      const double v = wave_sum(acc[i]);
      if (lane == 0) sh[i][wid] = v;
    }
  __syncthreads();
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) r += sh[i][q];
    part[((int64_t)sb * (kmax + 1) + i) * gridDim.x + blockIdx.x] = r;
  }
}

void launch_dots(const Geo& g, const Work& w, int j, int32_t B, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)w.nred, B);
  const size_t vs = (size_t)g.nn * B;
#define MLQ_DOTS(T, JB)                                                                                       \
  hipLaunchKernelGGL((k_dots<T, JB>), grid, dim3(kBlock), 0, s, g.nn, (const T*)w.w, (const T*)w.V, vs, j, \
                     w.kmax, w.dpart, w.inner_active)
#define MLQ_DOTS_T(T)            \
  if (j < 4)                     \
    MLQ_DOTS(T, 4);              \
  else if (j < 8)                \
    MLQ_DOTS(T, 8);              \
  else if (j < 16)               \
    MLQ_DOTS(T, 16);             \
  else                           \
    MLQ_DOTS(T, kMaxInner + 1);
  if (mixed) {
    MLQ_DOTS_T(float)
  } else {
    MLQ_DOTS_T(double)
  }
#undef MLQ_DOTS_T
#undef MLQ_DOTS
}

// Vs_{j+1} = w - sum_i hc_i Vs_i, partial |Vs_{j+1}|^2.  Each block first sums the
// npart projection partials (of k_dots, or of the apply kernel that fused them;
// one wave per coefficient, fixed order):
// h_ij = inv_eta_i sum_blk part, hc_i = h_ij inv_eta_i; block 0 stores column j of H.
// The projection coefficients of step j from the npart partials per sample (one wave per
// coefficient, fixed order): h_ij = inv_eta_i sum_blk part, hc_i = h_ij inv_eta_i, column j of H.
__device__ inline void sum_projections(int sb, int j, int kmax, int npart, const double* __restrict__ dpart,
                                       const double* __restrict__ inv_eta, double* __restrict__ H, double* c,
                                       bool store_h) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i <= j; i += kBlock / 64) {
    const double* pi = dpart + ((int64_t)sb * (kmax + 1) + i) * npart;
    double a = 0.0;
    for (int b = lane; b < npart; b += 64) a += pi[b];
    a = wave_sum(a);
    if (lane == 0) {
      const double ie = inv_eta[(int64_t)sb * (kmax + 1) + i];
      const double h = a * ie;
      c[i] = h * ie;
      if (store_h) H[((int64_t)sb * (kmax + 1) + i) * kmax + j] = h;
    }
  }
}

// Projection coefficients once per sample (into hc), for launches whose orthogonalisation blocks
// would otherwise each re-read every partial.
__global__ __launch_bounds__(kBlock) void k_hsum(int j, int kmax, int npart, const double* __restrict__ dpart,
                                                 const double* __restrict__ inv_eta, double* __restrict__ H,
                                                 double* __restrict__ hc, const int32_t* __restrict__ active) {
  const int sb = blockIdx.x;
  if (active[sb] == 0) return;
  sum_projections(sb, j, kmax, npart, dpart, inv_eta, H, hc + (int64_t)sb * (kmax + 1), true);
}

// npart > 0: the coefficients from the partials (each block); npart == 0: from hc (k_hsum).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_orth(int64_t nn, const T* __restrict__ w, T* __restrict__ V, size_t vs,
                                                 int j, int kmax, const double* __restrict__ dpart,
                                                 const double* __restrict__ inv_eta, double* __restrict__ H,
                                                 double* __restrict__ part, const int32_t* __restrict__ active,
                                                 int npart, const double* __restrict__ hc) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  __shared__ double sh[kBlock / 64];
  __shared__ double c[kMaxInner + 1];
  if (npart > 0) {
    sum_projections(sb, j, kmax, npart, dpart, inv_eta, H, c, blockIdx.x == 0);
  } else {
    for (int i = threadIdx.x; i <= j; i += kBlock) c[i] = hc[(int64_t)sb * (kmax + 1) + i];
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  const int64_t end = base + kRedChunk < nn ? base + kRedChunk : nn;
  const T* ws = w + (int64_t)sb * nn;
  T* vn = V + (size_t)(j + 1) * vs + (int64_t)sb * nn;
  // a thread's kRedChunk / kBlock nodes side by side, so that the loads of one basis vector at
  // all of them are in flight together (the same operations per node, in the same order)
  constexpr int NPT = kRedChunk / kBlock;
  double v[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int64_t t = base + threadIdx.x + (int64_t)q * kBlock;
    v[q] = t < end ? (double)ws[t] : 0.0;
  }
  for (int i = 0; i <= j; ++i) {
    const double ci = c[i];
    const T* vi = V + i * vs + (int64_t)sb * nn;
    T x[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int64_t t = base + threadIdx.x + (int64_t)q * kBlock;
      x[q] = t < end ? vi[t] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < NPT; ++q) v[q] -= ci * (double)x[q];
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    const int64_t t = base + threadIdx.x + (int64_t)q * kBlock;
    if (t < end) {
      const T vt = (T)v[q];
      vn[t] = vt;
      acc += (double)vt * (double)vt;
    }
  }
  acc = block_sum<kBlock>(acc, sh);
  if (threadIdx.x == 0) part[(int64_t)sb * gridDim.x + blockIdx.x] = acc;
}

void launch_orth(const Geo& g, const Work& w, int j, int32_t B, bool mixed, hipStream_t s, int32_t npart) {
  const dim3 grid((unsigned)w.nred, B);
  const size_t vs = (size_t)g.nn * B;
  // Many blocks per sample, each re-reading (j + 1) x npart partials: sum them once per sample
  // first (the same sums in the same order).
  int np = npart;
  if ((int64_t)w.nred * npart > kHsumMinReads) {
    hipLaunchKernelGGL(k_hsum, dim3(B), dim3(kBlock), 0, s, j, w.kmax, (int)npart, w.dpart, w.inv_eta, w.H, w.hc,
                       w.inner_active);
    np = 0;
  }
  if (mixed)
    hipLaunchKernelGGL((k_orth<float>), grid, dim3(kBlock), 0, s, g.nn, (const float*)w.w, (float*)w.V, vs, j,
                       w.kmax, w.dpart, w.inv_eta, w.H, w.part, w.inner_active, np, (const double*)w.hc);
  else
    hipLaunchKernelGGL((k_orth<double>), grid, dim3(kBlock), 0, s, g.nn, (const double*)w.w, (double*)w.V, vs, j,
                       w.kmax, w.dpart, w.inv_eta, w.H, w.part, w.inner_active, np, (const double*)w.hc);
}

// Norm of the new vector, Givens rotations of column j, residual estimate |g_{j+1}|.
// Also counts the samples still active after this iteration into *count (one integer
// atomic add per such sample; the order does not matter) and clears *clear, the counter of
// the next iteration (two counters alternate, so the host can read this one meanwhile).
__global__ __launch_bounds__(kBlock) void k_givens(const double* __restrict__ part, int32_t nred, int j, int kmax,
                                                   double tol, double* H, double* cs, double* sn, double* gv,
                                                   double* inv_eta, const double* __restrict__ beta,
                                                   int32_t* inner_active, int32_t* inner_k, int32_t* count,
                                                   int32_t* clear) {
  const int sb = blockIdx.x;
  if (sb == 0 && threadIdx.x == 0) *clear = 0;
  if (inner_active[sb] == 0) return;
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nred; i += kBlock) acc += part[(int64_t)sb * nred + i];
  const double nrm2 = block_sum<kBlock>(acc, sh);
  if (threadIdx.x != 0) return;
  const int64_t hb = (int64_t)sb * (kmax + 1) * kmax;
  double* Hs = H + hb;
  double* c = cs + (int64_t)sb * kmax;
  double* s = sn + (int64_t)sb * kmax;
  double* gs = gv + (int64_t)sb * (kmax + 1);
  const double hn = sqrt(nrm2);
  inv_eta[(int64_t)sb * (kmax + 1) + j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    const double a = Hs[i * kmax + j], b = Hs[(i + 1) * kmax + j];
    Hs[i * kmax + j] = c[i] * a + s[i] * b;
    Hs[(i + 1) * kmax + j] = -s[i] * a + c[i] * b;
  }
  const double a = Hs[j * kmax + j];
  const double r = hypot(a, hn);
  double cj = 1.0, sj = 0.0;
  if (r > 0.0) {
    cj = a / r;
    sj = hn / r;
  }
  c[j] = cj;
  s[j] = sj;
  Hs[j * kmax + j] = r;
  Hs[(j + 1) * kmax + j] = 0.0;
  gs[j + 1] = -sj * gs[j];
  gs[j] = cj * gs[j];
  const double res = fabs(gs[j + 1]);
  if (res <= tol * beta[sb] || hn == 0.0 || j + 1 >= kmax || !(res == res)) {
    inner_active[sb] = 0;
    inner_k[sb] = j + 1;
  } else {
    atomicAdd(count, 1);
  }
}

void launch_givens(const Geo& g, const Work& w, int j, int32_t B, double tol, hipStream_t s, int32_t nparts) {
  (void)g;
  hipLaunchKernelGGL(k_givens, dim3(B), dim3(kBlock), 0, s, w.part, nparts, j, w.kmax, tol, w.H, w.cs, w.sn, w.g,
                     w.inv_eta, w.beta, w.inner_active, w.inner_k, w.counter + 1 + (j & 1),
                     w.counter + 1 + ((j + 1) & 1));
}

// Back substitution R y = g on the rotated Hessenberg matrix; stores y_i, times inv_eta_i
// when scaled (the combination then runs over the unnormalised basis v_i).
__global__ void k_solve_y(int32_t B, int kmax, const double* __restrict__ H, const double* __restrict__ gv,
                          const double* __restrict__ inv_eta, const int32_t* __restrict__ newton_active,
                          const int32_t* __restrict__ inner_k, double* y, int64_t* iters, int scaled) {
  const int sb = blockIdx.x * blockDim.x + threadIdx.x;
  if (sb >= B || newton_active[sb] == 0) return;
  const int k = inner_k[sb];
  iters[2 * sb] += 1;
  iters[2 * sb + 1] += k;
  const double* Hs = H + (int64_t)sb * (kmax + 1) * kmax;
  const double* gs = gv + (int64_t)sb * (kmax + 1);
  double* ys = y + (int64_t)sb * kmax;
  for (int i = k - 1; i >= 0; --i) {
    double v = gs[i];
    for (int l = i + 1; l < k; ++l) v -= Hs[i * kmax + l] * ys[l];
    ys[i] = Hs[i * kmax + i] != 0.0 ? v / Hs[i * kmax + i] : 0.0;
  }
  if (scaled)
    for (int i = 0; i < k; ++i) ys[i] *= inv_eta[(int64_t)sb * (kmax + 1) + i];
}

void launch_solve_y(const Work& w, int32_t B, bool scaled, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_y, dim3((unsigned)cdiv(B, 64)), dim3(64), 0, s, B, w.kmax, w.H, w.g, w.inv_eta,
                     w.newton_active, w.inner_k, w.y, w.iters, scaled ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Activation time (Section 2.4): first crossing of u_th, linear in time.
__global__ void k_activation(const double* __restrict__ uk, const double* __restrict__ u, double* __restrict__ act,
                             int64_t total, double u_th, double t_k, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const double a = uk[i], b = u[i];
  if (a < u_th && b >= u_th && act[i] < 0.0) act[i] = t_k + dt * (u_th - a) / (b - a);
}

void launch_activation(const Work& w, int64_t nn, int32_t B, double u_th, double t_k, double dt, hipStream_t s) {
  launch_activation_between(w.uk, w.u, w.act, nn, B, u_th, t_k, dt, s);
}

void launch_activation_between(const double* uold, const double* unew, double* act, int64_t nn, int32_t B,
                               double u_th, double t_k, double dt, hipStream_t s) {
  const int64_t total = nn * B;
  hipLaunchKernelGGL(k_activation, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, uold, unew, act, total,
                     u_th, t_k, dt);
}

// All-at-once time blocks: U is [B][G][n] with slot 0 the block's initial state and slots 1 .. G - 1
// its unknown time levels.  Newton's first iterate of every slot q >= 1 (Section 3.3): mode 0 the
// initial state itself (the multiple-time-blocks start), 1 the reference solution r_(k0 + q) (global
// guess), 2 the initial state plus the reference's increment r_(k0 + q) - r_k0 (local guess).
__global__ void k_block_guess(double* __restrict__ U, int G, int64_t nn, int32_t B, const double* __restrict__ ref,
                              int k0, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * B) return;
  const int64_t b = i / nn, x = i - b * nn;
  double* Ub = U + b * G * nn;
  const double u0 = Ub[x];
  for (int q = 1; q < G; ++q) {
    double v = u0;
    if (mode == 1) v = ref[(int64_t)(k0 + q) * nn + x];
    if (mode == 2) v = u0 + (ref[(int64_t)(k0 + q) * nn + x] - ref[(int64_t)k0 * nn + x]);
    Ub[(int64_t)q * nn + x] = v;
  }
}

void launch_block_guess(double* U, int G, int64_t nn, int32_t B, const double* ref, int k0, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_block_guess, dim3((unsigned)cdiv(nn * B, kBlock)), dim3(kBlock), 0, s, U, G, nn, B, ref, k0,
                     mode);
}

// After a block: activation times of its steps (first crossing of u_th, linear in time between
// the time nodes t_(k0 + q - 1) and t_(k0 + q)), then slot 0 := the last slot (the next block's
// initial state).
__global__ void k_block_close(double* __restrict__ U, int G, int64_t nn, int32_t B, double* __restrict__ act,
                              double u_th, int k0, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * B) return;
  const int64_t b = i / nn, x = i - b * nn;
  double* Ub = U + b * G * nn;
  double a = act[i];
  double prev = Ub[x];
  for (int q = 1; q < G; ++q) {
    const double cur = Ub[(int64_t)q * nn + x];
    if (a < 0.0 && prev < u_th && cur >= u_th) a = (double)(k0 + q - 1) * dt + dt * (u_th - prev) / (cur - prev);
    prev = cur;
  }
  act[i] = a;
  Ub[x] = prev;
}

void launch_block_close(double* U, int G, int64_t nn, int32_t B, double* act, double u_th, int k0, double dt,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_block_close, dim3((unsigned)cdiv(nn * B, kBlock)), dim3(kBlock), 0, s, U, G, nn, B, act, u_th,
                     k0, dt);
}

// QoI: (1/|D|) sum_i w_i v_i with v = u (final) or the censored activation time.
__global__ __launch_bounds__(kBlock) void k_qoi(const double* __restrict__ u, const double* __restrict__ act,
                                                const double* __restrict__ wts, int64_t nn, int qoi, double t_stop,
                                                double vol, double* out) {
  __shared__ double sh[kBlock / 64];
  const int sb = blockIdx.x;
  const double* us = u + (int64_t)sb * nn;
  const double* as = act + (int64_t)sb * nn;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nn; i += kBlock) {
    const double v = qoi == MLQ_QOI_MEAN_U_FINAL ? us[i] : (as[i] < 0.0 ? t_stop : as[i]);
    acc += wts[i] * v;
  }
  acc = block_sum<kBlock>(acc, sh);
  if (threadIdx.x == 0) out[sb] = acc / vol;
}

void launch_qoi(const Work& w, const double* wts, int64_t nn, int32_t B, int qoi, double t_stop, double vol,
                double* qoi_out, hipStream_t s) {
  hipLaunchKernelGGL(k_qoi, dim3(B), dim3(kBlock), 0, s, w.uk, w.act, wts, nn, qoi, t_stop, vol, qoi_out);
}

// ---------------------------------------------------------------------------
// KL synthesis on the matrix cores, eq. (KLlowrank):
//   theta[b][p] = theta0[p] + sum_k (sqrt(lambda_k) Y[b][k]) phiT[k][p],
// a (B x M) (M x P) product with the basis stored mode-major (phiT, M x P).  MFMA
// 16x16x4 (f32 in mixed mode, f64 in FP64 mode) with samples as rows and elements as
// columns: lane l supplies A[l % 16][l / 16] = sqrt(lambda) Y of sample l % 16 and
// B[l / 16][l % 16] = phiT of element l % 16 (16 consecutive elements of one mode:
// one contiguous segment); its four results are rows 4 (l / 16) + r (f32) or
// l / 16 + 4 r (f64) of column l % 16, so the stores of a 16-lane group cover 16
// consecutive elements of one sample.  A wave tile is 16 elements by the 64 samples
// of the block's sample chunk (four 16 x 16 tiles); the block's four waves cover 64
// consecutive elements, and the block walks kKLTilesPerWave such groups with one
// staged chunk of sqrt(lambda) Y (128 modes at a time, in LDS).
constexpr int kKLModesPerStage = 128;

template <typename T>
struct MfmaKL;
template <>
struct MfmaKL<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct MfmaKL<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

constexpr int kKLTilesPerWave = 8;  // 16-element tiles a wave walks with one staged chunk

template <typename T>
__global__ __launch_bounds__(kBlock) void k_kl_mfma(const T* __restrict__ phiT, const double* __restrict__ sl,
                                                    const double* __restrict__ theta0, const double* __restrict__ Y,
                                                    int64_t P, int32_t M, int32_t B, T* __restrict__ theta) {
  typedef typename MfmaKL<T>::v4 v4;
  __shared__ T ys[kKLModesPerStage][64 + 1];
  const int b0 = blockIdx.y * 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int ks = 0; ks < M; ks += kKLModesPerStage) {
    const int mk = (M - ks) < kKLModesPerStage ? (M - ks) : kKLModesPerStage;
    __syncthreads();
    // consecutive threads read consecutive modes of one sample (Y is sample-major)
    for (int t = threadIdx.x; t < kKLModesPerStage * 64; t += kBlock) {
      const int bb = t / kKLModesPerStage, k = t % kKLModesPerStage;
      ys[k][bb] = (k < mk && b0 + bb < B) ? (T)(sl[ks + k] * Y[(int64_t)(b0 + bb) * M + ks + k]) : (T)0;
    }
    __syncthreads();
    for (int it = 0; it < kKLTilesPerWave; ++it) {
      const int64_t pt = (((int64_t)blockIdx.x * kKLTilesPerWave + it) * (kBlock / 64) + wid) * 16;
      if (pt >= P) break;
      const int64_t p = pt + li;
      const int64_t pa = p < P ? p : P - 1;  // clamped element (B column)
      v4 acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = v4{0, 0, 0, 0};
      // all basis values of the stage for this tile are loaded before the first product
      T a[kKLModesPerStage / 4];
#pragma unroll
      for (int q = 0; q < kKLModesPerStage / 4; ++q) {
        const int k = 4 * q + lk;
        a[q] = k < mk ? phiT[(int64_t)(ks + k) * P + pa] : (T)0;
      }
#pragma unroll
      for (int q = 0; q < kKLModesPerStage / 4; ++q) {
        if (4 * q >= mk) break;  // rows of ys past mk hold zeros
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = MfmaKL<T>::mma(ys[4 * q + lk][16 * c + li], a[q], acc[c]);
      }
      if (p < P) {
        const double t0 = ks == 0 ? (theta0 != nullptr ? theta0[p] : 0.0) : 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int b = b0 + 16 * c + MfmaKL<T>::row(lane, r);
            if (b < B) {
              T* o = theta + (int64_t)b * P + p;
              // modes beyond the first stage add to the partial field written before
              *o = ks == 0 ? (T)(t0 + (double)acc[c][r]) : (T)((double)*o + (double)acc[c][r]);
            }
          }
        }
      }
    }
  }
}

void launch_kl(const double* phi64T, const float* phi32T, const double* sqrt_lambda, const double* theta0,
               const double* Y, int64_t P, int32_t M, int32_t B, void* theta, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(P, 16 * (kBlock / 64) * kKLTilesPerWave), (unsigned)cdiv(B, 64));
  if (mixed)
    hipLaunchKernelGGL((k_kl_mfma<float>), grid, dim3(kBlock), 0, s, phi32T, sqrt_lambda, theta0, Y, P, M, B,
                       (float*)theta);
  else
    hipLaunchKernelGGL((k_kl_mfma<double>), grid, dim3(kBlock), 0, s, phi64T, sqrt_lambda, theta0, Y, P, M, B,
                       (double*)theta);
}

// dst (cols x rows) = transpose of src (rows x cols), FP64, through 32 x 33 LDS tiles.
__global__ void k_transpose_f64(const double* __restrict__ src, double* __restrict__ dst, int64_t rows,
                                int64_t cols) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows at a time
  for (int i = ty; i < 32; i += 8)
    if (r0 + i < rows && c0 + tx < cols) t[i][tx] = src[(r0 + i) * cols + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 32; i += 8)
    if (c0 + i < cols && r0 + tx < rows) dst[(c0 + i) * rows + r0 + tx] = t[tx][i];
}

void launch_transpose_f64(const double* src, double* dst, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows < 1 || cols < 1) return;
  hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)cdiv(cols, 32), (unsigned)cdiv(rows, 32)), dim3(256), 0, s,
                     src, dst, rows, cols);
}

// ---------------------------------------------------------------------------
// Shifted rank-1 lattice points mapped to N(0,1): y = Phi^-1(frac(((i z) mod N)/N + shift)).
// uniform != 0: y = 2x - 1 (the uniform coordinates on [-1, 1]) instead of Phi^-1(x).
__global__ void k_lattice(const int64_t* __restrict__ z, const double* __restrict__ shift, int32_t sdim, int64_t N,
                          int64_t first, int32_t count, int uniform, double* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)sdim * count) return;
  const int k = (int)(t % sdim);
  const int64_t i = first + t / sdim;
  const int64_t r = (i % N) * (z[k] % N) % N;
  double x = (double)r / (double)N + shift[k];
  if (x >= 1.0) x -= 1.0;
  if (uniform) {
    Y[t] = 2.0 * x - 1.0;
    return;
  }
  const double eps = 1.1102230246251565e-16;  // 2^-53
  x = x < eps ? eps : (x > 1.0 - eps ? 1.0 - eps : x);
  Y[t] = normcdfinv(x);
}

void launch_lattice(const int64_t* z, const double* shift, int32_t sdim, int64_t N, int64_t first, int32_t count,
                    bool uniform, double* Y, hipStream_t s) {
  const int64_t total = (int64_t)sdim * count;
  hipLaunchKernelGGL(k_lattice, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, z, shift, sdim, N, first,
                     count, uniform ? 1 : 0, Y);
}

// ---------------------------------------------------------------------------
// Halton points: coordinate k of point i is the radical inverse of i in the base of the
// (k+1)-th prime.  The digits of i, least significant first, are accumulated as the integer
// numerator r of r / p^J (J digits); both stay below 2^53 for i < 2^32 and p < 2^13, so the
// quotient is the exact rational rounded once.  Optional shift mod 1, then the map to uniform
// coordinates 2x - 1 or to Gaussian ones Phi^-1(x).

// The first kHaltonMaxDims primes, sieved at compile time.
struct PrimeTable {
  uint16_t p[kHaltonMaxDims];
};

constexpr PrimeTable make_primes() {
  constexpr int kLimit = 8192;  // the 1024th prime is 8161
  bool composite[kLimit] = {};
  PrimeTable t{};
  int n = 0;
  for (int c = 2; c < kLimit && n < kHaltonMaxDims; ++c) {
    if (composite[c]) continue;
    t.p[n++] = (uint16_t)c;
    for (int m = 2 * c; m < kLimit; m += c) composite[m] = true;
  }
  return t;
}

constexpr PrimeTable kPrimeTable = make_primes();
static_assert(kPrimeTable.p[kHaltonMaxDims - 1] == 8161, "prime table");
__constant__ PrimeTable kPrimes = kPrimeTable;

__global__ void k_halton(int32_t sdim, int64_t first, int32_t count, const double* __restrict__ shift,
                         int32_t uniform, double* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)sdim * count) return;
  const int k = (int)(t % sdim);
  const uint64_t p = kPrimes.p[k];
  uint64_t n = (uint64_t)(first + t / sdim), r = 0, q = 1;
  while (n > 0) {
    const uint64_t d = n / p;
    r = r * p + (n - d * p);
    n = d;
    q *= p;
  }
  double x = (double)r / (double)q;
  if (shift != nullptr) {
    x += shift[k];
    if (x >= 1.0) x -= 1.0;
  }
  if (uniform) {
    Y[t] = 2.0 * x - 1.0;
  } else {
    const double eps = 1.1102230246251565e-16;  // 2^-53
    x = x < eps ? eps : (x > 1.0 - eps ? 1.0 - eps : x);
    Y[t] = normcdfinv(x);
  }
}

void launch_halton(int32_t sdim, int64_t first, int32_t count, const double* shift, bool uniform, double* Y,
                   hipStream_t s) {
  const int64_t total = (int64_t)sdim * count;
  hipLaunchKernelGGL(k_halton, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, sdim, first, count, shift,
                     uniform ? 1 : 0, Y);
}

// ---------------------------------------------------------------------------
// Level difference and FP64 accumulation, one block, fixed order.
__global__ void k_accumulate(const double* __restrict__ ff, const double* __restrict__ fc, int32_t count,
                             double* acc) {
  __shared__ double sh[kBlock / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < count; i += kBlock) {
    const double y = ff[i] - (fc != nullptr ? fc[i] : 0.0);
    s1 += y;
    s2 += y * y;
  }
  s1 = block_sum<kBlock>(s1, sh);
  s2 = block_sum<kBlock>(s2, sh);
  if (threadIdx.x == 0) {
    acc[0] += (double)count;
    acc[1] += s1;
    acc[2] += s2;
  }
}

void launch_accumulate(const double* ff, const double* fc, int32_t count, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(kBlock), 0, s, ff, fc, count, acc);
}

}  // namespace mlq

namespace mlq {

// Newton bookkeeping: samples that failed stay frozen; the others start a step.
__global__ void k_newton_reset(const int32_t* __restrict__ status, int32_t* newton_active, int32_t B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) newton_active[i] = status[i] == MLQ_SAMPLE_OK ? 1 : 0;
}

__global__ void k_mark_failed(int32_t* status, int32_t* newton_active, int32_t B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B && newton_active[i] != 0) {
    status[i] = MLQ_SAMPLE_NOCONV;
    newton_active[i] = 0;
  }
}

void launch_newton_reset(const Work& w, int32_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_newton_reset, dim3((unsigned)cdiv(B, kBlock)), dim3(kBlock), 0, s, w.status,
                     w.newton_active, B);
}

void launch_mark_failed(const Work& w, int32_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_failed, dim3((unsigned)cdiv(B, kBlock)), dim3(kBlock), 0, s, w.status,
                     w.newton_active, B);
}

}  // namespace mlq

namespace mlq {

__global__ void k_cast_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

void launch_cast_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)cdiv(n, kBlock)), dim3(kBlock), 0, s, src, dst, n);
}

}  // namespace mlq

namespace mlq {

// ---------------------------------------------------------------------------
// Preconditioner P = M (I + D): exact inverse of the consistent Q1 mass, which is
// the Kronecker product of 1D masses M_a = h_a/6 tridiag(1, 4, 1) (2 on the end
// diagonals), followed by the pointwise division by (1 + d).  With right
// preconditioning the mass part of J P^-1 is the identity, so the Krylov
// operator is v -> v + dt/2 K P^-1 v.
//
// The 3D inverse runs as two passes: z-line solves (one thread per (x, y) column,
// the line in registers, the input scaled on the way in), then one workgroup per
// z-plane that stages the plane in LDS and solves its x lines and y lines before
// the pointwise output.  A 2D sample is one plane.  Every pass issues all of a
// thread's global loads before it uses the first one.
//
// Thomas elimination of tridiag(1, 4, 1) (2 at the ends); iv[i] = 1 / (pivot i)
// is precomputed per axis:  y_0 = v_0 iv_0,  y_i = (v_i - y_{i-1}) iv_i,
// x_{n-1} = y_{n-1},  x_i = y_i - iv_i x_{i+1}.
template <int N, typename T>
__device__ inline void thomas_regs(T (&v)[N], const T* __restrict__ iv) {
  T prev = v[0] * iv[0];
  v[0] = prev;
#pragma unroll
  for (int i = 1; i < N; ++i) {
    prev = (v[i] - prev) * iv[i];
    v[i] = prev;
  }
#pragma unroll
  for (int i = N - 2; i >= 0; --i) v[i] = v[i] - iv[i] * v[i + 1];
}

// The same elimination on a strided line a[i * stride] (LDS or global memory) of
// runtime length, in chunks of 16 entries whose loads are issued together.
template <typename T>
__device__ inline void line_solve(T* a, int n, int64_t stride, const T* __restrict__ iv) {
  constexpr int CH = 16;
  T prev = 0;
#pragma unroll 1
  for (int c0 = 0; c0 < n; c0 += CH) {
    T v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (c0 + i < n) v[i] = a[(c0 + i) * stride];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (c0 + i < n) {
        prev = (c0 + i == 0) ? v[i] * iv[0] : (v[i] - prev) * iv[c0 + i];
        v[i] = prev;
      }
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (c0 + i < n) a[(c0 + i) * stride] = v[i];
  }
  T nxt = prev;  // x_{n-1} = y_{n-1}
#pragma unroll 1
  for (int hi = n - 2; hi >= 0; hi -= CH) {
    T v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (hi - i >= 0) v[i] = a[(hi - i) * stride];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (hi - i >= 0) {
        nxt = v[i] - iv[hi - i] * nxt;
        v[i] = nxt;
      }
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (hi - i >= 0) a[(hi - i) * stride] = v[i];
  }
}

enum { kOutDivD = 1 };

__device__ inline double minv_scale(const double* __restrict__ inv_eta, int sb, int j, int kmax, double c6) {
  return c6 * (inv_eta != nullptr ? inv_eta[(int64_t)sb * (kmax + 1) + j] : 1.0);
}

// z lines: thread per (x, y) column of one sample (blockIdx.y); out = Mz^-1 (scale in).
template <typename T, int N>
__global__ __launch_bounds__(kBlock) void k_line_z(Geo g, const T* __restrict__ in, T* __restrict__ out,
                                                   const double* __restrict__ inv_eta, int j, int kmax, double c6,
                                                   const T* __restrict__ iv, const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  // time blocks (g.group > 1): sb is a virtual sample of sample sr, slot 0 the block's initial state
  const int grp = g.group > 1 ? g.group : 1, sr = sb / grp;
  if ((grp > 1 && sb == sr * grp) || active[sr] == 0) return;
  const int L = blockIdx.x * kBlock + threadIdx.x;
  if (L >= g.nx * g.ny) return;
  const int64_t stride = (int64_t)g.nx * g.ny;
  const int64_t base = (int64_t)sb * g.nn + L;
  const T s = (T)minv_scale(inv_eta, sr, j, kmax, c6);
  if constexpr (N > 0) {
    T v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = in[base + i * stride] * s;
    thomas_regs<N, T>(v, iv);
#pragma unroll
    for (int i = 0; i < N; ++i) out[base + i * stride] = v[i];
  } else {
    // runtime length: scaled copy into out, then the chunked elimination in place
    const int n = g.nz;
    for (int c0 = 0; c0 < n; c0 += 16) {
      T v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (c0 + i < n) v[i] = in[base + (c0 + i) * stride];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (c0 + i < n) out[base + (c0 + i) * stride] = v[i] * s;
    }
    line_solve<T>(out + base, n, stride, iv);
  }
}

// x and y lines of one z-plane (blockIdx.x) of one sample (blockIdx.y) in LDS, then
// the output divided by (1 + d).  The input is scaled by c6 inv_eta_j (inv_eta !=
// nullptr) or c6.  N: nx = ny when it is one of the unrolled sizes (each line solved in
// registers by one thread), else 0 (runtime size, chunked solves).  d is fetched after
// the sweeps, so the sweeps hold no prefetched registers.
template <typename T, int OUT, int N>
__global__ __launch_bounds__(kBlock) void k_plane_xy(Geo g, const T* __restrict__ in, T* __restrict__ out,
                                                     const double* __restrict__ inv_eta, int j, int kmax, double c6,
                                                     const T* __restrict__ ivx, const T* __restrict__ ivy,
                                                     const T* __restrict__ d, const int32_t* __restrict__ active) {
  extern __shared__ unsigned char smem_raw[];
  T* sh = reinterpret_cast<T*>(smem_raw);
  const int sb = blockIdx.y;
  const int grp = g.group > 1 ? g.group : 1, sr = sb / grp;
  if ((grp > 1 && sb == sr * grp) || active[sr] == 0) return;
  const int nx = N > 0 ? N : g.nx, ny = N > 0 ? N : g.ny;
  const int np = nx * ny;
  const int64_t base = (int64_t)sb * g.nn + (int64_t)blockIdx.x * np;
  const T s = (T)minv_scale(inv_eta, sr, j, kmax, c6);
  const int t0 = threadIdx.x;
  // entries t0 + q kBlock of the plane, in batches of PB whose loads are all issued first
  constexpr int PB = (N > 0 && N * N <= 24 * kBlock) ? (N * N + kBlock - 1) / kBlock : 16;
  for (int b0 = 0; b0 < np; b0 += PB * kBlock) {
    T r[PB];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (b0 + t0 + q * kBlock < np) r[q] = in[base + b0 + t0 + q * kBlock];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (b0 + t0 + q * kBlock < np) sh[b0 + t0 + q * kBlock] = r[q] * s;
  }
  __syncthreads();
  if constexpr (N > 0) {
    if (t0 < N) {
      T v[N];
      T* a = sh + t0 * N;
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = a[i];
      thomas_regs<N, T>(v, ivx);
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] = v[i];
    }
    __syncthreads();
    if (t0 < N) {
      T v[N];
      T* a = sh + t0;
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = a[i * N];
      thomas_regs<N, T>(v, ivy);
#pragma unroll
      for (int i = 0; i < N; ++i) a[i * N] = v[i];
    }
  } else {
    for (int r = t0; r < ny; r += kBlock) line_solve<T>(sh + r * nx, nx, 1, ivx);
    __syncthreads();
    for (int c = t0; c < nx; c += kBlock) line_solve<T>(sh + c, ny, nx, ivy);
  }
  __syncthreads();
  for (int b0 = 0; b0 < np; b0 += PB * kBlock) {
    T dv[PB];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (b0 + t0 + q * kBlock < np) dv[q] = d[base + b0 + t0 + q * kBlock];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (b0 + t0 + q * kBlock < np) {
        const int64_t o = base + b0 + t0 + q * kBlock;
        out[o] = sh[b0 + t0 + q * kBlock] / ((T)1 + dv[q]);
      }
  }
}

// dst <- P^-1 (scale src); tmp holds the z-solved field in 3D.
// N: common line length of all axes when it is one of the unrolled sizes, else 0.
template <typename T, int N>
static void minv_launch(const Geo& g, const T* src, T* tmp, T* dst, const double* inv_eta, int j, int kmax,
                        const T* tri, int nmax, const T* d, const int32_t* active, int32_t B, hipStream_t s) {
  const T* ivx = tri;
  const T* ivy = tri + nmax;
  const T* ivz = tri + 2 * nmax;
  const size_t sh = sizeof(T) * (size_t)g.nx * g.ny;
  const T* pin = src;
  const double* peta = inv_eta;
  double c6 = 36.0 / g.Hm;
  unsigned planes = 1;
  if (g.dim == 3) {
    hipLaunchKernelGGL((k_line_z<T, N>), dim3((unsigned)cdiv((int64_t)g.nx * g.ny, kBlock), B), dim3(kBlock), 0, s, g,
                       src, tmp, inv_eta, j, kmax, 216.0 / g.Hm, ivz, active);
    pin = tmp;
    peta = nullptr;
    c6 = 1.0;
    planes = (unsigned)g.nz;
  }
  hipLaunchKernelGGL((k_plane_xy<T, kOutDivD, N>), dim3(planes, B), dim3(kBlock), sh, s, g, pin, dst, peta, j, kmax,
                     c6, ivx, ivy, d, active);
}

template <typename T>
static void minv_dispatch(const Geo& g, const T* src, T* tmp, T* dst, const double* inv_eta, int j, int kmax,
                          const T* tri, int nmax, const T* d, const int32_t* active, int32_t B, hipStream_t s) {
  const bool cube = g.nx == g.ny && (g.dim == 2 || g.nz == g.nx);
  int n = cube ? g.nx : 0;
  // both passes hold whole lines in registers (FP64 lines of 129 run at one wave per
  // SIMD, which the 133 KB LDS plane of the xy pass imposes anyway)
#define MLQ_MINV(NN) minv_launch<T, NN>(g, src, tmp, dst, inv_eta, j, kmax, tri, nmax, d, active, B, s)
  switch (n) {
    case 9: MLQ_MINV(9); break;
    case 17: MLQ_MINV(17); break;
    case 33: MLQ_MINV(33); break;
    case 65: MLQ_MINV(65); break;
    case 129: MLQ_MINV(129); break;
    default: MLQ_MINV(0); break;
  }
#undef MLQ_MINV
}

// GMRES preconditioner step: z_j = P^-1 v_j (v_j = stored basis vector times inv_eta_j),
// kept as vector j of the preconditioned basis; w is scratch.
void launch_minv_basis(const Geo& g, const Work& w, const void* tri, int nmax, int j, int32_t B, bool mixed,
                       hipStream_t s) {
  const size_t vs = (size_t)g.nn * B;
  if (mixed)
    minv_dispatch<float>(g, (const float*)w.V + j * vs, (float*)w.w, (float*)w.z + j * vs, w.inv_eta, j, w.kmax,
                         (const float*)tri, nmax, (const float*)w.d, w.inner_active, B, s);
  else
    minv_dispatch<double>(g, (const double*)w.V + j * vs, (double*)w.w, (double*)w.z + j * vs, w.inv_eta, j, w.kmax,
                          (const double*)tri, nmax, (const double*)w.d, w.inner_active, B, s);
}

// Preconditioned operator: w = v_j + dt/2 K_G z  (the mass part of J P^-1 is the identity).
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_apply_pk(Geo g, const T* __restrict__ z, const T* __restrict__ vj,
                                                     const double* __restrict__ inv_eta, int j, int kmax,
                                                     const T* __restrict__ coef, T* __restrict__ w, T ck,
                                                     const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.nn) return;
  const T* zs = z + (int64_t)sb * g.nn;
  const T* cf = coef + (int64_t)sb * g.P * 2;
  int ix, iy, iz;
  node_xyz(i, g, ix, iy, iz);
  T xm[27], xk[27];
  load_nbhd<DIM, T>(
      ix, iy, iz, g,
      [&](int64_t jj, T& a, T& b) {
        a = 0;
        b = zs[jj];
      },
      xm, xk);
  T SM, SK;
  gather<DIM, T, T>(ix, iy, iz, g, cf, xm, xk, SM, SK);
  const int64_t o = (int64_t)sb * g.nn + i;
  const T sj = (T)inv_eta[(int64_t)sb * (kmax + 1) + j];
  w[o] = vj[o] * sj + ck * SK;
}

void launch_apply_pk(const Geo& g, const Work& w, int j, double ck, int32_t B, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)w.nblk, B);
  const size_t vs = (size_t)g.nn * B;
#define MLQ_APK(D, T)                                                                                         \
  hipLaunchKernelGGL((k_apply_pk<D, T>), grid, dim3(kBlock), 0, s, g, (const T*)w.z + j * vs, (const T*)w.V + j * vs, \
                     w.inv_eta, j, w.kmax, (const T*)w.coef, (T*)w.w, (T)ck, w.inner_active)
  if (g.dim == 3) {
    if (mixed) MLQ_APK(3, float); else MLQ_APK(3, double);
  } else {
    if (mixed) MLQ_APK(2, float); else MLQ_APK(2, double);
  }
#undef MLQ_APK
}

// Newton update, right preconditioning: u += P^-1 (sum_l y_l v_l).
// Newton update with right preconditioning on boxes: u += sum_l y_l z_l over the
// preconditioned basis (z_l = P^-1 v_l inv_eta_l, y_l from k_solve_y unscaled).  A thread takes
// kUpdNodes nodes a block apart, side by side: the loads of four basis vectors at all of its
// nodes (and the nodes' u) are in flight together; each node's sum runs in the order of l.
constexpr int kUpdNodes = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_zbasis(int64_t nn, const T* __restrict__ Z, size_t vs,
                                                          const double* __restrict__ y, int kmax,
                                                          const int32_t* __restrict__ inner_k, double* __restrict__ u,
                                                          const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  __shared__ double c[kMaxInner];
  const int k = inner_k[sb];
  for (int i = threadIdx.x; i < k; i += kBlock) c[i] = y[(int64_t)sb * kmax + i];
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kUpdNodes) + threadIdx.x;
  const int64_t base = (int64_t)sb * nn;
  double acc[kUpdNodes], uv[kUpdNodes];
#pragma unroll
  for (int r = 0; r < kUpdNodes; ++r) {
    const int64_t i = i0 + (int64_t)r * kBlock;
    acc[r] = 0.0;
    uv[r] = i < nn ? u[base + i] : 0.0;
  }
  for (int l0 = 0; l0 < k; l0 += 4) {
    T zv[kUpdNodes][4];
#pragma unroll
    for (int r = 0; r < kUpdNodes; ++r) {
      const int64_t i = i0 + (int64_t)r * kBlock;
#pragma unroll
      for (int q = 0; q < 4; ++q) zv[r][q] = (l0 + q < k && i < nn) ? Z[(l0 + q) * vs + base + i] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < kUpdNodes; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (l0 + q < k) acc[r] += c[l0 + q] * (double)zv[r][q];
  }
#pragma unroll
  for (int r = 0; r < kUpdNodes; ++r) {
    const int64_t i = i0 + (int64_t)r * kBlock;
    if (i < nn) u[base + i] = uv[r] + acc[r];
  }
}

void launch_update_zbasis(const Geo& g, const Work& w, int32_t B, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(g.nn, (int64_t)kBlock * kUpdNodes), B);
  const size_t vs = (size_t)g.nn * B;
  if (mixed)
    hipLaunchKernelGGL((k_update_zbasis<float>), grid, dim3(kBlock), 0, s, g.nn, (const float*)w.z, vs, w.y, w.kmax,
                       w.inner_k, w.u, w.newton_active);
  else
    hipLaunchKernelGGL((k_update_zbasis<double>), grid, dim3(kBlock), 0, s, g.nn, (const double*)w.z, vs, w.y,
                       w.kmax, w.inner_k, w.u, w.newton_active);
}

}  // namespace mlq


namespace mlq {

// Planes above 64 KB of LDS (129^2 in FP32 or FP64, non-unrolled sizes) need the
// dynamic LDS limit of the plane kernels raised.
hipError_t prepare_minv_kernels(size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  const int b = (int)bytes;
  hipError_t e = hipSuccess;
  auto set = [&](const void* k) {
    if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, b);
  };
  set((const void*)(k_plane_xy<double, kOutDivD, 0>));
  set((const void*)(k_plane_xy<float, kOutDivD, 0>));
  set((const void*)(k_plane_xy<float, kOutDivD, 129>));
  set((const void*)(k_plane_xy<double, kOutDivD, 129>));
  return e;
}

}  // namespace mlq
