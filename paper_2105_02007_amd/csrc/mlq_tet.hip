// P1 tetrahedral operators of the space-time solve (Section 3.1 eq. (semi-disc)
// with the P1 space of a tetrahedral mesh; Section 3.2 Jacobian).
//
// The stiffness depends on the sample through the fibre angle of each element,
//   K_e[a][b] = |T| ( sigma_t g_a . g_b + (sigma_l - sigma_t) (g_a . f)(g_b . f) ),
//   f = cos(theta) e_circ + sin(theta) e_long,
// (eq. (AdmV) with V = sigma_l f; g_a = grad phi_a).  Once per solve its values are
// gathered per stored entry of the vertex-adjacency pattern (each entry sums its
// element contributions in increasing element order: deterministic, no atomics) into
// kval[b][e].  The mass M (P1, |T| (1 + delta_ab) / 20) is shared by all samples.
// The pattern is stored slot-major and padded to the longest row (entry (s, i) at
// s * nv + i), so that in every operator application (one thread per row and sample,
// or per row and group of samples in the Jacobian apply; rows of one sample contiguous,
// samples on blockIdx.y) a wave reads the columns, mass and stiffness values of slot s
// for 64 consecutive rows in one coalesced load.  Within a row the slots follow
// increasing column order.
#include "mlq_internal.h"

namespace mlq {

namespace {

// XCD-aware block numbering: workgroups go to the 8 XCDs round-robin by linear id.  Give each
// XCD one contiguous range of (row block, sample group) blocks, so that the column gathers of
// neighbouring row blocks meet in one L2.  Within the range the sample groups of a row block
// are consecutive, so the shared pattern (columns, mass) of that block is fetched from HBM once
// and read from L2 by the other groups.  (bx, by) replace (blockIdx.x, blockIdx.y).
__device__ inline void xcd_block(int64_t& bx, int64_t& by) {
  const int64_t NB = (int64_t)gridDim.x * gridDim.y;
  const int64_t L = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
  const int64_t q = NB >> 3, r = NB & 7, x = L & 7;
  const int64_t W = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (L >> 3);
  by = W % gridDim.y;
  bx = W / gridDim.y;
}

__device__ inline double tet_iion(double u, const Ionic& io) {
  return io.alpha * (u - io.u_rest) * (u - io.u_th) * (u - io.u_peak);
}
__device__ inline double tet_diion(double u, const Ionic& io) {
  const double a = u - io.u_rest, b = u - io.u_th, c = u - io.u_peak;
  return io.alpha * (b * c + a * c + a * b);
}

// Fibre-angle model (model 0): f = cos(theta) e_circ + sin(theta) e_long,
// G = s_t I + (s_l - s_t) f f^T.  Isotropic model (1): G = max(theta, s_t) I, s_t the lower
// bound.  Vector model (2): the field is V = vmean + (theta_0, theta_1, theta_2) per element,
// component c of sample b at theta[(c B + b) P + e], and G = g I + (|V| - g) V V^T / V^T V
// (eq. (AdmV) with g = sigma_t).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tet_assemble(TetDev t, const T* __restrict__ theta, T* __restrict__ kval,
                                                         double sigma_t, double dsig, int model, int32_t B,
                                                         const double* __restrict__ vmean) {
  const int sb = blockIdx.y;
  const int64_t nz = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (nz >= t.nell) return;
  const T* th = theta + (int64_t)sb * t.nt;
  const int64_t cstride = (int64_t)B * t.nt;
  double acc = 0.0;
  for (int32_t c = t.ecptr[nz]; c < t.ecptr[nz + 1]; ++c) {
    const int32_t code = t.ecdat[c];
    const int64_t e = code >> 4;
    const int a = (code >> 2) & 3, b = code & 3;
    const double* G = t.geo + e * kTetGeo;
    const double ga0 = G[3 * a], ga1 = G[3 * a + 1], ga2 = G[3 * a + 2];
    const double gb0 = G[3 * b], gb1 = G[3 * b + 1], gb2 = G[3 * b + 2];
    const double gg = ga0 * gb0 + ga1 * gb1 + ga2 * gb2;
    if (model == 1) {
      const double v = (double)th[e];
      acc += G[18] * (v > sigma_t ? v : sigma_t) * gg;
    } else if (model == 2) {
      const double v0 = vmean[3 * e] + (double)th[e], v1 = vmean[3 * e + 1] + (double)th[cstride + e];
      const double v2 = vmean[3 * e + 2] + (double)th[2 * cstride + e];
      const double vv = v0 * v0 + v1 * v1 + v2 * v2;
      const double av = ga0 * v0 + ga1 * v1 + ga2 * v2;
      const double bv = gb0 * v0 + gb1 * v1 + gb2 * v2;
      acc += G[18] * (sigma_t * gg + (sqrt(vv) - sigma_t) * av * bv / vv);
    } else {
      double sn, cs;
      sincos((double)th[e], &sn, &cs);
      const double f0 = cs * G[12] + sn * G[15], f1 = cs * G[13] + sn * G[16], f2 = cs * G[14] + sn * G[17];
      const double af = ga0 * f0 + ga1 * f1 + ga2 * f2;
      const double bf = gb0 * f0 + gb1 * f1 + gb2 * f2;
      acc += G[18] * (sigma_t * gg + dsig * af * bf);
    }
  }
  kval[(int64_t)sb * t.nell + nz] = (T)acc;
}

// y = M ((1 + d) x) + ck K x.  A thread takes one row for kTetSamples samples, so that the
// shared pattern (columns, mass) is read once for all of them; each sample's sum runs over
// the slots in the same order as for one sample.
constexpr int kTetSamples = 4;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tet_apply(TetDev t, const T* __restrict__ kval, const T* __restrict__ x,
                                                      const T* __restrict__ d, T* __restrict__ y, T ck, int32_t B,
                                                      const int32_t* __restrict__ active) {
  constexpr int S = kTetSamples;
  int64_t bx, by;
  xcd_block(bx, by);
  const int sb0 = (int)by * S;
  bool on[S];
  bool any = false;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    on[q] = sb0 + q < B && (active == nullptr || active[sb0 + q] != 0);
    any = any || on[q];
  }
  if (!any) return;
  const int64_t i = bx * kBlock + threadIdx.x;
  if (i >= t.nv) return;
  const T* mv = nullptr;
  if constexpr (sizeof(T) == 4) mv = (const T*)t.em32; else mv = (const T*)t.em;
  T acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = 0;
  bool all = true;
#pragma unroll
  for (int q = 0; q < S; ++q) all = all && on[q];
  if (all) {
    // Every sample of the group active (the usual case): no per-sample branch in the slot loop, so
    // the gathers of all samples and of the next slot are in flight together. Same arithmetic, in
    // the same order, as the general loop below.
#pragma unroll 2
    for (int32_t sl = 0; sl < t.width; ++sl) {
      const int64_t e = (int64_t)sl * t.nv + i;
      const int64_t c = t.ecol[e];
      const T m = mv[e];
      T dv[S], xv[S], kv[S];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const int64_t j = (int64_t)(sb0 + q) * t.nv + c;
        dv[q] = d[j];
        xv[q] = x[j];
        kv[q] = kval[(int64_t)(sb0 + q) * t.nell + e];
      }
#pragma unroll
      for (int q = 0; q < S; ++q) acc[q] += (m * ((T)1 + dv[q]) + ck * kv[q]) * xv[q];
    }
#pragma unroll
    for (int q = 0; q < S; ++q) y[(int64_t)(sb0 + q) * t.nv + i] = acc[q];
    return;
  }
  for (int32_t sl = 0; sl < t.width; ++sl) {
    const int64_t e = (int64_t)sl * t.nv + i;
    const int64_t c = t.ecol[e];
    const T m = mv[e];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      if (!on[q]) continue;
      const int64_t so = (int64_t)(sb0 + q) * t.nv;
      const int64_t j = so + c;
      acc[q] += (m * ((T)1 + d[j]) + ck * kval[(int64_t)(sb0 + q) * t.nell + e]) * x[j];
    }
  }
#pragma unroll
  for (int q = 0; q < S; ++q)
    if (on[q]) y[(int64_t)(sb0 + q) * t.nv + i] = acc[q];
}

// F = M (u + dt I_ion(u)) + dt/2 K u - b (FP64), r0 = -F, d = dt I_ion'(u), partial norms.  A
// thread takes one row of kTetSamples samples, as the apply does: the column and the mass value
// of a slot are loaded once for the group, and the gathers of all samples are in flight together
// (samples past the batch or not active read another sample's values, which are discarded).  Per
// sample the sums run in the same order as one sample per thread would.
template <typename TI>
__global__ __launch_bounds__(kBlock) void k_tet_residual(TetDev t, Ionic io, const TI* __restrict__ kval,
                                                         const double* __restrict__ u, const double* __restrict__ bv,
                                                         TI* __restrict__ r0, TI* __restrict__ dout,
                                                         double* __restrict__ part,
                                                         const int32_t* __restrict__ active, int32_t B) {
  constexpr int S = kTetSamples;
  int64_t bx, by;
  xcd_block(bx, by);
  const int sb0 = (int)by * S;
  bool on[S];
  int sq[S];
  bool any = false;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    on[q] = sb0 + q < B && active[sb0 + q] != 0;
    sq[q] = min(sb0 + q, B - 1);
    any = any || on[q];
  }
  if (!any) return;
  const int64_t i = bx * kBlock + threadIdx.x;
  double n0[S], n1[S], n2[S];
#pragma unroll
  for (int q = 0; q < S; ++q) n0[q] = n1[q] = n2[q] = 0.0;
  if (i < t.nv) {
    const double ck = 0.5 * io.dt;
    double G[S];
#pragma unroll
    for (int q = 0; q < S; ++q) G[q] = 0.0;
#pragma unroll 2
    for (int32_t sl = 0; sl < t.width; ++sl) {
      const int64_t e = (int64_t)sl * t.nv + i;
      const int64_t c = t.ecol[e];
      const double m = t.em[e];
      double uj[S];
      TI kv[S];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        uj[q] = u[(int64_t)sq[q] * t.nv + c];
        kv[q] = kval[(int64_t)sq[q] * t.nell + e];
      }
#pragma unroll
      for (int q = 0; q < S; ++q) G[q] += m * (uj[q] + io.dt * tet_iion(uj[q], io)) + ck * (double)kv[q] * uj[q];
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
      if (!on[q]) continue;
      const int64_t so = (int64_t)(sb0 + q) * t.nv;
      const double b = bv[so + i];
      const double F = G[q] - b;
      r0[so + i] = (TI)(-F);
      dout[so + i] = (TI)(io.dt * tet_diion(u[so + i], io));
      n0[q] = F * F;
      n1[q] = G[q] * G[q];
      n2[q] = b * b;
    }
  }
  __shared__ double red[kBlock / 64][S][3];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    double v[3] = {n0[q], n1[q], n2[q]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    }
    if (lane == 0) {
      red[wid][q][0] = v[0];
      red[wid][q][1] = v[1];
      red[wid][q][2] = v[2];
    }
  }
  __syncthreads();
  bool onq = false;  // on[threadIdx.x] without a runtime index into a register array
#pragma unroll
  for (int q = 0; q < S; ++q) onq = onq || ((int)threadIdx.x == q && on[q]);
  if (onq) {
    const int q = threadIdx.x;
    double s0 = 0, s1 = 0, s2 = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      s0 += red[w][q][0];
      s1 += red[w][q][1];
      s2 += red[w][q][2];
    }
    double* p = part + ((int64_t)(sb0 + q) * gridDim.x + bx) * 3;
    p[0] = s0;
    p[1] = s1;
    p[2] = s2;
  }
}

// b = M u_k - dt/2 K u_k + load F (FP64), u = u_k
template <typename TI>
// Also, with uprev (u_{k-1}, may be NULL): the extrapolated Newton start 2 u_k - u_{k-1}
// (extrap) and the activation times of the step from t_prev = t_{k-1} to t_k into act.
__global__ __launch_bounds__(kBlock) void k_tet_rhs(TetDev t, const TI* __restrict__ kval,
                                                    const double* __restrict__ uk, const double* __restrict__ fload,
                                                    double load, double ck, double* __restrict__ bout,
                                                    double* __restrict__ ucopy, const double* __restrict__ uprev,
                                                    double* __restrict__ act, double u_th, double t_prev, double dt,
                                                    int extrap, int32_t B) {
  constexpr int S = kTetSamples;  // one row of kTetSamples samples per thread, as in the apply
  int64_t bx, by;
  xcd_block(bx, by);
  const int sb0 = (int)by * S;
  const int64_t i = bx * kBlock + threadIdx.x;
  if (i >= t.nv) return;
  int sq[S];
#pragma unroll
  for (int q = 0; q < S; ++q) sq[q] = min(sb0 + q, B - 1);  // past the batch: read, not stored
  double acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = 0.0;
#pragma unroll 2
  for (int32_t sl = 0; sl < t.width; ++sl) {
    const int64_t e = (int64_t)sl * t.nv + i;
    const int64_t c = t.ecol[e];
    const double m = t.em[e];
    double uj[S];
    TI kv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      uj[q] = uk[(int64_t)sq[q] * t.nv + c];
      kv[q] = kval[(int64_t)sq[q] * t.nell + e];
    }
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] += (m - ck * (double)kv[q]) * uj[q];
  }
  const double fl = load * fload[i];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (sb0 + q >= B) break;
    const int64_t so = (int64_t)(sb0 + q) * t.nv;
    bout[so + i] = acc[q] + fl;
    const double u0 = uk[so + i];
    double ustart = u0;
    if (uprev != nullptr) {
      const double um = uprev[so + i];
      if (extrap) ustart = 2.0 * u0 - um;
      // the activation time is read only where u crosses the threshold
      if (um < u_th && u0 >= u_th && act[so + i] < 0.0) act[so + i] = t_prev + dt * (u_th - um) / (u0 - um);
    }
    ucopy[so + i] = ustart;
  }
}

// GMRES preconditioner step (Jacobi on the whole Jacobian): z_j = v_j inv_eta_j / J_ii with
// J_ii = m_ii (1 + d_i) + ck k_ii, into the preconditioned basis.  The stiffness diagonal
// matters where the mesh is fine (near the apex dt sigma / h^2 is of order one there).  A thread
// takes kJacRows rows a block apart, side by side, with the loads of all of them in flight.
constexpr int kJacRows = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tet_jacobi(TetDev t, const T* __restrict__ v, const T* __restrict__ d,
                                                       const T* __restrict__ kval, T ck, T* __restrict__ z,
                                                       const double* __restrict__ inv_eta, int j, int kmax,
                                                       const int32_t* __restrict__ active) {
  const int sb = blockIdx.y;
  if (active[sb] == 0) return;
  const T* md = nullptr;
  if constexpr (sizeof(T) == 4) md = (const T*)t.mdiag32; else md = (const T*)t.mdiag;
  const T s = (T)inv_eta[(int64_t)sb * (kmax + 1) + j];
  const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kJacRows) + threadIdx.x;
  const int64_t base = (int64_t)sb * t.nv;
  const T* ks = kval + (int64_t)sb * t.nell;
  T vv[kJacRows], dv[kJacRows], kv[kJacRows], mv[kJacRows];
#pragma unroll
  for (int r = 0; r < kJacRows; ++r) {
    const int64_t i = min(i0 + (int64_t)r * kBlock, t.nv - 1);  // clamped: rows past the end are not stored
    vv[r] = v[base + i];
    dv[r] = d[base + i];
    kv[r] = ks[(int64_t)t.ediag[i] * t.nv + i];
    mv[r] = md[i];
  }
#pragma unroll
  for (int r = 0; r < kJacRows; ++r) {
    const int64_t i = i0 + (int64_t)r * kBlock;
    if (i < t.nv) z[base + i] = vv[r] * s / (mv[r] * ((T)1 + dv[r]) + ck * kv[r]);
  }
}

}  // namespace

void launch_tet_assemble(const TetDev& t, const void* theta, void* kval, int32_t B, double sigma_t, double dsig,
                         bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(t.nell, kBlock), B);
  if (mixed)
    hipLaunchKernelGGL((k_tet_assemble<float>), grid, dim3(kBlock), 0, s, t, (const float*)theta, (float*)kval,
                       sigma_t, dsig, t.model, B, t.vmean);
  else
    hipLaunchKernelGGL((k_tet_assemble<double>), grid, dim3(kBlock), 0, s, t, (const double*)theta, (double*)kval,
                       sigma_t, dsig, t.model, B, t.vmean);
}

void launch_tet_apply(const TetDev& t, const void* kval, const void* x, const void* d, void* y, double ck, int32_t B,
                      const int32_t* active, bool mixed, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(t.nv, kBlock), (unsigned)cdiv(B, kTetSamples));
  if (mixed)
    hipLaunchKernelGGL((k_tet_apply<float>), grid, dim3(kBlock), 0, s, t, (const float*)kval, (const float*)x,
                       (const float*)d, (float*)y, (float)ck, B, active);
  else
    hipLaunchKernelGGL((k_tet_apply<double>), grid, dim3(kBlock), 0, s, t, (const double*)kval, (const double*)x,
                       (const double*)d, (double*)y, ck, B, active);
}

void launch_tet_residual(const TetDev& t, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s) {
  // gridDim.x = w.nres blocks per sample; kTetSamples samples per block row
  const dim3 grid((unsigned)cdiv(t.nv, kBlock), (unsigned)cdiv(B, kTetSamples));
  if (mixed)
    hipLaunchKernelGGL((k_tet_residual<float>), grid, dim3(kBlock), 0, s, t, io, (const float*)w.coef, w.u, w.b,
                       (float*)w.V, (float*)w.d, w.part, w.newton_active, B);
  else
    hipLaunchKernelGGL((k_tet_residual<double>), grid, dim3(kBlock), 0, s, t, io, (const double*)w.coef, w.u, w.b,
                       (double*)w.V, (double*)w.d, w.part, w.newton_active, B);
}

void launch_tet_rhs(const TetDev& t, const Work& w, const double* fload, double load, double dt, int32_t B,
                    bool mixed, hipStream_t s, const double* uprev, bool extrap, double u_th, double t_prev) {
  const dim3 grid((unsigned)cdiv(t.nv, kBlock), (unsigned)cdiv(B, kTetSamples));
  if (mixed)
    hipLaunchKernelGGL((k_tet_rhs<float>), grid, dim3(kBlock), 0, s, t, (const float*)w.coef, w.uk, fload, load,
                       0.5 * dt, w.b, w.u, uprev, w.act, u_th, t_prev, dt, extrap ? 1 : 0, B);
  else
    hipLaunchKernelGGL((k_tet_rhs<double>), grid, dim3(kBlock), 0, s, t, (const double*)w.coef, w.uk, fload, load,
                       0.5 * dt, w.b, w.u, uprev, w.act, u_th, t_prev, dt, extrap ? 1 : 0, B);
}

void launch_tet_jacobi_basis(const TetDev& t, const Work& w, int j, double ck, int32_t B, bool mixed,
                             hipStream_t s) {
  const dim3 grid((unsigned)cdiv(t.nv, (int64_t)kBlock * kJacRows), B);
  const size_t vs = (size_t)t.nv * B;
  if (mixed)
    hipLaunchKernelGGL((k_tet_jacobi<float>), grid, dim3(kBlock), 0, s, t, (const float*)w.V + j * vs,
                       (const float*)w.d, (const float*)w.coef, (float)ck, (float*)w.z + j * vs, w.inv_eta, j, w.kmax,
                       w.inner_active);
  else
    hipLaunchKernelGGL((k_tet_jacobi<double>), grid, dim3(kBlock), 0, s, t, (const double*)w.V + j * vs,
                       (const double*)w.d, (const double*)w.coef, ck, (double*)w.z + j * vs, w.inv_eta, j, w.kmax,
                       w.inner_active);
}

}  // namespace mlq
