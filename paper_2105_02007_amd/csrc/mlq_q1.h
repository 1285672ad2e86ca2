// Q1 box element arithmetic and block reductions shared by the batched kernels
// (mlq_kernels.hip) and the per-sample persistent solver (mlq_small.hip).
#pragma once

#include "mlq_internal.h"

namespace mlq {

// ---------------------------------------------------------------------------
// 1D factors of the Q1 brick element matrices (Section 3.1, eq. (semi-disc)).
// Local node a of an element has bit k = offset along axis k.
//   mass      int phi_a phi_b           = h * mm(a, b)
//   stiffness int phi_a' phi_b'         = kk(a, b) / h
//   mixed     int phi_a phi_b'          = ss(b) / 2
__host__ __device__ constexpr double mm(int p, int q) { return p == q ? (1.0 / 3.0) : (1.0 / 6.0); }
__host__ __device__ constexpr double kk(int p, int q) { return p == q ? 1.0 : -1.0; }
__host__ __device__ constexpr double ss(int p) { return p ? 1.0 : -1.0; }

template <typename T>
__device__ inline T ld(const T* p) { return *p; }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum; result valid in every thread.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) r += sh[i];
  return r;
}

// Ionic current eq. (ionic_term) and its derivative.
__device__ inline double iion(double u, const Ionic& io) {
  return io.alpha * (u - io.u_rest) * (u - io.u_th) * (u - io.u_peak);
}
__device__ inline double diion(double u, const Ionic& io) {
  const double a = u - io.u_rest, b = u - io.u_th, c = u - io.u_peak;
  return io.alpha * (b * c + a * c + a * b);
}

// ---------------------------------------------------------------------------
// Matrix-free gather of the mass and anisotropic stiffness rows of node i.
// G_e = (cx0 + cx1 p_e) e_x e_x^T + (cy0 + cy1 p_e) e_y e_y^T + q_e (e_x e_y^T + e_y e_x^T)
//       [+ (cz0 + cz1 p_e) e_z e_z^T]  (the constants of the conductivity model in Geo), which
// equals eq. (AdmV) with V = sigma_l (cos t, sin t, 0), g = sigma_t for the fibre model
// (p = (sigma_l - sigma_t)/2 cos 2t, q = (sigma_l - sigma_t)/2 sin 2t) and v I for the
// isotropic one (p = v, q = 0).
// xm / xk: the 3^d neighbourhood values of the mass input and stiffness input.
// Returns SM = sum_e (M_e xm)_a / Hm and SK = sum_e (K_e xk)_a.
template <typename R, typename TC>
__host__ __device__ inline void gather3(int ix, int iy, int iz, const Geo& g, const TC* __restrict__ cf,
                               const R (&xm)[27], const R (&xk)[27], R& SM, R& SK) {
  SM = R(0);
  SK = R(0);
#pragma unroll
  for (int oz = -1; oz <= 0; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 0; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 0; ++ox) {
        const int ex = ix + ox, ey = iy + oy, ez = iz + oz;
        if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx - 1 || ey >= g.ny - 1 || ez >= g.nz - 1) continue;
        const int ax = -ox, ay = -oy, az = -oz;
        const int64_t e = ex + (int64_t)(g.nx - 1) * (ey + (int64_t)(g.ny - 1) * ez);
        const R p = (R)cf[2 * e], q = (R)cf[2 * e + 1];
        R sm = 0, sx = 0, sy = 0, sz = 0, sc = 0;
#pragma unroll
        for (int bz = 0; bz < 2; ++bz)
#pragma unroll
          for (int by = 0; by < 2; ++by)
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
              const int nb = (ox + bx + 1) + 3 * ((oy + by + 1) + 3 * (oz + bz + 1));
              sm += (R)(mm(ax, bx) * mm(ay, by) * mm(az, bz)) * xm[nb];
              sx += (R)(kk(ax, bx) * mm(ay, by) * mm(az, bz)) * xk[nb];
              sy += (R)(mm(ax, bx) * kk(ay, by) * mm(az, bz)) * xk[nb];
              sz += (R)(mm(ax, bx) * mm(ay, by) * kk(az, bz)) * xk[nb];
              sc += (R)(0.25 * (ss(ax) * ss(by) + ss(ay) * ss(bx)) * mm(az, bz)) * xk[nb];
            }
        SM += sm;
        SK += ((R)g.cx0 + (R)g.cx1 * p) * (R)g.Hxx * sx + ((R)g.cy0 + (R)g.cy1 * p) * (R)g.Hyy * sy +
              ((R)g.cz0 + (R)g.cz1 * p) * (R)g.Hzz * sz + q * (R)g.Hxy * sc;
      }
}

template <typename R, typename TC>
__host__ __device__ inline void gather2(int ix, int iy, const Geo& g, const TC* __restrict__ cf, const R (&xm)[27],
                               const R (&xk)[27], R& SM, R& SK) {
  SM = R(0);
  SK = R(0);
#pragma unroll
  for (int oy = -1; oy <= 0; ++oy)
#pragma unroll
    for (int ox = -1; ox <= 0; ++ox) {
      const int ex = ix + ox, ey = iy + oy;
      if (ex < 0 || ey < 0 || ex >= g.nx - 1 || ey >= g.ny - 1) continue;
      const int ax = -ox, ay = -oy;
      const int64_t e = ex + (int64_t)(g.nx - 1) * ey;
      const R p = (R)cf[2 * e], q = (R)cf[2 * e + 1];
      R sm = 0, sx = 0, sy = 0, sc = 0;
#pragma unroll
      for (int by = 0; by < 2; ++by)
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
          const int nb = (ox + bx + 1) + 3 * (oy + by + 1) + 9;  // middle plane of the 3x3x3 block
          sm += (R)(mm(ax, bx) * mm(ay, by)) * xm[nb];
          sx += (R)(kk(ax, bx) * mm(ay, by)) * xk[nb];
          sy += (R)(mm(ax, bx) * kk(ay, by)) * xk[nb];
          sc += (R)(0.25 * (ss(ax) * ss(by) + ss(ay) * ss(bx))) * xk[nb];
        }
      SM += sm;
      SK += ((R)g.cx0 + (R)g.cx1 * p) * (R)g.Hxx * sx + ((R)g.cy0 + (R)g.cy1 * p) * (R)g.Hyy * sy +
            q * (R)g.Hxy * sc;
    }
}

// Decode node index of a sample into grid coordinates.
__host__ __device__ inline void node_xyz(int64_t i, const Geo& g, int& ix, int& iy, int& iz) {
  ix = (int)(i % g.nx);
  const int64_t r = i / g.nx;
  iy = (int)(r % g.ny);
  iz = (int)(r / g.ny);
}

// Load the 3^d neighbourhood through a functor f(node_index) -> (mass input, stiffness input).
template <int DIM, typename R, typename F>
__host__ __device__ inline void load_nbhd(int ix, int iy, int iz, const Geo& g, F f, R (&xm)[27], R (&xk)[27]) {
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int nb = (dx + 1) + 3 * ((dy + 1) + 3 * (dz + 1));
        if (DIM == 2 && dz != 0) {
          xm[nb] = 0;
          xk[nb] = 0;
          continue;
        }
        const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        const bool in = jx >= 0 && jy >= 0 && jz >= 0 && jx < g.nx && jy < g.ny && jz < g.nz;
        if (in) {
          const int64_t j = jx + (int64_t)g.nx * (jy + (int64_t)g.ny * jz);
          f(j, xm[nb], xk[nb]);
        } else {
          xm[nb] = 0;
          xk[nb] = 0;
        }
      }
}

template <int DIM, typename R, typename TC>
__host__ __device__ inline void gather(int ix, int iy, int iz, const Geo& g, const TC* cf, const R (&xm)[27],
                              const R (&xk)[27], R& SM, R& SK) {
  if constexpr (DIM == 3)
    gather3<R, TC>(ix, iy, iz, g, cf, xm, xk, SM, SK);
  else
    gather2<R, TC>(ix, iy, g, cf, xm, xk, SM, SK);
}

}  // namespace mlq
