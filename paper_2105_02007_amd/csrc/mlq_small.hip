// Persistent per-sample solver for small 3D box levels.
//
// The same method as the batched host-steered path (Section 3.3: time stepping, i.e. time
// blocks of one step, each step's nonlinear system eq. (mono_disc) solved by Newton's method
// from the extrapolated start, every Newton system by right-preconditioned GMRES with
// P = M (I + D) and classical Gram-Schmidt; the stopping test of the fused 3D residual), but
// with the whole time loop of one sample inside one workgroup: no launch and no host round
// trip per iteration.  A coarse level of a multilevel estimator has thousands of samples of a
// few thousand nodes each; the batched path then issues several launches per GMRES iteration
// whose kernels each touch only a few hundred bytes per sample, and the level is bound by
// launch latency.  Here a grid of one wave of resident workgroups walks the batch (workgroup
// b takes samples b, b + G, ...), each sample's vectors stay in L2 between passes, and the
// preconditioner runs on a copy of the vector in LDS.
//
// Work layout: the batched workspace (Work), sample sb's vectors at offset sb * n of every
// [B][n] array, so both paths take the same workspace.
#include "mlq_internal.h"
#include "mlq_q1.h"

namespace mlq {

namespace {

constexpr int NT = kSmallThreads;

// Row of the stiffness K_G at node (ix, iy, iz) applied to the 3^3 neighbourhood xk (the
// stiffness half of gather3).
template <typename R, typename TC>
__device__ inline R stiff_row3(int ix, int iy, int iz, const Geo& g, const TC* __restrict__ cf, const R (&xk)[27]) {
  R SK = 0;
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
        R sx = 0, sy = 0, sz = 0, sc = 0;
#pragma unroll
        for (int bz = 0; bz < 2; ++bz)
#pragma unroll
          for (int by = 0; by < 2; ++by)
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
              const int nb = (ox + bx + 1) + 3 * ((oy + by + 1) + 3 * (oz + bz + 1));
              sx += (R)(kk(ax, bx) * mm(ay, by) * mm(az, bz)) * xk[nb];
              sy += (R)(mm(ax, bx) * kk(ay, by) * mm(az, bz)) * xk[nb];
              sz += (R)(mm(ax, bx) * mm(ay, by) * kk(az, bz)) * xk[nb];
              sc += (R)(0.25 * (ss(ax) * ss(by) + ss(ay) * ss(bx)) * mm(az, bz)) * xk[nb];
            }
        SK += ((R)g.cx0 + (R)g.cx1 * p) * (R)g.Hxx * sx + ((R)g.cy0 + (R)g.cy1 * p) * (R)g.Hyy * sy +
              ((R)g.cz0 + (R)g.cz1 * p) * (R)g.Hzz * sz + q * (R)g.Hxy * sc;
      }
  return SK;
}

// Row of the mass (divided by Hm) at node (ix, iy, iz) applied to the 3^3 neighbourhood xm.
template <typename R>
__device__ inline R mass_row3(int ix, int iy, int iz, const Geo& g, const R (&xm)[27]) {
  R SM = 0;
#pragma unroll
  for (int oz = -1; oz <= 0; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 0; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 0; ++ox) {
        const int ex = ix + ox, ey = iy + oy, ez = iz + oz;
        if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx - 1 || ey >= g.ny - 1 || ez >= g.nz - 1) continue;
        const int ax = -ox, ay = -oy, az = -oz;
        R sm = 0;
#pragma unroll
        for (int bz = 0; bz < 2; ++bz)
#pragma unroll
          for (int by = 0; by < 2; ++by)
#pragma unroll
            for (int bx = 0; bx < 2; ++bx) {
              const int nb = (ox + bx + 1) + 3 * ((oy + by + 1) + 3 * (oz + bz + 1));
              sm += (R)(mm(ax, bx) * mm(ay, by) * mm(az, bz)) * xm[nb];
            }
        SM += sm;
      }
  return SM;
}

// The 3^3 neighbourhood of node (ix, iy, iz) through f(node) (0 outside the grid).
template <typename R, typename F>
__device__ inline void load_nb(int ix, int iy, int iz, const Geo& g, F f, R (&x)[27]) {
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
        const bool in = jx >= 0 && jy >= 0 && jz >= 0 && jx < g.nx && jy < g.ny && jz < g.nz;
        x[(dx + 1) + 3 * ((dy + 1) + 3 * (dz + 1))] =
            in ? f(jx + (int64_t)g.nx * (jy + (int64_t)g.ny * jz)) : (R)0;
      }
}

// Thomas elimination of tridiag(1, 4, 1) (2 at the ends) on a strided line, iv = 1 / pivots.
template <typename T>
__device__ inline void thomas_line(T* a, int n, int stride, const T* __restrict__ iv) {
  T prev = a[0] * iv[0];
  a[0] = prev;
  for (int i = 1; i < n; ++i) {
    prev = (a[i * stride] - prev) * iv[i];
    a[i * stride] = prev;
  }
  for (int i = n - 2; i >= 0; --i) a[i * stride] = a[i * stride] - iv[i] * a[(i + 1) * stride];
}

template <typename TI>
__global__ __launch_bounds__(NT) void k_solve_small(SmallArgs a) {
  extern __shared__ unsigned char smem_raw[];
  TI* tz = reinterpret_cast<TI*>(smem_raw);  // n values: the preconditioner's vector, then z_j
  __shared__ double sh[NT / 64];
  __shared__ double red[NT / 64][kMaxInner + 1];
  __shared__ double s_g[kMaxInner + 1], s_ie[kMaxInner + 1], s_hc[kMaxInner + 1];
  __shared__ double s_cs[kMaxInner], s_sn[kMaxInner], s_y[kMaxInner];
  __shared__ int s_stop;
  const Geo& g = a.g;
  const Ionic& io = a.io;
  const int64_t n = g.nn;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const size_t vs = (size_t)n * a.B;
  const int kmax = a.kmax;
  const TI* ivx = (const TI*)a.tri;
  const TI* ivy = ivx + a.nmax;
  const TI* ivz = ivy + a.nmax;
  const double dt = io.dt, ck = 0.5 * dt, hm = g.Hm;
  const double lw = g.Hx * g.Hy * g.Hz;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t plane = (int64_t)nx * ny;
  const TI minv_c = (TI)(216.0 / hm);

  for (int sb = blockIdx.x; sb < a.B; sb += gridDim.x) {
    double* pk = a.w.uk + (int64_t)sb * n;     // u_k
    double* pkm1 = a.w.ukm1 + (int64_t)sb * n; // u_(k-1)
    double* pu = a.w.u + (int64_t)sb * n;      // Newton iterate
    double* act = a.w.act + (int64_t)sb * n;
    TI* d = (TI*)a.w.d + (int64_t)sb * n;
    TI* wv = (TI*)a.w.w + (int64_t)sb * n;
    TI* V = (TI*)a.w.V + (int64_t)sb * n;      // vector l at V + l vs (stored unnormalised, s_ie[l] = 1 / norm)
    TI* Z = (TI*)a.w.z + (int64_t)sb * n;      // preconditioned basis z_l = P^-1 v_l s_ie[l]
    const TI* cf = (const TI*)a.w.coef + (int64_t)sb * g.P * 2;
    double* H = a.w.H + (int64_t)sb * (kmax + 1) * kmax;
    for (int64_t i = t; i < n; i += NT) {
      pk[i] = 0.0;
      act[i] = (0.0 >= io.u_th) ? 0.0 : -1.0;
    }
    int status = MLQ_SAMPLE_OK;
    int64_t newton_its = 0, inner_its = 0;
    __syncthreads();
    for (int k = 0; k < a.n_steps && status == MLQ_SAMPLE_OK; ++k) {
      const double t0 = (double)k * dt, t1 = (double)(k + 1) * dt;
      const double r0 = (a.t_on <= t0 && t0 < a.t_off) ? a.amp : 0.0;
      const double r1 = (a.t_on <= t1 && t1 < a.t_off) ? a.amp : 0.0;
      const double load = 0.5 * dt * (r1 + r0);
      // Newton start (u_k or 2 u_k - u_(k-1)) and the activation times of the previous step
      for (int64_t i = t; i < n; i += NT) {
        const double u0 = pk[i];
        double s = u0;
        if (k > 0) {
          const double um = pkm1[i];
          if (a.extrap) s = 2.0 * u0 - um;
          if (um < io.u_th && u0 >= io.u_th && act[i] < 0.0)
            act[i] = (double)(k - 1) * dt + dt * (io.u_th - um) / (u0 - um);
        }
        pu[i] = s;
      }
      __syncthreads();
      for (int it = 0;; ++it) {
        // residual F = M ((u - u_k) + dt I_ion(u)) + dt/2 K (u + u_k) - load F_box, d = dt I_ion'(u),
        // r0 = -F into V_0; stopping test |F| <= tol (|w u| + |w u_k + load F_box|), w the lumped mass
        double n0 = 0.0, n1 = 0.0, n2 = 0.0;
        for (int64_t i = t; i < n; i += NT) {
          int ix, iy, iz;
          node_xyz(i, g, ix, iy, iz);
          // the stiffness and the mass parts one after the other (one 27-value neighbourhood live
          // at a time; the second reads hit the cache)
          double xn[27];
          load_nb<double>(ix, iy, iz, g, [&](int64_t q) { return pu[q] + pk[q]; }, xn);
          const double SK = stiff_row3<double, TI>(ix, iy, iz, g, cf, xn);
          load_nb<double>(ix, iy, iz, g, [&](int64_t q) {
            const double uu = pu[q];
            return (uu - pk[q]) + dt * iion(uu, io);
          }, xn);
          const double SM = mass_row3<double>(ix, iy, iz, g, xn);
          const double fb = load * a.fbox[i];
          const double F = hm * SM + ck * SK - fb;
          const double uo = pu[i];
          V[i] = (TI)(-F);
          d[i] = (TI)(dt * diion(uo, io));
          const double wl = lw * ((ix == 0 || ix == nx - 1) ? 0.5 : 1.0) * ((iy == 0 || iy == ny - 1) ? 0.5 : 1.0) *
                            ((iz == 0 || iz == nz - 1) ? 0.5 : 1.0);
          n0 += F * F;
          n1 += (wl * uo) * (wl * uo);
          n2 += (wl * pk[i] + fb) * (wl * pk[i] + fb);
        }
        const double F2 = block_sum<NT>(n0, sh);
        const double G2 = block_sum<NT>(n1, sh);
        const double B2 = block_sum<NT>(n2, sh);
        const double nf = sqrt(F2), den = sqrt(G2) + sqrt(B2);
        const double err = den == 0.0 ? 0.0 : nf / den;
        if (!(err == err) || !isfinite(nf)) {
          status = MLQ_SAMPLE_NAN;
          break;
        }
        if (err <= a.newton_tol || nf == 0.0) break;
        if (it >= a.max_newton) {
          status = MLQ_SAMPLE_NOCONV;
          break;
        }
        // GMRES on J e = -F from e = 0
        if (t == 0) {
          s_ie[0] = 1.0 / nf;
          s_g[0] = nf;
          s_stop = 0;
        }
        for (int j = t + 1; j <= kmax; j += NT) s_g[j] = 0.0;
        __syncthreads();
        int kin = 0;
        for (int j = 0; j < kmax; ++j) {
          // z_j = P^-1 v_j = (I + D)^-1 M^-1 v_j: M^-1 as three families of line solves (the
          // Kronecker factors of the Q1 mass), in LDS
          const TI sc = minv_c * (TI)s_ie[j];
          const TI* vj = V + (size_t)j * vs;
          for (int64_t i = t; i < n; i += NT) tz[i] = vj[i] * sc;
          __syncthreads();
          for (int L = t; L < nx * ny; L += NT) thomas_line<TI>(tz + L, nz, (int)plane, ivz);
          __syncthreads();
          for (int L = t; L < nx * nz; L += NT) thomas_line<TI>(tz + (L % nx) + plane * (L / nx), ny, nx, ivy);
          __syncthreads();
          for (int L = t; L < ny * nz; L += NT) thomas_line<TI>(tz + (int64_t)L * nx, nx, 1, ivx);
          __syncthreads();
          TI* zj = Z + (size_t)j * vs;
          for (int64_t i = t; i < n; i += NT) {
            const TI z = tz[i] / ((TI)1 + d[i]);
            tz[i] = z;
            zj[i] = z;
          }
          __syncthreads();
          // w = J z_j = v_j s_ie[j] + dt/2 K z_j (the mass part of J P^-1 is the identity), and the
          // classical Gram-Schmidt projections w . v_l (l <= j; the first eight in the same pass)
          constexpr int JF = 8;
          double acc[JF];
#pragma unroll
          for (int l = 0; l < JF; ++l) acc[l] = 0.0;
          const TI iej = (TI)s_ie[j];
          for (int64_t i = t; i < n; i += NT) {
            int ix, iy, iz;
            node_xyz(i, g, ix, iy, iz);
            TI xk[27];
            load_nb<TI>(ix, iy, iz, g, [&](int64_t q) { return tz[q]; }, xk);
            const TI wi = vj[i] * iej + (TI)ck * stiff_row3<TI, TI>(ix, iy, iz, g, cf, xk);
            wv[i] = wi;
#pragma unroll
            for (int l = 0; l < JF; ++l)
              if (l <= j) acc[l] += (double)wi * (double)V[(size_t)l * vs + i];
          }
#pragma unroll
          for (int l = 0; l < JF; ++l) {
            if (l > j) break;
            const double v = wave_sum(acc[l]);
            if (lane == 0) red[wid][l] = v;
          }
          for (int l = JF; l <= j; ++l) {  // later projections: one more pass each (rare)
            double s = 0.0;
            for (int64_t i = t; i < n; i += NT) s += (double)wv[i] * (double)V[(size_t)l * vs + i];
            s = wave_sum(s);
            if (lane == 0) red[wid][l] = s;
          }
          __syncthreads();
          for (int l = t; l <= j; l += NT) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NT / 64; ++q) s += red[q][l];
            const double h = s * s_ie[l];
            s_hc[l] = h * s_ie[l];
            H[(size_t)l * kmax + j] = h;
          }
          __syncthreads();
          // v_(j+1) = w - sum_l h_lj v_l (stored unnormalised) and its norm
          TI* vn = V + (size_t)(j + 1) * vs;
          double nacc = 0.0;
          for (int64_t i = t; i < n; i += NT) {
            double v = (double)wv[i];
            for (int l = 0; l <= j; ++l) v -= s_hc[l] * (double)V[(size_t)l * vs + i];
            const TI vt = (TI)v;
            vn[i] = vt;
            nacc += (double)vt * (double)vt;
          }
          const double nrm2 = block_sum<NT>(nacc, sh);
          if (t == 0) {
            // Givens rotations of column j and the residual estimate |g_(j+1)|
            const double hn = sqrt(nrm2);
            s_ie[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
            for (int i = 0; i < j; ++i) {
              const double x = H[(size_t)i * kmax + j], y = H[(size_t)(i + 1) * kmax + j];
              H[(size_t)i * kmax + j] = s_cs[i] * x + s_sn[i] * y;
              H[(size_t)(i + 1) * kmax + j] = -s_sn[i] * x + s_cs[i] * y;
            }
            const double x = H[(size_t)j * kmax + j];
            const double r = hypot(x, hn);
            double cj = 1.0, sj = 0.0;
            if (r > 0.0) {
              cj = x / r;
              sj = hn / r;
            }
            s_cs[j] = cj;
            s_sn[j] = sj;
            H[(size_t)j * kmax + j] = r;
            H[(size_t)(j + 1) * kmax + j] = 0.0;
            s_g[j + 1] = -sj * s_g[j];
            s_g[j] = cj * s_g[j];
            const double res = fabs(s_g[j + 1]);
            s_stop = (res <= a.inner_tol * nf || hn == 0.0 || j + 1 >= kmax || !(res == res)) ? 1 : 0;
          }
          __syncthreads();
          if (s_stop) {
            kin = j + 1;
            break;
          }
        }
        // back substitution R y = g, then u += sum_l y_l z_l
        if (t == 0) {
          for (int i = kin - 1; i >= 0; --i) {
            double v = s_g[i];
            for (int l = i + 1; l < kin; ++l) v -= H[(size_t)i * kmax + l] * s_y[l];
            const double r = H[(size_t)i * kmax + i];
            s_y[i] = r != 0.0 ? v / r : 0.0;
          }
        }
        __syncthreads();
        for (int64_t i = t; i < n; i += NT) {
          double s = 0.0;
          for (int l = 0; l < kin; ++l) s += s_y[l] * (double)Z[(size_t)l * vs + i];
          pu[i] += s;
        }
        __syncthreads();
        ++newton_its;
        inner_its += kin;
      }
      // u_(k-1) <- u_k <- u (the old u_(k-1) becomes the next iterate's storage)
      double* old = pkm1;
      pkm1 = pk;
      pk = pu;
      pu = old;
      __syncthreads();
    }
    // the last step's activation times, then the quantity of interest
    const double t_stop = (double)a.n_steps * dt;
    double acc = 0.0;
    for (int64_t i = t; i < n; i += NT) {
      if (a.n_steps > 0 && status == MLQ_SAMPLE_OK) {
        const double um = pkm1[i], u0 = pk[i];
        if (um < io.u_th && u0 >= io.u_th && act[i] < 0.0)
          act[i] = (double)(a.n_steps - 1) * dt + dt * (io.u_th - um) / (u0 - um);
      }
      const double v = a.qoi == MLQ_QOI_MEAN_U_FINAL ? pk[i] : (act[i] < 0.0 ? t_stop : act[i]);
      acc += a.wts[i] * v;
      if (a.u_out != nullptr) a.u_out[(int64_t)sb * n + i] = pk[i];
      if (a.act_out != nullptr) a.act_out[(int64_t)sb * n + i] = act[i];
    }
    acc = block_sum<NT>(acc, sh);
    if (t == 0) {
      a.qoi_out[sb] = acc / a.vol;
      a.status_out[sb] = status;
      a.iters_out[2 * sb] = newton_its;
      a.iters_out[2 * sb + 1] = inner_its;
    }
    __syncthreads();
  }
}

}  // namespace

bool small_solver_fits(const Geo& g, bool mixed) {
  return g.dim == 3 && !g.tet && g.group <= 1 && g.nn * (mixed ? 4 : 8) <= kSmallMaxLds;
}

hipError_t launch_solve_small(const SmallArgs& a, bool mixed, hipStream_t s) {
  const size_t lds = (size_t)a.g.nn * (mixed ? sizeof(float) : sizeof(double));
  const void* fn = mixed ? (const void*)k_solve_small<float> : (const void*)k_solve_small<double>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallMaxLds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds);
  if (e != hipSuccess) return e;
  const int64_t resident = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  const unsigned grid = (unsigned)(a.B < resident ? a.B : resident);
  if (mixed)
    hipLaunchKernelGGL(k_solve_small<float>, dim3(grid), dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL(k_solve_small<double>, dim3(grid), dim3(NT), lds, s, a);
  return hipGetLastError();
}

}  // namespace mlq
