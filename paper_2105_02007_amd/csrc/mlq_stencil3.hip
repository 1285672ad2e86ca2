// 3D Q1 operators of the space-time solve (Section 3.1 eq. (semi-disc),
// Section 3.2 Jacobian) on uniform brick meshes, as register-streaming kernels.
//
// One wave owns a 7 x 7 column of nodes of one sample and computes the 8 x 8
// elements around it (lane = i + 8 j <-> element (x0 - 1 + i, y0 - 1 + j)),
// marching up a chunk of 15 node planes.  Per slab of elements between two node
// planes every lane
//   1. holds its element's four corner values of the lower and the upper plane
//      in registers (neighbouring lanes hit the same cache lines),
//   2. computes the element's 8 outputs from the 8 nodal inputs with the
//      factored element operators below (one lane per element, no redundancy),
//   3. sums the contributions of the 4 + 4 elements around every owned node in
//      a fixed order, taking neighbour outputs by cross-lane shuffles (bottom
//      faces of this slab + top faces of the previous one).
// There is no LDS staging and no barrier; a ring of four plane register sets
// keeps the loads of the next planes in flight while a slab is computed.
//
// Element operators (edges hx, hy, hz; local node (a, b, c) in {0,1}^3;
// s(0) = -1, s(1) = +1; M1 = h/6 [[2,1],[1,2]]; K1 = 1/h [[1,-1],[-1,1]]).  With
//   G = sbar I + p (ex ex^T - ey ey^T) + q (ex ey^T + ey ex^T) + (st - sbar) ez ez^T
// (eq. (AdmV) for V = sigma_l (cos t, sin t, 0), p = ds/2 cos 2t, q = ds/2 sin 2t):
//   K_e = [(sbar + p) K1x (x) M1y + (sbar - p) M1x (x) K1y + q (C1x^T (x) C1y + C1x (x) C1y^T)] (x) M1z
//         + st M1x (x) M1y (x) K1z,      C1[i][j] = int phi_i phi_j' = s(j)/2,
// which on the z-mixed 2x2 layer u = (M1z x)_c reduces to
//   out_ab = s(a) [(sbar + p) X_b + q Dy / 4] + s(b) [(sbar - p) Y_a + q Dx / 4],
//   X = M1y dx / hx, Y = M1x dy / hy, dx_b = u_1b - u_0b, dy_a = u_a1 - u_a0,
//   Dx = dx_0 + dx_1, Dy = dy_0 + dy_1.
#include "mlq_internal.h"

namespace mlq {

namespace {

constexpr int NT = 256;           // threads per workgroup (four independent waves)

enum { kPK = 0, kFull = 1, kRes = 2, kRhs = 3 };

template <typename R>
struct Elem {
  // element outputs (8, index a + 2b + 4c) of M_e xm (scaled later) and K_e xk
  __host__ __device__ static inline void stiff(const R (&x)[8], R p, R q, const Geo& g, R (&o)[8]) {
    const R hx = (R)g.Hx, hy = (R)g.Hy, hz = (R)g.Hz;
    const R sb = (R)g.sbar, st = (R)g.st;
    const R z6 = hz / (R)6;
    // z-mix with M1z
    R m[2][4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
      m[0][ab] = z6 * ((R)2 * x[ab] + x[ab + 4]);
      m[1][ab] = z6 * (x[ab] + (R)2 * x[ab + 4]);
    }
    const R cx = hy / ((R)6 * hx), cy = hx / ((R)6 * hy);
    const R ap = sb + p, am = sb - p, q4 = (R)0.25 * q;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const R* u = m[c];
      const R dx0 = u[1] - u[0], dx1 = u[3] - u[2];  // b = 0, 1
      const R dy0 = u[2] - u[0], dy1 = u[3] - u[1];  // a = 0, 1
      const R X0 = cx * ((R)2 * dx0 + dx1), X1 = cx * (dx0 + (R)2 * dx1);
      const R Y0 = cy * ((R)2 * dy0 + dy1), Y1 = cy * (dy0 + (R)2 * dy1);
      const R Dx = dx0 + dx1, Dy = dy0 + dy1;
      const R A0 = ap * X0 + q4 * Dy, A1 = ap * X1 + q4 * Dy;
      const R B0 = am * Y0 + q4 * Dx, B1 = am * Y1 + q4 * Dx;
      o[4 * c + 0] = -A0 - B0;  // a = 0, b = 0
      o[4 * c + 1] = A0 - B1;   // a = 1, b = 0
      o[4 * c + 2] = -A1 + B0;  // a = 0, b = 1
      o[4 * c + 3] = A1 + B1;   // a = 1, b = 1
    }
    // st M1x (x) M1y (x) K1z
    R dz[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) dz[ab] = x[ab + 4] - x[ab];
    const R r0 = (R)2 * dz[0] + dz[1], r1 = dz[0] + (R)2 * dz[1];  // x-pass, b = 0
    const R r2 = (R)2 * dz[2] + dz[3], r3 = dz[2] + (R)2 * dz[3];  // x-pass, b = 1
    const R cz = st * hx * hy / ((R)36 * hz);
    const R t0 = cz * ((R)2 * r0 + r2), t1 = cz * ((R)2 * r1 + r3);
    const R t2 = cz * (r0 + (R)2 * r2), t3 = cz * (r1 + (R)2 * r3);
    o[0] -= t0; o[1] -= t1; o[2] -= t2; o[3] -= t3;
    o[4] += t0; o[5] += t1; o[6] += t2; o[7] += t3;
  }

  // M_e x (full mass, scaled by hx hy hz / 216)
  __host__ __device__ static inline void mass(const R (&x)[8], const Geo& g, R (&o)[8]) {
    const R f = (R)g.Hm / (R)216;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R t[4];
#pragma unroll
      for (int ab = 0; ab < 4; ++ab) t[ab] = (c == 0) ? ((R)2 * x[ab] + x[ab + 4]) : (x[ab] + (R)2 * x[ab + 4]);
      const R r0 = (R)2 * t[0] + t[1], r1 = t[0] + (R)2 * t[1];
      const R r2 = (R)2 * t[2] + t[3], r3 = t[2] + (R)2 * t[3];
      o[4 * c + 0] = f * ((R)2 * r0 + r2);
      o[4 * c + 1] = f * ((R)2 * r1 + r3);
      o[4 * c + 2] = f * (r0 + (R)2 * r2);
      o[4 * c + 3] = f * (r1 + (R)2 * r3);
    }
  }
};

__device__ inline double iion3(double u, const Ionic& io) {
  return io.alpha * (u - io.u_rest) * (u - io.u_th) * (u - io.u_peak);
}
__device__ inline double diion3(double u, const Ionic& io) {
  const double a = u - io.u_rest, b = u - io.u_th, c = u - io.u_peak;
  return io.alpha * (b * c + a * c + a * b);
}

template <typename T>
struct Args {
  Geo g;
  Ionic io;
  const T* x;         // kPK: z; kFull: x; kRes / kRhs: u (FP64, cast)
  const T* d;         // kFull: d
  const T* vj;        // kPK: basis vector
  const double* inv_eta;
  int j, kmax;
  const void* coef;   // [B][P][2], coefficient precision
  T* y;               // kPK: w; kFull: y
  const double* u;   // kRes / kRhs input (FP64)
  const double* bvec; // kRes: b
  double* bout;       // kRhs: b
  double* ucopy;      // kRhs: u := u_k
  const double* fbox; // kRhs
  double load;
  void* r0;           // kRes: -F (inner precision)
  void* dout;         // kRes: dt I'(u) (inner precision)
  double* part;       // kRes: partial norms
  double ck, cm;
  const int32_t* active;
  int tiles_x, tiles_y, zchunks;
};

}  // namespace

// Owned node (X, Y) = lane (X, Y) sums, in this order, vertex (1,1) of its own
// element, (0,1) of lane + 1, (1,0) of lane + 8 and (0,0) of lane + 9.
constexpr int WT = 7;   // owned nodes per wave along x and y
constexpr int WZ = 15;  // owned node planes per wave (WZ + 1 steps, a multiple of 4)

template <typename R>
__device__ inline R shdn(R v, int d) {
  return __shfl_down(v, d, 64);
}

template <typename R, typename TC, typename TI, int MODE>
__global__ __launch_bounds__(NT) void k_wave3(Args<R> A) {
  const Geo& g = A.g;
  const int sb = blockIdx.y;
  const bool sample_on = A.active == nullptr || A.active[sb] != 0;
  constexpr bool kMass = MODE != kPK;
  __shared__ double red[NT / 64][3];
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave: keep it (and everything derived
  // from it: tile, z-chunk, plane offsets) in scalar registers
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = blockIdx.x * (NT / 64) + wid;
  const int nwaves = A.tiles_x * A.tiles_y * A.zchunks;
  const bool wave_on = sample_on && gw < nwaves;
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  if (wave_on) {
    int t = gw;
    const int tx_i = t % A.tiles_x;
    t /= A.tiles_x;
    const int ty_i = t % A.tiles_y;
    const int zc = t / A.tiles_y;
    const int i = lane & 7, j = lane >> 3;
    const int ex = tx_i * WT - 1 + i, ey = ty_i * WT - 1 + j;  // this lane's element (= its node (0,0))
    const int zs = zc * WZ, ze = min(zs + WZ, g.nz);
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int64_t sbase = (int64_t)sb * g.nn;
    const TC* cf = (const TC*)A.coef + (int64_t)sb * g.P * 2;
    const int ex_n = g.nx - 1, ey_n = g.ny - 1;
    const bool elem_xy = ex >= 0 && ey >= 0 && ex < ex_n && ey < ey_n;
    const bool owner = i < WT && j < WT && ex + 1 < g.nx && ey + 1 < g.ny;
    // every load below uses an address clamped into the grid, so no lane branches around
    // a load and the compiler can count outstanding loads exactly; values of clamped
    // addresses only ever feed elements or nodes that are discarded
    const int cx0 = min(max(ex, 0), g.nx - 2), cy0 = min(max(ey, 0), g.ny - 2);
    const int64_t c00 = (int64_t)cy0 * g.nx + cx0;                     // corner (0,0) of the clamped element
    const int ocx = min(ex + 1, g.nx - 1), ocy = min(ey + 1, g.ny - 1);
    const int64_t oof = (int64_t)ocy * g.nx + ocx;                      // owned node (clamped)
    const int64_t ce = (int64_t)cx0 + (int64_t)ex_n * cy0;              // clamped element in its layer
    const int64_t layer = (int64_t)ex_n * ey_n;

    auto in_val = [&](int64_t o, R& vk, R& vm) {
      if constexpr (MODE == kPK) {
        vk = (R)A.x[o];
      } else if constexpr (MODE == kFull) {
        const R v = (R)A.x[o];
        vk = v;
        vm = v + (R)A.d[o] * v;
      } else if constexpr (MODE == kRes) {
        const double v = A.u[o];
        vk = (R)v;
        vm = (R)(v + A.io.dt * iion3(v, A.io));
      } else {
        const double v = A.u[o];
        vk = (R)v;
        vm = (R)v;
      }
    };
    struct Pl {
      R k[4], m[4];
    };
    auto fetch = [&](int k, Pl& r) {
      const int kk = min(max(k, 0), g.nz - 1);
      const int64_t pb = sbase + (int64_t)kk * plane + c00;
      in_val(pb, r.k[0], r.m[0]);
      in_val(pb + 1, r.k[1], r.m[1]);
      in_val(pb + g.nx, r.k[2], r.m[2]);
      in_val(pb + g.nx + 1, r.k[3], r.m[3]);
    };
    auto fetch_coef = [&](int k, R& p, R& q) {
      const int kk = min(max(k, 0), g.nz - 2);
      const int64_t eg = ce + layer * kk;
      p = (R)cf[2 * eg];
      q = (R)cf[2 * eg + 1];
    };

    auto fetch_pre = [&](int k, R& p0, R& p1) {
      const int kc = min(max(k, 0), g.nz - 1);
      const int64_t own = sbase + (int64_t)kc * plane + oof;
      p0 = 0;
      p1 = 0;
      if constexpr (MODE == kPK) p0 = A.vj[own];
      if constexpr (MODE == kRes) {
        p0 = (R)A.bvec[own];
        p1 = (R)A.u[own];
      }
      if constexpr (MODE == kRhs) {
        p0 = (R)A.fbox[own - sbase];
        p1 = (R)A.u[own];
      }
    };
    R sj = 0;
    if constexpr (MODE == kPK) sj = (R)A.inv_eta[(int64_t)sb * (A.kmax + 1) + A.j];

    // one slab: planes lo (k) and hi (k + 1) are resident; the loads of plane k + 3,
    // the coefficients of slab k + 2 and the node inputs of plane k + 2 are issued here
    R acc_top = 0;
    auto step = [&](int k, const Pl& lo, const Pl& hi, Pl& ld, R cp, R cq, R& lp, R& lq, R p0, R p1, R& lp0,
                    R& lp1) {
      fetch(k + 3, ld);
      fetch_coef(k + 2, lp, lq);
      fetch_pre(k + 2, lp0, lp1);
      const bool slab = k >= 0 && k <= g.nz - 2;
      R o[8];
      {
        R xin[8] = {lo.k[0], lo.k[1], lo.k[2], lo.k[3], hi.k[0], hi.k[1], hi.k[2], hi.k[3]};
        Elem<R>::stiff(xin, cp, cq, g, o);
        const R sc = (slab && elem_xy) ? (R)A.ck : (R)0;
#pragma unroll
        for (int c = 0; c < 8; ++c) o[c] *= sc;
        if constexpr (kMass) {
          R xm[8] = {lo.m[0], lo.m[1], lo.m[2], lo.m[3], hi.m[0], hi.m[1], hi.m[2], hi.m[3]};
          R om[8];
          Elem<R>::mass(xm, g, om);
          const R sm = (slab && elem_xy) ? (R)A.cm : (R)0;
#pragma unroll
          for (int c = 0; c < 8; ++c) o[c] += sm * om[c];
        }
      }
      // assemble the owned node: bottom faces of slab k (plane k), top faces (plane k + 1)
      const R bot = o[3] + shdn(o[2], 1) + shdn(o[1], 8) + shdn(o[0], 9);
      const R top = o[7] + shdn(o[6], 1) + shdn(o[5], 8) + shdn(o[4], 9);
      if (owner && k >= zs && k < ze) {
        const int64_t own = sbase + (int64_t)k * plane + oof;
        const R sres = acc_top + bot;
        if constexpr (MODE == kPK) {
          A.y[own] = p0 * sj + sres;
        } else if constexpr (MODE == kFull) {
          A.y[own] = sres;
        } else if constexpr (MODE == kRes) {
          const double G = (double)sres;
          const double bb = (double)p0;
          const double F = G - bb;
          ((TI*)A.r0)[own] = (TI)(-F);
          ((TI*)A.dout)[own] = (TI)(A.io.dt * diion3((double)p1, A.io));
          n0 += F * F;
          n1 += G * G;
          n2 += bb * bb;
        } else {
          A.bout[own] = (double)sres + A.load * (double)p0;
          A.ucopy[own] = (double)p1;
        }
      }
      acc_top = top;
    };

    // ring of four plane sets (P), coefficient sets (C) and node-input sets (Q), rotated by
    // unrolling four steps; a wave covers slabs zs - 1 .. zs + WZ - 1 (16 steps)
    const int k0 = zs - 1;
    Pl P0, P1, P2, P3;
    R C0p, C0q, C1p, C1q, C2p, C2q, C3p, C3q;
    R Q00, Q01, Q10, Q11, Q20, Q21, Q30, Q31;
    fetch(k0, P0);
    fetch(k0 + 1, P1);
    fetch(k0 + 2, P2);
    fetch_coef(k0, C0p, C0q);
    fetch_coef(k0 + 1, C1p, C1q);
    fetch_pre(k0, Q00, Q01);
    fetch_pre(k0 + 1, Q10, Q11);
    for (int it = 0; it < (WZ + 1) / 4; ++it) {
      const int k = k0 + 4 * it;
      step(k + 0, P0, P1, P3, C0p, C0q, C2p, C2q, Q00, Q01, Q20, Q21);
      step(k + 1, P1, P2, P0, C1p, C1q, C3p, C3q, Q10, Q11, Q30, Q31);
      step(k + 2, P2, P3, P1, C2p, C2q, C0p, C0q, Q20, Q21, Q00, Q01);
      step(k + 3, P3, P0, P2, C3p, C3q, C1p, C1q, Q30, Q31, Q10, Q11);
    }
  }
  if constexpr (MODE == kRes) {
    double v[3] = {n0, n1, n2};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    }
    if (lane == 0) {
      red[wid][0] = v[0];
      red[wid][1] = v[1];
      red[wid][2] = v[2];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s0 = 0, s1 = 0, s2 = 0;
      for (int w = 0; w < NT / 64; ++w) {
        s0 += red[w][0];
        s1 += red[w][1];
        s2 += red[w][2];
      }
      double* p = A.part + ((int64_t)sb * gridDim.x + blockIdx.x) * 3;
      p[0] = s0;
      p[1] = s1;
      p[2] = s2;
    }
  }
}

namespace {

template <typename R>
void wave_grid_of(const Geo& g, Args<R>& a, int32_t B, dim3& grid) {
  a.tiles_x = (int)cdiv(g.nx, WT);
  a.tiles_y = (int)cdiv(g.ny, WT);
  a.zchunks = (int)cdiv(g.nz, WZ);
  grid = dim3((unsigned)cdiv((int64_t)a.tiles_x * a.tiles_y * a.zchunks, NT / 64), (unsigned)B);
}

}  // namespace

int32_t stencil3_blocks(const Geo& g) {
  return (int32_t)cdiv(cdiv(g.nx, WT) * cdiv(g.ny, WT) * cdiv(g.nz, WZ), NT / 64);
}

void launch_apply_pk3(const Geo& g, const Work& w, int j, double ck, int32_t B, bool mixed, hipStream_t s) {
  const size_t vs = (size_t)g.nn * B;
  if (mixed) {
    Args<float> a{};
    a.g = g; a.x = (const float*)w.z; a.vj = (const float*)w.V + j * vs; a.inv_eta = w.inv_eta; a.j = j;
    a.kmax = w.kmax; a.coef = w.coef; a.y = (float*)w.w; a.ck = ck; a.cm = 0.0; a.active = w.inner_active;
    dim3 grid;
    wave_grid_of(g, a, B, grid);
    hipLaunchKernelGGL((k_wave3<float, float, float, kPK>), grid, dim3(NT), 0, s, a);
  } else {
    Args<double> a{};
    a.g = g; a.x = (const double*)w.z; a.vj = (const double*)w.V + j * vs; a.inv_eta = w.inv_eta; a.j = j;
    a.kmax = w.kmax; a.coef = w.coef; a.y = (double*)w.w; a.ck = ck; a.cm = 0.0; a.active = w.inner_active;
    dim3 grid;
    wave_grid_of(g, a, B, grid);
    hipLaunchKernelGGL((k_wave3<double, double, double, kPK>), grid, dim3(NT), 0, s, a);
  }
}

void launch_apply_full3(const Geo& g, const void* coef, const void* x, const void* d, void* y, double ck, int32_t B,
                        bool mixed, hipStream_t s) {
  if (mixed) {
    Args<float> a{};
    a.g = g; a.x = (const float*)x; a.d = (const float*)d; a.coef = coef; a.y = (float*)y; a.ck = ck; a.cm = 1.0;
    dim3 grid;
    wave_grid_of(g, a, B, grid);
    hipLaunchKernelGGL((k_wave3<float, float, float, kFull>), grid, dim3(NT), 0, s, a);
  } else {
    Args<double> a{};
    a.g = g; a.x = (const double*)x; a.d = (const double*)d; a.coef = coef; a.y = (double*)y; a.ck = ck; a.cm = 1.0;
    dim3 grid;
    wave_grid_of(g, a, B, grid);
    hipLaunchKernelGGL((k_wave3<double, double, double, kFull>), grid, dim3(NT), 0, s, a);
  }
}

void launch_residual3(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s) {
  Args<double> a{};
  a.g = g; a.io = io; a.u = w.u; a.bvec = w.b; a.coef = w.coef; a.r0 = w.V; a.dout = w.d; a.part = w.part;
  a.ck = 0.5 * io.dt; a.cm = 1.0; a.active = w.newton_active;
  dim3 grid;
  wave_grid_of(g, a, B, grid);
  if (mixed)
    hipLaunchKernelGGL((k_wave3<double, float, float, kRes>), grid, dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_wave3<double, double, double, kRes>), grid, dim3(NT), 0, s, a);
}

void launch_rhs3(const Geo& g, const Work& w, const double* fbox, double load_coef, double dt, int32_t B, bool mixed,
                 hipStream_t s) {
  Args<double> a{};
  a.g = g; a.u = w.uk; a.coef = w.coef; a.bout = w.b; a.ucopy = w.u; a.fbox = fbox; a.load = load_coef;
  a.ck = -0.5 * dt; a.cm = 1.0; a.active = nullptr;
  dim3 grid;
  wave_grid_of(g, a, B, grid);
  if (mixed)
    hipLaunchKernelGGL((k_wave3<double, float, float, kRhs>), grid, dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_wave3<double, double, double, kRhs>), grid, dim3(NT), 0, s, a);
}

}  // namespace mlq
