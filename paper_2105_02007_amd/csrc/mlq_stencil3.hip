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
//   G = G_xx ex ex^T + G_yy ey ey^T + G_xy (ex ey^T + ey ex^T) + G_zz ez ez^T
// (G_xx = cx0 + cx1 p, G_yy = cy0 + cy1 p, G_zz = cz0 + cz1 p, G_xy = q from the per-element
// coefficients; eq. (AdmV) for V = sigma_l (cos t, sin t, 0) is G_xx, G_yy = sbar +- p,
// G_zz = sigma_t with p = ds/2 cos 2t, q = ds/2 sin 2t; the isotropic model is G = v I):
//   K_e = [G_xx K1x (x) M1y + G_yy M1x (x) K1y + G_xy (C1x^T (x) C1y + C1x (x) C1y^T)] (x) M1z
//         + G_zz M1x (x) M1y (x) K1z,    C1[i][j] = int phi_i phi_j' = s(j)/2,
// which on the z-mixed 2x2 layer u = (M1z x)_c reduces to
//   out_ab = s(a) [G_xx X_b + G_xy Dy / 4] + s(b) [G_yy Y_a + G_xy Dx / 4],
//   X = M1y dx / hx, Y = M1x dy / hy, dx_b = u_1b - u_0b, dy_a = u_a1 - u_a0,
//   Dx = dx_0 + dx_1, Dy = dy_0 + dy_1.
#include <type_traits>

#include "mlq_internal.h"

namespace mlq {

namespace {

constexpr int NT = 256;           // threads per workgroup (four independent waves)

enum { kPK = 0, kFull = 1, kRes = 2, kRhs = 3, kCoup = 4, kResF = 5 };

template <typename R>
struct Elem {
  // element outputs (8, index a + 2b + 4c) of K_e x, with every constant folded into four
  // per-element scalars:
  //   AX = s G_xx hy hz / (36 hx),  BY = s G_yy hx hz / (36 hy),
  //   Q4 = s G_xy hz / 24,          CZ = s G_zz hx hy / (36 hz),
  // s = the operator's scale (0 for an element that contributes nothing).
  __host__ __device__ static inline void stiff_f(const R (&x)[8], R AX, R BY, R Q4, R CZ, R (&o)[8]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R u[4];
#pragma unroll
      for (int ab = 0; ab < 4; ++ab) u[ab] = c == 0 ? (R)2 * x[ab] + x[ab + 4] : x[ab] + (R)2 * x[ab + 4];
      const R dx0 = u[1] - u[0], dx1 = u[3] - u[2];
      const R dy0 = u[2] - u[0], dy1 = u[3] - u[1];
      const R qy = Q4 * (dy0 + dy1), qx = Q4 * (dx0 + dx1);
      const R A0 = AX * ((R)2 * dx0 + dx1) + qy, A1 = AX * (dx0 + (R)2 * dx1) + qy;
      const R B0 = BY * ((R)2 * dy0 + dy1) + qx, B1 = BY * (dy0 + (R)2 * dy1) + qx;
      o[4 * c + 0] = -A0 - B0;
      o[4 * c + 1] = A0 - B1;
      o[4 * c + 2] = -A1 + B0;
      o[4 * c + 3] = A1 + B1;
    }
    R dz[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) dz[ab] = CZ * (x[ab + 4] - x[ab]);
    const R r0 = (R)2 * dz[0] + dz[1], r1 = dz[0] + (R)2 * dz[1];
    const R r2 = (R)2 * dz[2] + dz[3], r3 = dz[2] + (R)2 * dz[3];
    const R t0 = (R)2 * r0 + r2, t1 = (R)2 * r1 + r3;
    const R t2 = r0 + (R)2 * r2, t3 = r1 + (R)2 * r3;
    o[0] -= t0; o[1] -= t1; o[2] -= t2; o[3] -= t3;
    o[4] += t0; o[5] += t1; o[6] += t2; o[7] += t3;
  }

  // f M1x (x) M1y (x) M1z x with the factor f = s hx hy hz / 216 applied once
  __host__ __device__ static inline void mass_f(const R (&x)[8], R f, R (&o)[8]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R t[4];
#pragma unroll
      for (int ab = 0; ab < 4; ++ab) t[ab] = f * ((c == 0) ? ((R)2 * x[ab] + x[ab + 4]) : (x[ab] + (R)2 * x[ab + 4]));
      const R r0 = (R)2 * t[0] + t[1], r1 = t[0] + (R)2 * t[1];
      const R r2 = (R)2 * t[2] + t[3], r3 = t[2] + (R)2 * t[3];
      o[4 * c + 0] = (R)2 * r0 + r2;
      o[4 * c + 1] = (R)2 * r1 + r3;
      o[4 * c + 2] = r0 + (R)2 * r2;
      o[4 * c + 3] = r1 + (R)2 * r3;
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
  const void* coef;   // CF = 0: [B][P][2] pairs (p, q), coefficient precision; else the field [B][P]
  double cfa;         // CF > 0: (s_l - s_t)/2 for the fibre angle, the floor for the isotropic field
  T* y;               // kPK: w; kFull: y
  const double* u;   // kRes / kRhs input (FP64); kResF: the Newton iterate (start 0)
  const double* ukp;  // kResF: u_k, the state at the start of the step
  const double* bvec; // kRes: b
  double* bout;       // kRhs: b
  double* ucopy;      // kRhs: u := u_k (or 2 u_k - u_{k-1} with extrap)
  const double* fbox; // kRhs
  // kRhs, previous time level (may be NULL): u_{k-1} for the extrapolated Newton start and for
  // the activation times of the step from t_{k-1} to t_k, which the kernel records in act
  const double* uprev;
  double* act;
  double u_th, t_prev, dt_act;
  int extrap;
  double load;
  void* r0;           // kRes: -F (inner precision)
  void* dout;         // kRes: dt I'(u) (inner precision)
  double* part;       // kRes: partial norms
  double ck, cm;
  const int32_t* active;
  // kRhs in a time block (g.group > 1): the load of time level q is dt/2 (rate(t_(k0+q)) +
  // rate(t_(k0+q-1))), rate = amp on [t_on, t_off)
  int k0;
  double t_on, t_off, amp, dt_load;
  int tiles_x, tiles_y, zchunks;
  int bps;            // workgroups per sample
  // kPK with fused projections: partials of w . v_i (i <= j) per wave
  const T* V;         // basis vectors v_0.., stride vs
  size_t vs;
  double* dpart;      // [B][kmax + 1][npart]
  int npart;          // partials per sample (= waves per sample)
};

}  // namespace

// Owned node (X, Y) = lane (X, Y) sums, in this order, vertex (1,1) of its own
// element, (0,1) of lane + 1, (1,0) of lane + LX and (0,0) of lane + LX + 1.
// Lane layouts of a wave: LX lanes along x times 64 / LX along y.  With 16 lanes along x
// every load of a plane reads rows of 16 consecutive nodes (one 128-byte line in FP64)
// instead of 8; it owns 15 x 3 nodes instead of 7 x 7 and wastes more of a small grid
// on partial tiles, so by default grids narrower than kWideMinNx nodes use the 8 x 8
// layout.  A level may fix the layout instead (g.lx, set by timing both).
constexpr int kWideMinNx = 48;
inline int wave_lx(const Geo& g) { return g.lx != 0 ? g.lx : (g.nx >= kWideMinNx ? 16 : 8); }
constexpr int WZ = 11;  // owned node planes per wave (WZ + 1 steps)

// steps between issuing a slab's loads and using them
template <typename R, int MODE>
constexpr int wave_prefetch() {
#ifdef MLQ_WAVE_PD
  return MLQ_WAVE_PD;
#else
  // the fused residual carries two FP64 values per corner and four per owned node: one slab
  // ahead keeps it at three waves per SIMD
  return MODE == kResF ? 1 : 2;
#endif
}

template <typename R>
__device__ inline R shdn(R v, int d) {
  return __shfl_down(v, d, 64);
}

// Element coefficients (CF): 0 = the pairs (p, q) read from memory; 1 = formed from the fibre
// angle theta of the element, p, q = cfa (cos 2t, sin 2t) with the library's accurate FP32 sincos
// (the same values the pair kernel k_coefs stores); 2 = the same with the hardware sine and cosine
// (an approximation good to about 1e-6, used where only the Krylov operator needs it); 3 = the
// isotropic field v, p = max(v, cfa), q = 0.  CF > 0 reads 4 bytes per element instead of 8.
// At least three waves per SIMD: the FP64 residual variants sit just above the register budget of
// three (168 VGPRs) and would otherwise drop to two; the other variants use far fewer registers.
template <typename R, typename TC, typename TI, int MODE, int JB, int LX, int CF>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_wave3(Args<R> A) {
  constexpr int LY = 64 / LX;
  constexpr int WTX = LX - 1, WTY = LY - 1;  // owned nodes per wave along x and y
  const Geo& g = A.g;
  // dt I_ion(u) = dt alpha (u - u_rest)(u - u_th)(u - u_peak) as a cubic in u, evaluated by Horner's
  // rule at every corner of the fused residual (fewer FP64 operations than the product form)
  const double ida = A.io.dt * A.io.alpha, ir = A.io.u_rest, it_ = A.io.u_th, ip = A.io.u_peak;
  const double ic3 = ida, ic2 = -ida * (ir + it_ + ip), ic1 = ida * (ir * it_ + ir * ip + it_ * ip),
               ic0 = -ida * ir * it_ * ip;
  // its derivative dt I_ion'(u) = (3 ic3 u + 2 ic2) u + ic1
  const double dc2 = 3.0 * ic3, dc1 = 2.0 * ic2;
  // Workgroups go to the 8 XCDs round-robin (linear id mod 8).  Renumber them so
  // that each XCD owns one contiguous range of (sample, tile) blocks: tiles that
  // share cache lines (x/y halos, the plane above a z-chunk) then meet in one L2.
  const int L = blockIdx.x, NB = gridDim.x;
  const int q = NB >> 3, r = NB & 7, xcd = L & 7;
  const int W = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + (L >> 3);
  const int sb = W / A.bps, blk = W - sb * A.bps;
  // time blocks: sb is a virtual sample (one time level); sr the sample it belongs to, whose
  // coefficients, flags and Krylov scalars it uses; slot 0 of a block holds its initial state
  const int grp = g.group > 1 ? g.group : 1;
  const int sr = sb / grp, slot = sb - sr * grp;
  const bool sample_on = (grp == 1 || slot != 0) && (A.active == nullptr || A.active[sr] != 0);
  constexpr bool kMass = MODE != kPK;
  __shared__ double red[NT / 64][3];
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave: keep it (and everything derived
  // from it: tile, z-chunk, plane offsets) in scalar registers
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gw = blk * (NT / 64) + wid;
  const int nwaves = A.tiles_x * A.tiles_y * A.zchunks;
  const bool wave_on = sample_on && gw < nwaves;
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  double dacc[JB > 0 ? JB : 1];
#pragma unroll
  for (int i = 0; i < (JB > 0 ? JB : 1); ++i) dacc[i] = 0.0;
  R wk[JB > 0 ? WZ : 1];  // w at the owned node of each plane of the wave (0 where not owned)
#pragma unroll
  for (int t = 0; t < (JB > 0 ? WZ : 1); ++t) wk[t] = 0;
  if (wave_on) {
    int t = gw;
    const int tx_i = t % A.tiles_x;
    t /= A.tiles_x;
    const int ty_i = t % A.tiles_y;
    const int zc = t / A.tiles_y;
    const int i = lane % LX, j = lane / LX;
    const int ex = tx_i * WTX - 1 + i, ey = ty_i * WTY - 1 + j;  // this lane's element (= its node (0,0))
    const int zs = zc * WZ, ze = min(zs + WZ, g.nz);
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int64_t sbase = (int64_t)sb * g.nn;
    constexpr int kCw = CF == 0 ? 2 : 1;  // stored values per element
    const TC* cf = (const TC*)A.coef + (int64_t)sr * g.P * kCw;
    const int ex_n = g.nx - 1, ey_n = g.ny - 1;
    const bool elem_xy = ex >= 0 && ey >= 0 && ex < ex_n && ey < ey_n;
    const bool owner = i < WTX && j < WTY && ex + 1 < g.nx && ey + 1 < g.ny;
    // every load below uses an address clamped into the grid, so no lane branches around
    // a load and the compiler can count outstanding loads exactly; values of clamped
    // addresses only ever feed elements or nodes that are discarded
    const int cx0 = min(max(ex, 0), g.nx - 2), cy0 = min(max(ey, 0), g.ny - 2);
    const int64_t c00 = (int64_t)cy0 * g.nx + cx0;                     // corner (0,0) of the clamped element
    const int ocx = min(ex + 1, g.nx - 1), ocy = min(ey + 1, g.ny - 1);
    const int64_t oof = (int64_t)ocy * g.nx + ocx;                      // owned node (clamped)
    const int64_t ce = (int64_t)cx0 + (int64_t)ex_n * cy0;              // clamped element in its layer
    const int64_t layer = (int64_t)ex_n * ey_n;
    // lumped-mass weight of the owned node without its z factor (stopping-test scale)
    const double wxy = g.Hx * g.Hy * g.Hz * ((ex + 1 == 0 || ex + 1 == g.nx - 1) ? 0.5 : 1.0) *
                       ((ey + 1 == 0 || ey + 1 == g.ny - 1) ? 0.5 : 1.0);

    // Loads and stores address a wave-uniform base (sample, plane) plus a 32-bit
    // per-lane byte offset that stays fixed while the wave marches up in z.
    const uint32_t lb = (uint32_t)c00 * (uint32_t)sizeof(R);     // corner (0,0), node arrays of type R
    const uint32_t lbd = (uint32_t)c00 * 8u;                      // same, FP64 node arrays
    const uint32_t ob = (uint32_t)oof * (uint32_t)sizeof(R);     // owned node, type R
    const uint32_t obd = (uint32_t)oof * 8u;                      // owned node, FP64
    const uint32_t eb = (uint32_t)ce * (uint32_t)(kCw * sizeof(TC)); // element (p, q) or field value
    auto at = [](auto* base, uint32_t byte_off) { return *(decltype(base))((const char*)base + byte_off); };
    const int nxs = g.nx;

    // Per-sample base pointers (64-bit, uniform) are formed once; a plane is then a
    // 32-bit byte offset (kk * plane fits in 32 bits for every mesh the library accepts).
    const uint32_t pbR = (uint32_t)plane * (uint32_t)sizeof(R), pbD = (uint32_t)plane * 8u;
    const uint32_t lbR = (uint32_t)layer * (uint32_t)(kCw * sizeof(TC));
    const R* xs = nullptr;
    const R* ds_ = nullptr;
    const double* us = nullptr;
    const double* uks = nullptr;
    const double* ups = nullptr;
    if constexpr (MODE == kPK || MODE == kFull || MODE == kCoup) xs = A.x + sbase;
    if constexpr (MODE == kFull) ds_ = A.d + sbase;
    if constexpr (MODE == kRes || MODE == kRhs) us = A.u + sbase;
    // kResF: the JB parameter carries the start kind (0: w.u, 1: u_k, 2: 2 u_k - u_(k-1)) so that
    // every load of the march is issued without a branch; absent optional inputs read u_k instead
    // (cache hits), their values unused
    constexpr int kStart = MODE == kResF ? JB : 0;
    const double* fbs = nullptr;
    if constexpr (MODE == kResF) {
      uks = A.ukp + sbase;
      us = kStart == 0 ? A.u + sbase : uks;
      ups = A.uprev != nullptr ? A.uprev + sbase : uks;
      fbs = A.load != 0.0 ? A.fbox : uks;
    }
    auto in_val = [&](uint32_t po, int dn, R& vk, R& vm) {
      if constexpr (MODE == kPK || MODE == kCoup) {
        vk = (R)at(xs + dn, lb + po);
      } else if constexpr (MODE == kFull) {
        const R v = (R)at(xs + dn, lb + po);
        vk = v;
        vm = v + (R)at(ds_ + dn, lb + po) * v;
      } else if constexpr (MODE == kResF) {
        // from the iterate u and u_k: the stiffness input u + u_k and the mass input
        // (u - u_k) + dt I_ion(u)
        const double a = at(uks + dn, lbd + po);
        double u = a;
        if constexpr (kStart == 0) u = at(us + dn, lbd + po);
        if constexpr (kStart == 2) u = 2.0 * a - at(ups + dn, lbd + po);
        vk = (R)(u + a);
        vm = (R)((u - a) + ((ic3 * u + ic2) * u + ic1) * u + ic0);
      } else {
        // kRes / kRhs: the mass input (u + dt I_ion(u), or u) is formed in step() from vk, so
        // that the register ring of planes holds one value per corner
        vk = (R)at(us + dn, lbd + po);
      }
    };
    struct Pl {
      R k[4], m[4];
    };
    auto fetch = [&](int k, Pl& r) {
      const uint32_t kk = (uint32_t)min(max(k, 0), g.nz - 1);
      const uint32_t po = kk * ((MODE == kRes || MODE == kRhs || MODE == kResF) ? pbD : pbR);
      in_val(po, 0, r.k[0], r.m[0]);
      in_val(po, 1, r.k[1], r.m[1]);
      in_val(po, nxs, r.k[2], r.m[2]);
      in_val(po, nxs + 1, r.k[3], r.m[3]);
    };
    auto fetch_coef = [&](int k, R& p, R& q) {
      const uint32_t kk = (uint32_t)min(max(k, 0), g.nz - 2);
      p = (R)at(cf, eb + kk * lbR);  // CF > 0: the field value, converted in step()
      q = CF == 0 ? (R)at(cf + 1, eb + kk * lbR) : (R)0;
    };
    const float cfa32 = (float)A.cfa;

    const R* vjs = nullptr;
    const double* bs = nullptr;
    if constexpr (MODE == kPK) vjs = A.vj + sbase;
    if constexpr (MODE == kRes) bs = A.bvec + sbase;
    auto fetch_pre = [&](int k, R& p0, R& p1, R& p2, R& p3) {
      const uint32_t kc = (uint32_t)min(max(k, 0), g.nz - 1);
      p0 = 0;
      p1 = 0;
      p2 = 0;
      p3 = 0;
      if constexpr (MODE == kResF) {
        // at the owned node: the iterate, u_k, u_(k-1) (activation) and the stimulus load
        const double a = at(uks, obd + kc * pbD);
        const double um = at(ups, obd + kc * pbD);
        double u = a;
        if constexpr (kStart == 0) u = at(us, obd + kc * pbD);
        if constexpr (kStart == 2) u = 2.0 * a - um;
        p0 = (R)u;
        p1 = (R)a;
        p2 = (R)um;
        p3 = (R)at(fbs, obd + kc * pbD);
      }
      if constexpr (MODE == kPK) p0 = at(vjs, ob + kc * pbR);
      if constexpr (MODE == kRes) {
        p0 = (R)at(bs, obd + kc * pbD);
        p1 = (R)at(us, obd + kc * pbD);
      }
      if constexpr (MODE == kRhs) {
        p0 = (R)at(A.fbox, obd + kc * pbD);
        p1 = (R)at(us, obd + kc * pbD);
      }
    };
    // folded constants of the element operators (uniform)
    const R KX = (R)(g.Hy / (6.0 * g.Hx) * g.Hz / 6.0), KY = (R)(g.Hx / (6.0 * g.Hy) * g.Hz / 6.0);
    const R KQ = (R)(0.25 * g.Hz / 6.0), KZ = (R)(g.Hx * g.Hy / (36.0 * g.Hz));
    const R KM = (R)(g.Hm / 216.0);
    const R CX0 = (R)g.cx0, CX1 = (R)g.cx1, CY0 = (R)g.cy0, CY1 = (R)g.cy1, CZ0 = (R)g.cz0, CZ1 = (R)g.cz1;
    R sj = 0;
    if constexpr (MODE == kPK) sj = (R)A.inv_eta[(int64_t)sr * (A.kmax + 1) + A.j];
    double load = A.load;
    if constexpr (MODE == kRhs) {
      if (grp > 1) {
        const double ta = (double)(A.k0 + slot - 1) * A.dt_load, tb = (double)(A.k0 + slot) * A.dt_load;
        const double ra = (A.t_on <= ta && ta < A.t_off) ? A.amp : 0.0;
        const double rb = (A.t_on <= tb && tb < A.t_off) ? A.amp : 0.0;
        load = 0.5 * A.dt_load * (rb + ra);
      }
    }

    // one slab: planes lo (k) and hi (k + 1), its coefficients and the node inputs of
    // plane k are resident (loaded PD steps earlier)
    R acc_top = 0;
    // kResF: the mass term is applied per plane (its z part x_(k-1) + 4 x_k + x_(k+1) formed once per
    // node and plane, then the element's x-y mass over it), not per slab; fm masks elements outside
    // the grid in x-y
    const R fm = elem_xy ? (R)A.cm * KM : (R)0;
    auto step = [&](int k, const Pl& pv, const Pl& lo, const Pl& hi, R cp, R cq, R p0, R p1, R p2, R p3) {
      const bool slab = k >= 0 && k <= g.nz - 2;
      if constexpr (CF == 1 || CF == 2) {
        const float t2 = 2.0f * (float)cp;
        float sv, cv;
        if constexpr (CF == 1)
          sincosf(t2, &sv, &cv);
        else
          __sincosf(t2, &sv, &cv);
        cp = (R)(cfa32 * cv);
        cq = (R)(cfa32 * sv);
      } else if constexpr (CF == 3) {
        const double v = (double)cp;
        cp = (R)(TC)(v > A.cfa ? v : A.cfa);
        cq = (R)0;
      }
      R o[8];
      {
        const bool on = slab && elem_xy;
        const R sc = on ? (R)A.ck : (R)0;
        R xin[8] = {lo.k[0], lo.k[1], lo.k[2], lo.k[3], hi.k[0], hi.k[1], hi.k[2], hi.k[3]};
        Elem<R>::stiff_f(xin, (CX0 + CX1 * cp) * (sc * KX), (CY0 + CY1 * cp) * (sc * KY), cq * (sc * KQ),
                         (CZ0 + CZ1 * cp) * (sc * KZ), o);
        if constexpr (MODE == kResF) {
          const R za = k > 0 ? (R)1 : (R)0, zc = k < g.nz - 1 ? (R)1 : (R)0, zb = (R)2 * (za + zc);
          R T[4];
#pragma unroll
          for (int ab = 0; ab < 4; ++ab) T[ab] = za * pv.m[ab] + zb * lo.m[ab] + zc * hi.m[ab];
          const R r0 = (R)2 * T[0] + T[1], r1 = T[0] + (R)2 * T[1];
          const R r2 = (R)2 * T[2] + T[3], r3 = T[2] + (R)2 * T[3];
          o[0] += fm * ((R)2 * r0 + r2);
          o[1] += fm * ((R)2 * r1 + r3);
          o[2] += fm * (r0 + (R)2 * r2);
          o[3] += fm * (r1 + (R)2 * r3);
        } else if constexpr (kMass) {
          R xm[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if constexpr (MODE == kRes) {
              const double v = (double)xin[c];
              xm[c] = (R)(v + A.io.dt * iion3(v, A.io));
            } else if constexpr (MODE == kRhs || MODE == kCoup) {
              xm[c] = xin[c];
            } else {
              xm[c] = c < 4 ? lo.m[c] : hi.m[c - 4];
            }
          }
          R om[8];
          Elem<R>::mass_f(xm, on ? (R)A.cm * KM : (R)0, om);
#pragma unroll
          for (int c = 0; c < 8; ++c) o[c] += om[c];
        }
      }
      // assemble the owned node: bottom faces of slab k (plane k), top faces (plane k + 1)
      const R bot = o[3] + shdn(o[2], 1) + shdn(o[1], LX) + shdn(o[0], LX + 1);
      const R top = o[7] + shdn(o[6], 1) + shdn(o[5], LX) + shdn(o[4], LX + 1);
      if (owner && k >= zs && k < ze) {
        const uint32_t kk = (uint32_t)k;
        const R sres = acc_top + bot;
        auto put = [&](auto* base, uint32_t byte_off, auto v) {
          *(decltype(base))((char*)base + byte_off) = v;
        };
        if constexpr (MODE == kPK) {
          const R wv = p0 * sj + sres;
          put(A.y + sbase, ob + kk * pbR, wv);
          if constexpr (JB > 0) {
            // w . v_j at once (p0 is v_j here); w is kept for the projections on v_0 ..
            // v_{j-1} after the march (the march is unrolled, so k - zs is a
            // compile-time index)
            dacc[0] += (double)wv * (double)p0;
            const int q = k - zs;
#pragma unroll
            for (int t = 0; t < WZ; ++t)
              if (t == q) wk[t] = wv;
          }
        } else if constexpr (MODE == kFull) {
          put(A.y + sbase, ob + kk * pbR, sres);
        } else if constexpr (MODE == kCoup) {
          put(A.y + sbase, ob + kk * pbR, at(A.y + sbase, ob + kk * pbR) + sres);
        } else if constexpr (MODE == kResF) {
          // F = M ((u - u_k) + dt I_ion(u)) + dt/2 K (u + u_k) - load F_box, the step equation's
          // residual G(u) - b without forming G(u) and b; the stopping test's scale is the
          // lumped mass of the two states, |w u| + |w u_k + load F_box| (w the node weight)
          const double uo = (double)p0, uko = (double)p1, fb = load * (double)p3;
          const double F = (double)sres - fb;
          const uint32_t oi = (uint32_t)oof * (uint32_t)sizeof(TI) + kk * (uint32_t)plane * (uint32_t)sizeof(TI);
          put((TI*)A.r0 + sbase, oi, (TI)(-F));
          put((TI*)A.dout + sbase, oi, (TI)((dc2 * uo + dc1) * uo + ic1));
          if constexpr (kStart != 0) put(A.ucopy + sbase, obd + kk * pbD, uo);
          if (A.uprev != nullptr) {  // activation in the step from t_(k-1) to t_k
            const double um = (double)p2;
            double* ap = (double*)((char*)(A.act + sbase) + obd + kk * pbD);
            if (um < A.u_th && uko >= A.u_th && *ap < 0.0)  // read only where u crosses the threshold
              *ap = A.t_prev + A.dt_act * (A.u_th - um) / (uko - um);
          }
          const double wl = (k == 0 || k == g.nz - 1) ? 0.5 * wxy : wxy;
          const double su = wl * uo, sk = wl * uko + fb;
          n0 += F * F;
          n1 += su * su;
          n2 += sk * sk;
        } else if constexpr (MODE == kRes) {
          const double G = (double)sres;
          const double bb = (double)p0;
          const double F = G - bb;
          const uint32_t oi = (uint32_t)oof * (uint32_t)sizeof(TI) + kk * (uint32_t)plane * (uint32_t)sizeof(TI);
          put((TI*)A.r0 + sbase, oi, (TI)(-F));
          put((TI*)A.dout + sbase, oi, (TI)(A.io.dt * diion3((double)p1, A.io)));
          n0 += F * F;
          n1 += G * G;
          n2 += bb * bb;
        } else {
          put(A.bout + sbase, obd + kk * pbD, (double)sres + load * (double)p0);
          const double uk = (double)p1;
          double ustart = uk;
          if (A.uprev != nullptr) {
            const double um = at(A.uprev + sbase, obd + kk * pbD);
            if (A.extrap) ustart = 2.0 * uk - um;
            double* ap = (double*)((char*)(A.act + sbase) + obd + kk * pbD);
            if (um < A.u_th && uk >= A.u_th && *ap < 0.0) *ap = A.t_prev + A.dt_act * (A.u_th - um) / (uk - um);
          }
          if (A.ucopy != nullptr) put(A.ucopy + sbase, obd + kk * pbD, ustart);
        }
      }
      acc_top = top;
    };

    // The march over slabs zs - 1 .. zs + WZ - 1 is unrolled, so every array below is
    // indexed by compile-time constants and lives in registers.  Step s consumes planes
    // s and s + 1, the coefficients and node inputs of s; the loads for step s + PD are
    // issued at step s.
    constexpr int NS = WZ + 1;
    constexpr int PD = wave_prefetch<R, MODE>();
    const int k0 = zs - 1;
    Pl P[NS + 1];
    R Cp[NS], Cq[NS], Q0[NS], Q1[NS], Q2[NS], Q3[NS];
#pragma unroll
    for (int t = 0; t <= PD; ++t) fetch(k0 + t, P[t]);
#pragma unroll
    for (int t = 0; t < PD; ++t) {
      fetch_coef(k0 + t, Cp[t], Cq[t]);
      fetch_pre(k0 + t, Q0[t], Q1[t], Q2[t], Q3[t]);
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (t + PD + 1 <= NS) fetch(k0 + t + PD + 1, P[t + PD + 1]);
      if (t + PD < NS) {
        fetch_coef(k0 + t + PD, Cp[t + PD], Cq[t + PD]);
        fetch_pre(k0 + t + PD, Q0[t + PD], Q1[t + PD], Q2[t + PD], Q3[t + PD]);
      }
      step(k0 + t, P[t > 0 ? t - 1 : 0], P[t], P[t + 1], Cp[t], Cq[t], Q0[t], Q1[t], Q2[t], Q3[t]);
    }
    if constexpr (MODE == kPK && JB > 0) {
      // projections w . v_i (i < j) over the wave's owned nodes, into dacc[i + 1]: all
      // loads of one basis vector are issued together (addresses clamped into the grid;
      // wk is 0 wherever the node is not owned)
      if (owner) {
#pragma unroll
        for (int i = 0; i + 1 < JB; ++i) {
          if (i >= A.j) break;
          R v[WZ];
#pragma unroll
          for (int t = 0; t < WZ; ++t) {
            const uint32_t kk = (uint32_t)min(zs + t, g.nz - 1);
            v[t] = at(A.V + i * A.vs + sbase, ob + kk * pbR);
          }
#pragma unroll
          for (int t = 0; t < WZ; ++t) dacc[i + 1] += (double)wk[t] * (double)v[t];
        }
      }
    }
  }
  if constexpr (MODE == kPK && JB > 0) {
    // one partial per workgroup: waves summed in a fixed order
    __shared__ double redp[NT / 64][JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) {
      double v = dacc[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) redp[wid][i] = v;
    }
    __syncthreads();
    // redp[.][0] holds w . v_j, redp[.][i + 1] holds w . v_i
    if ((int)threadIdx.x < JB && (int)threadIdx.x <= A.j) {
      const int i = threadIdx.x;
      const int src = i == A.j ? 0 : i + 1;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) v += redp[q][src];
      A.dpart[((int64_t)sb * (A.kmax + 1) + i) * A.npart + blk] = v;
    }
  }
  if constexpr (MODE == kRes || MODE == kResF) {
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
      double* p = A.part + ((int64_t)sb * A.bps + blk) * 3;
      p[0] = s0;
      p[1] = s1;
      p[2] = s2;
    }
  }
}

namespace {

template <typename R>
void wave_grid_of(const Geo& g, Args<R>& a, int32_t B, dim3& grid) {
  const int lx = wave_lx(g);
  a.tiles_x = (int)cdiv(g.nx, lx - 1);
  a.tiles_y = (int)cdiv(g.ny, 64 / lx - 1);
  a.zchunks = (int)cdiv(g.nz, WZ);
  a.bps = (int)cdiv((int64_t)a.tiles_x * a.tiles_y * a.zchunks, NT / 64);
  a.npart = a.bps;
  grid = dim3((unsigned)((int64_t)a.bps * B));
}

template <typename R, typename TC, typename TI, int MODE, int JB, int CF>
void launch_wave3_cf(const Geo& g, Args<R>& a, int32_t B, hipStream_t s) {
  dim3 grid;
  wave_grid_of(g, a, B, grid);
  if (wave_lx(g) == 16)
    hipLaunchKernelGGL((k_wave3<R, TC, TI, MODE, JB, 16, CF>), grid, dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_wave3<R, TC, TI, MODE, JB, 8, CF>), grid, dim3(NT), 0, s, a);
}

// FP64 (TC = double), and the FP64-arithmetic residual and right-hand side of mixed precision:
// the pairs (p, q) of k_coefs (their FP64 stencils are bound by latency and registers, where the
// accurate sine and cosine per element cost more than the 4 bytes they save).  Mixed precision
// (TC = float) otherwise reads the field itself: the Krylov apply (kPK) with the hardware sine
// and cosine, the public apply with the accurate ones (the values k_coefs stores).
template <typename R, typename TC, typename TI, int MODE, int JB = 0>
void launch_wave3(const Geo& g, Args<R>& a, int32_t B, hipStream_t s) {
  if constexpr (sizeof(TC) == 8 || MODE == kRes || MODE == kRhs || MODE == kResF) {
    launch_wave3_cf<R, TC, TI, MODE, JB, 0>(g, a, B, s);
  } else {
    a.cfa = g.cfa;
    if (g.iso)
      launch_wave3_cf<R, TC, TI, MODE, JB, 3>(g, a, B, s);
    else if (MODE == kPK)
      launch_wave3_cf<R, TC, TI, MODE, JB, 2>(g, a, B, s);
    else
      launch_wave3_cf<R, TC, TI, MODE, JB, 1>(g, a, B, s);
  }
}

}  // namespace

int32_t stencil3_blocks(const Geo& g) {
  const int lx = wave_lx(g);
  return (int32_t)cdiv(cdiv(g.nx, lx - 1) * cdiv(g.ny, 64 / lx - 1) * cdiv(g.nz, WZ), NT / 64);
}

void launch_apply_pk3(const Geo& g, const Work& w, int j, double ck, int32_t B, bool mixed, hipStream_t s, int jb) {
  const size_t vs = (size_t)g.nn * B;
  auto fill = [&](auto& a) {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(a.x)>>;
    a.g = g; a.x = (const T*)w.z + j * vs; a.vj = (const T*)w.V + j * vs; a.inv_eta = w.inv_eta;
    a.j = j; a.kmax = w.kmax; a.coef = mixed ? w.theta : w.coef; a.y = (T*)w.w; a.ck = ck; a.cm = 0.0;
    a.active = w.inner_active;
    a.V = (const T*)w.V; a.vs = vs; a.dpart = w.dpart;
  };
  if (mixed) {
    Args<float> a{};
    fill(a);
    if (jb == 0)
      launch_wave3<float, float, float, kPK, 0>(g, a, B, s);
    else if (jb == 1)
      launch_wave3<float, float, float, kPK, 1>(g, a, B, s);
    else if (jb <= 4)
      launch_wave3<float, float, float, kPK, 4>(g, a, B, s);
    else
      launch_wave3<float, float, float, kPK, 8>(g, a, B, s);
  } else {
    Args<double> a{};
    fill(a);
    if (jb == 0)
      launch_wave3<double, double, double, kPK, 0>(g, a, B, s);
    else if (jb == 1)
      launch_wave3<double, double, double, kPK, 1>(g, a, B, s);
    else if (jb <= 4)
      launch_wave3<double, double, double, kPK, 4>(g, a, B, s);
    else
      launch_wave3<double, double, double, kPK, 8>(g, a, B, s);
  }
}

void launch_apply_full3(const Geo& g, const void* coef, const void* x, const void* d, void* y, double ck, int32_t B,
                        bool mixed, hipStream_t s) {
  if (mixed) {
    Args<float> a{};
    a.g = g; a.x = (const float*)x; a.d = (const float*)d; a.coef = coef; a.y = (float*)y; a.ck = ck; a.cm = 1.0;
    launch_wave3<float, float, float, kFull>(g, a, B, s);
  } else {
    Args<double> a{};
    a.g = g; a.x = (const double*)x; a.d = (const double*)d; a.coef = coef; a.y = (double*)y; a.ck = ck; a.cm = 1.0;
    launch_wave3<double, double, double, kFull>(g, a, B, s);
  }
}

void launch_residual3(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s) {
  Args<double> a{};
  a.g = g; a.io = io; a.u = w.u; a.bvec = w.b; a.coef = w.coef; a.r0 = w.V; a.dout = w.d; a.part = w.part;
  a.ck = 0.5 * io.dt; a.cm = 1.0; a.active = w.newton_active;
  if (mixed)
    launch_wave3<double, float, float, kRes>(g, a, B, s);
  else
    launch_wave3<double, double, double, kRes>(g, a, B, s);
}

void launch_residual3f(const Geo& g, const Ionic& io, const Work& w, int32_t B, bool mixed, hipStream_t s, int start,
                       const double* uprev, const double* fbox, double load, double u_th, double t_prev) {
  Args<double> a{};
  a.g = g; a.io = io; a.u = w.u; a.ukp = w.uk; a.ucopy = w.u; a.uprev = uprev; a.act = w.act;
  a.u_th = u_th; a.t_prev = t_prev; a.dt_act = io.dt; a.fbox = fbox; a.load = load;
  a.coef = w.coef; a.r0 = w.V; a.dout = w.d; a.part = w.part; a.ck = 0.5 * io.dt; a.cm = 1.0;
  a.active = w.newton_active;
  // the start kind is the JB parameter of the kernel (compile time)
  auto go = [&](auto st) {
    constexpr int S = decltype(st)::value;
    if (mixed)
      launch_wave3<double, float, float, kResF, S>(g, a, B, s);
    else
      launch_wave3<double, double, double, kResF, S>(g, a, B, s);
  };
  if (start == 0)
    go(std::integral_constant<int, 0>{});
  else if (start == 1)
    go(std::integral_constant<int, 1>{});
  else
    go(std::integral_constant<int, 2>{});
}

void launch_rhs3_block(const Geo& g, const double* U, double* b, const void* coef, const double* fbox, int k0,
                       double dt, double t_on, double t_off, double amp, int32_t Bv, bool mixed, hipStream_t s) {
  Args<double> a{};
  // virtual sample v reads U at v - 1 (slot 0 of a block, its initial state, feeds slot 1)
  a.g = g; a.u = U - g.nn; a.coef = coef; a.bout = b; a.ucopy = nullptr; a.fbox = fbox; a.load = 0.0;
  a.ck = -0.5 * dt; a.cm = 1.0; a.active = nullptr; a.uprev = nullptr;
  a.k0 = k0; a.t_on = t_on; a.t_off = t_off; a.amp = amp; a.dt_load = dt;
  if (mixed)
    launch_wave3_cf<double, float, float, kRhs, 0, 0>(g, a, Bv, s);
  else
    launch_wave3_cf<double, double, double, kRhs, 0, 0>(g, a, Bv, s);
}

void launch_coupling3(const Geo& g, const void* x, void* wv, const void* coef_or_theta, double ck, int32_t Bv,
                      const int32_t* active, bool mixed, hipStream_t s) {
  if (mixed) {
    Args<float> a{};
    a.g = g; a.x = (const float*)x - g.nn; a.coef = coef_or_theta; a.y = (float*)wv; a.ck = ck; a.cm = -1.0;
    a.active = active;
    launch_wave3<float, float, float, kCoup>(g, a, Bv, s);
  } else {
    Args<double> a{};
    a.g = g; a.x = (const double*)x - g.nn; a.coef = coef_or_theta; a.y = (double*)wv; a.ck = ck; a.cm = -1.0;
    a.active = active;
    launch_wave3<double, double, double, kCoup>(g, a, Bv, s);
  }
}

void launch_rhs3(const Geo& g, const Work& w, const double* fbox, double load_coef, double dt, int32_t B, bool mixed,
                 hipStream_t s, const double* uprev, bool extrap, double u_th, double t_prev) {
  Args<double> a{};
  a.g = g; a.u = w.uk; a.coef = w.coef; a.bout = w.b; a.ucopy = w.u; a.fbox = fbox; a.load = load_coef;
  a.ck = -0.5 * dt; a.cm = 1.0; a.active = nullptr;
  a.uprev = uprev; a.act = w.act; a.u_th = u_th; a.t_prev = t_prev; a.dt_act = dt; a.extrap = extrap ? 1 : 0;
  if (mixed)
    launch_wave3<double, float, float, kRhs>(g, a, B, s);
  else
    launch_wave3<double, double, double, kRhs>(g, a, B, s);
}

}  // namespace mlq
