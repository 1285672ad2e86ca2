// Field quantities of interest (Section 2.4) streamed during a solve, and the transfer of
// space-time fields between nested box levels (Section 5, error measures: the tensor product
// of the space and the time interpolation).
//
// All of them are HBM-streaming kernels with no reuse beyond a cache line: one thread per
// output node, consecutive threads on consecutive nodes so that every wave reads whole
// 512-byte segments of each sample's state.
#include "mlq_internal.h"

namespace mlq {

// u_sum[i] += sum_b u[b n + i], samples added in order b = 0 .. B-1.
__global__ __launch_bounds__(kBlock) void k_field_sum(const double* __restrict__ u, int32_t B, int64_t n,
                                                      double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t b = 0; b < B; ++b) acc += u[(int64_t)b * n + i];
  dst[i] += acc;
}

void launch_field_sum(const double* u, int32_t B, int64_t n, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_field_sum, dim3((unsigned)cdiv(n, kBlock)), dim3(kBlock), 0, s, u, B, n, dst);
}

// act_sum[i] += sum_b a_b(i), a never-activated node (a < 0) counted at the stop time.
__global__ __launch_bounds__(kBlock) void k_act_sum(const double* __restrict__ act, int32_t B, int64_t n,
                                                    double t_stop, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t b = 0; b < B; ++b) {
    const double a = act[(int64_t)b * n + i];
    acc += a < 0.0 ? t_stop : a;
  }
  dst[i] += acc;
}

void launch_act_sum(const double* act, int32_t B, int64_t n, double t_stop, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_act_sum, dim3((unsigned)cdiv(n, kBlock)), dim3(kBlock), 0, s, act, B, n, t_stop, dst);
}

// out[(b np + p) ld + k] = sum_j w[p][j] u[b n + node[p][j]]: one thread per (sample, probe).
__global__ __launch_bounds__(kBlock) void k_probe(const double* __restrict__ u, int32_t B, int64_t n, ProbeTab tab,
                                                  int32_t k, int32_t ld, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * tab.n) return;
  const int b = t / tab.n, p = t % tab.n;
  const double* ub = u + (int64_t)b * n;
  double acc = 0.0;
  for (int j = 0; j < kProbeNodes; ++j) acc += tab.w[p * kProbeNodes + j] * ub[tab.node[p * kProbeNodes + j]];
  out[(int64_t)t * ld + k] = acc;
}

void launch_probe(const double* u, int32_t B, int64_t n, const ProbeTab& tab, int32_t k, int32_t ld, double* out,
                  hipStream_t s) {
  const int total = B * tab.n;
  hipLaunchKernelGGL(k_probe, dim3((unsigned)cdiv(total, kBlock)), dim3(kBlock), 0, s, u, B, n, tab, k, ld, out);
}

// sum[p ld + k] += sum_b sum_j w[p][j] u[b n + node[p][j]]: one wave per probe, its lanes over
// the samples, a fixed-order tree over the lanes.
__global__ __launch_bounds__(64) void k_probe_sum(const double* __restrict__ u, int32_t B, int64_t n, ProbeTab tab,
                                                  int32_t k, int32_t ld, double* __restrict__ sum) {
  const int p = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0;
  for (int b = lane; b < B; b += 64) {
    const double* ub = u + (int64_t)b * n;
    double v = 0.0;
    for (int j = 0; j < kProbeNodes; ++j) v += tab.w[p * kProbeNodes + j] * ub[tab.node[p * kProbeNodes + j]];
    acc += v;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) sum[(int64_t)p * ld + k] += acc;
}

void launch_probe_sum(const double* u, int32_t B, int64_t n, const ProbeTab& tab, int32_t k, int32_t ld, double* sum,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_probe_sum, dim3((unsigned)tab.n), dim3(64), 0, s, u, B, n, tab, k, ld, sum);
}

// dst[(r T_t + k') S_t + i'] += alpha * sum over the time and space stencils of src[(r T_f + k) S_f + i].
// Time: coarse node kc = floor(k' m_f / m_t) with weight 1 - th and kc + 1 with th,
// th = ((k' m_f) mod m_t) / m_t.  Space, per axis: coarse index q = floor(i'_a (n_f - 1) / (n_t - 1))
// with weight 1 - x, q + 1 with x, x = ((i'_a (n_f - 1)) mod (n_t - 1)) / (n_t - 1).  A stencil
// point of weight zero is not read (it may lie past the end of the grid).
// Threads in x cover (row, fine node); the space stencil is formed once per thread and reused
// for every output time node, which the y dimension strides over.
__global__ __launch_bounds__(kBlock) void k_transfer(XferGeo g, int64_t rows, double alpha,
                                                     const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t St = g.sn_t[0] * g.sn_t[1] * g.sn_t[2];
  const int64_t Sf = g.sn_f[0] * g.sn_f[1] * g.sn_f[2];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * St) return;
  const int64_t r = t / St;
  int64_t rem = t - r * St;
  const int64_t ip = rem;
  int64_t q[3];
  double x[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t ia = rem % g.sn_t[a];
    rem /= g.sn_t[a];
    if (g.sn_t[a] > 1) {
      const int64_t num = ia * (g.sn_f[a] - 1);
      q[a] = num / (g.sn_t[a] - 1);
      x[a] = (double)(num - q[a] * (g.sn_t[a] - 1)) / (double)(g.sn_t[a] - 1);
    } else {
      q[a] = 0;
      x[a] = 0.0;
    }
  }
  int64_t off[8];
  double ws[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    double w = 1.0;
    int64_t idx = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int o = (c >> a) & 1;
      w *= o ? x[a] : 1.0 - x[a];
      idx += (q[a] + o) * stride;
      stride *= g.sn_f[a];
    }
    off[c] = w == 0.0 ? 0 : idx;  // a zero-weight corner is never read
    ws[c] = w;
  }
  const double* sr = src + r * g.tn_f * Sf;
  double* dr = dst + r * g.tn_t * St + ip;
  for (int64_t kp = blockIdx.y; kp < g.tn_t; kp += gridDim.y) {
    int64_t kc = 0;
    double th = 0.0;
    if (g.tn_t > 1) {
      const int64_t num = kp * g.m_f;
      kc = num / g.m_t;
      th = (double)(num - kc * g.m_t) / (double)g.m_t;
    }
    double acc = 0.0;
    for (int dtm = 0; dtm < 2; ++dtm) {
      const double wt = dtm ? th : 1.0 - th;
      if (wt == 0.0) continue;
      const double* sk = sr + (kc + dtm) * Sf;
      double part = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (ws[c] != 0.0) part += ws[c] * sk[off[c]];
      acc += wt * part;
    }
    dr[kp * St] += alpha * acc;
  }
}

void launch_transfer(const XferGeo& g, int64_t rows, double alpha, const double* src, double* dst, hipStream_t s) {
  const int64_t nx = rows * g.sn_t[0] * g.sn_t[1] * g.sn_t[2];
  if (nx < 1 || g.tn_t < 1) return;
  const unsigned gy = (unsigned)(g.tn_t < 1024 ? g.tn_t : 1024);
  hipLaunchKernelGGL(k_transfer, dim3((unsigned)cdiv(nx, kBlock), gy), dim3(kBlock), 0, s, g, rows, alpha, src, dst);
}

// Transfer with explicit interpolation weights in space (non-nested meshes): target node i'
// takes sum_j w[i' K + j] src[node[i' K + j]] (indices clamped to the source grid), combined
// with the linear time interpolation of k_transfer.  One thread per (row, target node), the
// y dimension strides over the output time nodes.
__global__ __launch_bounds__(kBlock) void k_transfer_weighted(XferGeo g, int64_t rows, int64_t n_from, int64_t n_to,
                                                              int K, const int64_t* __restrict__ node,
                                                              const double* __restrict__ w, double alpha,
                                                              const double* __restrict__ src,
                                                              double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * n_to) return;
  const int64_t r = t / n_to;
  const int64_t ip = t - r * n_to;
  int64_t nd[kProbeNodes];
  double wt[kProbeNodes];
#pragma unroll
  for (int jj = 0; jj < kProbeNodes; ++jj) {
    if (jj < K) {
      const int64_t v = node[ip * K + jj];
      nd[jj] = v < 0 ? 0 : (v >= n_from ? n_from - 1 : v);
      wt[jj] = w[ip * K + jj];
    } else {
      nd[jj] = 0;
      wt[jj] = 0.0;
    }
  }
  const double* sr = src + r * g.tn_f * n_from;
  double* dr = dst + r * g.tn_t * n_to + ip;
  for (int64_t kp = blockIdx.y; kp < g.tn_t; kp += gridDim.y) {
    int64_t kc = 0;
    double th = 0.0;
    if (g.tn_t > 1) {
      const int64_t num = kp * g.m_f;
      kc = num / g.m_t;
      th = (double)(num - kc * g.m_t) / (double)g.m_t;
    }
    double acc = 0.0;
    for (int dtm = 0; dtm < 2; ++dtm) {
      const double wtt = dtm ? th : 1.0 - th;
      if (wtt == 0.0) continue;
      const double* sk = sr + (kc + dtm) * n_from;
      double part = 0.0;
#pragma unroll
      for (int jj = 0; jj < kProbeNodes; ++jj)
        if (wt[jj] != 0.0) part += wt[jj] * sk[nd[jj]];
      acc += wtt * part;
    }
    dr[kp * n_to] += alpha * acc;
  }
}

void launch_transfer_weighted(const XferGeo& g, int64_t rows, int64_t n_from, int64_t n_to, int K,
                              const int64_t* node, const double* w, double alpha, const double* src, double* dst,
                              hipStream_t s) {
  const int64_t nx = rows * n_to;
  if (nx < 1 || g.tn_t < 1) return;
  const unsigned gy = (unsigned)(g.tn_t < 1024 ? g.tn_t : 1024);
  hipLaunchKernelGGL(k_transfer_weighted, dim3((unsigned)cdiv(nx, kBlock), gy), dim3(kBlock), 0, s, g, rows, n_from,
                     n_to, K, node, w, alpha, src, dst);
}

// Squared norm in L^2((0, T); H^q(D)) of the space-time interpolant of one row of a field
// ((m + 1) x n nodal values on a Q1 box), integrated exactly: over element e and interval k,
// dt/3 (a'A_e a + a'A_e b + b'A_e b) with a, b the element's corner values at t_k, t_(k+1) and
// A_e the element mass (plus the Laplacian stiffness for q = 1), both Kronecker products of the
// 1D matrices h/6 [2 1; 1 2] and 1/h [1 -1; -1 1].  Threads stride over (element, interval);
// per-block partials part[r * gridDim.x + block] are summed in order by k_norm_final.
__global__ __launch_bounds__(kBlock) void k_st_norm(NormGeo g, const double* __restrict__ f,
                                                    double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  const int64_t r = blockIdx.y;
  const int64_t ex = g.n[0] - 1, ey = g.dim > 1 ? g.n[1] - 1 : 1, ez = g.dim > 2 ? g.n[2] - 1 : 1;
  const int64_t ne = ex * ey * ez;
  const int64_t nn = g.n[0] * (g.dim > 1 ? g.n[1] : 1) * (g.dim > 2 ? g.n[2] : 1);
  const int64_t total = ne * g.m;
  const int nc = 1 << g.dim;
  const double* fr = f + r * (g.m + 1) * nn;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / ne;
    int64_t e = t - k * ne;
    const int64_t ix = e % ex;
    e /= ex;
    const int64_t iy = e % ey;
    const int64_t iz = e / ey;
    const int64_t base = ix + g.n[0] * (iy + (g.dim > 1 ? g.n[1] : 1) * iz);
    double a[8], b[8];
    for (int c = 0; c < 8; ++c) {
      if (c >= nc) {
        a[c] = b[c] = 0.0;
        continue;
      }
      const int64_t off = (c & 1) + ((c >> 1) & 1) * g.n[0] + ((c >> 2) & 1) * g.n[0] * g.n[1];
      a[c] = fr[k * nn + base + off];
      b[c] = fr[(k + 1) * nn + base + off];
    }
    double qf = 0.0;
    for (int c = 0; c < nc; ++c) {
      for (int cp = 0; cp < nc; ++cp) {
        double mass = 1.0, stiff = 0.0;
        for (int ax = 0; ax < g.dim; ++ax) {
          const bool same = ((c >> ax) & 1) == ((cp >> ax) & 1);
          const double m1 = g.h[ax] * (same ? 2.0 : 1.0) / 6.0;
          const double s1 = (same ? 1.0 : -1.0) / g.h[ax];
          stiff = stiff * m1 + mass * s1;
          mass *= m1;
        }
        const double A = g.q ? mass + stiff : mass;
        qf += A * (a[c] * a[cp] + a[c] * b[cp] + b[c] * b[cp]);
      }
    }
    acc += g.dt / 3.0 * qf;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) s += sh[i];
    part[r * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_norm_final(const double* __restrict__ part, int nb, int64_t rows, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += part[r * nb + i];
  out[r] = s;
}

void launch_st_norm(const NormGeo& g, int64_t rows, const double* f, double* part, double* out, hipStream_t s) {
  int64_t ne = 1;
  for (int a = 0; a < g.dim; ++a) ne *= g.n[a] - 1;
  int64_t nb = cdiv(ne * g.m, kBlock);
  nb = nb < 1 ? 1 : (nb > kNormBlocks ? kNormBlocks : nb);
  hipLaunchKernelGGL(k_st_norm, dim3((unsigned)nb, (unsigned)rows), dim3(kBlock), 0, s, g, f, part);
  hipLaunchKernelGGL(k_norm_final, dim3((unsigned)cdiv(rows, kBlock)), dim3(kBlock), 0, s, part, (int)nb, rows, out);
}

// Squared H^q(0, T) norm of the linear interpolant of each row of (m + 1) values: one thread
// per row, sum_k dt/3 (a^2 + a b + b^2) (+ (b - a)^2 / dt for q = 1) in order k.
__global__ void k_time_norm(const double* __restrict__ f, int64_t rows, int64_t m, double dt, int q,
                            double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double* fr = f + r * (m + 1);
  double s = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    const double a = fr[k], b = fr[k + 1];
    s += dt / 3.0 * (a * a + a * b + b * b);
    if (q) s += (b - a) * (b - a) / dt;
  }
  out[r] = s;
}

void launch_time_norm(const double* f, int64_t rows, int64_t m, double dt, int q, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_time_norm, dim3((unsigned)cdiv(rows, kBlock)), dim3(kBlock), 0, s, f, rows, m, dt, q, out);
}

}  // namespace mlq
