// Discrete Karhunen-Loeve basis of the random field (fibre angle, or scalar
// conductivity; Section 2.3) on the nodes of a uniform Q1 box or a tetrahedral mesh,
// and its element-midpoint transfer to the element centres of a level (Section 4).
//
//   eq. (algEig)    M C M v = lambda M v,     C_ij = s^2 exp(-|x_i - x_j|_2 / l)
//                   (or s^2 exp(-|x_i - x_j|_2^2 / l), the squared-exponential kernel)
//   C ~ L L^T       pivoted Cholesky (largest remaining diagonal, lowest index on
//                   ties; columns of C evaluated on the fly on the GPU)
//   eq. (redEig)    L^T M L v~ = lambda v~ (R x R, cyclic Jacobi on the host)
//   v = L v~        v_i^T M v_j = lambda_i delta_ij;  psi = v / sqrt(lambda)
//
// Sign of each mode: its first entry of largest magnitude is positive (entries
// within a relative 1e-9 of the maximum count as ties).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mlq_internal.h"

namespace mlq {

namespace {

constexpr int kT = 256;

struct Box {
  int32_t dim;
  int64_t n[3];
  double lo[3], h[3];
  int64_t nn;
  const double* xyz;  // tetrahedral KL mesh: vertex coordinates (device), else nullptr
};

__host__ __device__ inline void box_xyz(const Box& b, int64_t i, double x[3]) {
  if (b.xyz != nullptr) {
    x[0] = b.xyz[3 * i];
    x[1] = b.xyz[3 * i + 1];
    x[2] = b.xyz[3 * i + 2];
    return;
  }
  const int64_t ix = i % b.n[0];
  const int64_t r = i / b.n[0];
  const int64_t iy = r % b.n[1];
  const int64_t iz = r / b.n[1];
  x[0] = b.lo[0] + b.h[0] * (double)ix;
  x[1] = b.lo[1] + b.h[1] * (double)iy;
  x[2] = b.dim == 3 ? b.lo[2] + b.h[2] * (double)iz : 0.0;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Block-level (max value, lowest index) and sum of d; partials per block.
__global__ __launch_bounds__(kT) void k_argmax_sum(const double* __restrict__ d, int64_t n, int use_abs,
                                                   double* __restrict__ pv, int64_t* __restrict__ pi,
                                                   double* __restrict__ ps) {
  __shared__ double sv[kT];
  __shared__ int64_t si[kT];
  __shared__ double ss[kT];
  const int64_t base = (int64_t)blockIdx.x * kT * 16;
  double bv = -1.0, sum = 0.0;
  int64_t bi = -1;
  for (int k = 0; k < 16; ++k) {
    const int64_t i = base + (int64_t)k * kT + threadIdx.x;
    if (i < n) {
      const double v = use_abs ? fabs(d[i]) : d[i];
      sum += d[i];
      if (bi < 0 || v > bv) {
        bv = v;
        bi = i;
      }
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  ss[threadIdx.x] = sum;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v2 = sv[threadIdx.x + o];
      const int64_t i2 = si[threadIdx.x + o];
      if (i2 >= 0 && (si[threadIdx.x] < 0 || v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x]))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
      ss[threadIdx.x] += ss[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
    ps[blockIdx.x] = ss[0];
  }
}

// Final reduction over block partials (one block).  out: [0] = max, [1] = sum; idx_out = argmax.
__global__ __launch_bounds__(kT) void k_argmax_final(const double* __restrict__ pv, const int64_t* __restrict__ pi,
                                                     const double* __restrict__ ps, int nb, double* out,
                                                     int64_t* idx_out) {
  __shared__ double sv[kT];
  __shared__ int64_t si[kT];
  __shared__ double ss[kT];
  double bv = -1.0, sum = 0.0;
  int64_t bi = -1;
  for (int b = threadIdx.x; b < nb; b += kT) {
    sum += ps[b];
    if (pi[b] >= 0 && (bi < 0 || pv[b] > bv || (pv[b] == bv && pi[b] < bi))) {
      bv = pv[b];
      bi = pi[b];
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  ss[threadIdx.x] = sum;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v2 = sv[threadIdx.x + o];
      const int64_t i2 = si[threadIdx.x + o];
      if (i2 >= 0 && (si[threadIdx.x] < 0 || v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x]))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
      ss[threadIdx.x] += ss[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sv[0];
    out[1] = ss[0];
    idx_out[0] = si[0];
  }
}

// Column r of the pivoted Cholesky factor (column-major L, n rows):
//   L[:, r] = (C[:, p] - L[:, :r] L[p, :r]^T) / sqrt(d_p),  d -= L[:, r]^2,  d_p = 0.
__global__ __launch_bounds__(kT) void k_chol_col(Box b, double* __restrict__ L, double* __restrict__ d, int r,
                                                 const int64_t* __restrict__ pivp, const double* __restrict__ stat,
                                                 double s2, double inv_len, int sqexp) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= b.nn) return;
  const int64_t p = pivp[0];
  const double dp = stat[0];
  double xi[3], xp[3];
  box_xyz(b, i, xi);
  box_xyz(b, p, xp);
  const double dx = xi[0] - xp[0], dy = xi[1] - xp[1], dz = xi[2] - xp[2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  double c = s2 * exp(-(sqexp ? r2 : sqrt(r2)) * inv_len);
  for (int j = 0; j < r; ++j) c -= L[(int64_t)j * b.nn + i] * L[(int64_t)j * b.nn + p];
  const double l = c / sqrt(dp);
  L[(int64_t)r * b.nn + i] = l;
  d[i] = (i == p) ? 0.0 : d[i] - l * l;
}

// Mass matrix (tensor-product Q1) applied to every column: grid (blocks, columns).
__global__ __launch_bounds__(kT) void k_mass_cols(Box b, const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= b.nn) return;
  const int64_t c = blockIdx.y;
  const double* x = X + c * b.nn;
  const int64_t ix = i % b.n[0], r = i / b.n[0], iy = r % b.n[1], iz = r / b.n[1];
  // separable stencil: (M1 (x) M1 (x) M1), M1 = h/6 tridiag(1, 4, 1), halved diagonal at the ends
  double acc = 0.0;
  const int zlo = b.dim == 3 ? -1 : 0, zhi = b.dim == 3 ? 1 : 0;
  for (int oz = zlo; oz <= zhi; ++oz) {
    const int64_t jz = iz + oz;
    if (jz < 0 || jz >= b.n[2]) continue;
    double wz = 1.0;
    if (b.dim == 3) wz = oz != 0 ? b.h[2] / 6.0 : ((iz == 0 || iz == b.n[2] - 1) ? 2.0 : 4.0) * b.h[2] / 6.0;
    for (int oy = -1; oy <= 1; ++oy) {
      const int64_t jy = iy + oy;
      if (jy < 0 || jy >= b.n[1]) continue;
      const double wy = oy != 0 ? b.h[1] / 6.0 : ((iy == 0 || iy == b.n[1] - 1) ? 2.0 : 4.0) * b.h[1] / 6.0;
      for (int ox = -1; ox <= 1; ++ox) {
        const int64_t jx = ix + ox;
        if (jx < 0 || jx >= b.n[0]) continue;
        const double wx = ox != 0 ? b.h[0] / 6.0 : ((ix == 0 || ix == b.n[0] - 1) ? 2.0 : 4.0) * b.h[0] / 6.0;
        acc += wx * wy * wz * x[jx + b.n[0] * (jy + b.n[1] * jz)];
      }
    }
  }
  Y[c * b.nn + i] = acc;
}

// P1 mass (CSR) applied to every column: grid (blocks, columns).
__global__ __launch_bounds__(kT) void k_mass_csr_cols(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ mval,
                                                      const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const int64_t c = blockIdx.y;
  const double* x = X + c * n;
  double acc = 0.0;
  for (int32_t nz = rowptr[i]; nz < rowptr[i + 1]; ++nz) acc += mval[nz] * x[col[nz]];
  Y[c * n + i] = acc;
}

// phi[p][k] = sum_a w[p][a] psi[k][v[p][a]]  (psi column-major n x M, phi row-major P x M)
__global__ __launch_bounds__(kT) void k_transfer_bary(const double* __restrict__ psi, int64_t n, int M,
                                                      const int32_t* __restrict__ v, const double* __restrict__ w,
                                                      int64_t P, double* __restrict__ phi) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= P * M) return;
  const int64_t p = t / M;
  const int k = (int)(t % M);
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) acc += w[4 * p + a] * psi[(int64_t)k * n + v[4 * p + a]];
  phi[t] = acc;
}

// Split-K Gram matrix: part[chunk][a][c] = sum_{rows in chunk} A[:, a] B[:, c] (A, B column-major, n rows).
constexpr int kGT = 16;       // tile edge
constexpr int kGChunk = 8192; // rows per chunk
__global__ __launch_bounds__(kGT * kGT) void k_gram(const double* __restrict__ A, const double* __restrict__ Bm,
                                                    int64_t n, int R, double* __restrict__ part) {
  __shared__ double sa[64][kGT + 1];
  __shared__ double sb[64][kGT + 1];
  const int ta = threadIdx.x % kGT, tc = threadIdx.x / kGT;
  const int a = blockIdx.x * kGT + ta, c = blockIdx.y * kGT + tc;
  const int64_t r0 = (int64_t)blockIdx.z * kGChunk;
  const int64_t r1 = r0 + kGChunk < n ? r0 + kGChunk : n;
  double acc = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    // load 64 rows x 16 columns of A (tile columns blockIdx.x) and of B (tile columns blockIdx.y)
    for (int t = threadIdx.x; t < 64 * kGT; t += kGT * kGT) {
      const int row = t % 64, col = t / 64;
      const int64_t gr = rb + row;
      const int ca = blockIdx.x * kGT + col, cb = blockIdx.y * kGT + col;
      sa[row][col] = (gr < r1 && ca < R) ? A[(int64_t)ca * n + gr] : 0.0;
      sb[row][col] = (gr < r1 && cb < R) ? Bm[(int64_t)cb * n + gr] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int row = 0; row < 64; ++row) acc += sa[row][ta] * sb[row][tc];
    __syncthreads();
  }
  if (a < R && c < R) part[((int64_t)blockIdx.z * R + a) * R + c] = acc;
}

__global__ void k_gram_sum(const double* __restrict__ part, int nchunk, int R, double* S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)R * R) return;
  double s = 0.0;
  for (int k = 0; k < nchunk; ++k) s += part[(int64_t)k * R * R + t];
  S[t] = s;
}

// psi[:, k] = L W[:, k] (column-major, n rows; W is R x M row-major in LDS chunks).
__global__ __launch_bounds__(kT) void k_combine(const double* __restrict__ L, int64_t n, int R,
                                                const double* __restrict__ W, int M, double* __restrict__ psi) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < R; ++j) acc += L[(int64_t)j * n + i] * W[(int64_t)j * M + k];
  psi[(int64_t)k * n + i] = acc;
}

// Sign convention: the first entry of largest magnitude is positive; entries
// within a relative 1e-9 of the maximum count as ties (symmetric meshes give
// +/- pairs of equal magnitude).  One block per column.
__global__ __launch_bounds__(kT) void k_sign_fix(double* psi, int64_t n) {
  __shared__ double sv[kT];
  __shared__ int64_t si[kT];
  double* col = psi + (int64_t)blockIdx.x * n;
  double bv = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) bv = fmax(bv, fabs(col[i]));
  sv[threadIdx.x] = bv;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sv[threadIdx.x] = fmax(sv[threadIdx.x], sv[threadIdx.x + o]);
    __syncthreads();
  }
  const double cut = sv[0] * (1.0 - 1e-9);
  int64_t first = -1;
  for (int64_t i = threadIdx.x; i < n; i += kT)
    if (fabs(col[i]) >= cut) {
      first = i;
      break;
    }
  si[threadIdx.x] = first;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int64_t a = si[threadIdx.x], b = si[threadIdx.x + o];
      si[threadIdx.x] = (a < 0) ? b : ((b < 0) ? a : (a < b ? a : b));
    }
    __syncthreads();
  }
  const bool flip = si[0] >= 0 && col[si[0]] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = threadIdx.x; i < n; i += kT) col[i] = -col[i];
}

// Element-midpoint transfer: phi[p][k] = Q1 interpolant of psi[:, k] (KL grid) at centre p of the level.
__global__ __launch_bounds__(kT) void k_transfer(Box kb, Box lb, const double* __restrict__ psi, int M,
                                                 double* __restrict__ phi, int64_t P) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= P * M) return;
  const int64_t p = t / M;
  const int k = (int)(t % M);
  const int64_t nex = lb.n[0] - 1, ney = lb.n[1] - 1;
  const int64_t ex = p % nex, r = p / nex, ey = r % ney, ez = r / ney;
  const int64_t e[3] = {ex, ey, ez};
  int64_t cell[3] = {0, 0, 0};
  double xi[3] = {0, 0, 0};
  for (int a = 0; a < kb.dim; ++a) {
    const double c = lb.lo[a] + ((double)e[a] + 0.5) * lb.h[a];
    const double rel = (c - kb.lo[a]) / kb.h[a];
    int64_t ci = (int64_t)floor(rel);
    ci = ci < 0 ? 0 : (ci > kb.n[a] - 2 ? kb.n[a] - 2 : ci);
    cell[a] = ci;
    xi[a] = rel - (double)ci;
  }
  const double* col = psi + (int64_t)k * kb.nn;
  double acc = 0.0;
  const int nloc = kb.dim == 3 ? 8 : 4;
  for (int a = 0; a < nloc; ++a) {
    double w = 1.0;
    int64_t id = 0, stride = 1;
    for (int ax = 0; ax < kb.dim; ++ax) {
      const int off = (a >> ax) & 1;
      w *= off ? xi[ax] : 1.0 - xi[ax];
      id += (cell[ax] + off) * stride;
      stride *= kb.n[ax];
    }
    acc += w * col[id];
  }
  phi[p * M + k] = acc;
}

// R1 -= R2 (flat)
__global__ __launch_bounds__(kT) void k_axpy_cols(double* __restrict__ R1, const double* __restrict__ R2, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < total) R1[i] -= R2[i];
}

// ---- exact top eigenpairs on box grids (subspace iteration; C by circulant embedding) ----
// The covariance matrix of a uniform grid is (block) Toeplitz: C_ij = k(x_i - x_j) depends on
// the index offset only.  Embedded in a circulant of 2 (n_a - 1) points per axis (offsets d and
// N_a - d carry the same value), its product with a vector is exact through the FFT.
struct Emb {
  int32_t dim;
  int64_t n[3], N[3];  // grid and embedding sizes per axis (1 on unused axes)
  int64_t ne, nh;      // embedding points, half-spectrum points (N0 / 2 + 1 along axis 0)
};

// First column of the embedded circulant: c[m] = k(offset(m)), offset_a = min(m_a, N_a - m_a) h_a.
__global__ __launch_bounds__(kT) void k_circ_col(Emb e, Box b, double s2, double inv_len, int sqexp,
                                                 double* __restrict__ c) {
  const int64_t m = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (m >= e.ne) return;
  int64_t r = m;
  double d2 = 0.0;
  for (int a = 0; a < e.dim; ++a) {
    const int64_t ma = r % e.N[a];
    r /= e.N[a];
    const int64_t o = ma < e.N[a] - ma ? ma : e.N[a] - ma;
    const double d = (double)o * b.h[a];
    d2 += d * d;
  }
  c[m] = s2 * exp(-(sqexp ? d2 : sqrt(d2)) * inv_len);
}

// Columns col0 .. col0 + nc - 1 of X (n rows) zero-padded into the embedding, E[c][m].
__global__ __launch_bounds__(kT) void k_embed(Emb e, const double* __restrict__ X, int64_t n, int64_t col0,
                                              double* __restrict__ E) {
  const int64_t m = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (m >= e.ne) return;
  const int c = blockIdx.y;
  int64_t r = m, i = 0, stride = 1;
  bool in = true;
  for (int a = 0; a < e.dim; ++a) {
    const int64_t ma = r % e.N[a];
    r /= e.N[a];
    in = in && ma < e.n[a];
    i += ma * stride;
    stride *= e.n[a];
  }
  E[(int64_t)c * e.ne + m] = in ? X[(col0 + c) * n + i] : 0.0;
}

// Y[:, col0 + c] = the grid part of E[c] times scale.
__global__ __launch_bounds__(kT) void k_extract(Emb e, const double* __restrict__ E, int64_t n, int64_t col0,
                                                double scale, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const int c = blockIdx.y;
  int64_t r = i, m = 0, stride = 1;
  for (int a = 0; a < e.dim; ++a) {
    const int64_t ia = r % e.n[a];
    r /= e.n[a];
    m += ia * stride;
    stride *= e.N[a];
  }
  Y[(col0 + c) * n + i] = E[(int64_t)c * e.ne + m] * scale;
}

// Spectrum times the circulant's eigenvalues (real: the circulant is symmetric).
__global__ __launch_bounds__(kT) void k_cmul(hipfftDoubleComplex* __restrict__ F, const hipfftDoubleComplex* __restrict__ ch,
                                             int64_t nh) {
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k >= nh) return;
  const int c = blockIdx.y;
  const double lam = ch[k].x;
  hipfftDoubleComplex& f = F[(int64_t)c * nh + k];
  f.x *= lam;
  f.y *= lam;
}

// Seeded standard normals (counter-based: splitmix64 of the index, Box-Muller).
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ __launch_bounds__(kT) void k_randn(double* __restrict__ X, int64_t total, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i >= total) return;
  const uint64_t a = mix64(seed ^ (2 * (uint64_t)i)), c = mix64(seed ^ (2 * (uint64_t)i + 1));
  const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53, u2 = (double)(c >> 11) * 0x1.0p-53;
  X[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// out[:, k] = sum_j A[:, j] Z[j][k] (A column-major n x R, Z row-major R x C, out column-major n x C);
// a thread forms 8 output columns of one row.
constexpr int kCB = 8;
__global__ __launch_bounds__(kT) void k_combine8(const double* __restrict__ A, int64_t n, int R,
                                                 const double* __restrict__ Z, int C, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int k0 = blockIdx.y * kCB;
  if (i >= n) return;
  double acc[kCB];
#pragma unroll
  for (int q = 0; q < kCB; ++q) acc[q] = 0.0;
  for (int j = 0; j < R; ++j) {
    const double a = A[(int64_t)j * n + i];
    const double* z = Z + (int64_t)j * C + k0;
#pragma unroll
    for (int q = 0; q < kCB; ++q)
      if (k0 + q < C) acc[q] += a * z[q];
  }
#pragma unroll
  for (int q = 0; q < kCB; ++q)
    if (k0 + q < C) out[(int64_t)(k0 + q) * n + i] = acc[q];
}

// Cyclic Jacobi eigen-decomposition of a symmetric R x R matrix (row-major, in place).
// On return A's diagonal holds the eigenvalues and V (row-major) the eigenvectors as columns.
void jacobi_eig(std::vector<double>& A, std::vector<double>& V, int R) {
  V.assign((size_t)R * R, 0.0);
  for (int i = 0; i < R; ++i) V[(size_t)i * R + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * R + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < R; ++i) {
      diag += a(i, i) * a(i, i);
      for (int j = i + 1; j < R; ++j) off += a(i, j) * a(i, j);
    }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < R - 1; ++p)
      for (int q = p + 1; q < R; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        // rotation annihilating a_pq (symmetric Schur decomposition of the 2x2 block)
        const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < R; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < R; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < R; ++k) {
          const double vkp = V[(size_t)k * R + p], vkq = V[(size_t)k * R + q];
          V[(size_t)k * R + p] = c * vkp - s * vkq;
          V[(size_t)k * R + q] = s * vkp + c * vkq;
        }
      }
  }
}

Box make_box(const mlq_kl_desc* kd) {
  Box b{};
  if (kd->mesh_kind == MLQ_MESH_P1_TET) {
    b.dim = 3;
    b.nn = kd->n_vert;
    return b;
  }
  b.dim = kd->dim;
  b.nn = 1;
  for (int a = 0; a < 3; ++a) {
    b.n[a] = a < kd->dim ? kd->n[a] : 1;
    b.lo[a] = a < kd->dim ? kd->lo[a] : 0.0;
    b.h[a] = a < kd->dim ? (kd->hi[a] - kd->lo[a]) / (double)(kd->n[a] - 1) : 1.0;
    b.nn *= b.n[a];
  }
  return b;
}

inline size_t al(size_t v) { return (v + 255) & ~size_t(255); }

struct KlWork {
  double *L, *ML, *d, *pv, *ps, *stat, *part, *S, *W;
  int64_t *pi, *idx;
  double *xyz, *mval;   // tetrahedral KL mesh
  int32_t *rowptr, *col;
  size_t bytes;
};

// ---- exact route: workspace and driver ----
Emb make_emb(const Box& b) {
  Emb e{};
  e.dim = b.dim;
  e.ne = 1;
  for (int a = 0; a < 3; ++a) {
    e.n[a] = a < b.dim ? b.n[a] : 1;
    e.N[a] = a < b.dim ? 2 * (b.n[a] - 1) : 1;
    e.ne *= e.N[a];
  }
  e.nh = (e.N[0] / 2 + 1) * e.N[1] * e.N[2];
  return e;
}

// Columns of the subspace: twice the modes (at least 16 more), at most the nodes.
int exact_block(int64_t n, int M) { return (int)std::min<int64_t>(n, std::max(2 * M, M + 16)); }

// Embedded columns transformed together (bounded so that the FFT buffers stay near 4 GB).
int exact_chunk(const Emb& e, int bcols) {
  const double per = 8.0 * (double)e.ne + 16.0 * (double)e.nh;
  return (int)std::max(1.0, std::min((double)bcols, 4.0e9 / per));
}

struct ExactWork {
  double *X, *MX, *Y, *MY, *E, *part, *S, *Z, *R1, *R2, *cvec;
  hipfftDoubleComplex *F, *ch;
  void* fft_work;
  size_t bytes;
};

ExactWork exact_carve(void* base, int64_t n, int bcols, int M, const Emb& e, int chunk, size_t fft_bytes) {
  ExactWork w{};
  char* p = (char*)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? (void*)(p + o) : nullptr;
    o = al(o + bytes);
    return r;
  };
  w.X = (double*)take(sizeof(double) * n * bcols);
  w.MX = (double*)take(sizeof(double) * n * bcols);
  w.Y = (double*)take(sizeof(double) * n * bcols);
  w.MY = (double*)take(sizeof(double) * n * bcols);
  w.R1 = (double*)take(sizeof(double) * n * M);
  w.R2 = (double*)take(sizeof(double) * n * M);
  w.E = (double*)take(sizeof(double) * e.ne * chunk);
  w.F = (hipfftDoubleComplex*)take(sizeof(hipfftDoubleComplex) * e.nh * chunk);
  w.cvec = (double*)take(sizeof(double) * e.ne);
  w.ch = (hipfftDoubleComplex*)take(sizeof(hipfftDoubleComplex) * e.nh);
  w.part = (double*)take(sizeof(double) * cdiv(n, kGChunk) * bcols * bcols);
  w.S = (double*)take(sizeof(double) * bcols * bcols);
  w.Z = (double*)take(sizeof(double) * bcols * bcols);
  w.fft_work = take(fft_bytes);
  w.bytes = o;
  return w;
}

// hipFFT plans of the embedding (real to complex and back, `batch` columns), with the work area
// left to the caller's workspace; *work_bytes receives its size.
hipfftResult exact_plans(const Emb& e, int batch, hipfftHandle* fwd, hipfftHandle* bwd, size_t* work_bytes) {
  int dims[3];
  const int rank = e.dim;
  for (int a = 0; a < rank; ++a) dims[a] = (int)e.N[rank - 1 - a];  // row-major: slowest axis first
  int inembed[3], onembed[3];
  for (int a = 0; a < rank; ++a) inembed[a] = onembed[a] = dims[a];
  onembed[rank - 1] = dims[rank - 1] / 2 + 1;
  size_t w1 = 0, w2 = 0;
  hipfftResult r = hipfftCreate(fwd);
  if (r == HIPFFT_SUCCESS) r = hipfftCreate(bwd);
  if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(*fwd, 0);
  if (r == HIPFFT_SUCCESS) r = hipfftSetAutoAllocation(*bwd, 0);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany(*fwd, rank, dims, inembed, 1, (int)e.ne, onembed, 1, (int)e.nh, HIPFFT_D2Z, batch, &w1);
  if (r == HIPFFT_SUCCESS)
    r = hipfftMakePlanMany(*bwd, rank, dims, onembed, 1, (int)e.nh, inembed, 1, (int)e.ne, HIPFFT_Z2D, batch, &w2);
  *work_bytes = std::max(w1, w2);
  return r;
}

size_t exact_workspace_bytes(const mlq_kl_desc* kd) {
  const Box b = make_box(kd);
  const Emb e = make_emb(b);
  const int bcols = exact_block(b.nn, kd->n_modes);
  const int chunk = exact_chunk(e, bcols);
  hipfftHandle f = 0, g = 0;
  size_t wb = 0;
  const hipfftResult r = exact_plans(e, chunk, &f, &g, &wb);
  if (f) hipfftDestroy(f);
  if (g) hipfftDestroy(g);
  if (r != HIPFFT_SUCCESS) return 0;
  return exact_carve(nullptr, b.nn, bcols, kd->n_modes, e, chunk, wb).bytes;
}

// Cholesky G = U^T U (upper U, row-major b x b) and its inverse in place of U; false if G is
// not positive definite.
bool chol_inv_upper(std::vector<double>& G, int b, std::vector<double>& Uinv) {
  std::vector<double> U((size_t)b * b, 0.0);
  for (int j = 0; j < b; ++j) {
    double d = G[(size_t)j * b + j];
    for (int k = 0; k < j; ++k) d -= U[(size_t)k * b + j] * U[(size_t)k * b + j];
    if (!(d > 0.0)) return false;
    const double ujj = std::sqrt(d);
    U[(size_t)j * b + j] = ujj;
    for (int i = j + 1; i < b; ++i) {
      double v = G[(size_t)j * b + i];
      for (int k = 0; k < j; ++k) v -= U[(size_t)k * b + j] * U[(size_t)k * b + i];
      U[(size_t)j * b + i] = v / ujj;
    }
  }
  Uinv.assign((size_t)b * b, 0.0);
  for (int c = 0; c < b; ++c) {  // solve U x = e_c by back substitution
    for (int i = c; i >= 0; --i) {
      double v = i == c ? 1.0 : 0.0;
      for (int k = i + 1; k <= c; ++k) v -= U[(size_t)i * b + k] * Uinv[(size_t)k * b + c];
      Uinv[(size_t)i * b + c] = v / U[(size_t)i * b + i];
    }
  }
  return true;
}

// The n_modes largest eigenpairs of eq. (algEig) on a box grid, C M psi = lambda psi with
// psi^T M psi = 1, by subspace iteration with Rayleigh-Ritz on bcols >= 2 n_modes columns:
//   Y = C (M X);  T = (M X)^T Y;  T W = W Theta;  X <- Y W Theta^-1 orthonormalised in the M inner
//   product (Cholesky of its Gram matrix), until every wanted Ritz pair has
//   |C M psi - lambda psi|_M <= eps lambda (eps = kd->eps); C is applied through the FFT of its
//   circulant embedding.  *rank_out = bcols, *resid_out = the largest relative residual.
mlq_status kl_modes_exact(const mlq_kl_desc* kd, void* ws, double* lambda_host, double* psi_dev, int32_t* rank_out,
                          double* resid_out, hipStream_t s, std::string& err) {
  const Box b = make_box(kd);
  const Emb e = make_emb(b);
  const int64_t n = b.nn;
  const int M = kd->n_modes;
  const int bc = exact_block(n, M);
  const int chunk = exact_chunk(e, bc);
  auto chk = [&](hipError_t x, const char* what) {
    if (x != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(x);
      return false;
    }
    return true;
  };
  hipfftHandle pf = 0, pb = 0;
  size_t wb = 0;
  struct PlanGuard {
    hipfftHandle* a;
    hipfftHandle* b;
    ~PlanGuard() {
      if (*a) hipfftDestroy(*a);
      if (*b) hipfftDestroy(*b);
    }
  } guard{&pf, &pb};
  if (exact_plans(e, chunk, &pf, &pb, &wb) != HIPFFT_SUCCESS) {
    err = "FFT plan creation failed";
    return MLQ_EHIP;
  }
  ExactWork w = exact_carve(ws, n, bc, M, e, chunk, wb);
  if (hipfftSetWorkArea(pf, w.fft_work) != HIPFFT_SUCCESS || hipfftSetWorkArea(pb, w.fft_work) != HIPFFT_SUCCESS ||
      hipfftSetStream(pf, s) != HIPFFT_SUCCESS || hipfftSetStream(pb, s) != HIPFFT_SUCCESS) {
    err = "FFT plan set-up failed";
    return MLQ_EHIP;
  }
  const double s2 = kd->std_dev * kd->std_dev;
  const int sq = kd->cov_kernel == MLQ_COV_SQEXP ? 1 : 0;
  // eigenvalues of the circulant: the FFT of its first column (one column of the batch plan)
  hipLaunchKernelGGL(k_circ_col, dim3((unsigned)cdiv(e.ne, kT)), dim3(kT), 0, s, e, b, s2, 1.0 / kd->corr_len, sq,
                     w.E);
  if (chunk > 1)
    hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(e.ne * (chunk - 1), kT)), dim3(kT), 0, s, w.E + e.ne,
                       e.ne * (chunk - 1), 0.0);
  if (hipfftExecD2Z(pf, w.E, w.F) != HIPFFT_SUCCESS) {
    err = "FFT failed";
    return MLQ_EHIP;
  }
  if (!chk(hipMemcpyAsync(w.ch, w.F, sizeof(hipfftDoubleComplex) * e.nh, hipMemcpyDeviceToDevice, s), "copy")) return MLQ_EHIP;
  const double inv_ne = 1.0 / (double)e.ne;
  // Y[:, c] = C X[:, c] for every column
  auto apply_c = [&](const double* X, double* Y) -> bool {
    for (int c0 = 0; c0 < bc; c0 += chunk) {
      const int nc = std::min(chunk, bc - c0);
      hipLaunchKernelGGL(k_embed, dim3((unsigned)cdiv(e.ne, kT), nc), dim3(kT), 0, s, e, X, n, (int64_t)c0, w.E);
      if (nc < chunk)
        hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(e.ne * (chunk - nc), kT)), dim3(kT), 0, s,
                           w.E + (int64_t)nc * e.ne, e.ne * (chunk - nc), 0.0);
      if (hipfftExecD2Z(pf, w.E, w.F) != HIPFFT_SUCCESS) return false;
      hipLaunchKernelGGL(k_cmul, dim3((unsigned)cdiv(e.nh, kT), chunk), dim3(kT), 0, s, w.F, w.ch, e.nh);
      if (hipfftExecZ2D(pb, w.F, w.E) != HIPFFT_SUCCESS) return false;
      hipLaunchKernelGGL(k_extract, dim3((unsigned)cdiv(n, kT), nc), dim3(kT), 0, s, e, w.E, n, (int64_t)c0, inv_ne, Y);
    }
    return true;
  };
  const int nchunk = (int)cdiv(n, kGChunk);
  // G = A^T B (bc x bc or the first cols columns), to the host
  auto gram = [&](const double* A, const double* Bm, int cols, std::vector<double>& G) -> bool {
    hipLaunchKernelGGL(k_gram, dim3((unsigned)cdiv(cols, kGT), (unsigned)cdiv(cols, kGT), nchunk), dim3(kGT * kGT), 0, s,
                       A, Bm, n, cols, w.part);
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)cdiv((int64_t)cols * cols, kT)), dim3(kT), 0, s, w.part, nchunk, cols,
                       w.S);
    G.resize((size_t)cols * cols);
    if (!chk(hipMemcpyAsync(G.data(), w.S, sizeof(double) * cols * cols, hipMemcpyDeviceToHost, s), "copy")) return false;
    if (!chk(hipStreamSynchronize(s), "sync")) return false;
    for (int i = 0; i < cols; ++i)
      for (int j = i + 1; j < cols; ++j) {
        const double v = 0.5 * (G[(size_t)i * cols + j] + G[(size_t)j * cols + i]);
        G[(size_t)i * cols + j] = G[(size_t)j * cols + i] = v;
      }
    return true;
  };
  auto combine = [&](const double* A, int R, const std::vector<double>& Zh, int C, double* out) -> bool {
    if (!chk(hipMemcpyAsync(w.Z, Zh.data(), sizeof(double) * R * C, hipMemcpyHostToDevice, s), "copy")) return false;
    hipLaunchKernelGGL(k_combine8, dim3((unsigned)cdiv(n, kT), (unsigned)cdiv(C, kCB)), dim3(kT), 0, s, A, n, R, w.Z,
                       C, out);
    return chk(hipStreamSynchronize(s), "sync");  // Zh is host memory of the caller's scope
  };
  auto mass = [&](const double* X, double* Y, int cols) {
    hipLaunchKernelGGL(k_mass_cols, dim3((unsigned)cdiv(n, kT), cols), dim3(kT), 0, s, b, X, Y);
  };
  // start: seeded normals, M-orthonormalised
  hipLaunchKernelGGL(k_randn, dim3((unsigned)cdiv(n * bc, kT)), dim3(kT), 0, s, w.Y, n * bc, (uint64_t)0x4B4C4558ull);
  mass(w.Y, w.MY, bc);
  std::vector<double> G, T, V, Uinv, Zh((size_t)bc * bc);
  if (!gram(w.Y, w.MY, bc, G)) return MLQ_EHIP;
  if (!chol_inv_upper(G, bc, Uinv)) {
    err = "start block not of full rank";
    return MLQ_EINVAL;
  }
  if (!combine(w.Y, bc, Uinv, bc, w.X) || !combine(w.MY, bc, Uinv, bc, w.MX)) return MLQ_EHIP;
  std::vector<double> theta(bc), prev(M, 0.0);
  double worst = 1.0;
  const int max_it = 400;
  for (int it = 0; it < max_it; ++it) {
    if (!apply_c(w.MX, w.Y)) {
      err = "FFT failed";
      return MLQ_EHIP;
    }
    if (!gram(w.MX, w.Y, bc, T)) return MLQ_EHIP;  // Rayleigh quotient (M X)^T C (M X)
    jacobi_eig(T, V, bc);
    std::vector<int> order(bc);
    for (int i = 0; i < bc; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return T[(size_t)x * bc + x] > T[(size_t)y * bc + y]; });
    for (int k = 0; k < bc; ++k) theta[k] = T[(size_t)order[k] * bc + order[k]];
    double change = 0.0;
    for (int k = 0; k < M; ++k) change = std::max(change, std::fabs(theta[k] - prev[k]) / std::fabs(theta[k]));
    for (int k = 0; k < M; ++k) prev[k] = theta[k];
    // residuals of the wanted Ritz pairs, formed explicitly once the values have settled
    if (change < 1e-12 || it == max_it - 1) {
      std::vector<double> W1((size_t)bc * M), W2((size_t)bc * M);
      for (int j = 0; j < bc; ++j)
        for (int k = 0; k < M; ++k) {
          W1[(size_t)j * M + k] = V[(size_t)j * bc + order[k]];
          W2[(size_t)j * M + k] = V[(size_t)j * bc + order[k]] * theta[k];
        }
      if (!combine(w.Y, bc, W1, M, w.R1) || !combine(w.X, bc, W2, M, w.R2)) return MLQ_EHIP;
      hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)cdiv(n * M, kT)), dim3(kT), 0, s, w.R1, w.R2, n * M);
      mass(w.R1, w.R2, M);
      std::vector<double> RR;
      if (!gram(w.R1, w.R2, M, RR)) return MLQ_EHIP;
      worst = 0.0;
      for (int k = 0; k < M; ++k)
        worst = std::max(worst, std::sqrt(std::max(RR[(size_t)k * M + k], 0.0)) / theta[k]);
      if (worst <= kd->eps || it == max_it - 1) {
        for (int k = 0; k < M; ++k) {
          if (!(theta[k] > 0.0)) {
            err = "non-positive KL eigenvalue among the requested modes";
            return MLQ_EINVAL;
          }
          lambda_host[k] = theta[k];
        }
        // psi = X W (the Ritz vectors, M-orthonormal)
        if (!combine(w.X, bc, W1, M, psi_dev)) return MLQ_EHIP;
        hipLaunchKernelGGL(k_sign_fix, dim3(M), dim3(kT), 0, s, psi_dev, n);
        if (!chk(hipGetLastError(), "launch") || !chk(hipStreamSynchronize(s), "sync")) return MLQ_EHIP;
        if (rank_out) *rank_out = bc;
        if (resid_out) *resid_out = worst;
        if (worst > kd->eps) {
          err = "subspace iteration did not reach the residual tolerance";
          return MLQ_ENOCONV;
        }
        return MLQ_OK;
      }
    }
    // next block: Y W Theta^-1 (Ritz-rotated and scaled, nearly M-orthonormal), then Cholesky
    mass(w.Y, w.MY, bc);
    if (!gram(w.Y, w.MY, bc, G)) return MLQ_EHIP;
    std::vector<double> WT((size_t)bc * bc), G2((size_t)bc * bc, 0.0);
    for (int j = 0; j < bc; ++j)
      for (int k = 0; k < bc; ++k) WT[(size_t)j * bc + k] = V[(size_t)j * bc + order[k]] / theta[k];
    // G2 = WT^T G WT
    std::vector<double> GW((size_t)bc * bc, 0.0);
    for (int i = 0; i < bc; ++i)
      for (int j = 0; j < bc; ++j) {
        const double g = G[(size_t)i * bc + j];
        if (g == 0.0) continue;
        for (int k = 0; k < bc; ++k) GW[(size_t)i * bc + k] += g * WT[(size_t)j * bc + k];
      }
    for (int i = 0; i < bc; ++i)
      for (int j = 0; j < bc; ++j) {
        const double wt = WT[(size_t)i * bc + j];
        for (int k = 0; k < bc; ++k) G2[(size_t)j * bc + k] += wt * GW[(size_t)i * bc + k];
      }
    if (!chol_inv_upper(G2, bc, Uinv)) {
      err = "subspace lost rank";
      return MLQ_EINVAL;
    }
    for (int i = 0; i < bc; ++i)
      for (int k = 0; k < bc; ++k) {
        double v = 0.0;
        for (int j = 0; j <= k; ++j) v += WT[(size_t)i * bc + j] * Uinv[(size_t)j * bc + k];
        Zh[(size_t)i * bc + k] = v;
      }
    if (!combine(w.Y, bc, Zh, bc, w.X) || !combine(w.MY, bc, Zh, bc, w.MX)) return MLQ_EHIP;
  }
  err = "subspace iteration did not converge";
  return MLQ_ENOCONV;
}

// The P1 mass matrix of a tetrahedral KL mesh (CSR on the host).
std::string kl_tet_mass(const mlq_kl_desc* kd, TetHost& h, bool values) {
  mlq_level_desc d{};
  d.dim = 3;
  d.mesh_kind = MLQ_MESH_P1_TET;
  d.n_vert = kd->n_vert;
  d.n_tet = kd->n_tet;
  d.xyz = kd->xyz;
  d.tets = kd->tets;
  std::vector<double> frame(values ? 3 * (size_t)kd->n_tet : 3, 0.0);  // unused by the mass
  d.e_circ = d.e_long = frame.data();
  return tet_build(&d, h, values);
}

KlWork kl_carve(void* base, int64_t n, int R, int M, int64_t nnz = -1) {
  KlWork w{};
  char* p = (char*)base;
  size_t o = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? (void*)(p + o) : nullptr;
    o = al(o + bytes);
    return r;
  };
  const int64_t nb = cdiv(n, kT * 16);
  const int64_t nchunk = cdiv(n, kGChunk);
  w.L = (double*)take(sizeof(double) * n * R);
  w.ML = (double*)take(sizeof(double) * n * R);
  w.d = (double*)take(sizeof(double) * n);
  w.pv = (double*)take(sizeof(double) * nb);
  w.ps = (double*)take(sizeof(double) * nb);
  w.pi = (int64_t*)take(sizeof(int64_t) * nb);
  w.stat = (double*)take(sizeof(double) * 4);
  w.idx = (int64_t*)take(sizeof(int64_t) * 4);
  w.part = (double*)take(sizeof(double) * nchunk * R * R);
  w.S = (double*)take(sizeof(double) * R * R);
  w.W = (double*)take(sizeof(double) * R * M);
  if (nnz >= 0) {
    w.xyz = (double*)take(sizeof(double) * 3 * n);
    w.rowptr = (int32_t*)take(sizeof(int32_t) * (n + 1));
    w.col = (int32_t*)take(sizeof(int32_t) * nnz);
    w.mval = (double*)take(sizeof(double) * nnz);
  }
  w.bytes = o;
  return w;
}

}  // namespace

mlq_status kl_validate(const mlq_kl_desc* kd) {
  if (kd == nullptr) return MLQ_EINVAL;
  int64_t n = 1;
  if (kd->mesh_kind == MLQ_MESH_P1_TET) {
    if (kd->n_vert < 4 || kd->n_vert > (int64_t(1) << 27) || kd->n_tet < 1 || kd->n_tet >= (int64_t(1) << 27) ||
        kd->xyz == nullptr || kd->tets == nullptr)
      return MLQ_EINVAL;
    n = kd->n_vert;
  } else {
    if (kd->mesh_kind != MLQ_MESH_Q1_BOX) return MLQ_EINVAL;
    if (kd->dim != 2 && kd->dim != 3) return MLQ_EINVAL;
    for (int a = 0; a < kd->dim; ++a) {
      if (kd->n[a] < 2 || !(kd->hi[a] > kd->lo[a])) return MLQ_EINVAL;
      n *= kd->n[a];
    }
  }
  if (kd->n_modes < 0 || kd->n_modes > 1024) return MLQ_EINVAL;  // 0: stochastic dimension query
  if (kd->max_rank < std::max(kd->n_modes, 1) || kd->max_rank > 4096 || kd->max_rank > n) return MLQ_EINVAL;
  if (!(kd->std_dev > 0.0) || !(kd->corr_len > 0.0) || !(kd->eps >= 0.0)) return MLQ_EINVAL;
  if (kd->cov_kernel != MLQ_COV_EXP && kd->cov_kernel != MLQ_COV_SQEXP) return MLQ_EINVAL;
  if (kd->method != MLQ_KL_CHOLESKY && kd->method != MLQ_KL_EXACT) return MLQ_EINVAL;
  if (kd->method == MLQ_KL_EXACT &&
      (kd->mesh_kind != MLQ_MESH_Q1_BOX || kd->n_modes < 1 || !(kd->eps > 0.0) || 2 * (int64_t)kd->n_modes > n))
    return MLQ_EINVAL;
  return MLQ_OK;
}

size_t kl_workspace_bytes(const mlq_kl_desc* kd) {
  if (kd->method == MLQ_KL_EXACT) return exact_workspace_bytes(kd);
  const Box b = make_box(kd);
  if (kd->mesh_kind == MLQ_MESH_P1_TET) {
    TetHost h;
    if (!kl_tet_mass(kd, h, false).empty()) return 0;
    return kl_carve(nullptr, b.nn, kd->max_rank, kd->n_modes, h.nnz).bytes;
  }
  return kl_carve(nullptr, b.nn, kd->max_rank, kd->n_modes).bytes;
}

// Returns MLQ_OK or MLQ_EHIP; error text in err.
mlq_status kl_modes(const mlq_kl_desc* kd, void* ws, double* lambda_host, double* psi_dev, int32_t* rank_out,
                    double* resid_out, hipStream_t s, std::string& err) {
  if (kd->method == MLQ_KL_EXACT) return kl_modes_exact(kd, ws, lambda_host, psi_dev, rank_out, resid_out, s, err);
  Box b = make_box(kd);
  const int64_t n = b.nn;
  const int Rmax = kd->max_rank, M = kd->n_modes;
  const bool tet = kd->mesh_kind == MLQ_MESH_P1_TET;
  TetHost th;
  if (tet) {
    err = kl_tet_mass(kd, th, true);
    if (!err.empty()) return MLQ_EINVAL;
  }
  KlWork w = kl_carve(ws, n, Rmax, M, tet ? th.nnz : -1);
  if (tet) {
    hipError_t e = hipMemcpyAsync(w.xyz, kd->xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w.rowptr, th.rowptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w.col, th.col.data(), sizeof(int32_t) * th.nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w.mval, th.mval.data(), sizeof(double) * th.nnz, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      err = std::string("KL mesh upload: ") + hipGetErrorString(e);
      return MLQ_EHIP;
    }
    b.xyz = w.xyz;
  }
  const int64_t nb = cdiv(n, kT * 16);
  const double s2 = kd->std_dev * kd->std_dev;
  const double tr0 = s2 * (double)n;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(e);
      return false;
    }
    return true;
  };
  hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, s, w.d, n, s2);
  double hstat[2];
  int rank = 0;
  double resid = tr0;
  for (int r = 0; r < Rmax; ++r) {
    hipLaunchKernelGGL(k_argmax_sum, dim3((unsigned)nb), dim3(kT), 0, s, w.d, n, 0, w.pv, w.pi, w.ps);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(kT), 0, s, w.pv, w.pi, w.ps, (int)nb, w.stat, w.idx);
    if (!chk(hipMemcpyAsync(hstat, w.stat, sizeof(hstat), hipMemcpyDeviceToHost, s), "copy")) return MLQ_EHIP;
    if (!chk(hipStreamSynchronize(s), "sync")) return MLQ_EHIP;
    resid = hstat[1];
    if (hstat[0] <= 0.0) break;                            // exact low rank reached
    if (r >= M && resid <= kd->eps * tr0) break;           // truncation criterion
    hipLaunchKernelGGL(k_chol_col, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, s, b, w.L, w.d, r, w.idx, w.stat, s2,
                       1.0 / kd->corr_len, kd->cov_kernel == MLQ_COV_SQEXP ? 1 : 0);
    rank = r + 1;
  }
  if (rank < M) {
    err = "covariance has numerical rank below n_modes";
    return MLQ_EINVAL;
  }
  if (M == 0) {  // query: the rank at which the truncation criterion holds is the dimension M
    if (rank_out) *rank_out = rank;
    if (resid_out) *resid_out = resid / tr0;
    return MLQ_OK;
  }
  if (rank == Rmax) {  // residual after the last column
    hipLaunchKernelGGL(k_argmax_sum, dim3((unsigned)nb), dim3(kT), 0, s, w.d, n, 0, w.pv, w.pi, w.ps);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(kT), 0, s, w.pv, w.pi, w.ps, (int)nb, w.stat, w.idx);
    if (!chk(hipMemcpyAsync(hstat, w.stat, sizeof(hstat), hipMemcpyDeviceToHost, s), "copy")) return MLQ_EHIP;
    if (!chk(hipStreamSynchronize(s), "sync")) return MLQ_EHIP;
    resid = hstat[1];
  }
  const int R = rank;
  // reduced eigenproblem eq. (redEig): S = L^T M L
  if (tet)
    hipLaunchKernelGGL(k_mass_csr_cols, dim3((unsigned)cdiv(n, kT), R), dim3(kT), 0, s, n, w.rowptr, w.col, w.mval,
                       w.L, w.ML);
  else
    hipLaunchKernelGGL(k_mass_cols, dim3((unsigned)cdiv(n, kT), R), dim3(kT), 0, s, b, w.L, w.ML);
  const int nchunk = (int)cdiv(n, kGChunk);
  hipLaunchKernelGGL(k_gram, dim3((unsigned)cdiv(R, kGT), (unsigned)cdiv(R, kGT), nchunk), dim3(kGT * kGT), 0, s,
                     w.L, w.ML, n, R, w.part);
  hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)cdiv((int64_t)R * R, kT)), dim3(kT), 0, s, w.part, nchunk, R, w.S);
  std::vector<double> S((size_t)R * R), V;
  if (!chk(hipMemcpyAsync(S.data(), w.S, sizeof(double) * R * R, hipMemcpyDeviceToHost, s), "copy S")) return MLQ_EHIP;
  if (!chk(hipStreamSynchronize(s), "sync")) return MLQ_EHIP;
  for (int i = 0; i < R; ++i)
    for (int j = i + 1; j < R; ++j) {
      const double v = 0.5 * (S[(size_t)i * R + j] + S[(size_t)j * R + i]);
      S[(size_t)i * R + j] = S[(size_t)j * R + i] = v;
    }
  jacobi_eig(S, V, R);
  std::vector<int> order(R);
  for (int i = 0; i < R; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return S[(size_t)x * R + x] > S[(size_t)y * R + y]; });
  std::vector<double> W((size_t)R * M);
  for (int k = 0; k < M; ++k) {
    const double lam = S[(size_t)order[k] * R + order[k]];
    if (!(lam > 0.0)) {
      err = "non-positive KL eigenvalue among the requested modes";
      return MLQ_EINVAL;
    }
    lambda_host[k] = lam;
    const double inv = 1.0 / std::sqrt(lam);
    for (int j = 0; j < R; ++j) W[(size_t)j * M + k] = V[(size_t)j * R + order[k]] * inv;
  }
  if (!chk(hipMemcpyAsync(w.W, W.data(), sizeof(double) * R * M, hipMemcpyHostToDevice, s), "copy W")) return MLQ_EHIP;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)cdiv(n, kT), M), dim3(kT), 0, s, w.L, n, R, w.W, M, psi_dev);
  hipLaunchKernelGGL(k_sign_fix, dim3(M), dim3(kT), 0, s, psi_dev, n);
  if (!chk(hipGetLastError(), "launch")) return MLQ_EHIP;
  if (!chk(hipStreamSynchronize(s), "sync")) return MLQ_EHIP;
  if (rank_out) *rank_out = R;
  if (resid_out) *resid_out = resid / tr0;
  return MLQ_OK;
}

mlq_status kl_transfer(const mlq_kl_desc* kd, const double* psi_dev, const int64_t* level_n, const double* level_lo,
                       const double* level_hi, double* phi_dev, hipStream_t s) {
  const Box kb = make_box(kd);
  Box lb{};
  lb.dim = kd->dim;
  lb.nn = 1;
  int64_t P = 1;
  for (int a = 0; a < 3; ++a) {
    lb.n[a] = a < kd->dim ? level_n[a] : 2;
    lb.lo[a] = a < kd->dim ? level_lo[a] : 0.0;
    lb.h[a] = a < kd->dim ? (level_hi[a] - level_lo[a]) / (double)(level_n[a] - 1) : 1.0;
    lb.nn *= lb.n[a];
    if (a < kd->dim) P *= level_n[a] - 1;
  }
  const int M = kd->n_modes;
  hipLaunchKernelGGL(k_transfer, dim3((unsigned)cdiv(P * M, kT)), dim3(kT), 0, s, kb, lb, psi_dev, M, phi_dev, P);
  return hipGetLastError() == hipSuccess ? MLQ_OK : MLQ_EHIP;
}

}  // namespace mlq

namespace mlq {

size_t kl_transfer_tet_bytes(int64_t P) { return al(sizeof(int32_t) * 4 * P) + al(sizeof(double) * 4 * P); }

// Point location in a tetrahedral mesh (uniform bucket grid over the mesh; the tetrahedron
// with the largest smallest barycentric coordinate, lowest index on ties within 1e-12; the
// search widens to the neighbouring cells for a point no candidate contains, and a point
// outside the mesh takes the best tetrahedron found there).  Output per point: the four
// vertices and the barycentric weights, negative ones clipped to 0 and renormalised.
mlq_status locate_points_tet(const mlq_kl_desc* kd, const double* pts, int64_t np, std::vector<int32_t>& vid,
                             std::vector<double>& wts, std::string& err) {
  TetHost h;
  err = kl_tet_mass(kd, h, true);  // gradients of the tetrahedra (geo)
  if (!err.empty()) return MLQ_EINVAL;
  const int64_t kn = kd->n_vert, kt = kd->n_tet;
  const double* kx = kd->xyz;
  const int32_t* kT4 = kd->tets;
  // bucket grid
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < kn; ++v)
    for (int m = 0; m < 3; ++m) {
      lo[m] = std::min(lo[m], kx[3 * v + m]);
      hi[m] = std::max(hi[m], kx[3 * v + m]);
    }
  const double cell = 2.0 * std::cbrt(h.vol / (double)kt);
  int64_t dims[3];
  for (int m = 0; m < 3; ++m) dims[m] = std::max<int64_t>(1, (int64_t)std::ceil((hi[m] - lo[m]) / cell));
  while (dims[0] * dims[1] * dims[2] > 8 * kt + 64)
    for (int m = 0; m < 3; ++m) dims[m] = std::max<int64_t>(1, dims[m] / 2);
  const double cw[3] = {(hi[0] - lo[0]) / dims[0] + 1e-300, (hi[1] - lo[1]) / dims[1] + 1e-300,
                        (hi[2] - lo[2]) / dims[2] + 1e-300};
  auto cidx = [&](const double* x, int m) {
    const int64_t c = (int64_t)std::floor((x[m] - lo[m]) / cw[m]);
    return std::min(std::max<int64_t>(c, 0), dims[m] - 1);
  };
  const int64_t ncell = dims[0] * dims[1] * dims[2];
  std::vector<int64_t> cptr(ncell + 1, 0);
  std::vector<int32_t> clist;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      for (int64_t c = 0; c < ncell; ++c) cptr[c + 1] += cptr[c];
      clist.assign(cptr[ncell], 0);
      fill.assign(cptr.begin(), cptr.end() - 1);
    }
    for (int64_t e = 0; e < kt; ++e) {
      double blo[3] = {1e300, 1e300, 1e300}, bhi[3] = {-1e300, -1e300, -1e300};
      for (int a = 0; a < 4; ++a)
        for (int m = 0; m < 3; ++m) {
          blo[m] = std::min(blo[m], kx[3 * (int64_t)kT4[4 * e + a] + m]);
          bhi[m] = std::max(bhi[m], kx[3 * (int64_t)kT4[4 * e + a] + m]);
        }
      int64_t c0[3], c1[3];
      for (int m = 0; m < 3; ++m) {
        c0[m] = cidx(blo, m);
        c1[m] = cidx(bhi, m);
      }
      for (int64_t z = c0[2]; z <= c1[2]; ++z)
        for (int64_t y = c0[1]; y <= c1[1]; ++y)
          for (int64_t x = c0[0]; x <= c1[0]; ++x) {
            const int64_t c = x + dims[0] * (y + dims[1] * z);
            if (pass == 0)
              cptr[c + 1]++;
            else
              clist[fill[c]++] = (int32_t)e;
          }
    }
  }
  auto bary = [&](int64_t e, const double* x, double lam[4]) {
    const double* G = h.geo.data() + e * kTetGeo;
    const double* p0 = kx + 3 * (int64_t)kT4[4 * e];
    const double d0 = x[0] - p0[0], d1 = x[1] - p0[1], d2 = x[2] - p0[2];
    double s1 = 0.0;
    for (int a = 1; a < 4; ++a) {
      lam[a] = G[3 * a] * d0 + G[3 * a + 1] * d1 + G[3 * a + 2] * d2;
      s1 += lam[a];
    }
    lam[0] = 1.0 - s1;
  };
  auto score = [&](int64_t e, const double* x) {
    double lam[4];
    bary(e, x, lam);
    return std::min(std::min(lam[0], lam[1]), std::min(lam[2], lam[3]));
  };
  vid.assign((size_t)4 * np, 0);
  wts.assign((size_t)4 * np, 0.0);
  std::vector<int32_t> cand;
  for (int64_t p = 0; p < np; ++p) {
    const double* x = pts + 3 * p;
    int64_t ci[3];
    for (int m = 0; m < 3; ++m) ci[m] = cidx(x, m);
    int64_t best_e = -1;
    for (int ring = 0; best_e < 0 || ring <= 1; ++ring) {
      cand.clear();
      for (int64_t z = std::max<int64_t>(0, ci[2] - ring); z <= std::min(dims[2] - 1, ci[2] + ring); ++z)
        for (int64_t y = std::max<int64_t>(0, ci[1] - ring); y <= std::min(dims[1] - 1, ci[1] + ring); ++y)
          for (int64_t xx = std::max<int64_t>(0, ci[0] - ring); xx <= std::min(dims[0] - 1, ci[0] + ring); ++xx) {
            const int64_t c = xx + dims[0] * (y + dims[1] * z);
            cand.insert(cand.end(), clist.begin() + cptr[c], clist.begin() + cptr[c + 1]);
          }
      if (cand.empty()) {
        if (ring > dims[0] + dims[1] + dims[2]) break;
        continue;
      }
      double best = -1e300;
      for (int32_t e : cand) best = std::max(best, score(e, x));
      int64_t pick = -1;
      for (int32_t e : cand)
        if (score(e, x) >= best - 1e-12 && (pick < 0 || e < pick)) pick = e;
      best_e = pick;
      if (best >= -1e-12) break;  // a containing tetrahedron: the rule is decided locally
      if (ring >= 1) break;       // outside: the best of the neighbouring cells
    }
    if (best_e < 0) {
      err = "point location failed";
      return MLQ_EINVAL;
    }
    double lam[4], sum = 0.0;
    bary(best_e, x, lam);
    for (int a = 0; a < 4; ++a) {
      lam[a] = std::max(lam[a], 0.0);
      sum += lam[a];
    }
    for (int a = 0; a < 4; ++a) {
      vid[4 * p + a] = kT4[4 * best_e + a];
      wts[4 * p + a] = lam[a] / sum;
    }
  }
  return MLQ_OK;
}

// Non-nested transfer: locate the centroids of the level's tetrahedra in the KL mesh, then
// interpolate the modes on the device.
mlq_status kl_transfer_tet(const mlq_kl_desc* kd, const double* psi_dev, int64_t nv, const double* xyz, int64_t nt,
                           const int32_t* tets, void* ws, double* phi_dev, hipStream_t s, std::string& err) {
  (void)nv;
  std::vector<double> cen((size_t)3 * nt, 0.0);
  for (int64_t p = 0; p < nt; ++p)
    for (int a = 0; a < 4; ++a)
      for (int m = 0; m < 3; ++m) cen[3 * p + m] += 0.25 * xyz[3 * (int64_t)tets[4 * p + a] + m];
  std::vector<int32_t> vid;
  std::vector<double> wts;
  const mlq_status st = locate_points_tet(kd, cen.data(), nt, vid, wts, err);
  if (st != MLQ_OK) return st;
  const int64_t kn = kd->n_vert;
  int32_t* dv = (int32_t*)ws;
  double* dw = (double*)((char*)ws + al(sizeof(int32_t) * 4 * nt));
  hipError_t e = hipMemcpyAsync(dv, vid.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dw, wts.data(), sizeof(double) * 4 * nt, hipMemcpyHostToDevice, s);
  const int M = kd->n_modes;
  if (e == hipSuccess)
    hipLaunchKernelGGL(k_transfer_bary, dim3((unsigned)cdiv(nt * M, kT)), dim3(kT), 0, s, psi_dev, kn, M, dv, dw, nt,
                       phi_dev);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host arrays must outlive the copies
  if (e != hipSuccess) {
    err = std::string("transfer: ") + hipGetErrorString(e);
    return MLQ_EHIP;
  }
  return MLQ_OK;
}

}  // namespace mlq
