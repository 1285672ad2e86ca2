// Host preparation of a P1 tetrahedral level: validation, the vertex-adjacency
// CSR of M and K, the consistent mass (Section 3.1: |T| (1 + delta_ab) / 20 per
// element), the element contributions of every nonzero in increasing element
// order, per-element gradients / fibre frame / volume, node weights w = M 1 and
// the stimulus load F = M chi of the stimulus ball.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "mlq_internal.h"

namespace mlq {

std::string tet_build(const mlq_level_desc* d, TetHost& h, bool values) {
  char msg[256];
  if (d->dim != 3) return "tetrahedral levels are 3D";
  const int64_t nv = d->n_vert, nt = d->n_tet;
  if (nv < 4 || nv > (int64_t(1) << 27)) return "n_vert must be in [4, 2^27]";
  if (nt < 1 || nt >= (int64_t(1) << 27)) return "n_tet must be in [1, 2^27)";
  if (d->xyz == nullptr || d->tets == nullptr || d->e_circ == nullptr || d->e_long == nullptr)
    return "xyz, tets, e_circ and e_long are required";
  if (!(d->stim_radius >= 0.0)) return "stim_radius must be >= 0";
  h.nv = nv;
  h.nt = nt;
  for (int64_t e = 0; e < 4 * nt; ++e)
    if (d->tets[e] < 0 || d->tets[e] >= nv) {
      std::snprintf(msg, sizeof msg, "tetrahedron %lld has a vertex index out of range", (long long)(e / 4));
      return msg;
    }
  // orientation (checked here so that sizing already rejects a bad mesh)
  for (int64_t e = 0; e < nt; ++e) {
    const double* p0 = d->xyz + 3 * (int64_t)d->tets[4 * e];
    double E[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) E[r][c] = d->xyz[3 * (int64_t)d->tets[4 * e + r + 1] + c] - p0[c];
    const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                       E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                       E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (!(det > 0.0)) {
      std::snprintf(msg, sizeof msg, "tetrahedron %lld is not positively oriented", (long long)e);
      return msg;
    }
  }
  // vertex -> incident tetrahedra (increasing element order)
  std::vector<int64_t> iptr(nv + 1, 0);
  for (int64_t e = 0; e < 4 * nt; ++e) iptr[d->tets[e] + 1]++;
  for (int64_t v = 0; v < nv; ++v) iptr[v + 1] += iptr[v];
  std::vector<int32_t> inc(4 * nt);
  {
    std::vector<int64_t> pos(iptr.begin(), iptr.end() - 1);
    for (int64_t e = 0; e < nt; ++e)
      for (int a = 0; a < 4; ++a) inc[pos[d->tets[4 * e + a]]++] = (int32_t)e;
  }
  // rows: sorted unique neighbours
  h.rowptr.assign(nv + 1, 0);
  std::vector<int32_t> nb;
  std::vector<std::vector<int32_t>> rows;  // filled only to size the CSR, then moved
  h.col.clear();
  for (int64_t v = 0; v < nv; ++v) {
    nb.clear();
    for (int64_t q = iptr[v]; q < iptr[v + 1]; ++q)
      for (int b = 0; b < 4; ++b) nb.push_back(d->tets[4 * (int64_t)inc[q] + b]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    if (h.col.size() + nb.size() > (size_t)INT32_MAX) return "too many nonzeros for 32-bit CSR indices";
    h.col.insert(h.col.end(), nb.begin(), nb.end());
    h.rowptr[v + 1] = (int32_t)h.col.size();
  }
  h.nnz = (int64_t)h.col.size();
  h.nc = 16 * nt;
  h.width = 0;
  for (int64_t v = 0; v < nv; ++v) {
    if (h.rowptr[v + 1] == h.rowptr[v]) return "a vertex belongs to no tetrahedron";
    h.width = std::max(h.width, h.rowptr[v + 1] - h.rowptr[v]);
  }
  h.nell = (int64_t)h.width * nv;
  if (h.nell > (int64_t)INT32_MAX) return "too many padded nonzeros for 32-bit indices";
  if (!values) return "";
  // element geometry: gradients (rows of inverse edge matrix), frame, volume
  h.geo.assign((size_t)nt * kTetGeo, 0.0);
  for (int64_t e = 0; e < nt; ++e) {
    const double* p[4];
    for (int a = 0; a < 4; ++a) p[a] = d->xyz + 3 * (int64_t)d->tets[4 * e + a];
    double E[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) E[r][c] = p[r + 1][c] - p[0][c];
    const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                       E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                       E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (!(det > 0.0)) {
      std::snprintf(msg, sizeof msg, "tetrahedron %lld is not positively oriented", (long long)e);
      return msg;
    }
    // inverse of E: inv[c][r] = cofactor(r, c) / det; grad phi_{r+1} = column r of inv
    double inv[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        inv[c][r] = (E[r1][c1] * E[r2][c2] - E[r1][c2] * E[r2][c1]) / det;
      }
    double* G = h.geo.data() + e * kTetGeo;
    for (int a = 1; a < 4; ++a)
      for (int m = 0; m < 3; ++m) G[3 * a + m] = inv[m][a - 1];
    for (int m = 0; m < 3; ++m) G[m] = -(G[3 + m] + G[6 + m] + G[9 + m]);
    for (int m = 0; m < 3; ++m) {
      G[12 + m] = d->e_circ[3 * e + m];
      G[15 + m] = d->e_long[3 * e + m];
    }
    G[18] = det / 6.0;
    h.vol += G[18];
  }
  // contributions per nonzero (increasing element, then local column) and the mass
  h.cptr.assign(h.nnz + 1, 0);
  h.cdat.assign(h.nc, 0);
  h.mval.assign(h.nnz, 0.0);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fill;
    if (pass == 1) fill.assign(h.cptr.begin(), h.cptr.end() - 1);
    for (int64_t v = 0; v < nv; ++v) {
      const int32_t* rb = h.col.data() + h.rowptr[v];
      const int32_t* re = h.col.data() + h.rowptr[v + 1];
      for (int64_t q = iptr[v]; q < iptr[v + 1]; ++q) {
        const int64_t e = inc[q];
        int a = 0;
        while (d->tets[4 * e + a] != v) ++a;
        for (int b = 0; b < 4; ++b) {
          const int32_t j = d->tets[4 * e + b];
          const int64_t nz = h.rowptr[v] + (std::lower_bound(rb, re, j) - rb);
          if (pass == 0) {
            h.cptr[nz + 1]++;
          } else {
            h.cdat[fill[nz]++] = (int32_t)((e << 4) | (4 * a + b));
            h.mval[nz] += h.geo[e * kTetGeo + 18] * (a == b ? 2.0 : 1.0) / 20.0;
          }
        }
      }
    }
    if (pass == 0)
      for (int64_t nz = 0; nz < h.nnz; ++nz) h.cptr[nz + 1] += h.cptr[nz];
  }
  // slot-major padded rows: entry (slot s, row v) at s * nv + v; a padded slot points at the
  // row itself with a zero value and no contributions
  h.ediag.assign(nv, -1);
  for (int64_t v = 0; v < nv; ++v)
    for (int32_t nz = h.rowptr[v]; nz < h.rowptr[v + 1]; ++nz)
      if (h.col[nz] == v) h.ediag[v] = nz - h.rowptr[v];
  h.ecol.assign(h.nell, 0);
  h.em.assign(h.nell, 0.0);
  h.ecptr.assign(h.nell + 1, 0);
  h.ecdat.assign(h.nc, 0);
  {
    int64_t c = 0;
    for (int32_t sl = 0; sl < h.width; ++sl)
      for (int64_t v = 0; v < nv; ++v) {
        const int64_t idx = (int64_t)sl * nv + v;
        if (sl < h.rowptr[v + 1] - h.rowptr[v]) {
          const int64_t nz = h.rowptr[v] + sl;
          h.ecol[idx] = h.col[nz];
          h.em[idx] = h.mval[nz];
          for (int32_t q = h.cptr[nz]; q < h.cptr[nz + 1]; ++q) h.ecdat[c++] = h.cdat[q];
        } else {
          h.ecol[idx] = (int32_t)v;
        }
        h.ecptr[idx + 1] = (int32_t)c;
      }
  }
  h.mdiag.assign(nv, 0.0);
  h.wts.assign(nv, 0.0);
  h.fload.assign(nv, 0.0);
  std::vector<double> chi(nv, 0.0);
  const double r2 = d->stim_radius * d->stim_radius;
  for (int64_t v = 0; v < nv; ++v) {
    double s = 0.0;
    for (int m = 0; m < 3; ++m) {
      const double t = d->xyz[3 * v + m] - d->stim_center[m];
      s += t * t;
    }
    chi[v] = s < r2 ? 1.0 : 0.0;
  }
  for (int64_t v = 0; v < nv; ++v)
    for (int32_t nz = h.rowptr[v]; nz < h.rowptr[v + 1]; ++nz) {
      const int32_t j = h.col[nz];
      if (j == v) h.mdiag[v] = h.mval[nz];
      h.wts[v] += h.mval[nz];
      h.fload[v] += h.mval[nz] * chi[j];
    }
  return "";
}

}  // namespace mlq
