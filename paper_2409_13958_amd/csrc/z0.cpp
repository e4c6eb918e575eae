// Element-exact near-field correction (paper Eq. hms_d2b and the correction
// radius "based on the average edge length" of Sec. 3.2.2), FP64.
//
// Each tetrahedron e carries the constant volume charge rho_e = -Ms_e div m
// and, on its faces that are surfaces of the body (outer boundary or a
// material interface after LCA gluing), the linear surface charge
// sigma = Ms_e m.n. For every tetrahedron whose centroid lies within
// kappa * hbar of the observer (minimum image), the exact potential of those
// charges replaces the point charges q_i^(e) that e contributes to the other
// nodes i:
//   u_Z,n = (1/4 pi) sum_e [ rho_e int_e 1/R + sum_f int_f sigma/R
//                            - sum_{i != n} q_i^(e) / |r_n - r_i| ].
// The integrals are closed forms: over a triangle, int 1/R and
// int (rho' - rho)/R from the edge formulas of Wilton et al. (IEEE TAP 1984)
// and Graglia (IEEE TAP 1993); over a tetrahedron, by the divergence
// theorem, int_e 1/R = (1/2) sum_f n_f.(r_f - r) int_f 1/R.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace pmfem {
namespace {

inline void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Triangle P[0..2]: unit normal n (right-handed in vertex order), twice the
// area, I0 = int 1/R, Ir = int (rho' - rho)/R, rho = projection of r.
struct TriInt {
  double n[3], area2, I0, Ir[3], rho[3];
};

void tri_integrals(const double* r, const double* P0, const double* P1, const double* P2, TriInt& o) {
  const double* P[3] = {P0, P1, P2};
  double e1[3], e2[3];
  sub3(P1, P0, e1);
  sub3(P2, P0, e2);
  cross3(e1, e2, o.n);
  o.area2 = std::sqrt(dot3(o.n, o.n));
  for (int i = 0; i < 3; ++i) o.n[i] /= o.area2;
  double rp[3];
  sub3(r, P0, rp);
  double d = dot3(o.n, rp);
  for (int i = 0; i < 3; ++i) o.rho[i] = r[i] - d * o.n[i];
  double ad = std::fabs(d);
  o.I0 = 0.0;
  o.Ir[0] = o.Ir[1] = o.Ir[2] = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double* Pa = P[i];
    const double* Pb = P[(i + 1) % 3];
    double l[3];
    sub3(Pb, Pa, l);
    double len = std::sqrt(dot3(l, l));
    double lh[3] = {l[0] / len, l[1] / len, l[2] / len};
    double uh[3];
    cross3(lh, o.n, uh);  // outward in-plane edge normal
    double a[3], b[3];
    sub3(Pa, o.rho, a);
    sub3(Pb, o.rho, b);
    double lm = dot3(a, lh), lp = dot3(b, lh);
    double t = dot3(a, uh);  // signed distance of rho from the edge line
    double R0sq = t * t + d * d;
    double Rp = std::sqrt(R0sq + lp * lp), Rm = std::sqrt(R0sq + lm * lm);
    double f = 0.0;
    if (R0sq > 1e-28 * len * len) {
      double R0 = std::sqrt(R0sq);
      f = std::asinh(lp / R0) - std::asinh(lm / R0);
    }
    double beta = 0.0;
    if (ad > 0.0 && t != 0.0)
      beta = std::atan(t * lp / (R0sq + ad * Rp)) - std::atan(t * lm / (R0sq + ad * Rm));
    o.I0 += t * f - ad * beta;
    double g = 0.5 * (R0sq * f + lp * Rp - lm * Rm);
    for (int k = 0; k < 3; ++k) o.Ir[k] += g * uh[k];
  }
}

struct Geom {
  double V, g[4][3];
};

bool geom(const double X[4][3], Geom& G) {
  double a[3], b[3], c[3], bc[3], ca[3], ab[3];
  sub3(X[1], X[0], a);
  sub3(X[2], X[0], b);
  sub3(X[3], X[0], c);
  cross3(b, c, bc);
  cross3(c, a, ca);
  cross3(a, b, ab);
  double v6 = dot3(a, bc);
  G.V = v6 / 6.0;
  for (int i = 0; i < 3; ++i) {
    G.g[1][i] = bc[i] / v6;
    G.g[2][i] = ca[i] / v6;
    G.g[3][i] = ab[i] / v6;
    G.g[0][i] = -(G.g[1][i] + G.g[2][i] + G.g[3][i]);
  }
  return v6 > 0.0;
}

struct Cells {
  int nc[3];
  double lo[3], size[3];
  int per[3];
  std::vector<int64_t> start;
  std::vector<int64_t> items;
  int cell_of(int a, double x) const {
    double v = (x - lo[a]) / size[a];
    int i = (int)std::floor(v);
    if (per[a]) {
      i %= nc[a];
      if (i < 0) i += nc[a];
    } else {
      i = std::min(std::max(i, 0), nc[a] - 1);
    }
    return i;
  }
};

}  // namespace

int build_z0(pmfem_ctx* c, const std::vector<uint8_t>& surface) {
  HostOps& o = c->ops;
  const int64_t T = c->n_tets, Np = o.n_unk;
  const double* X = c->xyz.data();
  const int32_t* tets = c->tets.data();
  const std::vector<int64_t>& uk = o.unk_of_node;
  const double rad = c->z0_radius * o.hbar;
  const double rad2 = rad * rad;
  o.z0_rowptr.assign(Np + 1, 0);
  if (rad <= 0.0) {
    o.z0_col.clear();
    o.z0_val.clear();
    return PMFEM_OK;
  }
  // centroids and a cell grid of size >= rad over them (periodic axes wrap)
  std::vector<double> cen(3 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 3; ++a)
      cen[3 * t + a] = 0.25 * (X[3 * tets[4 * t] + a] + X[3 * tets[4 * t + 1] + a] +
                               X[3 * tets[4 * t + 2] + a] + X[3 * tets[4 * t + 3] + a]);
  Cells cl;
  for (int a = 0; a < 3; ++a) {
    cl.per[a] = o.per[a];
    if (o.per[a]) {
      cl.lo[a] = 0.0;
      cl.nc[a] = std::max(1, (int)std::floor(c->L[a] / rad));
      cl.size[a] = c->L[a] / cl.nc[a];
    } else {
      double mn = 1e300, mx = -1e300;
      for (int64_t t = 0; t < T; ++t) {
        mn = std::min(mn, cen[3 * t + a]);
        mx = std::max(mx, cen[3 * t + a]);
      }
      for (int64_t n = 0; n < c->n_nodes; ++n) {
        mn = std::min(mn, X[3 * n + a]);
        mx = std::max(mx, X[3 * n + a]);
      }
      cl.lo[a] = mn;
      cl.nc[a] = std::max(1, (int)std::floor((mx - mn) / rad));
      cl.size[a] = (mx - mn) / cl.nc[a] + 1e-300;
    }
  }
  const int64_t ncell = (int64_t)cl.nc[0] * cl.nc[1] * cl.nc[2];
  cl.start.assign(ncell + 1, 0);
  std::vector<int64_t> cid(T);
  for (int64_t t = 0; t < T; ++t) {
    int i = cl.cell_of(0, cen[3 * t]), j = cl.cell_of(1, cen[3 * t + 1]), k = cl.cell_of(2, cen[3 * t + 2]);
    cid[t] = ((int64_t)k * cl.nc[1] + j) * cl.nc[0] + i;
    cl.start[cid[t] + 1]++;
  }
  for (int64_t q = 0; q < ncell; ++q) cl.start[q + 1] += cl.start[q];
  cl.items.resize(T);
  {
    std::vector<int64_t> fill(cl.start.begin(), cl.start.end() - 1);
    for (int64_t t = 0; t < T; ++t) cl.items[fill[cid[t]]++] = t;
  }
  // elements near observer u, with their minimum-image shift
  auto near_elems = [&](int64_t u, std::vector<int64_t>& el, std::vector<double>& sh) {
    el.clear();
    sh.clear();
    const double* r = X + 3 * o.node_of_unk[u];
    int ci[3];
    for (int a = 0; a < 3; ++a) ci[a] = cl.cell_of(a, r[a]);
    int lst[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, cnt[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      cnt[a] = 0;
      for (int d = -1; d <= 1; ++d) {
        int v = ci[a] + d;
        if (cl.per[a]) {
          v = ((v % cl.nc[a]) + cl.nc[a]) % cl.nc[a];
        } else if (v < 0 || v >= cl.nc[a]) {
          continue;
        }
        bool dup = false;
        for (int q = 0; q < cnt[a]; ++q) dup |= (lst[a][q] == v);
        if (!dup) lst[a][cnt[a]++] = v;
      }
    }
    for (int iz = 0; iz < cnt[2]; ++iz)
      for (int iy = 0; iy < cnt[1]; ++iy)
        for (int ix = 0; ix < cnt[0]; ++ix) {
          int64_t q = ((int64_t)lst[2][iz] * cl.nc[1] + lst[1][iy]) * cl.nc[0] + lst[0][ix];
          for (int64_t it = cl.start[q]; it < cl.start[q + 1]; ++it) {
            int64_t t = cl.items[it];
            double dv[3], s3[3], d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
              dv[a] = cen[3 * t + a] - r[a];
              s3[a] = o.per[a] ? -c->L[a] * std::nearbyint(dv[a] / c->L[a]) : 0.0;
              double w = dv[a] + s3[a];
              d2 += w * w;
            }
            if (d2 <= rad2) {
              el.push_back(t);
              sh.push_back(s3[0]);
              sh.push_back(s3[1]);
              sh.push_back(s3[2]);
            }
          }
        }
  };
  std::vector<int32_t> rowlen(Np);
  parallel_for(Np, [&](int64_t u) {
    std::vector<int64_t> el;
    std::vector<double> sh;
    near_elems(u, el, sh);
    std::vector<int64_t> cols;
    for (int64_t t : el)
      for (int b = 0; b < 4; ++b) cols.push_back(uk[tets[4 * t + b]]);
    std::sort(cols.begin(), cols.end());
    rowlen[u] = (int32_t)(std::unique(cols.begin(), cols.end()) - cols.begin());
  }, 512);
  for (int64_t u = 0; u < Np; ++u) {
    int64_t v = (int64_t)o.z0_rowptr[u] + rowlen[u];
    if (v > 2147483647LL) {
      c->err = "element correction exceeds 2^31 entries";
      return PMFEM_ENOMEM;
    }
    o.z0_rowptr[u + 1] = (int32_t)v;
  }
  const int64_t nnz = o.z0_rowptr[Np];
  o.z0_col.resize(nnz);
  o.z0_val.assign(4 * nnz, 0.0f);
  std::atomic<int> bad(0);
  parallel_for(Np, [&](int64_t u) {
    std::vector<int64_t> el;
    std::vector<double> sh;
    near_elems(u, el, sh);
    std::vector<int64_t> cols;
    for (int64_t t : el)
      for (int b = 0; b < 4; ++b) cols.push_back(uk[tets[4 * t + b]]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    std::vector<double> acc(3 * cols.size(), 0.0);
    const double* r = X + 3 * o.node_of_unk[u];
    for (size_t ie = 0; ie < el.size(); ++ie) {
      int64_t t = el[ie];
      double P[4][3];
      int vtx = -1;
      for (int b = 0; b < 4; ++b) {
        for (int a = 0; a < 3; ++a) P[b][a] = X[3 * tets[4 * t + b] + a] + sh[3 * ie + a];
        if (uk[tets[4 * t + b]] == u) vtx = b;
      }
      Geom G;
      geom(P, G);
      double ms = c->Ms[c->region[t]];
      double g0[4];
      for (int b = 0; b < 4; ++b) {
        double dv[3];
        sub3(r, P[b], dv);
        double dd = std::sqrt(dot3(dv, dv));
        if (b == vtx) {
          if (dd > 1e-6 * o.hbar) bad = 1;
          g0[b] = 0.0;
        } else {
          g0[b] = 1.0 / dd;
        }
      }
      double gsum = g0[0] + g0[1] + g0[2] + g0[3];
      // exact volume integral via the four faces
      double IV = 0.0;
      TriInt ti[4];
      bool have[4] = {false, false, false, false};
      double nout[4][3];
      for (int a = 0; a < 4; ++a) {
        int f0 = (a + 1) % 4, f1 = (a + 2) % 4, f2 = (a + 3) % 4;
        // outward normal of the face opposite a
        double e1[3], e2[3], nn[3], toa[3];
        sub3(P[f1], P[f0], e1);
        sub3(P[f2], P[f0], e2);
        cross3(e1, e2, nn);
        double nl = std::sqrt(dot3(nn, nn));
        sub3(P[a], P[f0], toa);
        double sg = dot3(nn, toa) > 0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; ++k) nout[a][k] = sg * nn[k] / nl;
        double pr[3];
        sub3(P[f0], r, pr);
        double dn = dot3(nout[a], pr);
        bool need_face = surface[4 * t + a] != 0;
        if (vtx == a || vtx < 0 || need_face) {
          // faces through the observer (vtx != a, vtx >= 0) have dn = 0
          tri_integrals(r, P[f0], P[f1], P[f2], ti[a]);
          have[a] = true;
          if (vtx == a || vtx < 0) IV += 0.5 * dn * ti[a].I0;
        }
      }
      double ex[4][3], pt[4][3];
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 3; ++k) {
          ex[j][k] = -ms * IV * G.g[j][k];
          pt[j][k] = -ms * G.V / 4.0 * gsum * G.g[j][k];
        }
      for (int a = 0; a < 4; ++a) {
        if (!surface[4 * t + a]) continue;
        int fv[3] = {(a + 1) % 4, (a + 2) % 4, (a + 3) % 4};
        const TriInt& T3 = ti[a];
        (void)have;
        // orientation of the triangle as passed: T3.n; outward normal nout[a]
        double area = 0.5 * T3.area2;
        for (int li = 0; li < 3; ++li) {
          int j = fv[li];
          // lambda_j on the face (barycentric in the plane) at rho, and its gradient
          const double* Pj1 = P[fv[(li + 1) % 3]];
          const double* Pj2 = P[fv[(li + 2) % 3]];
          double e[3], gs[3], v1[3], v2[3], cr[3];
          sub3(Pj2, Pj1, e);
          cross3(T3.n, e, gs);
          for (int k = 0; k < 3; ++k) gs[k] /= T3.area2;
          sub3(Pj1, T3.rho, v1);
          sub3(Pj2, T3.rho, v2);
          cross3(v1, v2, cr);
          double lam = dot3(cr, T3.n) / T3.area2;
          double Ifl = lam * T3.I0 + dot3(gs, T3.Ir);
          double share = 0.0;
          for (int q = 0; q < 3; ++q) share += g0[fv[q]] * (fv[q] == j ? 2.0 : 1.0);
          for (int k = 0; k < 3; ++k) {
            ex[j][k] += ms * Ifl * nout[a][k];
            pt[j][k] += ms * area / 12.0 * share * nout[a][k];
          }
        }
      }
      for (int j = 0; j < 4; ++j) {
        int64_t col = uk[tets[4 * t + j]];
        size_t pos = std::lower_bound(cols.begin(), cols.end(), col) - cols.begin();
        for (int k = 0; k < 3; ++k) acc[3 * pos + k] += (ex[j][k] - pt[j][k]) / (4.0 * kPi);
      }
    }
    int64_t base = o.z0_rowptr[u];
    for (size_t j = 0; j < cols.size(); ++j) {
      o.z0_col[base + j] = (int32_t)cols[j];
      for (int k = 0; k < 3; ++k) o.z0_val[4 * (base + j) + k] = (float)acc[3 * j + k];
      o.z0_val[4 * (base + j) + 3] = 0.0f;
    }
  }, 256);
  if (bad) {
    c->err = "an element vertex maps to the observer at another periodic image";
    return PMFEM_EMESH;
  }
  return PMFEM_OK;
}

}  // namespace pmfem
