// Host setup of the PM-FEM operators, FP64 arithmetic, run once per build.
//
//  1. PBC pairs (nodes equal modulo the lattice) by spatial hashing and
//     union-find LCA merge (Secs. 2.1, 2.2).
//  2. Folded positions (Eq. shift_hms), grid coordinates, boxes, and the
//     box-sorted numbering of the unknowns (Sec. 3.2.2).
//  3. Periodised P1 operators on one shared CSR pattern (Secs. 3.1, 3.2.1):
//     exchange  L_nk = -2 K_nk / (mu0 mu_n),  K_nk = sum_t A_t V_t gl_n . gl_k
//     charge    q_n  = sum_k D_nk . m_k,      D_nk = sum_t Ms_t V_t/4 gl_n
//     gradient  H_n -= sum_k G_nk u_k,        G_nk = D_kn / mu_n
//     where the tetrahedra keep their own geometry and their vertex indices
//     are replaced by LCA unknowns (Eqs. lapl_1, lapl_2).
//  4. Grid kernel K(g) = G^p(g Delta), K(0) = G_reg(0), and its spectrum.
//  5. Precorrection P_nk = [k != n] G0(r_nk*) - W_n^T K0 W_k over near boxes
//     (G0-only correction of Sec. 3.2.2), assembled with the factorisation
//     W_n^T K0 W_k = sum_a' W_k(a') Phi_n(a'), Phi_n = W_n^T K0.
//  6. Element-exact correction (z0.cpp).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "internal.h"

namespace pmfem {
namespace {

struct TetGeom {
  double V;
  double g[4][3];  // barycentric gradients
};

// Volume and barycentric gradients from the face cross products:
// grad(lambda_i) = (edge x edge of the opposite face) / (6 V).
inline bool tet_geom(const double* X0, const double* X1, const double* X2, const double* X3,
                     TetGeom& t) {
  double a[3], b[3], c[3];
  for (int i = 0; i < 3; ++i) {
    a[i] = X1[i] - X0[i];
    b[i] = X2[i] - X0[i];
    c[i] = X3[i] - X0[i];
  }
  double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
  double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  double v6 = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
  t.V = v6 / 6.0;
  if (!(v6 > 0.0)) return false;
  for (int i = 0; i < 3; ++i) {
    t.g[1][i] = bc[i] / v6;
    t.g[2][i] = ca[i] / v6;
    t.g[3][i] = ab[i] / v6;
    t.g[0][i] = -(t.g[1][i] + t.g[2][i] + t.g[3][i]);
  }
  return true;
}

int find_root(std::vector<int64_t>& par, int64_t i) {
  int64_t r = i;
  while (par[r] != r) r = par[r];
  while (par[i] != r) {
    int64_t n = par[i];
    par[i] = r;
    i = n;
  }
  return (int)r;
}

struct CellKey {
  int64_t x, y, z;
  bool operator==(const CellKey& o) const { return x == o.x && y == o.y && z == o.z; }
};
struct CellHash {
  size_t operator()(const CellKey& k) const {
    uint64_t h = (uint64_t)k.x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.y * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.z * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

int fail(pmfem_ctx* c, int code, const std::string& m) {
  c->err = m;
  return code;
}

// a product of the factors 2, 3, 5 and 7 (the radices of the FFT passes)
bool is_smooth7(int v) {
  if (v < 1) return false;
  for (int r : {2, 3, 5, 7})
    while (v % r == 0) v /= r;
  return v == 1;
}

}  // namespace

int host_build(pmfem_ctx* c) {
  HostOps& o = c->ops;
  o = HostOps();
  const int64_t N = c->n_nodes, T = c->n_tets;
  if (!c->have_mesh || !c->have_mat || !c->have_aim)
    return fail(c, PMFEM_ESTATE, "mesh, materials and AIM parameters must be set before build");
  if (c->precision < 0 || c->precision > 2)
    return fail(c, PMFEM_EINVAL, "precision must be 0 (FP32), 1 (BF16 grid) or 2 (BF16 hi + lo grid)");
  const int p = c->order_p, rb = c->near_boxes;
  if (p < 1 || p > 5) return fail(c, PMFEM_EINVAL, "order_p must be in [1, 5]");
  if (rb < 0 || rb > 3) return fail(c, PMFEM_EINVAL, "near_boxes must be in [0, 3]");
  if (!(c->z0_radius >= 0.0)) return fail(c, PMFEM_EINVAL, "z0_radius must be >= 0");
  for (int32_t r = 0; r < c->n_regions; ++r) {
    if (!(c->Ms[r] > 0.0)) return fail(c, PMFEM_EINVAL, "Ms must be > 0 in every region");
    if (!(c->Aex[r] >= 0.0)) return fail(c, PMFEM_EINVAL, "Aex must be >= 0");
  }
  for (int a = 0; a < 3; ++a)
    if (((c->mask >> a) & 1) && !(c->L[a] > 0.0))
      return fail(c, PMFEM_EINVAL, "period must be > 0 on periodic axes");
  // ---- mesh validation and orientation -------------------------------------
  std::vector<int32_t>& tets = c->tets;
  for (int64_t t = 0; t < T; ++t) {
    for (int a = 0; a < 4; ++a) {
      int32_t v = tets[4 * t + a];
      if (v < 0 || v >= N) return fail(c, PMFEM_EMESH, "tetrahedron vertex index out of range");
    }
    if (c->region[t] < 0 || c->region[t] >= c->n_regions)
      return fail(c, PMFEM_EMESH, "region id out of range");
  }
  const double* X = c->xyz.data();
  std::atomic<int> bad(0);
  parallel_for(T, [&](int64_t t) {
    int32_t* v = &tets[4 * t];
    TetGeom g;
    if (!tet_geom(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], X + 3 * v[3], g)) {
      if (g.V < 0.0) {
        std::swap(v[2], v[3]);
        if (!tet_geom(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], X + 3 * v[3], g)) bad = 1;
      } else {
        bad = 1;
      }
    }
  }, 4096);
  if (bad) return fail(c, PMFEM_EMESH, "degenerate tetrahedron (zero volume)");

  // ---- 1. PBC pairs and LCA -------------------------------------------------
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t n = 0; n < N; ++n)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], X[3 * n + a]);
      hi[a] = std::max(hi[a], X[3 * n + a]);
    }
  double scale = 0.0;
  for (int a = 0; a < 3; ++a) {
    scale = std::max(scale, hi[a] - lo[a]);
    if ((c->mask >> a) & 1) scale = std::max(scale, c->L[a]);
  }
  const double tol = (c->match_tol > 0 ? c->match_tol : 1e-9) * scale;
  std::vector<int64_t> par(N);
  std::iota(par.begin(), par.end(), 0);
  if (c->mask) {
    // Two nodes form a PBC pair when they coincide modulo the lattice (any
    // combination of periods: the combined shifts of Sec. 2.1 and the images
    // of protruding cells). Positions are wrapped into the cell on periodic
    // axes and hashed on a grid of cells much larger than the tolerance;
    // neighbouring cells are visited (cyclically on periodic axes) only for
    // points within the tolerance of a cell face.
    const double cell = tol * 64.0;
    int per[3];
    int64_t ncell[3];
    std::vector<double> w(3 * N);
    for (int a = 0; a < 3; ++a) {
      per[a] = (c->mask >> a) & 1;
      ncell[a] = per[a] ? (int64_t)std::ceil(c->L[a] / cell) : 0;
    }
    for (int64_t n = 0; n < N; ++n)
      for (int a = 0; a < 3; ++a) {
        double v = X[3 * n + a];
        if (per[a]) {
          v -= c->L[a] * std::floor(v / c->L[a]);
          if (v >= c->L[a]) v -= c->L[a];
        }
        w[3 * n + a] = v;
      }
    std::unordered_map<CellKey, std::vector<int32_t>, CellHash> hash;
    hash.reserve((size_t)N * 2);
    auto key_of = [&](const double* v) {
      return CellKey{(int64_t)std::floor(v[0] / cell), (int64_t)std::floor(v[1] / cell),
                     (int64_t)std::floor(v[2] / cell)};
    };
    for (int64_t n = 0; n < N; ++n) hash[key_of(&w[3 * n])].push_back((int32_t)n);
    std::vector<std::vector<int32_t>> match(N);
    parallel_for(N, [&](int64_t n) {
      const double* v = &w[3 * n];
      CellKey k0 = key_of(v);
      int64_t base[3] = {k0.x, k0.y, k0.z};
      int rng[3][2];
      for (int d = 0; d < 3; ++d) {
        double f = v[d] / cell - (double)base[d];
        rng[d][0] = f < 0.1 ? -1 : 0;
        rng[d][1] = f > 0.9 ? 1 : 0;
        if (per[d]) {  // the top cell of a periodic axis may be partial
          if (base[d] == ncell[d] - 1) rng[d][1] = 1;
          if (v[d] > c->L[d] - 2.0 * tol) rng[d][1] = 1;
        }
      }
      for (int dx = rng[0][0]; dx <= rng[0][1]; ++dx)
        for (int dy = rng[1][0]; dy <= rng[1][1]; ++dy)
          for (int dz = rng[2][0]; dz <= rng[2][1]; ++dz) {
            int64_t kk[3] = {base[0] + dx, base[1] + dy, base[2] + dz};
            for (int d = 0; d < 3; ++d)
              if (per[d]) kk[d] = ((kk[d] % ncell[d]) + ncell[d]) % ncell[d];
            auto it = hash.find(CellKey{kk[0], kk[1], kk[2]});
            if (it == hash.end()) continue;
            for (int32_t j : it->second) {
              if (j <= n) continue;
              double d2 = 0.0;
              for (int d = 0; d < 3; ++d) {
                double e = w[3 * j + d] - v[d];
                if (per[d]) e -= c->L[d] * std::nearbyint(e / c->L[d]);
                d2 += e * e;
              }
              if (d2 <= tol * tol) match[n].push_back(j);
            }
          }
    }, 4096);
    for (int64_t n = 0; n < N; ++n)
      for (int32_t j : match[n]) {
        int64_t ra = find_root(par, n), rb2 = find_root(par, j);
        if (ra != rb2) {
          if (ra < rb2) par[rb2] = ra; else par[ra] = rb2;
        }
      }
  }
  std::vector<int64_t> root(N);
  for (int64_t n = 0; n < N; ++n) root[n] = find_root(par, n);
  std::vector<int64_t> reps;
  for (int64_t n = 0; n < N; ++n)
    if (root[n] == n) reps.push_back(n);
  const int64_t Np = (int64_t)reps.size();
  o.n_nodes = N;
  o.n_unk = Np;

  // ---- 2. folded positions, grid, boxes, unknown order -----------------------
  std::vector<double> pos(3 * Np);
  double r0[3] = {0, 0, 0};
  for (int64_t i = 0; i < Np; ++i)
    for (int a = 0; a < 3; ++a) r0[a] += X[3 * reps[i] + a];
  for (int a = 0; a < 3; ++a) r0[a] /= (double)Np;
  for (int64_t i = 0; i < Np; ++i)
    for (int a = 0; a < 3; ++a) {
      double x = X[3 * reps[i] + a];
      if ((c->mask >> a) & 1) x -= c->L[a] * std::floor((x - r0[a]) / c->L[a] + 0.5);
      pos[3 * i + a] = x;
    }
  o.p = p;
  o.rb = rb;
  for (int a = 0; a < 3; ++a) {
    o.per[a] = (c->mask >> a) & 1;
    o.N[a] = c->grid[a];
    o.M[a] = o.per[a] ? o.N[a] : 2 * o.N[a];
    o.nbox[a] = o.per[a] ? o.N[a] : o.N[a] - 1;
    if (o.N[a] < p + 1) return fail(c, PMFEM_EGRID, "grid axis shorter than the stencil");
    if (!is_smooth7(o.M[a]) || o.M[a] < 4 || o.M[a] > 512)
      return fail(c, PMFEM_EGRID, "FFT extent must be a product of 2, 3, 5 and 7 in [4, 512]");
    if (o.per[a] && o.N[a] < 2 * (rb + p) + 1)
      return fail(c, PMFEM_EGRID, "periodic grid axis too short for the near region");
    if (o.per[a]) {
      o.delta[a] = c->L[a] / o.N[a];
      o.origin[a] = 0.0;
    } else {
      double mn = 1e300, mx = -1e300;
      for (int64_t i = 0; i < Np; ++i) {
        mn = std::min(mn, pos[3 * i + a]);
        mx = std::max(mx, pos[3 * i + a]);
      }
      if (!(mx > mn)) return fail(c, PMFEM_EGRID, "mesh has no extent along a non-periodic axis");
      o.origin[a] = mn;
      o.delta[a] = (mx - mn) / (o.N[a] - 1);
    }
  }
  const int shift = (p - 1) / 2;
  std::vector<double> s(3 * Np);
  std::vector<int32_t> bx(3 * Np), stu(3 * Np);
  std::vector<int64_t> boxlin(Np);
  for (int64_t i = 0; i < Np; ++i) {
    for (int a = 0; a < 3; ++a) {
      double v = (pos[3 * i + a] - o.origin[a]) / o.delta[a];
      int b;
      int st;
      if (o.per[a]) {
        v -= o.N[a] * std::floor(v / o.N[a]);
        b = (int)std::floor(v);
        if (b >= o.N[a]) b -= o.N[a];
        st = b - shift;
      } else {
        b = (int)std::floor(v);
        b = std::min(std::max(b, 0), o.N[a] - 2);
        st = std::min(std::max(b - shift, 0), o.N[a] - p - 1);
      }
      s[3 * i + a] = v;
      bx[3 * i + a] = b;
      stu[3 * i + a] = st;
    }
    boxlin[i] = ((int64_t)bx[3 * i + 2] * o.nbox[1] + bx[3 * i + 1]) * o.nbox[0] + bx[3 * i];
  }
  std::vector<int64_t> order(Np);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return boxlin[a] < boxlin[b]; });
  // permute everything into the box-sorted unknown order
  o.node_of_unk.resize(Np);
  o.pos.resize(3 * Np);
  {
    std::vector<double> s2(3 * Np);
    std::vector<int32_t> b2(3 * Np), st2(3 * Np);
    std::vector<int64_t> bl2(Np);
    for (int64_t u = 0; u < Np; ++u) {
      int64_t i = order[u];
      o.node_of_unk[u] = reps[i];
      bl2[u] = boxlin[i];
      for (int a = 0; a < 3; ++a) {
        o.pos[3 * u + a] = pos[3 * i + a];
        s2[3 * u + a] = s[3 * i + a];
        b2[3 * u + a] = bx[3 * i + a];
        st2[3 * u + a] = stu[3 * i + a];
      }
    }
    s.swap(s2);
    bx.swap(b2);
    stu.swap(st2);
    boxlin.swap(bl2);
  }
  {
    std::vector<int64_t> unk_of_rep(N, -1);
    for (int64_t u = 0; u < Np; ++u) unk_of_rep[o.node_of_unk[u]] = u;
    o.unk_of_node.resize(N);
    for (int64_t n = 0; n < N; ++n) o.unk_of_node[n] = unk_of_rep[root[n]];
  }
  const int64_t nbox = (int64_t)o.nbox[0] * o.nbox[1] * o.nbox[2];
  o.box_start.assign(nbox + 1, 0);
  for (int64_t u = 0; u < Np; ++u) o.box_start[boxlin[u] + 1]++;
  for (int64_t b = 0; b < nbox; ++b) o.box_start[b + 1] += o.box_start[b];
  o.pos4.resize(4 * Np);
  for (int64_t u = 0; u < Np; ++u) {
    uint32_t packed = 0;  // box coordinates, 10 bits per axis
    for (int a = 0; a < 3; ++a) {
      o.pos4[4 * u + a] = (float)(s[3 * u + a] - stu[3 * u + a]);
      packed |= (uint32_t)bx[3 * u + a] << (10 * a);
    }
    std::memcpy(&o.pos4[4 * u + 3], &packed, 4);
  }
  const std::vector<int64_t>& uk = o.unk_of_node;
  // a tetrahedron whose vertices merge into fewer than four unknowns spans a
  // whole period: the periodic faces cannot be matched consistently
  for (int64_t t = 0; t < T; ++t) {
    const int32_t* v = &tets[4 * t];
    for (int a2 = 0; a2 < 4; ++a2)
      for (int b2 = a2 + 1; b2 < 4; ++b2)
        if (uk[v[a2]] == uk[v[b2]])
          return fail(c, PMFEM_EPBC, "a tetrahedron spans a whole period (two vertices are images)");
  }

  // ---- 3. local operators ----------------------------------------------------
  std::vector<int64_t> inc_ptr(Np + 1, 0);
  for (int64_t t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a) inc_ptr[uk[tets[4 * t + a]] + 1]++;
  for (int64_t u = 0; u < Np; ++u) inc_ptr[u + 1] += inc_ptr[u];
  std::vector<int64_t> inc(inc_ptr[Np]);
  {
    std::vector<int64_t> fillp(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) inc[fillp[uk[tets[4 * t + a]]]++] = 4 * t + a;
  }
  std::vector<int32_t> rowlen(Np);
  parallel_for(Np, [&](int64_t u) {
    std::vector<int64_t> cols;
    for (int64_t e = inc_ptr[u]; e < inc_ptr[u + 1]; ++e) {
      int64_t t = inc[e] / 4;
      for (int b = 0; b < 4; ++b) cols.push_back(uk[tets[4 * t + b]]);
    }
    std::sort(cols.begin(), cols.end());
    rowlen[u] = (int32_t)(std::unique(cols.begin(), cols.end()) - cols.begin());
  }, 1024);
  o.loc_rowptr.assign(Np + 1, 0);
  for (int64_t u = 0; u < Np; ++u) o.loc_rowptr[u + 1] = o.loc_rowptr[u] + rowlen[u];
  const int64_t nnzL = o.loc_rowptr[Np];
  o.loc_col.resize(nnzL);
  o.loc_val.assign(8 * nnzL, 0.0f);
  o.mu.assign(Np, 0.0);
  parallel_for(Np, [&](int64_t u) {
    std::vector<int64_t> cols;
    for (int64_t e = inc_ptr[u]; e < inc_ptr[u + 1]; ++e) {
      int64_t t = inc[e] / 4;
      for (int b = 0; b < 4; ++b) cols.push_back(uk[tets[4 * t + b]]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    size_t nc = cols.size();
    std::vector<double> K(nc, 0.0), D(3 * nc, 0.0), G(3 * nc, 0.0);
    double mu = 0.0;
    for (int64_t e = inc_ptr[u]; e < inc_ptr[u + 1]; ++e) {
      int64_t t = inc[e] / 4;
      int a = (int)(inc[e] % 4);
      const int32_t* v = &tets[4 * t];
      TetGeom g;
      tet_geom(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], X + 3 * v[3], g);
      int r = c->region[t];
      double ms = c->Ms[r], A = c->Aex[r];
      mu += ms * g.V / 4.0;
      for (int b = 0; b < 4; ++b) {
        size_t j = std::lower_bound(cols.begin(), cols.end(), uk[v[b]]) - cols.begin();
        double dot = g.g[a][0] * g.g[b][0] + g.g[a][1] * g.g[b][1] + g.g[a][2] * g.g[b][2];
        K[j] += A * g.V * dot;
        for (int i = 0; i < 3; ++i) {
          D[3 * j + i] += ms * g.V / 4.0 * g.g[a][i];
          G[3 * j + i] += ms * g.V / 4.0 * g.g[b][i];
        }
      }
    }
    o.mu[u] = mu;
    int64_t base = o.loc_rowptr[u];
    for (size_t j = 0; j < nc; ++j) {
      o.loc_col[base + j] = (int32_t)cols[j];
      float* w = &o.loc_val[8 * (base + j)];
      w[0] = (float)(-2.0 * K[j] / (kMu0 * mu));
      for (int i = 0; i < 3; ++i) {
        w[1 + i] = (float)D[3 * j + i];
        w[4 + i] = (float)(G[3 * j + i] / mu);
      }
      w[7] = 0.0f;
    }
  }, 1024);

  // ---- surface faces (for the element-exact correction) ---------------------
  // face (t, a) = the face opposite local vertex a; bucket faces by their
  // smallest LCA unknown, then match the remaining pair inside each bucket.
  std::vector<uint8_t> surface(4 * T, 1);
  {
    std::vector<int64_t> fptr(Np + 1, 0);
    auto fkey = [&](int64_t t, int a, int64_t k[3]) {
      int q = 0;
      for (int b = 0; b < 4; ++b)
        if (b != a) k[q++] = uk[tets[4 * t + b]];
      std::sort(k, k + 3);
    };
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) {
        int64_t k[3];
        fkey(t, a, k);
        fptr[k[0] + 1]++;
      }
    for (int64_t u = 0; u < Np; ++u) fptr[u + 1] += fptr[u];
    std::vector<int64_t> faces(fptr[Np]);
    std::vector<int64_t> fill(fptr.begin(), fptr.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) {
        int64_t k[3];
        fkey(t, a, k);
        faces[fill[k[0]]++] = 4 * t + a;
      }
    std::atomic<int> tri(0);
    parallel_for(Np, [&](int64_t u) {
      int64_t b0 = fptr[u], b1 = fptr[u + 1];
      std::vector<std::pair<std::pair<int64_t, int64_t>, int64_t>> lst;
      for (int64_t i = b0; i < b1; ++i) {
        int64_t k[3];
        fkey(faces[i] / 4, (int)(faces[i] % 4), k);
        lst.push_back({{k[1], k[2]}, faces[i]});
      }
      std::sort(lst.begin(), lst.end());
      for (size_t i = 0; i < lst.size();) {
        size_t j = i + 1;
        while (j < lst.size() && lst[j].first == lst[i].first) ++j;
        if (j - i > 2) tri = 1;
        if (j - i == 2) {
          int64_t f1 = lst[i].second, f2 = lst[i + 1].second;
          if (c->region[f1 / 4] == c->region[f2 / 4]) {
            surface[f1] = 0;
            surface[f2] = 0;
          }
        }
        i = j;
      }
    }, 1024);
    if (tri) return fail(c, PMFEM_EMESH, "a face is shared by more than two tetrahedra");
  }
  // mean edge length over the unique edges of the input mesh
  {
    std::vector<int64_t> eptr(N + 1, 0);
    static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int64_t t = 0; t < T; ++t)
      for (int e = 0; e < 6; ++e)
        eptr[std::min(tets[4 * t + E[e][0]], tets[4 * t + E[e][1]]) + 1]++;
    for (int64_t n = 0; n < N; ++n) eptr[n + 1] += eptr[n];
    std::vector<int32_t> other(eptr[N]);
    std::vector<int64_t> fill(eptr.begin(), eptr.end() - 1);
    for (int64_t t = 0; t < T; ++t)
      for (int e = 0; e < 6; ++e) {
        int32_t a = tets[4 * t + E[e][0]], b = tets[4 * t + E[e][1]];
        other[fill[std::min(a, b)]++] = std::max(a, b);
      }
    std::vector<double> sum(N, 0.0);
    std::vector<int64_t> cnt(N, 0);
    parallel_for(N, [&](int64_t n) {
      std::sort(other.begin() + eptr[n], other.begin() + eptr[n + 1]);
      int32_t prev = -1;
      for (int64_t i = eptr[n]; i < eptr[n + 1]; ++i) {
        if (other[i] == prev) continue;
        prev = other[i];
        double d0 = X[3 * n] - X[3 * prev], d1 = X[3 * n + 1] - X[3 * prev + 1],
               d2 = X[3 * n + 2] - X[3 * prev + 2];
        sum[n] += std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        cnt[n]++;
      }
    }, 4096);
    double S = 0.0;
    int64_t C = 0;
    for (int64_t n = 0; n < N; ++n) {
      S += sum[n];
      C += cnt[n];
    }
    o.hbar = S / (double)C;
  }

  // ---- 4. grid kernel and spectrum -------------------------------------------
  {
    int Mx = o.M[0], My = o.M[1], Mz = o.M[2];
    // distinct |offset| per axis
    int na[3];
    for (int a = 0; a < 3; ++a) na[a] = o.per[a] ? o.N[a] / 2 + 1 : o.N[a];
    std::vector<double> rr(3 * (size_t)na[0] * na[1] * na[2]);
    for (int k = 0; k < na[2]; ++k)
      for (int j = 0; j < na[1]; ++j)
        for (int i = 0; i < na[0]; ++i) {
          size_t idx = ((size_t)k * na[1] + j) * na[0] + i;
          rr[3 * idx] = i * o.delta[0];
          rr[3 * idx + 1] = j * o.delta[1];
          rr[3 * idx + 2] = k * o.delta[2];
        }
    std::vector<double> tab(rr.size() / 3);
    pgf_eval(c->mask, c->L, 0.0, (int64_t)tab.size(), rr.data(), tab.data());
    auto offset = [&](int a, int i) -> int {
      if (o.per[a]) return i <= o.N[a] / 2 ? i : o.N[a] - i;
      if (i < o.N[a]) return i;
      if (i == o.N[a]) return -1;  // unused padding slot
      return o.M[a] - i;
    };
    o.kgrid.assign((size_t)Mx * My * Mz, 0.0);
    for (int k = 0; k < Mz; ++k)
      for (int j = 0; j < My; ++j)
        for (int i = 0; i < Mx; ++i) {
          int di = offset(0, i), dj = offset(1, j), dk = offset(2, k);
          if (di < 0 || dj < 0 || dk < 0) continue;
          o.kgrid[((size_t)k * My + j) * Mx + i] = tab[((size_t)dk * na[1] + dj) * na[0] + di];
        }
    std::vector<double> re(o.kgrid), im(re.size(), 0.0);
    fft3_inplace(re, im, o.M);
    int Hx = Mx / 2 + 1;
    o.khat.resize((size_t)Hx * My * Mz);
    double sc = 1.0 / (4.0 * kPi * (double)Mx * My * Mz);
    for (int k = 0; k < Mz; ++k)
      for (int j = 0; j < My; ++j)
        for (int i = 0; i < Hx; ++i)
          o.khat[((size_t)k * My + j) * Hx + i] = (float)(re[((size_t)k * My + j) * Mx + i] * sc);
  }

  // ---- 5. precorrection -----------------------------------------------------
  {
    const int R = rb + p;            // K0 table half-width
    const int TW = 2 * R + 1;
    const int E = 2 * rb + p + 1;    // Phi extent per axis, offsets [-rb, rb + p]
    std::vector<double> K0((size_t)TW * TW * TW);
    for (int z = -R; z <= R; ++z)
      for (int y = -R; y <= R; ++y)
        for (int x = -R; x <= R; ++x) {
          double d0 = x * o.delta[0], d1 = y * o.delta[1], d2 = z * o.delta[2];
          double d = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
          K0[((size_t)(z + R) * TW + (y + R)) * TW + (x + R)] = d > 0 ? 1.0 / d : 0.0;
        }
    auto weights = [&](int64_t u, double w[3][8]) {
      for (int a = 0; a < 3; ++a) {
        double xi = s[3 * u + a] - stu[3 * u + a];
        for (int i = 0; i <= p; ++i) {
          double v = 1.0;
          for (int j = 0; j <= p; ++j)
            if (j != i) v *= (xi - j) / (double)(i - j);
          w[a][i] = v;
        }
      }
    };
    // near boxes of u: per axis list of (target box, wraps, offset d)
    auto near_axis = [&](int64_t u, int a, int tb[16], int wr[16], int dd[16]) -> int {
      int n = 0;
      for (int d = -rb; d <= rb; ++d) {
        int t = bx[3 * u + a] + d;
        int w = 0;
        if (o.per[a]) {
          w = (int)std::floor((double)t / o.N[a]);
          t -= w * o.N[a];
        } else if (t < 0 || t >= o.nbox[a]) {
          continue;
        }
        tb[n] = t;
        wr[n] = w;
        dd[n] = d;
        ++n;
      }
      return n;
    };
    std::vector<int32_t> plen(Np);
    parallel_for(Np, [&](int64_t u) {
      int tb[3][16], wr[3][16], dd[3][16], cnt[3];
      for (int a = 0; a < 3; ++a) cnt[a] = near_axis(u, a, tb[a], wr[a], dd[a]);
      int64_t tot = 0;
      for (int iz = 0; iz < cnt[2]; ++iz)
        for (int iy = 0; iy < cnt[1]; ++iy)
          for (int ix = 0; ix < cnt[0]; ++ix) {
            int64_t b = ((int64_t)tb[2][iz] * o.nbox[1] + tb[1][iy]) * o.nbox[0] + tb[0][ix];
            tot += o.box_start[b + 1] - o.box_start[b];
          }
      plen[u] = (int32_t)tot;
    }, 1024);
    o.p_rowptr.assign(Np + 1, 0);
    int64_t acc = 0;
    for (int64_t u = 0; u < Np; ++u) {
      acc += plen[u];
      if (acc > 2147483647LL) return fail(c, PMFEM_ENOMEM, "precorrection exceeds 2^31 entries");
      o.p_rowptr[u + 1] = (int32_t)acc;
    }
    o.p_col.resize(acc);
    o.p_val.resize(acc);
    const double inv4pi = 1.0 / (4.0 * kPi);
    parallel_for(Np, [&](int64_t u) {
      double w[3][8];
      weights(u, w);
      // Phi(e) = sum_a W_u(a) K0(a - e), e in [-rb, rb+p]^3, separable in 3 passes
      std::vector<double> t1((size_t)TW * TW * E), t2((size_t)TW * E * E), phi((size_t)E * E * E);
      for (int x = 0; x < TW; ++x)
        for (int y = 0; y < TW; ++y)
          for (int ez = 0; ez < E; ++ez) {
            double v = 0.0;
            for (int az = 0; az <= p; ++az) {
              int dz = az - (ez - rb);  // az - e_z, e_z = ez - rb
              v += w[2][az] * K0[((size_t)(dz + R) * TW + y) * TW + x];
            }
            t1[((size_t)x * TW + y) * E + ez] = v;
          }
      for (int x = 0; x < TW; ++x)
        for (int ey = 0; ey < E; ++ey)
          for (int ez = 0; ez < E; ++ez) {
            double v = 0.0;
            for (int ay = 0; ay <= p; ++ay) {
              int dy = ay - (ey - rb);
              v += w[1][ay] * t1[((size_t)x * TW + (dy + R)) * E + ez];
            }
            t2[((size_t)x * E + ey) * E + ez] = v;
          }
      for (int ex = 0; ex < E; ++ex)
        for (int ey = 0; ey < E; ++ey)
          for (int ez = 0; ez < E; ++ez) {
            double v = 0.0;
            for (int ax = 0; ax <= p; ++ax) {
              int dx = ax - (ex - rb);
              v += w[0][ax] * t2[((size_t)(dx + R) * E + ey) * E + ez];
            }
            phi[((size_t)ex * E + ey) * E + ez] = v;
          }
      double xn[3];
      for (int a = 0; a < 3; ++a) xn[a] = o.origin[a] + s[3 * u + a] * o.delta[a];
      int tb[3][16], wr[3][16], dd[3][16], cnt[3];
      for (int a = 0; a < 3; ++a) cnt[a] = near_axis(u, a, tb[a], wr[a], dd[a]);
      int64_t out = o.p_rowptr[u];
      // column order: x box offset outermost, then z, then y, then node order
      for (int ix = 0; ix < cnt[0]; ++ix)
        for (int iz = 0; iz < cnt[2]; ++iz)
          for (int iy = 0; iy < cnt[1]; ++iy) {
            int64_t b = ((int64_t)tb[2][iz] * o.nbox[1] + tb[1][iy]) * o.nbox[0] + tb[0][ix];
            for (int32_t k = o.box_start[b]; k < o.box_start[b + 1]; ++k) {
              double wk[3][8];
              weights(k, wk);
              int e0[3];
              double dist2 = 0.0;
              const int* wrs[3] = {&wr[0][ix], &wr[1][iy], &wr[2][iz]};
              for (int a = 0; a < 3; ++a) {
                int stk = stu[3 * k + a];
                if (o.per[a]) stk += *wrs[a] * o.N[a];
                e0[a] = stk - stu[3 * u + a] + rb;   // index into Phi
                double xk = o.origin[a] + s[3 * k + a] * o.delta[a] + *wrs[a] * c->L[a] * o.per[a];
                double dlt = xn[a] - xk;
                dist2 += dlt * dlt;
              }
              double conv = 0.0;
              for (int ax = 0; ax <= p; ++ax)
                for (int ay = 0; ay <= p; ++ay) {
                  const double* row = &phi[((size_t)(e0[0] + ax) * E + (e0[1] + ay)) * E + e0[2]];
                  double v = 0.0;
                  for (int az = 0; az <= p; ++az) v += wk[2][az] * row[az];
                  conv += wk[0][ax] * wk[1][ay] * v;
                }
              double g0 = (k == u) ? 0.0 : 1.0 / std::sqrt(dist2);
              o.p_col[out] = k;
              o.p_val[out] = (float)((g0 - conv) * inv4pi);
              ++out;
            }
          }
    }, 256);
  }

  // ---- 6. element-exact correction --------------------------------------------
  int rc = build_z0(c, surface);
  if (rc != PMFEM_OK) return rc;
  return PMFEM_OK;
}

}  // namespace pmfem
