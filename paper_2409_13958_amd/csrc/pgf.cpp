// Periodic Green's function of the Laplacian at zero Bloch phase, FP64.
//
// Paper Eq. 2 writes G^p as lattice sums of G0 = 1/|r|; at k0 = 0 they
// diverge, and the paper evaluates G^p with "exponentially convergent sums"
// from a reference it does not reproduce. Here the sums are regularised by
// Ewald splitting 1/r = erfc(eta r)/r + erf(eta r)/r: the first part is
// summed over the lattice in real space, the second over the reciprocal
// lattice (Poisson summation along the periodic axes). Dropped divergent
// pieces are constants that cancel for a neutral cell. Conventions:
//   3D: zero average over the cell (background -pi/(eta^2 V));
//   2D: far field -2 pi |z| / A along the normal;
//   1D: far field -(2/L) ln(rho / L) - gamma/L across the axis.
// A point on a lattice site returns lim (G - 1/r), the interaction of a
// charge with its own images.
#include <cmath>
#include <vector>

#include "internal.h"

namespace pmfem {
namespace {

constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kRealCut = 6.2;    // erfc(6.2) ~ 1e-18
constexpr double kRecipCut = 12.5;  // exp(-(12.5/2)^2) ~ 1e-17

// exp(x^2) erfc(x) for x >= 0, with a continued fraction in the tail.
double erfcx_pos(double x) {
  if (x < 2.5) return std::exp(x * x) * std::erfc(x);
  double t = x;
  for (int n = 80; n >= 1; --n) t = x + 0.5 * n / t;
  return 1.0 / (kSqrtPi * t);
}

// exp(k z) erfc(k / (2 eta) + eta z) without overflow.
double exp_erfc(double k, double z, double eta) {
  double a = k / (2.0 * eta) + eta * z;
  if (a >= 0.0) return std::exp(-k * k / (4.0 * eta * eta) - eta * eta * z * z) * erfcx_pos(a);
  return std::exp(k * z) * std::erfc(a);
}

// Ein(x) = E1(x) + gamma + ln x, an entire function.
double ein(double x) {
  if (x <= 2.0) {
    double term = x, sum = x;
    for (int k = 2; k < 60; ++k) {
      term *= -x / k;
      double add = term / k;
      sum += add;
      if (std::fabs(add) < 1e-18 * std::fabs(sum)) break;
    }
    return sum;
  }
  return -std::expint(-x) + kEulerGamma + std::log(x);
}

double e1(double x) { return -std::expint(-x); }

// Gauss-Legendre nodes/weights on [0, 1].
struct GL {
  std::vector<double> x, w;
  explicit GL(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        pp = n * (z * p1 - p0) / (z * z - 1.0);
        double dz = p1 / pp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      x[i] = 0.5 * (1.0 - z);
      w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
    }
  }
};

// J(k, rho) = int_0^eta exp(-k^2/(4 t^2) - rho^2 t^2) dt/t, written with
// t = eta exp(-s) as int_0^inf exp(-k^2 e^{2s}/(4 eta^2) - rho^2 eta^2 e^{-2s}) ds;
// the integrand dies double-exponentially, so [0, S] with Gauss-Legendre suffices.
double incomplete_k0(double k, double rho, double eta) {
  static const GL gl(96);
  double a = k * k / (4.0 * eta * eta);
  double S = 0.5 * std::log(45.0 / a);
  if (S < 0.25) S = 0.25;
  double b = rho * rho * eta * eta, sum = 0.0;
  for (size_t i = 0; i < gl.x.size(); ++i) {
    double s = S * gl.x[i];
    sum += gl.w[i] * std::exp(-a * std::exp(2.0 * s) - b * std::exp(-2.0 * s));
  }
  return S * sum;
}

struct Lattice {
  int dim = 0;
  int per[3] = {0, 0, 0};
  int pa[3] = {0, 0, 0};   // periodic axes
  int na[3] = {0, 0, 0};   // non-periodic axes
  double L[3] = {0, 0, 0};
  double eta = 0.0;
  std::vector<double> R;   // real-space lattice vectors [nR][3]
  std::vector<double> K;   // reciprocal vectors of one half space [nK][3]
  std::vector<double> Kw;  // their weights (both +-k already included)
  double rmax = 0.0;       // max |reduced r| covered by the real sum
};

Lattice make_lattice(uint32_t mask, const double L[3], double eta, double rcover) {
  Lattice lt;
  int ip = 0, in = 0;
  for (int a = 0; a < 3; ++a) {
    lt.per[a] = (mask >> a) & 1;
    lt.L[a] = L[a];
    if (lt.per[a]) lt.pa[ip++] = a; else lt.na[in++] = a;
  }
  lt.dim = ip;
  lt.eta = eta;
  lt.rmax = rcover;
  double reach = kRealCut / eta + rcover;
  int nmax[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    if (lt.per[a]) nmax[a] = (int)std::ceil(reach / L[a]) + 1;
  for (int i = -nmax[0]; i <= nmax[0]; ++i)
    for (int j = -nmax[1]; j <= nmax[1]; ++j)
      for (int k = -nmax[2]; k <= nmax[2]; ++k) {
        double v[3] = {i * L[0] * lt.per[0], j * L[1] * lt.per[1], k * L[2] * lt.per[2]};
        if (std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) <= reach + 1e-300) {
          lt.R.push_back(v[0]);
          lt.R.push_back(v[1]);
          lt.R.push_back(v[2]);
        }
      }
  double kcut = kRecipCut * eta;
  int mmax[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    if (lt.per[a]) mmax[a] = (int)std::ceil(kcut * L[a] / (2.0 * kPi)) + 1;
  for (int i = 0; i <= mmax[0]; ++i)
    for (int j = -mmax[1]; j <= mmax[1]; ++j)
      for (int k = -mmax[2]; k <= mmax[2]; ++k) {
        // one of each +-k pair: first non-zero index positive
        if (!(i > 0 || (i == 0 && (j > 0 || (j == 0 && k > 0))))) continue;
        double kv[3] = {lt.per[0] ? 2 * kPi * i / L[0] : 0.0, lt.per[1] ? 2 * kPi * j / L[1] : 0.0,
                        lt.per[2] ? 2 * kPi * k / L[2] : 0.0};
        if ((!lt.per[0] && i) || (!lt.per[1] && j) || (!lt.per[2] && k)) continue;
        double kk = std::sqrt(kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]);
        if (kk > kcut) continue;
        double w = 0.0;
        if (lt.dim == 3) {
          double V = L[0] * L[1] * L[2];
          w = 2.0 * (4.0 * kPi / V) * std::exp(-kk * kk / (4.0 * eta * eta)) / (kk * kk);
        } else if (lt.dim == 2) {
          double A = L[lt.pa[0]] * L[lt.pa[1]];
          w = 2.0 * (kPi / A) / kk;  // times the z-dependent bracket
        } else {
          w = 2.0 * (2.0 / L[lt.pa[0]]);  // (4/L) per m >= 1, half space already
        }
        lt.K.push_back(kv[0]);
        lt.K.push_back(kv[1]);
        lt.K.push_back(kv[2]);
        lt.Kw.push_back(w);
      }
  return lt;
}

double eval_one(const Lattice& lt, const double rin[3]) {
  double r[3] = {rin[0], rin[1], rin[2]};
  for (int a = 0; a < 3; ++a)
    if (lt.per[a]) r[a] -= lt.L[a] * std::nearbyint(r[a] / lt.L[a]);
  const double eta = lt.eta;
  bool origin = (r[0] == 0.0 && r[1] == 0.0 && r[2] == 0.0);
  // real space
  double real = 0.0;
  size_t nR = lt.R.size() / 3;
  for (size_t i = 0; i < nR; ++i) {
    double d0 = r[0] + lt.R[3 * i], d1 = r[1] + lt.R[3 * i + 1], d2 = r[2] + lt.R[3 * i + 2];
    double d = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (d == 0.0) continue;
    if (eta * d > kRealCut + 1.0) continue;
    real += std::erfc(eta * d) / d;
  }
  if (origin) real -= 2.0 * eta / kSqrtPi;
  double recip = 0.0;
  size_t nK = lt.Kw.size();
  if (lt.dim == 3) {
    for (size_t i = 0; i < nK; ++i)
      recip += lt.Kw[i] * std::cos(lt.K[3 * i] * r[0] + lt.K[3 * i + 1] * r[1] + lt.K[3 * i + 2] * r[2]);
    double V = lt.L[0] * lt.L[1] * lt.L[2];
    recip -= kPi / (eta * eta * V);
  } else if (lt.dim == 2) {
    double z = r[lt.na[0]];
    for (size_t i = 0; i < nK; ++i) {
      double kk = std::sqrt(lt.K[3 * i] * lt.K[3 * i] + lt.K[3 * i + 1] * lt.K[3 * i + 1] +
                            lt.K[3 * i + 2] * lt.K[3 * i + 2]);
      double ph = std::cos(lt.K[3 * i] * r[0] + lt.K[3 * i + 1] * r[1] + lt.K[3 * i + 2] * r[2]);
      recip += lt.Kw[i] * ph * (exp_erfc(kk, z, eta) + exp_erfc(kk, -z, eta));
    }
    double A = lt.L[lt.pa[0]] * lt.L[lt.pa[1]];
    recip -= (2.0 * kPi / A) * (z * std::erf(eta * z) + std::exp(-eta * eta * z * z) / (eta * kSqrtPi));
  } else {
    int a = lt.pa[0];
    double Lp = lt.L[a];
    double x = r[a];
    double rho = std::sqrt(r[lt.na[0]] * r[lt.na[0]] + r[lt.na[1]] * r[lt.na[1]]);
    for (size_t i = 0; i < nK; ++i) {
      double kk = lt.K[3 * i + a];
      double J = (rho == 0.0) ? 0.5 * e1(kk * kk / (4.0 * eta * eta)) : incomplete_k0(kk, rho, eta);
      recip += lt.Kw[i] * std::cos(kk * x) * J;
    }
    recip -= (ein(eta * eta * rho * rho) - std::log(eta * eta * Lp * Lp)) / Lp;
  }
  return real + recip;
}

}  // namespace

double pgf_default_eta(uint32_t mask, const double L[3]) {
  double prod = 1.0;
  int d = 0;
  for (int a = 0; a < 3; ++a)
    if ((mask >> a) & 1) {
      prod *= L[a];
      ++d;
    }
  if (d == 0) return 0.0;
  return 1.2 * kSqrtPi / std::pow(prod, 1.0 / d);
}

void pgf_eval(uint32_t mask, const double L[3], double eta, int64_t n, const double* r,
              double* out) {
  if (mask == 0) {
    for (int64_t i = 0; i < n; ++i) {
      double d = std::sqrt(r[3 * i] * r[3 * i] + r[3 * i + 1] * r[3 * i + 1] + r[3 * i + 2] * r[3 * i + 2]);
      out[i] = d > 0.0 ? 1.0 / d : 0.0;
    }
    return;
  }
  if (eta <= 0.0) eta = pgf_default_eta(mask, L);
  // largest reduced |r| to cover
  double cover = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
      double v = r[3 * i + a];
      if ((mask >> a) & 1) v -= L[a] * std::nearbyint(v / L[a]);
      s += v * v;
    }
    cover = std::max(cover, std::sqrt(s));
  }
  Lattice lt = make_lattice(mask, L, eta, cover);
  parallel_for(n, [&](int64_t i) { out[i] = eval_one(lt, r + 3 * i); }, 64);
}

}  // namespace pmfem

extern "C" int pmfem_pgf_eval(uint32_t axis_mask, const double L[3], double eta, int64_t n,
                              const double* r, double* out) {
  if (n < 0 || (n > 0 && (!r || !out)) || !L || axis_mask > 7) return PMFEM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (((axis_mask >> a) & 1) && !(L[a] > 0.0)) return PMFEM_EINVAL;
  pmfem::pgf_eval(axis_mask, L, eta, n, r, out);
  return PMFEM_OK;
}
