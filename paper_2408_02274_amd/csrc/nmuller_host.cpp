// Host-side N-Mueller plan: surface quantities and near-field corrections.
//
// Singular moments follow Sec. III-D: closest point by golden-section search
// (eq. dist_min), Kress's sigmoidal map (eq. mk_cov_1, mk_cov_2), the
// clustering maps xi_alpha (eq. cov) and the mapped Fejer rule of
// eq. int_moments_cov; the Chebyshev expansion of the density (eq. phi_cheby,
// rp_exp) turns moments into nodal weights, and the local correction of
// Sec. III-H subtracts what the regular Fejer sum already counts.
#include "nmuller_host.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace ifgf {

namespace {

const double kPi = 3.141592653589793;
const double kGold = (std::sqrt(5.0) - 1.0) / 2.0;
using cd = std::complex<double>;

void cheb_nodes(int n, double* x) {
  for (int k = 0; k < n; ++k) x[k] = std::cos((k + 0.5) * kPi / n);
}

void fejer(int n, double* w) {
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int m = 1; m <= n / 2; ++m) s += std::cos(m * kPi * (2 * k + 1) / n) / (4.0 * m * m - 1.0);
    w[k] = (2.0 / n) * (1.0 - 2.0 * s);
  }
}

// T_0..T_{n-1}(x) and T'_0..T'_{n-1}(x)
inline void chebT(int n, double x, double* T, double* dT) {
  T[0] = 1.0;
  if (n > 1) T[1] = x;
  for (int k = 2; k < n; ++k) T[k] = 2.0 * x * T[k - 1] - T[k - 2];
  if (dT) {
    // T'_k = k U_{k-1}
    double um2 = 0.0, um1 = 1.0;  // U_{-1} = 0, U_0 = 1
    dT[0] = 0.0;
    for (int k = 1; k < n; ++k) {
      dT[k] = k * um1;
      double u = 2.0 * x * um1 - um2;
      um2 = um1;
      um1 = u;
    }
  }
}

// M[m][i] = (2/n) c_m T_m(x_i), c_0 = 1/2: node values -> coefficients
void transform_matrix(int n, std::vector<double>& M) {
  std::vector<double> x(n), T(n);
  cheb_nodes(n, x.data());
  M.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    chebT(n, x[i], T.data(), nullptr);
    for (int m = 0; m < n; ++m) M[m * n + i] = (2.0 / n) * (m == 0 ? 0.5 : 1.0) * T[m];
  }
}

// x^d for a small integer d >= 1 by repeated multiplication (the device
// builder forms the same products in the same order)
inline double ipow(double x, int d) {
  double p = x;
  for (int k = 1; k < d; ++k) p = p * x;
  return p;
}

// Kress map (eq. mk_cov_1, mk_cov_2) and its derivative
inline double knu(double t, int d) {
  double a = (kPi - t) / kPi;
  return (1.0 / d - 0.5) * a * a * a + (1.0 / d) * ((t - kPi) / kPi) + 0.5;
}
inline double kdnu(double t, int d) {
  double a = (kPi - t) / kPi;
  return -(3.0 / kPi) * (1.0 / d - 0.5) * a * a + 1.0 / (d * kPi);
}
inline double kw(double t, int d) {
  double a = ipow(knu(t, d), d), b = ipow(knu(2 * kPi - t, d), d);
  return 2 * kPi * a / (a + b);
}
inline double kdw(double t, int d) {
  double n1 = knu(t, d), n2 = knu(2 * kPi - t, d);
  double a = ipow(n1, d), b = ipow(n2, d);
  double da = d * ipow(n1, d - 1) * kdnu(t, d);
  double db = -d * ipow(n2, d - 1) * kdnu(2 * kPi - t, d);
  return 2 * kPi * (da * b - a * db) / ((a + b) * (a + b));
}

// clustering map xi_alpha (eq. cov): value and derivative at tau in [-1, 1]
inline void xi(double al, double t, int d, double* u, double* mu) {
  if (al == 1.0) {
    *u = al - ((1.0 + al) / kPi) * kw(kPi * std::fabs((t - 1.0) / 2.0), d);
    *mu = kdw(kPi * (1.0 - t) / 2.0, d);
  } else if (al == -1.0) {
    *u = al + ((1.0 - al) / kPi) * kw(kPi * std::fabs((t + 1.0) / 2.0), d);
    *mu = kdw(kPi * (1.0 + t) / 2.0, d);
  } else {
    double sg = (t > 0) - (t < 0);
    *u = al + ((sg - al) / kPi) * kw(kPi * std::fabs(t), d);
    *mu = (1.0 - al * sg) * kdw(kPi * std::fabs(t), d);
  }
}

struct PatchInterp {
  int nc;
  const double* A;  // [nc][nc][3]
  void eval(double u, double v, double* X) const {
    double Tu[16], Tv[16];
    chebT(nc, u, Tu, nullptr);
    chebT(nc, v, Tv, nullptr);
    X[0] = X[1] = X[2] = 0.0;
    for (int m = 0; m < nc; ++m)
      for (int n = 0; n < nc; ++n) {
        double t = Tu[m] * Tv[n];
        const double* a = A + 3 * (m * nc + n);
        X[0] += t * a[0];
        X[1] += t * a[1];
        X[2] += t * a[2];
      }
  }
  double dist2(const double* x, double u, double v) const {
    double X[3];
    eval(u, v, X);
    double a = x[0] - X[0], b = x[1] - X[1], c = x[2] - X[2];
    return a * a + b * b + c * c;
  }
};

template <class F>
double golden(F f, double lo, double hi, int iters) {
  double a = lo, b = hi;
  double c = b - kGold * (b - a), d = a + kGold * (b - a);
  double fc = f(c), fd = f(d);
  for (int it = 0; it < iters; ++it) {
    if (fc < fd) {
      b = d;
      d = c;
      fd = fc;
      c = b - kGold * (b - a);
      fc = f(c);
    } else {
      a = c;
      c = d;
      fc = fd;
      d = a + kGold * (b - a);
      fd = f(d);
    }
  }
  return 0.5 * (a + b);
}

}  // namespace

int build_surface(SurfaceGeo& g, int P, int nc, const double* x, const double* du,
                  const double* dv, std::string& err) {
  if (P < 1 || nc < 2 || nc > 16) {
    err = "need P >= 1 and 2 <= Nc <= 16";
    return -1;
  }
  g.P = P;
  g.nc = nc;
  g.n = (int64_t)P * nc * nc;
  const int64_t n = g.n;
  g.x.assign(x, x + 3 * n);
  g.du.assign(du, du + 3 * n);
  g.dv.assign(dv, dv + 3 * n);
  g.nrm.resize(3 * n);
  g.t1.resize(3 * n);
  g.t2.resize(3 * n);
  g.J.resize(n);
  g.w.resize(n);
  g.Q.resize(4 * n);
  g.gu.resize(3 * n);
  g.gv.resize(3 * n);
  std::vector<double> wf(nc);
  fejer(nc, wf.data());
  for (int64_t l = 0; l < n; ++l) {
    const double* a = &du[3 * l];
    const double* b = &dv[3 * l];
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double J = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(J > 0.0) || !std::isfinite(J)) {
      err = "degenerate parametrisation (|d_u eta x d_v eta| = 0) at node " + std::to_string(l);
      return -1;
    }
    double* nn = &g.nrm[3 * l];
    for (int k = 0; k < 3; ++k) nn[k] = c[k] / J;
    g.J[l] = J;
    int loc = (int)(l % (nc * nc));
    g.w[l] = wf[loc / nc] * wf[loc % nc] * J;
    double la = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double* t1 = &g.t1[3 * l];
    double* t2 = &g.t2[3 * l];
    for (int k = 0; k < 3; ++k) t1[k] = a[k] / la;
    t2[0] = nn[1] * t1[2] - nn[2] * t1[1];
    t2[1] = nn[2] * t1[0] - nn[0] * t1[2];
    t2[2] = nn[0] * t1[1] - nn[1] * t1[0];
    double guu = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    double guv = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double gvv = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double det = guu * gvv - guv * guv;
    double iuu = gvv / det, iuv = -guv / det, ivv = guu / det;
    for (int k = 0; k < 3; ++k) {
      g.gu[3 * l + k] = iuu * a[k] + iuv * b[k];
      g.gv[3 * l + k] = iuv * a[k] + ivv * b[k];
    }
    // b_u = a.du = c1 t1.du + c2 t2.du ; b_v = c1 t1.dv + c2 t2.dv
    double t1u = t1[0] * a[0] + t1[1] * a[1] + t1[2] * a[2];
    double t2u = t2[0] * a[0] + t2[1] * a[1] + t2[2] * a[2];
    double t1v = t1[0] * b[0] + t1[1] * b[1] + t1[2] * b[2];
    double t2v = t2[0] * b[0] + t2[1] * b[1] + t2[2] * b[2];
    // (a^u, a^v) = Ginv (b_u, b_v); Q = J Ginv [[t1u, t2u], [t1v, t2v]]
    g.Q[4 * l + 0] = J * (iuu * t1u + iuv * t1v);
    g.Q[4 * l + 1] = J * (iuu * t2u + iuv * t2v);
    g.Q[4 * l + 2] = J * (iuv * t1u + ivv * t1v);
    g.Q[4 * l + 3] = J * (iuv * t2u + ivv * t2v);
  }
  // differentiation matrix: values -> coefficients -> derivative recurrence -> values
  std::vector<double> M;
  transform_matrix(nc, M);
  std::vector<double> xn(nc), T(nc);
  cheb_nodes(nc, xn.data());
  g.Dcheb.assign(nc * nc, 0.0);
  for (int col = 0; col < nc; ++col) {
    std::vector<double> c(nc), d(nc + 1, 0.0);
    for (int m = 0; m < nc; ++m) c[m] = M[m * nc + col];
    for (int m = nc - 1; m >= 2; --m) d[m - 1] = d[m + 1] + 2.0 * m * c[m];
    if (nc > 1) d[0] = c[1] + 0.5 * d[2];
    for (int i = 0; i < nc; ++i) {
      chebT(nc, xn[i], T.data(), nullptr);
      double s = 0.0;
      for (int m = 0; m < nc; ++m) s += d[m] * T[m];
      g.Dcheb[i * nc + col] = s;
    }
  }
  return 0;
}

int sing_tables(const SurfaceGeo& g, const SingParams& sp, SingTables& t, std::string& err) {
  const int nc = g.nc, P = g.P;
  const int nq = nc * nc;
  t.nb = sp.nbeta > 0 ? sp.nbeta : 6 * nc;
  if (t.nb > 128) {
    err = "nbeta must be <= 128";
    return -1;
  }
  transform_matrix(nc, t.M);
  t.tn.resize(nc);
  t.tb.resize(t.nb);
  t.wb.resize(t.nb);
  cheb_nodes(nc, t.tn.data());
  cheb_nodes(t.nb, t.tb.data());
  fejer(t.nb, t.wb.data());
  t.gold = kGold;
  // per patch: Chebyshev coefficients of the node coordinates, bounding box, delta
  t.A.assign((size_t)P * nq * 3, 0.0);
  t.lo.resize(3 * (size_t)P);
  t.hi.resize(3 * (size_t)P);
  t.delta.resize(P);
  const std::vector<double>& M = t.M;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < P; ++p) {
    const double* xp = &g.x[(size_t)3 * p * nq];
    std::vector<double> tmp((size_t)nq * 3, 0.0);
    for (int m = 0; m < nc; ++m)          // tmp[m][j] = sum_i M[m][i] x[i][j]
      for (int j = 0; j < nc; ++j)
        for (int i = 0; i < nc; ++i)
          for (int c = 0; c < 3; ++c) tmp[3 * (m * nc + j) + c] += M[m * nc + i] * xp[3 * (i * nc + j) + c];
    double* Ap = &t.A[(size_t)3 * p * nq];
    for (int m = 0; m < nc; ++m)
      for (int nn = 0; nn < nc; ++nn) {
        double s[3] = {0, 0, 0};
        for (int j = 0; j < nc; ++j)
          for (int c = 0; c < 3; ++c) s[c] += M[nn * nc + j] * tmp[3 * (m * nc + j) + c];
        for (int c = 0; c < 3; ++c) Ap[3 * (m * nc + nn) + c] = s[c];
      }
    double* lo = &t.lo[3 * (size_t)p];
    double* hi = &t.hi[3 * (size_t)p];
    for (int c = 0; c < 3; ++c) {
      lo[c] = hi[c] = xp[c];
      for (int q = 0; q < nq; ++q) {
        lo[c] = std::min(lo[c], xp[3 * q + c]);
        hi[c] = std::max(hi[c], xp[3 * q + c]);
      }
    }
    double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
    t.delta[p] = sp.delta_factor * std::sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  }
  return 0;
}

int build_corrections(const SurfaceGeo& g, double k_int, double k_ext, const SingParams& sp,
                      Corrections& cor, std::string& err) {
  const int nc = g.nc, P = g.P;
  const int nq = nc * nc;
  const int64_t n = g.n;
  const int d = sp.d;
  SingTables t;
  if (sing_tables(g, sp, t, err)) return -1;
  const int nb = t.nb;
  const std::vector<double>& M = t.M;
  const std::vector<double>& tn = t.tn;
  const std::vector<double>& tb = t.tb;
  const std::vector<double>& wb = t.wb;
  const std::vector<double>& A = t.A;
  const std::vector<double>& lo = t.lo;
  const std::vector<double>& hi = t.hi;
  const std::vector<double>& delta = t.delta;

  // pass 1: singular pairs with their closest points
  std::vector<std::vector<int32_t>> rp(n);
  std::vector<std::vector<double>> ruv(n);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t l = 0; l < n; ++l) {
    const double* xl = &g.x[3 * l];
    for (int p = 0; p < P; ++p) {
      double gap2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        double gg = std::max(0.0, std::max(lo[3 * p + c] - xl[c], xl[c] - hi[3 * p + c]));
        gap2 += gg * gg;
      }
      if (std::sqrt(gap2) > 1.5 * delta[p]) continue;
      const double* xp = &g.x[(size_t)3 * p * nq];
      double u, v, dist;
      bool own = (l / nq) == p;
      if (own) {
        int loc = (int)(l % nq);
        u = tn[loc / nc];
        v = tn[loc % nc];
        dist = 0.0;
      } else {
        int kbest = 0;
        double best = 0.0;
        for (int q = 0; q < nq; ++q) {
          double a = xp[3 * q] - xl[0], b = xp[3 * q + 1] - xl[1], c = xp[3 * q + 2] - xl[2];
          double d2 = a * a + b * b + c * c;
          if (q == 0 || d2 < best) {
            best = d2;
            kbest = q;
          }
        }
        int i0 = kbest / nc, j0 = kbest % nc;
        double lo_u = (i0 + 1 < nc) ? tn[i0 + 1] : -1.0, hi_u = (i0 > 0) ? tn[i0 - 1] : 1.0;
        double lo_v = (j0 + 1 < nc) ? tn[j0 + 1] : -1.0, hi_v = (j0 > 0) ? tn[j0 - 1] : 1.0;
        PatchInterp pi{nc, &A[(size_t)3 * p * nq]};
        u = tn[i0];
        v = tn[j0];
        for (int s = 0; s < sp.sweeps; ++s) {
          u = golden([&](double uu) { return pi.dist2(xl, uu, v); }, lo_u, hi_u, sp.iters);
          v = golden([&](double vv) { return pi.dist2(xl, u, vv); }, lo_v, hi_v, sp.iters);
        }
        if (std::fabs(1.0 - std::fabs(u)) < 1e-6) u = u > 0 ? 1.0 : -1.0;
        if (std::fabs(1.0 - std::fabs(v)) < 1e-6) v = v > 0 ? 1.0 : -1.0;
        dist = std::sqrt(pi.dist2(xl, u, v));
      }
      if (dist <= delta[p]) {
        rp[l].push_back(p);
        ruv[l].push_back(u);
        ruv[l].push_back(v);
      }
    }
  }
  cor.nc = nc;
  cor.row_off.assign(n + 1, 0);
  for (int64_t l = 0; l < n; ++l) cor.row_off[l + 1] = cor.row_off[l] + (int64_t)rp[l].size();
  const int64_t npairs = cor.row_off[n];
  cor.pair_patch.resize(npairs);
  cor.vals.assign((size_t)npairs * 4 * nq * 2, 0.0);
  for (int64_t l = 0; l < n; ++l)
    std::copy(rp[l].begin(), rp[l].end(), cor.pair_patch.begin() + cor.row_off[l]);

  // pass 2: moments -> nodal weights -> corrections
  const double kk[2] = {k_int, k_ext};
  int bad = 0;
#pragma omp parallel reduction(+ : bad)
  {
    std::vector<double> U(nb), MU(nb), V(nb), MV(nb), Tu(nb * nc), dTu(nb * nc), Tv(nb * nc), dTv(nb * nc);
    std::vector<double> Bx(nb * nc * 3), Bu(nb * nc * 3);
    std::vector<cd> F(4 * nb * nb), Gm(4 * nb * nc), beta(4 * nq), tmp(4 * nq);
#pragma omp for schedule(dynamic, 16)
    for (int64_t l = 0; l < n; ++l) {
      const double* xl = &g.x[3 * l];
      const double* nl = &g.nrm[3 * l];
      for (int64_t e = cor.row_off[l]; e < cor.row_off[l + 1]; ++e) {
        int p = cor.pair_patch[e];
        double ua = ruv[l][2 * (e - cor.row_off[l])], va = ruv[l][2 * (e - cor.row_off[l]) + 1];
        const double* Ap = &A[(size_t)3 * p * nq];
        for (int i = 0; i < nb; ++i) {
          xi(ua, tb[i], d, &U[i], &MU[i]);
          xi(va, tb[i], d, &V[i], &MV[i]);
          chebT(nc, U[i], &Tu[i * nc], &dTu[i * nc]);
          chebT(nc, V[i], &Tv[i * nc], &dTv[i * nc]);
        }
        // Bx[i][n] = sum_m T_m(U_i) A[m][n], Bu with T'_m
        for (int i = 0; i < nb; ++i)
          for (int nn = 0; nn < nc; ++nn)
            for (int c = 0; c < 3; ++c) {
              double s = 0.0, su = 0.0;
              for (int m = 0; m < nc; ++m) {
                s += Tu[i * nc + m] * Ap[3 * (m * nc + nn) + c];
                su += dTu[i * nc + m] * Ap[3 * (m * nc + nn) + c];
              }
              Bx[(i * nc + nn) * 3 + c] = s;
              Bu[(i * nc + nn) * 3 + c] = su;
            }
        for (int i = 0; i < nb; ++i)
          for (int j = 0; j < nb; ++j) {
            double Y[3] = {0, 0, 0}, Yu[3] = {0, 0, 0}, Yv[3] = {0, 0, 0};
            for (int nn = 0; nn < nc; ++nn) {
              double tv = Tv[j * nc + nn], dtv = dTv[j * nc + nn];
              for (int c = 0; c < 3; ++c) {
                Y[c] += Bx[(i * nc + nn) * 3 + c] * tv;
                Yu[c] += Bu[(i * nc + nn) * 3 + c] * tv;
                Yv[c] += Bx[(i * nc + nn) * 3 + c] * dtv;
              }
            }
            double cr0 = Yu[1] * Yv[2] - Yu[2] * Yv[1], cr1 = Yu[2] * Yv[0] - Yu[0] * Yv[2],
                   cr2 = Yu[0] * Yv[1] - Yu[1] * Yv[0];
            double Jq = std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2);
            double dx = xl[0] - Y[0], dy = xl[1] - Y[1], dz = xl[2] - Y[2];
            double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            double nd = nl[0] * dx + nl[1] * dy + nl[2] * dz;
            double wgt = Jq * (MU[i] * wb[i]) * (MV[j] * wb[j]);
            for (int q = 0; q < 2; ++q) {
              cd G = std::exp(cd(0.0, kk[q] * r)) / (4.0 * kPi * r);
              cd KD = G * cd(-1.0 / r, kk[q]) * nd / r;
              F[(q * nb + i) * nb + j] = G * wgt;
              F[((2 + q) * nb + i) * nb + j] = KD * wgt;
            }
          }
        // beta_k[m][n] = sum_i Tu[i][m] sum_j F_k[i][j] Tv[j][n]
        for (int k = 0; k < 4; ++k) {
          for (int i = 0; i < nb; ++i)
            for (int nn = 0; nn < nc; ++nn) {
              cd s = 0.0;
              for (int j = 0; j < nb; ++j) s += F[(k * nb + i) * nb + j] * Tv[j * nc + nn];
              Gm[(k * nb + i) * nc + nn] = s;
            }
          for (int m = 0; m < nc; ++m)
            for (int nn = 0; nn < nc; ++nn) {
              cd s = 0.0;
              for (int i = 0; i < nb; ++i) s += Tu[i * nc + m] * Gm[(k * nb + i) * nc + nn];
              beta[k * nq + m * nc + nn] = s;
            }
          // W[i'][j'] = sum_m sum_n M[m][i'] beta[m][n] M[n][j']
          for (int m = 0; m < nc; ++m)
            for (int jj = 0; jj < nc; ++jj) {
              cd s = 0.0;
              for (int nn = 0; nn < nc; ++nn) s += beta[k * nq + m * nc + nn] * M[nn * nc + jj];
              tmp[k * nq + m * nc + jj] = s;
            }
          for (int ii = 0; ii < nc; ++ii)
            for (int jj = 0; jj < nc; ++jj) {
              cd s = 0.0;
              for (int m = 0; m < nc; ++m) s += M[m * nc + ii] * tmp[k * nq + m * nc + jj];
              beta[k * nq + ii * nc + jj] = s;  // reuse as W
            }
        }
        // C = W - [q != l] w_q K(x_l, x_q)
        double* out = &cor.vals[(size_t)e * 4 * nq * 2];
        for (int qq = 0; qq < nq; ++qq) {
          int64_t gq = (int64_t)p * nq + qq;
          cd Kq[4] = {0.0, 0.0, 0.0, 0.0};
          if (gq != l) {
            const double* xq = &g.x[3 * gq];
            double dx = xl[0] - xq[0], dy = xl[1] - xq[1], dz = xl[2] - xq[2];
            double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r > 0.0)) {
              ++bad;
              continue;
            }
            double nd = nl[0] * dx + nl[1] * dy + nl[2] * dz;
            for (int q = 0; q < 2; ++q) {
              cd G = std::exp(cd(0.0, kk[q] * r)) / (4.0 * kPi * r);
              Kq[q] = G * g.w[gq];
              Kq[2 + q] = G * cd(-1.0 / r, kk[q]) * nd / r * g.w[gq];
            }
          }
          for (int k = 0; k < 4; ++k) {
            cd c = beta[k * nq + qq] - Kq[k];
            out[(k * nq + qq) * 2] = c.real();
            out[(k * nq + qq) * 2 + 1] = c.imag();
          }
        }
      }
    }
  }
  if (bad) {
    err = "duplicate surface points";
    return -1;
  }
  return 0;
}

}  // namespace ifgf
