// Near-field corrections on gfx950 (Sec. III-B eq. patch_sing, Sec. III-D,
// Sec. III-H): the quadrature of the host builder, moved to the device so that
// a 1.6M-point surface needs seconds rather than minutes and its ~100 GB of
// FP64 weights never pass through host memory.
//
// Pass 1 (one thread per target x_l) decides for every patch p whether it is
// singular for x_l -- the distance from x_l to the patch surface, found by
// golden-section search on the patch's Chebyshev interpolant (eq. dist_min),
// is at most delta_p -- and keeps the closest point (u, v).  The decision is
// discrete, so it is taken with the host's operations in the host's order and
// with floating-point contraction off (the host library is compiled without
// it): +, -, * and sqrt round identically on both sides, and the pairs and
// closest points equal the host's bit for bit.  A count pass sizes the rows,
// a fill pass writes them.
//
// Pass 2 (one wavefront per target, its pairs in turn) maps the Fejer rule
// through the clustering maps xi_alpha (eq. cov; Kress's map eq. mk_cov_1,
// mk_cov_2), sums G and dG/dn against the Chebyshev basis of the patch
// (eq. int_moments_cov: lane i owns the Fejer row i, the column sum runs in
// registers), turns the moments into nodal weights with the values ->
// coefficients matrix (eq. phi_cheby, rp_exp) and subtracts what the regular
// Fejer sum already counts, w_q K(x_l, x_q) for q != l (Sec. III-H).  It too
// follows the host's operations and order with contraction off: the
// innermost Fejer points of a target's own patch lie ~1e-6 from it, where
// n . (x - y) is a difference of nearly equal numbers, and the D weights of
// that patch move by up to ~5e-4 of their largest entry when only the
// rounding of the geometry changes (FMA contraction alone does that).  So the
// geometry here rounds exactly as on the host, and the weights differ only
// through the last bits of sin and cos.
#include "corrections.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/ifgf.h"

namespace ifgf {
namespace {

constexpr double kPiD = 3.141592653589793;
constexpr int kMaxNb = 64;

struct SingDev {
  const double* x;     // [n][3] nodes, patch order
  const double* nrm;   // [n][3]
  const double* w;     // [n] regular weights w_i w_j J
  const double* A;     // [P][Nc^2][3] Chebyshev coefficients of eta_p
  const double* box;   // [P][8]: lo[3], hi[3], delta_p, 0
  const double* tn;    // [Nc] patch nodes
  const double* tb;    // [nb] Fejer nodes
  const double* wb;    // [nb] Fejer weights
  const double* M;     // [Nc][Nc] values -> coefficients
  int64_t n;
  int P, nb, d, sweeps, iters;
  double gold;
  double k[2];
};

// ---------------------------------------------------------------- pass 1
// T_0..T_{NC-1}(x) by the three-term recurrence.
template <int NC>
__device__ inline void cheb_exact(double x, double* T) {
#pragma clang fp contract(off)
  T[0] = 1.0;
  if (NC > 1) T[1] = x;
#pragma unroll
  for (int k = 2; k < NC; ++k) T[k] = 2.0 * x * T[k - 1] - T[k - 2];
}

// Squared distance from x to eta_p(u, v), eta_p the patch interpolant.  T_m(u)
// comes from the recurrence as the m loop advances (the loop stays rolled so
// that the coefficients are loaded per row instead of held in registers).
template <int NC>
__device__ inline double patch_dist2(const double* __restrict__ A, const double* x, double u, double v) {
#pragma clang fp contract(off)
  double Tv[NC];
  cheb_exact<NC>(v, Tv);
  double X0 = 0.0, X1 = 0.0, X2 = 0.0;
  double tm2 = 0.0, tm1 = 0.0;
#pragma unroll 1
  for (int m = 0; m < NC; ++m) {
    const double tm = m == 0 ? 1.0 : (m == 1 ? u : 2.0 * u * tm1 - tm2);
    const double* a = A + 3 * NC * m;
#pragma unroll
    for (int nn = 0; nn < NC; ++nn) {
      const double t = tm * Tv[nn];
      X0 += t * a[3 * nn];
      X1 += t * a[3 * nn + 1];
      X2 += t * a[3 * nn + 2];
    }
    tm2 = tm1;
    tm1 = tm;
  }
  const double a = x[0] - X0, b = x[1] - X1, c = x[2] - X2;
  return a * a + b * b + c * c;
}

// Golden-section minimisation of f on [lo, hi] with a fixed step count.
template <class F>
__device__ inline double golden_min(F f, double lo, double hi, int iters, double gold) {
#pragma clang fp contract(off)
  double a = lo, b = hi;
  double c = b - gold * (b - a), d = a + gold * (b - a);
  double fc = f(c), fd = f(d);
  for (int it = 0; it < iters; ++it) {
    if (fc < fd) {
      b = d;
      d = c;
      fd = fc;
      c = b - gold * (b - a);
      fc = f(c);
    } else {
      a = c;
      c = d;
      fc = fd;
      d = a + gold * (b - a);
      fd = f(d);
    }
  }
  return 0.5 * (a + b);
}

// FILL = false: cnt[l] = |S_l|.  FILL = true: the pairs of row l at row_off[l].
template <int NC, bool FILL>
__global__ void __launch_bounds__(256) k_sing_pairs(SingDev g, int64_t* __restrict__ cnt,
                                                    const int64_t* __restrict__ row_off,
                                                    int32_t* __restrict__ pair_patch, double* __restrict__ uv) {
#pragma clang fp contract(off)
  constexpr int NQ = NC * NC;
  __shared__ double sbox[256 * 8];
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool act = l < g.n;
  double xl[3] = {0.0, 0.0, 0.0};
  if (act)
    for (int c = 0; c < 3; ++c) xl[c] = g.x[3 * l + c];
  int64_t o = (FILL && act) ? row_off[l] : 0;
  int64_t count = 0;
  for (int p0 = 0; p0 < g.P; p0 += 256) {
    __syncthreads();
    for (int t = threadIdx.x; t < 256 * 8; t += 256) {
      const int pp = p0 + t / 8;
      sbox[t] = pp < g.P ? g.box[(int64_t)pp * 8 + t % 8] : 0.0;
    }
    __syncthreads();
    if (!act) continue;
    const int pe = min(256, g.P - p0);
    for (int j = 0; j < pe; ++j) {
      const double* bx = &sbox[8 * j];
      double gap2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double gg = fmax(0.0, fmax(bx[c] - xl[c], xl[c] - bx[3 + c]));
        gap2 += gg * gg;
      }
      if (sqrt(gap2) > 1.5 * bx[6]) continue;
      const int p = p0 + j;
      const double* xp = g.x + (int64_t)3 * p * NQ;
      const double* Ap = g.A + (int64_t)3 * p * NQ;
      double u, v, dist;
      if (l / NQ == p) {
        const int loc = (int)(l % NQ);
        u = g.tn[loc / NC];
        v = g.tn[loc % NC];
        dist = 0.0;
      } else {
        int kbest = 0;
        double best = 0.0;
        for (int q = 0; q < NQ; ++q) {
          const double a = xp[3 * q] - xl[0], b = xp[3 * q + 1] - xl[1], c = xp[3 * q + 2] - xl[2];
          const double d2 = a * a + b * b + c * c;
          if (q == 0 || d2 < best) {
            best = d2;
            kbest = q;
          }
        }
        const int i0 = kbest / NC, j0 = kbest % NC;
        const double lo_u = (i0 + 1 < NC) ? g.tn[i0 + 1] : -1.0, hi_u = (i0 > 0) ? g.tn[i0 - 1] : 1.0;
        const double lo_v = (j0 + 1 < NC) ? g.tn[j0 + 1] : -1.0, hi_v = (j0 > 0) ? g.tn[j0 - 1] : 1.0;
        u = g.tn[i0];
        v = g.tn[j0];
        for (int s = 0; s < g.sweeps; ++s) {
          u = golden_min([&](double uu) { return patch_dist2<NC>(Ap, xl, uu, v); }, lo_u, hi_u, g.iters, g.gold);
          v = golden_min([&](double vv) { return patch_dist2<NC>(Ap, xl, u, vv); }, lo_v, hi_v, g.iters, g.gold);
        }
        if (fabs(1.0 - fabs(u)) < 1e-6) u = u > 0 ? 1.0 : -1.0;
        if (fabs(1.0 - fabs(v)) < 1e-6) v = v > 0 ? 1.0 : -1.0;
        dist = sqrt(patch_dist2<NC>(Ap, xl, u, v));
      }
      if (dist <= bx[6]) {
        if (FILL) {
          pair_patch[o + count] = p;
          uv[2 * (o + count)] = u;
          uv[2 * (o + count) + 1] = v;
        }
        ++count;
      }
    }
  }
  if (!FILL && act) cnt[l] = count;
}

// ---------------------------------------------------------------- pass 2
// Kress's sigmoidal map w(t) (eq. mk_cov_1, mk_cov_2) and its derivative.
__device__ inline double kress_nu(double t, int d) {
#pragma clang fp contract(off)
  const double a = (kPiD - t) / kPiD;
  return (1.0 / d - 0.5) * a * a * a + (1.0 / d) * ((t - kPiD) / kPiD) + 0.5;
}
__device__ inline double kress_dnu(double t, int d) {
#pragma clang fp contract(off)
  const double a = (kPiD - t) / kPiD;
  return -(3.0 / kPiD) * (1.0 / d - 0.5) * a * a + 1.0 / (d * kPiD);
}
__device__ inline double ipow_dev(double x, int d) {
#pragma clang fp contract(off)
  double p = x;
  for (int k = 1; k < d; ++k) p = p * x;
  return p;
}
__device__ inline double kress_w(double t, int d) {
#pragma clang fp contract(off)
  const double a = ipow_dev(kress_nu(t, d), d), b = ipow_dev(kress_nu(2 * kPiD - t, d), d);
  return 2 * kPiD * a / (a + b);
}
__device__ inline double kress_dw(double t, int d) {
#pragma clang fp contract(off)
  const double n1 = kress_nu(t, d), n2 = kress_nu(2 * kPiD - t, d);
  const double a = ipow_dev(n1, d), b = ipow_dev(n2, d);
  const double da = d * ipow_dev(n1, d - 1) * kress_dnu(t, d);
  const double db = -d * ipow_dev(n2, d - 1) * kress_dnu(2 * kPiD - t, d);
  return 2 * kPiD * (da * b - a * db) / ((a + b) * (a + b));
}

// Clustering map xi_alpha (eq. cov) at tau in [-1, 1]: value and derivative,
// accumulating Fejer points at the closest point alpha.
__device__ inline void cluster_map(double al, double t, int d, double* u, double* mu) {
#pragma clang fp contract(off)
  if (al == 1.0) {
    *u = al - ((1.0 + al) / kPiD) * kress_w(kPiD * fabs((t - 1.0) / 2.0), d);
    *mu = kress_dw(kPiD * (1.0 - t) / 2.0, d);
  } else if (al == -1.0) {
    *u = al + ((1.0 - al) / kPiD) * kress_w(kPiD * fabs((t + 1.0) / 2.0), d);
    *mu = kress_dw(kPiD * (1.0 + t) / 2.0, d);
  } else {
    const double sg = (t > 0) - (t < 0);
    *u = al + ((sg - al) / kPiD) * kress_w(kPiD * fabs(t), d);
    *mu = (1.0 - al * sg) * kress_dw(kPiD * fabs(t), d);
  }
}

// T_k(x) and T'_k(x) = k U_{k-1}(x), k < NC.
template <int NC>
__device__ inline void cheb_td(double x, double* T, double* dT) {
#pragma clang fp contract(off)
  T[0] = 1.0;
  if (NC > 1) T[1] = x;
#pragma unroll
  for (int k = 2; k < NC; ++k) T[k] = 2.0 * x * T[k - 1] - T[k - 2];
  double um2 = 0.0, um1 = 1.0;
  dT[0] = 0.0;
#pragma unroll
  for (int k = 1; k < NC; ++k) {
    dT[k] = k * um1;
    const double un = 2.0 * x * um1 - um2;
    um2 = um1;
    um1 = un;
  }
}

template <int NC>
__global__ void __launch_bounds__(64) k_sing_weights(SingDev g, const int64_t* __restrict__ row_off,
                                                     const int32_t* __restrict__ pair_patch,
                                                     const double* __restrict__ uv, double2* __restrict__ vals,
                                                     unsigned* __restrict__ err) {
#pragma clang fp contract(off)
  constexpr int NQ = NC * NC;
  __shared__ double sTu[kMaxNb * NC], sdTu[kMaxNb * NC], sTv[kMaxNb * NC], sdTv[kMaxNb * NC];
  __shared__ double sMU[kMaxNb], sMV[kMaxNb];
  __shared__ double sA[NQ * 3];
  __shared__ double sM[NQ];
  __shared__ double2 sG[2][kMaxNb * NC];   // column sums of (G, dG/dn) x weights for one wavenumber
  __shared__ double2 sB[2][NQ], sT[2][NQ];
  const int lane = threadIdx.x;
  const int64_t l = blockIdx.x;
  const int nb = g.nb;
  const double xl0 = g.x[3 * l], xl1 = g.x[3 * l + 1], xl2 = g.x[3 * l + 2];
  const double nl0 = g.nrm[3 * l], nl1 = g.nrm[3 * l + 1], nl2 = g.nrm[3 * l + 2];
  for (int t = lane; t < NQ; t += 64) sM[t] = g.M[t];
  for (int64_t e = row_off[l]; e < row_off[l + 1]; ++e) {
    const int p = pair_patch[e];
    const double ua = uv[2 * e], va = uv[2 * e + 1];
    __syncthreads();
    for (int t = lane; t < NQ * 3; t += 64) sA[t] = g.A[(int64_t)p * NQ * 3 + t];
    if (lane < nb) {
      double U, MU, V, MV;
      cluster_map(ua, g.tb[lane], g.d, &U, &MU);
      cluster_map(va, g.tb[lane], g.d, &V, &MV);
      cheb_td<NC>(U, &sTu[lane * NC], &sdTu[lane * NC]);
      cheb_td<NC>(V, &sTv[lane * NC], &sdTv[lane * NC]);
      sMU[lane] = MU * g.wb[lane];
      sMV[lane] = MV * g.wb[lane];
    }
    __syncthreads();
    // rows of eta_p and d eta_p / du at u = U_i, as Chebyshev series in v
    double Bx[NC][3], Bu[NC][3];
#pragma unroll
    for (int nn = 0; nn < NC; ++nn)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double s = 0.0, su = 0.0;
        if (lane < nb) {
#pragma unroll
          for (int m = 0; m < NC; ++m) {
            const double a = sA[3 * (m * NC + nn) + c];
            s += sTu[lane * NC + m] * a;
            su += sdTu[lane * NC + m] * a;
          }
        }
        Bx[nn][c] = s;
        Bu[nn][c] = su;
      }
    for (int q = 0; q < 2; ++q) {
      const double kq = g.k[q];
      if (lane < nb) {
        double sr[NC], si[NC], dr[NC], di[NC];
#pragma unroll
        for (int nn = 0; nn < NC; ++nn) sr[nn] = si[nn] = dr[nn] = di[nn] = 0.0;
        const double mu = sMU[lane];
        for (int j = 0; j < nb; ++j) {
          const double* tv = &sTv[j * NC];
          const double* dtv = &sdTv[j * NC];
          double Y0 = 0, Y1 = 0, Y2 = 0, U0 = 0, U1 = 0, U2 = 0, V0 = 0, V1 = 0, V2 = 0;
#pragma unroll
          for (int nn = 0; nn < NC; ++nn) {
            const double t = tv[nn], dt = dtv[nn];
            Y0 += Bx[nn][0] * t;
            Y1 += Bx[nn][1] * t;
            Y2 += Bx[nn][2] * t;
            U0 += Bu[nn][0] * t;
            U1 += Bu[nn][1] * t;
            U2 += Bu[nn][2] * t;
            V0 += Bx[nn][0] * dt;
            V1 += Bx[nn][1] * dt;
            V2 += Bx[nn][2] * dt;
          }
          const double c0 = U1 * V2 - U2 * V1, c1 = U2 * V0 - U0 * V2, c2 = U0 * V1 - U1 * V0;
          const double Jq = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
          const double dx = xl0 - Y0, dy = xl1 - Y1, dz = xl2 - Y2;
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          const double nd = nl0 * dx + nl1 * dy + nl2 * dz;
          const double wgt = Jq * mu * sMV[j];
          double sn, cs;
          sincos(kq * r, &sn, &cs);
          const double den = 4.0 * kPiD * r;
          const double gr = cs / den, gi = sn / den;             // G
          const double ar = -1.0 / r;                            // G (-1/r + i k) nd / r
          const double kr = ((gr * ar - gi * kq) * nd) / r, ki = ((gr * kq + gi * ar) * nd) / r;
          const double fr = gr * wgt, fi = gi * wgt, hr = kr * wgt, hi = ki * wgt;
#pragma unroll
          for (int nn = 0; nn < NC; ++nn) {
            const double t = tv[nn];
            sr[nn] += fr * t;
            si[nn] += fi * t;
            dr[nn] += hr * t;
            di[nn] += hi * t;
          }
        }
#pragma unroll
        for (int nn = 0; nn < NC; ++nn) {
          sG[0][lane * NC + nn] = make_double2(sr[nn], si[nn]);
          sG[1][lane * NC + nn] = make_double2(dr[nn], di[nn]);
        }
      }
      __syncthreads();
      // moments beta[m][n] = sum_i T_m(U_i) colsum[i][n]
      for (int o = lane; o < 2 * NQ; o += 64) {
        const int kk = o / NQ, mn = o % NQ, m = mn / NC, nn = mn % NC;
        double re = 0.0, im = 0.0;
        for (int i = 0; i < nb; ++i) {
          const double t = sTu[i * NC + m];
          const double2 v = sG[kk][i * NC + nn];
          re += t * v.x;
          im += t * v.y;
        }
        sB[kk][mn] = make_double2(re, im);
      }
      __syncthreads();
      // nodal weights W = M^T beta M
      for (int o = lane; o < 2 * NQ; o += 64) {
        const int kk = o / NQ, mn = o % NQ, m = mn / NC, jj = mn % NC;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int nn = 0; nn < NC; ++nn) {
          const double mt = sM[nn * NC + jj];
          re += sB[kk][m * NC + nn].x * mt;
          im += sB[kk][m * NC + nn].y * mt;
        }
        sT[kk][mn] = make_double2(re, im);
      }
      __syncthreads();
      for (int o = lane; o < 2 * NQ; o += 64) {
        const int kk = o / NQ, mn = o % NQ, ii = mn / NC, jj = mn % NC;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
          const double mt = sM[m * NC + ii];
          re += mt * sT[kk][m * NC + jj].x;
          im += mt * sT[kk][m * NC + jj].y;
        }
        sB[kk][mn] = make_double2(re, im);
      }
      __syncthreads();
      // minus the regular Fejer term the IFGF sum already holds
      double2* out = vals + e * 4 * NQ;
      for (int qq = lane; qq < NQ; qq += 64) {
        const int64_t gq = (int64_t)p * NQ + qq;
        double ksr = 0.0, ksi = 0.0, kdr = 0.0, kdi = 0.0;
        if (gq != l) {
          const double dx = xl0 - g.x[3 * gq], dy = xl1 - g.x[3 * gq + 1], dz = xl2 - g.x[3 * gq + 2];
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          if (!(r > 0.0)) {
            atomicOr(err, 1u);
            continue;
          }
          const double nd = nl0 * dx + nl1 * dy + nl2 * dz;
          double sn, cs;
          sincos(kq * r, &sn, &cs);
          const double den = 4.0 * kPiD * r, wq = g.w[gq];
          const double gr = cs / den, gi = sn / den;
          const double ar = -1.0 / r;
          ksr = gr * wq;
          ksi = gi * wq;
          kdr = (((gr * ar - gi * kq) * nd) / r) * wq;
          kdi = (((gr * kq + gi * ar) * nd) / r) * wq;
        }
        const double2 ws = sB[0][qq], wd = sB[1][qq];
        out[q * NQ + qq] = make_double2(ws.x - ksr, ws.y - ksi);
        out[(2 + q) * NQ + qq] = make_double2(wd.x - kdr, wd.y - kdi);
      }
      __syncthreads();
    }
  }
}

template <int NC>
hipError_t launch_pairs(const SingDev& g, int64_t* cnt, const int64_t* row_off, int32_t* pp, double* uv, bool fill) {
  const dim3 grid((unsigned)((g.n + 255) / 256));
  if (fill)
    hipLaunchKernelGGL((k_sing_pairs<NC, true>), grid, dim3(256), 0, 0, g, cnt, row_off, pp, uv);
  else
    hipLaunchKernelGGL((k_sing_pairs<NC, false>), grid, dim3(256), 0, 0, g, cnt, row_off, pp, uv);
  return hipGetLastError();
}

template <int NC>
hipError_t launch_weights(const SingDev& g, const int64_t* row_off, const int32_t* pp, const double* uv,
                          double2* vals, unsigned* err) {
  hipLaunchKernelGGL((k_sing_weights<NC>), dim3((unsigned)g.n), dim3(64), 0, 0, g, row_off, pp, uv, vals, err);
  return hipGetLastError();
}

template <class F>
hipError_t with_nc(int nc, F f) {
  switch (nc) {
    case 4: return f.template operator()<4>();
    case 5: return f.template operator()<5>();
    case 6: return f.template operator()<6>();
    case 8: return f.template operator()<8>();
    case 10: return f.template operator()<10>();
    default: return hipErrorInvalidValue;
  }
}

template <class T>
T* upload(DeviceArena& ar, const std::vector<T>& v) {
  T* p = static_cast<T*>(ar.alloc(v.size() * sizeof(T)));
  if (p && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return p;
}

}  // namespace

bool device_corrections_supported(int nc, int nbeta) {
  const int nb = nbeta > 0 ? nbeta : 6 * nc;
  return (nc == 4 || nc == 5 || nc == 6 || nc == 8 || nc == 10) && nb <= kMaxNb;
}

int build_corrections_device(const SurfaceGeo& geo, double k_int, double k_ext, const SingParams& sp,
                             DeviceArena& ar, DevCorrections& dc, Corrections& cor, std::string& err) {
  const int nc = geo.nc, nq = nc * nc;
  const int64_t n = geo.n;
  if (!device_corrections_supported(nc, sp.nbeta)) {
    err = "the device correction builder needs Nc in {4, 5, 6, 8, 10} and at most 64 Fejer points";
    return IFGF_EINVAL;
  }
  if (n >= ((int64_t)1 << 31)) {
    err = "too many points for the device correction builder";
    return IFGF_EINVAL;
  }
  SingTables t;
  if (sing_tables(geo, sp, t, err)) return IFGF_EINVAL;
  std::vector<double> box((size_t)geo.P * 8, 0.0);
  for (int p = 0; p < geo.P; ++p) {
    for (int c = 0; c < 3; ++c) {
      box[8 * (size_t)p + c] = t.lo[3 * (size_t)p + c];
      box[8 * (size_t)p + 3 + c] = t.hi[3 * (size_t)p + c];
    }
    box[8 * (size_t)p + 6] = t.delta[p];
  }
  DeviceArena tmp;   // freed on return
  SingDev g{};
  g.x = upload(tmp, geo.x);
  g.nrm = upload(tmp, geo.nrm);
  g.w = upload(tmp, geo.w);
  g.A = upload(tmp, t.A);
  g.box = upload(tmp, box);
  g.tn = upload(tmp, t.tn);
  g.tb = upload(tmp, t.tb);
  g.wb = upload(tmp, t.wb);
  g.M = upload(tmp, t.M);
  int64_t* d_cnt = static_cast<int64_t*>(tmp.alloc(sizeof(int64_t) * n));
  unsigned* d_err = static_cast<unsigned*>(tmp.alloc(sizeof(unsigned)));
  if (!g.x || !g.nrm || !g.w || !g.A || !g.box || !g.tn || !g.tb || !g.wb || !g.M || !d_cnt || !d_err) {
    err = "device allocation or copy failed for the singular quadrature";
    return IFGF_ENOMEM;
  }
  g.n = n;
  g.P = geo.P;
  g.nb = t.nb;
  g.d = sp.d;
  g.sweeps = sp.sweeps;
  g.iters = sp.iters;
  g.gold = t.gold;
  g.k[0] = k_int;
  g.k[1] = k_ext;
  hipError_t e;
  auto fail = [&](hipError_t h, const char* where) {
    err = std::string(where) + ": " + hipGetErrorString(h);
    return IFGF_EHIP;
  };
  if ((e = hipMemset(d_err, 0, sizeof(unsigned))) != hipSuccess) return fail(e, "hipMemset");
  if ((e = with_nc(nc, [&]<int NC>() { return launch_pairs<NC>(g, d_cnt, nullptr, nullptr, nullptr, false); })) !=
      hipSuccess)
    return fail(e, "singular pair count");
  std::vector<int64_t> cnt(n);
  if ((e = hipMemcpy(cnt.data(), d_cnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost)) != hipSuccess)
    return fail(e, "hipMemcpy");
  cor.nc = nc;
  cor.row_off.assign(n + 1, 0);
  for (int64_t l = 0; l < n; ++l) cor.row_off[l + 1] = cor.row_off[l] + cnt[l];
  const int64_t npairs = cor.row_off[n];
  std::vector<int64_t>().swap(cnt);
  dc.npairs = npairs;
  dc.row_off = upload(ar, cor.row_off);
  dc.pair_patch = static_cast<int32_t*>(ar.alloc(sizeof(int32_t) * std::max<int64_t>(npairs, 1)));
  dc.vals = static_cast<double2*>(ar.alloc(sizeof(double2) * 4 * nq * (size_t)std::max<int64_t>(npairs, 1)));
  double* d_uv = static_cast<double*>(tmp.alloc(sizeof(double) * 2 * std::max<int64_t>(npairs, 1)));
  if (!dc.row_off || !dc.pair_patch || !dc.vals || !d_uv) {
    err = "device allocation failed for the near-field corrections (" + std::to_string(npairs) + " pairs, " +
          std::to_string((double)npairs * 4 * nq * 16 / (1 << 30)) + " GiB of weights)";
    return IFGF_ENOMEM;
  }
  if ((e = with_nc(nc, [&]<int NC>() { return launch_pairs<NC>(g, nullptr, dc.row_off, dc.pair_patch, d_uv, true); })) !=
      hipSuccess)
    return fail(e, "singular pair fill");
  if ((e = with_nc(nc, [&]<int NC>() { return launch_weights<NC>(g, dc.row_off, dc.pair_patch, d_uv, dc.vals, d_err); })) !=
      hipSuccess)
    return fail(e, "singular weights");
  unsigned bad = 0;
  if ((e = hipMemcpy(&bad, d_err, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess) return fail(e, "hipMemcpy");
  if (bad) {
    err = "duplicate surface points";
    return IFGF_EINVAL;
  }
  cor.pair_patch.resize(npairs);
  if (npairs > 0 &&
      (e = hipMemcpy(cor.pair_patch.data(), dc.pair_patch, sizeof(int32_t) * npairs, hipMemcpyDeviceToHost)) !=
          hipSuccess)
    return fail(e, "hipMemcpy");
  std::vector<double>().swap(cor.vals);
  return 0;
}

}  // namespace ifgf
