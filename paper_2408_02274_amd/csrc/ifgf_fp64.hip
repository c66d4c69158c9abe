// FP64 IFGF apply kernels for gfx950 (reference-precision path).
//
// Paper: Sec. III-G algorithm steps 2-3 and Sec. III-I (IFGF_Vec):
//  near      direct G and n.grad G sums from the 27 neighbour leaves (step 2a)
//  leaf      F^D_B at the interpolation points of B's relevant cones (step 2b),
//            with the analytic factor of eq. ifgf_ana_factor
//  targets   interpolation of F_B at cousin points times the centred factor
//            G(x, x_B), plus the normal derivative of that product (step 3a)
//  propagate interpolation of the children's F at the parent's interpolation
//            points times G(X, x_child)/G(X, x_parent), summed over children (3b)
//
// The interpolant is the tensor Chebyshev interpolant of Sec. III-F written in
// Lagrange form on the same nodes (identical polynomial), so no separate
// value-to-coefficient pass is needed.  Discrete choices (cone of a point)
// come from the plan's integer tables; only continuous quantities are
// recomputed here.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace ifgf {

namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)
constexpr double kEta = 0.5773502691896257;       // sqrt(3) / 3

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}
__device__ __forceinline__ double2 expi(double ph) {
  double s, c;
  sincos(ph, &s, &c);
  return make_double2(c, s);
}

// Lagrange basis values (and derivatives) at u on the P nodes x.
__device__ __forceinline__ void lagrange(int P, const double* x, const double* winv, double u,
                                         double* L) {
  for (int j = 0; j < P; ++j) {
    double p = winv[j];
    for (int m = 0; m < P; ++m)
      if (m != j) p *= (u - x[m]);
    L[j] = p;
  }
}
__device__ __forceinline__ void lagrange_d(int P, const double* x, const double* winv, double u,
                                           double* dL) {
  for (int j = 0; j < P; ++j) {
    double acc = 0.0;
    for (int m = 0; m < P; ++m) {
      if (m == j) continue;
      double p = 1.0;
      for (int l = 0; l < P; ++l)
        if (l != j && l != m) p *= (u - x[l]);
      acc += p;
    }
    dL[j] = acc * winv[j];
  }
}

// Interpolation point k of cone `cone` of a box centred at c with radius h.
__device__ __forceinline__ void cone_point(int ns, int na, double h, const double* c, int cone,
                                           int k, const InterpC& ic, double* X) {
  int ip = cone % (2 * na);
  int it = (cone / (2 * na)) % na;
  int is = cone / (2 * na * na);
  int kp = k % ic.Pa, kt = (k / ic.Pa) % ic.Pa, ks = k / (ic.Pa * ic.Pa);
  double ds = kEta / ns, da = kPi / na;
  double s = (is + 0.5) * ds + 0.5 * ds * ic.xs[ks];
  double t = (it + 0.5) * da + 0.5 * da * ic.xa[kt];
  double f = (ip + 0.5) * da + 0.5 * da * ic.xa[kp];
  double rr = h / s;
  double st, ct, sp, cp;
  sincos(t, &st, &ct);
  sincos(f, &sp, &cp);
  X[0] = c[0] + rr * (st * cp);
  X[1] = c[1] + rr * (st * sp);
  X[2] = c[2] + rr * ct;
}

// Spherical coordinates of offset d about a box centre and their affine
// images in the intervals of cone `cone`.
struct Local {
  double r, s, th, ph, us, ut, up;
};
__device__ __forceinline__ Local local_coords(double dx, double dy, double dz, double h, int ns,
                                              int na, int cone) {
  Local o;
  o.r = sqrt(dx * dx + dy * dy + dz * dz);
  o.s = h / o.r;
  double ct = dz / o.r;
  ct = fmin(1.0, fmax(-1.0, ct));
  o.th = acos(ct);
  o.ph = atan2(dy, dx);
  if (o.ph < 0.0) o.ph += kTwoPi;
  int ip = cone % (2 * na);
  int it = (cone / (2 * na)) % na;
  int is = cone / (2 * na * na);
  double ds = kEta / ns, da = kPi / na;
  o.us = (o.s - (is + 0.5) * ds) / (0.5 * ds);
  o.ut = (o.th - (it + 0.5) * da) / (0.5 * da);
  o.up = (o.ph - (ip + 0.5) * da) / (0.5 * da);
  return o;
}

__global__ void k_gather_weighted(const double2* __restrict__ dens, const int64_t* __restrict__ perm,
                                  const double* __restrict__ w, int64_t n, double2* __restrict__ a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * kNS) return;
  int64_t i = t / kNS;
  int m = (int)(t % kNS);
  double2 v = dens[(int64_t)m * n + perm[i]];
  double wi = w[i];
  a[t] = make_double2(v.x * wi, v.y * wi);
}

__global__ void __launch_bounds__(128) k_near(const int32_t* __restrict__ leaf_of_point, const int32_t* __restrict__ nbr_off,
                       const int32_t* __restrict__ nbr, const int32_t* __restrict__ start,
                       const int32_t* __restrict__ end, const double* __restrict__ xs,
                       const double* __restrict__ nrm, const double2* __restrict__ a, int64_t n,
                       double k0, double k1, double2* __restrict__ out_s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = xs[3 * i], yi = xs[3 * i + 1], zi = xs[3 * i + 2];
  const double nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
  double2 S[2][kNS], Dn[2][kND];
  for (int q = 0; q < 2; ++q) {
    for (int m = 0; m < kNS; ++m) S[q][m] = make_double2(0.0, 0.0);
    for (int m = 0; m < kND; ++m) Dn[q][m] = make_double2(0.0, 0.0);
  }
  const double kk[2] = {k0, k1};
  int32_t b = leaf_of_point[i];
  for (int32_t e = nbr_off[b]; e < nbr_off[b + 1]; ++e) {
    int32_t c = nbr[e];
    for (int32_t j = start[c]; j < end[c]; ++j) {
      if (j == i) continue;
      double dx = xi - xs[3 * j], dy = yi - xs[3 * j + 1], dz = zi - xs[3 * j + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double rinv = 1.0 / r;
      double nd = (nx * dx + ny * dy + nz * dz) * rinv;
      const double2* aj = a + (int64_t)j * kNS;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double2 G = expi(kk[q] * r);
        G.x *= kInv4Pi * rinv;
        G.y *= kInv4Pi * rinv;
        double2 gd = cmul(G, make_double2(-rinv * nd, kk[q] * nd));
#pragma unroll
        for (int m = 0; m < kNS; ++m) cfma(S[q][m], G, aj[m]);
#pragma unroll
        for (int m = 0; m < kND; ++m) cfma(Dn[q][m], gd, aj[m]);
      }
    }
  }
  double2* o = out_s + i * kOut;
  for (int q = 0; q < 2; ++q) {
    for (int m = 0; m < kNS; ++m) o[q * (kNS + kND) + m] = S[q][m];
    for (int m = 0; m < kND; ++m) o[q * (kNS + kND) + kNS + m] = Dn[q][m];
  }
}

__global__ void __launch_bounds__(128) k_leaf(DevLevel L, InterpC ic, const double* __restrict__ xs,
                       const double2* __restrict__ a, double k0, double k1,
                       double2* __restrict__ vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nslots * ic.npts) return;
  int64_t q = t / ic.npts;
  int k = (int)(t % ic.npts);
  int32_t b = L.slot_box[q];
  const double* c = L.centers + 3 * b;
  double X[3];
  cone_point(L.ns, L.na, L.h, c, L.slot_cone[q], k, ic, X);
  double ex = X[0] - c[0], ey = X[1] - c[1], ez = X[2] - c[2];
  double rxc = sqrt(ex * ex + ey * ey + ez * ez);
  double2 acc[2][kNS];
  for (int qq = 0; qq < 2; ++qq)
    for (int m = 0; m < kNS; ++m) acc[qq][m] = make_double2(0.0, 0.0);
  const double kk[2] = {k0, k1};
  for (int32_t j = L.start[b]; j < L.end[b]; ++j) {
    double dx = X[0] - xs[3 * j], dy = X[1] - xs[3 * j + 1], dz = X[2] - xs[3 * j + 2];
    double rxy = sqrt(dx * dx + dy * dy + dz * dz);
    double ratio = rxc / rxy;
    const double2* aj = a + (int64_t)j * kNS;
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      double2 g = expi(kk[qq] * (rxy - rxc));
      g.x *= ratio;
      g.y *= ratio;
#pragma unroll
      for (int m = 0; m < kNS; ++m) cfma(acc[qq][m], g, aj[m]);
    }
  }
  double2* o = vals + t * kCols;
  for (int qq = 0; qq < 2; ++qq)
    for (int m = 0; m < kNS; ++m) o[qq * kNS + m] = acc[qq][m];
}

__global__ void __launch_bounds__(64) k_targets(DevLevel L, InterpC ic, const double* __restrict__ xs,
                          const double* __restrict__ nrm, int64_t n, double k0, double k1,
                          const double2* __restrict__ vals, double2* __restrict__ out_s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t e0 = L.tp_off[i], e1 = L.tp_off[i + 1];
  if (e0 == e1) return;
  const double xi = xs[3 * i], yi = xs[3 * i + 1], zi = xs[3 * i + 2];
  const double nx = nrm[3 * i], ny = nrm[3 * i + 1], nz = nrm[3 * i + 2];
  const double kk[2] = {k0, k1};
  double2* o = out_s + i * kOut;
  double2 S[2][kNS], Dn[2][kND];
  for (int q = 0; q < 2; ++q) {
    for (int m = 0; m < kNS; ++m) S[q][m] = o[q * (kNS + kND) + m];
    for (int m = 0; m < kND; ++m) Dn[q][m] = o[q * (kNS + kND) + kNS + m];
  }
  const double ds = kEta / L.ns, da = kPi / L.na;
  for (int64_t e = e0; e < e1; ++e) {
    int32_t slot = L.tp_slot[e];
    int32_t B = L.slot_box[slot];
    int cone = L.slot_cone[slot];
    const double* c = L.centers + 3 * B;
    double dx = xi - c[0], dy = yi - c[1], dz = zi - c[2];
    Local lc = local_coords(dx, dy, dz, L.h, L.ns, L.na, cone);
    double Ls[8], Lt[8], Lp[8], dLs[8], dLt[8], dLp[8];
    lagrange(ic.Ps, ic.xs, ic.ws, lc.us, Ls);
    lagrange(ic.Pa, ic.xa, ic.wa, lc.ut, Lt);
    lagrange(ic.Pa, ic.xa, ic.wa, lc.up, Lp);
    lagrange_d(ic.Ps, ic.xs, ic.ws, lc.us, dLs);
    lagrange_d(ic.Pa, ic.xa, ic.wa, lc.ut, dLt);
    lagrange_d(ic.Pa, ic.xa, ic.wa, lc.up, dLp);
    double rinv = 1.0 / lc.r;
    double n_r = (nx * dx + ny * dy + nz * dz) * rinv;
    double st, ct, sp, cp;
    sincos(lc.th, &st, &ct);
    sincos(lc.ph, &sp, &cp);
    double n_th = nx * ct * cp + ny * ct * sp - nz * st;
    double n_ph = -nx * sp + ny * cp;
    double c_ph = (st > 0.0) ? n_ph / (lc.r * st) : 0.0;   // grad phi = phi-hat/(r sin theta)
    double c_s = -(L.h * rinv * rinv) * n_r;                // grad s = -(h/r^2) r-hat
    double c_t = n_th * rinv;                                // grad theta = theta-hat / r
    c_s *= 2.0 / ds;
    c_t *= 2.0 / da;
    c_ph *= 2.0 / da;
    const double2* V = vals + (int64_t)slot * ic.npts * kCols;
    for (int q = 0; q < 2; ++q) {
      double2 F[kNS], FD[kND];
      for (int m = 0; m < kNS; ++m) F[m] = make_double2(0.0, 0.0);
      for (int m = 0; m < kND; ++m) FD[m] = make_double2(0.0, 0.0);
      int k = 0;
      for (int a = 0; a < ic.Ps; ++a)
        for (int bb = 0; bb < ic.Pa; ++bb)
          for (int cc = 0; cc < ic.Pa; ++cc, ++k) {
            double w = Ls[a] * Lt[bb] * Lp[cc];
            double wd = c_s * dLs[a] * Lt[bb] * Lp[cc] + c_t * Ls[a] * dLt[bb] * Lp[cc] +
                        c_ph * Ls[a] * Lt[bb] * dLp[cc];
            const double2* v = V + (int64_t)k * kCols + q * kNS;
#pragma unroll
            for (int m = 0; m < kNS; ++m) {
              double2 vm = v[m];
              F[m].x += w * vm.x;
              F[m].y += w * vm.y;
              if (m < kND) {
                FD[m].x += wd * vm.x;
                FD[m].y += wd * vm.y;
              }
            }
          }
      double2 Gc = expi(kk[q] * lc.r);
      Gc.x *= kInv4Pi * rinv;
      Gc.y *= kInv4Pi * rinv;
      double2 dG = make_double2(-rinv * n_r, kk[q] * n_r);   // (i k - 1/r) n.r-hat
#pragma unroll
      for (int m = 0; m < kNS; ++m) cfma(S[q][m], Gc, F[m]);
#pragma unroll
      for (int m = 0; m < kND; ++m) {
        double2 t = cmul(dG, F[m]);
        t.x += FD[m].x;
        t.y += FD[m].y;
        cfma(Dn[q][m], Gc, t);
      }
    }
  }
  for (int q = 0; q < 2; ++q) {
    for (int m = 0; m < kNS; ++m) o[q * (kNS + kND) + m] = S[q][m];
    for (int m = 0; m < kND; ++m) o[q * (kNS + kND) + kNS + m] = Dn[q][m];
  }
}

__global__ void __launch_bounds__(64) k_propagate(DevLevel C, DevLevel P, InterpC ic, double k0, double k1,
                            const double2* __restrict__ vals_c, double2* __restrict__ vals_p) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P.nslots * ic.npts) return;
  int64_t q = t / ic.npts;
  int k = (int)(t % ic.npts);
  int32_t pb = P.slot_box[q];
  const double* cp = P.centers + 3 * pb;
  double X[3];
  cone_point(P.ns, P.na, P.h, cp, P.slot_cone[q], k, ic, X);
  double ex = X[0] - cp[0], ey = X[1] - cp[1], ez = X[2] - cp[2];
  double rp = sqrt(ex * ex + ey * ey + ez * ez);
  const double kk[2] = {k0, k1};
  double2 acc[kCols];
  for (int m = 0; m < kCols; ++m) acc[m] = make_double2(0.0, 0.0);
  int64_t base = P.pp_off[q];
  int32_t c0 = P.child_start[pb], c1 = P.child_end[pb];
  for (int32_t c = c0; c < c1; ++c) {
    int32_t slot = P.pp_slot[base + (int64_t)(c - c0) * ic.npts + k];
    const double* cc = C.centers + 3 * c;
    Local lc = local_coords(X[0] - cc[0], X[1] - cc[1], X[2] - cc[2], C.h, C.ns, C.na,
                            C.slot_cone[slot]);
    double Ls[8], Lt[8], Lp[8];
    lagrange(ic.Ps, ic.xs, ic.ws, lc.us, Ls);
    lagrange(ic.Pa, ic.xa, ic.wa, lc.ut, Lt);
    lagrange(ic.Pa, ic.xa, ic.wa, lc.up, Lp);
    double2 F[kCols];
    for (int m = 0; m < kCols; ++m) F[m] = make_double2(0.0, 0.0);
    const double2* V = vals_c + (int64_t)slot * ic.npts * kCols;
    int kk2 = 0;
    for (int a = 0; a < ic.Ps; ++a)
      for (int bb = 0; bb < ic.Pa; ++bb) {
        double wab = Ls[a] * Lt[bb];
        for (int cc2 = 0; cc2 < ic.Pa; ++cc2, ++kk2) {
          double w = wab * Lp[cc2];
          const double2* v = V + (int64_t)kk2 * kCols;
#pragma unroll
          for (int m = 0; m < kCols; ++m) {
            double2 vm = v[m];
            F[m].x += w * vm.x;
            F[m].y += w * vm.y;
          }
        }
      }
    double ratio = rp / lc.r;
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      double2 f = expi(kk[qq] * (lc.r - rp));     // G(X,x_c)/G(X,x_p)
      f.x *= ratio;
      f.y *= ratio;
#pragma unroll
      for (int m = 0; m < kNS; ++m) cfma(acc[qq * kNS + m], f, F[qq * kNS + m]);
    }
  }
  double2* o = vals_p + t * kCols;
  for (int m = 0; m < kCols; ++m) o[m] = acc[m];
}

__global__ void k_scatter_out(const double2* __restrict__ out_s, const int64_t* __restrict__ perm,
                              int64_t n, double2* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * kOut) return;
  int64_t i = t / kOut;
  int c = (int)(t % kOut);
  out[(int64_t)c * n + perm[i]] = out_s[t];
}

inline unsigned nblk(int64_t work, int bs) { return (unsigned)((work + bs - 1) / bs); }

}  // namespace

hipError_t launch_gather_weighted(const double2* dens, const int64_t* perm, const double* w,
                                  int64_t n, double2* a, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_weighted, dim3(nblk(n * kNS, 256)), dim3(256), 0, st, dens, perm, w,
                     n, a);
  return hipGetLastError();
}

hipError_t launch_near(const DevLevel& leaf, const int32_t* leaf_of_point, const double* xs,
                       const double* nrm, const double2* a, int64_t n, double k0, double k1,
                       double2* out_s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_near, dim3(nblk(n, 128)), dim3(128), 0, st, leaf_of_point, leaf.nbr_off,
                     leaf.nbr, leaf.start, leaf.end, xs, nrm, a, n, k0, k1, out_s);
  return hipGetLastError();
}

hipError_t launch_leaf(const DevLevel& leaf, const InterpC& ic, const double* xs,
                       const double2* a, double k0, double k1, double2* vals, hipStream_t st) {
  int64_t work = leaf.nslots * ic.npts;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf, dim3(nblk(work, 128)), dim3(128), 0, st, leaf, ic, xs, a, k0, k1,
                     vals);
  return hipGetLastError();
}

hipError_t launch_targets(const DevLevel& L, const InterpC& ic, const double* xs,
                          const double* nrm, int64_t n, double k0, double k1,
                          const double2* vals, double2* out_s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_targets, dim3(nblk(n, 64)), dim3(64), 0, st, L, ic, xs, nrm, n, k0, k1,
                     vals, out_s);
  return hipGetLastError();
}

hipError_t launch_propagate(const DevLevel& child, const DevLevel& parent, const InterpC& ic,
                            double k0, double k1, const double2* vals_child,
                            double2* vals_parent, hipStream_t st) {
  int64_t work = parent.nslots * ic.npts;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_propagate, dim3(nblk(work, 64)), dim3(64), 0, st, child, parent, ic, k0,
                     k1, vals_child, vals_parent);
  return hipGetLastError();
}

hipError_t launch_scatter_out(const double2* out_s, const int64_t* perm, int64_t n,
                              double2* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_out, dim3(nblk(n * kOut, 256)), dim3(256), 0, st, out_s, perm, n,
                     out);
  return hipGetLastError();
}

}  // namespace ifgf
