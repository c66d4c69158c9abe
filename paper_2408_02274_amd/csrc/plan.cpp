// Host-side IFGF plan (Sec. III-G algorithm step 1).
//
// Builds the linear octree of non-empty boxes (eq. rele_boxes), neighbour and
// cousin lists (eq. box_neighbor, box_cousin), per-level cone counts
// (Remark 2), and the relevant cone segments of every box, recursively from
// level 3 (eq. rele_cone): a cone is relevant if it contains a cousin point
// or an interpolation point of a relevant cone of the parent box.
//
// Geometric decisions (box of a point, cone of a point) are made once, in
// FP64, and handed to the apply kernels as integer tables.  They use only
// +, -, *, /, sqrt and floor, with floating-point contraction off, against
// tables of the cone boundary directions (cone_index): any implementation
// that forms the same products -- the oracle, the device planner -- takes
// the same decision, also for points exactly on a cone boundary.
#include "plan.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace ifgf {

static const double kPi = 3.141592653589793;
static const double kTwoPi = 2.0 * 3.141592653589793;
static const double kSqrt3 = std::sqrt(3.0);
static const double kEta = std::sqrt(3.0) / 3.0;   // cone domain radius (Sec. III-F)

void cone_dirs(int na, std::vector<double>& C, std::vector<double>& S) {
  const double da = kPi / na;
  C.resize(na + 1);
  S.resize(na + 1);
  for (int k = 0; k <= na; ++k) {
    C[k] = std::cos((double)k * da);
    S[k] = std::sin((double)k * da);
  }
}

int cone_index(double dx, double dy, double dz, double h, int ns, int na, const double* C, const double* S) {
  const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  const double s = h / r;
  double ct = dz / r;
  if (ct > 1.0) ct = 1.0;
  if (ct < -1.0) ct = -1.0;
  const double ds = kEta / ns;
  const double fs = std::floor(s / ds);
  const int64_t is = (int64_t)std::min(fs, (double)(ns - 1));
  // theta >= k da  <=>  cos theta <= C[k]: count k = 1..na-1 (C decreasing)
  int lo = 1, hi = na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ct <= C[mid]) lo = mid + 1;
    else hi = mid;
  }
  const int64_t it = lo - 1;
  // phi >= k da: the point on or counter-clockwise of boundary ray k, in its
  // half plane (the lower half turned by pi)
  const bool up = dy > 0.0 || (dy == 0.0 && dx >= 0.0);
  const double px = up ? dx : -dx, py = up ? dy : -dy;
  lo = 1;
  hi = na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] * py - S[mid] * px >= 0.0) lo = mid + 1;
    else hi = mid;
  }
  int64_t ip = (lo - 1) + (up ? 0 : na);
  if (dx == 0.0 && dy == 0.0) ip = 0;
  return (int)((is * na + it) * (2 * na) + ip);
}

static inline uint64_t morton(int64_t kx, int64_t ky, int64_t kz) {
  uint64_t key = 0;
  for (int b = 0; b < 20; ++b) {
    key |= (uint64_t)((kx >> b) & 1) << (3 * b + 2);
    key |= (uint64_t)((ky >> b) & 1) << (3 * b + 1);
    key |= (uint64_t)((kz >> b) & 1) << (3 * b);
  }
  return key;
}

// Chebyshev nodes cos((k + 1/2) pi / n).
static void cheb_nodes(int n, double* x) {
  for (int k = 0; k < n; ++k) x[k] = std::cos((k + 0.5) * kPi / n);
}

// Interpolation point k of cone `cone` of a box centred at c (radius h).
static inline void cone_point(const HostLevel& L, const double* c, int cone, int k,
                              int Ps, int Pa, const double* xs, const double* xa,
                              double* X) {
  int na = L.na, ns = L.ns;
  int ip = cone % (2 * na);
  int it = (cone / (2 * na)) % na;
  int is = cone / (2 * na * na);
  int kp = k % Pa, kt = (k / Pa) % Pa, ks = k / (Pa * Pa);
  double ds = kEta / ns, da = kPi / na;
  double s = (is + 0.5) * ds + 0.5 * ds * xs[ks];
  double t = (it + 0.5) * da + 0.5 * da * xa[kt];
  double f = (ip + 0.5) * da + 0.5 * da * xa[kp];
  double rr = L.h / s;
  double st = std::sin(t), ctt = std::cos(t), sp = std::sin(f), cp = std::cos(f);
  X[0] = c[0] + rr * (st * cp);
  X[1] = c[1] + rr * (st * sp);
  X[2] = c[2] + rr * ctt;
  (void)ns;
}

static int64_t find_box(const HostLevel& L, uint64_t key) {
  auto it = std::lower_bound(L.key.begin(), L.key.end(), (int64_t)key);
  if (it == L.key.end() || *it != (int64_t)key) return -1;
  return it - L.key.begin();
}

static int find_slot(const HostLevel& L, int64_t box, int cone) {
  const int32_t* b = L.slot_cone.data() + L.slot_off[box];
  const int32_t* e = L.slot_cone.data() + L.slot_off[box + 1];
  const int32_t* it = std::lower_bound(b, e, cone);
  if (it == e || *it != cone) return -1;
  return (int)(L.slot_off[box] + (it - b));
}

void build_target_tiles(HostLevel& L, int64_t n, int64_t chunk_pairs) {
  const int64_t np = L.tp_off.empty() ? 0 : L.tp_off[n];
  L.tt_slot.clear();
  L.tt_start.clear();
  L.tt_cnt.clear();
  L.tc_tile.assign(1, 0);
  L.tc_i0.assign(1, 0);
  L.tc_max_pairs = 0;
  if (np <= 0 || L.nslots <= 0) {
    L.ts_tgt.clear();
    L.ts_e.clear();
    L.tc_i0.push_back(n);
    L.tc_tile.push_back(0);
    return;
  }
  L.ts_tgt.resize(np);
  L.ts_e.resize(np);
  std::vector<int64_t> off(L.nslots + 1, 0);
  for (int64_t i0 = 0; i0 < n;) {
    const int64_t e0 = L.tp_off[i0];
    int64_t i1 = i0 + 1;
    while (i1 < n && L.tp_off[i1 + 1] - e0 <= chunk_pairs) ++i1;
    const int64_t e1 = L.tp_off[i1];
    L.tc_max_pairs = std::max(L.tc_max_pairs, e1 - e0);
    std::fill(off.begin(), off.end(), 0);
    for (int64_t e = e0; e < e1; ++e) off[L.tp_slot[e] + 1] += 1;
    for (int64_t s = 0; s < L.nslots; ++s) off[s + 1] += off[s];
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int64_t i = i0; i < i1; ++i)
      for (int64_t e = L.tp_off[i]; e < L.tp_off[i + 1]; ++e) {
        const int64_t pos = e0 + cur[L.tp_slot[e]]++;
        L.ts_tgt[pos] = (int32_t)i;
        L.ts_e[pos] = (int32_t)(e - e0);
      }
    for (int64_t s = 0; s < L.nslots; ++s)
      for (int64_t k = off[s]; k < off[s + 1]; k += 8) {
        L.tt_slot.push_back((int32_t)s);
        L.tt_start.push_back(e0 + k);
        L.tt_cnt.push_back((uint8_t)std::min<int64_t>(8, off[s + 1] - k));
      }
    L.tc_tile.push_back((int64_t)L.tt_slot.size());
    L.tc_i0.push_back(i1);
    i0 = i1;
  }
}

void build_prop_groups(HostLevel& Pl, const HostLevel& L, int npts) {
  const int64_t Q = Pl.nslots;
  std::vector<std::vector<int32_t>> gs(Q), gc(Q), gn(Q);
  std::vector<std::vector<uint8_t>> gp(Q);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < Q; ++q) {
    const int32_t pb = Pl.slot_box[q];
    const int nch = Pl.child_end[pb] - Pl.child_start[pb];
    std::vector<std::pair<int32_t, int>> tmp(npts);
    for (int j = 0; j < nch; ++j) {
      const int32_t* ps = &Pl.pp_slot[Pl.pp_off[q] + (int64_t)j * npts];
      for (int k = 0; k < npts; ++k) tmp[k] = {ps[k], k};
      std::stable_sort(tmp.begin(), tmp.end(),
                       [](const std::pair<int32_t, int>& a, const std::pair<int32_t, int>& b) {
                         return a.first < b.first;
                       });
      for (int k = 0; k < npts; ++k) {
        if (k == 0 || tmp[k].first != tmp[k - 1].first) {
          gs[q].push_back(tmp[k].first);
          gc[q].push_back(Pl.child_start[pb] + j);
          gn[q].push_back(0);
        }
        gn[q].back() += 1;
        gp[q].push_back((uint8_t)tmp[k].second);
      }
    }
  }
  Pl.pg_off.assign(Q + 1, 0);
  for (int64_t q = 0; q < Q; ++q) Pl.pg_off[q + 1] = Pl.pg_off[q] + (int64_t)gs[q].size();
  const int64_t G = Pl.pg_off[Q];
  Pl.pg_slot.resize(G);
  Pl.pg_cbox.resize(G);
  Pl.pg_count.resize(G);
  Pl.pg_start.resize(G);
  Pl.pg_pts.resize(Pl.pp_off[Q]);
  for (int64_t q = 0; q < Q; ++q) {
    int64_t g = Pl.pg_off[q];
    int64_t st = Pl.pp_off[q];
    std::copy(gp[q].begin(), gp[q].end(), Pl.pg_pts.begin() + st);
    for (size_t i = 0; i < gs[q].size(); ++i, ++g) {
      Pl.pg_slot[g] = gs[q][i];
      Pl.pg_cbox[g] = gc[q][i];
      Pl.pg_count[g] = gn[q][i];
      Pl.pg_start[g] = st;
      st += gn[q][i];
    }
  }
  Pl.pt_off.assign(Q + 1, 0);
  for (int64_t q = 0; q < Q; ++q) {
    int64_t nt = 0;
    for (int64_t g = Pl.pg_off[q]; g < Pl.pg_off[q + 1]; ++g) nt += (Pl.pg_count[g] + 15) / 16;
    Pl.pt_off[q + 1] = Pl.pt_off[q] + nt;
  }
  Pl.pt_g.resize(Pl.pt_off[Q]);
  Pl.pt_t0.resize(Pl.pt_off[Q]);
  Pl.pt_rec.resize(4 * Pl.pt_off[Q]);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t q = 0; q < Q; ++q) {
    int64_t t = Pl.pt_off[q];
    for (int64_t g = Pl.pg_off[q]; g < Pl.pg_off[q + 1]; ++g)
      for (int t0 = 0; t0 < Pl.pg_count[g]; t0 += 16, ++t) {
        Pl.pt_g[t] = (int32_t)g;
        Pl.pt_t0[t] = (uint8_t)t0;
        int32_t* r = &Pl.pt_rec[4 * t];
        r[0] = Pl.pg_slot[g];
        r[1] = (Pl.pg_cbox[g] << 5) | std::min(16, Pl.pg_count[g] - t0);
        r[2] = (int32_t)(Pl.pg_start[g] + t0);
        r[3] = L.slot_cone[Pl.pg_slot[g]];
      }
  }
  (void)L;
}

int build_host_plan(HostPlan& P, int64_t n, const double* x, const double* nrm,
                    const double* w, double k0, double k1, const PlanParams& pp,
                    std::string& err) {
  P.n = n;
  P.k[0] = k0;
  P.k[1] = k1;
  P.kmax = std::max(k0, k1);
  P.Ps = pp.Ps;
  P.Pa = pp.Pa;
  P.npts = pp.Ps * pp.Pa * pp.Pa;
  const int npts = P.npts;

  // bounding cube (reading A21) and depth (H_D <= leaf_wavelengths * lambda_min)
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) { lo[c] = x[c]; hi[c] = x[c]; }
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], x[3 * i + c]);
      hi[c] = std::max(hi[c], x[3 * i + c]);
    }
  double ext = 0.0;
  for (int c = 0; c < 3; ++c) {
    P.center[c] = 0.5 * (lo[c] + hi[c]);
    ext = std::max(ext, hi[c] - lo[c]);
  }
  P.H1 = ext > 0.0 ? ext * (1.0 + 1e-9) : 1.0;
  double lam = kTwoPi / P.kmax;
  int D = 1;
  while (std::ldexp(P.H1, -(D - 1)) > pp.leaf_wavelengths * lam) {
    ++D;
    if (D > 21) { err = "octree deeper than 21 levels"; return -1; }
  }
  P.D = D;
  for (int c = 0; c < 3; ++c) P.origin[c] = P.center[c] - 0.5 * P.H1;
  const double HD = std::ldexp(P.H1, -(D - 1));
  const int64_t nmax = (int64_t)1 << (D - 1);

  // leaf coordinates, Morton sort (stable by input index)
  std::vector<int64_t> kD(3 * n);
  std::vector<uint64_t> keyD(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) {
      double f = std::floor((x[3 * i + c] - P.origin[c]) / HD);
      int64_t k = (int64_t)f;
      k = std::max<int64_t>(0, std::min<int64_t>(nmax - 1, k));
      kD[3 * i + c] = k;
    }
    keyD[i] = morton(kD[3 * i], kD[3 * i + 1], kD[3 * i + 2]);
  }
  P.perm.resize(n);
  std::iota(P.perm.begin(), P.perm.end(), 0);
  std::stable_sort(P.perm.begin(), P.perm.end(),
                   [&](int64_t a, int64_t b) { return keyD[a] < keyD[b]; });
  P.xs.resize(3 * n);
  P.nrm.resize(3 * n);
  P.w.resize(n);
  std::vector<uint64_t> skey(n);
  std::vector<int64_t> skD(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = P.perm[i];
    for (int c = 0; c < 3; ++c) {
      P.xs[3 * i + c] = x[3 * j + c];
      P.nrm[3 * i + c] = nrm[3 * j + c];
      skD[3 * i + c] = kD[3 * j + c];
    }
    P.w[i] = w[j];
    skey[i] = keyD[j];
  }

  // cone counts per level (Remark 2; readings A2-A4)
  P.lev.assign(D + 1, HostLevel());
  {
    int ns = pp.ns_init, na = pp.na_init;
    for (int d = D; d >= 3; --d) {
      double Hd = std::ldexp(P.H1, -(d - 1));
      int a = (P.kmax * Hd > 0.5) ? 2 : 1;
      na *= a;
      if (pp.refine_radial) ns *= a;
      P.lev[d].ns = ns;
      P.lev[d].na = na;
      P.lev[d].ncones = (int64_t)ns * na * 2 * na;
      if (P.lev[d].ncones >= ((int64_t)1 << 31)) {
        err = "more than 2^31 cones per box at level " + std::to_string(d) + " (cone indices are 32-bit)";
        return -1;
      }
    }
  }

  // boxes per level
  for (int d = 1; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    L.d = d;
    L.H = std::ldexp(P.H1, -(d - 1));
    L.h = kSqrt3 / 2.0 * L.H;
    int shift = 3 * (D - d);
    for (int64_t i = 0; i < n; ++i) {
      uint64_t k = skey[i] >> shift;
      if (i == 0 || k != (skey[i - 1] >> shift)) {
        L.key.push_back((int64_t)k);
        L.start.push_back((int32_t)i);
        for (int c = 0; c < 3; ++c) L.coords.push_back((int32_t)(skD[3 * i + c] >> (D - d)));
      }
    }
    L.nb = (int64_t)L.key.size();
    L.end.resize(L.nb);
    for (int64_t b = 0; b < L.nb; ++b) L.end[b] = (b + 1 < L.nb) ? L.start[b + 1] : (int32_t)n;
    L.centers.resize(3 * L.nb);
    for (int64_t b = 0; b < L.nb; ++b)
      for (int c = 0; c < 3; ++c)
        L.centers[3 * b + c] = P.origin[c] + L.H * (L.coords[3 * b + c] + 0.5);
  }
  for (int d = 2; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    HostLevel& Pl = P.lev[d - 1];
    L.parent.resize(L.nb);
    for (int64_t b = 0; b < L.nb; ++b) L.parent[b] = (int32_t)find_box(Pl, (uint64_t)L.key[b] >> 3);
    Pl.child_start.assign(Pl.nb, 0);
    Pl.child_end.assign(Pl.nb, 0);
    for (int64_t b = L.nb - 1; b >= 0; --b) Pl.child_start[L.parent[b]] = (int32_t)b;
    for (int64_t b = 0; b < L.nb; ++b) Pl.child_end[L.parent[b]] = (int32_t)(b + 1);
  }
  P.leaf_of_point.resize(n);
  {
    HostLevel& L = P.lev[D];
    for (int64_t b = 0; b < L.nb; ++b)
      for (int32_t i = L.start[b]; i < L.end[b]; ++i) P.leaf_of_point[i] = (int32_t)b;
  }

  // neighbours: the 27 boxes with ||j - k||_inf <= 1 that are non-empty (A5)
  for (int d = 1; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    int64_t side = (int64_t)1 << (d - 1);
    L.nbr_off.assign(L.nb + 1, 0);
    std::vector<std::vector<int32_t>> tmp(L.nb);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < L.nb; ++b) {
      const int32_t* k = &L.coords[3 * b];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int64_t a = k[0] + dx, bb = k[1] + dy, c = k[2] + dz;
            if (a < 0 || bb < 0 || c < 0 || a >= side || bb >= side || c >= side) continue;
            int64_t j = find_box(L, morton(a, bb, c));
            if (j >= 0) tmp[b].push_back((int32_t)j);
          }
      std::sort(tmp[b].begin(), tmp[b].end());
    }
    for (int64_t b = 0; b < L.nb; ++b) L.nbr_off[b + 1] = L.nbr_off[b] + (int32_t)tmp[b].size();
    L.nbr.resize(L.nbr_off[L.nb]);
    for (int64_t b = 0; b < L.nb; ++b)
      std::copy(tmp[b].begin(), tmp[b].end(), L.nbr.begin() + L.nbr_off[b]);
  }
  // cousins: children of the parent's neighbours that are not neighbours
  for (int d = 3; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    HostLevel& Pl = P.lev[d - 1];
    std::vector<std::vector<int32_t>> tmp(L.nb);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < L.nb; ++b) {
      const int32_t* k = &L.coords[3 * b];
      int32_t pb = L.parent[b];
      for (int32_t e = Pl.nbr_off[pb]; e < Pl.nbr_off[pb + 1]; ++e) {
        int32_t pn = Pl.nbr[e];
        for (int32_t c = Pl.child_start[pn]; c < Pl.child_end[pn]; ++c) {
          const int32_t* kc = &L.coords[3 * c];
          int m = std::max(std::abs(kc[0] - k[0]), std::max(std::abs(kc[1] - k[1]), std::abs(kc[2] - k[2])));
          if (m > 1) tmp[b].push_back(c);
        }
      }
      std::sort(tmp[b].begin(), tmp[b].end());
    }
    L.cous_off.assign(L.nb + 1, 0);
    for (int64_t b = 0; b < L.nb; ++b) L.cous_off[b + 1] = L.cous_off[b] + (int32_t)tmp[b].size();
    L.cous.resize(L.cous_off[L.nb]);
    for (int64_t b = 0; b < L.nb; ++b)
      std::copy(tmp[b].begin(), tmp[b].end(), L.cous.begin() + L.cous_off[b]);
  }

  double xs_[kMaxP], xa_[kMaxP];
  cheb_nodes(P.Ps, xs_);
  cheb_nodes(P.Pa, xa_);

  const auto t_start = std::chrono::steady_clock::now();
  auto progress = [&](const char* what, int d, int64_t count) {
    if (!pp.verbose) return;
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[ifgf plan] %7.1f s  %s level %d: %lld\n", s, what, d, (long long)count);
    std::fflush(stderr);
  };
  // relevant cones, top-down from level 3 (eq. rele_cone)
  for (int d = 3; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    std::vector<double> Cv, Sv;
    cone_dirs(L.na, Cv, Sv);
    const double* Cd = Cv.data();
    const double* Sd = Sv.data();
    std::vector<std::vector<int32_t>> cones(L.nb);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < L.nb; ++b) {
      std::vector<int32_t>& cl = cones[b];
      const double* cb = &L.centers[3 * b];
      for (int32_t e = L.cous_off[b]; e < L.cous_off[b + 1]; ++e) {
        int32_t c = L.cous[e];
        for (int32_t i = L.start[c]; i < L.end[c]; ++i) {
          const double* xi = &P.xs[3 * i];
          cl.push_back(cone_index(xi[0] - cb[0], xi[1] - cb[1], xi[2] - cb[2], L.h, L.ns, L.na, Cd, Sd));
        }
      }
      if (d >= 4) {
        const HostLevel& Pl = P.lev[d - 1];
        int32_t pb = L.parent[b];
        const double* cp = &Pl.centers[3 * pb];
        for (int64_t q = Pl.slot_off[pb]; q < Pl.slot_off[pb + 1]; ++q) {
          for (int k = 0; k < npts; ++k) {
            double X[3];
            cone_point(Pl, cp, Pl.slot_cone[q], k, P.Ps, P.Pa, xs_, xa_, X);
            cl.push_back(cone_index(X[0] - cb[0], X[1] - cb[1], X[2] - cb[2], L.h, L.ns, L.na, Cd, Sd));
          }
        }
      }
      std::sort(cl.begin(), cl.end());
      cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
    }
    L.slot_off.assign(L.nb + 1, 0);
    for (int64_t b = 0; b < L.nb; ++b) L.slot_off[b + 1] = L.slot_off[b] + (int64_t)cones[b].size();
    L.nslots = L.slot_off[L.nb];
    L.slot_cone.resize(L.nslots);
    L.slot_box.resize(L.nslots);
    for (int64_t b = 0; b < L.nb; ++b) {
      std::copy(cones[b].begin(), cones[b].end(), L.slot_cone.begin() + L.slot_off[b]);
      std::fill(L.slot_box.begin() + L.slot_off[b], L.slot_box.begin() + L.slot_off[b + 1], (int32_t)b);
    }
    // target pairs: per sorted point, the slots of the cousins of its level-d box
    std::vector<int32_t> box_of(n);
    for (int64_t b = 0; b < L.nb; ++b)
      for (int32_t i = L.start[b]; i < L.end[b]; ++i) box_of[i] = (int32_t)b;
    L.tp_off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
      L.tp_off[i + 1] = L.tp_off[i] + (L.cous_off[box_of[i] + 1] - L.cous_off[box_of[i]]);
    L.tp_slot.resize(L.tp_off[n]);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
    for (int64_t i = 0; i < n; ++i) {
      int32_t T = box_of[i];
      const double* xi = &P.xs[3 * i];
      int64_t o = L.tp_off[i];
      for (int32_t e = L.cous_off[T]; e < L.cous_off[T + 1]; ++e, ++o) {
        int32_t B = L.cous[e];
        const double* cb = &L.centers[3 * B];
        int cone = cone_index(xi[0] - cb[0], xi[1] - cb[1], xi[2] - cb[2], L.h, L.ns, L.na, Cd, Sd);
        int s = find_slot(L, B, cone);
        if (s < 0) ++bad;
        L.tp_slot[o] = s;
      }
    }
    if (bad) { err = "internal: cousin target outside relevant cones"; return -1; }
    build_target_tiles(L, n, pp.target_chunk_pairs > 0 ? pp.target_chunk_pairs : kTargetChunkPairs);
    progress("relevant cones and target pairs", d, L.nslots);
    // propagation pairs into level d-1
    if (d >= 4) {
      HostLevel& Pl = P.lev[d - 1];
      Pl.pp_off.assign(Pl.nslots + 1, 0);
      for (int64_t q = 0; q < Pl.nslots; ++q) {
        int32_t pb = Pl.slot_box[q];
        Pl.pp_off[q + 1] = Pl.pp_off[q] + (int64_t)(Pl.child_end[pb] - Pl.child_start[pb]) * npts;
      }
      Pl.pp_slot.resize(Pl.pp_off[Pl.nslots]);
      int bad2 = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad2)
      for (int64_t q = 0; q < Pl.nslots; ++q) {
        int32_t pb = Pl.slot_box[q];
        const double* cp = &Pl.centers[3 * pb];
        int64_t o = Pl.pp_off[q];
        for (int32_t c = Pl.child_start[pb]; c < Pl.child_end[pb]; ++c) {
          const double* cc = &L.centers[3 * c];
          for (int k = 0; k < npts; ++k, ++o) {
            double X[3];
            cone_point(Pl, cp, Pl.slot_cone[q], k, P.Ps, P.Pa, xs_, xa_, X);
            int cone = cone_index(X[0] - cc[0], X[1] - cc[1], X[2] - cc[2], L.h, L.ns, L.na, Cd, Sd);
            int s = find_slot(L, c, cone);
            if (s < 0) ++bad2;
            Pl.pp_slot[o] = s;
          }
        }
      }
      if (bad2) { err = "internal: parent point outside relevant child cones"; return -1; }
      if (npts <= 256) {
        if (Pl.pp_off[Pl.nslots] >= ((int64_t)1 << 31)) {
          err = "too many propagation pairs on one level for the 32-bit tile records";
          return -1;
        }
        if (L.nb >= ((int64_t)1 << 26)) {
          err = "too many boxes on one level for the tile records (child box << 5 | count)";
          return -1;
        }
        build_prop_groups(Pl, L, npts);
        progress("propagation groups into", d - 1, Pl.pp_off[Pl.nslots]);
      }
    }
  }

  // unit counts
  {
    HostLevel& L = P.lev[D];
    int64_t near = 0;
    for (int64_t b = 0; b < L.nb; ++b) {
      int64_t src = 0;
      for (int32_t e = L.nbr_off[b]; e < L.nbr_off[b + 1]; ++e) src += L.end[L.nbr[e]] - L.start[L.nbr[e]];
      near += (int64_t)(L.end[b] - L.start[b]) * src;
    }
    P.near_pairs = near - n;
    int64_t lp = 0;
    if (D >= 3)
      for (int64_t q = 0; q < L.nslots; ++q) lp += (int64_t)npts * (L.end[L.slot_box[q]] - L.start[L.slot_box[q]]);
    P.leaf_pairs = lp;
  }
  return 0;
}

}  // namespace ifgf
