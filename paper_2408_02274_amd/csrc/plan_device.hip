// IFGF plan built on gfx950 (Sec. III-G algorithm step 1): Morton keys and a
// stable radix sort of the points, the non-empty boxes of every level
// (eq. rele_boxes) by scan and compaction, parents and children, neighbour
// and cousin lists (eq. box_neighbor, box_cousin), the relevant cone segments
// of every box from level 3 down (eq. rele_cone, Remark 2 cone counts), the
// cone slot of every (target, cousin box) and (parent interpolation point,
// child box) pair, and the propagation groups and tiles.
//
// The tables equal those of the host builder bit for bit: every discrete
// decision (the box of a point, the cone of a point) is taken with the
// host's formula and operation order, contraction off, using only +, -, *,
// /, sqrt and floor against host-computed tables of the cone boundary
// directions; the interpolation points take their sines and cosines from
// host tables as well.
//
// Relevant cones: each box owns a bitmap of its n_s x n_a x 2 n_a cones; the
// cousin targets and the parents' interpolation points set their bits with
// atomic ORs, an exclusive scan of the words' population counts numbers the
// set bits (box-major, cone-ascending: the slot order), and a pair's slot is
// then the scan value of its word plus the set bits below its cone.
//
// Propagation groups: for every (parent slot, child) the interpolation
// points are ranked by child cone slot (ties by point index: a stable sort)
// on one wavefront; equal slots form a group, groups are cut into tiles of
// at most 16 points.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "plan.hpp"
#include "util.hpp"

namespace ifgf {
namespace {

constexpr double kPiD = 3.141592653589793;
constexpr double kTwoPiD = 2.0 * 3.141592653589793;

inline unsigned nblocks(int64_t w, int bs) { return (unsigned)((w + bs - 1) / bs); }

__host__ __device__ inline uint64_t morton_key(int64_t kx, int64_t ky, int64_t kz) {
  uint64_t key = 0;
  for (int b = 0; b < 20; ++b) {
    key |= (uint64_t)((kx >> b) & 1) << (3 * b + 2);
    key |= (uint64_t)((ky >> b) & 1) << (3 * b + 1);
    key |= (uint64_t)((kz >> b) & 1) << (3 * b);
  }
  return key;
}

// Cone of the offset (dx, dy, dz) from a box centre (radius h), n_s x n_a x
// 2 n_a cones (Sec. III-F), decided as the host builder decides it: s = h / r
// against the radial intervals, cos theta against the boundary cosines C[k]
// and the azimuth by cross products with the boundary rays (C[k], S[k]) in
// the point's half plane.
__device__ inline int cone_of(double dx, double dy, double dz, double h, int ns, int na, double eta,
                              const double* __restrict__ C, const double* __restrict__ S) {
#pragma clang fp contract(off)
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double s = h / r;
  double ct = dz / r;
  if (ct > 1.0) ct = 1.0;
  if (ct < -1.0) ct = -1.0;
  const double ds = eta / ns;
  const double fs = floor(s / ds);
  const int64_t is = (int64_t)fmin(fs, (double)(ns - 1));
  int lo = 1, hi = na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ct <= C[mid]) lo = mid + 1;
    else hi = mid;
  }
  const int64_t it = lo - 1;
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

// Interpolation point k of cone `cone` of a box centred at c (radius h); the
// sines and cosines of its polar and azimuthal nodes come from host tables
// (ang[0..3]: sin, cos of theta [n_a][P_a]; sin, cos of phi [2 n_a][P_a]).
__device__ inline void cone_point_d(int ns, int na, double h, double eta, const double* c, int cone, int k, int Ps,
                                    int Pa, const double* xs, const double* const* ang, double* X) {
#pragma clang fp contract(off)
  const int ip = cone % (2 * na);
  const int it = (cone / (2 * na)) % na;
  const int is = cone / (2 * na * na);
  const int kp = k % Pa, kt = (k / Pa) % Pa, ks = k / (Pa * Pa);
  const double ds = eta / ns;
  const double s = (is + 0.5) * ds + 0.5 * ds * xs[ks];
  const double rr = h / s;
  const double st = ang[0][it * Pa + kt], ctt = ang[1][it * Pa + kt];
  const double sp = ang[2][ip * Pa + kp], cp = ang[3][ip * Pa + kp];
  X[0] = c[0] + rr * (st * cp);
  X[1] = c[1] + rr * (st * sp);
  X[2] = c[2] + rr * ctt;
}

__device__ inline int64_t find_key(const int64_t* key, int64_t nb, int64_t k) {
  int64_t lo = 0, hi = nb;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return (lo < nb && key[lo] == k) ? lo : -1;
}

// ----------------------------------------------------------------- points
__global__ void k_point_keys(const double* __restrict__ x, int64_t n, double o0, double o1, double o2, double HD,
                             int64_t nmax, uint64_t* __restrict__ key, int32_t* __restrict__ kD,
                             int32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double o[3] = {o0, o1, o2};
  int64_t k[3];
  for (int c = 0; c < 3; ++c) {
    const double f = floor((x[3 * i + c] - o[c]) / HD);
    int64_t v = (int64_t)f;
    v = v < 0 ? 0 : (v > nmax - 1 ? nmax - 1 : v);
    k[c] = v;
    kD[3 * i + c] = (int32_t)v;
  }
  key[i] = morton_key(k[0], k[1], k[2]);
  idx[i] = (int32_t)i;
}

__global__ void k_gather_points(const int32_t* __restrict__ perm, int64_t n, const double* __restrict__ x,
                                const int32_t* __restrict__ kD, double* __restrict__ xs, int32_t* __restrict__ skD) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  for (int c = 0; c < 3; ++c) {
    xs[3 * i + c] = x[3 * j + c];
    skD[3 * i + c] = kD[3 * j + c];
  }
}

// ----------------------------------------------------------------- boxes
__global__ void k_box_flags(const uint64_t* __restrict__ skey, int64_t n, int shift, int64_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (skey[i] >> shift) != (skey[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_box_make(const uint64_t* __restrict__ skey, const int32_t* __restrict__ skD,
                           const int64_t* __restrict__ flag, const int64_t* __restrict__ bid, int64_t n, int shift,
                           int cshift, int32_t* __restrict__ start, int64_t* __restrict__ key,
                           int32_t* __restrict__ coords, int32_t* __restrict__ box_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = bid[i] + flag[i] - 1;
  box_of[i] = (int32_t)b;
  if (!flag[i]) return;
  start[b] = (int32_t)i;
  key[b] = (int64_t)(skey[i] >> shift);
  for (int c = 0; c < 3; ++c) coords[3 * b + c] = skD[3 * i + c] >> cshift;
}

__global__ void k_box_finish(const int32_t* __restrict__ start, const int32_t* __restrict__ coords, int64_t nb,
                             int64_t n, double o0, double o1, double o2, double H, int32_t* __restrict__ end,
                             double* __restrict__ centers) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  end[b] = (b + 1 < nb) ? start[b + 1] : (int32_t)n;
  const double o[3] = {o0, o1, o2};
  for (int c = 0; c < 3; ++c) centers[3 * b + c] = o[c] + H * (coords[3 * b + c] + 0.5);
}

__global__ void k_parents(const int64_t* __restrict__ key, int64_t nb, const int64_t* __restrict__ pkey, int64_t pnb,
                          int32_t* __restrict__ parent) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  parent[b] = (int32_t)find_key(pkey, pnb, (int64_t)((uint64_t)key[b] >> 3));
}

__global__ void k_children(const int32_t* __restrict__ parent, int64_t nb, int32_t* __restrict__ cs,
                           int32_t* __restrict__ ce) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int32_t pb = parent[b];
  if (b == 0 || parent[b - 1] != pb) cs[pb] = (int32_t)b;
  if (b == nb - 1 || parent[b + 1] != pb) ce[pb] = (int32_t)(b + 1);
}

// FILL = false: cnt[b] = neighbours of b; FILL = true: the ascending list at off[b].
template <bool FILL>
__global__ void k_neighbours(const int64_t* __restrict__ key, const int32_t* __restrict__ coords, int64_t nb,
                             int64_t side, int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                             int32_t* __restrict__ nbr) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int32_t tmp[27];
  int m = 0;
  const int32_t* k = coords + 3 * b;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        const int64_t a = k[0] + dx, bb = k[1] + dy, c = k[2] + dz;
        if (a < 0 || bb < 0 || c < 0 || a >= side || bb >= side || c >= side) continue;
        const int64_t j = find_key(key, nb, (int64_t)morton_key(a, bb, c));
        if (j >= 0) tmp[m++] = (int32_t)j;
      }
  if (!FILL) {
    cnt[b] = m;
    return;
  }
  for (int i = 1; i < m; ++i) {   // insertion sort of <= 27 indices
    const int32_t v = tmp[i];
    int j = i - 1;
    while (j >= 0 && tmp[j] > v) {
      tmp[j + 1] = tmp[j];
      --j;
    }
    tmp[j + 1] = v;
  }
  for (int i = 0; i < m; ++i) nbr[off[b] + i] = tmp[i];
}

// Cousins: children of the parent's neighbours that are not neighbours.
template <bool FILL>
__global__ void k_cousins(const int32_t* __restrict__ coords, const int32_t* __restrict__ parent, int64_t nb,
                          const int64_t* __restrict__ pnbr_off, const int32_t* __restrict__ pnbr,
                          const int32_t* __restrict__ pcs, const int32_t* __restrict__ pce, int64_t* __restrict__ cnt,
                          const int64_t* __restrict__ off, int32_t* __restrict__ cous) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int32_t* k = coords + 3 * b;
  const int32_t pb = parent[b];
  int64_t m = 0, o = FILL ? off[b] : 0;
  for (int64_t e = pnbr_off[pb]; e < pnbr_off[pb + 1]; ++e) {
    const int32_t pn = pnbr[e];
    for (int32_t c = pcs[pn]; c < pce[pn]; ++c) {
      const int32_t* kc = coords + 3 * c;
      const int d = max(abs(kc[0] - k[0]), max(abs(kc[1] - k[1]), abs(kc[2] - k[2])));
      if (d > 1) {
        if (FILL) cous[o + m] = c;
        ++m;
      }
    }
  }
  if (!FILL) cnt[b] = m;
}

// ----------------------------------------------------------- relevant cones
struct LevelGeo {
  const double* centers;
  int64_t nb;
  double h;
  int ns, na;
  int64_t wpb;          // bitmap words per box
  const double* C;      // boundary directions [na + 1]
  const double* S;
  const double* ang[4]; // sin/cos of the polar [na][Pa] and azimuthal [2 na][Pa] interpolation nodes
};

// Cone of every (target, cousin box) pair, its bit set in the cousin's map.
template <bool CONVERT>
__global__ void k_target_cones(LevelGeo G, const double* __restrict__ xs, int64_t n, const int32_t* __restrict__ box_of,
                               const int64_t* __restrict__ cous_off, const int32_t* __restrict__ cous,
                               const int64_t* __restrict__ tp_off, int32_t* __restrict__ tp,
                               unsigned* __restrict__ bits, const int64_t* __restrict__ word_off, double eta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t T = box_of[i];
  int64_t o = tp_off[i];
  for (int64_t e = cous_off[T]; e < cous_off[T + 1]; ++e, ++o) {
    const int32_t B = cous[e];
    if (!CONVERT) {
      const double* cb = G.centers + 3 * (int64_t)B;
      const int cone =
          cone_of(xs[3 * i] - cb[0], xs[3 * i + 1] - cb[1], xs[3 * i + 2] - cb[2], G.h, G.ns, G.na, eta, G.C, G.S);
      tp[o] = cone;
      atomicOr(&bits[(int64_t)B * G.wpb + (cone >> 5)], 1u << (cone & 31));
    } else {
      const int cone = tp[o];
      const int64_t w = (int64_t)B * G.wpb + (cone >> 5);
      tp[o] = (int32_t)(word_off[w] + __popc(bits[w] & ((1u << (cone & 31)) - 1u)));
    }
  }
}

// Cone of every (parent interpolation point, child box) pair; one block per
// parent slot q, one thread per point.
template <bool CONVERT>
__global__ void k_parent_cones(LevelGeo C, LevelGeo P, const int32_t* __restrict__ pslot_box,
                               const int32_t* __restrict__ pslot_cone, const int32_t* __restrict__ pcs,
                               const int32_t* __restrict__ pce, const int64_t* __restrict__ pp_off, int npts, int Ps,
                               int Pa, const double* __restrict__ xs_nodes, int32_t* __restrict__ pp,
                               unsigned* __restrict__ bits, const int64_t* __restrict__ word_off, double eta) {
  const int64_t q = blockIdx.x;
  const int32_t pb = pslot_box[q];
  const int32_t c0 = pcs[pb], c1 = pce[pb];
  double xs[8];
  for (int t = 0; t < Ps; ++t) xs[t] = xs_nodes[t];
  for (int k = threadIdx.x; k < npts; k += blockDim.x) {
    double X[3];
    if (!CONVERT)
      cone_point_d(P.ns, P.na, P.h, eta, P.centers + 3 * (int64_t)pb, pslot_cone[q], k, Ps, Pa, xs, P.ang, X);
    for (int32_t c = c0; c < c1; ++c) {
      const int64_t o = pp_off[q] + (int64_t)(c - c0) * npts + k;
      if (!CONVERT) {
        const double* cc = C.centers + 3 * (int64_t)c;
        const int cone = cone_of(X[0] - cc[0], X[1] - cc[1], X[2] - cc[2], C.h, C.ns, C.na, eta, C.C, C.S);
        pp[o] = cone;
        atomicOr(&bits[(int64_t)c * C.wpb + (cone >> 5)], 1u << (cone & 31));
      } else {
        const int cone = pp[o];
        const int64_t w = (int64_t)c * C.wpb + (cone >> 5);
        pp[o] = (int32_t)(word_off[w] + __popc(bits[w] & ((1u << (cone & 31)) - 1u)));
      }
    }
  }
}

__global__ void k_popcount(const unsigned* __restrict__ bits, int64_t nw, int64_t* __restrict__ cnt) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  cnt[w] = __popc(bits[w]);
}

__global__ void k_slots(const unsigned* __restrict__ bits, const int64_t* __restrict__ word_off, int64_t nw,
                        int64_t wpb, int32_t* __restrict__ slot_cone, int32_t* __restrict__ slot_box) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  unsigned v = bits[w];
  int64_t o = word_off[w];
  const int64_t b = w / wpb;
  const int64_t base = (w % wpb) * 32;
  while (v) {
    const int j = __ffs(v) - 1;
    slot_cone[o] = (int32_t)(base + j);
    slot_box[o] = (int32_t)b;
    ++o;
    v &= v - 1u;
  }
}

__global__ void k_slot_off(const int64_t* __restrict__ word_off, int64_t nb, int64_t wpb, int64_t nslots,
                           int64_t* __restrict__ slot_off) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  slot_off[b] = b < nb ? word_off[b * wpb] : nslots;
}

__global__ void k_pair_counts(const int32_t* __restrict__ box_of, int64_t n, const int64_t* __restrict__ cous_off,
                              int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t T = box_of[i];
  cnt[i] = cous_off[T + 1] - cous_off[T];
}

__global__ void k_prop_counts(const int32_t* __restrict__ slot_box, int64_t Q, const int32_t* __restrict__ cs,
                              const int32_t* __restrict__ ce, int npts, int64_t* __restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const int32_t pb = slot_box[q];
  cnt[q] = (int64_t)(ce[pb] - cs[pb]) * npts;
}

// ------------------------------------------------------ propagation groups
// One wavefront per (parent slot q, child j), f = pp_off[q] / npts + j.
// FILL = false: groups and tiles of f; FILL = true: sorted points, records.
template <bool FILL>
__global__ void __launch_bounds__(64) k_prop_groups(const int64_t* __restrict__ pp_off, int64_t Q, int npts,
                                                    const int32_t* __restrict__ pp, const int32_t* __restrict__ pslot_box,
                                                    const int32_t* __restrict__ pcs,
                                                    const int32_t* __restrict__ cslot_cone,
                                                    int64_t* __restrict__ ngroups, int64_t* __restrict__ ntiles,
                                                    const int64_t* __restrict__ tile_off, uint8_t* __restrict__ pts,
                                                    int32_t* __restrict__ rec) {
  __shared__ int32_t s[256];
  __shared__ int32_t first[256];   // 1 if k is the first point of its slot
  __shared__ int32_t cntv[256];    // points of k's slot (first points only)
  const int64_t f = blockIdx.x;
  const int lane = threadIdx.x;
  // the parent slot q whose children hold f
  int64_t lo = 0, hi = Q;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (pp_off[mid] / npts <= f) lo = mid;
    else hi = mid;
  }
  const int64_t q = lo;
  const int64_t j = f - pp_off[q] / npts;
  const int64_t base = pp_off[q] + j * npts;
  for (int k = lane; k < npts; k += 64) s[k] = pp[base + k];
  __syncthreads();
  int64_t g = 0, t = 0;
  for (int k = lane; k < npts; k += 64) {
    int fst = 1, c = 0;
    for (int k2 = 0; k2 < npts; ++k2) {
      if (s[k2] == s[k]) {
        ++c;
        if (k2 < k) fst = 0;
      }
    }
    first[k] = fst;
    cntv[k] = c;
    if (fst) {
      ++g;
      t += (c + 15) / 16;
    }
  }
  if (!FILL) {
    for (int off = 32; off > 0; off >>= 1) {
      g += __shfl_xor(g, off, 64);
      t += __shfl_xor(t, off, 64);
    }
    if (lane == 0) {
      ngroups[f] = g;
      ntiles[f] = t;
    }
    return;
  }
  __syncthreads();
  const int32_t pb = pslot_box[q];
  const int32_t cbox = pcs[pb] + (int32_t)j;
  for (int k = lane; k < npts; k += 64) {
    const int32_t v = s[k];
    int rank = 0;
    int64_t tb = 0;
    for (int k2 = 0; k2 < npts; ++k2) {
      const int32_t v2 = s[k2];
      if (v2 < v || (v2 == v && k2 < k)) ++rank;
      if (first[k2] && v2 < v) tb += (cntv[k2] + 15) / 16;
    }
    pts[base + rank] = (uint8_t)k;
    if (first[k]) {
      // rank of the slot's first point = its group's first sorted position
      int64_t tile = tile_off[f] + tb;
      for (int t0 = 0; t0 < cntv[k]; t0 += 16, ++tile) {
        int32_t* r = rec + 4 * tile;
        r[0] = v;
        r[1] = (cbox << 5) | min(16, cntv[k] - t0);
        r[2] = (int32_t)(base + rank + t0);
        r[3] = cslot_cone[v];
      }
    }
  }
}

// ----------------------------------------------------------------- helpers
struct Dev {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  ~Dev() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(int64_t count) {
    void* p = nullptr;
    if (err != hipSuccess) return nullptr;
    const size_t bytes = std::max<size_t>(sizeof(T) * (size_t)std::max<int64_t>(count, 1), 256);
    if ((err = hipMalloc(&p, bytes)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  void release(void* p) {
    for (auto& q : ptrs)
      if (q == p) {
        (void)hipFree(q);
        q = nullptr;
      }
  }
};

template <class T>
hipError_t down(std::vector<T>& v, const T* d, int64_t count) {
  v.resize(count);
  if (count <= 0) return hipSuccess;
  return hipMemcpy(v.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost);
}

template <class T>
hipError_t up(const std::vector<T>& v, T* d) {
  if (v.empty()) return hipSuccess;
  return hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

// out[0..n) = exclusive sum of in, out[n] = total (out has n + 1 entries)
hipError_t scan_total(Dev& D, const int64_t* in, int64_t* out, int64_t n, int64_t* total) {
  *total = 0;
  if (n <= 0) return hipMemset(out, 0, sizeof(int64_t));
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n);
  if (e != hipSuccess) return e;
  void* tmp = D.alloc<char>((int64_t)bytes);
  if (!tmp) return D.err;
  if ((e = hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, n)) != hipSuccess) return e;
  D.release(tmp);
  int64_t last[2];
  if ((e = hipMemcpy(&last[0], out + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if ((e = hipMemcpy(&last[1], in + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  *total = last[0] + last[1];
  return hipMemcpy(out + n, total, sizeof(int64_t), hipMemcpyHostToDevice);
}

struct DevLevelTables {
  int64_t nb = 0;
  int64_t* key = nullptr;
  int32_t *coords = nullptr, *start = nullptr, *end = nullptr, *parent = nullptr, *cs = nullptr, *ce = nullptr;
  int32_t* box_of = nullptr;
  double* centers = nullptr;
  int64_t* nbr_off = nullptr;
  int32_t* nbr = nullptr;
  int64_t* cous_off = nullptr;
  int32_t* cous = nullptr;
  int64_t nslots = 0;
  int32_t *slot_cone = nullptr, *slot_box = nullptr;
};

}  // namespace

int build_device_plan(HostPlan& P, int64_t n, const double* x, const double* nrm, const double* w, double k0,
                      double k1, const PlanParams& pp, std::string& err) {
  if (n >= ((int64_t)1 << 31)) {
    err = "the device planner needs fewer than 2^31 points";
    return -1;
  }
  P.n = n;
  P.k[0] = k0;
  P.k[1] = k1;
  P.kmax = std::max(k0, k1);
  P.Ps = pp.Ps;
  P.Pa = pp.Pa;
  P.npts = pp.Ps * pp.Pa * pp.Pa;
  const int npts = P.npts;
  const double eta = std::sqrt(3.0) / 3.0;
  const double sqrt3 = std::sqrt(3.0);

  // bounding cube and depth: the host builder's formulas
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) lo[c] = hi[c] = x[c];
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
  const double lam = 2.0 * kPiD / P.kmax;
  int D = 1;
  while (std::ldexp(P.H1, -(D - 1)) > pp.leaf_wavelengths * lam) {
    ++D;
    if (D > 21) {
      err = "octree deeper than 21 levels";
      return -1;
    }
  }
  P.D = D;
  for (int c = 0; c < 3; ++c) P.origin[c] = P.center[c] - 0.5 * P.H1;
  const double HD = std::ldexp(P.H1, -(D - 1));
  const int64_t nmax = (int64_t)1 << (D - 1);

  const auto t_start = std::chrono::steady_clock::now();
  auto progress = [&](const char* what, int d, int64_t count) {
    if (!pp.verbose) return;
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[ifgf plan, device] %7.1f s  %s level %d: %lld\n", s, what, d, (long long)count);
    std::fflush(stderr);
  };
  Dev M;
  hipError_t e = hipSuccess;
  auto fail = [&](const char* where) {
    err = std::string("device planner, ") + where + ": " + hipGetErrorString(M.err != hipSuccess ? M.err : e);
    return -2;
  };
#define CK(expr, where)                              \
  do {                                               \
    if ((e = (expr)) != hipSuccess) return fail(where); \
  } while (0)
#define CKA(ptr, where)                  \
  do {                                   \
    if (!(ptr)) return fail(where);      \
  } while (0)

  // Morton keys of the leaves and a stable sort by key
  double* d_x = M.alloc<double>(3 * n);
  uint64_t* d_key = M.alloc<uint64_t>(n);
  uint64_t* d_skey = M.alloc<uint64_t>(n);
  int32_t* d_kD = M.alloc<int32_t>(3 * n);
  int32_t* d_idx = M.alloc<int32_t>(n);
  int32_t* d_perm = M.alloc<int32_t>(n);
  CKA(d_x && d_key && d_skey && d_kD && d_idx && d_perm, "allocation");
  CK(hipMemcpy(d_x, x, sizeof(double) * 3 * n, hipMemcpyHostToDevice), "copy");
  hipLaunchKernelGGL(k_point_keys, dim3(nblocks(n, 256)), dim3(256), 0, 0, d_x, n, P.origin[0], P.origin[1],
                     P.origin[2], HD, nmax, d_key, d_kD, d_idx);
  CK(hipGetLastError(), "keys");
  {
    const int end_bit = std::max(1, 3 * (D - 1));
    size_t bytes = 0;
    CK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, d_key, d_skey, d_idx, d_perm, (int)n, 0, end_bit),
       "sort");
    void* tmp = M.alloc<char>((int64_t)bytes);
    CKA(tmp, "allocation");
    CK(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, d_key, d_skey, d_idx, d_perm, (int)n, 0, end_bit), "sort");
    M.release(tmp);
  }
  double* d_xs = M.alloc<double>(3 * n);
  int32_t* d_skD = M.alloc<int32_t>(3 * n);
  CKA(d_xs && d_skD, "allocation");
  hipLaunchKernelGGL(k_gather_points, dim3(nblocks(n, 256)), dim3(256), 0, 0, d_perm, n, d_x, d_kD, d_xs, d_skD);
  CK(hipGetLastError(), "gather");
  M.release(d_key);
  M.release(d_idx);
  M.release(d_kD);
  {
    std::vector<int32_t> perm;
    CK(down(perm, d_perm, n), "copy");
    P.perm.assign(perm.begin(), perm.end());
  }
  CK(down(P.xs, d_xs, 3 * n), "copy");
  P.nrm.resize(3 * n);
  P.w.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t j = P.perm[i];
    for (int c = 0; c < 3; ++c) P.nrm[3 * i + c] = nrm[3 * j + c];
    P.w[i] = w[j];
  }

  // cone counts per level (Remark 2)
  P.lev.assign(D + 1, HostLevel());
  {
    int ns = pp.ns_init, na = pp.na_init;
    for (int d = D; d >= 3; --d) {
      const double Hd = std::ldexp(P.H1, -(d - 1));
      const int a = (P.kmax * Hd > 0.5) ? 2 : 1;
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

  // boxes, parents, children, neighbours and cousins of every level
  std::vector<DevLevelTables> T(D + 1);
  int64_t* d_flag = M.alloc<int64_t>(n);
  int64_t* d_bid = M.alloc<int64_t>(n + 1);
  CKA(d_flag && d_bid, "allocation");
  for (int d = 1; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    DevLevelTables& G = T[d];
    L.d = d;
    L.H = std::ldexp(P.H1, -(d - 1));
    L.h = sqrt3 / 2.0 * L.H;
    const int shift = 3 * (D - d);
    hipLaunchKernelGGL(k_box_flags, dim3(nblocks(n, 256)), dim3(256), 0, 0, d_skey, n, shift, d_flag);
    CK(hipGetLastError(), "box flags");
    int64_t nb = 0;
    CK(scan_total(M, d_flag, d_bid, n, &nb), "box scan");
    G.nb = L.nb = nb;
    G.key = M.alloc<int64_t>(nb);
    G.coords = M.alloc<int32_t>(3 * nb);
    G.start = M.alloc<int32_t>(nb);
    G.end = M.alloc<int32_t>(nb);
    G.centers = M.alloc<double>(3 * nb);
    G.box_of = M.alloc<int32_t>(n);
    CKA(G.key && G.coords && G.start && G.end && G.centers && G.box_of, "allocation");
    hipLaunchKernelGGL(k_box_make, dim3(nblocks(n, 256)), dim3(256), 0, 0, d_skey, d_skD, d_flag, d_bid, n, shift,
                       D - d, G.start, G.key, G.coords, G.box_of);
    hipLaunchKernelGGL(k_box_finish, dim3(nblocks(nb, 256)), dim3(256), 0, 0, G.start, G.coords, nb, n, P.origin[0],
                       P.origin[1], P.origin[2], L.H, G.end, G.centers);
    CK(hipGetLastError(), "boxes");
    CK(down(L.key, G.key, nb), "copy");
    CK(down(L.coords, G.coords, 3 * nb), "copy");
    CK(down(L.start, G.start, nb), "copy");
    CK(down(L.end, G.end, nb), "copy");
    CK(down(L.centers, G.centers, 3 * nb), "copy");
    if (d >= 2) {
      DevLevelTables& Pg = T[d - 1];
      HostLevel& Pl = P.lev[d - 1];
      G.parent = M.alloc<int32_t>(nb);
      Pg.cs = M.alloc<int32_t>(Pg.nb);
      Pg.ce = M.alloc<int32_t>(Pg.nb);
      CKA(G.parent && Pg.cs && Pg.ce, "allocation");
      CK(hipMemset(Pg.cs, 0, sizeof(int32_t) * Pg.nb), "memset");
      CK(hipMemset(Pg.ce, 0, sizeof(int32_t) * Pg.nb), "memset");
      hipLaunchKernelGGL(k_parents, dim3(nblocks(nb, 256)), dim3(256), 0, 0, G.key, nb, Pg.key, Pg.nb, G.parent);
      hipLaunchKernelGGL(k_children, dim3(nblocks(nb, 256)), dim3(256), 0, 0, G.parent, nb, Pg.cs, Pg.ce);
      CK(hipGetLastError(), "parents");
      CK(down(L.parent, G.parent, nb), "copy");
      CK(down(Pl.child_start, Pg.cs, Pg.nb), "copy");
      CK(down(Pl.child_end, Pg.ce, Pg.nb), "copy");
    }
    // neighbours (27 boxes with ||j - k||_inf <= 1 that are non-empty)
    {
      int64_t* cnt = M.alloc<int64_t>(nb);
      G.nbr_off = M.alloc<int64_t>(nb + 1);
      CKA(cnt && G.nbr_off, "allocation");
      const int64_t side = (int64_t)1 << (d - 1);
      hipLaunchKernelGGL((k_neighbours<false>), dim3(nblocks(nb, 256)), dim3(256), 0, 0, G.key, G.coords, nb, side,
                         cnt, nullptr, nullptr);
      int64_t tot = 0;
      CK(scan_total(M, cnt, G.nbr_off, nb, &tot), "neighbour scan");
      G.nbr = M.alloc<int32_t>(tot);
      CKA(G.nbr, "allocation");
      hipLaunchKernelGGL((k_neighbours<true>), dim3(nblocks(nb, 256)), dim3(256), 0, 0, G.key, G.coords, nb, side,
                         nullptr, G.nbr_off, G.nbr);
      CK(hipGetLastError(), "neighbours");
      M.release(cnt);
      std::vector<int64_t> off;
      CK(down(off, G.nbr_off, nb + 1), "copy");
      L.nbr_off.assign(off.begin(), off.end());
      CK(down(L.nbr, G.nbr, tot), "copy");
    }
  }
  M.release(d_flag);
  M.release(d_bid);
  {
    std::vector<int32_t> lop;
    CK(down(lop, T[D].box_of, n), "copy");
    P.leaf_of_point = lop;
  }
  for (int d = 3; d <= D; ++d) {
    DevLevelTables& G = T[d];
    DevLevelTables& Pg = T[d - 1];
    int64_t* cnt = M.alloc<int64_t>(G.nb);
    G.cous_off = M.alloc<int64_t>(G.nb + 1);
    CKA(cnt && G.cous_off, "allocation");
    hipLaunchKernelGGL((k_cousins<false>), dim3(nblocks(G.nb, 256)), dim3(256), 0, 0, G.coords, G.parent, G.nb,
                       Pg.nbr_off, Pg.nbr, Pg.cs, Pg.ce, cnt, nullptr, nullptr);
    int64_t tot = 0;
    CK(scan_total(M, cnt, G.cous_off, G.nb, &tot), "cousin scan");
    G.cous = M.alloc<int32_t>(tot);
    CKA(G.cous, "allocation");
    hipLaunchKernelGGL((k_cousins<true>), dim3(nblocks(G.nb, 256)), dim3(256), 0, 0, G.coords, G.parent, G.nb,
                       Pg.nbr_off, Pg.nbr, Pg.cs, Pg.ce, nullptr, G.cous_off, G.cous);
    CK(hipGetLastError(), "cousins");
    M.release(cnt);
    std::vector<int64_t> off;
    CK(down(off, G.cous_off, G.nb + 1), "copy");
    P.lev[d].cous_off.assign(off.begin(), off.end());
    CK(down(P.lev[d].cous, G.cous, tot), "copy");
  }

  // Chebyshev nodes of the cone grids
  std::vector<double> xs_n(pp.Ps), xa_n(pp.Pa);
  for (int k = 0; k < pp.Ps; ++k) xs_n[k] = std::cos((k + 0.5) * kPiD / pp.Ps);
  for (int k = 0; k < pp.Pa; ++k) xa_n[k] = std::cos((k + 0.5) * kPiD / pp.Pa);
  double* d_xsn = M.alloc<double>(pp.Ps);
  CKA(d_xsn, "allocation");
  CK(up(xs_n, d_xsn), "copy");
  // per level: boundary directions, and sin/cos of the polar and azimuthal
  // interpolation nodes (the host builder's values)
  std::vector<double*> d_C(D + 1, nullptr), d_S(D + 1, nullptr);
  std::vector<std::array<double*, 4>> d_ang(D + 1);
  for (int d = 3; d <= D; ++d) {
    const int na = P.lev[d].na;
    std::vector<double> C, S;
    cone_dirs(na, C, S);
    const double da = kPiD / na;
    std::vector<double> st(na * pp.Pa), ct(na * pp.Pa), sp(2 * na * pp.Pa), cp(2 * na * pp.Pa);
    for (int it = 0; it < na; ++it)
      for (int kt = 0; kt < pp.Pa; ++kt) {
        const double t = (it + 0.5) * da + 0.5 * da * xa_n[kt];
        st[it * pp.Pa + kt] = std::sin(t);
        ct[it * pp.Pa + kt] = std::cos(t);
      }
    for (int ip = 0; ip < 2 * na; ++ip)
      for (int kp = 0; kp < pp.Pa; ++kp) {
        const double f = (ip + 0.5) * da + 0.5 * da * xa_n[kp];
        sp[ip * pp.Pa + kp] = std::sin(f);
        cp[ip * pp.Pa + kp] = std::cos(f);
      }
    d_C[d] = M.alloc<double>(na + 1);
    d_S[d] = M.alloc<double>(na + 1);
    for (int a = 0; a < 4; ++a) d_ang[d][a] = M.alloc<double>(a < 2 ? na * pp.Pa : 2 * na * pp.Pa);
    CKA(d_C[d] && d_S[d] && d_ang[d][0] && d_ang[d][1] && d_ang[d][2] && d_ang[d][3], "allocation");
    CK(up(C, d_C[d]), "copy");
    CK(up(S, d_S[d]), "copy");
    CK(up(st, d_ang[d][0]), "copy");
    CK(up(ct, d_ang[d][1]), "copy");
    CK(up(sp, d_ang[d][2]), "copy");
    CK(up(cp, d_ang[d][3]), "copy");
  }

  // relevant cones, top-down from level 3 (eq. rele_cone)
  for (int d = 3; d <= D; ++d) {
    HostLevel& L = P.lev[d];
    DevLevelTables& G = T[d];
    const int64_t wpb = (L.ncones + 31) / 32;
    const int64_t nw = G.nb * wpb;
    unsigned* bits = M.alloc<unsigned>(nw);
    int64_t* tp_off = M.alloc<int64_t>(n + 1);
    int64_t* cnt = M.alloc<int64_t>(n);
    CKA(bits && tp_off && cnt, "allocation");
    CK(hipMemset(bits, 0, sizeof(unsigned) * nw), "memset");
    LevelGeo Cg{G.centers, G.nb, L.h, L.ns, L.na, wpb, d_C[d], d_S[d], {d_ang[d][0], d_ang[d][1], d_ang[d][2], d_ang[d][3]}};
    // cousin targets
    hipLaunchKernelGGL(k_pair_counts, dim3(nblocks(n, 256)), dim3(256), 0, 0, G.box_of, n, G.cous_off, cnt);
    int64_t ntp = 0;
    CK(scan_total(M, cnt, tp_off, n, &ntp), "pair scan");
    M.release(cnt);
    int32_t* tp = M.alloc<int32_t>(ntp);
    CKA(tp, "allocation");
    hipLaunchKernelGGL((k_target_cones<false>), dim3(nblocks(n, 256)), dim3(256), 0, 0, Cg, d_xs, n, G.box_of,
                       G.cous_off, G.cous, tp_off, tp, bits, nullptr, eta);
    CK(hipGetLastError(), "target cones");
    // interpolation points of the parents' relevant cones
    int64_t* pp_off = nullptr;
    int32_t* ppd = nullptr;
    int64_t npp = 0;
    HostLevel& Pl = P.lev[d - 1];
    DevLevelTables& Pg = T[d - 1];
    LevelGeo Pgeo{Pg.centers, Pg.nb, Pl.h, Pl.ns, Pl.na, 0, d_C[d - 1], d_S[d - 1],
                  {d_ang[d - 1][0], d_ang[d - 1][1], d_ang[d - 1][2], d_ang[d - 1][3]}};
    if (d >= 4) {
      const int64_t Q = Pg.nslots;
      int64_t* pc = M.alloc<int64_t>(Q);
      pp_off = M.alloc<int64_t>(Q + 1);
      CKA(pc && pp_off, "allocation");
      if (Q > 0)
        hipLaunchKernelGGL(k_prop_counts, dim3(nblocks(Q, 256)), dim3(256), 0, 0, Pg.slot_box, Q, Pg.cs, Pg.ce,
                           npts, pc);
      CK(scan_total(M, pc, pp_off, Q, &npp), "propagation scan");
      M.release(pc);
      ppd = M.alloc<int32_t>(npp);
      CKA(ppd, "allocation");
      if (Q > 0)
        hipLaunchKernelGGL((k_parent_cones<false>), dim3((unsigned)Q), dim3(256), 0, 0, Cg, Pgeo, Pg.slot_box,
                           Pg.slot_cone, Pg.cs, Pg.ce, pp_off, npts, pp.Ps, pp.Pa, d_xsn, ppd, bits, nullptr, eta);
      CK(hipGetLastError(), "parent cones");
    }
    // number the set bits: the slots of the level
    int64_t* wc = M.alloc<int64_t>(nw);
    int64_t* word_off = M.alloc<int64_t>(nw + 1);
    CKA(wc && word_off, "allocation");
    hipLaunchKernelGGL(k_popcount, dim3(nblocks(nw, 256)), dim3(256), 0, 0, bits, nw, wc);
    int64_t nslots = 0;
    CK(scan_total(M, wc, word_off, nw, &nslots), "slot scan");
    M.release(wc);
    if (nslots >= ((int64_t)1 << 31)) {
      err = "more than 2^31 relevant cones on one level";
      return -1;
    }
    G.nslots = L.nslots = nslots;
    G.slot_cone = M.alloc<int32_t>(nslots);
    G.slot_box = M.alloc<int32_t>(nslots);
    int64_t* slot_off = M.alloc<int64_t>(G.nb + 1);
    CKA(G.slot_cone && G.slot_box && slot_off, "allocation");
    hipLaunchKernelGGL(k_slots, dim3(nblocks(nw, 256)), dim3(256), 0, 0, bits, word_off, nw, wpb, G.slot_cone,
                       G.slot_box);
    hipLaunchKernelGGL(k_slot_off, dim3(nblocks(G.nb + 1, 256)), dim3(256), 0, 0, word_off, G.nb, wpb, nslots,
                       slot_off);
    // cones -> slots
    hipLaunchKernelGGL((k_target_cones<true>), dim3(nblocks(n, 256)), dim3(256), 0, 0, Cg, d_xs, n, G.box_of,
                       G.cous_off, G.cous, tp_off, tp, bits, word_off, eta);
    if (d >= 4 && Pg.nslots > 0)
      hipLaunchKernelGGL((k_parent_cones<true>), dim3((unsigned)Pg.nslots), dim3(256), 0, 0, Cg, Pgeo, Pg.slot_box,
                         Pg.slot_cone, Pg.cs, Pg.ce, pp_off, npts, pp.Ps, pp.Pa, d_xsn, ppd, bits, word_off, eta);
    CK(hipGetLastError(), "slots");
    CK(down(L.slot_off, slot_off, G.nb + 1), "copy");
    CK(down(L.slot_cone, G.slot_cone, nslots), "copy");
    CK(down(L.slot_box, G.slot_box, nslots), "copy");
    CK(down(L.tp_off, tp_off, n + 1), "copy");
    CK(down(L.tp_slot, tp, ntp), "copy");
    M.release(bits);
    M.release(word_off);
    M.release(slot_off);
    M.release(tp);
    M.release(tp_off);
    build_target_tiles(L, n, pp.target_chunk_pairs > 0 ? pp.target_chunk_pairs : kTargetChunkPairs);
    progress("relevant cones and target pairs", d, L.nslots);
    if (d >= 4) {
      const int64_t Q = Pg.nslots;
      CK(down(Pl.pp_off, pp_off, Q + 1), "copy");
      CK(down(Pl.pp_slot, ppd, npp), "copy");
      if (npts <= 256) {
        if (npp >= ((int64_t)1 << 31)) {
          err = "too many propagation pairs on one level for the 32-bit tile records";
          return -1;
        }
        if (L.nb >= ((int64_t)1 << 26)) {
          err = "too many boxes on one level for the tile records (child box << 5 | count)";
          return -1;
        }
        const int64_t F = npp / npts;   // (parent slot, child) pairs
        int64_t* ng = M.alloc<int64_t>(F);
        int64_t* nt = M.alloc<int64_t>(F);
        int64_t* goff = M.alloc<int64_t>(F + 1);
        int64_t* toff = M.alloc<int64_t>(F + 1);
        CKA(ng && nt && goff && toff, "allocation");
        if (F > 0)
          hipLaunchKernelGGL((k_prop_groups<false>), dim3((unsigned)F), dim3(64), 0, 0, pp_off, Q, npts, ppd,
                             Pg.slot_box, Pg.cs, G.slot_cone, ng, nt, nullptr, nullptr, nullptr);
        CK(hipGetLastError(), "propagation groups");
        int64_t ngt = 0, ntt = 0;
        CK(scan_total(M, ng, goff, F, &ngt), "group scan");
        CK(scan_total(M, nt, toff, F, &ntt), "tile scan");
        uint8_t* pts = M.alloc<uint8_t>(npp);
        int32_t* rec = M.alloc<int32_t>(4 * ntt);
        CKA(pts && rec, "allocation");
        if (F > 0)
          hipLaunchKernelGGL((k_prop_groups<true>), dim3((unsigned)F), dim3(64), 0, 0, pp_off, Q, npts, ppd,
                             Pg.slot_box, Pg.cs, G.slot_cone, nullptr, nullptr, toff, pts, rec);
        CK(hipGetLastError(), "propagation tiles");
        std::vector<int64_t> gf, tf;
        CK(down(gf, goff, F + 1), "copy");
        CK(down(tf, toff, F + 1), "copy");
        Pl.pg_off.assign(Q + 1, 0);
        Pl.pt_off.assign(Q + 1, 0);
        for (int64_t q = 0; q <= Q; ++q) {
          const int64_t fq = Pl.pp_off[q] / npts;
          Pl.pg_off[q] = gf[fq];
          Pl.pt_off[q] = tf[fq];
        }
        CK(down(Pl.pg_pts, pts, npp), "copy");
        CK(down(Pl.pt_rec, rec, 4 * ntt), "copy");
        M.release(ng);
        M.release(nt);
        M.release(goff);
        M.release(toff);
        M.release(pts);
        M.release(rec);
        progress("propagation groups into", d - 1, npp);
      }
      M.release(ppd);
      M.release(pp_off);
    }
  }

  // unit counts (the host builder's loops)
  {
    HostLevel& L = P.lev[D];
    int64_t near = 0;
    for (int64_t b = 0; b < L.nb; ++b) {
      int64_t src = 0;
      for (int32_t e2 = L.nbr_off[b]; e2 < L.nbr_off[b + 1]; ++e2) src += L.end[L.nbr[e2]] - L.start[L.nbr[e2]];
      near += (int64_t)(L.end[b] - L.start[b]) * src;
    }
    P.near_pairs = near - n;
    int64_t lp = 0;
    if (D >= 3)
      for (int64_t q = 0; q < L.nslots; ++q) lp += (int64_t)npts * (L.end[L.slot_box[q]] - L.start[L.slot_box[q]]);
    P.leaf_pairs = lp;
  }
#undef CK
#undef CKA
  return 0;
}

}  // namespace ifgf
