// C-ABI of libifgf: plan construction, upload and the IFGF apply driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ifgf.h"
#include "device.hpp"
#include "ifgf_mfma.hpp"
#include "plan.hpp"
#include "util.hpp"

using namespace ifgf;

// Optional per-kernel timing: HIP events recorded around each launch on the
// caller's stream; durations are collected when the statistics are read.
struct PhaseTimer {
  bool on = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
    double units;
  };
  std::vector<Rec> pending;
  struct Acc {
    int64_t launches = 0;
    double ms = 0.0, units = 0.0;
  };
  std::vector<std::pair<std::string, Acc>> acc;
  hipEvent_t begin(hipStream_t st) {
    hipEvent_t e = nullptr;
    if (on && hipEventCreate(&e) == hipSuccess) (void)hipEventRecord(e, st);
    return e;
  }
  void end(const char* name, hipEvent_t a, hipStream_t st, double units) {
    if (!on || !a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, st);
    pending.push_back({name, a, b, units});
  }
  void collect() {
    for (auto& r : pending) {
      float ms = 0.f;
      (void)hipEventSynchronize(r.b);
      (void)hipEventElapsedTime(&ms, r.a, r.b);
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
      Acc* a = nullptr;
      for (auto& kv : acc)
        if (kv.first == r.name) a = &kv.second;
      if (!a) {
        acc.push_back({r.name, Acc()});
        a = &acc.back().second;
      }
      a->launches += 1;
      a->ms += ms;
      a->units += r.units;
    }
    pending.clear();
  }
  void reset() {
    collect();
    acc.clear();
  }
};

struct ifgf_plan_s {
  HostPlan host;
  ifgf_options opt;
  InterpC ic;
  int device = 0;
  // device copies
  DeviceArena arena;
  int64_t* d_perm = nullptr;
  double* d_xs = nullptr;
  double* d_nrm = nullptr;
  double* d_w = nullptr;
  int32_t* d_leaf_of_point = nullptr;
  std::vector<DevLevel> lev;   // lev[d]
  // workspaces
  double2* d_a = nullptr;      // [n][8]
  double2* d_out_s = nullptr;  // [n][28]
  double2* d_vals[2] = {nullptr, nullptr};
  int64_t max_slots = 0;
  // level d uses cone buffer (D - d) & 1: each is sized for its own levels
  int64_t par_slots[2] = {0, 0};
  size_t vals_bytes = 0, res_bytes = 0;
  PhaseTimer timer;
  // matrix-core path (Pa = 5 or 6): K-slot cone layout, FP32 or FP64 cone data
  bool mfma = false;
  bool fp32 = false;
  void* d_af = nullptr;                 // weighted densities of a batch [n][R][16]
  int rcap = 1;                         // right-hand sides per pass the buffers hold
  int rsel = 1;                         // right-hand sides per pass in use (<= rcap)
  std::vector<PropGroups> groups;       // groups[d]: propagation into level d
  std::vector<TargetTiles> ttiles;      // ttiles[d]: target pairs by cone (matrix-core interpolation)
  // chunks of ttiles[d]: tiles [tc_tile[c], tc_tile[c+1]) hold targets [tc_i0[c], tc_i0[c+1])
  std::vector<std::vector<int64_t>> tc_tile, tc_i0;
  void* d_res = nullptr;                // per-pair target contributions [pairs][R][28] complex
  unsigned* d_err = nullptr;            // device error word (bit 0: a propagation lock wait gave up)
  int elem = 8;                         // bytes per real of the cone buffers and density copy
  int spin_limit = 1 << 22;             // attempts of the bounded lock wait
  int nk = 2;                           // kernels per pass: 2 (both), or 1 (one at a time, Remark 3)
};

namespace ifgf {
hipEvent_t timer_begin(ifgf_plan_s* p, hipStream_t st) { return p ? p->timer.begin(st) : nullptr; }
void timer_end(ifgf_plan_s* p, const char* name, hipEvent_t ev, hipStream_t st, double units) {
  if (p) p->timer.end(name, ev, st, units);
}
bool timing_on(ifgf_plan_s* p) { return p && p->timer.on; }
bool plan_verbose(ifgf_plan_s* p) { return p && p->opt.verbose; }
}  // namespace ifgf

namespace {

// Which kernel interpolates onto the cousin targets of level d: the
// matrix-core tiles (one right-hand side per pass; levels whose pair count
// fits the tile tables) or one thread per target otherwise.
// reals per cone row of the matrix-core buffers
size_t row_width(const ifgf_plan_s* p) { return p->nk == 2 ? (size_t)32 * p->rcap : 16; }

const char* target_path(const ifgf_plan_s* p, int d) {
  if (!p->mfma) return "generic";
  if (p->d_res && d < (int)p->ttiles.size() && p->ttiles[d].ntiles > 0) return "mfma_tiles";
  return "per_target";
}

// Bytes of the two cone buffers (level d uses buffer (D - d) & 1, each sized
// for the largest of its levels) with nk kernels per pass and R right-hand
// sides per pass: what Remark 3 computes from the relevant cone counts.
size_t cone_buffer_bytes(const HostPlan& H, bool mfma, int elem, int R, int nk, int npts) {
  int64_t slots[2] = {0, 0};
  for (int d = 3; d <= H.D; ++d) slots[(H.D - d) & 1] = std::max(slots[(H.D - d) & 1], H.lev[d].nslots);
  if (slots[0] == 0 && slots[1] == 0) return 0;
  size_t total = 0;
  for (int b = 0; b < 2; ++b) {
    const size_t sl = (size_t)std::max<int64_t>(slots[b], 1);
    total += mfma ? (size_t)elem * sl * kslot_rows(H.Ps, H.Pa, nk) * (nk == 2 ? 32 * R : 16)
                  : sizeof(double2) * sl * npts * kCols;
  }
  return total;
}

int tol_to_orders(double tol, int* Ps, int* Pa) {
  // With the cone rule of Remark 2 (radial and angular counts doubled per
  // level), the smallest orders whose interpolation error stays below tol in
  // every output block: the single-layer sums and, larger, their normal
  // derivatives, whose angular part needs Pa = 6 below 1.5e-4.  Measured
  // against direct sums on spheres of radius 1 to 5 wavelengths and an
  // ellipsoid.  tol >= 1e-3 gives the paper's (3, 5).
  if (tol >= 1e-3) { *Ps = 3; *Pa = 5; }
  else if (tol >= 1e-4) { *Ps = 4; *Pa = 6; }
  else if (tol >= 1e-5) { *Ps = 7; *Pa = 8; }
  else { *Ps = 8; *Pa = 8; }
  return 0;
}

void make_interp(InterpC& ic, int Ps, int Pa) {
  ic.Ps = Ps;
  ic.Pa = Pa;
  ic.npts = Ps * Pa * Pa;
  auto fill = [](int P, double* x, double* w) {
    for (int k = 0; k < P; ++k) x[k] = std::cos((k + 0.5) * 3.141592653589793 / P);
    for (int j = 0; j < P; ++j) {
      double p = 1.0;
      for (int m = 0; m < P; ++m)
        if (m != j) p *= (x[j] - x[m]);
      w[j] = 1.0 / p;
    }
  };
  std::memset(ic.xs, 0, sizeof(ic.xs));
  std::memset(ic.xa, 0, sizeof(ic.xa));
  std::memset(ic.ws, 0, sizeof(ic.ws));
  std::memset(ic.wa, 0, sizeof(ic.wa));
  fill(Ps, ic.xs, ic.ws);
  fill(Pa, ic.xa, ic.wa);
  for (int k = 0; k < 8; ++k) {
    ic.xsf[k] = (float)ic.xs[k];
    ic.xaf[k] = (float)ic.xa[k];
    ic.wsf[k] = (float)ic.ws[k];
    ic.waf[k] = (float)ic.wa[k];
  }
}

template <class T>
int upload(DeviceArena& ar, const std::vector<T>& v, T** dst) {
  *dst = nullptr;
  if (v.empty()) return 0;
  *dst = static_cast<T*>(ar.alloc(v.size() * sizeof(T)));
  if (!*dst) return IFGF_ENOMEM;
  hipError_t e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return set_hip_error(e, "hipMemcpy");
  return 0;
}

int validate(int64_t n, const double* x, const double* nrm, const double* w, double k0, double k1,
             double tol) {
  if (n < 1) return set_error(IFGF_EINVAL, "n must be >= 1");
  if (!x || !nrm || !w) return set_error(IFGF_EINVAL, "points, normals and weights are required");
  if (!(k0 > 0.0) || !(k1 > 0.0) || !std::isfinite(k0) || !std::isfinite(k1))
    return set_error(IFGF_EINVAL, "wavenumbers must be finite and > 0");
  if (!(tol >= 1e-10 && tol <= 1e-1)) return set_error(IFGF_EINVAL, "tol must lie in [1e-10, 1e-1]");
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(x[3 * i + c]) || !std::isfinite(nrm[3 * i + c]))
        return set_error(IFGF_EINVAL, "non-finite point or normal at index " + std::to_string(i));
    double nn = std::sqrt(nrm[3 * i] * nrm[3 * i] + nrm[3 * i + 1] * nrm[3 * i + 1] +
                          nrm[3 * i + 2] * nrm[3 * i + 2]);
    if (std::fabs(nn - 1.0) > 1e-6)
      return set_error(IFGF_EINVAL, "normal is not unit length at index " + std::to_string(i));
    if (!(w[i] > 0.0) || !std::isfinite(w[i]))
      return set_error(IFGF_EINVAL, "weight must be finite and > 0 at index " + std::to_string(i));
  }
  return 0;
}

}  // namespace

extern "C" {

void ifgf_default_options(ifgf_options* opt) {
  if (!opt) return;
  opt->Ps = 0;
  opt->Pa = 0;
  opt->ns_init = 1;
  opt->na_init = 2;
  opt->refine_radial = 1;
  opt->leaf_wavelengths = 0.25;
  opt->precision = IFGF_FP64;
  opt->max_nrhs = 1;
  opt->host_only = 0;
  opt->batch_columns = 1;
  opt->fp32_workspaces = 0;
  opt->verbose = 0;
  opt->deriv_mode = IFGF_DERIV_ANALYTIC;
  opt->target_chunk_pairs = 0;
  opt->plan_on_device = 1;
  opt->keep_pair_tables = 0;
  opt->kernel_at_a_time = 0;
  opt->cone_memory_budget = 0;
  opt->target_tiles = 1;
}

int ifgf_plan(ifgf_plan_t* out, int64_t n, const double* points, const double* normals,
              const double* weights, double k_int, double k_ext, double tol,
              const ifgf_options* optin) {
  clear_error();
  if (!out) return set_error(IFGF_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(n, points, normals, weights, k_int, k_ext, tol);
  if (rc) return rc;
  ifgf_options opt;
  ifgf_default_options(&opt);
  if (optin) opt = *optin;
  if (opt.ns_init <= 0) opt.ns_init = 1;
  if (opt.na_init <= 0) opt.na_init = 2;
  if (opt.leaf_wavelengths <= 0.0) opt.leaf_wavelengths = 0.25;
  if (opt.max_nrhs <= 0) opt.max_nrhs = 1;
  if (opt.batch_columns <= 0) opt.batch_columns = 1;
  if (opt.batch_columns != 1 && opt.batch_columns != 2 && opt.batch_columns != 4)
    return set_error(IFGF_EINVAL, "batch_columns must be 1, 2 or 4");
  if (opt.Ps <= 0 || opt.Pa <= 0) tol_to_orders(tol, &opt.Ps, &opt.Pa);
  if (opt.Ps > kMaxP || opt.Pa > kMaxP || opt.Ps < 1 || opt.Pa < 1)
    return set_error(IFGF_EINVAL, "Ps and Pa must lie in [1, 8]");
  if (opt.precision != IFGF_FP64 && opt.precision != IFGF_FP32)
    return set_error(IFGF_EINVAL, "precision must be IFGF_FP64 or IFGF_FP32");
  if (opt.deriv_mode != IFGF_DERIV_ANALYTIC && opt.deriv_mode != IFGF_DERIV_FD)
    return set_error(IFGF_EINVAL, "deriv_mode must be IFGF_DERIV_ANALYTIC or IFGF_DERIV_FD");
  if (opt.deriv_mode == IFGF_DERIV_FD && (opt.precision != IFGF_FP64 || opt.max_nrhs > 1 || opt.batch_columns > 1))
    return set_error(IFGF_EINVAL, "IFGF_DERIV_FD needs IFGF_FP64 and one right-hand side per apply");
  if (opt.kernel_at_a_time < -1 || opt.kernel_at_a_time > 1)
    return set_error(IFGF_EINVAL, "kernel_at_a_time must be -1, 0 or 1");
  if (opt.cone_memory_budget < 0) return set_error(IFGF_EINVAL, "cone_memory_budget must be >= 0");

  ifgf_plan_s* p = new (std::nothrow) ifgf_plan_s();
  if (!p) return set_error(IFGF_ENOMEM, "host allocation failed");
  p->opt = opt;
  PlanParams pp;
  pp.Ps = opt.Ps;
  pp.Pa = opt.Pa;
  pp.ns_init = opt.ns_init;
  pp.na_init = opt.na_init;
  pp.refine_radial = opt.refine_radial;
  pp.leaf_wavelengths = opt.leaf_wavelengths;
  pp.verbose = opt.verbose;
  if (opt.target_chunk_pairs < 0) return set_error(IFGF_EINVAL, "target_chunk_pairs must be >= 0");
  pp.target_chunk_pairs = opt.target_chunk_pairs > 0 ? opt.target_chunk_pairs : kTargetChunkPairs;
  std::string err;
  try {
    if (opt.plan_on_device && !opt.host_only) {
      const int prc = build_device_plan(p->host, n, points, normals, weights, k_int, k_ext, pp, err);
      if (prc) {
        delete p;
        return set_error(prc == -2 ? IFGF_EHIP : IFGF_EINVAL, err);
      }
    } else if (build_host_plan(p->host, n, points, normals, weights, k_int, k_ext, pp, err)) {
      delete p;
      return set_error(IFGF_EINVAL, err);
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return set_error(IFGF_ENOMEM, "host allocation failed while planning");
  }
  HostPlan& H = p->host;
  // duplicate points (excluded by the method: Sec. III-E) share a leaf
  {
    HostLevel& L = H.lev[H.D];
    for (int64_t b = 0; b < L.nb; ++b)
      for (int32_t i = L.start[b]; i < L.end[b]; ++i)
        for (int32_t j = i + 1; j < L.end[b]; ++j)
          if (H.xs[3 * i] == H.xs[3 * j] && H.xs[3 * i + 1] == H.xs[3 * j + 1] &&
              H.xs[3 * i + 2] == H.xs[3 * j + 2]) {
            delete p;
            return set_error(IFGF_EINVAL, "duplicate points (input indices " +
                                              std::to_string(H.perm[i]) + ", " +
                                              std::to_string(H.perm[j]) + ")");
          }
  }
  make_interp(p->ic, opt.Ps, opt.Pa);
  if (opt.host_only) {
    *out = p;
    return IFGF_OK;
  }
  (void)hipGetDevice(&p->device);

  DeviceArena& ar = p->arena;
  if ((rc = upload(ar, H.perm, &p->d_perm)) || (rc = upload(ar, H.xs, &p->d_xs)) ||
      (rc = upload(ar, H.nrm, &p->d_nrm)) || (rc = upload(ar, H.w, &p->d_w)) ||
      (rc = upload(ar, H.leaf_of_point, &p->d_leaf_of_point))) {
    delete p;
    return rc;
  }
  p->mfma = mfma_path_supported(opt.Ps, opt.Pa);
  p->fp32 = opt.precision == IFGF_FP32;
  if (p->fp32 && !p->mfma) {
    delete p;
    return set_error(IFGF_EINVAL, "IFGF_FP32 needs Pa = 5 or 6 and 3 <= Ps <= 6");
  }
  if (opt.deriv_mode == IFGF_DERIV_FD && !p->mfma) {
    delete p;
    return set_error(IFGF_EINVAL, "IFGF_DERIV_FD needs the matrix-core orders (Pa = 5 or 6, 3 <= Ps <= 6)");
  }
  if (p->mfma && !opt.keep_pair_tables)
    for (int d = 1; d <= H.D; ++d) std::vector<int32_t>().swap(H.lev[d].pp_slot);
  p->groups.assign(H.D + 1, PropGroups());
  p->ttiles.assign(H.D + 1, TargetTiles());
  p->tc_tile.assign(H.D + 1, std::vector<int64_t>());
  p->tc_i0.assign(H.D + 1, std::vector<int64_t>());
  int64_t max_pairs = 0;
  p->lev.assign(H.D + 1, DevLevel());
  for (int d = 1; d <= H.D; ++d) {
    HostLevel& L = H.lev[d];
    DevLevel& G = p->lev[d];
    G.d = d;
    G.h = L.h;
    G.ns = L.ns;
    G.na = L.na;
    G.nb = L.nb;
    G.nslots = L.nslots;
    if ((rc = upload(ar, L.centers, &G.centers)) || (rc = upload(ar, L.start, &G.start)) ||
        (rc = upload(ar, L.end, &G.end)) || (rc = upload(ar, L.child_start, &G.child_start)) ||
        (rc = upload(ar, L.child_end, &G.child_end)) || (rc = upload(ar, L.slot_box, &G.slot_box)) ||
        (rc = upload(ar, L.slot_cone, &G.slot_cone)) || (rc = upload(ar, L.tp_off, &G.tp_off)) ||
        (rc = upload(ar, L.tp_slot, &G.tp_slot)) || (rc = upload(ar, L.pp_off, &G.pp_off)) ||
        (rc = upload(ar, L.pp_slot, &G.pp_slot))) {
      delete p;
      return rc;
    }
    if (d == H.D) {
      if ((rc = upload(ar, L.nbr_off, &G.nbr_off)) || (rc = upload(ar, L.nbr, &G.nbr))) {
        delete p;
        return rc;
      }
    }
    if (p->mfma && !L.pg_off.empty()) {
      PropGroups& PG = p->groups[d];
      int64_t* to = nullptr;
      int32_t* rec = nullptr;
      uint8_t* pt = nullptr;
      if ((rc = upload(ar, L.pt_off, &to)) || (rc = upload(ar, L.pt_rec, &rec)) || (rc = upload(ar, L.pg_pts, &pt))) {
        delete p;
        return rc;
      }
      PG.toff = to;
      PG.rec = reinterpret_cast<const int4*>(rec);
      PG.pts = pt;
    }
    // only the offsets stay on the host (statistics)
    std::vector<int32_t>().swap(L.pt_rec);
    std::vector<int32_t>().swap(L.pt_g);
    std::vector<uint8_t>().swap(L.pt_t0);
    std::vector<int64_t>().swap(L.pg_start);
    std::vector<int32_t>().swap(L.pg_slot);
    std::vector<int32_t>().swap(L.pg_cbox);
    std::vector<int32_t>().swap(L.pg_count);
    std::vector<uint8_t>().swap(L.pg_pts);
    if (p->mfma && d >= 3 && !L.tt_slot.empty() && opt.target_tiles) {
      TargetTiles& TT = p->ttiles[d];
      int32_t *sl = nullptr, *tg = nullptr, *ee = nullptr;
      int64_t* stt = nullptr;
      uint8_t* cn = nullptr;
      if ((rc = upload(ar, L.tt_slot, &sl)) || (rc = upload(ar, L.tt_start, &stt)) ||
          (rc = upload(ar, L.tt_cnt, &cn)) || (rc = upload(ar, L.ts_tgt, &tg)) || (rc = upload(ar, L.ts_e, &ee))) {
        delete p;
        return rc;
      }
      TT.ntiles = (int64_t)L.tt_slot.size();
      TT.slot = sl;
      TT.start = stt;
      TT.cnt = cn;
      TT.tgt = tg;
      TT.e = ee;
      p->tc_tile[d] = L.tc_tile;
      p->tc_i0[d] = L.tc_i0;
      max_pairs = std::max(max_pairs, L.tc_max_pairs);
    }
    std::vector<int32_t>().swap(L.tt_slot);
    std::vector<int64_t>().swap(L.tt_start);
    std::vector<uint8_t>().swap(L.tt_cnt);
    std::vector<int32_t>().swap(L.ts_tgt);
    std::vector<int32_t>().swap(L.ts_e);
    if (d >= 3) {
      p->max_slots = std::max(p->max_slots, L.nslots);
      p->par_slots[(H.D - d) & 1] = std::max(p->par_slots[(H.D - d) & 1], L.nslots);
    }
    // the host copies of the large pair tables are no longer needed
    if (!opt.keep_pair_tables) {
      std::vector<int32_t>().swap(L.tp_slot);
      std::vector<int32_t>().swap(L.pp_slot);
    }
  }
  if (opt.deriv_mode == IFGF_DERIV_FD)
    for (int d = 3; d <= H.D; ++d)
      if (H.lev[d].tp_off.back() > 0 && p->ttiles[d].ntiles == 0) {
        delete p;
        return set_error(IFGF_EINVAL, "IFGF_DERIV_FD needs the target tiles of every level");
      }
  // right-hand sides stacked into the cone-data columns (matrix-core path)
  p->rcap = p->mfma ? std::min(std::min(opt.max_nrhs, opt.batch_columns), max_batch_columns(p->fp32, opt.Ps, opt.Pa))
                    : 1;
  if (p->rcap == 3) p->rcap = 2;
  p->elem = (p->fp32 && opt.fp32_workspaces) ? 4 : 8;
  // Kernels per pass (Remark 3): both, or one at a time with half the cone
  // memory.  -1 picks one at a time when the cone buffers of both kernels
  // exceed the budget: cone_memory_budget, else the free device memory less
  // the workspaces still to be allocated.
  if (opt.kernel_at_a_time != 0) {
    if (!p->mfma) {
      delete p;
      return set_error(IFGF_EINVAL, "kernel_at_a_time needs the matrix-core orders (Pa = 5 or 6, 3 <= Ps <= 6)");
    }
    p->nk = 1;
    if (opt.kernel_at_a_time == -1) {
      size_t budget = (size_t)opt.cone_memory_budget;
      if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipError_t e = hipMemGetInfo(&fr, &tot); e != hipSuccess) {
          delete p;
          return set_hip_error(e, "hipMemGetInfo");
        }
        const size_t rest = sizeof(double2) * n * (kNS + (size_t)kOut * p->rcap) + (size_t)p->elem * 16 * n * p->rcap +
                            (size_t)p->elem * 56 * (size_t)max_pairs * p->rcap;
        budget = fr > rest ? fr - rest : 0;
      }
      p->nk = cone_buffer_bytes(H, true, p->elem, p->rcap, 2, p->ic.npts) > budget ? 1 : 2;
    }
    if (p->nk == 1) p->rcap = 1;
  }
  p->rsel = p->rcap;
  p->d_a = static_cast<double2*>(ar.alloc(sizeof(double2) * n * kNS));
  p->d_out_s = static_cast<double2*>(ar.alloc(sizeof(double2) * n * kOut * p->rcap));
  p->d_err = static_cast<unsigned*>(ar.alloc(sizeof(unsigned)));
  if (!p->d_a || !p->d_out_s || !p->d_err) {
    delete p;
    return set_error(IFGF_ENOMEM, "device workspace allocation failed");
  }
  if (hipError_t e = hipMemset(p->d_err, 0, sizeof(unsigned)); e != hipSuccess) {
    delete p;
    return set_hip_error(e, "hipMemset");
  }
  // A matrix-core plan can run in either precision (ifgf_set_precision), so
  // its density copy and cone buffers are sized for FP64 -- unless it was
  // built FP32-only (fp32_workspaces), which halves them.
  if (p->mfma) {
    p->d_af = ar.alloc((size_t)p->elem * 16 * (size_t)n * p->rcap);
    if (!p->d_af) {
      delete p;
      return set_error(IFGF_ENOMEM, "device workspace allocation failed");
    }
  }
  if (max_pairs > 0) {
    p->res_bytes = (size_t)p->elem * 28 * p->nk * (size_t)max_pairs * p->rcap;
    p->d_res = ar.alloc(p->res_bytes);
    if (!p->d_res) {
      delete p;
      return set_error(IFGF_ENOMEM, "device workspace allocation failed");
    }
  }
  if (p->max_slots > 0) {
    for (int b = 0; b < 2; ++b) {
      const size_t slots = (size_t)std::max<int64_t>(p->par_slots[b], 1);
      const size_t vb = p->mfma ? (size_t)p->elem * slots * kslot_rows(opt.Ps, opt.Pa, p->nk) * row_width(p)
                                : sizeof(double2) * slots * p->ic.npts * kCols;
      p->d_vals[b] = static_cast<double2*>(ar.alloc(vb));
      p->vals_bytes += vb;
    }
    if (!p->d_vals[0] || !p->d_vals[1]) {
      delete p;
      return set_error(IFGF_ENOMEM, "device cone-grid allocation failed");
    }
  }
  *out = p;
  return IFGF_OK;
}

int ifgf_apply(ifgf_plan_t p, const void* densities, int nrhs, void* out, void* stream) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  if (!densities || !out) return set_error(IFGF_EINVAL, "densities and out are required");
  if (nrhs < 1 || nrhs > p->opt.max_nrhs)
    return set_error(IFGF_EINVAL, "nrhs must lie in [1, max_nrhs]");
  if (p->opt.host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const HostPlan& H = p->host;
  const int64_t n = H.n;
  const double k0 = H.k[0], k1 = H.k[1];
  PhaseTimer& T = p->timer;
  if (p->mfma && H.D >= 3) {
    // matrix-core path: R right-hand sides per pass share the geometry
    const int rmax = std::min(p->rsel, max_batch_columns(p->fp32, H.Ps, H.Pa));
    for (int r0 = 0; r0 < nrhs;) {
      const int rem = nrhs - r0;
      const int R = (rem >= 4 && rmax >= 4) ? 4 : ((rem >= 2 && rmax >= 2) ? 2 : 1);
      const double2* dens = static_cast<const double2*>(densities) + (int64_t)r0 * kNS * n;
      hipError_t e;
      for (int r = 0; r < R; ++r) {
        hipEvent_t ev = T.begin(st);
        if ((e = launch_gather_weighted(dens + (int64_t)r * kNS * n, p->d_perm, p->d_w, n, p->d_a, st)) !=
            hipSuccess)
          return set_hip_error(e, "gather");
        T.end("gather", ev, st, (double)n);
        ev = T.begin(st);
        if ((e = launch_near(p->lev[H.D], p->d_leaf_of_point, p->d_xs, p->d_nrm, p->d_a, n, k0, k1,
                             p->d_out_s + (int64_t)r * kOut * n, st)) != hipSuccess)
          return set_hip_error(e, "near");
        T.end("near", ev, st, (double)H.near_pairs);
      }
      if ((e = mf_gather(p->fp32, R, dens, p->d_perm, p->d_w, n, p->d_af, st)) != hipSuccess)
        return set_hip_error(e, "gather batch");
      // both kernels in one pass (nk = 2), or one pass per kernel (nk = 1,
      // Remark 3): pass kq runs the kernel of wavenumber k_kq alone
      const int nk = p->nk;
      for (int kq = 0; kq < 3 - nk; ++kq) {
      const double ka = nk == 2 ? k0 : H.k[kq], kb = nk == 2 ? k1 : H.k[kq];
      int cur = 0;
      hipEvent_t ev = T.begin(st);
      if ((e = mf_leaf(p->fp32, H.Ps, H.Pa, R, nk, p->lev[H.D], p->ic, p->d_xs, p->d_af, ka, kb, p->d_vals[cur],
                       st)) != hipSuccess)
        return set_hip_error(e, "leaf");
      T.end("leaf", ev, st, (double)H.leaf_pairs * R);
      for (int d = H.D; d >= 3; --d) {
        ev = T.begin(st);
        if (p->d_res && p->ttiles[d].ntiles > 0) {
          // cone-major tiles on the matrix cores, then the per-target sums,
          // one chunk of consecutive targets at a time (bounded result buffer)
          const std::vector<int64_t>& ct = p->tc_tile[d];
          const std::vector<int64_t>& ci = p->tc_i0[d];
          for (size_t c = 0; c + 1 < ct.size(); ++c) {
            TargetTiles sub = p->ttiles[d];
            sub.slot += ct[c];
            sub.start += ct[c];
            sub.cnt += ct[c];
            sub.ntiles = ct[c + 1] - ct[c];
            if ((e = mf_targets_tiles(p->fp32, H.Ps, H.Pa, R, nk, p->lev[d], p->ic, sub, p->d_xs, p->d_nrm, ka, kb,
                                      p->d_vals[cur], p->d_res, p->opt.deriv_mode == IFGF_DERIV_FD, st)) !=
                    hipSuccess ||
                (e = mf_targets_reduce(p->fp32, p->lev[d], R, nk, kq, n, ci[c], ci[c + 1], p->d_res, p->d_out_s,
                                       st)) != hipSuccess)
              return set_hip_error(e, "targets");
          }
        } else if ((e = mf_targets(p->fp32, H.Ps, H.Pa, R, nk, p->lev[d], p->ic, p->d_xs, p->d_nrm, n, ka, kb,
                                   p->d_vals[cur], p->d_out_s, kq, st)) != hipSuccess) {
          return set_hip_error(e, "targets");
        }
        T.end("targets", ev, st, (double)H.lev[d].tp_off.back() * R);
        if (d > 3) {
          ev = T.begin(st);
          if ((e = mf_propagate(p->fp32, H.Ps, H.Pa, R, nk, p->lev[d], p->lev[d - 1], p->ic, p->groups[d - 1], ka,
                                kb, p->d_vals[cur], p->d_vals[cur ^ 1], p->spin_limit, p->d_err, st)) !=
              hipSuccess)
            return set_hip_error(e, "propagate");
          T.end("propagate", ev, st, (double)H.lev[d - 1].pp_off.back() * R);
          cur ^= 1;
        }
      }
      }
      for (int r = 0; r < R; ++r) {
        hipEvent_t ev = T.begin(st);
        double2* o = static_cast<double2*>(out) + (int64_t)(r0 + r) * kOut * n;
        if ((e = launch_scatter_out(p->d_out_s + (int64_t)r * kOut * n, p->d_perm, n, o, st)) != hipSuccess)
          return set_hip_error(e, "scatter");
        T.end("scatter", ev, st, (double)n);
      }
      r0 += R;
    }
    return IFGF_OK;
  }
  for (int r = 0; r < nrhs; ++r) {
    const double2* dens = static_cast<const double2*>(densities) + (int64_t)r * kNS * n;
    double2* o = static_cast<double2*>(out) + (int64_t)r * kOut * n;
    hipError_t e;
    hipEvent_t ev = T.begin(st);
    if ((e = launch_gather_weighted(dens, p->d_perm, p->d_w, n, p->d_a, st)) != hipSuccess)
      return set_hip_error(e, "gather");
    T.end("gather", ev, st, (double)n);
    ev = T.begin(st);
    if ((e = launch_near(p->lev[H.D], p->d_leaf_of_point, p->d_xs, p->d_nrm, p->d_a, n, k0, k1,
                         p->d_out_s, st)) != hipSuccess)
      return set_hip_error(e, "near");
    T.end("near", ev, st, (double)H.near_pairs);
    if (H.D >= 3) {
      int cur = 0;
      ev = T.begin(st);
      if ((e = launch_leaf(p->lev[H.D], p->ic, p->d_xs, p->d_a, k0, k1, p->d_vals[cur], st)) !=
          hipSuccess)
        return set_hip_error(e, "leaf");
      T.end("leaf", ev, st, (double)H.leaf_pairs);
      for (int d = H.D; d >= 3; --d) {
        ev = T.begin(st);
        if ((e = launch_targets(p->lev[d], p->ic, p->d_xs, p->d_nrm, n, k0, k1, p->d_vals[cur],
                                p->d_out_s, st)) != hipSuccess)
          return set_hip_error(e, "targets");
        T.end("targets", ev, st, (double)H.lev[d].tp_off.back());
        if (d > 3) {
          ev = T.begin(st);
          if ((e = launch_propagate(p->lev[d], p->lev[d - 1], p->ic, k0, k1, p->d_vals[cur],
                                    p->d_vals[cur ^ 1], st)) != hipSuccess)
            return set_hip_error(e, "propagate");
          T.end("propagate", ev, st, (double)H.lev[d - 1].pp_off.back());
          cur ^= 1;
        }
      }
    }
    ev = T.begin(st);
    if ((e = launch_scatter_out(p->d_out_s, p->d_perm, n, o, st)) != hipSuccess)
      return set_hip_error(e, "scatter");
    T.end("scatter", ev, st, (double)n);
  }
  return IFGF_OK;
}

int ifgf_plan_counts(ifgf_plan_t p, int64_t* counts, int ncount) {
  clear_error();
  if (!p || !counts) return set_error(IFGF_EINVAL, "plan and counts are required");
  const HostPlan& H = p->host;
  std::vector<int64_t> v = {H.n, H.D, H.Ps, H.Pa, H.near_pairs,
                            H.D >= 3 ? H.lev[H.D].nslots : 0, H.leaf_pairs};
  for (int d = 3; d <= H.D; ++d) {
    const HostLevel& L = H.lev[d];
    int64_t tp = L.tp_off.empty() ? 0 : L.tp_off.back();
    int64_t pp = (d >= 4 && !H.lev[d - 1].pp_off.empty()) ? H.lev[d - 1].pp_off.back() : 0;
    v.push_back(L.nslots);
    v.push_back(tp);
    v.push_back(pp);
    v.push_back((int64_t)L.ns * 65536 + L.na);
  }
  for (int i = 0; i < ncount; ++i) counts[i] = i < (int)v.size() ? v[i] : 0;
  return IFGF_OK;
}

int ifgf_plan_table(ifgf_plan_t p, int which, int64_t* buf, int64_t cap, int64_t* count) {
  clear_error();
  if (!p || !count) return set_error(IFGF_EINVAL, "plan and count are required");
  const HostPlan& H = p->host;
  std::vector<int64_t> v;
  if (which == 0) {
    v = H.perm;
  } else if (which > 1000 && which - 1000 <= H.D && which - 1000 >= 3) {
    const HostLevel& L = H.lev[which - 1000];
    v.resize(L.nslots);
    for (int64_t s = 0; s < L.nslots; ++s) v[s] = (int64_t)L.slot_box[s] * L.ncones + L.slot_cone[s];
  } else if (which > 2000 && which - 2000 <= H.D && which - 2000 >= 3) {
    const HostLevel& L = H.lev[which - 2000];
    if (L.tp_slot.size() != (size_t)(L.tp_off.empty() ? 0 : L.tp_off.back()))
      return set_error(IFGF_ENOTPLANNED, "pair tables are kept only by host_only plans");
    v.assign(L.tp_slot.begin(), L.tp_slot.end());
  } else if (which > 3000 && which - 3000 < H.D && which - 3000 >= 3) {
    const HostLevel& L = H.lev[which - 3000];
    if (L.pp_slot.size() != (size_t)(L.pp_off.empty() ? 0 : L.pp_off.back()))
      return set_error(IFGF_ENOTPLANNED, "pair tables are kept only by host_only plans");
    v.assign(L.pp_slot.begin(), L.pp_slot.end());
  } else {
    return set_error(IFGF_EINVAL, "unknown table id");
  }
  *count = (int64_t)v.size();
  if (buf) {
    if (cap < (int64_t)v.size()) return set_error(IFGF_EINVAL, "buffer too small");
    std::memcpy(buf, v.data(), v.size() * sizeof(int64_t));
  }
  return IFGF_OK;
}

int ifgf_stats(ifgf_plan_t p, char* json, size_t cap) {
  clear_error();
  if (!p || !json) return set_error(IFGF_EINVAL, "plan and json are required");
  const HostPlan& H = p->host;
  std::string s = "{\"n\":" + std::to_string(H.n) + ",\"D\":" + std::to_string(H.D) +
                  ",\"Ps\":" + std::to_string(H.Ps) + ",\"Pa\":" + std::to_string(H.Pa) +
                  ",\"near_pairs\":" + std::to_string(H.near_pairs) +
                  ",\"leaf_pairs\":" + std::to_string(H.leaf_pairs) +
                  ",\"device_bytes\":" + std::to_string(p->arena.bytes()) +
                  ",\"workspace_elem_bytes\":" + std::to_string(p->elem) +
                  ",\"cone_buffer_bytes\":" + std::to_string(p->vals_bytes) +
                  ",\"kernels_per_pass\":" + std::to_string(p->opt.host_only ? 0 : p->nk) +
                  ",\"cone_buffer_bytes_by_mode\":[" +
                  std::to_string(cone_buffer_bytes(H, mfma_path_supported(H.Ps, H.Pa), 8, 1, 2, p->ic.npts)) + "," +
                  std::to_string(mfma_path_supported(H.Ps, H.Pa)
                                     ? cone_buffer_bytes(H, true, 8, 1, 1, p->ic.npts) : (size_t)0) + "]" +
                  ",\"target_result_bytes\":" + std::to_string(p->res_bytes) + ",\"levels\":[";
  for (int d = 3; d <= H.D; ++d) {
    const HostLevel& L = H.lev[d];
    s += std::string(d > 3 ? "," : "") + "{\"d\":" + std::to_string(d) + ",\"boxes\":" +
         std::to_string(L.nb) + ",\"ns\":" + std::to_string(L.ns) + ",\"na\":" +
         std::to_string(L.na) + ",\"slots\":" + std::to_string(L.nslots) +
         ",\"prop_groups\":" + std::to_string(L.pg_off.empty() ? 0 : L.pg_off.back()) +
         ",\"prop_tiles\":" + std::to_string(L.pt_off.empty() ? 0 : L.pt_off.back()) +
         ",\"target_path\":\"" + target_path(p, d) + "\"}";
  }
  unsigned derr = 0;
  if (p->d_err && hipMemcpy(&derr, p->d_err, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(IFGF_EHIP, "reading the device error word");
  s += "],\"device_error\":" + std::to_string(derr) + ",\"timing\":{";
  p->timer.collect();
  bool first = true;
  for (auto& kv : p->timer.acc) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s\"%s\":{\"launches\":%lld,\"ms\":%.6f,\"units\":%.1f}",
                  first ? "" : ",", kv.first.c_str(), (long long)kv.second.launches, kv.second.ms,
                  kv.second.units);
    s += buf;
    first = false;
  }
  s += "}}";
  if (s.size() + 1 > cap) return set_error(IFGF_EINVAL, "json buffer too small");
  std::memcpy(json, s.c_str(), s.size() + 1);
  return IFGF_OK;
}

int ifgf_autotune(ifgf_plan_t p, void* stream, int* chosen) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  if (p->opt.host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  if (p->timer.on) return set_error(IFGF_EINVAL, "switch per-kernel timing off before tuning");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = p->host.n;
  const int top = p->nk == 1 ? 1 : std::min(p->rcap, max_batch_columns(p->fp32, p->host.Ps, p->host.Pa));
  int best = 1;
  if (p->mfma && top > 1) {
    DeviceArena tmp;
    void* dens = tmp.alloc(sizeof(double2) * kNS * (size_t)n * top);
    void* out = tmp.alloc(sizeof(double2) * kOut * (size_t)n * top);
    hipEvent_t a = nullptr, b = nullptr;
    if (!dens || !out) return set_error(IFGF_ENOMEM, "autotune buffers");
    hipError_t e;
    if ((e = hipMemsetAsync(dens, 0, sizeof(double2) * kNS * (size_t)n * top, st)) != hipSuccess ||
        (e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess)
      return set_hip_error(e, "autotune setup");
    double best_ms = 1e300;
    const int saved = p->rsel;
    for (int R = 1; R <= top; R *= 2) {
      p->rsel = R;
      int rc = ifgf_apply(p, dens, R, out, stream);   // warm-up
      if (!rc) {
        (void)hipEventRecord(a, st);
        rc = ifgf_apply(p, dens, R, out, stream);
        (void)hipEventRecord(b, st);
      }
      float ms = 0.f;
      if (rc || (e = hipEventSynchronize(b)) != hipSuccess || (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) {
        p->rsel = saved;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return rc ? rc : set_hip_error(e, "autotune timing");
      }
      const double per = ms / R;
      if (per < best_ms) {
        best_ms = per;
        best = R;
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  p->rsel = best;
  if (chosen) *chosen = best;
  return IFGF_OK;
}

int ifgf_set_precision(ifgf_plan_t p, int precision, int* previous) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  if (precision != IFGF_FP64 && precision != IFGF_FP32)
    return set_error(IFGF_EINVAL, "precision must be IFGF_FP64 or IFGF_FP32");
  if (p->opt.host_only) return set_error(IFGF_ENOTPLANNED, "plan was built with host_only");
  if (precision == IFGF_FP32 && !p->mfma)
    return set_error(IFGF_EINVAL, "IFGF_FP32 needs Pa = 5 or 6 and 3 <= Ps <= 6");
  if (precision == IFGF_FP32 && p->opt.deriv_mode == IFGF_DERIV_FD)
    return set_error(IFGF_EINVAL, "the forward-difference derivative is FP64 only");
  if (precision == IFGF_FP64 && p->elem < 8)
    return set_error(IFGF_EINVAL, "the plan was built with fp32_workspaces: its buffers hold FP32 cone data only");
  if (previous) *previous = p->fp32 ? IFGF_FP32 : IFGF_FP64;
  p->fp32 = precision == IFGF_FP32;
  p->opt.precision = precision;
  return IFGF_OK;
}

int ifgf_precisions(ifgf_plan_t p) {
  if (!p || p->opt.host_only) return 0;
  int m = p->elem >= 8 ? 1 : 0;
  if (p->mfma && p->opt.deriv_mode != IFGF_DERIV_FD) m |= 2;
  return m;
}

int ifgf_check(ifgf_plan_t p, void* stream, unsigned* flags) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  if (flags) *flags = 0;
  if (p->opt.host_only || !p->d_err) return IFGF_OK;
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_hip_error(e, "hipStreamSynchronize");
  unsigned w = 0;
  if ((e = hipMemcpy(&w, p->d_err, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess)
    return set_hip_error(e, "hipMemcpy");
  if (flags) *flags = w;
  if (w == 0) return IFGF_OK;
  if ((e = hipMemset(p->d_err, 0, sizeof(unsigned))) != hipSuccess) return set_hip_error(e, "hipMemset");
  return set_error(IFGF_EDEVICE, "a propagation wavefront gave up waiting for its accumulator lock; "
                                 "the sums of the applies since the last check are incomplete");
}

int ifgf_set_normals(ifgf_plan_t p, const double* normals) {
  clear_error();
  if (!p || !normals) return set_error(IFGF_EINVAL, "null argument");
  HostPlan& H = p->host;
  std::vector<double> s(3 * (size_t)H.n);
  for (int64_t i = 0; i < H.n; ++i) {
    const int64_t j = H.perm[i];
    const double a = normals[3 * j], b = normals[3 * j + 1], c = normals[3 * j + 2];
    if (!(std::fabs(std::sqrt(a * a + b * b + c * c) - 1.0) <= 1e-6))
      return set_error(IFGF_EINVAL, "normal is not unit length at index " + std::to_string(j));
    s[3 * i] = a;
    s[3 * i + 1] = b;
    s[3 * i + 2] = c;
  }
  H.nrm = s;
  if (p->opt.host_only || !p->d_nrm) return IFGF_OK;
  hipError_t e = hipMemcpy(p->d_nrm, s.data(), sizeof(double) * s.size(), hipMemcpyHostToDevice);
  return e == hipSuccess ? IFGF_OK : set_hip_error(e, "hipMemcpy");
}

int ifgf_set_lock_spin_limit(ifgf_plan_t p, int limit) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  if (limit < 0) return set_error(IFGF_EINVAL, "limit must be >= 0");
  p->spin_limit = limit;
  return IFGF_OK;
}

int ifgf_set_timing(ifgf_plan_t p, int on) {
  clear_error();
  if (!p) return set_error(IFGF_EINVAL, "plan is NULL");
  p->timer.reset();
  p->timer.on = on != 0;
  return IFGF_OK;
}

void ifgf_destroy(ifgf_plan_t p) {
  if (!p) return;
  p->timer.reset();
  delete p;
}

const char* ifgf_last_error(void) { return last_error_cstr(); }

}  // extern "C"
