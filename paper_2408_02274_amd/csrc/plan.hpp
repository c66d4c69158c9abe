// Host-side IFGF plan: box octree, cone structure and relevant-cone tables.
//
// Paper: Sec. III-F (cone segments), Sec. III-G (octree, neighbours, cousins,
// relevant cones eq. rele_cone, Remark 2 cone counts, algorithm step 1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ifgf {

constexpr int kMaxP = 8;      // largest Ps / Pa supported by the kernels

struct HostLevel {
  int d = 0;
  double H = 0.0, h = 0.0;     // box side and radius h = sqrt(3) H / 2
  int ns = 0, na = 0;          // cone counts (levels >= 3)
  int64_t ncones = 0;          // ns * na * 2 na
  int64_t nb = 0;              // non-empty ("relevant") boxes, Morton order
  std::vector<int64_t> key;
  std::vector<int32_t> coords;             // [nb][3] integer box coordinates
  std::vector<double> centers;             // [nb][3]
  std::vector<int32_t> start, end;         // point range in sorted order
  std::vector<int32_t> parent;             // box index at level d-1
  std::vector<int32_t> child_start, child_end;  // box range at level d+1
  std::vector<int32_t> nbr_off, nbr;       // neighbours (CSR, self included)
  std::vector<int32_t> cous_off, cous;     // cousins (CSR), levels >= 3
  // relevant cones, slots ordered by (box, cone)
  std::vector<int64_t> slot_off;           // [nb+1]
  std::vector<int32_t> slot_cone, slot_box;
  int64_t nslots = 0;
  // interpolation onto cousin points: for sorted target i, the relevant cone
  // slot of each cousin box of box(i), in cousin-list order
  std::vector<int64_t> tp_off;             // [n+1]
  std::vector<int32_t> tp_slot;
  // propagation (levels >= 4): for parent slot q at level d-1, child j of its
  // box and interpolation point k, the child's cone slot at level d
  std::vector<int64_t> pp_off;             // [nslots(d-1)+1], stride nchild*npts
  std::vector<int32_t> pp_slot;
  // the same pairs grouped by child cone: for parent slot q of this level the
  // groups [pg_off[q], pg_off[q+1]); a group lists the interpolation points
  // pg_pts[pg_start .. +pg_count) of q that lie in child cone slot pg_slot of
  // child box pg_cbox (children in order, points ascending)
  std::vector<int64_t> pg_off, pg_start;
  std::vector<int32_t> pg_slot, pg_cbox, pg_count;
  std::vector<uint8_t> pg_pts;
  // 16-point tiles of those groups: for parent slot q the tiles
  // [pt_off[q], pt_off[q+1]); tile t covers points pt_t0[t] .. +16 of group pt_g[t]
  std::vector<int64_t> pt_off;
  std::vector<int32_t> pt_g;
  std::vector<uint8_t> pt_t0;
  // one record per tile, everything the propagation needs to start it:
  // [tile][4] = child cone slot, child box << 5 | number of points (<= 16),
  // index of the tile's first point in pg_pts, child cone index (a cone index
  // needs up to 31 bits: 2^30 cones per box at level 3 of a 40-wavelength body)
  std::vector<int32_t> pt_rec;
  // the target pairs in chunks of consecutive targets (chunk c: targets
  // [tc_i0[c], tc_i0[c+1]), pairs from tp_off[tc_i0[c]], at most
  // tc_max_pairs of them), within a chunk grouped by cone slot (targets
  // ascending within a slot) and cut into tiles of at most 8 targets: tile t
  // covers entries [tt_start[t], tt_start[t] + tt_cnt[t]) of ts_tgt (sorted
  // target) and ts_e (its pair index relative to the chunk's first pair), all
  // of slot tt_slot[t]; the tiles of chunk c are [tc_tile[c], tc_tile[c+1])
  std::vector<int32_t> ts_tgt, ts_e;
  std::vector<int32_t> tt_slot;
  std::vector<int64_t> tt_start;
  std::vector<uint8_t> tt_cnt;
  std::vector<int64_t> tc_tile, tc_i0;
  int64_t tc_max_pairs = 0;
};

struct HostPlan {
  int64_t n = 0;
  double k[2] = {0.0, 0.0};
  double kmax = 0.0;
  int Ps = 3, Pa = 5, npts = 75;
  int D = 1;
  double H1 = 1.0;
  double center[3] = {0, 0, 0}, origin[3] = {0, 0, 0};
  std::vector<int64_t> perm;               // sorted position -> input index
  std::vector<double> xs, nrm, w;          // sorted points, normals, weights
  std::vector<HostLevel> lev;              // lev[d], d = 1..D
  std::vector<int32_t> leaf_of_point;      // sorted point -> leaf box
  int64_t near_pairs = 0, leaf_pairs = 0;
};

// Pairs per chunk of the per-pair target results: 1 GiB of FP64 results.
constexpr int64_t kTargetChunkPairs = ((int64_t)1 << 30) / (56 * 8);

struct PlanParams {
  int Ps = 3, Pa = 5, ns_init = 1, na_init = 2, refine_radial = 1;
  double leaf_wavelengths = 0.25;
  int verbose = 0;   // progress lines on stderr
  int64_t target_chunk_pairs = 0;   // target pairs per result chunk (0: kTargetChunkPairs)
};

// Returns 0 on success, else fills err.
int build_host_plan(HostPlan& P, int64_t n, const double* x, const double* nrm,
                    const double* w, double k0, double k1, const PlanParams& pp,
                    std::string& err);

// The same tables built by kernels on the current device (host arrays in,
// HostPlan filled on the host; device temporaries freed on return).  Returns
// 0 on success, -1 for a size limit, -2 for a HIP error; fills err.
int build_device_plan(HostPlan& P, int64_t n, const double* x, const double* nrm,
                      const double* w, double k0, double k1, const PlanParams& pp,
                      std::string& err);

// Cut the target pairs of level L into chunks of consecutive targets with at
// most chunk_pairs pairs each, group each chunk's pairs by cone slot and cut
// them into tiles of at most 8 targets.
void build_target_tiles(HostLevel& L, int64_t n, int64_t chunk_pairs);


// Group the propagation pairs of parent level Pl (children at level L) by
// child cone slot (requires npts <= 256).
void build_prop_groups(HostLevel& Pl, const HostLevel& L, int npts);

// cos and sin of the cone boundary angles k pi / na, k = 0..na.
void cone_dirs(int na, std::vector<double>& C, std::vector<double>& S);

// Cone index of the offset (dx,dy,dz) from a box centre (box radius h) with
// ns x na x 2na cones (Sec. III-F): i_s = min(floor(s / ds), ns - 1) with
// s = h / r; i_theta counts the boundaries k = 1..na-1 with cos theta <= C[k];
// i_phi counts those whose ray (C[k], S[k]) has the point on or
// counter-clockwise of it, in the point's half plane (y > 0 or y = 0 <= x;
// the lower half turned by pi, plus na); i_phi = 0 on the z axis.
int cone_index(double dx, double dy, double dz, double h, int ns, int na, const double* C, const double* S);

}  // namespace ifgf
