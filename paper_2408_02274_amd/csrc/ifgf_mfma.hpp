// Matrix-core IFGF path: cone data in K-slot order (Pa = 5 or 6), FP32 or FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace ifgf {

// Propagation work list for one parent level: the tiles of parent cone slot
// q are [toff[q], toff[q+1]); rec[t] = (child cone slot, child box << 5 |
// points in the tile, index of the tile's first parent point in pts, child
// cone) and pts holds the parent interpolation point numbers of the groups.
struct PropGroups {
  const int64_t* toff = nullptr;
  const int4* rec = nullptr;
  const uint8_t* pts = nullptr;
};

// Target pairs of one level grouped by cone slot, in tiles of at most 8
// targets: tile t covers entries [start[t], start[t] + cnt[t]) of tgt (sorted
// target) and e (the pair's index in the target-major pair list).
struct TargetTiles {
  int64_t ntiles = 0;
  const int32_t* slot = nullptr;
  const int64_t* start = nullptr;
  const uint8_t* cnt = nullptr;
  const int32_t* tgt = nullptr;
  const int32_t* e = nullptr;
};

bool mfma_path_supported(int Ps, int Pa);
// rows per cone in K-slot order: both kernels per pass (nk = 2, rows of 32 R
// reals) or one kernel per pass (nk = 1, rows of 16 reals; Remark 3)
int kslot_rows(int Ps, int Pa, int nk);
// Right-hand sides per pass: cone rows hold R groups of 32 reals, R in {1, 2, 4}
// (FP32) or {1, 2} (FP64), as far as the propagation's LDS allows.
int max_batch_columns(bool fp32, int Ps, int Pa);

// a: [n][R][16] weighted densities of dens[r][8][n], r < R
hipError_t mf_gather(bool fp32, int R, const double2* dens, const int64_t* perm, const double* w, int64_t n,
                     void* a, hipStream_t st);
// nk = 2: both kernels (k0, k1) per pass; nk = 1 (R = 1 only): the kernel of
// wavenumber k0 alone, whose results go to the 14 outputs of kernel index qo
hipError_t mf_leaf(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                   const double* xs, const void* a, double k0, double k1, void* V, hipStream_t st);
// spin_limit bounds the wait for the FP32 accumulator lock; a wavefront that
// gives up skips its tile and sets bit 0 of *err (device word).
hipError_t mf_propagate(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& C, const DevLevel& P,
                        const InterpC& ic, const PropGroups& G, double k0, double k1, const void* Vc, void* Vp,
                        int spin_limit, unsigned* err, hipStream_t st);
// out_s: [R][n][28], accumulated
hipError_t mf_targets(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                      const double* xs, const double* nrm, int64_t n, double k0, double k1, const void* V,
                      double2* out_s, int qo, hipStream_t st);

// Target interpolation on the matrix cores (R right-hand sides per pass): per pair e
// the 14 nk complex contributions of each of R right-hand sides into res
// [pairs][R][14 nk] (complex in the cone precision), then out_s[r][i] += sum of
// res over the pairs of target i.
// fd: normal derivatives by the forward difference of the paper (FP64 only)
hipError_t mf_targets_tiles(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                            const TargetTiles& TT, const double* xs, const double* nrm, double k0, double k1,
                            const void* V, void* res, bool fd, hipStream_t st);
// out_s[r][i] += the per-pair results of targets i in [i0, i1), whose pairs
// start at tp_off[i0] in res, for r < R (out_s holds n points per r); nk = 1
// adds them to the 14 outputs of kernel index qo
hipError_t mf_targets_reduce(bool fp32, const DevLevel& L, int R, int nk, int qo, int64_t n, int64_t i0, int64_t i1,
                             const void* res, double2* out_s, hipStream_t st);

}  // namespace ifgf
