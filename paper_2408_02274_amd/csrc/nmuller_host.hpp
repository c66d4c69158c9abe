// Host-side N-Mueller plan: surface quantities and near-field corrections.
//
// Paper: Sec. III-A (patches, open Chebyshev grid, point order), Sec. III-C
// (Fejer weights), Sec. III-D (rectangular-polar singular moments), Sec. III-H
// (local corrections).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ifgf {

struct SurfaceGeo {
  int P = 0, nc = 0;
  int64_t n = 0;
  std::vector<double> x, du, dv;    // [n][3] input
  std::vector<double> nrm, t1, t2;  // [n][3]
  std::vector<double> J, w;         // [n]
  // (J a^u, J a^v) = Q (c1, c2) for a tangent field a = c1 t1 + c2 t2: Q [n][4] row-major
  std::vector<double> Q;
  // surface gradient: grad f = (gu f_u + gv f_v) with gu = iuu du + iuv dv,
  // gv = iuv du + ivv dv: [n][3] each
  std::vector<double> gu, gv;
  std::vector<double> Dcheb;        // [nc][nc] values -> derivative values at the nodes
};

struct SingParams {
  double delta_factor = 1.0;
  int nbeta = 0;   // 0 -> 6 nc
  int d = 4;
  int sweeps = 4, iters = 40;
};

// Near-field corrections in block form: for target l the singular patches
// pair_patch[row_off[l] .. row_off[l+1]) and for each pair 4 x nc^2 complex
// weights, kernel order (S k_int, S k_ext, D k_int, D k_ext), node order of the
// patch (i*nc + j).
struct Corrections {
  int nc = 0;
  std::vector<int64_t> row_off;     // [n+1]
  std::vector<int32_t> pair_patch;  // [npairs]
  std::vector<double> vals;         // [npairs][4][nc*nc][2]
};

// Inputs of the singular quadrature shared by the host and device builders:
// Chebyshev coefficients of each patch's node coordinates A [P][Nc^2][3]
// (coefficient (m, n) of eta_p), the patch node bounding boxes lo, hi [P][3]
// and radii delta [P] of eq. patch_sing, the Chebyshev nodes tn [Nc] of the
// patches, the Fejer rule (tb, wb) [nb] of eq. int_moments_cov, the
// values -> coefficients matrix M [Nc][Nc] and the golden-section ratio.
struct SingTables {
  int nb = 0;
  double gold = 0.0;
  std::vector<double> A, lo, hi, delta, tn, tb, wb, M;
};

int build_surface(SurfaceGeo& g, int P, int nc, const double* x, const double* du,
                  const double* dv, std::string& err);
int sing_tables(const SurfaceGeo& g, const SingParams& sp, SingTables& t, std::string& err);
int build_corrections(const SurfaceGeo& g, double k_int, double k_ext, const SingParams& sp,
                      Corrections& c, std::string& err);

}  // namespace ifgf
