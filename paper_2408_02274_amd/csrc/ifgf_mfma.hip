// IFGF apply kernels on the matrix cores (MFMA 16x16x4, FP32 or FP64).
//
// Paper: Sec. III-G algorithm steps 2b (leaf cone values), 3a (interpolation
// onto cousin points times the centred factor, plus its normal derivative)
// and 3b (interpolation onto parent interpolation points times the
// re-centring factor G(X, x_child) / G(X, x_parent), summed over children).
//
// Cone data layout ("K-slot" order, Pa = 5 or 6).  A cone with Ps x Pa x Pa
// nodes (a, b, c) -> point p = Pa (Pa a + b) + c is stored as K = 4 * KS rows
// with nab = Pa Ps, tc = Pa - 4 and KS = nab + ceil(tc nab / 4):
//   c < 4  : row 4 * ab + c                      (ab = Pa a + b)
//   c >= 4 : row 4 * nab + tc * ab + (c - 4)
// remaining rows (up to an even number KS2 of 4-row k-steps) are zero
// padding.  A row holds R groups of 32 reals, one group per right-hand side of
// the batch: the real parts of the 16 complex columns (column = 8 * kernel +
// density) then their imaginary parts.  With this order the MFMA lane group
// g = lane / 16 supplies the phi-node c = g in the first nab k-steps and
// c = 4 + g mod tc in the others, so the interpolation weight of a lane is
// one product of per-point Lagrange factors.
//
// In memory the (row, column) values of a cone are stored in the order the
// matrix cores consume them (see kofs): for each pair of k-steps and each
// right-hand side, lane l = 16 g + c of a wavefront finds the four B operands
// it needs -- (row 4 j + g, column c), (row 4 j + g, column 16 + c) for
// j = 2 jp and j = 2 jp + 1 -- in four consecutive reals, so one 16-byte
// (FP32) load per lane feeds four MFMAs and a wavefront reads 1 KB of
// contiguous memory per load.
//
// One kernel at a time (Remark 3): a pass carries the 8 densities of one of
// the two kernels only, so a row holds 16 reals (the real parts of the 8
// complex columns, then their imaginary parts) and the cone buffers take half
// the memory.  The rows are padded to a multiple of four k-steps (K1 rows)
// and stored in consumption order per quad of k-steps (see kofs1): lane
// l = 16 g + c finds (row 4 j + g, column c) for the four k-steps j of a quad
// in four consecutive reals.  The real and imaginary parts of a column then
// come out of one MFMA in lanes c and c + 8, which swap them for the complex
// factors of the epilogues.
//
// The interpolant is the tensor Chebyshev interpolant of Sec. III-F in
// Lagrange form on the same nodes (identical polynomial).  Geometry is
// evaluated in cone-centred coordinates so that FP32 keeps relative accuracy:
// phases use r_child - r_parent = (|d|^2 - 2 Y.d) / (r_child + r_parent).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "ifgf_mfma.hpp"

namespace ifgf {

namespace {

constexpr double kPiD = 3.141592653589793;
constexpr double kInv4PiD = 0.07957747154594767;
constexpr double kEtaD = 0.5773502691896257;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <class T> struct MF;
template <> struct MF<float> {
  using acc = f4v;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row of element r held by lane l
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MF<double> {
  using acc = d4v;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <class T> __device__ __forceinline__ void tsincos(T x, T* s, T* c);
template <> __device__ __forceinline__ void tsincos<float>(float x, float* s, float* c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void tsincos<double>(double x, double* s, double* c) { sincos(x, s, c); }
template <class T> __device__ __forceinline__ T tacos(T x);
template <> __device__ __forceinline__ float tacos<float>(float x) { return acosf(x); }
template <> __device__ __forceinline__ double tacos<double>(double x) { return acos(x); }
template <class T> __device__ __forceinline__ T tatan2(T y, T x);
template <> __device__ __forceinline__ float tatan2<float>(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double tatan2<double>(double y, double x) { return atan2(y, x); }
template <class T> __device__ __forceinline__ T tsqrt(T x);
template <> __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }
template <> __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }

// Chebyshev nodes and Lagrange denominators in the working precision
template <class T> struct Nodes;
template <> struct Nodes<float> {
  __device__ static const float* xs(const InterpC& c) { return c.xsf; }
  __device__ static const float* xa(const InterpC& c) { return c.xaf; }
  __device__ static const float* ws(const InterpC& c) { return c.wsf; }
  __device__ static const float* wa(const InterpC& c) { return c.waf; }
};
template <> struct Nodes<double> {
  __device__ static const double* xs(const InterpC& c) { return c.xs; }
  __device__ static const double* xa(const InterpC& c) { return c.xa; }
  __device__ static const double* ws(const InterpC& c) { return c.ws; }
  __device__ static const double* wa(const InterpC& c) { return c.wa; }
};

// Lagrange basis on P Chebyshev nodes x with inverse denominators w
template <int P, class T, class X>
__device__ __forceinline__ void lag(const X* x, const X* w, T u, T* L) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    T p = (T)w[j];
#pragma unroll
    for (int m = 0; m < P; ++m)
      if (m != j) p *= (u - (T)x[m]);
    L[j] = p;
  }
}
template <int P, class T, class X>
__device__ __forceinline__ void lag_d(const X* x, const X* w, T u, T* dL) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    T acc = 0;
#pragma unroll
    for (int m = 0; m < P; ++m) {
      if (m == j) continue;
      T p = 1;
#pragma unroll
      for (int l = 0; l < P; ++l)
        if (l != j && l != m) p *= (u - (T)x[l]);
      acc += p;
    }
    dL[j] = acc * (T)w[j];
  }
}

// node (s, theta, phi) of point p of cone `cone` and the unit direction
template <int PA, class T>
__device__ __forceinline__ void cone_node(int ns, int na, int cone, int p, const InterpC& ic, T* s,
                                          T* ux, T* uy, T* uz) {
  const int ip = cone % (2 * na);
  const int it = (cone / (2 * na)) % na;
  const int is = cone / (2 * na * na);
  const int c = p % PA, b = (p / PA) % PA, a = p / (PA * PA);
  const double ds = kEtaD / ns, da = kPiD / na;
  *s = (T)((is + 0.5) * ds + 0.5 * ds * ic.xs[a]);
  T t = (T)((it + 0.5) * da + 0.5 * da * ic.xa[b]);
  T f = (T)((ip + 0.5) * da + 0.5 * da * ic.xa[c]);
  T st, ct, sp, cp;
  tsincos<T>(t, &st, &ct);
  tsincos<T>(f, &sp, &cp);
  *ux = st * cp;
  *uy = st * sp;
  *uz = ct;
}

// local coordinates of offset (zx, zy, zz) in cone `cone` (ns, na)
template <class T>
__device__ __forceinline__ void local3(T zx, T zy, T zz, T h, int ns, int na, int cone, T* r, T* us,
                                       T* ut, T* up, T* th, T* ph) {
  *r = tsqrt<T>(zx * zx + zy * zy + zz * zz);
  T s = h / *r;
  T ct = zz / *r;
  ct = ct > (T)1 ? (T)1 : (ct < (T)-1 ? (T)-1 : ct);
  *th = tacos<T>(ct);
  *ph = tatan2<T>(zy, zx);
  if (*ph < (T)0) *ph += (T)(2.0 * kPiD);
  const int ip = cone % (2 * na);
  const int it = (cone / (2 * na)) % na;
  const int is = cone / (2 * na * na);
  const T ds = (T)(kEtaD / ns), da = (T)(kPiD / na);
  *us = (s - ((T)is + (T)0.5) * ds) / ((T)0.5 * ds);
  *ut = (*th - ((T)it + (T)0.5) * da) / ((T)0.5 * da);
  *up = (*ph - ((T)ip + (T)0.5) * da) / ((T)0.5 * da);
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8),
// each XCD with its own L2.  Map blocks so that every XCD works on one
// contiguous range of work items: neighbouring cones (which share child cones
// and cousin data) then meet in the same L2.  A bijection of [0, nblocks).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t x = bid & 7, i = bid >> 3;
  const int64_t per = nblocks >> 3, rem = nblocks & 7;
  return x * per + (x < rem ? x : rem) + i;
}

// K-slot geometry of a Ps x PA x PA cone
template <int PS, int PA> struct KSlot {
  static constexpr int NAB = PS * PA;               // (radial, polar) node pairs
  static constexpr int TC = PA - 4;                 // phi-nodes past the first four
  static constexpr int KS = NAB + (TC * NAB + 3) / 4;   // k-steps that carry nodes
  static constexpr int KS2 = KS + (KS & 1);         // k-steps stored (even)
  static constexpr int K = 4 * KS2;                 // rows stored per cone
  static constexpr int KS4 = (KS + 3) & ~3;         // k-steps stored, one kernel per pass
  static constexpr int K1 = 4 * KS4;                // rows stored per cone, one kernel per pass
  static constexpr int NPTS = NAB * PA;
};

// Offset of (row, column) within one cone of R right-hand sides (32 R reals
// per row) in matrix-core consumption order: k-step pair jp = row / 8,
// right-hand side r = column / 32, lane 16 (row mod 4) + column mod 16,
// then (k-step parity, real/imaginary half).
template <int R>
__device__ __forceinline__ int kofs(int row, int col) {
  const int j = row >> 2, g = row & 3;
  const int r = col >> 5, h = (col >> 4) & 1, c = col & 15;
  return (((j >> 1) * R + r) * 64 + 16 * g + c) * 4 + 2 * (j & 1) + h;
}

// Offset of (row, column) within one cone of a one-kernel pass (16 reals
// per row): k-step quad j / 4, lane 16 (row mod 4) + column, then k-step
// j mod 4.
__device__ __forceinline__ int kofs1(int row, int col) {
  const int j = row >> 2, g = row & 3;
  return ((j >> 2) * 64 + 16 * g + col) * 4 + (j & 3);
}

template <class T> struct Vec4;
template <> struct Vec4<float> { using type = f4v; };
template <> struct Vec4<double> { using type = d4v; };

// reals per cone row: R groups of 32 (both kernels), or 16 (one kernel)
constexpr int row_reals(int R, int NK) { return NK == 2 ? 32 * R : 16; }
// LDS of the propagation kernel: accumulator (W reals per point), per-wavefront
// geometry records (4 wavefronts x 16 rows x tb tiles x (10 + 2 Pa) values),
// parent-point geometry, lock
constexpr int64_t prop_lds_bytes_tb(int Ps, int Pa, int W, int elem, int tb) {
  return (int64_t)Ps * Pa * Pa * (W + 1) * elem + 4 * 16 * tb * (10 + 2 * Pa) * elem +
         (int64_t)Ps * Pa * Pa * 4 * elem + 4;
}
// Tiles a wavefront prepares per geometry phase: 4, or 2 where that keeps an
// FP64 block within 80 KB of LDS (two blocks per compute unit).
constexpr int prop_tiles_per_batch(int Ps, int Pa, int W, int elem) {
  return (elem == 8 && prop_lds_bytes_tb(Ps, Pa, W, elem, 4) > 80 * 1024) ? 2 : 4;
}
constexpr int64_t prop_lds_bytes(int Ps, int Pa, int W, int elem) {
  return prop_lds_bytes_tb(Ps, Pa, W, elem, prop_tiles_per_batch(Ps, Pa, W, elem));
}
constexpr int64_t kLdsLimit = 160 * 1024;
// tiles of the target interpolation whose records a wavefront computes together
constexpr int target_tiles_per_wave(int elem) { return elem == 4 ? 4 : 2; }
// pairs of k-steps whose B operands a propagation wavefront keeps in flight
// (FP64 operands take twice the registers)
constexpr int prop_prefetch(int elem) { return elem == 4 ? 6 : 3; }

template <int PA>
__device__ __forceinline__ int point_of_row(int row, int nab) {
  constexpr int TC = PA - 4;
  if (row < 4 * nab) return PA * (row >> 2) + (row & 3);
  const int m = row - 4 * nab;
  return m < TC * nab ? PA * (m / TC) + 4 + m % TC : -1;
}
template <int PA>
__device__ __forceinline__ int row_of_point(int p, int nab) {
  constexpr int TC = PA - 4;
  const int c = p % PA, ab = p / PA;
  return c < 4 ? 4 * ab + c : 4 * nab + TC * ab + (c - 4);
}

// ---------------------------------------------------------------------------
// weighted densities in sorted order: a[i][r][m] = w_i phi_{r,m}(perm[i]) for
// the R right-hand sides dens[r][m][.]
template <class T>
__global__ void k_gather(const double2* __restrict__ dens, const int64_t* __restrict__ perm,
                         const double* __restrict__ w, int64_t n, int R, T* __restrict__ a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 8 * R) return;
  int64_t i = t / (8 * R);
  int r = (int)((t / 8) % R);
  int m = (int)(t % 8);
  double2 v = dens[((int64_t)r * 8 + m) * n + perm[i]];
  a[2 * t] = (T)(v.x * w[i]);
  a[2 * t + 1] = (T)(v.y * w[i]);
}

// sin and cos of a leaf phase k (|X - y| - |X - c|), and the divisions of the
// leaf geometry.  The phase is below a quarter turn at the leaf level (boxes
// of at most a quarter wavelength), where the FP32 form takes the hardware
// sine and cosine (argument in revolutions) and a reciprocal-based divide;
// the FP64 form keeps the library functions.
template <class T> __device__ __forceinline__ void leaf_sincos(T x, T* s, T* c) { tsincos<T>(x, s, c); }
template <> __device__ __forceinline__ void leaf_sincos<float>(float x, float* s, float* c) {
  const float rev = x * (float)(0.5 / kPiD);
  *s = __builtin_amdgcn_sinf(rev);
  *c = __builtin_amdgcn_cosf(rev);
}
template <class T> __device__ __forceinline__ T leaf_div(T a, T b) { return a / b; }
template <> __device__ __forceinline__ float leaf_div<float>(float a, float b) { return __fdividef(a, b); }

// leaf cone values: thread per (slot, row, right-hand side).  NK = 1: the
// 8 columns of kernel k0 only (one kernel per pass).
template <int PS, int PA, class T, int R, int NK>
__global__ void __launch_bounds__(256) k_leaf_k(DevLevel L, InterpC ic, const double* __restrict__ xs, const T* __restrict__ a,
                         double k0, double k1, T* __restrict__ V) {
  constexpr int NAB = KSlot<PS, PA>::NAB;
  constexpr int K = NK == 2 ? KSlot<PS, PA>::K : KSlot<PS, PA>::K1;
  constexpr int W = row_reals(R, NK);
  int64_t t = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= L.nslots * K * R) return;
  int64_t q = t / (K * R);
  int row = (int)((t / R) % K);
  const int r = (int)(t % R);
  // NK = 2: column c (real part) and 16 + c (imaginary part) sit side by
  // side; NK = 1: column c of the 16 reals at o[4 c]
  T* o = V + q * (int64_t)K * W + (NK == 2 ? kofs<R>(row, 32 * r) : kofs1(row, 0));
  int p = point_of_row<PA>(row, NAB);
  if (p < 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if constexpr (NK == 2) {
        o[4 * c] = (T)0;
        o[4 * c + 1] = (T)0;
      } else {
        o[4 * c] = (T)0;
      }
    }
    return;
  }
  int32_t b = L.slot_box[q];
  const double* c = L.centers + 3 * b;
  T s, ux, uy, uz;
  cone_node<PA, T>(L.ns, L.na, L.slot_cone[q], p, ic, &s, &ux, &uy, &uz);
  const T rxc = (T)L.h / s;
  const T Yx = rxc * ux, Yy = rxc * uy, Yz = rxc * uz;
  T acc[16 * NK];
#pragma unroll
  for (int m = 0; m < 16 * NK; ++m) acc[m] = (T)0;
  const T kk[2] = {(T)k0, (T)k1};
  for (int32_t j = L.start[b]; j < L.end[b]; ++j) {
    const T yx = (T)(xs[3 * j] - c[0]), yy = (T)(xs[3 * j + 1] - c[1]), yz = (T)(xs[3 * j + 2] - c[2]);
    const T dx = Yx - yx, dy = Yy - yy, dz = Yz - yz;
    const T rxy = tsqrt<T>(dx * dx + dy * dy + dz * dz);
    const T diff = leaf_div<T>(yx * yx + yy * yy + yz * yz - (T)2 * (Yx * yx + Yy * yy + Yz * yz), rxy + rxc);
    const T ratio = leaf_div<T>(rxc, rxy);
    const T* aj = a + ((int64_t)j * R + r) * 16;
#pragma unroll
    for (int qq = 0; qq < NK; ++qq) {
      T sn, cs;
      leaf_sincos<T>(kk[qq] * diff, &sn, &cs);
      const T gr = ratio * cs, gi = ratio * sn;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const T ar = aj[2 * m], ai = aj[2 * m + 1];
        acc[qq * 8 + m] += gr * ar - gi * ai;
        acc[8 * NK + qq * 8 + m] += gr * ai + gi * ar;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if constexpr (NK == 2) {
      o[4 * c] = acc[c];
      o[4 * c + 1] = acc[16 + c];
    } else {
      o[4 * c] = acc[c];
    }
  }
}

// ---------------------------------------------------------------------------
// propagation: one workgroup per parent cone slot, 4 wavefronts.  The tiles
// (16 parent points of one child cone) are dealt round-robin to the
// wavefronts.  A wavefront takes its tiles TB (4, or 2 for large FP64 cones)
// at a time: one lane per point evaluates the child-cone coordinates,
// Lagrange factors and re-centring factor of its point into wave-private LDS,
// then the TB MFMA tiles run.  NK = 1: one kernel per pass (wavenumber k0).
template <int PS, int PA, class T, int R, int NK>
__global__ void __launch_bounds__(256) k_prop_mfma(DevLevel C, DevLevel P, InterpC ic, PropGroups G,
                                                   double k0, double k1, const T* __restrict__ Vc,
                                                   T* __restrict__ Vp, int spin_limit,
                                                   unsigned* __restrict__ err) {
  constexpr int NAB = KSlot<PS, PA>::NAB;
  constexpr int TC = KSlot<PS, PA>::TC;
  constexpr int KS = KSlot<PS, PA>::KS;
  constexpr int K = NK == 2 ? KSlot<PS, PA>::K : KSlot<PS, PA>::K1;
  constexpr int NPTS = KSlot<PS, PA>::NPTS;
  // per-lane geometry record: Ls [0, PS), Lt [OT, OT + PA), Lp [OP, OP + PA),
  // re-centring factors [OF, OF + 4)
  constexpr int OT = 6, OP = OT + PA, OF = OP + PA, GW = OF + 4;
  constexpr int W = row_reals(R, NK);   // reals per cone row
  constexpr int TB = prop_tiles_per_batch(PS, PA, W, sizeof(T));
  __shared__ T acc[NPTS][W + 1];
  __shared__ T gbuf[4][16 * TB][GW];    // per wavefront: TB tiles x 16 rows
  __shared__ T geo[NPTS][4];            // parent points about the parent centre, and r_p
  __shared__ int acc_lock;              // held by the wavefront adding a tile into acc
  const int64_t q = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, gl = lane >> 4;
  for (int i = tid; i < NPTS * (W + 1); i += 256) (&acc[0][0])[i] = (T)0;
  if (tid == 0) acc_lock = 0;
  const int32_t pb = P.slot_box[q];
  const int pcone = P.slot_cone[q];
  const double* cp = P.centers + 3 * pb;
  if (tid < NPTS) {
    T s, ux, uy, uz;
    cone_node<PA, T>(P.ns, P.na, pcone, tid, ic, &s, &ux, &uy, &uz);
    const T rp = (T)P.h / s;
    geo[tid][0] = rp * ux;
    geo[tid][1] = rp * uy;
    geo[tid][2] = rp * uz;
    geo[tid][3] = rp;
  }
  __syncthreads();
  const T kk[2] = {(T)k0, (T)k1};
  const T two_ds = (T)(2.0 * C.ns / kEtaD), two_da = (T)(2.0 * C.na / kPiD);
  T(*gb)[GW] = gbuf[wave];
  const int64_t t_beg = G.toff[q], t_end = G.toff[q + 1];
  // this wavefront owns tiles t_beg + wave + 4 i, taken TB at a time; the
  // records of the next TB are fetched while the current ones run
  // rb / rn: the TB records, wave-uniform; mine / mine_n: this lane's own
  // record for the geometry phase (tile gl of the TB)
  int4 rb[TB], rn[TB], mine, mine_n;
  int nb = 0;
#pragma unroll
  for (int b = 0; b < TB; ++b) {
    const int64_t tl = t_beg + wave + 4 * b;
    rb[b] = tl < t_end ? G.rec[tl] : make_int4(0, 0, 0, 0);
    nb += tl < t_end ? 1 : 0;
  }
  {
    const int64_t tl = t_beg + wave + 4 * gl;
    mine = (gl < TB && tl < t_end) ? G.rec[tl] : make_int4(0, 0, 0, 0);
  }
  // B operands: one 16-byte (FP32) load per lane and right-hand side per
  // pair of k-steps (NK = 1: per quad of k-steps), issued PD - 1 loads ahead
  // of its use into a ring of registers; a scheduling barrier after each
  // load's k-steps keeps the compiler from sinking the loads next to their
  // use (an L2 hit takes far longer than the MFMAs they feed).  The first
  // loads of a tile are requested before the epilogue of the tile before it.
  using V4 = typename Vec4<T>::type;
  constexpr int SPL = NK == 2 ? 2 : 4;  // k-steps per load
  constexpr int NP = NK == 2 ? KSlot<PS, PA>::KS2 / 2 : KSlot<PS, PA>::KS4 / 4;
  constexpr int PD = prop_prefetch(sizeof(T));
  V4 ring[PD][R];
  auto first_pairs = [&](int32_t child_slot) {
    const T* vs = Vc + (int64_t)child_slot * K * W + 4 * lane;
#pragma unroll
    for (int i = 0; i < PD - 1 && i < NP; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) ring[i][r] = *reinterpret_cast<const V4*>(vs + (int64_t)(i * R + r) * 256);
  };
  if (nb > 0) first_pairs(rb[0].x);
  for (int64_t tb = t_beg + wave; tb < t_end; tb += 4 * TB) {
    int nn = 0;
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int64_t tl = tb + 4 * TB + 4 * b;
      rn[b] = tl < t_end ? G.rec[tl] : make_int4(0, 0, 0, 0);
      nn += tl < t_end ? 1 : 0;
    }
    {
      const int64_t tl = tb + 4 * TB + 4 * gl;
      mine_n = (gl < TB && tl < t_end) ? G.rec[tl] : make_int4(0, 0, 0, 0);
    }
    // geometry: lane -> (tile lane / 16, row lane % 16); the lane keeps its
    // parent point index for the epilogues, which read it across lanes
    int pme = 0;
    {
      const int b = gl;
      if (b < nb) {
        const int4 rr = mine;
        const int cnt = rr.y & 31;
        const bool valid = r16 < cnt;
        const int p = valid ? (int)G.pts[rr.z + r16] : 0;
        pme = p;
        const int cone = rr.w;
        const double* cc = C.centers + 3 * (int64_t)(rr.y >> 5);
        const T dx = (T)(cc[0] - cp[0]), dy = (T)(cc[1] - cp[1]), dz = (T)(cc[2] - cp[2]);
        const T Yx = geo[p][0], Yy = geo[p][1], Yz = geo[p][2], rp = geo[p][3];
        const T zx = Yx - dx, zy = Yy - dy, zz = Yz - dz;
        const T rc = tsqrt<T>(zx * zx + zy * zy + zz * zz);
        const T rci = (T)1 / rc;
        T ct = zz * rci;
        ct = ct > (T)1 ? (T)1 : (ct < (T)-1 ? (T)-1 : ct);
        const T th = tacos<T>(ct);
        T ph = tatan2<T>(zy, zx);
        if (ph < (T)0) ph += (T)(2.0 * kPiD);
        const int ip = cone % (2 * C.na);
        const int it = (cone / (2 * C.na)) % C.na;
        const int is = cone / (2 * C.na * C.na);
        const T us = (T)C.h * rci * two_ds - (T)(2 * is + 1);
        const T ut = th * two_da - (T)(2 * it + 1);
        const T up = ph * two_da - (T)(2 * ip + 1);
        T L[PS], Lt[PA], Lp[PA];
        lag<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us, L);
        lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut, Lt);
        lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up, Lp);
        const T vm = valid ? (T)1 : (T)0;
#pragma unroll
        for (int z = 0; z < PS; ++z) gb[lane][z] = L[z] * vm;
#pragma unroll
        for (int z = 0; z < PA; ++z) {
          gb[lane][OT + z] = Lt[z];
          gb[lane][OP + z] = Lp[z];
        }
        // re-centring factor G(X, x_child) / G(X, x_parent) = (rp / rc) exp(i k (rc - rp))
        const T diff = (dx * dx + dy * dy + dz * dz - (T)2 * (Yx * dx + Yy * dy + Yz * dz)) / (rc + rp);
        const T ratio = rp * rci;
#pragma unroll
        for (int qq = 0; qq < NK; ++qq) {
          T sn, cs;
          tsincos<T>(kk[qq] * diff, &sn, &cs);
          gb[lane][OF + 2 * qq] = ratio * cs;
          gb[lane][OF + 1 + 2 * qq] = ratio * sn;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      if (b >= nb) break;
      const int cnt = rb[b].y & 31;
      const T* Vs = Vc + (int64_t)rb[b].x * K * W + 4 * lane;
      const T* me = gb[16 * b + r16];
      T Ls[PS], Lt[PA];
#pragma unroll
      for (int z = 0; z < PS; ++z) Ls[z] = me[z];
#pragma unroll
      for (int z = 0; z < PA; ++z) Lt[z] = me[OT + z];
      const T lpg = me[OP + gl];
      // phi-node of this lane in the tail k-steps: 4 + gl mod tc
      const T lp4 = me[OP + 4 + (TC == 1 ? 0 : (gl & 1))];
      // st(ab) = Ls[a] Lt[b]: tabulated in registers, or formed per k-step
      // for large FP64 cones (the table's registers would cost occupancy)
      constexpr bool kTab = sizeof(T) == 4 || NAB <= 25;
      T st[kTab ? NAB : 1];
      if constexpr (kTab) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) st[ab] = Ls[ab / PA] * Lt[ab % PA];
      }
      auto stv = [&](int ab) -> T {
        if constexpr (kTab) return st[ab];
        else return Ls[ab / PA] * Lt[ab % PA];
      };
      typename MF<T>::acc c0[R], c1[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        c0[r] = typename MF<T>::acc{0, 0, 0, 0};
        c1[r] = typename MF<T>::acc{0, 0, 0, 0};
      }
#pragma unroll
      for (int j = 0; j < KS; ++j) {
        const int jp = j / SPL;
        if (j % SPL == 0 && jp + PD - 1 < NP) {
#pragma unroll
          for (int r = 0; r < R; ++r)
            ring[(jp + PD - 1) % PD][r] = *reinterpret_cast<const V4*>(Vs + (int64_t)((jp + PD - 1) * R + r) * 256);
        }
        T av;
        if (j < NAB) {
          av = stv(j) * lpg;
        } else if constexpr (TC == 1) {
          // slot 4 j + gl holds phi-node 4 of (a, b) pair m = 4 (j - NAB) + gl
          const int m0 = 4 * (j - NAB);
          T sel = (m0 < NAB) ? stv(m0 < NAB ? m0 : 0) : (T)0;
          sel = (gl == 1) ? ((m0 + 1 < NAB) ? stv(m0 + 1 < NAB ? m0 + 1 : 0) : (T)0) : sel;
          sel = (gl == 2) ? ((m0 + 2 < NAB) ? stv(m0 + 2 < NAB ? m0 + 2 : 0) : (T)0) : sel;
          sel = (gl == 3) ? ((m0 + 3 < NAB) ? stv(m0 + 3 < NAB ? m0 + 3 : 0) : (T)0) : sel;
          av = sel * lp4;
        } else {
          // slot 4 j + gl holds phi-node 4 + (gl & 1) of pair m = 2 (j - NAB) + gl / 2
          const int m0 = 2 * (j - NAB);
          T sel = (m0 < NAB) ? stv(m0 < NAB ? m0 : 0) : (T)0;
          sel = (gl >= 2) ? ((m0 + 1 < NAB) ? stv(m0 + 1 < NAB ? m0 + 1 : 0) : (T)0) : sel;
          av = sel * lp4;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const V4& b4 = ring[jp % PD][r];
          if constexpr (NK == 2) {
            c0[r] = MF<T>::mma(av, (j & 1) ? b4[2] : b4[0], c0[r]);
            c1[r] = MF<T>::mma(av, (j & 1) ? b4[3] : b4[1], c1[r]);
          } else {
            c0[r] = MF<T>::mma(av, b4[j & 3], c0[r]);
          }
        }
        if (j % SPL == SPL - 1) __builtin_amdgcn_sched_barrier(0);
      }
      // the next tile (of this batch, else the first of the next batch)
      if (b + 1 < nb) first_pairs(rb[b + 1 < TB ? b + 1 : 0].x);
      else if (nn > 0) first_pairs(rn[0].x);
      __builtin_amdgcn_sched_barrier(0);
      // NK = 2: lane holds rows MF::row(lane, e), complex column r16 (kernel
      // r16 / 8) in c0 (real) and c1 (imaginary part).  NK = 1: lane holds
      // real column r16 of kernel k0 in c0; lanes r16 < 8 hold real parts,
      // lanes r16 + 8 the imaginary parts of the same columns
      const int qq = NK == 2 ? r16 >> 3 : 0;
      if constexpr (NK == 1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) c1[0][e] = __shfl_xor(c0[0][e], 8);
      }
      const bool re_lane = r16 < 8;
      if constexpr (sizeof(T) == 4) {
        int po[4];
        T zr[4][R], zi[4][R];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int orow = MF<T>::row(lane, e);
          po[e] = __builtin_amdgcn_ds_bpermute((16 * b + orow) << 2, pme);
          const int ro = orow < cnt ? orow : 0;
          const T fr = gb[16 * b + ro][OF + 2 * qq], fi = gb[16 * b + ro][OF + 1 + 2 * qq];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if constexpr (NK == 2) {
              const T vr = c0[r][e], vi = c1[r][e];
              zr[e][r] = fr * vr - fi * vi;
              zi[e][r] = fr * vi + fi * vr;
            } else {
              // own value and the partner lane's: (re, im) of column r16 mod 8
              const T vr = re_lane ? c0[r][e] : c1[r][e], vi = re_lane ? c1[r][e] : c0[r][e];
              zr[e][r] = re_lane ? fr * vr - fi * vi : fr * vi + fi * vr;
            }
          }
        }
        // The rows of one tile are distinct parent points, so the tile is added
        // with plain loads and stores; other wavefronts of the block add tiles
        // of other child boxes into the same points, hence the block lock
        // around the read-add-write (cheaper than per-element LDS atomics).
        // The wait is bounded (spin_limit attempts).  A wavefront that gives up
        // neither adds its tile nor releases the lock; it records the failure
        // in the device error word, which the host turns into IFGF_EDEVICE.
        int got = 0;
        if (lane == 0) {
          int expected = 0;
#pragma unroll 1
          for (int spin = 0; spin < spin_limit; ++spin) {
            if (__hip_atomic_compare_exchange_strong(&acc_lock, &expected, 1, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
              got = 1;
              break;
            }
            expected = 0;
            __builtin_amdgcn_s_sleep(1);
          }
          if (!got) atomicOr(err, 1u);
        }
        got = __builtin_amdgcn_readfirstlane(got);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (got) {
          T oldr[4][R], oldi[4][R];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (MF<T>::row(lane, e) < cnt) {
#pragma unroll
              for (int r = 0; r < R; ++r) {
                oldr[e][r] = acc[po[e]][32 * r + r16];
                if constexpr (NK == 2) oldi[e][r] = acc[po[e]][32 * r + 16 + r16];
              }
            }
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (MF<T>::row(lane, e) < cnt) {
#pragma unroll
              for (int r = 0; r < R; ++r) {
                acc[po[e]][32 * r + r16] = oldr[e][r] + zr[e][r];
                if constexpr (NK == 2) acc[po[e]][32 * r + 16 + r16] = oldi[e][r] + zi[e][r];
              }
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) __hip_atomic_store(&acc_lock, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      } else {
        // FP64: native LDS add of doubles, no lock (the extra registers of
        // the locked form would halve the occupancy of this kernel)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int orow = MF<T>::row(lane, e);
          const int pe = __builtin_amdgcn_ds_bpermute((16 * b + orow) << 2, pme);
          if (orow < cnt) {
            const T fr = gb[16 * b + orow][OF + 2 * qq], fi = gb[16 * b + orow][OF + 1 + 2 * qq];
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if constexpr (NK == 2) {
                const T vr = c0[r][e], vi = c1[r][e];
                atomicAdd(&acc[pe][32 * r + r16], fr * vr - fi * vi);
                atomicAdd(&acc[pe][32 * r + 16 + r16], fr * vi + fi * vr);
              } else {
                const T vr = re_lane ? c0[r][e] : c1[r][e], vi = re_lane ? c1[r][e] : c0[r][e];
                atomicAdd(&acc[pe][r16], re_lane ? fr * vr - fi * vi : fr * vi + fi * vr);
              }
            }
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int b = 0; b < TB; ++b) rb[b] = rn[b];
    mine = mine_n;
    nb = nn;
  }
  __syncthreads();
  // contiguous stores in consumption order: offset i -> (row, column)
  T* out = Vp + q * (int64_t)K * W;
  for (int i = tid; i < K * W; i += 256) {
    int row, col;
    if constexpr (NK == 2) {
      const int h = i & 1, jo = (i >> 1) & 1, li = (i >> 2) & 63, blk = i >> 8;
      const int r = blk % R, jp = blk / R;
      row = 4 * (2 * jp + jo) + (li >> 4);
      col = 32 * r + 16 * h + (li & 15);
    } else {
      const int jj = i & 3, li = (i >> 2) & 63, jq = i >> 8;
      row = 4 * (4 * jq + jj) + (li >> 4);
      col = li & 15;
    }
    const int p = point_of_row<PA>(row, NAB);
    out[i] = p >= 0 ? acc[p][col] : (T)0;
  }
}

// ---------------------------------------------------------------------------
// interpolation onto cousin targets: two threads per target, one per
// wavenumber q (the 16 columns of a cone row split 8 + 8 by kernel); each
// loops over the target's cousin cones.  blockIdx.y selects the right-hand
// side r of the batch of R.  NK = 1 (one kernel per pass): one thread per
// target for kernel k0, whose 14 sums go to outputs 14 qo .. 14 qo + 13.
template <int PS, int PA, class T, int R, int NK>
__global__ void __launch_bounds__(64) k_targets_k(DevLevel L, InterpC ic, const double* __restrict__ xs,
                            const double* __restrict__ nrm, int64_t n, double k0, double k1,
                            const T* __restrict__ V, double2* __restrict__ out_s, int qo) {
  constexpr int NAB = KSlot<PS, PA>::NAB;
  constexpr int TC = KSlot<PS, PA>::TC;
  constexpr int K = NK == 2 ? KSlot<PS, PA>::K : KSlot<PS, PA>::K1;
  const int64_t g = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t i = NK == 2 ? g >> 1 : g;
  const int q = NK == 2 ? (int)(g & 1) : 0;
  if (i >= n) return;
  const int64_t e0 = L.tp_off[i], e1 = L.tp_off[i + 1];
  if (e0 == e1) return;
  const T nx = (T)nrm[3 * i], ny = (T)nrm[3 * i + 1], nz = (T)nrm[3 * i + 2];
  const T kq = (T)(q == 0 ? k0 : k1);
  const int rr = blockIdx.y;
  double2* o = out_s + ((int64_t)rr * n + i) * 28 + (NK == 2 ? q : qo) * 14;
  T Sr[8], Si[8], Dr[6], Di[6];
#pragma unroll
  for (int m = 0; m < 8; ++m) { Sr[m] = (T)0; Si[m] = (T)0; }
#pragma unroll
  for (int m = 0; m < 6; ++m) { Dr[m] = (T)0; Di[m] = (T)0; }
  for (int64_t e = e0; e < e1; ++e) {
    const int32_t slot = L.tp_slot[e];
    const int32_t B = L.slot_box[slot];
    const int cone = L.slot_cone[slot];
    const double* c = L.centers + 3 * B;
    const T zx = (T)(xs[3 * i] - c[0]), zy = (T)(xs[3 * i + 1] - c[1]), zz = (T)(xs[3 * i + 2] - c[2]);
    T r, us, ut, up, th, ph;
    local3<T>(zx, zy, zz, (T)L.h, L.ns, L.na, cone, &r, &us, &ut, &up, &th, &ph);
    T Ls[PS], Lt[PA], Lp[PA], dLs[PS], dLt[PA], dLp[PA];
    lag<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us, Ls);
    lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut, Lt);
    lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up, Lp);
    lag_d<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us, dLs);
    lag_d<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut, dLt);
    lag_d<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up, dLp);
    const T rinv = (T)1 / r;
    const T n_r = (nx * zx + ny * zy + nz * zz) * rinv;
    T st, ct, sp, cp;
    tsincos<T>(th, &st, &ct);
    tsincos<T>(ph, &sp, &cp);
    const T n_th = nx * ct * cp + ny * ct * sp - nz * st;
    const T n_ph = -nx * sp + ny * cp;
    T c_ph = st > (T)0 ? n_ph / (r * st) : (T)0;     // grad phi = phi-hat / (r sin theta)
    T c_s = -((T)L.h * rinv * rinv) * n_r;           // grad s = -(h / r^2) r-hat
    T c_t = n_th * rinv;                             // grad theta = theta-hat / r
    c_s *= (T)2 / ((T)(kEtaD / L.ns));
    c_t *= (T)2 / ((T)(kPiD / L.na));
    c_ph *= (T)2 / ((T)(kPiD / L.na));
    // F: interpolant of this kernel's 8 columns (re, im); FD: its n.grad for
    // the 6 Cartesian densities (re, im)
    T F[16], FD[12];
#pragma unroll
    for (int m = 0; m < 16; ++m) F[m] = (T)0;
#pragma unroll
    for (int m = 0; m < 12; ++m) FD[m] = (T)0;
    const T* Vs = V + (int64_t)slot * K * row_reals(R, NK);
    // radial index a runs in a rolled loop; Ls/dLs rotate so indices stay static
#pragma unroll 1
    for (int a = 0; a < PS; ++a) {
      const T la = Ls[0], dla = dLs[0];
#pragma unroll
      for (int z = 0; z + 1 < PS; ++z) {
        Ls[z] = Ls[z + 1];
        dLs[z] = dLs[z + 1];
      }
#pragma unroll
      for (int b = 0; b < PA; ++b) {
        const int ab = PA * a + b;
        const T lst = la * Lt[b];
        const T dst = c_s * dla * Lt[b] + c_t * la * dLt[b];
        const T phs = c_ph * la * Lt[b];
        // phi index cc in a rolled loop; Lp/dLp rotate cyclically (restored after PA steps)
#pragma unroll 1
        for (int cc = 0; cc < PA; ++cc) {
          const int row = cc < 4 ? 4 * ab + cc : 4 * NAB + TC * ab + (cc - 4);
          const T w = lst * Lp[0];
          const T wd = dst * Lp[0] + phs * dLp[0];
          {
            const T l0 = Lp[0], d0 = dLp[0];
#pragma unroll
            for (int z = 0; z + 1 < PA; ++z) {
              Lp[z] = Lp[z + 1];
              dLp[z] = dLp[z + 1];
            }
            Lp[PA - 1] = l0;
            dLp[PA - 1] = d0;
          }
          // NK = 2: column 8 q + m, real part at vr[4 m], imaginary part at
          // vr[4 m + 1]; NK = 1: real part at vr[4 m], imaginary at vr[4 (8 + m)]
          const T* vr = Vs + (NK == 2 ? kofs<R>(row, 32 * rr + 8 * q) : kofs1(row, 0));
          constexpr int IM = NK == 2 ? 1 : 32;
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            F[m] += w * vr[4 * m];
            F[8 + m] += w * vr[4 * m + IM];
          }
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            FD[m] += wd * vr[4 * m];
            FD[6 + m] += wd * vr[4 * m + IM];
          }
        }
      }
    }
    T sn, cs;
    tsincos<T>(kq * r, &sn, &cs);
    const T gr = cs * (T)kInv4PiD * rinv, gi = sn * (T)kInv4PiD * rinv;
    const T dgr = -rinv * n_r, dgi = kq * n_r;   // (i k - 1/r) n.r-hat
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const T fr = F[m], fi = F[8 + m];
      Sr[m] += gr * fr - gi * fi;
      Si[m] += gr * fi + gi * fr;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const T fr = F[m], fi = F[8 + m];
      const T tr = dgr * fr - dgi * fi + FD[m];
      const T ti = dgr * fi + dgi * fr + FD[6 + m];
      Dr[m] += gr * tr - gi * ti;
      Di[m] += gr * ti + gi * tr;
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    double2 v = o[m];
    o[m] = make_double2(v.x + (double)Sr[m], v.y + (double)Si[m]);
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double2 v = o[8 + m];
    o[8 + m] = make_double2(v.x + (double)Dr[m], v.y + (double)Di[m]);
  }
}

// ---------------------------------------------------------------------------
// interpolation onto cousin targets on the matrix cores: one wavefront per
// tile of up to 8 targets that fall in one cone.  MFMA row 2t carries the
// interpolation weights of target t, row 2t + 1 the weights of the normal
// derivative of the interpolant (chain rule through (s, theta, phi)); both
// are contracted with the cone's 32 value columns at once.  The epilogue
// applies the centred factor G(x, x_B) and its gradient and writes the 28
// complex contributions of each (target, cousin) pair to res; a second
// kernel sums them per target.
// FD (the paper's forward difference, Sec. III-I): row 2t + 1 instead holds
// the interpolation weights at x + h n in the cone of x (extrapolating where
// x + h n leaves it), and the normal derivative is (G(x + h n, x_B)
// F(x + h n) - G(x, x_B) F(x)) / h, h = 1e-6.
// NK = 1 (one kernel per pass): the 8 columns of kernel k0 only; a pair's
// 14 contributions go to res[(e R + r) 28].
template <int PS, int PA, class T, bool FD, int R, int NK>
__global__ void __launch_bounds__(256) k_targets_mfma(DevLevel L, InterpC ic, TargetTiles TT,
                                                      const double* __restrict__ xs,
                                                      const double* __restrict__ nrm, double k0, double k1,
                                                      const T* __restrict__ V, T* __restrict__ res) {
  constexpr int NAB = KSlot<PS, PA>::NAB;
  constexpr int TC = KSlot<PS, PA>::TC;
  constexpr int KS = KSlot<PS, PA>::KS;
  constexpr int K = NK == 2 ? KSlot<PS, PA>::K : KSlot<PS, PA>::K1;
  constexpr int WR = row_reals(R, NK);   // reals per cone row
  // per-target record: Ls, c_s dLs, Lt, c_t dLt, Lp, c_ph dLp, then
  // Re G_q, Im G_q (q = 0, 1), -n.r-hat / r, n.r-hat; with FD the derivative
  // slots hold Ls, Lt, Lp at x + h n and Re G_q, Im G_q there follow
  constexpr int OLS = 0, OSD = PS, OLT = 2 * PS, OTD = 2 * PS + PA, OLP = 2 * PS + 2 * PA,
                OPD = 2 * PS + 3 * PA, OG = 2 * PS + 4 * PA, TW = OG + (FD ? 10 : 6);
  constexpr double kFdH = 1e-6;
  // A wavefront takes TBT consecutive tiles: all their target records are
  // computed at once, lane l for target l mod 8 of tile l / 8, then the
  // tiles run on the matrix cores one after the other.
  constexpr int TBT = target_tiles_per_wave(sizeof(T));
  __shared__ T rec[4][8 * TBT][TW];
  __shared__ T outb[4][16][33];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, gl = lane >> 4;
  const int64_t tile0 = (xcd_remap(blockIdx.x, gridDim.x) * 4 + wave) * TBT;
  if (tile0 >= TT.ntiles) return;   // whole wavefront; only wavefront barriers follow
  const int nt = (int)(TT.ntiles - tile0 < TBT ? TT.ntiles - tile0 : TBT);
  T(*rw)[TW] = rec[wave];
  if (lane < 8 * TBT) {
    T* o = rw[lane];
    const int tl = lane >> 3, k = lane & 7;
    const int cntl = tl < nt ? (int)TT.cnt[tile0 + tl] : 0;
    if (k < cntl) {
      const int32_t slot = TT.slot[tile0 + tl];
      const int cone = L.slot_cone[slot];
      const double* c = L.centers + 3 * L.slot_box[slot];
      const int64_t i = TT.tgt[TT.start[tile0 + tl] + k];
      const T nx = (T)nrm[3 * i], ny = (T)nrm[3 * i + 1], nz = (T)nrm[3 * i + 2];
      const T zx = (T)(xs[3 * i] - c[0]), zy = (T)(xs[3 * i + 1] - c[1]), zz = (T)(xs[3 * i + 2] - c[2]);
      T r, us, ut, up, th, ph;
      local3<T>(zx, zy, zz, (T)L.h, L.ns, L.na, cone, &r, &us, &ut, &up, &th, &ph);
      T Ls[PS], Lt[PA], Lp[PA], dLs[PS], dLt[PA], dLp[PA];
      lag<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us, Ls);
      lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut, Lt);
      lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up, Lp);
      lag_d<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us, dLs);
      lag_d<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut, dLt);
      lag_d<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up, dLp);
      const T rinv = (T)1 / r;
      const T n_r = (nx * zx + ny * zy + nz * zz) * rinv;
      T sth, cth, sph, cph;
      tsincos<T>(th, &sth, &cth);
      tsincos<T>(ph, &sph, &cph);
      const T n_th = nx * cth * cph + ny * cth * sph - nz * sth;
      const T n_ph = -nx * sph + ny * cph;
      T c_ph = sth > (T)0 ? n_ph / (r * sth) : (T)0;   // grad phi = phi-hat / (r sin theta)
      T c_s = -((T)L.h * rinv * rinv) * n_r;           // grad s = -(h / r^2) r-hat
      T c_t = n_th * rinv;                             // grad theta = theta-hat / r
      c_s *= (T)2 / ((T)(kEtaD / L.ns));
      c_t *= (T)2 / ((T)(kPiD / L.na));
      c_ph *= (T)2 / ((T)(kPiD / L.na));
      if constexpr (FD) {
        // x + h n in the cone of x, its Lagrange weights and centred factor
        const T zx2 = zx + (T)kFdH * nx, zy2 = zy + (T)kFdH * ny, zz2 = zz + (T)kFdH * nz;
        T r2, us2, ut2, up2, th2, ph2;
        local3<T>(zx2, zy2, zz2, (T)L.h, L.ns, L.na, cone, &r2, &us2, &ut2, &up2, &th2, &ph2);
        lag<PS, T>(Nodes<T>::xs(ic), Nodes<T>::ws(ic), us2, dLs);
        lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), ut2, dLt);
        lag<PA, T>(Nodes<T>::xa(ic), Nodes<T>::wa(ic), up2, dLp);
        c_s = c_t = c_ph = (T)1;
#pragma unroll
        for (int q = 0; q < NK; ++q) {
          T sn, cs;
          tsincos<T>((T)(q == 0 ? k0 : k1) * r2, &sn, &cs);
          o[OG + 6 + q] = cs * (T)kInv4PiD / r2;
          o[OG + 8 + q] = sn * (T)kInv4PiD / r2;
        }
      }
#pragma unroll
      for (int z = 0; z < PS; ++z) {
        o[OLS + z] = Ls[z];
        o[OSD + z] = c_s * dLs[z];
      }
#pragma unroll
      for (int z = 0; z < PA; ++z) {
        o[OLT + z] = Lt[z];
        o[OTD + z] = c_t * dLt[z];
        o[OLP + z] = Lp[z];
        o[OPD + z] = c_ph * dLp[z];
      }
#pragma unroll
      for (int q = 0; q < NK; ++q) {
        T sn, cs;
        tsincos<T>((T)(q == 0 ? k0 : k1) * r, &sn, &cs);
        o[OG + q] = cs * (T)kInv4PiD * rinv;
        o[OG + 2 + q] = sn * (T)kInv4PiD * rinv;
      }
      o[OG + 4] = -rinv * n_r;
      o[OG + 5] = n_r;
    } else {
      for (int z = 0; z < TW; ++z) o[z] = (T)0;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
  for (int ti = 0; ti < nt; ++ti) {
  const int64_t tile = tile0 + ti;
  const int32_t slot = TT.slot[tile];
  const int64_t kbeg = TT.start[tile];
  const int cnt = TT.cnt[tile];
  if (ti > 0) {
    // the epilogue of the tile before has read the output buffer
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // A operand of row r16 (target t, value or derivative) at node (a, b, c):
  //   value:      Ls[a] Lt[b] Lp[c]
  //   derivative: (c_s dLs[a]) Lt[b] Lp[c] + Ls[a] (c_t dLt[b]) Lp[c] + Ls[a] Lt[b] (c_ph dLp[c])
  // = Lt[b] U[a] + (c_t dLt[b]) W[a] with per-lane U, W for the phi-node c
  const int t = r16 >> 1;
  const T kv = (r16 & 1) ? (T)0 : (T)1, kd = (T)1 - kv;
  const T* me = rw[8 * ti + t];
  // (FD: value rows Lt[b] U[a], U = Ls Lp; difference rows Lt2[b] W[a], W = Ls2 Lp2)
  T U[PS], W[PS], Ltv[PA], Tdv[PA];
  if constexpr (FD) {
    const T f1 = kv * me[OLP + gl], f2 = kd * me[OPD + gl];
#pragma unroll
    for (int a = 0; a < PS; ++a) {
      U[a] = me[OLS + a] * f1;
      W[a] = me[OSD + a] * f2;
    }
  } else {
    const T f1 = kv * me[OLP + gl] + kd * me[OPD + gl], f2 = kd * me[OLP + gl];
#pragma unroll
    for (int a = 0; a < PS; ++a) {
      U[a] = me[OLS + a] * f1 + me[OSD + a] * f2;
      W[a] = me[OLS + a] * f2;
    }
  }
  {
#pragma unroll
    for (int b = 0; b < PA; ++b) {
      Ltv[b] = me[OLT + b];
      Tdv[b] = me[OTD + b];
    }
  }
  // phi-node of this lane in the tail k-steps: 4 + gl mod tc
  const int ct4 = 4 + (TC == 1 ? 0 : (gl & 1));
  const T g1 = FD ? kv * me[OLP + ct4] : kv * me[OLP + ct4] + kd * me[OPD + ct4];
  const T g2 = FD ? kd * me[OPD + ct4] : kd * me[OLP + ct4];
  typename MF<T>::acc c0[R], c1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) c0[r] = c1[r] = typename MF<T>::acc{0, 0, 0, 0};
  // R right-hand sides: each cone row holds R groups of 32 values, pair jp
  // of right-hand side r at (jp R + r) 256 reals (MFMA consumption order);
  // NK = 1: quad jp of k-steps at jp 256 reals
  const T* Vs = V + (int64_t)slot * K * WR + 4 * lane;
  // B operands of a pair (quad) of k-steps are requested PD - 1 loads ahead
  // of their use (see the propagation kernel)
  using V4 = typename Vec4<T>::type;
  constexpr int SPL = NK == 2 ? 2 : 4;  // k-steps per load
  constexpr int NP = NK == 2 ? KSlot<PS, PA>::KS2 / 2 : KSlot<PS, PA>::KS4 / 4;
  constexpr int PD = prop_prefetch(sizeof(T));
  V4 ring[PD][R];
#pragma unroll
  for (int i = 0; i < PD - 1 && i < NP; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r) ring[i][r] = *reinterpret_cast<const V4*>(Vs + (int64_t)(i * R + r) * 256);
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const int jp = j / SPL;
    if (j % SPL == 0 && jp + PD - 1 < NP)
#pragma unroll
      for (int r = 0; r < R; ++r)
        ring[(jp + PD - 1) % PD][r] = *reinterpret_cast<const V4*>(Vs + (int64_t)((jp + PD - 1) * R + r) * 256);
    T av;
    if (j < NAB) {
      av = Ltv[j % PA] * U[j / PA] + Tdv[j % PA] * W[j / PA];   // (a, b) = j, phi-node gl
    } else {
      const int ab = (4 * (j - NAB) + gl) / TC;                // phi-node ct4 of pair ab
      if (ab < NAB) {
        const T lsa = me[OLS + ab / PA], sda = me[OSD + ab / PA];
        if constexpr (FD)
          av = me[OLT + ab % PA] * lsa * g1 + me[OTD + ab % PA] * sda * g2;
        else
          av = me[OLT + ab % PA] * (lsa * g1 + sda * g2) + me[OTD + ab % PA] * lsa * g2;
      } else {
        av = (T)0;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const V4& b4 = ring[jp % PD][r];
      if constexpr (NK == 2) {
        c0[r] = MF<T>::mma(av, (j & 1) ? b4[2] : b4[0], c0[r]);
        c1[r] = MF<T>::mma(av, (j & 1) ? b4[3] : b4[1], c1[r]);
      } else {
        c0[r] = MF<T>::mma(av, b4[j & 3], c0[r]);
      }
    }
    if (j % SPL == SPL - 1) __builtin_amdgcn_sched_barrier(0);
  }
  T(*ob)[33] = outb[wave];
  // epilogue, one right-hand side at a time through the wavefront's LDS
  // buffer: lane -> target lane / 8, density m = lane % 8, both kernels;
  // results of right-hand side r at res[(e R + r) 56] (NK = 1: column m of
  // ob holds the real, column 8 + m the imaginary part; res[(e R + r) 28])
  const int tt = lane >> 3, m = lane & 7;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r > 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = MF<T>::row(lane, e);
      ob[row][r16] = c0[r][e];
      if constexpr (NK == 2) ob[row][16 + r16] = c1[r][e];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (tt < cnt) {
    const int64_t e = TT.e[kbeg + tt];
    const T* g = rw[8 * ti + tt] + OG;
    T* out = res + (e * R + r) * 28 * NK;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      const int col = 8 * q + m, cim = NK == 2 ? 16 + col : 8 + m;
      const T fr = ob[2 * tt][col], fi = ob[2 * tt][cim];
      const T gr = g[q], gi = g[2 + q];
      out[2 * (14 * q + m)] = gr * fr - gi * fi;
      out[2 * (14 * q + m) + 1] = gr * fi + gi * fr;
      if (m < 6) {
        const T dr = ob[2 * tt + 1][col], di = ob[2 * tt + 1][cim];
        if constexpr (FD) {
          const T g2r = g[6 + q], g2i = g[8 + q];
          const T ih = (T)(1.0 / kFdH);
          out[2 * (14 * q + 8 + m)] = ((g2r * dr - g2i * di) - (gr * fr - gi * fi)) * ih;
          out[2 * (14 * q + 8 + m) + 1] = ((g2r * di + g2i * dr) - (gr * fi + gi * fr)) * ih;
        } else {
          const T dgr = g[4], dgi = (T)(q == 0 ? k0 : k1) * g[5];   // (i k - 1/r) n.r-hat
          const T tr = dgr * fr - dgi * fi + dr, ti = dgr * fi + dgi * fr + di;
          out[2 * (14 * q + 8 + m)] = gr * tr - gi * ti;
          out[2 * (14 * q + 8 + m) + 1] = gr * ti + gi * tr;
        }
      }
    }
  }
  }
  }
}

// out_s[r][i][ko + k] += sum over the target pairs e of i of
// res[(e - e0) R + r][k], k < nk (28, or the 14 of one kernel), for targets
// i0 <= i < i1 whose pairs start at e0 = tp_off[i0] and right-hand sides r < R
// (FP64 sums; out_s holds n points of 28 outputs per right-hand side)
template <class T>
__global__ void __launch_bounds__(256) k_targets_reduce(const int64_t* __restrict__ tp_off, int64_t n, int64_t i0,
                                                        int64_t i1, int R, int nk, int ko, const T* __restrict__ res,
                                                        double2* __restrict__ out_s) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (i1 - i0) * nk;
  if (g >= per * R) return;
  const int r = (int)(g / per);
  const int64_t i = i0 + (g % per) / nk;
  const int k = (int)(g % nk);
  const int64_t e0 = tp_off[i0];
  double re = 0.0, im = 0.0;
  for (int64_t e = tp_off[i] - e0; e < tp_off[i + 1] - e0; ++e) {
    re += (double)res[(e * R + r) * 2 * nk + 2 * k];
    im += (double)res[(e * R + r) * 2 * nk + 2 * k + 1];
  }
  const int64_t o = (int64_t)r * 28 * n + i * 28 + ko + k;
  const double2 v = out_s[o];
  out_s[o] = make_double2(v.x + re, v.y + im);
}

inline unsigned nblk(int64_t w, int bs) { return (unsigned)((w + bs - 1) / bs); }

template <int PS, int PA, class T, int R, int NK>
hipError_t leaf_t(const DevLevel& L, const InterpC& ic, const double* xs, const void* a, double k0,
                  double k1, void* V, hipStream_t st) {
  constexpr int K = NK == 2 ? KSlot<PS, PA>::K : KSlot<PS, PA>::K1;
  int64_t work = L.nslots * K * R;
  if (work <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_leaf_k<PS, PA, T, R, NK>), dim3(nblk(work, 256)), dim3(256), 0, st, L, ic, xs,
                     static_cast<const T*>(a), k0, k1, static_cast<T*>(V));
  return hipGetLastError();
}
template <int PS, int PA, class T, int R, int NK>
hipError_t prop_t(const DevLevel& C, const DevLevel& P, const InterpC& ic, const PropGroups& G,
                  double k0, double k1, const void* Vc, void* Vp, int spin_limit, unsigned* err,
                  hipStream_t st) {
  if constexpr (prop_lds_bytes(PS, PA, row_reals(R, NK), sizeof(T)) > kLdsLimit) {
    return hipErrorInvalidValue;   // excluded by max_batch_columns
  } else {
    if (P.nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_prop_mfma<PS, PA, T, R, NK>), dim3((unsigned)P.nslots), dim3(256), 0, st, C, P, ic, G, k0,
                       k1, static_cast<const T*>(Vc), static_cast<T*>(Vp), spin_limit, err);
    return hipGetLastError();
  }
}
template <int PS, int PA, class T, int R, int NK>
hipError_t targets_t(const DevLevel& L, const InterpC& ic, const double* xs, const double* nrm,
                     int64_t n, double k0, double k1, const void* V, double2* out_s, int qo, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_targets_k<PS, PA, T, R, NK>), dim3(nblk(NK * n, 64), R), dim3(64), 0, st, L, ic, xs, nrm, n,
                     k0, k1, static_cast<const T*>(V), out_s, qo);
  return hipGetLastError();
}
template <int PS, int PA, class T, int R, int NK>
hipError_t targets_tiles_t(const DevLevel& L, const InterpC& ic, const TargetTiles& TT, const double* xs,
                           const double* nrm, double k0, double k1, const void* V, void* res, bool fd,
                           hipStream_t st) {
  if (TT.ntiles <= 0) return hipSuccess;
  if (fd) {
    if constexpr (std::is_same<T, double>::value && R == 1)
      hipLaunchKernelGGL((k_targets_mfma<PS, PA, T, true, 1, NK>), dim3(nblk(TT.ntiles, 4 * target_tiles_per_wave(sizeof(T)))), dim3(256), 0, st, L,
                         ic, TT, xs, nrm, k0, k1, static_cast<const T*>(V), static_cast<T*>(res));
    else
      return hipErrorInvalidValue;   // the forward difference is FP64 with one right-hand side only
  } else {
    hipLaunchKernelGGL((k_targets_mfma<PS, PA, T, false, R, NK>), dim3(nblk(TT.ntiles, 4 * target_tiles_per_wave(sizeof(T)))), dim3(256), 0, st, L,
                       ic, TT, xs, nrm, k0, k1, static_cast<const T*>(V), static_cast<T*>(res));
  }
  return hipGetLastError();
}

// Calls f.template operator()<PS, PA>() for the supported orders (Pa = 5 or
// 6, 3 <= Ps <= 6); hipErrorInvalidValue otherwise.
template <class F>
hipError_t with_orders(int Ps, int Pa, F&& f) {
  if (Pa == 5) {
    switch (Ps) {
      case 3: return f.template operator()<3, 5>();
      case 4: return f.template operator()<4, 5>();
      case 5: return f.template operator()<5, 5>();
      case 6: return f.template operator()<6, 5>();
    }
  } else if (Pa == 6) {
    switch (Ps) {
      case 3: return f.template operator()<3, 6>();
      case 4: return f.template operator()<4, 6>();
      case 5: return f.template operator()<5, 6>();
      case 6: return f.template operator()<6, 6>();
    }
  }
  return hipErrorInvalidValue;
}

// R = 1, 2 or 4 right-hand sides per pass with both kernels (NK = 2); FP64
// takes at most 2 (the LDS of the propagation at R = 4 would exceed a
// workgroup's 160 KB).  One kernel per pass (NK = 1) takes R = 1 only.
template <class T, class F>
hipError_t with_columns(int R, int nk, F&& f) {
  if (nk == 1) return R == 1 ? f.template operator()<1, 1>() : hipErrorInvalidValue;
  if (nk != 2) return hipErrorInvalidValue;
  switch (R) {
    case 1: return f.template operator()<1, 2>();
    case 2: return f.template operator()<2, 2>();
    case 4:
      if constexpr (std::is_same<T, float>::value) return f.template operator()<4, 2>();
      break;
  }
  return hipErrorInvalidValue;
}

template <class T>
hipError_t dispatch_leaf(int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic, const double* xs,
                         const void* a, double k0, double k1, void* V, hipStream_t st) {
  return with_orders(Ps, Pa, [&]<int PS, int PA>() {
    return with_columns<T>(R, nk, [&]<int RR, int NK>() {
      return leaf_t<PS, PA, T, RR, NK>(L, ic, xs, a, k0, k1, V, st);
    });
  });
}
template <class T>
hipError_t dispatch_prop(int Ps, int Pa, int R, int nk, const DevLevel& C, const DevLevel& P, const InterpC& ic,
                         const PropGroups& G, double k0, double k1, const void* Vc, void* Vp, int spin_limit,
                         unsigned* err, hipStream_t st) {
  return with_orders(Ps, Pa, [&]<int PS, int PA>() {
    return with_columns<T>(R, nk, [&]<int RR, int NK>() {
      return prop_t<PS, PA, T, RR, NK>(C, P, ic, G, k0, k1, Vc, Vp, spin_limit, err, st);
    });
  });
}
template <class T>
hipError_t dispatch_targets(int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic, const double* xs,
                            const double* nrm, int64_t n, double k0, double k1, const void* V,
                            double2* out_s, int qo, hipStream_t st) {
  return with_orders(Ps, Pa, [&]<int PS, int PA>() {
    return with_columns<T>(R, nk, [&]<int RR, int NK>() {
      return targets_t<PS, PA, T, RR, NK>(L, ic, xs, nrm, n, k0, k1, V, out_s, qo, st);
    });
  });
}
template <class T>
hipError_t dispatch_targets_tiles(int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                                  const TargetTiles& TT, const double* xs, const double* nrm, double k0, double k1,
                                  const void* V, void* res, bool fd, hipStream_t st) {
  return with_orders(Ps, Pa, [&]<int PS, int PA>() {
    return with_columns<T>(R, nk, [&]<int RR, int NK>() {
      return targets_tiles_t<PS, PA, T, RR, NK>(L, ic, TT, xs, nrm, k0, k1, V, res, fd, st);
    });
  });
}

}  // namespace

bool mfma_path_supported(int Ps, int Pa) { return (Pa == 5 || Pa == 6) && Ps >= 3 && Ps <= 6; }

int kslot_rows(int Ps, int Pa, int nk) {
  const int nab = Pa * Ps, tc = Pa - 4;
  const int ks = nab + (tc * nab + 3) / 4;
  return nk == 1 ? 4 * ((ks + 3) & ~3) : 4 * (ks + (ks & 1));
}

int max_batch_columns(bool fp32, int Ps, int Pa) {
  for (int R = fp32 ? 4 : 2; R > 1; R /= 2)
    if (prop_lds_bytes(Ps, Pa, row_reals(R, 2), fp32 ? 4 : 8) <= kLdsLimit) return R;
  return 1;
}

hipError_t mf_gather(bool fp32, int R, const double2* dens, const int64_t* perm, const double* w, int64_t n,
                     void* a, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_gather<float>, dim3(nblk(n * 8 * R, 256)), dim3(256), 0, st, dens, perm, w, n, R,
                       static_cast<float*>(a));
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(nblk(n * 8 * R, 256)), dim3(256), 0, st, dens, perm, w, n, R,
                       static_cast<double*>(a));
  return hipGetLastError();
}

hipError_t mf_leaf(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                   const double* xs, const void* a, double k0, double k1, void* V, hipStream_t st) {
  return fp32 ? dispatch_leaf<float>(Ps, Pa, R, nk, L, ic, xs, a, k0, k1, V, st)
              : dispatch_leaf<double>(Ps, Pa, R, nk, L, ic, xs, a, k0, k1, V, st);
}

hipError_t mf_propagate(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& C, const DevLevel& P,
                        const InterpC& ic, const PropGroups& G, double k0, double k1, const void* Vc, void* Vp,
                        int spin_limit, unsigned* err, hipStream_t st) {
  return fp32 ? dispatch_prop<float>(Ps, Pa, R, nk, C, P, ic, G, k0, k1, Vc, Vp, spin_limit, err, st)
              : dispatch_prop<double>(Ps, Pa, R, nk, C, P, ic, G, k0, k1, Vc, Vp, spin_limit, err, st);
}

hipError_t mf_targets(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                      const double* xs, const double* nrm, int64_t n, double k0, double k1, const void* V,
                      double2* out_s, int qo, hipStream_t st) {
  return fp32 ? dispatch_targets<float>(Ps, Pa, R, nk, L, ic, xs, nrm, n, k0, k1, V, out_s, qo, st)
              : dispatch_targets<double>(Ps, Pa, R, nk, L, ic, xs, nrm, n, k0, k1, V, out_s, qo, st);
}

hipError_t mf_targets_tiles(bool fp32, int Ps, int Pa, int R, int nk, const DevLevel& L, const InterpC& ic,
                            const TargetTiles& TT, const double* xs, const double* nrm, double k0, double k1,
                            const void* V, void* res, bool fd, hipStream_t st) {
  return fp32 ? dispatch_targets_tiles<float>(Ps, Pa, R, nk, L, ic, TT, xs, nrm, k0, k1, V, res, fd, st)
              : dispatch_targets_tiles<double>(Ps, Pa, R, nk, L, ic, TT, xs, nrm, k0, k1, V, res, fd, st);
}

hipError_t mf_targets_reduce(bool fp32, const DevLevel& L, int R, int nk, int qo, int64_t n, int64_t i0, int64_t i1,
                             const void* res, double2* out_s, hipStream_t st) {
  if (i1 <= i0) return hipSuccess;
  if (nk != 1 && nk != 2) return hipErrorInvalidValue;
  const int w = 14 * nk, ko = nk == 1 ? 14 * qo : 0;
  const unsigned nb = nblk((i1 - i0) * w * R, 256);
  if (fp32)
    hipLaunchKernelGGL(k_targets_reduce<float>, dim3(nb), dim3(256), 0, st, L.tp_off, n, i0, i1, R, w, ko,
                       static_cast<const float*>(res), out_s);
  else
    hipLaunchKernelGGL(k_targets_reduce<double>, dim3(nb), dim3(256), 0, st, L.tp_off, n, i0, i1, R, w, ko,
                       static_cast<const double*>(res), out_s);
  return hipGetLastError();
}

}  // namespace ifgf
