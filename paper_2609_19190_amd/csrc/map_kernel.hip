// Fused spatial-mapping kernel for gfx950 (CDNA4, wave64).
//
// What it computes: for every VOI voxel c, the features of its cubic
// neighbourhood V(c) = cube(2r+1) ∩ image ∩ mask (paper: "Software design
// and extraction modes" -- spatial maps; Table 2 -- 18 first-order, 24 GLCM,
// 16 GLRLM, 16 GLSZM, 14 GLDM, 5 NGTDM maps; feature equations per IBSI as
// the paper defers to it, with the readings stated in fr.h).
//
// How: one wavefront (= one workgroup) owns a contiguous run of compact
// mask indices and handles its voxels one after another, all 64 lanes on
// one voxel:
//   gather   lane per cube position: levels + raw values into LDS
//   levels   local compaction of the levels present (L <= LMAX), so every
//            table is L-sized instead of Ng-sized
//   count    lane per cube position, one pass over the 26 neighbours:
//            equal-level neighbour bitmask, GLCM counts (13 forward
//            offsets, LDS atomics; equal pairs folded into one diagonal add),
//            GLCM row sums, GLDM dependence, NGTDM exact integer sums,
//            zone labels by minimum-label propagation over equal-level bits
//   runs     GLRLM: a run starts where the backward neighbour bit is clear;
//            walk the forward bits
//   features FP64, wave-shuffle reductions; integer numerators kept exact
//            where a feature is a ratio of integer sums; GLCM features via
//            the sum/difference histograms; MCC as the spectral radius of
//            D^-1/2 P D^-1/2 - v v^T (v = sqrt(px)), by Householder
//            tridiagonalisation and Sturm-count multisection (64 probes per
//            round across the lanes)
// Nothing here is a dense contraction, so no MFMA; the bound is LDS and
// VALU (FP64) work per voxel.
#include <math.h>
#include <stddef.h>

#include <type_traits>
#include <utility>

#include "fr_internal.h"
#include "map_device.h"

namespace fr {
namespace {

constexpr int kNFO = 18, kNGLCM = 24, kNGLRLM = 16, kNGLSZM = 16, kNGLDM = 14, kNNGTDM = 5;

// One deferred MCC problem: a neighbourhood with 2..NL present levels whose
// MCC is computed later, together with up to three others (one per 16-lane
// row of the wave).
template <int NL>
struct McProblemT {
  float* dst;  // address of this voxel's MCC map value
  int n;       // number of present levels
  // co-occurrence counts of the present levels, upper triangle (entry
  // (a, b), a <= b, at b (b + 1) / 2 + a; the row sums and N_P follow from
  // them exactly)
  uint16_t g[NL * (NL + 1) / 2];
};
using McProblem = McProblemT<32>;  // 17..32 levels (or 2..32 without a small pool)
using McSmall = McProblemT<16>;    // 2..16 levels
template <typename P, int N>
struct McSlots {
  P s[N];
};
template <typename P>
struct McSlots<P, 0> {};
static_assert(sizeof(McProblem) == kMccProblemBytes, "stash entry size");
static_assert(sizeof(McSmall) <= sizeof(McProblem), "stash entry size");

// Every neighbourhood with at most 32 present levels defers its MCC: four
// problems per flush.  A problem's result depends only on the problem (not
// on the instance or on what shares its flush).  Wider problems (64-level
// instances) are computed at the flush that follows their voxel, from the
// GLCM that is still in LDS.
template <int R, int LMAX>
constexpr int kMcSlots = 4;
// Problems with <= 16 levels have a pool of their own (four small slots),
// so both kinds of flush run with four problems; the radius-3, 32-level
// instance (whose LDS budget is tighter: eight workgroups per CU) keeps
// them in its large slots instead.
template <int R, int LMAX>
constexpr int kSmallSlots = (R == 3 && LMAX == 32) ? 0 : 4;

// MOUT: the MCC problems with <= 32 levels go to a global stash for the
// MCC kernel (no deferred-problem slots in LDS).
template <int R, int LMAX, bool MOUT = false>
struct Smem {
  static constexpr int S = 2 * R + 1;
  static constexpr int C = S * S * S;
  static constexpr int CP = (C + 63) / 64 * 64;
  static constexpr int SP = R == 1 ? 64 : (R == 2 ? 128 : 512);  // sort size, 64 * pow2 >= C
  // zone hash slots: more than the distinct (level, size) pairs, which are
  // at most |V| (27, 125) or, for radius 3, 178 (sizes 1, 2 for 64 levels
  // and 3 for 50 use 342 voxels)
  static constexpr int HT = R == 1 ? 64 : 256;
  // GLCM |i-j| and i+j histograms over level values 1..Ng (Ng <= 255)
  static constexpr int PD = 256;
  static constexpr int PS = 512;
  // words of the packed 16-bit upper triangle of the co-occurrence table
  static constexpr int kTriWords = (LMAX * (LMAX + 1) / 2 + 1) / 2;
  static constexpr int SQ = S + 2;                                // padded cube side
  static constexpr int PC = (SQ * SQ * SQ + 3) / 4 * 4;
  uint8_t cl[CP];        // level per cube position (0: not in V)
  uint8_t clp[PC];       // the same levels in a cube with a zero border of 1
  // level values 1..255; at most LMAX of them present in one neighbourhood
  // (a neighbourhood with more is handed to a wider instance)
  static constexpr int LV = 256;
  static constexpr int LVW = LV / 4;
  uint8_t lflag[LV];     // level present in V
  uint8_t lmap[LV];      // level -> compact index
  uint8_t lval[LMAX];    // compact index -> level
  uint32_t hist[LMAX];   // level histogram
  uint32_t pxc[LMAX];    // GLCM row sums
  // this voxel's maps: a member, or (radius 3 with 32 levels, where LDS
  // decides the occupancy) the zone-size table, free once the zones are
  // counted and out of reach of the overlays b and c below
  static constexpr bool kFeatInZcnt = R == 3 && LMAX == 32;
  float feat_m[kFeatInZcnt ? 1 : 96];
  McSlots<McProblem, MOUT ? 0 : kMcSlots<R, LMAX>> mq;  // deferred MCC problems
  McSlots<McSmall, MOUT ? 0 : kSmallSlots<R, LMAX>> ms;  // deferred MCC problems, <= 16 levels
  // The counting tables (a), the GLCM feature histograms (c) and the MCC
  // work space (b) share one region; b and c keep a.glcm in place and put
  // their arrays past it, over tables whose features are already done.
  union U {
    struct A {
      // compact co-occurrence counts, row stride L, two 16-bit counts per
      // word (entry e in half e & 1 of word e >> 1; all counts add up to
      // twice the forward pairs, at most 26 (2r+1)^3 < 2^16)
      uint32_t glcm[kTriWords];
      // equal-level neighbour bits; once the runs are counted, the sorted raw
      // values of V (float) for the order statistics
      uint32_t same[CP];
      uint32_t parent[CP]; // zone labels
      uint32_t zcnt[CP / 2];  // zone sizes at roots (16-bit, packed as the GLCM)
      uint32_t glrlm[LMAX * S];
      uint32_t gldm[(LMAX * 27 + 1) / 2];  // 16-bit counts, packed
      uint32_t ngn[LMAX];
      unsigned long long ngS[LMAX];
      uint32_t zpl[LMAX];
      uint32_t zps[CP / 2];  // zones per size (16-bit, packed)
      uint32_t hkey[HT];
      uint32_t hcnt[HT / 2];  // zones per (level, size) key (16-bit, packed)
    } a;
    struct C {
      uint32_t glcm[kTriWords];  // a.glcm
      uint32_t pd[PD];                 // |i-j| histogram of the GLCM
      uint32_t ps[PS];                 // i+j histogram of the GLCM
    } c;
    struct B {
      uint32_t glcm[kTriWords];  // a.glcm, still read by the MCC
      int pl[LMAX];                    // compact level of present level i
      double d[LMAX];                  // tridiagonal form: diagonal
      double e2[LMAX];                 // and squared sub-diagonal
      float* big_dst;                  // a pending problem with > 32 levels
      int big_n;
    } b;
  } u;
  __device__ float* feat() { return kFeatInZcnt ? (float*)u.a.zcnt : feat_m; }
};


// Packed 16-bit counts (GLCM, GLDM, zone tables): entry e in half e & 1 of
// word e >> 1; every count stays below 2^16 (at most 26 (2r+1)^3).
__device__ inline void gadd(uint32_t* g, int e, uint32_t v) {
  atomicAdd(&g[e >> 1], v << ((e & 1) << 4));
}
__device__ inline uint32_t gget(const uint32_t* g, int e) {
  return (g[e >> 1] >> ((e & 1) << 4)) & 0xffffu;
}
// The co-occurrence table holds the upper triangle of the symmetric matrix,
// entry (r, c), r <= c, at c (c + 1) / 2 + r (the counting pass adds each
// unequal pair once, at (min, max)).
__device__ inline int tri(int r, int c) { return c * (c + 1) / 2 + r; }
__device__ inline uint32_t gsym(const uint32_t* g, int r, int c) {
  return gget(g, r <= c ? tri(r, c) : tri(c, r));
}

// Wavefront reductions on the VALU (DPP), every call site with all 64
// lanes active; the result is a wave-uniform scalar.
__device__ inline double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline long long readlane_l(long long x, int l) {
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return ((long long)hi << 32) | (unsigned)lo;
}
// the two values a 64-bit x takes after a permlane16 (R16) or permlane32
// swap of a register with itself: lane i gets x of lane i and of i ^ 16 (32)
template <bool R16>
__device__ inline void swap_pair(long long b, long long& p0, long long& p1) {
  if (R16) {
    const auto lo = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
    p0 = ((long long)hi[0] << 32) | (unsigned)lo[0];
    p1 = ((long long)hi[1] << 32) | (unsigned)lo[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
    p0 = ((long long)hi[0] << 32) | (unsigned)lo[0];
    p1 = ((long long)hi[1] << 32) | (unsigned)lo[1];
  }
}
// One DPP step on a 64-bit value (bit moves): a single 64-bit move for the
// row broadcasts (row_newbcast), two 32-bit moves for the other patterns.
// Steps that write every lane need no identity; the row broadcasts of
// row_bcast:15/31 write only some rows and give the identity bits `id` to
// the others.
template <int CTRL>
__device__ inline long long dpp64(long long b) {
  return __builtin_amdgcn_mov_dpp(b, CTRL, 0xf, 0xf, true);
}
template <int CTRL, int ROWMASK>
__device__ inline long long dpp64m(long long b, long long id) {
  return __builtin_amdgcn_update_dpp(id, b, CTRL, ROWMASK, 0xf, false);
}
// Reduce across the wavefront: four steps inside each row of 16 lanes
// (quad_perm twice, half-row mirror, row mirror: every lane then holds its
// row total), then two row broadcasts fold rows 0..3 into lane 63, which is
// read back as a uniform scalar.
template <typename Op>
__device__ inline long long wfold64(long long v, long long id, Op op) {
  v = op(v, dpp64<0xb1>(v));             // quad_perm [1,0,3,2]
  v = op(v, dpp64<0x4e>(v));             // quad_perm [2,3,0,1]
  v = op(v, dpp64<0x141>(v));            // row_half_mirror
  v = op(v, dpp64<0x140>(v));            // row_mirror
  v = op(v, dpp64m<0x142, 0xa>(v, id));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp64m<0x143, 0xc>(v, id));  // row_bcast:31 into rows 2, 3
  return readlane_l(v, 63);
}
__device__ inline double wsum(double v) {
  return __longlong_as_double(wfold64(__double_as_longlong(v), 0ll, [](long long a, long long b) {
    return __double_as_longlong(__longlong_as_double(a) + __longlong_as_double(b));
  }));
}
__device__ inline long long wsumi(long long v) {
  return wfold64(v, 0ll, [](long long a, long long b) { return a + b; });
}
__device__ inline double wmaxd_nonneg(double v) {  // identity 0.0: inputs are >= 0
  return __longlong_as_double(wfold64(__double_as_longlong(v), 0ll, [](long long a, long long b) {
    return __double_as_longlong(fmax(__longlong_as_double(a), __longlong_as_double(b)));
  }));
}
__device__ inline unsigned wmaxu(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xb1, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4e, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ inline int wscan_excl(int v, int lane, int* total) {
  // inclusive scan by DPP (no LDS round trips): shifts by 1, 2, 4, 8 inside
  // each 16-lane row (zero shifted in), then lane 15 of a row added to the
  // next row (rows 1, 3) and lane 31 to rows 2 and 3; every lane active
  (void)lane;
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  *total = __builtin_amdgcn_readlane(x, 63);
  return x - v;
}

// Eight wavefront sums at once.  A permlane32 swap adds lanes l and l+32
// while keeping values 0-3 in the low half and 4-7 in the high half; a
// permlane16 swap does the same for row pairs; each row then holds two
// values, reduced in its two 8-lane halves by DPP (row mirror, half-row
// mirror, quad permutes).  Total k ends in lane 8 k.
__device__ inline double fold32d(double x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((int)bx, (int)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((int)(bx >> 32), (int)(by >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]) +
         __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
}
__device__ inline double fold16d(double x, double y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((int)bx, (int)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((int)(bx >> 32), (int)(by >> 32), false, false);
  return __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]) +
         __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
}
template <int CTRL>
__device__ inline double dppd(double x) {
  return __longlong_as_double(dpp64<CTRL>(__double_as_longlong(x)));
}
__device__ inline void wsum8d(double (&v)[8]) {
  const double a0 = fold32d(v[0], v[4]), a1 = fold32d(v[1], v[5]);
  const double a2 = fold32d(v[2], v[6]), a3 = fold32d(v[3], v[7]);
  const double b0 = fold16d(a0, a2), b1 = fold16d(a1, a3);  // row r: values 2r', 2r'+1
  const bool hi8 = (threadIdx.x & 8) != 0;
  double c = (hi8 ? b1 : b0) + dppd<0x140>(hi8 ? b0 : b1);  // row_mirror
  c += dppd<0x141>(c);                                        // row_half_mirror
  c += dppd<0x4e>(c);
  c += dppd<0xb1>(c);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = readlane_d(c, 8 * k);
}
__device__ inline int fold32i(int x, int y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  return r[0] + r[1];
}
__device__ inline int fold16i(int x, int y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  return r[0] + r[1];
}
// 32-bit integer version (callers guarantee every total fits in int32).
__device__ inline void wsum8i(int (&v)[8]) {
  const int a0 = fold32i(v[0], v[4]), a1 = fold32i(v[1], v[5]);
  const int a2 = fold32i(v[2], v[6]), a3 = fold32i(v[3], v[7]);
  const int b0 = fold16i(a0, a2), b1 = fold16i(a1, a3);
  const bool hi8 = (threadIdx.x & 8) != 0;
  int c = (hi8 ? b1 : b0) + __builtin_amdgcn_mov_dpp(hi8 ? b0 : b1, 0x140, 0xf, 0xf, true);
  c += __builtin_amdgcn_mov_dpp(c, 0x141, 0xf, 0xf, true);
  c += __builtin_amdgcn_mov_dpp(c, 0x4e, 0xf, 0xf, true);
  c += __builtin_amdgcn_mov_dpp(c, 0xb1, 0xf, 0xf, true);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_readlane(c, 8 * k);
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) inside [-x, x)
// (Sturm): the sign changes of the leading principal minors
//   p_0 = 1, p_1 = d_0 - y, p_i = (d_{i-1} - y) p_{i-1} - e_{i-2}^2 p_{i-2}
// count the eigenvalues below y; the sequences for y = x and y = -x run
// interleaved, without divisions.  The matrices here have n <= 64 and
// entries of magnitude below 3, so |p_i| < 6^64 never overflows.  A zero
// minor takes a tiny value of the previous minor's sign, the convention of
// the ratio form.  Sign changes are counted on the sign bits.
// D[i] = d_i and E2[i] = e_i^2 are LDS arrays read as broadcasts.
__device__ inline int sign_change(double a, double b) {
  return (int)(((uint32_t)(__double_as_longlong(a) >> 32) ^ (uint32_t)(__double_as_longlong(b) >> 32)) >> 31);
}
// SEQ 3: Sturm count of [-x, x) (eigenvalues below x minus those below -x);
// SEQ 1: eigenvalues below x only; SEQ 2: eigenvalues below -x only.  The
// counts of 1 and 2 are the two terms of 3, computed the same way.
template <int SEQ = 3>
__device__ inline int sturm_span_r(const double* D, const double* E2, int n, double x) {
  const double d0 = D[0];
  double ap = d0 - x, am = d0 + x, bp = 1.0, bm = 1.0;
  ap = ap == 0.0 ? 0x1p-1000 : ap;
  am = am == 0.0 ? 0x1p-1000 : am;
  int cnt = 0;
  if constexpr (SEQ & 1) cnt += sign_change(ap, 1.0);
  if constexpr (SEQ & 2) cnt += SEQ == 3 ? -sign_change(am, 1.0) : sign_change(am, 1.0);
  for (int i = 1; i < n; ++i) {
    const double di = D[i], e2 = E2[i - 1];
    if constexpr (SEQ & 1) {
      double np = fma(di - x, ap, -e2 * bp);
      np = np == 0.0 ? copysign(0x1p-1000, ap) : np;
      cnt += sign_change(np, ap);
      bp = ap;
      ap = np;
    }
    if constexpr (SEQ & 2) {
      double nm = fma(di + x, am, -e2 * bm);
      nm = nm == 0.0 ? copysign(0x1p-1000, am) : nm;
      cnt += SEQ == 3 ? -sign_change(nm, am) : sign_change(nm, am);
      bm = am;
      am = nm;
    }
  }
  return cnt;
}

// ---- MCC of four neighbourhoods at once --------------------------------
// Row r of 16 lanes holds problem r; lane j of the row is column j.  Values
// move inside a row by DPP (row broadcast of lane I, row mirrors), so the
// four problems never mix and each one's result does not depend on its row.
#define FR_INLINE __attribute__((always_inline))
// The lane index through an opaque move: nothing derived from it is
// hoisted out of the voxel loop, where it would stay live (and spill)
// across the large MCC flush.
__device__ FR_INLINE inline int opaque_lane() {
  int lane;
  asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"((int)threadIdx.x));
  return lane;
}
template <int B, int E, typename F>
__device__ FR_INLINE inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
template <int I>
__device__ inline double rbc(double v) {  // lane I of this row
  return __longlong_as_double(dpp64<0x150 + I>(__double_as_longlong(v)));
}
__device__ inline double rsum(double v) {  // row total in every lane of the row
  long long b = __double_as_longlong(v);
  b = __double_as_longlong(__longlong_as_double(b) + __longlong_as_double(dpp64<0xb1>(b)));
  b = __double_as_longlong(__longlong_as_double(b) + __longlong_as_double(dpp64<0x4e>(b)));
  b = __double_as_longlong(__longlong_as_double(b) + __longlong_as_double(dpp64<0x141>(b)));
  b = __double_as_longlong(__longlong_as_double(b) + __longlong_as_double(dpp64<0x140>(b)));
  return __longlong_as_double(b);
}
__device__ inline double rmax(double v) {
  long long b = __double_as_longlong(v);
  b = __double_as_longlong(fmax(__longlong_as_double(b), __longlong_as_double(dpp64<0xb1>(b))));
  b = __double_as_longlong(fmax(__longlong_as_double(b), __longlong_as_double(dpp64<0x4e>(b))));
  b = __double_as_longlong(fmax(__longlong_as_double(b), __longlong_as_double(dpp64<0x141>(b))));
  b = __double_as_longlong(fmax(__longlong_as_double(b), __longlong_as_double(dpp64<0x140>(b))));
  return __longlong_as_double(b);
}

// Sturm count of [-x, x) for the row's tridiagonal (D[i] = d_i and
// E2[i] = e_i^2 already broadcast to every lane of the row), N = 16 or 32
// entries; SEQ as for sturm_span_r.
template <int N, int SEQ = 3>
__device__ FR_INLINE inline int sturm_row(const double (&D)[N], const double (&E2)[N], int n, double x) {
  const double d0 = D[0];
  double ap = d0 - x, am = d0 + x, bp = 1.0, bm = 1.0;
  ap = ap == 0.0 ? 0x1p-1000 : ap;
  am = am == 0.0 ? 0x1p-1000 : am;
  int cnt = 0;
  if constexpr (SEQ & 1) cnt += sign_change(ap, 1.0);
  if constexpr (SEQ & 2) cnt += SEQ == 3 ? -sign_change(am, 1.0) : sign_change(am, 1.0);
  static_for<1, N>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    const double di = D[i], e2 = E2[i - 1];
    if (i < n) {
      if constexpr (SEQ & 1) {
        double np = fma(di - x, ap, -e2 * bp);
        np = np == 0.0 ? copysign(0x1p-1000, ap) : np;
        cnt += sign_change(np, ap);
        bp = ap;
        ap = np;
      }
      if constexpr (SEQ & 2) {
        double nm = fma(di + x, am, -e2 * bm);
        nm = nm == 0.0 ? copysign(0x1p-1000, am) : nm;
        cnt += SEQ == 3 ? -sign_change(nm, am) : sign_change(nm, am);
        bm = am;
        am = nm;
      }
    }
  });
  return cnt;
}

// Slot of the stash that row r takes: the r-th set bit of mask (-1: none).
__device__ inline int row_slot(unsigned mask, int r) {
  int slot = -1, c = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if ((mask >> s) & 1u) {
      if (c == r) slot = s;
      ++c;
    }
  }
  return slot;
}

// 6 rounds of 17-way Sturm multisection of [0, min(gb, 1)] for the row's
// tridiagonal (16 probes per row; width <= 1 / 17^6); the spectrum of B
// lies in [-1, 1] (that of D^-1/2 P D^-1/2 without its top eigenvalue 1).
template <typename F>
__device__ FR_INLINE inline double multisect_row(double gb, int r, int j, F&& count_is_n, double* lo_out) {
  double lo = 0.0, hi = fmin(gb, 1.0) * (1.0 + 1e-12) + 1e-300;
  const double frac = (double)(j + 1) / 17.0;
  bool done = false;
#pragma unroll 1
  for (int round = 0; round < 6; ++round) {
    // a row stops refining once its bracket is below 1e-8 + 2e-6 lo (the
    // midpoint then errs by under 5e-9 + 1e-6 of the value, far inside
    // the parity bound) or after round 6 (1 / 17^6); so its result depends
    // on its own problem only.  The wave stops when every row has.
    done = done || (hi - lo) <= 1e-8 + 2e-6 * lo;
    if (__ballot(!done) == 0ull) break;
    const double x = lo + (hi - lo) * frac;
    const uint64_t bal = __ballot(count_is_n(x));
    const uint32_t rb = (uint32_t)(bal >> (16 * r)) & 0xffffu;
    if (done) {
    } else if (rb == 0u) {
      lo = lo + (hi - lo) * ((double)16 / 17.0);
    } else {
      const int t = __ffs(rb) - 1;
      const double xt = lo + (hi - lo) * ((double)(t + 1) / 17.0);
      const double xp = t > 0 ? lo + (hi - lo) * ((double)t / 17.0) : lo;
      hi = xt;
      lo = xp;
    }
  }
  if (lo_out) *lo_out = lo;
  return 0.5 * (lo + hi);
}

// The MCC of the row's problem: the spectral radius of its tridiagonal.
// First the multisection on the largest eigenvalue alone (one Sturm
// sequence a probe); when no eigenvalue lies below minus the lower end of
// its final bracket, the largest eigenvalue is the radius and every probe
// gave what the two-sided count of [-x, x) gives (a probe above the largest
// eigenvalue is above minus the smallest), so the result is the two-sided
// search's.  Otherwise the two-sided search runs (for the whole wave; a row
// keeps the result of the search its own problem calls for).
template <int N>
__device__ FR_INLINE inline double radius_row(const double (&D)[N], const double (&E2)[N], int n, double gb, int r,
                                              int j) {
  double lo = 0.0;
  double m = multisect_row(gb, r, j, [&](double x) FR_INLINE { return sturm_row<N, 1>(D, E2, n, x) == n; }, &lo);
  const bool ok = sturm_row<N, 2>(D, E2, n, lo) == 0;
  if (__ballot(!ok) != 0ull) {
    const double m2 =
        multisect_row(gb, r, j, [&](double x) FR_INLINE { return sturm_row<N, 3>(D, E2, n, x) == n; }, nullptr);
    if (!ok) m = m2;
  }
  return m;
}

// Eight rows of a Householder step (rows 8b .. 8b + 7 of B) with the row
// broadcast fused into the FMA: v_fmac_f64 with a
// row_newbcast operand, one instruction per product where the compiler
// emits a DPP move and an FMA.  H: the rows are lanes 8..15 of their 16-row
// copy instead of 0..7.  mv8 adds col[t] * v_{8b+t} to pp[t & 3]; up8
// subtracts q_{8b+t} v + v_{8b+t} q from col[t] (in that order, the
// rounding of the two-FMA form).  The leading s_nop 4 covers the DPP read
// hazards after a VALU write of the broadcast source (2 wait states) or of
// EXEC (5).
#define FR_MV(L, A, C) "v_fmac_f64_dpp " A ", %4, " C " row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t"
template <bool H>
__device__ FR_INLINE inline void mv8(double (&pp)[4], double vr, const double* c) {
  if constexpr (!H)
    asm volatile("s_nop 4\n\t" FR_MV(0, "%0", "%5") FR_MV(1, "%1", "%6") FR_MV(2, "%2", "%7") FR_MV(3, "%3", "%8")
                 FR_MV(4, "%0", "%9") FR_MV(5, "%1", "%10") FR_MV(6, "%2", "%11") FR_MV(7, "%3", "%12")
                 : "+v"(pp[0]), "+v"(pp[1]), "+v"(pp[2]), "+v"(pp[3])
                 : "v"(vr), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]), "v"(c[7]));
  else
    asm volatile("s_nop 4\n\t" FR_MV(8, "%0", "%5") FR_MV(9, "%1", "%6") FR_MV(10, "%2", "%7") FR_MV(11, "%3", "%8")
                 FR_MV(12, "%0", "%9") FR_MV(13, "%1", "%10") FR_MV(14, "%2", "%11") FR_MV(15, "%3", "%12")
                 : "+v"(pp[0]), "+v"(pp[1]), "+v"(pp[2]), "+v"(pp[3])
                 : "v"(vr), "v"(c[0]), "v"(c[1]), "v"(c[2]), "v"(c[3]), "v"(c[4]), "v"(c[5]), "v"(c[6]), "v"(c[7]));
}
#undef FR_MV
// c[t] += bq_t (-v) + bv_t (-q) for the eight rows, in that order.
#define FR_UP(L, C) "v_fmac_f64_dpp " C ", %9, %10 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t" \
                    "v_fmac_f64_dpp " C ", %8, %11 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t"
template <bool H>
__device__ FR_INLINE inline void up8(double* c, double vr, double qr, double nv, double nq) {
  if constexpr (!H)
    asm volatile("s_nop 4\n\t" FR_UP(0, "%0") FR_UP(1, "%1") FR_UP(2, "%2") FR_UP(3, "%3") FR_UP(4, "%4")
                 FR_UP(5, "%5") FR_UP(6, "%6") FR_UP(7, "%7")
                 : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4]), "+v"(c[5]), "+v"(c[6]), "+v"(c[7])
                 : "v"(vr), "v"(qr), "v"(nv), "v"(nq));
  else
    asm volatile("s_nop 4\n\t" FR_UP(8, "%0") FR_UP(9, "%1") FR_UP(10, "%2") FR_UP(11, "%3") FR_UP(12, "%4")
                 FR_UP(13, "%5") FR_UP(14, "%6") FR_UP(15, "%7")
                 : "+v"(c[0]), "+v"(c[1]), "+v"(c[2]), "+v"(c[3]), "+v"(c[4]), "+v"(c[5]), "+v"(c[6]), "+v"(c[7])
                 : "v"(vr), "v"(qr), "v"(nv), "v"(nq));
}
#undef FR_UP
// The same for two columns per lane (cA, cB: columns j and j + 16 of a
// 17..32-level problem in a 16-lane row), each broadcast feeding both.
#define FR_MV2(L, A, B, CA, CB)                                                    \
  "v_fmac_f64_dpp " A ", %4, " CA " row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t" \
  "v_fmac_f64_dpp " B ", %4, " CB " row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t"
#define FR_MV2_ALL(L0, L1, L2, L3, L4, L5, L6, L7)                                              \
  "s_nop 4\n\t" FR_MV2(L0, "%0", "%2", "%5", "%13") FR_MV2(L1, "%1", "%3", "%6", "%14")           \
      FR_MV2(L2, "%0", "%2", "%7", "%15") FR_MV2(L3, "%1", "%3", "%8", "%16")                      \
          FR_MV2(L4, "%0", "%2", "%9", "%17") FR_MV2(L5, "%1", "%3", "%10", "%18")                 \
              FR_MV2(L6, "%0", "%2", "%11", "%19") FR_MV2(L7, "%1", "%3", "%12", "%20")
template <bool H>
__device__ FR_INLINE inline void mv8w(double (&pA)[2], double (&pB)[2], double vsrc, const double* cA,
                                      const double* cB) {
  if constexpr (!H)
    asm volatile(FR_MV2_ALL(0, 1, 2, 3, 4, 5, 6, 7)
                 : "+v"(pA[0]), "+v"(pA[1]), "+v"(pB[0]), "+v"(pB[1])
                 : "v"(vsrc), "v"(cA[0]), "v"(cA[1]), "v"(cA[2]), "v"(cA[3]), "v"(cA[4]), "v"(cA[5]), "v"(cA[6]),
                   "v"(cA[7]), "v"(cB[0]), "v"(cB[1]), "v"(cB[2]), "v"(cB[3]), "v"(cB[4]), "v"(cB[5]), "v"(cB[6]),
                   "v"(cB[7]));
  else
    asm volatile(FR_MV2_ALL(8, 9, 10, 11, 12, 13, 14, 15)
                 : "+v"(pA[0]), "+v"(pA[1]), "+v"(pB[0]), "+v"(pB[1])
                 : "v"(vsrc), "v"(cA[0]), "v"(cA[1]), "v"(cA[2]), "v"(cA[3]), "v"(cA[4]), "v"(cA[5]), "v"(cA[6]),
                   "v"(cA[7]), "v"(cB[0]), "v"(cB[1]), "v"(cB[2]), "v"(cB[3]), "v"(cB[4]), "v"(cB[5]), "v"(cB[6]),
                   "v"(cB[7]));
}
#undef FR_MV2_ALL
#undef FR_MV2
// cA[t] += q_i (-vA) + v_i (-qA), cB[t] += q_i (-vB) + v_i (-qB), i the
// row of t; %16 / %17: v and q sources, %18..%21: -vA, -vB, -qA, -qB.
#define FR_UP2(L, CA, CB)                                                            \
  "v_fmac_f64_dpp " CA ", %17, %18 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t" \
  "v_fmac_f64_dpp " CB ", %17, %19 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t" \
  "v_fmac_f64_dpp " CA ", %16, %20 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t" \
  "v_fmac_f64_dpp " CB ", %16, %21 row_newbcast:" #L " row_mask:0xf bank_mask:0xf\n\t"
#define FR_UP2_ALL(L0, L1, L2, L3, L4, L5, L6, L7)                                                   \
  "s_nop 4\n\t" FR_UP2(L0, "%0", "%8") FR_UP2(L1, "%1", "%9") FR_UP2(L2, "%2", "%10") FR_UP2(L3, "%3", "%11") \
      FR_UP2(L4, "%4", "%12") FR_UP2(L5, "%5", "%13") FR_UP2(L6, "%6", "%14") FR_UP2(L7, "%7", "%15")
template <bool H>
__device__ FR_INLINE inline void up8w(double* cA, double* cB, double vsrc, double qsrc, double nvA, double nvB,
                                      double nqA, double nqB) {
  if constexpr (!H)
    asm volatile(FR_UP2_ALL(0, 1, 2, 3, 4, 5, 6, 7)
                 : "+v"(cA[0]), "+v"(cA[1]), "+v"(cA[2]), "+v"(cA[3]), "+v"(cA[4]), "+v"(cA[5]), "+v"(cA[6]),
                   "+v"(cA[7]), "+v"(cB[0]), "+v"(cB[1]), "+v"(cB[2]), "+v"(cB[3]), "+v"(cB[4]), "+v"(cB[5]),
                   "+v"(cB[6]), "+v"(cB[7])
                 : "v"(vsrc), "v"(qsrc), "v"(nvA), "v"(nvB), "v"(nqA), "v"(nqB));
  else
    asm volatile(FR_UP2_ALL(8, 9, 10, 11, 12, 13, 14, 15)
                 : "+v"(cA[0]), "+v"(cA[1]), "+v"(cA[2]), "+v"(cA[3]), "+v"(cA[4]), "+v"(cA[5]), "+v"(cA[6]),
                   "+v"(cA[7]), "+v"(cB[0]), "+v"(cB[1]), "+v"(cB[2]), "+v"(cB[3]), "+v"(cB[4]), "+v"(cB[5]),
                   "+v"(cB[6]), "+v"(cB[7])
                 : "v"(vsrc), "v"(qsrc), "v"(nvA), "v"(nvB), "v"(nqA), "v"(nqB));
}
#undef FR_UP2_ALL
#undef FR_UP2

// MCC (spectral radius of B = D^-1/2 P D^-1/2 - v v^T over the present
// levels) of up to four stashed problems with n <= 16, row r taking the
// r-th slot of mask: Householder tridiagonalisation with one column per
// lane, then the row's Sturm multisection; row r writes its value to dst.
template <typename P>
__device__ FR_INLINE inline void mcc_narrow(const P* slots, unsigned mask) {
  const int lane = opaque_lane(), r = lane >> 4, j = lane & 15;
  const int slot = row_slot(mask, r);
  const P& q = slots[slot >= 0 ? slot : 0];
  const int n = slot >= 0 ? q.n : 0;
  const bool lok = j < n;
  const int tj = j * (j + 1) / 2;
  uint32_t gc[16];  // column j of the counts
  uint32_t rowc = 0;
  static_for<0, 16>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    const int e = a <= j ? tj + a : a * (a + 1) / 2 + j;  // in the slot for any a, j
    gc[a] = (a < n && lok) ? (uint32_t)q.g[e] : 0u;
    rowc += gc[a];
  });
  const double rtb = sqrt((double)rowc), irtb = lok ? 1.0 / rtb : 0.0;
  const double invN = 1.0 / rsum((double)rowc);  // N_P
  double col[16];
  static_for<0, 16>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    const double rta = rbc<a>(rtb), irta = rbc<a>(irtb);
    col[a] = (a < n && lok) ? (double)gc[a] * (irta * irtb) - rta * rtb * invN : 0.0;
  });
  double e_lane = 0.0;
  // steps past the wave's largest n - 2 change nothing in any row: skipped
  const int kend = (int)wmaxu((unsigned)n) - 1;
  static_for<0, 14>([&](auto kc) FR_INLINE {
    constexpr int k = decltype(kc)::value;
    if (k >= kend) return;
    const double xi = (j > k && j < n) ? col[k] : 0.0;
    const double a2 = rsum(xi * xi);
    const double x0 = rbc<k + 1>(xi);
    const double alpha = a2 == 0.0 ? 0.0 : (x0 >= 0.0 ? -sqrt(a2) : sqrt(a2));
    const double beta = a2 == 0.0 ? 0.0 : 1.0 / (a2 - x0 * alpha);  // 2 / v.v
    const double vi = j == k + 1 ? x0 - alpha : xi;
    double pj = 0.0;
    static_for<k + 1, 16>([&](auto ic) FR_INLINE {
      constexpr int i = decltype(ic)::value;
      pj += col[i] * rbc<i>(vi);
    });
    pj *= beta;  // p = beta T v
    const double Kc = 0.5 * beta * rsum(vi * pj);
    const double qj = pj - Kc * vi;
    if (j > k) {  // T -= v q^T + q v^T
      static_for<k + 1, 16>([&](auto ic) FR_INLINE {
        constexpr int i = decltype(ic)::value;
        col[i] -= rbc<i>(vi) * qj + rbc<i>(qj) * vi;
      });
    }
    if (j == k) e_lane = alpha;  // also the last step k = n - 2 (a sign flip)
  });
  double d = 0.0;
  static_for<0, 16>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    if (j == i) d = col[i];
  });
  if (n == 16 && j == 14) e_lane = col[15];  // last sub-diagonal entry (step 14 not run)
  const double dl = lok ? d : 0.0;
  const double el = j < n - 1 ? e_lane : 0.0;
  const double em = __longlong_as_double(dpp64<0x111>(__double_as_longlong(el)));  // e_{j-1}
  const double gb = rmax(lok ? fabs(dl) + fabs(el) + (j >= 1 ? fabs(em) : 0.0) : 0.0);
  const double e2l = el * el;
  double Db[16], Eb[16];  // the row's d_i and e_i^2, in every lane of the row
  static_for<0, 16>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    Db[i] = rbc<i>(dl);
    Eb[i] = rbc<i>(e2l);
  });
  // the two-sided search directly: with at most 16 levels the smallest
  // eigenvalue dominates often enough that searching the largest first
  // costs more than it saves (measured)
  const double mcc =
      multisect_row(gb, r, j, [&](double x) FR_INLINE { return sturm_row<16, 3>(Db, Eb, n, x) == n; }, nullptr);
  if (j == 0 && slot >= 0) *q.dst = (float)mcc;
}

// The same for problems with 17 <= n <= 32: lane j of row r holds columns
// j (cA) and j + 16 (cB) of its problem.
__device__ FR_INLINE inline void mcc_wide(const McProblem* slots, unsigned mask) {
  const int lane = opaque_lane(), r = lane >> 4, j = lane & 15, jb = j + 16;
  const int slot = row_slot(mask, r);
  const McProblem& q = slots[slot >= 0 ? slot : 0];
  const int n = slot >= 0 ? q.n : 0;
  const bool okA = j < n, okB = jb < n;
  const int tA = j * (j + 1) / 2, tB = jb * (jb + 1) / 2;
  uint32_t gcA[32], gcB[32];  // columns j and j + 16 of the counts
  uint32_t rcA = 0, rcB = 0;
  static_for<0, 32>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    const int eA = a <= j ? tA + a : a * (a + 1) / 2 + j;  // in the slot for any a, j
    const int eB = a <= jb ? tB + a : a * (a + 1) / 2 + jb;
    gcA[a] = (a < n && okA) ? (uint32_t)q.g[eA] : 0u;
    gcB[a] = (a < n && okB) ? (uint32_t)q.g[eB] : 0u;
    rcA += gcA[a];
    rcB += gcB[a];
  });
  const double rtA = sqrt((double)rcA), irtA = okA ? 1.0 / rtA : 0.0;
  const double rtB = sqrt((double)rcB), irtB = okB ? 1.0 / rtB : 0.0;
  const double invN = 1.0 / rsum((double)rcA + (double)rcB);  // N_P
  double cA[32], cB[32];
  static_for<0, 32>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    const double rta = a < 16 ? rbc<a & 15>(rtA) : rbc<a & 15>(rtB);
    const double irta = a < 16 ? rbc<a & 15>(irtA) : rbc<a & 15>(irtB);
    cA[a] = (a < n && okA) ? (double)gcA[a] * (irta * irtA) - rta * rtA * invN : 0.0;
    cB[a] = (a < n && okB) ? (double)gcB[a] * (irta * irtB) - rta * rtB * invN : 0.0;
  });
  double eA = 0.0, eB = 0.0;
  // steps k = 0 .. nmax - 2 (a step past a problem's own n - 2 changes
  // nothing in it); runtime loops over four groups of steps, each group's
  // body covering the rows from its first step on (rows <= k get v_i = 0
  // and q_i = 0, so they are unchanged) -- a quarter of the code of a full
  // unroll
  const int nmax = (int)wmaxu((unsigned)n);
  const int kend = nmax - 1;
  auto steps = [&](auto k0c, auto k1c) FR_INLINE {
    constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
#pragma unroll 1
    for (int k = K0; k < K1 && k < kend; ++k) {
      double ckA = 0.0, ckB = 0.0;  // row k of the lane's columns
      static_for<K0, K1>([&](auto cc) FR_INLINE {
        constexpr int c = decltype(cc)::value;
        if (k == c) {
          ckA = cA[c];
          ckB = cB[c];
        }
      });
      // column k below the diagonal; by symmetry B[i][k] = cA[k] of lane i
      const double xA = (j > k && j < n) ? ckA : 0.0;
      const double xB = (jb > k && jb < n) ? ckB : 0.0;
      const double a2 = rsum(xA * xA + xB * xB);
      const double x0 = rsum((j == k + 1 ? xA : 0.0) + (jb == k + 1 ? xB : 0.0));
      const double alpha = a2 == 0.0 ? 0.0 : (x0 >= 0.0 ? -sqrt(a2) : sqrt(a2));
      const double beta = a2 == 0.0 ? 0.0 : 1.0 / (a2 - x0 * alpha);  // 2 / v.v
      const double vA = j == k + 1 ? x0 - alpha : xA;
      const double vB = jb == k + 1 ? x0 - alpha : xB;
      // rows from K0 + 1 on, in blocks of eight behind one uniform branch
      // each (block b only if 8 b < nmax: rows past every problem's n hold
      // zeros); two partial sums per column for latency
      double pA2[2] = {0.0, 0.0}, pB2[2] = {0.0, 0.0};
      static_for<(K0 + 1) / 8, 4>([&](auto bc) FR_INLINE {
        constexpr int b = decltype(bc)::value;
        if (8 * b < nmax) {
          if constexpr (8 * b >= K0 + 1) {
            mv8w<(b & 1) != 0>(pA2, pB2, b < 2 ? vA : vB, &cA[8 * b], &cB[8 * b]);
          } else {
            static_for<K0 + 1, 8 * b + 8>([&](auto ic) FR_INLINE {
              constexpr int i = decltype(ic)::value;
              const double vi = i < 16 ? rbc<i & 15>(vA) : rbc<i & 15>(vB);
              pA2[i & 1] = fma(cA[i], vi, pA2[i & 1]);
              pB2[i & 1] = fma(cB[i], vi, pB2[i & 1]);
            });
          }
        }
      });
      const double pA = (pA2[0] + pA2[1]) * beta;  // p = beta T v
      const double pB = (pB2[0] + pB2[1]) * beta;
      const double Kc = 0.5 * beta * rsum(vA * pA + vB * pB);
      // q = p - K v on the trailing columns, 0 on the finished ones (whose
      // v is 0 too), so the update leaves those unchanged
      const double qA = j > k ? pA - Kc * vA : 0.0, qB = jb > k ? pB - Kc * vB : 0.0;
      const double nvA = -vA, nvB = -vB, nqA = -qA, nqB = -qB;
      static_for<(K0 + 1) / 8, 4>([&](auto bc) FR_INLINE {  // T -= v q^T + q v^T
        constexpr int b = decltype(bc)::value;
        if (8 * b < nmax) {
          if constexpr (8 * b >= K0 + 1) {
            up8w<(b & 1) != 0>(&cA[8 * b], &cB[8 * b], b < 2 ? vA : vB, b < 2 ? qA : qB, nvA, nvB, nqA, nqB);
          } else {
            static_for<K0 + 1, 8 * b + 8>([&](auto ic) FR_INLINE {
              constexpr int i = decltype(ic)::value;
              const double vi = i < 16 ? rbc<i & 15>(vA) : rbc<i & 15>(vB);
              const double qi = i < 16 ? rbc<i & 15>(qA) : rbc<i & 15>(qB);
              cA[i] = fma(-vi, qA, fma(-qi, vA, cA[i]));
              cB[i] = fma(-vi, qB, fma(-qi, vB, cB[i]));
            });
          }
        }
      });
      if (j == k) eA = alpha;  // also the last step k = n - 2 (a sign flip)
      if (jb == k) eB = alpha;
    }
  };
  steps(std::integral_constant<int, 0>{}, std::integral_constant<int, 8>{});
  steps(std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
  steps(std::integral_constant<int, 16>{}, std::integral_constant<int, 24>{});
  steps(std::integral_constant<int, 24>{}, std::integral_constant<int, 30>{});
  double dA = 0.0, dB = 0.0;
  static_for<0, 32>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    if (j == i) dA = cA[i];
    if (jb == i) dB = cB[i];
  });
  if (n == 32 && j == 14) eB = cB[31];  // last sub-diagonal entry (step 30 not run)
  const double dlA = okA ? dA : 0.0, dlB = okB ? dB : 0.0;
  const double elA = j < n - 1 ? eA : 0.0, elB = jb < n - 1 ? eB : 0.0;
  // e_{j-1} and e_{j+15}: lane 0 of the B half takes e_15 from lane 15 of A
  const double emA = __longlong_as_double(dpp64<0x111>(__double_as_longlong(elA)));
  double emB = __longlong_as_double(dpp64<0x111>(__double_as_longlong(elB)));
  const double e15 = rbc<15>(elA);
  if (j == 0) emB = e15;
  const double gA = okA ? fabs(dlA) + fabs(elA) + (j >= 1 ? fabs(emA) : 0.0) : 0.0;
  const double gB = okB ? fabs(dlB) + fabs(elB) + fabs(emB) : 0.0;
  const double gb = rmax(fmax(gA, gB));
  const double e2A = elA * elA, e2B = elB * elB;
  double Db[32], Eb[32];  // the row's d_i and e_i^2, in every lane of the row
  static_for<0, 16>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    Db[i] = rbc<i>(dlA);
    Eb[i] = rbc<i>(e2A);
    Db[i + 16] = rbc<i>(dlB);
    Eb[i + 16] = rbc<i>(e2B);
  });
  const double mcc = radius_row<32>(Db, Eb, n, gb, r, j);
  if (j == 0 && slot >= 0) *q.dst = (float)mcc;
}


// MCC of the pending problem with 33 <= n <= 64 present levels (64-level
// instances), straight from the GLCM still in LDS: one problem per wave,
// lane j holding column j of B in registers.  Each step stages v (then q)
// in LDS and reads it back so that lane n of every 16-lane row holds
// v_n, v_{16+n}, v_{32+n}, v_{48+n}; a row broadcast of lane i & 15 of copy
// i >> 4 then gives v_i to every lane, fused into the FMA that uses it
// (mv8, up8; a single 64-bit DPP move on the partial blocks).  Householder
// steps in runtime loops over groups of eight (each group's body covers the
// rows from its first step on; rows <= k get v_i = q_i = 0 and stay
// unchanged), then 4 rounds of 65-way Sturm multisection on the tridiagonal
// form (width <= 1 / 65^4).
template <int R, int LMAX, bool MOUT>
__device__ FR_INLINE inline void mcc_big(Smem<R, LMAX, MOUT>& sm) {
  const int lane = opaque_lane();
  const int n = __builtin_amdgcn_readfirstlane(sm.u.b.big_n);
  const bool ok = lane < n;
  const int plj = ok ? sm.u.b.pl[lane] : 0;
  const uint32_t rowc = ok ? sm.pxc[plj] : 0u;  // GLCM row sum of present level j
  const double rtj = sqrt((double)rowc), irtj = ok ? 1.0 / rtj : 0.0;
  const double invN = 1.0 / wsum((double)rowc);  // N_P
  // rt and 1/rt are 0 past n, so every entry outside n x n is 0 without a
  // select (and the code stays free of branches)
  uint32_t gv[64];  // column j of the counts: all LDS reads issued first
  static_for<0, 64>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    gv[a] = gsym(sm.u.a.glcm, __builtin_amdgcn_readlane(plj, a), plj);
  });
  __builtin_amdgcn_sched_barrier(0);
  double col[64];
  static_for<0, 64>([&](auto ac) FR_INLINE {
    constexpr int a = decltype(ac)::value;
    const double rta = readlane_d(rtj, a), irta = readlane_d(irtj, a);
    col[a] = (double)gv[a] * (irta * irtj) - rta * rtj * invN;
  });
  double e_lane = 0.0;
  double* hv = sm.u.b.d;  // staging of v and q (the tridiagonal form comes later)
  double* hq = sm.u.b.e2;
  const int ln = lane & 15;
  const int kend = n - 1 < 62 ? n - 1 : 62;  // steps k <= n - 2 (k = 62 is not needed)
  auto steps = [&](auto k0c, auto k1c) FR_INLINE {
    constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
#pragma unroll 1
    for (int k = K0; k < K1 && k < kend; ++k) {
      double ck = 0.0;  // row k of the lane's column
      static_for<K0, K1>([&](auto cc) FR_INLINE {
        constexpr int c = decltype(cc)::value;
        ck = k == c ? col[c] : ck;
      });
      // column k below the diagonal; by symmetry B[i][k] = col[k] of lane i
      const double x = lane > k ? ck : 0.0;
      const double a2 = wsum(x * x);
      const double x0 = readlane_d(x, k + 1);
      const double alpha = a2 == 0.0 ? 0.0 : (x0 >= 0.0 ? -sqrt(a2) : sqrt(a2));
      const double beta = a2 == 0.0 ? 0.0 : 1.0 / (a2 - x0 * alpha);  // 2 / v.v
      const double v = lane == k + 1 ? x0 - alpha : x;
      double vr[4];  // vr[m] = v_{16 m + n} in lane n of every row
      hv[lane] = v;
      __syncthreads();
      static_for<0, 4>([&](auto mc) FR_INLINE { vr[decltype(mc)::value] = hv[16 * decltype(mc)::value + ln]; });
      // rows from K0 + 1 on, in blocks of eight behind one uniform branch
      // each (block b only if 8 b < n); rows past n inside a block hold
      // zeros and have v_i = q_i = 0.  Four independent sums for latency.
      double pp[4] = {0.0, 0.0, 0.0, 0.0};
      static_for<(K0 + 1) / 8, 8>([&](auto bc) FR_INLINE {
        constexpr int b = decltype(bc)::value;
        if (8 * b < n) {
          if constexpr (8 * b >= K0 + 1) {
            mv8<(b & 1) != 0>(pp, vr[b >> 1], &col[8 * b]);
          } else {
            static_for<K0 + 1, 8 * b + 8>([&](auto ic) FR_INLINE {
              constexpr int i = decltype(ic)::value;
              pp[i & 3] = fma(col[i], rbc<i & 15>(vr[i >> 4]), pp[i & 3]);
            });
          }
        }
      });
      double p = (pp[0] + pp[1]) + (pp[2] + pp[3]);
      p *= beta;  // p = beta T v
      const double Kc = 0.5 * beta * wsum(v * p);
      const double q = lane > k ? p - Kc * v : 0.0;
      double qr[4];  // the same copies of q
      hq[lane] = q;
      __syncthreads();
      static_for<0, 4>([&](auto mc) FR_INLINE { qr[decltype(mc)::value] = hq[16 * decltype(mc)::value + ln]; });
      const double nv = -v, nq = -q;
      static_for<(K0 + 1) / 8, 8>([&](auto bc) FR_INLINE {  // T -= v q^T + q v^T
        constexpr int b = decltype(bc)::value;
        if (8 * b < n) {
          if constexpr (8 * b >= K0 + 1) {
            up8<(b & 1) != 0>(&col[8 * b], vr[b >> 1], qr[b >> 1], nv, nq);
          } else {
            static_for<K0 + 1, 8 * b + 8>([&](auto ic) FR_INLINE {
              constexpr int i = decltype(ic)::value;
              col[i] = fma(-rbc<i & 15>(vr[i >> 4]), q, fma(-rbc<i & 15>(qr[i >> 4]), v, col[i]));
            });
          }
        }
      });
      if (lane == k) e_lane = alpha;  // also the last step k = n - 2 (a sign flip)
    }
  };
  steps(std::integral_constant<int, 0>{}, std::integral_constant<int, 8>{});
  steps(std::integral_constant<int, 8>{}, std::integral_constant<int, 16>{});
  steps(std::integral_constant<int, 16>{}, std::integral_constant<int, 24>{});
  steps(std::integral_constant<int, 24>{}, std::integral_constant<int, 32>{});
  steps(std::integral_constant<int, 32>{}, std::integral_constant<int, 40>{});
  steps(std::integral_constant<int, 40>{}, std::integral_constant<int, 48>{});
  steps(std::integral_constant<int, 48>{}, std::integral_constant<int, 56>{});
  steps(std::integral_constant<int, 56>{}, std::integral_constant<int, 62>{});
  double d = 0.0;
  static_for<0, 64>([&](auto ic) FR_INLINE {
    constexpr int i = decltype(ic)::value;
    if (lane == i) d = col[i];
  });
  if (n == 64 && lane == 62) e_lane = col[63];  // last sub-diagonal entry (step 62 not run)
  const double dl = ok ? d : 0.0;
  const double el = lane < n - 1 ? e_lane : 0.0;
  const double em = __shfl_up(el, 1);  // e_{lane-1}
  const double gb = wmaxd_nonneg(ok ? fabs(dl) + fabs(el) + (lane >= 1 ? fabs(em) : 0.0) : 0.0);
  __syncthreads();  // the last step's reads of hv and hq are done
  if (ok) {
    sm.u.b.d[lane] = dl;
    sm.u.b.e2[lane] = el * el;
  }
  __syncthreads();
  // the spectrum of B lies in [-1, 1]; the largest eigenvalue alone first,
  // the two-sided count only when the smallest may be the larger in size
  // (as radius_row)
  const double hi0 = fmin(gb, 1.0) * (1.0 + 1e-12) + 1e-300;
  const double frac = (double)(lane + 1) / 65.0;
  auto search = [&](auto seqc, double& lo, double& hi) FR_INLINE {
    constexpr int SEQ = decltype(seqc)::value;
    lo = 0.0;
    hi = hi0;
#pragma unroll 1
    for (int round = 0; round < 4; ++round) {
      const double xr = lo + (hi - lo) * frac;
      const uint64_t bal = __ballot(sturm_span_r<SEQ>(sm.u.b.d, sm.u.b.e2, n, xr) == n);
      if (bal == 0ull) {
        lo = readlane_d(xr, 63);
      } else {
        const int t = __ffsll((unsigned long long)bal) - 1;
        const double xt = readlane_d(xr, t);
        const double xp = t > 0 ? readlane_d(xr, t - 1) : lo;
        hi = xt;
        lo = xp;
      }
    }
  };
  double lo, hi;
  search(std::integral_constant<int, 1>{}, lo, hi);
  if (sturm_span_r<2>(sm.u.b.d, sm.u.b.e2, n, lo) != 0) search(std::integral_constant<int, 3>{}, lo, hi);
  if (lane == 0) *sm.u.b.big_dst = (float)(0.5 * (lo + hi));
}

// Computes the pending MCC problems: the one with more than 32 levels (if
// big), the first ns problems of the small pool and the first nq of the
// large pool (a large slot with <= 16 levels goes to the one-column pass).
// Which routine takes a problem depends only on its n, so a result does
// not depend on the other problems of the flush.
template <int R, int LMAX, bool MOUT>
__device__ FR_INLINE inline void mcc_flush(Smem<R, LMAX, MOUT>& sm, int ns, int nq, bool big) {
  __syncthreads();
  if constexpr (LMAX > 32) {
    if (big) mcc_big(sm);
  }
  if constexpr (!MOUT) mcc_flush_pools(sm, ns, nq);
  __syncthreads();
}

// The LDS pools' problems of a flush (see mcc_flush).
template <int R, int LMAX>
__device__ FR_INLINE inline void mcc_flush_pools(Smem<R, LMAX, false>& sm, int ns, int nq) {
  if constexpr (kSmallSlots<R, LMAX> > 0) {
    if (ns) mcc_narrow(sm.ms.s, (1u << ns) - 1u);
  }
  if (nq) {
    unsigned narrow = 0u, wide = 0u;
    for (int s = 0; s < nq; ++s) {
      if (sm.mq.s[s].n <= 16)
        narrow |= 1u << s;
      else
        wide |= 1u << s;
    }
    if constexpr (kSmallSlots<R, LMAX> == 0) {
      if (narrow) mcc_narrow(sm.mq.s, narrow);
    }
    if (wide) mcc_wide(sm.mq.s, wide);
  }
}

// Bitonic sort of 64 NPL values held in registers, the NIN values of each
// lane's `in` first (+inf beyond; +inf sorts last), element e = lane * NPL
// + r: stages whose partner is in the same lane are register
// compare-exchanges, the others exchange with lane ^ (j / NPL).  No
// barriers.  Writes the first NOUT of the sorted values to srt.
// x of lane (lane ^ M), M a power of two below 64, without the LDS
// crossbar: DPP quad permutes (1, 2), row rotates (4: by 4 or 12 depending
// on lane bit 2; 8), and the gfx950 row / half swaps (16, 32).
template <int M>
__device__ inline float xor_lane(float x, int lane) {
  const int b = __float_as_int(x);
  if constexpr (M == 1) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0xb1, 0xf, 0xf, false));
  } else if constexpr (M == 2) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x4e, 0xf, 0xf, false));
  } else if constexpr (M == 4) {
    const int r4 = __builtin_amdgcn_mov_dpp(b, 0x124, 0xf, 0xf, false);   // row_ror:4 (lane - 4)
    const int r12 = __builtin_amdgcn_mov_dpp(b, 0x12c, 0xf, 0xf, false);  // row_ror:12 (lane + 4)
    return __int_as_float((lane & 4) ? r4 : r12);
  } else if constexpr (M == 8) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(b, 0x128, 0xf, 0xf, false));  // row_ror:8
  } else if constexpr (M == 16) {
    // swapping a register with itself: the odd rows find the partner in the
    // first result, the even rows in the second
    const auto r = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    return __int_as_float((lane & 16) ? r[0] : r[1]);
  } else {
    static_assert(M == 32, "xor_lane: M in 1..32");
    const auto r = __builtin_amdgcn_permlane32_swap(b, b, false, false);  // halves, likewise
    return __int_as_float((lane & 32) ? r[0] : r[1]);
  }
}

template <int NPL, int NIN, int NOUT>
__device__ inline void sort_regs(const float (&in)[NIN], float* srt, int lane) {
  constexpr int NE = 64 * NPL;
  static_assert(NE <= 512 && NIN <= NPL, "sort size");
  float v[NPL];
#pragma unroll
  for (int r = 0; r < NPL; ++r) v[r] = r < NIN ? in[r] : INFINITY;
  static_for<1, 10>([&](auto kl) FR_INLINE {  // k = 2^kl up to NE <= 512
    constexpr int k = 1 << decltype(kl)::value;
    if constexpr (k <= NE) {
    const bool up = ((lane * NPL) & k) == 0 || k < NPL;
    static_for<0, decltype(kl)::value>([&](auto jl) FR_INLINE {  // j = k / 2, k / 4, ..., 1
      constexpr int j = k >> (1 + decltype(jl)::value);
      if constexpr (j >= NPL) {
        constexpr int m = j / NPL;
        const bool keep_lo = ((lane & m) == 0) == up;
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          const float y = xor_lane<m>(v[r], lane);
          v[r] = keep_lo ? fminf(v[r], y) : fmaxf(v[r], y);
        }
      } else {
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          if (r & j) continue;
          const bool u = k < NPL ? ((r & k) == 0) : up;
          const float a = v[r], b = v[r | j];
          v[r] = u ? fminf(a, b) : fmaxf(a, b);
          v[r | j] = u ? fmaxf(a, b) : fminf(a, b);
        }
      }
    });
    }
  });
#pragma unroll
  for (int r = 0; r < NPL; ++r)
    if (lane * NPL + r < NOUT) srt[lane * NPL + r] = v[r];
}

// Run/zone/dependence emphasis features from per-entry sums.
struct Emph {
  long long n, si, si2, sj, sj2;  // totals (after emph_reduce)
  double si2j2;                   // total of c i^2 j^2, an integer below 2^53
  uint32_t pn, psi, psi2, psj, psj2;  // the lane's partial sums
  double psi2j2;
  double invj2, invi2, invi2j2, i2invj2, j2invi2, clogc;
};
// One matrix entry: count c (at most 13 (2r+1)^3 < 2^24) at level value i
// (<= 255) and index j (run length, zone size or dependence count, <= 343).
// The sums of c, c i, c i^2, c j, c j^2 stay below 2^31 (at most 13|V|
// entries, c i <= 1.2e6, c i^2 <= 2.9e8): 32-bit arithmetic, 24-bit
// multiplies.  Sum c i^2 j^2 does not (a uniform 7^3 neighbourhood at level
// 255 gives 5.9e9 for the dependence counts): it is summed in FP64, where
// every term and partial sum is an integer below 2^53, so exactly and in
// any order.
__device__ inline void emph_add(Emph& a, uint32_t c, int i, int j) {
  const double ci = (double)c;
  const uint32_t ui = (uint32_t)i, uj = (uint32_t)j;
  const uint32_t i2u = __umul24(ui, ui), j2u = __umul24(uj, uj);
  const double i2 = (double)i2u, j2 = (double)j2u;
  const double ri2 = frcp(i2), rj2 = frcp(j2);
  const uint32_t cis = __umul24(c, ui), cjs = __umul24(c, uj);
  a.pn += c;
  a.psi += cis;
  a.psi2 += __umul24(cis, ui);
  a.psj += cjs;
  a.psj2 += __umul24(cjs, uj);
  a.psi2j2 += ci * (i2 * j2);
  a.invj2 += ci * rj2;
  a.invi2 += ci * ri2;
  a.invi2j2 += ci * ri2 * rj2;
  a.i2invj2 += ci * i2 * rj2;
  a.j2invi2 += ci * j2 * ri2;
  if (c > 1) a.clogc += ci * flog2(ci);
}
// The integer sums fit in 32 bits (see emph_add); x1, x2: two more
// per-lane integer partials (squared row / column totals, each total below
// 2^31) reduced in the same pass.
__device__ inline void emph_reduce(Emph& a, long long& x1, long long& x2) {
  int vi[8] = {(int)a.pn, (int)a.psi, (int)a.psi2, (int)a.psj, (int)a.psj2, 0, (int)x1, (int)x2};
  wsum8i(vi);
  a.n = vi[0];
  a.si = vi[1];
  a.si2 = vi[2];
  a.sj = vi[3];
  a.sj2 = vi[4];
  x1 = vi[6];
  x2 = vi[7];
  double vd[8] = {a.invj2, a.invi2, a.invi2j2, a.i2invj2, a.j2invi2, a.clogc, a.psi2j2, 0.0};
  wsum8d(vd);
  a.invj2 = vd[0];
  a.invi2 = vd[1];
  a.invi2j2 = vd[2];
  a.i2invj2 = vd[3];
  a.j2invi2 = vd[4];
  a.clogc = vd[5];
  a.si2j2 = vd[6];
}
// The 16-value set shared by GLRLM and GLSZM: gln/rln are the sums of
// squared row/column totals; units = Np (13|V| for runs) or Nv (|V|).
__device__ inline void emph16(const Emph& a, long long gln, long long rln, double units,
                              float* f) {
  const double N = (double)a.n;
  const double rN = 1.0 / N, rN2 = rN * rN;  // one division; the rest multiply
  f[0] = (float)(a.invj2 * rN);
  f[1] = (float)((double)a.sj2 * rN);
  f[2] = (float)((double)gln * rN);
  f[3] = (float)((double)gln * rN2);
  f[4] = (float)((double)rln * rN);
  f[5] = (float)((double)rln * rN2);
  f[6] = (float)(N / units);
  f[7] = (float)((double)(a.n * a.si2 - a.si * a.si) * rN2);
  f[8] = (float)((double)(a.n * a.sj2 - a.sj * a.sj) * rN2);
  f[9] = (float)(flog2(N) - a.clogc * rN);
  f[10] = (float)(a.invi2 * rN);
  f[11] = (float)((double)a.si2 * rN);
  f[12] = (float)(a.invi2j2 * rN);
  f[13] = (float)(a.i2invj2 * rN);
  f[14] = (float)(a.j2invi2 * rN);
  f[15] = (float)(a.si2j2 * rN);
}

template <typename T, int R, int LMAX, bool DEBUG, bool MOUT = false>
__device__ __attribute__((always_inline)) inline void map_voxel(Smem<R, LMAX, MOUT>& sm, const MapArgs& a, int32_t lin, int64_t it,
                                                               int& ns, int& nq, bool& big) {
  using SM = Smem<R, LMAX, MOUT>;
  constexpr int S = SM::S, C = SM::C, CP = SM::CP, SP = SM::SP, HT = SM::HT;
  constexpr int NIT = CP / 64;
  const int lane = opaque_lane();
  const T* __restrict__ vol = (const T*)a.vol;
  const uint32_t fam = a.families;
  const bool fFO = fam & 1u, fGLCM = fam & 2u, fGLRLM = fam & 4u, fGLSZM = fam & 8u,
             fGLDM = fam & 16u, fNGTDM = fam & 32u;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int cx = lin % nx, cy = (lin / nx) % ny, cz = lin / (nx * ny);

  // ---- gather the cube ------------------------------------------------
  // the raw values stay in registers (xq) until their sort; their sums for
  // the moments are taken here
  int K = 0;
  float xq[NIT];
  double s1 = 0.0, s2 = 0.0;
  // every load of the cube first (levels and raw values of the positions
  // inside the image, whatever their level), so that they are all in
  // flight together instead of one round trip per position
  int gl[NIT];
  float xl[NIT];
#pragma unroll
  for (int q = 0; q < NIT; ++q) {
    const int c = lane + 64 * q;
    gl[q] = 0;
    xl[q] = INFINITY;
    if (c < C) {
      const int x = c % S, y = (c / S) % S, z = c / (S * S);
      const int gx = cx + x - R, gy = cy + y - R, gz = cz + z - R;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
        const int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
        gl[q] = a.levels[gi];
        xl[q] = (float)vol[gi];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NIT; ++q) {
    const int c = lane + 64 * q;
    const int g = gl[q];
    const float xr = g ? xl[q] : INFINITY;
    if (g) sm.lflag[g] = 1;
    sm.cl[c] = (uint8_t)g;
    if (c < C) {
      const int x = c % S, y = (c / S) % S, z = c / (S * S);
      sm.clp[((z + 1) * SM::SQ + (y + 1)) * SM::SQ + (x + 1)] = (uint8_t)g;
    }
    xq[q] = xr;
    if (fFO && g) {
      const double xd = (double)xr;
      s1 += xd;
      s2 += xd * xd;
    }
    sm.u.a.parent[c] = (uint32_t)c;
    if (!(c & 1)) sm.u.a.zcnt[c >> 1] = 0;
    K += __popcll(__ballot(g != 0));
  }
  __syncthreads();

  // ---- local level compaction -----------------------------------------
  int L;
  {
    const uint32_t fw = lane < SM::LVW ? ((const uint32_t*)sm.lflag)[lane] : 0u;
    const int f0 = (fw & 0xffu) != 0, f1 = (fw & 0xff00u) != 0, f2 = (fw & 0xff0000u) != 0,
              f3 = (fw & 0xff000000u) != 0;
    int pre = wscan_excl(f0 + f1 + f2 + f3, lane, &L);
    if (f0) { sm.lmap[4 * lane] = (uint8_t)pre; sm.lval[pre++] = (uint8_t)(4 * lane); }
    if (f1) { sm.lmap[4 * lane + 1] = (uint8_t)pre; sm.lval[pre++] = (uint8_t)(4 * lane + 1); }
    if (f2) { sm.lmap[4 * lane + 2] = (uint8_t)pre; sm.lval[pre++] = (uint8_t)(4 * lane + 2); }
    if (f3) { sm.lmap[4 * lane + 3] = (uint8_t)pre; sm.lval[pre++] = (uint8_t)(4 * lane + 3); }
    if (lane < SM::LVW) ((uint32_t*)sm.lflag)[lane] = 0u;  // ready for the next voxel
  }
  if constexpr (C > LMAX) {
    if (L > LMAX) {  // more present levels than these tables hold: a wider pass maps it
      if (lane == 0) a.over[atomicAdd(a.over_count, 1)] = make_int2(a.over_job, (int)it);
      return;
    }
  }
  // clear the L-sized tables
  for (int e = lane; e < (L * (L + 1) / 2 + 1) / 2; e += 64) sm.u.a.glcm[e] = 0;
  for (int e = lane; e < L * S; e += 64) sm.u.a.glrlm[e] = 0;
  for (int e = lane; e < (L * 27 + 1) / 2; e += 64) sm.u.a.gldm[e] = 0;
  if (lane < L) {
    sm.hist[lane] = 0;
    sm.pxc[lane] = 0;
    sm.u.a.ngn[lane] = 0;
    sm.u.a.ngS[lane] = 0ull;
    sm.u.a.zpl[lane] = 0;
  }
  for (int e = lane; e < CP / 2; e += 64) sm.u.a.zps[e] = 0;
  for (int e = lane; e < HT; e += 64) {
    sm.u.a.hkey[e] = 0;
    if (e < HT / 2) sm.u.a.hcnt[e] = 0;
  }
  __syncthreads();

  // ---- counting pass: lane per cube position --------------------------
  // All 26 neighbour levels are loaded at once from the zero-bordered cube
  // (no bounds tests), then folded with bit arithmetic; only the GLCM
  // atomics of unequal forward pairs are predicated.
  constexpr int SQ = SM::SQ;
#pragma unroll 1
  for (int q = 0; q < NIT; ++q) {
    const int c = lane + 64 * q;
    const int g = (c < C) ? sm.cl[c] : 0;
    if (g) {
      const int x = c % S, y = (c / S) % S, z = c / (S * S);
      const uint8_t* nb = &sm.clp[((z + 1) * SQ + (y + 1)) * SQ + (x + 1)];
      int h[26];
#pragma unroll
      for (int n = 0; n < 26; ++n) h[n] = nb[(ndz(n) * SQ + ndy(n)) * SQ + ndx(n)];
      uint32_t same = 0;
      int cnt = 0, lsum = 0;
#pragma unroll
      for (int n = 0; n < 26; ++n) {
        cnt += min(h[n], 1);  // no compare: the carry chain it makes needs wait states
        lsum += h[n];
        same |= (uint32_t)(h[n] == g) << n;
      }
      const int l = sm.lmap[g];
      sm.u.a.same[c] = same;
      if (fGLSZM) {  // first zone label: the smallest equal-level neighbour index
        // (neighbours 13..25 precede c; one of another level gives ~0)
        const uint32_t nsame = ~same;
        uint32_t m0 = (uint32_t)c;
#pragma unroll
        for (int n = 13; n < 26; ++n)
          m0 = min(m0, (uint32_t)(c + (ndz(n) * S + ndy(n)) * S + ndx(n)) |
                           (uint32_t)((int32_t)(nsame << (31 - n)) >> 31));
        sm.u.a.parent[c] = m0;
      }
      atomicAdd(&sm.hist[l], 1u);
      if (fGLCM) {
        int mm[13];
#pragma unroll
        for (int n = 0; n < 13; ++n) mm[n] = sm.lmap[h[n]];
#pragma unroll
        for (int n = 0; n < 13; ++n) {
          if (h[n] != 0 && h[n] != g) {
            gadd(sm.u.a.glcm, l < mm[n] ? tri(l, mm[n]) : tri(mm[n], l), 1u);
          }
        }
        const int eq = __popc(same & 0x1FFFu);
        if (eq) gadd(sm.u.a.glcm, tri(l, l), 2u * eq);
        atomicAdd(&sm.pxc[l], (uint32_t)cnt);
      }
      if (fGLDM) gadd(sm.u.a.gldm, l * 27 + __popc(same), 1u);
      if (fNGTDM && cnt) {
        atomicAdd(&sm.u.a.ngn[l], 1u);
        const int dd = g * cnt - lsum;
        atomicAdd(&sm.u.a.ngS[l], (unsigned long long)(dd < 0 ? -dd : dd) * kLcmOver[cnt]);
      }
    }
  }
  __syncthreads();

  // ---- zones: minimum-label propagation over equal-level neighbours ----
  // label[c] starts at the smallest equal-level neighbour index (or c); each
  // pass takes the minimum over the equal-level 26-neighbours and one
  // pointer jump, and a voxel whose label drops also lowers the label of the
  // voxel it pointed to (hooking).  Labels only decrease and always name a
  // voxel of the same zone, so the fixed point (a pass that changes
  // nothing) labels every zone with its smallest cube index.
  // At radius 3 every neighbour label is read, in or out of the cube: the
  // index stays within the 32-bit counting tables around the label array
  // (the static_assert below), and a neighbour whose bit in same is clear
  // gives ~0 to the minimum (two VALU operations a neighbour, no address
  // select).
  if (fGLSZM) {
    using A = typename SM::U::A;
    constexpr int kLab = (int)(offsetof(A, parent) / 4);
    constexpr int kReach = S * S + S + 1;  // largest |neighbour index offset|
    static_assert(kLab >= kReach && offsetof(A, parent) % 4 == 0 &&
                      offsetof(A, ngS) / 4 >= (size_t)(kLab + C + kReach),
                  "the label array has 32-bit tables on both sides");
    uint32_t* lab = sm.u.a.parent;
    const uint32_t* tab = reinterpret_cast<const uint32_t*>(&sm.u.a);
    while (true) {
      bool changed = false;
#pragma unroll 1
      for (int q = 0; q < NIT; ++q) {
        const int c = lane + 64 * q;
        if (c < C && sm.cl[c]) {
          uint32_t m = lab[c];
          if constexpr (R == 3) {
            const uint32_t nsb = ~sm.u.a.same[c];
            uint32_t nl[26];
#pragma unroll
            for (int n = 0; n < 26; ++n) nl[n] = tab[kLab + c + (ndz(n) * S + ndy(n)) * S + ndx(n)];
#pragma unroll
            for (int n = 0; n < 26; ++n) m = min(m, nl[n] | (uint32_t)((int32_t)(nsb << (31 - n)) >> 31));
          } else {  // measured faster below radius 3: the read address selected
            const uint32_t sb = sm.u.a.same[c];
            uint32_t nl[26];
#pragma unroll
            for (int n = 0; n < 26; ++n)
              nl[n] = lab[(sb >> n) & 1u ? c + (ndz(n) * S + ndy(n)) * S + ndx(n) : c];
#pragma unroll
            for (int n = 0; n < 26; ++n) m = min(m, nl[n]);
          }
          m = min(m, lab[m]);
          const uint32_t cur = lab[c];
          if (m < cur) {  // atomics: a concurrent hook is never raised again
            atomicMin(&lab[c], m);
            atomicMin(&lab[cur], m);
            changed = true;
          }
        }
      }
      __syncthreads();
      if (__ballot(changed) == 0ull) break;
    }
  }

  // ---- runs and zone sizes --------------------------------------------
#pragma unroll
  for (int q = 0; q < NIT; ++q) {
    const int c = lane + 64 * q;
    const int g = (c < C) ? sm.cl[c] : 0;
    if (g) {
      const uint32_t same = sm.u.a.same[c];
      if (fGLRLM) {
        const int l = sm.lmap[g];
        // a run of direction d starts here when the backward neighbour is
        // not of this level; the runs of all 13 directions are walked
        // together, one step of each per round (13 independent LDS reads in
        // flight instead of 13 chains one after another)
        const uint32_t starts = ~(same >> 13) & 0x1FFFu;
        uint32_t act = starts & same;  // bit d: the run of direction d goes on
        // step[d]: positions walked so far; the position reached is
        // c + step[d] * (forward offset of d, positive), its byte address
        // one multiply-add.  Radius 3 only: below it, the form with a
        // position per direction measured faster.
        uint32_t step[13];
#pragma unroll
        for (int d = 0; d < 13; ++d) step[d] = 0u;
        int cc[13];
#pragma unroll
        for (int d = 0; d < 13; ++d) cc[d] = c;
        const char* sb0 = reinterpret_cast<const char*>(sm.u.a.same) + 4 * c;
        while (act) {
          uint32_t sv[13];
#pragma unroll
          for (int d = 0; d < 13; ++d) {
            const uint32_t on = (act >> d) & 1u;
            step[d] += on;
            if constexpr (R != 3) cc[d] += on ? (fdz(d) * S + fdy(d)) * S + fdx(d) : 0;
          }
#pragma unroll
          for (int d = 0; d < 13; ++d) {
            if constexpr (R == 3)
              sv[d] = *reinterpret_cast<const uint32_t*>(
                  sb0 + step[d] * (uint32_t)(4 * ((fdz(d) * S + fdy(d)) * S + fdx(d))));
            else
              sv[d] = sm.u.a.same[cc[d]];
          }
          uint32_t go = 0;
#pragma unroll
          for (int d = 0; d < 13; ++d) go |= sv[d] & (1u << d);
          act &= go;
        }
#pragma unroll
        for (int d = 0; d < 13; ++d)
          if ((starts >> d) & 1u) atomicAdd(&sm.u.a.glrlm[l * S + (int)step[d]], 1u);
      }
      if (fGLSZM) gadd(sm.u.a.zcnt, (int)sm.u.a.parent[c], 1u);
    }
  }
  // sort of the raw values for the order statistics
  if (fFO) {
    __syncthreads();
    sort_regs<SP / 64, NIT, CP>(xq, (float*)sm.u.a.same, lane);
  }
  __syncthreads();

  // ---- zones: per root ------------------------------------------------
  Emph ez = {};
  if (fGLSZM) {
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
      const int c = lane + 64 * q;
      const int g = (c < C) ? sm.cl[c] : 0;
      if (g && sm.u.a.parent[c] == (uint32_t)c) {
        const int s = (int)gget(sm.u.a.zcnt, c);
        const int l = sm.lmap[g];
        emph_add(ez, 1, g, s);  // c log2 c = 0 for c = 1; the entropy comes from the hash
        atomicAdd(&sm.u.a.zpl[l], 1u);
        gadd(sm.u.a.zps, s - 1, 1u);
        const uint32_t key = ((uint32_t)l << 16 | (uint32_t)s) + 1u;
        // multiplicative hash: the product's high bits mix level and size
        uint32_t h = (key * 2654435761u) >> (32 - __builtin_ctz((unsigned)HT));
        while (true) {
          const uint32_t old = atomicCAS(&sm.u.a.hkey[h], 0u, key);
          if (old == 0u || old == key) {
            gadd(sm.u.a.hcnt, (int)h, 1u);
            break;
          }
          h = (h + 1) & (HT - 1);
        }
        if (DEBUG) {
          const int64_t base = it * (int64_t)a.ng * C;
          atomicAdd(&a.d_glszm[base + (int64_t)(g - 1) * C + (s - 1)], 1);
        }
      }
    }
  }
  __syncthreads();

  if (DEBUG) {
    const int ng = a.ng;
    for (int e = lane; e < L * L; e += 64) {
      const int l = e / L, m = e % L;
      a.d_glcm[it * ng * ng + (int64_t)(sm.lval[l] - 1) * ng + (sm.lval[m] - 1)] = (int32_t)gsym(sm.u.a.glcm, l, m);
    }
    for (int e = lane; e < L * S; e += 64) {
      const int l = e / S, j = e % S;
      a.d_glrlm[it * ng * S + (int64_t)(sm.lval[l] - 1) * S + j] = (int32_t)sm.u.a.glrlm[e];
    }
    for (int e = lane; e < L * 27; e += 64) {
      const int l = e / 27, j = e % 27;
      a.d_gldm[it * ng * 27 + (int64_t)(sm.lval[l] - 1) * 27 + j] = (int32_t)gget(sm.u.a.gldm, e);
    }
    if (lane < L) {
      const int64_t o = it * ng + (sm.lval[lane] - 1);
      a.d_ngn[o] = (int32_t)sm.u.a.ngn[lane];
      a.d_ngS[o] = (int64_t)sm.u.a.ngS[lane];
      a.d_hist[o] = (int32_t)sm.hist[lane];
    }
  }

  // map offsets of the families in the output
  int off = 0;
  const int oFO = off;    off += fFO ? kNFO : 0;
  const int oGLCM = off;  off += fGLCM ? kNGLCM : 0;
  const int oGLRLM = off; off += fGLRLM ? kNGLRLM : 0;
  const int oGLSZM = off; off += fGLSZM ? kNGLSZM : 0;
  const int oGLDM = off;  off += fGLDM ? kNGLDM : 0;
  const int oNGTDM = off; off += fNGTDM ? kNNGTDM : 0;
  const int count = off;
  float* F = sm.feat();
  if constexpr (SM::kFeatInZcnt) {
    using U = typename SM::U;
    static_assert(offsetof(typename U::A, zcnt) >= sizeof(typename U::B) &&
                      offsetof(typename U::A, zcnt) >= sizeof(typename U::C) &&
                      sizeof(U::A::zcnt) >= 96 * sizeof(float),
                  "the maps overlay the zone sizes");
  }
  const double Kd = (double)K;

  // ---- first order ----------------------------------------------------
  if (fFO) {
    const double rKd = 1.0 / Kd;  // one division; the rest multiply
    double ent = 0.0, uni = 0.0;
    if (lane < L) {
      const double p = (double)sm.hist[lane] * rKd;
      ent = -p * flog2(p);
      uni = p * p;
    }
    double r1[8] = {s1, s2, ent, uni, 0.0, 0.0, 0.0, 0.0};
    wsum8d(r1);
    const double S1 = r1[0], S2 = r1[1];
    ent = r1[2];
    uni = r1[3];
    const double mu = S1 * rKd;
    const float* srt = (const float*)sm.u.a.same;  // sorted: the K values of V first
    const double mn = srt[0], mx = srt[K - 1];
    auto pct = [&](double qq) -> double {
      const double h = (double)(K - 1) * qq;
      const double lo = floor(h);
      const int i = (int)lo;
      const double fr = h - lo;
      if (i + 1 >= K) return (double)srt[K - 1];
      const double a0 = srt[i], a1 = srt[i + 1];
      return a0 + fr * (a1 - a0);
    };
    const double p10 = pct(0.10), p25 = pct(0.25), p50 = pct(0.50), p75 = pct(0.75),
                 p90 = pct(0.90);
    double m2 = 0, m3 = 0, m4 = 0, mad = 0, rs = 0, rn = 0;
#pragma unroll
    for (int q = 0; q < NIT; ++q) {
      const int c = lane + 64 * q;
      if (c < K) {
        const double x = srt[c];
        const double d = x - mu;
        const double d2 = d * d;
        m2 += d2;
        m3 += d2 * d;
        m4 += d2 * d2;
        mad += fabs(d);
        if (x >= p10 && x <= p90) {
          rs += x;
          rn += 1.0;
        }
      }
    }
    double r2[8] = {m2, m3, m4, mad, rs, rn, 0.0, 0.0};
    wsum8d(r2);
    m2 = r2[0] * rKd;
    m3 = r2[1] * rKd;
    m4 = r2[2] * rKd;
    mad = r2[3] * rKd;
    rs = r2[4];
    rn = r2[5];
    double rmad = NAN;
    if (rn > 0.0) {
      const double rmu = rs / rn;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < NIT; ++q) {
        const int c = lane + 64 * q;
        if (c < K) {
          const double x = srt[c];
          if (x >= p10 && x <= p90) acc += fabs(x - rmu);
        }
      }
      rmad = wsum(acc) / rn;
    }
    const bool flat = (mn == mx);
    if (lane == 0) {
      F[oFO + 0] = (float)S2;
      F[oFO + 1] = (float)(a.voxel_volume * S2);
      F[oFO + 2] = (float)ent;
      F[oFO + 3] = (float)mn;
      F[oFO + 4] = (float)p10;
      F[oFO + 5] = (float)p90;
      F[oFO + 6] = (float)mx;
      F[oFO + 7] = (float)mu;
      F[oFO + 8] = (float)p50;
      F[oFO + 9] = (float)(p75 - p25);
      F[oFO + 10] = (float)(mx - mn);
      F[oFO + 11] = (float)mad;
      F[oFO + 12] = (float)rmad;
      F[oFO + 13] = (float)sqrt(S2 * rKd);
      F[oFO + 14] = flat ? 0.f : (float)(m3 / (m2 * sqrt(m2)));  // m2^1.5
      F[oFO + 15] = flat ? 0.f : (float)(m4 / (m2 * m2) - 3.0);
      F[oFO + 16] = (float)m2;
      F[oFO + 17] = (float)uni;
    }
  }

  // ---- GLRLM ----------------------------------------------------------
  if (fGLRLM) {
    Emph er = {};
    uint32_t nzb = 0;  // bit t: entry lane + 64 t is nonzero (L*S <= 448)
    for (int t = 0; lane + 64 * t < L * S; ++t) nzb |= (sm.u.a.glrlm[lane + 64 * t] != 0u) << t;
    while (nzb) {
      const int e = lane + 64 * (__ffs(nzb) - 1);
      nzb &= nzb - 1;
      emph_add(er, sm.u.a.glrlm[e], sm.lval[e / S], e % S + 1);
    }
    long long gln = 0, rln = 0;
    if (lane < L) {
      long long t = 0;
      for (int j = 0; j < S; ++j) t += sm.u.a.glrlm[lane * S + j];
      gln = t * t;
    }
    if (lane < S) {
      long long t = 0;
      for (int l = 0; l < L; ++l) t += sm.u.a.glrlm[l * S + lane];
      rln = t * t;
    }
    emph_reduce(er, gln, rln);
    float f[16];
    emph16(er, gln, rln, 13.0 * Kd, f);
    if (lane < 16) F[oGLRLM + lane] = f[lane];
  }

  // ---- GLSZM ----------------------------------------------------------
  if (fGLSZM) {
    double hl = 0.0;
    uint32_t nzb = 0;  // bit t: slot lane + 64 t holds a key (HT <= 256)
    for (int t = 0; lane + 64 * t < HT; ++t) nzb |= (gget(sm.u.a.hcnt, lane + 64 * t) != 0u) << t;
    while (nzb) {  // only the occupied slots pay for a logarithm
      const double c = (double)gget(sm.u.a.hcnt, lane + 64 * (__ffs(nzb) - 1));
      nzb &= nzb - 1;
      hl += c * flog2(c);
    }
    ez.clogc = hl;  // zones count once each; the entropy term comes from the hash
    long long gln = 0, szn = 0;
    if (lane < L) {
      const long long t = sm.u.a.zpl[lane];
      gln = t * t;
    }
    for (int s = lane; s < C; s += 64) {
      const long long t = gget(sm.u.a.zps, s);
      szn += t * t;
    }
    emph_reduce(ez, gln, szn);
    float f[16];
    emph16(ez, gln, szn, Kd, f);
    if (lane < 16) F[oGLSZM + lane] = f[lane];
  }

  // ---- GLDM -----------------------------------------------------------
  if (fGLDM) {
    Emph ed = {};
    uint32_t nzb = 0;  // bit t: entry lane + 64 t is nonzero (L*27 <= 1728)
    for (int t = 0; lane + 64 * t < L * 27; ++t) nzb |= (gget(sm.u.a.gldm, lane + 64 * t) != 0u) << t;
    while (nzb) {
      const int e = lane + 64 * (__ffs(nzb) - 1);
      nzb &= nzb - 1;
      emph_add(ed, gget(sm.u.a.gldm, e), sm.lval[e / 27], e % 27 + 1);
    }
    long long gln = 0, dn = 0;
    if (lane < L) {
      const long long t = sm.hist[lane];
      gln = t * t;
    }
    if (lane < 27) {
      long long t = 0;
      for (int l = 0; l < L; ++l) t += gget(sm.u.a.gldm, l * 27 + lane);
      dn = t * t;
    }
    emph_reduce(ed, gln, dn);
    const double N = (double)ed.n;
    const double rN = 1.0 / N, rN2 = rN * rN;  // one division; the rest multiply
    if (lane == 0) {
      float* f = F + oGLDM;
      f[0] = (float)(ed.invj2 * rN);
      f[1] = (float)((double)ed.sj2 * rN);
      f[2] = (float)((double)gln * rN);
      f[3] = (float)((double)dn * rN);
      f[4] = (float)((double)dn * rN2);
      f[5] = (float)((double)(ed.n * ed.si2 - ed.si * ed.si) * rN2);
      f[6] = (float)((double)(ed.n * ed.sj2 - ed.sj * ed.sj) * rN2);
      f[7] = (float)(flog2(N) - ed.clogc * rN);
      f[8] = (float)(ed.invi2 * rN);
      f[9] = (float)((double)ed.si2 * rN);
      f[10] = (float)(ed.invi2j2 * rN);
      f[11] = (float)(ed.i2invj2 * rN);
      f[12] = (float)(ed.j2invi2 * rN);
      f[13] = (float)(ed.si2j2 * rN);
    }
  }

  // ---- NGTDM ----------------------------------------------------------
  if (fNGTDM) {
    long long n_i = 0, sum_n = 0, sum_ni = 0, sum_ni2 = 0, pres = 0, pj = 0, pj2 = 0;
    double s_i = 0.0, ps_acc = 0.0;
    int i_lev = 0, anys = 0;
    // s_i as a double in place of its integer numerator (no later reader of
    // the integer), so the pairwise terms read it converted once per level
    double* sd = reinterpret_cast<double*>(sm.u.a.ngS);
    if (lane < L) {
      n_i = sm.u.a.ngn[lane];
      const unsigned long long Si = sm.u.a.ngS[lane];
      i_lev = sm.lval[lane];
      s_i = (double)Si * kRcpLcm26;
      sd[lane] = s_i;
      if (n_i) {
        pres = 1;
        pj = i_lev;
        pj2 = (long long)i_lev * i_lev;
        anys = Si != 0ull;
      }
      sum_n = n_i;
      sum_ni = n_i * i_lev;
      sum_ni2 = n_i * i_lev * i_lev;
      ps_acc = (double)n_i * s_i;
    }
    // pairwise terms over present levels: both terms are symmetric in
    // (i, j) and vanish for i = j, so the pairs i < j, enumerated compactly
    // (e = j (j - 1) / 2 + i), one per lane, count twice
    long long bden = 0;
    double cplx = 0.0;
    __syncthreads();  // sd complete
    {
      const int npair = L * (L - 1) / 2;
      for (int e0 = 0; e0 < npair; e0 += 64) {
        const int e = e0 + lane;
        if (e < npair) {
          int jc = (int)((1.0f + sqrtf(8.0f * (float)e + 1.0f)) * 0.5f);
          jc += (jc + 1) * jc / 2 <= e;  // exact: largest jc with jc (jc - 1) / 2 <= e
          jc -= jc * (jc - 1) / 2 > e;
          const int i = e - jc * (jc - 1) / 2;
          // counts <= (2r+1)^3 and levels <= 255: the products fit in 32 bits
          const int ni = (int)sm.u.a.ngn[i], nj = (int)sm.u.a.ngn[jc];
          if (ni && nj) {
            const int il = sm.lval[i], jl = sm.lval[jc];
            const int t = il * ni - jl * nj;
            bden += 2 * (t < 0 ? -t : t);
            const double si = sd[i], sj = sd[jc];
            cplx += 2.0 * fabs((double)(il - jl)) * ((double)ni * si + (double)nj * sj) *
                    frcp((double)(ni + nj));
          }
        }
      }
    }
    // every integer total is below 2^31: |V| <= 343, at most 64 present
    // levels of value <= 255 (sum n_i i^2 <= 2.3e7, bden <= 1.2e7)
    int ri[8] = {(int)sum_n, (int)pres, (int)pj, (int)pj2, (int)sum_ni, (int)sum_ni2, (int)bden, 0};
    wsum8i(ri);
    double rd[8] = {s_i, ps_acc, cplx, 0.0, 0.0, 0.0, 0.0, 0.0};
    wsum8d(rd);
    const long long Nvc = ri[0];
    if (Nvc == 0) {
      if (lane < kNNGTDM) F[oNGTDM + lane] = NAN;
    } else {
      const long long Ngp = ri[1], A1 = ri[2], A2 = ri[3];
      const long long Sn1 = ri[4], Sn2 = ri[5];
      const double ssum = rd[0];
      const double Nd = (double)Nvc;
      const double psum = rd[1] / Nd;  // sum_i p_i s_i
      const bool any_s = __ballot(anys) != 0ull;
      bden = ri[6];
      cplx = rd[2];
      if (lane == 0) {
        float* f = F + oNGTDM;
        // sum_ij p_i p_j (i-j)^2 = 2 Var_p(i);  sum_ij (p_i+p_j)(i-j)^2 =
        // 2 sum_i p_i (Ngp i^2 - 2 i A1 + A2)
        const double c1 = 2.0 * (double)(Nvc * Sn2 - Sn1 * Sn1) / (Nd * Nd);
        const double strn = 2.0 * (double)(Ngp * Sn2 - 2 * A1 * Sn1 + A2 * Nvc) / Nd;
        f[0] = any_s ? (float)(1.0 / psum) : 1e6f;
        f[1] = Ngp <= 1 ? 0.f : (float)(c1 / (double)(Ngp * (Ngp - 1)) * (ssum / Nd));
        f[2] = bden == 0 ? 0.f : (float)(psum / ((double)bden / Nd));
        f[3] = (float)(cplx / Nd);
        f[4] = any_s ? (float)(strn / ssum) : 0.f;
      }
    }
  }

  // ---- GLCM (last: its eigen work space overlays the tables above) -----
  if (fGLCM) {
    __syncthreads();
    // the |i-j| and i+j histograms overlay tables whose features are done:
    // clear the ranges the features read (|i-j| < Ng, i+j <= 2 Ng)
    for (int e = lane; e < a.ng; e += 64) sm.u.c.pd[e] = 0;
    for (int e = lane; e <= 2 * a.ng; e += 64) sm.u.c.ps[e] = 0;
    __syncthreads();
    long long rowc = 0, s1x = 0, s2x = 0;
    double hxp = 0.0;
    int lv = 0;
    if (lane < L) {
      rowc = sm.pxc[lane];
      lv = sm.lval[lane];
      s1x = rowc * lv;
      s2x = rowc * lv * lv;
      if (rowc) hxp = (double)rowc * flog2((double)rowc);
    }
    const long long NP = wsumi(rowc);
    if (NP == 0) {
      if (lane < kNGLCM) F[oGLCM + lane] = NAN;
    } else {
      const uint64_t presb = __ballot(lane < L && rowc > 0);
      const int nlev = __popcll(presb);
      const double Nd = (double)NP;
      const double lgN = flog2(Nd);
      // entries of the upper triangle (r <= c), one per lane, enumerated
      // compactly (e = c (c + 1) / 2 + r); an entry off the diagonal stands
      // for the two symmetric ones (weight 2)
      const int ntri = L * (L + 1) / 2;
      long long e2 = 0;
      double plogp = 0.0;
      unsigned pmax = 0;
      for (int e0 = 0; e0 < ntri; e0 += 64) {
        const int e = e0 + lane;
        if (e < ntri) {
          int c = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
          c += (c + 1) * (c + 2) / 2 <= e;  // exact floor of the root
          c -= c * (c + 1) / 2 > e;
          const int r = e - c * (c + 1) / 2;
          const uint32_t P = gget(sm.u.a.glcm, e);
          if (P) {
            const uint32_t w = r == c ? 1u : 2u;
            e2 += (long long)(w * P) * P;
            plogp += (double)w * ((double)P * flog2((double)P));
            pmax = max(pmax, P);
            const int i = sm.lval[r], j = sm.lval[c];
            atomicAdd(&sm.u.c.pd[i > j ? i - j : j - i], w * P);
            atomicAdd(&sm.u.c.ps[i + j], w * P);
          }
        }
      }
      int gi[8] = {(int)s1x, (int)s2x, (int)e2, 0, 0, 0, 0, 0};  // totals below 2^31
      wsum8i(gi);
      const long long S1x = gi[0], S2x = gi[1];
      e2 = gi[2];
      double gd[8] = {hxp, plogp, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      wsum8d(gd);
      const double HX = lgN - gd[0] / Nd;
      plogp = gd[1];
      pmax = wmaxu(pmax);
      __syncthreads();
      const int ng = a.ng;
      const double mu = (double)S1x / Nd;
      long long sd1 = 0, sd2 = 0, ss1 = 0, ss2 = 0;
      double dlog = 0, slog = 0, iv = 0, idm = 0, idmn = 0, id = 0, idn = 0, ct = 0, cs = 0, cp = 0;
      const double ngd = (double)ng;
      const double rng = 1.0 / ngd, rng2 = rng * rng;
      for (int k = lane; k < ng; k += 64) {
        const uint32_t c = sm.u.c.pd[k];
        if (c) {
          const double cd = (double)c, kd = (double)k;
          sd1 += (long long)c * k;
          sd2 += (long long)c * k * k;
          dlog += cd * flog2(cd);
          if (k > 0) iv += cd * frcp(kd * kd);
          idm += cd * frcp(1.0 + kd * kd);
          idmn += cd * frcp(1.0 + kd * kd * rng2);
          id += cd * frcp(1.0 + kd);
          idn += cd * frcp(1.0 + kd * rng);
        }
      }
      for (int k = 2 + lane; k <= 2 * ng; k += 64) {
        const uint32_t c = sm.u.c.ps[k];
        if (c) {
          const double cd = (double)c, t = (double)k - 2.0 * mu;
          ss1 += (long long)c * k;
          ss2 += (long long)c * k * k;
          slog += cd * flog2(cd);
          ct += cd * t * t;
          cs += cd * t * t * t;
          cp += cd * t * t * t * t;
        }
      }
      // totals below 2^31: the largest, sum over i+j of c k^2, is at most
      // N_P (2 Ng)^2 = 6,516 x 510^2 = 1.7e9 for a 7^3 cube
      int hi[8] = {(int)sd1, (int)sd2, (int)ss1, (int)ss2, 0, 0, 0, 0};
      wsum8i(hi);
      sd1 = hi[0];
      sd2 = hi[1];
      ss1 = hi[2];
      ss2 = hi[3];
      double h1[8] = {dlog, slog, iv, idm, idmn, id, idn, ct};
      wsum8d(h1);
      dlog = h1[0];
      slog = h1[1];
      iv = h1[2];
      idm = h1[3];
      idmn = h1[4];
      id = h1[5];
      idn = h1[6];
      ct = h1[7];
      double h2[8] = {cs, cp, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      wsum8d(h2);
      cs = h2[0];
      cp = h2[1];
      const long long sij = (ss2 - sd2) / 4;  // sum_ij i j P
      const double N2 = Nd * Nd;
      const double var = (double)(NP * S2x - S1x * S1x) / N2;
      const double HXY = lgN - plogp / Nd;

      // MCC: spectral radius of B = D^-1/2 P D^-1/2 - v v^T over present levels
      double mcc = 1.0;
      bool deferred = false;
      if (nlev > 1) {
        const int n = nlev;
        if (lane < L && rowc > 0) {
          const int pos = __popcll(presb & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
          sm.u.b.pl[pos] = lane;
        }
        __syncthreads();
        if (n <= 32) {  // stash the problem; a flush (or the MCC kernel) computes four at once
          // upper triangle, column c of the lower half-wave and column
          // n - 1 - c of the upper one per pass
          auto stash = [&](uint16_t* gq, float** dq, int* nqp) FR_INLINE {
            const int l = lane & 31;
            const int plr = l < n ? sm.u.b.pl[l] : 0;
            for (int c0 = 0; 2 * c0 < n; ++c0) {
              const int c = lane < 32 ? c0 : n - 1 - c0;
              if (l <= c && (lane < 32 || c > c0))
                gq[c * (c + 1) / 2 + l] = (uint16_t)gsym(sm.u.a.glcm, plr, sm.u.b.pl[c]);
            }
            if (lane == 0) {
              *nqp = n;
              *dq = a.stage ? a.stage + it * kStageStride + (oGLCM + 15)
                            : a.out + (int64_t)(oGLCM + 15) * a.n_out + it;
            }
          };
          if constexpr (MOUT) {
            // problems with <= 16 levels fill the stash from its start,
            // wider ones from its end (one problem per voxel at most, so
            // the two never meet)
            const bool small = n <= 16;
            int slot = 0;
            if (lane == 0) slot = atomicAdd(&a.mcc_count[small ? 0 : 1], 1);
            slot = __shfl(slot, 0);
            if (small) {
              McSmall* q = (McSmall*)a.mcc + slot;
              stash(q->g, &q->dst, &q->n);
            } else {
              McProblem* q = (McProblem*)(a.mcc + a.mcc_cap * kMccProblemBytes) - (slot + 1);
              stash(q->g, &q->dst, &q->n);
            }
          } else {
            bool to_small = false;
            if constexpr (kSmallSlots<R, LMAX> > 0) to_small = n <= 16;
            if (to_small) {
              if constexpr (kSmallSlots<R, LMAX> > 0) stash(sm.ms.s[ns].g, &sm.ms.s[ns].dst, &sm.ms.s[ns].n);
              ++ns;
            } else {
              stash(sm.mq.s[nq].g, &sm.mq.s[nq].dst, &sm.mq.s[nq].n);
              ++nq;
            }
          }
          deferred = true;
          mcc = NAN;
        }
        if constexpr (LMAX > 32) {
          if (!deferred) {  // > 32 levels: computed at the flush after this voxel
            if (lane == 0) {
              sm.u.b.big_n = n;
              sm.u.b.big_dst = a.stage ? a.stage + it * kStageStride + (oGLCM + 15)
                                       : a.out + (int64_t)(oGLCM + 15) * a.n_out + it;
            }
            big = true;
            mcc = NAN;
          }
        }
      }

      const double rNd = 1.0 / Nd, rN2 = rNd * rNd;  // one division; the rest multiply
      if (lane == 0) {
        float* f = F + oGLCM;
        f[0] = (float)((double)sij * rNd);
        f[1] = (float)mu;
        f[2] = (float)(cp * rNd);
        f[3] = (float)(cs * rNd);
        f[4] = (float)(ct * rNd);
        f[5] = (float)((double)sd2 * rNd);
        f[6] = nlev <= 1 ? 1.f
                         : (float)((double)(NP * sij - S1x * S1x) / (double)(NP * S2x - S1x * S1x));
        f[7] = (float)((double)sd1 * rNd);
        f[8] = (float)(lgN - dlog * rNd);
        f[9] = (float)((double)(NP * sd2 - sd1 * sd1) * rN2);
        f[10] = (float)((double)e2 * rN2);
        f[11] = (float)HXY;
        f[12] = nlev <= 1 ? 0.f : (float)((HXY - 2.0 * HX) / HX);
        const double t = 1.0 - exp(-2.0 * (2.0 * HX - HXY));
        f[13] = (float)sqrt(t > 0.0 ? t : 0.0);
        f[14] = (float)(idm * rNd);
        f[15] = (float)mcc;
        f[16] = (float)(idmn * rNd);
        f[17] = (float)(id * rNd);
        f[18] = (float)(idn * rNd);
        f[19] = (float)(iv * rNd);
        f[20] = (float)((double)pmax * rNd);
        f[21] = (float)((double)ss1 * rNd);
        f[22] = (float)(lgN - slog * rNd);
        f[23] = (float)var;
      }
    }
  }

  __syncthreads();
  if (a.stage) {  // one contiguous row per voxel; the transpose kernel scatters it
    // whole rows (a deferred MCC is a placeholder here; the flush overwrites it
    // after its barrier, whose release fence completes these stores first)
    float* row = a.stage + it * kStageStride;
    for (int k = lane; k < count; k += 64) row[k] = F[k];
  } else {
    for (int k = lane; k < count; k += 64) a.out[(int64_t)k * a.n_out + it] = F[k];
  }
  __syncthreads();
}

// MOUT: the MCC problems with <= 32 levels go to the stash of a.mcc, so the
// kernel needs no LDS slots for them; the 32-level instance then holds no
// MCC code at all and needs far fewer registers (three waves per SIMD),
// while the 64-level one still solves its wider problems itself.
template <typename T, int R, int LMAX, bool DEBUG, bool MOUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MOUT && LMAX == 32 ? 3 : 2))) void k_map(MapArgs arg) {
  static_assert(!MOUT || !DEBUG, "stash only from production instances");
  __shared__ Smem<R, LMAX, MOUT> sm;
  const DiscParams* P = arg.params;
  if (P->err != kJobOk) return;  // a data error of the discretisation: write nothing
  MapArgs a = arg;
  a.ng = P->ng;
  if (threadIdx.x < Smem<R, LMAX>::LVW) ((uint32_t*)sm.lflag)[threadIdx.x] = 0u;
  for (int e = threadIdx.x; e < Smem<R, LMAX>::PC / 4; e += 64) ((uint32_t*)sm.clp)[e] = 0u;
  __syncthreads();
  int ns = 0, nq = 0;  // deferred MCC problems in sm.ms and sm.mq
  bool big = false;    // a problem with > 32 levels pending
  // balanced partition (n < 2^31): the counts differ by at most one; with
  // an item list, n is the list's length as the previous pass left it
  const int64_t n = a.items ? (int64_t)*a.items_count : a.n_items;
  const int64_t i0 = (int64_t)blockIdx.x * n / a.nblk;
  const int64_t i1 = ((int64_t)blockIdx.x + 1) * n / a.nblk;
  for (int64_t k = i0; k < i1; ++k) {
    const int64_t it = a.items ? (int64_t)a.items[k].y : k;
    const int64_t m = DEBUG ? a.sample[it] : it;
    if (m < 0 || m >= a.n_list) {  // out-of-range sample index: NaN maps, no matrices
      for (int q = threadIdx.x; q < 93; q += 64)
        if (q < __popc(a.families & 1u) * 18 + __popc(a.families & 2u) * 24 +
                    __popc(a.families & 4u) * 16 + __popc(a.families & 8u) * 16 +
                    __popc(a.families & 16u) * 14 + __popc(a.families & 32u) * 5)
          a.out[(int64_t)q * a.n_out + it] = NAN;
    } else {
      map_voxel<T, R, LMAX, DEBUG, MOUT>(sm, a, a.list[m], it, ns, nq, big);
    }
    if constexpr (!MOUT) {
      // one flush site (the flush code is large): after a voxel with more
      // than 32 levels, when a pool is full, and after the last voxel
      const bool last = k + 1 == i1;
      const int fs = (ns == kSmallSlots<R, LMAX> || last) ? ns : 0;
      const int fq = (nq == kMcSlots<R, LMAX> || last) ? nq : 0;
      if (big || fs || fq) {
        mcc_flush(sm, fs, fq, big);
        ns -= fs;
        nq -= fq;
        big = false;
      }
    } else if constexpr (LMAX > 32) {
      if (big) {  // the smaller problems went to the stash
        mcc_flush(sm, 0, 0, true);
        big = false;
      }
    }
  }
}

// The MCC of the problems a map pass stashed: groups of four problems of
// one kind per wave (a 16-lane row each), the <= 16-level ones first; each
// result goes to its problem's output address.  A problem's result depends
// only on the problem, as in the in-kernel flush.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_mcc(
    const int32_t* __restrict__ n_mcc, const int32_t* __restrict__ err,
    const unsigned char* __restrict__ stash, int64_t cap) {
  if (err && *err != kJobOk) return;
  const int nn = n_mcc[0], nw = n_mcc[1];
  const int gn = (nn + 3) / 4, gw = (nw + 3) / 4;
  for (int g = blockIdx.x; g < gn + gw; g += gridDim.x) {
    if (g < gn) {
      const int c = min(4, nn - 4 * g);
      mcc_narrow((const McSmall*)stash + 4 * g, (1u << c) - 1u);
    } else {
      // wide problem k is the (k + 1)-th entry from the end: slot s of the
      // group's window is problem k0 + c - 1 - s
      const int k0 = 4 * (g - gn), c = min(4, nw - k0);
      const McProblem* win = (const McProblem*)(stash + cap * kMccProblemBytes) - (k0 + c);
      mcc_wide(win, (1u << c) - 1u);
    }
  }
}

// Workgroups for n voxels: a whole number of waves of the resident
// workgroups (so no partial last wave leaves CUs idle), at least 8 voxels
// each (a sweep over 4..48 on the PET workload put the optimum there) and
// at most 8 waves, but never under 4 voxels per workgroup (a workgroup's
// deferred MCC problems should fill the rows of its flushes).
inline int64_t plain_blocks(int64_t n, int64_t resident) {
  if (resident < 1) resident = 1;
  int64_t per = (n + resident * 8 - 1) / (resident * 8);
  if (per < 8) per = 8;
  const int64_t waves = (n + resident * per - 1) / (resident * per);
  int64_t nblk = waves * resident;
  const int64_t cap = (n + 3) / 4;
  if (nblk > cap) nblk = cap;
  return nblk < 1 ? 1 : nblk;
}

template <typename T, int R, int LMAX, bool MOUT = false>
int resident_t() {
  static int resident = 0;  // resident workgroups of this instance on the device
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_map<T, R, LMAX, false, MOUT>, 64,
                                                     0) != hipSuccess) {
      (void)hipGetLastError();
      cus = 256;
      per_cu = 1;
    }
    resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  return resident;
}

template <typename T, int R, int LMAX>
hipError_t launch_t(MapArgs a, bool debug, hipStream_t st) {
  const bool mout = !debug && a.mcc;
  const int resident = mout ? resident_t<T, R, LMAX, true>() : resident_t<T, R, LMAX>();
  // an item list's length is known only on the device: one whole wave of
  // resident workgroups, each taking its share of whatever the list holds
  a.nblk = a.items ? resident : plain_blocks(a.n_items, resident);
  if (debug)
    hipLaunchKernelGGL((k_map<T, R, LMAX, true, false>), dim3((unsigned)a.nblk), dim3(64), 0, st, a);
  else if (mout)
    hipLaunchKernelGGL((k_map<T, R, LMAX, false, true>), dim3((unsigned)a.nblk), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_map<T, R, LMAX, false, false>), dim3((unsigned)a.nblk), dim3(64), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_r(const MapArgs& a, int radius, int lmax, bool debug, hipStream_t st) {
  if (radius == 1) return launch_t<T, 1, 32>(a, debug, st);
  if (radius == 2) return lmax <= 32 ? launch_t<T, 2, 32>(a, debug, st) : launch_t<T, 2, 64>(a, debug, st);
  return lmax <= 32 ? launch_t<T, 3, 32>(a, debug, st) : launch_t<T, 3, 64>(a, debug, st);
}

template <typename T>
int resident_r(int radius, int lmax) {
  if (radius == 1) return resident_t<T, 1, 32>();
  if (radius == 2) return lmax <= 32 ? resident_t<T, 2, 32>() : resident_t<T, 2, 64>();
  return lmax <= 32 ? resident_t<T, 3, 32>() : resident_t<T, 3, 64>();
}

// Tile transpose of the staging rows: 64 voxels x up to 96 maps per block
// through LDS, so both the row reads and the per-map writes (64 consecutive
// floats) are contiguous.
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ stage,
                                                   float* __restrict__ out, int64_t n,
                                                   int count, const DiscParams* __restrict__ params) {
  __shared__ float tile[64][kStageStride + 1];
  if (params->err != kJobOk) return;
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int t = threadIdx.x;
  for (int e = t; e < 64 * kStageStride; e += 256) {
    const int v = e / kStageStride, k = e % kStageStride;
    if (m0 + v < n && k < count) tile[v][k] = stage[(m0 + v) * kStageStride + k];
  }
  __syncthreads();
  for (int e = t; e < 64 * count; e += 256) {
    const int k = e / 64, v = e % 64;
    if (m0 + v < n) out[(int64_t)k * n + m0 + v] = tile[v][k];
  }
}

template <typename T, int R, int LMAX, bool MOUT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MOUT ? 3 : 2))) void k_map_batch(
    const BatchJob* __restrict__ jobs, const DiscParams* __restrict__ params,
    const int2* __restrict__ items, int32_t n_items_host, const int32_t* __restrict__ n_items_dev,
    int32_t vpw, int2* over, int32_t* over_count, int32_t* queue, unsigned char* mcc,
    int64_t mcc_cap, int32_t* mcc_count) {
  static_assert(!MOUT || LMAX == 32, "stash only from the 32-level instance");
  __shared__ Smem<R, LMAX, MOUT> sm;
  const int32_t n_items = n_items_dev ? *n_items_dev : n_items_host;
  if (threadIdx.x < Smem<R, LMAX>::LVW) ((uint32_t*)sm.lflag)[threadIdx.x] = 0u;
  for (int e = threadIdx.x; e < Smem<R, LMAX>::PC / 4; e += 64) ((uint32_t*)sm.clp)[e] = 0u;
  __syncthreads();
  int ns = 0, nq = 0;  // deferred MCC problems in sm.ms and sm.mq
  bool big = false;    // a problem with > 32 levels pending
  // work distribution: items blockIdx.x, + gridDim.x, ... (static), or the
  // next item of the queue (dynamic); one loop over their voxels, so that
  // the flush has a single site
  int64_t w = (int64_t)blockIdx.x - (int64_t)gridDim.x;
  int64_t m = 0, m1 = 0;
  MapArgs a;
  const BatchJob* J = nullptr;
  for (;;) {
    while (m >= m1) {  // next item of a job without error
      if (queue) {
        int q = 0;
        if (threadIdx.x == 0) q = atomicAdd(queue, 1);
        w = __shfl(q, 0);
      } else {
        w += gridDim.x;
      }
      if (w >= n_items) break;
      // no item table: one job (index 0), item w starts at voxel w * vpw
      const int2 it2 = items ? items[w] : make_int2(0, w * vpw);
      const DiscParams& P = params[it2.x];
      if (P.err != kJobOk) continue;
      J = &jobs[it2.x];
      a.params = &P;
      a.vol = J->vol;
      a.levels = J->levels;
      a.list = J->list;
      a.sample = nullptr;
      a.out = J->out;
      a.stage = J->stage;
      a.n_out = J->n_mask;
      a.n_items = J->n_mask;
      a.n_list = J->n_mask;
      a.nx = J->nx;
      a.ny = J->ny;
      a.nz = J->nz;
      a.ng = P.ng;
      a.families = J->families;
      a.voxel_volume = J->voxel_volume;
      a.nblk = 0;
      a.d_glcm = a.d_glrlm = a.d_glszm = a.d_gldm = a.d_ngn = a.d_hist = nullptr;
      a.d_ngS = nullptr;
      a.items = nullptr;
      a.items_count = nullptr;
      a.over = over;
      a.over_count = over_count;
      a.over_job = it2.x;
      a.radius = J->radius;
      a.opt = J->opt;
      a.mcc = mcc;
      a.mcc_cap = mcc_cap;
      a.mcc_count = mcc_count;
      m = it2.y;
      m1 = (int64_t)it2.y + vpw;
      if (m1 > J->n_mask) m1 = J->n_mask;
    }
    const bool more = w < n_items;
    if (more) {
      map_voxel<T, R, LMAX, false, MOUT>(sm, a, a.list[m], m, ns, nq, big);
      ++m;
    }
    if constexpr (!MOUT) {
      const int fs = (ns == kSmallSlots<R, LMAX> || !more) ? ns : 0;
      const int fq = (nq == kMcSlots<R, LMAX> || !more) ? nq : 0;
      if (big || fs || fq) {
        mcc_flush(sm, fs, fq, big);
        ns -= fs;
        nq -= fq;
        big = false;
      }
    }
    if (!more) break;
  }
}

// The fused batched pass: every fixed radius of one raw type in one
// persistent kernel.  The LDS holds one radius's layout at a time (a union
// of the three); a workgroup switches layout when its next item's job has
// another radius (items come grouped by radius, so rarely), after flushing
// the MCC problems stashed in the old layout (64-level form).
struct FusedNone {};
template <int LMAX, bool MOUT>
union FusedSmem {
  std::conditional_t<LMAX == 32, Smem<1, 32, MOUT>, FusedNone> s1;
  Smem<2, LMAX, MOUT> s2;
  Smem<3, LMAX, MOUT> s3;
};

template <int R, int LMAX, bool MOUT>
__device__ FR_INLINE inline void fused_layout(Smem<R, LMAX, MOUT>& sm) {
  if (threadIdx.x < Smem<R, LMAX, MOUT>::LVW) ((uint32_t*)sm.lflag)[threadIdx.x] = 0u;
  for (int e = threadIdx.x; e < Smem<R, LMAX, MOUT>::PC / 4; e += 64) ((uint32_t*)sm.clp)[e] = 0u;
  __syncthreads();
}

template <typename T, int LMAX>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LMAX == 32 ? 3 : 2))) void k_map_fused(
    const BatchJob* __restrict__ jobs, const DiscParams* __restrict__ params,
    const int2* __restrict__ items, int32_t n_items_host, const int32_t* __restrict__ n_items_dev,
    int2* over, int32_t* over_count, int32_t* queue, unsigned char* mcc, int64_t mcc_cap,
    int32_t* mcc_count) {
  constexpr bool MOUT = true;  // problems with <= 32 levels go to the stash
  __shared__ FusedSmem<LMAX, MOUT> sm;
  const int32_t n_items = n_items_dev ? *n_items_dev : n_items_host;
  int cur = 0;         // radius whose layout the LDS holds (0: none yet)
  int ns = 0, nq = 0;  // deferred MCC problems (64-level form)
  bool big = false;
  auto flush = [&](bool) FR_INLINE {
    if constexpr (LMAX > 32) {  // a problem with more than 32 levels, solved here
      if (big) {
        if (cur == 2)
          mcc_flush(sm.s2, 0, 0, true);
        else
          mcc_flush(sm.s3, 0, 0, true);
        big = false;
      }
    }
  };
  int64_t m = 0, m1 = 0;
  MapArgs a;
  const BatchJob* J = nullptr;
  for (;;) {
    int R = cur;
    while (m >= m1) {  // next item of a job without error
      int q = 0;
      if (threadIdx.x == 0) q = atomicAdd(queue, 1);
      const int w = __shfl(q, 0);
      if (w >= n_items) break;
      const int2 it2 = items[w];
      const DiscParams& P = params[it2.x];
      if (P.err != kJobOk) continue;
      J = &jobs[it2.x];
      a.params = &P;
      a.vol = J->vol;
      a.levels = J->levels;
      a.list = J->list;
      a.sample = nullptr;
      a.out = J->out;
      a.stage = J->stage;
      a.n_out = J->n_mask;
      a.n_items = J->n_mask;
      a.n_list = J->n_mask;
      a.nx = J->nx;
      a.ny = J->ny;
      a.nz = J->nz;
      a.ng = P.ng;
      a.families = J->families;
      a.voxel_volume = J->voxel_volume;
      a.nblk = 0;
      a.d_glcm = a.d_glrlm = a.d_glszm = a.d_gldm = a.d_ngn = a.d_hist = nullptr;
      a.d_ngS = nullptr;
      a.items = nullptr;
      a.items_count = nullptr;
      a.over = over;
      a.over_count = over_count;
      a.over_job = it2.x;
      a.radius = J->radius;
      a.opt = J->opt;
      a.mcc = mcc;
      a.mcc_cap = mcc_cap;
      a.mcc_count = mcc_count;
      R = __builtin_amdgcn_readfirstlane(J->radius);
      m = it2.y;
      m1 = (int64_t)it2.y + (LMAX == 32 ? J->vpw : 1);
      if (m1 > J->n_mask) m1 = J->n_mask;
    }
    const bool more = m < m1;
    if (!more || R != cur) {  // end, or another radius's layout
      flush(true);
      if (!more) break;
      if (R == 1) {
        if constexpr (LMAX == 32) fused_layout(sm.s1);
      } else if (R == 2) {
        fused_layout(sm.s2);
      } else {
        fused_layout(sm.s3);
      }
      cur = R;
    }
    if (R == 1) {
      if constexpr (LMAX == 32) map_voxel<T, 1, 32, false, MOUT>(sm.s1, a, a.list[m], m, ns, nq, big);
    } else if (R == 2) {
      map_voxel<T, 2, LMAX, false, MOUT>(sm.s2, a, a.list[m], m, ns, nq, big);
    } else {
      map_voxel<T, 3, LMAX, false, MOUT>(sm.s3, a, a.list[m], m, ns, nq, big);
    }
    ++m;
    flush(false);
  }
}

__global__ __launch_bounds__(256) void k_transpose_batch(const BatchJob* __restrict__ jobs,
                                                         const DiscParams* __restrict__ params,
                                                         const int2* __restrict__ items) {
  __shared__ float tile[64][kStageStride + 1];
  const int2 it2 = items ? items[blockIdx.x] : make_int2(0, (int)blockIdx.x * 64);
  const BatchJob& J = jobs[it2.x];
  if (params[it2.x].err != kJobOk) return;
  const int64_t n = J.n_mask, m0 = it2.y;
  const int count = J.count;
  const int t = threadIdx.x;
  for (int e = t; e < 64 * kStageStride; e += 256) {
    const int v = e / kStageStride, k = e % kStageStride;
    if (m0 + v < n && k < count) tile[v][k] = J.stage[(m0 + v) * kStageStride + k];
  }
  __syncthreads();
  for (int e = t; e < 64 * count; e += 256) {
    const int k = e / 64, v = e % 64;
    if (m0 + v < n) J.out[(int64_t)k * n + m0 + v] = tile[v][k];
  }
}

template <typename T, int R, int LMAX>
hipError_t launch_b(const BatchJob* jobs, const DiscParams* params, const int2* items,
                    int32_t n_items, const int32_t* n_items_dev, int32_t vpw, int grid, int2* over,
                    int32_t* over_count, int32_t* queue, unsigned char* mcc, int64_t mcc_cap,
                    int32_t* mcc_count, hipStream_t st) {
  if constexpr (LMAX == 32) {
    if (mcc) {
      hipLaunchKernelGGL((k_map_batch<T, R, 32, true>), dim3((unsigned)grid), dim3(64), 0, st, jobs, params,
                         items, n_items, n_items_dev, vpw, over, over_count, queue, mcc, mcc_cap, mcc_count);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_map_batch<T, R, LMAX, false>), dim3((unsigned)grid), dim3(64), 0, st, jobs, params,
                     items, n_items, n_items_dev, vpw, over, over_count, queue, nullptr, (int64_t)0,
                     nullptr);
  return hipGetLastError();
}

template <typename T, int R, int LMAX, bool MOUT>
int occ_b() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_map_batch<T, R, LMAX, MOUT>, 64, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <typename T>
hipError_t launch_b_r(const BatchJob* jobs, const DiscParams* params, const int2* items,
                      int32_t n_items, const int32_t* n_items_dev, int32_t vpw, int radius,
                      int lmax, int grid, int2* over, int32_t* over_count, int32_t* queue,
                      unsigned char* mcc, int64_t mcc_cap, int32_t* mcc_count, hipStream_t st) {
  if (radius == 1)
    return launch_b<T, 1, 32>(jobs, params, items, n_items, n_items_dev, vpw, grid, over, over_count,
                              queue, mcc, mcc_cap, mcc_count, st);
  if (radius == 2)
    return lmax <= 32 ? launch_b<T, 2, 32>(jobs, params, items, n_items, n_items_dev, vpw, grid, over,
                                           over_count, queue, mcc, mcc_cap, mcc_count, st)
                      : launch_b<T, 2, 64>(jobs, params, items, n_items, n_items_dev, vpw, grid, over,
                                           over_count, queue, nullptr, 0, nullptr, st);
  return lmax <= 32 ? launch_b<T, 3, 32>(jobs, params, items, n_items, n_items_dev, vpw, grid, over,
                                         over_count, queue, mcc, mcc_cap, mcc_count, st)
                    : launch_b<T, 3, 64>(jobs, params, items, n_items, n_items_dev, vpw, grid, over,
                                         over_count, queue, nullptr, 0, nullptr, st);
}

template <typename T>
int occ_b_r(int radius, int lmax, bool stash) {
  if (radius == 1) return stash ? occ_b<T, 1, 32, true>() : occ_b<T, 1, 32, false>();
  if (radius == 2)
    return lmax > 32 ? occ_b<T, 2, 64, false>() : (stash ? occ_b<T, 2, 32, true>() : occ_b<T, 2, 32, false>());
  return lmax > 32 ? occ_b<T, 3, 64, false>() : (stash ? occ_b<T, 3, 32, true>() : occ_b<T, 3, 32, false>());
}

template <typename T, int LMAX>
int occ_f() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_map_fused<T, LMAX>, 64, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace

hipError_t launch_map_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                            int32_t n_items, const int32_t* n_items_dev, int32_t vpw, int dtype,
                            int radius, int lmax, int grid, int2* over, int32_t* over_count,
                            int32_t* queue, unsigned char* mcc, int64_t mcc_cap, int32_t* mcc_count,
                            hipStream_t st) {
  if (n_items <= 0 && !n_items_dev) return hipSuccess;
  if (dtype == 1)
    return launch_b_r<int16_t>(jobs, params, items, n_items, n_items_dev, vpw, radius, lmax, grid,
                               over, over_count, queue, mcc, mcc_cap, mcc_count, st);
  return launch_b_r<float>(jobs, params, items, n_items, n_items_dev, vpw, radius, lmax, grid, over,
                           over_count, queue, mcc, mcc_cap, mcc_count, st);
}

hipError_t launch_map_fused(const BatchJob* jobs, const DiscParams* params, const int2* items,
                            int32_t n_items, const int32_t* n_items_dev, int dtype, int lmax,
                            int grid, int2* over, int32_t* over_count, int32_t* queue,
                            unsigned char* mcc, int64_t mcc_cap, int32_t* mcc_count, hipStream_t st) {
  if (n_items <= 0 && !n_items_dev) return hipSuccess;
  const dim3 g((unsigned)grid), b(64);
  if (dtype == 1) {
    if (lmax <= 32)
      hipLaunchKernelGGL((k_map_fused<int16_t, 32>), g, b, 0, st, jobs, params, items, n_items, n_items_dev,
                         over, over_count, queue, mcc, mcc_cap, mcc_count);
    else
      hipLaunchKernelGGL((k_map_fused<int16_t, 64>), g, b, 0, st, jobs, params, items, n_items, n_items_dev,
                         over, over_count, queue, mcc, mcc_cap, mcc_count);
  } else {
    if (lmax <= 32)
      hipLaunchKernelGGL((k_map_fused<float, 32>), g, b, 0, st, jobs, params, items, n_items, n_items_dev,
                         over, over_count, queue, mcc, mcc_cap, mcc_count);
    else
      hipLaunchKernelGGL((k_map_fused<float, 64>), g, b, 0, st, jobs, params, items, n_items, n_items_dev,
                         over, over_count, queue, mcc, mcc_cap, mcc_count);
  }
  return hipGetLastError();
}

int map_fused_blocks_per_cu(int dtype, int lmax) {
  if (dtype == 1) return lmax <= 32 ? occ_f<int16_t, 32>() : occ_f<int16_t, 64>();
  return lmax <= 32 ? occ_f<float, 32>() : occ_f<float, 64>();
}

int map_batch_blocks_per_cu(int dtype, int radius, int lmax, bool stash) {
  return dtype == 1 ? occ_b_r<int16_t>(radius, lmax, stash) : occ_b_r<float>(radius, lmax, stash);
}

hipError_t launch_transpose_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                                  int32_t n_items, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_batch, dim3((unsigned)n_items), dim3(256), 0, st, jobs, params, items);
  return hipGetLastError();
}

hipError_t launch_mcc(const int32_t* n_mcc, const int32_t* err, const unsigned char* stash,
                      int64_t cap, hipStream_t st) {
  static int grid = 0;  // resident workgroups of k_mcc: a persistent grid
  if (grid == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_mcc, 64, 0) != hipSuccess) {
      (void)hipGetLastError();
      cus = 256;
      per_cu = 1;
    }
    grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  hipLaunchKernelGGL(k_mcc, dim3((unsigned)grid), dim3(64), 0, st, n_mcc, err, stash, cap);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* stage, float* out, int64_t n, int count,
                            const DiscParams* params, hipStream_t st) {
  const int64_t nb = (n + 63) / 64;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)nb), dim3(256), 0, st, stage, out, n, count, params);
  return hipGetLastError();
}

int map_resident(int dtype, int radius, int lmax) {
  return dtype == 1 ? resident_r<int16_t>(radius, lmax) : resident_r<float>(radius, lmax);
}

hipError_t launch_map(const MapArgs& a, int dtype, int radius, int lmax, bool debug,
                      hipStream_t st) {
  if (dtype == 1) return launch_r<int16_t>(a, radius, lmax, debug, st);
  return launch_r<float>(a, radius, lmax, debug, st);
}

}  // namespace fr
