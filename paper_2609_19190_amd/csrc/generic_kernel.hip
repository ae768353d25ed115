// Generic spatial-mapping kernel for gfx950: the neighbourhoods the fused
// fixed-radius kernel does not take.
//
// It computes exactly the maps of the fused kernel (paper: "Software design
// and extraction modes" -- spatial maps; Table 2's 93 maps; IBSI feature
// definitions) for
//   - neighbourhoods holding more present gray levels than the 64-level
//     tables of the fused kernel (up to 255),
//   - kernel radii above 3 (up to kGenericMaxRadius),
//   - the IBSI extraction variants the paper lists among its settings: GLCM
//     neighbour distance > 1, GLDM coarseness alpha > 0, and GLCM / GLRLM
//     features averaged over the 13 directions instead of merged.
// One workgroup of 256 threads (four waves) maps one voxel at a time and is
// persistent over its share of the items.  The cube (levels, raw values,
// equal-level bits, zone labels) lives in LDS; the tables indexed by present
// levels (GLCM L x L, GLRLM, GLDM, zone sizes, the zone (level, size) hash)
// and the MCC matrix live in a global scratch slice of the workgroup.  Table
// entries are only ever incremented by atomics and read by agent-scope
// atomic loads, so no stale vector-L1 line is read; the MCC matrix is
// column-owned (thread j alone reads and writes column j), so plain loads
// and stores are coherent for it.
#include <math.h>

#include "fr_internal.h"
#include "map_device.h"

namespace fr {
namespace {

constexpr int NT = kGenericThreads;                 // 256
constexpr int NW = NT / 64;                         // waves per workgroup
constexpr int RMAXG = kGenericMaxRadius;
constexpr int SMAXG = 2 * RMAXG + 1;
constexpr int CMAXG = SMAXG * SMAXG * SMAXG;        // 1331
constexpr int CPADG = (CMAXG + NT - 1) / NT * NT;   // 1536
constexpr int SORTG = 2048;                         // power of two >= CMAXG
constexpr int HTG = 4096;                           // zone hash slots (> 2 x zones)
constexpr int kNRed = 16;                           // values per block reduction

struct GSmem {
  uint8_t cl[CPADG];      // level per cube position (0: not in V)
  uint8_t lflag[256];     // level present in V
  uint8_t lmap[256];      // level -> compact index
  uint8_t lval[256];      // compact index -> level
  float cr[SORTG];        // raw values (+inf outside V), sorted in place
  uint32_t same[CPADG];   // equal-level neighbour bits (bit n: neighbour n)
  uint32_t lab[CPADG];    // zone labels
  uint32_t zcnt[CPADG];   // zone sizes at roots
  uint32_t hist[256];     // level histogram (compact index)
  uint32_t pxc[256];      // GLCM row sums of the current pass
  uint32_t ngn[256];      // NGTDM n_i
  uint32_t zpl[256];      // zones per level
  unsigned long long ngS[256];  // NGTDM s_i * lcm(1..26)
  uint32_t pd[256];       // |i-j| histogram of the GLCM pass
  uint32_t ps[512];       // i+j histogram of the GLCM pass
  int pl[256];            // compact index of the k-th present GLCM level
  double va[256];         // MCC: Householder v, then the diagonal d
  double vb[256];         // MCC: q, then the squared sub-diagonal e^2
  double ve[256];         // MCC: sub-diagonal e
  double red[NW][kNRed];  // block reductions
  long long redl[NW][kNRed];
  float feat[96];         // this voxel's maps
  int iv[4];              // block-wide integers (flags, counters, broadcasts)
  double dv[2];           // block-wide doubles (broadcasts)
};

// Layout of a workgroup's global scratch slice for lcap present levels.
struct GLayout {
  size_t glcm, glrlm, gldm, zps, hkey, hcnt, mat, total;
};
__host__ __device__ inline size_t galign(size_t x) { return (x + 255) / 256 * 256; }
__host__ __device__ inline GLayout glayout(int lcap) {
  GLayout g;
  size_t o = 0;
  g.glcm = o;  o = galign(o + sizeof(uint32_t) * (size_t)lcap * lcap);
  g.glrlm = o; o = galign(o + sizeof(uint32_t) * (size_t)lcap * SMAXG);
  g.gldm = o;  o = galign(o + sizeof(uint32_t) * (size_t)lcap * 27);
  g.zps = o;   o = galign(o + sizeof(uint32_t) * CMAXG);
  g.hkey = o;  o = galign(o + sizeof(uint32_t) * HTG);
  g.hcnt = o;  o = galign(o + sizeof(uint32_t) * HTG);
  g.mat = o;   o = galign(o + sizeof(double) * (size_t)lcap * lcap);
  g.total = o;
  return g;
}

__device__ inline uint32_t gld(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void gzero(uint32_t* p) {
  __hip_atomic_store(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- block reductions (every thread receives the totals) ---------------
template <int N>
__device__ inline void bsum(GSmem& sm, double (&v)[N]) {
  static_assert(N <= kNRed, "reduction width");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) sm.red[w][k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double x = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) x += sm.red[q][k];
    v[k] = x;
  }
  __syncthreads();
}
template <int N>
__device__ inline void bsuml(GSmem& sm, long long (&v)[N]) {
  static_assert(N <= kNRed, "reduction width");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    long long x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) sm.redl[w][k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    long long x = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) x += sm.redl[q][k];
    v[k] = x;
  }
  __syncthreads();
}
__device__ inline double bmax(GSmem& sm, double v) {  // v >= 0
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (lane == 0) sm.red[w][0] = v;
  __syncthreads();
  double x = 0.0;
#pragma unroll
  for (int q = 0; q < NW; ++q) x = fmax(x, sm.red[q][0]);
  __syncthreads();
  return x;
}
// Exclusive prefix sum over the 256 threads; *total receives the sum.
__device__ inline int bscan(GSmem& sm, int v, int* total) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm.redl[w][0] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const int t = (int)sm.redl[q][0];
    before += q < w ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

// Run / zone / dependence emphasis sums of one table.
struct GEmph {
  long long n, si, si2, sj, sj2, si2j2;
  double invj2, invi2, invi2j2, i2invj2, j2invi2, clogc;
};
__device__ inline void gemph_add(GEmph& e, long long c, int i, int j) {
  const double cd = (double)c, i2 = (double)i * i, j2 = (double)j * j;
  e.n += c;
  e.si += c * i;
  e.si2 += c * i * i;
  e.sj += c * j;
  e.sj2 += c * j * j;
  e.si2j2 += c * (long long)(i * i) * (long long)(j * j);
  e.invj2 += cd / j2;
  e.invi2 += cd / i2;
  e.invi2j2 += cd / (i2 * j2);
  e.i2invj2 += cd * i2 / j2;
  e.j2invi2 += cd * j2 / i2;
  if (c > 1) e.clogc += cd * flog2(cd);
}
// Block totals of e; x1, x2 two more integer partials reduced alongside.
__device__ inline void gemph_reduce(GSmem& sm, GEmph& e, long long& x1, long long& x2) {
  long long vl[8] = {e.n, e.si, e.si2, e.sj, e.sj2, e.si2j2, x1, x2};
  bsuml(sm, vl);
  e.n = vl[0]; e.si = vl[1]; e.si2 = vl[2]; e.sj = vl[3]; e.sj2 = vl[4]; e.si2j2 = vl[5];
  x1 = vl[6];
  x2 = vl[7];
  double vd[6] = {e.invj2, e.invi2, e.invi2j2, e.i2invj2, e.j2invi2, e.clogc};
  bsum(sm, vd);
  e.invj2 = vd[0]; e.invi2 = vd[1]; e.invi2j2 = vd[2]; e.i2invj2 = vd[3]; e.j2invi2 = vd[4];
  e.clogc = vd[5];
}
// GLRLM / GLSZM: the 16 maps (units = Np or Nv).
__device__ inline void gemph16(const GEmph& e, long long gln, long long rln, double units, double* f) {
  const double N = (double)e.n;
  f[0] = e.invj2 / N;
  f[1] = (double)e.sj2 / N;
  f[2] = (double)gln / N;
  f[3] = (double)gln / (N * N);
  f[4] = (double)rln / N;
  f[5] = (double)rln / (N * N);
  f[6] = N / units;
  f[7] = (double)(e.n * e.si2 - e.si * e.si) / (N * N);
  f[8] = (double)(e.n * e.sj2 - e.sj * e.sj) / (N * N);
  f[9] = flog2(N) - e.clogc / N;
  f[10] = e.invi2 / N;
  f[11] = (double)e.si2 / N;
  f[12] = e.invi2j2 / N;
  f[13] = e.i2invj2 / N;
  f[14] = e.j2invi2 / N;
  f[15] = (double)e.si2j2 / N;
}

// Eigenvalues below y of the tridiagonal (d, e^2) (Sturm, ratio form; a
// pivot of exactly zero is replaced by a tiny negative one).
__device__ inline int sturm_below(const double* d, const double* e2, int n, double y) {
  double q = d[0] - y;
  if (fabs(q) < 1e-300) q = -1e-300;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - y) - e2[i - 1] / q;
    if (fabs(q) < 1e-300) q = -1e-300;
    cnt += q < 0.0;
  }
  return cnt;
}

// MCC of the GLCM pass: spectral radius of B = D^-1/2 P D^-1/2 - v v^T over
// the n present levels (v = sqrt(px)).  Householder tridiagonalisation with
// thread j owning column j of B in `mat` (row stride ns), then 4 rounds of
// 257-way Sturm multisection of [0, min(Gershgorin bound, 1)].
__device__ double gmcc(GSmem& sm, const uint32_t* glcm, int L, double* mat, int ns, int n, long long NP) {
  const int t = threadIdx.x;
  const double invN = 1.0 / (double)NP;
  // sqrt of the row sums of the present levels
  if (t < n) {
    const double r = sqrt((double)sm.pxc[sm.pl[t]]);
    sm.va[t] = r;
    sm.vb[t] = 1.0 / r;
  }
  __syncthreads();
  if (t < n) {
    const int pj = sm.pl[t];
    const double rj = sm.va[t], irj = sm.vb[t];
    for (int i = 0; i < n; ++i) {
      const int pi = sm.pl[i];
      const uint32_t P = gld(&glcm[pi < pj ? pi * L + pj : pj * L + pi]);
      mat[(size_t)i * ns + t] = (double)P * (sm.vb[i] * irj) - sm.va[i] * rj * invN;
    }
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const double x = (t > k && t < n) ? mat[(size_t)k * ns + t] : 0.0;
    double r1[1] = {x * x};
    bsum(sm, r1);
    const double a2 = r1[0];
    if (t == k + 1) sm.dv[0] = x;
    __syncthreads();
    const double x0 = sm.dv[0];
    const double alpha = a2 == 0.0 ? 0.0 : (x0 >= 0.0 ? -sqrt(a2) : sqrt(a2));
    const double beta = a2 == 0.0 ? 0.0 : 1.0 / (a2 - x0 * alpha);
    const double v = t == k + 1 ? x0 - alpha : x;
    sm.va[t] = v;  // zero for t <= k and t >= n
    if (t == 0) sm.ve[k] = alpha;
    __syncthreads();
    double p = 0.0;
    if (t > k && t < n) {
      for (int i = k + 1; i < n; ++i) p += mat[(size_t)i * ns + t] * sm.va[i];
      p *= beta;
    }
    double r2[1] = {v * p};
    bsum(sm, r2);
    const double Kc = 0.5 * beta * r2[0];
    const double q = (t > k && t < n) ? p - Kc * v : 0.0;
    sm.vb[t] = q;
    __syncthreads();
    if (t > k && t < n)
      for (int i = k + 1; i < n; ++i)
        mat[(size_t)i * ns + t] -= sm.va[i] * q + sm.vb[i] * v;
    __syncthreads();
  }
  // tridiagonal: d_i = B[i][i], e_k (k < n - 2) from the steps, e_{n-2} = B[n-1][n-2]
  double dl = 0.0;
  if (t < n) dl = mat[(size_t)t * ns + t];
  if (t == n - 2) sm.ve[n - 2] = mat[(size_t)(n - 1) * ns + t];
  __syncthreads();
  const double el = t < n - 1 ? sm.ve[t] : 0.0;
  const double em = (t >= 1 && t < n) ? sm.ve[t - 1] : 0.0;
  const double gl = t < n ? fabs(dl) + fabs(el) + fabs(em) : 0.0;
  const double gb = bmax(sm, gl);
  if (t < n) {
    sm.va[t] = dl;
    sm.vb[t] = el * el;
  }
  __syncthreads();
  double lo = 0.0, hi = fmin(gb, 1.0) * (1.0 + 1e-12) + 1e-300;
  for (int round = 0; round < 4; ++round) {
    const double x = lo + (hi - lo) * ((double)(t + 1) / (double)(NT + 1));
    const int c = sturm_below(sm.va, sm.vb, n, x) - sturm_below(sm.va, sm.vb, n, -x);
    if (t == 0) sm.iv[2] = NT;
    __syncthreads();
    if (c == n) atomicMin(&sm.iv[2], t);
    __syncthreads();
    const int b = sm.iv[2];
    __syncthreads();
    if (b == NT) {
      lo = lo + (hi - lo) * ((double)NT / (double)(NT + 1));
    } else {
      const double xb = lo + (hi - lo) * ((double)(b + 1) / (double)(NT + 1));
      const double xa = b > 0 ? lo + (hi - lo) * ((double)b / (double)(NT + 1)) : lo;
      hi = xb;
      lo = xa;
    }
  }
  return 0.5 * (lo + hi);
}

// Bitonic sort of cr[0 .. ns) (ns a power of two) in LDS.
__device__ inline void bsort(float* cr, int ns) {
  for (int k = 2; k <= ns; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < ns; i += NT) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const float a = cr[i], b = cr[p];
          if ((a > b) == up) {
            cr[i] = b;
            cr[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

struct GCtx {
  int R, S, C, L, K, ng, dist, alpha;
  bool averaged;
  uint32_t fam;
};

// Cube index of (x, y, z) or -1 outside the cube.
__device__ inline int cidx(const GCtx& g, int x, int y, int z) {
  return (x < 0 || y < 0 || z < 0 || x >= g.S || y >= g.S || z >= g.S) ? -1 : (z * g.S + y) * g.S + x;
}

// GLCM features of the current pass (tables in glcm / pxc) into f[24];
// returns false when the pass has no voxel pair (features undefined).
__device__ bool glcm_pass_features(GSmem& sm, const GCtx& g, const uint32_t* glcm, double* mat,
                                   int ns, double* f) {
  const int t = threadIdx.x, L = g.L;
  long long rowc = 0, s1x = 0, s2x = 0, nl = 0;
  double hxp = 0.0;
  if (t < L) {
    rowc = sm.pxc[t];
    const int lv = sm.lval[t];
    s1x = rowc * lv;
    s2x = rowc * lv * lv;
    nl = rowc > 0;
    if (rowc) hxp = (double)rowc * flog2((double)rowc);
  }
  long long ri[4] = {rowc, s1x, s2x, nl};
  bsuml(sm, ri);
  const long long NP = ri[0], S1x = ri[1], S2x = ri[2];
  const int nlev = (int)ri[3];
  if (NP == 0) return false;
  // compact list of the present levels (increasing compact index)
  {
    int tot = 0;
    const int pre = bscan(sm, (t < L && rowc > 0) ? 1 : 0, &tot);
    if (t < L && rowc > 0) sm.pl[pre] = t;
  }
  for (int e = t; e < g.ng; e += NT) sm.pd[e] = 0;
  for (int e = t; e <= 2 * g.ng; e += NT) sm.ps[e] = 0;
  __syncthreads();
  const double Nd = (double)NP, lgN = flog2(Nd);
  long long e2 = 0;
  double plogp = 0.0, pmax = 0.0;
  for (int e = t; e < L * L; e += NT) {
    const int r = e / L, c = e % L;
    if (r > c) continue;
    const uint32_t P = gld(&glcm[e]);
    if (!P) continue;
    const uint32_t w = r == c ? 1u : 2u;
    e2 += (long long)(w * P) * P;
    plogp += (double)w * ((double)P * flog2((double)P));
    pmax = fmax(pmax, (double)P);
    const int i = sm.lval[r], j = sm.lval[c];
    atomicAdd(&sm.pd[i > j ? i - j : j - i], w * P);
    atomicAdd(&sm.ps[i + j], w * P);
  }
  const double pm = bmax(sm, pmax);
  double gd[2] = {hxp, plogp};
  bsum(sm, gd);
  const double HX = lgN - gd[0] / Nd;
  plogp = gd[1];
  const double mu = (double)S1x / Nd;
  long long sd1 = 0, sd2 = 0, ss1 = 0, ss2 = 0;
  double dlog = 0, slog = 0, iv = 0, idm = 0, idmn = 0, id = 0, idn = 0, ct = 0, cs = 0, cp = 0;
  const double ngd = (double)g.ng;
  for (int k = t; k < g.ng; k += NT) {
    const uint32_t c = sm.pd[k];
    if (c) {
      const double cd = (double)c, kd = (double)k;
      sd1 += (long long)c * k;
      sd2 += (long long)c * k * k;
      dlog += cd * flog2(cd);
      if (k > 0) iv += cd / (kd * kd);
      idm += cd / (1.0 + kd * kd);
      idmn += cd / (1.0 + kd * kd / (ngd * ngd));
      id += cd / (1.0 + kd);
      idn += cd / (1.0 + kd / ngd);
    }
  }
  for (int k = 2 + t; k <= 2 * g.ng; k += NT) {
    const uint32_t c = sm.ps[k];
    if (c) {
      const double cd = (double)c, tt = (double)k - 2.0 * mu;
      ss1 += (long long)c * k;
      ss2 += (long long)c * k * k;
      slog += cd * flog2(cd);
      ct += cd * tt * tt;
      cs += cd * tt * tt * tt;
      cp += cd * tt * tt * tt * tt;
    }
  }
  long long hl[5] = {sd1, sd2, ss1, ss2, e2};
  bsuml(sm, hl);
  sd1 = hl[0]; sd2 = hl[1]; ss1 = hl[2]; ss2 = hl[3]; e2 = hl[4];
  double hd[10] = {dlog, slog, iv, idm, idmn, id, idn, ct, cs, cp};
  bsum(sm, hd);
  dlog = hd[0]; slog = hd[1]; iv = hd[2]; idm = hd[3]; idmn = hd[4]; id = hd[5]; idn = hd[6];
  ct = hd[7]; cs = hd[8]; cp = hd[9];
  const long long sij = (ss2 - sd2) / 4;  // sum_ij i j P
  const double HXY = lgN - plogp / Nd;
  const double mcc = nlev > 1 ? gmcc(sm, glcm, L, mat, ns, nlev, NP) : 1.0;
  f[0] = (double)sij / Nd;
  f[1] = mu;
  f[2] = cp / Nd;
  f[3] = cs / Nd;
  f[4] = ct / Nd;
  f[5] = (double)sd2 / Nd;
  f[6] = nlev <= 1 ? 1.0 : (double)(NP * sij - S1x * S1x) / (double)(NP * S2x - S1x * S1x);
  f[7] = (double)sd1 / Nd;
  f[8] = lgN - dlog / Nd;
  f[9] = (double)(NP * sd2 - sd1 * sd1) / (Nd * Nd);
  f[10] = (double)e2 / (Nd * Nd);
  f[11] = HXY;
  f[12] = nlev <= 1 ? 0.0 : (HXY - 2.0 * HX) / HX;
  const double tq = 1.0 - exp(-2.0 * (2.0 * HX - HXY));
  f[13] = sqrt(tq > 0.0 ? tq : 0.0);
  f[14] = idm / Nd;
  f[15] = mcc;
  f[16] = idmn / Nd;
  f[17] = id / Nd;
  f[18] = idn / Nd;
  f[19] = iv / Nd;
  f[20] = pm / Nd;
  f[21] = (double)ss1 / Nd;
  f[22] = lgN - slog / Nd;
  f[23] = (double)(NP * S2x - S1x * S1x) / (Nd * Nd);
  return true;
}

template <typename T>
__device__ void gmap_voxel(GSmem& sm, const MapArgs& a, int32_t lin, int64_t it, char* scratch,
                           int lcap, const GLayout& lay) {
  const int t = threadIdx.x;
  GCtx g;
  g.R = a.radius;
  g.S = 2 * g.R + 1;
  g.C = g.S * g.S * g.S;
  g.ng = a.ng;
  g.dist = a.opt.glcm_dist;
  g.alpha = a.opt.gldm_alpha;
  g.averaged = a.opt.averaged != 0;
  g.fam = a.families;
  const T* __restrict__ vol = (const T*)a.vol;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int cx = lin % nx, cy = (lin / nx) % ny, cz = lin / (nx * ny);
  uint32_t* glcm = (uint32_t*)(scratch + lay.glcm);
  uint32_t* glrlm = (uint32_t*)(scratch + lay.glrlm);
  uint32_t* gldm = (uint32_t*)(scratch + lay.gldm);
  uint32_t* zps = (uint32_t*)(scratch + lay.zps);
  uint32_t* hkey = (uint32_t*)(scratch + lay.hkey);
  uint32_t* hcnt = (uint32_t*)(scratch + lay.hcnt);
  double* mat = (double*)(scratch + lay.mat);
  const bool debug = a.d_glcm != nullptr;
  const int S = g.S, C = g.C;

  // ---- gather ---------------------------------------------------------
  int kloc = 0;
  int ns_sort = 64;
  while (ns_sort < C) ns_sort <<= 1;
  for (int c = t; c < ns_sort; c += NT) {
    int lev = 0;
    float xr = INFINITY;
    if (c < C) {
      const int x = c % S, y = (c / S) % S, z = c / (S * S);
      const int gx = cx + x - g.R, gy = cy + y - g.R, gz = cz + z - g.R;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
        const int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
        lev = a.levels[gi];
        if (lev) {
          xr = (float)vol[gi];
          sm.lflag[lev] = 1;
          kloc++;
        }
      }
      sm.cl[c] = (uint8_t)lev;
      sm.lab[c] = (uint32_t)c;
      sm.zcnt[c] = 0;
    }
    sm.cr[c] = xr;
  }
  __syncthreads();
  {
    long long kk[1] = {kloc};
    bsuml(sm, kk);
    g.K = (int)kk[0];
  }
  // ---- local level compaction -----------------------------------------
  {
    const int f = sm.lflag[t] != 0;
    int tot = 0;
    const int pre = bscan(sm, f, &tot);
    if (f) {
      sm.lmap[t] = (uint8_t)pre;
      sm.lval[pre] = (uint8_t)t;
    }
    g.L = tot;
    sm.lflag[t] = 0;
  }
  const int L = g.L;
  const int count = a.count;
  if (L > lcap) {  // cannot happen for a launch sized by the host; write NaN
    for (int k = t; k < count; k += NT) sm.feat[k] = NAN;
    __syncthreads();
  } else {
    // clear the tables
    for (int e = t; e < L * 27; e += NT) gzero(&gldm[e]);
    for (int e = t; e < C; e += NT) gzero(&zps[e]);
    for (int e = t; e < HTG; e += NT) {
      gzero(&hkey[e]);
      gzero(&hcnt[e]);
    }
    if (t < L) {
      sm.hist[t] = 0;
      sm.ngn[t] = 0;
      sm.ngS[t] = 0ull;
      sm.zpl[t] = 0;
    }
    __syncthreads();

    // ---- counting pass: histogram, equal-level bits, GLDM, NGTDM, moments
    double s1 = 0.0, s2 = 0.0;
    for (int c = t; c < C; c += NT) {
      const int lev = sm.cl[c];
      if (!lev) continue;
      const int x = c % S, y = (c / S) % S, z = c / (S * S);
      const int l = sm.lmap[lev];
      uint32_t same = 0;
      int cnt = 0, lsum = 0, dep = 0;
      for (int nb = 0; nb < 26; ++nb) {
        const int u = cidx(g, x + ndx(nb), y + ndy(nb), z + ndz(nb));
        const int h = u >= 0 ? sm.cl[u] : 0;
        if (!h) continue;
        cnt++;
        lsum += h;
        if (h == lev) same |= 1u << nb;
        if (abs(h - lev) <= g.alpha) dep++;
      }
      sm.same[c] = same;
      atomicAdd(&sm.hist[l], 1u);
      if (g.fam & 16u) atomicAdd(&gldm[l * 27 + dep], 1u);
      if ((g.fam & 32u) && cnt) {
        atomicAdd(&sm.ngn[l], 1u);
        const int dd = lev * cnt - lsum;
        atomicAdd(&sm.ngS[l], (unsigned long long)(dd < 0 ? -dd : dd) * kLcmOver[cnt]);
      }
      const double xr = (double)sm.cr[c];
      s1 += xr;
      s2 += xr * xr;
    }
    __syncthreads();

    // ---- zones: minimum-label propagation over equal-level neighbours ---
    if (g.fam & 8u) {
      for (;;) {
        if (t == 0) sm.iv[0] = 0;
        __syncthreads();
        for (int c = t; c < C; c += NT) {
          if (!sm.cl[c]) continue;
          const uint32_t sb = sm.same[c];
          const int x = c % S, y = (c / S) % S, z = c / (S * S);
          uint32_t m = sm.lab[c];
          for (int nb = 0; nb < 26; ++nb)
            if ((sb >> nb) & 1u) m = min(m, sm.lab[cidx(g, x + ndx(nb), y + ndy(nb), z + ndz(nb))]);
          m = min(m, sm.lab[m]);
          const uint32_t cur = sm.lab[c];
          if (m < cur) {
            atomicMin(&sm.lab[c], m);
            atomicMin(&sm.lab[cur], m);
            sm.iv[0] = 1;
          }
        }
        __syncthreads();
        const int changed = sm.iv[0];
        __syncthreads();
        if (!changed) break;
      }
      for (int c = t; c < C; c += NT)
        if (sm.cl[c]) atomicAdd(&sm.zcnt[sm.lab[c]], 1u);
    }
    // order statistics
    if (g.fam & 1u) {
      __syncthreads();
      bsort(sm.cr, ns_sort);
    }
    __syncthreads();

    // ---- zones: per root ------------------------------------------------
    GEmph ez = {};
    if (g.fam & 8u) {
      for (int c = t; c < C; c += NT) {
        const int lev = sm.cl[c];
        if (!lev || sm.lab[c] != (uint32_t)c) continue;
        const int s = (int)sm.zcnt[c];
        const int l = sm.lmap[lev];
        gemph_add(ez, 1, lev, s);
        atomicAdd(&sm.zpl[l], 1u);
        atomicAdd(&zps[s - 1], 1u);
        const uint32_t key = ((uint32_t)l << 16 | (uint32_t)s) + 1u;
        uint32_t h = (key * 2654435761u) >> 20;  // 12 bits: HTG = 4096
        for (;;) {
          const uint32_t old = atomicCAS(&hkey[h], 0u, key);
          if (old == 0u || old == key) {
            atomicAdd(&hcnt[h], 1u);
            break;
          }
          h = (h + 1) & (HTG - 1);
        }
        if (debug) atomicAdd(&a.d_glszm[it * (int64_t)g.ng * C + (int64_t)(lev - 1) * C + (s - 1)], 1);
      }
    }
    __syncthreads();
    if (debug) {
      const int ng = g.ng;
      for (int e = t; e < L * 27; e += NT)
        a.d_gldm[it * ng * 27 + (int64_t)(sm.lval[e / 27] - 1) * 27 + e % 27] = (int32_t)gld(&gldm[e]);
      if (t < L) {
        const int64_t o = it * ng + (sm.lval[t] - 1);
        a.d_ngn[o] = (int32_t)sm.ngn[t];
        a.d_ngS[o] = (int64_t)sm.ngS[t];
        a.d_hist[o] = (int32_t)sm.hist[t];
      }
    }

    int off = 0;
    const int oFO = off;    off += (g.fam & 1u) ? 18 : 0;
    const int oGLCM = off;  off += (g.fam & 2u) ? 24 : 0;
    const int oGLRLM = off; off += (g.fam & 4u) ? 16 : 0;
    const int oGLSZM = off; off += (g.fam & 8u) ? 16 : 0;
    const int oGLDM = off;  off += (g.fam & 16u) ? 14 : 0;
    const int oNGTDM = off;
    const double Kd = (double)g.K;
    double f[24];

    // ---- first order ----------------------------------------------------
    if (g.fam & 1u) {
      const int K = g.K;
      double ent = 0.0, uni = 0.0;
      if (t < L) {
        const double p = (double)sm.hist[t] / Kd;
        ent = -p * flog2(p);
        uni = p * p;
      }
      double r1[4] = {s1, s2, ent, uni};
      bsum(sm, r1);
      const double S1 = r1[0], S2 = r1[1];
      const double mu = S1 / Kd;
      const float* srt = sm.cr;
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
      const double p10 = pct(0.10), p25 = pct(0.25), p50 = pct(0.50), p75 = pct(0.75), p90 = pct(0.90);
      double m[6] = {0, 0, 0, 0, 0, 0};
      for (int e = t; e < K; e += NT) {
        const double x = srt[e], d = x - mu, d2 = d * d;
        m[0] += d2;
        m[1] += d2 * d;
        m[2] += d2 * d2;
        m[3] += fabs(d);
        if (x >= p10 && x <= p90) {
          m[4] += x;
          m[5] += 1.0;
        }
      }
      bsum(sm, m);
      const double m2 = m[0] / Kd, m3 = m[1] / Kd, m4 = m[2] / Kd, mad = m[3] / Kd;
      double rmad = NAN;
      if (m[5] > 0.0) {
        const double rmu = m[4] / m[5];
        double acc[1] = {0.0};
        for (int e = t; e < K; e += NT) {
          const double x = srt[e];
          if (x >= p10 && x <= p90) acc[0] += fabs(x - rmu);
        }
        bsum(sm, acc);
        rmad = acc[0] / m[5];
      }
      const bool flat = mn == mx;
      if (t == 0) {
        float* F = sm.feat + oFO;
        F[0] = (float)S2;
        F[1] = (float)(a.voxel_volume * S2);
        F[2] = (float)r1[2];
        F[3] = (float)mn;
        F[4] = (float)p10;
        F[5] = (float)p90;
        F[6] = (float)mx;
        F[7] = (float)mu;
        F[8] = (float)p50;
        F[9] = (float)(p75 - p25);
        F[10] = (float)(mx - mn);
        F[11] = (float)mad;
        F[12] = (float)rmad;
        F[13] = (float)sqrt(S2 / Kd);
        F[14] = flat ? 0.f : (float)(m3 / (m2 * sqrt(m2)));
        F[15] = flat ? 0.f : (float)(m4 / (m2 * m2) - 3.0);
        F[16] = (float)m2;
        F[17] = (float)r1[3];
      }
    }

    // ---- GLSZM ----------------------------------------------------------
    if (g.fam & 8u) {
      double hl = 0.0;
      for (int e = t; e < HTG; e += NT) {
        const uint32_t c = gld(&hcnt[e]);
        if (c > 1) hl += (double)c * flog2((double)c);
      }
      ez.clogc = hl;
      long long gln = 0, szn = 0;
      if (t < L) gln = (long long)sm.zpl[t] * sm.zpl[t];
      for (int e = t; e < C; e += NT) {
        const long long z = gld(&zps[e]);
        szn += z * z;
      }
      gemph_reduce(sm, ez, gln, szn);
      gemph16(ez, gln, szn, Kd, f);
      if (t == 0)
        for (int k = 0; k < 16; ++k) sm.feat[oGLSZM + k] = (float)f[k];
    }

    // ---- GLDM -----------------------------------------------------------
    if (g.fam & 16u) {
      GEmph ed = {};
      for (int e = t; e < L * 27; e += NT) {
        const uint32_t c = gld(&gldm[e]);
        if (c) gemph_add(ed, c, sm.lval[e / 27], e % 27 + 1);
      }
      long long gln = 0, dn = 0;
      if (t < L) gln = (long long)sm.hist[t] * sm.hist[t];
      if (t < 27) {
        long long s = 0;
        for (int l = 0; l < L; ++l) s += gld(&gldm[l * 27 + t]);
        dn = s * s;
      }
      gemph_reduce(sm, ed, gln, dn);
      const double N = (double)ed.n;
      if (t == 0) {
        float* F = sm.feat + oGLDM;
        F[0] = (float)(ed.invj2 / N);
        F[1] = (float)((double)ed.sj2 / N);
        F[2] = (float)((double)gln / N);
        F[3] = (float)((double)dn / N);
        F[4] = (float)((double)dn / (N * N));
        F[5] = (float)((double)(ed.n * ed.si2 - ed.si * ed.si) / (N * N));
        F[6] = (float)((double)(ed.n * ed.sj2 - ed.sj * ed.sj) / (N * N));
        F[7] = (float)(flog2(N) - ed.clogc / N);
        F[8] = (float)(ed.invi2 / N);
        F[9] = (float)((double)ed.si2 / N);
        F[10] = (float)(ed.invi2j2 / N);
        F[11] = (float)(ed.i2invj2 / N);
        F[12] = (float)(ed.j2invi2 / N);
        F[13] = (float)((double)ed.si2j2 / N);
      }
    }

    // ---- NGTDM ----------------------------------------------------------
    if (g.fam & 32u) {
      long long vi[7] = {0, 0, 0, 0, 0, 0, 0};
      double vs[3] = {0.0, 0.0, 0.0};
      if (t < L) {
        const long long ni = sm.ngn[t];
        const int il = sm.lval[t];
        const double si = (double)sm.ngS[t] * kRcpLcm26;
        vi[0] = ni;
        if (ni) {
          vi[1] = 1;
          vi[2] = il;
          vi[3] = (long long)il * il;
          vi[6] = sm.ngS[t] != 0ull;
        }
        vi[4] = ni * il;
        vi[5] = ni * il * il;
        vs[0] = si;
        vs[1] = (double)ni * si;
      }
      long long bden = 0;
      double cplx = 0.0;
      for (int e = t; e < L * L; e += NT) {
        const int i = e / L, j = e % L;
        if (i >= j) continue;
        const long long ni = sm.ngn[i], nj = sm.ngn[j];
        if (!ni || !nj) continue;
        const int il = sm.lval[i], jl = sm.lval[j];
        const long long tt = (long long)il * ni - (long long)jl * nj;
        bden += 2 * (tt < 0 ? -tt : tt);
        const double si = (double)sm.ngS[i] * kRcpLcm26, sj = (double)sm.ngS[j] * kRcpLcm26;
        cplx += 2.0 * fabs((double)(il - jl)) * ((double)ni * si + (double)nj * sj) / (double)(ni + nj);
      }
      long long rl[8] = {vi[0], vi[1], vi[2], vi[3], vi[4], vi[5], vi[6], bden};
      bsuml(sm, rl);
      vs[2] = cplx;
      bsum(sm, vs);
      const long long Nvc = rl[0];
      if (t == 0) {
        float* F = sm.feat + oNGTDM;
        if (Nvc == 0) {
          for (int k = 0; k < 5; ++k) F[k] = NAN;
        } else {
          const long long Ngp = rl[1], A1 = rl[2], A2 = rl[3], Sn1 = rl[4], Sn2 = rl[5];
          const bool any_s = rl[6] != 0;
          const double ssum = vs[0], Nd = (double)Nvc, psum = vs[1] / Nd;
          const double c1 = 2.0 * (double)(Nvc * Sn2 - Sn1 * Sn1) / (Nd * Nd);
          const double strn = 2.0 * (double)(Ngp * Sn2 - 2 * A1 * Sn1 + A2 * Nvc) / Nd;
          F[0] = any_s ? (float)(1.0 / psum) : 1e6f;
          F[1] = Ngp <= 1 ? 0.f : (float)(c1 / (double)(Ngp * (Ngp - 1)) * (ssum / Nd));
          F[2] = rl[7] == 0 ? 0.f : (float)(psum / ((double)rl[7] / Nd));
          F[3] = (float)(vs[2] / Nd);
          F[4] = any_s ? (float)(strn / ssum) : 0.f;
        }
      }
    }

    // ---- GLRLM: merged (one pass over the 13 directions) or averaged ----
    if (g.fam & 4u) {
      const int passes = g.averaged ? 13 : 1;
      double acc[16];
      for (int k = 0; k < 16; ++k) acc[k] = 0.0;
      for (int pass = 0; pass < passes; ++pass) {
        const int d0 = g.averaged ? pass : 0, d1 = g.averaged ? pass + 1 : 13;
        for (int e = t; e < L * S; e += NT) gzero(&glrlm[e]);
        __syncthreads();
        for (int c = t; c < C; c += NT) {
          const int lev = sm.cl[c];
          if (!lev) continue;
          const int x = c % S, y = (c / S) % S, z = c / (S * S);
          const int l = sm.lmap[lev];
          for (int d = d0; d < d1; ++d) {
            const int up = cidx(g, x - fdx(d), y - fdy(d), z - fdz(d));
            if (up >= 0 && sm.cl[up] == lev) continue;  // not the start of a run
            int len = 1, px = x + fdx(d), py = y + fdy(d), pz = z + fdz(d);
            for (;;) {
              const int u = cidx(g, px, py, pz);
              if (u < 0 || sm.cl[u] != lev) break;
              len++;
              px += fdx(d);
              py += fdy(d);
              pz += fdz(d);
            }
            atomicAdd(&glrlm[l * S + len - 1], 1u);
          }
        }
        __syncthreads();
        GEmph er = {};
        for (int e = t; e < L * S; e += NT) {
          const uint32_t c = gld(&glrlm[e]);
          if (c) {
            gemph_add(er, c, sm.lval[e / S], e % S + 1);
            if (debug) atomicAdd(&a.d_glrlm[it * g.ng * S + (int64_t)(sm.lval[e / S] - 1) * S + e % S], (int)c);
          }
        }
        long long gln = 0, rln = 0;
        if (t < L) {
          long long s = 0;
          for (int j = 0; j < S; ++j) s += gld(&glrlm[t * S + j]);
          gln = s * s;
        }
        if (t < S) {
          long long s = 0;
          for (int l = 0; l < L; ++l) s += gld(&glrlm[l * S + t]);
          rln = s * s;
        }
        gemph_reduce(sm, er, gln, rln);
        gemph16(er, gln, rln, (double)(d1 - d0) * Kd, f);
        for (int k = 0; k < 16; ++k) acc[k] += f[k];
        __syncthreads();
      }
      if (t == 0)
        for (int k = 0; k < 16; ++k) sm.feat[oGLRLM + k] = (float)(acc[k] / (double)passes);
    }

    // ---- GLCM: merged (one pass) or averaged over the directions with pairs
    if (g.fam & 2u) {
      const int passes = g.averaged ? 13 : 1;
      double acc[24];
      for (int k = 0; k < 24; ++k) acc[k] = 0.0;
      int defined = 0;
      const int dist = g.dist;
      for (int pass = 0; pass < passes; ++pass) {
        const int d0 = g.averaged ? pass : 0, d1 = g.averaged ? pass + 1 : 13;
        for (int e = t; e < L * L; e += NT) gzero(&glcm[e]);
        if (t < L) sm.pxc[t] = 0;
        __syncthreads();
        for (int c = t; c < C; c += NT) {
          const int lev = sm.cl[c];
          if (!lev) continue;
          const int x = c % S, y = (c / S) % S, z = c / (S * S);
          const int l = sm.lmap[lev];
          for (int d = d0; d < d1; ++d) {
            const int u = cidx(g, x + dist * fdx(d), y + dist * fdy(d), z + dist * fdz(d));
            const int h = u >= 0 ? sm.cl[u] : 0;
            if (!h) continue;
            const int lh = sm.lmap[h];
            if (lh == l) {
              atomicAdd(&glcm[l * L + l], 2u);
              atomicAdd(&sm.pxc[l], 2u);
            } else {
              atomicAdd(&glcm[l < lh ? l * L + lh : lh * L + l], 1u);
              atomicAdd(&sm.pxc[l], 1u);
              atomicAdd(&sm.pxc[lh], 1u);
            }
          }
        }
        __syncthreads();
        if (debug) {
          const int ng = g.ng;
          for (int e = t; e < L * L; e += NT) {
            const int r = e / L, c = e % L;
            const uint32_t P = gld(&glcm[r <= c ? e : c * L + r]);
            if (P) atomicAdd(&a.d_glcm[it * ng * ng + (int64_t)(sm.lval[r] - 1) * ng + (sm.lval[c] - 1)], (int)P);
          }
        }
        const bool ok = glcm_pass_features(sm, g, glcm, mat, lcap, f);
        if (ok) {
          defined++;
          for (int k = 0; k < 24; ++k) acc[k] += f[k];
        }
        __syncthreads();
      }
      if (t == 0)
        for (int k = 0; k < 24; ++k)
          sm.feat[oGLCM + k] = defined ? (float)(acc[k] / (double)defined) : NAN;
    }
  }
  __syncthreads();
  if (a.stage) {
    float* row = a.stage + it * kStageStride;
    for (int k = t; k < count; k += NT) row[k] = sm.feat[k];
  } else {
    for (int k = t; k < count; k += NT) a.out[(int64_t)k * a.n_out + it] = sm.feat[k];
  }
  __syncthreads();
}

// The job's MapArgs from the batch job table.
__device__ inline MapArgs job_args(const BatchJob& J, const DiscParams* P) {
  MapArgs a = {};
  a.params = P;
  a.vol = J.vol;
  a.levels = J.levels;
  a.list = J.list;
  a.out = J.out;
  a.stage = J.stage;
  a.n_out = J.n_mask;
  a.n_items = J.n_mask;
  a.n_list = J.n_mask;
  a.nx = J.nx;
  a.ny = J.ny;
  a.nz = J.nz;
  a.ng = P->ng;
  a.families = J.families;
  a.count = J.count;
  a.voxel_volume = J.voxel_volume;
  a.radius = J.radius;
  a.opt = J.opt;
  return a;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_map_generic(MapArgs one, const BatchJob* __restrict__ jobs,
                                                    const DiscParams* __restrict__ params,
                                                    const int2* __restrict__ items,
                                                    const int32_t* __restrict__ n_items_dev,
                                                    int32_t n_items_host, char* scratch,
                                                    size_t per_wg, int lcap) {
  __shared__ GSmem sm;
  const int t = threadIdx.x;
  sm.lflag[t] = 0;
  __syncthreads();
  const GLayout lay = glayout(lcap);
  char* slice = scratch + (size_t)blockIdx.x * per_wg;
  const int64_t n = n_items_dev ? (int64_t)*n_items_dev : (int64_t)n_items_host;
  const int64_t i0 = (int64_t)blockIdx.x * n / gridDim.x;
  const int64_t i1 = ((int64_t)blockIdx.x + 1) * n / gridDim.x;
  for (int64_t k = i0; k < i1; ++k) {
    const int2 item = items ? items[k] : make_int2(0, (int)k);
    MapArgs a;
    if (jobs) {
      const DiscParams* P = &params[item.x];
      if (P->err != kJobOk) continue;
      a = job_args(jobs[item.x], P);
    } else {
      if (one.params->err != kJobOk) return;
      a = one;
      a.ng = one.params->ng;
    }
    const int64_t it = item.y;
    const int64_t m = a.sample ? a.sample[it] : it;
    if (m < 0 || m >= a.n_list) {  // out-of-range sample index: NaN maps, no matrices
      for (int q = t; q < a.count; q += NT) a.out[(int64_t)q * a.n_out + it] = NAN;
      continue;
    }
    gmap_voxel<T>(sm, a, a.list[m], it, slice, lcap, lay);
  }
}

}  // namespace

size_t generic_scratch_bytes(int lcap) { return glayout(lcap < 1 ? 1 : lcap).total; }

hipError_t launch_map_generic(const MapArgs& a, const BatchJob* jobs, const DiscParams* params,
                              const int2* items, const int32_t* n_items_dev, int32_t n_items,
                              int dtype, void* scratch, int lcap, int grid, hipStream_t st) {
  if (!n_items_dev && n_items <= 0) return hipSuccess;
  if (lcap < 1 || lcap > 255 || grid < 1) return hipErrorInvalidValue;
  const size_t scratch_per_wg = generic_scratch_bytes(lcap);
  if (dtype == 1)
    hipLaunchKernelGGL(k_map_generic<int16_t>, dim3((unsigned)grid), dim3(NT), 0, st, a, jobs, params,
                       items, n_items_dev, n_items, (char*)scratch, scratch_per_wg, lcap);
  else
    hipLaunchKernelGGL(k_map_generic<float>, dim3((unsigned)grid), dim3(NT), 0, st, a, jobs, params,
                       items, n_items_dev, n_items, (char*)scratch, scratch_per_wg, lcap);
  return hipGetLastError();
}

}  // namespace fr
