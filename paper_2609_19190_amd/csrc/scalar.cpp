// Whole-VOI ("scalar") radiomic features on the host, in FP64.
//
// The paper runs scalar extraction on the CPU, where it measured it faster
// than its GPU backend (Results, scalar benchmark; Discussion): one VOI is
// one neighbourhood, so there is no per-voxel parallelism to exploit.  The
// features are those of the spatial maps with the neighbourhood taken to be
// the whole mask: V = {voxels with mask != 0}, texture relations restricted
// to V, the 13 directions merged, 26-connected zones, GLDM alpha = 0, NGTDM
// over the 26-neighbours in V of voxels that have at least one.  A map value
// at a voxel whose cube covers the VOI therefore equals the scalar value.
//
// Matrices are counted exactly in integers (NGTDM s_i as an exact multiple
// of 1 / lcm(1..26)); features are FP64 sums over the present entries.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_error.h"

namespace {


fr_status cfail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status cfail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fr::set_error(buf);
  return code;
}

// One representative of each +- pair of the 26 unit offsets.
const int kDir[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},   {1, 1, 0},  {1, -1, 0},
                         {1, 0, 1},  {1, 0, -1}, {0, 1, 1},   {0, 1, -1}, {1, 1, 1},
                         {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

constexpr int64_t kLcm = 26771144400LL;  // lcm(1, ..., 26)

struct Grid {
  int nx, ny, nz;
  std::vector<uint8_t> lev;  // level per voxel, 0 outside V
  bool inside(int x, int y, int z) const {
    return x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
  }
  int64_t at(int x, int y, int z) const { return ((int64_t)z * ny + y) * nx + x; }
  int level(int x, int y, int z) const { return inside(x, y, z) ? lev[at(x, y, z)] : 0; }
};

double plog2p(double p) { return p > 0.0 ? p * log2(p) : 0.0; }

// ---- discretisation (IBSI fixed bin number / width, FP64, no contraction)
int discretise(const std::vector<double>& x, int mode, double value, double lower,
               std::vector<uint8_t>& g, int* ng_out) {
#pragma clang fp contract(off)
  const double mn = *std::min_element(x.begin(), x.end());
  const double mx = *std::max_element(x.begin(), x.end());
  g.resize(x.size());
  if (mode == FR_FBN) {
    const int ng = (int)value;
    const double range = mx - mn;
    for (size_t i = 0; i < x.size(); ++i) {
      int q = 1;
      if (range > 0.0) {
        const double t = x[i] - mn;
        q = (int)floor(((double)ng * t) / range) + 1;
        if (q > ng) q = ng;
      }
      g[i] = (uint8_t)q;
    }
    *ng_out = ng;
    return FR_OK;
  }
  const double lo = isfinite(lower) ? lower : mn;
  const double top = floor((mx - lo) / value) + 1.0;
  if (!(top <= 255.0)) return FR_E_RANGE;
  for (size_t i = 0; i < x.size(); ++i) {
    double q = floor((x[i] - lo) / value) + 1.0;
    if (q < 1.0) q = 1.0;
    g[i] = (uint8_t)q;
  }
  *ng_out = top < 1.0 ? 1 : (int)top;
  return FR_OK;
}

// ---- first order -------------------------------------------------------
void first_order(const std::vector<double>& x, const std::vector<uint8_t>& g, int ng,
                 double voxel_volume, double* f) {
  const size_t K = x.size();
  const double Kd = (double)K;
  std::vector<double> s(x);
  std::sort(s.begin(), s.end());
  auto pct = [&](double q) {
    const double h = (Kd - 1.0) * q;
    const size_t i = (size_t)floor(h);
    if (i + 1 >= K) return s[K - 1];
    return s[i] + (h - floor(h)) * (s[i + 1] - s[i]);
  };
  double s1 = 0.0, s2 = 0.0;
  for (double v : x) {
    s1 += v;
    s2 += v * v;
  }
  const double mu = s1 / Kd;
  double m2 = 0, m3 = 0, m4 = 0, mad = 0;
  for (double v : x) {
    const double d = v - mu;
    m2 += d * d;
    m3 += d * d * d;
    m4 += d * d * d * d;
    mad += fabs(d);
  }
  m2 /= Kd;
  m3 /= Kd;
  m4 /= Kd;
  mad /= Kd;
  const double p10 = pct(0.10), p25 = pct(0.25), p50 = pct(0.50), p75 = pct(0.75), p90 = pct(0.90);
  double rsum = 0.0;
  size_t rn = 0;
  for (double v : x)
    if (v >= p10 && v <= p90) {
      rsum += v;
      rn++;
    }
  double rmad = NAN;
  if (rn > 0) {
    const double rmu = rsum / (double)rn;
    double acc = 0.0;
    for (double v : x)
      if (v >= p10 && v <= p90) acc += fabs(v - rmu);
    rmad = acc / (double)rn;
  }
  std::vector<int64_t> h(ng + 1, 0);
  for (uint8_t q : g) h[q]++;
  double ent = 0.0, uni = 0.0;
  for (int i = 1; i <= ng; ++i) {
    const double p = (double)h[i] / Kd;
    ent -= plog2p(p);
    uni += p * p;
  }
  const bool flat = s.front() == s.back();
  f[0] = s2;
  f[1] = voxel_volume * s2;
  f[2] = ent;
  f[3] = s.front();
  f[4] = p10;
  f[5] = p90;
  f[6] = s.back();
  f[7] = mu;
  f[8] = p50;
  f[9] = p75 - p25;
  f[10] = s.back() - s.front();
  f[11] = mad;
  f[12] = rmad;
  f[13] = sqrt(s2 / Kd);
  f[14] = flat ? 0.0 : m3 / pow(m2, 1.5);
  f[15] = flat ? 0.0 : m4 / (m2 * m2) - 3.0;
  f[16] = m2;
  f[17] = uni;
}

// ---- MCC: spectral radius of a symmetric matrix ---------------------------
// Householder reduction to tridiagonal form (a, b), then bisection on the
// Sturm counts of the interval [-x, x) down to the last bit.
double spectral_radius(std::vector<double> A, int n) {
  std::vector<double> a(n), b(n, 0.0), v(n), p(n), w(n);
  auto M = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int k = 0; k + 2 < n; ++k) {
    double s = 0.0;
    for (int i = k + 1; i < n; ++i) s += M(i, k) * M(i, k);
    if (s == 0.0) {
      b[k] = 0.0;
      continue;
    }
    const double x0 = M(k + 1, k);
    const double alpha = x0 >= 0.0 ? -sqrt(s) : sqrt(s);
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = M(i, k);
    const double beta = 1.0 / (s - x0 * alpha);  // 2 / |v|^2
    for (int i = k + 1; i < n; ++i) {
      double acc = 0.0;
      for (int j = k + 1; j < n; ++j) acc += M(i, j) * v[j];
      p[i] = beta * acc;
    }
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) pv += p[i] * v[i];
    const double c = 0.5 * beta * pv;
    for (int i = k + 1; i < n; ++i) w[i] = p[i] - c * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) M(i, j) -= v[i] * w[j] + w[i] * v[j];
    b[k] = alpha;
  }
  for (int i = 0; i < n; ++i) a[i] = M(i, i);
  if (n >= 2) b[n - 2] = M(n - 1, n - 2);
  // eigenvalues below y: sign changes of the ratio sequence
  auto below = [&](double y) {
    int cnt = 0;
    double q = a[0] - y;
    if (q < 0.0) cnt++;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = 1e-300;
      q = (a[i] - y) - b[i - 1] * b[i - 1] / q;
      if (q < 0.0) cnt++;
    }
    return cnt;
  };
  double hi = 0.0;
  for (int i = 0; i < n; ++i)
    hi = std::max(hi, fabs(a[i]) + (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < n ? fabs(b[i]) : 0.0));
  hi = hi * (1.0 + 1e-12) + 1e-300;
  double lo = 0.0;
  // largest |eigenvalue| = the smallest x with every eigenvalue in [-x, x)
  for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (below(mid) - below(-mid) == n)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// ---- GLCM ------------------------------------------------------------------
void glcm_features(const Grid& G, int ng, double* f) {
  std::vector<int64_t> P((size_t)(ng + 1) * (ng + 1), 0);
  auto at = [&](int i, int j) -> int64_t& { return P[(size_t)i * (ng + 1) + j]; };
  for (int z = 0; z < G.nz; ++z)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int a = G.lev[G.at(x, y, z)];
        if (!a) continue;
        for (const auto& d : kDir) {
          const int b = G.level(x + d[0], y + d[1], z + d[2]);
          if (!b) continue;
          at(a, b)++;
          at(b, a)++;
        }
      }
  int64_t NP = 0;
  std::vector<int64_t> row(ng + 1, 0);
  for (int i = 1; i <= ng; ++i)
    for (int j = 1; j <= ng; ++j) {
      NP += at(i, j);
      row[i] += at(i, j);
    }
  if (NP == 0) {
    for (int k = 0; k < 24; ++k) f[k] = NAN;
    return;
  }
  const double N = (double)NP;
  std::vector<int> present;
  for (int i = 1; i <= ng; ++i)
    if (row[i]) present.push_back(i);
  double mu = 0.0, hx = 0.0;
  for (int i = 1; i <= ng; ++i) {
    const double px = (double)row[i] / N;
    mu += i * px;
    hx -= plog2p(px);
  }
  double ac = 0, cp = 0, cs = 0, ct = 0, con = 0, je = 0, jent = 0, pmax = 0, var = 0;
  std::vector<double> pd(ng, 0.0), ps(2 * ng + 1, 0.0);
  for (int i = 1; i <= ng; ++i) {
    var += (i - mu) * (i - mu) * (double)row[i] / N;
    for (int j = 1; j <= ng; ++j) {
      if (!at(i, j)) continue;
      const double p = (double)at(i, j) / N;
      const double t = i + j - 2.0 * mu;
      ac += i * j * p;
      cp += t * t * t * t * p;
      cs += t * t * t * p;
      ct += t * t * p;
      con += (double)(i - j) * (i - j) * p;
      je += p * p;
      jent -= plog2p(p);
      pmax = std::max(pmax, p);
      pd[std::abs(i - j)] += p;
      ps[i + j] += p;
    }
  }
  double da = 0, dent = 0, idm = 0, idmn = 0, id = 0, idn = 0, iv = 0;
  for (int k = 0; k < ng; ++k) {
    const double p = pd[k];
    if (p <= 0.0) continue;
    da += k * p;
    dent -= plog2p(p);
    idm += p / (1.0 + (double)k * k);
    idmn += p / (1.0 + (double)k * k / ((double)ng * ng));
    id += p / (1.0 + k);
    idn += p / (1.0 + (double)k / ng);
    if (k > 0) iv += p / ((double)k * k);
  }
  double dv = 0.0;
  for (int k = 0; k < ng; ++k) dv += (k - da) * (k - da) * pd[k];
  double sa = 0, sent = 0;
  for (int k = 2; k <= 2 * ng; ++k) {
    sa += k * ps[k];
    sent -= plog2p(ps[k]);
  }
  const int nlev = (int)present.size();
  double mcc = 1.0;
  if (nlev > 1) {
    std::vector<double> B((size_t)nlev * nlev);
    for (int a = 0; a < nlev; ++a)
      for (int b = 0; b < nlev; ++b) {
        const double rr = sqrt((double)row[present[a]] * (double)row[present[b]]);
        B[(size_t)a * nlev + b] = (double)at(present[a], present[b]) / rr - rr / N;
      }
    mcc = spectral_radius(B, nlev);
  }
  f[0] = ac;
  f[1] = mu;
  f[2] = cp;
  f[3] = cs;
  f[4] = ct;
  f[5] = con;
  f[6] = nlev <= 1 ? 1.0 : (ac - mu * mu) / var;
  f[7] = da;
  f[8] = dent;
  f[9] = dv;
  f[10] = je;
  f[11] = jent;
  f[12] = nlev <= 1 ? 0.0 : (jent - 2.0 * hx) / hx;
  const double t = 1.0 - exp(-2.0 * (2.0 * hx - jent));
  f[13] = sqrt(t > 0.0 ? t : 0.0);
  f[14] = idm;
  f[15] = mcc;
  f[16] = idmn;
  f[17] = id;
  f[18] = idn;
  f[19] = iv;
  f[20] = pmax;
  f[21] = sa;
  f[22] = sent;
  f[23] = var;
}

// ---- run / zone / dependence families ------------------------------------
// Entries (i, j, c): c runs / zones / voxels of gray level i (1..ng) and
// length / size / dependence j.  Np is the denominator of the percentage
// feature.  The 16 features in the GLRLM / GLSZM order: SE, LE, GLN, GLNN,
// LN, LNN, percentage, GLV, LV, entropy, LGE, HGE, SLGE, SHGE, LLGE, LHGE.
struct Entry {
  int i;
  int64_t j, c;
};

void emphasis(const std::vector<Entry>& E, int ng, double Np, double* f) {
  int64_t Nt = 0;
  std::vector<int64_t> ri(ng + 1, 0);
  std::vector<std::pair<int64_t, int64_t>> cj;  // (j, c), summed per j below
  for (const Entry& e : E) {
    Nt += e.c;
    ri[e.i] += e.c;
    cj.push_back({e.j, e.c});
  }
  std::sort(cj.begin(), cj.end());
  const double N = (double)Nt;
  double se = 0, le = 0, mi = 0, mj = 0, ent = 0, lge = 0, hge = 0, slge = 0, shge = 0, llge = 0, lhge = 0;
  for (const Entry& e : E) {
    const double p = (double)e.c / N, di = e.i, dj = (double)e.j;
    se += p / (dj * dj);
    le += p * dj * dj;
    mi += p * di;
    mj += p * dj;
    ent -= plog2p(p);
    lge += p / (di * di);
    hge += p * di * di;
    slge += p / (di * di * dj * dj);
    shge += p * di * di / (dj * dj);
    llge += p * dj * dj / (di * di);
    lhge += p * di * di * dj * dj;
  }
  double gln = 0, ln = 0, gv = 0, lv = 0;
  for (int i = 1; i <= ng; ++i) {
    gln += (double)ri[i] * (double)ri[i];
    gv += (i - mi) * (i - mi) * (double)ri[i] / N;
  }
  for (size_t q = 0; q < cj.size();) {
    const int64_t j = cj[q].first;
    int64_t c = 0;
    for (; q < cj.size() && cj[q].first == j; ++q) c += cj[q].second;
    ln += (double)c * (double)c;
    lv += (j - mj) * (j - mj) * (double)c / N;
  }
  f[0] = se;
  f[1] = le;
  f[2] = gln / N;
  f[3] = gln / (N * N);
  f[4] = ln / N;
  f[5] = ln / (N * N);
  f[6] = N / Np;
  f[7] = gv;
  f[8] = lv;
  f[9] = ent;
  f[10] = lge;
  f[11] = hge;
  f[12] = slge;
  f[13] = shge;
  f[14] = llge;
  f[15] = lhge;
}

// Non-zero entries of a dense [ng+1][nj+1] count table.
std::vector<Entry> entries(const std::vector<int64_t>& T, int ng, int nj) {
  std::vector<Entry> E;
  for (int i = 1; i <= ng; ++i)
    for (int j = 1; j <= nj; ++j)
      if (T[(size_t)i * (nj + 1) + j]) E.push_back({i, j, T[(size_t)i * (nj + 1) + j]});
  return E;
}

void glrlm_features(const Grid& G, int ng, int64_t K, double* f) {
  const int maxlen = std::max(G.nx, std::max(G.ny, G.nz));
  std::vector<int64_t> R((size_t)(ng + 1) * (maxlen + 1), 0);
  for (const auto& d : kDir)
    for (int z = 0; z < G.nz; ++z)
      for (int y = 0; y < G.ny; ++y)
        for (int x = 0; x < G.nx; ++x) {
          const int a = G.lev[G.at(x, y, z)];
          if (!a || G.level(x - d[0], y - d[1], z - d[2]) == a) continue;  // not a run start
          int len = 1;
          while (G.level(x + len * d[0], y + len * d[1], z + len * d[2]) == a) len++;
          R[(size_t)a * (maxlen + 1) + len]++;
        }
  emphasis(entries(R, ng, maxlen), ng, 13.0 * (double)K, f);
}

void glszm_features(const Grid& G, int ng, int64_t K, double* f) {
  const int64_t N = (int64_t)G.nx * G.ny * G.nz;
  std::vector<int64_t> parent(N);
  std::iota(parent.begin(), parent.end(), 0);
  auto root = [&](int64_t u) {
    while (parent[u] != u) {
      parent[u] = parent[parent[u]];
      u = parent[u];
    }
    return u;
  };
  for (int z = 0; z < G.nz; ++z)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int a = G.lev[G.at(x, y, z)];
        if (!a) continue;
        for (const auto& d : kDir) {
          const int xn = x + d[0], yn = y + d[1], zn = z + d[2];
          if (G.level(xn, yn, zn) != a) continue;
          const int64_t r1 = root(G.at(x, y, z)), r2 = root(G.at(xn, yn, zn));
          if (r1 != r2) parent[std::max(r1, r2)] = std::min(r1, r2);
        }
      }
  std::vector<int64_t> size(N, 0);
  for (int64_t u = 0; u < N; ++u)
    if (G.lev[u]) size[root(u)]++;
  std::vector<std::pair<int, int64_t>> zones;  // (level, size) per zone
  for (int64_t u = 0; u < N; ++u)
    if (G.lev[u] && parent[u] == u) zones.push_back({G.lev[u], size[u]});
  std::sort(zones.begin(), zones.end());
  std::vector<Entry> E;
  for (size_t q = 0; q < zones.size();) {
    size_t r = q;
    while (r < zones.size() && zones[r] == zones[q]) r++;
    E.push_back({zones[q].first, zones[q].second, (int64_t)(r - q)});
    q = r;
  }
  emphasis(E, ng, (double)K, f);
}

void gldm_features(const Grid& G, int ng, double* f) {
  std::vector<int64_t> D((size_t)(ng + 1) * 28, 0);
  for (int z = 0; z < G.nz; ++z)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int a = G.lev[G.at(x, y, z)];
        if (!a) continue;
        int k = 1;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
              if ((dx || dy || dz) && G.level(x + dx, y + dy, z + dz) == a) k++;
        D[(size_t)a * 28 + k]++;
      }
  double e[16];
  emphasis(entries(D, ng, 27), ng, 1.0, e);
  // GLDM order: SDE, LDE, GLN, DN, DNN, GLV, DV, DE, LGLE, HGLE, SDLGLE,
  // SDHGLE, LDLGLE, LDHGLE
  const int pick[14] = {0, 1, 2, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15};
  for (int k = 0; k < 14; ++k) f[k] = e[pick[k]];
}

void ngtdm_features(const Grid& G, int ng, double* f) {
  std::vector<int64_t> n(ng + 1, 0);
  std::vector<__int128> S(ng + 1, 0);  // s_i * lcm(1..26), exact
  for (int z = 0; z < G.nz; ++z)
    for (int y = 0; y < G.ny; ++y)
      for (int x = 0; x < G.nx; ++x) {
        const int a = G.lev[G.at(x, y, z)];
        if (!a) continue;
        int W = 0, A = 0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (!(dx || dy || dz)) continue;
              const int b = G.level(x + dx, y + dy, z + dz);
              if (b) {
                W++;
                A += b;
              }
            }
        if (!W) continue;
        n[a]++;
        S[a] += (__int128)std::abs(a * W - A) * (kLcm / W);
      }
  int64_t Nv = 0;
  __int128 Stot = 0;
  for (int i = 1; i <= ng; ++i) {
    Nv += n[i];
    Stot += S[i];
  }
  if (Nv == 0) {
    for (int k = 0; k < 5; ++k) f[k] = NAN;
    return;
  }
  const double Nd = (double)Nv;
  std::vector<int> pres;
  for (int i = 1; i <= ng; ++i)
    if (n[i]) pres.push_back(i);
  std::vector<double> p(ng + 1, 0.0), s(ng + 1, 0.0);
  for (int i : pres) {
    p[i] = (double)n[i] / Nd;
    s[i] = (double)S[i] / (double)kLcm;
  }
  double psum = 0.0, ssum = (double)Stot / (double)kLcm;
  for (int i : pres) psum += p[i] * s[i];
  const int Ngp = (int)pres.size();
  double con = 0, bden = 0, cpx = 0, str = 0;
  int64_t bint = 0;
  for (int i : pres)
    for (int j : pres) {
      const double dij = (double)(i - j);
      con += p[i] * p[j] * dij * dij;
      bint += std::llabs((int64_t)i * n[i] - (int64_t)j * n[j]);
      bden += fabs(i * p[i] - j * p[j]);
      cpx += fabs(dij) * (p[i] * s[i] + p[j] * s[j]) / (p[i] + p[j]);
      str += (p[i] + p[j]) * dij * dij;
    }
  f[0] = Stot == 0 ? 1e6 : 1.0 / psum;
  f[1] = Ngp <= 1 ? 0.0 : con / ((double)Ngp * (Ngp - 1)) * ssum / Nd;
  f[2] = bint == 0 ? 0.0 : psum / bden;
  f[3] = cpx / Nd;
  f[4] = Stot == 0 ? 0.0 : str / ssum;
}

}  // namespace

extern "C" {

fr_status fr_scalar(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                    const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                    double disc_value, double disc_lower, uint32_t families, double* out,
                    int32_t out_capacity) {
  fr::clear_error();
  if (!volume || !mask || !spacing_mm || !out) return cfail(FR_E_ARG, "null pointer argument");
  if (nx <= 0 || ny <= 0 || nz <= 0) return cfail(FR_E_ARG, "dims must be positive");
  if (dtype != FR_I16 && dtype != FR_F32) return cfail(FR_E_ARG, "dtype %d unknown", dtype);
  if (disc_mode != FR_FBW && disc_mode != FR_FBN) return cfail(FR_E_ARG, "discretisation mode unknown");
  if (!(disc_value > 0.0) || !isfinite(disc_value)) return cfail(FR_E_ARG, "bin value must be finite and > 0");
  if (disc_mode == FR_FBN && (disc_value != floor(disc_value) || disc_value > 255.0))
    return cfail(FR_E_RANGE, "bin count must be an integer in 1..255");
  for (int i = 0; i < 3; ++i)
    if (!(spacing_mm[i] > 0.0) || !isfinite(spacing_mm[i]))
      return cfail(FR_E_ARG, "spacing_mm[%d] must be finite and > 0", i);
  if (families == 0 || (families & ~(uint32_t)FR_ALL))
    return cfail(FR_E_RANGE, "families mask 0x%x invalid", families);
  static const int cnt[6] = {18, 24, 16, 16, 14, 5};
  int32_t count = 0;
  for (int q = 0; q < 6; ++q)
    if (families & (1u << q)) count += cnt[q];
  if (out_capacity < count) return cfail(FR_E_CAPACITY, "out holds %d doubles, %d needed", out_capacity, count);
  const int64_t N = (int64_t)nx * ny * nz;
  std::vector<double> x;
  std::vector<int64_t> where;
  for (int64_t i = 0; i < N; ++i)
    if (mask[i]) {
      where.push_back(i);
      x.push_back(dtype == FR_I16 ? (double)((const int16_t*)volume)[i] : (double)((const float*)volume)[i]);
    }
  if (x.empty()) return cfail(FR_E_EMPTY_MASK, "the mask holds no voxel");
  std::vector<uint8_t> g;
  int ng = 0;
  if (discretise(x, disc_mode, disc_value, disc_lower, g, &ng) != FR_OK)
    return cfail(FR_E_RANGE, "fixed bin width gives more than 255 gray levels");
  Grid G{nx, ny, nz, std::vector<uint8_t>(N, 0)};
  for (size_t m = 0; m < where.size(); ++m) G.lev[where[m]] = g[m];
  const int64_t K = (int64_t)x.size();
  double* f = out;
  if (families & FR_FIRSTORDER) {
    first_order(x, g, ng, spacing_mm[0] * spacing_mm[1] * spacing_mm[2], f);
    f += 18;
  }
  if (families & FR_GLCM) {
    glcm_features(G, ng, f);
    f += 24;
  }
  if (families & FR_GLRLM) {
    glrlm_features(G, ng, K, f);
    f += 16;
  }
  if (families & FR_GLSZM) {
    glszm_features(G, ng, K, f);
    f += 16;
  }
  if (families & FR_GLDM) {
    gldm_features(G, ng, f);
    f += 14;
  }
  if (families & FR_NGTDM) ngtdm_features(G, ng, f);
  return FR_OK;
}

const char* fr_scalar_last_error(void) { return fr::last_error(); }

}  // extern "C"
