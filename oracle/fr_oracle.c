/*
 * fr_oracle.c -- plain, slow, FP64 CPU ORACLE for radiomic spatial mapping.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (paper: "Software design and extraction modes" -- spatial
 * mapping returns, for every VOI voxel, features of that voxel's local
 * neighbourhood, as maps aligned with the source image; Table 2 -- the 93
 * shared spatial maps: 18 first-order ("statistics"), 24 GLCM, 16 GLRLM,
 * 16 GLSZM, 14 NGLDM/GLDM, 5 NGTDM).  The paper defers the feature equations
 * to IBSI ("IBSI compliance tests"); the readings it leaves open are fixed
 * here:
 *
 *   neighbourhood  V(c) = { u : |u-c|_inf <= r, u inside the image, mask[u] }
 *   discretisation FBN  g = floor(Ng (X - Xmin) / (Xmax - Xmin)) + 1, g <= Ng
 *                  FBW  g = floor((X - Xlo) / w) + 1, g >= 1; Ng = max level
 *                  Xmin/Xmax over the whole VOI; Xlo = given bound or Xmin
 *   GLCM   13 offsets at Chebyshev distance 1, counted both ways (symmetric),
 *          merged over directions before the features
 *   GLRLM  maximal equal-level runs inside V along the 13 directions, merged;
 *          Np = 13 |V|
 *   GLSZM  26-connected equal-level zones inside V
 *   GLDM   alpha = 0, dependence k(v) = 1 + #{26-neighbours in V, same level}
 *   NGTDM  s_i = sum over v with level i and >=1 neighbour in V of
 *          |i - mean level of those neighbours|
 *
 * Extraction variants (the IBSI configuration elements the paper lists
 * among its settings: GLCM distance, NGLDM coarseness, direction
 * aggregation), selected by the *_ex entry points:
 *   GLCM distance d   pairs (v, v + d m) for the 13 direction vectors m
 *   GLDM alpha        u depends on v when |g_u - g_v| <= alpha
 *   averaged          GLCM and GLRLM features computed from each
 *                     direction's own matrix, then their mean (GLRLM: Np =
 *                     |V| per direction; a direction without a GLCM pair is
 *                     left out of the GLCM mean, NaN when no direction has one)
 *
 * Everything is the plain definition: integer matrices counted by direct
 * enumeration, features by double sums over the matrices in FP64.  The only
 * iterative step is the eigenvalue problem of the maximal correlation
 * coefficient, solved by cyclic Jacobi rotations on a symmetric matrix that
 * is diagonally similar to the defining matrix Q.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_EMPTY (-2)
#define OR_E_RANGE (-3)
#define OR_E_NOMEM (-4)

#define OR_I16 1
#define OR_F32 2
#define OR_FBW 1
#define OR_FBN 2

#define F_FO 1u
#define F_GLCM 2u
#define F_GLRLM 4u
#define F_GLSZM 8u
#define F_GLDM 16u
#define F_NGTDM 32u

#define N_FO 18
#define N_GLCM 24
#define N_GLRLM 16
#define N_GLSZM 16
#define N_GLDM 14
#define N_NGTDM 5

/* lcm(1..26): the neighbour count c of a voxel is 1..26, so
 * (g*c - sum) * (LCM / c) is an exact integer image of |g - sum/c| * LCM. */
#define OR_LCM26 26771144400LL

/* One representative (dx,dy,dz) of each +/- pair of the 26-neighbourhood. */
static const int OR_DIR[13][3] = {
    {1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0},   {1, -1, 0},
    {1, 0, 1},  {1, 0, -1}, {0, 1, 1},  {0, 1, -1},  {1, 1, 1},
    {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

static double rawval(const void *vol, int dtype, int64_t i) {
  if (dtype == OR_I16) return (double)((const int16_t *)vol)[i];
  return (double)((const float *)vol)[i];
}

/* ------------------------------------------------------------------------ */
/* Discretisation (IBSI fixed bin number / fixed bin width).                 */
/* ------------------------------------------------------------------------ */
int or_discretise(const void *vol, int dtype, int nx, int ny, int nz,
                  const uint8_t *mask, int mode, double value, double lower,
                  uint8_t *levels, int *ng_out, double *xmin_out,
                  double *xmax_out) {
  if (!vol || !mask || !levels || nx <= 0 || ny <= 0 || nz <= 0) return OR_E_ARG;
  if (dtype != OR_I16 && dtype != OR_F32) return OR_E_ARG;
  if (!(value > 0.0) || !isfinite(value)) return OR_E_ARG;
  const int64_t n = (int64_t)nx * ny * nz;
  double xmin = INFINITY, xmax = -INFINITY;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; i++) {
    if (!mask[i]) continue;
    double x = rawval(vol, dtype, i);
    if (x < xmin) xmin = x;
    if (x > xmax) xmax = x;
    cnt++;
  }
  if (cnt == 0) return OR_E_EMPTY;
  int ng;
  if (mode == OR_FBN) {
    if (value != floor(value) || value > 255.0) return OR_E_RANGE;
    ng = (int)value;
    const double range = xmax - xmin;
    for (int64_t i = 0; i < n; i++) {
      if (!mask[i]) { levels[i] = 0; continue; }
      int g = 1;
      if (range > 0.0) {
        double t = rawval(vol, dtype, i) - xmin;
        double q = ((double)ng * t) / range;
        g = (int)floor(q) + 1;
        if (g > ng) g = ng;
      }
      levels[i] = (uint8_t)g;
    }
  } else if (mode == OR_FBW) {
    const double lo = isfinite(lower) ? lower : xmin;
    double qmax = floor((xmax - lo) / value) + 1.0;
    if (qmax > 255.0) return OR_E_RANGE;
    ng = qmax < 1.0 ? 1 : (int)qmax;
    for (int64_t i = 0; i < n; i++) {
      if (!mask[i]) { levels[i] = 0; continue; }
      double t = rawval(vol, dtype, i) - lo;
      double g = floor(t / value) + 1.0;
      if (g < 1.0) g = 1.0;
      levels[i] = (uint8_t)g;
    }
  } else {
    return OR_E_ARG;
  }
  if (ng_out) *ng_out = ng;
  if (xmin_out) *xmin_out = xmin;
  if (xmax_out) *xmax_out = xmax;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Neighbourhood: a box of the image with a membership flag per voxel.       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int bx, by, bz;      /* box dims */
  uint8_t *member;     /* [bz][by][bx] 1 = voxel in V */
  uint8_t *lev;        /* level of the voxel (valid where member) */
  double *raw;         /* raw value (valid where member) */
  int K;               /* |V| */
} nbhd;

static int nb_in(const nbhd *b, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= b->bx || y >= b->by || z >= b->bz) return 0;
  return b->member[((int64_t)z * b->by + y) * b->bx + x];
}
static int nb_lev(const nbhd *b, int x, int y, int z) {
  return b->lev[((int64_t)z * b->by + y) * b->bx + x];
}

/* Fill V for the cube of radius r around (cx,cy,cz); r < 0 means the whole
 * bounding box of the mask (scalar extraction). */
static int nb_build(nbhd *b, const uint8_t *levels, const void *vol, int dtype,
                    int nx, int ny, int nz, int r, int cx, int cy, int cz,
                    int box_cap) {
  int x0, y0, z0, x1, y1, z1;
  if (r >= 0) {
    x0 = cx - r; x1 = cx + r; y0 = cy - r; y1 = cy + r; z0 = cz - r; z1 = cz + r;
  } else {
    x0 = nx; y0 = ny; z0 = nz; x1 = -1; y1 = -1; z1 = -1;
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++)
          if (levels[((int64_t)z * ny + y) * nx + x]) {
            x0 = x < x0 ? x : x0; x1 = x > x1 ? x : x1;
            y0 = y < y0 ? y : y0; y1 = y > y1 ? y : y1;
            z0 = z < z0 ? z : z0; z1 = z > z1 ? z : z1;
          }
    if (x1 < 0) return OR_E_EMPTY;
  }
  b->bx = x1 - x0 + 1; b->by = y1 - y0 + 1; b->bz = z1 - z0 + 1;
  if ((int64_t)b->bx * b->by * b->bz > box_cap) return OR_E_RANGE;
  b->K = 0;
  for (int z = 0; z < b->bz; z++)
    for (int y = 0; y < b->by; y++)
      for (int x = 0; x < b->bx; x++) {
        int64_t bi = ((int64_t)z * b->by + y) * b->bx + x;
        int gx = x + x0, gy = y + y0, gz = z + z0;
        b->member[bi] = 0; b->lev[bi] = 0; b->raw[bi] = 0.0;
        if (gx < 0 || gy < 0 || gz < 0 || gx >= nx || gy >= ny || gz >= nz) continue;
        int64_t gi = ((int64_t)gz * ny + gy) * nx + gx;
        if (!levels[gi]) continue;   /* level 0 <=> outside the VOI mask */
        b->member[bi] = 1;
        b->lev[bi] = levels[gi];
        b->raw[bi] = rawval(vol, dtype, gi);
        b->K++;
      }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Integer matrices of one neighbourhood, by direct enumeration.             */
/* ------------------------------------------------------------------------ */
typedef struct {
  int ng, lmax, zmax;
  int dist, alpha, averaged;  /* extraction variant (defaults 1, 0, 0)    */
  int64_t *glcm;    /* [ng][ng] symmetric co-occurrence counts            */
  int64_t *glcm_dir;  /* averaged only: [13][ng][ng] per direction      */
  int64_t *glrlm_dir; /* averaged only: [13][ng][lmax] per direction     */
  int64_t *glrlm;   /* [ng][lmax] run counts, column j-1 = run length j     */
  int64_t *glszm;   /* [ng][zmax] zone counts, column s-1 = zone size s     */
  int64_t *gldm;    /* [ng][27] dependence counts, column k-1 = k           */
  int64_t *ng_n;    /* [ng] NGTDM voxel counts n_i                          */
  int64_t *ng_S;    /* [ng] NGTDM s_i * lcm(1..26), exact                    */
  double *ng_s;     /* [ng] NGTDM s_i, FP64 definitional                    */
  int64_t *hist;    /* [ng] level histogram                                */
  double *vals;     /* [K] raw values of V                                  */
  int K;
  int *queue;       /* zone flood-fill work space [box]                      */
  uint8_t *seen;    /* [box]                                               */
} mats;

static void count_matrices(const nbhd *b, mats *m) {
  const int ng = m->ng;
  memset(m->glcm, 0, sizeof(int64_t) * ng * ng);
  memset(m->glrlm, 0, sizeof(int64_t) * ng * m->lmax);
  memset(m->glszm, 0, sizeof(int64_t) * ng * m->zmax);
  memset(m->gldm, 0, sizeof(int64_t) * ng * 27);
  memset(m->ng_n, 0, sizeof(int64_t) * ng);
  memset(m->ng_S, 0, sizeof(int64_t) * ng);
  memset(m->hist, 0, sizeof(int64_t) * ng);
  for (int i = 0; i < ng; i++) m->ng_s[i] = 0.0;
  if (m->averaged) {
    memset(m->glcm_dir, 0, sizeof(int64_t) * 13 * ng * ng);
    memset(m->glrlm_dir, 0, sizeof(int64_t) * 13 * ng * m->lmax);
  }
  m->K = 0;
  const int64_t nbox = (int64_t)b->bx * b->by * b->bz;
  memset(m->seen, 0, (size_t)nbox);

  for (int z = 0; z < b->bz; z++)
    for (int y = 0; y < b->by; y++)
      for (int x = 0; x < b->bx; x++) {
        if (!nb_in(b, x, y, z)) continue;
        const int g = nb_lev(b, x, y, z);
        const int64_t bi = ((int64_t)z * b->by + y) * b->bx + x;
        m->vals[m->K++] = b->raw[bi];
        m->hist[g - 1]++;

        /* GLCM: each unordered pair at offset +-dist*m is reached once
         * through the 13 representative vectors m and recorded in both
         * orders (and in its direction's matrix when averaging). */
        for (int d = 0; d < 13; d++) {
          int ux = x + m->dist * OR_DIR[d][0], uy = y + m->dist * OR_DIR[d][1];
          int uz = z + m->dist * OR_DIR[d][2];
          if (!nb_in(b, ux, uy, uz)) continue;
          int h = nb_lev(b, ux, uy, uz);
          m->glcm[(g - 1) * ng + (h - 1)]++;
          m->glcm[(h - 1) * ng + (g - 1)]++;
          if (m->averaged) {
            m->glcm_dir[(int64_t)d * ng * ng + (g - 1) * ng + (h - 1)]++;
            m->glcm_dir[(int64_t)d * ng * ng + (h - 1) * ng + (g - 1)]++;
          }
        }

        /* GLRLM: a run starts where the previous voxel along d is not in V or
         * has another level; walk forward while the level stays equal. */
        for (int d = 0; d < 13; d++) {
          int px = x - OR_DIR[d][0], py = y - OR_DIR[d][1], pz = z - OR_DIR[d][2];
          if (nb_in(b, px, py, pz) && nb_lev(b, px, py, pz) == g) continue;
          int len = 1;
          int qx = x + OR_DIR[d][0], qy = y + OR_DIR[d][1], qz = z + OR_DIR[d][2];
          while (nb_in(b, qx, qy, qz) && nb_lev(b, qx, qy, qz) == g) {
            len++;
            qx += OR_DIR[d][0]; qy += OR_DIR[d][1]; qz += OR_DIR[d][2];
          }
          m->glrlm[(g - 1) * m->lmax + (len - 1)]++;
          if (m->averaged) m->glrlm_dir[(int64_t)d * ng * m->lmax + (g - 1) * m->lmax + (len - 1)]++;
        }

        /* GLDM and NGTDM: the 26 neighbours of v that are in V. */
        int same = 0, cnt = 0;
        int64_t lsum = 0;
        for (int dz = -1; dz <= 1; dz++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
              if (!dx && !dy && !dz) continue;
              if (!nb_in(b, x + dx, y + dy, z + dz)) continue;
              int h = nb_lev(b, x + dx, y + dy, z + dz);
              cnt++;
              lsum += h;
              if (abs(h - g) <= m->alpha) same++;
            }
        m->gldm[(g - 1) * 27 + same]++;   /* k = 1 + dependent, column k-1 */
        if (cnt > 0) {
          m->ng_n[g - 1]++;
          m->ng_s[g - 1] += fabs((double)g - (double)lsum / (double)cnt);
          int64_t diff = (int64_t)g * cnt - lsum;
          if (diff < 0) diff = -diff;
          m->ng_S[g - 1] += diff * (OR_LCM26 / cnt);
        }
      }

  /* GLSZM: flood fill of 26-connected equal-level components (breadth
   * first, from every not yet visited voxel in raster order). */
  for (int z = 0; z < b->bz; z++)
    for (int y = 0; y < b->by; y++)
      for (int x = 0; x < b->bx; x++) {
        int64_t bi = ((int64_t)z * b->by + y) * b->bx + x;
        if (!b->member[bi] || m->seen[bi]) continue;
        const int g = b->lev[bi];
        int head = 0, tail = 0, size = 0;
        m->queue[tail++] = (int)bi;
        m->seen[bi] = 1;
        while (head < tail) {
          int cur = m->queue[head++];
          size++;
          int cx = cur % b->bx, cy = (cur / b->bx) % b->by, cz = cur / (b->bx * b->by);
          for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
              for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                int ux = cx + dx, uy = cy + dy, uz = cz + dz;
                if (!nb_in(b, ux, uy, uz)) continue;
                int64_t ui = ((int64_t)uz * b->by + uy) * b->bx + ux;
                if (m->seen[ui] || b->lev[ui] != g) continue;
                m->seen[ui] = 1;
                m->queue[tail++] = (int)ui;
              }
        }
        m->glszm[(g - 1) * m->zmax + (size - 1)]++;
      }
}

/* ------------------------------------------------------------------------ */
/* First-order features (Table 2 "Statistics", IBSI definitions).            */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Linear interpolation between order statistics: h = (N-1) q, 0-based. */
static double pct_sorted(const double *s, int n, double q) {
  double h = (double)(n - 1) * q;
  double lo = floor(h);
  int i = (int)lo;
  double frac = h - lo;
  if (i + 1 >= n) return s[n - 1];
  return s[i] + frac * (s[i + 1] - s[i]);
}

int or_firstorder_features(const double *vals, int K, const int64_t *hist,
                           int ng, double voxel_volume, double *f) {
  if (K <= 0) return OR_E_ARG;
  double *s = (double *)malloc(sizeof(double) * K);
  if (!s) return OR_E_NOMEM;
  memcpy(s, vals, sizeof(double) * K);
  qsort(s, K, sizeof(double), cmp_double);
  const double N = (double)K;
  double sum = 0.0, sum2 = 0.0;
  for (int i = 0; i < K; i++) { sum += vals[i]; sum2 += vals[i] * vals[i]; }
  const double mu = sum / N;
  double m2 = 0.0, m3 = 0.0, m4 = 0.0, mad = 0.0;
  for (int i = 0; i < K; i++) {
    double d = vals[i] - mu;
    m2 += d * d; m3 += d * d * d; m4 += d * d * d * d; mad += fabs(d);
  }
  m2 /= N; m3 /= N; m4 /= N; mad /= N;
  const double mn = s[0], mx = s[K - 1];
  const double p10 = pct_sorted(s, K, 0.10), p25 = pct_sorted(s, K, 0.25);
  const double p50 = pct_sorted(s, K, 0.50), p75 = pct_sorted(s, K, 0.75);
  const double p90 = pct_sorted(s, K, 0.90);
  /* robust subset: values inside [P10, P90] */
  double rs = 0.0; int rn = 0;
  for (int i = 0; i < K; i++)
    if (vals[i] >= p10 && vals[i] <= p90) { rs += vals[i]; rn++; }
  const double rmu = rs / (double)rn;
  double rmad = 0.0;
  for (int i = 0; i < K; i++)
    if (vals[i] >= p10 && vals[i] <= p90) rmad += fabs(vals[i] - rmu);
  rmad /= (double)rn;
  double ent = 0.0, uni = 0.0;
  for (int i = 0; i < ng; i++) {
    if (!hist[i]) continue;
    double p = (double)hist[i] / N;
    ent -= p * log2(p);
    uni += p * p;
  }
  const int flat = (mn == mx);
  f[0] = sum2;                                   /* Energy */
  f[1] = voxel_volume * sum2;                    /* TotalEnergy */
  f[2] = ent;                                    /* Entropy */
  f[3] = mn;                                     /* Minimum */
  f[4] = p10;                                    /* 10Percentile */
  f[5] = p90;                                    /* 90Percentile */
  f[6] = mx;                                     /* Maximum */
  f[7] = mu;                                     /* Mean */
  f[8] = p50;                                    /* Median */
  f[9] = p75 - p25;                              /* InterquartileRange */
  f[10] = mx - mn;                               /* Range */
  f[11] = mad;                                   /* MeanAbsoluteDeviation */
  f[12] = rmad;                                  /* RobustMeanAbsoluteDeviation */
  f[13] = sqrt(sum2 / N);                        /* RootMeanSquared */
  f[14] = flat ? 0.0 : m3 / pow(m2, 1.5);        /* Skewness */
  f[15] = flat ? 0.0 : m4 / (m2 * m2) - 3.0;     /* Kurtosis (excess) */
  f[16] = m2;                                    /* Variance */
  f[17] = uni;                                   /* Uniformity */
  free(s);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Symmetric eigenvalues by cyclic Jacobi rotations (textbook method).       */
/* a is n x n, overwritten; eigenvalues returned in w.                       */
/* ------------------------------------------------------------------------ */
static void jacobi_eigenvalues(double *a, int n, double *w) {
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; p++)
      for (int q = p + 1; q < n; q++) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double app = a[p * n + p], aqq = a[q * n + q];
        /* rotation angle that zeroes a[p][q]: cot(2 phi) = (aqq - app) / (2 apq) */
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; k++) { /* columns p, q */
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; k++) { /* rows p, q */
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  for (int i = 0; i < n; i++) w[i] = a[i * n + i];
}

/* ------------------------------------------------------------------------ */
/* GLCM features (Table 2 GLCM; IBSI/PyRadiomics definitions).              */
/* P: [ng][ng] symmetric counts.  ng_norm: the VOI gray-level count used by  */
/* the normalised inverse difference (moment).  extra (optional, 4 values):  */
/* HX, HY, HXY1, HXY2 as defined, for the identity checks in the tests.      */
/* ------------------------------------------------------------------------ */
int or_glcm_features(const int64_t *P, int ng, double ng_norm, double *f,
                     double *extra) {
  int64_t NP = 0;
  for (int i = 0; i < ng * ng; i++) NP += P[i];
  if (NP == 0) {
    for (int k = 0; k < N_GLCM; k++) f[k] = NAN;
    if (extra) for (int k = 0; k < 4; k++) extra[k] = NAN;
    return OR_OK;
  }
  double *p = (double *)malloc(sizeof(double) * ng * ng);
  double *px = (double *)calloc(ng, sizeof(double));
  double *py = (double *)calloc(ng, sizeof(double));
  double *psum = (double *)calloc(2 * ng + 1, sizeof(double));
  double *pdif = (double *)calloc(ng, sizeof(double));
  if (!p || !px || !py || !psum || !pdif) return OR_E_NOMEM;
  for (int a = 0; a < ng; a++)
    for (int b = 0; b < ng; b++) p[a * ng + b] = (double)P[a * ng + b] / (double)NP;
  for (int a = 0; a < ng; a++)
    for (int b = 0; b < ng; b++) {
      px[a] += p[a * ng + b];
      py[b] += p[a * ng + b];
      psum[(a + 1) + (b + 1)] += p[a * ng + b];
      pdif[abs(a - b)] += p[a * ng + b];
    }
  double ux = 0.0, uy = 0.0;
  for (int a = 0; a < ng; a++) { ux += (a + 1) * px[a]; uy += (a + 1) * py[a]; }
  double sx2 = 0.0, sy2 = 0.0, HX = 0.0, HY = 0.0;
  int nlev = 0;
  for (int a = 0; a < ng; a++) {
    double i = a + 1;
    sx2 += (i - ux) * (i - ux) * px[a];
    sy2 += (i - uy) * (i - uy) * py[a];
    if (px[a] > 0) { HX -= px[a] * log2(px[a]); nlev++; }
    if (py[a] > 0) HY -= py[a] * log2(py[a]);
  }
  double autoc = 0, cprom = 0, cshade = 0, ctend = 0, contrast = 0, corr = 0;
  double energy = 0, HXY = 0, HXY1 = 0, HXY2 = 0, idm = 0, idmn = 0, id = 0, idn = 0;
  double maxp = 0;
  for (int a = 0; a < ng; a++)
    for (int b = 0; b < ng; b++) {
      const double i = a + 1, j = b + 1, v = p[a * ng + b];
      if (px[a] > 0 && py[b] > 0) HXY2 -= px[a] * py[b] * log2(px[a] * py[b]);
      if (v == 0.0) continue;
      const double s = i + j - ux - uy;
      autoc += i * j * v;
      cprom += s * s * s * s * v;
      cshade += s * s * s * v;
      ctend += s * s * v;
      contrast += (i - j) * (i - j) * v;
      corr += (i - ux) * (j - uy) * v;
      energy += v * v;
      HXY -= v * log2(v);
      HXY1 -= v * log2(px[a] * py[b]);
      idm += v / (1.0 + (i - j) * (i - j));
      idmn += v / (1.0 + (i - j) * (i - j) / (ng_norm * ng_norm));
      id += v / (1.0 + fabs(i - j));
      idn += v / (1.0 + fabs(i - j) / ng_norm);
      if (v > maxp) maxp = v;
    }
  double da = 0, de = 0, dv = 0, ivar = 0;
  for (int k = 0; k < ng; k++) {
    if (pdif[k] <= 0) continue;
    da += k * pdif[k];
    de -= pdif[k] * log2(pdif[k]);
    if (k > 0) ivar += pdif[k] / ((double)k * k);
  }
  for (int k = 0; k < ng; k++)
    if (pdif[k] > 0) dv += (k - da) * (k - da) * pdif[k];
  double sa = 0, se = 0;
  for (int k = 2; k <= 2 * ng; k++) {
    if (psum[k] <= 0) continue;
    sa += k * psum[k];
    se -= psum[k] * log2(psum[k]);
  }
  /* maximal correlation coefficient: Q(i,j) = sum_k p(i,k) p(j,k) / (px(i) py(k))
   * over present levels; its eigenvalues equal those of the symmetric
   * S = Dx^(1/2) Q Dx^(-1/2); MCC = sqrt(second largest eigenvalue). */
  double mcc = 1.0;
  if (nlev > 1) {
    int *lv = (int *)malloc(sizeof(int) * ng);
    int n = 0;
    for (int a = 0; a < ng; a++) if (px[a] > 0) lv[n++] = a;
    double *Q = (double *)malloc(sizeof(double) * n * n);
    double *S = (double *)malloc(sizeof(double) * n * n);
    double *w = (double *)malloc(sizeof(double) * n);
    for (int a = 0; a < n; a++)
      for (int b = 0; b < n; b++) {
        double q = 0.0;
        for (int c = 0; c < ng; c++) {
          if (py[c] <= 0) continue;
          q += p[lv[a] * ng + c] * p[lv[b] * ng + c] / (px[lv[a]] * py[c]);
        }
        Q[a * n + b] = q;
      }
    for (int a = 0; a < n; a++)
      for (int b = 0; b < n; b++)
        S[a * n + b] = Q[a * n + b] * sqrt(px[lv[a]]) / sqrt(px[lv[b]]);
    for (int a = 0; a < n; a++)   /* remove rounding asymmetry */
      for (int b = a + 1; b < n; b++) {
        double m = 0.5 * (S[a * n + b] + S[b * n + a]);
        S[a * n + b] = S[b * n + a] = m;
      }
    jacobi_eigenvalues(S, n, w);
    qsort(w, n, sizeof(double), cmp_double);   /* ascending */
    double l2 = w[n - 2];
    mcc = sqrt(l2 > 0.0 ? l2 : 0.0);
    free(lv); free(Q); free(S); free(w);
  }
  const double hxmax = HX > HY ? HX : HY;
  f[0] = autoc;                                      /* Autocorrelation */
  f[1] = ux;                                         /* JointAverage */
  f[2] = cprom;                                      /* ClusterProminence */
  f[3] = cshade;                                     /* ClusterShade */
  f[4] = ctend;                                      /* ClusterTendency */
  f[5] = contrast;                                   /* Contrast */
  f[6] = nlev <= 1 ? 1.0 : corr / sqrt(sx2 * sy2);   /* Correlation */
  f[7] = da;                                         /* DifferenceAverage */
  f[8] = de;                                         /* DifferenceEntropy */
  f[9] = dv;                                         /* DifferenceVariance */
  f[10] = energy;                                    /* JointEnergy */
  f[11] = HXY;                                       /* JointEntropy */
  f[12] = nlev <= 1 ? 0.0 : (HXY - HXY1) / hxmax;    /* Imc1 */
  {
    double t = 1.0 - exp(-2.0 * (HXY2 - HXY));       /* Imc2 */
    f[13] = sqrt(t > 0.0 ? t : 0.0);
  }
  f[14] = idm;                                       /* Idm */
  f[15] = mcc;                                       /* MCC */
  f[16] = idmn;                                      /* Idmn */
  f[17] = id;                                        /* Id */
  f[18] = idn;                                       /* Idn */
  f[19] = ivar;                                      /* InverseVariance */
  f[20] = maxp;                                      /* MaximumProbability */
  f[21] = sa;                                        /* SumAverage */
  f[22] = se;                                        /* SumEntropy */
  f[23] = sx2;                                       /* SumSquares */
  if (extra) { extra[0] = HX; extra[1] = HY; extra[2] = HXY1; extra[3] = HXY2; }
  free(p); free(px); free(py); free(psum); free(pdif);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Run/zone/dependence "emphasis" features.  M is [ng][ncol]; column c holds */
/* length/size/dependence j = c + 1.                                          */
/* ------------------------------------------------------------------------ */
/* GLRLM (16) and GLSZM (16) share one formula set; "units" = Np (voxels
 * covered by runs, 13 |V| when merged) or Nv (= |V| for zones). */
int or_runzone_features(const int64_t *M, int ng, int ncol, double units, double *f) {
  int64_t Nr = 0;
  for (int i = 0; i < ng * ncol; i++) Nr += M[i];
  if (Nr == 0) { for (int k = 0; k < 16; k++) f[k] = NAN; return OR_OK; }
  const double N = (double)Nr;
  double sre = 0, lre = 0, gln = 0, rln = 0, mui = 0, muj = 0, ent = 0;
  double lgl = 0, hgl = 0, srlgl = 0, srhgl = 0, lrlgl = 0, lrhgl = 0;
  for (int a = 0; a < ng; a++) {
    double rowsum = 0;
    for (int c = 0; c < ncol; c++) rowsum += (double)M[a * ncol + c];
    gln += rowsum * rowsum;
  }
  for (int c = 0; c < ncol; c++) {
    double colsum = 0;
    for (int a = 0; a < ng; a++) colsum += (double)M[a * ncol + c];
    rln += colsum * colsum;
  }
  for (int a = 0; a < ng; a++)
    for (int c = 0; c < ncol; c++) {
      if (!M[a * ncol + c]) continue;
      const double i = a + 1, j = c + 1, p = (double)M[a * ncol + c] / N;
      sre += p / (j * j);
      lre += p * j * j;
      mui += p * i;
      muj += p * j;
      ent -= p * log2(p);
      lgl += p / (i * i);
      hgl += p * i * i;
      srlgl += p / (i * i * j * j);
      srhgl += p * i * i / (j * j);
      lrlgl += p * j * j / (i * i);
      lrhgl += p * i * i * j * j;
    }
  double glv = 0, rv = 0;
  for (int a = 0; a < ng; a++)
    for (int c = 0; c < ncol; c++) {
      if (!M[a * ncol + c]) continue;
      const double i = a + 1, j = c + 1, p = (double)M[a * ncol + c] / N;
      glv += p * (i - mui) * (i - mui);
      rv += p * (j - muj) * (j - muj);
    }
  f[0] = sre; f[1] = lre; f[2] = gln / N; f[3] = gln / (N * N);
  f[4] = rln / N; f[5] = rln / (N * N); f[6] = N / units;
  f[7] = glv; f[8] = rv; f[9] = ent; f[10] = lgl; f[11] = hgl;
  f[12] = srlgl; f[13] = srhgl; f[14] = lrlgl; f[15] = lrhgl;
  return OR_OK;
}

/* GLDM (14): D is [ng][ncol], column c = dependence k = c + 1. */
int or_gldm_features(const int64_t *D, int ng, int ncol, double *f) {
  int64_t Nt = 0;
  for (int i = 0; i < ng * ncol; i++) Nt += D[i];
  if (Nt == 0) { for (int k = 0; k < N_GLDM; k++) f[k] = NAN; return OR_OK; }
  const double N = (double)Nt;
  double sde = 0, lde = 0, gln = 0, dn = 0, mui = 0, muj = 0, ent = 0;
  double lgl = 0, hgl = 0, sdlgl = 0, sdhgl = 0, ldlgl = 0, ldhgl = 0;
  for (int a = 0; a < ng; a++) {
    double rowsum = 0;
    for (int c = 0; c < ncol; c++) rowsum += (double)D[a * ncol + c];
    gln += rowsum * rowsum;
  }
  for (int c = 0; c < ncol; c++) {
    double colsum = 0;
    for (int a = 0; a < ng; a++) colsum += (double)D[a * ncol + c];
    dn += colsum * colsum;
  }
  for (int a = 0; a < ng; a++)
    for (int c = 0; c < ncol; c++) {
      if (!D[a * ncol + c]) continue;
      const double i = a + 1, j = c + 1, p = (double)D[a * ncol + c] / N;
      sde += p / (j * j);
      lde += p * j * j;
      mui += p * i;
      muj += p * j;
      ent -= p * log2(p);
      lgl += p / (i * i);
      hgl += p * i * i;
      sdlgl += p / (i * i * j * j);
      sdhgl += p * i * i / (j * j);
      ldlgl += p * j * j / (i * i);
      ldhgl += p * i * i * j * j;
    }
  double glv = 0, dv = 0;
  for (int a = 0; a < ng; a++)
    for (int c = 0; c < ncol; c++) {
      if (!D[a * ncol + c]) continue;
      const double i = a + 1, j = c + 1, p = (double)D[a * ncol + c] / N;
      glv += p * (i - mui) * (i - mui);
      dv += p * (j - muj) * (j - muj);
    }
  f[0] = sde; f[1] = lde; f[2] = gln / N; f[3] = dn / N; f[4] = dn / (N * N);
  f[5] = glv; f[6] = dv; f[7] = ent; f[8] = lgl; f[9] = hgl;
  f[10] = sdlgl; f[11] = sdhgl; f[12] = ldlgl; f[13] = ldhgl;
  return OR_OK;
}

/* NGTDM (5): n[i] voxel counts, s[i] absolute-difference sums, level i+1. */
int or_ngtdm_features(const int64_t *n, const double *s, int ng, double *f) {
  int64_t Nvc_i = 0;
  for (int i = 0; i < ng; i++) Nvc_i += n[i];
  if (Nvc_i == 0) { for (int k = 0; k < N_NGTDM; k++) f[k] = NAN; return OR_OK; }
  const double Nvc = (double)Nvc_i;
  double *p = (double *)malloc(sizeof(double) * ng);
  int ngp = 0;
  double ps = 0.0, ssum = 0.0;
  int any_s = 0;
  for (int i = 0; i < ng; i++) {
    p[i] = (double)n[i] / Nvc;
    if (n[i]) ngp++;
    ps += p[i] * s[i];
    ssum += s[i];
    if (n[i] && s[i] != 0.0) any_s = 1;
  }
  double c1 = 0, bden = 0, cplx = 0, strn = 0;
  int64_t bden_int = 0;
  for (int a = 0; a < ng; a++) {
    if (!n[a]) continue;
    for (int b = 0; b < ng; b++) {
      if (!n[b]) continue;
      const double i = a + 1, j = b + 1;
      c1 += p[a] * p[b] * (i - j) * (i - j);
      bden += fabs(i * p[a] - j * p[b]);
      int64_t t = (int64_t)(a + 1) * n[a] - (int64_t)(b + 1) * n[b];
      bden_int += t < 0 ? -t : t;
      cplx += fabs(i - j) * (p[a] * s[a] + p[b] * s[b]) / (p[a] + p[b]);
      strn += (p[a] + p[b]) * (i - j) * (i - j);
    }
  }
  f[0] = any_s ? 1.0 / ps : 1e6;                                     /* Coarseness */
  f[1] = ngp <= 1 ? 0.0 : (c1 / ((double)ngp * (ngp - 1))) * (ssum / Nvc); /* Contrast */
  f[2] = bden_int == 0 ? 0.0 : ps / bden;                            /* Busyness */
  f[3] = cplx / Nvc;                                                 /* Complexity */
  f[4] = any_s ? strn / ssum : 0.0;                                  /* Strength */
  free(p);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Driver: features of one neighbourhood, per selected family.               */
/* ------------------------------------------------------------------------ */
int or_map_count(uint32_t families) {
  int n = 0;
  if (families & F_FO) n += N_FO;
  if (families & F_GLCM) n += N_GLCM;
  if (families & F_GLRLM) n += N_GLRLM;
  if (families & F_GLSZM) n += N_GLSZM;
  if (families & F_GLDM) n += N_GLDM;
  if (families & F_NGTDM) n += N_NGTDM;
  return n;
}

static const char *FO_NAMES[N_FO] = {
    "Energy", "TotalEnergy", "Entropy", "Minimum", "10Percentile", "90Percentile",
    "Maximum", "Mean", "Median", "InterquartileRange", "Range",
    "MeanAbsoluteDeviation", "RobustMeanAbsoluteDeviation", "RootMeanSquared",
    "Skewness", "Kurtosis", "Variance", "Uniformity"};
static const char *GLCM_NAMES[N_GLCM] = {
    "Autocorrelation", "JointAverage", "ClusterProminence", "ClusterShade",
    "ClusterTendency", "Contrast", "Correlation", "DifferenceAverage",
    "DifferenceEntropy", "DifferenceVariance", "JointEnergy", "JointEntropy",
    "Imc1", "Imc2", "Idm", "MCC", "Idmn", "Id", "Idn", "InverseVariance",
    "MaximumProbability", "SumAverage", "SumEntropy", "SumSquares"};
static const char *GLRLM_NAMES[N_GLRLM] = {
    "ShortRunEmphasis", "LongRunEmphasis", "GrayLevelNonUniformity",
    "GrayLevelNonUniformityNormalized", "RunLengthNonUniformity",
    "RunLengthNonUniformityNormalized", "RunPercentage", "GrayLevelVariance",
    "RunVariance", "RunEntropy", "LowGrayLevelRunEmphasis",
    "HighGrayLevelRunEmphasis", "ShortRunLowGrayLevelEmphasis",
    "ShortRunHighGrayLevelEmphasis", "LongRunLowGrayLevelEmphasis",
    "LongRunHighGrayLevelEmphasis"};
static const char *GLSZM_NAMES[N_GLSZM] = {
    "SmallAreaEmphasis", "LargeAreaEmphasis", "GrayLevelNonUniformity",
    "GrayLevelNonUniformityNormalized", "SizeZoneNonUniformity",
    "SizeZoneNonUniformityNormalized", "ZonePercentage", "GrayLevelVariance",
    "ZoneVariance", "ZoneEntropy", "LowGrayLevelZoneEmphasis",
    "HighGrayLevelZoneEmphasis", "SmallAreaLowGrayLevelEmphasis",
    "SmallAreaHighGrayLevelEmphasis", "LargeAreaLowGrayLevelEmphasis",
    "LargeAreaHighGrayLevelEmphasis"};
static const char *GLDM_NAMES[N_GLDM] = {
    "SmallDependenceEmphasis", "LargeDependenceEmphasis", "GrayLevelNonUniformity",
    "DependenceNonUniformity", "DependenceNonUniformityNormalized",
    "GrayLevelVariance", "DependenceVariance", "DependenceEntropy",
    "LowGrayLevelEmphasis", "HighGrayLevelEmphasis",
    "SmallDependenceLowGrayLevelEmphasis", "SmallDependenceHighGrayLevelEmphasis",
    "LargeDependenceLowGrayLevelEmphasis", "LargeDependenceHighGrayLevelEmphasis"};
static const char *NGTDM_NAMES[N_NGTDM] = {"Coarseness", "Contrast", "Busyness",
                                           "Complexity", "Strength"};

/* Name of map k in canonical order, written as "family_Feature". */
int or_map_name(uint32_t families, int k, char *buf, int buflen) {
  const char *fam[6] = {"firstorder", "glcm", "glrlm", "glszm", "gldm", "ngtdm"};
  const char **tab[6] = {FO_NAMES, GLCM_NAMES, GLRLM_NAMES, GLSZM_NAMES, GLDM_NAMES, NGTDM_NAMES};
  const int cnt[6] = {N_FO, N_GLCM, N_GLRLM, N_GLSZM, N_GLDM, N_NGTDM};
  for (int q = 0; q < 6; q++) {
    if (!(families & (1u << q))) continue;
    if (k < cnt[q]) {
      int w = 0;
      for (const char *s = fam[q]; *s && w < buflen - 1; s++) buf[w++] = *s;
      if (w < buflen - 1) buf[w++] = '_';
      for (const char *s = tab[q][k]; *s && w < buflen - 1; s++) buf[w++] = *s;
      buf[w] = 0;
      return OR_OK;
    }
    k -= cnt[q];
  }
  return OR_E_RANGE;
}

typedef struct {
  mats m;
  nbhd b;
  double *feat; /* all 93 */
} work;

static int work_alloc(work *w, int ng, int lmax, int zmax, int64_t box, const int *opt) {
  memset(w, 0, sizeof(*w));
  w->m.ng = ng; w->m.lmax = lmax; w->m.zmax = zmax;
  w->m.dist = opt ? opt[0] : 1;
  w->m.alpha = opt ? opt[1] : 0;
  w->m.averaged = opt ? opt[2] : 0;
  if (w->m.averaged) {
    w->m.glcm_dir = (int64_t *)malloc(sizeof(int64_t) * 13 * ng * ng);
    w->m.glrlm_dir = (int64_t *)malloc(sizeof(int64_t) * 13 * ng * lmax);
    if (!w->m.glcm_dir || !w->m.glrlm_dir) return OR_E_NOMEM;
  }
  w->m.glcm = (int64_t *)malloc(sizeof(int64_t) * ng * ng);
  w->m.glrlm = (int64_t *)malloc(sizeof(int64_t) * ng * lmax);
  w->m.glszm = (int64_t *)malloc(sizeof(int64_t) * (int64_t)ng * zmax);
  w->m.gldm = (int64_t *)malloc(sizeof(int64_t) * ng * 27);
  w->m.ng_n = (int64_t *)malloc(sizeof(int64_t) * ng);
  w->m.ng_S = (int64_t *)malloc(sizeof(int64_t) * ng);
  w->m.ng_s = (double *)malloc(sizeof(double) * ng);
  w->m.hist = (int64_t *)malloc(sizeof(int64_t) * ng);
  w->m.vals = (double *)malloc(sizeof(double) * box);
  w->m.queue = (int *)malloc(sizeof(int) * box);
  w->m.seen = (uint8_t *)malloc(box);
  w->b.member = (uint8_t *)malloc(box);
  w->b.lev = (uint8_t *)malloc(box);
  w->b.raw = (double *)malloc(sizeof(double) * box);
  w->feat = (double *)malloc(sizeof(double) * 93);
  if (!w->m.glcm || !w->m.glrlm || !w->m.glszm || !w->m.gldm || !w->m.ng_n ||
      !w->m.ng_S || !w->m.ng_s || !w->m.hist || !w->m.vals || !w->m.queue ||
      !w->m.seen || !w->b.member || !w->b.lev || !w->b.raw || !w->feat)
    return OR_E_NOMEM;
  return OR_OK;
}

static void work_free(work *w) {
  free(w->m.glcm_dir); free(w->m.glrlm_dir);
  free(w->m.glcm); free(w->m.glrlm); free(w->m.glszm); free(w->m.gldm);
  free(w->m.ng_n); free(w->m.ng_S); free(w->m.ng_s); free(w->m.hist);
  free(w->m.vals); free(w->m.queue); free(w->m.seen);
  free(w->b.member); free(w->b.lev); free(w->b.raw); free(w->feat);
}

static int features_of(work *w, uint32_t families, double ng_norm, double voxel_volume) {
  mats *m = &w->m;
  double *f = w->feat;
  int k = 0, rc;
  if (families & F_FO) {
    rc = or_firstorder_features(m->vals, m->K, m->hist, m->ng, voxel_volume, f + k);
    if (rc) return rc;
    k += N_FO;
  }
  if (families & F_GLCM) {
    if (!m->averaged) {
      rc = or_glcm_features(m->glcm, m->ng, ng_norm, f + k, NULL);
      if (rc) return rc;
    } else {  /* mean over the directions that have at least one pair */
      double fd[N_GLCM];
      int nd = 0;
      for (int q = 0; q < N_GLCM; q++) f[k + q] = 0.0;
      for (int d = 0; d < 13; d++) {
        const int64_t *P = m->glcm_dir + (int64_t)d * m->ng * m->ng;
        int64_t tot = 0;
        for (int i = 0; i < m->ng * m->ng; i++) tot += P[i];
        if (!tot) continue;
        rc = or_glcm_features(P, m->ng, ng_norm, fd, NULL);
        if (rc) return rc;
        for (int q = 0; q < N_GLCM; q++) f[k + q] += fd[q];
        nd++;
      }
      for (int q = 0; q < N_GLCM; q++) f[k + q] = nd ? f[k + q] / nd : NAN;
    }
    k += N_GLCM;
  }
  if (families & F_GLRLM) {
    if (!m->averaged) {
      or_runzone_features(m->glrlm, m->ng, m->lmax, 13.0 * m->K, f + k);
    } else {  /* mean over the 13 directions, Np = |V| each */
      double fd[N_GLRLM];
      for (int q = 0; q < N_GLRLM; q++) f[k + q] = 0.0;
      for (int d = 0; d < 13; d++) {
        or_runzone_features(m->glrlm_dir + (int64_t)d * m->ng * m->lmax, m->ng, m->lmax,
                            (double)m->K, fd);
        for (int q = 0; q < N_GLRLM; q++) f[k + q] += fd[q] / 13.0;
      }
    }
    k += N_GLRLM;
  }
  if (families & F_GLSZM) {
    or_runzone_features(m->glszm, m->ng, m->zmax, (double)m->K, f + k);
    k += N_GLSZM;
  }
  if (families & F_GLDM) {
    or_gldm_features(m->gldm, m->ng, 27, f + k);
    k += N_GLDM;
  }
  if (families & F_NGTDM) {
    or_ngtdm_features(m->ng_n, m->ng_s, m->ng, f + k);
    k += N_NGTDM;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Public: per-voxel matrices of one centre voxel (for bit-exact checks).    */
/* levels: discretised volume (0 outside mask).  radius < 0 -> whole VOI.    */
/* Output buffers are dense over actual levels 1..ng (row a = level a+1).    */
/* ------------------------------------------------------------------------ */
/* opt (may be NULL): {GLCM distance, GLDM alpha, averaged}; the GLCM and
 * GLRLM returned are the merged ones (the sum of the direction matrices). */
int or_matrices_ex(const uint8_t *levels, const void *vol, int dtype, int nx, int ny,
                   int nz, int radius, int cx, int cy, int cz, int ng, int lmax,
                   int zmax, int64_t *glcm, int64_t *glrlm, int64_t *glszm,
                   int64_t *gldm, int64_t *ngtdm_n, int64_t *ngtdm_S,
                   double *ngtdm_s, int64_t *hist, double *vals, int *K_out,
                   const int *opt) {
  if (!levels || !vol || ng <= 0 || ng > 255) return OR_E_ARG;
  int64_t box = radius >= 0 ? (int64_t)(2 * radius + 1) * (2 * radius + 1) * (2 * radius + 1)
                            : (int64_t)nx * ny * nz;
  work w;
  int rc = work_alloc(&w, ng, lmax, zmax, box, opt);
  if (rc) { work_free(&w); return rc; }
  rc = nb_build(&w.b, levels, vol, dtype, nx, ny, nz, radius, cx, cy, cz, (int)box);
  if (rc) { work_free(&w); return rc; }
  if (radius < 0) {
    int ext = w.b.bx > w.b.by ? w.b.bx : w.b.by;
    if (w.b.bz > ext) ext = w.b.bz;
    if (lmax < ext || zmax < w.b.K) { work_free(&w); return OR_E_RANGE; }
  }
  count_matrices(&w.b, &w.m);
  memcpy(glcm, w.m.glcm, sizeof(int64_t) * ng * ng);
  memcpy(glrlm, w.m.glrlm, sizeof(int64_t) * ng * lmax);
  memcpy(glszm, w.m.glszm, sizeof(int64_t) * (int64_t)ng * zmax);
  memcpy(gldm, w.m.gldm, sizeof(int64_t) * ng * 27);
  memcpy(ngtdm_n, w.m.ng_n, sizeof(int64_t) * ng);
  memcpy(ngtdm_S, w.m.ng_S, sizeof(int64_t) * ng);
  memcpy(ngtdm_s, w.m.ng_s, sizeof(double) * ng);
  memcpy(hist, w.m.hist, sizeof(int64_t) * ng);
  if (vals) memcpy(vals, w.m.vals, sizeof(double) * w.m.K);
  if (K_out) *K_out = w.m.K;
  work_free(&w);
  return OR_OK;
}

int or_matrices(const uint8_t *levels, const void *vol, int dtype, int nx, int ny,
                int nz, int radius, int cx, int cy, int cz, int ng, int lmax,
                int zmax, int64_t *glcm, int64_t *glrlm, int64_t *glszm,
                int64_t *gldm, int64_t *ngtdm_n, int64_t *ngtdm_S,
                double *ngtdm_s, int64_t *hist, double *vals, int *K_out) {
  return or_matrices_ex(levels, vol, dtype, nx, ny, nz, radius, cx, cy, cz, ng, lmax, zmax,
                        glcm, glrlm, glszm, gldm, ngtdm_n, ngtdm_S, ngtdm_s, hist, vals,
                        K_out, NULL);
}

/* ------------------------------------------------------------------------ */
/* Public: spatial map for a sample of mask voxels (all if sample == NULL).  */
/* out is [count][nsample] FP64, map k of sample s at out[k*nsample + s].    */
/* The sample holds compact indices: the m-th mask voxel in raster order.    */
/* ------------------------------------------------------------------------ */
typedef struct {
  const uint8_t *levels;
  const void *vol;
  int dtype, nx, ny, nz, radius, ng;
  uint32_t families;
  double ng_norm, voxel_volume;
  const int64_t *lin;    /* linear voxel index of each sample */
  int64_t nsample, s0, s1;
  double *out;
  const int *opt;
  int rc;
} job;

static void *map_worker(void *arg) {
  job *j = (job *)arg;
  const int S = 2 * j->radius + 1;
  work w;
  j->rc = work_alloc(&w, j->ng, S, S * S * S, (int64_t)S * S * S, j->opt);
  if (j->rc) { work_free(&w); return NULL; }
  const int count = or_map_count(j->families);
  for (int64_t s = j->s0; s < j->s1; s++) {
    int64_t li = j->lin[s];
    int cx = (int)(li % j->nx), cy = (int)((li / j->nx) % j->ny), cz = (int)(li / ((int64_t)j->nx * j->ny));
    int rc = nb_build(&w.b, j->levels, j->vol, j->dtype, j->nx, j->ny, j->nz, j->radius, cx, cy, cz, S * S * S);
    if (rc) { j->rc = rc; break; }
    count_matrices(&w.b, &w.m);
    rc = features_of(&w, j->families, j->ng_norm, j->voxel_volume);
    if (rc) { j->rc = rc; break; }
    for (int k = 0; k < count; k++) j->out[(int64_t)k * j->nsample + s] = w.feat[k];
  }
  work_free(&w);
  return NULL;
}

/* opt (may be NULL): {GLCM distance >= 1, GLDM alpha >= 0, averaged 0/1}. */
int or_map_ex(const void *vol, int dtype, int nx, int ny, int nz, const uint8_t *mask,
              const double *spacing, int mode, double value, double lower, int radius,
              uint32_t families, const int64_t *sample, int64_t nsample, double *out,
              int nthreads, const int *opt) {
  if (!vol || !mask || !spacing || !out || radius < 1 || radius > 16) return OR_E_ARG;
  if (opt && (opt[0] < 1 || opt[1] < 0 || (opt[2] != 0 && opt[2] != 1))) return OR_E_ARG;
  if (!families || (families & ~63u)) return OR_E_RANGE;
  const int64_t n = (int64_t)nx * ny * nz;
  uint8_t *levels = (uint8_t *)malloc(n);
  if (!levels) return OR_E_NOMEM;
  int ng;
  double xmin, xmax;
  int rc = or_discretise(vol, dtype, nx, ny, nz, mask, mode, value, lower, levels, &ng, &xmin, &xmax);
  if (rc) { free(levels); return rc; }
  /* compact index -> linear voxel index (raster order) */
  int64_t M = 0;
  for (int64_t i = 0; i < n; i++) if (mask[i]) M++;
  int64_t *all = (int64_t *)malloc(sizeof(int64_t) * M);
  int64_t q = 0;
  for (int64_t i = 0; i < n; i++) if (mask[i]) all[q++] = i;
  int64_t ns = sample ? nsample : M;
  int64_t *lin = (int64_t *)malloc(sizeof(int64_t) * (ns > 0 ? ns : 1));
  for (int64_t s = 0; s < ns; s++) {
    int64_t m = sample ? sample[s] : s;
    if (m < 0 || m >= M) { free(levels); free(all); free(lin); return OR_E_RANGE; }
    lin[s] = all[m];
  }
  if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > ns) nthreads = ns > 0 ? (int)ns : 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
  job *jobs = (job *)malloc(sizeof(job) * nthreads);
  for (int t = 0; t < nthreads; t++) {
    job *j = &jobs[t];
    j->levels = levels; j->vol = vol; j->dtype = dtype;
    j->nx = nx; j->ny = ny; j->nz = nz; j->radius = radius; j->ng = ng;
    j->families = families; j->ng_norm = (double)ng;
    j->voxel_volume = spacing[0] * spacing[1] * spacing[2];
    j->lin = lin; j->nsample = ns;
    j->s0 = ns * t / nthreads; j->s1 = ns * (t + 1) / nthreads;
    j->out = out; j->opt = opt; j->rc = 0;
    pthread_create(&th[t], NULL, map_worker, j);
  }
  rc = OR_OK;
  for (int t = 0; t < nthreads; t++) {
    pthread_join(th[t], NULL);
    if (jobs[t].rc) rc = jobs[t].rc;
  }
  free(th); free(jobs); free(levels); free(all); free(lin);
  return rc;
}

int or_map(const void *vol, int dtype, int nx, int ny, int nz, const uint8_t *mask,
           const double *spacing, int mode, double value, double lower, int radius,
           uint32_t families, const int64_t *sample, int64_t nsample, double *out,
           int nthreads) {
  return or_map_ex(vol, dtype, nx, ny, nz, mask, spacing, mode, value, lower, radius, families,
                   sample, nsample, out, nthreads, NULL);
}

/* ------------------------------------------------------------------------ */
/* Public: scalar extraction -- the same features over the whole VOI.        */
/* ------------------------------------------------------------------------ */
int or_scalar(const void *vol, int dtype, int nx, int ny, int nz, const uint8_t *mask,
              const double *spacing, int mode, double value, double lower,
              uint32_t families, double *out) {
  if (!vol || !mask || !spacing || !out) return OR_E_ARG;
  if (!families || (families & ~63u)) return OR_E_RANGE;
  const int64_t n = (int64_t)nx * ny * nz;
  uint8_t *levels = (uint8_t *)malloc(n);
  int ng; double xmin, xmax;
  int rc = or_discretise(vol, dtype, nx, ny, nz, mask, mode, value, lower, levels, &ng, &xmin, &xmax);
  if (rc) { free(levels); return rc; }
  int ext = nx > ny ? nx : ny; if (nz > ext) ext = nz;
  int64_t M = 0;
  for (int64_t i = 0; i < n; i++) if (mask[i]) M++;
  work w;
  rc = work_alloc(&w, ng, ext, (int)M, n, NULL);
  if (!rc) rc = nb_build(&w.b, levels, vol, dtype, nx, ny, nz, -1, 0, 0, 0, (int)n);
  if (!rc) {
    count_matrices(&w.b, &w.m);
    rc = features_of(&w, families, (double)ng, spacing[0] * spacing[1] * spacing[2]);
    if (!rc) memcpy(out, w.feat, sizeof(double) * or_map_count(families));
  }
  work_free(&w);
  free(levels);
  return rc;
}
