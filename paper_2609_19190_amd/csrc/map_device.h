// Device helpers shared by the map kernels of this library (the fused
// fixed-radius kernel and the generic kernel): the 13 GLCM/GLRLM direction
// representatives, the exact NGTDM scale table and two FP64 primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fr {
namespace {

// lcm(1..26) / c for c = 1..26: NGTDM differences |g c - sum| scaled by it
// are exact integers (s_i * lcm(1..26)).
__constant__ unsigned long long kLcmOver[27] = {
    0ull,           26771144400ull, 13385572200ull, 8923714800ull, 6692786100ull,
    5354228880ull,  4461857400ull,  3824449200ull,  3346393050ull, 2974571600ull,
    2677114440ull,  2433740400ull,  2230928700ull,  2059318800ull, 1912224600ull,
    1784742960ull,  1673196525ull,  1574773200ull,  1487285800ull, 1409007600ull,
    1338557220ull,  1274816400ull,  1216870200ull,  1163962800ull, 1115464350ull,
    1070845776ull,  1029659400ull};
constexpr double kLcm26 = 26771144400.0;
constexpr double kRcpLcm26 = 1.0 / kLcm26;

// 13 forward neighbour offsets (dx, dy, dz), one of each +/- pair; bit d of
// the equal-level mask is forward direction d, bit 13 + d its opposite.
__host__ __device__ constexpr int fdx(int d) {
  return d == 0 ? 1 : d == 1 ? 0 : d == 2 ? 0 : d == 3 ? 1 : d == 4 ? -1 : d == 5 ? 1
       : d == 6 ? -1 : d == 7 ? 0 : d == 8 ? 0 : d == 9 ? 1 : d == 10 ? -1 : d == 11 ? 1 : -1;
}
__host__ __device__ constexpr int fdy(int d) {
  return d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 0 : d == 3 ? 1 : d == 4 ? 1 : d == 5 ? 0
       : d == 6 ? 0 : d == 7 ? 1 : d == 8 ? -1 : d == 9 ? 1 : d == 10 ? 1 : d == 11 ? -1 : -1;
}
__host__ __device__ constexpr int fdz(int d) {
  return d == 0 ? 0 : d == 1 ? 0 : d == 2 ? 1 : d == 3 ? 0 : d == 4 ? 0 : 1;
}
__host__ __device__ constexpr int ndx(int n) { return n < 13 ? fdx(n) : -fdx(n - 13); }
__host__ __device__ constexpr int ndy(int n) { return n < 13 ? fdy(n) : -fdy(n - 13); }
__host__ __device__ constexpr int ndz(int n) { return n < 13 ? fdz(n) : -fdz(n - 13); }

// 1/x from the hardware reciprocal refined by one Newton step (relative
// error ~1e-16; used where a quotient feeds a sum or a sign test).
__device__ inline double frcp(double x) {
  const double r0 = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r0, 1.0), r0, r0);
}

// log2 of a positive finite normal x, for the entropy terms: x = m 2^e with
// m in [1/sqrt 2, sqrt 2), ln m = 2 atanh(s), s = (m - 1) / (m + 1) (|s| <=
// 0.1716), by the odd series of atanh to s^15.  The first omitted term,
// 2 s^17 / 17 <= 1.2e-14 in ln m, bounds the error at about 2e-14 absolute
// in log2 (some hundred ulps near m = sqrt 2; the entropies it feeds are
// compared at 1e-5 relative).  Exact for powers of two.  About a third of
// the instructions of the library's double-double log2.
__device__ inline double flog2(double x) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) * frcp(m + 1.0), s2 = s * s;
  double t = 1.0 / 15.0;
  t = fma(t, s2, 1.0 / 13.0);
  t = fma(t, s2, 1.0 / 11.0);
  t = fma(t, s2, 1.0 / 9.0);
  t = fma(t, s2, 1.0 / 7.0);
  t = fma(t, s2, 1.0 / 5.0);
  t = fma(t, s2, 1.0 / 3.0);
  t = fma(t, s2, 1.0);
  constexpr double k2OverLn2 = 2.8853900817779268;  // 2 / ln 2
  return fma(s * t, k2OverLn2, (double)e);
}

}  // namespace
}  // namespace fr
