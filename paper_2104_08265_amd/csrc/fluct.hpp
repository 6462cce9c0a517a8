// Binomial fluctuation of rasterised charge (arXiv:2104.08265 Sec. 4.3.1, Table 2: the
// fluctuation is binomial; generating the random numbers dominated the CPU time, so
// the generator is counter-based and inline here, with no pool and no host traffic).
//
// Draw stream, version WCT_FLUCT_SPEC_VERSION = 2:
//  * generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed low,
//    seed high); cells (b, 2m) and (b, 2m+1) share the block with counter
//    (b*ceil(N_t/2) + m, depo_id, event, plane << 24);
//  * variate: u = ((x >> 6) * 2^27 + (y >> 5)) * 2^-53, exact, in [0, 1), with
//    (x, y) = words (0, 1) for the even tick and words (2, 3) for the odd tick;
//  * count: Binomial(N = floor(Q + 1/2), p = A_b * B_k) by inversion from 0 when
//    N*p' < 10 (p' = min(p, 1-p)), otherwise by a chop-down search alternating below
//    and above the mode; p > 1/2 is sampled as N minus a draw with 1-p.
// Every operation is an IEEE-754 double +, -, *, / (this file must be compiled with
// floating-point contraction off), frexp, ldexp, rint, floor, in a fixed order, so the
// counts do not depend on the device, the schedule or the compiler's choices.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wct {

// Host and device: the host build serves the CPU checks of the sampler.
#define WCT_HD __host__ __device__ __forceinline__

// Small tables, filled on the host with correctly rounded divisions (kept in LDS for
// the loops that index them at run time).
struct DetTables {
  double inv[256];      // inv[j] = 1/j (inv[0] = 0)
  double inv_fact[17];  // 1/j!
  double fact[19];      // j! (exact)
};

// The same values as compile-time constants for the fully unrolled series (erf, log,
// exp): each entry is one correctly rounded division, as on the host, and unrolled use
// keeps them out of vector registers.
constexpr DetTables make_det_const() {
  DetTables t{};
  t.inv[0] = 0.0;
  for (int j = 1; j < 256; ++j) t.inv[j] = 1.0 / (double)j;
  double f = 1.0;
  t.fact[0] = 1.0;
  t.inv_fact[0] = 1.0;
  for (int j = 1; j < 19; ++j) {
    f = f * (double)j;
    t.fact[j] = f;
    if (j <= 16) t.inv_fact[j] = 1.0 / f;
  }
  return t;
}
constexpr DetTables kDet = make_det_const();

// The part of the tables the sampler indexes at run time (inversion: 1/(k+1) for
// k < kInversionCap; ln(n!) for n <= 18), small enough for LDS next to a raster tile.
struct DetTablesSmall {
  double inv[129];
  double fact[19];
};

constexpr double kTwoOverSqrtPi = 1.1283791670955126;
constexpr double kSqrt2 = 1.4142135623730951;
constexpr double kSqrtHalf = 0.7071067811865476;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kLog2e = 1.4426950408889634;
constexpr double kHalfLn2Pi = 0.91893853320467274;
constexpr int kErfTerms = 60;
constexpr double kMuSwitch = 10.0;
constexpr int64_t kInversionCap = 128;

struct Philox4 {
  uint32_t w0, w1, w2, w3;
};

WCT_HD Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Philox4{c0, c1, c2, c3};
}

WCT_HD double uniform53(uint32_t w0, uint32_t w1) {
  return ((double)(w0 >> 6) * 134217728.0 + (double)(w1 >> 5)) * 0x1p-53;
}

// Whether the predicate holds on any active lane of the wave (on the host: for the one
// caller).
WCT_HD bool wave_any(bool v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __ballot(v) != 0;
#else
  return v;
#endif
}

// The series' added terms a_j = x^(2j+1) / (j! (2j+1)) shrink in magnitude from j >= x^2
// on.  Once one of them is at most 2^-55 |acc| (below a quarter unit in the last place of
// acc), it and every later one leave acc unchanged under round-to-nearest, so the sum
// stops there with the bits of the full kErfTerms-term sum.  The test runs at a few
// checkpoints only, and the lanes of a wave stop together (a lane that could stop keeps
// adding terms that change nothing).
WCT_HD double det_erf(double x) {
  const double mx2 = -(x * x);
  double term = x, acc = x;
  bool more = true;  // this lane's sum may still change
#pragma unroll
  for (int j = 1; j < kErfTerms; ++j) {
    term = (term * mx2) * kDet.inv[j];
    const double a = term * kDet.inv[2 * j + 1];
    acc = acc + a;
    if (j >= 24 && j % 6 == 0) {
      more = more && !((double)j >= -mx2 && fabs(a) <= fabs(acc) * 0x1p-55);
      if (!wave_any(more)) break;
    }
  }
  return kTwoOverSqrtPi * acc;
}

WCT_HD double det_log(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double poly = kDet.inv[23];
#pragma unroll
  for (int j = 10; j >= 0; --j) poly = poly * s2 + kDet.inv[2 * j + 1];
  return (s * poly) * 2.0 + (double)e * kLn2;
}

WCT_HD double det_exp(double x) {
  const double n = rint(x * kLog2e);
  const double r = x - n * kLn2;
  double poly = kDet.inv_fact[16];
#pragma unroll
  for (int j = 15; j >= 0; --j) poly = poly * r + kDet.inv_fact[j];
  return ldexp(poly, (int)n);
}

template <typename Tab>
WCT_HD double det_lfact(int64_t n, const Tab& tb) {
  // one det_log call site: the argument is n! (exact) for small n, else n
  const double x = (double)n;
  const double lg = det_log(n <= 18 ? tb.fact[n] : x);
  if (n <= 18) return lg;
  const double r = 1.0 / x;
  const double r2 = r * r;
  const double series = r * ((1.0 / 12.0) - r2 * ((1.0 / 360.0) - r2 * ((1.0 / 1260.0) - r2 * (1.0 / 1680.0))));
  return (x + 0.5) * lg - x + kHalfLn2Pi + series;
}

// ln(n!) for n < kLfactTable is read from a table the plan fills with det_lfact itself
// (same code, same bits); larger n are evaluated.
constexpr int kLfactTable = 1 << 17;
template <typename Tab>
WCT_HD double lfact_of(int64_t n, const double* __restrict__ lf, const Tab& tb) {
  return (lf && n < kLfactTable) ? lf[n] : det_lfact(n, tb);
}

// Count k of Binomial(N, p) from the uniform u: inversion from k = 0 when N p' < 10
// (p' = min(p, 1 - p)), else a chop-down search that starts at the mode and alternates a
// step below with a step above; p > 1/2 is drawn as N minus a draw with 1 - p.  The
// cheap cases are decided first (binom_quick), the two searches are separate entry
// points (binom_regime_draw), so that a caller can gather the cells of one regime and
// run them together.  Lanes that run a search together share N (0 < N < 2^31):
// integers enter the arithmetic as doubles kept up to date by exact +-1 steps, and in
// the inversion every lane still searching has taken the same number of steps, so the
// step's table entry is one shared read, issued two steps ahead.
WCT_HD int binom_regime(int64_t N, double p) {
  const double pp = p > 0.5 ? 1.0 - p : p;
  return (double)N * pp < kMuSwitch ? 0 : 1;
}

// The count when the cheap tests decide it (>= 0), else -1 - (regime of the search).
// Zero bound: the inversion returns 0 when u < F(0), the computed q^N.  The rounded q is
// at least 1 - (p + 2^-53), so by Bernoulli's inequality the exact power of it is at
// least 1 - N p - N 2^-53; the square-and-multiply adds at most 128 roundings (< 2e-14)
// and mu = N p carries < 2e-15.  Hence u below (1 - mu) - (1e-12 + 2.5e-16 N) implies
// u < F(0): the search would return 0.
// The tests are combined without branches (the same comparisons and the same mu).  The
// kernels call it with 32-bit counts (Int = int), the host checks with int64_t.
template <typename Int>
WCT_HD Int binom_quick(Int N, double p, double u) {
  const double Nf = (double)N;
  const double mu = Nf * p;  // the zero bound's mean (used where p <= 1/2)
  const bool none = (N <= 0) | !(p > 0.0);
  const bool all = p >= 1.0;
  const bool zero = (p <= 0.5) & (mu < kMuSwitch) & (u < (1.0 - mu) - (1.0e-12 + Nf * 2.5e-16));
  const double pp = p > 0.5 ? 1.0 - p : p;
  const Int search = Nf * pp < kMuSwitch ? -1 : -2;  // -1 - binom_regime(N, p)
  return none ? Int(0) : (all ? N : (zero ? Int(0) : search));
}

#if defined(WCT_HOST_LOCKSTEP)
inline thread_local int wct_host_extra_passes = 0;
#endif

// wave_any for the sampler's loops, which end on it (uniform control); the host check
// of the lockstep property can make it report more passes.
WCT_HD bool any_lane(bool v) {
#if !defined(__HIP_DEVICE_COMPILE__) && defined(WCT_HOST_LOCKSTEP)
  // the caller sets extra passes that a lane takes after its own search has ended, as it
  // does beside slower lanes of its wave
  if (wct_host_extra_passes > 0) {
    --wct_host_extra_passes;
    return true;
  }
#endif
  return wave_any(v);
}

template <typename Tab>
WCT_HD int binom_inversion_shared(int N, double pp, double q, double u, const Tab& tb) {
  // q^N by left-to-right square-and-multiply: the leading bit of N gives q exactly, then
  // each lower bit squares, and each set one multiplies by q (N is shared by the lanes, so
  // the bit tests are scalar)
  double f = q;
  const int top = 31 - __builtin_clz((unsigned)N);
  for (int i = top - 1; i >= 0; --i) {
    f = f * f;
    if ((N >> i) & 1) {  // a uniform branch: the product only where the bit is set
      f = f * q;
#if defined(__HIP_DEVICE_COMPILE__)
      // keeps the compiler from turning the branch into an unconditional product and a
      // 64-bit select (three vector instructions for every bit instead of one per set bit)
      __asm__ volatile("" : "+v"(f));
#endif
    }
  }
  // F(k) = F(k-1) + f(k), f(k) = f(k-1) * (r (N - k + 1)) / k, while u >= F and k < cap.
  // Every lane takes the shared steps s = 0, 1, ... (the loop ends once no lane has
  // u >= F, or at the cap) and counts those it takes while u >= F: F never decreases, so
  // that count is the step at which its own search stops, and each lane's F and f up to
  // that step are the search's own.  The loop control is then uniform (no per-lane exit),
  // two steps per pass, and 1/k is a scalar load from the constant table.
  const double r = pp / q;
  double F = f;
  const int cap = N < kInversionCap ? N : (int)kInversionCap;
  double nk = (double)N;  // N - s
  int k = 0;
  int s = 0;
  double i1 = kDet.inv[1], i2 = kDet.inv[2];  // 1/(s + 1), 1/(s + 2), loaded a pass ahead
  for (; s + 2 <= cap; s += 2) {
    if (!any_lane(u >= F)) break;
    const double n1 = kDet.inv[s + 3], n2 = kDet.inv[s + 4];
    k += u >= F ? 1 : 0;
    f = (f * (r * nk)) * i1;
    F = F + f;
    nk = nk - 1.0;
    k += u >= F ? 1 : 0;
    f = (f * (r * nk)) * i2;
    F = F + f;
    nk = nk - 1.0;
    i1 = n1;
    i2 = n2;
  }
  if (s < cap) k += u >= F ? 1 : 0;  // an odd cap: one last step (its f is not needed)
  return k;
}

template <typename Tab>
WCT_HD int binom_chopdown_shared(int N, double lfN, double pp, double q, double u, const Tab& tb,
                                 const double* __restrict__ lf) {
  // mode m = floor((N + 1) p'), P(m) = exp(ln N! - ln m! - ln (N - m)! + m ln p' + (N - m) ln q)
  const double Nf = (double)N;
  int m = (int)floor((Nf + 1.0) * pp);
  if (m > N) m = N;
  // the table reads go first: their latency overlaps the two logarithms
  const double lfm = lfact_of(m, lf, tb), lfnm = lfact_of(N - m, lf, tb);
  const double lp = det_log(pp), lq = det_log(q);
  const double x = lfN - lfm - lfnm + (double)m * lp + (double)(N - m) * lq;
  const double pm = det_exp(x);
  double v = u - pm;
  int lo = m, hi = m;
  double plo = pm, phi = pm;
  double dlo = (double)m, dnlo = (double)(N - m + 1);     // lo, N - lo + 1
  double dnhi = (double)(N - m), dhi1 = (double)m + 1.0;  // N - hi, hi + 1
  // Each pass takes a step below (while the lower side is neither at 0 nor underflowed),
  // subtracts its probability from v, then a step above under the same rule; the count
  // is the index at which v first drops below 0 (m if v = u - P(m) already is), or m once
  // neither side can step.  A side
  // that cannot step is stepped anyway: at lo = 0 (or hi = N) its factor lo (or N - hi) is
  // 0, and an underflowed probability stays 0, so the probability added is a zero and v is
  // unchanged.  A lane whose v is already negative keeps stepping with its count fixed.
  // So every lane runs the same instructions and the loop ends, for the wave, once no lane
  // is still searching (uniform control, no per-lane exits).
  int k = m;
  bool searching = !(v < 0.0);  // u below P(m): the mode
  for (;;) {
    searching = searching & (((lo > 0) & (plo > 0.0)) | ((hi < N) & (phi > 0.0)));
    if (!any_lane(searching)) break;
    plo = plo * (dlo * q) / (dnlo * pp);
    lo -= 1;
    dlo = dlo - 1.0;
    dnlo = dnlo + 1.0;
    v = v - plo;
    const bool hit_lo = searching & (v < 0.0);
    k = hit_lo ? lo : k;
    searching = searching & !hit_lo;
    phi = phi * (dnhi * pp) / (dhi1 * q);
    hi += 1;
    dnhi = dnhi - 1.0;
    dhi1 = dhi1 + 1.0;
    v = v - phi;
    const bool hit_hi = searching & (v < 0.0);
    k = hit_hi ? hi : k;
    searching = searching & !hit_hi;
  }
  return k;
}

// The search of regime REGIME (binom_regime) for 0 < N < 2^31 and 0 < p < 1; lfN is
// ln(N!) as lfact_of gives it.
template <int REGIME, typename Tab>
WCT_HD int binom_regime_draw(int N, double lfN, double p, double u, const Tab& tb, const double* __restrict__ lf) {
  const bool flip = p > 0.5;
  const double pp = flip ? 1.0 - p : p;
  const double q = 1.0 - pp;
  const int k =
      REGIME == 0 ? binom_inversion_shared(N, pp, q, u, tb) : binom_chopdown_shared(N, lfN, pp, q, u, tb, lf);
  return flip ? N - k : k;
}

// Normal-approximation mode (Sec. 4.3.1: the Kokkos port drew normal deviates with the
// Box-Muller transform).  A cell's count is min(max(floor(N p + sqrt(N p (1 - p)) z + 1/2),
// 0), N); the cells (b, 2m) and (b, 2m+1) take the two normals of one Box-Muller pair
// from their shared Philox block: u1 = 1 - uniform53(words 0, 1) in (0, 1], u2 =
// uniform53(words 2, 3), r = sqrt(-2 ln u1), z = r cos(2 pi u2) (even tick) and
// r sin(2 pi u2) (odd tick).  sqrt, cos and sin below use +, -, *, / only, like the
// sampler, so the counts are reproducible bit for bit.

// sqrt(x), x >= 0: x = m 2^e with e even and m in [1/2, 2); seven Newton steps on
// y = 1/sqrt(m) from y = 3/2 - m/2 (quadratic convergence from a start within 30%), then
// sqrt(x) = (m y) 2^(e/2); within two units in the last place.
constexpr int kRsqrtSteps = 7;
WCT_HD double det_sqrt(double x) {
  if (!(x > 0.0)) return 0.0;
  int e;
  double m = frexp(x, &e);
  if (e & 1) {
    m = m * 2.0;
    e = e - 1;
  }
  double y = 1.5 - m * 0.5;
#pragma unroll
  for (int i = 0; i < kRsqrtSteps; ++i) y = y * (1.5 - ((m * y) * y) * 0.5);
  return ldexp(m * y, e / 2);
}

// cos(2 pi u) and sin(2 pi u) for u in [0, 1): t = 4u (exact), quadrant j = floor(t),
// f = t - j; g = 1 - f (exact) when f > 1/2, else f; x = g pi/2 in [0, pi/4]; sin x and
// cos x by their Maclaurin series to x^15 and x^16 (Horner form, 1/j! correctly rounded);
// the complement swaps the pair and the quadrant rotates it.
constexpr double kHalfPi = 1.5707963267948966;
WCT_HD void det_sincos2pi(double u, double* c_out, double* s_out) {
  const double t = u * 4.0;
  const double jf = floor(t);
  const double f = t - jf;
  const bool swap = f > 0.5;
  const double g = swap ? 1.0 - f : f;
  const double x = g * kHalfPi;
  const double x2 = x * x;
  double s = kDet.inv_fact[15];
#pragma unroll
  for (int n = 13; n >= 1; n -= 2) s = kDet.inv_fact[n] - x2 * s;
  s = x * s;
  double c = kDet.inv_fact[16];
#pragma unroll
  for (int n = 14; n >= 0; n -= 2) c = kDet.inv_fact[n] - x2 * c;
  const double sp = swap ? c : s, cp = swap ? s : c;  // sin, cos of (pi/2) f
  const int j = (int)jf;
  *c_out = j == 0 ? cp : (j == 1 ? -sp : (j == 2 ? -cp : sp));
  *s_out = j == 0 ? sp : (j == 1 ? cp : (j == 2 ? -sp : -cp));
}

// The two normals of a tick pair's Philox block (even tick first).
WCT_HD void box_muller_pair(const Philox4& ph, double* z_even, double* z_odd) {
  const double u1 = 1.0 - uniform53(ph.w0, ph.w1);
  const double u2 = uniform53(ph.w2, ph.w3);
  const double r = det_sqrt(-2.0 * det_log(u1));
  double c, s;
  det_sincos2pi(u2, &c, &s);
  *z_even = r * c;
  *z_odd = r * s;
}

// The normal approximation's count for N >= 0 electrons, probability p in [0, 1], normal z.
WCT_HD int normal_count(int N, double p, double z) {
  const double Nf = (double)N;
  const double mu = Nf * p;
  const double var = mu * (1.0 - p);
  const double sd = det_sqrt(var > 0.0 ? var : 0.0);
  const double x = floor((mu + sd * z) + 0.5);
  return (int)(x < 0.0 ? 0.0 : (x > Nf ? Nf : x));
}

}  // namespace wct
