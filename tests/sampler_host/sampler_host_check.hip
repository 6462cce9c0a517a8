// Host build of the HIP path's binomial sampler (fluct.hpp): the cheap tests, then the
// search of the cell's regime, exactly as the raster kernels combine them, and the
// HIP path's Philox4x32-10 and 53-bit uniform.  The tests compare its output with the
// oracle's.
// Usage: sampler_host_check binom   stdin lines "N p u" (p, u as C99 hex floats)
//                                   -> one count per line
//        sampler_host_check binom_lockstep   the same, each search continuing for
//                                   (line number mod 9) passes after its own end, as a
//                                   lane does beside slower lanes of its wave
//        sampler_host_check philox  stdin lines "c0 c1 c2 c3 k0 k1" (decimal)
//                                   -> "w0 w1 w2 w3 u_even u_odd" (u as hex floats)
//        sampler_host_check erf     stdin lines "x" (hex float) -> det_erf(x) (hex float)
//        sampler_host_check normal  stdin lines "w0 w1 w2 w3 N p_even p_odd" (words and N
//                                   decimal, p as hex floats) -> "z_even z_odd n_even
//                                   n_odd sqrt(x) cos sin" for the normal-approximation
//                                   mode (x = p_even * 1e6, cos and sin of 2 pi p_odd)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fluct.hpp"

using namespace wct;

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  if (std::strcmp(argv[1], "philox") == 0) {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
      const Philox4 r = philox4x32_10(c0, c1, c2, c3, k0, k1);
      std::printf("%u %u %u %u %a %a\n", r.w0, r.w1, r.w2, r.w3, uniform53(r.w0, r.w1), uniform53(r.w2, r.w3));
    }
    return 0;
  }
  if (std::strcmp(argv[1], "erf") == 0) {
    char bx[64];
    while (std::scanf("%63s", bx) == 1) std::printf("%a\n", det_erf(std::strtod(bx, nullptr)));
    return 0;
  }
  if (std::strcmp(argv[1], "normal") == 0) {
    unsigned w0, w1, w2, w3;
    int N;
    char be[64], bo[64];
    while (std::scanf("%u %u %u %u %d %63s %63s", &w0, &w1, &w2, &w3, &N, be, bo) == 7) {
      const double pe = std::strtod(be, nullptr), po = std::strtod(bo, nullptr);
      double ze, zo, c, s;
      box_muller_pair(Philox4{w0, w1, w2, w3}, &ze, &zo);
      det_sincos2pi(po, &c, &s);
      std::printf("%a %a %d %d %a %a %a\n", ze, zo, normal_count(N, pe, ze), normal_count(N, po, zo),
                  det_sqrt(pe * 1e6), c, s);
    }
    return 0;
  }
  const bool lockstep = std::strcmp(argv[1], "binom_lockstep") == 0;
  if (std::strcmp(argv[1], "binom") != 0 && !lockstep) return 2;
  static const DetTables full = make_det_const();
  DetTablesSmall tb;
  for (int i = 0; i < 129; ++i) tb.inv[i] = full.inv[i];
  for (int i = 0; i < 19; ++i) tb.fact[i] = full.fact[i];
  // the plan's ln(n!) table: det_lfact over the full tables, as the device fills it
  std::vector<double> lf(kLfactTable);
  for (int i = 0; i < kLfactTable; ++i) lf[i] = det_lfact((int64_t)i, full);
  long long N;
  double p, u;
  char bp[64], bu[64];
  long line = 0;
  while (std::scanf("%lld %63s %63s", &N, bp, bu) == 3) {
    ++line;
    p = std::strtod(bp, nullptr);
    u = std::strtod(bu, nullptr);
    int64_t k = binom_quick(N, p, u);
    if (k < 0) {
      const int n = (int)N;
      wct_host_extra_passes = lockstep ? (int)(line % 9) : 0;
      const double lfN = lfact_of(n, lf.data(), tb);
      k = k == -1 ? binom_regime_draw<0>(n, lfN, p, u, tb, lf.data()) : binom_regime_draw<1>(n, lfN, p, u, tb, lf.data());
    }
    std::printf("%lld\n", (long long)k);
  }
  return 0;
}
