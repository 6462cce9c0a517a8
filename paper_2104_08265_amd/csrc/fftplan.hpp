// Host-side planning of the LDS transforms: radix sequences and twiddle tables.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "fftvariants.hpp"

namespace wct {

// exp(-2 pi i m / n) with the angle reduced exactly and evaluated in long double.
inline cx<double> wexp(int64_t m, int64_t n) {
  m %= n;
  if (m < 0) m += n;
  const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
  return mk((double)cosl(a), (double)sinl(a));
}

// Radix policies (the autotuner may try several):
//  0: fewest passes over radices {10, 9, 8, 6, 5, 4, 3, 2}, odd radices first;
//  1: fewest passes over radices {8, 5, 4, 3, 2}, odd radices first;
//  2: as 0 but in descending radix order.
// Odd radices first keep the early passes (small stride Ns) free of the power-of-two
// LDS write strides that even radices produce there.
inline bool plan_radices(int n, int policy, std::vector<int>& out) {
  out.clear();
  int a = 0, b = 0, c = 0, r = n;
  while (r % 2 == 0) r /= 2, ++a;
  while (r % 3 == 0) r /= 3, ++b;
  while (r % 5 == 0) r /= 5, ++c;
  if (r != 1 || n < 1) return false;
  struct Rad { int r, a, b, c; };
  std::vector<Rad> set = policy == 1
      ? std::vector<Rad>{{8, 3, 0, 0}, {5, 0, 0, 1}, {4, 2, 0, 0}, {3, 0, 1, 0}, {2, 1, 0, 0}}
      : std::vector<Rad>{{10, 1, 0, 1}, {9, 0, 2, 0}, {8, 3, 0, 0}, {6, 1, 1, 0},
                         {5, 0, 0, 1},  {4, 2, 0, 0}, {3, 0, 1, 0}, {2, 1, 0, 0}};
  // DP over exponents: fewest passes; ties prefer a plan with an odd radix (to lead
  // with), then the larger smallest radix
  const int A = a + 1, B = b + 1, Cc = c + 1;
  std::vector<int> best(A * B * Cc, 1 << 20), minr(A * B * Cc, 0), pick(A * B * Cc, -1), odd(A * B * Cc, 0);
  best[0] = 0;
  minr[0] = 1 << 20;
  for (int ia = 0; ia < A; ++ia)
    for (int ib = 0; ib < B; ++ib)
      for (int ic = 0; ic < Cc; ++ic) {
        const int id = (ia * B + ib) * Cc + ic;
        if (id == 0) continue;
        for (int k = 0; k < (int)set.size(); ++k) {
          const Rad& R = set[k];
          if (R.a > ia || R.b > ib || R.c > ic) continue;
          const int pid = ((ia - R.a) * B + (ib - R.b)) * Cc + (ic - R.c);
          if (best[pid] >= (1 << 20)) continue;
          const int np = best[pid] + 1, mr = std::min(minr[pid], R.r), od = odd[pid] | (R.r & 1);
          if (np < best[id] || (np == best[id] && (od > odd[id] || (od == odd[id] && mr > minr[id])))) {
            best[id] = np;
            minr[id] = mr;
            odd[id] = od;
            pick[id] = k;
          }
        }
      }
  for (int ia = a, ib = b, ic = c; ia || ib || ic;) {
    const int id = (ia * B + ib) * Cc + ic;
    const Rad& R = set[pick[id]];
    out.push_back(R.r);
    ia -= R.a, ib -= R.b, ic -= R.c;
  }
  if (policy == 2) {
    std::sort(out.begin(), out.end(), [](int x, int y) { return x > y; });
  } else {
    std::stable_sort(out.begin(), out.end(), [](int x, int y) {
      const bool ox = x % 2 == 1, oy = y % 2 == 1;
      if (ox != oy) return ox;  // odd radices first
      return ox ? x > y : x < y;
    });
  }
  return (int)out.size() <= kMaxPass;
}

// Stockham plan for the radices `rad` (in pass order) and its twiddle table: pass p
// with stride Ns and radix R keeps W_{Ns R}^{r k} for k < Ns, 1 <= r < R at
// tw_off[p] + k (R-1) + r - 1.
inline bool build_fft_radices(int n, const std::vector<int>& rad, FftPlan& fp, std::vector<cx<double>>& tw) {
  std::memset(&fp, 0, sizeof(fp));
  fp.n = n;
  fp.variant = -1;
  if (rad.empty() || (int)rad.size() > kMaxPass) return false;
  int64_t prod = 1;
  for (int r : rad) prod *= r;
  if (prod != n) return false;
  tw.clear();
  int Ns = 1;
  fp.npass = (int)rad.size();
  for (int p = 0; p < fp.npass; ++p) {
    const int R = rad[p];
    fp.radix[p] = R;
    fp.tw_off[p] = (int)tw.size();
    for (int k = 0; k < Ns; ++k)
      for (int q = 1; q < R; ++q) tw.push_back(wexp((int64_t)q * k, (int64_t)Ns * R));
    Ns *= R;
  }
  if (tw.empty()) tw.push_back(mk(1.0, 0.0));
  return true;
}

// Runtime plan of a radix policy.
inline bool build_fft(int n, int policy, FftPlan& fp, std::vector<cx<double>>& tw) {
  std::vector<int> rad;
  if (!plan_radices(n, policy, rad)) return false;
  return build_fft_radices(n, rad, fp, tw);
}

// Plan of compiled variant v (fftvariants.hpp).
inline bool build_fft_variant(const FftVariantDesc& d, int v, FftPlan& fp, std::vector<cx<double>>& tw) {
  std::vector<int> rad(d.radix, d.radix + d.npass);
  if (!build_fft_radices(d.n, rad, fp, tw)) return false;
  fp.variant = v;
  return true;
}

}  // namespace wct
