// Host check of the LDS Stockham transforms: runs the product's butterfly functions
// (bf_load / bf_store from fft.hpp) and plans (fftplan.hpp) over all butterflies of every
// pass on the CPU, exactly as a workgroup does (all loads of a pass, then all stores),
// and compares forward and inverse transforms with a direct long-double DFT.
// Usage: fft_host_check n policy C   -> prints "rel_fwd_f64 rel_inv_f64 rel_fwd_f32 rel_inv_f32 radices"
//        fft_host_check variants      -> one line per compiled variant (fftvariants.hpp): its radices
//          run with the compiled passes' butterflies (bfc_*), forward with the variant's table,
//          inverse with the reversed radices (as the column passes do), same error columns.
#include <cstdio>
#include <string>
#include <cstdlib>
#include <random>
#include <vector>

#include "fft.hpp"
#include "fftplan.hpp"

using namespace wct;

template <int R, typename T, bool INV, int C>
static void host_pass(std::vector<cx<T>>& buf, int n, int Ns, const cx<T>* tw) {
  const int nr = n / R, nbf = nr * C;
  std::vector<cx<T>> v((size_t)nbf * R);
  cx<T> w[R];
  for (int idx = 0; idx < nbf; ++idx) bf_load<R, T, C>(buf.data(), idx, nr, &v[(size_t)idx * R]);
  for (int idx = 0; idx < nbf; ++idx) {
    if (Ns > 1) bf_twiddles<R, T, C>(idx, Ns, tw, w);
    bf_store<R, T, INV, C>(buf.data(), idx, Ns, w, &v[(size_t)idx * R]);
  }
}

// Compiled-plan pass: bfc_* butterflies; POW = twiddles from one entry and its powers
// (the column transforms' policy).
template <typename T, bool INV, int C, int N, int R, int NS, bool POW>
static void host_ct_pass(std::vector<cx<T>>& buf, const cx<T>* tw) {
  constexpr int NR = N / R, NB = NR * C;
  std::vector<cx<T>> v((size_t)NB * R);
  cx<T> w[R];
  for (int idx = 0; idx < NB; ++idx) bfc_load<R, T, C, NR>(buf.data(), idx, &v[(size_t)idx * R]);
  for (int idx = 0; idx < NB; ++idx) {
    if constexpr (NS > 1) {
      if (POW) bfc_twiddles_pow<R, T, C, NS>(idx, tw, w);
      else bfc_twiddles<R, T, C, NS>(idx, tw, w);
    }
    bfc_store<R, T, INV, C, NS>(buf.data(), idx, w, &v[(size_t)idx * R]);
  }
}
template <typename T, bool INV, int C, int N, bool POW, int NS, int TWO, int R, int... Rest>
static void host_ct_fft(std::vector<cx<T>>& buf, const cx<T>* tw) {
  host_ct_pass<T, INV, C, N, R, NS, POW>(buf, tw + TWO);
  if constexpr (sizeof...(Rest) > 0) host_ct_fft<T, INV, C, N, POW, NS * R, TWO + NS * (R - 1), Rest...>(buf, tw);
}
template <typename T, bool INV, int C, int N, bool POW, int... Rs>
static void host_ct_list(std::vector<cx<T>>& buf, const cx<T>* tw, IntList<Rs...>) {
  host_ct_fft<T, INV, C, N, POW, 1, 0, Rs...>(buf, tw);
}

template <typename T, bool INV, int C>
static void host_fft(std::vector<cx<T>>& buf, const FftPlan& fp, const std::vector<cx<T>>& tw) {
  int Ns = 1;
  for (int p = 0; p < fp.npass; ++p) {
    const cx<T>* t = tw.data() + fp.tw_off[p];
    switch (fp.radix[p]) {
      case 2: host_pass<2, T, INV, C>(buf, fp.n, Ns, t); break;
      case 3: host_pass<3, T, INV, C>(buf, fp.n, Ns, t); break;
      case 4: host_pass<4, T, INV, C>(buf, fp.n, Ns, t); break;
      case 5: host_pass<5, T, INV, C>(buf, fp.n, Ns, t); break;
      case 6: host_pass<6, T, INV, C>(buf, fp.n, Ns, t); break;
      case 8: host_pass<8, T, INV, C>(buf, fp.n, Ns, t); break;
      case 9: host_pass<9, T, INV, C>(buf, fp.n, Ns, t); break;
      case 10: host_pass<10, T, INV, C>(buf, fp.n, Ns, t); break;
      default: std::abort();
    }
    Ns *= fp.radix[p];
  }
}

template <typename T, int C>
static void run(int n, int policy, const std::vector<cx<long double>>& x, const std::vector<cx<long double>>& X,
                double* efwd, double* einv, FftPlan* out_plan) {
  FftPlan fp;
  std::vector<cx<double>> twd;
  if (!build_fft(n, policy, fp, twd)) std::abort();
  *out_plan = fp;
  std::vector<cx<T>> tw(twd.size());
  for (size_t i = 0; i < tw.size(); ++i) tw[i] = mk((T)twd[i].x, (T)twd[i].y);
  std::vector<cx<T>> buf(x.size());
  for (size_t i = 0; i < x.size(); ++i) buf[i] = mk((T)x[i].x, (T)x[i].y);
  host_fft<T, false, C>(buf, fp, tw);
  long double num = 0, den = 0;
  for (size_t i = 0; i < X.size(); ++i) {
    const long double dx = buf[i].x - X[i].x, dy = buf[i].y - X[i].y;
    num += dx * dx + dy * dy;
    den += X[i].x * X[i].x + X[i].y * X[i].y;
  }
  *efwd = (double)sqrtl(num / den);
  host_fft<T, true, C>(buf, fp, tw);  // unnormalised inverse: n * x
  num = den = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    const long double dx = buf[i].x / n - x[i].x, dy = buf[i].y / n - x[i].y;
    num += dx * dx + dy * dy;
    den += x[i].x * x[i].x + x[i].y * x[i].y;
  }
  *einv = (double)sqrtl(num / den);
}

static void dft_ref(int n, int C, const std::vector<cx<long double>>& x, std::vector<cx<long double>>& X);

template <typename T>
static std::vector<cx<T>> table(const std::vector<int>& rad, int n) {
  FftPlan fp;
  std::vector<cx<double>> twd;
  if (!build_fft_radices(n, rad, fp, twd)) std::abort();
  std::vector<cx<T>> tw(twd.size());
  for (size_t i = 0; i < tw.size(); ++i) tw[i] = mk((T)twd[i].x, (T)twd[i].y);
  return tw;
}

template <typename T>
static double rel(const std::vector<cx<T>>& got, const std::vector<cx<long double>>& ref, long double scale) {
  long double num = 0, den = 0;
  for (size_t i = 0; i < ref.size(); ++i) {
    const long double dx = got[i].x / scale - ref[i].x, dy = got[i].y / scale - ref[i].y;
    num += dx * dx + dy * dy;
    den += ref[i].x * ref[i].x + ref[i].y * ref[i].y;
  }
  return (double)sqrtl(num / den);
}

// Forward with the variant's radices, inverse with them reversed; returns (fwd, inv) errors.
template <typename T, int C, int NT, int... Rs>
static void check_variant(double* ef, double* ei) {
  constexpr int N = (1 * ... * Rs);
  constexpr bool POW = C > 1;
  std::mt19937_64 rng(777 + N);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<cx<long double>> x((size_t)N * C), X;
  for (auto& v : x) v = mk((long double)U(rng), (long double)U(rng));
  dft_ref(N, C, x, X);
  std::vector<cx<T>> buf(x.size());
  for (size_t i = 0; i < x.size(); ++i) buf[i] = mk((T)x[i].x, (T)x[i].y);
  const std::vector<int> rad = {Rs...};
  std::vector<int> rev(rad.rbegin(), rad.rend());
  const std::vector<cx<T>> tw = table<T>(rad, N), twr = table<T>(rev, N);
  host_ct_list<T, false, C, N, POW>(buf, tw.data(), IntList<Rs...>{});
  *ef = rel(buf, X, 1.0L);
  host_ct_list<T, true, C, N, POW>(buf, twr.data(), typename RevList<IntList<Rs...>>::type{});
  *ei = rel(buf, x, (long double)N);
}

static int run_variants() {
#define WCT_CHECK_VARIANT(K, TT, NT, MW, ...)                                                        \
  {                                                                                              \
    double ef = 0, ei = 0, ef32 = 0, ei32 = 0;                                                   \
    check_variant<double, (K == 0 ? 1 : K == 1 ? kChunk : kChunk / 2), NT, __VA_ARGS__>(&ef, &ei);  \
    check_variant<float, (K == 0 ? 1 : K == 1 ? kChunk : kChunk / 2), NT, __VA_ARGS__>(&ef32, &ei32); \
    std::printf("%d %d %d %.3e %.3e %.3e %.3e %s\n", K, (int)sizeof(TT), NT, ef, ei, ef32, ei32, #__VA_ARGS__); \
  }
  WCT_FFT_VARIANTS(WCT_CHECK_VARIANT)
#undef WCT_CHECK_VARIANT
  return 0;
}

static void dft_ref(int n, int C, const std::vector<cx<long double>>& x, std::vector<cx<long double>>& X) {
  X.assign((size_t)n * C, mk(0.0L, 0.0L));
  const long double tau = 6.283185307179586476925286766559005768L;
  std::vector<long double> tc(n), ts(n);
  for (int m = 0; m < n; ++m) {
    tc[m] = cosl(-tau * (long double)m / n);
    ts[m] = sinl(-tau * (long double)m / n);
  }
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < n; ++k) {
      long double sx = 0, sy = 0;
      for (int m = 0; m < n; ++m) {
        const int q = (int)(((long long)m * k) % n);
        const cx<long double> v = x[(size_t)m * C + c];
        sx += v.x * tc[q] - v.y * ts[q];
        sy += v.x * ts[q] + v.y * tc[q];
      }
      X[(size_t)k * C + c] = mk(sx, sy);
    }
}

int main(int argc, char** argv) {
  if (argc == 2 && std::string(argv[1]) == "variants") return run_variants();
  if (argc < 4) return 2;
  const int n = std::atoi(argv[1]), policy = std::atoi(argv[2]), C = std::atoi(argv[3]);
  std::mt19937_64 rng(12345 + n);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<cx<long double>> x((size_t)n * C), X((size_t)n * C);
  for (auto& v : x) v = mk((long double)U(rng), (long double)U(rng));
  const long double tau = 6.283185307179586476925286766559005768L;
  std::vector<long double> tc(n), ts(n);
  for (int m = 0; m < n; ++m) {
    tc[m] = cosl(-tau * (long double)m / n);
    ts[m] = sinl(-tau * (long double)m / n);
  }
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < n; ++k) {
      long double sx = 0, sy = 0;
      for (int m = 0; m < n; ++m) {
        const int q = (int)(((long long)m * k) % n);
        const long double cr = tc[q], ci = ts[q];
        const cx<long double> v = x[(size_t)m * C + c];
        sx += v.x * cr - v.y * ci;
        sy += v.x * ci + v.y * cr;
      }
      X[(size_t)k * C + c] = mk(sx, sy);
    }
  double f64f, f64i, f32f, f32i;
  FftPlan fp;
  if (C == 1) {
    run<double, 1>(n, policy, x, X, &f64f, &f64i, &fp);
    run<float, 1>(n, policy, x, X, &f32f, &f32i, &fp);
  } else {
    run<double, 4>(n, policy, x, X, &f64f, &f64i, &fp);
    run<float, 4>(n, policy, x, X, &f32f, &f32i, &fp);
  }
  std::printf("%.3e %.3e %.3e %.3e", f64f, f64i, f32f, f32i);
  for (int p = 0; p < fp.npass; ++p) std::printf(" %d", fp.radix[p]);
  std::printf("\n");
  return 0;
}
