// Host check of the LDS Stockham transforms: runs the product's butterfly functions
// (bf_load / bf_store from fft.hpp) and plans (fftplan.hpp) over all butterflies of every
// pass on the CPU, exactly as a workgroup does (all loads of a pass, then all stores),
// and compares forward and inverse transforms with a direct long-double DFT.
// Usage: fft_host_check n policy C   -> prints "maxrel_fwd_f64 maxrel_inv_f64 maxrel_fwd_f32 radices"
#include <cstdio>
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
  for (int idx = 0; idx < nbf; ++idx) bf_load<R, T, C>(buf.data(), idx, nr, &v[(size_t)idx * R]);
  for (int idx = 0; idx < nbf; ++idx) bf_store<R, T, INV, C>(buf.data(), idx, Ns, tw, &v[(size_t)idx * R]);
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

int main(int argc, char** argv) {
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
