// FP64 host-side preparation of the kernels the passes multiply by.
#include "mvd_host.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <thread>

namespace mvdh {

namespace {

int n_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return (int)std::min(h, 32u);
}

// Run f(i) for i in [0, n) on a few threads; the first exception thrown by
// f is rethrown on the calling thread once every thread has finished.
void parallel_for(int n, const std::function<void(int)>& f) {
  const int nt = std::min(n, n_threads());
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&] {
      try {
        for (int i = next++; i < n; i = next++) f(i);
      } catch (...) {
        std::lock_guard<std::mutex> lock(mu);
        if (!err) err = std::current_exception();
        next = n;
      }
    });
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace

bool all_within(const float* x, int64_t n, float lo, float hi) {
  constexpr int64_t chunk = 1 << 20;
  const int nc = (int)((n + chunk - 1) / chunk);
  std::atomic<bool> ok{true};
  parallel_for(nc, [&](int c) {
    if (!ok.load(std::memory_order_relaxed)) return;
    const int64_t a = (int64_t)c * chunk, b = std::min(n, a + chunk);
    // comparisons are false for NaN; the last one rejects +inf when hi is +inf
    int64_t nbad = 0;
    for (int64_t i = a; i < b; ++i) nbad += !(x[i] >= lo && x[i] <= hi && x[i] < INFINITY);
    if (nbad) ok = false;
  });
  return ok;
}

namespace {

// f[i] += b[i] * w for i < n, in real arithmetic (vectorises)
inline void cmac(cd* f, const cd* b, cd w, size_t n) {
  const double wr = w.real(), wi = w.imag();
  const double* bp = reinterpret_cast<const double*>(b);
  double* fp = reinterpret_cast<double*>(f);
  for (size_t i = 0; i < n; ++i) {
    const double br = bp[2 * i], bi = bp[2 * i + 1];
    fp[2 * i] += br * wr - bi * wi;
    fp[2 * i + 1] += br * wi + bi * wr;
  }
}

inline int wrap(long long k, long long d, int n) {
  long long m = (k * d) % n;
  if (m < 0) m += n;
  return (int)m;
}

// Centred DFT of K on a periodic grid (gx, gy, gz), full complex [kz][ky][kx]:
// F[k] = sum_d K[c + d] exp(-2 pi i k.d / g).
std::vector<cd> dft_grid(const Kern& K, int gx, int gy, int gz) {
  const auto tx = twiddles(gx), ty = twiddles(gy), tz = twiddles(gz);
  const int cx = (K.kx - 1) / 2, cy = (K.ky - 1) / 2, cz = (K.kz - 1) / 2;
  std::vector<cd> A((size_t)K.kz * K.ky * gx);
  for (int z = 0; z < K.kz; ++z)
    for (int y = 0; y < K.ky; ++y)
      for (int k = 0; k < gx; ++k) {
        // phase index k (x - cx) mod gx, stepped by k along x
        int idx = wrap(k, -cx, gx);
        cd s = 0;
        for (int x = 0; x < K.kx; ++x) {
          s += K.at(z, y, x) * tx[idx];
          idx += k;
          if (idx >= gx) idx -= gx;
        }
        A[((size_t)z * K.ky + y) * gx + k] = s;
      }
  std::vector<cd> B((size_t)K.kz * gy * gx);
  for (int z = 0; z < K.kz; ++z)
    for (int k = 0; k < gy; ++k)
      for (int y = 0; y < K.ky; ++y) {
        const cd w = ty[wrap(k, y - cy, gy)];
        cmac(&B[((size_t)z * gy + k) * gx], &A[((size_t)z * K.ky + y) * gx], w, gx);
      }
  std::vector<cd> F((size_t)gz * gy * gx);
  for (int k = 0; k < gz; ++k)
    for (int z = 0; z < K.kz; ++z) {
      const cd w = tz[wrap(k, z - cz, gz)];
      cmac(&F[(size_t)k * gy * gx], &B[(size_t)z * gy * gx], w, (size_t)gy * gx);
    }
  return F;
}

// Inverse DFT of S on the grid, evaluated only at offsets d in the centred
// window (wx, wy, wz); real part, divided by the grid size.
std::vector<double> idft_window(const std::vector<cd>& S, int gx, int gy, int gz, int wx, int wy,
                                int wz) {
  const auto tx = twiddles(gx), ty = twiddles(gy), tz = twiddles(gz);
  const int cx = (wx - 1) / 2, cy = (wy - 1) / 2, cz = (wz - 1) / 2;
  std::vector<cd> T1((size_t)wz * gy * gx);
  for (int z = 0; z < wz; ++z)
    for (int k = 0; k < gz; ++k) {
      const cd w = std::conj(tz[wrap(k, z - cz, gz)]);
      cmac(&T1[(size_t)z * gy * gx], &S[(size_t)k * gy * gx], w, (size_t)gy * gx);
    }
  std::vector<cd> T2((size_t)wz * wy * gx);
  for (int z = 0; z < wz; ++z)
    for (int y = 0; y < wy; ++y)
      for (int k = 0; k < gy; ++k) {
        const cd w = std::conj(ty[wrap(k, y - cy, gy)]);
        cmac(&T2[((size_t)z * wy + y) * gx], &T1[((size_t)z * gy + k) * gx], w, gx);
      }
  const double inv = 1.0 / ((double)gx * gy * gz);
  std::vector<double> out((size_t)wz * wy * wx);
  for (int z = 0; z < wz; ++z)
    for (int y = 0; y < wy; ++y)
      for (int x = 0; x < wx; ++x) {
        // phase index k (x - cx) mod gx, stepped by x - cx along k
        const int step = wrap(1, x - cx, gx);
        int idx = 0;
        cd s = 0;
        const cd* t = &T2[((size_t)z * wy + y) * gx];
        for (int k = 0; k < gx; ++k) {
          s += t[k] * std::conj(tx[idx]);
          idx += step;
          if (idx >= gx) idx -= gx;
        }
        out[((size_t)z * wy + y) * wx + x] = s.real() * inv;
      }
  return out;
}

void normalize(Kern& K) {
  double s = 0;
  for (double v : K.a) s += v;
  if (!(s > 0) || !std::isfinite(s)) throw std::invalid_argument("kernel sum must be positive");
  for (double& v : K.a) v /= s;
}

}  // namespace

bool is_smooth5(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

std::vector<int> factorize(int n) {
  std::vector<int> r;
  while (n % 8 == 0) {
    r.push_back(8);
    n /= 8;
  }
  if (n % 4 == 0) {
    r.push_back(4);
    n /= 4;
  }
  if (n % 2 == 0) {
    r.push_back(2);
    n /= 2;
  }
  while (n % 3 == 0) {
    r.push_back(3);
    n /= 3;
  }
  while (n % 5 == 0) {
    r.push_back(5);
    n /= 5;
  }
  if (n != 1) throw std::invalid_argument("length is not 5-smooth");
  return r;
}

std::vector<cd> twiddles(int n) {
  std::vector<cd> t(n);
  const double a = -2.0 * M_PI / n;
  for (int m = 0; m < n; ++m) t[m] = cd(std::cos(a * m), std::sin(a * m));
  return t;
}

Kern prepare_psf(const float* p, int kx, int ky, int kz) {
  if (kx < 1 || ky < 1 || kz < 1) throw std::invalid_argument("PSF extents must be >= 1");
  Kern K;
  K.kx = kx | 1;
  K.ky = ky | 1;
  K.kz = kz | 1;
  K.a.assign((size_t)K.kx * K.ky * K.kz, 0.0);
  for (int z = 0; z < kz; ++z)
    for (int y = 0; y < ky; ++y)
      for (int x = 0; x < kx; ++x) {
        const float v = p[((size_t)z * ky + y) * kx + x];
        if (!std::isfinite(v) || v < 0) throw std::invalid_argument("PSF values must be finite and >= 0");
        K.at(z, y, x) = v;
      }
  normalize(K);
  return K;
}

Kern mirror(const Kern& k) {
  Kern m = k;
  for (int z = 0; z < k.kz; ++z)
    for (int y = 0; y < k.ky; ++y)
      for (int x = 0; x < k.kx; ++x) m.at(z, y, x) = k.at(k.kz - 1 - z, k.ky - 1 - y, k.kx - 1 - x);
  return m;
}

Kern compound_kernel(const std::vector<Kern>& P, int v, int variant) {
  const int n = (int)P.size();
  Kern K = mirror(P[v]);
  if (variant == 0 || n == 1) return K;
  if (variant == 3) {
    for (double& a : K.a) a = std::pow(a, n);
    normalize(K);
    return K;
  }
  if (variant != 1 && variant != 2) throw std::invalid_argument("unknown variant");
  // grid on which the partner factor's circular convolution equals the
  // linear one inside the window of P_v
  int mx = 0, my = 0, mz = 0;
  for (int w = 0; w < n; ++w) {
    mx = std::max(mx, P[w].kx);
    my = std::max(my, P[w].ky);
    mz = std::max(mz, P[w].kz);
  }
  const int f = variant == 1 ? 2 : 1;
  const int gx = P[v].kx + f * mx, gy = P[v].ky + f * my, gz = P[v].kz + f * mz;
  const std::vector<cd> Fv = dft_grid(P[v], gx, gy, gz);
  std::vector<std::vector<double>> fac(n);
  parallel_for(n, [&](int w) {
    if (w == v) return;
    std::vector<cd> S = dft_grid(P[w], gx, gy, gz);
    for (size_t i = 0; i < S.size(); ++i) {
      cd s = std::conj(Fv[i]) * S[i];        // P_v* (x) P_w
      if (variant == 1) s *= std::conj(S[i]);  // (x) P_w*
      S[i] = s;
    }
    fac[w] = idft_window(S, gx, gy, gz, K.kx, K.ky, K.kz);
  });
  for (int w = 0; w < n; ++w) {
    if (w == v) continue;
    for (size_t i = 0; i < K.a.size(); ++i) K.a[i] *= fac[w][i];
  }
  normalize(K);
  return K;
}

std::vector<Kern> compound_kernels(const std::vector<Kern>& P, int variant) {
  std::vector<Kern> K(P.size());
  parallel_for((int)P.size(), [&](int v) { K[v] = compound_kernel(P, v, variant); });
  return K;
}

std::vector<std::vector<double>> compound_kernels_vjp(const std::vector<Kern>& P, int variant,
                                                      const std::vector<std::vector<double>>& Kbar) {
  const int n = (int)P.size();
  std::vector<std::vector<double>> g(n);
  for (int w = 0; w < n; ++w) g[w].assign(P[w].a.size(), 0.0);
  if ((int)Kbar.size() != n) throw std::invalid_argument("one Kbar per view");
  for (int v = 0; v < n; ++v)
    if (!Kbar[v].empty() && Kbar[v].size() != P[v].a.size())
      throw std::invalid_argument("Kbar does not have the kernel's window");
  // dst += mirror(src) on the window of P[v]
  auto add_mirror = [&](std::vector<double>& dst, const Kern& shape, const std::vector<double>& src) {
    Kern t = shape;
    t.a = src;
    const Kern m = mirror(t);
    for (size_t i = 0; i < dst.size(); ++i) dst[i] += m.a[i];
  };
  if (variant == 0 || n == 1) {
    for (int v = 0; v < n; ++v)
      if (!Kbar[v].empty()) add_mirror(g[v], P[v], Kbar[v]);
    return g;
  }
  if (variant == 3) {
    // K = U / sum U with U = Mv^n
    for (int v = 0; v < n; ++v) {
      if (Kbar[v].empty()) continue;
      const Kern Mv = mirror(P[v]);
      const size_t nk = Mv.a.size();
      std::vector<double> U(nk);
      double S = 0;
      for (size_t i = 0; i < nk; ++i) S += (U[i] = std::pow(Mv.a[i], n));
      double kk = 0;
      for (size_t i = 0; i < nk; ++i) kk += Kbar[v][i] * U[i] / S;
      std::vector<double> Mbar(nk);
      for (size_t i = 0; i < nk; ++i) Mbar[i] = (Kbar[v][i] - kk) / S * n * std::pow(Mv.a[i], n - 1);
      add_mirror(g[v], P[v], Mbar);
    }
    return g;
  }
  if (variant != 1 && variant != 2) throw std::invalid_argument("unknown variant");
  const bool eff = variant == 1;
  int mx = 0, my = 0, mz = 0;
  for (int w = 0; w < n; ++w) {
    mx = std::max(mx, P[w].kx);
    my = std::max(my, P[w].ky);
    mz = std::max(mz, P[w].kz);
  }
  // Per view v, one grid on which circular equals linear convolution for
  // every term below: the autocorrelation P_w (x) P_w* fits (2 k_max - 1),
  // and the window of K_v correlated with a partner term of radius up to
  // r_v + r_w (or 2 r_w) never wraps (k_v + k_max).
  struct Grid {
    int x, y, z;
  };
  std::vector<Grid> grid(n);
  for (int v = 0; v < n; ++v)
    grid[v] = {std::max(P[v].kx + mx, 2 * mx - 1), std::max(P[v].ky + my, 2 * my - 1),
               std::max(P[v].kz + mz, 2 * mz - 1)};
  // spectra of every PSF on every view's grid, and the partner factors
  std::vector<std::vector<std::vector<cd>>> Sp(n, std::vector<std::vector<cd>>(n));
  parallel_for(n * n, [&](int i) {
    const int v = i / n, w = i % n;
    if (!Kbar[v].empty()) Sp[v][w] = dft_grid(P[w], grid[v].x, grid[v].y, grid[v].z);
  });
  std::vector<std::vector<std::vector<double>>> fac(n, std::vector<std::vector<double>>(n));
  parallel_for(n * n, [&](int i) {
    const int v = i / n, w = i % n;
    if (w == v || Kbar[v].empty()) return;
    const auto& Fv = Sp[v][v];
    const auto& Sw = Sp[v][w];
    std::vector<cd> X(Fv.size());
    for (size_t k = 0; k < X.size(); ++k) {
      cd t = std::conj(Fv[k]) * Sw[k];  // P_v* (x) P_w
      if (eff) t *= std::conj(Sw[k]);   // (x) P_w*
      X[k] = t;
    }
    fac[v][w] = idft_window(X, grid[v].x, grid[v].y, grid[v].z, P[v].kx, P[v].ky, P[v].kz);
  });
  // K_v = U / sum U, U = Mv . prod_w fac_w: dL/dU, and the direct factor's term
  std::vector<std::vector<double>> Ubar(n), Mbar(n);
  std::vector<Kern> Mv(n);
  for (int v = 0; v < n; ++v) {
    if (Kbar[v].empty()) continue;
    Mv[v] = mirror(P[v]);
    const size_t nk = Mv[v].a.size();
    std::vector<double> U = Mv[v].a;
    for (int w = 0; w < n; ++w)
      if (w != v)
        for (size_t i = 0; i < nk; ++i) U[i] *= fac[v][w][i];
    double S = 0;
    for (double x : U) S += x;
    double kk = 0;
    for (size_t i = 0; i < nk; ++i) kk += Kbar[v][i] * U[i] / S;
    Ubar[v].resize(nk);
    for (size_t i = 0; i < nk; ++i) Ubar[v][i] = (Kbar[v][i] - kk) / S;
    Mbar[v].resize(nk);
    for (size_t i = 0; i < nk; ++i) {
      double p = Ubar[v][i];
      for (int w = 0; w < n; ++w)
        if (w != v) p *= fac[v][w][i];
      Mbar[v][i] = p;
    }
  }
  // each partner factor fac_w = crop(Mv (x) P_w (x) Mw) (EFF) or crop(Mv (x)
  // P_w) (OPT1): with T = dL/dfac_w, the correlations of T with the other
  // operands (on the grid of v)
  std::vector<std::vector<double>> mv_part(n * n), pw_part(n * n), mw_part(n * n);
  parallel_for(n * n, [&](int i) {
    const int v = i / n, w = i % n;
    if (w == v || Kbar[v].empty()) return;
    const size_t nk = Mv[v].a.size();
    const Grid& G = grid[v];
    Kern T = Mv[v];
    for (size_t k = 0; k < nk; ++k) {
      double p = Ubar[v][k] * Mv[v].a[k];
      for (int u = 0; u < n; ++u)
        if (u != v && u != w) p *= fac[v][u][k];
      T.a[k] = p;
    }
    const std::vector<cd> Th = dft_grid(T, G.x, G.y, G.z);
    const auto& Fv = Sp[v][v];
    const auto& Sw = Sp[v][w];
    std::vector<cd> X(Th.size());
    // Mv: correlation with P_w (x) Mw (EFF, a real spectrum |S_w|^2) or P_w
    for (size_t k = 0; k < X.size(); ++k) X[k] = eff ? Th[k] * std::norm(Sw[k]) : Th[k] * std::conj(Sw[k]);
    mv_part[i] = idft_window(X, G.x, G.y, G.z, P[v].kx, P[v].ky, P[v].kz);
    // P_w: correlation with Mv (x) Mw (EFF) or Mv
    for (size_t k = 0; k < X.size(); ++k) X[k] = eff ? Th[k] * Fv[k] * Sw[k] : Th[k] * Fv[k];
    pw_part[i] = idft_window(X, G.x, G.y, G.z, P[w].kx, P[w].ky, P[w].kz);
    if (eff) {
      // Mw: correlation with Mv (x) P_w
      for (size_t k = 0; k < X.size(); ++k) X[k] = Th[k] * Fv[k] * std::conj(Sw[k]);
      mw_part[i] = idft_window(X, G.x, G.y, G.z, P[w].kx, P[w].ky, P[w].kz);
    }
  });
  for (int v = 0; v < n; ++v) {
    if (Kbar[v].empty()) continue;
    for (int w = 0; w < n; ++w) {
      if (w == v) continue;
      const int i = v * n + w;
      for (size_t k = 0; k < Mbar[v].size(); ++k) Mbar[v][k] += mv_part[i][k];
      for (size_t k = 0; k < g[w].size(); ++k) g[w][k] += pw_part[i][k];
      if (eff) add_mirror(g[w], P[w], mw_part[i]);
    }
    add_mirror(g[v], P[v], Mbar[v]);
  }
  return g;
}

std::vector<std::vector<double>> compound_kernel_vjp(const std::vector<Kern>& P, int v, int variant,
                                                     const std::vector<double>& Kbar) {
  std::vector<std::vector<double>> all(P.size());
  all[v] = Kbar;
  if (Kbar.size() != P[v].a.size()) throw std::invalid_argument("Kbar does not have the kernel's window");
  return compound_kernels_vjp(P, variant, all);
}

namespace {

// x and y stages of the spectrum of a centred kernel on an (nx, ny) grid,
// plane by plane in parallel; store(dz, ky, kx, value) receives every
// kx <= nx / 2.
template <class Store>
void spectrum_xy_planes(const Kern& K, int nx, int ny, Store&& store) {
  const int M = nx / 2;
  const auto tx = twiddles(nx), ty = twiddles(ny);
  const int cx = (K.kx - 1) / 2, cy = (K.ky - 1) / 2;
  const int W = M + 1;
  parallel_for(K.kz, [&](int z) {
    // x stage of every kernel row, real and imaginary parts apart so the
    // y stage's inner loop vectorises
    std::vector<double> re((size_t)K.ky * W), im((size_t)K.ky * W), sr(W), si(W);
    for (int y = 0; y < K.ky; ++y)
      for (int k = 0; k <= M; ++k) {
        // phase index k (x - cx) mod nx, stepped by k along x
        int idx = wrap(k, -cx, nx);
        cd s = 0;
        for (int x = 0; x < K.kx; ++x) {
          s += K.at(z, y, x) * tx[idx];
          idx += k;
          if (idx >= nx) idx -= nx;
        }
        re[(size_t)y * W + k] = s.real();
        im[(size_t)y * W + k] = s.imag();
      }
    for (int k = 0; k < ny; ++k) {
      std::fill(sr.begin(), sr.end(), 0.0);
      std::fill(si.begin(), si.end(), 0.0);
      for (int y = 0; y < K.ky; ++y) {
        const double wr = ty[wrap(k, y - cy, ny)].real(), wi = ty[wrap(k, y - cy, ny)].imag();
        const double* ar = &re[(size_t)y * W];
        const double* ai = &im[(size_t)y * W];
        for (int x = 0; x < W; ++x) {
          sr[x] += ar[x] * wr - ai[x] * wi;
          si[x] += ar[x] * wi + ai[x] * wr;
        }
      }
      for (int x = 0; x < W; ++x) store(z, k, x, sr[x], si[x]);
    }
  });
}

}  // namespace

std::vector<cd> spectrum_xy(const Kern& K, int nx, int ny) {
  const int W = nx / 2 + 1;
  std::vector<cd> A2((size_t)K.kz * ny * W);
  spectrum_xy_planes(K, nx, ny, [&](int z, int ky, int kx, double r, double i) {
    A2[((size_t)z * ny + ky) * W + kx] = cd(r, i);
  });
  return A2;
}

void spectrum_xy_f32(const Kern& K, int nx, int ny, double scale, int d0, int Mp, int64_t h_main, float* out) {
  const int M = nx / 2;
  spectrum_xy_planes(K, nx, ny, [&](int z, int ky, int kx, double r, double i) {
    const size_t d = (size_t)(z + d0);
    const size_t o = kx < M ? (d * ny + ky) * Mp + kx : (size_t)h_main + d * ny + ky;
    out[2 * o] = (float)(r * scale);
    out[2 * o + 1] = (float)(i * scale);
  });
}

void spectrum_host(const Kern& K, int nx, int ny, int nz, float* main_out, float* nyq_out) {
  const int M = nx / 2;
  const auto A2 = spectrum_xy(K, nx, ny);
  const auto tz = twiddles(nz);
  const int cz = (K.kz - 1) / 2;
  const double invV = 1.0 / ((double)nx * ny * nz);
  parallel_for(nz, [&](int kz) {
    for (int ky = 0; ky < ny; ++ky)
      for (int kx = 0; kx <= M; ++kx) {
        cd s = 0;
        for (int z = 0; z < K.kz; ++z) s += A2[((size_t)z * ny + ky) * (M + 1) + kx] * tz[wrap(kz, z - cz, nz)];
        s *= invV;
        float* o = kx < M ? main_out + 2 * (((size_t)kz * ny + ky) * M + kx) : nyq_out + 2 * ((size_t)kz * ny + ky);
        o[0] = (float)s.real();
        o[1] = (float)s.imag();
      }
  });
}

}  // namespace mvdh
