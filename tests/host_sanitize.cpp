// Host FP64 preparation code under AddressSanitizer and UBSan: PSF
// preparation (odd and even extents, rejection of bad values), compound
// kernels and their adjoint for every variant, kernel spectra, plans.
// Built and run by tests/test_host_sanitize.py; exits non-zero on a failure.
#include <cmath>
#include <cstdio>
#include <random>
#include <stdexcept>
#include <vector>

#include "mvd_host.h"

using namespace mvdh;

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::fprintf(stderr, "check failed: %s line %d\n", #c, __LINE__); \
      ++fails;                                                \
    }                                                         \
  } while (0)

int main() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<float> u(0.01f, 1.0f);
  const int ext[3][3] = {{5, 3, 7}, {4, 5, 3}, {3, 3, 6}};
  std::vector<Kern> P;
  for (auto& e : ext) {
    std::vector<float> g((size_t)e[0] * e[1] * e[2]);
    for (float& x : g) x = u(rng);
    Kern K = prepare_psf(g.data(), e[0], e[1], e[2]);
    CHECK(K.kx % 2 == 1 && K.ky % 2 == 1 && K.kz % 2 == 1);
    double s = 0;
    for (double a : K.a) s += a;
    CHECK(std::fabs(s - 1.0) < 1e-12);
    P.push_back(K);
  }
  // bad values are rejected
  {
    std::vector<float> g(27, 1.0f);
    g[5] = -1.0f;
    bool thrown = false;
    try {
      prepare_psf(g.data(), 3, 3, 3);
    } catch (const std::invalid_argument&) {
      thrown = true;
    }
    CHECK(thrown);
    std::vector<float> z(8, 0.0f);
    thrown = false;
    try {
      prepare_psf(z.data(), 2, 2, 2);
    } catch (const std::invalid_argument&) {
      thrown = true;
    }
    CHECK(thrown);
  }
  // every view's kernel at once (in parallel) equals the one-view builds;
  // an exception on a worker thread reaches the caller
  for (int variant = 0; variant < 4; ++variant) {
    const auto all = compound_kernels(P, variant);
    CHECK(all.size() == 3);
    for (int v = 0; v < 3; ++v) CHECK(all[v].a == compound_kernel(P, v, variant).a);
  }
  {
    bool thrown = false;
    try {
      compound_kernels(P, 7);
    } catch (const std::invalid_argument&) {
      thrown = true;
    }
    CHECK(thrown);
  }
  for (int variant = 0; variant < 4; ++variant)
    for (int v = 0; v < 3; ++v) {
      Kern K = compound_kernel(P, v, variant);
      CHECK(K.kx == P[v].kx && K.ky == P[v].ky && K.kz == P[v].kz);
      double s = 0;
      for (double a : K.a) s += a;
      CHECK(std::fabs(s - 1.0) < 1e-10);
      std::vector<double> kbar(K.a.size());
      for (size_t i = 0; i < kbar.size(); ++i) kbar[i] = std::sin(0.37 * (double)i);
      const auto g = compound_kernel_vjp(P, v, variant, kbar);
      CHECK(g.size() == 3);
      for (int w = 0; w < 3; ++w) {
        CHECK(g[w].size() == P[w].a.size());
        for (double x : g[w]) CHECK(std::isfinite(x));
      }
      bool thrown = false;
      try {
        compound_kernel_vjp(P, v, variant, std::vector<double>(3, 0.0));
      } catch (const std::invalid_argument&) {
        thrown = true;
      }
      CHECK(thrown);
    }
  // spectra on a small grid and every plan factorisation up to 1024
  {
    const int nx = 20, ny = 12, nz = 10;
    std::vector<float> main_out((size_t)nz * ny * (nx / 2) * 2), nyq((size_t)nz * ny * 2);
    spectrum_host(P[0], nx, ny, nz, main_out.data(), nyq.data());
    for (float x : main_out) CHECK(std::isfinite(x));
    // DC term: the kernel's sum times 1/V
    CHECK(std::fabs(main_out[0] - 1.0f / (nx * ny * nz)) < 1e-7f);
    // the device layout of the kernel planes: one plane of margin on each
    // side of the window, rows padded to 16 complex, the Nyquist column apart
    const int kzw = P[0].kz + 2, M = nx / 2, Mp = 16;
    const int64_t h_main = (int64_t)Mp * ny * kzw;
    std::vector<float> planes((size_t)(h_main + (int64_t)ny * kzw) * 2, -7.0f);
    spectrum_xy_f32(P[0], nx, ny, 0.5, 1, Mp, h_main, planes.data());
    const auto A2 = spectrum_xy(P[0], nx, ny);
    for (int d = 0; d < kzw; ++d)
      for (int ky = 0; ky < ny; ++ky)
        for (int kx = 0; kx < Mp; ++kx) {
          const size_t o = ((size_t)d * ny + ky) * Mp + kx;
          if (d == 0 || d == kzw - 1 || kx >= M) {
            CHECK(planes[2 * o] == -7.0f && planes[2 * o + 1] == -7.0f);
          } else {
            const cd a = A2[((size_t)(d - 1) * ny + ky) * (M + 1) + kx] * 0.5;
            CHECK(std::fabs(planes[2 * o] - (float)a.real()) <= 1e-6f * (1.0f + std::fabs((float)a.real())));
            CHECK(std::fabs(planes[2 * o + 1] - (float)a.imag()) <= 1e-6f * (1.0f + std::fabs((float)a.imag())));
          }
        }
    for (int d = 1; d + 1 < kzw; ++d)
      for (int ky = 0; ky < ny; ++ky) {
        const size_t o = (size_t)h_main + (size_t)d * ny + ky;
        const cd a = A2[((size_t)(d - 1) * ny + ky) * (M + 1) + M] * 0.5;
        CHECK(std::fabs(planes[2 * o] - (float)a.real()) <= 1e-6f * (1.0f + std::fabs((float)a.real())));
      }
    for (int n = 1; n <= 1024; ++n)
      if (is_smooth5(n)) {
        int prod = 1;
        for (int r : factorize(n)) prod *= r;
        CHECK(prod == n);
      }
  }
  if (fails) std::fprintf(stderr, "%d failures\n", fails);
  else std::printf("host sanitize: ok\n");
  return fails ? 1 : 0;
}
