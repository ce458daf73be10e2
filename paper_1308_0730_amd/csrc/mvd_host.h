// FP64 host-side preparation: PSF normalisation, compound kernels, kernel
// spectra, FFT plans and twiddle tables.  No device code.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace mvdh {

using cd = std::complex<double>;

// A centred kernel with odd extents, [z][y][x] doubles.
struct Kern {
  int kx = 0, ky = 0, kz = 0;
  std::vector<double> a;
  double& at(int z, int y, int x) { return a[((size_t)z * ky + y) * kx + x]; }
  double at(int z, int y, int x) const { return a[((size_t)z * ky + y) * kx + x]; }
};

bool is_smooth5(int n);
// True if every x[i] is finite and in [lo, hi] (checked on several threads).
bool all_within(const float* x, int64_t n, float lo, float hi);
// Radices (8, 4, 2, 3, 5) of a 5-smooth length, largest first.
std::vector<int> factorize(int n);

// Normalise to sum one and pad even extents with a trailing zero plane.
// Throws std::invalid_argument on negative / non-finite values or zero sum.
Kern prepare_psf(const float* p, int kx, int ky, int kz);
Kern mirror(const Kern& k);

// Compound back-projection kernel of view v (0 = RL, 1 = EFF, 2 = OPT1,
// 3 = OPT2), in the window of P_v, normalised.  The partner factors
// P_v* (x) P_w (x) P_w* (EFF) and P_v* (x) P_w (OPT1) are evaluated exactly
// by a direct DFT on a grid large enough that circular equals linear
// convolution, then cropped to the window.
Kern compound_kernel(const std::vector<Kern>& P, int v, int variant);
// The compound kernels of every view, computed in parallel.
std::vector<Kern> compound_kernels(const std::vector<Kern>& P, int variant);

// Adjoint of compound_kernel: given Kbar = dL/dK_v on K_v's window (the
// window of P_v), dL/dP_w for every prepared PSF (same extents as P[w].a;
// zero for PSFs K_v does not depend on).  FP64, by the same direct DFTs on
// a grid where circular equals linear convolution.
std::vector<std::vector<double>> compound_kernel_vjp(const std::vector<Kern>& P, int v, int variant,
                                                     const std::vector<double>& Kbar);
// The same for every view's kernel at once (Kbar[v] empty: no gradient for
// K_v): the sum over v of the gradients, computed in parallel.
std::vector<std::vector<double>> compound_kernels_vjp(const std::vector<Kern>& P, int variant,
                                                      const std::vector<std::vector<double>>& Kbar);

// Stages x and y of the spectrum of a centred kernel on a volume grid:
// A2[dz][ky][kx], kx in [0, nx/2], for every kernel plane dz.
std::vector<cd> spectrum_xy(const Kern& K, int nx, int ny);
// The same scaled by `scale` and rounded to FP32, written in the device
// layout of kernel planes: plane dz goes to plane dz + d0, kx < nx / 2 at
// ((dz + d0) ny + ky) Mp + kx and kx = nx / 2 at h_main + (dz + d0) ny + ky
// (complex: real then imaginary float); nothing else of out is written.
void spectrum_xy_f32(const Kern& K, int nx, int ny, double scale, int d0, int Mp, int64_t h_main, float* out);
// exp(-2 pi i m / n), m < n.
std::vector<cd> twiddles(int n);
// Full spectrum on the host (all three stages), scaled by 1/V, split into
// the main part [kz][ky][kx < nx/2] and the Nyquist plane [kz][ky].
void spectrum_host(const Kern& K, int nx, int ny, int nz, float* main_out, float* nyq_out);

}  // namespace mvdh
