// Descriptors shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>

#define MVD_MAX_STAGES 12

// Mixed-radix Stockham plan of one 1-D complex FFT length (radices 2, 3, 4,
// 5, 8).  Per stage s: the radix, Ns (product of the earlier radices), the
// twiddle stride L / (Ns R), and multipliers m with floor(j / d) =
// umulhi(j, m) for the divisions by Ns and by L / R (exact for j, d < 2^16;
// unused when the divisor is 1).  tw is the offset of the length-L table
// exp(-2 pi i m / L) in the twiddle pool.
struct FftPlan {
  int L;
  int nst;
  int tw;
  int pad;
  int radix[MVD_MAX_STAGES];
  int ns[MVD_MAX_STAGES];
  int tws[MVD_MAX_STAGES];
  unsigned ns_magic[MVD_MAX_STAGES];
  unsigned nb_magic[MVD_MAX_STAGES];
};

// Spectrum roles: which kernel spectrum a convolution pass multiplies by.
enum { ROLE_P = 0, ROLE_EFF = 1, ROLE_OPT1 = 2, ROLE_OPT2 = 3, N_ROLES = 4 };

// One volume (a block of the batched form) as the kernels see it.
// Volumes are [z][y][x] float32; the half spectrum is kept as a main part
// [z][y][kx < M] (M = nx/2 complex per row) followed by the kx = M
// (Nyquist) plane [z][y], complex float32 interleaved.
//
// Kernels are stored as their x and y transform stages only, at the kz
// planes of a common centred window (kz odd, centre cz = (kz - 1) / 2): the
// same layout as a half spectrum with nz replaced by kz (main part
// [d][ky][kx < M], then [d][ky] for kx = M), scaled by 1/V.  The z pass
// places tap d at circular offset d - cz of each length-nz line and
// transforms it next to the data.
struct JobDesc {
  int nx, ny, nz, M;
  int nviews;
  int plan_x, plan_y, plan_z;  // plans of lengths M, ny, nz
  int pp;                      // offset of exp(-2 pi i k / nx), k < M, in the twiddle pool
  int Mp;                      // row pitch of the main half spectrum (complex): M rounded up
                               // to 16, so every row starts on a 128-byte line
  int64_t V;
  int64_t spec_main;           // Mp * ny * nz
  int64_t spec_elems;          // spec_main + ny * nz
  int64_t h_main;              // Mp * ny * kz: start of a kernel's kx = M taps
  int64_t h_elems;             // h_main + ny * kz: complex entries per view of H[role]
  float* psi;
  float* spec;                 // complex interleaved, spec_elems entries
  const float* phi;            // [nviews][V]
  const float* w;              // [nviews][V] or nullptr
  const float* H[N_ROLES];     // [nviews][h_elems] complex kernel planes; nullptr if not built
  float eps, lamp;
  int kz, cz;                  // kernel window along z and its centre
  float* acc;                  // [V] combined-update factor (product or sum over views), or nullptr
  float* saved;                // spec_elems complex: x/y-stage spectrum of psi kept over a combined
                               // iteration, or nullptr
  // Block-wise form: the block's grid is a window of the volume's estimate
  // vol (vnx x vny x vnz, periodic); grid voxel g sits at volume voxel
  // (s + g) mod vn per axis.  The block's own voxels are the grid voxels
  // [h, h + e) per axis (no wrap: they sit at o + g - h).  The forward x
  // pass reads the window and the update writes the own voxels, both in the
  // volume; psi is then nullptr.  vol is nullptr otherwise.
  float* vol;
  int vnx, vny, vnz;
  int sx, sy, sz;
  int ox, oy, oz;
  int hx, hy, hz;
  int ex, ey, ez;
};

// Linear boundary: a view holds this value on the grid voxels outside the
// volume (where it has no data); the ratio pass takes q = 1 there.  Views
// are >= 0 on the volume, so the marker is never a measured value.
#define MVD_NO_DATA (-1.0f)

// Options of the x passes (bit set).  SPEC: write the forward x transform
// of the new psi (update modes).  FIRST: the first view of a combined
// iteration (the factor starts from this view's value).  GEO: combine by
// product and |V|-th root, else by sum and division by |V|.
enum { XOPT_SPEC = 1, XOPT_FIRST = 2, XOPT_GEO = 4 };

// x pass modes 0 (forward of psi) and 2 (update) of the block-wise form take
// this bit: the forward pass reads the block's window of the volume, the
// update reads and writes the own voxels in the volume (JobDesc.vol).
enum { XMODE_WIN = 8 };

// Per-workgroup partial results of the x passes (one entry per x tile).
struct Partial {
  double flux;
  unsigned int ratio_clamps;
  unsigned int neg_clamps;
};

enum PassKind { PASS_X = 0, PASS_Y = 1, PASS_Z = 2 };

#if defined(__HIPCC__)
#define MVD_HD __host__ __device__
#else
#define MVD_HD
#endif

MVD_HD inline int mvd_cdiv(int a, int b) { return (a + b - 1) / b; }

// Number of tiles of a job for a pass.  x: rows of RW; y and z: TX adjacent
// lines of the main part plus TX lines of the Nyquist plane.
MVD_HD inline int mvd_tiles(const JobDesc& j, int kind, int param) {
  if (kind == PASS_X) return mvd_cdiv(j.ny * j.nz, param);
  if (kind == PASS_Y) return mvd_cdiv(j.M, param) * j.nz + mvd_cdiv(j.nz, param);
  return mvd_cdiv(j.M, param) * j.ny + mvd_cdiv(j.ny, param);
}

// Multiplier for floor(j / d) = umulhi(j, m), d >= 2, j, d < 2^16.
MVD_HD inline unsigned mvd_magic(unsigned d) {
  return d < 2 ? 0u : (unsigned)((0x100000000ull + d - 1) / d);
}
