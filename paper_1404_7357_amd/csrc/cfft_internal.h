// Host-side interfaces between the C-ABI layer (cfft_api.cpp) and the kernel
// launchers (*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfft {

constexpr int kMaxPairsPerLaunch = 64;
constexpr int kMaxOrder = 7;
constexpr int kSpecPChunk = 4;   // spectra kernel: centres per unrolled chunk
constexpr int kMaxGroups = 32;   // basis shape groups (kind, a, b) a geometry may hold

// Sampling of one axis: k(n) = k0 + n dk, D(j) = d0 + j dd.
struct Axis {
  int n;
  double k_first, dk;   // spectral samples
  double d_first, dd;   // output displacements
};

// Contour of a grid: ray (beta_I = gamma beta) or parabolic (beta_I =
// gamma beta (1 - beta/beta_end) below beta_end, real beyond).
struct Contour {
  double gamma;
  int parabolic;
  double beta_end;
};

struct GreenParams {
  Axis x, y;
  double gamma, k0;
  double eps_re, tan_delta, h;
  int parabolic;
  double beta_end;
};

// Separable geometry of a basis set: bases sharing (kind, a, b) form a
// group; inside a group every basis sits on the product of the group's
// distinct x- and y-centres, so its spectrum factorises in kx and ky.
struct GeomGroup {
  int kind;
  int np, nr;         // distinct x-centres (p), distinct y-centres (r)
  int xoff, yoff;     // offsets into the x / y centre arrays
  int ioff;           // offset into the [np][nr] basis index array (-1 = empty slot)
  int uoff;           // row offset of this group's x tables (U rows)
  int poff;           // offset of this group's centres in the per-row w tables,
                      // each group padded to a multiple of kSpecPChunk
  int uniform;        // 1: x-centres and y-centres are each equally spaced
  double a, b;
  double dxc, dyc;    // centre spacings when uniform (0 for a single centre)
};

struct GeomDevice {
  int ngroups;
  int nbasis;
  int total_p;        // sum of np
  int total_r;        // sum of nr
  int total_idx;      // sum of np*nr
  int ppad;           // sum of np rounded up per group to kSpecPChunk
  int ngroups_x;      // groups [0, ngroups_x) carry x-directed current, the rest y
  GeomGroup* groups;  // device copies
  double* xs;         // [total_p]
  double* ys;         // [total_r]
  int* index;         // [total_idx]
};

// Column tiles of the column pass: the default shape, tiles of half its
// width, or (columns of 1024 points and more) the other number of points per
// thread, 8 or 16, with its own widest tile.  The two alternatives are the
// autotuner's candidates beside the default.
enum { kColTileDefault = 0, kColTileHalf = 1, kColTileAltR = 2 };

struct PassParams {
  Axis x, y;
  double gamma;
  int order;
  int precision;      // 0 FP64, 1 MIXED (storage precision)
  int hi_compute;     // MIXED only: transforms in FP64 on the FP32-stored data
  int tensor;         // 1: tensor-product truncation (one intermediate per pair)
  int parabolic;      // 1: parabolic contour (per-sample ratio; N_t row transforms)
  double beta_end;
  int band;           // 1: x2 zero-padded grid, integrand only on n in [N/4, 3N/4) per axis
  int col_tile;       // kColTile*: column tile of the column pass
  int stream_out;     // 1: the row pass writes the intermediates with non-temporal
                      // stores (a launch's intermediates too large to stay in the
                      // memory-side cache until the column pass reads them)
};

// Intermediate arrays per pair between the row and column passes.
inline int inter_slots(const PassParams& p) { return p.tensor ? 1 : p.order + 1; }

// Launchers; all return hipSuccess or the launch error.
hipError_t launch_green(const GreenParams& p, double2* g, hipStream_t s);
__host__ __device__ int green_threads(const GreenParams& p);   // quadrant samples evaluated

hipError_t launch_spectra_tables(const Axis& x, const Axis& y, double gamma, const GeomDevice& geo,
                                 double2* utab, hipStream_t s);
size_t spectra_tables_len(const Axis& x, const Axis& y, const GeomDevice& geo);
hipError_t launch_spectra(const Axis& x, const Axis& y, double gamma, const GeomDevice& geo,
                          const double2* utab, const double2* q, int nmbf, double2* scratch,
                          void* spec, int precision, hipStream_t s);
// Spectra on the parabolic contour (no per-axis separation): per sample.
hipError_t launch_spectra_direct(const Axis& x, const Axis& y, const Contour& c, const GeomDevice& geo,
                                 const double2* q, int nmbf, double2* scratch, void* spec, int precision,
                                 hipStream_t s);
size_t spectra_direct_scratch_len(const GeomDevice& geo, int nmbf);
size_t spectra_scratch_len(const Axis& y, const GeomDevice& geo, int nmbf);
size_t spectra_lds_bytes(const GeomDevice& geo, int nmbf);
size_t adj_spectra_lds_bytes(const GeomDevice& geo, int nmbf);
constexpr size_t kMaxDynamicLds = 65536;   // dynamic LDS a launch may ask for

// Row + column passes for one chunk of <= kMaxPairsPerLaunch pairs.
hipError_t launch_row_pass(const PassParams& p, const double2* g, const void* spec,
                           const int* pm, const int* pn, int npairs, void* inter,
                           const void* twx, hipStream_t s);
hipError_t launch_col_pass(const PassParams& p, const void* inter, int npairs, void* z,
                           const void* twy, hipStream_t s);

hipError_t launch_lookup(const PassParams& p, const void* z, int npairs, const double* pts,
                         int npts, double2* out, hipStream_t s);
hipError_t launch_lookup_quadratic(const PassParams& p, const void* z, int npairs, const double* pts,
                                  int npts, double2* out, hipStream_t s);
// Reduced-matrix fill; slot[m * kFillMaxMbf + n] = pair index of (m, n) or -1.
constexpr int kFillMaxMbf = 16;
hipError_t launch_fill(const PassParams& p, const void* z, const short* slot, int nmbf, const double* pos,
                       int nelem, int order, double2* out, hipStream_t s);

// Deterministic adjoints of the interpolations (cfft_scatter.hip): the
// cotangents scattered onto the FP64 table gradient dz (accumulated into);
// ws holds scatter_workspace_bytes(points) bytes (0: too many points).
constexpr int kScatterMaxPairs = kFillMaxMbf * kFillMaxMbf;
size_t scatter_workspace_bytes(long long npoints);
hipError_t launch_lookup_backward(const PassParams& p, const double2* dout, int npairs, const double* pts,
                                  int npts, double2* dz, bool quadratic, void* ws, hipStream_t s);
hipError_t launch_fill_backward(const PassParams& p, const int* pm, const int* pn, int npairs, int nmbf,
                                const double* pos, int nelem, int order, const double2* dout, double2* dz,
                                void* ws, hipStream_t s);

// Adjoint.
hipError_t launch_adj_col_pass(const PassParams& p, const double2* dz, int npairs, double2* inter,
                               const void* twy, hipStream_t s);
hipError_t launch_adj_row_pass(const PassParams& p, const double2* inter, int npairs, double2* gi,
                               const void* twx, hipStream_t s);
hipError_t launch_adj_integrand(const PassParams& p, const double2* gi, const double2* g,
                                const double2* spec, const int* pm, const int* pn, int npairs,
                                int nmbf, double2* gg, double2* gspec, int accumulate, hipStream_t s);
hipError_t launch_adj_green(const GreenParams& p, const double2* gg, double* partial, int nblocks,
                            hipStream_t s);
hipError_t launch_reduce_sum(const double* partial, int n, int count, double* out, hipStream_t s);
hipError_t launch_adj_spectra(const Axis& x, const Axis& y, const GeomDevice& geo,
                              const double2* utab, const double2* gspec, int nmbf, double2* rowacc,
                              double2* gq, hipStream_t s);

// Size of the adjoint scratch (host helper).
size_t adj_spectra_scratch(const Axis& y, const GeomDevice& geo, int nmbf);

}  // namespace cfft
