// Adjoints of the table interpolations (bilinear and second-order lookup,
// reduced-matrix fill; Sec. III-B.3, last paragraph), deterministic.
//
// Every interpolated value is a weighted sum over a small stencil of table
// nodes (2 x 2 bilinear, 3 x 3 second order) anchored at one base cell.  Its
// adjoint scatters the cotangent, times the same weights, back onto that
// stencil.  Floating-point addition is not associative, so the order in which
// many points add into one node must be fixed for the result to repeat bit
// for bit.  Here:
//   1. every point gets the key (colour, base cell) and the points are sorted
//      by key (stable radix sort: points of one cell keep their order);
//   2. each run of equal keys (the points of one base cell) sums its
//      contributions to its stencil in that order, in registers;
//   3. the runs add their sums into the table colour by colour: two base
//      cells of one colour (equal cell indices modulo the stencil width on
//      both axes) have disjoint stencils, so within one colour no two threads
//      touch the same node, and the colours follow one another on the stream.
// No atomics are used; every node's sum has the same order on every run.
#include <hipcub/hipcub.hpp>

#include "cfft_device.h"
#include "cfft_internal.h"

namespace cfft {

constexpr unsigned kNoCell = 0xffffffffu;

struct ScatterArgs {
  int order;            // 1 bilinear, 2 second order
  int fill;             // 0: points of a lookup, 1: element pairs of a fill
  int nx, ny;
  double x0, ddx, y0, ddy;
  const double* pts;    // lookup: [npts][2]
  int npts;
  const double* pos;    // fill: element positions [nelem][2]
  int nelem, nmbf;
  const double2* dout;  // cotangents (layout of the forward output)
  double2* dz;          // [npairs][ny][nx], accumulated into
  int npairs;
  int pm[kScatterMaxPairs], pn[kScatterMaxPairs];   // fill: (m, n) of table k
};

__host__ __device__ __forceinline__ int stencil_width(int order) { return order == 1 ? 2 : 3; }

// Fractional table index of point q (lookup point or element pair i, j);
// false for a fill's self pair.
__device__ __forceinline__ bool point_uv(const ScatterArgs& a, int q, double& ux, double& uy) {
  double dx, dy;
  if (a.fill) {
    const int i = q / a.nelem, j = q - (q / a.nelem) * a.nelem;
    if (i == j) return false;
    dx = a.pos[2 * i] - a.pos[2 * j];
    dy = a.pos[2 * i + 1] - a.pos[2 * j + 1];
  } else {
    dx = a.pts[2 * q];
    dy = a.pts[2 * q + 1];
  }
  ux = (dx - a.x0) / a.ddx;
  uy = (dy - a.y0) / a.ddy;
  return true;
}

// Base cell (j1, j2) of the stencil and the per-axis weights of point q.
__device__ __forceinline__ bool point_stencil(const ScatterArgs& a, int q, int& j1, int& j2, double (&wx)[3],
                                              double (&wy)[3]) {
  double ux, uy, tx, ty;
  if (!point_uv(a, q, ux, uy)) return false;
  if (a.order == 1) {
    if (!cell_at(ux, uy, a.nx, a.ny, j1, j2, tx, ty)) return false;
    wx[0] = 1.0 - tx;
    wx[1] = tx;
    wy[0] = 1.0 - ty;
    wy[1] = ty;
    wx[2] = wy[2] = 0.0;
    return true;
  }
  int c1, c2;
  if (!stencil_at(ux, uy, a.nx, a.ny, c1, c2, tx, ty)) return false;
  lagrange3(tx, wx);
  lagrange3(ty, wy);
  j1 = c1 - 1;   // the 3 x 3 stencil starts one node before its centre
  j2 = c2 - 1;
  return true;
}

__global__ void __launch_bounds__(256) scatter_keys_kernel(ScatterArgs a, int npoints, unsigned* keys, unsigned* idx) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npoints) return;
  int j1, j2;
  double wx[3], wy[3];
  unsigned key = kNoCell;
  if (point_stencil(a, q, j1, j2, wx, wy)) {
    const int w = stencil_width(a.order);
    const unsigned colour = (unsigned)((j1 % w) + w * (j2 % w));
    key = colour * (unsigned)(a.nx * a.ny) + (unsigned)(j2 * a.nx + j1);
  }
  keys[q] = key;
  idx[q] = (unsigned)q;
}

// One thread per (run of one base cell, table k), for the runs of one colour:
// the run's contributions summed in sorted order, then added to the stencil.
__global__ void __launch_bounds__(256) scatter_colour_kernel(ScatterArgs a, unsigned colour, const unsigned* runs,
                                                             const int* counts, const int* offsets,
                                                             const int* nruns, const unsigned* order) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= *nruns) return;
  const unsigned key = runs[r];
  const unsigned ncell = (unsigned)(a.nx * a.ny);
  if (key == kNoCell || key / ncell != colour) return;
  const int w = stencil_width(a.order);
  double2 acc[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[b][c] = make_double2(0.0, 0.0);
  const int am = a.nelem * a.nmbf;
  for (int t = offsets[r], e = offsets[r] + counts[r]; t < e; ++t) {
    const int q = (int)order[t];
    int j1, j2;
    double wx[3], wy[3];
    point_stencil(a, q, j1, j2, wx, wy);
    double2 g;
    if (a.fill) {
      const int i = q / a.nelem, j = q - (q / a.nelem) * a.nelem;
      g = a.dout[(size_t)(i * a.nmbf + a.pm[k]) * am + j * a.nmbf + a.pn[k]];
    } else {
      g = a.dout[(size_t)k * a.npts + q];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double wt = wy[b] * wx[c];
        acc[b][c] = make_double2(acc[b][c].x + wt * g.x, acc[b][c].y + wt * g.y);
      }
  }
  const unsigned cell = key % ncell;
  const int j1 = (int)(cell % (unsigned)a.nx), j2 = (int)(cell / (unsigned)a.nx);
  double2* dz = a.dz + (size_t)k * ncell;
  for (int b = 0; b < w; ++b)
    for (int c = 0; c < w; ++c) {
      double2& d = dz[(size_t)(j2 + b) * a.nx + j1 + c];
      d = make_double2(d.x + acc[b][c].x, d.y + acc[b][c].y);
    }
}

namespace {
size_t al256(size_t v) { return (v + 255) / 256 * 256; }

struct ScatterLayout {
  size_t keys, idx, skeys, sidx, runs, counts, offsets, nruns, temp, total;
  size_t t_sort, t_rle, t_scan;
};

hipError_t scatter_layout(int n, ScatterLayout& L) {
  L.t_sort = L.t_rle = L.t_scan = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, L.t_sort, (const unsigned*)nullptr, (unsigned*)nullptr,
                                                    (const unsigned*)nullptr, (unsigned*)nullptr, n);
  if (e == hipSuccess)
    e = hipcub::DeviceRunLengthEncode::Encode(nullptr, L.t_rle, (const unsigned*)nullptr, (unsigned*)nullptr,
                                              (int*)nullptr, (int*)nullptr, n);
  if (e == hipSuccess)
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, L.t_scan, (const int*)nullptr, (int*)nullptr, n);
  if (e != hipSuccess) return e;
  const size_t u = al256(sizeof(unsigned) * (size_t)n);
  L.keys = 0;
  L.idx = L.keys + u;
  L.skeys = L.idx + u;
  L.sidx = L.skeys + u;
  L.runs = L.sidx + u;
  L.counts = L.runs + u;
  L.offsets = L.counts + u;
  L.nruns = L.offsets + u;
  L.temp = L.nruns + 256;
  L.total = L.temp + al256(std::max(L.t_sort, std::max(L.t_rle, L.t_scan)));
  return hipSuccess;
}

ScatterArgs scatter_args(const PassParams& p, int order, const double2* dout, double2* dz) {
  ScatterArgs a{};
  a.order = order;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.x0 = p.x.d_first;
  a.ddx = p.x.dd;
  a.y0 = p.y.d_first;
  a.ddy = p.y.dd;
  a.dout = dout;
  a.dz = dz;
  return a;
}

hipError_t run_scatter(const ScatterArgs& a, int npoints, void* ws, hipStream_t s) {
  ScatterLayout L;
  hipError_t e = scatter_layout(npoints, L);
  if (e != hipSuccess) return e;
  char* b = (char*)ws;
  unsigned *keys = (unsigned*)(b + L.keys), *idx = (unsigned*)(b + L.idx);
  unsigned *skeys = (unsigned*)(b + L.skeys), *sidx = (unsigned*)(b + L.sidx), *runs = (unsigned*)(b + L.runs);
  int *counts = (int*)(b + L.counts), *offsets = (int*)(b + L.offsets), *nruns = (int*)(b + L.nruns);
  void* temp = b + L.temp;
  const unsigned blocks = (unsigned)((npoints + 255) / 256);
  hipLaunchKernelGGL(scatter_keys_kernel, dim3(blocks), dim3(256), 0, s, a, npoints, keys, idx);
  e = hipGetLastError();
  size_t tb = L.t_sort;
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortPairs(temp, tb, keys, skeys, idx, sidx, npoints, 0, 32, s);
  tb = L.t_rle;
  if (e == hipSuccess) e = hipcub::DeviceRunLengthEncode::Encode(temp, tb, skeys, runs, counts, nruns, npoints, s);
  tb = L.t_scan;
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, offsets, npoints, s);
  const int w = stencil_width(a.order);
  for (int c = 0; c < w * w && e == hipSuccess; ++c) {
    hipLaunchKernelGGL(scatter_colour_kernel, dim3(blocks, (unsigned)a.npairs), dim3(256), 0, s, a, (unsigned)c, runs,
                       counts, offsets, nruns, sidx);
    e = hipGetLastError();
  }
  return e;
}
}  // namespace

size_t scatter_workspace_bytes(long long npoints) {
  ScatterLayout L;
  if (npoints < 1 || npoints > (1LL << 30) || scatter_layout((int)npoints, L) != hipSuccess) return 0;
  return L.total;
}

hipError_t launch_lookup_backward(const PassParams& p, const double2* dout, int npairs, const double* pts, int npts,
                                  double2* dz, bool quadratic, void* ws, hipStream_t s) {
  ScatterArgs a = scatter_args(p, quadratic ? 2 : 1, dout, dz);
  a.fill = 0;
  a.pts = pts;
  a.npts = npts;
  a.npairs = npairs;
  return run_scatter(a, npts, ws, s);
}

hipError_t launch_fill_backward(const PassParams& p, const int* pm, const int* pn, int npairs, int nmbf,
                                const double* pos, int nelem, int order, const double2* dout, double2* dz, void* ws,
                                hipStream_t s) {
  if (npairs > kScatterMaxPairs) return hipErrorInvalidValue;
  ScatterArgs a = scatter_args(p, order, dout, dz);
  a.fill = 1;
  a.pos = pos;
  a.nelem = nelem;
  a.nmbf = nmbf;
  a.npairs = npairs;
  for (int k = 0; k < npairs; ++k) {
    a.pm[k] = pm[k];
    a.pn[k] = pn[k];
  }
  return run_scatter(a, nelem * nelem, ws, s);
}

}  // namespace cfft
