// MBF spectra on the ray contour (eq. FTMBF), FP64, and their adjoint.
//
// Bases that share (kind, a, b) form a group whose members sit on the product
// of the group's distinct x- and y-centres.  Their transforms factorise:
//   F_j(k_c) = SX_g(kx) SY_g(ky) U_gp(kx) V_gr(ky),
//   U_gp = exp(-i kcx X_p),  V_gr = exp(-i kcy Y_r),
// so   M_m(k_c) = sum_g SX_g SY_g sum_p U_gp [ sum_r conj(q_m,j(g,p,r)) V_gr ].
// The inner sum over r is done once per row (LDS), the outer one per sample.
// The reflected spectrum M#_m(k_c) = sum_j q_mj F_j(-k_c) uses U#, V# =
// exp(+i k_c .) and the even shape factors.
#include "cfft_device.h"
#include "cfft_internal.h"

namespace cfft {

__device__ __forceinline__ double2 at_byte(const double2* row, unsigned byte_off) {
  return *(const double2*)((const char*)row + byte_off);
}

__device__ __forceinline__ bool is_ydir(int kind) { return kind == 1 || kind == 3; }
__device__ __forceinline__ bool is_cos(int kind) { return kind == 2 || kind == 3; }

// Shape factor along the current: triangle a sinc^2(k a/2) or half-cosine
// (a/2)[sinc((k a - pi)/2) + sinc((k a + pi)/2)]; across: b sinc(k b/2).
__device__ __forceinline__ double2 along_factor(int kind, double a, double2 k) {
  if (is_cos(kind)) {
    const double2 ka = cscale(k, a);
    const double2 s1 = csinc(cscale(make_double2(ka.x - M_PI, ka.y), 0.5));
    const double2 s2 = csinc(cscale(make_double2(ka.x + M_PI, ka.y), 0.5));
    return cscale(cadd(s1, s2), 0.5 * a);
  }
  const double2 s = csinc(cscale(k, 0.5 * a));
  return cscale(cmul(s, s), a);
}
__device__ __forceinline__ double2 across_factor(double b, double2 k) {
  return cscale(csinc(cscale(k, 0.5 * b)), b);
}

// exp(-i (1 + i gamma) k X) and exp(+i (1 + i gamma) k X).
__device__ __forceinline__ void phase_pair(double k, double gamma, double X, double2& u, double2& uh) {
  double s, c;
  sincos(k * X, &s, &c);
  const double e = exp(gamma * k * X);
  const double ei = 1.0 / e;
  u = make_double2(e * c, -e * s);
  uh = make_double2(ei * c, ei * s);
}

// Geometry tables of one grid (built once per grid and basis set):
//   x part, rows of length nx: [2 (uoff+p)] = SX_g U, [2 (uoff+p) + 1] = SX_g U#
//                              (the x shape factors are even in k),
//                              [2 total_p + g] = SX_g
//   y part (at vtab_offset), rows of length ny: [2 (yoff+r)] = V,
//                              [2 (yoff+r) + 1] = V#, [2 total_r + g] = SY_g
__host__ __device__ inline size_t vtab_offset(int nx, const GeomDevice& geo) {
  return (size_t)(2 * geo.total_p + geo.ngroups) * nx;
}

__device__ __forceinline__ int group_of(const GeomDevice& geo, int row, bool by_r) {
  int g = 0;
  while (g + 1 < geo.ngroups && (by_r ? geo.groups[g + 1].yoff : geo.groups[g + 1].uoff) <= row) ++g;
  return g;
}

__global__ void spectra_tables_kernel(Axis x, Axis y, double gamma, GeomDevice geo, double2* __restrict__ utab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  const int nxrows = geo.total_p + geo.ngroups;
  if (row < nxrows) {
    if (i >= x.n) return;
    const double k = x.k_first + i * x.dk;
    if (row < geo.total_p) {
      const int g = group_of(geo, row, false);
      const GeomGroup gr = geo.groups[g];
      double2 u, uh;
      phase_pair(k, gamma, geo.xs[gr.xoff + (row - gr.uoff)], u, uh);
      const double2 kc = make_double2(k, gamma * k);
      const double2 sx = is_ydir(gr.kind) ? across_factor(gr.b, kc) : along_factor(gr.kind, gr.a, kc);
      utab[(size_t)(2 * row) * x.n + i] = cmul(sx, u);
      utab[(size_t)(2 * row + 1) * x.n + i] = cmul(sx, uh);
    } else {
      const int g = row - geo.total_p;
      const GeomGroup gr = geo.groups[g];
      const double2 kc = make_double2(k, gamma * k);
      utab[(size_t)(2 * geo.total_p + g) * x.n + i] =
          is_ydir(gr.kind) ? across_factor(gr.b, kc) : along_factor(gr.kind, gr.a, kc);
    }
  } else {
    if (i >= y.n) return;
    double2* vtab = utab + vtab_offset(x.n, geo);
    const int vr = row - nxrows;
    const double k = y.k_first + i * y.dk;
    if (vr < geo.total_r) {
      const GeomGroup gr = geo.groups[group_of(geo, vr, true)];
      double2 v, vh;
      phase_pair(k, gamma, geo.ys[vr], v, vh);
      vtab[(size_t)(2 * vr) * y.n + i] = v;
      vtab[(size_t)(2 * vr + 1) * y.n + i] = vh;
      (void)gr;
    } else {
      const int g = vr - geo.total_r;
      const GeomGroup gr = geo.groups[g];
      const double2 kc = make_double2(k, gamma * k);
      vtab[(size_t)(2 * geo.total_r + g) * y.n + i] =
          is_ydir(gr.kind) ? along_factor(gr.kind, gr.a, kc) : across_factor(gr.b, kc);
    }
  }
}

size_t spectra_tables_len(const Axis& x, const Axis& y, const GeomDevice& geo) {
  return (size_t)(2 * geo.total_p + geo.ngroups) * x.n + (size_t)(2 * geo.total_r + geo.ngroups) * y.n;
}

hipError_t launch_spectra_tables(const Axis& x, const Axis& y, double gamma, const GeomDevice& geo, double2* utab,
                                 hipStream_t s) {
  const int nmax = x.n > y.n ? x.n : y.n;
  dim3 grid((nmax + 127) / 128, geo.total_p + geo.total_r + 2 * geo.ngroups);
  hipLaunchKernelGGL(spectra_tables_kernel, grid, dim3(128), 0, s, x, y, gamma, geo, utab);
  return hipGetLastError();
}

constexpr int kSpecThreads = 256;   // spectra kernel block size
constexpr int kSpecRows = 2;         // rows per spectra block
constexpr int kMChunk = 4;   // MBFs per pass of the parabolic (direct) kernel

// MBFs per pass of the separable per-sample kernel: 3 or 4, whichever pads
// the MBF count less (M = 6: 6 not 8 slots, M = 9: 9 not 12; ties take 4).
// The w tables hold mpad = the padded count of MBF slots.
static int spectra_mchunk(int nmbf) {
  const int p3 = (nmbf + 2) / 3 * 3, p4 = (nmbf + 3) / 4 * 4;
  return p3 < p4 ? 3 : 4;
}
static int spectra_mpad(int nmbf) {
  const int mc = spectra_mchunk(nmbf);
  return (nmbf + mc - 1) / mc * mc;
}

// Per-row contraction over y-centres, one thread per table entry
//   v = 0:  w [n2][m][pp] = SY_g(n2) sum_r conj(q_m,j(g,p,r)) V_gr(n2)
//   v = 1:  w#[n2][m][pp] = SY_g(n2) sum_r      q_m,j(g,p,r)  V#_gr(n2)
// stored as wtab[n2][v][mpad][ppad] with pp = poff_g + p.  Slots past a
// group's centre count and MBFs past nmbf hold zero, so the per-sample
// kernel runs whole chunks without bounds tests.  The row index n2 runs
// fastest over the threads: the V tables (rows of length ny) are read with
// coalesced loads, while the basis index and the coefficient of an entry are
// the same for a whole wave (when 64 divides ny) and come through scalar
// loads.
// One w entry: pair slot pp of MBF m in variant v at row n2.
__device__ __forceinline__ double2 w_entry(const Axis& x, const Axis& y, const GeomDevice& geo,
                                           const double2* __restrict__ utab, const double2* __restrict__ q, int nmbf,
                                           int v, int m, int pp, int n2) {
  int g = 0;
  while (g + 1 < geo.ngroups && geo.groups[g + 1].poff <= pp) ++g;
  const GeomGroup gr = geo.groups[g];
  const int p = pp - gr.poff;
  double2 acc = make_double2(0.0, 0.0);
  if (m < nmbf && p < gr.np) {
    const double2* vtab = utab + vtab_offset(x.n, geo);
    const int* irow = geo.index + gr.ioff + (size_t)p * gr.nr;
    const double2* qm = q + (size_t)m * geo.nbasis;
    // eight independent index, coefficient and V loads in flight at a time
    for (int r0 = 0; r0 < gr.nr; r0 += 8) {
      int jj[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) jj[k] = r0 + k < gr.nr ? irow[r0 + k] : -1;
      double2 qq[8], vv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        qq[k] = jj[k] >= 0 ? qm[jj[k]] : make_double2(0.0, 0.0);
        vv[k] = jj[k] >= 0 ? vtab[(size_t)(2 * (gr.yoff + r0 + k) + v) * y.n + n2] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc = cadd(acc, v == 0 ? cmulc(vv[k], qq[k]) : cmul(qq[k], vv[k]));   // conj(q) V or q V#
    }
    acc = cmul(acc, vtab[(size_t)(2 * geo.total_r + g) * y.n + n2]);
  }
  return acc;
}

constexpr int kRowsThreads = 256;
__global__ void __launch_bounds__(kRowsThreads)
spectra_rows_kernel(Axis x, Axis y, GeomDevice geo, const double2* __restrict__ utab,
                    const double2* __restrict__ q, int nmbf, int mpad, double2* __restrict__ wtab) {
  const int ppad = geo.ppad;
  const int per_v = mpad * ppad;
  const long long e = (long long)blockIdx.x * kRowsThreads + threadIdx.x;
  if (e >= (long long)2 * per_v * y.n) return;
  const int n2 = (int)(e % y.n);
  const int ent = (int)(e / y.n);
  const int v = ent / per_v;
  const int m = (ent % per_v) / ppad;
  const int pp = ent % ppad;
  wtab[((size_t)n2 * 2 + v) * per_v + (size_t)m * ppad + pp] = w_entry(x, y, geo, utab, q, nmbf, v, m, pp, n2);
}

// Per-sample sums of one block: thread = sample n1 (byte offset boff in a
// table row), rows n2_0 .. n2_0 + RB - 1 with w tables wrow[r] ([mpad][ppad]):
//   M_m^c(n1, n2) = sum_{g of component c} sum_p (SX_g U_gp)(n1) w[n2][m][p].
// A U value is loaded once and used for every row.  Padded centres use a
// clamped U times a zero w.
template <int RB, int MC, typename O>
__device__ __forceinline__ void spectra_block(const GeomDevice& geo, const double2* __restrict__ utab, size_t rs,
                                              unsigned boff, const double2* const (&wrow)[RB], int v, int nmbf,
                                              int mpad, int n1, int n2_0, int ny, O* __restrict__ spec) {
  const int ppad = geo.ppad;
  const size_t plane = rs * (size_t)ny;
  for (int m0 = 0; m0 < mpad; m0 += MC) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double2 acc[RB][MC];
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < MC; ++i) acc[r][i] = make_double2(0.0, 0.0);
      const int g0 = c == 0 ? 0 : geo.ngroups_x;
      const int g1 = c == 0 ? geo.ngroups_x : geo.ngroups;
      for (int g = g0; g < g1; ++g) {
        const GeomGroup gr = geo.groups[g];
        const int pend = (gr.np + kSpecPChunk - 1) / kSpecPChunk * kSpecPChunk;
        const size_t woff = (size_t)m0 * ppad + gr.poff;
        for (int p0 = 0; p0 < pend; p0 += kSpecPChunk) {
          double2 u[kSpecPChunk];
#pragma unroll
          for (int k = 0; k < kSpecPChunk; ++k) {
            const int prow = gr.uoff + min(p0 + k, gr.np - 1);
            u[k] = at_byte(utab + (size_t)(2 * prow + v) * rs, boff);
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const double2* wg = wrow[r] + woff + p0;
#pragma unroll
            for (int k = 0; k < kSpecPChunk; ++k) {
#pragma unroll
              for (int i = 0; i < MC; ++i) acc[r][i] = cfma(acc[r][i], u[k], wg[(size_t)i * ppad + k]);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (n2_0 + r >= ny) continue;
#pragma unroll
        for (int i = 0; i < MC; ++i) {
          if (m0 + i < nmbf)
            spec[((size_t)(m0 + i) * 4 + 2 * v + c) * plane + (size_t)(n2_0 + r) * rs + n1] = from_d<O>(acc[r][i]);
        }
      }
    }
  }
}

// w tables from spectra_rows_kernel; every thread of a block reads the same
// entries (wave-uniform addresses, served by scalar loads).  Block =
// kSpecThreads samples of kSpecRows rows and one variant v (blockIdx.z:
// 0 = M with U and w, 1 = M# with U# and w#).  O is the stored type:
// complex128 for FP64 grids, complex64 (rounded from the FP64 sums) for
// mixed ones.
template <typename O, int MC>
__global__ void __launch_bounds__(kSpecThreads)
spectra_kernel(Axis x, Axis y, GeomDevice geo, const double2* __restrict__ utab,
               const double2* __restrict__ wtab, int nmbf, int mpad, O* __restrict__ spec) {
  constexpr int RB = kSpecRows;
  const int n2_0 = blockIdx.y * RB;
  const int v = blockIdx.z;
  const int n1 = blockIdx.x * kSpecThreads + threadIdx.x;
  if (n1 >= x.n) return;
  const double2* wrow[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) wrow[r] = wtab + ((size_t)min(n2_0 + r, y.n - 1) * 2 + v) * mpad * geo.ppad;
  spectra_block<RB, MC, O>(geo, utab, (size_t)x.n, (unsigned)n1 * (unsigned)sizeof(double2), wrow, v, nmbf, mpad, n1,
                       n2_0, y.n, spec);
}

// Dynamic LDS of the spectra adjoint's row kernel: the testing and reflected
// accumulators of every MBF and distinct x-centre.
size_t adj_spectra_lds_bytes(const GeomDevice& geo, int nmbf) { return sizeof(double2) * 2 * (size_t)nmbf * geo.total_p; }

size_t spectra_lds_bytes(const GeomDevice& geo, int nmbf) {
  (void)nmbf;
  return sizeof(double2) * (size_t)(2 * geo.total_r + geo.ngroups);
}


size_t spectra_scratch_len(const Axis& y, const GeomDevice& geo, int nmbf) {
  return (size_t)y.n * 2 * spectra_mpad(nmbf) * geo.ppad;
}

hipError_t launch_spectra(const Axis& x, const Axis& y, double gamma, const GeomDevice& geo, const double2* utab,
                          const double2* q, int nmbf, double2* scratch, void* spec, int precision, hipStream_t s) {
  (void)gamma;
  const int mpad = spectra_mpad(nmbf);
  dim3 grid((x.n + kSpecThreads - 1) / kSpecThreads, (y.n + kSpecRows - 1) / kSpecRows, 2);
  const long long rows_entries = (long long)2 * mpad * geo.ppad * y.n;
  hipLaunchKernelGGL(spectra_rows_kernel, dim3((unsigned)((rows_entries + kRowsThreads - 1) / kRowsThreads)),
                     dim3(kRowsThreads), 0, s, x, y, geo, utab, q, nmbf, mpad, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool three = spectra_mchunk(nmbf) == 3;
  if (precision == 0) {
    if (three)
      hipLaunchKernelGGL((spectra_kernel<double2, 3>), grid, dim3(kSpecThreads), 0, s, x, y, geo, utab, scratch, nmbf,
                         mpad, (double2*)spec);
    else
      hipLaunchKernelGGL((spectra_kernel<double2, 4>), grid, dim3(kSpecThreads), 0, s, x, y, geo, utab, scratch, nmbf,
                         mpad, (double2*)spec);
  } else {
    if (three)
      hipLaunchKernelGGL((spectra_kernel<float2, 3>), grid, dim3(kSpecThreads), 0, s, x, y, geo, utab, scratch, nmbf,
                         mpad, (float2*)spec);
    else
      hipLaunchKernelGGL((spectra_kernel<float2, 4>), grid, dim3(kSpecThreads), 0, s, x, y, geo, utab, scratch, nmbf,
                         mpad, (float2*)spec);
  }
  return hipGetLastError();
}

// ------------------------------------------------ parabolic contour
// On the parabolic contour k_c = (1 + i g(|k|)) k couples kx and ky, so the
// transforms no longer split into x and y tables: each sample sums its bases
// directly, F_j(k_c) = SX(kcx) SY(kcy) exp(-i k_c . c_j) with
// exp(-i k_c . c) = exp(g k.c) (cos k.c - i sin k.c) and, for the reflected
// spectrum, exp(+i k_c . c) = exp(-g k.c) (cos k.c + i sin k.c) (the shape
// factors are even).  Groups whose centres are equally spaced in x and y use
// per-axis recurrences instead (one complex product per centre step).  One
// thread per sample; the coefficients of a basis are the same for every
// thread (wave-uniform loads); MBFs in chunks of kMChunk.
constexpr int kDirectThreads = 256;
template <typename O>
__global__ void __launch_bounds__(kDirectThreads)
spectra_direct_kernel(Axis x, Axis y, Contour cont, GeomDevice geo, const double2* __restrict__ q,
                      const double2* __restrict__ qd, int nmbf, O* __restrict__ spec) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= x.n * y.n) return;
  const int n1 = idx % x.n, n2 = idx / x.n;
  const double kx = x.k_first + n1 * x.dk;
  const double ky = y.k_first + n2 * y.dk;
  double g, slope;
  contour_ratio(hypot(kx, ky), cont.gamma, cont.parabolic, cont.beta_end, g, slope);
  const double2 kcx = make_double2(kx, g * kx), kcy = make_double2(ky, g * ky);
  const size_t plane = (size_t)x.n * y.n;
  for (int m0 = 0; m0 < nmbf; m0 += kMChunk) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double2 acc[kMChunk], acch[kMChunk];
#pragma unroll
      for (int i = 0; i < kMChunk; ++i) acc[i] = acch[i] = make_double2(0.0, 0.0);
      const int g0 = c == 0 ? 0 : geo.ngroups_x;
      const int g1 = c == 0 ? geo.ngroups_x : geo.ngroups;
      for (int gi = g0; gi < g1; ++gi) {
        const GeomGroup gr = geo.groups[gi];
        const double2 sx = is_ydir(gr.kind) ? across_factor(gr.b, kcx) : along_factor(gr.kind, gr.a, kcx);
        const double2 sy = is_ydir(gr.kind) ? along_factor(gr.kind, gr.a, kcy) : across_factor(gr.b, kcy);
        const double2 shape = cmul(sx, sy);
        if (gr.uniform) {
          // equally spaced centres: the x and y phase factors follow by
          // recurrence, U_{p+1} = U_p Rx, V_{r+1} = V_r Ry, and the sum over r
          // is formed once per x-centre: M += shape U_p sum_r conj(q) V_r
          double2 u, uh, rx, rxh, v0, v0h, ry, ryh;
          phase_pair(kx, g, geo.xs[gr.xoff], u, uh);
          phase_pair(kx, g, gr.dxc, rx, rxh);
          phase_pair(ky, g, geo.ys[gr.yoff], v0, v0h);
          phase_pair(ky, g, gr.dyc, ry, ryh);
          double2 ga[kMChunk], gah[kMChunk];
#pragma unroll
          for (int i = 0; i < kMChunk; ++i) ga[i] = gah[i] = make_double2(0.0, 0.0);
          for (int p = 0; p < gr.np; ++p) {
            double2 w[kMChunk], wh[kMChunk];
#pragma unroll
            for (int i = 0; i < kMChunk; ++i) w[i] = wh[i] = make_double2(0.0, 0.0);
            double2 v = v0, vh = v0h;
            // coefficients in slot order (zero for empty slots): no index lookups
            const double2* qrow = qd + gr.ioff + (size_t)p * gr.nr;
#pragma unroll 4
            for (int r = 0; r < gr.nr; ++r) {
#pragma unroll
              for (int i = 0; i < kMChunk; ++i) {
                if (m0 + i < nmbf) {
                  const double2 qv = qrow[(size_t)(m0 + i) * geo.total_idx + r];
                  w[i] = cfma(w[i], v, make_double2(qv.x, -qv.y));   // conj(q) V
                  wh[i] = cfma(wh[i], vh, qv);                       // q V#
                }
              }
              v = cmul(v, ry);
              vh = cmul(vh, ryh);
            }
#pragma unroll
            for (int i = 0; i < kMChunk; ++i) {
              ga[i] = cfma(ga[i], u, w[i]);
              gah[i] = cfma(gah[i], uh, wh[i]);
            }
            u = cmul(u, rx);
            uh = cmul(uh, rxh);
          }
#pragma unroll
          for (int i = 0; i < kMChunk; ++i) {
            acc[i] = cfma(acc[i], shape, ga[i]);
            acch[i] = cfma(acch[i], shape, gah[i]);
          }
          continue;
        }
        for (int p = 0; p < gr.np; ++p) {
          const double xc = geo.xs[gr.xoff + p];
          for (int r = 0; r < gr.nr; ++r) {
            const int j = geo.index[gr.ioff + p * gr.nr + r];
            if (j < 0) continue;
            const double kd = kx * xc + ky * geo.ys[gr.yoff + r];
            double sn, cs;
            sincos(kd, &sn, &cs);
            const double e = exp(g * kd);
            const double ei = 1.0 / e;
            const double2 f = cmul(shape, make_double2(e * cs, -e * sn));
            const double2 fh = cmul(shape, make_double2(ei * cs, ei * sn));
#pragma unroll
            for (int i = 0; i < kMChunk; ++i) {
              if (m0 + i < nmbf) {
                const double2 qv = q[(size_t)(m0 + i) * geo.nbasis + j];
                acc[i] = cfma(acc[i], f, make_double2(qv.x, -qv.y));   // conj(q) F
                acch[i] = cfma(acch[i], fh, qv);                       // q F#
              }
            }
          }
        }
      }
      const size_t o = (size_t)n2 * x.n + n1;
#pragma unroll
      for (int i = 0; i < kMChunk; ++i) {
        if (m0 + i < nmbf) {
          spec[((size_t)(m0 + i) * 4 + c) * plane + o] = from_d<O>(acc[i]);
          spec[((size_t)(m0 + i) * 4 + 2 + c) * plane + o] = from_d<O>(acch[i]);
        }
      }
    }
  }
}

// qd[m][slot] = q[m][index[slot]] (0 for empty slots), slot order of the groups.
__global__ void gather_slots_kernel(GeomDevice geo, const double2* __restrict__ q, int nmbf,
                                    double2* __restrict__ qd) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nmbf * geo.total_idx) return;
  const int m = e / geo.total_idx, li = e % geo.total_idx;
  const int j = geo.index[li];
  qd[e] = j < 0 ? make_double2(0.0, 0.0) : q[(size_t)m * geo.nbasis + j];
}

size_t spectra_direct_scratch_len(const GeomDevice& geo, int nmbf) { return (size_t)nmbf * geo.total_idx; }

hipError_t launch_spectra_direct(const Axis& x, const Axis& y, const Contour& c, const GeomDevice& geo,
                                 const double2* q, int nmbf, double2* scratch, void* spec, int precision,
                                 hipStream_t s) {
  const int ng = nmbf * geo.total_idx;
  hipLaunchKernelGGL(gather_slots_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, geo, q, nmbf, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = x.n * y.n;
  if (precision == 0)
    hipLaunchKernelGGL(spectra_direct_kernel<double2>, dim3((n + kDirectThreads - 1) / kDirectThreads),
                       dim3(kDirectThreads), 0, s, x, y, c, geo, q, scratch, nmbf, (double2*)spec);
  else
    hipLaunchKernelGGL(spectra_direct_kernel<float2>, dim3((n + kDirectThreads - 1) / kDirectThreads),
                       dim3(kDirectThreads), 0, s, x, y, c, geo, q, scratch, nmbf, (float2*)spec);
  return hipGetLastError();
}

// ------------------------------------------------ adjoint
// Gradient of L w.r.t. q from the gradient w.r.t. the spectra (gspec, same
// layout as spec, in the d/dRe + i d/dIm convention):
//   gq_mj = sum_n conj(gM_m(n)) F_j(k_c(n)) + gM#_m(n) conj(F_j(-k_c(n))).
// Per row n2 the sums over n1 are reduced per (m, g, p), one wave per
// (m, p) item (lane-strided sums, then a butterfly over the wave's lanes),
// then multiplied by the row factors and written to rowacc[n2][m][j]; two
// more kernels sum rowacc over rows in a fixed order (row classes modulo
// kAdjSplit in place, then the classes).
constexpr int kAdjThreads = 256;
constexpr int kAdjSplit = 64;

__global__ void __launch_bounds__(kAdjThreads)
adj_spectra_rows_kernel(Axis x, Axis y, GeomDevice geo, const double2* __restrict__ utab,
                        const double2* __restrict__ gspec, int nmbf, double2* __restrict__ rowacc) {
  extern __shared__ double2 sh[];
  // a1, a2: [nmbf][total_p]
  double2* a1 = sh;
  double2* a2 = sh + nmbf * geo.total_p;
  __shared__ GeomGroup grp[kMaxGroups];
  const int n2 = blockIdx.x;
  if ((int)threadIdx.x < geo.ngroups) grp[threadIdx.x] = geo.groups[threadIdx.x];
  __syncthreads();
  const size_t plane = (size_t)x.n * y.n;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nitems = nmbf * geo.total_p;
  for (int it = wave; it < nitems; it += kAdjThreads / 64) {
    const int m = it / geo.total_p;
    const int prow = it - m * geo.total_p;   // U row uoff_g + p of the group g holding it
    int g = 0;
    while (g + 1 < geo.ngroups && grp[g + 1].uoff <= prow) ++g;
    const int comp = is_ydir(grp[g].kind) ? 1 : 0;
    double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
    for (int n1 = lane; n1 < x.n; n1 += 64) {
      const double2 u = utab[(size_t)(2 * prow) * x.n + n1];        // SX U
      const double2 uh = utab[(size_t)(2 * prow + 1) * x.n + n1];   // SX U#
      const double2 gm = gspec[((size_t)m * 4 + comp) * plane + (size_t)n2 * x.n + n1];
      const double2 gmh = gspec[((size_t)m * 4 + 2 + comp) * plane + (size_t)n2 * x.n + n1];
      s1 = cadd(s1, cmulc(u, gm));      // conj(gM) SX U  (conj applied below)
      s2 = cadd(s2, cmulc(gmh, uh));    // gM# conj(SX U#)
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1.x += __shfl_xor(s1.x, off, 64);
      s1.y += __shfl_xor(s1.y, off, 64);
      s2.x += __shfl_xor(s2.x, off, 64);
      s2.y += __shfl_xor(s2.y, off, 64);
    }
    if (lane == 0) {
      a1[it] = s1;
      a2[it] = s2;
    }
  }
  __syncthreads();
  // rowacc[n2][m][j] = SY V_r a1[p] + conj(SY V#_r) a2[p]
  const int nent = nmbf * geo.total_idx;
  for (int e = threadIdx.x; e < nent; e += blockDim.x) {
    const int m = e / geo.total_idx;
    const int li = e % geo.total_idx;
    int g = 0;
    while (g + 1 < geo.ngroups && grp[g + 1].ioff <= li) ++g;
    const GeomGroup gr = grp[g];
    const int j = geo.index[li];
    if (j < 0) continue;
    const int p = (li - gr.ioff) / gr.nr;
    const int r = (li - gr.ioff) % gr.nr;
    const double2* vtab = utab + vtab_offset(x.n, geo);
    const double2 sy = vtab[(size_t)(2 * geo.total_r + g) * y.n + n2];
    const double2 v = vtab[(size_t)(2 * (gr.yoff + r)) * y.n + n2];
    const double2 vh = vtab[(size_t)(2 * (gr.yoff + r) + 1) * y.n + n2];
    const double2 t1 = cmul(cmul(sy, v), a1[m * geo.total_p + gr.uoff + p]);
    const double2 t2 = cmulc(a2[m * geo.total_p + gr.uoff + p], cmul(sy, vh));
    rowacc[((size_t)n2 * nmbf + m) * geo.nbasis + j] = cadd(t1, t2);
  }
}

// In place: rowacc[s][e] <- sum over rows r = s, s + kAdjSplit, ... of
// rowacc[r][e], for s < min(kAdjSplit, nrows) (fixed order; thread (s, e) is
// the only one to read or write any row of its class at column e).
__global__ void adj_spectra_split_kernel(double2* __restrict__ rowacc, int nrows, int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= count || s >= nrows) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int r = s; r < nrows; r += kAdjSplit) acc = cadd(acc, rowacc[(size_t)r * count + e]);
  rowacc[(size_t)s * count + e] = acc;
}

// gq[m][j] = sum_n2 rowacc[n2][m][j]  (fixed summation order)
__global__ void adj_spectra_sum_kernel(const double2* __restrict__ rowacc, int nrows, int count,
                                       double2* __restrict__ gq) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int r = 0; r < nrows; ++r) acc = cadd(acc, rowacc[(size_t)r * count + e]);
  gq[e] = acc;
}

size_t adj_spectra_scratch(const Axis& y, const GeomDevice& geo, int nmbf) {
  return sizeof(double2) * (size_t)y.n * nmbf * geo.nbasis;
}

hipError_t launch_adj_spectra(const Axis& x, const Axis& y, const GeomDevice& geo,
                              const double2* utab, const double2* gspec, int nmbf, double2* rowacc,
                              double2* gq, hipStream_t s) {
  const size_t lds = adj_spectra_lds_bytes(geo, nmbf);
  hipLaunchKernelGGL(adj_spectra_rows_kernel, dim3(y.n), dim3(kAdjThreads), lds, s, x, y, geo, utab,
                     gspec, nmbf, rowacc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int count = nmbf * geo.nbasis;
  hipLaunchKernelGGL(adj_spectra_split_kernel, dim3((count + 255) / 256, kAdjSplit), dim3(256), 0, s, rowacc, y.n,
                     count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_spectra_sum_kernel, dim3((count + 255) / 256), dim3(256), 0, s, rowacc,
                     y.n < kAdjSplit ? y.n : kAdjSplit, count, gq);
  return hipGetLastError();
}

}  // namespace cfft
