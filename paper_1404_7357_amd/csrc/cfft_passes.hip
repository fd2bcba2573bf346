// The C-FFT passes (Sec. III-B.3, eqs. fftexp and fftarry; Appendix change
// of variables), their adjoint, and the table lookup.
//
// With s(n) = (-1)^n, K = dkx dky / 4 pi^2, sigma = exp(-i pi (nx+ny)/2) and
// the ray weight W = (1 + i gamma)^2, the table is
//   Z(j1,j2) = K sigma W s(j1+j2) sum_b Dy(j2)^b/b! DFT_n2[ s(n2) (gamma ky)^b S_{P-b} ](j2)
//   S_c(j1,n2) = sum_{a<=c} Dx(j1)^a/a! DFT_n1[ s(n1) (gamma kx)^a H(n1,n2) ](j1)
//   H = M_m . G . M#_n
// which is the total-degree-P Taylor expansion of E_I with every
// displacement factor moved outside its transform.  With the tensor-product
// truncation (a <= P and b <= P, not in the paper) every column term reads
// the full row sum S_P, so only S_P is stored.
//
// Row pass: a block assembles H of one row from G and the spectra (FP64),
// then for a = 0..P multiplies by gamma kx, runs an in-register/LDS Stockham
// FFT along n1, folds the result into the running partial sum S (FP64
// accumulators) and writes S_a (S_P only, tensor truncation).
// Column pass: one block handles a tile of C adjacent columns of one pair;
// each wave loads whole C-column row segments of S_{P-b} straight into
// registers, FFTs every column along n2 (LDS exchanges), accumulates
// Dy^b/b! times the result in FP64 and writes the scaled table.
//
// Precision.  Every pass kernel has a storage type Vs (spectra,
// intermediates and table in HBM: complex128 on FP64 grids, complex64 on
// mixed grids) and a compute type Vc (butterflies, twiddles and LDS
// exchanges of the transforms).  FP64 grids compute in FP64.  Mixed grids
// compute in FP32, except where the Taylor recombination would amplify FP32
// rounding past the mixed path's error target (long transforms): there they
// compute in FP64 on the FP32-stored data, so the HBM traffic stays that of
// the mixed path.  The integrand, the Taylor weights, the partial sums S_c
// and the column accumulators are FP64 in every case.
#include <algorithm>
#include <map>
#include <type_traits>
#include <vector>

#include "cfft_device.h"
#include "cfft_internal.h"

namespace cfft {

// LDS padding of the row transforms: one pad slot per 2^row_pad<V>() elements
// (16-byte elements: every 16; 8-byte elements: every 8).
template <typename V> __host__ __device__ constexpr int row_pad() { return sizeof(V) == 16 ? 4 : 3; }

// Minimum waves per SIMD requested for the row pass (1: no constraint).  The
// FP32 rows of 1024 points and more take 4 waves per SIMD at the price of a
// small spill (-9% on the frequency sweep); shorter rows lose from it.
template <typename Vc, int N> constexpr int row_min_waves() { return (sizeof(Vc) == 8 && N >= 1024) ? 4 : 1; }

// Whether the row pass rebuilds its per-point factors and store addresses in
// every term (from an opaque copy of the thread index) instead of keeping
// them live across the term loop: only in the FP32 rows of 1024 points and
// more, whose kernels otherwise spill at the 128 registers of their
// occupancy target (elsewhere the rebuilt factors cost 3%).
template <typename Vc, int N> constexpr bool row_opaque_t() { return sizeof(Vc) == 8 && N >= 1024; }

// Points per thread of the row transforms.  In the FP64 rows of 4096 points,
// 16 points per thread take 256 registers and one wave per SIMD, and 4 points
// per thread (radix-4 stages, 1024 threads, four waves per SIMD) took 11%
// longer than 8: two more LDS exchanges per transform.
template <typename Vc, int N> __host__ __device__ constexpr int row_r() { return 8; }

// Whether the row pass runs its Taylor terms two at a time through one
// sequence of transform stages (fft_forward2): in the FP64 transforms of
// rows of 2048 points and more (one 512- or 256-thread block per row, two
// waves per SIMD at about 200 registers, latency-bound), where the second
// transform's registers still fit that occupancy and its LDS region fits
// beside the first.
template <typename Vc, int N> constexpr bool row_paired() { return sizeof(Vc) == 16 && N >= 2048; }

// Whether the row pass keeps its blocks resident and loops over rows: FP64
// rows of 4096 points (one block per CU, each row ~25 us), where a fresh
// block per row costs about 4% in dispatch and start-up (4096^2 FP64:
// 14.24 -> 13.68 ms).  The loop raises the kernel to 256 registers: at 2048
// points that halves the resident blocks (the pass lost 27%), and with FP32
// storage (a larger spill) it gained nothing.
template <typename Vs, typename Vc, int N> constexpr bool row_persistent() {
  return sizeof(Vs) == 16 && row_paired<Vc, N>() && N >= 4096;
}

template <int N, int R> struct RowCfg {
  static constexpr int T = N / R;
  static constexpr int ROWS = T >= 64 ? 1 : 64 / T;
  static constexpr int THREADS = ROWS * T;
};

struct RowArgs {
  int tensor;   // tensor-product truncation: only S_P is stored, in slot 0
  int stream_out;   // write the intermediates with non-temporal stores (see PassParams)
  int band;     // x2 zero-padded grid: integrand only on n in [N/4, 3N/4) per axis
  int parabolic;                // per-sample contour ratio (see row_terms_general)
  double ky0, dky, beta_end;
  const double2* g;
  const void* spec;   // Vs elements
  void* inter;        // Vs elements
  const void* tw;     // Vc elements
  int nx, ny, order, npairs;
  double kx0, dkx, x0, ddx, gamma;
  double rinv[kMaxOrder + 1];   // 1/i (the Taylor weights need no division)
  int pm[kMaxPairsPerLaunch];
  int pn[kMaxPairsPerLaunch];
};

// Sample n of an axis of n_len samples lies in the band of a x2 zero-padded grid.
__device__ __forceinline__ bool in_band(int n, int n_len) { return n >= n_len / 4 && n < 3 * (n_len / 4); }

// Contour weight W = (1 + i g)(1 + i beta_I') at the sample (kx, ky).
template <typename Args>
__device__ __forceinline__ double2 contour_weight(const Args& a, double kx, double ky) {
  double g, slope;
  contour_ratio(hypot(kx, ky), a.gamma, a.parabolic, a.beta_end, g, slope);
  return cmul(make_double2(1.0, g), make_double2(1.0, slope));
}

// Row terms when the contour ratio g varies per sample (parabolic contour):
// (g ky)^b is no longer constant along a row, so for b = 0..P the row pass
// forms S'_b = sum_{a <= P-b} Dx^a/a! DFT_n1[ (g kx)^a (g ky)^b f ] and
// stores it in slot b; the column pass then applies no ky factor.  That is
// (P+1)(P+2)/2 row transforms, the N_t of eq. fftarry.  f already carries
// s(n1) and the contour weight.
template <typename Vs, typename Vc, int N, int R, bool WAVE, int PS, typename Args>
__device__ __forceinline__ void row_terms_general(const Args& a, const Vc (&f)[R], Vc* lds, const Vc* ltw, int t,
                                                  int n2, Vs* dst0, size_t slot_stride, bool store) {
  constexpr int T = N / R;
  using Rc = typename real_of<Vc>::type;
  const double ky = a.ky0 + n2 * a.dky;
  double gkx[R], gky[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double kx = a.kx0 + (t + T * r) * a.dkx;
    double g, slope;
    contour_ratio(hypot(kx, ky), a.gamma, a.parabolic, a.beta_end, g, slope);
    gkx[r] = g * kx;
    gky[r] = g * ky;
  }
  for (int b = 0; b <= a.order; ++b) {
    double2 S[R];
#pragma unroll
    for (int r = 0; r < R; ++r) S[r] = make_double2(0.0, 0.0);
    for (int ao = 0; ao + b <= a.order; ++ao) {
      Vc x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double w = 1.0;
        for (int i = 0; i < ao; ++i) w *= gkx[r];
        for (int i = 0; i < b; ++i) w *= gky[r];
        x[r] = cscale(f[r], (Rc)w);
      }
      fft_forward<Vc, N, R, WAVE, PS>(x, lds, ltw, t);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double dx = a.x0 + (t + T * r) * a.ddx;
        double cf = 1.0;
        for (int i = 1; i <= ao; ++i) cf *= dx * a.rinv[i];
        const double2 xv = to_d(x[r]);
        S[r] = make_double2(S[r].x + cf * xv.x, S[r].y + cf * xv.y);
      }
    }
    if (store) {
#pragma unroll
      for (int r = 0; r < R; ++r) dst0[(size_t)b * slot_stride + t + T * r] = from_d<Vs>(S[r]);
    }
  }
}

// Integrand samples s(n1) W H(n1, n2) of the R points of thread t on row n2
// (H = Mx_m (Gxx Mx#_n + Gxy My#_n) + My_m (Gxy Mx#_n + Gyy My#_n)).  The
// loads of all points are issued without branches (a row past the end reads
// row row0 and is zeroed by a select) so that they are in flight together.
// On a zero-padded grid (BAND) the point n1 = t + T r lies in the band
// [N/4, 3N/4) exactly when R/4 <= r < 3R/4 (T = N/R), the same for every
// thread, so the other points are neither loaded nor computed.
template <bool BAND, typename Vs, typename Vc, int N, int R>
__device__ __forceinline__ void row_inputs(const RowArgs& a, int t, int n2, bool valid, int row0, int m, int n,
                                           size_t plane, Vc (&f)[R]) {
  constexpr int T = N / R;
  const size_t rowb = (size_t)(valid ? n2 : row0) * N;
  const Vs* sp = (const Vs*)a.spec;
  const Vs* spm = sp + (size_t)m * 4 * plane + rowb;
  const Vs* spn = sp + ((size_t)n * 4 + 2) * plane + rowb;
  const double2* gr = a.g + rowb;
  auto live = [](int r) { return !BAND || (4 * r >= R && 4 * r < 3 * R); };
  double2 h[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    h[r] = make_double2(0.0, 0.0);
    if (!live(r)) continue;
    const int n1 = t + T * r;
    const double2 gxx = gr[n1], gxy = gr[plane + n1], gyy = gr[2 * plane + n1];
    const double2 mx = to_d(spm[n1]), my = to_d(spm[plane + n1]);
    const double2 mxh = to_d(spn[n1]), myh = to_d(spn[plane + n1]);
    h[r] = cadd(cmul(mx, cadd(cmul(gxx, mxh), cmul(gxy, myh))), cmul(my, cadd(cmul(gxy, mxh), cmul(gyy, myh))));
  }
  if (a.parabolic) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (live(r)) h[r] = cmul(h[r], contour_weight(a, a.kx0 + (t + T * r) * a.dkx, a.ky0 + n2 * a.dky));
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double2 v = (live(r) && ((t + T * r) & 1)) ? make_double2(-h[r].x, -h[r].y) : h[r];
    f[r] = from_d<Vc>(valid ? v : make_double2(0.0, 0.0));
  }
}

template <typename Vs, typename Vc, int N, int R>
__global__ void __launch_bounds__((RowCfg<N, R>::THREADS), (row_min_waves<Vc, N>())) row_pass_kernel(RowArgs a) {
  using Cfg = RowCfg<N, R>;
  constexpr int T = Cfg::T, ROWS = Cfg::ROWS;
  using Rc = typename real_of<Vc>::type;
  __shared__ Vc lds[(row_paired<Vc, N>() ? 2 : 1) * ROWS * lds_len<row_pad<Vc>()>(N)];
  __shared__ Vc ltw[TwLds<N>::LEN];
  load_twiddles<Vc, N>(ltw, (const Vc*)a.tw, threadIdx.x, Cfg::THREADS);
  __syncthreads();   // twiddle tables ready
  // One row (ROWS rows) of one pair: logical block lid.
  auto process = [&](const int lid) {
    const int pair = lid % a.npairs;
    const int rb = lid / a.npairs;
    const int grp = threadIdx.x / T;
    const int t = threadIdx.x % T;
    // zero-padded grid: only the rows of the band are launched (the others
    // are zero and the column pass does not read them)
    const int row0 = a.band ? a.ny / 4 : 0;
    const int n2 = row0 + rb * ROWS + grp;
    const bool valid = n2 < a.ny - row0;
    const size_t plane = (size_t)a.nx * a.ny;
    const int m = a.pm[pair], n = a.pn[pair];
    Vs* inter = (Vs*)a.inter;

    Vc f[R];
    if (a.band) row_inputs<true, Vs, Vc, N, R>(a, t, n2, valid, row0, m, n, plane, f);
    else row_inputs<false, Vs, Vc, N, R>(a, t, n2, valid, row0, m, n, plane, f);
    Vc* my_lds = lds + grp * lds_len<row_pad<Vc>()>(N);
    if (a.parabolic) {
      const size_t slot = (size_t)a.ny * N;
      row_terms_general<Vs, Vc, N, R, (T <= 64), row_pad<Vc>()>(
          a, f, my_lds, ltw, t, valid ? n2 : 0, inter + ((size_t)pair * (a.order + 1) * a.ny + (valid ? n2 : 0)) * N,
          slot, valid);
      return;
    }
    double2 S[R];
  #pragma unroll
    for (int r = 0; r < R; ++r) S[r] = make_double2(0.0, 0.0);
    const int nsl = a.tensor ? 1 : a.order + 1;
    // Fold the transform xx of term ao into S and store S_ao.
    auto accumulate = [&](int ao, int tb, const Vc(&xx)[R]) {
      const bool keep = !a.tensor || ao == a.order;
      Vs* dst = inter + (((size_t)pair * nsl + (a.tensor ? 0 : ao)) * a.ny + (valid ? n2 : 0)) * N;
  #pragma unroll
      for (int r = 0; r < R; ++r) {
        // Dx(j1)^a / a!, rebuilt per term (cheaper than keeping it live)
        const double dx = a.x0 + (tb + T * r) * a.ddx;
        double cf = 1.0;
        for (int i = 1; i <= ao; ++i) cf *= dx * a.rinv[i];
        const double2 xv = to_d(xx[r]);
        S[r] = make_double2(S[r].x + cf * xv.x, S[r].y + cf * xv.y);
        if (valid && keep) {
          if (a.stream_out) store_nt(dst + tb + T * r, from_d<Vs>(S[r]));
          else dst[tb + T * r] = from_d<Vs>(S[r]);
        }
      }
    };
    // f <- (gamma kx) f: the input of the next term
    auto next_term = [&](int tb) {
  #pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n1 = tb + T * r;
        f[r] = cscale(f[r], (Rc)(a.gamma * (a.kx0 + n1 * a.dkx)));
      }
    };
    for (int ao = 0; ao <= a.order;) {
      // opaque copy of t: the per-point factors and store addresses are
      // rebuilt per term instead of being hoisted and held across the loop
      int tb = t;
      if constexpr (row_opaque_t<Vc, N>()) asm volatile("" : "+v"(tb));
      if (ao > 0) next_term(tb);
      Vc x[R];
  #pragma unroll
      for (int r = 0; r < R; ++r) x[r] = f[r];
      if constexpr (row_paired<Vc, N>()) {
        if (ao < a.order) {
          // terms ao and ao + 1 through one sequence of stages
          next_term(tb);
          Vc z[R];
  #pragma unroll
          for (int r = 0; r < R; ++r) z[r] = f[r];
          fft_forward2<Vc, N, R, (T <= 64), row_pad<Vc>()>(x, z, my_lds, my_lds + lds_len<row_pad<Vc>()>(N), ltw, t);
          accumulate(ao, tb, x);
          accumulate(ao + 1, tb, z);
          ao += 2;
          continue;
        }
      }
      fft_forward<Vc, N, R, (T <= 64), row_pad<Vc>()>(x, my_lds, ltw, t);
      accumulate(ao, tb, x);
      ++ao;
    }
  };
  if constexpr (row_persistent<Vs, Vc, N>()) {
    // persistent blocks (as many as fit the device at once) take the logical
    // blocks vb = blockIdx.x + i gridDim.x in turn; gridDim.x is a multiple
    // of 8, so every one stays on its block's XCD and the remap keeps its
    // order
    const int total = (((a.band ? a.ny / 2 : a.ny) + ROWS - 1) / ROWS) * a.npairs;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) process(xcd_remap(vb, total));
  } else {
    process(xcd_remap(blockIdx.x, gridDim.x));
  }
}

// Grouped row pass (N <= 1024): one block per (row, group of up to NPW pairs
// sharing the testing MBF m), one transform of T = N/8 threads per pair.  The
// block first forms, once for all its pairs,
//   A_x = s(n1) (Mx_m Gxx + My_m Gxy),  A_y = s(n1) (Mx_m Gxy + My_m Gyy)
// in LDS (FP64); each transform then needs only the reflected spectra of its
// own basis MBF n, H = A_x Mx#_n + A_y My#_n.  That reads (5 + 2 NPW)/NPW
// input arrays per pair instead of 7.
struct RowGArgs {
  int tensor;
  int stream_out;
  int band;
  int parabolic;
  double ky0, dky, beta_end;
  const double2* g;
  const void* spec;   // Vs elements
  void* inter;        // Vs elements
  const void* tw;     // Vc elements
  int nx, ny, order, ngroups;
  double kx0, dkx, x0, ddx, gamma;
  double rinv[kMaxOrder + 1];
  int gm[kMaxPairsPerLaunch];      // testing MBF of each group
  int gfirst[kMaxPairsPerLaunch];  // first slot of the group in gpair
  int gcnt[kMaxPairsPerLaunch];    // pairs in the group (<= NPW)
  int gpair[kMaxPairsPerLaunch];   // pair index (position in the launch) per slot
  int pn[kMaxPairsPerLaunch];      // basis MBF per pair index
};

template <int N, int NPW> struct RowGCfg {
  static constexpr int R = 8;
  static constexpr int T = N / R;
  static constexpr int THREADS = NPW * T;
};

// A tables of the grouped row pass (see above) for row n2, in LDS.  The loads
// of all of a thread's entries are issued without branches so that they are
// in flight together; the contour weight follows in a loop of its own.  On a
// zero-padded grid (BAND) only the band [N/4, 3N/4) is formed: the
// transforms never read the entries outside it.
template <bool BAND, typename Vs, int N, int THREADS>
__device__ __forceinline__ void grouped_a_tables(const RowGArgs& a, int m, int n2, size_t row, size_t plane,
                                                 double2* ax, double2* ay) {
  constexpr int LEN = BAND ? N / 2 : N;
  constexpr int I0 = BAND ? N / 4 : 0;
  constexpr int PER = LEN / THREADS;
  static_assert(PER * THREADS == LEN, "whole rows per block");
  const Vs* sp = (const Vs*)a.spec;
  double2 vx[PER], vy[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = I0 + threadIdx.x + THREADS * u;
    const double2 gxx = a.g[row + i], gxy = a.g[plane + row + i], gyy = a.g[2 * plane + row + i];
    const double2 mx = to_d(sp[((size_t)m * 4 + 0) * plane + row + i]);
    const double2 my = to_d(sp[((size_t)m * 4 + 1) * plane + row + i]);
    vx[u] = cfma(cmul(mx, gxx), my, gxy);
    vy[u] = cfma(cmul(mx, gxy), my, gyy);
  }
  if (a.parabolic) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = I0 + threadIdx.x + THREADS * u;
      const double2 wc = contour_weight(a, a.kx0 + i * a.dkx, a.ky0 + n2 * a.dky);
      vx[u] = cmul(vx[u], wc);
      vy[u] = cmul(vy[u], wc);
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = I0 + threadIdx.x + THREADS * u;
    ax[i] = (i & 1) ? make_double2(-vx[u].x, -vx[u].y) : vx[u];
    ay[i] = (i & 1) ? make_double2(-vy[u].x, -vy[u].y) : vy[u];
  }
}

// Integrand samples H = A_x Mx#_n + A_y My#_n of the R points of thread t
// (zero for an inactive transform slot, whose loads stay in the plane of
// pair 0).  On a zero-padded grid only the points R/4 <= r < 3R/4 lie in
// the band (n1 = t + T r, T = N/R) and are loaded.
template <bool BAND, typename Vs, typename Vc, int N, int R>
__device__ __forceinline__ void grouped_inputs(const Vs* sp, int n, size_t row, size_t plane, int t, bool active,
                                               const double2* ax, const double2* ay, Vc (&f)[R]) {
  constexpr int T = N / R;
  auto live = [](int r) { return !BAND || (4 * r >= R && 4 * r < 3 * R); };
  const Vs* spn = sp + ((size_t)n * 4 + 2) * plane + row;
  double2 mxh[R], myh[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!live(r)) continue;
    mxh[r] = to_d(spn[t + T * r]);
    myh[r] = to_d(spn[plane + t + T * r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int n1 = t + T * r;
    f[r] = from_d<Vc>(live(r) && active ? cfma(cmul(ax[n1], mxh[r]), ay[n1], myh[r]) : make_double2(0.0, 0.0));
  }
}

// The grouped row pass asks for the row pass's occupancy, except that the
// two-pair blocks of FP32 rows of 1024 points settle for 3 waves per SIMD
// (their A tables take the registers 4 waves would need).
template <typename Vc, int N, int NPW> constexpr int rowg_min_waves() {
  return (NPW == 2 && row_min_waves<Vc, N>() == 4) ? 3 : row_min_waves<Vc, N>();
}

template <typename Vs, typename Vc, int N, int NPW>
__global__ void __launch_bounds__(NPW * (N / 8), (rowg_min_waves<Vc, N, NPW>())) row_pass_grouped_kernel(RowGArgs a) {
  using Cfg = RowGCfg<N, NPW>;
  constexpr int T = Cfg::T, R = Cfg::R;
  using Rc = typename real_of<Vc>::type;
  __shared__ double2 ax[N], ay[N];
  __shared__ Vc lds[NPW * lds_len<row_pad<Vc>()>(N)];
  __shared__ Vc ltw[TwLds<N>::LEN];
  load_twiddles<Vc, N>(ltw, (const Vc*)a.tw, threadIdx.x, Cfg::THREADS);
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int grp = lid % a.ngroups;
  const int n2 = lid / a.ngroups + (a.band ? a.ny / 4 : 0);   // zero-padded grid: band rows only
  const int w = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const size_t plane = (size_t)a.nx * a.ny;
  const int m = a.gm[grp];
  const size_t row = (size_t)n2 * N;
  const Vs* sp = (const Vs*)a.spec;
  if (a.band) grouped_a_tables<true, Vs, N, Cfg::THREADS>(a, m, n2, row, plane, ax, ay);
  else grouped_a_tables<false, Vs, N, Cfg::THREADS>(a, m, n2, row, plane, ax, ay);
  __syncthreads();   // A tables and twiddle tables ready
  const bool active = w < a.gcnt[grp];
  if constexpr (T <= 64) {
    if (!active) return;   // transforms are wave-local: nothing left to wait for
  }
  const int pair = active ? a.gpair[a.gfirst[grp] + w] : 0;
  const int n = a.pn[pair];
  Vc f[R];
  if (a.band) grouped_inputs<true, Vs, Vc, N, R>(sp, n, row, plane, t, active, ax, ay, f);
  else grouped_inputs<false, Vs, Vc, N, R>(sp, n, row, plane, t, active, ax, ay, f);
  Vc* my_lds = lds + w * lds_len<row_pad<Vc>()>(N);
  Vs* inter = (Vs*)a.inter;
  if (a.parabolic) {
    row_terms_general<Vs, Vc, N, R, (T <= 64), row_pad<Vc>()>(
        a, f, my_lds, ltw, t, n2, inter + ((size_t)pair * (a.order + 1) * a.ny + n2) * N, (size_t)a.ny * N, active);
    return;
  }
  double2 S[R];
#pragma unroll
  for (int r = 0; r < R; ++r) S[r] = make_double2(0.0, 0.0);
  for (int ao = 0; ao <= a.order; ++ao) {
    int tb = t;
    if constexpr (row_opaque_t<Vc, N>()) asm volatile("" : "+v"(tb));
    if (ao > 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n1 = tb + T * r;
        f[r] = cscale(f[r], (Rc)(a.gamma * (a.kx0 + n1 * a.dkx)));
      }
    }
    Vc x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = f[r];
    fft_forward<Vc, N, R, (T <= 64), row_pad<Vc>()>(x, my_lds, ltw, t);
    const bool keep = !a.tensor || ao == a.order;
    const int nsl = a.tensor ? 1 : a.order + 1;
    Vs* dst = inter + (((size_t)pair * nsl + (a.tensor ? 0 : ao)) * a.ny + n2) * N;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double dx = a.x0 + (tb + T * r) * a.ddx;
      double cf = 1.0;
      for (int i = 1; i <= ao; ++i) cf *= dx * a.rinv[i];
      const double2 xv = to_d(x[r]);
      S[r] = make_double2(S[r].x + cf * xv.x, S[r].y + cf * xv.y);
      if (active && keep) {
        if (a.stream_out) store_nt(dst + tb + T * r, from_d<Vs>(S[r]));
        else dst[tb + T * r] = from_d<Vs>(S[r]);
      }
    }
  }
}

struct ColArgs {
  int tensor;   // every term reads slot 0 (the full row sum S_P)
  int parabolic;   // term b reads slot b and carries no (gamma ky)^b factor
  int band;     // x2 zero-padded grid: rows outside [N/4, 3N/4) are zero and not read
  int tile;     // kColTile*: the default tile or one of the autotuner's alternatives
  const void* inter;   // Vs elements
  void* z;             // Vs elements
  const void* tw;      // Vc elements
  int nx, ny, order, npairs;
  double ky0, dky, y0, ddy, gamma;
  double2 scale;   // K sigma W
  double rinv[kMaxOrder + 1];
};

// Column-pass tile: C adjacent columns per block and R points per thread of
// each column transform.  The widest C that keeps a block within 64-byte row
// pieces, its LDS budget (80 KiB: two blocks per CU; 152 KiB with more than
// 8 points per thread: one block) and 512 threads (1024 for FP32 transforms
// of 2048 points and more).  RF != 0 imposes R (the autotuner's alternative
// number of points per thread).
template <typename Vs, typename Vc, int N, int RF = 0> struct ColShape {
  static constexpr int lds_per_col() { return (lds_len(N) + 4) * (int)sizeof(Vc); }
  // FP64 transforms of 4096 points: two-column tiles of 8 points per thread
  // (1024 threads, one block per CU).  Measured on the 4096^2 table against
  // one-column tiles of 8 or 16 points per thread and two-column tiles of 16,
  // each with and without loading the next term during the transform, it
  // was the fastest in both storage precisions (one-column tiles move 16-byte
  // row pieces; 16 points per thread leave one wave per SIMD).
  static constexpr bool wide4096 = sizeof(Vc) == 16 && N >= 4096;
  static constexpr int R_DEFAULT = wide4096 ? 8 : (sizeof(Vc) == 8 && N >= 4096) ? 16 : 8;
  static constexpr int R = RF ? RF : R_DEFAULT;
  // the other number of points per thread, offered for columns of 1024
  // points and more
  static constexpr int R_ALT = R_DEFAULT == 8 ? 16 : 8;
  static constexpr int pick_c() {
    if (wide4096 && R == 8) return 2;
    int c = 64 / (int)sizeof(Vs);
    const int max_threads = (sizeof(Vc) == 8 && N >= 2048 && R == 8) ? 1024 : 512;
    const int cap = R > 8 ? 155648 : 81920;
    while (c > 1 && (c * lds_per_col() > cap || c * (N / R) > max_threads)) c /= 2;
    return c;
  }
  static constexpr int C = pick_c();
};

// Minimum waves per SIMD requested for the column pass (1: no constraint).
// Tiles of more than 8 points per thread fill a CU's LDS with one block, so
// they take the register budget of that block; the FP32 transforms of 8
// points take 4 waves per SIMD (two 512-thread blocks per CU) at the price
// of a small spill (-17% at 512^2).
template <typename Vc, int R> constexpr int col_min_waves() { return (sizeof(Vc) == 8 && R == 8) ? 4 : 1; }

template <int N, int C, int R> struct ColCfg {
  static constexpr int T = N / R;
  static constexpr int THREADS = C * T;
  static constexpr int LDP = lds_len(N) + 4;
};

// Column-pass block.  Thread tid works on column c = tid % C of the tile at
// transform position t = tid / C, holding R points at stride T = N/R.  A
// wave therefore covers 64/C consecutive rows of all C columns, so every
// global load and store moves whole C-column row segments straight between
// HBM and registers; LDS is used only for the FFT exchanges (one region of
// LDP entries per column).
template <typename Vs, typename Vc, int N, int C, int R>
__global__ void __launch_bounds__(C * (N / R), (col_min_waves<Vc, R>())) col_pass_kernel(ColArgs a) {
  using Cfg = ColCfg<N, C, R>;
  constexpr int T = Cfg::T, LDP = Cfg::LDP;
  using Rc = typename real_of<Vc>::type;
  __shared__ Vc lds[C * LDP];
  __shared__ Vc ltw[TwLds<N>::LEN];
  load_twiddles<Vc, N>(ltw, (const Vc*)a.tw, threadIdx.x, Cfg::THREADS);
  const int ntile = a.nx / C;
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = lid % ntile;
  const int pair = lid / ntile;
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const int j1 = tile * C + c;
  const size_t plane = (size_t)N * a.nx;
  const int nsl = a.tensor ? 1 : a.order + 1;
  const Vs* col0 = (const Vs*)a.inter + (size_t)pair * nsl * plane + j1;

  double2 Z[R];
#pragma unroll
  for (int r = 0; r < R; ++r) Z[r] = make_double2(0.0, 0.0);
  // Term b reads S_{P-b} (total degree), S'_b (parabolic) or S_P (tensor).
  // n2 = t + T r lies in the band [N/4, 3N/4) of a zero-padded grid exactly
  // when 2R/8 <= r < 6R/8; outside it the intermediates are zero (never
  // written by the row pass) and are not read.
  auto load_term = [&](Vs(&dst)[R], int b, int tt) {
    const Vs* src = col0 + (size_t)(a.tensor ? 0 : a.parabolic ? b : a.order - b) * plane;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (a.band && (8 * r < 2 * R || 8 * r >= 6 * R)) dst[r] = from_d<Vs>(make_double2(0.0, 0.0));
      else dst[r] = src[(size_t)(tt + T * r) * a.nx];
    }
  };
  Vs nxt[R];
  Vc* my_lds = lds + c * LDP;
  __syncthreads();   // twiddle tables ready
  for (int b = 0; b <= a.order; ++b) {
    // an opaque copy of t keeps the per-point weights and addresses inside
    // the term loop (hoisted, they would stay live in registers across it)
    int tb = t;
    asm volatile("" : "+v"(tb));
    load_term(nxt, b, tb);
    Vc x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // s(n2) (gamma ky)^b, rebuilt per term (a few multiplies)
      const int n2 = tb + T * r;
      double w = (n2 & 1) ? -1.0 : 1.0;
      if (!a.parabolic) {
        const double gk = a.gamma * (a.ky0 + n2 * a.dky);
        for (int i = 0; i < b; ++i) w *= gk;
      }
      x[r] = cscale(from_d<Vc>(to_d(nxt[r])), (Rc)w);
    }
    fft_forward<Vc, N, R>(x, my_lds, ltw, t);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j2 = tb + T * r;
      const double dy = a.y0 + j2 * a.ddy;
      double cf = 1.0;
      for (int i = 1; i <= b; ++i) cf *= dy * a.rinv[i];
      const double2 xv = to_d(x[r]);
      Z[r].x += cf * xv.x;
      Z[r].y += cf * xv.y;
    }
  }
  Vs* dst = (Vs*)a.z + (size_t)pair * plane + j1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j2 = t + T * r;
    double2 v = cmul(Z[r], a.scale);
    if ((j1 + j2) & 1) v = make_double2(-v.x, -v.y);
    // streaming stores for whole 64-byte row pieces; narrower tiles store
    // through the cache, where the neighbouring tiles' pieces complete a
    // line before it is written back (streaming 16-32 byte pieces out one
    // by one cost 40% more time at 4096^2)
    if constexpr (C * sizeof(Vs) >= 64) store_nt(dst + (size_t)j2 * a.nx, from_d<Vs>(v));
    else dst[(size_t)j2 * a.nx] = from_d<Vs>(v);
  }
}

// ------------------------------------------------ dispatch over sizes
static void fill_rinv(double* r) {
  r[0] = 1.0;
  for (int i = 1; i <= kMaxOrder; ++i) r[i] = 1.0 / i;
}

template <typename Vs, typename Vc, int N>
static hipError_t row_launch(const RowArgs& args, hipStream_t s) {
  constexpr int R = row_r<Vc, N>();
  using Cfg = RowCfg<N, R>;
  const int rows = args.band ? args.ny / 2 : args.ny;
  const int nblk = ((rows + Cfg::ROWS - 1) / Cfg::ROWS) * args.npairs;
  int grid = nblk;
  if constexpr (row_persistent<Vs, Vc, N>()) {
    // blocks resident at once on this device, in multiples of 8 (XCDs)
    static thread_local int cached_dev = -1, cached_resident = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != cached_dev) {
      int per_cu = 0, cus = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, row_pass_kernel<Vs, Vc, N, R>, Cfg::THREADS, 0);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      cached_resident = std::max(8, per_cu * cus / 8 * 8);
      cached_dev = dev;
    }
    grid = std::min(nblk, cached_resident);
  }
  hipLaunchKernelGGL((row_pass_kernel<Vs, Vc, N, R>), dim3(grid), dim3(Cfg::THREADS), 0, s, args);
  return hipGetLastError();
}

template <typename Vs, typename Vc, int N, int C, int R>
static hipError_t col_launch_tile(const ColArgs& args, hipStream_t s) {
  if (args.nx % C != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((col_pass_kernel<Vs, Vc, N, C, R>), dim3((args.nx / C) * args.npairs),
                     dim3(ColCfg<N, C, R>::THREADS), 0, s, args);
  return hipGetLastError();
}

template <typename Vs, typename Vc, int N>
static hipError_t col_launch(const ColArgs& args, hipStream_t s) {
  using Sh = ColShape<Vs, Vc, N>;
  constexpr int C0 = Sh::C, R = Sh::R;
  // the autotuner's alternatives: tiles of half the width (more, smaller
  // blocks; shorter row pieces), or, for columns of 1024 points and more,
  // the other number of points per thread with its own widest tile
  if constexpr (C0 > 1) {
    if (args.tile == kColTileHalf) return col_launch_tile<Vs, Vc, N, C0 / 2, R>(args, s);
  }
  if constexpr (N >= 1024) {
    using Alt = ColShape<Vs, Vc, N, Sh::R_ALT>;
    if (args.tile == kColTileAltR) return col_launch_tile<Vs, Vc, N, Alt::C, Alt::R>(args, s);
  }
  return col_launch_tile<Vs, Vc, N, C0, R>(args, s);
}

#define CFFT_SIZE_SWITCH(n, F, ...)      \
  switch (n) {                           \
    case 16: return F<16>(__VA_ARGS__);     \
    case 32: return F<32>(__VA_ARGS__);     \
    case 64: return F<64>(__VA_ARGS__);     \
    case 128: return F<128>(__VA_ARGS__);   \
    case 256: return F<256>(__VA_ARGS__);   \
    case 512: return F<512>(__VA_ARGS__);   \
    case 1024: return F<1024>(__VA_ARGS__); \
    case 2048: return F<2048>(__VA_ARGS__); \
    case 4096: return F<4096>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;   \
  }

// Grouped launch: pairs are grouped by testing MBF into groups of <= NPW
// (4 when every MBF's pair count is a multiple of 4, else 2).
template <typename Vs, typename Vc, int N>
static hipError_t rowg_launch(const RowArgs& ra, hipStream_t s) {
  RowGArgs a;
  a.g = ra.g;
  a.spec = ra.spec;
  a.inter = ra.inter;
  a.tw = ra.tw;
  a.nx = ra.nx;
  a.ny = ra.ny;
  a.order = ra.order;
  a.tensor = ra.tensor;
  a.stream_out = ra.stream_out;
  a.band = ra.band;
  a.parabolic = ra.parabolic;
  a.ky0 = ra.ky0;
  a.dky = ra.dky;
  a.beta_end = ra.beta_end;
  a.kx0 = ra.kx0;
  a.dkx = ra.dkx;
  a.x0 = ra.x0;
  a.ddx = ra.ddx;
  a.gamma = ra.gamma;
  for (int i = 0; i <= kMaxOrder; ++i) a.rinv[i] = ra.rinv[i];
  for (int i = 0; i < kMaxPairsPerLaunch; ++i) a.pn[i] = ra.pn[i];
  // pair indices per testing MBF, in list order
  std::map<int, std::vector<int>> by_m;
  std::vector<int> order_m;
  for (int i = 0; i < ra.npairs; ++i) {
    if (!by_m.count(ra.pm[i])) order_m.push_back(ra.pm[i]);
    by_m[ra.pm[i]].push_back(i);
  }
  bool all4 = true;
  for (auto& kv : by_m) all4 = all4 && (kv.second.size() % 4 == 0);
  const int npw = all4 ? 4 : 2;
  int ng = 0, slot = 0;
  for (int m : order_m) {
    const auto& v = by_m[m];
    for (size_t j = 0; j < v.size(); j += npw) {
      a.gm[ng] = m;
      a.gfirst[ng] = slot;
      a.gcnt[ng] = (int)std::min<size_t>(npw, v.size() - j);
      for (int k = 0; k < a.gcnt[ng]; ++k) a.gpair[slot++] = v[j + k];
      ++ng;
    }
  }
  for (int i = ng; i < kMaxPairsPerLaunch; ++i) a.gm[i] = a.gfirst[i] = a.gcnt[i] = 0;
  for (int i = slot; i < kMaxPairsPerLaunch; ++i) a.gpair[i] = 0;
  a.ngroups = ng;
  const int nblk = ng * (ra.band ? ra.ny / 2 : ra.ny);
  if (npw == 4) {
    hipLaunchKernelGGL((row_pass_grouped_kernel<Vs, Vc, N, 4>), dim3(nblk), dim3(RowGCfg<N, 4>::THREADS), 0, s, a);
  } else {
    hipLaunchKernelGGL((row_pass_grouped_kernel<Vs, Vc, N, 2>), dim3(nblk), dim3(RowGCfg<N, 2>::THREADS), 0, s, a);
  }
  return hipGetLastError();
}

template <typename Vs, typename Vc, int N> static hipError_t row_any(const RowArgs& a, hipStream_t s) {
  if constexpr (N >= 128 && N <= 1024) return rowg_launch<Vs, Vc, N>(a, s);
  else return row_launch<Vs, Vc, N>(a, s);
}
template <int N> static hipError_t row_fp64(const RowArgs& a, hipStream_t s) { return row_any<double2, double2, N>(a, s); }
template <int N> static hipError_t row_fp32(const RowArgs& a, hipStream_t s) { return row_any<float2, float2, N>(a, s); }
template <int N> static hipError_t row_fp32_hi(const RowArgs& a, hipStream_t s) {
  return row_any<float2, double2, N>(a, s);
}
template <int N> static hipError_t col_fp64(const ColArgs& a, hipStream_t s) {
  return col_launch<double2, double2, N>(a, s);
}
template <int N> static hipError_t col_fp32(const ColArgs& a, hipStream_t s) {
  return col_launch<float2, float2, N>(a, s);
}
template <int N> static hipError_t col_fp32_hi(const ColArgs& a, hipStream_t s) {
  return col_launch<float2, double2, N>(a, s);
}

hipError_t launch_row_pass(const PassParams& p, const double2* g, const void* spec, const int* pm,
                           const int* pn, int npairs, void* inter, const void* twx, hipStream_t s) {
  if (npairs < 1 || npairs > kMaxPairsPerLaunch) return hipErrorInvalidValue;
  RowArgs a;
  a.g = g;
  a.spec = spec;
  a.inter = inter;
  a.tw = twx;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.order = p.order;
  a.tensor = p.tensor;
  a.stream_out = p.stream_out;
  a.band = p.band;
  a.parabolic = p.parabolic;
  a.ky0 = p.y.k_first;
  a.dky = p.y.dk;
  a.beta_end = p.beta_end;
  a.npairs = npairs;
  a.kx0 = p.x.k_first;
  a.dkx = p.x.dk;
  a.x0 = p.x.d_first;
  a.ddx = p.x.dd;
  a.gamma = p.gamma;
  fill_rinv(a.rinv);
  for (int i = 0; i < kMaxPairsPerLaunch; ++i) {
    a.pm[i] = i < npairs ? pm[i] : 0;
    a.pn[i] = i < npairs ? pn[i] : 0;
  }
  if (p.precision == 0) {
    CFFT_SIZE_SWITCH(p.x.n, row_fp64, a, s)
  }
  if (p.hi_compute) {
    CFFT_SIZE_SWITCH(p.x.n, row_fp32_hi, a, s)
  }
  CFFT_SIZE_SWITCH(p.x.n, row_fp32, a, s)
}

static double2 table_scale(const PassParams& p) {
  const double K = p.x.dk * p.y.dk / (4.0 * M_PI * M_PI);
  const int half = (p.x.n + p.y.n) / 2;
  const double sigma = (half & 1) ? -1.0 : 1.0;
  // ray: W = (1 + i gamma)^2 is constant and applied here; parabolic: W
  // varies per sample and the row pass has applied it
  if (p.parabolic) return make_double2(K * sigma, 0.0);
  const double wr = 1.0 - p.gamma * p.gamma, wi = 2.0 * p.gamma;
  return make_double2(K * sigma * wr, K * sigma * wi);
}

hipError_t launch_col_pass(const PassParams& p, const void* inter, int npairs, void* z, const void* twy,
                           hipStream_t s) {
  ColArgs a;
  a.inter = inter;
  a.z = z;
  a.tw = twy;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.order = p.order;
  a.tensor = p.tensor;
  a.parabolic = p.parabolic;
  a.band = p.band;
  a.tile = p.col_tile;
  a.npairs = npairs;
  a.ky0 = p.y.k_first;
  a.dky = p.y.dk;
  a.y0 = p.y.d_first;
  a.ddy = p.y.dd;
  a.gamma = p.gamma;
  a.scale = table_scale(p);
  fill_rinv(a.rinv);
  if (p.precision == 0) {
    CFFT_SIZE_SWITCH(p.y.n, col_fp64, a, s)
  }
  if (p.hi_compute) {
    CFFT_SIZE_SWITCH(p.y.n, col_fp32_hi, a, s)
  }
  CFFT_SIZE_SWITCH(p.y.n, col_fp32, a, s)
}

// ------------------------------------------------ adjoint passes (FP64)
// With h = conj(K sigma W) s(j1+j2) gZ, the adjoint of the table map is
//   U_b(j1,n2) = IDFT_j2[ Dy^b/b! h ](n2),  V_c = sum_{b<=c} (gamma ky)^b U_b
//   gH(n1,n2)  = s(n1+n2) sum_a (gamma kx)^a IDFT_j1[ Dx^a/a! V_{P-a} ](n1)
// (unnormalised inverse DFTs; all weights are real).  Tensor truncation:
// V_{P-a} is replaced by V_P for every a, so only V_P is stored.
struct AdjColArgs {
  int tensor;   // only the full sum V_P is stored, in slot 0
  const double2* dz;
  double2* inter;
  const double2* tw;
  int nx, ny, order, npairs;
  double ky0, dky, y0, ddy, gamma;
  double2 cscale;  // conj(K sigma W)
  double rinv[kMaxOrder + 1];
};

// Adjoint column tile: FP64, 8 points per thread, up to four columns (64-byte
// row pieces) within 80 KiB of LDS and 512 threads.
template <int N> constexpr int adj_col_tile() {
  int c = 4;
  while (c > 1 && (c * (lds_len(N) + 4) * 16 > 81920 || c * (N / 8) > 512)) c /= 2;
  return c;
}

template <int N, int C>
__global__ void __launch_bounds__(C * (N / 8)) adj_col_kernel(AdjColArgs a) {
  constexpr int R = 8;
  using Cfg = ColCfg<N, C, R>;
  constexpr int T = Cfg::T, LDP = Cfg::LDP;
  __shared__ double2 lds[C * LDP];
  __shared__ double2 ltw[TwLds<N>::LEN];
  load_twiddles<double2, N>(ltw, a.tw, threadIdx.x, Cfg::THREADS);
  const int ntile = a.nx / C;
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = lid % ntile;
  const int pair = lid / ntile;
  const int c = threadIdx.x % C;
  const int t = threadIdx.x / C;
  const int j1 = tile * C + c;
  const size_t plane = (size_t)N * a.nx;
  const double2* src = a.dz + (size_t)pair * plane + j1;
  double2 h0[R], acc[R];
  double cf[R], pw[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j2 = t + T * r;
    double2 v = cmul(src[(size_t)j2 * a.nx], a.cscale);
    if ((j1 + j2) & 1) v = make_double2(-v.x, -v.y);
    h0[r] = v;
    acc[r] = make_double2(0.0, 0.0);
    cf[r] = 1.0;
    pw[r] = 1.0;
  }
  double2* my_lds = lds + c * LDP;
  __syncthreads();   // twiddle tables ready
  for (int b = 0; b <= a.order; ++b) {
    double2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j2 = t + T * r;
      if (b > 0) cf[r] *= (a.y0 + j2 * a.ddy) * a.rinv[b];
      x[r] = cscale(h0[r], cf[r]);
    }
    fft_inverse<double2, N, R>(x, my_lds, ltw, t);
    const bool keep = !a.tensor || b == a.order;
    const int nsl = a.tensor ? 1 : a.order + 1;
    double2* dst = a.inter + ((size_t)pair * nsl + (a.tensor ? 0 : b)) * plane + j1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n2 = t + T * r;
      if (b > 0) pw[r] *= a.gamma * (a.ky0 + n2 * a.dky);
      acc[r] = cadd(acc[r], cscale(x[r], pw[r]));
      if (keep) dst[(size_t)n2 * a.nx] = acc[r];
    }
  }
}

struct AdjRowArgs {
  int tensor;
  const double2* inter;
  double2* gi;
  const double2* tw;
  int nx, ny, order, npairs;
  double kx0, dkx, x0, ddx, gamma;
  double rinv[kMaxOrder + 1];
};

template <int N>
__global__ void __launch_bounds__((RowCfg<N, 8>::THREADS)) adj_row_kernel(AdjRowArgs a) {
  using Cfg = RowCfg<N, 8>;
  constexpr int T = Cfg::T, R = 8, ROWS = Cfg::ROWS;
  __shared__ double2 lds[ROWS * lds_len<row_pad<double2>()>(N)];
  __shared__ double2 ltw[TwLds<N>::LEN];
  load_twiddles<double2, N>(ltw, a.tw, threadIdx.x, Cfg::THREADS);
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int pair = lid % a.npairs;
  const int rb = lid / a.npairs;
  const int grp = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int n2 = rb * ROWS + grp;
  const bool valid = n2 < a.ny;
  double2 acc[R];
  double cf[R], pw[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    acc[r] = make_double2(0.0, 0.0);
    cf[r] = 1.0;
    pw[r] = 1.0;
  }
  double2* my_lds = lds + grp * lds_len<row_pad<double2>()>(N);
  __syncthreads();   // twiddle tables ready
  for (int ao = 0; ao <= a.order; ++ao) {
    const int nsl = a.tensor ? 1 : a.order + 1;
    const double2* src =
        a.inter + (((size_t)pair * nsl + (a.tensor ? 0 : a.order - ao)) * a.ny + (valid ? n2 : 0)) * N;
    double2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j1 = t + T * r;
      if (ao > 0) cf[r] *= (a.x0 + j1 * a.ddx) * a.rinv[ao];
      x[r] = valid ? cscale(src[j1], cf[r]) : make_double2(0.0, 0.0);
    }
    fft_inverse<double2, N, R, (T <= 64), row_pad<double2>()>(x, my_lds, ltw, t);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n1 = t + T * r;
      if (ao > 0) pw[r] *= a.gamma * (a.kx0 + n1 * a.dkx);
      acc[r] = cadd(acc[r], cscale(x[r], pw[r]));
    }
  }
  if (!valid) return;
  double2* dst = a.gi + ((size_t)pair * a.ny + n2) * N;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int n1 = t + T * r;
    double2 v = acc[r];
    if ((n1 + n2) & 1) v = make_double2(-v.x, -v.y);
    dst[n1] = v;
  }
}

template <int N>
static hipError_t adj_col_launch(const AdjColArgs& args, hipStream_t s) {
  constexpr int C = adj_col_tile<N>();
  using Cfg = ColCfg<N, C, 8>;
  if (args.nx % C != 0) return hipErrorInvalidValue;
  const int nblk = (args.nx / C) * args.npairs;
  hipLaunchKernelGGL((adj_col_kernel<N, C>), dim3(nblk), dim3(Cfg::THREADS), 0, s, args);
  return hipGetLastError();
}

template <int N>
static hipError_t adj_row_launch(const AdjRowArgs& args, hipStream_t s) {
  using Cfg = RowCfg<N, 8>;
  const int nblk = ((args.ny + Cfg::ROWS - 1) / Cfg::ROWS) * args.npairs;
  hipLaunchKernelGGL((adj_row_kernel<N>), dim3(nblk), dim3(Cfg::THREADS), 0, s, args);
  return hipGetLastError();
}

hipError_t launch_adj_col_pass(const PassParams& p, const double2* dz, int npairs, double2* inter,
                               const void* twy, hipStream_t s) {
  AdjColArgs a;
  a.dz = dz;
  a.inter = inter;
  a.tw = (const double2*)twy;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.order = p.order;
  a.tensor = p.tensor;
  a.npairs = npairs;
  a.ky0 = p.y.k_first;
  a.dky = p.y.dk;
  a.y0 = p.y.d_first;
  a.ddy = p.y.dd;
  a.gamma = p.gamma;
  const double2 sc = table_scale(p);
  a.cscale = make_double2(sc.x, -sc.y);
  fill_rinv(a.rinv);
  CFFT_SIZE_SWITCH(p.y.n, adj_col_launch, a, s)
}

hipError_t launch_adj_row_pass(const PassParams& p, const double2* inter, int npairs, double2* gi,
                               const void* twx, hipStream_t s) {
  AdjRowArgs a;
  a.inter = inter;
  a.gi = gi;
  a.tw = (const double2*)twx;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.order = p.order;
  a.tensor = p.tensor;
  a.npairs = npairs;
  a.kx0 = p.x.k_first;
  a.dkx = p.x.dk;
  a.x0 = p.x.d_first;
  a.ddx = p.x.dd;
  a.gamma = p.gamma;
  fill_rinv(a.rinv);
  CFFT_SIZE_SWITCH(p.x.n, adj_row_launch, a, s)
}

// ------------------------------------------------ integrand adjoint
// For every sample, with gH_p the gradient w.r.t. H of pair p = (m, n):
//   gG_xx += gH conj(Mx_m Mx#_n), gG_xy += gH conj(Mx_m My#_n + My_m Mx#_n),
//   gG_yy += gH conj(My_m My#_n),
//   gMx_m += gH conj(Gxx Mx#_n + Gxy My#_n), gMy_m += gH conj(Gxy Mx#_n + Gyy My#_n),
//   gMx#_n += gH conj(Mx_m Gxx + My_m Gxy),  gMy#_n += gH conj(Mx_m Gxy + My_m Gyy).
struct AdjIntArgs {
  const double2* gi;
  const double2* g;
  const double2* spec;
  double2* gg;
  double2* gspec;
  int n, npairs, nmbf, accumulate;
  int nx, ny, band;   // zero-padded grid: samples outside the band carry no integrand
  int pm[kMaxPairsPerLaunch];
  int pn[kMaxPairsPerLaunch];
};

__global__ void __launch_bounds__(256) adj_integrand_kernel(AdjIntArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.n) return;
  // the forward zeroes the integrand outside the band of a zero-padded grid,
  // so nothing flows back to the Green's function or spectra there
  const bool silent = a.band && !(in_band(idx % a.nx, a.nx) && in_band(idx / a.nx, a.ny));
  const size_t plane = (size_t)a.n;
  const double2 gxx = a.g[idx], gxy = a.g[plane + idx], gyy = a.g[2 * plane + idx];
  double2 ggxx = make_double2(0.0, 0.0), ggxy = ggxx, ggyy = ggxx;
  if (a.accumulate) {
    ggxx = a.gg[idx];
    ggxy = a.gg[plane + idx];
    ggyy = a.gg[2 * plane + idx];
  }
  for (int mm = 0; mm < a.nmbf; ++mm) {
    // testing-side gradients of MBF mm and basis-side gradients of MBF mm
    double2 gmx = make_double2(0.0, 0.0), gmy = gmx, gmxh = gmx, gmyh = gmx;
    bool touched = false;
    const double2 mx = a.spec[((size_t)mm * 4 + 0) * plane + idx];
    const double2 my = a.spec[((size_t)mm * 4 + 1) * plane + idx];
    const double2 mxh_self = a.spec[((size_t)mm * 4 + 2) * plane + idx];
    const double2 myh_self = a.spec[((size_t)mm * 4 + 3) * plane + idx];
    for (int p = 0; p < (silent ? 0 : a.npairs); ++p) {
      const int m = a.pm[p], n = a.pn[p];
      if (m != mm && n != mm) continue;
      touched = true;
      const double2 gh = a.gi[(size_t)p * plane + idx];
      if (m == mm) {
        const double2 nxh = a.spec[((size_t)n * 4 + 2) * plane + idx];
        const double2 nyh = a.spec[((size_t)n * 4 + 3) * plane + idx];
        gmx = cadd(gmx, cmulc(gh, cadd(cmul(gxx, nxh), cmul(gxy, nyh))));
        gmy = cadd(gmy, cmulc(gh, cadd(cmul(gxy, nxh), cmul(gyy, nyh))));
        // Green's function gradient once per pair (on its testing MBF)
        ggxx = cadd(ggxx, cmulc(gh, cmul(mx, nxh)));
        ggxy = cadd(ggxy, cmulc(gh, cadd(cmul(mx, nyh), cmul(my, nxh))));
        ggyy = cadd(ggyy, cmulc(gh, cmul(my, nyh)));
      }
      if (n == mm) {
        const double2 tx = a.spec[((size_t)m * 4 + 0) * plane + idx];
        const double2 ty = a.spec[((size_t)m * 4 + 1) * plane + idx];
        gmxh = cadd(gmxh, cmulc(gh, cadd(cmul(tx, gxx), cmul(ty, gxy))));
        gmyh = cadd(gmyh, cmulc(gh, cadd(cmul(tx, gxy), cmul(ty, gyy))));
      }
    }
    (void)mxh_self;
    (void)myh_self;
    double2* gs = a.gspec + (size_t)mm * 4 * plane + idx;
    if (a.accumulate) {
      if (touched) {
        gs[0] = cadd(gs[0], gmx);
        gs[plane] = cadd(gs[plane], gmy);
        gs[2 * plane] = cadd(gs[2 * plane], gmxh);
        gs[3 * plane] = cadd(gs[3 * plane], gmyh);
      }
    } else {
      gs[0] = gmx;
      gs[plane] = gmy;
      gs[2 * plane] = gmxh;
      gs[3 * plane] = gmyh;
    }
  }
  a.gg[idx] = ggxx;
  a.gg[plane + idx] = ggxy;
  a.gg[2 * plane + idx] = ggyy;
}

// The same gradients for at most NM MBFs, with one pass over the pairs: the
// sample's spectra of every MBF and the gradient accumulators stay in
// registers (the MBF of a pair is wave-uniform, so selecting its registers
// costs unrolled uniform branches), and each pair's integrand gradient is
// read once.  The generic kernel above re-reads it and the spectra per MBF.
template <int NM>
__global__ void __launch_bounds__(256) adj_integrand_small_kernel(AdjIntArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.n) return;
  const bool silent = a.band && !(in_band(idx % a.nx, a.nx) && in_band(idx / a.nx, a.ny));
  const size_t plane = (size_t)a.n;
  const double2 zero = make_double2(0.0, 0.0);
  const double2 gxx = a.g[idx], gxy = a.g[plane + idx], gyy = a.g[2 * plane + idx];
  double2 ggxx = zero, ggxy = zero, ggyy = zero;
  if (a.accumulate) {
    ggxx = a.gg[idx];
    ggxy = a.gg[plane + idx];
    ggyy = a.gg[2 * plane + idx];
  }
  double2 sx[NM], sy[NM], sxh[NM], syh[NM], gmx[NM], gmy[NM], gmxh[NM], gmyh[NM];
#pragma unroll
  for (int mm = 0; mm < NM; ++mm) {
    gmx[mm] = gmy[mm] = gmxh[mm] = gmyh[mm] = zero;
    sx[mm] = sy[mm] = sxh[mm] = syh[mm] = zero;
    if (mm < a.nmbf && !silent) {
      const double2* sp = a.spec + (size_t)mm * 4 * plane + idx;
      sx[mm] = sp[0];
      sy[mm] = sp[plane];
      sxh[mm] = sp[2 * plane];
      syh[mm] = sp[3 * plane];
    }
  }
  for (int p = 0; p < (silent ? 0 : a.npairs); ++p) {
    const int m = a.pm[p], n = a.pn[p];
    const double2 gh = a.gi[(size_t)p * plane + idx];
    double2 mx = zero, my = zero, nxh = zero, nyh = zero;
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) {
      if (mm == m) {
        mx = sx[mm];
        my = sy[mm];
      }
      if (mm == n) {
        nxh = sxh[mm];
        nyh = syh[mm];
      }
    }
    const double2 cx = cmulc(gh, cadd(cmul(gxx, nxh), cmul(gxy, nyh)));
    const double2 cy = cmulc(gh, cadd(cmul(gxy, nxh), cmul(gyy, nyh)));
    const double2 chx = cmulc(gh, cadd(cmul(mx, gxx), cmul(my, gxy)));
    const double2 chy = cmulc(gh, cadd(cmul(mx, gxy), cmul(my, gyy)));
    ggxx = cadd(ggxx, cmulc(gh, cmul(mx, nxh)));
    ggxy = cadd(ggxy, cmulc(gh, cadd(cmul(mx, nyh), cmul(my, nxh))));
    ggyy = cadd(ggyy, cmulc(gh, cmul(my, nyh)));
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) {
      if (mm == m) {
        gmx[mm] = cadd(gmx[mm], cx);
        gmy[mm] = cadd(gmy[mm], cy);
      }
      if (mm == n) {
        gmxh[mm] = cadd(gmxh[mm], chx);
        gmyh[mm] = cadd(gmyh[mm], chy);
      }
    }
  }
#pragma unroll
  for (int mm = 0; mm < NM; ++mm) {
    if (mm >= a.nmbf) break;
    double2* gs = a.gspec + (size_t)mm * 4 * plane + idx;
    if (a.accumulate) {
      bool touched = false;
      for (int p = 0; p < a.npairs; ++p) touched = touched || a.pm[p] == mm || a.pn[p] == mm;
      if (touched && !silent) {
        gs[0] = cadd(gs[0], gmx[mm]);
        gs[plane] = cadd(gs[plane], gmy[mm]);
        gs[2 * plane] = cadd(gs[2 * plane], gmxh[mm]);
        gs[3 * plane] = cadd(gs[3 * plane], gmyh[mm]);
      }
    } else {
      gs[0] = gmx[mm];
      gs[plane] = gmy[mm];
      gs[2 * plane] = gmxh[mm];
      gs[3 * plane] = gmyh[mm];
    }
  }
  a.gg[idx] = ggxx;
  a.gg[plane + idx] = ggxy;
  a.gg[2 * plane + idx] = ggyy;
}

hipError_t launch_adj_integrand(const PassParams& p, const double2* gi, const double2* g, const double2* spec,
                                const int* pm, const int* pn, int npairs, int nmbf, double2* gg, double2* gspec,
                                int accumulate, hipStream_t s) {
  if (npairs < 1 || npairs > kMaxPairsPerLaunch) return hipErrorInvalidValue;
  AdjIntArgs a;
  a.gi = gi;
  a.g = g;
  a.spec = spec;
  a.gg = gg;
  a.gspec = gspec;
  a.n = p.x.n * p.y.n;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.band = p.band;
  a.npairs = npairs;
  a.nmbf = nmbf;
  a.accumulate = accumulate;
  for (int i = 0; i < kMaxPairsPerLaunch; ++i) {
    a.pm[i] = i < npairs ? pm[i] : 0;
    a.pn[i] = i < npairs ? pn[i] : 0;
  }
  if (nmbf <= 4)
    hipLaunchKernelGGL(adj_integrand_small_kernel<4>, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(adj_integrand_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------ lookup
struct LookupArgs {
  const void* z;
  const double* pts;
  double2* out;
  int nx, ny, npairs, npts, precision;
  double x0, ddx, y0, ddy;
};

__device__ __forceinline__ bool cell_of(const LookupArgs& a, int q, int& j1, int& j2, double& tx, double& ty) {
  return cell_at((a.pts[2 * q] - a.x0) / a.ddx, (a.pts[2 * q + 1] - a.y0) / a.ddy, a.nx, a.ny, j1, j2, tx, ty);
}

__device__ __forceinline__ double2 table_at(const void* z, int precision, size_t i) {
  return precision == 0 ? ((const double2*)z)[i] : to_d(((const float2*)z)[i]);
}

// Bilinear value of one table plane (base = first entry of the plane).
__device__ __forceinline__ double2 bilinear_at(const void* z, int precision, size_t base, int nx, int j1, int j2,
                                               double tx, double ty) {
  const size_t i00 = base + (size_t)j2 * nx + j1;
  const double2 z00 = table_at(z, precision, i00), z01 = table_at(z, precision, i00 + 1);
  const double2 z10 = table_at(z, precision, i00 + nx), z11 = table_at(z, precision, i00 + nx + 1);
  const double w00 = (1 - tx) * (1 - ty), w01 = tx * (1 - ty), w10 = (1 - tx) * ty, w11 = tx * ty;
  return make_double2(w00 * z00.x + w01 * z01.x + w10 * z10.x + w11 * z11.x,
                      w00 * z00.y + w01 * z01.y + w10 * z10.y + w11 * z11.y);
}

__global__ void lookup_kernel(LookupArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.npairs * a.npts) return;
  const int p = e / a.npts, q = e % a.npts;
  int j1, j2;
  double tx, ty;
  if (!cell_of(a, q, j1, j2, tx, ty)) {
    a.out[e] = make_double2(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  a.out[e] = bilinear_at(a.z, a.precision, (size_t)p * a.nx * a.ny, a.nx, j1, j2, tx, ty);
}

__device__ __forceinline__ double2 quadratic_at(const void* z, int precision, size_t base, int nx, int c1, int c2,
                                                double tx, double ty) {
  double wx[3], wy[3];
  lagrange3(tx, wx);
  lagrange3(ty, wy);
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const size_t row = base + (size_t)(c2 + b - 1) * nx + (c1 - 1);
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 v = table_at(z, precision, row + i);
      s = make_double2(s.x + wx[i] * v.x, s.y + wx[i] * v.y);
    }
    acc = make_double2(acc.x + wy[b] * s.x, acc.y + wy[b] * s.y);
  }
  return acc;
}

__global__ void lookup_quadratic_kernel(LookupArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.npairs * a.npts) return;
  const int p = e / a.npts, q = e % a.npts;
  int c1, c2;
  double tx, ty;
  if (!stencil_at((a.pts[2 * q] - a.x0) / a.ddx, (a.pts[2 * q + 1] - a.y0) / a.ddy, a.nx, a.ny, c1, c2, tx, ty)) {
    a.out[e] = make_double2(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  a.out[e] = quadratic_at(a.z, a.precision, (size_t)p * a.nx * a.ny, a.nx, c1, c2, tx, ty);
}

// Reduced-matrix fill (Sec. II eq. MBF; Sec. III-B.1 and III-B.3): one
// block per matrix row r = i*M + m and 256 consecutive columns c = j*M + n,
// so the row segment is written with coalesced stores; each thread reads
// the table of pair (m, n) around D = r_i - r_j.  Self blocks (i == j) and
// unlisted (m, n) are not written.
struct FillArgs {
  const void* z;
  const double* pos;
  double2* out;
  int nx, ny, precision, nelem, nmbf, ncb;
  double x0, ddx, y0, ddy;
  short slot[kFillMaxMbf * kFillMaxMbf];   // pair index of (m, n), -1 when not listed
};

// Block = 256 consecutive columns of matrix row i M + m.  The blocks are
// ordered with the testing MBF m outermost and the element i next, and each
// XCD takes a contiguous range of them: the rows one XCD fills in turn then
// share most of their displacements r_i - r_j (a layout's displacements
// cluster), so the stencil lines of the M tables of one m stay in that
// XCD's L2 instead of coming from the memory-side cache for every row.
template <int ORDER>
__global__ __launch_bounds__(256) void fill_kernel(FillArgs a) {
  const int am = a.nelem * a.nmbf;
  const int lid = xcd_remap(blockIdx.x, gridDim.x);
  const int rr = lid / a.ncb;   // m * nelem + i
  const int c = (lid - rr * a.ncb) * 256 + threadIdx.x;
  if (c >= am) return;
  const int m = rr / a.nelem, i = rr - m * a.nelem;
  const int r = i * a.nmbf + m;
  const int j = c / a.nmbf, n = c - j * a.nmbf;
  if (i == j) return;
  const int p = a.slot[m * kFillMaxMbf + n];
  if (p < 0) return;
  const double ux = (a.pos[2 * i] - a.pos[2 * j] - a.x0) / a.ddx;
  const double uy = (a.pos[2 * i + 1] - a.pos[2 * j + 1] - a.y0) / a.ddy;
  const size_t base = (size_t)p * a.nx * a.ny;
  double2 v = make_double2(__builtin_nan(""), __builtin_nan(""));
  int c1, c2;
  double tx, ty;
  if (ORDER == 1) {
    if (cell_at(ux, uy, a.nx, a.ny, c1, c2, tx, ty)) v = bilinear_at(a.z, a.precision, base, a.nx, c1, c2, tx, ty);
  } else {
    if (stencil_at(ux, uy, a.nx, a.ny, c1, c2, tx, ty)) v = quadratic_at(a.z, a.precision, base, a.nx, c1, c2, tx, ty);
  }
  a.out[(size_t)r * am + c] = v;
}

hipError_t launch_fill(const PassParams& p, const void* z, const short* slot, int nmbf, const double* pos, int nelem,
                       int order, double2* out, hipStream_t s) {
  FillArgs a;
  a.z = z;
  a.pos = pos;
  a.out = out;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.precision = p.precision;
  a.nelem = nelem;
  a.nmbf = nmbf;
  const int am = nelem * nmbf;
  a.ncb = (am + 255) / 256;
  a.x0 = p.x.d_first;
  a.ddx = p.x.dd;
  a.y0 = p.y.d_first;
  a.ddy = p.y.dd;
  for (int k = 0; k < kFillMaxMbf * kFillMaxMbf; ++k) a.slot[k] = slot[k];
  const dim3 grid((unsigned)((long long)am * a.ncb));
  if (order == 1)
    hipLaunchKernelGGL(fill_kernel<1>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(fill_kernel<2>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

static LookupArgs lookup_args(const PassParams& p, const void* z, int npairs, const double* pts, int npts,
                              double2* out) {
  LookupArgs a;
  a.z = z;
  a.pts = pts;
  a.out = out;
  a.nx = p.x.n;
  a.ny = p.y.n;
  a.npairs = npairs;
  a.npts = npts;
  a.precision = p.precision;
  a.x0 = p.x.d_first;
  a.ddx = p.x.dd;
  a.y0 = p.y.d_first;
  a.ddy = p.y.dd;
  return a;
}

hipError_t launch_lookup(const PassParams& p, const void* z, int npairs, const double* pts, int npts, double2* out,
                         hipStream_t s) {
  const LookupArgs a = lookup_args(p, z, npairs, pts, npts, out);
  const long long n = (long long)npairs * npts;
  hipLaunchKernelGGL(lookup_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lookup_quadratic(const PassParams& p, const void* z, int npairs, const double* pts, int npts,
                                  double2* out, hipStream_t s) {
  const LookupArgs a = lookup_args(p, z, npairs, pts, npts, out);
  const long long n = (long long)npairs * npts;
  hipLaunchKernelGGL(lookup_quadratic_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace cfft
