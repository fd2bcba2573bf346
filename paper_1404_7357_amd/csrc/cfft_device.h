// Device-side building blocks for gfx950: complex arithmetic in FP64/FP32,
// the radiating square root, and an LDS-exchanged Stockham FFT whose
// butterflies run in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfft {

// ---------------------------------------------------------------- complex
template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };

template <typename V> struct real_of;
template <> struct real_of<double2> { using type = double; };
template <> struct real_of<float2> { using type = float; };

__device__ __forceinline__ double2 mk(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ float2 mk(float x, float y) { return make_float2(x, y); }

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return mk(a.x * s, a.y * s); }
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk(a.x, -a.y); }
// acc + a b with four fused multiply-adds
template <typename V> __device__ __forceinline__ V cfma(V acc, V a, V b) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// multiply by i, by -i
template <typename V> __device__ __forceinline__ V cmul_i(V a) { return mk(-a.y, a.x); }
template <typename V> __device__ __forceinline__ V cmul_mi(V a) { return mk(a.y, -a.x); }

__device__ __forceinline__ double2 to_d(double2 a) { return a; }
__device__ __forceinline__ double2 to_d(float2 a) { return make_double2(a.x, a.y); }
template <typename V> __device__ __forceinline__ V from_d(double2 a);
template <> __device__ __forceinline__ double2 from_d<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}

// Smith's division (no intermediate overflow for large operands).
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}

__device__ __forceinline__ double2 cexp(double2 z) {
  double s, c;
  sincos(z.y, &s, &c);
  const double e = exp(z.x);
  return make_double2(e * c, e * s);
}

// exp(z) - 1 without cancellation for small |z|.
__device__ __forceinline__ double2 cexpm1(double2 z) {
  double s, c;
  sincos(z.y, &s, &c);
  const double em1 = expm1(z.x);
  // Re: e^x cos y - 1 = (e^x - 1) cos y - 2 sin^2(y/2)
  const double sh = sin(0.5 * z.y);
  return make_double2(em1 * c - 2.0 * sh * sh, (em1 + 1.0) * s);
}

// Principal square root.
__device__ __forceinline__ double2 csqrt_principal(double2 z) {
  if (z.x == 0.0 && z.y == 0.0) return make_double2(0.0, z.y);
  const double r = hypot(z.x, z.y);
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

// Vertical wavenumber on the radiating branch: the root whose cut lies on the
// positive imaginary axis, i.e. arg in (-3pi/4, pi/4].  On the closed lower
// half plane (passive media, deformed contour) this is Im <= 0, Re >= 0 when
// propagating; elsewhere it continues analytically.
__device__ __forceinline__ double2 csqrt_radiating(double2 z) {
  double2 w = csqrt_principal(z);
  if (w.y > w.x) w = make_double2(-w.x, -w.y);
  return w;
}

// sin(z)/z for complex z with the removable point handled by its series.
__device__ __forceinline__ double2 csinc(double2 z) {
  const double a2 = z.x * z.x + z.y * z.y;
  if (a2 < 1e-8) {
    const double2 z2 = cmul(z, z);
    const double2 z4 = cmul(z2, z2);
    return make_double2(1.0 - z2.x / 6.0 + z4.x / 120.0, -z2.y / 6.0 + z4.y / 120.0);
  }
  double s, c;
  sincos(z.x, &s, &c);
  const double sh = sinh(z.y), ch = cosh(z.y);
  return cdiv(make_double2(s * ch, c * sh), z);
}

// Local contour ratio g = beta_I/beta at |k| = beta and the path slope
// beta_I' = d beta_I/d beta: ray, g = beta_I' = gamma; parabolic (beta_I =
// gamma beta (1 - beta/beta_end) below beta_end, real beyond),
// g = gamma (1 - beta/beta_end), beta_I' = gamma (1 - 2 beta/beta_end).  The
// slope jumps at beta_end; a sample there (within a relative 1e-9, so that
// the rounding of beta does not decide) takes the mean slope -gamma/2.
__device__ __forceinline__ void contour_ratio(double beta, double gamma, int parabolic, double beta_end,
                                              double& g, double& slope) {
  if (!parabolic) {
    g = slope = gamma;
    return;
  }
  g = beta < beta_end ? gamma * (1.0 - beta / beta_end) : 0.0;
  if (fabs(beta - beta_end) <= 1e-9 * beta_end) slope = -0.5 * gamma;
  else slope = beta < beta_end ? gamma * (1.0 - 2.0 * beta / beta_end) : 0.0;
}

// Non-temporal (streaming) store for data written once; it moves
// the whole complex value in one instruction.
template <typename V> __device__ __forceinline__ void store_nt(V* p, V v) {
  using Rl = typename real_of<V>::type;
  typedef Rl pair_t __attribute__((ext_vector_type(2)));
  pair_t w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<pair_t*>(p));
}

// ---------------------------------------------------------------- FFT
__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// LDS slot of exchange element i: one pad entry after every 2^S elements.  A
// radix-8 stage writes 8 consecutive elements per thread (stride 128 B for
// complex128), which without padding puts many lanes of one LDS access on
// the same banks; the pad spreads them.  The best S depends on how the lanes
// of a transform sit in a wave (one transform per wave: S = 4; four
// interleaved column transforms: S = 3 with a per-column offset).
template <int S = 3> __host__ __device__ constexpr int lds_slot(int i) { return i + (i >> S); }
// LDS entries needed by one length-N exchange buffer.
template <int S = 3> __host__ __device__ constexpr int lds_len(int n) { return n + (n >> S); }

// In-register forward DFT of 2, 4 or 8 points (omega = exp(-2 pi i / n)).
template <typename V> __device__ __forceinline__ void dft2(V& a, V& b) {
  const V t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename V> __device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
  const V s02 = cadd(x0, x2), d02 = csub(x0, x2);
  const V s13 = cadd(x1, x3), d13 = csub(x1, x3);
  x0 = cadd(s02, s13);
  x2 = csub(s02, s13);
  x1 = cadd(d02, cmul_mi(d13));
  x3 = csub(d02, cmul_mi(d13));
}

template <typename V> __device__ __forceinline__ void dft8(V* x) {
  using R = typename real_of<V>::type;
  const R h = (R)0.70710678118654752440;
  V e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  V o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // o_k *= omega8^k
  o1 = mk((R)((o1.x + o1.y) * h), (R)((o1.y - o1.x) * h));
  o2 = cmul_mi(o2);
  o3 = mk((R)((o3.y - o3.x) * h), (R)(-(o3.x + o3.y) * h));
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

template <typename V, int RHO> __device__ __forceinline__ void dft_small(V* y) {
  if constexpr (RHO == 2) dft2(y[0], y[1]);
  else if constexpr (RHO == 4) dft4(y[0], y[1], y[2], y[3]);
  else dft8(y);
}

// Twiddles w(m) = exp(-2 pi i m / N) live in LDS as two short tables,
// lo[j] = w(j) (j < 64) and hi[j] = w(64 j) (j < N/64), so that
// w(m) = hi[m >> 6] lo[m & 63]: 64 + N/64 entries per block instead of N,
// read through the LDS pipe instead of competing with the streaming global
// loads and stores.
template <int N> struct TwLds {
  static constexpr int LO = N < 64 ? N : 64;
  static constexpr int HI = N <= 64 ? 0 : N / 64;
  static constexpr int LEN = LO + HI;
};

// Fill the LDS tables from the full global table w(0..N-1); all threads of
// the block take part; a barrier must follow before the first use.
template <typename V, int N>
__device__ __forceinline__ void load_twiddles(V* ltw, const V* __restrict__ gtw, int tid, int nthreads) {
  for (int i = tid; i < TwLds<N>::LEN; i += nthreads)
    ltw[i] = i < TwLds<N>::LO ? gtw[i] : gtw[64 * (i - TwLds<N>::LO)];
}

template <typename V, int N> __device__ __forceinline__ V tw_at(const V* ltw, int m) {
  if constexpr (N <= 64) return ltw[m];
  else return cmul(ltw[TwLds<N>::LO + (m >> 6)], ltw[m & 63]);
}

// Barrier between the LDS writes and reads of one exchange.  When every
// thread of a transform sits in one wave (WAVE), no other wave touches its
// LDS region and a wave's LDS instructions execute in issue order, so it is
// enough to keep the compiler from moving LDS accesses across this point;
// otherwise the whole block synchronises.
template <bool WAVE> __device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham stage of radix RHO on a length-N transform spread over
// T = N/R threads, each holding R points at stride T (x[r] = data[t + T r]).
// L is the length of the sub-transforms already done.  Non-final stages
// exchange through `lds` (lds_len(N) entries, padded slots); the final stage leaves the outputs in
// registers in the same stride-T order.
template <typename V, int N, int R, int RHO, bool LAST, bool WAVE, int PS>
__device__ __forceinline__ void stockham_stage(V (&x)[R], V* lds, const V* ltw, int t, int L) {
  constexpr int T = N / R;
  constexpr int BPT = R / RHO;
#pragma unroll
  for (int mb = 0; mb < BPT; ++mb) {
    const int i = t + T * mb;
    const int k = i & (L - 1);
    V y[RHO];
#pragma unroll
    for (int j = 0; j < RHO; ++j) y[j] = x[mb + j * BPT];
    if (L > 1) {
      const int step = N / (L * RHO);
      if constexpr (RHO == 8) {
        // w^j for j = 1..7 from one table lookup w = w(k step): products of
        // at most three factors after the lookup (w^2 = w w, w^3 = w^2 w,
        // w^4 = w^2 w^2, w^5 = w^4 w, w^6 = w^3 w^3, w^7 = w^4 w^3), which
        // replaces six LDS lookups per stage with the same number of complex
        // products.  k step < N/8, so for N <= 512 the lookup is lo[] alone.
        const int m = k * step;
        V w1;
        if constexpr (N / RHO <= 64) w1 = ltw[m];
        else w1 = tw_at<V, N>(ltw, m);
        const V w2 = cmul(w1, w1);
        const V w4 = cmul(w2, w2);
        const V w3 = cmul(w2, w1);
        y[1] = cmul(y[1], w1);
        y[2] = cmul(y[2], w2);
        y[5] = cmul(y[5], cmul(w4, w1));
        y[4] = cmul(y[4], w4);
        y[3] = cmul(y[3], w3);
        y[6] = cmul(y[6], cmul(w3, w3));
        y[7] = cmul(y[7], cmul(w4, w3));
      } else {
#pragma unroll
        for (int j = 1; j < RHO; ++j) y[j] = cmul(y[j], tw_at<V, N>(ltw, j * k * step));
      }
    }
    dft_small<V, RHO>(y);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RHO; ++q) x[mb + q * BPT] = y[q];
    } else {
      const int base = (i - k) * RHO + k;
#pragma unroll
      for (int q = 0; q < RHO; ++q) lds[lds_slot<PS>(base + q * L)] = y[q];
    }
  }
  if constexpr (!LAST) {
    exchange_sync<WAVE>();
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = lds[lds_slot<PS>(t + T * r)];
    exchange_sync<WAVE>();
  }
}

// Forward DFT X[j] = sum_n x[n] exp(-2 pi i n j / N), N = 2^m, 8 <= N.
// Radices: one leading radix-2 or radix-4 stage when log2 N is not a
// multiple of 3, then radix-8 stages.  All threads of the block must call
// it (it contains block barriers), unless WAVE: then the N/R threads of each
// transform must be lanes of one wave, and only they synchronise.
template <typename V, int N, int R, bool WAVE = false, int PS = 3>
__device__ __forceinline__ void fft_forward(V (&x)[R], V* lds, const V* ltw, int t) {
  static_assert(R == 8 || R == 16 || R == 32, "8, 16 or 32 points per thread");
  static_assert(!WAVE || N / R <= 64, "a wave-local transform needs at most 64 threads");
  // Keep the twiddle addressing inside the caller's term loop: without this
  // the compiler hoists every stage's twiddle loads out of the loop and keeps
  // them live across it, which costs ~60 VGPRs and halves occupancy.
  asm volatile("" : "+v"(t));
  constexpr int LOG = ilog2c(N);
  constexpr int NR8 = LOG / 3;
  constexpr int REM = LOG % 3;
  int L = 1;
  if constexpr (REM == 1) {
    stockham_stage<V, N, R, 2, NR8 == 0, WAVE, PS>(x, lds, ltw, t, L);
    L *= 2;
  } else if constexpr (REM == 2) {
    stockham_stage<V, N, R, 4, NR8 == 0, WAVE, PS>(x, lds, ltw, t, L);
    L *= 4;
  }
  if constexpr (NR8 >= 1) {
    if constexpr (NR8 >= 2) {
#pragma unroll
      for (int s = 0; s < NR8 - 1; ++s) {
        stockham_stage<V, N, R, 8, false, WAVE, PS>(x, lds, ltw, t, L);
        L *= 8;
      }
    }
    stockham_stage<V, N, R, 8, true, WAVE, PS>(x, lds, ltw, t, L);
  }
}

// Two independent transforms of the same length through one sequence of
// stages: a stage's twiddles are formed once for both, and the two exchanges
// (each transform in its own LDS region, lx and lz) share one pair of
// barriers.  Each transform sees exactly the operations of fft_forward, so
// the results are the same bit for bit; what changes is that a wave has two
// independent butterfly chains to issue from between its LDS waits.
template <typename V, int N, int R, int RHO, bool LAST, bool WAVE, int PS>
__device__ __forceinline__ void stockham_stage2(V (&x)[R], V (&z)[R], V* lx, V* lz, const V* ltw, int t, int L) {
  constexpr int T = N / R;
  constexpr int BPT = R / RHO;
#pragma unroll
  for (int mb = 0; mb < BPT; ++mb) {
    const int i = t + T * mb;
    const int k = i & (L - 1);
    V y[RHO], u[RHO];
#pragma unroll
    for (int j = 0; j < RHO; ++j) {
      y[j] = x[mb + j * BPT];
      u[j] = z[mb + j * BPT];
    }
    if (L > 1) {
      const int step = N / (L * RHO);
      if constexpr (RHO == 8) {
        // the powers w^j as in stockham_stage, formed once for both transforms
        const int m = k * step;
        V w1;
        if constexpr (N / RHO <= 64) w1 = ltw[m];
        else w1 = tw_at<V, N>(ltw, m);
        const V w2 = cmul(w1, w1);
        const V w4 = cmul(w2, w2);
        const V w3 = cmul(w2, w1);
        const V w5 = cmul(w4, w1);
        const V w6 = cmul(w3, w3);
        const V w7 = cmul(w4, w3);
        y[1] = cmul(y[1], w1);
        u[1] = cmul(u[1], w1);
        y[2] = cmul(y[2], w2);
        u[2] = cmul(u[2], w2);
        y[5] = cmul(y[5], w5);
        u[5] = cmul(u[5], w5);
        y[4] = cmul(y[4], w4);
        u[4] = cmul(u[4], w4);
        y[3] = cmul(y[3], w3);
        u[3] = cmul(u[3], w3);
        y[6] = cmul(y[6], w6);
        u[6] = cmul(u[6], w6);
        y[7] = cmul(y[7], w7);
        u[7] = cmul(u[7], w7);
      } else {
#pragma unroll
        for (int j = 1; j < RHO; ++j) {
          const V w = tw_at<V, N>(ltw, j * k * step);
          y[j] = cmul(y[j], w);
          u[j] = cmul(u[j], w);
        }
      }
    }
    dft_small<V, RHO>(y);
    dft_small<V, RHO>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RHO; ++q) {
        x[mb + q * BPT] = y[q];
        z[mb + q * BPT] = u[q];
      }
    } else {
      const int base = (i - k) * RHO + k;
#pragma unroll
      for (int q = 0; q < RHO; ++q) {
        lx[lds_slot<PS>(base + q * L)] = y[q];
        lz[lds_slot<PS>(base + q * L)] = u[q];
      }
    }
  }
  if constexpr (!LAST) {
    exchange_sync<WAVE>();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      x[r] = lx[lds_slot<PS>(t + T * r)];
      z[r] = lz[lds_slot<PS>(t + T * r)];
    }
    exchange_sync<WAVE>();
  }
}

// fft_forward of two independent inputs at once (see stockham_stage2).
template <typename V, int N, int R, bool WAVE = false, int PS = 3>
__device__ __forceinline__ void fft_forward2(V (&x)[R], V (&z)[R], V* lx, V* lz, const V* ltw, int t) {
  static_assert(R == 8, "8 points per thread");
  asm volatile("" : "+v"(t));
  constexpr int LOG = ilog2c(N);
  constexpr int NR8 = LOG / 3;
  constexpr int REM = LOG % 3;
  int L = 1;
  if constexpr (REM == 1) {
    stockham_stage2<V, N, R, 2, NR8 == 0, WAVE, PS>(x, z, lx, lz, ltw, t, L);
    L *= 2;
  } else if constexpr (REM == 2) {
    stockham_stage2<V, N, R, 4, NR8 == 0, WAVE, PS>(x, z, lx, lz, ltw, t, L);
    L *= 4;
  }
  if constexpr (NR8 >= 1) {
    if constexpr (NR8 >= 2) {
#pragma unroll
      for (int s = 0; s < NR8 - 1; ++s) {
        stockham_stage2<V, N, R, 8, false, WAVE, PS>(x, z, lx, lz, ltw, t, L);
        L *= 8;
      }
    }
    stockham_stage2<V, N, R, 8, true, WAVE, PS>(x, z, lx, lz, ltw, t, L);
  }
}

// Inverse (unnormalised) DFT: conj(DFT(conj x)).
template <typename V, int N, int R, bool WAVE = false, int PS = 3>
__device__ __forceinline__ void fft_inverse(V (&x)[R], V* lds, const V* ltw, int t) {
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = cconj(x[r]);
  fft_forward<V, N, R, WAVE, PS>(x, lds, ltw, t);
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = cconj(x[r]);
}

// ---------------------------------------------------------------- table stencils
// Bilinear cell of the fractional table index (ux, uy): rejects NaN,
// negative and beyond-the-last-cell points before any cast.
__device__ __forceinline__ bool cell_at(double ux, double uy, int nx, int ny, int& j1, int& j2, double& tx,
                                        double& ty) {
  if (!(ux >= 0.0) || !(uy >= 0.0) || !(ux < (double)(nx - 1)) || !(uy < (double)(ny - 1))) return false;
  j1 = (int)floor(ux);
  j2 = (int)floor(uy);
  if (j1 > nx - 2 || j2 > ny - 2) return false;
  tx = ux - j1;
  ty = uy - j2;
  return true;
}

// Second-order interpolation (Sec. III-B.3, last paragraph): per axis the
// nodes c - 1, c, c + 1 around the nearest node c = round(u), kept in
// [1, n-2], with the quadratic Lagrange weights in t = u - c.  Points need
// 0 <= u <= n - 1 on both axes; others (and NaN) yield NaN.
__device__ __forceinline__ bool stencil_at(double ux, double uy, int nx, int ny, int& c1, int& c2, double& tx,
                                           double& ty) {
  if (!(ux >= 0.0) || !(uy >= 0.0) || !(ux <= (double)(nx - 1)) || !(uy <= (double)(ny - 1))) return false;
  c1 = min(max((int)floor(ux + 0.5), 1), nx - 2);
  c2 = min(max((int)floor(uy + 0.5), 1), ny - 2);
  tx = ux - c1;
  ty = uy - c2;
  return true;
}

__device__ __forceinline__ void lagrange3(double t, double (&w)[3]) {
  w[0] = 0.5 * t * (t - 1.0);
  w[1] = (1.0 - t) * (1.0 + t);
  w[2] = 0.5 * t * (t + 1.0);
}

// XCD-aware remap of the block index: the hardware deals consecutive block
// ids round-robin to the 8 XCDs; this returns a logical id such that
// consecutive logical ids run on the same XCD (and so share its L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int NXCD = 8;
  const int per = nblocks / NXCD;
  const int full = per * NXCD;
  if (bid >= full) return bid;
  return (bid % NXCD) * per + bid / NXCD;
}

}  // namespace cfft
