// Grounded-slab spectral dyadic Green's function minus the effective
// homogeneous medium and its image (Sec. II, Sec. III-A of the paper), on
// the contour k_c = (1 + i g) k (g = gamma on the ray, g = g(|k|) on the
// parabolic contour), in FP64.  One thread per quadrant
// sample, writing its mirror images; interleaved complex128 output
// [3][ny][nx] with x fastest.
//
// The same templated evaluation runs on forward-mode dual numbers in the
// adjoint, giving dG/d eps_r and dG/dh analytically.
#include "cfft_device.h"
#include "cfft_internal.h"

namespace cfft {

// ------------------------------------------------ scalar / dual complex ops
template <int ND> struct dc {
  double2 v;
  double2 d[ND];
};

__device__ __forceinline__ double2 lift0(double2 a) { return a; }
__device__ __forceinline__ double2 o_add(double2 a, double2 b) { return cadd(a, b); }
__device__ __forceinline__ double2 o_sub(double2 a, double2 b) { return csub(a, b); }
__device__ __forceinline__ double2 o_mul(double2 a, double2 b) { return cmul(a, b); }
__device__ __forceinline__ double2 o_div(double2 a, double2 b) { return cdiv(a, b); }
__device__ __forceinline__ double2 o_cmul(double2 a, double2 c) { return cmul(a, c); }
__device__ __forceinline__ double2 o_rmul(double2 a, double r) { return cscale(a, r); }
__device__ __forceinline__ double2 o_neg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 o_sqrt(double2 a) { return csqrt_radiating(a); }
__device__ __forceinline__ double2 o_expm1(double2 a) { return cexpm1(a); }
__device__ __forceinline__ double2 o_const(double2 c, double2) { return c; }

template <int ND> __device__ __forceinline__ dc<ND> o_const(double2 c, dc<ND>) {
  dc<ND> r;
  r.v = c;
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = make_double2(0.0, 0.0);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_add(const dc<ND>& a, const dc<ND>& b) {
  dc<ND> r;
  r.v = cadd(a.v, b.v);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cadd(a.d[i], b.d[i]);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_sub(const dc<ND>& a, const dc<ND>& b) {
  dc<ND> r;
  r.v = csub(a.v, b.v);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = csub(a.d[i], b.d[i]);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_mul(const dc<ND>& a, const dc<ND>& b) {
  dc<ND> r;
  r.v = cmul(a.v, b.v);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cadd(cmul(a.d[i], b.v), cmul(a.v, b.d[i]));
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_div(const dc<ND>& a, const dc<ND>& b) {
  dc<ND> r;
  r.v = cdiv(a.v, b.v);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cdiv(csub(a.d[i], cmul(r.v, b.d[i])), b.v);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_cmul(const dc<ND>& a, double2 c) {
  dc<ND> r;
  r.v = cmul(a.v, c);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cmul(a.d[i], c);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_rmul(const dc<ND>& a, double s) {
  dc<ND> r;
  r.v = cscale(a.v, s);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cscale(a.d[i], s);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_neg(const dc<ND>& a) { return o_rmul(a, -1.0); }
template <int ND> __device__ __forceinline__ dc<ND> o_sqrt(const dc<ND>& a) {
  dc<ND> r;
  r.v = csqrt_radiating(a.v);
  const double2 inv2 = cdiv(make_double2(0.5, 0.0), r.v);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cmul(a.d[i], inv2);
  return r;
}
template <int ND> __device__ __forceinline__ dc<ND> o_expm1(const dc<ND>& a) {
  dc<ND> r;
  r.v = cexpm1(a.v);
  const double2 e = make_double2(r.v.x + 1.0, r.v.y);
#pragma unroll
  for (int i = 0; i < ND; ++i) r.d[i] = cmul(a.d[i], e);
  return r;
}

// Immittance differences dZ_TE, dZ_TM at beta_c^2 = (1 + i gamma)^2 beta^2.
//   kz0 = sqrt(k0^2 - beta_c^2), kz1 = sqrt(eps k0^2 - beta_c^2) (radiating root),
//   t = tan(kz1 h) = i E1/(2 + E1), E1 = expm1(-2 i kz1 h)  (bounded at large beta)
//   Z_TE = i k0 t / (kz1 + i kz0 t)
//   Z_TM = i kz1 kz0 t / (k0 (eps kz0 + i kz1 t))
//   eps_e = (eps + 1)/2, ke = sqrt(eps_e k0^2 - beta_c^2), e_h = -expm1(-2 i ke h)
//   Zh_TE = k0 e_h / (2 ke),  Zh_TM = ke e_h / (2 k0 eps_e)
template <typename C>
__device__ __forceinline__ void immittance_diff(double beta, double gamma, double k0, const C& eps,
                                                const C& h, C& dte, C& dtm) {
  const double b2 = beta * beta;
  const C bc2 = o_const(make_double2((1.0 - gamma * gamma) * b2, 2.0 * gamma * b2), eps);
  const C k02 = o_const(make_double2(k0 * k0, 0.0), eps);
  const C kz0 = o_sqrt(o_sub(k02, bc2));
  const C kz1 = o_sqrt(o_sub(o_mul(eps, k02), bc2));
  const C e1 = o_expm1(o_cmul(o_mul(kz1, h), make_double2(0.0, -2.0)));
  const C t = o_div(o_cmul(e1, make_double2(0.0, 1.0)), o_add(o_const(make_double2(2.0, 0.0), eps), e1));
  const C kz0t_i = o_cmul(o_mul(kz0, t), make_double2(0.0, 1.0));
  const C zte = o_div(o_cmul(t, make_double2(0.0, k0)), o_add(kz1, kz0t_i));
  const C kz1t_i = o_cmul(o_mul(kz1, t), make_double2(0.0, 1.0));
  const C ztm = o_div(o_cmul(o_mul(kz0, kz1t_i), make_double2(1.0, 0.0)),
                      o_rmul(o_add(o_mul(eps, kz0), kz1t_i), k0));
  const C epse = o_rmul(o_add(eps, o_const(make_double2(1.0, 0.0), eps)), 0.5);
  const C ke = o_sqrt(o_sub(o_mul(epse, k02), bc2));
  const C eh = o_neg(o_expm1(o_cmul(o_mul(ke, h), make_double2(0.0, -2.0))));
  const C hte = o_div(o_rmul(eh, 0.5 * k0), ke);
  const C htm = o_div(o_mul(ke, eh), o_rmul(epse, 2.0 * k0));
  dte = o_sub(zte, hte);
  dtm = o_sub(ztm, htm);
}

// Dyadic: Gxx = -(c^2 dTM + s^2 dTE), Gyy = -(s^2 dTM + c^2 dTE),
// Gxy = -c s (dTM - dTE); at beta = 0 the isotropic limit -dTE * I.
template <typename C>
__device__ __forceinline__ void green_dyadic(double kx, double ky, double gamma, double k0, const C& eps,
                                             const C& h, C& gxx, C& gxy, C& gyy) {
  const double beta = hypot(kx, ky);
  C dte, dtm;
  immittance_diff(beta, gamma, k0, eps, h, dte, dtm);
  double c = 1.0, s = 0.0;
  if (beta > 0.0) {
    c = kx / beta;
    s = ky / beta;
  } else {
    dtm = dte;
  }
  gxx = o_neg(o_add(o_rmul(dtm, c * c), o_rmul(dte, s * s)));
  gyy = o_neg(o_add(o_rmul(dtm, s * s), o_rmul(dte, c * c)));
  gxy = o_rmul(o_sub(dtm, dte), -c * s);
}

// Mirror symmetry of the sample grid: k(N/2 + h) = h dk = -k(N/2 - h), and
// index 0 (k = -k_max) is the mirror of h = N/2.  The immittances depend on
// beta only; Gxx and Gyy are even and Gxy odd in each of kx and ky.  One
// thread therefore evaluates the dyadic at (h1 dkx, h2 dky), h in [0, N/2],
// and writes the up to four mirrored samples (n1, n2) = (N/2 +- h1, N/2 +- h2)
// that exist, negating Gxy where exactly one of kx, ky changes sign (the
// same value a direct evaluation at the negated wavenumber gives).
__host__ __device__ int green_threads(const GreenParams& p) { return (p.x.n / 2 + 1) * (p.y.n / 2 + 1); }

struct Mirror {
  int h1, h2;
};
__device__ __forceinline__ bool mirror_of(const GreenParams& p, int idx, Mirror& m) {
  const int hx = p.x.n / 2, hy = p.y.n / 2;
  if (idx >= (hx + 1) * (hy + 1)) return false;
  m.h1 = idx % (hx + 1);
  m.h2 = idx / (hx + 1);
  return true;
}
// Sample q (0..3) of the mirror set: bit 0 selects N/2 - h1, bit 1 N/2 - h2.
// Returns the flat sample index, or -1 where that mirror does not exist.
__device__ __forceinline__ int mirror_sample(const GreenParams& p, const Mirror& m, int q) {
  const int hx = p.x.n / 2, hy = p.y.n / 2;
  const bool fx = q & 1, fy = q & 2;
  const int n1 = fx ? hx - m.h1 : hx + m.h1;
  const int n2 = fy ? hy - m.h2 : hy + m.h2;
  if (n1 >= p.x.n || n2 >= p.y.n) return -1;   // h = N/2 has only its minus mirror
  if ((fx && m.h1 == 0) || (fy && m.h2 == 0)) return -1;   // h = 0 is its own mirror
  return n2 * p.x.n + n1;
}

__global__ void __launch_bounds__(256) green_kernel(GreenParams p, double2* __restrict__ g) {
  Mirror mr;
  if (!mirror_of(p, blockIdx.x * blockDim.x + threadIdx.x, mr)) return;
  const int n = p.x.n * p.y.n;
  const double kx = mr.h1 * p.x.dk;
  const double ky = mr.h2 * p.y.dk;
  const double2 eps = make_double2(p.eps_re, -p.eps_re * p.tan_delta);
  const double2 h = make_double2(p.h, 0.0);
  double ratio, slope;
  contour_ratio(hypot(kx, ky), p.gamma, p.parabolic, p.beta_end, ratio, slope);
  double2 gxx, gxy, gyy;
  green_dyadic(kx, ky, ratio, p.k0, eps, h, gxx, gxy, gyy);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = mirror_sample(p, mr, q);
    if (i < 0) continue;
    const bool odd = (q == 1) || (q == 2);
    g[i] = gxx;
    g[n + i] = odd ? make_double2(-gxy.x, -gxy.y) : gxy;
    g[2 * n + i] = gyy;
  }
}

hipError_t launch_green(const GreenParams& p, double2* g, hipStream_t s) {
  const int n = green_threads(p);
  hipLaunchKernelGGL(green_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g);
  return hipGetLastError();
}

// ------------------------------------------------ adjoint
// partial[block][2] = sum over the block's samples of
//   Re sum_c conj(gG_c) dG_c/d theta,  theta in (eps_r', h).
__global__ void __launch_bounds__(256) adj_green_kernel(GreenParams p, const double2* __restrict__ gg,
                                                        double* __restrict__ partial) {
  __shared__ double red[2][256];
  const int n = p.x.n * p.y.n;
  const int nq = green_threads(p);
  double acc0 = 0.0, acc1 = 0.0;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nq; idx += gridDim.x * blockDim.x) {
    Mirror mr;
    mirror_of(p, idx, mr);
    const double kx = mr.h1 * p.x.dk;
    const double ky = mr.h2 * p.y.dk;
    dc<2> eps, h;
    eps.v = make_double2(p.eps_re, -p.eps_re * p.tan_delta);
    eps.d[0] = make_double2(1.0, -p.tan_delta);
    eps.d[1] = make_double2(0.0, 0.0);
    h.v = make_double2(p.h, 0.0);
    h.d[0] = make_double2(0.0, 0.0);
    h.d[1] = make_double2(1.0, 0.0);
    dc<2> gxx, gxy, gyy;
    green_dyadic(kx, ky, p.gamma, p.k0, eps, h, gxx, gxy, gyy);
    // the mirrored samples share dGxx, dGyy; dGxy flips sign with Gxy
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = mirror_sample(p, mr, q);
      if (i < 0) continue;
      const double sg = (q == 1 || q == 2) ? -1.0 : 1.0;
      const double2 a = gg[i], b = gg[n + i], c = gg[2 * n + i];
      // Re(conj(a) d) = a.x d.x + a.y d.y
      acc0 += a.x * gxx.d[0].x + a.y * gxx.d[0].y + sg * (b.x * gxy.d[0].x + b.y * gxy.d[0].y) +
              c.x * gyy.d[0].x + c.y * gyy.d[0].y;
      acc1 += a.x * gxx.d[1].x + a.y * gxx.d[1].y + sg * (b.x * gxy.d[1].x + b.y * gxy.d[1].y) +
              c.x * gyy.d[1].x + c.y * gyy.d[1].y;
    }
  }
  red[0][threadIdx.x] = acc0;
  red[1][threadIdx.x] = acc1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = red[0][0];
    partial[2 * blockIdx.x + 1] = red[1][0];
  }
}

hipError_t launch_adj_green(const GreenParams& p, const double2* gg, double* partial, int nblocks,
                            hipStream_t s) {
  hipLaunchKernelGGL(adj_green_kernel, dim3(nblocks), dim3(256), 0, s, p, gg, partial);
  return hipGetLastError();
}

// out[c] = sum_i partial[i * count + c], fixed order (deterministic).
__global__ void reduce_sum_kernel(const double* __restrict__ partial, int n, int count, double* __restrict__ out) {
  __shared__ double red[256];
  for (int c = 0; c < count; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i * count + c];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_sum(const double* partial, int n, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, partial, n, count, out);
  return hipGetLastError();
}

}  // namespace cfft
