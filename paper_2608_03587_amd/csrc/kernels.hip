// HIP kernels (gfx950) of the DEC beam-propagation hot path.
//
// The operators are sparse stencils (about six off-diagonal neighbours per
// vertex), so every kernel here is bandwidth/latency bound: one thread per
// (vertex, field) pair, gathers through the sliced-ELL layout of kernels.hpp,
// neighbours made local in memory by the Hilbert vertex order, and the
// pointwise work (RK4 stage update, Kerr phase, absorber damping, the next
// substep's |psi|^2 phi) fused into the gather kernels so each pass reads and
// writes every vector once.  No matrix cores: there is no dense contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "kernels.hpp"

// The build compiles this file twice in parallel: DECBPM_PART 1 emits the
// complex64 instantiations and the precision-independent launchers, 2 the
// complex128 ones (3, the default, emits everything in one object).
#ifndef DECBPM_PART
#define DECBPM_PART 3
#endif

namespace decbpm {

namespace {

// ---- scalar math (HIP's device math library) ----
__device__ inline float d_exp(float x) { return expf(x); }
__device__ inline double d_exp(double x) { return exp(x); }
__device__ inline float d_expm1(float x) { return expm1f(x); }
__device__ inline double d_expm1(double x) { return expm1(x); }
__device__ inline float d_log1p(float x) { return log1pf(x); }
__device__ inline double d_log1p(double x) { return log1p(x); }
__device__ inline void d_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline void d_sincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline bool d_finite(float x) { return isfinite(x); }
__device__ inline bool d_finite(double x) { return isfinite(x); }

// integral of e^{-2 w z} over [0, tau]
template <typename T>
__device__ inline T phi_w(T w, T tau) {
  return w > T(0) ? -d_expm1(T(-2) * w * tau) / (T(2) * w) : tau;
}

// Integral over [0, tau] of N(I e^{-2 w z}): the intensity a row contributes to
// the Kerr phase of an exact substep of length tau (the response N of d.nk;
// |psi|^2 decays as I e^{-2 w z} along the substep).  Kerr: I phi(w, tau);
// cubic-quintic: I phi(w, tau) - s I^2 phi(2w, tau); saturable (I_s):
// (I_s/(2w)) log((1 + a)/(1 + a e)), a = I/I_s, e = e^{-2 w tau}, taken as
// log1p(a (1 - e)/(1 + a e)) with 1 - e = -expm1(-2 w tau) (full precision
// for small a and small w tau), and tau I/(1 + a) at w = 0.
template <typename T>
__device__ inline T nl_int(const DevOps<T>& d, T I, T w, T tau) {
  if (d.nk == 0) return I * phi_w(w, tau);
  if (d.nk == 2) return I * phi_w(w, tau) - d.npar * I * I * phi_w(T(2) * w, tau);
  const T a = I / d.npar;
  if (w <= T(0)) return tau * I / (T(1) + a);
  const T ome = -d_expm1(T(-2) * w * tau);
  return d.npar / (T(2) * w) * d_log1p(a * ome / (T(1) + a * (T(1) - ome)));
}

template <typename T>
struct CT;
template <>
struct CT<float> {
  using C = float2;
};
template <>
struct CT<double> {
  using C = double2;
};

// Logical block index: with xcd_remap, hardware block b (dispatched round-robin
// over the 8 XCDs) takes logical block (b % 8) * (grid/8) + b / 8, so each XCD
// walks one contiguous stretch of the Hilbert-ordered rows and the halo of
// neighbouring blocks stays in the same L2.
__device__ inline int64_t logical_block(int32_t remap) {
  int64_t b = blockIdx.x;
  if (remap) {
    const int64_t per = gridDim.x >> 3;
    b = (b & 7) * per + (b >> 3);
  }
  return b;
}

template <int FB, typename T>
__device__ inline void split(int64_t idx, const DevOps<T>& d, int64_t& row, int32_t& f) {
  if (FB == 1) {  // one field per row
    row = idx;
    f = 0;
  } else if (FB == 2) {  // power-of-two field count
    row = idx >> d.lgF;
    f = int32_t(idx & ((int64_t(1) << d.lgF) - 1));
  } else {
    row = idx / d.F;
    f = int32_t(idx - row * d.F);
  }
}

inline unsigned grid_for(int64_t threads, int block, int remap) {
  int64_t g = (threads + block - 1) / block;
  if (remap) g = (g + 7) / 8 * 8;
  if (g < 1) g = 1;
  return unsigned(g);
}

// Visit the stored neighbours (q, weight) of `row`.  With KMAX > 0 every
// index and weight of the row is loaded before the first use, so a thread
// has all its gathers in flight at once instead of a chain of W dependent
// index -> value round trips.
template <int KMAX, typename T, typename W_t, typename Fn>
__device__ inline void for_neighbours(const DevOps<T>& d, const W_t* __restrict__ wt, int64_t row, Fn&& fn) {
  const int64_t info = d.sl_info[row >> 6];
  const int W = int(info & 0xff);
  const int64_t base = (info >> 8) + (row & 63);
  if constexpr (KMAX > 0) {
    int32_t q[KMAX];
    W_t c[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < W) {
        q[k] = d.col[base + 64 * k];
        c[k] = wt[base + 64 * k];
      } else {
        q[k] = 0;
        c[k] = W_t(0);
      }
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < W) fn(q[k], c[k]);
  } else {
    for (int k = 0; k < W; ++k) fn(d.col[base + 64 * k], wt[base + 64 * k]);
  }
}

// ---------------------------------------------------------------------------
// RK4 stage: y = psi + coef * A x,  A = -i H_lin.
//   B4 = false: H_lin x = p1 L x - v x (one gather of x)
//   B4 = true : t = L x is given; H_lin x = p1 t + beta4 L t - v x (gather of t)
// WS: also write s = |y|^2 phi(w, tau_s) for the Kerr substep that follows.
template <typename T, int FB, int KMAX, bool B4, bool WS>
__global__ void __launch_bounds__(1024) k_stage(DevOps<T> d, const typename CT<T>::C* __restrict__ x,
                                                const typename CT<T>::C* __restrict__ t,
                                                const typename CT<T>::C* psi, typename CT<T>::C* y, T coef,
                                                T* __restrict__ s_out, T tau_s) {
  using C = typename CT<T>::C;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const C* __restrict__ g = B4 ? t : x;
  const C gr = g[idx];
  const C xr = B4 ? x[idx] : gr;
  const C p = psi[idx];
  const T vr = d.v[row];
  T ar = T(0), ai = T(0);
  const int64_t FF = FB == 1 ? 1 : d.F;
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const C gq = g[int64_t(q) * FF + f];
    ar += c * (gr.x - gq.x);
    ai += c * (gr.y - gq.y);
  });
  T hr, hi;
  if (B4) {
    hr = d.p1 * gr.x + d.beta4 * ar - vr * xr.x;
    hi = d.p1 * gr.y + d.beta4 * ai - vr * xr.y;
  } else {
    hr = d.p1 * ar - vr * xr.x;
    hi = d.p1 * ai - vr * xr.y;
  }
  C out;
  out.x = p.x + coef * hi;  // -i (hr + i hi) = hi - i hr
  out.y = p.y - coef * hr;
  y[idx] = out;
  if (WS) s_out[idx] = nl_int(d, out.x * out.x + out.y * out.y, d.w[row], tau_s);
}

// t = L x
template <typename T, int FB, int KMAX>
__global__ void __launch_bounds__(1024) k_lap(DevOps<T> d, const typename CT<T>::C* __restrict__ x,
                                              typename CT<T>::C* __restrict__ t) {
  using C = typename CT<T>::C;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const C xr = x[idx];
  T ar = T(0), ai = T(0);
  const int64_t FF = FB == 1 ? 1 : d.F;
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const C xq = x[int64_t(q) * FF + f];
    ar += c * (xr.x - xq.x);
    ai += c * (xr.y - xq.y);
  });
  C out;
  out.x = ar;
  out.y = ai;
  t[idx] = out;
}

// y = a L z + b x (F = 1)
template <typename T, int KMAX>
__global__ void __launch_bounds__(1024) k_lapc(DevOps<T> d, const typename CT<T>::C* __restrict__ z,
                                               const typename CT<T>::C* __restrict__ x, T a, T b,
                                               typename CT<T>::C* __restrict__ y) {
  using C = typename CT<T>::C;
  const int64_t row = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  if (row >= d.n_rows) return;
  const C zr = z[row];
  const C xr = x[row];
  T ar = T(0), ai = T(0);
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const C zq = z[q];
    ar += c * (zr.x - zq.x);
    ai += c * (zr.y - zq.y);
  });
  C out;
  out.x = a * ar + b * xr.x;
  out.y = a * ai + b * xr.y;
  y[row] = out;
}

template <typename T, int FB>
__global__ void __launch_bounds__(1024) k_prep_s(DevOps<T> d, const typename CT<T>::C* __restrict__ psi,
                                                 T* __restrict__ s, T tau) {
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const auto p = psi[idx];
  s[idx] = nl_int(d, p.x * p.x + p.y * p.y, d.w[row], tau);
}

// Exact Kerr/absorber flow over tau:
//   psi_out = psi_in e^{-w tau} exp(i gamma Theta),  Theta = M s,  s = |psi|^2 phi(w, tau).
template <typename T, int FB, int KMAX, bool DEC>
__global__ void __launch_bounds__(1024) k_kerr(DevOps<T> d, const typename CT<T>::C* psi_in,
                                               typename CT<T>::C* psi_out, const T* __restrict__ s, T tau,
                                               T gamma) {
  using C = typename CT<T>::C;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const C p = psi_in[idx];
  const T wv = d.w[row];
  T th = d.mdiag[row] * s[idx];
  if (DEC) {
    const int64_t FF = FB == 1 ? 1 : d.F;
    for_neighbours<KMAX>(d, d.mw, row, [&](int32_t q, T m) { th += m * s[int64_t(q) * FF + f]; });
  }
  const T damp = d_exp(-wv * tau);
  T sn, cs;
  d_sincos(gamma * th, &sn, &cs);
  C out;
  out.x = damp * (p.x * cs - p.y * sn);
  out.y = damp * (p.x * sn + p.y * cs);
  psi_out[idx] = out;
}

template <typename T, int FB>
__global__ void k_perm_in(DevOps<T> d, const int32_t* __restrict__ perm, const typename CT<T>::C* __restrict__ src,
                          typename CT<T>::C* __restrict__ dst, int scale_inv_h0) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const int64_t F = FB == 1 ? 1 : d.F;
  auto v = src[int64_t(perm[row]) * F + f];
  if (scale_inv_h0) {
    const T s = T(1.0 / d.h0[row]);
    v.x *= s;
    v.y *= s;
  }
  dst[idx] = v;
}

template <typename T, int FB>
__global__ void k_perm_out(DevOps<T> d, const int32_t* __restrict__ perm, const typename CT<T>::C* __restrict__ src,
                           typename CT<T>::C* __restrict__ dst, int scale_h0, int* flag) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int64_t row;
  int32_t f;
  split<FB>(idx, d, row, f);
  if (row >= d.n_rows) return;
  const int64_t F = FB == 1 ? 1 : d.F;
  auto v = src[idx];
  if (scale_h0) {
    const T s = T(d.h0[row]);
    v.x *= s;
    v.y *= s;
  }
  if (flag && !(d_finite(v.x) && d_finite(v.y))) atomicOr(flag, 1);
  dst[int64_t(perm[row]) * F + f] = v;
}

// Batched caller layout <-> device layout.  Device element (row, f) is
// row * F + f; the caller's is cbase[row] + f for the first fcount[row]
// fields of the row's mesh, and the device's further fields (padding up to F)
// are zero on the way in and dropped on the way out.
// fmaj: the device layout is field-major (field f of row r at f * n_rows + r).
template <typename T>
__global__ void k_bperm_in(int64_t n_rows, int32_t F, const int64_t* __restrict__ cbase,
                           const int32_t* __restrict__ fcount, const typename CT<T>::C* __restrict__ src,
                           typename CT<T>::C* __restrict__ dst, int fmaj) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n_rows * F) return;
  const int64_t row = idx / F;
  const int32_t f = int32_t(idx - row * F);
  typename CT<T>::C v;
  v.x = v.y = T(0);
  if (f < fcount[row]) v = src[cbase[row] + f];
  dst[fmaj ? int64_t(f) * n_rows + row : idx] = v;
}

template <typename T>
__global__ void k_bperm_out(int64_t n_rows, int32_t F, const int64_t* __restrict__ cbase,
                            const int32_t* __restrict__ fcount, const typename CT<T>::C* __restrict__ src,
                            typename CT<T>::C* __restrict__ dst, int* flag, int fmaj) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n_rows * F) return;
  const int64_t row = idx / F;
  const int32_t f = int32_t(idx - row * F);
  if (f >= fcount[row]) return;
  const auto v = src[fmaj ? int64_t(f) * n_rows + row : idx];
  if (!(d_finite(v.x) && d_finite(v.y))) atomicOr(flag, 1);
  dst[cbase[row] + f] = v;
}

template <typename T>
__global__ void k_fill(int64_t n, typename CT<T>::C* x, T re, T im) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  typename CT<T>::C v;
  v.x = re;
  v.y = im;
  x[i] = v;
}

template <typename T>
__global__ void k_copy(int64_t n, const typename CT<T>::C* __restrict__ src, typename CT<T>::C* __restrict__ dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = src[i];
}

// ---- deterministic FP64 block reduction of two values ----
constexpr int RED_BLOCK = 256;

__device__ inline void block_sum2(double& a, double& b, double* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[2 * wave] = a;
    sh[2 * wave + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < nw; ++k) {
      sa += sh[2 * k];
      sb += sh[2 * k + 1];
    }
    a = sa;
    b = sb;
  }
}

template <typename T, bool DEC>
__global__ void __launch_bounds__(RED_BLOCK) k_diag(DevOps<T> d, const typename CT<T>::C* __restrict__ psi, T gamma,
                                                    double* __restrict__ partials) {
  using C = typename CT<T>::C;
  __shared__ double sh[2 * (RED_BLOCK / 64)];
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double P = 0.0, E = 0.0;
  if (row < d.n_rows) {
    const C pr = psi[row];
    const T a = pr.x * pr.x + pr.y * pr.y;
    const int64_t info = d.sl_info[row >> 6];
    const int W = int(info & 0xff);
    const int64_t base = (info >> 8) + (row & 63);
    T lr = T(0), li = T(0), ma = d.mdiag[row] * a;
    for (int k = 0; k < W; ++k) {
      const int64_t e = base + int64_t(k) * 64;
      const C pq = psi[d.col[e]];
      const T c = d.lw[e];
      lr += c * (pr.x - pq.x);
      li += c * (pr.y - pq.y);
      if (DEC) ma += d.mw[e] * (pq.x * pq.x + pq.y * pq.y);
    }
    const double h0 = d.h0[row];
    P = h0 * double(a);
    E = h0 * (double(d.p1) * (double(pr.x) * lr + double(pr.y) * li) +
              double(d.beta4) * (double(lr) * lr + double(li) * li) - double(d.v[row]) * a -
              0.5 * double(gamma) * double(a) * double(ma));
  }
  block_sum2(P, E, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = P;
    partials[2 * blockIdx.x + 1] = E;
  }
}

template <typename T>
__global__ void __launch_bounds__(RED_BLOCK) k_overlap(int64_t n, const double* __restrict__ h0c,
                                                       const typename CT<T>::C* __restrict__ a,
                                                       const typename CT<T>::C* __restrict__ b,
                                                       double* __restrict__ partials) {
  __shared__ double sh[2 * (RED_BLOCK / 64)];
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double re = 0.0, im = 0.0;
  if (j < n) {
    const auto x = a[j];
    const auto y = b[j];
    const double h = h0c[j];
    re = h * (double(x.x) * y.x + double(x.y) * y.y);  // conj(a) b
    im = h * (double(x.x) * y.y - double(x.y) * y.x);
  }
  block_sum2(re, im, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = re;
    partials[2 * blockIdx.x + 1] = im;
  }
}

// Sums the per-block partials in a fixed order (one block).
__global__ void __launch_bounds__(RED_BLOCK) k_finish2(const double* __restrict__ partials, int n_blocks,
                                                       double* __restrict__ out) {
  __shared__ double sh[2 * (RED_BLOCK / 64)];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n_blocks; k += blockDim.x) {
    a += partials[2 * k];
    b += partials[2 * k + 1];
  }
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// ---- adjoint ----
template <typename T, int KMAX, bool B4>
__global__ void __launch_bounds__(1024) k_adj_stage(DevOps<T> d, const typename CT<T>::C* __restrict__ u_in,
                                                    const typename CT<T>::C* __restrict__ t,
                                                    typename CT<T>::C* __restrict__ u_out,
                                                    typename CT<T>::C* __restrict__ acc, int init,
                                                    const typename CT<T>::C* __restrict__ yf, T coef, double cdn,
                                                    double* __restrict__ gdn) {
  using C = typename CT<T>::C;
  const int64_t row = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  if (row >= d.n_rows) return;
  const C* __restrict__ g = B4 ? t : u_in;
  const C gr = g[row];
  const C ur = B4 ? u_in[row] : gr;
  const C yv = yf[row];
  const T vr = d.v[row];
  T ar = T(0), ai = T(0);
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const C gq = g[q];
    ar += c * (gr.x - gq.x);
    ai += c * (gr.y - gq.y);
  });
  T hr, hi;
  if (B4) {
    hr = d.p1 * gr.x + d.beta4 * ar - vr * ur.x;
    hi = d.p1 * gr.y + d.beta4 * ai - vr * ur.y;
  } else {
    hr = d.p1 * ar - vr * ur.x;
    hi = d.p1 * ai - vr * ur.y;
  }
  C uo;
  uo.x = coef * hi;
  uo.y = -coef * hr;
  if (u_out) u_out[row] = uo;
  C a0 = init ? ur : acc[row];
  a0.x += uo.x;
  a0.y += uo.y;
  acc[row] = a0;
  // Re(i conj(u) y) = -(u.x y.y - u.y y.x)
  gdn[row] += cdn * d.h0[row] * -(double(ur.x) * yv.y - double(ur.y) * yv.x);
}

template <typename T>
__global__ void k_adj_prep(DevOps<T> d, const typename CT<T>::C* __restrict__ psi_in,
                           const typename CT<T>::C* __restrict__ psi_out, const typename CT<T>::C* __restrict__ lam,
                           typename CT<T>::C* __restrict__ sm, T tau, T gamma) {
  const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (row >= d.n_rows) return;
  const auto pi = psi_in[row];
  const auto po = psi_out[row];
  const auto l = lam[row];
  typename CT<T>::C o;
  o.x = (pi.x * pi.x + pi.y * pi.y) * phi_w(d.w[row], tau);
  o.y = -gamma * (l.x * po.y - l.y * po.x);  // gamma Re(i conj(l) psi_out)
  sm[row] = o;
}

template <typename T, int KMAX, bool DEC>
__global__ void __launch_bounds__(1024) k_adj_kerr(DevOps<T> d, const typename CT<T>::C* __restrict__ psi_in,
                                                   const typename CT<T>::C* lam_out,
                                                   const typename CT<T>::C* __restrict__ sm,
                                                   typename CT<T>::C* lam_in, T tau, T gamma) {
  using C = typename CT<T>::C;
  const int64_t row = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  if (row >= d.n_rows) return;
  const C own = sm[row];
  const C l = lam_out[row];
  const C p = psi_in[row];
  const T wv = d.w[row];
  T th = d.mdiag[row] * own.x, mm = d.mdiag[row] * own.y;
  if (DEC)
    for_neighbours<KMAX>(d, d.mw, row, [&](int32_t q, T m) {
      const C v = sm[q];
      th += m * v.x;
      mm += m * v.y;
    });
  const T damp = d_exp(-wv * tau);
  T sn, cs;
  d_sincos(gamma * th, &sn, &cs);
  const T two_phi_mm = T(2) * phi_w(wv, tau) * mm;
  C o;
  o.x = damp * (cs * l.x + sn * l.y) + two_phi_mm * p.x;  // conj(E) l + 2 phi (M mu) psi
  o.y = damp * (cs * l.y - sn * l.x) + two_phi_mm * p.y;
  lam_in[row] = o;
}

template <typename T>
__global__ void k_hcombine(DevOps<T> d, const typename CT<T>::C* __restrict__ x,
                           const typename CT<T>::C* __restrict__ t, const typename CT<T>::C* __restrict__ t2,
                           typename CT<T>::C* __restrict__ y) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= d.n_rows * d.F) return;
  const int64_t row = idx / d.F;
  const auto xv = x[idx];
  const auto tv = t[idx];
  const T vr = d.v[row];
  typename CT<T>::C o;
  o.x = d.p1 * tv.x - vr * xv.x;
  o.y = d.p1 * tv.y - vr * xv.y;
  if (t2) {
    const auto t2v = t2[idx];
    o.x += d.beta4 * t2v.x;
    o.y += d.beta4 * t2v.y;
  }
  y[idx] = o;
}

template <typename T>
__global__ void k_set_v(int64_t n, const T* __restrict__ v0, const double* __restrict__ dn,
                        const int32_t* __restrict__ perm, T* __restrict__ v) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  v[r] = dn ? T(double(v0[r]) + dn[perm[r]]) : v0[r];
}

__global__ void k_gdn_out(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ g,
                          double* __restrict__ out) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  out[perm[r]] = g[r];
}

__global__ void k_zero_f64(int64_t n, double* x) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  x[r] = 0.0;
}

// ---- batched kernels: VF adjacent fields of one row per thread ----
// With many fields per row (field-minor layout) a thread owns VF consecutive
// fields, so every gather of a neighbour is one 32-byte vector load and the
// row's operator entries are fetched once per VF fields.
template <typename T, int VF>
struct alignas(sizeof(typename CT<T>::C) * VF) CVec {
  typename CT<T>::C v[VF];
};
template <typename T, int VF>
struct alignas(sizeof(T) * VF) RVec {
  T v[VF];
};

template <typename T, int VF>
__device__ inline void split_w(int64_t idx, const DevOps<T>& d, int64_t& row, int64_t& e0) {
  const int64_t per = d.F / VF;  // threads per row
  row = idx / per;
  e0 = row * d.F + (idx - row * per) * VF;  // first element of this thread
}

template <typename T, int VF, int KMAX, bool B4, bool WS>
__global__ void __launch_bounds__(1024) k_stage_w(DevOps<T> d, const typename CT<T>::C* __restrict__ x,
                                                  const typename CT<T>::C* __restrict__ t,
                                                  const typename CT<T>::C* psi, typename CT<T>::C* y, T coef,
                                                  T* __restrict__ s_out, T tau_s) {
  using V = CVec<T, VF>;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row, e0;
  split_w<T, VF>(idx, d, row, e0);
  if (row >= d.n_rows) return;
  const int64_t fo = e0 - row * d.F;  // field offset inside the row
  const auto* __restrict__ g = reinterpret_cast<const V*>(B4 ? t : x);
  const V gr = g[e0 / VF];
  const V xr = B4 ? reinterpret_cast<const V*>(x)[e0 / VF] : gr;
  const V p = reinterpret_cast<const V*>(psi)[e0 / VF];
  const T vr = d.v[row];
  T ar[VF], ai[VF];
#pragma unroll
  for (int f = 0; f < VF; ++f) ar[f] = ai[f] = T(0);
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const V gq = g[(int64_t(q) * d.F + fo) / VF];
#pragma unroll
    for (int f = 0; f < VF; ++f) {
      ar[f] += c * (gr.v[f].x - gq.v[f].x);
      ai[f] += c * (gr.v[f].y - gq.v[f].y);
    }
  });
  V out;
  RVec<T, VF> so;
  const T ph = WS ? phi_w(d.w[row], tau_s) : T(0);
#pragma unroll
  for (int f = 0; f < VF; ++f) {
    T hr, hi;
    if (B4) {
      hr = d.p1 * gr.v[f].x + d.beta4 * ar[f] - vr * xr.v[f].x;
      hi = d.p1 * gr.v[f].y + d.beta4 * ai[f] - vr * xr.v[f].y;
    } else {
      hr = d.p1 * ar[f] - vr * xr.v[f].x;
      hi = d.p1 * ai[f] - vr * xr.v[f].y;
    }
    out.v[f].x = p.v[f].x + coef * hi;
    out.v[f].y = p.v[f].y - coef * hr;
    so.v[f] = (out.v[f].x * out.v[f].x + out.v[f].y * out.v[f].y) * ph;
  }
  reinterpret_cast<V*>(y)[e0 / VF] = out;
  if (WS) reinterpret_cast<RVec<T, VF>*>(s_out)[e0 / VF] = so;
}

template <typename T, int VF, int KMAX>
__global__ void __launch_bounds__(1024) k_lap_w(DevOps<T> d, const typename CT<T>::C* __restrict__ x,
                                                typename CT<T>::C* __restrict__ t) {
  using V = CVec<T, VF>;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row, e0;
  split_w<T, VF>(idx, d, row, e0);
  if (row >= d.n_rows) return;
  const int64_t fo = e0 - row * d.F;
  const auto* __restrict__ g = reinterpret_cast<const V*>(x);
  const V xr = g[e0 / VF];
  V out;
#pragma unroll
  for (int f = 0; f < VF; ++f) out.v[f].x = out.v[f].y = T(0);
  for_neighbours<KMAX>(d, d.lw, row, [&](int32_t q, T c) {
    const V xq = g[(int64_t(q) * d.F + fo) / VF];
#pragma unroll
    for (int f = 0; f < VF; ++f) {
      out.v[f].x += c * (xr.v[f].x - xq.v[f].x);
      out.v[f].y += c * (xr.v[f].y - xq.v[f].y);
    }
  });
  reinterpret_cast<V*>(t)[e0 / VF] = out;
}

template <typename T, int VF>
__global__ void __launch_bounds__(1024) k_prep_w(DevOps<T> d, const typename CT<T>::C* __restrict__ psi,
                                                 T* __restrict__ s, T tau) {
  using V = CVec<T, VF>;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row, e0;
  split_w<T, VF>(idx, d, row, e0);
  if (row >= d.n_rows) return;
  const V p = reinterpret_cast<const V*>(psi)[e0 / VF];
  const T ph = phi_w(d.w[row], tau);
  RVec<T, VF> o;
#pragma unroll
  for (int f = 0; f < VF; ++f) o.v[f] = (p.v[f].x * p.v[f].x + p.v[f].y * p.v[f].y) * ph;
  reinterpret_cast<RVec<T, VF>*>(s)[e0 / VF] = o;
}

template <typename T, int VF, int KMAX, bool DEC>
__global__ void __launch_bounds__(1024) k_kerr_w(DevOps<T> d, const typename CT<T>::C* psi_in,
                                                 typename CT<T>::C* psi_out, const T* __restrict__ s, T tau,
                                                 T gamma) {
  using V = CVec<T, VF>;
  using R = RVec<T, VF>;
  const int64_t idx = logical_block(d.xcd_remap) * blockDim.x + threadIdx.x;
  int64_t row, e0;
  split_w<T, VF>(idx, d, row, e0);
  if (row >= d.n_rows) return;
  const int64_t fo = e0 - row * d.F;
  const auto* __restrict__ sv = reinterpret_cast<const R*>(s);
  const V p = reinterpret_cast<const V*>(psi_in)[e0 / VF];
  const R own = sv[e0 / VF];
  const T md = d.mdiag[row];
  T th[VF];
#pragma unroll
  for (int f = 0; f < VF; ++f) th[f] = md * own.v[f];
  if (DEC)
    for_neighbours<KMAX>(d, d.mw, row, [&](int32_t q, T m) {
      const R sq = sv[(int64_t(q) * d.F + fo) / VF];
#pragma unroll
      for (int f = 0; f < VF; ++f) th[f] += m * sq.v[f];
    });
  const T damp = d_exp(-d.w[row] * tau);
  V out;
#pragma unroll
  for (int f = 0; f < VF; ++f) {
    T sn, cs;
    d_sincos(gamma * th[f], &sn, &cs);
    out.v[f].x = damp * (p.v[f].x * cs - p.v[f].y * sn);
    out.v[f].y = damp * (p.v[f].x * sn + p.v[f].y * cs);
  }
  reinterpret_cast<V*>(psi_out)[e0 / VF] = out;
}

// ---- batched kernels on LDS tiles (one halo ring, all fields of every slot) ----
// A workgroup stages the gathered vector for its tile's rows and their
// one-ring halo in LDS (32 bytes of fields per thread), then every neighbour
// gather of its rows reads LDS instead of L2.
template <typename T, int VF, int KMAX, bool B4, bool WS>
__global__ void __launch_bounds__(1024) k_bstage(DevOps<T> d, TileOps<T> tl, const typename CT<T>::C* __restrict__ x,
                                                 const typename CT<T>::C* __restrict__ t,
                                                 const typename CT<T>::C* psi, typename CT<T>::C* y, T coef,
                                                 T* __restrict__ s_out, T tau_s) {
  static_assert(KMAX > 0, "tiled batched kernels need a bounded row width");
  using V = CVec<T, VF>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int32_t* hd = tl.hdr + 8 * tile;
  const int c0 = hd[0], c1 = c0 + hd[1];
  const int32_t* __restrict__ ext = tl.ext + hd[4];
  const int32_t* __restrict__ lsl = tl.lsl + hd[5];
  const int64_t ebase = tl.ent_base[tile];
  const int64_t row0 = tile * int64_t(tl.TS);
  const int tpr = d.F / VF;
  V* X = reinterpret_cast<V*>(smem);
  const auto* __restrict__ g = reinterpret_cast<const V*>(B4 ? t : x);
  // this thread's element (one per thread: the workgroup covers the tile's rows x fields)
  const int e = threadIdx.x;
  const bool mine = e < c0 * tpr;
  const int slot = e / tpr, fv = e - slot * tpr;
  const int64_t r = row0 + slot;
  V p, xr;
  T vr = T(0), ph = T(0);
  int W = 0;
  int qq[KMAX];
  T cc[KMAX];
  if (mine) {
    p = reinterpret_cast<const V*>(psi)[r * tpr + fv];
    if (B4) xr = reinterpret_cast<const V*>(x)[r * tpr + fv];
    vr = d.v[r];
    if (WS) ph = phi_w(d.w[r], tau_s);
    const int32_t info = lsl[slot >> 6];
    W = info & 0xff;
    const int64_t base = ebase + (info >> 8) + (slot & 63);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      qq[k] = k < W ? int(tl.lcol[base + 64 * k]) : 0;
      cc[k] = k < W ? tl.llw[base + 64 * k] : T(0);
    }
  }
  for (int i = threadIdx.x; i < c1 * tpr; i += blockDim.x) {
    const int sl = i / tpr, f = i - sl * tpr;
    const int64_t rr = sl < c0 ? row0 + sl : int64_t(ext[sl - c0]);
    X[i] = g[rr * tpr + f];
  }
  __syncthreads();
  if (!mine) return;
  const V gr = X[e];
  if (!B4) xr = gr;
  T ar[VF], ai[VF];
#pragma unroll
  for (int f = 0; f < VF; ++f) ar[f] = ai[f] = T(0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < W) {
      const V gq = X[qq[k] * tpr + fv];
#pragma unroll
      for (int f = 0; f < VF; ++f) {
        ar[f] += cc[k] * (gr.v[f].x - gq.v[f].x);
        ai[f] += cc[k] * (gr.v[f].y - gq.v[f].y);
      }
    }
  V out;
  RVec<T, VF> so;
#pragma unroll
  for (int f = 0; f < VF; ++f) {
    T hr, hi;
    if (B4) {
      hr = d.p1 * gr.v[f].x + d.beta4 * ar[f] - vr * xr.v[f].x;
      hi = d.p1 * gr.v[f].y + d.beta4 * ai[f] - vr * xr.v[f].y;
    } else {
      hr = d.p1 * ar[f] - vr * xr.v[f].x;
      hi = d.p1 * ai[f] - vr * xr.v[f].y;
    }
    out.v[f].x = p.v[f].x + coef * hi;
    out.v[f].y = p.v[f].y - coef * hr;
    so.v[f] = (out.v[f].x * out.v[f].x + out.v[f].y * out.v[f].y) * ph;
  }
  reinterpret_cast<V*>(y)[r * tpr + fv] = out;
  if (WS) reinterpret_cast<RVec<T, VF>*>(s_out)[r * tpr + fv] = so;
}

template <typename T, int VF, int KMAX>
__global__ void __launch_bounds__(1024) k_blap(DevOps<T> d, TileOps<T> tl, const typename CT<T>::C* __restrict__ x,
                                               typename CT<T>::C* __restrict__ t) {
  static_assert(KMAX > 0, "tiled batched kernels need a bounded row width");
  using V = CVec<T, VF>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int32_t* hd = tl.hdr + 8 * tile;
  const int c0 = hd[0], c1 = c0 + hd[1];
  const int32_t* __restrict__ ext = tl.ext + hd[4];
  const int32_t* __restrict__ lsl = tl.lsl + hd[5];
  const int64_t ebase = tl.ent_base[tile];
  const int64_t row0 = tile * int64_t(tl.TS);
  const int tpr = d.F / VF;
  V* X = reinterpret_cast<V*>(smem);
  const auto* __restrict__ g = reinterpret_cast<const V*>(x);
  const int e = threadIdx.x;
  const bool mine = e < c0 * tpr;
  const int slot = e / tpr, fv = e - slot * tpr;
  const int64_t r = row0 + slot;
  int W = 0;
  int qq[KMAX];
  T cc[KMAX];
  if (mine) {
    const int32_t info = lsl[slot >> 6];
    W = info & 0xff;
    const int64_t base = ebase + (info >> 8) + (slot & 63);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      qq[k] = k < W ? int(tl.lcol[base + 64 * k]) : 0;
      cc[k] = k < W ? tl.llw[base + 64 * k] : T(0);
    }
  }
  for (int i = threadIdx.x; i < c1 * tpr; i += blockDim.x) {
    const int sl = i / tpr, f = i - sl * tpr;
    const int64_t rr = sl < c0 ? row0 + sl : int64_t(ext[sl - c0]);
    X[i] = g[rr * tpr + f];
  }
  __syncthreads();
  if (!mine) return;
  const V xr = X[e];
  V out;
#pragma unroll
  for (int f = 0; f < VF; ++f) out.v[f].x = out.v[f].y = T(0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < W) {
      const V xq = X[qq[k] * tpr + fv];
#pragma unroll
      for (int f = 0; f < VF; ++f) {
        out.v[f].x += cc[k] * (xr.v[f].x - xq.v[f].x);
        out.v[f].y += cc[k] * (xr.v[f].y - xq.v[f].y);
      }
    }
  reinterpret_cast<V*>(t)[r * tpr + fv] = out;
}

template <typename T, int VF, int KMAX>
__global__ void __launch_bounds__(1024) k_bkerr(DevOps<T> d, TileOps<T> tl, const typename CT<T>::C* psi_in,
                                                typename CT<T>::C* psi_out, const T* __restrict__ s, T tau, T gamma) {
  using V = CVec<T, VF>;
  using R = RVec<T, VF>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int32_t* hd = tl.hdr + 8 * tile;
  const int c0 = hd[0], c1 = c0 + hd[1];
  const int32_t* __restrict__ ext = tl.ext + hd[4];
  const int32_t* __restrict__ lsl = tl.lsl + hd[5];
  const int64_t ebase = tl.ent_base[tile];
  const int64_t row0 = tile * int64_t(tl.TS);
  const int tpr = d.F / VF;
  R* S = reinterpret_cast<R*>(smem);
  const auto* __restrict__ sv = reinterpret_cast<const R*>(s);
  for (int e = threadIdx.x; e < c1 * tpr; e += blockDim.x) {
    const int slot = e / tpr, fv = e - slot * tpr;
    const int64_t r = slot < c0 ? row0 + slot : int64_t(ext[slot - c0]);
    S[e] = sv[r * tpr + fv];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < c0 * tpr; e += blockDim.x) {
    const int slot = e / tpr, fv = e - slot * tpr;
    const int64_t r = row0 + slot;
    const V p = reinterpret_cast<const V*>(psi_in)[r * tpr + fv];
    const R own = S[e];
    const T md = d.mdiag[r];
    T th[VF];
#pragma unroll
    for (int f = 0; f < VF; ++f) th[f] = md * own.v[f];
    const int32_t info = lsl[slot >> 6];
    const int W = info & 0xff;
    const int64_t base = ebase + (info >> 8) + (slot & 63);
    if constexpr (KMAX > 0) {
      int qq[KMAX];
      T mm[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        qq[k] = k < W ? int(tl.lcol[base + 64 * k]) : 0;
        mm[k] = k < W ? tl.lmw[base + 64 * k] : T(0);
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k < W) {
          const R sq = S[qq[k] * tpr + fv];
#pragma unroll
          for (int f = 0; f < VF; ++f) th[f] += mm[k] * sq.v[f];
        }
    } else {
      for (int k = 0; k < W; ++k) {
        const R sq = S[int(tl.lcol[base + 64 * k]) * tpr + fv];
        const T m = tl.lmw[base + 64 * k];
#pragma unroll
        for (int f = 0; f < VF; ++f) th[f] += m * sq.v[f];
      }
    }
    const T damp = d_exp(-d.w[r] * tau);
    V out;
#pragma unroll
    for (int f = 0; f < VF; ++f) {
      T sn, cs;
      d_sincos(gamma * th[f], &sn, &cs);
      out.v[f].x = damp * (p.v[f].x * cs - p.v[f].y * sn);
      out.v[f].y = damp * (p.v[f].x * sn + p.v[f].y * cs);
    }
    reinterpret_cast<V*>(psi_out)[r * tpr + fv] = out;
  }
}

// ---- fused z-step kernels on LDS tiles ----
// One workgroup per tile.  The tile's rows and halo rings are staged in LDS;
// each stage of the kind is computed on the rings it needs, separated by
// workgroup barriers only.  Thread j of the workgroup owns slots j, j + B, ...
// (at most J of them) in every phase, and loads their operator rows (indices,
// L and M weights) and per-row scalars into registers once, while the field
// values are being staged, so the phases after the first barrier touch only
// LDS and registers.
template <typename T, int KMAX, bool DEC, int KIND, int J>
__global__ void __launch_bounds__(1024) k_fused(DevOps<T> d, TileOps<T> tl, const typename CT<T>::C* __restrict__ in_x,
                                                const typename CT<T>::C* __restrict__ in_psi,
                                                typename CT<T>::C* __restrict__ out_psi,
                                                typename CT<T>::C* __restrict__ out_y,
                                                typename CT<T>::C* __restrict__ out_rec, T h, T tau, T gamma) {
  using C = typename CT<T>::C;
  static_assert(KMAX > 0, "fused kernels need a bounded row width");
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;  // whole workgroup leaves together
  const int32_t* hd = tl.hdr + 8 * tile;
  const int c0 = hd[0], c1 = c0 + hd[1], c2 = c1 + hd[2], c3 = c2 + hd[3];
  const int32_t* __restrict__ ext = tl.ext + hd[4];
  const int32_t* __restrict__ lsl = tl.lsl + hd[5];
  const int64_t ebase = tl.ent_base[tile];
  const int64_t row0 = tile * int64_t(tl.TS);
  const int MS = tl.max_slots;
  const int B = blockDim.x;
  C* X = reinterpret_cast<C*>(smem);
  C* P = X + MS;
  C* Y = P + MS;
  T* S = reinterpret_cast<T*>(Y + MS);
  // ring extents (a triangle-averaged Kerr step gathers one ring, a lumped one none)
  int nX = 0, nP = 0, nA = 0;
  if (KIND == FUSED_S4_NL_S1) {
    nA = DEC ? c2 : c1;  // rows of stage 4
    nX = DEC ? c3 : c2;
    nP = nA;
  } else if (KIND == FUSED_S2_S3) {
    nA = c1;
    nX = c2;
    nP = c1;
  } else if (KIND == FUSED_NL_S1) {
    nA = c1;
    nP = DEC ? c2 : c1;
  } else {  // FUSED_S4_NL
    nA = DEC ? c1 : c0;
    nX = DEC ? c2 : c1;
    nP = nA;
  }
  const int nLoad = nX > nP ? nX : nP;
  // stage the field values of every slot
  for (int i = threadIdx.x; i < nLoad; i += B) {
    const int32_t r = i < c0 ? int32_t(row0 + i) : ext[i - c0];
    if (i < nX) X[i] = in_x[r];
    if (i < nP) {
      const C p = in_psi[r];
      P[i] = p;
      if (KIND == FUSED_NL_S1) S[i] = nl_int(d, p.x * p.x + p.y * p.y, d.w[r], tau);
    }
  }
  // registers: the operator rows of this thread's compute slots (all phases use prefixes of [0, nA))
  int q[J][KMAX];
  T cl[J][KMAX];
  T cm[J][DEC ? KMAX : 1];
  int wd[J];
  int32_t rr[J];
  T vv[J], ww[J], md[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + j * B;
    wd[j] = 0;
    rr[j] = 0;
    vv[j] = ww[j] = md[j] = T(0);
    if (i < nA) {
      const int32_t r = i < c0 ? int32_t(row0 + i) : ext[i - c0];
      rr[j] = r;
      vv[j] = d.v[r];
      ww[j] = d.w[r];
      md[j] = d.mdiag[r];
      const int32_t info = lsl[i >> 6];
      wd[j] = info & 0xff;
      const int64_t base = ebase + (info >> 8) + (i & 63);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < wd[j]) {
          q[j][k] = tl.lcol[base + 64 * k];
          cl[j][k] = tl.llw[base + 64 * k];
          if (DEC) cm[j][k] = tl.lmw[base + 64 * k];
        } else {
          q[j][k] = i;
          cl[j][k] = T(0);
          if (DEC) cm[j][k] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        q[j][k] = 0;
        cl[j][k] = T(0);
        if (DEC) cm[j][k] = T(0);
      }
    }
  }
  __syncthreads();

  // base + coef * (-i) (p1 L v - V v) for register slot j (slot index i), v gathered from V_
  auto stage = [&](const C* V_, const C* base_, int j, int i, T coef) {
    const C vr = V_[i];
    T ar = T(0), ai = T(0);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      {  // padded slots: self column, zero weight
        const C vq = V_[q[j][k]];
        ar += cl[j][k] * (vr.x - vq.x);
        ai += cl[j][k] * (vr.y - vq.y);
      }
    const T hr = d.p1 * ar - vv[j] * vr.x;
    const T hi = d.p1 * ai - vv[j] * vr.y;
    const C b = base_[i];
    C o;
    o.x = b.x + coef * hi;
    o.y = b.y - coef * hr;
    return o;
  };
  // exact Kerr/absorber flow of register slot j of Src, reading |psi|^2 phi from S
  auto kerr = [&](const C* Src, int j, int i) {
    T th = md[j] * S[i];
    if (DEC) {
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        th += cm[j][k] * S[q[j][k]];
    }
    const T damp = d_exp(-ww[j] * tau);
    T sn, cs;
    d_sincos(gamma * th, &sn, &cs);
    const C p = Src[i];
    C o;
    o.x = damp * (p.x * cs - p.y * sn);
    o.y = damp * (p.x * sn + p.y * cs);
    return o;
  };

  if (KIND == FUSED_S4_NL_S1 || KIND == FUSED_S4_NL) {
#pragma unroll
    for (int j = 0; j < J; ++j) {  // stage 4: psi_new = psi + h A y3
      const int i = threadIdx.x + j * B;
      if (i < nA) {
        const C o = stage(X, P, j, i, h);
        Y[i] = o;
        S[i] = nl_int(d, o.x * o.x + o.y * o.y, ww[j], tau);
        if (out_rec && i < c0) out_rec[rr[j]] = o;  // state before the Kerr substep (adjoint recompute)
      }
    }
    __syncthreads();
    const int nNL = KIND == FUSED_S4_NL ? c0 : c1;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        const C o = kerr(Y, j, i);
        if (KIND == FUSED_S4_NL_S1) X[i] = o;
        if (i < c0) out_psi[rr[j]] = o;
      }
    }
    if (KIND == FUSED_S4_NL_S1) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = threadIdx.x + j * B;
        if (i < c0) out_y[rr[j]] = stage(X, X, j, i, T(0.25) * h);
      }
    }
  } else if (KIND == FUSED_NL_S1) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < c1) {
        const C o = kerr(P, j, i);
        X[i] = o;
        if (i < c0) out_psi[rr[j]] = o;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < c0) out_y[rr[j]] = stage(X, X, j, i, T(0.25) * h);
    }
  } else {  // FUSED_S2_S3
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < c1) {
        const C o = stage(X, P, j, i, h / T(3));
        Y[i] = o;
        if (out_rec && i < c0) out_rec[rr[j]] = o;  // y2 (adjoint recompute)
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < c0) out_y[rr[j]] = stage(Y, P, j, i, T(0.5) * h);
    }
  }
}

// ---- one kernel per z step on LDS tiles with five halo rings ----
// The whole merged Strang step, LIN(h) then NL(tau): the four Horner stages
// of RK4 and the Kerr/absorber flow, on a tile whose halo is wide enough for
// every stage (stage k on rings 0..4-k; the triangle-averaged Kerr step of
// ring 0 needs stage 4 on ring 1).  Input: the state after the previous
// Kerr substep; output: the state after this one (owned rows).
// LDS array of complex values for the tile kernels, interleaved: one 8- or
// 16-byte access per element.  (Split real and imaginary planes, two narrower
// accesses per gather, measured about 20% slower in the step kernels.)
template <typename T>
struct CplxAoS {
  using C = typename CT<T>::C;
  C* p;
  __device__ C get(int i) const { return p[i]; }
  __device__ void put(int i, const C& v) const { p[i] = v; }
  // the element at byte offset off (a neighbour slot held pre-scaled)
  __device__ C get_b(int off) const { return *reinterpret_cast<const C*>(reinterpret_cast<const char*>(p) + off); }
};

// Fixed LDS layout of the complex64 persistent split step (template flag FX):
// the per-slot buffers sit at constant offsets of kFixSlots slots each in
// static LDS, and the neighbour slots are held as byte offsets (StepTile BO),
// so that every gather carries its buffer's offset in the LDS instruction
// instead of an address computed per neighbour.  For tiles of at most
// kFixSlots slots; two workgroups with four such buffers fit one compute
// unit's LDS.  (The one-kernel step, its adjoint pair and the batched field
// loop measured no faster with it, so they keep the runtime-sized layout.)
constexpr int kFixSlots = 2432;

// DEC_BPM_FIXED_LDS=0 keeps the runtime-sized LDS layout everywhere (read once
// per process).
static bool fixed_lds_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("DEC_BPM_FIXED_LDS");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Whether a complex64 tile set takes the fixed layout.
template <typename T>
static bool fixed_lds(const TileOps<T>& tl) {
  return sizeof(T) == 4 && tl.max_slots <= kFixSlots && fixed_lds_enabled();
}
// Threads per workgroup the step-tile kernels are compiled for.  With two
// compute slots per thread the complex128 kernels hold twice the operator
// registers of the complex64 ones, so their workgroups are capped at 640
// threads (up to 170 VGPRs per lane instead of 128; no spills).  The
// persistent kernel keeps the 1024 bound: there, keeping every tile resident
// (more waves per CU) matters more than the spills.
struct NoHook {
  __device__ void operator()() const {}
};

template <typename T, int J>
struct StepBound {
  static constexpr int value = (sizeof(T) == 8 && J >= 2) ? 640 : 1024;
};

// One tile of the one-kernel z step: the operator rows of its compute slots
// in registers (J slots per thread), the LIN(h) stages in Horner form on the
// LDS-staged state, then the Kerr/absorber flow over tau on the owned rows.
// Rings: the state is staged on rings 0..4+o (o = 1 for the triangle-averaged
// Kerr gather, 0 for the lumped one), each stage shrinks the valid region by
// one ring.  Tiles use the step layout: every slot listed at a fixed per-tile
// stride, rings sorted by degree so that the width of a 64-slot slice (one
// wavefront) is nearly every row's degree; the neighbour loops run to that
// wave-uniform width, padded entries pointing at their own slot with weight 0.
// CL: the L weights are complex (a perfectly matched layer stretches the
// Hodge stars); their imaginary parts ride in a second register array.
// LM: the M weights of the owned slots sit in LDS (TS x KP words, entry k of
// slot i at i * KP + k with the odd row length KP = KMAX | 1, so that the 64
// lanes of a wave reading entry k hit distinct banks and each entry is an
// immediate offset from one address per slot) instead of registers, for
// kernels that hold more per-slot state than the register file leaves room for.
template <typename T, int KMAX, bool DEC, int J, bool CL = false, bool LM = false, bool BO = false>
struct StepTile {
  using C = typename CT<T>::C;
  // BO: neighbour slots held as byte offsets into a complex LDS buffer
  // (slot * sizeof(C)) and the real per-slot buffer S laid out at the same
  // stride, so that with buffers at constant LDS offsets a gather needs no
  // address arithmetic (the offset goes into the LDS instruction)
  static constexpr int QSC = BO ? int(sizeof(C)) : 1;
  static constexpr int SST = BO ? 2 : 1;  // elements of T per S slot
  int nLoad, n1, n2, n3, n4, nNL;
  const int32_t* hd;
  const int32_t* ext;
  int q[J][KMAX];  // neighbour slots
  T cl[J][KMAX];
  T cli[J][CL ? KMAX : 1];
  T cm[J][(DEC && !LM) ? KMAX : 1];
  T* cml;  // LM: the LDS table of the M weights
  static constexpr int KP = KMAX | 1;
  int wd[J];  // slice width (wave-uniform)
  int32_t rr[J];
  T vv[J], ww[J], md[J];
  uint32_t dpk;  // depth of each register slot's row, 8 bits per slot (split step only)

  __device__ int32_t slot_row(int i) const { return ext[i]; }
  __device__ int nb(int j, int k) const { return q[j][k]; }

  // kerr_only: load the rows the NL substep alone needs (rings 0..1, the
  // reach of the M gather), not every compute slot's
  // m_lds (LM): where the M weight table goes; it is read after the caller's next barrier.
  // m_owned: only the owned slots get M weights and M_pp (the split step's Kerr
  // substep runs on them alone; the unsplit kernels gather M on the halo too)
  __device__ void init(const DevOps<T>& d, const TileOps<T>& tl, int64_t tile, bool kerr_only = false,
                       T* m_lds = nullptr, bool m_owned = false) {
    cml = m_lds;
    hd = tl.hdr + int64_t(tl.hdr_stride) * tile;  // hd[k]: slots in rings 0..k; hd[15]: rings
    ext = tl.ext + tile * int64_t(tl.ext_stride);
    const int32_t* __restrict__ lsl = tl.lsl + tile * int64_t(tl.lsl_stride);
    const int64_t ebase = tl.ent_base[tile];
    const int R = hd[15];
    nLoad = hd[R];
    n1 = hd[R - 1];  // slots with operator rows
    n2 = hd[R - 2];
    n3 = hd[R - 3];
    n4 = hd[R - 4];
    nNL = hd[0];
    const int nRows = kerr_only ? hd[1] : n1;
    const int B = blockDim.x;
    dpk = 0;
    if (tl.dep != nullptr) {
      const uint8_t* dp = tl.dep + tile * int64_t(tl.ext_stride);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = threadIdx.x + j * B;
        if (i < nNL) dpk |= uint32_t(dp[i]) << (8 * j);
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      rr[j] = 0;
      vv[j] = ww[j] = md[j] = T(0);
      int w = 0;
      int64_t base = 0;
      if (i < nRows) {
        const int32_t r = ext[i];
        rr[j] = r;
        vv[j] = d.v[r];
        ww[j] = d.w[r];
        if (!m_owned || i < nNL) md[j] = d.mdiag[r];
        const int32_t info = lsl[i >> 6];
        w = info & 0xff;
        base = ebase + (info >> 8) + (i & 63);
      }
      // lanes past n1 in a wave whose slice starts below n1 read the same slice word
      wd[j] = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < w) {
          q[j][k] = tl.lcol[base + 64 * k] * QSC;
          cl[j][k] = tl.llw[base + 64 * k];
          if constexpr (DEC && LM) {
            if (i < nNL) cml[i * KP + k] = tl.lmw[base + 64 * k];
          } else if constexpr (DEC) {
            cm[j][k] = (!m_owned || i < nNL) ? tl.lmw[base + 64 * k] : T(0);
          }
          if constexpr (CL) cli[j][k] = tl.llwi[base + 64 * k];
        } else {
          q[j][k] = (i < n1 ? i : 0) * QSC;
          cl[j][k] = T(0);
          if constexpr (DEC && !LM) cm[j][k] = T(0);
          if constexpr (CL) cli[j][k] = T(0);
        }
      }
    }
  }

  // Conjugates the complex L weights held in registers (CL): the adjoint of a
  // complex-stretched L in the conj(H0~)^{-1} g variables applies conj(L).
  __device__ void conj_l() {
    if constexpr (CL) {
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int k = 0; k < KMAX; ++k) cli[j][k] = -cli[j][k];
    }
  }

  // M weight k of register slot j (an owned slot when LM)
  __device__ T mw(int j, int k) const {
    if constexpr (LM)
      return cml[(int(threadIdx.x) + j * int(blockDim.x)) * KP + k];
    else
      return cm[j][k];
  }

  // Tells the compiler the neighbour slots may change here, so that a loop
  // over z steps recomputes their LDS addresses in each phase instead of
  // keeping one address per (neighbour, phase buffer) live across the loop.
  __device__ void opaque_neighbours() {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int k = 0; k < KMAX; ++k) asm volatile("" : "+v"(q[j][k]));
  }

  // sum_k c_k (vr - V_[q_k]) over the first N entries of register slot j
  template <int N, typename V>
  __device__ void lsum_n(const V& V_, int j, const C& vr, T& ar, T& ai) const {
    C vq[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if constexpr (BO)
        vq[k] = V_.get_b(nb(j, k));
      else
        vq[k] = V_.get(nb(j, k));
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const T dx = vr.x - vq[k].x, dy = vr.y - vq[k].y;
      if constexpr (CL) {  // (cl + i cli) (dx + i dy)
        ar += cl[j][k] * dx - cli[j][k] * dy;
        ai += cl[j][k] * dy + cli[j][k] * dx;
      } else {
        ar += cl[j][k] * dx;
        ai += cl[j][k] * dy;
      }
    }
  }
  template <int N, typename V>
  __device__ void lsum_w(int W, const V& V_, int j, const C& vr, T& ar, T& ai) const {
    if constexpr (N > 0) {
      if (W == N) {
        lsum_n<N>(V_, j, vr, ar, ai);
        return;
      }
      lsum_w<N - 1>(W, V_, j, vr, ar, ai);
    }
  }
  // th + sum_k m_k S[q_k] over the first N entries of register slot j
  template <int N>
  __device__ T msum_n(const T* S, int j, T th) const {
    T sq[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if constexpr (BO)
        sq[k] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(S) + nb(j, k));
      else
        sq[k] = S[nb(j, k)];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) th += mw(j, k) * sq[k];
    return th;
  }
  template <int N>
  __device__ T msum_w(int W, const T* S, int j, T th) const {
    if constexpr (N > 0) {
      if (W == N) return msum_n<N>(S, j, th);
      return msum_w<N - 1>(W, S, j, th);
    } else {
      return th;
    }
  }

  // (th, mm) + sum_k m_k (SM[q_k].x, SM[q_k].y) over the first N entries of register slot j
  template <int N>
  __device__ void msum2_n(const C* SM, int j, T& th, T& mm) const {
    C sq[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if constexpr (BO)
        sq[k] = *reinterpret_cast<const C*>(reinterpret_cast<const char*>(SM) + nb(j, k));
      else
        sq[k] = SM[nb(j, k)];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      th += mw(j, k) * sq[k].x;
      mm += mw(j, k) * sq[k].y;
    }
  }
  template <int N>
  __device__ void msum2_w(int W, const C* SM, int j, T& th, T& mm) const {
    if constexpr (N > 0) {
      if (W == N) {
        msum2_n<N>(SM, j, th, mm);
        return;
      }
      msum2_w<N - 1>(W, SM, j, th, mm);
    }
  }

  // coef * (-i) (p1 L v - V v) at register slot j (own value vr, neighbours from V_)
  template <typename V>
  __device__ C link(const DevOps<T>& d, const V& V_, const C& vr, int j, T coef) const {
    T ar = T(0), ai = T(0);
    lsum_w<KMAX>(wd[j], V_, j, vr, ar, ai);
    const T hr = d.p1 * ar - vv[j] * vr.x;
    const T hi = d.p1 * ai - vv[j] * vr.y;
    C o;
    o.x = coef * hi;
    o.y = -coef * hr;
    return o;
  }

  // base + coef * (-i) (p1 L v - V v) at register slot j: the slot's own value
  // vr and base come from registers, only the neighbours are gathered from V_
  template <typename V>
  __device__ C stage(const DevOps<T>& d, const V& V_, const C& vr, const C& base, int j, T coef) const {
    T ar = T(0), ai = T(0);
    lsum_w<KMAX>(wd[j], V_, j, vr, ar, ai);
    const T hr = d.p1 * ar - vv[j] * vr.x;
    const T hi = d.p1 * ai - vv[j] * vr.y;
    C r;
    r.x = base.x + coef * hi;
    r.y = base.y - coef * hr;
    return r;
  }

  // LIN(h) then NL(tau) of the state staged in P (slots < nLoad); X, Y, S are
  // LDS scratch of the same slot count.  Calls out(slot, r, value) for every
  // owned row r (P is no longer read by then), and rec(k, r, value) with the stage vectors y1, y2, y3 (k = 0..2)
  // and the state before the Kerr substep (k = 3) of every owned row.  Every
  // thread of the workgroup must call it (it holds barriers).  A thread keeps
  // the values of its own slots (the state, the latest stage, |b|^2 phi) in
  // registers; LDS serves the neighbour gathers only.
  // after_p() runs once P is no longer read (after the first barrier): a
  // caller may start refilling P from there.  before_nl() runs before the
  // barrier that opens the Kerr phase: what it writes to P is visible to
  // every thread after that barrier.
  template <typename V, typename Out, typename Rec, typename AfterP = NoHook, typename BeforeNL = NoHook>
  __device__ void step(const DevOps<T>& d, const V& P, const V& X, const V& Y, T* S, T h, T tau, T gamma, Out out,
                       Rec rec, AfterP after_p = AfterP(), BeforeNL before_nl = BeforeNL()) const {
    const int B = blockDim.x;
    C p[J], cur[J];
    T so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n1) {
        p[j] = P.get(i);
        cur[j] = stage(d, P, p[j], p[j], j, T(0.25) * h);  // y1
        Y.put(i, cur[j]);
        if (i < nNL) rec(0, rr[j], cur[j]);
      }
    }
    __syncthreads();
    after_p();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n2) {
        cur[j] = stage(d, Y, cur[j], p[j], j, h / T(3));  // y2
        X.put(i, cur[j]);
        if (i < nNL) rec(1, rr[j], cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n3) {
        cur[j] = stage(d, X, cur[j], p[j], j, T(0.5) * h);  // y3
        Y.put(i, cur[j]);
        if (i < nNL) rec(2, rr[j], cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n4) {  // state before the Kerr substep
        cur[j] = stage(d, Y, cur[j], p[j], j, h);
        so[j] = nl_int(d, cur[j].x * cur[j].x + cur[j].y * cur[j].y, ww[j], tau);
        S[i * SST] = so[j];
        if (i < nNL) rec(3, rr[j], cur[j]);
      }
    }
    before_nl();
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        T th = md[j] * so[j];
        if constexpr (DEC) th = msum_w<KMAX>(wd[j], S, j, th);
        const T damp = d_exp(-ww[j] * tau);
        T sn, cs;
        d_sincos(gamma * th, &sn, &cs);
        const C b = cur[j];
        C r;
        r.x = damp * (b.x * cs - b.y * sn);
        r.y = damp * (b.x * sn + b.y * cs);
        out(i, rr[j], r);
      }
    }
  }

  // The z step split around the neighbour wait of the persistent launch.
  // Before mid(), every stage is computed on the owned slots whose inputs are
  // owned rows of the previous state: stage k (k = 1..4) where the row's
  // distance to the nearest row the tile does not own is at least k + 1, the
  // Kerr flow where it is at least 6 (5 for the lumped form, whose gather is
  // the row itself).  mid() waits for the neighbour tiles and stages the halo
  // (false: the wait gave up, the step is abandoned).  After it, every other
  // slot.  Per slot the operations and their order are those of step(), so
  // the result is the same.  out_deep(slot, row, value) receives the owned
  // rows finished before the wait (no other tile reads them: their distance
  // exceeds the five halo rings), out(slot, row, value) the rest.
  template <typename V, typename OutDeep, typename Out, typename Mid>
  __device__ bool step_split(const DevOps<T>& d, const V& P, const V& X, const V& Y, T* S, T h, T tau, T gamma,
                             OutDeep out_deep, Out out, Mid mid) const {
    const int B = blockDim.x;
    constexpr int KD = DEC ? 6 : 5;
    C p[J], cur[J];
    T so[J];
    auto early = [&](int i, int j, int lim) { return i < nNL && int((dpk >> (8 * j)) & 0xffu) >= lim; };
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (early(i, j, 2)) {
        p[j] = P.get(i);
        cur[j] = stage(d, P, p[j], p[j], j, T(0.25) * h);  // y1
        Y.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (early(i, j, 3)) {
        cur[j] = stage(d, Y, cur[j], p[j], j, h / T(3));  // y2
        X.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (early(i, j, 4)) {
        cur[j] = stage(d, X, cur[j], p[j], j, T(0.5) * h);  // y3
        Y.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (early(i, j, 5)) {  // state before the Kerr substep
        cur[j] = stage(d, Y, cur[j], p[j], j, h);
        so[j] = nl_int(d, cur[j].x * cur[j].x + cur[j].y * cur[j].y, ww[j], tau);
        S[i * SST] = so[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (early(i, j, KD)) out_deep(i, rr[j], kerr_of(d, S, j, cur[j], so[j], tau, gamma));
    }
    if (!mid()) return false;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n1 && !early(i, j, 2)) {
        p[j] = P.get(i);
        cur[j] = stage(d, P, p[j], p[j], j, T(0.25) * h);  // y1
        Y.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n2 && !early(i, j, 3)) {
        cur[j] = stage(d, Y, cur[j], p[j], j, h / T(3));  // y2
        X.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n3 && !early(i, j, 4)) {
        cur[j] = stage(d, X, cur[j], p[j], j, T(0.5) * h);  // y3
        Y.put(i, cur[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n4 && !early(i, j, 5)) {
        cur[j] = stage(d, Y, cur[j], p[j], j, h);
        so[j] = nl_int(d, cur[j].x * cur[j].x + cur[j].y * cur[j].y, ww[j], tau);
        S[i * SST] = so[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL && !early(i, j, KD)) out(i, rr[j], kerr_of(d, S, j, cur[j], so[j], tau, gamma));
    }
    return true;
  }

  // The Kerr/absorber flow of register slot j (state b, its |b|^2 phi in so),
  // the neighbours' |.|^2 phi from S: step()'s last phase for one slot.
  __device__ C kerr_of(const DevOps<T>& d, const T* S, int j, const C& b, T so_j, T tau, T gamma) const {
    T th = md[j] * so_j;
    if constexpr (DEC) th = msum_w<KMAX>(wd[j], S, j, th);
    const T damp = d_exp(-ww[j] * tau);
    T sn, cs;
    d_sincos(gamma * th, &sn, &cs);
    C r;
    r.x = damp * (b.x * cs - b.y * sn);
    r.y = damp * (b.x * sn + b.y * cs);
    return r;
  }

  // NL(tau) alone of a field held in the caller's vertex order (row r at
  // src[perm[r]]; device order if perm is null), for the owned rows: |psi|^2 phi(w, tau) is staged in S on
  // rings 0..1 (the reach of the M gather; ring 0 for the lumped form), then
  // out(slot, r, value) receives each owned row's result.  Every thread of the
  // workgroup must call it (it holds a barrier).
  template <typename Out>
  __device__ void kerr_from(const DevOps<T>& d, const C* __restrict__ src, const int32_t* __restrict__ perm, T* S,
                            T tau, T gamma, Out out) const {
    const int B = blockDim.x;
    const int nS = DEC ? hd[1] : nNL;
    C p[J];
    T so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nS) {
        p[j] = src[perm ? perm[rr[j]] : rr[j]];
        so[j] = nl_int(d, p[j].x * p[j].x + p[j].y * p[j].y, ww[j], tau);
        S[i * SST] = so[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        T th = md[j] * so[j];
        if constexpr (DEC) th = msum_w<KMAX>(wd[j], S, j, th);
        const T damp = d_exp(-ww[j] * tau);
        T sn, cs;
        d_sincos(gamma * th, &sn, &cs);
        C r;
        r.x = damp * (p[j].x * cs - p[j].y * sn);
        r.y = damp * (p[j].x * sn + p[j].y * cs);
        out(i, rr[j], r);
      }
    }
  }

  // The same z step with the beta4 L^2 term: H v = p1 L v + beta4 L(L v) - V v.
  // Each stage takes two gather phases (t = L v into T, then L t), so the
  // state is staged on 8 halo rings (9 with the triangle-averaged Kerr
  // gather) and each stage shrinks the valid region by two rings.
  template <typename V, typename Out>
  __device__ void step_b4(const DevOps<T>& d, const V& P, const V& X, const V& Y, const V& Tb, T* S, T h, T tau,
                          T gamma, Out out) const {
    const int B = blockDim.x;
    const int R = hd[15];
    C p[J], cur[J], tl[J];
    T so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n1) {
        p[j] = P.get(i);
        cur[j] = p[j];
      }
    }
    const T coefs[4] = {T(0.25) * h, h / T(3), T(0.5) * h, h};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const V& Vin = k == 0 ? P : ((k & 1) ? Y : X);  // y1 -> Y, y2 -> X, y3 -> Y
      const V& Vout = (k & 1) ? X : Y;
      const int na = hd[R - 1 - 2 * k], nb_ = hd[R - 2 - 2 * k];
#pragma unroll
      for (int j = 0; j < J; ++j) {  // t = L v
        const int i = threadIdx.x + j * B;
        if (i < na) {
          T ar = T(0), ai = T(0);
          lsum_w<KMAX>(wd[j], Vin, j, cur[j], ar, ai);
          tl[j].x = ar;
          tl[j].y = ai;
          Tb.put(i, tl[j]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < J; ++j) {  // y = p + coef (-i) (p1 t + beta4 L t - V v)
        const int i = threadIdx.x + j * B;
        if (i < nb_) {
          T ar = T(0), ai = T(0);
          lsum_w<KMAX>(wd[j], Tb, j, tl[j], ar, ai);
          const T hr = d.p1 * tl[j].x + d.beta4 * ar - vv[j] * cur[j].x;
          const T hi = d.p1 * tl[j].y + d.beta4 * ai - vv[j] * cur[j].y;
          C y;
          y.x = p[j].x + coefs[k] * hi;
          y.y = p[j].y - coefs[k] * hr;
          cur[j] = y;
          if (k < 3) Vout.put(i, y);
          else {
            so[j] = nl_int(d, y.x * y.x + y.y * y.y, ww[j], tau);
            S[i * SST] = so[j];
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        T th = md[j] * so[j];
        if constexpr (DEC) th = msum_w<KMAX>(wd[j], S, j, th);
        const T damp = d_exp(-ww[j] * tau);
        T sn, cs;
        d_sincos(gamma * th, &sn, &cs);
        const C b = cur[j];
        C r;
        r.x = damp * (b.x * cs - b.y * sn);
        r.y = damp * (b.x * sn + b.y * cs);
        out(i, rr[j], r);
      }
    }
  }

  // ---- VF fields per slot (batched handles: the fields of a row are contiguous) ----
  // sum_k c_k (vr - V_[q_k]) over the first N entries of register slot j, per field
  template <int N, int VF>
  __device__ void lsumv_n(const CVec<T, VF>* V_, int j, const CVec<T, VF>& vr, T* ar, T* ai) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const CVec<T, VF> vq = V_[nb(j, k)];
#pragma unroll
      for (int f = 0; f < VF; ++f) {
        ar[f] += cl[j][k] * (vr.v[f].x - vq.v[f].x);
        ai[f] += cl[j][k] * (vr.v[f].y - vq.v[f].y);
      }
    }
  }
  template <int N, int VF>
  __device__ void lsumv_w(int W, const CVec<T, VF>* V_, int j, const CVec<T, VF>& vr, T* ar, T* ai) const {
    if constexpr (N > 0) {
      if (W == N) {
        lsumv_n<N>(V_, j, vr, ar, ai);
        return;
      }
      lsumv_w<N - 1>(W, V_, j, vr, ar, ai);
    }
  }
  template <int N, int VF>
  __device__ void msumv_n(const RVec<T, VF>* S, int j, T* th) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const RVec<T, VF> sq = S[nb(j, k)];
#pragma unroll
      for (int f = 0; f < VF; ++f) th[f] += cm[j][k] * sq.v[f];
    }
  }
  template <int N, int VF>
  __device__ void msumv_w(int W, const RVec<T, VF>* S, int j, T* th) const {
    if constexpr (N > 0) {
      if (W == N) {
        msumv_n<N>(S, j, th);
        return;
      }
      msumv_w<N - 1>(W, S, j, th);
    }
  }
  template <int VF>
  __device__ CVec<T, VF> stagev(const DevOps<T>& d, const CVec<T, VF>* V_, const CVec<T, VF>& vr,
                                const CVec<T, VF>& base, int j, T coef) const {
    T ar[VF], ai[VF];
#pragma unroll
    for (int f = 0; f < VF; ++f) ar[f] = ai[f] = T(0);
    lsumv_w<KMAX>(wd[j], V_, j, vr, ar, ai);
    CVec<T, VF> r;
#pragma unroll
    for (int f = 0; f < VF; ++f) {
      const T hr = d.p1 * ar[f] - vv[j] * vr.v[f].x;
      const T hi = d.p1 * ai[f] - vv[j] * vr.v[f].y;
      r.v[f].x = base.v[f].x + coef * hi;
      r.v[f].y = base.v[f].y - coef * hr;
    }
    return r;
  }

  // The z step of step() for VF fields per slot (same per-field arithmetic).
  template <int VF, typename Out>
  __device__ void step_vec(const DevOps<T>& d, const CVec<T, VF>* P, CVec<T, VF>* X, CVec<T, VF>* Y,
                           RVec<T, VF>* S, T h, T tau, T gamma, Out out) const {
    const int B = blockDim.x;
    CVec<T, VF> p[J], cur[J];
    RVec<T, VF> so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n1) {
        p[j] = P[i];
        cur[j] = stagev<VF>(d, P, p[j], p[j], j, T(0.25) * h);  // y1
        Y[i] = cur[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n2) {
        cur[j] = stagev<VF>(d, Y, cur[j], p[j], j, h / T(3));  // y2
        X[i] = cur[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n3) {
        cur[j] = stagev<VF>(d, X, cur[j], p[j], j, T(0.5) * h);  // y3
        Y[i] = cur[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < n4) {  // state before the Kerr substep
        cur[j] = stagev<VF>(d, Y, cur[j], p[j], j, h);
        const T ph = phi_w(ww[j], tau);
#pragma unroll
        for (int f = 0; f < VF; ++f)
          so[j].v[f] = (cur[j].v[f].x * cur[j].v[f].x + cur[j].v[f].y * cur[j].v[f].y) * ph;
        S[i * SST] = so[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        T th[VF];
#pragma unroll
        for (int f = 0; f < VF; ++f) th[f] = md[j] * so[j].v[f];
        if constexpr (DEC) msumv_w<KMAX>(wd[j], S, j, th);
        const T damp = d_exp(-ww[j] * tau);
        CVec<T, VF> r;
#pragma unroll
        for (int f = 0; f < VF; ++f) {
          T sn, cs;
          d_sincos(gamma * th[f], &sn, &cs);
          const C b = cur[j].v[f];
          r.v[f].x = damp * (b.x * cs - b.y * sn);
          r.v[f].y = damp * (b.x * sn + b.y * cs);
        }
        out(i, rr[j], r);
      }
    }
  }

  // One step of classical RK4 on the whole right-hand side
  //   F(v) = -i (p1 L v - V v) + i gamma (M |v|^2) v - w v
  // (the Kerr term inside every stage).  Stage k evaluates F on rings
  // 0..4-k, gathering its input v from A and |v|^2 from SA (rings 0..5-k), and
  // writes the next stage's input and its |.|^2 to B and SB; the buffers then
  // swap.  The state is staged in A and SA (rings 0..4); own values stay in
  // registers.  Calls out(slot, r, value) for every owned row.
  template <typename Out>
  __device__ void step_unsplit(const DevOps<T>& d, C* A, C* Bv, T* SA, T* SB, T h, T gamma, Out out) const {
    const int B = blockDim.x;
    C p[J], cur[J], acc[J];
    T so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[3]) {
        p[j] = A[i];
        cur[j] = p[j];
        so[j] = SA[i];
        acc[j].x = acc[j].y = T(0);
      }
    }
    const T cnext[3] = {T(0.5) * h, T(0.5) * h, h};
    const T wsum[4] = {T(1), T(2), T(2), T(1)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      C* Vin = (k & 1) ? Bv : A;
      C* Vout = (k & 1) ? A : Bv;
      T* Sin = (k & 1) ? SB : SA;
      T* Sout = (k & 1) ? SA : SB;
      const int nk = hd[3 - k];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = threadIdx.x + j * B;
        if (i < nk) {
          T ar = T(0), ai = T(0);
          lsum_w<KMAX>(wd[j], CplxAoS<T>{Vin}, j, cur[j], ar, ai);
          T th = md[j] * so[j];
          if constexpr (DEC) th = msum_w<KMAX>(wd[j], Sin, j, th);
          const T hr = d.p1 * ar - vv[j] * cur[j].x;
          const T hi = d.p1 * ai - vv[j] * cur[j].y;
          C f;  // -i (hr + i hi) + i gamma th v - w v
          f.x = hi - gamma * th * cur[j].y - ww[j] * cur[j].x;
          f.y = -hr + gamma * th * cur[j].x - ww[j] * cur[j].y;
          acc[j].x += wsum[k] * f.x;
          acc[j].y += wsum[k] * f.y;
          if (k < 3) {
            cur[j].x = p[j].x + cnext[k] * f.x;
            cur[j].y = p[j].y + cnext[k] * f.y;
            so[j] = cur[j].x * cur[j].x + cur[j].y * cur[j].y;
            Vout[i] = cur[j];
            Sout[i] = so[j];
          }
        }
      }
      if (k < 3) __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[0]) {
        C r;
        r.x = p[j].x + (h / T(6)) * acc[j].x;
        r.y = p[j].y + (h / T(6)) * acc[j].y;
        out(i, rr[j], r);
      }
    }
  }

  // One trial step of the Dormand-Prince 5(4) pair on the whole right-hand
  // side F of step_unsplit.  Stage s (0..6) evaluates k_s = F(y_s) on rings
  // 0..6-s, gathering y_s from A/SA or B/SB (rings 0..7-s), and forms the next
  // stage input y_{s+1} = psi + h sum_j a_{s+1,j} k_j on the same rows.  The
  // seventh stage input is the fifth-order solution y5 (first same as last),
  // so k_6 = F(y5) completes the embedded estimate e = h sum_j (b_j - b*_j) k_j.
  // Calls out(slot, r, y5) for every owned row and returns this thread's sum
  // over its owned rows of (|e| / (atol + rtol max(|psi|, |y5|)))^2.
  template <typename Out>
  __device__ double step_dp5(const DevOps<T>& d, C* A, C* Bv, T* SA, T* SB, T h, T gamma, T rtol, T atol,
                             Out out) const {
    // Dormand and Prince (1980): stage coefficients a (row s+1 builds y_{s+1}),
    // fifth-order weights (= row 7) and the differences to the fourth-order ones
    constexpr double a[7][6] = {
        {0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
    };
    constexpr double eb[7] = {35.0 / 384 - 5179.0 / 57600,      0.0, 500.0 / 1113 - 7571.0 / 16695,
                              125.0 / 192 - 393.0 / 640,        -2187.0 / 6784 + 92097.0 / 339200,
                              11.0 / 84 - 187.0 / 2100,         -1.0 / 40};
    const int B = blockDim.x;
    C p[J], cur[J], k[J][7];
    T so[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[6]) {
        p[j] = A[i];
        cur[j] = p[j];
        so[j] = SA[i];
      }
    }
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      C* Vin = (s & 1) ? Bv : A;
      C* Vout = (s & 1) ? A : Bv;
      T* Sin = (s & 1) ? SB : SA;
      T* Sout = (s & 1) ? SA : SB;
      const int ns = hd[6 - s];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = threadIdx.x + j * B;
        if (i < ns) {
          T ar = T(0), ai = T(0);
          lsum_w<KMAX>(wd[j], CplxAoS<T>{Vin}, j, cur[j], ar, ai);
          T th = md[j] * so[j];
          if constexpr (DEC) th = msum_w<KMAX>(wd[j], Sin, j, th);
          const T hr = d.p1 * ar - vv[j] * cur[j].x;
          const T hi = d.p1 * ai - vv[j] * cur[j].y;
          k[j][s].x = hi - gamma * th * cur[j].y - ww[j] * cur[j].x;
          k[j][s].y = -hr + gamma * th * cur[j].x - ww[j] * cur[j].y;
          if (s < 6) {
            T yx = T(0), yy = T(0);
#pragma unroll
            for (int q2 = 0; q2 <= s; ++q2) {
              if (a[s + 1][q2] != 0.0) {
                yx += T(a[s + 1][q2]) * k[j][q2].x;
                yy += T(a[s + 1][q2]) * k[j][q2].y;
              }
            }
            cur[j].x = p[j].x + h * yx;
            cur[j].y = p[j].y + h * yy;
            so[j] = cur[j].x * cur[j].x + cur[j].y * cur[j].y;
            Vout[i] = cur[j];
            Sout[i] = so[j];
          }
        }
      }
      if (s < 6) __syncthreads();
    }
    double q = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[0]) {
        T ex = T(0), ey = T(0);
#pragma unroll
        for (int s = 0; s < 7; ++s) {
          if (eb[s] != 0.0) {
            ex += T(eb[s]) * k[j][s].x;
            ey += T(eb[s]) * k[j][s].y;
          }
        }
        ex *= h;
        ey *= h;
        const T m0 = sqrt(p[j].x * p[j].x + p[j].y * p[j].y);
        const T m1 = sqrt(so[j]);
        const T sc = atol + rtol * (m0 > m1 ? m0 : m1);
        const T rx = ex / sc, ry = ey / sc;
        q += double(rx * rx + ry * ry);
        out(i, rr[j], cur[j]);
      }
    }
    return q;
  }

  // One step of the nonlinear mode iteration: y = R4(-h A) phi with
  // A = H_lin - gamma diag(M |phi|^2), the nonlinearity frozen at phi, in
  // Horner form.  The innermost product g = A phi is taken on rings 0..3 with
  // the |phi|^2 gather (SA); theta stays in registers for the three outer
  // products (rings 0..2, 0..1, 0), which gather from the other buffer.  Adds
  // over the owned rows, H0-weighted: acc[0] += Re(conj(phi) g),
  // acc[1] += |g - mu_prev phi|^2, acc[2] += |phi|^2, acc[3] += |y|^2, and
  // calls out(slot, r, y).
  template <typename Out>
  __device__ void step_mode(const DevOps<T>& d, C* A, C* Bv, const T* SA, T h, T gamma, T mu_prev, double (&acc)[4],
                            Out out) const {
    const int B = blockDim.x;
    C p[J], cur[J];
    T th[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[3]) {
        p[j] = A[i];
        cur[j] = p[j];
        th[j] = md[j] * SA[i];
      }
    }
    const T cf[4] = {h / T(4), h / T(3), h / T(2), h};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      C* Vin = (k & 1) ? Bv : A;
      C* Vout = (k & 1) ? A : Bv;
      const int nk = hd[3 - k];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = threadIdx.x + j * B;
        if (i < nk) {
          T ar = T(0), ai = T(0);
          lsum_w<KMAX>(wd[j], CplxAoS<T>{Vin}, j, cur[j], ar, ai);
          if (k == 0) {
            if constexpr (DEC) th[j] = msum_w<KMAX>(wd[j], SA, j, th[j]);
            th[j] *= gamma;
          }
          C g;  // A cur = p1 L cur - v cur - gamma theta cur
          g.x = d.p1 * ar - (vv[j] + th[j]) * cur[j].x;
          g.y = d.p1 * ai - (vv[j] + th[j]) * cur[j].y;
          if (k == 0 && i < hd[0]) {
            const double w0 = d.h0[rr[j]];
            acc[0] += w0 * (double(p[j].x) * g.x + double(p[j].y) * g.y);
            const double ex = double(g.x) - double(mu_prev) * p[j].x, ey = double(g.y) - double(mu_prev) * p[j].y;
            acc[1] += w0 * (ex * ex + ey * ey);
            acc[2] += w0 * (double(p[j].x) * p[j].x + double(p[j].y) * p[j].y);
          }
          cur[j].x = p[j].x - cf[k] * g.x;
          cur[j].y = p[j].y - cf[k] * g.y;
          if (k < 3) Vout[i] = cur[j];
        }
      }
      if (k < 3) __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < hd[0]) {
        acc[3] += d.h0[rr[j]] * (double(cur[j].x) * cur[j].x + double(cur[j].y) * cur[j].y);
        out(i, rr[j], cur[j]);
      }
    }
  }
};

// One whole z step, LIN(h) then NL(tau), per tile of rows (five halo rings).
// Stores a step's result: in device order, or (out_perm given) at the
// caller's index out_perm[r], flagging a non-finite value in bit 0 of *flag.
template <typename C>
__device__ inline void put_result(C* __restrict__ out, const int32_t* __restrict__ out_perm, int* flag, int32_t r,
                                  const C& v) {
  if (out_perm) {
    if (!(d_finite(v.x) && d_finite(v.y))) atomicOr(flag, 1);
    out[out_perm[r]] = v;
  } else {
    out[r] = v;
  }
}

// One whole z step: LIN(h) then NL(tau).  out_perm: see put_result.
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_step(DevOps<T> d, TileOps<T> tl, const typename CT<T>::C* __restrict__ in_psi,
                                               typename CT<T>::C* __restrict__ out_psi, T h, T tau, T gamma,
                                               const int32_t* __restrict__ out_perm, int* flag) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  C* base = reinterpret_cast<C*>(smem);
  const CplxAoS<T> P{base}, X{base + MS}, Y{base + 2 * MS};
  T* S = reinterpret_cast<T*>(base + 3 * MS);
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile, false, nullptr, true);
  for (int i = threadIdx.x; i < st.nLoad; i += blockDim.x) P.put(i, in_psi[st.slot_row(i)]);
  __syncthreads();
  st.step(d, P, X, Y, S, h, tau, gamma, [&](int, int32_t r, const C& v) { put_result(out_psi, out_perm, flag, r, v); },
          [](int, int32_t, const C&) {});
}

// NL(tau) of the caller's field (caller order, row r at src[perm[r]]) into a
// device-order state buffer, on the step tiles: the first half step of a
// propagate, with the same per-row arithmetic as the persistent launch's.
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_kerr_tile(DevOps<T> d, TileOps<T> tl,
                                                                        const typename CT<T>::C* __restrict__ src,
                                                                        const int32_t* __restrict__ perm,
                                                                        typename CT<T>::C* __restrict__ dst, T tau,
                                                                        T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  T* S = reinterpret_cast<T*>(smem);
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile, true);
  st.kerr_from(d, src, perm, S, tau, gamma, [&](int, int32_t r, const C& v) { dst[r] = v; });
}

// One z step of every field of a batch on one-field step tiles.  The device
// layout is field-major (field f of row r at f * n_rows + r).  The work is
// the n_tiles * nf (tile, field) pairs in tile-major order, cut into n_wg
// contiguous runs of equal length, one per workgroup, so that every
// workgroup does the same number of field steps whatever the tile count.
// Along its run a workgroup loads a tile's operator rows into registers once
// and steps that tile's fields one after another; the next field's state is
// fetched into registers while the current one runs its later stages (P is
// last read by stage 1) and moved into P before the Kerr phase's barrier, so
// that consecutive fields of a tile need no barrier between them.  LM: the M
// weights are kept in LDS after S (the per-field state leaves them no room in
// registers).
template <typename T, int KMAX, bool DEC, int J, int LS, bool LM>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_step_fields(DevOps<T> d, TileOps<T> tl,
                                                                          const typename CT<T>::C* __restrict__ in,
                                                                          typename CT<T>::C* __restrict__ out, T h,
                                                                          T tau, T gamma, int32_t nf, int32_t n_wg) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t wg = logical_block(d.xcd_remap);
  if (wg >= n_wg) return;
  const int MS = tl.max_slots;
  const int B = blockDim.x;
  C* base = reinterpret_cast<C*>(smem);
  const CplxAoS<T> P{base}, X{base + MS}, Y{base + 2 * MS};
  T* S = reinterpret_cast<T*>(base + 3 * MS);
  const int64_t units = int64_t(tl.n_tiles) * nf;
  int64_t u = wg * units / n_wg;
  const int64_t u_end = (wg + 1) * units / n_wg;
  while (u < u_end) {
    const int64_t tile = u / nf;
    const int32_t f0 = int32_t(u - tile * nf);
    const int32_t f1 = int32_t(f0 + (u_end - u < nf - f0 ? u_end - u : nf - f0));
    StepTile<T, KMAX, DEC, J, false, LM> st;
    st.init(d, tl, tile, false, S + MS, true);
    int32_t pr[LS];
#pragma unroll
    for (int l = 0; l < LS; ++l) {
      const int i = threadIdx.x + l * B;
      pr[l] = i < st.nLoad ? st.slot_row(i) : -1;
    }
    const int64_t off0 = int64_t(f0) * d.n_rows;
#pragma unroll
    for (int l = 0; l < LS; ++l)
      if (pr[l] >= 0) P.put(threadIdx.x + l * B, in[off0 + pr[l]]);
    __syncthreads();
    for (int32_t f = f0; f < f1; ++f) {
      st.opaque_neighbours();
      const int64_t off = int64_t(f) * d.n_rows;
      const bool more = f + 1 < f1;
      C pv[LS];
      // the next field's state: fetched into registers once P is free, put
      // into P before the Kerr phase's barrier (which then orders it before
      // the next field's first gather)
      st.step(d, P, X, Y, S, h, tau, gamma, [&](int, int32_t r, const C& v) { out[off + r] = v; },
              [](int, int32_t, const C&) {},
              [&]() {
                if (more) {
#pragma unroll
                  for (int l = 0; l < LS; ++l)
                    if (pr[l] >= 0) pv[l] = in[off + d.n_rows + pr[l]];
                }
              },
              [&]() {
                if (more) {
#pragma unroll
                  for (int l = 0; l < LS; ++l)
                    if (pr[l] >= 0) P.put(threadIdx.x + l * B, pv[l]);
                }
              });
      // every read of this tile's LDS is done before the next tile's load
      // overwrites it (the next field of the same tile needs no barrier here:
      // its first phase reads P, complete since the Kerr phase's barrier, and
      // writes Y, which this field's Kerr phase does not read)
      if (!more) __syncthreads();
    }
    u += f1 - f0;
  }
}

// NL(tau) of every field of a batch (field-major device layout) on one-field
// step tiles, as k_kerr_tile does for one field: the first half step.
template <typename T, int KMAX, bool DEC, int J>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_kerr_fields(DevOps<T> d, TileOps<T> tl,
                                                                          const typename CT<T>::C* __restrict__ in,
                                                                          typename CT<T>::C* __restrict__ out, T tau,
                                                                          T gamma, int32_t nf) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  T* S = reinterpret_cast<T*>(smem);
  StepTile<T, KMAX, DEC, J> st;
  st.init(d, tl, tile, true);
  for (int32_t f = 0; f < nf; ++f) {
    const int64_t off = int64_t(f) * d.n_rows;
    st.kerr_from(d, in + off, nullptr, S, tau, gamma, [&](int, int32_t r, const C& v) { out[off + r] = v; });
    __syncthreads();
  }
}

// One whole z step for a batched handle: workgroup b handles step tile
// b / G and the b % G-th group of VF fields (G = F / VF) of every row of it, so
// the G workgroups of a tile run back to back on one XCD and share its
// operator rows in L2.
template <typename T, int KMAX, bool DEC, int J, int VF>
__global__ void __launch_bounds__(1024) k_bstep(DevOps<T> d, TileOps<T> tl, const CVec<T, VF>* __restrict__ in_psi,
                                                CVec<T, VF>* __restrict__ out_psi, T h, T tau, T gamma) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int G = d.F / VF;
  const int64_t b = logical_block(d.xcd_remap);
  const int64_t tile = b / G;
  const int grp = int(b - tile * G);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  CVec<T, VF>* P = reinterpret_cast<CVec<T, VF>*>(smem);
  CVec<T, VF>* X = P + MS;
  CVec<T, VF>* Y = X + MS;
  RVec<T, VF>* S = reinterpret_cast<RVec<T, VF>*>(Y + MS);
  StepTile<T, KMAX, DEC, J> st;
  st.init(d, tl, tile);
  for (int i = threadIdx.x; i < st.nLoad; i += blockDim.x) P[i] = in_psi[int64_t(st.slot_row(i)) * G + grp];
  __syncthreads();
  st.template step_vec<VF>(d, P, X, Y, S, h, tau, gamma,
                           [&](int, int32_t r, const CVec<T, VF>& v) { out_psi[int64_t(r) * G + grp] = v; });
}

// One unsplit classical RK4 step per tile (the Kerr term inside every stage).
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_rk4u(DevOps<T> d, TileOps<T> tl,
                                                                  const typename CT<T>::C* __restrict__ in_psi,
                                                                  typename CT<T>::C* __restrict__ out_psi, T h,
                                                                  T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  C* A = reinterpret_cast<C*>(smem);
  C* Bv = A + MS;
  T* SA = reinterpret_cast<T*>(Bv + MS);
  T* SB = SA + MS;
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile);
  for (int i = threadIdx.x; i < st.hd[4]; i += blockDim.x) {
    const C v = in_psi[st.slot_row(i)];
    A[i] = v;
    SA[i] = v.x * v.x + v.y * v.y;
  }
  __syncthreads();
  st.step_unsplit(d, A, Bv, SA, SB, h, gamma, [&](int, int32_t r, const C& v) { out_psi[r] = v; });
}

// One RK4 stage of Eq. 1's operator sum with terms up to p4 L^4 on tiles of
// D halo rings (D = 4 with p4, else 3): out = base + coef (-i)(sum_n p_n L^n x
// - V x) on the owned rows, the powers of L by Horner on the LDS-staged x,
// t_D = p_D x, t_n = p_n x + L t_{n+1}, sum = L t_1; each product shrinks the
// valid region by one ring.  With s_out, the stage's result also gives the
// next Kerr substep's integral N-integral(|out|^2, w, tau_s).
template <typename T, int KMAX, int J>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_hstage(DevOps<T> d, TileOps<T> tl,
                                                                    const typename CT<T>::C* __restrict__ x,
                                                                    const typename CT<T>::C* __restrict__ base,
                                                                    typename CT<T>::C* __restrict__ out, T coef,
                                                                    T p3, T p4, T* __restrict__ s_out, T tau_s) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  const int B = blockDim.x;
  C* sm = reinterpret_cast<C*>(smem);
  const CplxAoS<T> X{sm}, TA{sm + MS}, TB{sm + 2 * MS};
  StepTile<T, KMAX, false, J> st;
  st.init(d, tl, tile);
  const int D = st.hd[15];  // rings of the tile: the number of products
  for (int i = threadIdx.x; i < st.nLoad; i += B) X.put(i, x[st.slot_row(i)]);
  const T pc[5] = {T(0), d.p1, d.beta4, p3, p4};
  C xv[J], tv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + j * B;
    xv[j] = i < st.n1 ? x[st.slot_row(i)] : C{T(0), T(0)};
    tv[j].x = pc[D] * xv[j].x;
    tv[j].y = pc[D] * xv[j].y;
  }
  __syncthreads();
  // product k (k = 1..D-1): t_{D-k} = p_{D-k} x + L t_{D-k+1} on rings 0..D-k;
  // the first product gathers x itself (t_D = p_D x), scaled afterwards
  for (int k = 1; k < D; ++k) {
    const CplxAoS<T>& src = k == 1 ? X : (k % 2 ? TB : TA);
    const CplxAoS<T>& dst = k % 2 ? TA : TB;
    const int nk = st.hd[D - k];
    const T pn = pc[D - k];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < nk) {
        T ar = T(0), ai = T(0);
        if (k == 1) {
          st.template lsum_w<KMAX>(st.wd[j], src, j, xv[j], ar, ai);
          ar *= pc[D];
          ai *= pc[D];
        } else {
          st.template lsum_w<KMAX>(st.wd[j], src, j, tv[j], ar, ai);
        }
        tv[j].x = pn * xv[j].x + ar;
        tv[j].y = pn * xv[j].y + ai;
        dst.put(i, tv[j]);
      }
    }
    __syncthreads();
  }
  // the last product on the owned rows: h = L t_1 - V x, out = base + coef (-i) h
  const CplxAoS<T>& last = (D - 1) % 2 ? TA : TB;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + j * B;
    if (i < st.nNL) {
      T ar = T(0), ai = T(0);
      st.template lsum_w<KMAX>(st.wd[j], last, j, tv[j], ar, ai);
      const int32_t r = st.rr[j];
      const T hr = ar - st.vv[j] * xv[j].x;
      const T hi = ai - st.vv[j] * xv[j].y;
      const C b = base[r];
      C o;
      o.x = b.x + coef * hi;
      o.y = b.y - coef * hr;
      out[r] = o;
      if (s_out) s_out[r] = nl_int(d, o.x * o.x + o.y * o.y, st.ww[j], tau_s);
    }
  }
}

// ---- device-coherent access between workgroups of one launch ----
// Device-coherent (agent scope) element access for state exchanged between
// workgroups of one persistent launch, which may run on different XCDs.
__device__ inline float2 coherent_load(const float2* p) {
  const uint64_t u =
      __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<float2*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 r;
  __builtin_memcpy(&r, &u, sizeof(r));
  return r;
}
__device__ inline double2 coherent_load(const double2* p) {
  uint64_t* q = reinterpret_cast<uint64_t*>(const_cast<double2*>(p));
  const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double2 r;
  __builtin_memcpy(&r.x, &a, 8);
  __builtin_memcpy(&r.y, &b, 8);
  return r;
}
__device__ inline void coherent_store(float2* p, const float2& v) {
  uint64_t u;
  __builtin_memcpy(&u, &v, sizeof(u));
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void coherent_store(double2* p, const double2& v) {
  uint64_t a, b;
  __builtin_memcpy(&a, &v.x, 8);
  __builtin_memcpy(&b, &v.y, 8);
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
  __hip_atomic_store(q, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wave's stores have been acknowledged (vmcnt = 0; the
// export and LDS counters are left at their maxima).  With every exchanged
// element written and read by agent-scope accesses, this orders the state
// stores before the flag store without a cache write-back or invalidate.
__device__ inline void wait_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ inline double coherent_load(const double* p) {
  const uint64_t u =
      __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double r;
  __builtin_memcpy(&r, &u, 8);
  return r;
}
__device__ inline void coherent_store(double* p, double v) {
  uint64_t u;
  __builtin_memcpy(&u, &v, 8);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Accept/reject rule of the standard embedded-pair controller (Hairer,
// Norsett and Wanner, Solving ODEs I, section II.4): accept when the error
// norm is below 1, scale the step by min(facmax, max(0.2, 0.9 err^(-1/5)))
// with facmax = 1 right after a rejection, clip the next trial to z_end.
__device__ inline void dp5_decide(Dp5Ctl* ctl, double sumsq, double inv_n) {
  Dp5Ctl c = *ctl;
  const double err = sqrt(sumsq * inv_n);
  c.err = err;
  if (!isfinite(err)) {
    c.status = 2;
    c.done = 1;
    c.rejected += 1;
    *ctl = c;
    return;
  }
  double fac;
  if (err < 1.0) {
    c.z = c.z_trial;
    c.cur ^= 1;
    c.accepted += 1;
    c.last_h = c.h_step;
    fac = err == 0.0 ? c.facmax : fmin(c.facmax, 0.9 * pow(err, -0.2));
    if (c.prev_rejected) fac = fmin(1.0, fac);
    c.prev_rejected = 0;
  } else {
    fac = fmax(0.2, 0.9 * pow(err, -0.2));
    c.rejected += 1;
    c.prev_rejected = 1;
  }
  c.h_abs = c.h_step * fac;
  if (c.z >= c.z_end) {
    c.done = 1;
  } else if (c.accepted + c.rejected >= c.max_attempts) {
    c.done = 1;
    c.status = 1;
  } else {
    const double zt = c.z + c.h_abs;
    c.z_trial = zt < c.z_end ? zt : c.z_end;
    c.h_step = c.z_trial - c.z;
    if (c.h_step < 10.0 * (nextafter(c.z, INFINITY) - c.z)) {
      c.done = 1;
      c.status = 3;
    }
  }
  *ctl = c;
}

// One Dormand-Prince 5(4) trial per tile of the seven-ring tiles.  The
// controller state says which buffer holds the state (x[cur]) and the trial
// step; the candidate goes to x[1 - cur].  Each tile publishes its share of
// the squared error norm (agent-scope store, acknowledged before it counts
// itself in); the workgroup that arrives last sums the shares in tile order,
// runs the controller and resets the arrival count for the next trial.
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__(1024) k_dp5(DevOps<T> d, TileOps<T> tl, typename CT<T>::C* x0,
                                              typename CT<T>::C* x1, Dp5Ctl* ctl, double* __restrict__ partial,
                                              uint32_t* __restrict__ arrivals, T gamma, T rtol, T atol,
                                              double inv_n) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ int last;
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles || ctl->done) return;
  const int cur = ctl->cur;
  const T h = T(ctl->h_step);
  const C* in_psi = cur ? x1 : x0;
  C* out_psi = cur ? x0 : x1;
  const int MS = tl.max_slots;
  C* A = reinterpret_cast<C*>(smem);
  C* Bv = A + MS;
  T* SA = reinterpret_cast<T*>(Bv + MS);
  T* SB = SA + MS;
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile);
  for (int i = threadIdx.x; i < st.hd[7]; i += blockDim.x) {
    const C v = in_psi[st.slot_row(i)];
    A[i] = v;
    SA[i] = v.x * v.x + v.y * v.y;
  }
  __syncthreads();
  double q = st.step_dp5(d, A, Bv, SA, SB, h, gamma, rtol, atol, [&](int, int32_t r, const C& v) { out_psi[r] = v; });
  const int nw = int(blockDim.x + 63) / 64;
  for (int off = 32; off > 0; off >>= 1) q += __shfl_down(q, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    coherent_store(partial + tile, t);
    wait_stores();
    last = __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
           uint32_t(tl.n_tiles - 1);
  }
  __syncthreads();
  if (!last) return;
  double t = 0.0;
  for (int k = threadIdx.x; k < tl.n_tiles; k += blockDim.x) t += coherent_load(partial + k);
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  __syncthreads();  // red[] reuse
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < nw; ++w) sum += red[w];
    __hip_atomic_store(arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    dp5_decide(ctl, sum, inv_n);
  }
}

// The adaptive run with every seven-ring tile resident (cooperative launch):
// the trials of k_dp5 back to back, each ended by a grid-wide exchange of the
// tiles' error shares (agent-scope stores, acknowledged, then an iteration
// counter); every tile sums all shares in tile order and runs the controller
// itself, so all take the same decision; tile 0 keeps the state in memory.
// The global wait orders the buffer reuse (a trial writes x[1 - cur], which no
// tile still reads) and the shares alternate between two halves of `partial`
// (2 * n_tiles doubles).
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__(1024) k_dp5_persist(DevOps<T> d, TileOps<T> tl, typename CT<T>::C* x0,
                                                      typename CT<T>::C* x1, Dp5Ctl* ctl, double* __restrict__ partial,
                                                      int32_t* flags, int32_t* status, int32_t spin_limit, T gamma,
                                                      T rtol, T atol, double inv_n) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  __shared__ Dp5Ctl cs;
  __shared__ int32_t abort_s;
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  const int nw = int(blockDim.x + 63) / 64;
  C* A = reinterpret_cast<C*>(smem);
  C* Bv = A + MS;
  T* SA = reinterpret_cast<T*>(Bv + MS);
  T* SB = SA + MS;
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile);
  if (threadIdx.x == 0) cs = *ctl;
  __syncthreads();
  for (int32_t it = 0; !cs.done; ++it) {
    st.opaque_neighbours();
    const C* in_psi = cs.cur ? x1 : x0;
    C* out_psi = cs.cur ? x0 : x1;
    const T h = T(cs.h_step);
    for (int i = threadIdx.x; i < st.hd[7]; i += blockDim.x) {
      const C v = coherent_load(in_psi + st.slot_row(i));
      A[i] = v;
      SA[i] = v.x * v.x + v.y * v.y;
    }
    __syncthreads();
    double q = st.step_dp5(d, A, Bv, SA, SB, h, gamma, rtol, atol,
                           [&](int, int32_t r, const C& v) { coherent_store(out_psi + r, v); });
    for (int off = 32; off > 0; off >>= 1) q += __shfl_down(q, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    double* half = partial + int64_t(it & 1) * tl.n_tiles;
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w];
      coherent_store(half + tile, t);
    }
    wait_stores();  // every wave: its rows and the share acknowledged
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + tile, it + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < 64) {  // wait for every tile's trial it
      bool ok = true;
      for (int32_t spins = 0;; ++spins) {
        bool all = true;
        for (int k = threadIdx.x; k < tl.n_tiles; k += 64)
          all = all && __hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= it + 1;
        if (__all(all)) break;
        if (spins >= spin_limit) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (threadIdx.x == 0) {
        abort_s = ok ? 0 : 1;
        if (!ok) __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (abort_s) return;
    double t = 0.0;
    for (int k = threadIdx.x; k < tl.n_tiles; k += blockDim.x) t += coherent_load(half + k);
    for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
    __syncthreads();  // red[] reuse
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < nw; ++w) sum += red[w];
      dp5_decide(&cs, sum, inv_n);
      if (tile == 0) *ctl = cs;
    }
    __syncthreads();
  }
}

__global__ void k_dp5_init(Dp5Ctl* ctl, uint32_t* arrivals, double z_end, double h0, int64_t max_attempts,
                           double facmax) {
  if (threadIdx.x != 0) return;
  Dp5Ctl c;
  c.z = 0.0;
  c.z_end = z_end;
  c.h_abs = h0;
  c.z_trial = h0 < z_end ? h0 : z_end;
  c.h_step = c.z_trial;
  c.last_h = 0.0;
  c.err = 0.0;
  c.facmax = facmax;
  c.accepted = c.rejected = 0;
  c.max_attempts = max_attempts;
  c.cur = 0;
  c.prev_rejected = 0;
  c.done = z_end <= 0.0 || max_attempts <= 0;
  c.status = (z_end > 0.0 && max_attempts <= 0) ? 1 : 0;
  *ctl = c;
  *arrivals = 0u;
}

// Gradient-flow mode iteration on the step tiles: x[cur] * s is the current
// iterate phi_k (power P); the kernel writes y = R4(-h A_k) phi_k to
// x[1 - cur] and four H0-weighted partial sums per tile; the workgroup that
// arrives last sums them in tile order and updates the state: the Rayleigh
// quotient mu_k, the residual with the previous quotient, the stopping test
// (k > 0, tol > 0, r <= tol |mu|: phi_k is the result), else s = sqrt(P /
// P(y)), cur flips and k advances.
__device__ inline void mode_decide(ModeCtl* ctl, const double (&S)[4]) {
  ModeCtl c = *ctl;
  const double mu = S[0] / S[2];
  const double r = sqrt(S[1] / S[2]);
  c.mu = mu;
  c.res = r;
  if (c.iter > 0 && c.tol > 0.0 && r <= c.tol * fabs(mu)) {
    c.done = 1;
    c.status = 0;
    *ctl = c;
    return;
  }
  if (!(S[3] > 0.0) || !isfinite(S[3]) || !isfinite(mu)) {
    c.done = 1;
    c.status = 2;
    *ctl = c;
    return;
  }
  c.s = sqrt(c.power / S[3]);
  c.cur ^= 1;
  c.mu_prev = mu;
  c.iter += 1;
  if (c.iter >= c.max_iter) {
    c.done = 1;
    c.status = c.tol > 0.0 ? 1 : 0;
  }
  *ctl = c;
}

template <typename T, int KMAX, bool DEC, int J>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_mode(DevOps<T> d, TileOps<T> tl, typename CT<T>::C* x0,
                                                                  typename CT<T>::C* x1, ModeCtl* ctl,
                                                                  double* __restrict__ partial,
                                                                  uint32_t* __restrict__ arrivals, T h, T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16][4];
  __shared__ int last;
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles || ctl->done) return;
  const int cur = ctl->cur;
  const T sc = T(ctl->s);
  const T mu_prev = T(ctl->mu_prev);
  const C* in_psi = cur ? x1 : x0;
  C* out_psi = cur ? x0 : x1;
  const int MS = tl.max_slots;
  C* A = reinterpret_cast<C*>(smem);
  C* Bv = A + MS;
  T* SA = reinterpret_cast<T*>(Bv + MS);
  StepTile<T, KMAX, DEC, J> st;
  st.init(d, tl, tile);
  for (int i = threadIdx.x; i < st.hd[4]; i += blockDim.x) {
    C v = in_psi[st.slot_row(i)];
    v.x *= sc;
    v.y *= sc;
    A[i] = v;
    SA[i] = v.x * v.x + v.y * v.y;
  }
  __syncthreads();
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  st.step_mode(d, A, Bv, SA, h, gamma, mu_prev, acc, [&](int, int32_t r, const C& v) { out_psi[r] = v; });
  const int nw = int(blockDim.x + 63) / 64;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_down(acc[c], off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w][threadIdx.x];
    coherent_store(partial + 4 * tile + threadIdx.x, t);
    wait_stores();
  }
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
           uint32_t(tl.n_tiles - 1);
  __syncthreads();
  if (!last) return;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < tl.n_tiles; k += blockDim.x)
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] += coherent_load(partial + 4 * k + c);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    for (int off = 32; off > 0; off >>= 1) t[c] += __shfl_down(t[c], off, 64);
  }
  __syncthreads();  // red[] reuse
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) red[threadIdx.x >> 6][c] = t[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < nw; ++w)
#pragma unroll
      for (int c = 0; c < 4; ++c) S[c] += red[w][c];
    __hip_atomic_store(arrivals, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mode_decide(ctl, S);
  }
}

// The mode iteration with every step tile resident (cooperative launch): the
// iterations of k_mode back to back, each ended by a grid-wide exchange
// instead of a kernel boundary.  A tile publishes its four sums and its new
// rows (agent-scope stores, acknowledged), then its iteration counter; it
// waits for every tile's counter (bounded: status bit 2 and exit), sums all
// tiles' shares in tile order and takes the stopping decision itself, so
// every tile reaches the same one; tile 0 keeps the controller state in
// memory.  The global wait also orders the buffer reuse: x[1 - cur] is only
// written after every tile has read it as the previous iteration's input,
// and the shares alternate between two halves of `partial` (8 * n_tiles
// doubles), so a tile still summing iteration k's shares is never overwritten.
template <typename T, int KMAX, bool DEC, int J>
__global__ void __launch_bounds__(1024) k_mode_persist(DevOps<T> d, TileOps<T> tl, typename CT<T>::C* x0,
                                                       typename CT<T>::C* x1, ModeCtl* ctl,
                                                       double* __restrict__ partial, int32_t* flags, int32_t* status,
                                                       int32_t spin_limit, T h, T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16][4];
  __shared__ ModeCtl cs;
  __shared__ int32_t abort_s;
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  const int nw = int(blockDim.x + 63) / 64;
  C* A = reinterpret_cast<C*>(smem);
  C* Bv = A + MS;
  T* SA = reinterpret_cast<T*>(Bv + MS);
  StepTile<T, KMAX, DEC, J> st;
  st.init(d, tl, tile);
  if (threadIdx.x == 0) cs = *ctl;
  __syncthreads();
  for (int32_t it = 0; !cs.done; ++it) {
    st.opaque_neighbours();
    const C* in_psi = cs.cur ? x1 : x0;
    C* out_psi = cs.cur ? x0 : x1;
    const T sc = T(cs.s);
    const T mu_prev = T(cs.mu_prev);
    for (int i = threadIdx.x; i < st.hd[4]; i += blockDim.x) {
      C v = coherent_load(in_psi + st.slot_row(i));
      v.x *= sc;
      v.y *= sc;
      A[i] = v;
      SA[i] = v.x * v.x + v.y * v.y;
    }
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    st.step_mode(d, A, Bv, SA, h, gamma, mu_prev, acc,
                 [&](int, int32_t r, const C& v) { coherent_store(out_psi + r, v); });
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      for (int off = 32; off > 0; off >>= 1) acc[c] += __shfl_down(acc[c], off, 64);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = acc[c];
    }
    __syncthreads();
    double* half = partial + int64_t(it & 1) * 4 * tl.n_tiles;
    if (threadIdx.x < 4) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += red[w][threadIdx.x];
      coherent_store(half + 4 * tile + threadIdx.x, t);
    }
    wait_stores();  // every wave: its rows and shares acknowledged
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + tile, it + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < 64) {  // wait for every tile's iteration it
      bool ok = true;
      for (int32_t spins = 0;; ++spins) {
        bool all = true;
        for (int k = threadIdx.x; k < tl.n_tiles; k += 64)
          all = all && __hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= it + 1;
        if (__all(all)) break;
        if (spins >= spin_limit) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (threadIdx.x == 0) {
        abort_s = ok ? 0 : 1;
        if (!ok) __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (abort_s) return;
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < tl.n_tiles; k += blockDim.x)
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] += coherent_load(half + 4 * k + c);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      for (int off = 32; off > 0; off >>= 1) t[c] += __shfl_down(t[c], off, 64);
    __syncthreads();  // red[] reuse
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[threadIdx.x >> 6][c] = t[c];
    __syncthreads();
    if (threadIdx.x == 0) {
      double S[4] = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < nw; ++w)
#pragma unroll
        for (int c = 0; c < 4; ++c) S[c] += red[w][c];
      mode_decide(&cs, S);
      if (tile == 0) *ctl = cs;
    }
    __syncthreads();
  }
}

// Starts a mode iteration from x[0] with power p0 = pw[0] (a power reduction
// of x[0]): s = sqrt(P / p0); a start with no power or a non-finite one ends
// at once with status 2.
__global__ void k_mode_init(ModeCtl* ctl, uint32_t* arrivals, const double* pw, double power, double tol,
                            int64_t max_iter) {
  if (threadIdx.x != 0) return;
  ModeCtl c;
  const double p0 = pw[0];
  c.s = sqrt(power / p0);
  c.power = power;
  c.mu_prev = 0.0;
  c.mu = c.res = 0.0;
  c.tol = tol;
  c.iter = 0;
  c.max_iter = max_iter;
  c.cur = 0;
  c.done = 0;
  c.status = 0;
  c.pad = 0;
  if (!(p0 > 0.0) || !isfinite(c.s)) {
    c.done = 1;
    c.status = 2;
  }
  *ctl = c;
  *arrivals = 0u;
}

// x[:] *= s (device order, F = 1)
template <typename T>
__global__ void k_scale(typename CT<T>::C* x, int64_t n, T s) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    x[i].x *= s;
    x[i].y *= s;
  }
}

// One whole z step with the beta4 L^2 term per tile (8 or 9 halo rings).
template <typename T, int KMAX, bool DEC, int J>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_step_b4(DevOps<T> d, TileOps<T> tl,
                                                                     const typename CT<T>::C* __restrict__ in_psi,
                                                                     typename CT<T>::C* __restrict__ out_psi, T h,
                                                                     T tau, T gamma,
                                                                     const int32_t* __restrict__ out_perm, int* flag) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  C* base = reinterpret_cast<C*>(smem);
  const CplxAoS<T> P{base}, X{base + MS}, Y{base + 2 * MS}, Tb{base + 3 * MS};
  T* S = reinterpret_cast<T*>(base + 4 * MS);
  StepTile<T, KMAX, DEC, J> st;
  st.init(d, tl, tile, false, nullptr, true);
  for (int i = threadIdx.x; i < st.nLoad; i += blockDim.x) P.put(i, in_psi[st.slot_row(i)]);
  __syncthreads();
  st.step_b4(d, P, X, Y, Tb, S, h, tau, gamma,
             [&](int, int32_t r, const C& v) { put_result(out_psi, out_perm, flag, r, v); });
}

// The one-kernel step that also records, for the adjoint's forward recompute,
// the stage vectors y1, y2, y3 and the state before the Kerr substep.
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_step_rec(DevOps<T> d, TileOps<T> tl,
                                                   const typename CT<T>::C* __restrict__ in_psi,
                                                   typename CT<T>::C* __restrict__ out_psi,
                                                   typename CT<T>::C* __restrict__ o_y1,
                                                   typename CT<T>::C* __restrict__ o_y2,
                                                   typename CT<T>::C* __restrict__ o_y3,
                                                   typename CT<T>::C* __restrict__ o_b, T h, T tau, T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  C* base = reinterpret_cast<C*>(smem);
  const CplxAoS<T> P{base}, X{base + MS}, Y{base + 2 * MS};
  T* S = reinterpret_cast<T*>(base + 3 * MS);
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile, false, nullptr, true);
  for (int i = threadIdx.x; i < st.nLoad; i += blockDim.x) P.put(i, in_psi[st.slot_row(i)]);
  __syncthreads();
  st.step(d, P, X, Y, S, h, tau, gamma, [&](int, int32_t r, const C& v) { out_psi[r] = v; },
          [&](int k, int32_t r, const C& v) {
            C* o = k == 0 ? o_y1 : (k == 1 ? o_y2 : (k == 2 ? o_y3 : o_b));
            o[r] = v;
          });
}

// One reverse z step of the adjoint in the lambda = H0^{-1} g variables on the
// step tiles (the transpose of the one-kernel step): the Kerr/absorber adjoint
// lam_b = conj(E) lam' + 2 phi b (M mu), mu = gamma Re(i conj(lam') a), then the
// four links of the reverse Horner chain u1 = -h A lam_b, u2 = -(h/2) A u1,
// u3 = -(h/3) A u2, u4 = -(h/4) A u3; lam = lam_b + u1 + u2 + u3 + u4, and the
// index-perturbation gradient grows by
// H0 Re(i [h conj(lam_b) y3 + h/2 conj(u1) y2 + h/3 conj(u2) y1 + h/4 conj(u3) a0]).
// Inputs: lam' (adjoint of the state a after the step), a, the state b before
// the Kerr substep, the step's y1..y3 and its input state a0.  lam_out must not
// alias lam_in (other tiles read lam_in's halo).  CL (complex L weights of a
// perfectly matched layer) also takes sig = H0~ / H0 per row (device order).
template <typename T, int KMAX, bool DEC, int J, bool CL = false>
__global__ void __launch_bounds__((StepBound<T, J>::value)) k_step_adj(DevOps<T> d, TileOps<T> tl,
                                                   const typename CT<T>::C* __restrict__ lam_in,
                                                   const typename CT<T>::C* __restrict__ fa,
                                                   const typename CT<T>::C* __restrict__ fb,
                                                   const typename CT<T>::C* __restrict__ y3,
                                                   const typename CT<T>::C* __restrict__ y2,
                                                   const typename CT<T>::C* __restrict__ y1,
                                                   const typename CT<T>::C* __restrict__ fa0,
                                                   typename CT<T>::C* __restrict__ lam_out,
                                                   double* __restrict__ gdn, T h, T tau, T gamma,
                                                   const typename CT<T>::C* __restrict__ sig) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int MS = tl.max_slots;
  const int B = blockDim.x;
  C* LB = reinterpret_cast<C*>(smem);  // lam' -> lam_b -> u2
  C* U = LB + MS;                      // b -> u1 -> u3
  C* SM = U + MS;                      // (|b|^2 phi, mu) per slot
  StepTile<T, KMAX, DEC, J, CL> st;
  st.init(d, tl, tile);
  st.conj_l();
  // CL (a perfectly matched layer, L~ = H0~^{-1} K~): the Kerr adjoint runs in
  // the lam = H0^{-1} g variables (M and the objective keep the real H0), the
  // linear chain in lam~ = conj(H0~)^{-1} g = lam / conj(sigma), where it
  // applies conj(L~); sigma = H0~ / H0 per row (1 outside the layer)
  auto to_tilde = [&](const C& l, const C& sg) {  // l / conj(sg)
    const T n2 = sg.x * sg.x + sg.y * sg.y;
    C o;
    o.x = (l.x * sg.x - l.y * sg.y) / n2;
    o.y = (l.y * sg.x + l.x * sg.y) / n2;
    return o;
  };
  auto from_tilde = [&](const C& l, const C& sg) {  // conj(sg) l
    C o;
    o.x = sg.x * l.x + sg.y * l.y;
    o.y = sg.x * l.y - sg.y * l.x;
    return o;
  };
  int cr[5];  // slots in rings 0..k
#pragma unroll
  for (int k = 0; k < 5; ++k) cr[k] = st.hd[k];
  // Kerr adjoint rows: rings 0..4 (triangle-averaged: gathered in a phase of
  // its own; lumped: pointwise, done while staging)
  for (int i = threadIdx.x; i < st.nLoad; i += B) {
    const int32_t r = st.slot_row(i);
    const C l = lam_in[r];
    const C aa = fa[r];
    const C bb = fb[r];
    const T w = d.w[r];
    C sm;
    sm.x = (bb.x * bb.x + bb.y * bb.y) * phi_w(w, tau);
    sm.y = -gamma * (l.x * aa.y - l.y * aa.x);  // gamma Re(i conj(lam) a)
    SM[i] = sm;
    if (DEC) {
      LB[i] = l;
      U[i] = bb;
    } else {
      const T md = d.mdiag[r];
      const T th = md * sm.x, mm = md * sm.y;
      const T damp = d_exp(-w * tau);
      T sn, cs;
      d_sincos(gamma * th, &sn, &cs);
      const T two_phi_mm = T(2) * phi_w(w, tau) * mm;
      C o;
      o.x = damp * (cs * l.x + sn * l.y) + two_phi_mm * bb.x;
      o.y = damp * (cs * l.y - sn * l.x) + two_phi_mm * bb.y;
      if constexpr (CL) o = to_tilde(o, sig[r]);
      LB[i] = o;
    }
  }
  // owned rows: forward vectors and the gradient accumulator
  C fy3[J], fy2[J], fy1[J], fa0r[J];
  C sg[J];  // CL: sigma of the slot's row (rings 0..4)
  double h0[J], g0[J], gd[J];  // H0, gradient so far, this step's sum of Re(i conj(u) y) terms
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + j * B;
    h0[j] = g0[j] = gd[j] = 0.0;
    if constexpr (CL) {
      sg[j].x = T(1);
      sg[j].y = T(0);
      if (i < cr[4]) sg[j] = sig[st.rr[j]];
    }
    if (i < cr[0]) {
      const int32_t r = st.rr[j];
      fy3[j] = y3[r];
      fy2[j] = y2[r];
      fy1[j] = y1[r];
      fa0r[j] = fa0[r];
      h0[j] = d.h0[r];
      g0[j] = gdn[r];
    }
  }
  __syncthreads();
  // Re(i conj(u) y) = -(u.x y.y - u.y y.x), u taken back to the lam variables
  auto rdn = [&](const C& ut, const C& y, int j) {
    C u = ut;
    if constexpr (CL) u = from_tilde(ut, sg[j]);
    return -(double(u.x) * y.y - double(u.y) * y.x);
  };
  C cur[J], acc[J];
  if constexpr (DEC) {
#pragma unroll
    for (int j = 0; j < J; ++j) {  // Kerr/absorber adjoint, rings 0..4
      const int i = threadIdx.x + j * B;
      if (i < cr[4]) {
        const C own = SM[i];
        T th = st.md[j] * own.x, mm = st.md[j] * own.y;
        st.template msum2_w<KMAX>(st.wd[j], SM, j, th, mm);
        const T damp = d_exp(-st.ww[j] * tau);
        T sn, cs;
        d_sincos(gamma * th, &sn, &cs);
        const C l = LB[i];
        const C p = U[i];
        const T two_phi_mm = T(2) * phi_w(st.ww[j], tau) * mm;
        C o;
        o.x = damp * (cs * l.x + sn * l.y) + two_phi_mm * p.x;
        o.y = damp * (cs * l.y - sn * l.x) + two_phi_mm * p.y;
        if constexpr (CL) o = to_tilde(o, sg[j]);
        cur[j] = o;
        LB[i] = o;  // only this thread reads LB[i] and U[i] in this phase
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = threadIdx.x + j * B;
      if (i < cr[3]) cur[j] = LB[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {  // link 1, rings 0..3
    const int i = threadIdx.x + j * B;
    if (i < cr[3]) {
      const C u1 = st.link(d, CplxAoS<T>{LB}, cur[j], j, -h);
      U[i] = u1;
      if (i < cr[0]) {
        gd[j] += double(h) * rdn(cur[j], fy3[j], j) + 0.5 * double(h) * rdn(u1, fy2[j], j);
        acc[j].x = cur[j].x + u1.x;
        acc[j].y = cur[j].y + u1.y;
      }
      cur[j] = u1;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {  // link 2, rings 0..2
    const int i = threadIdx.x + j * B;
    if (i < cr[2]) {
      const C u2 = st.link(d, CplxAoS<T>{U}, cur[j], j, T(-0.5) * h);
      LB[i] = u2;
      if (i < cr[0]) {
        gd[j] += double(h) / 3.0 * rdn(u2, fy1[j], j);
        acc[j].x += u2.x;
        acc[j].y += u2.y;
      }
      cur[j] = u2;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {  // link 3, rings 0..1
    const int i = threadIdx.x + j * B;
    if (i < cr[1]) {
      const C u3 = st.link(d, CplxAoS<T>{LB}, cur[j], j, -h / T(3));
      U[i] = u3;
      if (i < cr[0]) {
        gd[j] += 0.25 * double(h) * rdn(u3, fa0r[j], j);
        acc[j].x += u3.x;
        acc[j].y += u3.y;
      }
      cur[j] = u3;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {  // link 4, owned rows
    const int i = threadIdx.x + j * B;
    if (i < cr[0]) {
      const C u4 = st.link(d, CplxAoS<T>{U}, cur[j], j, T(-0.25) * h);
      C l;
      l.x = acc[j].x + u4.x;
      l.y = acc[j].y + u4.y;
      if constexpr (CL) l = from_tilde(l, sg[j]);
      lam_out[st.rr[j]] = l;
      gdn[st.rr[j]] = g0[j] + h0[j] * gd[j];
    }
  }
}

// ---- persistent z stepping on resident tiles ----
// n_steps z steps in one launch, one workgroup per tile, all resident (an
// ordinary launch of a grid that fits, or a cooperative one).  The operator
// rows stay in registers for the whole
// launch; per step only the state crosses memory.  The state alternates
// between buf0 (before even steps) and buf1.  Flags only grow: a tile
// publishes flags[tile] = base + k once the state its step k - 1 produced is
// stored (k = 0 being the starting state when the launch makes it itself), and
// before reading a state it waits for every tile that owns one of its halo
// rows to have published it.  The halo relation is symmetric, so that wait
// also guarantees the neighbours have finished reading the buffer this tile is
// about to overwrite.  Exchanged elements and flags are agent-scope atomic
// accesses (coherent across XCDs); each wave waits for its state stores to be
// acknowledged before the workgroup barrier that precedes the flag store, and
// the state loads follow the barrier that ends the flag wait, so no L2
// write-back or invalidate is needed.  Each wait is bounded: after spin_limit
// polls the tile sets bit 1 of *status and leaves, and its neighbours then
// time out in turn, so every workgroup exits.
// With io.in (split-step body) the launch starts from the caller's field: each
// tile applies NL(tau_first) to its owned rows (reading rings 0..1 through the
// permutation) and publishes them as the starting state.  With io.out the last
// step applies NL(tau_last) and writes the caller's field through the
// permutation.  The caller's field is read only before a tile's first flag and
// written only after its first wait, which every tile reading those rows has
// passed, so out may alias in.
// BODY 0: the merged split step; BODY 1: one unsplit classical RK4 step of the
// whole right-hand side (the stage inputs and their |.|^2 double-buffered in
// the same LDS; the owned state and its |.|^2 written back after the step).
// CL: complex L weights (a perfectly matched layer), in complex64.
// FX (split-step body, complex64): the fixed LDS layout (see kFixSlots).

template <typename T>
struct PersistArgs {
  using C = typename CT<T>::C;
  const C* in;
  C* out;
  const int32_t* perm;
  int32_t base;
  T tau_first, tau_last;
};

template <typename T, int KMAX, bool DEC, int J, int LS, int BODY, bool CL = false, bool FX = false>
__global__ void __launch_bounds__(1024) k_persist(DevOps<T> d, TileOps<T> tl, const int32_t* __restrict__ nb_ptr,
                                                  const int32_t* __restrict__ nb_list, typename CT<T>::C* buf0,
                                                  typename CT<T>::C* buf1, int32_t* flags, int32_t* status,
                                                  int32_t n_steps, int32_t spin_limit, T h, T gamma,
                                                  PersistArgs<T> io) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t nb_s[64];
  __shared__ int32_t abort_s;
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  static_assert(!FX || (BODY == 0 && sizeof(T) == 4), "the fixed layout is for the complex64 split step");
  const int MS = FX ? kFixSlots : tl.max_slots;
  const int B = blockDim.x;
  C* base = reinterpret_cast<C*>(smem);
  if constexpr (FX) {  // static LDS: its address is a constant the gathers can carry
    __shared__ __align__(16) unsigned char fx_lds[4 * kFixSlots * sizeof(C)];
    base = reinterpret_cast<C*>(fx_lds);
  }
  const CplxAoS<T> P{base}, X{base + MS}, Y{base + 2 * MS};
  T* S = reinterpret_cast<T*>(base + 3 * MS);
  C* UA = base;  // BODY 1: stage buffers A, B and their |.|^2
  C* UB = base + MS;
  T* USA = reinterpret_cast<T*>(base + 2 * MS);
  T* USB = USA + MS;
  StepTile<T, KMAX, DEC, J, CL, false, FX> st;
  st.init(d, tl, tile, false, nullptr, BODY == 0);
  int32_t pr[LS];  // rows of this thread's state slots
#pragma unroll
  for (int l = 0; l < LS; ++l) {
    const int i = threadIdx.x + l * B;
    pr[l] = i < st.nLoad ? st.slot_row(i) : -1;
  }
  const int32_t nb0 = nb_ptr[tile];
  const int n_nb = nb_ptr[tile + 1] - nb0;
  if (threadIdx.x < n_nb) nb_s[threadIdx.x] = nb_list[nb0 + threadIdx.x];
  const bool pro = BODY == 0 && io.in != nullptr;
  if (pro) {  // the starting state: NL(tau_first) of the caller's field, owned rows
    st.kerr_from(d, io.in, io.perm, S, io.tau_first, gamma, [&](int i, int32_t r, const C& v) {
      coherent_store(buf0 + r, v);
      P.put(i, v);
    });
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + tile, io.base + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if constexpr (BODY == 0) {  // the starting state is in buf0: its owned rows into P
#pragma unroll
    for (int l = 0; l < LS; ++l)
      if (pr[l] >= 0 && int(threadIdx.x) + l * B < st.nNL) P.put(threadIdx.x + l * B, coherent_load(buf0 + pr[l]));
  }
  __syncthreads();
  // wait until every neighbour tile has published `need`; false if the wait gave up
  auto wait_nb = [&](int32_t need) -> bool {
    if (threadIdx.x < 64) {  // one wave polls all neighbour flags at once
      // lanes without a neighbour poll this tile's own flag, which already
      // holds the value (published at the end of the previous step)
      const int32_t* fl = flags + (int(threadIdx.x) < n_nb ? nb_s[threadIdx.x] : int32_t(tile));
      bool ok = true;
      for (int32_t spins = 0;; ++spins) {
        if (__all(__hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need)) break;
        if (spins >= spin_limit) {
          ok = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (threadIdx.x == 0) {
        abort_s = ok ? 0 : 1;
        if (!ok) __hip_atomic_fetch_or(status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    return !abort_s;
  };
  // stage slots first.. of the state in src: the owned slots (ring 0) stay in
  // LDS from the previous step (or the prologue), so only the halo is loaded
  auto stage_state = [&](const C* src, int first) {
    C pv[LS];  // issue every load before the first use
#pragma unroll
    for (int l = 0; l < LS; ++l)
      if (pr[l] >= 0 && int(threadIdx.x) + l * B >= first) pv[l] = coherent_load(src + pr[l]);
#pragma unroll
    for (int l = 0; l < LS; ++l)
      if (pr[l] >= 0 && int(threadIdx.x) + l * B >= first) {
        if constexpr (BODY == 0) {
          P.put(threadIdx.x + l * B, pv[l]);
        } else {
          UA[threadIdx.x + l * B] = pv[l];
          USA[threadIdx.x + l * B] = pv[l].x * pv[l].x + pv[l].y * pv[l].y;
        }
      }
    __syncthreads();
  };
  for (int32_t s = 0; s < n_steps; ++s) {
    st.opaque_neighbours();
    const C* src = (s & 1) ? buf1 : buf0;
    C* dst = (s & 1) ? buf0 : buf1;
    const int32_t need = io.base + s + (pro ? 1 : 0);  // flag of the state step s reads
    const bool fin = io.out != nullptr && s == n_steps - 1;  // the last step: the result goes to the caller's field
    if constexpr (BODY == 0) {
      // the split step: the owned rows that need no halo are stepped while the
      // neighbours finish; the rest after the wait
      auto mid = [&]() -> bool {
        if ((s > 0 || pro) && !wait_nb(need)) return false;
        stage_state(src, st.nNL);
        return true;
      };
      if (fin) {
        auto res = [&](int, int32_t r, const C& v) { put_result(io.out, io.perm, status, r, v); };
        if (!st.step_split(d, P, X, Y, S, h, io.tau_last, gamma, res, res, mid)) return;
        break;
      }
      // rows deeper than the halo rings are read by no other tile: they stay in
      // LDS, and reach the state buffer only when the launch ends there
      const bool keep = io.out == nullptr && s == n_steps - 1;
      if (!st.step_split(d, P, X, Y, S, h, h, gamma,
                         [&](int i, int32_t r, const C& v) {
                           if (keep) dst[r] = v;
                           P.put(i, v);
                         },
                         [&](int i, int32_t r, const C& v) {
                           coherent_store(dst + r, v);
                           P.put(i, v);  // the next step's owned state
                         },
                         mid))
        return;
    } else {
      if ((s > 0 || pro) && !wait_nb(need)) return;
      stage_state(src, s == 0 ? 0 : st.nNL);
      if (fin) {
        st.step_unsplit(d, UA, UB, USA, USB, h, gamma,
                        [&](int, int32_t r, const C& v) { put_result(io.out, io.perm, status, r, v); });
        break;
      }
      // the last stage reads B only, so the owned state can go back into A
      st.step_unsplit(d, UA, UB, USA, USB, h, gamma, [&](int i, int32_t r, const C& v) {
        coherent_store(dst + r, v);
        UA[i] = v;
        USA[i] = v.x * v.x + v.y * v.y;
      });
    }
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flags + tile, need + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_zero_i32(int64_t n, int32_t* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// ---- fused adjoint kernels on LDS tiles (lambda = H0^{-1} g variables) ----
// AD1: Kerr/absorber adjoint (rings 0..2), chain links 1 and 2 of the reverse
//      RK4 (rings 0..1, ring 0):  lam_b = conj(E) lam + 2 phi b (M mu),
//      u1 = -h A lam_b,  u2 = -(h/2) A u1;  writes u2, acc = lam_b + u1 + u2 and
//      adds the link-1..3 terms of dJ/d(dn) (forward vectors y3, y2, y1).
// AD2: links 3 and 4: u3 = -(h/3) A u2 (rings 0..1), u4 = -(h/4) A u3;
//      lam_new = acc + u3 + u4; adds the link-4 term (forward state a).
template <typename T, int KMAX, bool DEC, int KIND, int J>
__global__ void __launch_bounds__(1024) k_fused_adj(DevOps<T> d, TileOps<T> tl,
                                                    const typename CT<T>::C* __restrict__ vin,
                                                    const typename CT<T>::C* __restrict__ fa,
                                                    const typename CT<T>::C* __restrict__ fb,
                                                    const typename CT<T>::C* __restrict__ y3,
                                                    const typename CT<T>::C* __restrict__ y2,
                                                    const typename CT<T>::C* __restrict__ y1,
                                                    typename CT<T>::C* __restrict__ out_u,
                                                    typename CT<T>::C* __restrict__ acc,
                                                    double* __restrict__ gdn, T h, T tau, T gamma) {
  using C = typename CT<T>::C;
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t tile = logical_block(d.xcd_remap);
  if (tile >= tl.n_tiles) return;
  const int32_t* hd = tl.hdr + 8 * tile;
  const int c0 = hd[0], c1 = c0 + hd[1], c2 = c1 + hd[2], c3 = c2 + hd[3];
  const int32_t* __restrict__ ext = tl.ext + hd[4];
  const int32_t* __restrict__ lsl = tl.lsl + hd[5];
  const int64_t ebase = tl.ent_base[tile];
  const int64_t row0 = tile * int64_t(tl.TS);
  const int MS = tl.max_slots;
  const int B = blockDim.x;
  C* Lm = reinterpret_cast<C*>(smem);  // AD1: lam -> lam_b; AD2: u2
  C* U = Lm + MS;                      // AD1: u1; AD2: u3
  C* Bs = U + MS;                      // AD1: b (state before the Kerr substep)
  C* SM = Bs + MS;                     // AD1: (s, mu) per slot
  const int nNL = c2;                  // AD1: Kerr adjoint rows
  const int nLoad = KIND == 1 ? (DEC ? c3 : c2) : c2;
  for (int i = threadIdx.x; i < nLoad; i += B) {
    const int32_t r = i < c0 ? int32_t(row0 + i) : ext[i - c0];
    const C l = vin[r];
    if (KIND == 1) {
      const C bb = fb[r];
      const C aa = fa[r];
      C sm;
      sm.x = (bb.x * bb.x + bb.y * bb.y) * phi_w(d.w[r], tau);
      sm.y = -gamma * (l.x * aa.y - l.y * aa.x);  // gamma Re(i conj(lam) a)
      SM[i] = sm;
      if (i < nNL) {
        Bs[i] = bb;
        Lm[i] = l;
      }
    } else {
      Lm[i] = l;
    }
  }
  int q[J][KMAX];
  T cl[J][KMAX];
  T cm[J][DEC ? KMAX : 1];
  int wd[J];
  int32_t rr[J];
  T vv[J], ww[J], md[J];
  C fy3[J], fy2[J], fy1[J], fac[J];
  double h0[J], gd[J];
  const int nRows = c2;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + j * B;
    wd[j] = 0;
    rr[j] = 0;
    vv[j] = ww[j] = md[j] = T(0);
    h0[j] = gd[j] = 0.0;
    if (i < nRows) {
      const int32_t r = i < c0 ? int32_t(row0 + i) : ext[i - c0];
      rr[j] = r;
      vv[j] = d.v[r];
      ww[j] = d.w[r];
      md[j] = d.mdiag[r];
      const int32_t info = lsl[i >> 6];
      wd[j] = info & 0xff;
      const int64_t base = ebase + (info >> 8) + (i & 63);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < wd[j]) {
          q[j][k] = tl.lcol[base + 64 * k];
          cl[j][k] = tl.llw[base + 64 * k];
          if (DEC) cm[j][k] = tl.lmw[base + 64 * k];
        } else {
          q[j][k] = i;
          cl[j][k] = T(0);
          if (DEC) cm[j][k] = T(0);
        }
      }
      if (i < c0) {  // owned rows: forward vectors, accumulators
        h0[j] = d.h0[r];
        gd[j] = gdn[r];
        if (KIND == 1) {
          fy3[j] = y3[r];
          fy2[j] = y2[r];
          fy1[j] = y1[r];
        } else {
          fac[j] = acc[r];
          fy1[j] = fa[r];
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        q[j][k] = 0;
        cl[j][k] = T(0);
        if (DEC) cm[j][k] = T(0);
      }
    }
  }
  __syncthreads();

  // coef * (-i) (p1 L v - V v) at register slot j, v gathered from V_
  auto link = [&](const C* V_, int j, int i, T coef) {
    const C vr = V_[i];
    T ar = T(0), ai = T(0);
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      {  // padded slots: self column, zero weight
        const C vq = V_[q[j][k]];
        ar += cl[j][k] * (vr.x - vq.x);
        ai += cl[j][k] * (vr.y - vq.y);
      }
    const T hr = d.p1 * ar - vv[j] * vr.x;
    const T hi = d.p1 * ai - vv[j] * vr.y;
    C o;
    o.x = coef * hi;
    o.y = -coef * hr;
    return o;
  };
  // Re(i conj(u) y) = -(u.x y.y - u.y y.x)
  auto rdn = [](const C& u, const C& y) { return -(double(u.x) * y.y - double(u.y) * y.x); };

  if (KIND == 1) {
#pragma unroll
    for (int j = 0; j < J; ++j) {  // Kerr/absorber adjoint
      const int i = threadIdx.x + j * B;
      if (i < nNL) {
        const C own = SM[i];
        T th = md[j] * own.x, mm = md[j] * own.y;
        if (DEC) {
#pragma unroll
          for (int k = 0; k < KMAX; ++k)
            {  // padded slots: self column, zero weight
              const C v = SM[q[j][k]];
              th += cm[j][k] * v.x;
              mm += cm[j][k] * v.y;
            }
        }
        const T damp = d_exp(-ww[j] * tau);
        T sn, cs;
        d_sincos(gamma * th, &sn, &cs);
        const C l = Lm[i];
        const C p = Bs[i];
        const T two_phi_mm = T(2) * phi_w(ww[j], tau) * mm;
        C o;
        o.x = damp * (cs * l.x + sn * l.y) + two_phi_mm * p.x;
        o.y = damp * (cs * l.y - sn * l.x) + two_phi_mm * p.y;
        Lm[i] = o;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {  // link 1
      const int i = threadIdx.x + j * B;
      if (i < c1) U[i] = link(Lm, j, i, -h);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {  // link 2, accumulators
      const int i = threadIdx.x + j * B;
      if (i < c0) {
        const C lb = Lm[i];
        const C u1 = U[i];
        const C u2 = link(U, j, i, T(-0.5) * h);
        out_u[rr[j]] = u2;
        C a;
        a.x = lb.x + u1.x + u2.x;
        a.y = lb.y + u1.y + u2.y;
        acc[rr[j]] = a;
        gdn[rr[j]] = gd[j] + h0[j] * (double(h) * rdn(lb, fy3[j]) + 0.5 * double(h) * rdn(u1, fy2[j]) +
                                      double(h) / 3.0 * rdn(u2, fy1[j]));
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {  // link 3
      const int i = threadIdx.x + j * B;
      if (i < c1) U[i] = link(Lm, j, i, -h / T(3));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {  // link 4, new adjoint state
      const int i = threadIdx.x + j * B;
      if (i < c0) {
        const C u3 = U[i];
        const C u4 = link(U, j, i, T(-0.25) * h);
        C l;
        l.x = fac[j].x + u3.x + u4.x;
        l.y = fac[j].y + u3.y + u4.y;
        out_u[rr[j]] = l;
        gdn[rr[j]] = gd[j] + h0[j] * 0.25 * double(h) * rdn(u3, fy1[j]);
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
#define DECBPM_C(T, p) reinterpret_cast<const typename CT<T>::C*>(p)
#define DECBPM_M(T, p) reinterpret_cast<typename CT<T>::C*>(p)

template <typename T>
inline int fb_of(const DevOps<T>& d) {
  return d.F == 1 ? 1 : (d.lgF >= 0 ? 2 : 0);
}
inline int kmax_of(int wmax) { return wmax <= 8 ? 8 : (wmax <= 12 ? 12 : 0); }

// Expand BODY for the (rows-per-field mode, unroll) pair of `d`.
#define DECBPM_DISPATCH_FB_K(d, BODY)            \
  switch (fb_of(d) * 100 + kmax_of((d).wmax)) {  \
    case 108: { constexpr int FB = 1, KM = 8; BODY; } break;   \
    case 112: { constexpr int FB = 1, KM = 12; BODY; } break;  \
    case 100: { constexpr int FB = 1, KM = 0; BODY; } break;   \
    case 208: { constexpr int FB = 2, KM = 8; BODY; } break;   \
    case 212: { constexpr int FB = 2, KM = 12; BODY; } break;  \
    case 200: { constexpr int FB = 2, KM = 0; BODY; } break;   \
    case 8: { constexpr int FB = 0, KM = 8; BODY; } break;     \
    case 12: { constexpr int FB = 0, KM = 12; BODY; } break;   \
    default: { constexpr int FB = 0, KM = 0; BODY; } break;    \
  }
#define DECBPM_DISPATCH_K(d, BODY)                               \
  switch (kmax_of((d).wmax)) {                                   \
    case 8: { constexpr int KM = 8; BODY; } break;               \
    case 12: { constexpr int KM = 12; BODY; } break;             \
    default: { constexpr int KM = 0; BODY; } break;              \
  }
#define DECBPM_DISPATCH_FB(d, BODY)                               \
  switch (fb_of(d)) {                                             \
    case 1: { constexpr int FB = 1; BODY; } break;                \
    case 2: { constexpr int FB = 2; BODY; } break;                \
    default: { constexpr int FB = 0; BODY; } break;               \
  }

// Fields per thread of the batched kernels: 32 bytes of complex values.
template <typename T>
inline int vf_of(const DevOps<T>& d) {
  constexpr int VF = int(32 / sizeof(typename CT<T>::C));
  return (d.F > 1 && d.F % VF == 0) ? VF : 1;
}

#define DECBPM_DISPATCH_W(d, BODY)                                   \
  switch (kmax_of((d).wmax)) {                                       \
    case 8: { constexpr int KM = 8; constexpr int VF = int(32 / sizeof(typename CT<T>::C)); BODY; } break;   \
    case 12: { constexpr int KM = 12; constexpr int VF = int(32 / sizeof(typename CT<T>::C)); BODY; } break; \
    default: { constexpr int KM = 0; constexpr int VF = int(32 / sizeof(typename CT<T>::C)); BODY; } break;  \
  }

template <typename T>
void launch_stage(const DevOps<T>& d, const void* x, const void* t, const void* psi, void* y, double coef,
                  void* s_out, double tau_s, int block, hipStream_t st) {
  if (vf_of(d) > 1) {
    const unsigned gw = grid_for(d.n_rows * d.F / vf_of(d), block, d.xcd_remap);
    T* sw = reinterpret_cast<T*>(s_out);
    const int mode = (t != nullptr) * 2 + (s_out != nullptr);
#define DECBPM_STAGE_W(B4, WS)                                                                                \
  hipLaunchKernelGGL((k_stage_w<T, VF, KM, B4, WS>), dim3(gw), dim3(block), 0, st, d, DECBPM_C(T, x),          \
                     DECBPM_C(T, t), DECBPM_C(T, psi), DECBPM_M(T, y), T(coef), sw, T(tau_s))
    DECBPM_DISPATCH_W(d, {
      if (mode == 0) DECBPM_STAGE_W(false, false);
      else if (mode == 1) DECBPM_STAGE_W(false, true);
      else if (mode == 2) DECBPM_STAGE_W(true, false);
      else DECBPM_STAGE_W(true, true);
    })
#undef DECBPM_STAGE_W
    return;
  }
  const unsigned g = grid_for(d.n_rows * d.F, block, d.xcd_remap);
  T* s = reinterpret_cast<T*>(s_out);
#define DECBPM_STAGE(B4, WS)                                                                                 \
  hipLaunchKernelGGL((k_stage<T, FB, KM, B4, WS>), dim3(g), dim3(block), 0, st, d, DECBPM_C(T, x),            \
                     DECBPM_C(T, t), DECBPM_C(T, psi), DECBPM_M(T, y), T(coef), s, T(tau_s))
  const int mode = (t != nullptr) * 2 + (s_out != nullptr);
  DECBPM_DISPATCH_FB_K(d, {
    if (mode == 0) DECBPM_STAGE(false, false);
    else if (mode == 1) DECBPM_STAGE(false, true);
    else if (mode == 2) DECBPM_STAGE(true, false);
    else DECBPM_STAGE(true, true);
  })
#undef DECBPM_STAGE
}

template <typename T>
void launch_lap(const DevOps<T>& d, const void* x, void* t, int block, hipStream_t st) {
  if (vf_of(d) > 1) {
    const unsigned gw = grid_for(d.n_rows * d.F / vf_of(d), block, d.xcd_remap);
    DECBPM_DISPATCH_W(d, hipLaunchKernelGGL((k_lap_w<T, VF, KM>), dim3(gw), dim3(block), 0, st, d, DECBPM_C(T, x),
                                            DECBPM_M(T, t)))
    return;
  }
  const unsigned g = grid_for(d.n_rows * d.F, block, d.xcd_remap);
  DECBPM_DISPATCH_FB_K(d, hipLaunchKernelGGL((k_lap<T, FB, KM>), dim3(g), dim3(block), 0, st, d, DECBPM_C(T, x),
                                             DECBPM_M(T, t)))
}

template <typename T>
void launch_lapc(const DevOps<T>& d, const void* z, const void* x, double a, double b, void* y, int block,
                 hipStream_t st) {
  const unsigned g = grid_for(d.n_rows, block, d.xcd_remap);
  DECBPM_DISPATCH_K(d, hipLaunchKernelGGL((k_lapc<T, KM>), dim3(g), dim3(block), 0, st, d, DECBPM_C(T, z),
                                          DECBPM_C(T, x), T(a), T(b), DECBPM_M(T, y)))
}

template <typename T>
void launch_prep_s(const DevOps<T>& d, const void* psi, void* s, double tau, int block, hipStream_t st) {
  if (vf_of(d) > 1) {
    constexpr int VF = int(32 / sizeof(typename CT<T>::C));
    const unsigned gw = grid_for(d.n_rows * d.F / VF, block, d.xcd_remap);
    hipLaunchKernelGGL((k_prep_w<T, VF>), dim3(gw), dim3(block), 0, st, d, DECBPM_C(T, psi), reinterpret_cast<T*>(s),
                       T(tau));
    return;
  }
  const unsigned g = grid_for(d.n_rows * d.F, block, d.xcd_remap);
  DECBPM_DISPATCH_FB(d, hipLaunchKernelGGL((k_prep_s<T, FB>), dim3(g), dim3(block), 0, st, d, DECBPM_C(T, psi),
                                           reinterpret_cast<T*>(s), T(tau)))
}

template <typename T>
void launch_kerr(const DevOps<T>& d, const void* psi_in, void* psi_out, const void* s, double tau, double gamma,
                 int block, hipStream_t st) {
  const T* sp = reinterpret_cast<const T*>(s);
  if (vf_of(d) > 1) {
    const unsigned gw = grid_for(d.n_rows * d.F / vf_of(d), block, d.xcd_remap);
    if (d.mw) {
      DECBPM_DISPATCH_W(d, hipLaunchKernelGGL((k_kerr_w<T, VF, KM, true>), dim3(gw), dim3(block), 0, st, d,
                                              DECBPM_C(T, psi_in), DECBPM_M(T, psi_out), sp, T(tau), T(gamma)))
    } else {
      constexpr int VF = int(32 / sizeof(typename CT<T>::C));
      hipLaunchKernelGGL((k_kerr_w<T, VF, 0, false>), dim3(gw), dim3(block), 0, st, d, DECBPM_C(T, psi_in),
                         DECBPM_M(T, psi_out), sp, T(tau), T(gamma));
    }
    return;
  }
  const unsigned g = grid_for(d.n_rows * d.F, block, d.xcd_remap);
  if (d.mw) {
    DECBPM_DISPATCH_FB_K(d, hipLaunchKernelGGL((k_kerr<T, FB, KM, true>), dim3(g), dim3(block), 0, st, d,
                                               DECBPM_C(T, psi_in), DECBPM_M(T, psi_out), sp, T(tau), T(gamma)))
  } else {
    DECBPM_DISPATCH_FB(d, hipLaunchKernelGGL((k_kerr<T, FB, 0, false>), dim3(g), dim3(block), 0, st, d,
                                             DECBPM_C(T, psi_in), DECBPM_M(T, psi_out), sp, T(tau), T(gamma)))
  }
}

template <typename T>
void launch_fused(const DevOps<T>& d, const TileOps<T>& tl, int kind, const void* in_x, const void* in_psi,
                  void* out_psi, void* out_y, void* out_rec, double h, double tau, double gamma, int block,
                  hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (3 * sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;  // slots per thread (1 or 2)
#define DECBPM_FUSED(KM, DEC, KIND, JJ)                                                                          \
  hipLaunchKernelGGL((k_fused<T, KM, DEC, KIND, JJ>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in_x), \
                     DECBPM_C(T, in_psi), DECBPM_M(T, out_psi), DECBPM_M(T, out_y), DECBPM_M(T, out_rec), T(h),  \
                     T(tau), T(gamma))
#define DECBPM_FUSED_J(KM, DEC, KIND) \
  if (J <= 1) DECBPM_FUSED(KM, DEC, KIND, 1); else DECBPM_FUSED(KM, DEC, KIND, 2);
#define DECBPM_FUSED_K(KM, DEC)                                  \
  switch (kind) {                                                \
    case FUSED_S4_NL_S1: DECBPM_FUSED_J(KM, DEC, 0); break;      \
    case FUSED_S2_S3: DECBPM_FUSED_J(KM, DEC, 1); break;         \
    case FUSED_NL_S1: DECBPM_FUSED_J(KM, DEC, 2); break;         \
    default: DECBPM_FUSED_J(KM, DEC, 3); break;                  \
  }
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_FUSED_K(8, true) } else { DECBPM_FUSED_K(8, false) }
  } else {
    if (dec) { DECBPM_FUSED_K(12, true) } else { DECBPM_FUSED_K(12, false) }
  }
#undef DECBPM_FUSED_K
#undef DECBPM_FUSED_J
#undef DECBPM_FUSED
}

template <typename T>
void launch_fused_adj(const DevOps<T>& d, const TileOps<T>& tl, int kind, const void* vin, const void* fa,
                      const void* fb, const void* y3, const void* y2, const void* y1, void* out_u, void* acc,
                      double* gdn, double h, double tau, double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * 4 * sizeof(typename CT<T>::C);
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_FADJ(KM, DEC, KIND, JJ)                                                                            \
  hipLaunchKernelGGL((k_fused_adj<T, KM, DEC, KIND, JJ>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, vin), \
                     DECBPM_C(T, fa), DECBPM_C(T, fb), DECBPM_C(T, y3), DECBPM_C(T, y2), DECBPM_C(T, y1),          \
                     DECBPM_M(T, out_u), DECBPM_M(T, acc), gdn, T(h), T(tau), T(gamma))
#define DECBPM_FADJ_J(KM, DEC, KIND) \
  if (J <= 1) DECBPM_FADJ(KM, DEC, KIND, 1); else DECBPM_FADJ(KM, DEC, KIND, 2);
#define DECBPM_FADJ_K(KM, DEC)                    \
  if (kind == 1) { DECBPM_FADJ_J(KM, DEC, 1) }    \
  else { DECBPM_FADJ_J(KM, DEC, 2) }
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_FADJ_K(8, true) } else { DECBPM_FADJ_K(8, false) }
  } else {
    if (dec) { DECBPM_FADJ_K(12, true) } else { DECBPM_FADJ_K(12, false) }
  }
#undef DECBPM_FADJ_K
#undef DECBPM_FADJ_J
#undef DECBPM_FADJ
}

template <typename T>
void launch_bstage(const DevOps<T>& d, const TileOps<T>& tl, const void* x, const void* t, const void* psi, void* y,
                   double coef, void* s_out, double tau_s, hipStream_t st) {
  constexpr int VF = int(32 / sizeof(typename CT<T>::C));
  const int tpr = d.F / VF;
  const int block = std::min(1024, std::max(64, (tl.TS * tpr + 63) / 64 * 64));
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * d.F * sizeof(typename CT<T>::C);
  T* sw = reinterpret_cast<T*>(s_out);
  const int mode = (t != nullptr) * 2 + (s_out != nullptr);
#define DECBPM_BSTAGE(B4, WS)                                                                                      \
  hipLaunchKernelGGL((k_bstage<T, VF, KM, B4, WS>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, x),         \
                     DECBPM_C(T, t), DECBPM_C(T, psi), DECBPM_M(T, y), T(coef), sw, T(tau_s))
  if (kmax_of(d.wmax) == 8) {
    constexpr int KM = 8;
    if (mode == 0) DECBPM_BSTAGE(false, false);
    else if (mode == 1) DECBPM_BSTAGE(false, true);
    else if (mode == 2) DECBPM_BSTAGE(true, false);
    else DECBPM_BSTAGE(true, true);
  } else {
    constexpr int KM = 12;
    if (mode == 0) DECBPM_BSTAGE(false, false);
    else if (mode == 1) DECBPM_BSTAGE(false, true);
    else if (mode == 2) DECBPM_BSTAGE(true, false);
    else DECBPM_BSTAGE(true, true);
  }
#undef DECBPM_BSTAGE
}

template <typename T>
void launch_blap(const DevOps<T>& d, const TileOps<T>& tl, const void* x, void* t, hipStream_t st) {
  constexpr int VF = int(32 / sizeof(typename CT<T>::C));
  const int tpr = d.F / VF;
  const int block = std::min(1024, std::max(64, (tl.TS * tpr + 63) / 64 * 64));
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * d.F * sizeof(typename CT<T>::C);
  if (kmax_of(d.wmax) == 8)
    hipLaunchKernelGGL((k_blap<T, VF, 8>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, x), DECBPM_M(T, t));
  else
    hipLaunchKernelGGL((k_blap<T, VF, 12>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, x), DECBPM_M(T, t));
}

template <typename T>
void launch_bkerr(const DevOps<T>& d, const TileOps<T>& tl, const void* psi_in, void* psi_out, const void* s,
                  double tau, double gamma, hipStream_t st) {
  constexpr int VF = int(32 / sizeof(typename CT<T>::C));
  const int tpr = d.F / VF;
  const int block = std::min(1024, std::max(64, (tl.TS * tpr + 63) / 64 * 64));
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * d.F * sizeof(T);
  const T* sp = reinterpret_cast<const T*>(s);
  DECBPM_DISPATCH_K(d, hipLaunchKernelGGL((k_bkerr<T, VF, KM>), dim3(g), dim3(block), shmem, st, d, tl,
                                          DECBPM_C(T, psi_in), DECBPM_M(T, psi_out), sp, T(tau), T(gamma)))
}

template <typename T>
void launch_bstep(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h, double tau,
                  double gamma, int block, hipStream_t st) {
  constexpr int VF = int(32 / sizeof(typename CT<T>::C));  // 32 bytes of each state vector per slot
  const int G = d.F / VF;
  const unsigned g = grid_for(int64_t(tl.n_tiles) * G * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (3 * sizeof(CVec<T, VF>) + sizeof(RVec<T, VF>));
  const int J = (tl.max_compute + block - 1) / block;
  using V = CVec<T, VF>;
#define DECBPM_BSTEP(KM, DEC, JJ)                                                                                   \
  hipLaunchKernelGGL((k_bstep<T, KM, DEC, JJ, VF>), dim3(g), dim3(block), shmem, st, d, tl,                         \
                     reinterpret_cast<const V*>(in_psi), reinterpret_cast<V*>(out_psi), T(h), T(tau), T(gamma))
#define DECBPM_BSTEP_J(KM, DEC) \
  if (J <= 1) DECBPM_BSTEP(KM, DEC, 1); else DECBPM_BSTEP(KM, DEC, 2);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_BSTEP_J(8, true) } else { DECBPM_BSTEP_J(8, false) }
  } else {
    if (dec) { DECBPM_BSTEP_J(12, true) } else { DECBPM_BSTEP_J(12, false) }
  }
#undef DECBPM_BSTEP_J
#undef DECBPM_BSTEP
}

template <typename T>
void launch_step(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h, double tau,
                 double gamma, int block, hipStream_t st, const int32_t* out_perm, int* flag) {
  if (d.F > 1) {  // batched handle: VF fields per slot
    launch_bstep<T>(d, tl, in_psi, out_psi, h, tau, gamma, block, st);
    return;
  }
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (3 * sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_STEP(KM, DEC, JJ, CLX)                                                                          \
  hipLaunchKernelGGL((k_step<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in_psi), \
                     DECBPM_M(T, out_psi), T(h), T(tau), T(gamma), out_perm, flag)
  // complex L weights (perfectly matched layer): their own instantiation
#define DECBPM_STEP_J(KM, DEC)                                                   \
  if (tl.llwi) {                                                                 \
    if (J <= 1) DECBPM_STEP(KM, DEC, 1, true); else DECBPM_STEP(KM, DEC, 2, true); \
  } else {                                                                       \
    if (J <= 1) DECBPM_STEP(KM, DEC, 1, false); else DECBPM_STEP(KM, DEC, 2, false); \
  }
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_STEP_J(8, true) } else { DECBPM_STEP_J(8, false) }
  } else {
    if (dec) { DECBPM_STEP_J(12, true) } else { DECBPM_STEP_J(12, false) }
  }
#undef DECBPM_STEP_J
#undef DECBPM_STEP
}

#if DECBPM_PART & 1
void launch_dp5_init(Dp5Ctl* ctl, uint32_t* arrivals, double z_end, double h0, int64_t max_attempts, double facmax,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_dp5_init, dim3(1), dim3(64), 0, st, ctl, arrivals, z_end, h0, max_attempts, facmax);
}
#endif

template <typename T>
void launch_dp5(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, Dp5Ctl* ctl, double* partial,
                uint32_t* arrivals, double gamma, double rtol, double atol, double inv_n, int block, hipStream_t st) {
  using C = typename CT<T>::C;
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * 2 * (sizeof(C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_DP5C(KM, DEC, JJ, CLX)                                                                              \
  hipLaunchKernelGGL((k_dp5<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl, static_cast<C*>(x0),     \
                     static_cast<C*>(x1), ctl, partial, arrivals, T(gamma), T(rtol), T(atol), inv_n)
  // complex L weights (a PML): the imaginary parts in a second register array
  const bool cl = tl.llwi != nullptr;
#define DECBPM_DP5(KM, DEC, JJ)           \
  if (cl) DECBPM_DP5C(KM, DEC, JJ, true); \
  else DECBPM_DP5C(KM, DEC, JJ, false)
  // complex128 tiles keep every compute slot on its own thread (J = 1): two
  // slots of rows with 12 neighbours need more than the 128 registers of a
  // 1024-thread workgroup, and halving the workgroup costs more than the spills
#define DECBPM_DP5_J(KM, DEC)                          \
  if constexpr (sizeof(T) == 8) DECBPM_DP5(KM, DEC, 1); \
  else if (J <= 1) DECBPM_DP5(KM, DEC, 1);              \
  else DECBPM_DP5(KM, DEC, 2);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_DP5_J(8, true) } else { DECBPM_DP5_J(8, false) }
  } else {
    if (dec) { DECBPM_DP5_J(12, true) } else { DECBPM_DP5_J(12, false) }
  }
#undef DECBPM_DP5_J
#undef DECBPM_DP5
#undef DECBPM_DP5C
}

#if DECBPM_PART & 1
void launch_mode_init(ModeCtl* ctl, uint32_t* arrivals, const double* pw, double power, double tol, int64_t max_iter,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mode_init, dim3(1), dim3(64), 0, st, ctl, arrivals, pw, power, tol, max_iter);
}
#endif

template <typename T>
void launch_scale(int64_t n, void* x, double s, int block, hipStream_t st) {
  const unsigned g = unsigned((n + block - 1) / block);
  if (g) hipLaunchKernelGGL((k_scale<T>), dim3(g), dim3(block), 0, st, static_cast<typename CT<T>::C*>(x), n, T(s));
}

template <typename T>
void launch_mode(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, ModeCtl* ctl, double* partial,
                 uint32_t* arrivals, double h, double gamma, int block, hipStream_t st) {
  using C = typename CT<T>::C;
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (2 * sizeof(C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_MODE(KM, DEC, JJ)                                                                                  \
  hipLaunchKernelGGL((k_mode<T, KM, DEC, JJ>), dim3(g), dim3(block), shmem, st, d, tl, static_cast<C*>(x0),        \
                     static_cast<C*>(x1), ctl, partial, arrivals, T(h), T(gamma))
#define DECBPM_MODE_J(KM, DEC) \
  if (J <= 1) DECBPM_MODE(KM, DEC, 1); else DECBPM_MODE(KM, DEC, 2);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_MODE_J(8, true) } else { DECBPM_MODE_J(8, false) }
  } else {
    if (dec) { DECBPM_MODE_J(12, true) } else { DECBPM_MODE_J(12, false) }
  }
#undef DECBPM_MODE_J
#undef DECBPM_MODE
}

template <typename T>
static const void* dp5_persist_kernel(const DevOps<T>& d, const TileOps<T>& tl, int block) {
  const int J = (tl.max_compute + block - 1) / block;
  const bool dec = tl.lmw != nullptr;
#define DECBPM_DP(KM, DEC, JJ)                                                        \
  (tl.llwi != nullptr ? reinterpret_cast<const void*>(&k_dp5_persist<T, KM, DEC, JJ, true>) \
                      : reinterpret_cast<const void*>(&k_dp5_persist<T, KM, DEC, JJ, false>))
#define DECBPM_DP_J(KM, DEC) return J <= 1 ? DECBPM_DP(KM, DEC, 1) : DECBPM_DP(KM, DEC, 2);
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_DP_J(8, true) } else { DECBPM_DP_J(8, false) }
  } else {
    if (dec) { DECBPM_DP_J(12, true) } else { DECBPM_DP_J(12, false) }
  }
#undef DECBPM_DP_J
#undef DECBPM_DP
}

template <typename T>
int dp5_persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block) {
  if (tl.max_compute > 2 * block) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = size_t(tl.max_slots) * 2 * (sizeof(typename CT<T>::C) + sizeof(T));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dp5_persist_kernel<T>(d, tl, block), block, lds) !=
      hipSuccess)
    return 0;
  return cus * per_cu;
}

template <typename T>
hipError_t launch_dp5_persist(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, Dp5Ctl* ctl,
                              double* partial, int32_t* flags, int32_t* status, int32_t spin_limit, double gamma,
                              double rtol, double atol, double inv_n, int block, hipStream_t st) {
  using C = typename CT<T>::C;
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(tl.n_tiles, 256, 0)), dim3(256), 0, st, int64_t(tl.n_tiles), flags);
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  DevOps<T> dd = d;
  TileOps<T> tt = tl;
  C* b0 = static_cast<C*>(x0);
  C* b1 = static_cast<C*>(x1);
  T tg = T(gamma), tr = T(rtol), ta = T(atol);
  void* args[] = {&dd, &tt, &b0, &b1, &ctl, &partial, &flags, &status, &spin_limit, &tg, &tr, &ta, &inv_n};
  const size_t lds = size_t(tl.max_slots) * 2 * (sizeof(C) + sizeof(T));
  return hipLaunchCooperativeKernel(dp5_persist_kernel<T>(d, tl, block), dim3(g), dim3(block), args, unsigned(lds),
                                    st);
}

template <typename T>
static const void* mode_persist_kernel(const DevOps<T>& d, const TileOps<T>& tl, int block) {
  const int J = (tl.max_compute + block - 1) / block;
  const bool dec = tl.lmw != nullptr;
#define DECBPM_MP(KM, DEC, JJ) reinterpret_cast<const void*>(&k_mode_persist<T, KM, DEC, JJ>)
#define DECBPM_MP_J(KM, DEC) return J <= 1 ? DECBPM_MP(KM, DEC, 1) : DECBPM_MP(KM, DEC, 2);
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_MP_J(8, true) } else { DECBPM_MP_J(8, false) }
  } else {
    if (dec) { DECBPM_MP_J(12, true) } else { DECBPM_MP_J(12, false) }
  }
#undef DECBPM_MP_J
#undef DECBPM_MP
}

template <typename T>
int mode_persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block) {
  if (tl.max_compute > 2 * block) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = size_t(tl.max_slots) * (2 * sizeof(typename CT<T>::C) + sizeof(T));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mode_persist_kernel<T>(d, tl, block), block, lds) !=
      hipSuccess)
    return 0;
  return cus * per_cu;
}

template <typename T>
hipError_t launch_mode_persist(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, ModeCtl* ctl,
                               double* partial, int32_t* flags, int32_t* status, int32_t spin_limit, double h,
                               double gamma, int block, hipStream_t st) {
  using C = typename CT<T>::C;
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(tl.n_tiles, 256, 0)), dim3(256), 0, st, int64_t(tl.n_tiles), flags);
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  DevOps<T> dd = d;
  TileOps<T> tt = tl;
  C* b0 = static_cast<C*>(x0);
  C* b1 = static_cast<C*>(x1);
  T th = T(h), tg = T(gamma);
  void* args[] = {&dd, &tt, &b0, &b1, &ctl, &partial, &flags, &status, &spin_limit, &th, &tg};
  const size_t lds = size_t(tl.max_slots) * (2 * sizeof(C) + sizeof(T));
  return hipLaunchCooperativeKernel(mode_persist_kernel<T>(d, tl, block), dim3(g), dim3(block), args, unsigned(lds),
                                    st);
}

template <typename T>
void launch_unsplit(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h,
                    double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * 2 * (sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_RK4UC(KM, DEC, JJ, CLX)                                                                           \
  hipLaunchKernelGGL((k_rk4u<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in_psi), \
                     DECBPM_M(T, out_psi), T(h), T(gamma))
  const bool cl = tl.llwi != nullptr;  // complex L weights (a PML)
#define DECBPM_RK4U(KM, DEC, JJ)           \
  if (cl) DECBPM_RK4UC(KM, DEC, JJ, true); \
  else DECBPM_RK4UC(KM, DEC, JJ, false)
#define DECBPM_RK4U_J(KM, DEC) \
  if (J <= 1) DECBPM_RK4U(KM, DEC, 1); else DECBPM_RK4U(KM, DEC, 2);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_RK4U_J(8, true) } else { DECBPM_RK4U_J(8, false) }
  } else {
    if (dec) { DECBPM_RK4U_J(12, true) } else { DECBPM_RK4U_J(12, false) }
  }
#undef DECBPM_RK4U_J
#undef DECBPM_RK4U
#undef DECBPM_RK4UC
}

template <typename T>
void launch_hstage(const DevOps<T>& d, const TileOps<T>& tl, const void* x, const void* base, void* out, double coef,
                   double p3, double p4, void* s_out, double tau_s, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * 3 * sizeof(typename CT<T>::C);
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_HS(KM, JJ)                                                                                        \
  hipLaunchKernelGGL((k_hstage<T, KM, JJ>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, x),             \
                     DECBPM_C(T, base), DECBPM_M(T, out), T(coef), T(p3), T(p4), static_cast<T*>(s_out), T(tau_s))
  if (kmax_of(d.wmax) == 8) {
    if (J <= 1) DECBPM_HS(8, 1); else DECBPM_HS(8, 2);
  } else {
    if (J <= 1) DECBPM_HS(12, 1); else DECBPM_HS(12, 2);
  }
#undef DECBPM_HS
}

template <typename T>
void launch_step_b4(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h,
                    double tau, double gamma, int block, hipStream_t st, const int32_t* out_perm, int* flag) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (4 * sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_STEP4(KM, DEC, JJ)                                                                              \
  hipLaunchKernelGGL((k_step_b4<T, KM, DEC, JJ>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in_psi),  \
                     DECBPM_M(T, out_psi), T(h), T(tau), T(gamma), out_perm, flag)
#define DECBPM_STEP4_J(KM, DEC) \
  if (J <= 1) DECBPM_STEP4(KM, DEC, 1); else if (J == 2) DECBPM_STEP4(KM, DEC, 2); else DECBPM_STEP4(KM, DEC, 3);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_STEP4_J(8, true) } else { DECBPM_STEP4_J(8, false) }
  } else {
    if (dec) { DECBPM_STEP4_J(12, true) } else { DECBPM_STEP4_J(12, false) }
  }
#undef DECBPM_STEP4_J
#undef DECBPM_STEP4
}

template <typename T>
void launch_kerr_tile(const DevOps<T>& d, const TileOps<T>& tl, const void* src, const int32_t* perm, void* dst,
                      double tau, double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * sizeof(T);
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_KT(KM, DEC, JJ, CLX)                                                                               \
  hipLaunchKernelGGL((k_kerr_tile<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, src), \
                     perm, DECBPM_M(T, dst), T(tau), T(gamma))
  // the operator rows are not used past rings 0..1, so complex L weights need no instance of their own
#define DECBPM_KT_J(KM, DEC) \
  if (J <= 1) DECBPM_KT(KM, DEC, 1, false); else if (J == 2) DECBPM_KT(KM, DEC, 2, false); else DECBPM_KT(KM, DEC, 3, false);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_KT_J(8, true) } else { DECBPM_KT_J(8, false) }
  } else {
    if (dec) { DECBPM_KT_J(12, true) } else { DECBPM_KT_J(12, false) }
  }
#undef DECBPM_KT_J
#undef DECBPM_KT
}

template <typename T>
void launch_step_rec(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, void* y1, void* y2,
                     void* y3, void* b, double h, double tau, double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * (3 * sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_STEPRC(KM, DEC, JJ, CLX)                                                                           \
  hipLaunchKernelGGL((k_step_rec<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl,                  \
                     DECBPM_C(T, in_psi), DECBPM_M(T, out_psi), DECBPM_M(T, y1), DECBPM_M(T, y2), DECBPM_M(T, y3), \
                     DECBPM_M(T, b), T(h), T(tau), T(gamma))
#define DECBPM_STEPR(KM, DEC, JJ)                       \
  if (tl.llwi) DECBPM_STEPRC(KM, DEC, JJ, true); \
  else DECBPM_STEPRC(KM, DEC, JJ, false)
#define DECBPM_STEPR_J(KM, DEC) \
  if (J <= 1) { DECBPM_STEPR(KM, DEC, 1); } else { DECBPM_STEPR(KM, DEC, 2); }
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_STEPR_J(8, true) } else { DECBPM_STEPR_J(8, false) }
  } else {
    if (dec) { DECBPM_STEPR_J(12, true) } else { DECBPM_STEPR_J(12, false) }
  }
#undef DECBPM_STEPR_J
#undef DECBPM_STEPR
#undef DECBPM_STEPRC
}

template <typename T>
void launch_step_adj(const DevOps<T>& d, const TileOps<T>& tl, const void* lam_in, const void* fa, const void* fb,
                     const void* y3, const void* y2, const void* y1, const void* fa0, void* lam_out, double* gdn,
                     double h, double tau, double gamma, const void* sig, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * 3 * sizeof(typename CT<T>::C);
  const int J = (tl.max_compute + block - 1) / block;
#define DECBPM_STEPAC(KM, DEC, JJ, CLX)                                                                          \
  hipLaunchKernelGGL((k_step_adj<T, KM, DEC, JJ, CLX>), dim3(g), dim3(block), shmem, st, d, tl,                 \
                     DECBPM_C(T, lam_in), DECBPM_C(T, fa), DECBPM_C(T, fb), DECBPM_C(T, y3), DECBPM_C(T, y2),   \
                     DECBPM_C(T, y1), DECBPM_C(T, fa0), DECBPM_M(T, lam_out), gdn, T(h), T(tau), T(gamma),     \
                     DECBPM_C(T, sig))
#define DECBPM_STEPA(KM, DEC, JJ)                       \
  if (tl.llwi) DECBPM_STEPAC(KM, DEC, JJ, true); \
  else DECBPM_STEPAC(KM, DEC, JJ, false)
#define DECBPM_STEPA_J(KM, DEC) \
  if (J <= 1) { DECBPM_STEPA(KM, DEC, 1); } else { DECBPM_STEPA(KM, DEC, 2); }
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_STEPA_J(8, true) } else { DECBPM_STEPA_J(8, false) }
  } else {
    if (dec) { DECBPM_STEPA_J(12, true) } else { DECBPM_STEPA_J(12, false) }
  }
#undef DECBPM_STEPA_J
#undef DECBPM_STEPA
#undef DECBPM_STEPAC
}

// Persistent kernel instance for a body; tiles with complex L weights have
// instances in complex64 only (nullptr otherwise).
template <typename T, int KM, bool DEC, int JJ>
static const void* persist_instance(int body, bool cl, bool fx) {
  if constexpr (sizeof(T) == 4) {
    if (fx && body == 0)
      return cl ? reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 0, true, true>)
                : reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 0, false, true>);
  }
  if (cl) {
    if constexpr (sizeof(T) == 4) {
      return body ? reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 1, true>)
                  : reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 0, true>);
    }
    return nullptr;
  }
  return body ? reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 1>)
              : reinterpret_cast<const void*>(&k_persist<T, KM, DEC, JJ, 3, 0>);
}

// Whether the persistent launch of a body takes the fixed LDS layout.
template <typename T>
static bool persist_fixed(const TileOps<T>& tl, int body) {
  return body == 0 && fixed_lds<T>(tl);
}

// Kernel instance of the persistent step for a tile set and block size.
template <typename T>
static const void* persist_kernel(const DevOps<T>& d, const TileOps<T>& tl, int block, int body) {
  const int J = (tl.max_compute + block - 1) / block;
  const bool dec = tl.lmw != nullptr;
  const bool cl = tl.llwi != nullptr;
  const bool fx = persist_fixed<T>(tl, body);
#define DECBPM_PK(KM, DEC, JJ) persist_instance<T, KM, DEC, JJ>(body, cl, fx)
#define DECBPM_PK_J(KM, DEC) return J <= 1 ? DECBPM_PK(KM, DEC, 1) : DECBPM_PK(KM, DEC, 2);
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_PK_J(8, true) } else { DECBPM_PK_J(8, false) }
  } else {
    if (dec) { DECBPM_PK_J(12, true) } else { DECBPM_PK_J(12, false) }
  }
#undef DECBPM_PK_J
#undef DECBPM_PK
}

template <typename T>
size_t persist_lds(const TileOps<T>& tl, int body) {
  // the fixed layout is static LDS of the kernel (four buffers of kFixSlots
  // complex-sized slots, S at the complex stride): no dynamic LDS
  if (persist_fixed<T>(tl, body)) return 0;
  return size_t(tl.max_slots) * (3 * sizeof(typename CT<T>::C) + sizeof(T));
}

template <typename T>
int persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block, int body) {
  if (tl.max_slots > 3 * block || tl.max_compute > 2 * block) return 0;
  const void* k = persist_kernel<T>(d, tl, block, body);
  if (!k) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, persist_lds<T>(tl, body)) != hipSuccess)
    return 0;
  return cus * per_cu;
}

template <typename T>
hipError_t launch_persist(const DevOps<T>& d, const TileOps<T>& tl, const int32_t* nb_ptr, const int32_t* nb_list,
                          void* buf0, void* buf1, int32_t* flags, int32_t* status, int32_t n_steps,
                          int32_t spin_limit, double h, double gamma, int block, hipStream_t st, int body,
                          const PersistIO& io, bool coop) {
  using C = typename CT<T>::C;
  const void* k = persist_kernel<T>(d, tl, block, body);
  if (!k) return hipErrorInvalidDeviceFunction;
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  DevOps<T> dd = d;
  TileOps<T> tt = tl;
  C* b0 = static_cast<C*>(buf0);
  C* b1 = static_cast<C*>(buf1);
  T th = T(h), tg = T(gamma);
  PersistArgs<T> pa{static_cast<const C*>(io.in), static_cast<C*>(io.out), io.perm, io.base, T(io.tau_first),
                    T(io.tau_last)};
  void* args[] = {&dd, &tt, const_cast<int32_t**>(&nb_ptr), const_cast<int32_t**>(&nb_list), &b0, &b1, &flags, &status,
                  &n_steps, &spin_limit, &th, &tg, &pa};
  if (coop) return hipLaunchCooperativeKernel(k, dim3(g), dim3(block), args, unsigned(persist_lds<T>(tl, body)), st);
  return hipLaunchKernel(k, dim3(g), dim3(block), args, size_t(persist_lds<T>(tl, body)), st);
}

template <typename T>
void launch_perm_in(const DevOps<T>& d, const int32_t* perm, const void* src, void* dst, int scale_inv_h0, int block,
                    hipStream_t st) {
  const unsigned g = grid_for(d.n_rows * d.F, block, 0);
  DECBPM_DISPATCH_FB(d, hipLaunchKernelGGL((k_perm_in<T, FB>), dim3(g), dim3(block), 0, st, d, perm,
                                           DECBPM_C(T, src), DECBPM_M(T, dst), scale_inv_h0))
}

template <typename T>
void launch_perm_out(const DevOps<T>& d, const int32_t* perm, const void* src, void* dst, int scale_h0, int* flag,
                     int block, hipStream_t st) {
  const unsigned g = grid_for(d.n_rows * d.F, block, 0);
  DECBPM_DISPATCH_FB(d, hipLaunchKernelGGL((k_perm_out<T, FB>), dim3(g), dim3(block), 0, st, d, perm,
                                           DECBPM_C(T, src), DECBPM_M(T, dst), scale_h0, flag))
}

template <typename T>
void launch_bperm(const DevOps<T>& d, const int64_t* cbase, const int32_t* fcount, const void* src, void* dst,
                  bool out, int* flag, int block, hipStream_t st, bool field_major) {
  const unsigned g = grid_for(d.n_rows * d.F, block, 0);
  if (out)
    hipLaunchKernelGGL((k_bperm_out<T>), dim3(g), dim3(block), 0, st, d.n_rows, d.F, cbase, fcount,
                       DECBPM_C(T, src), DECBPM_M(T, dst), flag, int(field_major));
  else
    hipLaunchKernelGGL((k_bperm_in<T>), dim3(g), dim3(block), 0, st, d.n_rows, d.F, cbase, fcount,
                       DECBPM_C(T, src), DECBPM_M(T, dst), int(field_major));
}

// Workgroups of `kernel` resident on the whole device at once (compute units
// times the blocks one unit holds), at least one.
template <typename K>
int resident_workgroups(K kernel, int block, size_t shmem) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    ncu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, shmem) != hipSuccess) per = 1;
  return (ncu > 0 ? ncu : 1) * (per > 0 ? per : 1);
}

template <typename T>
void launch_step_fields(const DevOps<T>& d, const TileOps<T>& tl, const void* in, void* out, double h, double tau,
                        double gamma, int block, hipStream_t st) {
  const size_t shmem0 = size_t(tl.max_slots) * (3 * sizeof(typename CT<T>::C) + sizeof(T));
  const int J = (tl.max_compute + block - 1) / block;
  const int LS = (tl.max_slots + block - 1) / block;
  const int32_t nf = d.F;
  const int64_t units = int64_t(tl.n_tiles) * nf;
  int dev = 0, lds_cap = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lds_cap = 0;
  // the M weights go to LDS (TS x (KMAX | 1) after S) where they fit
  auto lm_bytes = [&](int km) { return size_t(km | 1) * size_t(tl.TS) * sizeof(T); };
  // the operator rows take J slots per thread; the state LS (at most three slots of every ring).
  // One wave of workgroups, each given the same number of (tile, field) steps.
#define DECBPM_SF(KM, DEC, JJ, LL)                                                                                \
  do {                                                                                                            \
    const bool lm = DEC && shmem0 + lm_bytes(KM) <= size_t(lds_cap);                                              \
    auto* kern = lm ? &k_step_fields<T, KM, DEC, JJ, LL, true> : &k_step_fields<T, KM, DEC, JJ, LL, false>;       \
    const size_t shmem = shmem0 + (lm ? lm_bytes(KM) : 0);                                                        \
    const int64_t res = resident_workgroups(kern, block, shmem);                                                  \
    const int32_t n_wg = int32_t(units < res ? units : res);                                                      \
    const unsigned g = grid_for(int64_t(n_wg) * block, block, d.xcd_remap);                                       \
    hipLaunchKernelGGL(kern, dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in), DECBPM_M(T, out), T(h),     \
                       T(tau), T(gamma), nf, n_wg);                                                               \
  } while (0)
#define DECBPM_SF_J(KM, DEC)                                                           \
  if (J <= 1) {                                                                        \
    if (LS <= 2) DECBPM_SF(KM, DEC, 1, 2); else DECBPM_SF(KM, DEC, 1, 3);                \
  } else {                                                                             \
    if (LS <= 2) DECBPM_SF(KM, DEC, 2, 2); else DECBPM_SF(KM, DEC, 2, 3);                \
  }
  // rows of up to 10 entries (most meshes of degree 9 or 10) get their own
  // unroll: two fewer registers per slot and table than the 12-wide form
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_SF_J(8, true) } else { DECBPM_SF_J(8, false) }
  } else if (d.wmax <= 10) {
    if (dec) { DECBPM_SF_J(10, true) } else { DECBPM_SF_J(10, false) }
  } else {
    if (dec) { DECBPM_SF_J(12, true) } else { DECBPM_SF_J(12, false) }
  }
#undef DECBPM_SF_J
#undef DECBPM_SF
}

template <typename T>
void launch_kerr_fields(const DevOps<T>& d, const TileOps<T>& tl, const void* in, void* out, double tau,
                        double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(int64_t(tl.n_tiles) * block, block, d.xcd_remap);
  const size_t shmem = size_t(tl.max_slots) * sizeof(T);
  const int J = (tl.max_compute + block - 1) / block;
  const int32_t nf = d.F;
#define DECBPM_KF(KM, DEC, JJ)                                                                                   \
  hipLaunchKernelGGL((k_kerr_fields<T, KM, DEC, JJ>), dim3(g), dim3(block), shmem, st, d, tl, DECBPM_C(T, in),  \
                     DECBPM_M(T, out), T(tau), T(gamma), nf)
#define DECBPM_KF_J(KM, DEC) \
  if (J <= 1) DECBPM_KF(KM, DEC, 1); else DECBPM_KF(KM, DEC, 2);
  const bool dec = tl.lmw != nullptr;
  if (kmax_of(d.wmax) == 8) {
    if (dec) { DECBPM_KF_J(8, true) } else { DECBPM_KF_J(8, false) }
  } else {
    if (dec) { DECBPM_KF_J(12, true) } else { DECBPM_KF_J(12, false) }
  }
#undef DECBPM_KF_J
#undef DECBPM_KF
}

template <typename T>
void launch_fill(const DevOps<T>& d, void* x, double re, double im, int block, hipStream_t st) {
  const int64_t n = d.n_rows * d.F;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, block, 0)), dim3(block), 0, st, n, DECBPM_M(T, x), T(re), T(im));
}

template <typename T>
void launch_copy(int64_t n, const void* src, void* dst, int block, hipStream_t st) {
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n, block, 0)), dim3(block), 0, st, n, DECBPM_C(T, src),
                     DECBPM_M(T, dst));
}

template <typename T>
void launch_diag(const DevOps<T>& d, const void* psi, double gamma, double* partials, int n_blocks, double* out,
                 hipStream_t st) {
  if (d.mw)
    hipLaunchKernelGGL((k_diag<T, true>), dim3(n_blocks), dim3(RED_BLOCK), 0, st, d, DECBPM_C(T, psi), T(gamma),
                       partials);
  else
    hipLaunchKernelGGL((k_diag<T, false>), dim3(n_blocks), dim3(RED_BLOCK), 0, st, d, DECBPM_C(T, psi), T(gamma),
                       partials);
  hipLaunchKernelGGL(k_finish2, dim3(1), dim3(RED_BLOCK), 0, st, partials, n_blocks, out);
}

template <typename T>
void launch_overlap(int64_t n, const double* h0c, const void* a, const void* b, double* partials, int n_blocks,
                    double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_overlap<T>), dim3(n_blocks), dim3(RED_BLOCK), 0, st, n, h0c, DECBPM_C(T, a), DECBPM_C(T, b),
                     partials);
  hipLaunchKernelGGL(k_finish2, dim3(1), dim3(RED_BLOCK), 0, st, partials, n_blocks, out);
}

template <typename T>
void launch_adj_stage(const DevOps<T>& d, const void* u_in, const void* t, void* u_out, void* acc, int init,
                      const void* yf, double coef, double cdn, double* gdn, int block, hipStream_t st) {
  const unsigned g = grid_for(d.n_rows, block, d.xcd_remap);
  if (t) {
    DECBPM_DISPATCH_K(d, hipLaunchKernelGGL((k_adj_stage<T, KM, true>), dim3(g), dim3(block), 0, st, d,
                                            DECBPM_C(T, u_in), DECBPM_C(T, t), DECBPM_M(T, u_out), DECBPM_M(T, acc),
                                            init, DECBPM_C(T, yf), T(coef), cdn, gdn))
  } else {
    DECBPM_DISPATCH_K(d, hipLaunchKernelGGL((k_adj_stage<T, KM, false>), dim3(g), dim3(block), 0, st, d,
                                            DECBPM_C(T, u_in), DECBPM_C(T, t), DECBPM_M(T, u_out), DECBPM_M(T, acc),
                                            init, DECBPM_C(T, yf), T(coef), cdn, gdn))
  }
}

template <typename T>
void launch_adj_prep(const DevOps<T>& d, const void* psi_in, const void* psi_out, const void* lam_out, void* sm,
                     double tau, double gamma, int block, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_prep<T>), dim3(grid_for(d.n_rows, block, 0)), dim3(block), 0, st, d,
                     DECBPM_C(T, psi_in), DECBPM_C(T, psi_out), DECBPM_C(T, lam_out), DECBPM_M(T, sm), T(tau),
                     T(gamma));
}

template <typename T>
void launch_adj_kerr(const DevOps<T>& d, const void* psi_in, const void* lam_out, const void* sm, void* lam_in,
                     double tau, double gamma, int block, hipStream_t st) {
  const unsigned g = grid_for(d.n_rows, block, d.xcd_remap);
  if (d.mw) {
    DECBPM_DISPATCH_K(d, hipLaunchKernelGGL((k_adj_kerr<T, KM, true>), dim3(g), dim3(block), 0, st, d,
                                            DECBPM_C(T, psi_in), DECBPM_C(T, lam_out), DECBPM_C(T, sm),
                                            DECBPM_M(T, lam_in), T(tau), T(gamma)))
  } else {
    hipLaunchKernelGGL((k_adj_kerr<T, 0, false>), dim3(g), dim3(block), 0, st, d, DECBPM_C(T, psi_in),
                       DECBPM_C(T, lam_out), DECBPM_C(T, sm), DECBPM_M(T, lam_in), T(tau), T(gamma));
  }
}

template <typename T>
void launch_hcombine(const DevOps<T>& d, const void* x, const void* t, const void* t2, void* y, int block,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_hcombine<T>), dim3(grid_for(d.n_rows * d.F, block, 0)), dim3(block), 0, st, d,
                     DECBPM_C(T, x), DECBPM_C(T, t), DECBPM_C(T, t2), DECBPM_M(T, y));
}

template <typename T>
void launch_set_v(int64_t n, const T* v0, const double* dn, const int32_t* perm, T* v, int block, hipStream_t st) {
  hipLaunchKernelGGL((k_set_v<T>), dim3(grid_for(n, block, 0)), dim3(block), 0, st, n, v0, dn, perm, v);
}

#if DECBPM_PART & 1
void launch_gdn_out(int64_t n, const int32_t* perm, const double* gdn, double* out, int block, hipStream_t st) {
  hipLaunchKernelGGL(k_gdn_out, dim3(grid_for(n, block, 0)), dim3(block), 0, st, n, perm, gdn, out);
}
#endif

#if DECBPM_PART & 1
void launch_zero_i32(int64_t n, int32_t* x, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(n, 256, 0)), dim3(256), 0, st, n, x);
}

void launch_zero_f64(int64_t n, double* x, int block, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(n, block, 0)), dim3(block), 0, st, n, x);
}
#endif

#define DECBPM_INSTANTIATE(T)                                                                                     \
  template void launch_stage<T>(const DevOps<T>&, const void*, const void*, const void*, void*, double, void*,     \
                                double, int, hipStream_t);                                                       \
  template void launch_lap<T>(const DevOps<T>&, const void*, void*, int, hipStream_t);                             \
  template void launch_prep_s<T>(const DevOps<T>&, const void*, void*, double, int, hipStream_t);                  \
  template void launch_kerr<T>(const DevOps<T>&, const void*, void*, const void*, double, double, int, hipStream_t); \
  template void launch_perm_in<T>(const DevOps<T>&, const int32_t*, const void*, void*, int, int, hipStream_t);    \
  template void launch_perm_out<T>(const DevOps<T>&, const int32_t*, const void*, void*, int, int*, int,            \
                                   hipStream_t);                                                                 \
  template void launch_fill<T>(const DevOps<T>&, void*, double, double, int, hipStream_t);                         \
  template void launch_copy<T>(int64_t, const void*, void*, int, hipStream_t);                                    \
  template void launch_diag<T>(const DevOps<T>&, const void*, double, double*, int, double*, hipStream_t);         \
  template void launch_overlap<T>(int64_t, const double*, const void*, const void*, double*, int, double*,        \
                                  hipStream_t);                                                                  \
  template void launch_adj_stage<T>(const DevOps<T>&, const void*, const void*, void*, void*, int, const void*,   \
                                    double, double, double*, int, hipStream_t);                                  \
  template void launch_adj_prep<T>(const DevOps<T>&, const void*, const void*, const void*, void*, double, double, \
                                   int, hipStream_t);                                                            \
  template void launch_adj_kerr<T>(const DevOps<T>&, const void*, const void*, const void*, void*, double, double, \
                                   int, hipStream_t);                                                            \
  template void launch_hcombine<T>(const DevOps<T>&, const void*, const void*, const void*, void*, int,           \
                                   hipStream_t);                                                                 \
  template void launch_set_v<T>(int64_t, const T*, const double*, const int32_t*, T*, int, hipStream_t);          \
  template void launch_step<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, double, double, double,   \
                               int, hipStream_t, const int32_t*, int*);                                          \
  template void launch_kerr_tile<T>(const DevOps<T>&, const TileOps<T>&, const void*, const int32_t*, void*,      \
                                    double, double, int, hipStream_t);                                           \
  template void launch_bperm<T>(const DevOps<T>&, const int64_t*, const int32_t*, const void*, void*, bool, int*,  \
                                int, hipStream_t, bool);                                                         \
  template void launch_step_fields<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, double, double,     \
                                      double, int, hipStream_t);                                                 \
  template void launch_kerr_fields<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, double, double, int, \
                                      hipStream_t);                                                              \
  template int persist_capacity<T>(const DevOps<T>&, const TileOps<T>&, int, int);                                \
  template void launch_step_b4<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, double, double, double, \
                                  int, hipStream_t, const int32_t*, int*);                                       \
  template void launch_unsplit<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, double, double, int,    \
                                  hipStream_t);                                                                  \
  template void launch_hstage<T>(const DevOps<T>&, const TileOps<T>&, const void*, const void*, void*, double,    \
                                 double, double, void*, double, int, hipStream_t);                               \
  template void launch_lapc<T>(const DevOps<T>&, const void*, const void*, double, double, void*, int,         \
                               hipStream_t);                                                                     \
  template void launch_dp5<T>(const DevOps<T>&, const TileOps<T>&, void*, void*, Dp5Ctl*, double*, uint32_t*,     \
                              double, double, double, double, int, hipStream_t);                                 \
  template void launch_mode<T>(const DevOps<T>&, const TileOps<T>&, void*, void*, ModeCtl*, double*, uint32_t*,   \
                               double, double, int, hipStream_t);                                                \
  template void launch_scale<T>(int64_t, void*, double, int, hipStream_t);                                        \
  template int mode_persist_capacity<T>(const DevOps<T>&, const TileOps<T>&, int);                                \
  template int dp5_persist_capacity<T>(const DevOps<T>&, const TileOps<T>&, int);                                 \
  template hipError_t launch_dp5_persist<T>(const DevOps<T>&, const TileOps<T>&, void*, void*, Dp5Ctl*, double*,  \
                                            int32_t*, int32_t*, int32_t, double, double, double, double, int,      \
                                            hipStream_t);                                                         \
  template hipError_t launch_mode_persist<T>(const DevOps<T>&, const TileOps<T>&, void*, void*, ModeCtl*, double*, \
                                             int32_t*, int32_t*, int32_t, double, double, int, hipStream_t);      \
  template void launch_step_rec<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, void*, void*, void*,    \
                                   void*, double, double, double, int, hipStream_t);                             \
  template void launch_step_adj<T>(const DevOps<T>&, const TileOps<T>&, const void*, const void*, const void*,     \
                                   const void*, const void*, const void*, const void*, void*, double*, double,   \
                                   double, double, const void*, int, hipStream_t);                               \
  template hipError_t launch_persist<T>(const DevOps<T>&, const TileOps<T>&, const int32_t*, const int32_t*, void*, \
                                        void*, int32_t*, int32_t*, int32_t, int32_t, double, double, int,        \
                                        hipStream_t, int, const PersistIO&, bool);                                     \
  template void launch_bstage<T>(const DevOps<T>&, const TileOps<T>&, const void*, const void*, const void*, void*, \
                                 double, void*, double, hipStream_t);                                            \
  template void launch_blap<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, hipStream_t);           \
  template void launch_bkerr<T>(const DevOps<T>&, const TileOps<T>&, const void*, void*, const void*, double,     \
                                double, hipStream_t);                                                            \
  template void launch_fused<T>(const DevOps<T>&, const TileOps<T>&, int, const void*, const void*, void*, void*,  \
                                void*, double, double, double, int, hipStream_t);                                \
  template void launch_fused_adj<T>(const DevOps<T>&, const TileOps<T>&, int, const void*, const void*,          \
                                    const void*, const void*, const void*, const void*, void*, void*, double*,   \
                                    double, double, double, int, hipStream_t);

#if DECBPM_PART & 1
DECBPM_INSTANTIATE(float)
#endif
#if DECBPM_PART & 2
DECBPM_INSTANTIATE(double)
#endif

}  // namespace decbpm
