// Least-squares reconstruction with the matched SRT pair: conjugate gradients
// on the normal equations A^T A f = A^T g (the CGLS arrangement), applying
// only the forward (Alg. 1) and the adjoint (Alg. 2) of a plan. An exactly
// matched adjoint is what makes these iterations consistent (Sec. 3.2).
//
// Per batch item b, an independent problem:
//   r = g - A f,  s = A^T r,  p = s,  gamma = ||s||^2
//   repeat:  q = A p,  alpha = gamma / ||q||^2
//            f += alpha p,  r -= alpha q
//            s = A^T r,  gamma' = ||s||^2,  p = s + (gamma'/gamma) p
// All vector work and the scalars stay on the device: inner products are
// reduced in FP64 in a fixed order (so runs are bitwise repeatable), and the
// step lengths are read by the update kernels from device memory, so an
// iteration never waits for the host.
//
// Nonnegative least squares, min 0.5 ||A f - g||^2 subject to f >= 0, by
// accelerated projected gradient (FISTA; Beck and Teboulle 2009, Sec. 4, the
// projection onto f >= 0 as the proximal step), with a fixed step 1/L,
// L >= ||A||^2:
//   y_1 = f_0, t_1 = 1
//   f_k = max(0, y_k - (1/L) A^T (A y_k - g))
//   y_{k+1} = f_k + ((t_k - 1)/t_{k+1}) (f_k - f_{k-1}),
//   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
// The weights do not depend on the data and are computed on the host; one
// fused kernel does the projection and the extrapolation. ||A||^2, the
// largest eigenvalue of A^T A, is estimated by power iteration from the
// all-ones volume (A has no negative entries, so the dominant eigenvector of
// A^T A can be taken nonnegative and the start overlaps it).
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "srt_internal.h"

namespace srt {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;  // partial sums per batch item

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// 16-byte vectors of T (4 floats or 2 doubles), used when every batch item's
// vector starts 16-byte aligned (its length is a multiple of the width).
template <typename T> struct V;
template <> struct V<float> { using t = float4; static constexpr int n = 4; };
template <> struct V<double> { using t = double2; static constexpr int n = 2; };

// Where element j (0 <= j < n) of batch item b of B sits: the items'
// vectors are cut into runs of `run` elements and the runs of all items
// interleaved, run k of item b at (k * B + b) * run. With run == n the items
// lie one after another (b * n + j); data vectors in stage 2's layout
// [h][l][b][a] have run == n_angles. A grid-stride walk over j steps the run
// index and the offset within the run instead of dividing per element.
struct ItemWalk {
  int64_t run, B, b, k, o, dk, dO;
  __device__ ItemWalk(int64_t j0, int64_t stride, int64_t run_, int B_, int b_)
      : run(run_), B(B_), b(b_), k(j0 / run_), o(j0 % run_), dk(stride / run_), dO(stride % run_) {}
  __device__ int64_t pos() const { return (k * B + b) * run + o; }
  __device__ void next() {
    k += dk;
    o += dO;
    if (o >= run) {
      o -= run;
      ++k;
    }
  }
};

// part[b * kRedBlocks + blk] = sum over this block's share of item b of x*y,
// in FP64: each thread sums a fixed stride of the item's elements (in the
// item's own order j, whatever the layout), then a fixed tree. In the vector
// form n and run count 16-byte vectors.
template <typename T, bool VEC>
__global__ __launch_bounds__(kRedThreads) void k_dot_partial(const T *__restrict__ x,
                                                             const T *__restrict__ y, int64_t n,
                                                             int64_t run,
                                                             double *__restrict__ part) {
  __shared__ double red[kRedThreads];
  const int b = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
  const int64_t stride = (int64_t)kRedBlocks * kRedThreads;
  const int64_t j0 = (int64_t)blk * kRedThreads + t;
  double acc = 0.0;
  if constexpr (VEC) {
    using VT = typename V<T>::t;
    constexpr int W = V<T>::n;
    const VT *xv = reinterpret_cast<const VT *>(x), *yv = reinterpret_cast<const VT *>(y);
    auto term = [&](int64_t q) {
      const VT a = xv[q], c = yv[q];
      const T *as = reinterpret_cast<const T *>(&a), *cs = reinterpret_cast<const T *>(&c);
#pragma unroll
      for (int k = 0; k < W; ++k) acc += (double)as[k] * (double)cs[k];
    };
    if (run == n) {  // items one after another: plain offsets
      for (int64_t i = j0; i < n / W; i += stride) term((int64_t)b * (n / W) + i);
    } else {
      ItemWalk it(j0, stride, run / W, gridDim.y, b);
      for (int64_t i = j0; i < n / W; i += stride, it.next()) term(it.pos());
    }
  } else {
    if (run == n) {
      for (int64_t i = j0; i < n; i += stride) acc += (double)x[b * n + i] * (double)y[b * n + i];
    } else {
      ItemWalk it(j0, stride, run, gridDim.y, b);
      for (int64_t i = j0; i < n; i += stride, it.next()) {
        const int64_t q = it.pos();
        acc += (double)x[q] * (double)y[q];
      }
    }
  }
  red[t] = acc;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) part[(size_t)b * kRedBlocks + blk] = red[0];
}

// out[b] = sum of item b's partials in block order; optionally hist[b] = sqrt.
__global__ void k_dot_final(const double *__restrict__ part, int batch, double *__restrict__ out,
                            double *__restrict__ hist) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double s = 0.0;
  for (int i = 0; i < kRedBlocks; ++i) s += part[(size_t)b * kRedBlocks + i];
  out[b] = s;
  if (hist) hist[b] = sqrt(s);
}

__device__ __forceinline__ double ratio(double num, double den) { return den > 0.0 ? num / den : 0.0; }

// y = a * x + y  (XPAY false)  or  y = x + a * y  (XPAY true), per batch item
// b with a = sign * num[b] / den[b] (a zero denominator gives a = 0); items
// laid out in runs as for k_dot_partial.
template <typename T, bool VEC, bool XPAY>
__global__ void k_update(T *__restrict__ y, const T *__restrict__ x, const double *__restrict__ num,
                         const double *__restrict__ den, double sign, int64_t n, int64_t run) {
  const int b = blockIdx.y;
  const T a = (T)(sign * ratio(num[b], den[b]));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto op = [&](T xv, T yv) { return XPAY ? fma(a, yv, xv) : fma(a, xv, yv); };
  if constexpr (VEC) {
    using VT = typename V<T>::t;
    constexpr int W = V<T>::n;
    VT *yv = reinterpret_cast<VT *>(y);
    const VT *xv = reinterpret_cast<const VT *>(x);
    auto one = [&](int64_t q) {
      VT u = yv[q];
      const VT w = xv[q];
      T *us = reinterpret_cast<T *>(&u);
      const T *ws = reinterpret_cast<const T *>(&w);
#pragma unroll
      for (int k = 0; k < W; ++k) us[k] = op(ws[k], us[k]);
      yv[q] = u;
    };
    if (run == n) {  // items one after another: plain offsets
      for (int64_t i = j0; i < n / W; i += stride) one((int64_t)b * (n / W) + i);
    } else {
      ItemWalk it(j0, stride, run / W, gridDim.y, b);
      for (int64_t i = j0; i < n / W; i += stride, it.next()) one(it.pos());
    }
  } else {
    if (run == n) {
      for (int64_t i = j0; i < n; i += stride) y[b * n + i] = op(x[b * n + i], y[b * n + i]);
    } else {
      ItemWalk it(j0, stride, run, gridDim.y, b);
      for (int64_t i = j0; i < n; i += stride, it.next()) {
        const int64_t q = it.pos();
        y[q] = op(x[q], y[q]);
      }
    }
  }
}

// r = g - r   (r holds A f on entry)
template <typename T>
__global__ void k_rsub(T *__restrict__ r, const T *__restrict__ g, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = g[i] - r[i];
}

struct Layout {
  size_t r, q, s, p, ws, scal, part, hist, total;  // byte offsets
  size_t ws_bytes;
};

Layout layout(const srt_plan *p, int32_t batch, int32_t n_iter) {
  const Geometry &g = p->geo;
  const size_t es = dtype_size(p->vdtype);
  const size_t vol = (size_t)batch * g.mz * g.ms * g.ms * es;
  const size_t dat = (size_t)batch * g.na * g.nh * g.nl * es;
  Layout L{};
  size_t o = 0;
  L.r = o; o += align_up(dat);
  L.q = o; o += align_up(dat);
  L.s = o; o += align_up(vol);
  L.p = o; o += align_up(vol);
  L.ws_bytes = workspace_bytes(p, batch);
  L.ws = o; o += align_up(L.ws_bytes);
  L.scal = o; o += align_up(sizeof(double) * 3 * batch);  // gamma, gamma', delta
  L.part = o; o += align_up(sizeof(double) * kRedBlocks * batch);
  L.hist = o; o += align_up(sizeof(double) * (size_t)(n_iter + 1) * batch);
  L.total = o;
  return L;
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <typename T>
Status run(srt_plan *plan, T *f, const T *g, int32_t B, int32_t n_iter, double *resid, char *w,
           const Layout &L, hipStream_t st) {
  const Geometry &geo = plan->geo;
  const int64_t nv = (int64_t)geo.mz * geo.ms * geo.ms, nd = (int64_t)geo.na * geo.nh * geo.nl;
  T *r = (T *)(w + L.r), *q = (T *)(w + L.q), *s = (T *)(w + L.s), *p = (T *)(w + L.p);
  void *ws = w + L.ws;
  double *gam = (double *)(w + L.scal), *gam2 = gam + B, *del = gam + 2 * B;
  double *part = (double *)(w + L.part), *hist = (double *)(w + L.hist);
  constexpr int W = V<T>::n;
  // Data-space vectors (r, q) stay in stage 2's layout [h][l][b][a]: items in
  // runs of n_angles (one run when B == 1). Volume vectors are item by item.
  const int64_t drun = B > 1 ? geo.na : nd;
  // vector kernels when every run is a whole number of 16-byte vectors and
  // the caller's arrays are 16-byte aligned (workspace arrays are)
  const bool fv = nv % W == 0 && (uintptr_t)f % 16 == 0;
  auto dot = [&](const T *x, const T *y, int64_t n, int64_t run, bool vec, double *out,
                 double *h) -> Status {
    if (vec)
      hipLaunchKernelGGL((k_dot_partial<T, true>), dim3(kRedBlocks, B), dim3(kRedThreads), 0, st, x, y, n, run, part);
    else
      hipLaunchKernelGGL((k_dot_partial<T, false>), dim3(kRedBlocks, B), dim3(kRedThreads), 0, st, x, y, n, run, part);
    hipLaunchKernelGGL(k_dot_final, dim3((B + 63) / 64), dim3(64), 0, st, part, B, out, h);
    SRT_HIP(hipGetLastError());
    return Status{};
  };
  auto update = [&](T *y, const T *x, int64_t n, int64_t run, bool vec, bool xpay,
                    const double *num, const double *den, double sign) -> Status {
    const dim3 grid(grid_for(vec ? n / W : n), B);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, y, x, num, den, sign, n, run);
    };
    if (xpay) {
      if (vec) go(k_update<T, true, true>); else go(k_update<T, false, true>);
    } else {
      if (vec) go(k_update<T, true, false>); else go(k_update<T, false, false>);
    }
    SRT_HIP(hipGetLastError());
    return Status{};
  };
  auto fwd = [&](const T *in, T *out) {
    return apply_plan(plan, in, out, B, ws, L.ws_bytes, st, false, true);
  };
  auto adj = [&](const T *in, T *out) {
    return apply_plan(plan, in, out, B, ws, L.ws_bytes, st, true, true);
  };
  const bool vv = nv % W == 0, dv = nd % W == 0 && drun % W == 0;  // workspace vectors

  SRT_TRY(fwd(f, r));
  SRT_TRY(data_to_stage2(plan, g, q, B, st));  // q is free until the first iteration
  hipLaunchKernelGGL(k_rsub<T>, dim3(grid_for(nd * B)), dim3(256), 0, st, r, q, nd * B);
  SRT_HIP(hipGetLastError());
  SRT_TRY(adj(r, s));
  SRT_HIP(hipMemcpyAsync(p, s, sizeof(T) * nv * B, hipMemcpyDeviceToDevice, st));
  SRT_TRY(dot(s, s, nv, nv, vv, gam, hist));
  for (int k = 1; k <= n_iter; ++k) {
    SRT_TRY(fwd(p, q));
    SRT_TRY(dot(q, q, nd, drun, dv, del, nullptr));
    SRT_TRY(update(f, p, nv, nv, fv, false, gam, del, 1.0));     // f += alpha p
    SRT_TRY(update(r, q, nd, drun, dv, false, gam, del, -1.0));  // r -= alpha q
    SRT_TRY(adj(r, s));
    SRT_TRY(dot(s, s, nv, nv, vv, gam2, hist + (size_t)k * B));
    SRT_TRY(update(p, s, nv, nv, vv, true, gam2, gam, 1.0));     // p = s + beta p
    std::swap(gam, gam2);
  }
  if (resid) {
    SRT_HIP(hipMemcpyAsync(resid, hist, sizeof(double) * (size_t)(n_iter + 1) * B,
                           hipMemcpyDeviceToHost, st));
    SRT_HIP(hipStreamSynchronize(st));
  }
  return Status{};
}

// One FISTA step after the gradient s = A^T (g - A y) (note the sign: the
// residual kernel forms g - A y), flat over the whole batch:
//   x = y + step * s;  f_new = max(0, x) (NaN stays NaN);
//   y = f_new + beta * (f_new - f);  f = f_new
template <typename T, bool VEC>
__global__ void k_fista(T *__restrict__ f, T *__restrict__ y, const T *__restrict__ s, T step,
                        T beta, int64_t n) {
  auto one = [&](T &fv, T &yv, T sv) {
    const T x = yv + step * sv;
    const T fn = x < (T)0 ? (T)0 : x;
    yv = fn + beta * (fn - fv);
    fv = fn;
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if constexpr (VEC) {
    using VT = typename V<T>::t;
    constexpr int W = V<T>::n;
    VT *fv = reinterpret_cast<VT *>(f), *yv = reinterpret_cast<VT *>(y);
    const VT *sv = reinterpret_cast<const VT *>(s);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n / W; i += stride) {
      VT a = fv[i], c = yv[i];
      const VT d = sv[i];
      T *as = reinterpret_cast<T *>(&a), *cs = reinterpret_cast<T *>(&c);
      const T *ds = reinterpret_cast<const T *>(&d);
#pragma unroll
      for (int k = 0; k < W; ++k) one(as[k], cs[k], ds[k]);
      fv[i] = a;
      yv[i] = c;
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      one(f[i], y[i], s[i]);
  }
}

template <typename T>
__global__ void k_fill(T *__restrict__ v, T val, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = val;
}

// v = w / sqrt(nw[0]) (zero when nw[0] is zero)
template <typename T>
__global__ void k_normalize(T *__restrict__ v, const T *__restrict__ w,
                            const double *__restrict__ nw, int64_t n) {
  const double d = nw[0];
  const T inv = d > 0.0 ? (T)(1.0 / sqrt(d)) : (T)0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = w[i] * inv;
}

struct NnlsLayout {
  size_t r, g2, s, y, ws, scal, part, hist, total;  // byte offsets
  size_t ws_bytes;
};

NnlsLayout nnls_layout(const srt_plan *p, int32_t batch, int32_t n_iter) {
  const Geometry &g = p->geo;
  const size_t es = dtype_size(p->vdtype);
  const size_t vol = (size_t)batch * g.mz * g.ms * g.ms * es;
  const size_t dat = (size_t)batch * g.na * g.nh * g.nl * es;
  NnlsLayout L{};
  size_t o = 0;
  L.r = o; o += align_up(dat);
  L.g2 = o; o += align_up(dat);  // the data in stage 2's layout
  L.s = o; o += align_up(vol);
  L.y = o; o += align_up(vol);
  L.ws_bytes = workspace_bytes(p, batch);
  L.ws = o; o += align_up(L.ws_bytes);
  L.scal = o; o += align_up(sizeof(double) * 3 * batch);
  L.part = o; o += align_up(sizeof(double) * kRedBlocks * batch);
  L.hist = o; o += align_up(sizeof(double) * (size_t)(n_iter > 0 ? n_iter : 1) * batch);
  L.total = o;
  return L;
}

template <typename T>
Status dot_into(const T *x, const T *y, int64_t n, int64_t run, int32_t B, bool vec, double *part,
                double *out, double *h, hipStream_t st) {
  if (vec)
    hipLaunchKernelGGL((k_dot_partial<T, true>), dim3(kRedBlocks, B), dim3(kRedThreads), 0, st, x, y, n, run, part);
  else
    hipLaunchKernelGGL((k_dot_partial<T, false>), dim3(kRedBlocks, B), dim3(kRedThreads), 0, st, x, y, n, run, part);
  hipLaunchKernelGGL(k_dot_final, dim3((B + 63) / 64), dim3(64), 0, st, part, B, out, h);
  SRT_HIP(hipGetLastError());
  return Status{};
}

template <typename T>
Status run_nnls(srt_plan *plan, T *f, const T *g, int32_t B, int32_t n_iter, double step,
                double *resid, char *w, const NnlsLayout &L, hipStream_t st) {
  const Geometry &geo = plan->geo;
  const int64_t nv = (int64_t)geo.mz * geo.ms * geo.ms, nd = (int64_t)geo.na * geo.nh * geo.nl;
  T *r = (T *)(w + L.r), *g2 = (T *)(w + L.g2), *s = (T *)(w + L.s), *y = (T *)(w + L.y);
  void *ws = w + L.ws;
  double *part = (double *)(w + L.part), *hist = (double *)(w + L.hist);
  double *scal = (double *)(w + L.scal);
  constexpr int W = V<T>::n;
  // the residual stays in stage 2's layout [h][l][b][a] (runs of n_angles)
  const int64_t drun = B > 1 ? geo.na : nd;
  const bool dv = nd % W == 0 && drun % W == 0;
  const bool fv = (nv * B) % W == 0 && (uintptr_t)f % 16 == 0;
  SRT_HIP(hipMemcpyAsync(y, f, sizeof(T) * nv * B, hipMemcpyDeviceToDevice, st));
  SRT_TRY(data_to_stage2(plan, g, g2, B, st));
  double t = 1.0;
  for (int k = 0; k < n_iter; ++k) {
    const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double beta = (t - 1.0) / t_next;
    t = t_next;
    SRT_TRY(apply_plan(plan, y, r, B, ws, L.ws_bytes, st, false, true));  // r = A y
    hipLaunchKernelGGL(k_rsub<T>, dim3(grid_for(nd * B)), dim3(256), 0, st, r, g2, nd * B);
    SRT_HIP(hipGetLastError());                                              // r = g - A y
    SRT_TRY(dot_into<T>(r, r, nd, drun, B, dv, part, scal, hist + (size_t)k * B, st));
    SRT_TRY(apply_plan(plan, r, s, B, ws, L.ws_bytes, st, true, true));   // s = A^T (g - A y)
    const dim3 grid(grid_for(fv ? nv * B / W : nv * B));
    if (fv)
      hipLaunchKernelGGL((k_fista<T, true>), grid, dim3(256), 0, st, f, y, s, (T)step, (T)beta, nv * B);
    else
      hipLaunchKernelGGL((k_fista<T, false>), grid, dim3(256), 0, st, f, y, s, (T)step, (T)beta, nv * B);
    SRT_HIP(hipGetLastError());
  }
  if (resid) {
    if (n_iter > 0)
      SRT_HIP(hipMemcpyAsync(resid, hist, sizeof(double) * (size_t)n_iter * B,
                             hipMemcpyDeviceToHost, st));
    SRT_HIP(hipStreamSynchronize(st));
  }
  return Status{};
}

template <typename T>
Status run_opnorm2(srt_plan *plan, int32_t n_iter, double *norm2, char *w, const NnlsLayout &L,
                   hipStream_t st) {
  const Geometry &geo = plan->geo;
  const int64_t nv = (int64_t)geo.mz * geo.ms * geo.ms, nd = (int64_t)geo.na * geo.nh * geo.nl;
  T *u = (T *)(w + L.r), *wv = (T *)(w + L.s), *v = (T *)(w + L.y);
  void *ws = w + L.ws;
  double *part = (double *)(w + L.part), *sc = (double *)(w + L.scal);
  constexpr int W = V<T>::n;
  const bool vv = nv % W == 0, dv = nd % W == 0;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(nv)), dim3(256), 0, st, v, (T)1, nv);
  SRT_HIP(hipGetLastError());
  for (int k = 0; k < n_iter; ++k) {
    // u = A v, kept in stage 2's layout (one item: a single run)
    SRT_TRY(apply_plan(plan, v, u, 1, ws, L.ws_bytes, st, false, true));
    SRT_TRY(dot_into<T>(u, u, nd, nd, 1, dv, part, sc, nullptr, st));      // ||A v||^2
    SRT_TRY(dot_into<T>(v, v, nv, nv, 1, vv, part, sc + 1, nullptr, st));  // ||v||^2
    SRT_TRY(apply_plan(plan, u, wv, 1, ws, L.ws_bytes, st, true, true));  // w = A^T A v
    SRT_TRY(dot_into<T>(wv, wv, nv, nv, 1, vv, part, sc + 2, nullptr, st));
    hipLaunchKernelGGL(k_normalize<T>, dim3(grid_for(nv)), dim3(256), 0, st, v, wv, sc + 2, nv);
    SRT_HIP(hipGetLastError());
  }
  double h[2] = {0.0, 0.0};
  if (n_iter > 0) SRT_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st));
  SRT_HIP(hipStreamSynchronize(st));
  *norm2 = h[1] > 0.0 ? h[0] / h[1] : 0.0;
  return Status{};
}

}  // namespace
}  // namespace srt

extern "C" {

srt_status srt_cgls_workspace(const srt_plan *plan, int32_t batch, int32_t n_iter, size_t *bytes) {
  using namespace srt;
  if (!plan || plan->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan").code;
  if (!bytes || batch <= 0 || n_iter < 0)
    return fail(SRT_EINVAL, "bytes must be non-NULL, batch >= 1 and n_iter >= 0").code;
  *bytes = layout(plan, batch, n_iter).total;
  return SRT_OK;
}

srt_status srt_cgls(srt_plan *plan, void *vol, const void *data, int32_t batch, int32_t n_iter,
                    double *resid, void *workspace, size_t workspace_bytes, void *hip_stream) {
  using namespace srt;
  if (!plan || plan->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan").code;
  if (!vol || !data) return fail(SRT_EINVAL, "NULL volume or data").code;
  if (batch <= 0 || batch > 65535 || n_iter < 0)
    return fail(SRT_EINVAL, "batch must be in [1, 65535] and n_iter >= 0").code;
  const Layout L = layout(plan, batch, n_iter);
  if (!workspace || workspace_bytes < L.total)
    return fail(SRT_EINVAL, "workspace is NULL or smaller than srt_cgls_workspace reports").code;
  // workspace vectors are read and written 16 bytes at a time
  if ((uintptr_t)workspace % 16 != 0)
    return fail(SRT_EINVAL, "workspace must be 16-byte aligned").code;
  const size_t esz = plan->vdtype == SRT_F64 ? 8 : 4;
  if ((uintptr_t)vol % esz != 0 || (uintptr_t)data % esz != 0)
    return fail(SRT_EINVAL, "volume and data must be aligned to their element size").code;
  DeviceScope ds(plan->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice").code;
  hipStream_t st = (hipStream_t)hip_stream;
  char *w = (char *)workspace;
  if (plan->vdtype == SRT_F64)
    return run<double>(plan, (double *)vol, (const double *)data, batch, n_iter, resid, w, L, st).code;
  return run<float>(plan, (float *)vol, (const float *)data, batch, n_iter, resid, w, L, st).code;
}

srt_status srt_nnls_workspace(const srt_plan *plan, int32_t batch, int32_t n_iter, size_t *bytes) {
  using namespace srt;
  if (!plan || plan->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan").code;
  if (!bytes || batch <= 0 || batch > 65535 || n_iter < 0)
    return fail(SRT_EINVAL, "bytes must be non-NULL, batch in [1, 65535] and n_iter >= 0").code;
  *bytes = nnls_layout(plan, batch, n_iter).total;
  return SRT_OK;
}

srt_status srt_nnls(srt_plan *plan, void *vol, const void *data, int32_t batch, int32_t n_iter,
                    double step, double *resid, void *workspace, size_t workspace_bytes,
                    void *hip_stream) {
  using namespace srt;
  if (!plan || plan->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan").code;
  if (!vol || !data) return fail(SRT_EINVAL, "NULL volume or data").code;
  if (batch <= 0 || batch > 65535 || n_iter < 0)
    return fail(SRT_EINVAL, "batch must be in [1, 65535] and n_iter >= 0").code;
  if (!(std::isfinite(step) && step > 0.0))
    return fail(SRT_EINVAL, "step must be finite and > 0").code;
  const NnlsLayout L = nnls_layout(plan, batch, n_iter);
  if (!workspace || workspace_bytes < L.total)
    return fail(SRT_EINVAL, "workspace is NULL or smaller than srt_nnls_workspace reports").code;
  if ((uintptr_t)workspace % 16 != 0)
    return fail(SRT_EINVAL, "workspace must be 16-byte aligned").code;
  const size_t esz = plan->vdtype == SRT_F64 ? 8 : 4;
  if ((uintptr_t)vol % esz != 0 || (uintptr_t)data % esz != 0)
    return fail(SRT_EINVAL, "volume and data must be aligned to their element size").code;
  DeviceScope ds(plan->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice").code;
  hipStream_t st = (hipStream_t)hip_stream;
  char *w = (char *)workspace;
  if (plan->vdtype == SRT_F64)
    return run_nnls<double>(plan, (double *)vol, (const double *)data, batch, n_iter, step, resid,
                            w, L, st).code;
  return run_nnls<float>(plan, (float *)vol, (const float *)data, batch, n_iter, step, resid, w,
                         L, st).code;
}

srt_status srt_opnorm2(srt_plan *plan, int32_t n_iter, double *norm2, void *workspace,
                       size_t workspace_bytes, void *hip_stream) {
  using namespace srt;
  if (!plan || plan->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan").code;
  if (!norm2 || n_iter < 0) return fail(SRT_EINVAL, "norm2 must be non-NULL and n_iter >= 0").code;
  const NnlsLayout L = nnls_layout(plan, 1, 0);
  if (!workspace || workspace_bytes < L.total)
    return fail(SRT_EINVAL, "workspace is NULL or smaller than srt_nnls_workspace(plan, 1, 0)").code;
  if ((uintptr_t)workspace % 16 != 0)
    return fail(SRT_EINVAL, "workspace must be 16-byte aligned").code;
  DeviceScope ds(plan->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice").code;
  hipStream_t st = (hipStream_t)hip_stream;
  char *w = (char *)workspace;
  if (plan->vdtype == SRT_F64) return run_opnorm2<double>(plan, n_iter, norm2, w, L, st).code;
  return run_opnorm2<float>(plan, n_iter, norm2, w, L, st).code;
}

}  // extern "C"
