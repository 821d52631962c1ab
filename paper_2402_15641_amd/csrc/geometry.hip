// FP64 arc-length geometry of the two circular Radon transforms.
//
// A12 (Sec. 2, circle transform in a z-slice, measure rho dphi): row a*nr + m
// holds, for every pixel p = j*ms + i, the length of the circle of radius
// rho[m] about the centre (cx[a], cy[a]) of column a inside p.
// A34 (Sec. 2, half-circle transform, measure l dtheta, theta in [0, pi]):
// row h*nl + l holds, for every cell (rho cell m, z slice k) with column
// index m*mz + k, the length of the half circle of radius radii[l] about
// (z = zpos[h], rho = 0) inside that cell. The rho grid is the radii unless
// the plan was given one of its own.
//
// Each row is produced by one thread that walks its circle quadrant by
// quadrant. Inside a quadrant both coordinates are monotone in the angle, so
// the crossings with the two families of cell edges come out as two sorted
// sequences; merging them yields the breakpoints in angular order, and every
// piece between breakpoints lies in the single cell that holds its mid-angle
// point. The piece's weight is radius * (angle difference). Pieces of one
// cell cut apart by a quadrant boundary or revisited later are emitted
// separately and summed when the matrix is assembled.
//
// Piecewise-linear basis (Sec. 3.1 allows other bases): the same walk runs
// over the lattice of basis nodes instead of cell edges, and every piece
// spreads its integral over the four corners of its lattice cell with the
// exact integrals of the bilinear tents along the arc. Stage 1 nodes are the
// voxel centres plus one virtual (zero) node half a voxel outside each end;
// stage 2 nodes are the z voxel centres (virtual nodes likewise) times the
// radii, with a zero node at rho = 0 and one a spacing past the last radius.
// Entries at virtual nodes are not emitted.
#include <hipcub/hipcub.hpp>

#include "srt_internal.h"

// Count and fill passes must see bit-identical arithmetic: no FMA contraction.
#pragma clang fp contract(off)

namespace srt {
namespace {

constexpr double kHalfPi = 1.5707963267948966;
constexpr double kTwoPi = 6.283185307179586;

// Cell edges x0 + i*h, i = 0..n (n cells).
struct UniformEdges {
  double x0, h;
  int n;
  __device__ double pos(int i) const { return x0 + h * (double)i; }
  __device__ double width(int) const { return h; }
  // Number of edges at or below v.
  __device__ int count_le(double v) const {
    double f = floor((v - x0) / h);
    int i = f < -1.0 ? 0 : (f > (double)n ? n + 1 : (int)f + 1);
    while (i > 0 && pos(i - 1) > v) --i;
    while (i <= n && pos(i) <= v) ++i;
    return i;
  }
  // Number of edges strictly below v.
  __device__ int count_lt(double v) const {
    int i = count_le(v);
    while (i > 0 && pos(i - 1) >= v) --i;
    return i;
  }
};

// Edges of the rho cells: midpoints between consecutive grid radii, outer
// edges half a spacing beyond the first and the last (n = grid size).
struct RhoEdges {
  const double *r;
  int n;
  __device__ double pos(int i) const {
    if (n == 1) return i == 0 ? 0.5 * r[0] : 1.5 * r[0];
    if (i == 0) return r[0] - 0.5 * (r[1] - r[0]);
    if (i == n) return r[n - 1] + 0.5 * (r[n - 1] - r[n - 2]);
    return 0.5 * (r[i] + r[i - 1]);
  }
  __device__ int count_le(double v) const {  // edges are increasing
    int lo = 0, hi = n + 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (pos(mid) <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
  __device__ int count_lt(double v) const {
    int lo = 0, hi = n + 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (pos(mid) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
};

// Nodes of the linear basis along rho: 0, the grid radii, and the last one
// plus the last spacing (a single radius r gives 0, r, 2r); n = nl + 1 cells.
struct RhoNodes {
  const double *r;
  int nl, n;
  __device__ RhoNodes(const double *radii, int count) : r(radii), nl(count), n(count + 1) {}
  __device__ double pos(int i) const {
    if (i == 0) return 0.0;
    if (i <= nl) return r[i - 1];
    return r[nl - 1] + (nl > 1 ? r[nl - 1] - r[nl - 2] : r[0]);
  }
  __device__ double width(int i) const { return pos(i + 1) - pos(i); }
  __device__ int count_le(double v) const {
    int lo = 0, hi = n + 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (pos(mid) <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
  __device__ int count_lt(double v) const {
    int lo = 0, hi = n + 1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (pos(mid) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
};

template <class E>
__device__ int cell_of(const E &e, double v) {
  int i = e.count_le(v) - 1;
  return (i >= 0 && i < e.n) ? i : -1;
}

// Walks quadrants [0, nq) of the circle (cx + r cos t, cy + r sin t) over the
// cell grid XE x YE and calls emit(ix, iy, t0, t1, cos tm, sin tm) for each
// piece [t0, t1] inside cell (ix, iy), tm = (t0 + t1) / 2.
template <class XE, class YE, class Emit>
__device__ void walk_arc(double cx, double cy, double r, int nq, const XE &xe,
                         const YE &ye, Emit &emit) {
  for (int q = 0; q < nq; ++q) {
    const double ta = kHalfPi * (double)q, tb = kHalfPi * (double)(q + 1);
    const bool right = (q == 0 || q == 3);  // cos t >= 0
    const bool upper = (q <= 1);            // sin t >= 0
    const bool x_down = (q <= 1);           // x decreases as t grows
    const bool y_up = (q == 0 || q == 3);   // y increases as t grows
    const double xlo = right ? cx : cx - r, xhi = right ? cx + r : cx;
    const double ylo = upper ? cy : cy - r, yhi = upper ? cy + r : cy;
    // Edges strictly inside the quadrant's coordinate ranges.
    const int xi0 = xe.count_le(xlo), xi1 = xe.count_lt(xhi) - 1;
    const int yi0 = ye.count_le(ylo), yi1 = ye.count_lt(yhi) - 1;
    const int nx = xi1 >= xi0 ? xi1 - xi0 + 1 : 0;
    const int ny = yi1 >= yi0 ? yi1 - yi0 + 1 : 0;

    auto x_cross = [&](int k) {
      const double X = xe.pos(x_down ? xi1 - k : xi0 + k);
      const double dx = X - cx;
      const double dy = sqrt(fmax((r - dx) * (r + dx), 0.0));
      double t = atan2(upper ? dy : -dy, dx);
      if (t < 0.0) t += kTwoPi;
      return fmin(fmax(t, ta), tb);
    };
    auto y_cross = [&](int k) {
      const double Y = ye.pos(y_up ? yi0 + k : yi1 - k);
      const double dy = Y - cy;
      const double dx = sqrt(fmax((r - dy) * (r + dy), 0.0));
      double t = atan2(dy, right ? dx : -dx);
      if (t < 0.0) t += kTwoPi;
      return fmin(fmax(t, ta), tb);
    };

    int kx = 0, ky = 0;
    double tx = nx > 0 ? x_cross(0) : tb;
    double ty = ny > 0 ? y_cross(0) : tb;
    double tprev = ta;
    for (;;) {
      double tn;
      bool last = false;
      if (kx < nx && (ky >= ny || tx <= ty)) {
        tn = tx;
        ++kx;
        tx = kx < nx ? x_cross(kx) : tb;
      } else if (ky < ny) {
        tn = ty;
        ++ky;
        ty = ky < ny ? y_cross(ky) : tb;
      } else {
        tn = tb;
        last = true;
      }
      tn = fmax(tn, tprev);
      if (tn > tprev) {
        const double tm = 0.5 * (tprev + tn);
        double s, c;
        sincos(tm, &s, &c);
        const int ix = cell_of(xe, cx + r * c);
        const int iy = cell_of(ye, cy + r * s);
        if (ix >= 0 && iy >= 0) emit(ix, iy, tprev, tn, c, s);
      }
      tprev = tn;
      if (last) break;
    }
  }
}

// One emitter serves both passes (a single instantiation of the walk, so the
// fill pass reproduces the count pass exactly). With keys == nullptr it only
// counts; otherwise it writes at most `limit` entries and reports a mismatch.
struct PieceEmit {
  double r;
  uint64_t row_key;
  int64_t stride;      // column index = iy * stride + ix
  int live;            // iy >= live is dropped
  uint64_t *keys;
  double *vals;
  int64_t limit;
  int64_t k = 0;
  __device__ void operator()(int ix, int iy, double t0, double t1, double, double) {
    if (iy >= live) return;
    if (keys && k < limit) {
      keys[k] = row_key + (uint64_t)iy * (uint64_t)stride + (uint64_t)ix;
      vals[k] = r * (t1 - t0);
    }
    ++k;
  }
};

// sin(x) - x, without the cancellation of the direct form for small |x|:
// below 1/2 the Taylor series through x^15 (truncation under 1e-17
// relative), above it sin(x) - x directly (at most a factor 24 of
// cancellation).
__device__ double sin_minus_x(double x) {
  if (fabs(x) >= 0.5) return sin(x) - x;
  const double x2 = x * x;
  double p = -1.0 / 1307674368000.0;  // -1/15!
  p = p * x2 + 1.0 / 6227020800.0;    //  1/13!
  p = p * x2 - 1.0 / 39916800.0;      // -1/11!
  p = p * x2 + 1.0 / 362880.0;        //  1/9!
  p = p * x2 - 1.0 / 5040.0;          // -1/7!
  p = p * x2 + 1.0 / 120.0;           //  1/5!
  p = p * x2 - 1.0 / 6.0;             // -1/3!
  return p * x2 * x;
}

// Linear-basis emitter. A piece [t0, t1] in lattice cell (ix, iy) with
// corners (X0, Y0) and sides (hx, hy) carries the bilinear weights
// (1-u)(1-v), u(1-v), (1-u)v, uv with u = (cx + r cos t - X0) / hx and
// v = (cy + r sin t - Y0) / hy; their integrals (measure r dt) follow in
// closed form. Written about the mid-angle tm with d = t1 - t0, s = t - tm:
//   u = um + (r/hx) (cos tm (cos s - 1) - sin tm sin s), and v likewise, so
//   int u dt  = um d + A,   A = (r/hx) cos tm * 2 (sin(d/2) - d/2)
//   int v dt  = vm d + B,   B = (r/hy) sin tm * 2 (sin(d/2) - d/2)
//   int uv dt = um vm d + um B + vm A + C,
//   C = r^2/(hx hy) sin tm cos tm ((sin d - d) - 4 (sin(d/2) - d/2))
// (terms odd in s integrate to zero). The four weights sum to r d.
// Lattice node (nx, ny) is emitted as column (ny - 1) * stride + (nx - 1)
// when 1 <= nx <= nx_real and 1 <= ny <= ny_keep (virtual nodes and rho
// nodes beyond `live` are dropped).
template <class XE, class YE>
struct LinearEmit {
  const XE &xe;
  const YE &ye;
  double cx, cy, r;
  uint64_t row_key;
  int64_t stride;
  int nx_real, ny_keep;
  uint64_t *keys;
  double *vals;
  int64_t limit;
  int64_t k = 0;
  __device__ void put(int nx, int ny, double w) {
    if (nx < 1 || nx > nx_real || ny < 1 || ny > ny_keep) return;
    if (keys && k < limit) {
      keys[k] = row_key + (uint64_t)(ny - 1) * (uint64_t)stride + (uint64_t)(nx - 1);
      vals[k] = w;
    }
    ++k;
  }
  __device__ void operator()(int ix, int iy, double t0, double t1, double c, double s) {
    double w00 = 0.0, w10 = 0.0, w01 = 0.0, w11 = 0.0;
    if (keys) {
      const double hx = xe.width(ix), hy = ye.width(iy);
      const double um = (cx + r * c - xe.pos(ix)) / hx;
      const double vm = (cy + r * s - ye.pos(iy)) / hy;
      const double d = t1 - t0;
      const double e1 = 2.0 * sin_minus_x(0.5 * d);
      const double A = (r / hx) * c * e1;
      const double B = (r / hy) * s * e1;
      const double C = (r / hx) * (r / hy) * s * c * (sin_minus_x(d) - 2.0 * e1);
      const double uv = um * vm * d + um * B + vm * A + C;
      w11 = r * uv;
      w10 = r * (um * d + A - uv);
      w01 = r * (vm * d + B - uv);
      w00 = r * (d - um * d - A - vm * d - B + uv);
    }
    put(ix, iy, w00);
    put(ix + 1, iy, w10);
    put(ix, iy + 1, w01);
    put(ix + 1, iy + 1, w11);
  }
};

// A12 row a*nr + m: circle of radius rho[m] about the column centre over the
// pixel grid.
// Pass 1 (counts != nullptr) stores the piece count; pass 2 fills.
__global__ void a12_kernel(Geometry g, const int64_t *__restrict__ offs,
                           int64_t *__restrict__ counts, uint64_t *__restrict__ keys,
                           double *__restrict__ vals, int *__restrict__ mismatch) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int64_t)g.na * g.nr) return;
  const int a = (int)(row / g.nr), m = (int)(row % g.nr);
  const double cx = g.cx[a], cy = g.cy[a], r = g.rho[m];
  const bool fill = counts == nullptr;
  const uint64_t key = (uint64_t)row * (uint64_t)g.ms * (uint64_t)g.ms;
  uint64_t *kp = fill ? keys + offs[row] : nullptr;
  double *vp = fill ? vals + offs[row] : nullptr;
  const int64_t lim = fill ? offs[row + 1] - offs[row] : 0;
  int64_t k;
  if (g.basis == SRT_BASIS_LINEAR) {
    const UniformEdges xe{g.x0 - 0.5 * g.dxy, g.dxy, g.ms + 1};  // nodes 0 .. ms+1
    LinearEmit<UniformEdges, UniformEdges> e{xe, xe, cx, cy, r, key, g.ms, g.ms, g.ms,
                                             kp, vp, lim};
    walk_arc(cx, cy, r, 4, xe, xe, e);
    k = e.k;
  } else {
    const UniformEdges xe{g.x0, g.dxy, g.ms};
    PieceEmit e{r, key, g.ms, g.ms, kp, vp, lim};
    walk_arc(cx, cy, r, 4, xe, xe, e);
    k = e.k;
  }
  if (!fill) counts[row] = k;
  else if (k != lim) atomicOr(mismatch, 1);
}

// A34 row h*nl + l: upper half circle about (zpos[h], 0) over the (z, rho)
// cells; rho cells at or beyond `live` are dropped.
__global__ void a34_kernel(Geometry g, int live, const int64_t *__restrict__ offs,
                           int64_t *__restrict__ counts, uint64_t *__restrict__ keys,
                           double *__restrict__ vals, int *__restrict__ mismatch) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int64_t)g.nh * g.nl) return;
  const int h = (int)(row / g.nl), l = (int)(row % g.nl);
  const double cz = g.zpos[h], r = g.radii[l];
  const bool fill = counts == nullptr;
  const uint64_t key = (uint64_t)row * (uint64_t)live * (uint64_t)g.mz;
  uint64_t *kp = fill ? keys + offs[row] : nullptr;
  double *vp = fill ? vals + offs[row] : nullptr;
  const int64_t lim = fill ? offs[row + 1] - offs[row] : 0;
  int64_t k;
  if (g.basis == SRT_BASIS_LINEAR) {
    const UniformEdges ze{g.z0 - 0.5 * g.dz, g.dz, g.mz + 1};  // nodes 0 .. mz+1
    const RhoNodes re(g.rho, g.nr);
    LinearEmit<UniformEdges, RhoNodes> e{ze, re, cz, 0.0, r, key, g.mz, g.mz, live,
                                         kp, vp, lim};
    walk_arc(cz, 0.0, r, 2, ze, re, e);
    k = e.k;
  } else {
    const UniformEdges ze{g.z0, g.dz, g.mz};
    const RhoEdges re{g.rho, g.nr};
    PieceEmit e{r, key, g.mz, live, kp, vp, lim};
    walk_arc(cz, 0.0, r, 2, ze, re, e);
    k = e.k;
  }
  if (!fill) counts[row] = k;
  else if (k != lim) atomicOr(mismatch, 1);
}

// Count pass, exclusive scan, fill pass.
template <class Launch>
Status pieces(int64_t nrows, hipStream_t s, Launch launch, Coo *out) {
  int64_t *counts = nullptr, *offs = nullptr;
  int *mismatch = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  Status st;
  auto cleanup = [&]() {
    (void)hipFree(counts);
    (void)hipFree(offs);
    (void)hipFree(tmp);
    (void)hipFree(mismatch);
  };
  const int threads = 256;
  const unsigned blocks = (unsigned)((nrows + threads - 1) / threads);
  hipError_t e = hipMalloc(&counts, sizeof(int64_t) * (nrows + 1));
  if (e == hipSuccess) e = hipMalloc(&offs, sizeof(int64_t) * (nrows + 1));
  if (e == hipSuccess) e = hipMalloc(&mismatch, sizeof(int));
  if (e != hipSuccess) {
    cleanup();
    return fail(SRT_ENOMEM, "device allocation for geometry counts failed");
  }
  e = hipMemsetAsync(counts + nrows, 0, sizeof(int64_t), s);
  if (e == hipSuccess) e = hipMemsetAsync(mismatch, 0, sizeof(int), s);
  if (e == hipSuccess) {
    launch(blocks, threads, (const int64_t *)nullptr, counts, (uint64_t *)nullptr,
           (double *)nullptr, mismatch);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, counts, offs, nrows + 1, s);
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes);
  if (e == hipSuccess)
    e = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, counts, offs, nrows + 1, s);
  int64_t total = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&total, offs + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "geometry count pass");
  }
  out->n = total;
  e = hipMalloc(&out->keys, sizeof(uint64_t) * (total > 0 ? total : 1));
  if (e == hipSuccess) e = hipMalloc(&out->vals, sizeof(double) * (total > 0 ? total : 1));
  if (e != hipSuccess) {
    cleanup();
    return fail(SRT_ENOMEM, "device allocation for geometry pieces failed");
  }
  launch(blocks, threads, (const int64_t *)offs, (int64_t *)nullptr, out->keys, out->vals,
         mismatch);
  e = hipGetLastError();
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, mismatch, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "geometry fill pass");
  if (bad) return fail(SRT_EDEVICE, "geometry fill pass disagrees with the count pass");
  return st;
}

}  // namespace

Status a12_pieces(const Geometry &g, hipStream_t s, Coo *out) {
  const int64_t nrows = (int64_t)g.na * g.nr;
  return pieces(nrows, s,
                [&](unsigned b, int t, const int64_t *offs, int64_t *counts, uint64_t *keys,
                    double *vals, int *mm) {
                  hipLaunchKernelGGL(a12_kernel, dim3(b), dim3(t), 0, s, g, offs, counts,
                                     keys, vals, mm);
                },
                out);
}

Status a34_pieces(const Geometry &g, int32_t live, hipStream_t s, Coo *out) {
  const int64_t nrows = (int64_t)g.nh * g.nl;
  return pieces(nrows, s,
                [&](unsigned b, int t, const int64_t *offs, int64_t *counts, uint64_t *keys,
                    double *vals, int *mm) {
                  hipLaunchKernelGGL(a34_kernel, dim3(b), dim3(t), 0, s, g, (int)live, offs,
                                     counts, keys, vals, mm);
                },
                out);
}

}  // namespace srt
