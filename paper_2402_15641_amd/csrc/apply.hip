// Forward (Alg. 1) and matched adjoint (Alg. 2) applies.
//
// Both CRT stages are sparse-times-dense products in which the sparse weight
// does not depend on the dense index: A12_a is shared by every z-slice and
// batch item, A34 by every column angle and batch item (Sec. 2: sensors of a
// column share the first transform; all columns share the second). The dense
// index therefore runs across the lanes of a wavefront, the weight and the
// column index of a nonzero are wave-uniform (scalar loads), and every
// nonzero costs one coalesced row read plus one FMA per lane.
//
// Layouts between the stages (row index first, dense index last):
//   Ft [p][b][k]          pixel-major volume      (Alg. 1 reshape to M_s^2 x M_z)
//   G  [a][l'][b][k]      stage-1 output           (rows a*L + l')
//   Gt [l'][k][b][a]      stage-2 input            (rows l'*mz + k, angles fastest)
//   Yt [h][l][b][a]       stage-2 output           (rows h*nl + l)
//   data [b][a][h][l]     caller layout
// L = live rho cells (circles of larger radius miss the grid).
#include <algorithm>

#include "srt_internal.h"

namespace srt {
namespace {

template <typename T, typename WT>
__device__ __forceinline__ T load_w(const WT *__restrict__ v, int e);
template <>
__device__ __forceinline__ float load_w<float, float>(const float *__restrict__ v, int e) {
  return v[e];
}
template <>
__device__ __forceinline__ float load_w<float, uint16_t>(const uint16_t *__restrict__ v, int e) {
  return __uint_as_float((uint32_t)v[e] << 16);  // bf16 -> f32, exact
}
template <>
__device__ __forceinline__ float load_w<float, _Float16>(const _Float16 *__restrict__ v, int e) {
  return (float)v[e];
}
template <>
__device__ __forceinline__ double load_w<double, double>(const double *__restrict__ v, int e) {
  return v[e];
}

template <typename T, int V> struct Vec;
template <> struct Vec<float, 1> { using type = float; };
template <> struct Vec<float, 2> { using type = float2; };
template <> struct Vec<float, 4> { using type = float4; };
template <> struct Vec<double, 1> { using type = double; };
template <> struct Vec<double, 2> { using type = double2; };

// Y[o][d] = out_scale * sum_e vals[e] * X[cols[e]][d], one wavefront per output
// row o, lanes over the dense index d (V consecutive values per lane).
// Output row o reads CSR row (o / grp_out) * grp_in + o % grp_out, which drops
// empty trailing rows of every group without touching the matrix.
template <typename T, typename WT, int V>
__global__ __launch_bounds__(256) void spmm_rows(const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ cols,
                                                 const WT *__restrict__ vals,
                                                 const T *__restrict__ X, T *__restrict__ Y,
                                                 int nrows_out, int grp_out, int grp_in, int D,
                                                 T out_scale) {
  using VT = typename Vec<T, V>::type;
  const int lane = threadIdx.x & 63;
  const int o = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + ((int)threadIdx.x >> 6));
  if (o >= nrows_out) return;
  const int src = (o / grp_out) * grp_in + (o % grp_out);
  const int d = (int)blockIdx.y * (64 * V) + lane * V;
  const bool active = d < D;
  T acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = T(0);
  const int e0 = rowptr[src], e1 = rowptr[src + 1];
  if (active) {
#pragma unroll 4
    for (int e = e0; e < e1; ++e) {
      const int c = cols[e];
      const T w = load_w<T, WT>(vals, e);
      const VT x = *reinterpret_cast<const VT *>(X + (size_t)c * D + d);
      const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = fma(w, xs[v], acc[v]);
    }
    VT out;
    T *os = reinterpret_cast<T *>(&out);
#pragma unroll
    for (int v = 0; v < V; ++v) os[v] = acc[v] * out_scale;
    *reinterpret_cast<VT *>(Y + (size_t)o * D + d) = out;
  }
}

// Batched 2-D transpose through LDS:
//   out[b1*ob1 + b2*ob2 + c*ocs + r] = in[b1*ib1 + b2*ib2 + r*irs + c]
// for r < R, c < C, b1 < n1, b2 < n2. Reads are coalesced along c, writes
// along r. Grid: x = n1*n2*ceil(C/64), y = ceil(R/64).
struct TDesc {
  int R, C, n1, n2;
  int64_t irs, ib1, ib2, ocs, ob1, ob2;
};

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ in,
                                                        T *__restrict__ out, TDesc t) {
  __shared__ T tile[64][65];
  const int ctiles = (t.C + 63) / 64;
  const int bx = blockIdx.x;
  const int ct = bx % ctiles;
  const int b = bx / ctiles;
  const int b1 = b / t.n2, b2 = b % t.n2;
  const int r0 = blockIdx.y * 64, c0 = ct * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const T *ib = in + b1 * t.ib1 + b2 * t.ib2;
  T *ob = out + b1 * t.ob1 + b2 * t.ob2;
#pragma unroll 4
  for (int rr = ty; rr < 64; rr += 4) {
    const int r = r0 + rr, c = c0 + tx;
    if (r < t.R && c < t.C) tile[rr][tx] = ib[(int64_t)r * t.irs + c];
  }
  __syncthreads();
#pragma unroll 4
  for (int cc = ty; cc < 64; cc += 4) {
    const int c = c0 + cc, r = r0 + tx;
    if (r < t.R && c < t.C) ob[(int64_t)c * t.ocs + r] = tile[tx][cc];
  }
}

template <typename T>
Status transpose(const T *in, T *out, const TDesc &t, hipStream_t s) {
  if (t.R <= 0 || t.C <= 0 || t.n1 <= 0 || t.n2 <= 0) return Status{};
  const int64_t gx = (int64_t)t.n1 * t.n2 * ((t.C + 63) / 64);
  const int64_t gy = (t.R + 63) / 64;
  if (gx > INT32_MAX || gy > 65535) return fail(SRT_ENOTSUP, "transpose grid too large");
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, in,
                     out, t);
  SRT_HIP(hipGetLastError());
  return Status{};
}

template <typename T, typename WT>
Status spmm(const Csr &m, const T *X, T *Y, int nrows_out, int grp_out, int grp_in, int D,
            hipStream_t s) {
  if (nrows_out <= 0 || D <= 0) return Status{};
  const T scale = (T)(1.0 / m.scale);
  const WT *w = (const WT *)m.vals;
  int V = 1;
  if (sizeof(T) == 4) {
    if (D % 4 == 0 && D >= 128) V = 4;
    else if (D % 2 == 0 && D >= 64) V = 2;
  } else if (D % 2 == 0 && D >= 64) {
    V = 2;
  }
  const unsigned gx = (unsigned)((nrows_out + 3) / 4);
  const unsigned gy = (unsigned)((D + 64 * V - 1) / (64 * V));
  if (gy > 65535) return fail(SRT_ENOTSUP, "dense width too large");
  switch (V) {
    case 4:
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((spmm_rows<T, WT, 4>), dim3(gx, gy), dim3(256), 0, s, m.rowptr, m.cols,
                           w, X, Y, nrows_out, grp_out, grp_in, D, scale);
      break;
    case 2:
      hipLaunchKernelGGL((spmm_rows<T, WT, 2>), dim3(gx, gy), dim3(256), 0, s, m.rowptr, m.cols, w,
                         X, Y, nrows_out, grp_out, grp_in, D, scale);
      break;
    default:
      hipLaunchKernelGGL((spmm_rows<T, WT, 1>), dim3(gx, gy), dim3(256), 0, s, m.rowptr, m.cols, w,
                         X, Y, nrows_out, grp_out, grp_in, D, scale);
  }
  SRT_HIP(hipGetLastError());
  return Status{};
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t buffer_elems(const srt_plan *p, int32_t B) {
  const Geometry &g = p->geo;
  const size_t L = (size_t)std::max(p->live, 1);
  const size_t v = (size_t)g.ms * g.ms * g.mz;
  const size_t gsz = (size_t)g.na * L * g.mz;
  const size_t y = (size_t)g.nh * g.nl * g.na;
  return (size_t)B * std::max(v, std::max(gsz, y));
}

template <typename T, typename WT>
Status forward_impl(srt_plan *p, const T *vol, T *data, int32_t B, T *P, T *Q, hipStream_t s) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  if (L == 0) {  // no circle meets the grid: the transform is identically zero
    SRT_HIP(hipMemsetAsync(data, 0, sizeof(T) * (size_t)B * g.na * NR, s));
    return Status{};
  }
  // vol[b][k][p] -> Ft[p][b][k]
  SRT_TRY(transpose<T>(vol, P, TDesc{g.mz, M2, B, 1, M2, (int64_t)g.mz * M2, 0, D1, g.mz, 0}, s));
  // Stage 1 (Alg. 1 first product): G[a][l'][b][k]
  SRT_TRY((spmm<T, WT>(p->a12, P, Q, g.na * L, L, L, D1, s)));
  // G[a][l'][b][k] -> Gt[l'][k][b][a]
  SRT_TRY(transpose<T>(Q, P,
                       TDesc{g.na, g.mz, L, B, (int64_t)L * D1, D1, g.mz, D2,
                             (int64_t)g.mz * D2, g.na},
                       s));
  // Stage 2 (Alg. 1 second product): Yt[h][l][b][a]
  SRT_TRY((spmm<T, WT>(p->a34, P, Q, NR, NR, NR, D2, s)));
  // Yt[r][b][a] -> data[b][a][r]
  SRT_TRY(transpose<T>(Q, data, TDesc{NR, g.na, B, 1, D2, g.na, 0, NR, (int64_t)g.na * NR, 0}, s));
  return Status{};
}

template <typename T, typename WT>
Status adjoint_impl(srt_plan *p, const T *data, T *vol, int32_t B, T *P, T *Q, hipStream_t s) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  if (L == 0) {
    SRT_HIP(hipMemsetAsync(vol, 0, sizeof(T) * (size_t)B * g.mz * M2, s));
    return Status{};
  }
  // data[b][a][r] -> Yt[r][b][a]
  SRT_TRY(transpose<T>(data, P, TDesc{g.na, NR, B, 1, NR, (int64_t)g.na * NR, 0, D2, g.na, 0}, s));
  // Alg. 2 first product: Gt'[l'][k][b][a] = A34^T Yt
  SRT_TRY((spmm<T, WT>(p->a34t, P, Q, L * g.mz, L * g.mz, L * g.mz, D2, s)));
  // Gt'[l'][k][b][a] -> G'[a][l'][b][k]
  SRT_TRY(transpose<T>(Q, P,
                       TDesc{g.mz, g.na, L, B, D2, (int64_t)g.mz * D2, g.na, (int64_t)L * D1, D1,
                             g.mz},
                       s));
  // Alg. 2 second product, summed over columns: Ft'[p][b][k] = sum_a A12_a^T G'_a
  SRT_TRY((spmm<T, WT>(p->a12t, P, Q, M2, M2, M2, D1, s)));
  // Ft'[p][b][k] -> vol[b][k][p]
  SRT_TRY(transpose<T>(Q, vol, TDesc{M2, g.mz, B, 1, D1, g.mz, 0, M2, (int64_t)g.mz * M2, 0}, s));
  return Status{};
}

Status get_workspace(srt_plan *p, int32_t B, void *ws, size_t ws_bytes, hipStream_t s, void **P,
                     void **Q) {
  const size_t one = align_up(buffer_elems(p, B) * dtype_size(p->vdtype));
  const size_t need = 2 * one;
  if (ws) {
    if (ws_bytes < need) return fail(SRT_EINVAL, "workspace smaller than srt_plan_footprint reports");
  } else {
    if (p->own_ws_bytes < need) {
      SRT_HIP(hipStreamSynchronize(s));
      (void)hipFree(p->own_ws);
      p->own_ws = nullptr;
      p->own_ws_bytes = 0;
      if (hipMalloc(&p->own_ws, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SRT_ENOMEM, "device allocation for workspace failed");
      }
      p->own_ws_bytes = need;
    }
    ws = p->own_ws;
  }
  *P = ws;
  *Q = (char *)ws + one;
  return Status{};
}

struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

Status apply(srt_plan *p, const void *in, void *out, int32_t B, void *ws, size_t ws_bytes,
             hipStream_t s, bool adjoint) {
  if (!p || p->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan");
  if (!in || !out) return fail(SRT_EINVAL, "NULL input or output");
  if (B <= 0) return fail(SRT_EINVAL, "batch must be >= 1");
  const Geometry &g = p->geo;
  if ((int64_t)B * g.mz > INT32_MAX / 4 || (int64_t)B * g.na > INT32_MAX / 4)
    return fail(SRT_ENOTSUP, "batch too large");
  DeviceScope ds(p->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  void *P = nullptr, *Q = nullptr;
  SRT_TRY(get_workspace(p, B, ws, ws_bytes, s, &P, &Q));
  if (p->vdtype == SRT_F64) {
    using T = double;
    return adjoint ? adjoint_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s)
                   : forward_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s);
  }
  using T = float;
  switch (p->wdtype) {
    case SRT_BF16:
      return adjoint ? adjoint_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s)
                     : forward_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s);
    case SRT_F16:
      return adjoint ? adjoint_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s)
                     : forward_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s);
    default:
      return adjoint ? adjoint_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s)
                     : forward_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s);
  }
}

}  // namespace

size_t workspace_bytes(const srt_plan *p, int32_t batch) {
  return 2 * align_up(buffer_elems(p, batch) * dtype_size(p->vdtype));
}

}  // namespace srt

extern "C" {

srt_status srt_forward(srt_plan *plan, const void *vol, void *data, int32_t batch,
                       void *workspace, size_t workspace_bytes, void *hip_stream) {
  return srt::apply(plan, vol, data, batch, workspace, workspace_bytes, (hipStream_t)hip_stream,
                    false)
      .code;
}

srt_status srt_adjoint(srt_plan *plan, const void *data, void *vol, int32_t batch,
                       void *workspace, size_t workspace_bytes, void *hip_stream) {
  return srt::apply(plan, data, vol, batch, workspace, workspace_bytes, (hipStream_t)hip_stream,
                    true)
      .code;
}

}  // extern "C"
