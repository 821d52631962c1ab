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

// Weight conversion to the accumulation type (bf16 and f16 are exact in f32).
template <typename T, typename WT>
__device__ __forceinline__ T to_acc(WT w);
template <> __device__ __forceinline__ float to_acc<float, float>(float w) { return w; }
template <> __device__ __forceinline__ float to_acc<float, uint16_t>(uint16_t w) {
  return __uint_as_float((uint32_t)w << 16);
}
template <> __device__ __forceinline__ float to_acc<float, _Float16>(_Float16 w) { return (float)w; }
template <> __device__ __forceinline__ double to_acc<double, double>(double w) { return w; }

template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

// An operator entry as staged in LDS: local column and weight.
template <typename T> struct LdsEnt {
  int32_t col;
  T w;
};

// Tile geometry shared by the kernel and its launcher.
template <typename T> struct TileShape {
  static constexpr int VS = 16 / sizeof(T);      // values per 16-byte vector
  static constexpr int NV = 4;                   // vectors per lane
  static constexpr int DW = 8 * NV * VS;         // dense values per slice (8 lanes per row)
  static constexpr int PIECES = DW / VS;         // 16-byte pieces per staged dense row
  static constexpr int RPG = kRB / (kNW * 8);    // rows per lane group per wavefront
};

// One workgroup = one row block x one slice of the dense index; slices are
// outermost in the grid so the current slice of the dense operand stays in
// the last-level cache while every block streams through it.
//
// Per chunk the whole workgroup stages the chunk's dense rows (DW values
// each), its entries (converted to the accumulation type) and its per-row
// entry offsets into LDS with one batch of coalesced loads. A wavefront is
// 8 groups of 8 lanes: group q works on rows q, q+8, q+16, q+24 of the
// wavefront's 32 rows, and each lane of a group owns NV vectors of the dense
// slice (lane li holds values m*8*VS + li*VS .. +VS, m < NV, so a group reads
// 8 consecutive 16-byte words per vector: conflict-free). Every entry is one
// broadcast LDS read of (column, weight), one address computation and
// NV*VS fused multiply-adds per lane.
template <typename T, typename WT>
__device__ __forceinline__ void tiled_body(const int32_t *__restrict__ blk_rows,
                                           const int32_t *__restrict__ blk_chunk,
                                           const int32_t *__restrict__ chunk_cols,
                                           const int32_t *__restrict__ chunk_ncols,
                                           const int32_t *__restrict__ chunk_ent,
                                           const int32_t *__restrict__ seg,
                                           const int32_t *__restrict__ ent_col,
                                           const WT *__restrict__ ent_w, const T *__restrict__ X,
                                           T *__restrict__ Y, int nblk, int D, T scale) {
  using S = TileShape<T>;
  using V16 = typename Vec16<T>::type;
  constexpr int VS = S::VS, NV = S::NV, DW = S::DW, PIECES = S::PIECES, RPG = S::RPG;
  constexpr int NT = kNW * 64;
  constexpr int DENSE_PER_T = kC * PIECES / NT;
  constexpr int ENT_PER_T = (kE + NT - 1) / NT;
  __shared__ V16 lds_dense[kC * PIECES];
  __shared__ LdsEnt<T> lds_ent[kE];
  __shared__ int32_t lds_seg[kRB + 1];

  const int bid = blockIdx.x;
  const int blk = bid % nblk, slice = bid / nblk;
  const int d0 = slice * DW;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, grp = lane >> 3, li = lane & 7;

  V16 acc[RPG][NV];
#pragma unroll
  for (int j = 0; j < RPG; ++j)
#pragma unroll
    for (int m = 0; m < NV; ++m) acc[j][m] = V16{};

  const bool vec_ok = (D % VS) == 0;
  const int c0 = blk_chunk[blk], c1 = blk_chunk[blk + 1];
  for (int c = c0; c < c1; ++c) {
    const int n = chunk_ncols[c];
    const int ce0 = chunk_ent[c], ne = chunk_ent[c + 1] - ce0;
    // ---- stage: every load of the chunk is issued before any LDS store
    V16 dv[DENSE_PER_T];
    int32_t ec[ENT_PER_T];
    WT ew[ENT_PER_T];
    int32_t sv = 0;
#pragma unroll
    for (int k = 0; k < DENSE_PER_T; ++k) {
      const int i = tid + k * NT;
      const int u = i / PIECES, q = i % PIECES;
      const int d = d0 + q * VS;
      dv[k] = V16{};
      if (u < n) {
        const T *src = X + (size_t)chunk_cols[(size_t)c * kC + u] * D + d;
        if (vec_ok) {
          if (d < D) dv[k] = *reinterpret_cast<const V16 *>(src);
        } else {
          T *dd = reinterpret_cast<T *>(&dv[k]);
#pragma unroll
          for (int v = 0; v < VS; ++v) dd[v] = d + v < D ? src[v] : T(0);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < ENT_PER_T; ++k) {
      const int i = tid + k * NT;
      if (i < ne) {
        ec[k] = ent_col[ce0 + i];
        ew[k] = ent_w[ce0 + i];
      }
    }
    if (tid <= kRB) sv = seg[(size_t)c * (kRB + 1) + tid];
#pragma unroll
    for (int k = 0; k < DENSE_PER_T; ++k) lds_dense[tid + k * NT] = dv[k];
#pragma unroll
    for (int k = 0; k < ENT_PER_T; ++k) {
      const int i = tid + k * NT;
      if (i < ne) lds_ent[i] = LdsEnt<T>{ec[k] * PIECES, to_acc<T, WT>(ew[k])};
    }
    if (tid <= kRB) lds_seg[tid] = sv;
    __syncthreads();
    // ---- consume
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const int pos = wave * (8 * RPG) + j * 8 + grp;
      const int e0 = lds_seg[pos], e1 = lds_seg[pos + 1];
#pragma unroll 2
      for (int e = e0; e < e1; ++e) {
        const LdsEnt<T> en = lds_ent[e];
        const V16 *g = lds_dense + en.col + li;
#pragma unroll
        for (int m = 0; m < NV; ++m) {
          const V16 x = g[m * 8];
          const T *xs = reinterpret_cast<const T *>(&x);
          T *as = reinterpret_cast<T *>(&acc[j][m]);
#pragma unroll
          for (int v = 0; v < VS; ++v) as[v] = fma(en.w, xs[v], as[v]);
        }
      }
    }
    __syncthreads();
  }
  // ---- write: each row once
#pragma unroll
  for (int j = 0; j < RPG; ++j) {
    const int pos = wave * (8 * RPG) + j * 8 + grp;
    const int row = blk_rows[(size_t)blk * kRB + pos];
    if (row < 0) continue;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int d = d0 + m * 8 * VS + li * VS;
      T *y = Y + (size_t)row * D + d;
      const T *as = reinterpret_cast<const T *>(&acc[j][m]);
      if (vec_ok && d < D) {
        V16 o;
        T *os = reinterpret_cast<T *>(&o);
#pragma unroll
        for (int v = 0; v < VS; ++v) os[v] = as[v] * scale;
        *reinterpret_cast<V16 *>(y) = o;
      } else if (!vec_ok) {
#pragma unroll
        for (int v = 0; v < VS; ++v)
          if (d + v < D) y[v] = as[v] * scale;
      }
    }
  }
}

// One named kernel per stage so traces tell the stages apart.
#define SRT_STAGE_KERNEL(NAME)                                                                 \
  template <typename T, typename WT>                                                           \
  __global__ __launch_bounds__(kNW * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void NAME( \
      const int32_t *__restrict__ blk_rows, const int32_t *__restrict__ blk_chunk,             \
      const int32_t *__restrict__ chunk_cols, const int32_t *__restrict__ chunk_ncols,         \
      const int32_t *__restrict__ chunk_ent, const int32_t *__restrict__ seg,                  \
      const int32_t *__restrict__ ent_col, const WT *__restrict__ ent_w,                       \
      const T *__restrict__ X, T *__restrict__ Y, int nblk, int D, T scale) {                  \
    tiled_body<T, WT>(blk_rows, blk_chunk, chunk_cols, chunk_ncols, chunk_ent, seg, ent_col,   \
                      ent_w, X, Y, nblk, D, scale);                                            \
  }
SRT_STAGE_KERNEL(stage1_fwd)  // A12_a applied to every slice: G = A12 F
SRT_STAGE_KERNEL(stage2_fwd)  // A34 applied to every column: Y = A34 G
SRT_STAGE_KERNEL(stage2_adj)  // G' = A34^T Y
SRT_STAGE_KERNEL(stage1_adj)  // F' = sum_a A12_a^T G'_a
#undef SRT_STAGE_KERNEL

enum class Stage { s1_fwd, s2_fwd, s2_adj, s1_adj };

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
Status spmm(Stage st, const Tiled &m, const T *X, T *Y, int D, hipStream_t s) {
  if (m.nblk <= 0 || D <= 0) return Status{};
  constexpr int DW = TileShape<T>::DW;
  const int64_t nslices = (D + DW - 1) / DW;
  const int64_t grid = m.nblk * nslices;
  if (grid > INT32_MAX) return fail(SRT_ENOTSUP, "launch grid too large");
  const T scale = (T)(1.0 / m.scale);
  const WT *w = (const WT *)m.ent_w;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kNW * 64), 0, s, m.blk_rows, m.blk_chunk,
                       m.chunk_cols, m.chunk_ncols, m.chunk_ent, m.seg, m.ent_col, w, X, Y,
                       (int)m.nblk, D, scale);
  };
  switch (st) {
    case Stage::s1_fwd: go(stage1_fwd<T, WT>); break;
    case Stage::s2_fwd: go(stage2_fwd<T, WT>); break;
    case Stage::s2_adj: go(stage2_adj<T, WT>); break;
    case Stage::s1_adj: go(stage1_adj<T, WT>); break;
  }
  SRT_HIP(hipGetLastError());
  return Status{};
}

// Records HIP events between stages when the plan is timing its applies.
struct Marks {
  StageEvents *rec = nullptr;
  hipStream_t s = nullptr;
  Status at(int i) const {
    if (rec) SRT_HIP(hipEventRecord(rec->ev[i], s));
    return Status{};
  }
};

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
Status forward_impl(srt_plan *p, const T *vol, T *data, int32_t B, T *P, T *Q, hipStream_t s,
                    const Marks &mk) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  SRT_TRY(mk.at(0));
  if (L == 0) {  // no circle meets the grid: the transform is identically zero
    SRT_HIP(hipMemsetAsync(data, 0, sizeof(T) * (size_t)B * g.na * NR, s));
    for (int i = 1; i <= kStages; ++i) SRT_TRY(mk.at(i));
    return Status{};
  }
  // vol[b][k][p] -> Ft[p][b][k]
  SRT_TRY(transpose<T>(vol, P, TDesc{g.mz, M2, B, 1, M2, (int64_t)g.mz * M2, 0, D1, g.mz, 0}, s));
  SRT_TRY(mk.at(1));
  // Stage 1 (Alg. 1 first product): G[a][l'][b][k]
  SRT_TRY((spmm<T, WT>(Stage::s1_fwd, p->t12, P, Q, D1, s)));
  SRT_TRY(mk.at(2));
  // G[a][l'][b][k] -> Gt[l'][k][b][a]
  SRT_TRY(transpose<T>(Q, P,
                       TDesc{g.na, g.mz, L, B, (int64_t)L * D1, D1, g.mz, D2,
                             (int64_t)g.mz * D2, g.na},
                       s));
  SRT_TRY(mk.at(3));
  // Stage 2 (Alg. 1 second product): Yt[h][l][b][a]
  SRT_TRY((spmm<T, WT>(Stage::s2_fwd, p->t34, P, Q, D2, s)));
  SRT_TRY(mk.at(4));
  // Yt[r][b][a] -> data[b][a][r]
  SRT_TRY(transpose<T>(Q, data, TDesc{NR, g.na, B, 1, D2, g.na, 0, NR, (int64_t)g.na * NR, 0}, s));
  SRT_TRY(mk.at(5));
  return Status{};
}

template <typename T, typename WT>
Status adjoint_impl(srt_plan *p, const T *data, T *vol, int32_t B, T *P, T *Q, hipStream_t s,
                    const Marks &mk) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  SRT_TRY(mk.at(0));
  if (L == 0) {
    SRT_HIP(hipMemsetAsync(vol, 0, sizeof(T) * (size_t)B * g.mz * M2, s));
    for (int i = 1; i <= kStages; ++i) SRT_TRY(mk.at(i));
    return Status{};
  }
  // data[b][a][r] -> Yt[r][b][a]
  SRT_TRY(transpose<T>(data, P, TDesc{g.na, NR, B, 1, NR, (int64_t)g.na * NR, 0, D2, g.na, 0}, s));
  SRT_TRY(mk.at(1));
  // Alg. 2 first product: Gt'[l'][k][b][a] = A34^T Yt
  SRT_TRY((spmm<T, WT>(Stage::s2_adj, p->t34t, P, Q, D2, s)));
  SRT_TRY(mk.at(2));
  // Gt'[l'][k][b][a] -> G'[a][l'][b][k]
  SRT_TRY(transpose<T>(Q, P,
                       TDesc{g.mz, g.na, L, B, D2, (int64_t)g.mz * D2, g.na, (int64_t)L * D1, D1,
                             g.mz},
                       s));
  SRT_TRY(mk.at(3));
  // Alg. 2 second product, summed over columns: Ft'[p][b][k] = sum_a A12_a^T G'_a
  SRT_TRY((spmm<T, WT>(Stage::s1_adj, p->t12t, P, Q, D1, s)));
  SRT_TRY(mk.at(4));
  // Ft'[p][b][k] -> vol[b][k][p]
  SRT_TRY(transpose<T>(Q, vol, TDesc{M2, g.mz, B, 1, D1, g.mz, 0, M2, (int64_t)g.mz * M2, 0}, s));
  SRT_TRY(mk.at(5));
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
  Marks mk;
  mk.s = s;
  if (p->timing) {
    StageEvents rec;
    for (int i = 0; i <= kStages; ++i) {
      hipError_t e = hipEventCreate(&rec.ev[i]);
      if (e != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(rec.ev[j]);
        return hip_fail(e, "hipEventCreate");
      }
    }
    p->timed[adjoint ? 1 : 0].push_back(rec);
    mk.rec = &p->timed[adjoint ? 1 : 0].back();
  }
  if (p->vdtype == SRT_F64) {
    using T = double;
    return adjoint ? adjoint_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk)
                   : forward_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk);
  }
  using T = float;
  switch (p->wdtype) {
    case SRT_BF16:
      return adjoint
                 ? adjoint_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk)
                 : forward_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk);
    case SRT_F16:
      return adjoint
                 ? adjoint_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk)
                 : forward_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk);
    default:
      return adjoint ? adjoint_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk)
                     : forward_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk);
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
