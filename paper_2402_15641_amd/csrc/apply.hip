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

// Tile geometry shared by the kernel and its launcher. A wavefront is
// GROUPS lane groups of LPG lanes; a group works on one row at a time and its
// lanes split the dense slice: lane li holds NV vectors of VS values, vector m
// at slice offset (m * LPG + li) * VS. One vector load of a group therefore
// covers LPG * 16 = 256 contiguous bytes, i.e. every LDS bank once.
template <typename T> struct TileShape {
  static constexpr int VS = 16 / sizeof(T);      // values per 16-byte vector
  static constexpr int LPG = 16;                 // lanes per group
  static constexpr int GROUPS = 64 / LPG;        // groups per wavefront
  static constexpr int NV = 2;                   // vectors per lane
  static constexpr int DW = LPG * NV * VS;       // dense values per slice
  static constexpr int PIECES = DW / VS;         // 16-byte pieces per staged dense row
  static_assert(kNW * GROUPS == kNQ, "one quad per lane group");
  static constexpr int NT = kNW * 64;            // threads per workgroup
  static constexpr int E = sizeof(T) == 4 ? kE32 : kE64;  // entries per chunk
  static constexpr int DENSE_PER_T = kC * PIECES / NT;
  static constexpr int ENT_PER_T = (E + NT - 1) / NT;
};

// One chunk's staged data while it travels from memory to LDS.
template <typename T, typename WT> struct InFlight {
  typename Vec16<T>::type dv[TileShape<T>::DENSE_PER_T];
  int32_t ec[TileShape<T>::ENT_PER_T];
  WT ew[TileShape<T>::ENT_PER_T];
  int32_t sv;
};

// One workgroup (one per CU) = one row block x one slice of the dense
// index; slices are outermost in the grid so the current slice of the dense
// operand stays in the last-level cache while every block streams through it.
//
// Chunks are double-buffered in LDS: while the wavefronts consume chunk c
// from one buffer, the loads of chunk c+1 (its dense rows, entries and
// per-row offsets) are in flight into registers and land in the other buffer
// afterwards; the columns of chunk c+2 are fetched one step earlier still.
// A wavefront is GROUPS lane groups (see TileShape); each group runs one
// quad (kQ rows) in lockstep: per step it reads kQ entries (one per quad row,
// padded so the rows advance together), kQ * NV dense vectors and does
// kQ * NV * VS fused multiply-adds per lane.
template <typename T, typename WT, bool VEC>
__device__ __forceinline__ void tiled_body(const int32_t *__restrict__ blk_rows,
                                           const int32_t *__restrict__ blk_chunk,
                                           const int32_t *__restrict__ chunk_cols,
                                           const int32_t *__restrict__ chunk_ncols,
                                           const int32_t *__restrict__ chunk_ent,
                                           const int32_t *__restrict__ qseg,
                                           const int32_t *__restrict__ ent_col,
                                           const WT *__restrict__ ent_w, const T *__restrict__ X,
                                           T *__restrict__ Y, int nblk, int D, T scale) {
  using S = TileShape<T>;
  using V16 = typename Vec16<T>::type;
  constexpr int VS = S::VS, NV = S::NV, DW = S::DW, PIECES = S::PIECES;
  constexpr int LPG = S::LPG, GROUPS = S::GROUPS;
  constexpr int NT = S::NT, DPT = S::DENSE_PER_T, EPT = S::ENT_PER_T, E = S::E;
  __shared__ V16 lds_dense[2][(kC + 1) * PIECES];  // column kC stays zero (padding)
  __shared__ LdsEnt<T> lds_ent[2][E];
  __shared__ int32_t lds_seg[2][kNQ + 1];

  const int bid = blockIdx.x;
  const int blk = bid % nblk, slice = bid / nblk;
  const int d0 = slice * DW;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, grp = lane / LPG, li = lane % LPG;
  const int q = tid % PIECES;            // piece within a dense row
  const int d_piece = d0 + q * VS;
  // VEC: the dense width D is a multiple of VS, so rows are read and written
  // in whole 16-byte vectors (otherwise element by element).
  constexpr bool vec_ok = VEC;

  V16 acc[kQ][NV];
#pragma unroll
  for (int j = 0; j < kQ; ++j)
#pragma unroll
    for (int m = 0; m < NV; ++m) acc[j][m] = V16{};
  if (tid < PIECES) {
    lds_dense[0][kC * PIECES + tid] = V16{};
    lds_dense[1][kC * PIECES + tid] = V16{};
  }

  const int c0 = blk_chunk[blk], c1 = blk_chunk[blk + 1];

  // Column of the dense row behind this thread's k-th piece of chunk c.
  auto load_cols = [&](int c, int32_t *cols) {
#pragma unroll
    for (int k = 0; k < DPT; ++k) cols[k] = chunk_cols[(size_t)c * kC + (tid + k * NT) / PIECES];
  };
  auto issue = [&](int c, const int32_t *cols, InFlight<T, WT> &st) {
    const int n = chunk_ncols[c];
    const int ce0 = chunk_ent[c], ne = chunk_ent[c + 1] - ce0;
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int u = (tid + k * NT) / PIECES;
      st.dv[k] = V16{};
      if (u < n) {
        const T *src = X + (size_t)cols[k] * D + d_piece;
        if constexpr (VEC) {
          if (d_piece < D) st.dv[k] = *reinterpret_cast<const V16 *>(src);
        } else {
          T *dd = reinterpret_cast<T *>(&st.dv[k]);
#pragma unroll
          for (int v = 0; v < VS; ++v)
            if (d_piece + v < D) dd[v] = src[v];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * NT;
      st.ec[k] = 0;
      st.ew[k] = WT{};
      if (i < ne) {
        st.ec[k] = ent_col[ce0 + i];
        st.ew[k] = ent_w[ce0 + i];
      }
    }
    st.sv = tid <= kNQ ? qseg[(size_t)c * (kNQ + 1) + tid] : 0;
  };
  auto commit = [&](int buf, const InFlight<T, WT> &st) {
#pragma unroll
    for (int k = 0; k < DPT; ++k) lds_dense[buf][tid + k * NT] = st.dv[k];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = tid + k * NT;
      if (i < E) lds_ent[buf][i] = LdsEnt<T>{st.ec[k] * PIECES, to_acc<T, WT>(st.ew[k])};
    }
    if (tid <= kNQ) lds_seg[buf][tid] = st.sv;
  };

  if (c0 < c1) {
    int32_t cols_next[DPT], cols_after[DPT];
    InFlight<T, WT> st;
    load_cols(c0, cols_next);
    issue(c0, cols_next, st);
    if (c0 + 1 < c1) load_cols(c0 + 1, cols_next);
    commit(0, st);
    __syncthreads();
    for (int c = c0; c < c1; ++c) {
      // Keep each chunk's loads inside its own iteration: if the compiler
      // rotates some of them behind the barrier, the loop head waits for them.
      asm volatile("" ::: "memory");
      const int cur = (c - c0) & 1;
      const bool more = c + 1 < c1;
      if (more) {
        issue(c + 1, cols_next, st);
        if (c + 2 < c1) load_cols(c + 2, cols_after);
      }
      // ---- consume chunk c: this lane group's quad, kQ rows in lockstep
      {
        const int q = wave * GROUPS + grp;
        const int e0 = lds_seg[cur][q], e1 = lds_seg[cur][q + 1];
        for (int e = e0; e < e1; e += kQ) {
          LdsEnt<T> en[kQ];
#pragma unroll
          for (int j = 0; j < kQ; ++j) en[j] = lds_ent[cur][e + j];
          V16 x[kQ][NV];
#pragma unroll
          for (int j = 0; j < kQ; ++j)
#pragma unroll
            for (int m = 0; m < NV; ++m) x[j][m] = lds_dense[cur][en[j].col + li + m * LPG];
#pragma unroll
          for (int j = 0; j < kQ; ++j)
#pragma unroll
            for (int m = 0; m < NV; ++m) {
              const T *xs = reinterpret_cast<const T *>(&x[j][m]);
              T *as = reinterpret_cast<T *>(&acc[j][m]);
#pragma unroll
              for (int v = 0; v < VS; ++v) as[v] = fma(en[j].w, xs[v], as[v]);
            }
        }
      }
      if (more) {
        commit(cur ^ 1, st);
#pragma unroll
        for (int k = 0; k < DPT; ++k) cols_next[k] = cols_after[k];
      }
      __syncthreads();
    }
  }
  // ---- write: each row once
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    const int slot = (wave * GROUPS + grp) * kQ + j;
    const int row = blk_rows[(size_t)blk * kRB + slot];
    if (row < 0) continue;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
      const int d = d0 + (m * LPG + li) * VS;
      T *y = Y + (size_t)row * D + d;
      const T *as = reinterpret_cast<const T *>(&acc[j][m]);
      if constexpr (VEC) {
        if (d < D) {
          V16 o;
          T *os = reinterpret_cast<T *>(&o);
#pragma unroll
          for (int v = 0; v < VS; ++v) os[v] = as[v] * scale;
          *reinterpret_cast<V16 *>(y) = o;
        }
      } else {
#pragma unroll
        for (int v = 0; v < VS; ++v)
          if (d + v < D) y[v] = as[v] * scale;
      }
    }
  }
}

// One named kernel per stage so traces tell the stages apart.
#define SRT_STAGE_KERNEL(NAME)                                                                 \
  template <typename T, typename WT, bool VEC>                                                 \
  __global__ __launch_bounds__(kNW * 64) void NAME(                                           \
      const int32_t *__restrict__ blk_rows, const int32_t *__restrict__ blk_chunk,             \
      const int32_t *__restrict__ chunk_cols, const int32_t *__restrict__ chunk_ncols,         \
      const int32_t *__restrict__ chunk_ent, const int32_t *__restrict__ qseg,                 \
      const int32_t *__restrict__ ent_col, const WT *__restrict__ ent_w,                       \
      const T *__restrict__ X, T *__restrict__ Y, int nblk, int D, T scale) {                  \
    tiled_body<T, WT, VEC>(blk_rows, blk_chunk, chunk_cols, chunk_ncols, chunk_ent, qseg,      \
                           ent_col, ent_w, X, Y, nblk, D, scale);                              \
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
                       m.chunk_cols, m.chunk_ncols, m.chunk_ent, m.qseg, m.ent_col, w, X, Y,
                       (int)m.nblk, D, scale);
  };
  const bool vec = D % TileShape<T>::VS == 0;
  switch (st) {
    case Stage::s1_fwd: vec ? go(stage1_fwd<T, WT, true>) : go(stage1_fwd<T, WT, false>); break;
    case Stage::s2_fwd: vec ? go(stage2_fwd<T, WT, true>) : go(stage2_fwd<T, WT, false>); break;
    case Stage::s2_adj: vec ? go(stage2_adj<T, WT, true>) : go(stage2_adj<T, WT, false>); break;
    case Stage::s1_adj: vec ? go(stage1_adj<T, WT, true>) : go(stage1_adj<T, WT, false>); break;
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
