// Row-blocked, chunked format of a CRT operator for the LDS-staged product.
//
// Every nonzero of A12 or A34 multiplies a whole row of the dense operand
// (the slices of F for stage 1, the column angles of G for stage 2), and that
// row is needed again by every nonzero in the same column -- but only rows
// whose arcs pass through the same cell share columns. Rows whose arcs lie
// close together (one sensor column and neighbouring radii, neighbouring
// heights, a compact tile of pixels or of rho-z cells) share most cells, so
// the rows are grouped into geometrically compact blocks of kRB rows. One
// workgroup owns a block and one slice of the dense index. It walks the union
// of the block's columns in chunks; per chunk it stages the chunk's dense
// rows, entries and quad offsets into LDS, and every row of the block then
// consumes them from LDS. The rows' accumulators stay in registers across
// chunks, so every output element is written once, in a fixed order.
//
// Quads: the kernel runs kQ rows ("a quad", consecutive block slots) in
// lockstep on one lane group. Within a chunk the quad's row segments are
// padded to the same length and interleaved (entry k of quad row j at
// 4k + j), padding entries pointing at an all-zero LDS column (index kC) with
// weight 0. Chunks are cut greedily along the block's ascending columns so
// that both the column count (<= kC) and the padded entry count (<= max_ent)
// fit the LDS budget.
//
// Format:
//   blk_rows[b*kRB + slot]        global row at block slot (-1: none)
//   blk_chunk[b] .. [b+1]         chunks of block b (consecutive ids)
//   chunk_cols[c*kC + u]          global column of local column u of chunk c
//   chunk_ncols[c]                columns in chunk c
//   chunk_ent[c] .. [c+1]         padded entries of chunk c
//   qseg[c*(kNQ+1) + q]           first entry of quad q, relative to chunk_ent[c]
//   ent_col[e], ent_w[e]          local column and weight of entry e (16-bit
//                                 weights: one packed word, see Tiled::packed)
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "srt_internal.h"

namespace srt {
namespace {

unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

struct Buf {
  void *p = nullptr;
  ~Buf() { (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 8); }
  template <class T> T *as() const { return (T *)p; }
};

__device__ __forceinline__ void block_of(const RowGrid &g, int64_t row, int64_t *blk, int *slot) {
  const int64_t i1 = row / g.n2, i2 = row - i1 * g.n2;
  const int64_t nb1 = (g.n1 + g.b1 - 1) / g.b1, nb2 = (g.n2 + g.b2 - 1) / g.b2;
  const int64_t q1 = i1 / g.b1, q2 = i2 / g.b2, t = q1 / g.tile;
  const int64_t w = nb1 - t * g.tile < g.tile ? nb1 - t * g.tile : g.tile;  // last tile may be short
  *blk = t * g.tile * nb2 + q2 * w + (q1 - t * g.tile);
  *slot = g.along_i1 ? (int)((i2 % g.b2) * g.b1 + i1 % g.b1) : (int)((i1 % g.b1) * g.b2 + i2 % g.b2);
}

// Inverse of block_of's numbering: the (i1 group, i2 group) of block blk.
__device__ __forceinline__ void block_groups(const RowGrid &g, int64_t blk, int64_t *q1,
                                             int64_t *q2) {
  const int64_t nb1 = (g.n1 + g.b1 - 1) / g.b1, nb2 = (g.n2 + g.b2 - 1) / g.b2;
  const int64_t t = blk / (g.tile * nb2), rem = blk - t * g.tile * nb2;
  const int64_t w = nb1 - t * g.tile < g.tile ? nb1 - t * g.tile : g.tile;
  *q2 = rem / w;
  *q1 = t * g.tile + rem % w;
}

__device__ int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_rows(const int32_t *__restrict__ rowptr, int64_t nrows, RowGrid g,
                       int32_t *__restrict__ blk_rows, int32_t *__restrict__ row_of) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  int64_t b;
  int slot;
  block_of(g, r, &b, &slot);
  blk_rows[b * kRB + slot] = (int32_t)r;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) row_of[e] = (int32_t)r;
}

// Key (block, column) and the entry's own index, to sort entries by block and column.
__global__ void k_bc_keys(const int32_t *__restrict__ row_of, const int32_t *__restrict__ cols,
                          int64_t nnz, RowGrid g, uint64_t *__restrict__ keys,
                          int32_t *__restrict__ idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int64_t b;
  int slot;
  block_of(g, row_of[e], &b, &slot);
  keys[e] = ((uint64_t)b << 32) | (uint32_t)cols[e];
  idx[e] = (int32_t)e;
}

// Slot of every entry in (block, column) order.
__global__ void k_sorted_slots(const int32_t *__restrict__ idx_sorted,
                               const int32_t *__restrict__ row_of, int64_t nnz, RowGrid g,
                               uint8_t *__restrict__ slot_sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  int64_t b;
  int slot;
  block_of(g, row_of[idx_sorted[i]], &b, &slot);
  slot_sorted[i] = (uint8_t)slot;
}

// Sort key of distinct (block, column) key j under a polar column order:
// block in the high word, the column's angle about the centre of the block's
// numbering tile, scaled to [0, 2^32), in the low word.
__global__ void k_polar_keys(const uint64_t *__restrict__ ukeys, int64_t nu, RowGrid g,
                             ColumnOrder o, uint64_t *__restrict__ okeys,
                             int32_t *__restrict__ oidx) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nu) return;
  const int64_t b = (int64_t)(ukeys[j] >> 32);
  const int64_t col = (int64_t)(ukeys[j] & 0xffffffffu);
  int64_t q1, q2;
  block_groups(g, b, &q1, &q2);
  // the centre of the block's numbering tile: blocks that run side by side
  // walk the same sectors (measured 1% faster than each block's own centre)
  const int64_t t = q1 / g.tile;
  const int64_t r0 = t * g.tile * g.b1;
  const int64_t r1 = r0 + g.tile * g.b1 < g.n1 ? r0 + g.tile * g.b1 : g.n1;
  double px, py, cx = 0.0, cy = 0.0;
  if (o.kind == 1) {  // pixel about the mean position of the block's sensor columns
    for (int64_t r = r0; r < r1; ++r) {
      cx += o.cx[r];
      cy += o.cy[r];
    }
    px = o.x0 + ((double)(col % o.ms) + 0.5) * o.dxy;
    py = o.x0 + ((double)(col / o.ms) + 0.5) * o.dxy;
  } else {  // (rho, z) cell about the block's mean sensor height on the axis
    for (int64_t r = r0; r < r1; ++r) cy += o.zpos[r];
    px = o.rho[col / o.mz];
    py = o.z0 + ((double)(col % o.mz) + 0.5) * o.dz;
  }
  const double n = (double)(r1 - r0);
  const double a = atan2(py - cy / n, px - cx / n);  // (-pi, pi]
  double u = (a + M_PI) / (2.0 * M_PI);
  u = u < 0.0 ? 0.0 : (u >= 1.0 ? 0.0 : u);
  okeys[j] = ((uint64_t)b << 32) | (uint64_t)(u * 4294967296.0);
  oidx[j] = (int32_t)j;
}

// ustart[b]: first distinct (block, col) key of block b, b in [0, nblk].
__global__ void k_ustart(const uint64_t *__restrict__ ukeys, int64_t nu, int64_t nblk,
                         int64_t *__restrict__ ustart) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblk) return;
  ustart[b] = lower_bound_u64(ukeys, nu, (uint64_t)b << 32);
}

// Greedy cut of each block's distinct columns (in chunking order) into chunks with at
// most kC columns and at most max_ent entries once every quad's rows are
// padded to the quad's longest segment. One wavefront per block: lane l holds
// the open chunk's entry counts of slots l*SPL .. l*SPL+SPL-1 in registers; the
// lanes of a quad agree on its longest segment by shuffles, and the padded
// entries a column adds are summed over the wavefront. A column that breaks a
// limit closes the chunk and opens a new one holding it alone (that always
// fits: at most one entry per row, so at most kQ padded entries per quad).
constexpr int kChunkThreads = 64;
constexpr int kSPL = kRB / kChunkThreads;  // slots per lane
static_assert(kRB % kChunkThreads == 0 && (kSPL == 2 || kSPL == 4) && kQ == 4,
              "a quad spans two lanes (two slots each) or one lane (four slots)");
__global__ __launch_bounds__(kChunkThreads) void k_chunking(
    const int64_t *__restrict__ ustart, const int32_t *__restrict__ ucount,
    const int64_t *__restrict__ upos, const uint8_t *__restrict__ slot_sorted,
    const int32_t *__restrict__ uorder, int64_t nblk, int max_ent,
    int32_t *__restrict__ uchunk, int32_t *__restrict__ ulocal, int64_t *__restrict__ nch) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  if (b == nblk) {
    if (lane == 0) nch[b] = 0;
    return;
  }
  int cnt[kSPL];
#pragma unroll
  for (int t = 0; t < kSPL; ++t) cnt[t] = 0;
  int qmax = 0;  // longest segment of this lane's quad in the open chunk
  // the quad's padded entries are counted by its first lane only
  const bool quad_lead = kSPL == 4 || (lane & 1) == 0;
  int32_t chunk = 0, ncol = 0, padded = 0;
  const int64_t j0 = ustart[b], j1 = ustart[b + 1];
  for (int64_t jj = j0; jj < j1; ++jj) {
    // the block's distinct columns in chunking order (a permutation within
    // the block's range)
    const int64_t j = uorder ? uorder[jj] : jj;
    const int64_t e0 = upos[j];
    const int n = ucount[j];
    for (;;) {
      int nc[kSPL];
#pragma unroll
      for (int t = 0; t < kSPL; ++t) nc[t] = cnt[t];
      for (int i = 0; i < n; ++i) {
        const int sl = slot_sorted[e0 + i];
#pragma unroll
        for (int t = 0; t < kSPL; ++t) nc[t] += sl == lane * kSPL + t;
      }
      int m = nc[0];
#pragma unroll
      for (int t = 1; t < kSPL; ++t) m = max(m, nc[t]);
      if (kSPL == 2) m = max(m, __shfl_xor(m, 1));
      int add = quad_lead && m > qmax ? kQ * (m - qmax) : 0;
#pragma unroll
      for (int o = kChunkThreads / 2; o > 0; o >>= 1) add += __shfl_xor(add, o);
      if (ncol > 0 && (ncol + 1 > kC || padded + add > max_ent)) {
#pragma unroll
        for (int t = 0; t < kSPL; ++t) cnt[t] = 0;
        qmax = 0;
        ++chunk;
        ncol = 0;
        padded = 0;
        continue;  // the column again, alone in the new chunk
      }
#pragma unroll
      for (int t = 0; t < kSPL; ++t) cnt[t] = nc[t];
      qmax = max(qmax, m);
      padded += add;
      break;
    }
    if (lane == 0) {
      uchunk[j] = chunk;
      ulocal[j] = ncol;
    }
    ++ncol;
  }
  if (lane == 0) nch[b] = j1 > j0 ? chunk + 1 : 0;
}

__global__ void k_chunk_cols(const uint64_t *__restrict__ ukeys, int64_t nu,
                             const int64_t *__restrict__ chunk0, const int32_t *__restrict__ uchunk,
                             const int32_t *__restrict__ ulocal, int32_t *__restrict__ chunk_cols,
                             int32_t *__restrict__ chunk_ncols) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nu) return;
  const int64_t b = (int64_t)(ukeys[j] >> 32);
  const int64_t c = chunk0[b] + uchunk[j];
  chunk_cols[c * kC + ulocal[j]] = (int32_t)(uint32_t)(ukeys[j] & 0xffffffffu);
  atomicMax(&chunk_ncols[c], ulocal[j] + 1);
}

__global__ void k_blk_chunk(const int64_t *__restrict__ chunk0, int64_t nblk,
                            int32_t *__restrict__ blk_chunk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= nblk) blk_chunk[b] = (int32_t)chunk0[b];
}

// For the entries of distinct key j (contiguous in (block, column) order):
// chunk, local column and the (chunk, slot) sort key.
__global__ void k_entry_keys(const uint64_t *__restrict__ ukeys, const int32_t *__restrict__ ucount,
                             const int64_t *__restrict__ upos, int64_t nu,
                             const int64_t *__restrict__ chunk0, const int32_t *__restrict__ uchunk,
                             const int32_t *__restrict__ ulocal,
                             const uint8_t *__restrict__ slot_sorted, uint64_t *__restrict__ key2,
                             int32_t *__restrict__ local, int32_t *__restrict__ seq) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nu) return;
  const int64_t b = (int64_t)(ukeys[j] >> 32);
  const int64_t c = chunk0[b] + uchunk[j];
  for (int64_t i = upos[j]; i < upos[j] + ucount[j]; ++i) {
    key2[i] = (uint64_t)c * kRB + slot_sorted[i];
    local[i] = ulocal[j];
    seq[i] = (int32_t)i;
  }
}

// rawstart[sid] = first entry of segment sid = chunk * kRB + slot.
__global__ void k_rawstart(const uint64_t *__restrict__ key2s, int64_t nnz, int64_t nseg,
                           int64_t *__restrict__ rawstart) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nseg) return;
  rawstart[t] = lower_bound_u64(key2s, nnz, (uint64_t)t);
}

// Padded length of quad (chunk, q): kQ times its longest row segment.
__global__ void k_quad_len(const int64_t *__restrict__ rawstart, int64_t nquad,
                           int64_t *__restrict__ qlen) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nquad) return;
  if (t == nquad) {
    qlen[t] = 0;
    return;
  }
  int64_t m = 0;
  for (int j = 0; j < kQ; ++j) {
    const int64_t len = rawstart[t * kQ + j + 1] - rawstart[t * kQ + j];
    m = len > m ? len : m;
  }
  qlen[t] = kQ * m;
}

// The quads of a block, placed on the stage kernels' wavefronts. A wavefront
// steps through a chunk as long as its longest quad while the lanes of its
// shorter quads idle (masked lanes cost almost as much as active ones), so the
// quads that share a wavefront should have similar lengths chunk by chunk.
// Local search from the identity placement: swap two quads of different
// wavefronts whenever that lowers the sum over the block's chunks of each
// wavefront's longest quad, in a fixed pair order, until a pass makes no swap
// (at most kPermPasses passes). One wavefront per block; its lanes split the
// chunks. Blocks of more than kPermMaxChunks chunks keep the identity.
// perm[b * kNQ + q] = position of quad q (its rows keep their order).
constexpr int kPermPasses = 8;
// a quad's steps in a chunk are at most max_ent / kQ
using QuadSteps = std::conditional_t<(kE32 / kQ < 256), uint8_t, uint16_t>;
static_assert(kE32 >= kE64 && kE32 / kQ < 65536, "quad steps fit their type");
constexpr int kPermMaxChunks = 32768 / (kNQ * (int)sizeof(QuadSteps));  // 32 KB of LDS
__global__ __launch_bounds__(64) void k_quad_place(const int64_t *__restrict__ chunk0,
                                                   const int64_t *__restrict__ qlen,
                                                   int32_t *__restrict__ perm) {
  static_assert(kNQ <= 64, "one lane per quad position");
  __shared__ QuadSteps steps[kPermMaxChunks * kNQ];  // [chunk][quad]
  __shared__ int inv[kNQ];                           // position -> quad
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t c0 = chunk0[b], C = chunk0[b + 1] - c0;
  if (lane < kNQ) inv[lane] = lane;
  const bool search = C > 1 && C <= kPermMaxChunks;
  if (search)
    for (int64_t i = lane; i < C * kNQ; i += 64) steps[i] = (QuadSteps)(qlen[c0 * kNQ + i] / kQ);
  __syncthreads();
  for (int pass = 0; search && pass < kPermPasses; ++pass) {
    bool swapped = false;
    for (int pa = 0; pa < kNQ; ++pa)
      for (int pb = pa + 1; pb < kNQ; ++pb) {
        const int wa = pa / kQuadsPerWave, wb = pb / kQuadsPerWave;
        if (wa == wb) continue;
        const int qa = inv[pa], qb = inv[pb];
        int d = 0;  // change of the two wavefronts' summed longest quads
        for (int64_t c = lane; c < C; c += 64) {
          const QuadSteps *sc = steps + c * kNQ;
          int oa = 0, na = 0, ob = 0, nb = 0;
#pragma unroll
          for (int k = 0; k < kQuadsPerWave; ++k) {
            const int xa = wa * kQuadsPerWave + k, xb = wb * kQuadsPerWave + k;
            const int va = sc[inv[xa]], vb = sc[inv[xb]];
            oa = max(oa, va);
            ob = max(ob, vb);
            na = max(na, xa == pa ? (int)sc[qb] : va);
            nb = max(nb, xb == pb ? (int)sc[qa] : vb);
          }
          d += na + nb - oa - ob;
        }
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
        if (d < 0) {  // the same sum on every lane: a uniform decision
          __syncthreads();
          if (lane == 0) {
            inv[pa] = qb;
            inv[pb] = qa;
          }
          __syncthreads();
          swapped = true;
        }
      }
    if (!swapped) break;
  }
  if (lane < kNQ) perm[b * kNQ + inv[lane]] = lane;
}

// cblk[c] = the block of chunk c.
__global__ void k_chunk_blk(const int64_t *__restrict__ chunk0, int64_t nblk,
                            int32_t *__restrict__ cblk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  for (int64_t c = chunk0[b]; c < chunk0[b + 1]; ++c) cblk[c] = (int32_t)b;
}

// Quad lengths by position: qpos[c * kNQ + perm(q)] = qlen[c * kNQ + q].
__global__ void k_place_qlen(const int64_t *__restrict__ qlen, const int32_t *__restrict__ cblk,
                             const int32_t *__restrict__ perm, int64_t nquad,
                             int64_t *__restrict__ qpos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nquad) return;
  if (t == nquad) {
    qpos[t] = 0;
    return;
  }
  const int64_t c = t / kNQ;
  qpos[c * kNQ + perm[(int64_t)cblk[c] * kNQ + t % kNQ]] = qlen[t];
}

// Block rows by position: slot q * kQ + j moves to perm(q) * kQ + j.
__global__ void k_place_rows(const int32_t *__restrict__ rows, const int32_t *__restrict__ perm,
                             int64_t nblk, int32_t *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblk * kNQ) return;
  const int64_t b = t / kNQ;
  const int q = (int)(t % kNQ), p = perm[t];
  for (int j = 0; j < kQ; ++j) out[b * kRB + p * kQ + j] = rows[b * kRB + q * kQ + j];
}

__global__ void k_chunk_meta2(const int64_t *__restrict__ qstart, int64_t nchunk,
                              int32_t *__restrict__ chunk_ent, int32_t *__restrict__ qseg) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nchunk * (kNQ + 1)) {
    const int64_t c = t / (kNQ + 1), q = t % (kNQ + 1);
    qseg[t] = (int32_t)(qstart[c * kNQ + q] - qstart[c * kNQ]);
  }
  if (t <= nchunk) chunk_ent[t] = (int32_t)qstart[t * kNQ];
}

__global__ void k_pad_fill(int64_t n, int32_t *__restrict__ ent_col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ent_col[i] = kC;
}

// Packed 16-bit entries: a staged row's LDS offset in the low half of the word.
__host__ __device__ constexpr uint32_t packed_row(int u) {
  return ((uint32_t)u * kStagedRowBytes) >> kPackShift;
}

// Packed padding entries: weight 0, the all-zero row kC.
__global__ void k_pad_fill_packed(int64_t n, uint32_t *__restrict__ pack) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pack[i] = packed_row(kC);
}

// Entry i (in (chunk, slot) order) goes to row j = slot % kQ of its quad at
// padded position kQ * k + j, k = its rank within the row segment.
template <typename W>
__global__ void k_scatter(const uint64_t *__restrict__ key2s, const int32_t *__restrict__ perm2,
                          int64_t nnz, const int64_t *__restrict__ rawstart,
                          const int64_t *__restrict__ qstart, const int32_t *__restrict__ cblk,
                          const int32_t *__restrict__ place, const int32_t *__restrict__ local,
                          const int32_t *__restrict__ idx_sorted, const W *__restrict__ vals,
                          int32_t *__restrict__ ent_col, W *__restrict__ ent_w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int64_t sid = (int64_t)key2s[i];
  const int64_t c = sid / kRB;
  const int slot = (int)(sid % kRB);
  const int64_t k = i - rawstart[sid];
  const int pos = place[(int64_t)cblk[c] * kNQ + slot / kQ];
  const int64_t dst = qstart[c * kNQ + pos] + kQ * k + slot % kQ;
  const int32_t src = perm2[i];  // position in (block, column) order
  ent_col[dst] = local[src];
  ent_w[dst] = vals[idx_sorted[src]];
}

// As k_scatter, into the packed 16-bit layout: entry dst is word dst, the
// weight's bits in its high half, the local column's staged row in the low.
__global__ void k_scatter_packed(const uint64_t *__restrict__ key2s, const int32_t *__restrict__ perm2,
                                 int64_t nnz, const int64_t *__restrict__ rawstart,
                                 const int64_t *__restrict__ qstart, const int32_t *__restrict__ cblk,
                                 const int32_t *__restrict__ place, const int32_t *__restrict__ local,
                                 const int32_t *__restrict__ idx_sorted,
                                 const uint16_t *__restrict__ vals, uint32_t *__restrict__ pack) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int64_t sid = (int64_t)key2s[i];
  const int64_t c = sid / kRB;
  const int slot = (int)(sid % kRB);
  const int64_t k = i - rawstart[sid];
  const int pos = place[(int64_t)cblk[c] * kNQ + slot / kQ];
  const int64_t dst = qstart[c * kNQ + pos] + kQ * k + slot % kQ;
  const int32_t src = perm2[i];
  pack[dst] = ((uint32_t)vals[idx_sorted[src]] << 16) | packed_row(local[src]);
}

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

template <typename In, typename F>
Status scan_to_i64(const In *in, int64_t *out, int64_t n, hipStream_t s, F oom) {
  size_t b = 0;
  Buf tmp;
  SRT_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, b, in, out, (int)n, s));
  if (tmp.alloc(b)) return oom();
  SRT_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, b, in, out, (int)n, s));
  return Status{};
}

}  // namespace

size_t Tiled::bytes() const {
  return sizeof(int32_t) * ((size_t)nblk * kRB + nblk + 1 + (size_t)nchunk * (kC + 1) + nchunk + 1 +
                            (size_t)nchunk * (kNQ + 1)) +
         (packed ? 4 : sizeof(int32_t) + dtype_size(wdtype)) * (size_t)nnz;
}

void Tiled::release() {
  for (void *p : {(void *)blk_rows, (void *)blk_chunk, (void *)chunk_cols, (void *)chunk_ncols,
                  (void *)chunk_ent, (void *)qseg, (void *)ent_col, ent_w})
    (void)hipFree(p);
  *this = Tiled{};
}

Status build_tiled(const Csr &m, const RowGrid &g, int max_ent, const ColumnOrder &order,
                   hipStream_t s, Tiled *out) {
  if (g.n1 * g.n2 != m.nrows || g.b1 * g.b2 != kRB || max_ent < kRB)
    return fail(SRT_EDEVICE, "row grid does not match the operator");
  const int64_t nnz = m.nnz, nrows = m.nrows;
  const int64_t nblk = ((g.n1 + g.b1 - 1) / g.b1) * ((g.n2 + g.b2 - 1) / g.b2);
  const int t = 256;
  Tiled &T = *out;
  T.nblk = nblk;
  T.wdtype = m.wdtype;
  T.scale = m.scale;
  T.ncols = m.ncols;
  auto oom = [] { return fail(SRT_ENOMEM, "device allocation for the tiled operator failed"); };
  if (nnz >= INT32_MAX / 2) return fail(SRT_ENOTSUP, "operator too large for the tiled format");
  if (hipMalloc(&T.blk_rows, sizeof(int32_t) * (nblk > 0 ? nblk * kRB : 1)) != hipSuccess ||
      hipMalloc(&T.blk_chunk, sizeof(int32_t) * (nblk + 1)) != hipSuccess)
    return oom();
  if (nblk > 0) SRT_HIP(hipMemsetAsync(T.blk_rows, 0xff, sizeof(int32_t) * nblk * kRB, s));

  // 1. entries in (block, column) order, with their slots
  Buf row_of, bc, bc_sorted, idx, idx_sorted, slot_sorted, ukeys, ucount, upos, nu_d, ustart,
      uchunk, ulocal, nch, chunk0;
  if (row_of.alloc(4 * nnz) || bc.alloc(8 * nnz) || bc_sorted.alloc(8 * nnz) || idx.alloc(4 * nnz) ||
      idx_sorted.alloc(4 * nnz) || slot_sorted.alloc(nnz) || ukeys.alloc(8 * nnz) ||
      ucount.alloc(4 * (nnz + 1)) || upos.alloc(8 * (nnz + 1)) || nu_d.alloc(8) ||
      ustart.alloc(8 * (nblk + 1)) || uchunk.alloc(4 * nnz) || ulocal.alloc(4 * nnz) ||
      nch.alloc(8 * (nblk + 1)) || chunk0.alloc(8 * (nblk + 1)))
    return oom();
  if (nrows > 0)
    hipLaunchKernelGGL(k_rows, dim3(nblocks(nrows, t)), dim3(t), 0, s, m.rowptr, nrows, g,
                       T.blk_rows, row_of.as<int32_t>());
  int64_t nu = 0;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_bc_keys, dim3(nblocks(nnz, t)), dim3(t), 0, s, row_of.as<int32_t>(),
                       m.cols, nnz, g, bc.as<uint64_t>(), idx.as<int32_t>());
    const int kbits = 32 + bits_for((uint64_t)nblk);
    size_t b1 = 0, b2 = 0;
    Buf tmp;
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, bc.as<uint64_t>(),
                                               bc_sorted.as<uint64_t>(), idx.as<int32_t>(),
                                               idx_sorted.as<int32_t>(), (int)nnz, 0, kbits, s));
    SRT_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, b2, bc_sorted.as<uint64_t>(),
                                                  ukeys.as<uint64_t>(), ucount.as<int32_t>(),
                                                  nu_d.as<int64_t>(), (int)nnz, s));
    if (tmp.alloc(b1 > b2 ? b1 : b2)) return oom();
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, b1, bc.as<uint64_t>(),
                                               bc_sorted.as<uint64_t>(), idx.as<int32_t>(),
                                               idx_sorted.as<int32_t>(), (int)nnz, 0, kbits, s));
    SRT_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp.p, b2, bc_sorted.as<uint64_t>(),
                                                  ukeys.as<uint64_t>(), ucount.as<int32_t>(),
                                                  nu_d.as<int64_t>(), (int)nnz, s));
    SRT_HIP(hipMemcpyAsync(&nu, nu_d.p, 8, hipMemcpyDeviceToHost, s));
    SRT_HIP(hipStreamSynchronize(s));
    hipLaunchKernelGGL(k_sorted_slots, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                       idx_sorted.as<int32_t>(), row_of.as<int32_t>(), nnz, g,
                       slot_sorted.as<uint8_t>());
    SRT_TRY(scan_to_i64(ucount.as<int32_t>(), upos.as<int64_t>(), nu, s, oom));
  }
  // 2. chunks, cut along each block's columns in the requested order
  hipLaunchKernelGGL(k_ustart, dim3(nblocks(nblk + 1, t)), dim3(t), 0, s, ukeys.as<uint64_t>(), nu,
                     nblk, ustart.as<int64_t>());
  Buf okeys, okeys_sorted, oidx, uorder;
  if (order.kind != 0 && nu > 0) {
    if (okeys.alloc(8 * nu) || okeys_sorted.alloc(8 * nu) || oidx.alloc(4 * nu) ||
        uorder.alloc(4 * nu))
      return oom();
    hipLaunchKernelGGL(k_polar_keys, dim3(nblocks(nu, t)), dim3(t), 0, s, ukeys.as<uint64_t>(), nu,
                       g, order, okeys.as<uint64_t>(), oidx.as<int32_t>());
    // stable: columns at equal angles keep their index order
    const int kbits = 32 + bits_for((uint64_t)nblk);
    size_t b = 0;
    Buf tmpo;
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, okeys.as<uint64_t>(),
                                               okeys_sorted.as<uint64_t>(), oidx.as<int32_t>(),
                                               uorder.as<int32_t>(), (int)nu, 0, kbits, s));
    if (tmpo.alloc(b)) return oom();
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(tmpo.p, b, okeys.as<uint64_t>(),
                                               okeys_sorted.as<uint64_t>(), oidx.as<int32_t>(),
                                               uorder.as<int32_t>(), (int)nu, 0, kbits, s));
  }
  hipLaunchKernelGGL(k_chunking, dim3((unsigned)(nblk + 1)), dim3(kChunkThreads), 0, s,
                     ustart.as<int64_t>(), ucount.as<int32_t>(), upos.as<int64_t>(),
                     slot_sorted.as<uint8_t>(), order.kind != 0 ? uorder.as<int32_t>() : nullptr,
                     nblk, max_ent, uchunk.as<int32_t>(), ulocal.as<int32_t>(), nch.as<int64_t>());
  SRT_TRY(scan_to_i64(nch.as<int64_t>(), chunk0.as<int64_t>(), nblk + 1, s, oom));
  int64_t nchunk = 0;
  SRT_HIP(hipMemcpyAsync(&nchunk, chunk0.as<int64_t>() + nblk, 8, hipMemcpyDeviceToHost, s));
  SRT_HIP(hipStreamSynchronize(s));
  if (nchunk * (kNQ + 1) >= INT32_MAX || nchunk * kC >= INT32_MAX || nchunk * kRB >= INT32_MAX)
    return fail(SRT_ENOTSUP, "too many operator chunks");
  T.nchunk = nchunk;
  if (hipMalloc(&T.chunk_cols, sizeof(int32_t) * (nchunk > 0 ? nchunk * kC : 1)) != hipSuccess ||
      hipMalloc(&T.chunk_ncols, sizeof(int32_t) * (nchunk > 0 ? nchunk : 1)) != hipSuccess ||
      hipMalloc(&T.chunk_ent, sizeof(int32_t) * (nchunk + 1)) != hipSuccess ||
      hipMalloc(&T.qseg, sizeof(int32_t) * (nchunk > 0 ? nchunk * (kNQ + 1) : 1)) != hipSuccess)
    return oom();
  if (nchunk > 0) {
    SRT_HIP(hipMemsetAsync(T.chunk_cols, 0, sizeof(int32_t) * nchunk * kC, s));
    SRT_HIP(hipMemsetAsync(T.chunk_ncols, 0, sizeof(int32_t) * nchunk, s));
  }
  hipLaunchKernelGGL(k_blk_chunk, dim3(nblocks(nblk + 1, t)), dim3(t), 0, s, chunk0.as<int64_t>(),
                     nblk, T.blk_chunk);
  if (nu > 0)
    hipLaunchKernelGGL(k_chunk_cols, dim3(nblocks(nu, t)), dim3(t), 0, s, ukeys.as<uint64_t>(), nu,
                       chunk0.as<int64_t>(), uchunk.as<int32_t>(), ulocal.as<int32_t>(),
                       T.chunk_cols, T.chunk_ncols);
  // 3. entries in (chunk, slot) order and their padded quad positions
  const int64_t nseg = nchunk * kRB, nquad = nchunk * kNQ;
  Buf key2, key2s, local, seq, perm2, rawstart, qlen, qstart;
  if (key2.alloc(8 * nnz) || key2s.alloc(8 * nnz) || local.alloc(4 * nnz) || seq.alloc(4 * nnz) ||
      perm2.alloc(4 * nnz) || rawstart.alloc(8 * (nseg + 1)) || qlen.alloc(8 * (nquad + 1)) ||
      qstart.alloc(8 * (nquad + 1)))
    return oom();
  if (nnz > 0) {
    hipLaunchKernelGGL(k_entry_keys, dim3(nblocks(nu, t)), dim3(t), 0, s, ukeys.as<uint64_t>(),
                       ucount.as<int32_t>(), upos.as<int64_t>(), nu, chunk0.as<int64_t>(),
                       uchunk.as<int32_t>(), ulocal.as<int32_t>(), slot_sorted.as<uint8_t>(),
                       key2.as<uint64_t>(), local.as<int32_t>(), seq.as<int32_t>());
    const int kbits = bits_for((uint64_t)nseg + kRB);
    size_t b = 0;
    Buf tmp3;
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, key2.as<uint64_t>(), key2s.as<uint64_t>(),
                                               seq.as<int32_t>(), perm2.as<int32_t>(), (int)nnz, 0,
                                               kbits, s));
    if (tmp3.alloc(b)) return oom();
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp3.p, b, key2.as<uint64_t>(), key2s.as<uint64_t>(),
                                               seq.as<int32_t>(), perm2.as<int32_t>(), (int)nnz, 0,
                                               kbits, s));
  }
  hipLaunchKernelGGL(k_rawstart, dim3(nblocks(nseg + 1, t)), dim3(t), 0, s, key2s.as<uint64_t>(), nnz,
                     nseg, rawstart.as<int64_t>());
  hipLaunchKernelGGL(k_quad_len, dim3(nblocks(nquad + 1, t)), dim3(t), 0, s, rawstart.as<int64_t>(),
                     nquad, qlen.as<int64_t>());
  // 4. quads placed on wavefronts by length (positions), rows and lengths moved with them
  Buf place, cblk, qpos, rows0;
  if (place.alloc(4 * (size_t)nblk * kNQ) || cblk.alloc(4 * (size_t)(nchunk > 0 ? nchunk : 1)) ||
      qpos.alloc(8 * (nquad + 1)) || rows0.alloc(4 * (size_t)nblk * kRB))
    return oom();
  if (nblk > 0) {
    hipLaunchKernelGGL(k_quad_place, dim3((unsigned)nblk), dim3(64), 0, s, chunk0.as<int64_t>(),
                       qlen.as<int64_t>(), place.as<int32_t>());
    hipLaunchKernelGGL(k_chunk_blk, dim3(nblocks(nblk, t)), dim3(t), 0, s, chunk0.as<int64_t>(),
                       nblk, cblk.as<int32_t>());
    SRT_HIP(hipMemcpyAsync(rows0.p, T.blk_rows, 4 * (size_t)nblk * kRB, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_place_rows, dim3(nblocks(nblk * kNQ, t)), dim3(t), 0, s,
                       rows0.as<int32_t>(), place.as<int32_t>(), nblk, T.blk_rows);
  }
  hipLaunchKernelGGL(k_place_qlen, dim3(nblocks(nquad + 1, t)), dim3(t), 0, s, qlen.as<int64_t>(),
                     cblk.as<int32_t>(), place.as<int32_t>(), nquad, qpos.as<int64_t>());
  SRT_TRY(scan_to_i64(qpos.as<int64_t>(), qstart.as<int64_t>(), nquad + 1, s, oom));
  int64_t npad = 0;
  SRT_HIP(hipMemcpyAsync(&npad, qstart.as<int64_t>() + nquad, 8, hipMemcpyDeviceToHost, s));
  SRT_HIP(hipStreamSynchronize(s));
  if (npad >= INT32_MAX) return fail(SRT_ENOTSUP, "too many padded operator entries");
  T.nnz = npad;
  const size_t wsz = dtype_size(m.wdtype);
  // npad is a multiple of kQ (every quad segment is), so a quad step's four
  // packed words form one 16-byte unit
  T.packed = wsz == 2;
  if (T.packed) {
    if (hipMalloc(&T.ent_w, 4 * (size_t)(npad > 0 ? npad : 4)) != hipSuccess) return oom();
    if (npad > 0)
      hipLaunchKernelGGL(k_pad_fill_packed, dim3(nblocks(npad, t)), dim3(t), 0, s, npad,
                         (uint32_t *)T.ent_w);
  } else {
    if (hipMalloc(&T.ent_col, sizeof(int32_t) * (npad > 0 ? npad : 1)) != hipSuccess ||
        hipMalloc(&T.ent_w, wsz * (npad > 0 ? npad : 1)) != hipSuccess)
      return oom();
    if (npad > 0) {
      hipLaunchKernelGGL(k_pad_fill, dim3(nblocks(npad, t)), dim3(t), 0, s, npad, T.ent_col);
      SRT_HIP(hipMemsetAsync(T.ent_w, 0, wsz * npad, s));
    }
  }
  hipLaunchKernelGGL(k_chunk_meta2, dim3(nblocks(nchunk * (kNQ + 1) + 1, t)), dim3(t), 0, s,
                     qstart.as<int64_t>(), nchunk, T.chunk_ent, T.qseg);
  if (nnz > 0) {
    switch (wsz) {
      case 8:
        hipLaunchKernelGGL(k_scatter<uint64_t>, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           key2s.as<uint64_t>(), perm2.as<int32_t>(), nnz, rawstart.as<int64_t>(),
                           qstart.as<int64_t>(), cblk.as<int32_t>(), place.as<int32_t>(),
                           local.as<int32_t>(), idx_sorted.as<int32_t>(),
                           (const uint64_t *)m.vals, T.ent_col, (uint64_t *)T.ent_w);
        break;
      case 4:
        hipLaunchKernelGGL(k_scatter<uint32_t>, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           key2s.as<uint64_t>(), perm2.as<int32_t>(), nnz, rawstart.as<int64_t>(),
                           qstart.as<int64_t>(), cblk.as<int32_t>(), place.as<int32_t>(),
                           local.as<int32_t>(), idx_sorted.as<int32_t>(),
                           (const uint32_t *)m.vals, T.ent_col, (uint32_t *)T.ent_w);
        break;
      default:
        hipLaunchKernelGGL(k_scatter_packed, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           key2s.as<uint64_t>(), perm2.as<int32_t>(), nnz, rawstart.as<int64_t>(),
                           qstart.as<int64_t>(), cblk.as<int32_t>(), place.as<int32_t>(),
                           local.as<int32_t>(), idx_sorted.as<int32_t>(),
                           (const uint16_t *)m.vals, (uint32_t *)T.ent_w);
    }
  }
  SRT_HIP(hipGetLastError());
  SRT_HIP(hipStreamSynchronize(s));
  return Status{};
}

}  // namespace srt
