// Forward (Alg. 1) and matched adjoint (Alg. 2) applies.
//
// Both CRT stages are sparse-times-dense products in which the sparse weight
// does not depend on the dense index: A12_a is shared by every z-slice and
// batch item, A34 by every column angle and batch item (Sec. 2: sensors of a
// column share the first transform; all columns share the second). The dense
// index therefore runs across the lanes of a lane group: a nonzero's column
// and weight are the same for all of the group's lanes, and every nonzero
// costs one contiguous read of a staged dense row plus one FMA per lane and
// dense value. Rows of the operator are grouped into blocks whose dense rows
// are staged once in LDS for all of the block's rows (see tiled.hip).
//
// Layouts between the stages (row index first, dense index last):
//   Ft [p][b][k]          pixel-major volume      (Alg. 1 reshape to M_s^2 x M_z)
//   G  [a][l'][b][k]      stage-1 output           (rows a*L + l')
//   Gt [l'][k][b][a]      stage-2 input            (rows l'*mz + k, angles fastest)
//   Yt [h][l][b][a]       stage-2 output           (rows h*nl + l)
//   data [b][a][h][l]     caller layout
// L = live rho cells (circles of larger radius miss the grid).
#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>

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

// Tile geometry shared by the kernel and its launcher. A wavefront is
// GROUPS lane groups of LPG lanes; a group works on one quad of rows at a
// time and its lanes split the dense slice: lane li holds NV vectors of VS
// values, vector m at slice offset (m * LPG + li) * VS. One vector load of a
// group therefore covers LPG * 16 = 256 contiguous bytes, i.e. every LDS bank
// once.
template <typename T> struct TileShape {
  static constexpr int VS = 16 / sizeof(T);      // values per 16-byte vector
  static constexpr int LPG = 16;                 // lanes per group
  static constexpr int GROUPS = 64 / LPG;        // groups per wavefront
  static constexpr int NV = 2;                   // vectors per lane
  static constexpr int DW = LPG * NV * VS;       // dense values per slice
  static constexpr int PIECES = DW / VS;         // 16-byte pieces per staged dense row
  static_assert(kNW * GROUPS == kNQ, "one quad per lane group");
  static_assert(GROUPS == kQuadsPerWave, "quad positions follow the builder's placement");
  static_assert(PIECES == 32, "a staged dense row is half a wavefront of 16-byte pieces");
  static constexpr int NT = kNW * 64;            // threads per workgroup
  static constexpr int E = sizeof(T) == 4 ? kE32 : kE64;  // entries per chunk
  static constexpr int PAIRS_PER_WAVE = kC / 2 / kNW;     // dense row pairs a wave stages
  static_assert(kC % (2 * kNW) == 0, "dense rows split evenly over the wavefronts");
};

// The hardware deals workgroups round-robin to the 8 XCDs (id % 8), each
// with its own L2. Renumbering so that XCD x gets a contiguous range of the
// (slice-major) work order makes the blocks that run side by side on one XCD
// neighbours in the operator, which share dense rows through that L2.
constexpr int kXcds = 8;
// Each XCD takes K consecutive work items, then jumps ahead by 8K, so that all
// XCDs work on nearby blocks at once (ids past the last whole group of 8K keep
// their hardware order).
__device__ __forceinline__ int xcd_chunked(int id, int n, int K) {
  const int G = kXcds * K, full = n / G * G;
  if (id >= full) return id;
  const int x = id % kXcds, k = id / kXcds;
  return (k / K) * G + x * K + (k % K);
}
__device__ __forceinline__ int xcd_local(int id, int n) {
  const int x = id % kXcds, k = id / kXcds;
  const int q = n / kXcds, r = n % kXcds;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

// Asynchronous copies straight from global memory into LDS, 16 or 4 bytes
// per lane: lane l writes dst + l * size, where dst is the same for the
// whole wavefront. Lanes that are switched off write nothing. Completion is
// counted like any other vector load (vmcnt).
__device__ __forceinline__ void lds_dma16(const void *src, void *dst) {
  __builtin_amdgcn_global_load_lds((gbl_void_t *)src, (lds_void_t *)dst, 16, 0, 0);
}
__device__ __forceinline__ void lds_dma4(const void *src, void *dst) {
  __builtin_amdgcn_global_load_lds((gbl_void_t *)src, (lds_void_t *)dst, 4, 0, 0);
}

// The same copies through a buffer resource (base, byte size): a 32-bit
// byte offset per lane, and reads past the end return zeros instead of
// touching memory. While global_load_lds copies are in flight the compiler
// waits for every outstanding LDS read at once (lgkmcnt(0)); with buffer
// copies in flight it keeps waiting for the LDS reads one by one, which is
// what lets the consume loop overlap its reads with its FMAs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}
// The 16-byte buffer copy is written as one asm block rather than through
// the LDS-copy builtin. For the builtin the compiler cannot tell that the
// copies into the next chunk's buffer never alias the reads of the current
// one, and it holds the first step of every chunk until all of this
// wavefront's copies have landed (vmcnt). Hidden from it, a copy is awaited
// only where the kernel says so: wait_vmem before the barrier that publishes
// the buffer. The "memory" clobber keeps memory accesses on their side of the
// copy. The block sets M0 (the LDS destination, the same for the whole
// wavefront) for the copy and restores it; the copy has no register outputs.
__device__ __forceinline__ void buf_dma16(__amdgpu_buffer_rsrc_t r, uint32_t off, void *dst) {
  const uint32_t lds = (uint32_t)(uintptr_t)(lds_void_t *)dst;
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %3\n\t"
      "s_nop 0\n\t"
      "buffer_load_dwordx4 %1, %2, 0 offen lds\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(off), "s"(r), "s"(lds)
      : "memory");
}

// Waits until every vector memory operation of this wavefront (loads and
// LDS copies) has completed: vmcnt(0), other counters untouched.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Four consecutive weights from LDS (stored format) as accumulation type.
template <typename T, typename WT> struct Quad4;
template <> struct Quad4<float, float> {
  static __device__ __forceinline__ void load(const uint32_t *raw, int e, float w[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(raw + e);
    w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
  }
};
// A packed 16-bit entry (one 32-bit word): the weight's bits in the high
// half, the LDS offset of its staged dense row in the low half (shifted by
// kPackShift). Each costs one instruction to take apart: a mask (or a
// conversion) for the weight, a mask-and-or for this lane's address.
template <typename WT> __device__ __forceinline__ float packed_weight(uint32_t word);
template <> __device__ __forceinline__ float packed_weight<uint16_t>(uint32_t w) {  // bfloat16
  return __uint_as_float(w & 0xffff0000u);
}
template <> __device__ __forceinline__ float packed_weight<_Float16>(uint32_t w) {
  // converted once per step; left to itself the compiler folds the
  // conversion into every FMA (v_fma_mix_f32), which measured slower
  float f = (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  asm volatile("" : "+v"(f));
  return f;
}
// Byte offset, from the chunk's first staged row, of this lane's first piece
// of the entry's row (row offsets are multiples of 512 bytes, lane_byte < 256).
__device__ __forceinline__ uint32_t packed_offset(uint32_t w, uint32_t lane_byte) {
  return ((w & 0xffffu) << kPackShift) | lane_byte;
}
template <> struct Quad4<double, double> {
  static __device__ __forceinline__ void load(const uint32_t *raw, int e, double w[4]) {
    const double2 a = *reinterpret_cast<const double2 *>(raw + 2 * e);
    const double2 b = *reinterpret_cast<const double2 *>(raw + 2 * e + 4);
    w[0] = a.x; w[1] = a.y; w[2] = b.x; w[3] = b.y;
  }
};

// One chunk's worth of LDS: staged dense rows (row kC stays zero and is what
// padding entries point at) and the entries, in one array per buffer: their
// local columns, then their weights (as stored); 16-bit weights come packed
// with their rows' offsets, one word per entry, and need no column part. The
// column (or packed) part has room for one quad step more than a chunk holds,
// so the read of the step after a segment's last stays inside the buffer
// (its values are not used). The quads' entry offsets and first entries
// travel in registers.
template <typename T, typename WT> struct ChunkLds {
  using V16 = typename Vec16<T>::type;
  static constexpr bool PACKED = sizeof(WT) == 2;
  static constexpr int E = TileShape<T>::E;
  static constexpr int CWORDS = E + kQ;
  static constexpr int WWORDS = PACKED ? 0 : E * (int)sizeof(WT) / 4;
  static constexpr int EWORDS = CWORDS + WWORDS;
  V16 *dense;
  int32_t *col;  // local columns (unpacked layouts)
  uint32_t *w;   // weights (unpacked layouts: after the columns) or packed words
};

// One workgroup (one per CU) = one row block x one slice of the dense index.
//
// Chunks are double-buffered in LDS. While the wavefronts consume chunk c
// from one buffer, chunk c+1 (its dense rows, entries and quad offsets) is
// copied from memory straight into the other buffer by LDS DMA, each
// wavefront issuing its share and waiting for it only at the end of chunk c;
// the column list of chunk c+2 is fetched one step earlier still. The two
// buffers are separate LDS arrays and the chunk loop is unrolled by two, so
// the compiler sees that the copies in flight never alias the buffer being
// read.
//
// A wavefront is GROUPS lane groups (see TileShape); each group runs one
// quad (kQ rows) in lockstep: per step it reads kQ entries (one per quad row,
// padded so the rows advance together), kQ * NV dense vectors and does
// kQ * NV * VS fused multiply-adds per lane. The next step's entries are read
// before this step's products, so their LDS latency overlaps the dense reads.
// A group's offsets into chunk c+1 and its first step's entries are loaded
// from memory into registers while chunk c is consumed (the offsets one chunk
// earlier still), so a chunk starts with its dense reads, not with two
// dependent LDS round trips.
// MODE 1: the dense width D is a multiple of VS and the dense operand spans
// less than 4 GiB, so rows are staged in 16-byte pieces through buffer
// copies. MODE 2: 16-byte pieces through global copies (operand of 4 GiB or
// more). MODE 0: D is not a multiple of VS; rows are staged word by word.
template <typename T, typename WT, int MODE>
__device__ __forceinline__ void tiled_body(const int32_t *__restrict__ blk_rows,
                                           const int32_t *__restrict__ blk_chunk,
                                           const int32_t *__restrict__ chunk_cols,
                                           const int32_t *__restrict__ chunk_ncols,
                                           const int32_t *__restrict__ chunk_ent,
                                           const int32_t *__restrict__ qseg,
                                           const int32_t *__restrict__ ent_col,
                                           const WT *__restrict__ ent_w, const T *__restrict__ X,
                                           T *__restrict__ Y, int nblk, int D, T scale,
                                           int remap, int slice_inner, uint32_t xbytes) {
  constexpr bool VEC = MODE != 0, BUF = MODE == 1, PACKED = ChunkLds<T, WT>::PACKED;
  using S = TileShape<T>;
  using V16 = typename Vec16<T>::type;
  using L = ChunkLds<T, WT>;
  constexpr int VS = S::VS, NV = S::NV, DW = S::DW, PIECES = S::PIECES;
  constexpr int LPG = S::LPG, GROUPS = S::GROUPS, E = S::E, PPW = S::PAIRS_PER_WAVE;
  __shared__ V16 dense0[(kC + 1) * PIECES], dense1[(kC + 1) * PIECES];
  // a step's entries are read with one base address and constant offsets
  __shared__ __align__(16) uint32_t ent0[L::EWORDS], ent1[L::EWORDS];
  const L buf0{dense0, reinterpret_cast<int32_t *>(ent0), PACKED ? ent0 : ent0 + L::CWORDS};
  const L buf1{dense1, reinterpret_cast<int32_t *>(ent1), PACKED ? ent1 : ent1 + L::CWORDS};

  // remap < 0: a contiguous range per XCD; 0: hardware order; K > 0: chunks of K
  const int bid = remap < 0 ? xcd_local(blockIdx.x, gridDim.x)
                  : remap == 0 ? (int)blockIdx.x : xcd_chunked(blockIdx.x, gridDim.x, remap);
  // work order: slices outermost (slice-major), or innermost (a block's
  // slices consecutively, so its entries are re-read from L2)
  const int nsl = (int)gridDim.x / nblk;
  const int blk = slice_inner ? bid / nsl : bid % nblk;
  const int slice = slice_inner ? bid % nsl : bid / nblk;
  const int d0 = slice * DW;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, grp = lane / LPG, li = lane % LPG;
  const uint32_t lane_byte = (uint32_t)li * 16u;  // this lane's first piece of a staged row

  V16 acc[kQ][NV];
#pragma unroll
  for (int j = 0; j < kQ; ++j)
#pragma unroll
    for (int m = 0; m < NV; ++m) acc[j][m] = V16{};
  if (tid < PIECES) {
    dense0[kC * PIECES + tid] = V16{};
    dense1[kC * PIECES + tid] = V16{};
  }

  const int c0 = blk_chunk[blk], c1 = blk_chunk[blk + 1];

  // Dense row staged by this lane's k-th copy: rows come in pairs, one per
  // half wavefront, each half copying the row's PIECES 16-byte pieces.
  const int half = lane >> 5, piece = lane & 31;
  auto load_cols = [&](int c, int32_t *cols) {
#pragma unroll
    for (int k = 0; k < PPW; ++k)
      cols[k] = chunk_cols[(size_t)c * kC + 2 * (wave + kNW * k) + half];
  };
  // Issues this wavefront's share of the copies of chunk c into buffer b.
  auto stage = [&](int c, const L &b, const int32_t *cols) {
    const int n = chunk_ncols[c];
    const int ce0 = chunk_ent[c], ne = chunk_ent[c + 1] - ce0;
    if constexpr (VEC) {
      const int d = d0 + piece * VS;
      if constexpr (BUF) {
        // resource from the slice start to the operand's end
        const auto r = buf_rsrc(X + d0, xbytes - (uint32_t)(d0 * sizeof(T)));
        const uint32_t rowb = (uint32_t)D * sizeof(T);
#pragma unroll
        for (int k = 0; k < PPW; ++k) {
          const int p = wave + kNW * k;
          if (2 * p + half < n && d < D)
            buf_dma16(r, (uint32_t)cols[k] * rowb + piece * 16u, b.dense + 2 * p * PIECES);
        }
      } else {
#pragma unroll
        for (int k = 0; k < PPW; ++k) {
          const int p = wave + kNW * k;
          if (2 * p + half < n && d < D)
            lds_dma16(X + (size_t)cols[k] * D + d, b.dense + 2 * p * PIECES);
        }
      }
    } else {
      // D is not a multiple of VS: copy 4-byte words of each row's slice;
      // a row's slice is 2 * 64 words, one wavefront copy per half.
      constexpr int WPV = 16 / 4;  // words per 16-byte piece
      for (int i = wave; i < 2 * kC; i += kNW) {
        const int u = i >> 1;
        if (u >= n) break;
        const int col = chunk_cols[(size_t)c * kC + u];
        const int word = (i & 1) * 64 + lane;           // word within the row's slice
        const int elem = d0 + word * 4 / (int)sizeof(T);  // first value it holds
        if (elem < D)
          lds_dma4(reinterpret_cast<const uint32_t *>(X + (size_t)col * D + d0) + word,
                   b.dense + u * PIECES + (i & 1) * (64 / WPV));
      }
    }
    // weight words (packed: one word per entry)
    const int nw = PACKED ? ne : ne * (int)sizeof(WT) / 4;
    const uint32_t *wsrc = PACKED ? reinterpret_cast<const uint32_t *>(ent_w) + ce0
                                  : reinterpret_cast<const uint32_t *>(ent_w + ce0);
    if constexpr (BUF) {
      // entry words in 16-byte pieces: a chunk holds whole quads (ne and nw
      // are multiples of 4 words) and starts on a 16-byte boundary
      if constexpr (!PACKED) {
        const auto rc = buf_rsrc(ent_col + ce0, (uint32_t)ne * 4u);
        for (int j = wave; j * 256 < ne; j += kNW) {
          const int i = j * 64 + lane;
          if (4 * i < ne) buf_dma16(rc, (uint32_t)i * 16u, b.col + j * 256);
        }
      }
      const auto rw = buf_rsrc(wsrc, (uint32_t)nw * 4u);
      for (int j = wave; j * 256 < nw; j += kNW) {
        const int i = j * 64 + lane;
        if (4 * i < nw) buf_dma16(rw, (uint32_t)i * 16u, b.w + j * 256);
      }
    } else {
      if constexpr (!PACKED) {
        for (int j = wave; j * 64 < ne; j += kNW) {
          const int i = j * 64 + lane;
          if (i < ne) lds_dma4(ent_col + ce0 + i, b.col + j * 64);
        }
      }
      for (int j = wave; j * 64 < nw; j += kNW) {
        const int i = j * 64 + lane;
        if (i < nw) lds_dma4(wsrc + i, b.w + j * 64);
      }
    }
  };
  // This lane group's quad: its entry range in chunk c and its first step's
  // entries (columns and weights), read from memory, not from LDS.
  const int q = wave * GROUPS + grp;
  struct HeadU {  // unpacked layouts: the first step's columns
    int e0, e1;
    int4 cn;
  };
  struct HeadP {  // packed layout: the first step's words
    int e0, e1;
    uint4 un;
  };
  using Head = std::conditional_t<PACKED, HeadP, HeadU>;
  auto load_range = [&](int c, Head &h) {
    const int32_t *qs = qseg + (size_t)c * (kNQ + 1) + q;
    h.e0 = qs[0];
    h.e1 = qs[1];
  };
  auto load_first = [&](int c, Head &h) {
    // an empty segment reads the chunk's first entries instead (in range)
    const int e = chunk_ent[c] + (h.e0 < h.e1 ? h.e0 : 0);
    if constexpr (PACKED)
      h.un = *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint32_t *>(ent_w) + e);
    else
      h.cn = *reinterpret_cast<const int4 *>(ent_col + e);
  };
  // This lane group's quad over one staged chunk. Per step: this step's
  // weights (unpacked layouts), its kQ * NV dense pieces, then the next
  // step's columns or packed words, whose LDS latency overlaps the products.
  // The column registers are the only values carried from step to step.
  auto fmas = [&](const V16 (&x)[kQ][NV], const T (&ww)[kQ]) {
#pragma unroll
    for (int j = 0; j < kQ; ++j)
#pragma unroll
      for (int m = 0; m < NV; ++m) {
        const T *xs = reinterpret_cast<const T *>(&x[j][m]);
        T *as = reinterpret_cast<T *>(&acc[j][m]);
#pragma unroll
        for (int v = 0; v < VS; ++v) as[v] = fma(ww[j], xs[v], as[v]);
      }
  };
  auto consume = [&](const L &b, const Head &h) {
    const int e0 = h.e0, e1 = h.e1;
    // Keep the loop's own entry reads where they are written (a step ahead):
    // without this the compiler merges them with these first reads into one
    // read at the top of the loop, which stalls every step on it.
    if constexpr (PACKED) {
      uint4 un = h.un;
      asm volatile("" : "+v"(un.x), "+v"(un.y), "+v"(un.z), "+v"(un.w));
      const char *rows = reinterpret_cast<const char *>(b.dense);
      // the loop runs on the entry address alone (one add and one compare a step)
      for (const uint32_t *pe = b.w + e0, *pend = b.w + e1; pe < pend; pe += kQ) {
        const uint32_t wd[kQ] = {un.x, un.y, un.z, un.w};
        T ww[kQ];
        V16 x[kQ][NV];
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
          ww[j] = packed_weight<WT>(wd[j]);
          const uint32_t off = packed_offset(wd[j], lane_byte);
#pragma unroll
          for (int m = 0; m < NV; ++m)
            x[j][m] = *reinterpret_cast<const V16 *>(rows + off + m * LPG * 16);
        }
        un = *reinterpret_cast<const uint4 *>(pe + kQ);
        fmas(x, ww);
      }
    } else {
      int4 cn = h.cn;
      asm volatile("" : "+v"(cn.x), "+v"(cn.y), "+v"(cn.z), "+v"(cn.w));
      for (const int32_t *pc = b.col + e0, *pend = b.col + e1; pc < pend; pc += kQ) {
        T ww[kQ];
        if constexpr (sizeof(WT) == 4)  // the weights sit CWORDS words after their columns
          Quad4<T, WT>::load(reinterpret_cast<const uint32_t *>(pc + L::CWORDS), 0, ww);
        else
          Quad4<T, WT>::load(b.w, (int)(pc - b.col), ww);
        const int cj[kQ] = {cn.x, cn.y, cn.z, cn.w};
        V16 x[kQ][NV];
#pragma unroll
        for (int j = 0; j < kQ; ++j)
#pragma unroll
          for (int m = 0; m < NV; ++m) x[j][m] = b.dense[cj[j] * PIECES + li + m * LPG];
        cn = *reinterpret_cast<const int4 *>(pc + kQ);
        fmas(x, ww);
      }
    }
  };

  if (c0 < c1) {
    int32_t cols_a[PPW], cols_b[PPW];
    Head hc, hn, hnn;  // chunk c, c+1 (range and first entries), c+2 (range)
    if constexpr (VEC) load_cols(c0, cols_a);
    stage(c0, buf0, cols_a);
    if (VEC && c0 + 1 < c1) load_cols(c0 + 1, cols_b);
    load_range(c0, hc);
    if (c0 + 1 < c1) load_range(c0 + 1, hn);
    load_first(c0, hc);
    wait_vmem();
    __syncthreads();
    // one chunk: copy the next into `nxt`, consume `cur`, wait, publish
    auto step = [&](int c, const L &cur, const L &nxt, const int32_t *cols_next,
                    int32_t *cols_after) {
      if (c + 1 < c1) {
        stage(c + 1, nxt, cols_next);
        if (VEC && c + 2 < c1) load_cols(c + 2, cols_after);
        load_first(c + 1, hn);
        if (c + 2 < c1) load_range(c + 2, hnn);
      }
      consume(cur, hc);
      wait_vmem();
      __syncthreads();
      hc = hn;
      hn = hnn;
    };
    for (int c = c0; c < c1; c += 2) {
      step(c, buf0, buf1, cols_b, cols_a);
      if (c + 1 >= c1) break;
      step(c + 1, buf1, buf0, cols_a, cols_b);
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
  template <typename T, typename WT, int MODE>                                                 \
  __global__ __launch_bounds__(kNW * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void NAME(                                           \
      const int32_t *__restrict__ blk_rows, const int32_t *__restrict__ blk_chunk,             \
      const int32_t *__restrict__ chunk_cols, const int32_t *__restrict__ chunk_ncols,         \
      const int32_t *__restrict__ chunk_ent, const int32_t *__restrict__ qseg,                 \
      const int32_t *__restrict__ ent_col, const WT *__restrict__ ent_w,                       \
      const T *__restrict__ X, T *__restrict__ Y, int nblk, int D, T scale, int remap,         \
      int slice_inner, uint32_t xbytes) {                                                      \
    tiled_body<T, WT, MODE>(blk_rows, blk_chunk, chunk_cols, chunk_ncols, chunk_ent, qseg,     \
                            ent_col, ent_w, X, Y, nblk, D, scale, remap, slice_inner, xbytes); \
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

// The same transpose with 16-byte accesses: loads along c, stores along r
// (each a run of 16 lanes covering one 256-byte row segment of the tile).
// Needs R, C, every stride and both base addresses to be whole 16-byte
// vectors. The tile's odd row pitch keeps both phases free of LDS bank
// conflicts (the lanes of one access hit 64 distinct banks).
template <typename T>
__global__ __launch_bounds__(256) void transpose_vec_kernel(const T *__restrict__ in,
                                                            T *__restrict__ out, TDesc t) {
  using V16 = typename Vec16<T>::type;
  constexpr int VS = 16 / sizeof(T);  // values per vector
  constexpr int LPR = 64 / VS;        // lanes per 64-value row segment
  constexpr int RPP = 256 / LPR;      // rows per pass of the workgroup
  __shared__ T tile[64][65];
  const int ctiles = (t.C + 63) / 64;
  const int bx = blockIdx.x;
  const int ct = bx % ctiles;
  const int b = bx / ctiles;
  const int b1 = b / t.n2, b2 = b % t.n2;
  const int r0 = blockIdx.y * 64, c0 = ct * 64;
  const int tid = threadIdx.x, seg = (tid % LPR) * VS, sub = tid / LPR;
  const T *ib = in + b1 * t.ib1 + b2 * t.ib2;
  T *ob = out + b1 * t.ob1 + b2 * t.ob2;
#pragma unroll
  for (int i = 0; i < 64 / RPP; ++i) {
    const int rr = sub + RPP * i, r = r0 + rr, c = c0 + seg;
    if (r < t.R && c < t.C) {  // C is a whole number of vectors: c < C covers c + VS - 1
      const V16 v = *reinterpret_cast<const V16 *>(ib + (int64_t)r * t.irs + c);
      const T *vs = reinterpret_cast<const T *>(&v);
#pragma unroll
      for (int k = 0; k < VS; ++k) tile[rr][seg + k] = vs[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 64 / RPP; ++i) {
    const int cc = sub + RPP * i, c = c0 + cc, r = r0 + seg;
    if (c < t.C && r < t.R) {
      V16 v;
      T *vs = reinterpret_cast<T *>(&v);
#pragma unroll
      for (int k = 0; k < VS; ++k) vs[k] = tile[seg + k][cc];
      *reinterpret_cast<V16 *>(ob + (int64_t)c * t.ocs + r) = v;
    }
  }
}

template <typename T>
Status transpose(const T *in, T *out, const TDesc &t, hipStream_t s) {
  if (t.R <= 0 || t.C <= 0 || t.n1 <= 0 || t.n2 <= 0) return Status{};
  const int64_t gx = (int64_t)t.n1 * t.n2 * ((t.C + 63) / 64);
  const int64_t gy = (t.R + 63) / 64;
  if (gx > INT32_MAX || gy > 65535) return fail(SRT_ENOTSUP, "transpose grid too large");
  constexpr int64_t VS = 16 / sizeof(T);
  const bool vec = t.R % VS == 0 && t.C % VS == 0 && t.irs % VS == 0 && t.ib1 % VS == 0 &&
                   t.ib2 % VS == 0 && t.ocs % VS == 0 && t.ob1 % VS == 0 && t.ob2 % VS == 0 &&
                   reinterpret_cast<uintptr_t>(in) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(transpose_vec_kernel<T>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s,
                       in, out, t);
  else
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
  // Work order, measured at 256^3: a contiguous range per XCD for both
  // forward stages and the stage-1 adjoint; chunks of 16 for the stage-2
  // adjoint (5% faster than round-robin, 7-8% faster than ranges), which also
  // runs a block's slices consecutively (2% faster; 13% slower for stage 1).
  const int remap = st == Stage::s2_adj ? 16 : -1;
  const int slice_inner = st == Stage::s2_adj ? 1 : 0;
  // Buffer copies address the dense operand with 32-bit byte offsets.
  const uint64_t xb = (uint64_t)m.ncols * (uint64_t)D * sizeof(T);
  const int mode = D % TileShape<T>::VS != 0 ? 0 : (xb < (1ull << 32) ? 1 : 2);
  const uint32_t xbytes = mode == 1 ? (uint32_t)xb : 0u;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kNW * 64), 0, s, m.blk_rows, m.blk_chunk,
                       m.chunk_cols, m.chunk_ncols, m.chunk_ent, m.qseg, m.ent_col, w, X, Y,
                       (int)m.nblk, D, scale, remap, slice_inner, xbytes);
  };
#define SRT_GO(K)                                \
  (mode == 1 ? go(K<T, WT, 1>) : mode == 2 ? go(K<T, WT, 2>) : go(K<T, WT, 0>))
  switch (st) {
    case Stage::s1_fwd: SRT_GO(stage1_fwd); break;
    case Stage::s2_fwd: SRT_GO(stage2_fwd); break;
    case Stage::s2_adj: SRT_GO(stage2_adj); break;
    case Stage::s1_adj: SRT_GO(stage1_adj); break;
  }
#undef SRT_GO
  SRT_HIP(hipGetLastError());
  return Status{};
}

// Clears an output with a kernel rather than a memset, so that an apply
// captured into a HIP graph holds kernel nodes only.
template <typename T>
__global__ void k_zero(T *__restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (T)0;
}

template <typename T>
Status zero(T *y, int64_t n, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  if (blocks > 0) hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, y, n);
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

// With `stage2` the data stay in stage 2's layout Yt[h][l][b][a] (angles
// fastest, items interleaved): the forward leaves out its last layout pass and
// the adjoint its first. The solvers keep their data-space vectors that way.
template <typename T, typename WT>
Status forward_impl(srt_plan *p, const T *vol, T *data, int32_t B, T *P, T *Q, hipStream_t s,
                    const Marks &mk, bool stage2) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  SRT_TRY(mk.at(0));
  if (L == 0) {  // no circle meets the grid: the transform is identically zero
    SRT_TRY(zero<T>(data, (int64_t)B * g.na * NR, s));
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
  SRT_TRY((spmm<T, WT>(Stage::s2_fwd, p->t34, P, stage2 ? data : Q, D2, s)));
  SRT_TRY(mk.at(4));
  // Yt[r][b][a] -> data[b][a][r]
  if (!stage2)
    SRT_TRY(transpose<T>(Q, data, TDesc{NR, g.na, B, 1, D2, g.na, 0, NR, (int64_t)g.na * NR, 0}, s));
  SRT_TRY(mk.at(5));
  return Status{};
}

template <typename T, typename WT>
Status adjoint_impl(srt_plan *p, const T *data, T *vol, int32_t B, T *P, T *Q, hipStream_t s,
                    const Marks &mk, bool stage2) {
  const Geometry &g = p->geo;
  const int L = p->live, M2 = g.ms * g.ms, NR = g.nh * g.nl;
  const int D1 = B * g.mz, D2 = B * g.na;
  SRT_TRY(mk.at(0));
  if (L == 0) {
    SRT_TRY(zero<T>(vol, (int64_t)B * g.mz * M2, s));
    for (int i = 1; i <= kStages; ++i) SRT_TRY(mk.at(i));
    return Status{};
  }
  // data[b][a][r] -> Yt[r][b][a]
  if (!stage2)
    SRT_TRY(transpose<T>(data, P, TDesc{g.na, NR, B, 1, NR, (int64_t)g.na * NR, 0, D2, g.na, 0}, s));
  SRT_TRY(mk.at(1));
  // Alg. 2 first product: Gt'[l'][k][b][a] = A34^T Yt
  SRT_TRY((spmm<T, WT>(Stage::s2_adj, p->t34t, stage2 ? data : P, Q, D2, s)));
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

// Checks shared by every apply entry point.
Status check_apply(const srt_plan *p, const void *in, const void *out, int32_t B) {
  if (!p || p->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is NULL or not a live plan");
  if (!in || !out) return fail(SRT_EINVAL, "NULL input or output");
  if (B <= 0) return fail(SRT_EINVAL, "batch must be >= 1");
  // The layout passes read and write the caller's arrays element by element
  // (16 bytes at a time where aligned); the stage kernels copy and store the
  // workspace buffers in 16-byte pieces.
  const size_t esz = dtype_size(p->vdtype);
  if (reinterpret_cast<uintptr_t>(in) % esz != 0 || reinterpret_cast<uintptr_t>(out) % esz != 0)
    return fail(SRT_EINVAL, "input and output must be aligned to their element size");
  const Geometry &g = p->geo;
  if ((int64_t)B * g.mz > INT32_MAX / 4 || (int64_t)B * g.na > INT32_MAX / 4)
    return fail(SRT_ENOTSUP, "batch too large");
  return Status{};
}

// The value/weight type dispatch of one apply over workspace buffers P, Q.
Status run(srt_plan *p, const void *in, void *out, int32_t B, void *P, void *Q, hipStream_t s,
           const Marks &mk, bool adjoint, bool stage2 = false) {
  if (p->vdtype == SRT_F64) {
    using T = double;
    return adjoint ? adjoint_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2)
                   : forward_impl<T, double>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2);
  }
  using T = float;
  switch (p->wdtype) {
    case SRT_BF16:
      return adjoint
                 ? adjoint_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2)
                 : forward_impl<T, uint16_t>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2);
    case SRT_F16:
      return adjoint
                 ? adjoint_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2)
                 : forward_impl<T, _Float16>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2);
    default:
      return adjoint ? adjoint_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2)
                     : forward_impl<T, float>(p, (const T *)in, (T *)out, B, (T *)P, (T *)Q, s, mk, stage2);
  }
}

Status apply(srt_plan *p, const void *in, void *out, int32_t B, void *ws, size_t ws_bytes,
             hipStream_t s, bool adjoint, bool stage2 = false) {
  SRT_TRY(check_apply(p, in, out, B));
  if (ws && reinterpret_cast<uintptr_t>(ws) % 16 != 0)
    return fail(SRT_EINVAL, "workspace must be 16-byte aligned");
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
  if (p->mode != SRT_OP_ONTHEFLY) return run(p, in, out, B, P, Q, s, mk, adjoint, stage2);
  // On the fly: regenerate the two operators this direction applies, apply
  // them, and release them once the stream has finished with them.
  SRT_TRY(build_operators(p, s, adjoint ? kAdjointTiles : kForwardTiles));
  Status st = run(p, in, out, B, P, Q, s, mk, adjoint, stage2);
  const hipError_t e = hipStreamSynchronize(s);
  release_operators(p);
  if (!st.ok()) return st;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return Status{};
}

// ---- the allocation-free forward (srt_forward_noalloc)
// Its workspace is this file-scope array: every device the library runs on
// holds one copy of it, at its own address, until the process ends. In host
// code `scratch` names a host-side stand-in, not device memory; the device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is passed to kernels.
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device `dev`, looked up on the
// first call for that device.
Status scratch_address(int dev, void **out) {
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return fail(SRT_ENOTSUP, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!a) return fail(SRT_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    addr[dev] = a;
  }
  *out = addr[dev];
  return Status{};
}

Status forward_noalloc(srt_plan *p, const void *vol, void *data, int32_t B, hipStream_t s) {
  SRT_TRY(check_apply(p, vol, data, B));
  if (p->mode == SRT_OP_ONTHEFLY)
    return fail(SRT_EINVAL, "srt_forward_noalloc: an on-the-fly plan allocates its operators "
                            "in every apply");
  const size_t need = workspace_bytes(p, B);
  if (need > kScratchBytes)
    return fail(SRT_EINVAL, "srt_forward_noalloc: this plan and batch need " + std::to_string(need) +
                                " bytes of workspace, more than its " +
                                std::to_string(kScratchBytes) + "-byte scratch array");
  DeviceScope ds(p->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  void *base = nullptr;
  SRT_TRY(scratch_address(p->device, &base));
  const size_t one = need / 2;  // two equal, 256-byte aligned buffers
  Marks mk;  // no stage timing: recording it would allocate events
  mk.s = s;
  return run(p, vol, data, B, base, (char *)base + one, s, mk, false);
}

}  // namespace

Status apply_plan(srt_plan *p, const void *in, void *out, int32_t batch, void *ws,
                  size_t ws_bytes, hipStream_t s, bool adjoint, bool stage2) {
  return apply(p, in, out, batch, ws, ws_bytes, s, adjoint, stage2);
}

Status data_to_stage2(srt_plan *p, const void *data, void *out, int32_t B, hipStream_t s) {
  SRT_TRY(check_apply(p, data, out, B));
  DeviceScope ds(p->device);
  if (ds.err != hipSuccess) return hip_fail(ds.err, "hipSetDevice");
  const Geometry &g = p->geo;
  const int NR = g.nh * g.nl, D2 = B * g.na;
  const TDesc d{g.na, NR, B, 1, NR, (int64_t)g.na * NR, 0, D2, g.na, 0};
  if (p->vdtype == SRT_F64) return transpose<double>((const double *)data, (double *)out, d, s);
  return transpose<float>((const float *)data, (float *)out, d, s);
}

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

srt_status srt_forward_noalloc(srt_plan *plan, const void *vol, void *data, int32_t batch,
                               void *hip_stream) {
  try {
    return srt::forward_noalloc(plan, vol, data, batch, (hipStream_t)hip_stream).code;
  } catch (...) {
    return srt::fail(SRT_ENOMEM, "host exception in srt_forward_noalloc").code;
  }
}

}  // extern "C"
