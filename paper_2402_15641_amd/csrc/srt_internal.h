// Internal declarations shared by the translation units of libsrt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "srt.h"

namespace srt {

// Thread-local error text behind srt_last_error().
void set_error(const std::string &msg);

// A status plus message; `ok()` when status == SRT_OK.
struct Status {
  srt_status code = SRT_OK;
  bool ok() const { return code == SRT_OK; }
};

Status fail(srt_status code, const std::string &msg);
Status hip_fail(hipError_t e, const char *what);

#define SRT_HIP(call)                                     \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::srt::hip_fail(e_, #call); \
  } while (0)

#define SRT_TRY(expr)                 \
  do {                                \
    ::srt::Status s_ = (expr);        \
    if (!s_.ok()) return s_;          \
  } while (0)

// One sparse operator in CSR form on the device. Column indices ascend in
// every row; values are arc lengths times `scale`, stored in `wdtype`.
struct Csr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int32_t *rowptr = nullptr;  // nrows + 1
  int32_t *cols = nullptr;    // nnz
  void *vals = nullptr;       // nnz elements of wdtype
  srt_dtype wdtype = SRT_F32;
  double scale = 1.0;         // stored = arc length * scale (power of two)
  size_t bytes() const;
  void release();
};

// Geometry as the device sees it (device arrays owned by the plan).
struct Geometry {
  int32_t ms = 0, mz = 0;
  double x0 = 0, z0 = 0, dxy = 0, dz = 0;
  int32_t na = 0, nh = 0, nl = 0;
  const double *cx = nullptr;      // device [na] column centre x
  const double *cy = nullptr;      // device [na] column centre y
  const double *zpos = nullptr;    // device [nh]
  const double *radii = nullptr;   // device [nl] sphere radii (stage-2 half circles)
  const double *rho = nullptr;     // device [nr] radial grid of the stage-2 image
  int32_t nr = 0;                  // (stage-1 circle radii); may alias radii
  int32_t basis = SRT_BASIS_CONSTANT;  // voxel basis the weights integrate
};

// Raw COO pieces of an operator: one entry per arc piece (duplicates allowed),
// key = row * ncols + col.
struct Coo {
  int64_t n = 0;
  uint64_t *keys = nullptr;
  double *vals = nullptr;
};

// Geometry kernels (geometry.hip). `live` bounds the rho cells kept in A34.
Status a12_pieces(const Geometry &g, hipStream_t s, Coo *out);
Status a34_pieces(const Geometry &g, int32_t live, hipStream_t s, Coo *out);

// Sparse build (sparse_build.hip): sort pieces by (row, col), merge duplicates,
// form CSR of the operator and of its transpose, round weights.
Status build_csr_pair(Coo *pieces, int64_t nrows, int64_t ncols, srt_dtype wdtype,
                      hipStream_t s, Csr *op, Csr *op_t);
// Finds L = 1 + the largest radius index any column's circle reaches (0 if
// none) from the A12 pieces and renumbers their rows a * nl + l as a * L + l.
Status compact_a12(Coo *pieces, int32_t nl, int64_t npix, hipStream_t s, int32_t *live);

// ---- row-blocked operator format (tiled.hip)
// Workgroup shape of the stage kernels. Two shapes were measured at 256^3:
// 8 wavefronts per workgroup (128 rows, 64 staged columns per chunk, two
// workgroups per CU) ran the forward stages 5-10% faster than 16 wavefronts
// (256 rows, 128 columns, one workgroup per CU) and the pair 2% faster: a
// second workgroup keeps a CU busy while the first waits at a chunk barrier,
// at the price of less reuse of each staged column.
#ifndef SRT_WG_WAVES
#define SRT_WG_WAVES 8
#endif
#if SRT_WG_WAVES == 16
constexpr int kRB = 256;   // rows per block (one workgroup)
constexpr int kC = 128;    // columns staged in LDS per chunk
constexpr int kE32 = 1920; // padded entries staged in LDS per chunk (FP32 values)
constexpr int kE64 = 960;  // padded entries staged in LDS per chunk (FP64 values)
#else
constexpr int kRB = 128;
constexpr int kC = 64;
constexpr int kE32 = 940;  // two workgroups' double buffers fit one CU's LDS
constexpr int kE64 = 468;
#endif
constexpr int kQ = 4;      // rows per quad: a lane group runs a quad in lockstep
// whole quads per chunk, so that every step's four entries start on a
// 16-byte boundary in LDS (the read one step past a segment's end included)
static_assert(kE32 % kQ == 0 && kE64 % kQ == 0, "entries per chunk come in whole quads");
constexpr int kNQ = kRB / kQ;  // quads per block
// Quads per wavefront in the stage kernels: quad position p runs on lane group
// p % kQuadsPerWave of wavefront p / kQuadsPerWave.
constexpr int kQuadsPerWave = 4;
// One staged dense row in LDS: 32 pieces of 16 bytes (128 FP32 or 64 FP64
// values of the row's slice).
constexpr int kStagedRowBytes = 512;
// Packed 16-bit entries are one 32-bit word each: the weight's bits in the
// high half and, in the low half, the LDS byte offset of the entry's staged
// dense row (local column u at u * kStagedRowBytes) shifted right by
// kPackShift, so that the offset of the all-zero row kC fits 16 bits.
constexpr int kPackShift = (kC + 1) * kStagedRowBytes <= 65536 ? 0 : 5;
static_assert(((kC + 1) * kStagedRowBytes >> kPackShift) <= 65536, "row offsets fit 16 bits");
constexpr int kNW = SRT_WG_WAVES;  // wavefronts per workgroup

// The operator's rows viewed as an n1 x n2 grid (row = i1 * n2 + i2), cut
// into b1 x b2 blocks (b1 * b2 == kRB; edge blocks are partly empty). Within
// a block, rows are numbered into the kernel's processing slots; a lane group
// runs kQ consecutive slots in lockstep and a wavefront 4 * kQ, so
// consecutive slots should be rows with the same amount of work per chunk. along_i1 numbers slots along i1
// first (slot = r2 * b1 + r1), otherwise along i2 (slot = r1 * b2 + r2).
//
// Blocks are numbered in tiles of `tile` groups along i1: inside a tile the
// i1 group steps fastest, then the i2 group, then the tile (tile 1: row-major
// over (i1 group, i2 group)). The apply kernels deal consecutive block numbers
// to the same XCD, so this picks which neighbouring blocks run side by side
// and share staged dense rows through that XCD's L2.
struct RowGrid {
  int64_t n1 = 0, n2 = 0;
  int64_t b1 = 0, b2 = 0;
  bool along_i1 = false;  // consecutive block slots step along i1 (else along i2)
  int64_t tile = 1;       // i1 groups per tile of the block numbering
};

// Order in which a block's distinct columns are cut into chunks. In column
// index order (kind 0) a chunk of A12 is a strip of pixel rows and a chunk of
// A34 a strip of rho cells, which the block's arcs cross with very different
// lengths. Sorted by their polar angle about the block's centre, a chunk is a
// narrow sector that every arc of the block crosses with nearly the same
// length, so rows run side by side with little padding, divergence or
// barrier wait (CPU emulation at 256^3: useful issue slots 0.48 -> 0.82 for
// A12, 0.62 -> 0.79 for A34). The centre used is that of the block's
// numbering tile (the mean of its tile's sensor columns or heights), so that
// blocks running side by side walk the same sectors.
struct ColumnOrder {
  int kind = 0;  // 0: column index; 1: A12 about the block's columns; 2: A34 about its heights
  // kind 1: pixel p = j * ms + i at (x0 + (i + 1/2) dxy, x0 + (j + 1/2) dxy);
  // row index i1 = sensor column, at (cx[i1], cy[i1])
  const double *cx = nullptr, *cy = nullptr;
  int32_t ms = 0;
  double x0 = 0, dxy = 0;
  // kind 2: column m * mz + k at (rho[m], z0 + (k + 1/2) dz); row index i1 =
  // sensor height zpos[i1]
  const double *zpos = nullptr, *rho = nullptr;
  int32_t mz = 0;
  double z0 = 0, dz = 0;
};

struct Tiled {
  int64_t nblk = 0, nchunk = 0, nnz = 0, ncols = 0;  // nnz counts padding entries
  int32_t *blk_rows = nullptr;     // [nblk * kRB], -1 where a block has no row
  int32_t *blk_chunk = nullptr;    // [nblk + 1]
  int32_t *chunk_cols = nullptr;   // [nchunk * kC]
  int32_t *chunk_ncols = nullptr;  // [nchunk]
  int32_t *chunk_ent = nullptr;    // [nchunk + 1] first entry of each chunk
  int32_t *qseg = nullptr;         // [nchunk * (kNQ + 1)] quad offsets within the chunk
  int32_t *ent_col = nullptr;      // [nnz] local column (kC = the all-zero padding column)
  void *ent_w = nullptr;           // [nnz] weights in wdtype (0 for padding)
  // With 16-bit weights the entries are packed instead: ent_col is null and
  // ent_w holds one 32-bit word per entry, its weight (as stored) in the high
  // half and its staged row's LDS offset (kPackShift) in the low half.
  bool packed = false;
  srt_dtype wdtype = SRT_F32;
  double scale = 1.0;
  size_t bytes() const;
  void release();
};

// Builds the row-blocked format of a CSR operator (weights copied as stored);
// chunks hold at most kC columns and max_ent entries after padding.
Status build_tiled(const Csr &m, const RowGrid &g, int max_ent, const ColumnOrder &order,
                   hipStream_t s, Tiled *out);

}  // namespace srt

namespace srt {
constexpr int kStages = 5;
// HIP events of one timed apply: ev[i] .. ev[i+1] brackets stage i.
struct StageEvents {
  hipEvent_t ev[kStages + 1];
};
}  // namespace srt

struct srt_plan {
  uint32_t magic = 0;
  int32_t device = 0;
  srt_dtype vdtype = SRT_F32, wdtype = SRT_F32;
  // SRT_OP_STORED: the operators below stay resident. SRT_OP_ONTHEFLY: they
  // are empty between applies; each apply regenerates what it needs from the
  // geometry and releases it again.
  srt_opmode mode = SRT_OP_STORED;
  int64_t nnz12 = 0, nnz34 = 0;      // operator sizes, kept for either mode
  double scale12 = 1.0, scale34 = 1.0;
  size_t op_bytes = 0;               // bytes of all operators when built
  srt::Geometry geo;
  double *d_geom = nullptr;  // angles | zpos | radii
  int32_t live = 0;          // live rho cells
  srt::Csr a12, a12t, a34, a34t;      // CSR operators (export and format source)
  srt::Tiled t12, t12t, t34, t34t;    // row-blocked copies used by the applies
  void *own_ws = nullptr;
  size_t own_ws_bytes = 0;
  bool timing = false;
  std::vector<srt::StageEvents> timed[2];  // [0] forward, [1] adjoint
};

namespace srt {
constexpr uint32_t kPlanMagic = 0x53525431u;  // "SRT1"
// Row-blocked operators build_operators makes (the CSR pair of each operator
// is always built): bit per apply direction's needs.
constexpr unsigned kTileA12 = 1, kTileA12t = 2, kTileA34 = 4, kTileA34t = 8;
constexpr unsigned kForwardTiles = kTileA12 | kTileA34, kAdjointTiles = kTileA12t | kTileA34t;
constexpr unsigned kAllTiles = kForwardTiles | kAdjointTiles;
// Builds the plan's operators from its geometry on stream s (FP64 geometry,
// CSR pairs, the requested row-blocked copies) and sets `live`; on failure
// everything built is released.
Status build_operators(srt_plan *p, hipStream_t s, unsigned tiles);
void release_operators(srt_plan *p);
size_t operator_bytes(const srt_plan *p);
size_t workspace_bytes(const srt_plan *p, int32_t batch);
// One forward (Alg. 1) or adjoint (Alg. 2) apply of `batch` items on stream s
// (what srt_forward / srt_adjoint run; arguments validated there as well).
// With `stage2` the data side (the forward's output, the adjoint's input) is
// in stage 2's layout [h][l][b][a] instead of [b][a][h][l]: angles fastest,
// the batch items interleaved in runs of n_angles.
Status apply_plan(srt_plan *p, const void *in, void *out, int32_t batch, void *ws,
                  size_t ws_bytes, hipStream_t s, bool adjoint, bool stage2 = false);

// Data [b][a][h][l] laid out as stage 2's [h][l][b][a] (`out` holds as many
// elements), on stream s.
Status data_to_stage2(srt_plan *p, const void *data, void *out, int32_t batch, hipStream_t s);

// Makes `dev` the current device for the scope's lifetime.
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
size_t dtype_size(srt_dtype t);
void clear_timing(srt_plan *p);
}  // namespace srt
