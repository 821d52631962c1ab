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
// of the block's columns in chunks of at most kC columns and kE entries; per
// chunk it stages, in one batch of coalesced loads, the chunk's dense rows,
// its entries and its per-row offsets into LDS, and every row of the block
// then consumes them from LDS. The rows' accumulators stay in registers across
// chunks, so every output element is written once, in a fixed summation order.
//
// Format (built on the device from the CSR operator):
//   blk_rows[b*kRB + pos]         global row at block position pos (-1: none)
//   blk_chunk[b] .. [b+1]         chunks of block b (consecutive ids)
//   chunk_cols[c*kC + u]          global column of local column u of chunk c
//   chunk_ncols[c]                columns in chunk c
//   chunk_ent[c] .. [c+1]         entries of chunk c, ordered by row position
//   seg[c*(kRB+1) + pos]          first entry of row pos, relative to chunk_ent[c]
//   ent_col[e], ent_w[e]          local column and weight of entry e
#include <hipcub/hipcub.hpp>

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

__device__ __forceinline__ void block_of(const RowGrid &g, int64_t row, int64_t *blk, int *pos) {
  const int64_t i1 = row / g.n2, i2 = row - i1 * g.n2;
  const int64_t nb2 = (g.n2 + g.b2 - 1) / g.b2;
  *blk = (i1 / g.b1) * nb2 + i2 / g.b2;
  *pos = (int)((i1 % g.b1) * g.b2 + i2 % g.b2);
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
  int pos;
  block_of(g, r, &b, &pos);
  blk_rows[b * kRB + pos] = (int32_t)r;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) row_of[e] = (int32_t)r;
}

__global__ void k_bc_keys(const int32_t *__restrict__ row_of, const int32_t *__restrict__ cols,
                          int64_t nnz, RowGrid g, uint64_t *__restrict__ keys) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int64_t b;
  int pos;
  block_of(g, row_of[e], &b, &pos);
  keys[e] = ((uint64_t)b << 32) | (uint32_t)cols[e];
}

// ustart[b]: first distinct (block, col) key of block b, b in [0, nblk].
__global__ void k_ustart(const uint64_t *__restrict__ ukeys, int64_t nu, int64_t nblk,
                         int64_t *__restrict__ ustart) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblk) return;
  ustart[b] = lower_bound_u64(ukeys, nu, (uint64_t)b << 32);
}

// Greedy cut of each block's distinct columns (ascending) into chunks of at
// most kC columns and kE entries. One thread per block.
__global__ void k_chunking(const int64_t *__restrict__ ustart, const int32_t *__restrict__ ucount,
                           int64_t nblk, int32_t *__restrict__ uchunk, int32_t *__restrict__ ulocal,
                           int64_t *__restrict__ nch) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nblk) return;
  if (b == nblk) {
    nch[b] = 0;
    return;
  }
  int32_t chunk = 0, ncol = 0, nent = 0;
  for (int64_t j = ustart[b]; j < ustart[b + 1]; ++j) {
    if (ncol == kC || nent + ucount[j] > kE) {
      ++chunk;
      ncol = 0;
      nent = 0;
    }
    uchunk[j] = chunk;
    ulocal[j] = ncol++;
    nent += ucount[j];
  }
  nch[b] = ustart[b + 1] > ustart[b] ? chunk + 1 : 0;
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

__global__ void k_entry_keys(const int32_t *__restrict__ row_of, const uint64_t *__restrict__ bc,
                             int64_t nnz, RowGrid g, const uint64_t *__restrict__ ukeys,
                             const int64_t *__restrict__ ustart, const int64_t *__restrict__ chunk0,
                             const int32_t *__restrict__ uchunk, const int32_t *__restrict__ ulocal,
                             uint64_t *__restrict__ key2, int32_t *__restrict__ local,
                             int32_t *__restrict__ idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int64_t b;
  int pos;
  block_of(g, row_of[e], &b, &pos);
  const int64_t j = ustart[b] + lower_bound_u64(ukeys + ustart[b], ustart[b + 1] - ustart[b], bc[e]);
  const int64_t c = chunk0[b] + uchunk[j];
  local[e] = ulocal[j];
  key2[e] = (uint64_t)c * kRB + (uint64_t)pos;
  idx[e] = (int32_t)e;
}

template <typename W>
__global__ void k_gather(const int32_t *__restrict__ perm, int64_t nnz,
                         const int32_t *__restrict__ local, const W *__restrict__ vals,
                         int32_t *__restrict__ ent_col, W *__restrict__ ent_w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t e = perm[i];
  ent_col[i] = local[e];
  ent_w[i] = vals[e];
}

__global__ void k_chunk_ent(const uint64_t *__restrict__ key2s, int64_t nnz, int64_t nchunk,
                            int32_t *__restrict__ chunk_ent) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > nchunk) return;
  chunk_ent[c] = (int32_t)lower_bound_u64(key2s, nnz, (uint64_t)c * kRB);
}

__global__ void k_seg(const uint64_t *__restrict__ key2s, int64_t nnz, int64_t nchunk,
                      const int32_t *__restrict__ chunk_ent, int32_t *__restrict__ seg) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nchunk * (kRB + 1)) return;
  const int64_t c = t / (kRB + 1), p = t % (kRB + 1);
  seg[t] = (int32_t)(lower_bound_u64(key2s, nnz, (uint64_t)c * kRB + (uint64_t)p) - chunk_ent[c]);
}

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

template <typename F>
Status scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, F oom) {
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
                            (size_t)nchunk * (kRB + 1) + (size_t)nnz) +
         dtype_size(wdtype) * (size_t)nnz;
}

void Tiled::release() {
  for (void *p : {(void *)blk_rows, (void *)blk_chunk, (void *)chunk_cols, (void *)chunk_ncols,
                  (void *)chunk_ent, (void *)seg, (void *)ent_col, ent_w})
    (void)hipFree(p);
  *this = Tiled{};
}

Status build_tiled(const Csr &m, const RowGrid &g, hipStream_t s, Tiled *out) {
  if (g.n1 * g.n2 != m.nrows || g.b1 * g.b2 != kRB)
    return fail(SRT_EDEVICE, "row grid does not match the operator");
  const int64_t nnz = m.nnz, nrows = m.nrows;
  const int64_t nblk = ((g.n1 + g.b1 - 1) / g.b1) * ((g.n2 + g.b2 - 1) / g.b2);
  const int t = 256;
  Tiled &T = *out;
  T.nblk = nblk;
  T.nnz = nnz;
  T.wdtype = m.wdtype;
  T.scale = m.scale;
  T.ncols = m.ncols;
  auto oom = [] { return fail(SRT_ENOMEM, "device allocation for the tiled operator failed"); };
  if (hipMalloc(&T.blk_rows, sizeof(int32_t) * (nblk > 0 ? nblk * kRB : 1)) != hipSuccess ||
      hipMalloc(&T.blk_chunk, sizeof(int32_t) * (nblk + 1)) != hipSuccess)
    return oom();
  if (nblk > 0) SRT_HIP(hipMemsetAsync(T.blk_rows, 0xff, sizeof(int32_t) * nblk * kRB, s));

  Buf row_of, bc, bc_sorted, ukeys, ucount, nu_d, ustart, uchunk, ulocal, nch, chunk0;
  if (row_of.alloc(4 * nnz) || bc.alloc(8 * nnz) || bc_sorted.alloc(8 * nnz) ||
      ukeys.alloc(8 * nnz) || ucount.alloc(4 * nnz) || nu_d.alloc(8) ||
      ustart.alloc(8 * (nblk + 1)) || uchunk.alloc(4 * nnz) || ulocal.alloc(4 * nnz) ||
      nch.alloc(8 * (nblk + 1)) || chunk0.alloc(8 * (nblk + 1)))
    return oom();
  if (nrows > 0)
    hipLaunchKernelGGL(k_rows, dim3(nblocks(nrows, t)), dim3(t), 0, s, m.rowptr, nrows, g,
                       T.blk_rows, row_of.as<int32_t>());
  int64_t nu = 0;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_bc_keys, dim3(nblocks(nnz, t)), dim3(t), 0, s, row_of.as<int32_t>(),
                       m.cols, nnz, g, bc.as<uint64_t>());
    const int kbits = 32 + bits_for((uint64_t)nblk);
    size_t b1 = 0, b2 = 0;
    Buf tmp;
    SRT_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, b1, bc.as<uint64_t>(),
                                              bc_sorted.as<uint64_t>(), (int)nnz, 0, kbits, s));
    SRT_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, b2, bc_sorted.as<uint64_t>(),
                                                  ukeys.as<uint64_t>(), ucount.as<int32_t>(),
                                                  nu_d.as<int64_t>(), (int)nnz, s));
    if (tmp.alloc(b1 > b2 ? b1 : b2)) return oom();
    SRT_HIP(hipcub::DeviceRadixSort::SortKeys(tmp.p, b1, bc.as<uint64_t>(),
                                              bc_sorted.as<uint64_t>(), (int)nnz, 0, kbits, s));
    SRT_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp.p, b2, bc_sorted.as<uint64_t>(),
                                                  ukeys.as<uint64_t>(), ucount.as<int32_t>(),
                                                  nu_d.as<int64_t>(), (int)nnz, s));
    SRT_HIP(hipMemcpyAsync(&nu, nu_d.p, 8, hipMemcpyDeviceToHost, s));
    SRT_HIP(hipStreamSynchronize(s));
  }
  hipLaunchKernelGGL(k_ustart, dim3(nblocks(nblk + 1, t)), dim3(t), 0, s, ukeys.as<uint64_t>(), nu,
                     nblk, ustart.as<int64_t>());
  hipLaunchKernelGGL(k_chunking, dim3(nblocks(nblk + 1, 64)), dim3(64), 0, s, ustart.as<int64_t>(),
                     ucount.as<int32_t>(), nblk, uchunk.as<int32_t>(), ulocal.as<int32_t>(),
                     nch.as<int64_t>());
  SRT_TRY(scan_i64(nch.as<int64_t>(), chunk0.as<int64_t>(), nblk + 1, s, oom));
  int64_t nchunk = 0;
  SRT_HIP(hipMemcpyAsync(&nchunk, chunk0.as<int64_t>() + nblk, 8, hipMemcpyDeviceToHost, s));
  SRT_HIP(hipStreamSynchronize(s));
  if (nchunk * (kRB + 1) >= INT32_MAX || nchunk * kC >= INT32_MAX)
    return fail(SRT_ENOTSUP, "too many operator chunks");
  T.nchunk = nchunk;
  if (hipMalloc(&T.chunk_cols, sizeof(int32_t) * (nchunk > 0 ? nchunk * kC : 1)) != hipSuccess ||
      hipMalloc(&T.chunk_ncols, sizeof(int32_t) * (nchunk > 0 ? nchunk : 1)) != hipSuccess ||
      hipMalloc(&T.chunk_ent, sizeof(int32_t) * (nchunk + 1)) != hipSuccess ||
      hipMalloc(&T.seg, sizeof(int32_t) * (nchunk > 0 ? nchunk * (kRB + 1) : 1)) != hipSuccess ||
      hipMalloc(&T.ent_col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess ||
      hipMalloc(&T.ent_w, dtype_size(m.wdtype) * (nnz > 0 ? nnz : 1)) != hipSuccess)
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
  Buf key2, key2s, local, idx, perm;
  if (nnz > 0) {
    if (key2.alloc(8 * nnz) || key2s.alloc(8 * nnz) || local.alloc(4 * nnz) || idx.alloc(4 * nnz) ||
        perm.alloc(4 * nnz))
      return oom();
    hipLaunchKernelGGL(k_entry_keys, dim3(nblocks(nnz, t)), dim3(t), 0, s, row_of.as<int32_t>(),
                       bc.as<uint64_t>(), nnz, g, ukeys.as<uint64_t>(), ustart.as<int64_t>(),
                       chunk0.as<int64_t>(), uchunk.as<int32_t>(), ulocal.as<int32_t>(),
                       key2.as<uint64_t>(), local.as<int32_t>(), idx.as<int32_t>());
    const int kbits = bits_for((uint64_t)nchunk * kRB + kRB);
    size_t b = 0;
    Buf tmp3;
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b, key2.as<uint64_t>(), key2s.as<uint64_t>(),
                                               idx.as<int32_t>(), perm.as<int32_t>(), (int)nnz, 0,
                                               kbits, s));
    if (tmp3.alloc(b)) return oom();
    SRT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp3.p, b, key2.as<uint64_t>(), key2s.as<uint64_t>(),
                                               idx.as<int32_t>(), perm.as<int32_t>(), (int)nnz, 0,
                                               kbits, s));
    switch (dtype_size(m.wdtype)) {
      case 8:
        hipLaunchKernelGGL(k_gather<uint64_t>, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           perm.as<int32_t>(), nnz, local.as<int32_t>(), (const uint64_t *)m.vals,
                           T.ent_col, (uint64_t *)T.ent_w);
        break;
      case 4:
        hipLaunchKernelGGL(k_gather<uint32_t>, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           perm.as<int32_t>(), nnz, local.as<int32_t>(), (const uint32_t *)m.vals,
                           T.ent_col, (uint32_t *)T.ent_w);
        break;
      default:
        hipLaunchKernelGGL(k_gather<uint16_t>, dim3(nblocks(nnz, t)), dim3(t), 0, s,
                           perm.as<int32_t>(), nnz, local.as<int32_t>(), (const uint16_t *)m.vals,
                           T.ent_col, (uint16_t *)T.ent_w);
    }
  }
  hipLaunchKernelGGL(k_chunk_ent, dim3(nblocks(nchunk + 1, t)), dim3(t), 0, s, key2s.as<uint64_t>(),
                     nnz, nchunk, T.chunk_ent);
  if (nchunk > 0)
    hipLaunchKernelGGL(k_seg, dim3(nblocks(nchunk * (kRB + 1), t)), dim3(t), 0, s,
                       key2s.as<uint64_t>(), nnz, nchunk, T.chunk_ent, T.seg);
  SRT_HIP(hipGetLastError());
  SRT_HIP(hipStreamSynchronize(s));
  return Status{};
}

}  // namespace srt
