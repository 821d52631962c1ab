// Assembly of CSR operators from arc pieces, plus their explicit transposes.
//
// The pieces of one row come from one circle walk; pieces of one cell are
// summed (Sec. 3.1 weights are per-cell arc lengths). Keys row * ncols + col
// are radix-sorted (stable), equal keys are summed in walk order, and the CSR
// row pointers are found by binary search over the sorted keys, so the
// result is deterministic. The transpose used by the matched adjoint
// (Alg. 2) is formed from the same merged FP64 entries, so A and its
// transpose hold bit-identical weights.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

#include "srt_internal.h"

namespace srt {
namespace {

// Round v (>= 0) to the nearest value with `mant` fraction bits and minimum
// normal exponent `emin` (ties to even): one rounding, directly from FP64.
__device__ double round_to_format(double v, int mant, int emin) {
  if (v == 0.0) return 0.0;
  const int e = ilogb(v);
  const double q = ldexp(1.0, (e > emin ? e : emin) - mant);
  return rint(v / q) * q;
}

__global__ void store_weights(const double *__restrict__ in, int64_t n, double scale,
                              int wdtype, void *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = in[i] * scale;
  switch (wdtype) {
    case SRT_F64:
      ((double *)out)[i] = v;
      break;
    case SRT_F32:
      ((float *)out)[i] = (float)v;
      break;
    case SRT_BF16: {
      const float f = (float)round_to_format(v, 7, -126);  // exact in FP32
      ((uint16_t *)out)[i] = (uint16_t)(__float_as_uint(f) >> 16);
      break;
    }
    case SRT_F16: {
      const float f = (float)round_to_format(v, 10, -14);  // exact in FP16
      ((_Float16 *)out)[i] = (_Float16)f;
      break;
    }
  }
}

__global__ void split_keys(const uint64_t *__restrict__ keys, int64_t n, uint64_t ncols,
                           int32_t *__restrict__ cols, uint64_t *__restrict__ tkeys,
                           uint64_t nrows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  const uint64_t r = k / ncols, c = k - r * ncols;
  cols[i] = (int32_t)c;
  if (tkeys) tkeys[i] = c * nrows + r;
}

// rowptr[r] = number of keys below r * ncols (binary search, r in [0, nrows]).
__global__ void row_pointers(const uint64_t *__restrict__ keys, int64_t n, uint64_t ncols,
                             int64_t nrows, int32_t *__restrict__ rowptr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nrows) return;
  const uint64_t target = (uint64_t)r * ncols;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < target) lo = mid + 1; else hi = mid;
  }
  rowptr[r] = (int32_t)lo;
}

// Largest radius index (plus one) among the pieces of the stacked A12, whose
// keys are (a * nl + l) * npix + col. Grid-stride; the maximum is taken per
// wavefront first, so only one lane per wavefront touches the shared counter.
__global__ void live_kernel(const uint64_t *__restrict__ keys, int64_t n, uint64_t npix, int nl,
                            int *__restrict__ live) {
  int m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = max(m, (int)((keys[i] / npix) % (uint64_t)nl) + 1);
  for (int o = warpSize / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & (warpSize - 1)) == 0 && m > 0) atomicMax(live, m);
}

// Renumbers rows a * nl + l (l < live) as a * live + l.
__global__ void compact_kernel(uint64_t *__restrict__ keys, int64_t n, uint64_t npix, int nl,
                               int live) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = keys[i];
  const uint64_t row = k / npix, col = k - row * npix;
  const uint64_t a = row / (uint64_t)nl, l = row - a * (uint64_t)nl;
  keys[i] = (a * (uint64_t)live + l) * npix + col;
}

int key_bits(uint64_t max_key) {
  int b = 1;
  while (b < 64 && (max_key >> b) != 0) ++b;
  return b;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { (void)hipFree(p); }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes > 0 ? bytes : 1); }
  template <class T> T *as() const { return (T *)p; }
};

// Sorts (keys, vals) in place by key; the merged result goes to ukeys/uvals.
Status sort_merge(uint64_t *keys, double *vals, int64_t n, int bits, hipStream_t s,
                  DevBuf &ukeys, DevBuf &uvals, int64_t *n_unique) {
  DevBuf k2, v2, tmp, nruns;
  if (k2.alloc(sizeof(uint64_t) * n) != hipSuccess || v2.alloc(sizeof(double) * n) != hipSuccess ||
      ukeys.alloc(sizeof(uint64_t) * n) != hipSuccess ||
      uvals.alloc(sizeof(double) * n) != hipSuccess || nruns.alloc(sizeof(int64_t)) != hipSuccess)
    return fail(SRT_ENOMEM, "device allocation for operator sort failed");
  hipcub::DoubleBuffer<uint64_t> dk(keys, k2.as<uint64_t>());
  hipcub::DoubleBuffer<double> dv(vals, v2.as<double>());
  size_t b1 = 0, b2 = 0;
  SRT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, b1, dk, dv, (int)n, 0, bits, s));
  SRT_HIP(hipcub::DeviceReduce::ReduceByKey(nullptr, b2, dk.Current(), ukeys.as<uint64_t>(),
                                            dv.Current(), uvals.as<double>(),
                                            nruns.as<int64_t>(), hipcub::Sum(), (int)n, s));
  if (tmp.alloc(b1 > b2 ? b1 : b2) != hipSuccess)
    return fail(SRT_ENOMEM, "device allocation for sort scratch failed");
  SRT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, b1, dk, dv, (int)n, 0, bits, s));
  SRT_HIP(hipcub::DeviceReduce::ReduceByKey(tmp.p, b2, dk.Current(), ukeys.as<uint64_t>(),
                                            dv.Current(), uvals.as<double>(),
                                            nruns.as<int64_t>(), hipcub::Sum(), (int)n, s));
  SRT_HIP(hipMemcpyAsync(n_unique, nruns.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SRT_HIP(hipStreamSynchronize(s));
  return Status{};
}

// CSR from sorted unique keys and their FP64 values.
Status make_csr(const uint64_t *ukeys, const double *uvals, int64_t nnz, int64_t nrows,
                int64_t ncols, srt_dtype wdtype, double scale, hipStream_t s, Csr *out,
                uint64_t *tkeys_out) {
  out->nrows = nrows;
  out->ncols = ncols;
  out->nnz = nnz;
  out->wdtype = wdtype;
  out->scale = scale;
  if (hipMalloc(&out->rowptr, sizeof(int32_t) * (nrows + 1)) != hipSuccess ||
      hipMalloc(&out->cols, sizeof(int32_t) * (nnz > 0 ? nnz : 1)) != hipSuccess ||
      hipMalloc(&out->vals, dtype_size(wdtype) * (nnz > 0 ? nnz : 1)) != hipSuccess)
    return fail(SRT_ENOMEM, "device allocation for CSR operator failed");
  const int t = 256;
  hipLaunchKernelGGL(row_pointers, dim3(blocks_for(nrows + 1, t)), dim3(t), 0, s, ukeys, nnz,
                     (uint64_t)ncols, nrows, out->rowptr);
  if (nnz > 0) {
    hipLaunchKernelGGL(split_keys, dim3(blocks_for(nnz, t)), dim3(t), 0, s, ukeys, nnz,
                       (uint64_t)ncols, out->cols, tkeys_out, (uint64_t)nrows);
    hipLaunchKernelGGL(store_weights, dim3(blocks_for(nnz, t)), dim3(t), 0, s, uvals, nnz,
                       scale, (int)wdtype, out->vals);
  }
  SRT_HIP(hipGetLastError());
  return Status{};
}

}  // namespace

size_t Csr::bytes() const {
  return sizeof(int32_t) * (size_t)(nrows + 1) + (sizeof(int32_t) + dtype_size(wdtype)) * (size_t)nnz;
}

void Csr::release() {
  (void)hipFree(rowptr);
  (void)hipFree(cols);
  (void)hipFree(vals);
  rowptr = nullptr;
  cols = nullptr;
  vals = nullptr;
}

Status build_csr_pair(Coo *pieces, int64_t nrows, int64_t ncols, srt_dtype wdtype,
                      hipStream_t s, Csr *op, Csr *op_t) {
  const int64_t n = pieces->n;
  if (n >= (int64_t)INT32_MAX)
    return fail(SRT_ENOTSUP, "operator has more than 2^31-1 arc pieces");
  const uint64_t max_key = (uint64_t)nrows * (uint64_t)ncols;
  DevBuf ukeys, uvals;
  int64_t nnz = 0;
  if (n > 0) {
    SRT_TRY(sort_merge(pieces->keys, pieces->vals, n, key_bits(max_key), s, ukeys, uvals, &nnz));
  } else if (ukeys.alloc(8) != hipSuccess || uvals.alloc(8) != hipSuccess) {
    return fail(SRT_ENOMEM, "device allocation failed");
  }
  (void)hipFree(pieces->keys);
  (void)hipFree(pieces->vals);
  pieces->keys = nullptr;
  pieces->vals = nullptr;

  // Storage scale: a power of two bringing the largest weight into (1/2, 1]
  // for 16-bit weights (exact in any binary format); 1 otherwise.
  double scale = 1.0;
  if ((wdtype == SRT_BF16 || wdtype == SRT_F16) && nnz > 0) {
    DevBuf tmp, mx;
    size_t b = 0;
    if (mx.alloc(sizeof(double)) != hipSuccess) return fail(SRT_ENOMEM, "allocation failed");
    SRT_HIP(hipcub::DeviceReduce::Max(nullptr, b, uvals.as<double>(), mx.as<double>(), (int)nnz, s));
    if (tmp.alloc(b) != hipSuccess) return fail(SRT_ENOMEM, "allocation failed");
    SRT_HIP(hipcub::DeviceReduce::Max(tmp.p, b, uvals.as<double>(), mx.as<double>(), (int)nnz, s));
    double m = 0;
    SRT_HIP(hipMemcpyAsync(&m, mx.p, sizeof(double), hipMemcpyDeviceToHost, s));
    SRT_HIP(hipStreamSynchronize(s));
    if (m > 0) {
      const int e = std::ilogb(m);
      const bool pow2 = (m == std::ldexp(1.0, e));
      scale = std::ldexp(1.0, pow2 ? -e : -e - 1);
    }
  }

  DevBuf tkeys;
  if (tkeys.alloc(sizeof(uint64_t) * (nnz > 0 ? nnz : 1)) != hipSuccess)
    return fail(SRT_ENOMEM, "device allocation for transpose keys failed");
  SRT_TRY(make_csr(ukeys.as<uint64_t>(), uvals.as<double>(), nnz, nrows, ncols, wdtype, scale, s,
                   op, tkeys.as<uint64_t>()));
  SRT_HIP(hipStreamSynchronize(s));

  // Transpose: sort the same merged entries by (col, row); keys are unique.
  DevBuf tk2, tv2;
  if (nnz > 0) {
    DevBuf tvals;
    if (tvals.alloc(sizeof(double) * nnz) != hipSuccess)
      return fail(SRT_ENOMEM, "device allocation for transpose failed");
    SRT_HIP(hipMemcpyAsync(tvals.p, uvals.p, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    int64_t nnz_t = 0;
    SRT_TRY(sort_merge(tkeys.as<uint64_t>(), tvals.as<double>(), nnz, key_bits(max_key), s, tk2,
                       tv2, &nnz_t));
    if (nnz_t != nnz) return fail(SRT_EDEVICE, "transpose changed the number of entries");
  } else if (tk2.alloc(8) != hipSuccess || tv2.alloc(8) != hipSuccess) {
    return fail(SRT_ENOMEM, "device allocation failed");
  }
  SRT_TRY(make_csr(tk2.as<uint64_t>(), tv2.as<double>(), nnz, ncols, nrows, wdtype, scale, s,
                   op_t, nullptr));
  SRT_HIP(hipStreamSynchronize(s));
  return Status{};
}

Status compact_a12(Coo *pieces, int32_t nl, int64_t npix, hipStream_t s, int32_t *live) {
  DevBuf d;
  if (d.alloc(sizeof(int)) != hipSuccess) return fail(SRT_ENOMEM, "allocation failed");
  SRT_HIP(hipMemsetAsync(d.p, 0, sizeof(int), s));
  if (pieces->n > 0)
    hipLaunchKernelGGL(live_kernel, dim3((unsigned)std::min<int64_t>(blocks_for(pieces->n, 256), 8192)),
                       dim3(256), 0, s,
                       pieces->keys, pieces->n, (uint64_t)npix, (int)nl, d.as<int>());
  SRT_HIP(hipGetLastError());
  int h = 0;
  SRT_HIP(hipMemcpyAsync(&h, d.p, sizeof(int), hipMemcpyDeviceToHost, s));
  SRT_HIP(hipStreamSynchronize(s));
  *live = h;
  if (pieces->n > 0 && h > 0)
    hipLaunchKernelGGL(compact_kernel, dim3(blocks_for(pieces->n, 256)), dim3(256), 0, s,
                       pieces->keys, pieces->n, (uint64_t)npix, (int)nl, h);
  SRT_HIP(hipGetLastError());
  return Status{};
}

}  // namespace srt
