// Pattern transpose of P on the device: P^T's row pointers and column ids and,
// for every entry q of P, its position in P^T (so that P^T's values follow
// P's with one permutation).  A stable radix sort of (column of q, q) keeps
// the entries of every column in ascending P-row order, the order in which a
// serial transpose would list them.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace hamg {

namespace {

__global__ void k_row_of(int64_t n, const int64_t* __restrict__ ptr, int32_t* __restrict__ row_of) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    for (int64_t q = ptr[r]; q < ptr[r + 1]; ++q) row_of[q] = (int32_t)r;
}

__global__ void k_iota(int64_t n, int32_t* __restrict__ v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (int32_t)i;
}

// position d of P^T holds entry q = sorted[d]: its P^T column is q's P row
__global__ void k_transpose_fill(int64_t nnz, const int32_t* __restrict__ sorted,
                                 const int32_t* __restrict__ row_of, int32_t* __restrict__ tcol,
                                 int64_t* __restrict__ perm) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < nnz;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = sorted[d];
    tcol[d] = row_of[q];
    perm[q] = d;
  }
}

// tptr[c] = first position whose sorted column is >= c (c = 0 .. nc)
__global__ void k_col_starts(int64_t nc, int64_t nnz, const int32_t* __restrict__ keys,
                             int64_t* __restrict__ tptr) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < c) lo = mid + 1; else hi = mid;
    }
    tptr[c] = lo;
  }
}

unsigned grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

hipError_t transpose_pattern(int64_t n, int64_t nc, int64_t nnz, const int64_t* ptr,
                             const int32_t* col, int64_t* tptr, int32_t* tcol, int64_t* perm,
                             hipStream_t st) {
  if (nnz <= 0) {
    hipLaunchKernelGGL(k_col_starts, dim3(grid_of(nc + 1)), dim3(256), 0, st, nc, (int64_t)0, col, tptr);
    return hipGetLastError();
  }
  if (nnz > (int64_t)INT32_MAX || nc > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  int end_bit = 1;
  while (end_bit < 31 && ((int64_t)1 << end_bit) <= nc) ++end_bit;
  int32_t *keys_out = nullptr, *vals_in = nullptr, *vals_out = nullptr, *row_of = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  hipError_t e = hipSuccess;
  auto check = [&](hipError_t r) {
    if (e == hipSuccess && r != hipSuccess) e = r;
    return e == hipSuccess;
  };
  const size_t b = (size_t)nnz * sizeof(int32_t);
  if (check(hipMalloc(&keys_out, b)) && check(hipMalloc(&vals_in, b)) &&
      check(hipMalloc(&vals_out, b)) && check(hipMalloc(&row_of, b))) {
    hipLaunchKernelGGL(k_row_of, dim3(grid_of(n)), dim3(256), 0, st, n, ptr, row_of);
    hipLaunchKernelGGL(k_iota, dim3(grid_of(nnz)), dim3(256), 0, st, nnz, vals_in);
    if (check(hipGetLastError()) &&
        check(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, col, keys_out, vals_in, vals_out,
                                                 (int)nnz, 0, end_bit, st)) &&
        check(hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 1))) &&
        check(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, col, keys_out, vals_in, vals_out,
                                                 (int)nnz, 0, end_bit, st))) {
      hipLaunchKernelGGL(k_transpose_fill, dim3(grid_of(nnz)), dim3(256), 0, st, nnz, vals_out,
                         row_of, tcol, perm);
      hipLaunchKernelGGL(k_col_starts, dim3(grid_of(nc + 1)), dim3(256), 0, st, nc, nnz, keys_out,
                         tptr);
      check(hipGetLastError());
    }
  }
  // the scratch arrays are released once the stream has used them
  check(hipStreamSynchronize(st));
  for (void* p : {(void*)keys_out, (void*)vals_in, (void*)vals_out, (void*)row_of, tmp})
    if (p) (void)hipFree(p);
  return e;
}

}  // namespace hamg
