// Device helpers of the row kernels (Krylov and coupled baseline): row
// partition with XCD-contiguous ranges, small vector loads/stores, and the
// deterministic block / partial-record reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace crh {

constexpr int MAXBLK = 1024;   // upper bound on workgroups of the row kernels
constexpr int NPART = 4;       // doubles per partial record

struct Part {
  int64_t nf;
  int nblk;
  int64_t chunk;
};

__device__ __forceinline__ int logical_block(int nblk) {
  const int per = nblk >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

template <typename T, int D>
struct Vec {
  T v[D];
};

template <typename T, int D>
__device__ __forceinline__ Vec<T, D> ldv(const T* __restrict__ p, int64_t f) {
  Vec<T, D> r;
  if constexpr (D == 2) {
    using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    V2 t = *reinterpret_cast<const V2*>(p + f * 2);
    r.v[0] = t.x;
    r.v[1] = t.y;
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) r.v[i] = p[f * D + i];
  }
  return r;
}

template <typename T, int D>
__device__ __forceinline__ void stv(T* __restrict__ p, int64_t f, const Vec<T, D>& r) {
  if constexpr (D == 2) {
    using V2 = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    V2 t;
    t.x = r.v[0];
    t.y = r.v[1];
    *reinterpret_cast<V2*>(p + f * 2) = t;
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) p[f * D + i] = r.v[i];
  }
}

// one face row of the block-ELL product; In(c) returns the input vector at face c
template <int D, typename T, class In>
__device__ __forceinline__ Vec<T, D> spmv_row(const T* __restrict__ G, const int32_t* __restrict__ cols, int64_t nf,
                                              int64_t f, const In& in) {
  constexpr int DD = D * D, NS = 2 * D + 1;
  int c[NS];
  c[0] = (int)f;
#pragma unroll
  for (int s = 1; s < NS; ++s) c[s] = cols[(int64_t)(s - 1) * nf + f];
  Vec<T, D> xv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) xv[s] = in(c[s]);
  Vec<T, D> w;
#pragma unroll
  for (int i = 0; i < D; ++i) w.v[i] = T(0);
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) w.v[i] += G[(int64_t)(s * DD + i * D + j) * nf + f] * xv[s].v[j];
  return w;
}

template <int M>
__device__ __forceinline__ void block_sum(double (&v)[M]) {
  __shared__ double sh[M][NT / 64];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double x = v[m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[m] = x;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) sh[m][w] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = (sh[m][0] + sh[m][1]) + (sh[m][2] + sh[m][3]);
  __syncthreads();
}

// every workgroup reduces the same partial records in the same order
template <int M>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nblk, int first, double (&v)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT)
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] += part[(int64_t)i * NPART + first + m];
  block_sum<M>(v);
}

// Partial records stored field-major (part[field * nblk + block]): a consumer
// that needs k fields reads k contiguous arrays of nblk doubles.
template <int M>
__device__ __forceinline__ void reduce_fields(const double* __restrict__ part, int nblk, const int (&fields)[M],
                                              double (&v)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT)
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] += part[(int64_t)fields[m] * nblk + i];
  block_sum<M>(v);
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }


}  // namespace crh
