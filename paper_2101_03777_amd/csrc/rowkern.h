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

// ---------------------------------------------------------------------------
// Element-factor form of the scaled Stokes operator Ds G Ds (Ds = 1/dsq, one
// scale per face).  G = sum_K H_K G_K H_K^t with, for Stokes,
//   G_K[(j,i),(l,i')] = c_j c_l (delta_ii' (S_K^{-1})_jl - V_ji V_li' / B_K)
// (Section 3.2 items 4-5; A^_K = S_K (x) I_d), so the scaled element matrix is
//   delta_ii' Sh_jl - Vh_ji Vh_li',   Sh_jl = c_j c_l (S_K^{-1})_jl / (s_j s_l),
//                                     Vh_ji = c_j V_ji sqrt(1/B_K) / s_j,
// with s_j the scale of local face j.  Per element that is N(N+1)/2 + N D
// numbers (12 in 2D, 22 in 3D) instead of the (2d+1) d^2 numbers per face of
// the assembled rows.  Rows of exterior faces are zero.  A face row sums the
// row of its local face in its two elements; the element data of each
// element is read by its d+1 faces, mostly from cache.
// ---------------------------------------------------------------------------
template <int D>
struct EfoLayout {
  static constexpr int N = D + 1;
  static constexpr int NSYM = N * (N + 1) / 2;
  static constexpr int NF = NSYM + N * D;  // planes per element
  // packed upper triangle (row-major) index of (a, b), a <= b
  __host__ __device__ static constexpr int tri(int a, int b) { return a * N - a * (a - 1) / 2 + (b - a); }
  __host__ __device__ static constexpr int sym(int j, int l) { return j <= l ? tri(j, l) : tri(l, j); }
  __host__ __device__ static constexpr int vh(int l, int i) { return NSYM + l * D + i; }
};

template <typename T>
struct Efo {
  const T* __restrict__ F;           // [NF][ne]
  const int32_t* __restrict__ egat;  // [N][ne] face read for local face l (zero weight if exterior)
  const int32_t* __restrict__ fel;   // [2][nf] the two elements of a face
  const int32_t* __restrict__ floc;  // [nf] local index in the first | in the second << 8
  int64_t ne;
};

template <int D, typename T, class In>
__device__ __forceinline__ Vec<T, D> efo_row(const Efo<T>& E, int64_t nf, int64_t f, const In& in) {
  using L = EfoLayout<D>;
  constexpr int N = L::N;
  const int lc = E.floc[f];
  Vec<T, D> w;
#pragma unroll
  for (int i = 0; i < D; ++i) w.v[i] = T(0);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t K = E.fel[(int64_t)side * nf + f];
    const int j = (lc >> (8 * side)) & 0xff;
    Vec<T, D> xv[N];
#pragma unroll
    for (int l = 0; l < N; ++l) xv[l] = in(E.egat[(int64_t)l * E.ne + K]);
    T vh[N][D];
    T t = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l)
#pragma unroll
      for (int i = 0; i < D; ++i) {
        vh[l][i] = E.F[(int64_t)L::vh(l, i) * E.ne + K];
        t += vh[l][i] * xv[l].v[i];
      }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const T sh = E.F[(int64_t)L::sym(j, l) * E.ne + K];
#pragma unroll
      for (int i = 0; i < D; ++i) w.v[i] += sh * xv[l].v[i];
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T vj = vh[0][i];
#pragma unroll
      for (int l = 1; l < N; ++l) vj = j == l ? vh[l][i] : vj;
      w.v[i] -= vj * t;
    }
  }
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

// Stop words.  The first kernel of an iteration decides in every workgroup,
// from the same partial sums, whether the iteration runs; the workgroup with
// logical index 0 records the decision in a stop word that the other
// workgroups of the same launch also read.  The waves of one workgroup may
// therefore see different values of that word.  block_sum_stop takes each
// wave's view along with its sums and returns the OR over the workgroup, so
// that all waves of a workgroup leave together, after the barrier, and every
// wave that continues used complete sums.  (Any workgroup that saw the word
// still clear reaches the same decision as the one that wrote it.)
template <int M>
__device__ __forceinline__ bool block_sum_stop(double (&v)[M], int seen) {
  __shared__ double sh[M][NT / 64];
  __shared__ int sf[NT / 64];
  int s = seen != 0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double x = v[m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[m] = x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s |= __shfl_xor(s, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) sh[m][w] = v[m];
    sf[w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = (sh[m][0] + sh[m][1]) + (sh[m][2] + sh[m][3]);
  s = (sf[0] | sf[1]) | (sf[2] | sf[3]);
  __syncthreads();
  return s != 0;
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

// reduce_partials with the workgroup-uniform stop view of block_sum_stop
template <int M>
__device__ __forceinline__ bool reduce_partials_stop(const double* __restrict__ part, int nblk, int first,
                                                     double (&v)[M], int seen) {
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT)
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] += part[(int64_t)i * NPART + first + m];
  return block_sum_stop<M>(v, seen);
}

// reduce_fields with the workgroup-uniform stop view of block_sum_stop:
// returns true if any wave of the workgroup saw the stop word set
template <int M>
__device__ __forceinline__ bool reduce_fields_stop(const double* __restrict__ part, int nblk, const int (&fields)[M],
                                                   double (&v)[M], int seen) {
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT)
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] += part[(int64_t)fields[m] * nblk + i];
  return block_sum_stop<M>(v, seen);
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }


}  // namespace crh
