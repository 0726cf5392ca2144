// Device helpers shared by the element kernels: simplex geometry and flag bits.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace crh {

// ---------------------------------------------------------------------------
// geometry: |K|, a_{K,j} = |sigma_j| n_{K,sigma_j} (outward), x_K.
// With E = [x_1 - x_0, ..., x_d - x_0], grad(lambda_j) is row j-1 of E^{-1} and
// a_j = -d |K| grad(lambda_j), i.e. minus sign(det E) / (d-1)! times row j-1 of
// adj(E); a_0 closes the surface.
// ---------------------------------------------------------------------------
template <int D>
struct Geo {
  double X[D + 1][D];
  double a[D + 1][D];
  double vol;
  double xK[D];
};

template <int D>
__device__ __forceinline__ void load_geometry(const double* __restrict__ ecoord, int64_t ne, int64_t k, Geo<D>& g) {
#pragma unroll
  for (int j = 0; j <= D; ++j)
#pragma unroll
    for (int r = 0; r < D; ++r) g.X[j][r] = ecoord[(j * D + r) * ne + k];
  double E[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) E[r][c] = g.X[c + 1][r] - g.X[0][r];
  if constexpr (D == 2) {
    double det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
    double sg = det > 0.0 ? 1.0 : -1.0;
    g.a[1][0] = -sg * E[1][1];
    g.a[1][1] = sg * E[0][1];
    g.a[2][0] = sg * E[1][0];
    g.a[2][1] = -sg * E[0][0];
    g.vol = 0.5 * fabs(det);
  } else {
    double e[3][3];  // e[c] = column c
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 3; ++r) e[c][r] = E[r][c];
    double cr[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double* p = e[(j + 1) % 3];
      const double* q = e[(j + 2) % 3];
      cr[j][0] = p[1] * q[2] - p[2] * q[1];
      cr[j][1] = p[2] * q[0] - p[0] * q[2];
      cr[j][2] = p[0] * q[1] - p[1] * q[0];
    }
    double det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
    double h = det > 0.0 ? -0.5 : 0.5;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int r = 0; r < 3; ++r) g.a[j + 1][r] = h * cr[j][r];
    g.vol = fabs(det) / 6.0;
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    double s = 0.0, x = 0.0;
#pragma unroll
    for (int j = 1; j <= D; ++j) s += g.a[j][r];
    g.a[0][r] = -s;
#pragma unroll
    for (int j = 0; j <= D; ++j) x += g.X[j][r];
    g.xK[r] = x / (D + 1);
  }
}

__device__ __forceinline__ bool interior(uint32_t fl, int j) { return (fl >> j) & 1u; }
__device__ __forceinline__ double csign(uint32_t fl, int j) { return ((fl >> (8 + j)) & 1u) ? -1.0 : 1.0; }

}  // namespace crh
