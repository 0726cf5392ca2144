// Element matrix of the Navier-Stokes Newton step, shared by the elimination
// (elements.hip) and the coupled baseline (coupled.hip).
//
// A_K = S_K (x) I_d + d/du [N_K(u, u)] at ubar, with N_K the element vector of
// the convection form b_h (second form of eq. defbh, Section 2 item 6) and
// F_{s,t} the flux through the co-volume face between faces s and t, in the
// closed form of Section 2 item 6.  Local unknowns are indexed j*d + i (local
// face j, component i).
#pragma once

#include "geometry.h"

namespace crh {

template <int D>
struct NsPack {
  static constexpr int N = D + 1;
  static constexpr int NU = N * D;
  static constexpr int SIZE = NU * NU + 2 * NU + 1;  // A^{-1}, l, r, 1/B
};

// A(r, c) of a local NU x NU matrix: in registers (2D), or in the calling
// thread's column of an LDS array (3D: 144 doubles per element)
// Non-homogeneous Dirichlet data seen from an element: the exterior face of
// each local face (-1 interior; ebf == nullptr: no data), the data in canonical
// exterior order, and the divergence right-hand side e_K written by the
// elimination.
struct Bnd {
  const int32_t* ebf;  // [d+1][ne]
  const double* g;     // [nbf][d]
  double* ek;          // [ne]
};

// the data at the element's local faces, zero on interior faces
template <int D>
__device__ __forceinline__ void load_bnd(const Bnd& b, uint32_t fl, int64_t ne, int64_t k, double (&Gb)[D + 1][D]) {
#pragma unroll
  for (int j = 0; j <= D; ++j) {
    const bool ext = b.ebf != nullptr && !((fl >> j) & 1u);
    const int64_t e = ext ? b.ebf[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < D; ++i) Gb[j][i] = ext ? b.g[e * D + i] : 0.0;
  }
}

template <int NU>
struct RegMat {
  double (&m)[NU][NU];
  __device__ double& operator()(int r, int c) const { return m[r][c]; }
};

template <int NU>
struct LdsMat {
  double* base;  // entry (0, 0) of this thread; consecutive entries `stride` doubles apart
  int stride;
  __device__ double& operator()(int r, int c) const { return base[(r * NU + c) * stride]; }
};

// Ub: the linearisation velocity at the local faces (the boundary data on
// exterior faces); Gb: the boundary data (zero on interior faces).  Rows and
// columns of exterior faces are removed from A, and Rb receives the columns of
// exterior faces times their data, -sum_r A[s, r] g_r, for the right-hand side.
template <int D, class M>
__device__ __forceinline__ void ns_local(const Geo<D>& g, uint32_t fl, const double (&Ub)[D + 1][D], double mu,
                                         double nu, const M& A, double (&Nuu)[D + 1][D],
                                         const double (&Gb)[D + 1][D], double (&Rb)[D + 1][D]) {
  constexpr int N = D + 1;
#pragma unroll
  for (int s = 0; s < N; ++s)
#pragma unroll
    for (int i = 0; i < D; ++i) Rb[s][i] = 0.0;
  const double m = mu * g.vol / N, iv = nu / g.vol;
  double F[N][N], gx[N][N][D], Um[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double t = Ub[0][j];
#pragma unroll
    for (int q = 1; q < N; ++q) t += Ub[q][j];
    Um[j] = t / N;
  }
#pragma unroll
  for (int s = 0; s < N; ++s)
#pragma unroll
    for (int t = 0; t < N; ++t) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        gx[s][t][j] = (g.a[t][j] - g.a[s][j]) / N;
        double w = Ub[s][j] + Ub[t][j] - Um[j];
        v += w * gx[s][t][j];
      }
      F[s][t] = s == t ? 0.0 : v;
    }
#pragma unroll
  for (int s = 0; s < N; ++s)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < N; ++t) v += 0.5 * F[s][t] * (Ub[t][i] - Ub[s][i]);
      Nuu[s][i] = v;
    }
#pragma unroll
  for (int s = 0; s < N; ++s) {
    double rowF = F[s][0];
#pragma unroll
    for (int t = 1; t < N; ++t) rowF += F[s][t];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          double v = 0.0;
          if (i == j) {
            double ar = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) ar += g.a[s][q] * g.a[r][q];
            v += (s == r ? m : 0.0) + iv * ar;
            v += 0.5 * ((s == r ? 0.0 : F[s][r]) - (s == r ? rowF : 0.0));
          }
#pragma unroll
          for (int t = 0; t < N; ++t) {
            if (t == s) continue;
            double coef = (r == s ? 1.0 : 0.0) + (r == t ? 1.0 : 0.0) - 1.0 / N;
            v += 0.5 * coef * gx[s][t][j] * (Ub[t][i] - Ub[s][i]);
          }
          bool in = interior(fl, s) && interior(fl, r);
          if (interior(fl, s) && !interior(fl, r)) Rb[s][i] -= v * Gb[r][j];
          A(s * D + i, r * D + j) = in ? v : ((s == r && i == j) ? 1.0 : 0.0);
        }
  }
}

// the linearisation velocity at the local faces: interior faces from ulin,
// exterior faces from the boundary data Gb (zero without data)
template <int D>
__device__ __forceinline__ void load_ubar(const double* __restrict__ ulin, const int32_t* __restrict__ eface,
                                          uint32_t fl, int64_t ne, int64_t k, const double (&Gb)[D + 1][D],
                                          double (&Ub)[D + 1][D]) {
#pragma unroll
  for (int j = 0; j <= D; ++j) {
    bool in = ulin != nullptr && interior(fl, j);
    int f = in ? eface[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < D; ++i) Ub[j][i] = in ? ulin[(int64_t)f * D + i] : Gb[j][i];
  }
}

}  // namespace crh
