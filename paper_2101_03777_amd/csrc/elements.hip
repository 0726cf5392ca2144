// Element-wise kernels of the hybrid method (steps a1-a3, a5, a6), FP64.
//
// Paper: Chenier & Eymard, arXiv 2101.03777.
//   Section 2 items 1-4: geometry, CR basis, lumped mass, right-hand side eq. defrhs.
//   Section 2 item 6:    convection form b_h (eq. defbh), Newton Jacobian.
//   Section 3.1:         element matrices S_K, A_K, D_K, R_K.
//   Section 3.2:         E_K, C_K, B_K, G_K, s_K (items 4-5, 7), recovery (items 2, 4).
//
// One thread per element for elimination and recovery (the dense local algebra
// lives in registers: (d+1)x(d+1) in the Stokes case, where A^_K = S_K (x) I_d,
// and 6x6 for the 2D Newton step), one thread per interior face for the
// gather assembly of G: the (sigma, sigma') block of G comes from the unique
// element holding both faces and the diagonal block from the face's two
// elements, so assembly needs no atomics.
#include <cmath>
#include <mutex>
#include <utility>

#include "internal.h"
#include "geometry.h"
#include "rowkern.h"
#include "convection.h"

// Workgroup partials of the allocation-free recovery (cr_recover_noalloc):
// one double per element workgroup of the copy-mismatch pass, so at most
// NOALLOC_PARTIALS * 128 elements.  Each device holds its own copy for the
// life of the process; host code uses the address hipGetSymbolAddress returns
// for the current device, never this name.
constexpr int64_t NOALLOC_PARTIALS = 32768;  // 256 KiB
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

namespace crh {
namespace {

constexpr int BS = 128;  // threads per block for element/face kernels

enum : int { ERR_SINGULAR = 1, ERR_NONFINITE = 2, ERR_ZERODIAG = 4 };

__device__ __forceinline__ void report(int32_t* err, int bits, int64_t id) {
  atomicOr(err, bits);
  atomicMin(err + 1, (int32_t)id);
}

// In-place Gauss-Jordan inverse of an N x N matrix held in registers.  With
// PIVOT, rows are exchanged by compile-time-indexed conditional swaps so that
// the largest remaining entry of each column becomes the pivot (partial
// pivoting without dynamic register indexing).  Returns false on a zero pivot.
template <int N, bool PIVOT>
__device__ __forceinline__ bool gj_inverse(double (&A)[N][N], double (&Inv)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) Inv[r][c] = r == c ? 1.0 : 0.0;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    if constexpr (PIVOT) {
#pragma unroll
      for (int r = c + 1; r < N; ++r) {
        bool sw = fabs(A[r][c]) > fabs(A[c][c]);
#pragma unroll
        for (int q = 0; q < N; ++q) {
          double t0 = A[c][q], t1 = A[r][q];
          A[c][q] = sw ? t1 : t0;
          A[r][q] = sw ? t0 : t1;
          double u0 = Inv[c][q], u1 = Inv[r][q];
          Inv[c][q] = sw ? u1 : u0;
          Inv[r][q] = sw ? u0 : u1;
        }
      }
    }
    double piv = A[c][c];
    ok = ok && (piv != 0.0);
    double ip = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < N; ++q) {
      A[c][q] *= ip;
      Inv[c][q] *= ip;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      double f = A[r][c];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        A[r][q] -= f * A[c][q];
        Inv[r][q] -= f * Inv[c][q];
      }
    }
  }
  return ok;
}


// packed symmetric index of (j, l), j <= l, in an N x N upper triangle (row-major)
template <int N>
__device__ __forceinline__ constexpr int sym(int j, int l) {
  return j <= l ? j * N - j * (j - 1) / 2 + (l - j) : l * N - l * (l - 1) / 2 + (j - l);
}

// ---------------------------------------------------------------------------
// Stokes pack: S_K^{-1} (symmetric, N(N+1)/2), V = A^_K^{-1} D_K as [N][D], 1/B_K.
// For K0 the pack stores V = 0 and 1/B = 0, which turns every formula below
// into its K0 form (G_K0 = C A^{-1} C, s_K0 = C A^{-1} R, P_K0 = 0).
// ---------------------------------------------------------------------------
template <int D>
struct StokesPack {
  static constexpr int N = D + 1;
  static constexpr int NS = N * (N + 1) / 2;
  static constexpr int SIZE = NS + N * D + 1;
};

template <int D>
struct StokesFactors {
  double Si[D + 1][D + 1];
  double V[D + 1][D];
  double invB;
};

template <int D>
__device__ __forceinline__ void load_stokes_pack(const double* __restrict__ pack, int64_t ne, int64_t k,
                                                 StokesFactors<D>& F) {
  constexpr int N = D + 1;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int l = j; l < N; ++l) {
      double v = pack[(int64_t)sym<N>(j, l) * ne + k];
      F.Si[j][l] = v;
      F.Si[l][j] = v;
    }
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) F.V[j][i] = pack[(int64_t)(StokesPack<D>::NS + j * D + i) * ne + k];
  F.invB = pack[(int64_t)(StokesPack<D>::SIZE - 1) * ne + k];
}

// R_K (eq. defrhs plus the lumped-mass transient term) and s_K from the factors.
// (R_K)_{j,i} = a_j^(i) fbar.(x_sigma_j - x_K) with x_sigma_j - x_K = (x_K - x_j)/d.
// With boundary data the columns of the exterior faces of S_K (stiffness only,
// the lumped mass is diagonal) times the data leave the interior rows, and
// e_K = a . g becomes the right-hand side of the divergence row.
template <int D>
__device__ __forceinline__ void stokes_rhs(const Geo<D>& g, uint32_t fl, const StokesFactors<D>& F,
                                           const double* __restrict__ fbar, const double* __restrict__ uprev,
                                           const int32_t* __restrict__ eface, double mu, double nu, const Bnd& bnd,
                                           int64_t ne, int64_t k, double* __restrict__ RK, double* __restrict__ sK,
                                           int32_t* err) {
  constexpr int N = D + 1;
  double fb[D];
  bool fin = true;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    fb[i] = fbar[k * D + i];
    fin = fin && isfinite(fb[i]);
  }
  double R[N][D];
  const double m = mu * g.vol / N;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double proj = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) proj += fb[i] * (g.xK[i] - g.X[j][i]);
    proj *= 1.0 / D;
    bool in = interior(fl, j);
    int f = in ? eface[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double r = g.a[j][i] * proj;
      if (uprev != nullptr && in) {
        double u = uprev[(int64_t)f * D + i];
        fin = fin && isfinite(u);
        r += m * u;
      }
      R[j][i] = in ? r : 0.0;
    }
  }
  if (!fin) report(err, ERR_NONFINITE, k);
  double ediv = 0.0;
  if (bnd.ebf != nullptr) {
    double Gb[N][D];
    load_bnd<D>(bnd, fl, ne, k, Gb);
    const double iv = nu / g.vol;
#pragma unroll
    for (int l = 0; l < N; ++l) {
#pragma unroll
      for (int i = 0; i < D; ++i) ediv += g.a[l][i] * Gb[l][i];
      if (interior(fl, l)) continue;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (!interior(fl, j)) continue;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) s += g.a[j][q] * g.a[l][q];
#pragma unroll
        for (int i = 0; i < D; ++i) R[j][i] -= iv * s * Gb[l][i];
      }
    }
    if (bnd.ek != nullptr) bnd.ek[k] = ediv;
  }
  double vr = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) vr += F.V[j][i] * R[j][i];
  vr = (vr - ediv) * F.invB;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double c = csign(fl, j);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) t += F.Si[j][l] * R[l][i];
      RK[(int64_t)(j * D + i) * ne + k] = R[j][i];
      sK[(int64_t)(j * D + i) * ne + k] = c * (t - F.V[j][i] * vr);
    }
  }
}

// a1 + a2, Stokes: S_K (Section 3.1) with the lumped mass |K|/(d+1) per face
// (Section 2 item 3) and grad(phi_j) = a_j/|K|; A^_K = S_K (x) I_d (E_K = 0 for
// mu > 0, Section 3.2 item 6; for mu = 0 the Stokes E_K is diagonal per face and
// is added to S_K); B_K = D_K^t A^_K^{-1} D_K with D_K = -a (Section 3.2 item 4).
// Rows and columns of exterior faces are replaced by the identity and their
// entries of D_K and R_K by zero, which removes them from every product.
template <int D>
__global__ void __launch_bounds__(BS) k_elim_stokes(int64_t ne, const double* __restrict__ ecoord,
                                                    const uint32_t* __restrict__ eflags,
                                                    const int32_t* __restrict__ eface,
                                                    const int32_t* __restrict__ enb,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ fbar,
                                                    const double* __restrict__ uprev, double mu, double nu,
                                                    Bnd bnd, double* __restrict__ pack, double* __restrict__ RK,
                                                    double* __restrict__ sK, int32_t* err) {
  constexpr int N = D + 1;
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  const double m = mu * g.vol / N, iv = nu / g.vol;
  double e[N];  // diagonal E_K (steady Stokes): -lambda_K on M1, +lambda_L on faces facing M1
#pragma unroll
  for (int j = 0; j < N; ++j) e[j] = 0.0;
  if (lam != nullptr) {
    if (fl & F_M1) {
#pragma unroll
      for (int j = 0; j < N; ++j) e[j] = -lam[k];
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        int nb = enb[j * ne + k];
        if (interior(fl, j) && nb >= 0 && (eflags[nb] & F_M1)) e[j] = lam[nb];
      }
    }
  }
  double S[N][N];
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int l = 0; l < N; ++l) {
      double v = iv * (g.a[j][0] * g.a[l][0] + g.a[j][1] * g.a[l][1] + (D == 3 ? g.a[j][D - 1] * g.a[l][D - 1] : 0.0));
      if (j == l) v += m + e[j];
      bool in = interior(fl, j) && interior(fl, l);
      S[j][l] = in ? v : (j == l ? 1.0 : 0.0);
    }
  StokesFactors<D> F;
  bool ok = gj_inverse<N, false>(S, F.Si);
  double B = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) v -= F.Si[j][l] * (interior(fl, l) ? g.a[l][i] : 0.0);
      F.V[j][i] = v;
      B -= (interior(fl, j) ? g.a[j][i] : 0.0) * v;
    }
  // symmetric (mu > 0) case: B_K > 0; steady M1 elements have a negative definite A^_K, B_K < 0
  if (!ok || !isfinite(B) || !(fabs(B) > 0.0) || (lam == nullptr && !(B > 0.0))) report(err, ERR_SINGULAR, k);
  const bool k0 = fl & F_K0;
  F.invB = k0 ? 0.0 : 1.0 / B;
  if (k0) {
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < D; ++i) F.V[j][i] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int l = j; l < N; ++l) pack[(int64_t)sym<N>(j, l) * ne + k] = F.Si[j][l];
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) pack[(int64_t)(StokesPack<D>::NS + j * D + i) * ne + k] = F.V[j][i];
  pack[(int64_t)(StokesPack<D>::SIZE - 1) * ne + k] = F.invB;
  stokes_rhs<D>(g, fl, F, fbar, uprev, eface, mu, nu, bnd, ne, k, RK, sK, err);
}

// a6: new right-hand side from stored factors (same G).
template <int D>
__global__ void __launch_bounds__(BS) k_rhs_stokes(int64_t ne, const double* __restrict__ ecoord,
                                                   const uint32_t* __restrict__ eflags,
                                                   const int32_t* __restrict__ eface,
                                                   const double* __restrict__ fbar,
                                                   const double* __restrict__ uprev, double mu, double nu, Bnd bnd,
                                                   const double* __restrict__ pack, double* __restrict__ RK,
                                                   double* __restrict__ sK, int32_t* err) {
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  StokesFactors<D> F;
  load_stokes_pack<D>(pack, ne, k, F);
  stokes_rhs<D>(g, eflags[k], F, fbar, uprev, eface, mu, nu, bnd, ne, k, RK, sK, err);
}

// ---------------------------------------------------------------------------
// Navier-Stokes Newton step (N = d+1 faces, NU = N d local unknowns, index j*d+i).
// A_K = S_K (x) I_d + d/du [N_K(u, u)] at ubar, where
//   N_K(w, z)_{s,i} = 1/2 sum_{t != s} F_{s,t}(w) (z_{t,i} - z_{s,i}),
//   F_{s,t}(w) = (W_s + W_t - sum_q W_q / N) . (a_t - a_s) / N
// (second form of eq. defbh and the flux closed form of Section 2 item 6), and
// R_K = R_f + N_K(ubar, ubar) (Newton right-hand side).  Exterior faces carry
// U = 0 inside the sums; their rows and columns are removed.
// ---------------------------------------------------------------------------
// In-place Gauss-Jordan inverse of an NU x NU matrix behind an accessor, with
// partial pivoting (row exchanges, recorded 4 bits per step, undone as column
// exchanges in reverse order at the end).  Runtime loops: for matrices kept in
// LDS.  Returns false on a zero or non-finite pivot.
template <int NU, class M>
__device__ bool gj_inverse_inplace(const M& A) {
  static_assert(NU <= 16, "pivot record holds 4 bits per step");
  uint64_t piv = 0;
  bool ok = true;
  for (int k = 0; k < NU; ++k) {
    int p = k;
    double best = fabs(A(k, k));
    for (int r = k + 1; r < NU; ++r) {
      const double v = fabs(A(r, k));
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv |= (uint64_t)p << (4 * k);
    if (p != k)
      for (int c = 0; c < NU; ++c) {
        const double t = A(k, c);
        A(k, c) = A(p, c);
        A(p, c) = t;
      }
    const double pv = A(k, k);
    if (!(pv != 0.0) || !isfinite(pv)) ok = false;
    const double ip = 1.0 / pv;
    A(k, k) = 1.0;
    for (int c = 0; c < NU; ++c) A(k, c) *= ip;
    for (int r = 0; r < NU; ++r) {
      if (r == k) continue;
      const double f = A(r, k);
      A(r, k) = 0.0;
      for (int c = 0; c < NU; ++c) A(r, c) -= f * A(k, c);
    }
  }
  for (int k = NU - 1; k >= 0; --k) {
    const int p = (int)((piv >> (4 * k)) & 15u);
    if (p != k)
      for (int r = 0; r < NU; ++r) {
        const double t = A(r, k);
        A(r, k) = A(r, p);
        A(r, p) = t;
      }
  }
  return ok;
}

// lambda_K = lscale ||A_K||_inf over the interior rows/columns, for K in M1 (Section 3.2 item 7)
template <int D, class M>
__device__ __forceinline__ void ns_lambda_elem(int64_t ne, int64_t k, const double* __restrict__ ecoord,
                                               uint32_t fl, const int32_t* __restrict__ eface,
                                               const double* __restrict__ ulin, double mu, double nu, double lscale,
                                               const Bnd& bnd, const M& A, double* __restrict__ lam) {
  constexpr int NU = NsPack<D>::NU;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  double Ub[D + 1][D], Nuu[D + 1][D], Gb[D + 1][D], Rb[D + 1][D];
  load_bnd<D>(bnd, fl, ne, k, Gb);
  load_ubar<D>(ulin, eface, fl, ne, k, Gb, Ub);
  ns_local<D>(g, fl, Ub, mu, nu, A, Nuu, Gb, Rb);
  double mx = 0.0;
#pragma unroll
  for (int r = 0; r < NU; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NU; ++c) s += interior(fl, c / D) ? fabs(A(r, c)) : 0.0;
    mx = interior(fl, r / D) ? fmax(mx, s) : mx;
  }
  lam[k] = lscale * mx;
}

__global__ void __launch_bounds__(BS) k_ns_lambda(int64_t ne, const double* __restrict__ ecoord,
                                                  const uint32_t* __restrict__ eflags,
                                                  const int32_t* __restrict__ eface,
                                                  const double* __restrict__ ulin, double mu, double nu,
                                                  double lscale, Bnd bnd, double* __restrict__ lam) {
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  const uint32_t fl = eflags[k];
  if (!(fl & F_M1)) {
    lam[k] = 0.0;
    return;
  }
  double A[6][6];
  ns_lambda_elem<2>(ne, k, ecoord, fl, eface, ulin, mu, nu, lscale, bnd, RegMat<6>{A}, lam);
}

// threads per block of the 3D Newton-step element kernels (LDS: 144 doubles per thread)
constexpr int BS_NS3 = 64;
constexpr size_t LDS_NS3 = sizeof(double) * 144 * BS_NS3;

__global__ void __launch_bounds__(BS_NS3) k_ns_lambda3(int64_t ne, const double* __restrict__ ecoord,
                                                       const uint32_t* __restrict__ eflags,
                                                       const int32_t* __restrict__ eface,
                                                       const double* __restrict__ ulin, double mu, double nu,
                                                       double lscale, Bnd bnd, double* __restrict__ lam) {
  extern __shared__ double lds_ns[];
  int64_t k = (int64_t)blockIdx.x * BS_NS3 + threadIdx.x;
  if (k >= ne) return;
  const uint32_t fl = eflags[k];
  if (!(fl & F_M1)) {
    lam[k] = 0.0;
    return;
  }
  ns_lambda_elem<3>(ne, k, ecoord, fl, eface, ulin, mu, nu, lscale, bnd, LdsMat<12>{lds_ns + threadIdx.x, BS_NS3},
                    lam);
}

// Stokes steady (mu = 0) lambda: same rule with the Stokes element matrix
template <int D>
__global__ void __launch_bounds__(BS) k_stokes_lambda(int64_t ne, const double* __restrict__ ecoord,
                                                      const uint32_t* __restrict__ eflags, double mu, double nu,
                                                      double lscale, double* __restrict__ lam) {
  constexpr int N = D + 1;
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  const uint32_t fl = eflags[k];
  if (!(fl & F_M1)) {
    lam[k] = 0.0;
    return;
  }
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const double m = mu * g.vol / N, iv = nu / g.vol;
  double mx = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) v += g.a[j][i] * g.a[l][i];
      v = iv * v + (j == l ? m : 0.0);
      s += interior(fl, l) ? fabs(v) : 0.0;
    }
    mx = interior(fl, j) ? fmax(mx, s) : mx;
  }
  lam[k] = lscale * mx;
}

struct NsFactors {
  double Ai[6][6];
  double l[6], r[6];
  double invB;
};

__device__ __forceinline__ void load_ns_pack(const double* __restrict__ pack, int64_t ne, int64_t k, NsFactors& F) {
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) F.Ai[a][b] = pack[(int64_t)(a * 6 + b) * ne + k];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    F.l[a] = pack[(int64_t)(36 + a) * ne + k];
    F.r[a] = pack[(int64_t)(42 + a) * ne + k];
  }
  F.invB = pack[(int64_t)48 * ne + k];
}

// a1 + a2, 2D Newton step: A^_K = A_K + E_K (E_K from the M1/M2 partition when
// mu = 0), general inverse, l = A^{-1} D, r = A^{-t} D, B = D^t A^{-1} D, and
// s_K = C (A^{-1} R - l (r^t R) / B).
__global__ void __launch_bounds__(BS) k_elim_ns(int64_t ne, const double* __restrict__ ecoord,
                                                const uint32_t* __restrict__ eflags,
                                                const int32_t* __restrict__ eface,
                                                const int32_t* __restrict__ enb, const double* __restrict__ lam,
                                                const double* __restrict__ fbar, const double* __restrict__ uprev,
                                                const double* __restrict__ ulin, double mu, double nu, Bnd bnd,
                                                double* __restrict__ pack, double* __restrict__ RK,
                                                double* __restrict__ sK, int32_t* err) {
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  Geo<2> g;
  load_geometry<2>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  double Ub[3][2], A[6][6], Nuu[3][2], Gb[3][2], Rb[3][2];
  load_bnd<2>(bnd, fl, ne, k, Gb);
  load_ubar<2>(ulin, eface, fl, ne, k, Gb, Ub);
  bool fin = true;
#pragma unroll
  for (int j = 0; j < 3; ++j) fin = fin && isfinite(Ub[j][0]) && isfinite(Ub[j][1]);
  ns_local<2>(g, fl, Ub, mu, nu, RegMat<6>{A}, Nuu, Gb, Rb);
  if (lam != nullptr) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double e = 0.0;
      if (fl & F_M1) {
        e = -lam[k];
      } else {
        int nb = enb[j * ne + k];
        if (nb >= 0 && (eflags[nb] & F_M1)) e = lam[nb];
      }
      if (interior(fl, j)) {
        A[j * 2][j * 2] += e;
        A[j * 2 + 1][j * 2 + 1] += e;
      }
    }
  }
  NsFactors F;
  bool ok = gj_inverse<6, true>(A, F.Ai);
  double Dv[6];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i) Dv[j * 2 + i] = interior(fl, j) ? -g.a[j][i] : 0.0;
  double B = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double lv = 0.0, rv = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      lv += F.Ai[a][b] * Dv[b];
      rv += F.Ai[b][a] * Dv[b];
    }
    F.l[a] = lv;
    F.r[a] = rv;
    B += Dv[a] * lv;
  }
  if (!ok || !isfinite(B) || !(fabs(B) > 0.0)) report(err, ERR_SINGULAR, k);
  const bool k0 = fl & F_K0;
  F.invB = k0 ? 0.0 : 1.0 / B;
  if (k0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) F.l[a] = F.r[a] = 0.0;
  }
  // right-hand side: eq. defrhs + Newton completion + transient lumped mass
  double fb[2] = {fbar[k * 2], fbar[k * 2 + 1]};
  fin = fin && isfinite(fb[0]) && isfinite(fb[1]);
  double R[6];
  const double m = mu * g.vol / 3.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double proj = 0.5 * (fb[0] * (g.xK[0] - g.X[j][0]) + fb[1] * (g.xK[1] - g.X[j][1]));
    bool in = interior(fl, j);
    int f = in ? eface[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double rr = g.a[j][i] * proj + Nuu[j][i] + Rb[j][i];
      if (uprev != nullptr && in) rr += m * uprev[(int64_t)f * 2 + i];
      R[j * 2 + i] = in ? rr : 0.0;
    }
  }
  if (!fin) report(err, ERR_NONFINITE, k);
  // divergence right-hand side of the boundary data: e_K = -D_K[bnd] . g = a . g
  double ediv = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 2; ++i) ediv += g.a[j][i] * Gb[j][i];
  if (bnd.ek != nullptr) bnd.ek[k] = ediv;
  double rR = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) rR += F.r[a] * R[a];
  rR = (rR - ediv) * F.invB;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) t += F.Ai[a][b] * R[b];
    RK[(int64_t)a * ne + k] = R[a];
    sK[(int64_t)a * ne + k] = csign(fl, a / 2) * (t - F.l[a] * rR);
  }
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b < 6; ++b) pack[(int64_t)(a * 6 + b) * ne + k] = F.Ai[a][b];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    pack[(int64_t)(36 + a) * ne + k] = F.l[a];
    pack[(int64_t)(42 + a) * ne + k] = F.r[a];
  }
  pack[(int64_t)48 * ne + k] = F.invB;
}

// a1 + a2, 3D Newton step: as k_elim_ns with the 12 x 12 local matrix of a
// tetrahedron, built and inverted (partial pivoting) in the thread's column of
// an LDS array, since it does not fit in registers with its inverse.
__global__ void __launch_bounds__(BS_NS3) k_elim_ns3(int64_t ne, const double* __restrict__ ecoord,
                                                     const uint32_t* __restrict__ eflags,
                                                     const int32_t* __restrict__ eface,
                                                     const int32_t* __restrict__ enb, const double* __restrict__ lam,
                                                     const double* __restrict__ fbar,
                                                     const double* __restrict__ uprev,
                                                     const double* __restrict__ ulin, double mu, double nu,
                                                     Bnd bnd, double* __restrict__ pack, double* __restrict__ RK,
                                                     double* __restrict__ sK, int32_t* err) {
  constexpr int D = 3, N = 4, NU = 12;
  extern __shared__ double lds_ns[];
  int64_t k = (int64_t)blockIdx.x * BS_NS3 + threadIdx.x;
  if (k >= ne) return;
  const LdsMat<NU> A{lds_ns + threadIdx.x, BS_NS3};
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  double Ub[N][D], Nuu[N][D], Gb[N][D], Rb[N][D];
  load_bnd<D>(bnd, fl, ne, k, Gb);
  load_ubar<D>(ulin, eface, fl, ne, k, Gb, Ub);
  bool fin = true;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) fin = fin && isfinite(Ub[j][i]);
  ns_local<D>(g, fl, Ub, mu, nu, A, Nuu, Gb, Rb);
  if (lam != nullptr) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double e = 0.0;
      if (fl & F_M1) {
        e = -lam[k];
      } else {
        int nb = enb[j * ne + k];
        if (nb >= 0 && (eflags[nb] & F_M1)) e = lam[nb];
      }
      if (interior(fl, j))
#pragma unroll
        for (int i = 0; i < D; ++i) A(j * D + i, j * D + i) += e;
    }
  }
  const bool ok = gj_inverse_inplace<NU>(A);
  double Dv[NU], lv[NU], rv[NU];
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) Dv[j * D + i] = interior(fl, j) ? -g.a[j][i] : 0.0;
  double B = 0.0;
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    double l = 0.0, r = 0.0;
#pragma unroll
    for (int b = 0; b < NU; ++b) {
      l += A(a, b) * Dv[b];
      r += A(b, a) * Dv[b];
    }
    lv[a] = l;
    rv[a] = r;
    B += Dv[a] * l;
  }
  if (!ok || !isfinite(B) || !(fabs(B) > 0.0)) report(err, ERR_SINGULAR, k);
  const bool k0 = fl & F_K0;
  const double invB = k0 ? 0.0 : 1.0 / B;
  if (k0) {
#pragma unroll
    for (int a = 0; a < NU; ++a) lv[a] = rv[a] = 0.0;
  }
  // right-hand side: eq. defrhs + Newton completion + transient lumped mass
  double fb[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    fb[i] = fbar[k * D + i];
    fin = fin && isfinite(fb[i]);
  }
  double R[NU];
  const double m = mu * g.vol / N;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double proj = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) proj += fb[i] * (g.xK[i] - g.X[j][i]);
    proj *= 1.0 / D;
    bool in = interior(fl, j);
    int f = in ? eface[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double rr = g.a[j][i] * proj + Nuu[j][i] + Rb[j][i];
      if (uprev != nullptr && in) rr += m * uprev[(int64_t)f * D + i];
      R[j * D + i] = in ? rr : 0.0;
    }
  }
  if (!fin) report(err, ERR_NONFINITE, k);
  double ediv = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) ediv += g.a[j][i] * Gb[j][i];
  if (bnd.ek != nullptr) bnd.ek[k] = ediv;
  double rR = 0.0;
#pragma unroll
  for (int a = 0; a < NU; ++a) rR += rv[a] * R[a];
  rR = (rR - ediv) * invB;
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < NU; ++b) t += A(a, b) * R[b];
    RK[(int64_t)a * ne + k] = R[a];
    sK[(int64_t)a * ne + k] = csign(fl, a / D) * (t - lv[a] * rR);
  }
  for (int a = 0; a < NU; ++a)
    for (int b = 0; b < NU; ++b) pack[(int64_t)(a * NU + b) * ne + k] = A(a, b);
#pragma unroll
  for (int a = 0; a < NU; ++a) {
    pack[(int64_t)(NU * NU + a) * ne + k] = lv[a];
    pack[(int64_t)(NU * NU + NU + a) * ne + k] = rv[a];
  }
  pack[(int64_t)(NU * NU + 2 * NU) * ne + k] = invB;
}

// ---------------------------------------------------------------------------
// a3: gather assembly of G (Section 3.2 item 5: G = sum_K H_K G_K H_K^t) into
// block-ELL, one thread per interior face row f.  Slot 0 is the diagonal block
// (sum over the two elements of f); slots 1..d the other faces of the owner K
// in local order, slots d+1..2d those of the other element L.  Exterior faces
// give a zero block pointing at f itself.  Writes the unscaled G, S, and the
// Jacobi scale dsq = sqrt|diag G|; a second pass scales.
//   Stokes: G_K[(j,i),(l,i')] = c_j c_l (delta_ii' S^{-1}_jl - V_ji V_li' / B)
//   NS:     G_K[(j,i),(l,i')] = c_j c_l (A^{-1}[(j,i),(l,i')] - l_(j,i) r_(l,i') / B)
// ---------------------------------------------------------------------------
template <int D, bool NSK>
struct BlockSrc;

template <int D>
struct BlockSrc<D, false> {
  StokesFactors<D> F;
  __device__ void load(const double* pack, int64_t ne, int64_t k) { load_stokes_pack<D>(pack, ne, k, F); }
  __device__ double g(int j, int i, int l, int ip) const {
    return (i == ip ? F.Si[j][l] : 0.0) - F.V[j][i] * F.V[l][ip] * F.invB;
  }
};

// Newton step, any d: entries read from the pack where they are used (the 3D
// pack holds 169 numbers per element)
template <int D>
struct BlockSrc<D, true> {
  static constexpr int NU = NsPack<D>::NU;
  const double* pack;
  int64_t ne, k;
  double invB;
  __device__ void load(const double* p, int64_t n, int64_t kk) {
    pack = p;
    ne = n;
    k = kk;
    invB = pack[(int64_t)(NU * NU + 2 * NU) * ne + k];
  }
  __device__ double g(int j, int i, int l, int ip) const {
    const int a = j * D + i, b = l * D + ip;
    return pack[(int64_t)(a * NU + b) * ne + k] -
           pack[(int64_t)(NU * NU + a) * ne + k] * pack[(int64_t)(NU * NU + NU + b) * ne + k] * invB;
  }
};

template <>
struct BlockSrc<2, true> {
  NsFactors F;
  __device__ void load(const double* pack, int64_t ne, int64_t k) { load_ns_pack(pack, ne, k, F); }
  __device__ double g(int j, int i, int l, int ip) const {
    return F.Ai[j * 2 + i][l * 2 + ip] - F.l[j * 2 + i] * F.r[l * 2 + ip] * F.invB;
  }
};

// FULL = false: only the diagonal blocks (for the Jacobi scale), S and the
// column table; the block rows of G (G may be NULL) are not written.
template <int D, bool NSK, bool FULL = true>
__global__ void __launch_bounds__(BS) k_face_assemble(int64_t nf, int64_t ne, const int32_t* __restrict__ fel,
                                                      const int32_t* __restrict__ floc,
                                                      const int32_t* __restrict__ eface,
                                                      const uint32_t* __restrict__ eflags,
                                                      const double* __restrict__ pack,
                                                      const double* __restrict__ sK, int32_t* __restrict__ cols,
                                                      double* __restrict__ G, double* __restrict__ dsq,
                                                      double* __restrict__ bs, int32_t* err) {
  constexpr int N = D + 1, DD = D * D;
  int64_t f = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (f >= nf) return;
  const int64_t e2[2] = {fel[f], fel[nf + f]};
  const int lc = floc[f];
  const int jj[2] = {lc & 0xff, (lc >> 8) & 0xff};
  double diag[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int ip = 0; ip < D; ++ip) diag[i][ip] = 0.0;
  double Sf[D];
#pragma unroll
  for (int i = 0; i < D; ++i) Sf[i] = 0.0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t K = e2[side];
    const int j = jj[side];
    BlockSrc<D, NSK> src;
    src.load(pack, ne, K);
    const uint32_t fl = eflags[K];
    const double cj = csign(fl, j);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Sf[i] += sK[(int64_t)(j * D + i) * ne + K];
#pragma unroll
      for (int ip = 0; ip < D; ++ip) diag[i][ip] += src.g(j, i, j, ip);
    }
    int slot = 1 + side * D;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      if (l == j) continue;
      const bool in = interior(fl, l);
      const int64_t col = in ? eface[l * ne + K] : f;
      const double c = cj * csign(fl, l);
      cols[(int64_t)(slot - 1) * nf + f] = (int32_t)col;
      if constexpr (FULL) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int ip = 0; ip < D; ++ip) {
            G[(int64_t)(slot * DD + i * D + ip) * nf + f] = in ? c * src.g(j, i, l, ip) : 0.0;
          }
      }
      ++slot;
    }
  }
  // one Jacobi scale per face, sqrt of the mean |diagonal| over its d components
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if constexpr (FULL) {
#pragma unroll
      for (int ip = 0; ip < D; ++ip) G[(int64_t)(i * D + ip) * nf + f] = diag[i][ip];
    }
    const double dg = fabs(diag[i][i]);
    if (!(dg > 0.0) || !isfinite(dg)) report(err, ERR_ZERODIAG, f);
    dsum += dg;
  }
  const double sq = sqrt(dsum / D);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    dsq[f * D + i] = sq;
    bs[f * D + i] = Sf[i] / sq;
  }
}

// l = A^_K^{-1} D_K and 1/B_K of K0 (the pack stores zeros for K0), from its
// geometry and the stored inverse: D_K = -a restricted to interior faces.
template <int D>
__device__ __forceinline__ void k0_schur(const double* __restrict__ ecoord, int64_t ne, int64_t k, uint32_t fl,
                                         StokesFactors<D>& F) {
  constexpr int N = D + 1;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  double B = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) v -= F.Si[j][l] * (interior(fl, l) ? g.a[l][i] : 0.0);
      F.V[j][i] = v;
      B -= (interior(fl, j) ? g.a[j][i] : 0.0) * v;
    }
  F.invB = 1.0 / B;
}

// Element factors of the scaled Stokes operator (EfoLayout, rowkern.h) from
// the Stokes pack and the face scales, one thread per element; FP64 and an
// FP32 rounding.  egat[l] is the face of local face l, or any interior face of
// the element for an exterior one (its weights are zero).  K0 gets its Schur
// term like every other element: the operator of the element form is
// G' = G - u u^t / B_K0 with u = C_K0 l_K0, whose null vector is z
// (C_K z_K = -D_K on every element).
template <int D>
__global__ void __launch_bounds__(BS) k_efo_build(int64_t ne, const double* __restrict__ pack,
                                                  const double* __restrict__ ecoord,
                                                  const int32_t* __restrict__ eface,
                                                  const uint32_t* __restrict__ eflags,
                                                  const double* __restrict__ dsq, double* __restrict__ F64,
                                                  float* __restrict__ F32, int32_t* __restrict__ egat) {
  using L = EfoLayout<D>;
  constexpr int N = D + 1;
  const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  StokesFactors<D> F;
  load_stokes_pack<D>(pack, ne, k, F);
  const uint32_t fl = eflags[k];
  if (fl & F_K0) k0_schur<D>(ecoord, ne, k, fl, F);
  int32_t fc[N], any = -1;
  double wl[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    fc[l] = eface[(int64_t)l * ne + k];
    const bool in = interior(fl, l);
    if (in && any < 0) any = fc[l];
    wl[l] = in ? csign(fl, l) / dsq[(int64_t)fc[l] * D] : 0.0;
  }
  const double rb = sqrt(F.invB);
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int l = j; l < N; ++l) {
      const double v = wl[j] * wl[l] * F.Si[j][l];
      F64[(int64_t)L::tri(j, l) * ne + k] = v;
      F32[(int64_t)L::tri(j, l) * ne + k] = (float)v;
    }
#pragma unroll
  for (int l = 0; l < N; ++l)
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double v = wl[l] * F.V[l][i] * rb;
      F64[(int64_t)L::vh(l, i) * ne + k] = v;
      F32[(int64_t)L::vh(l, i) * ne + k] = (float)v;
    }
#pragma unroll
  for (int l = 0; l < N; ++l) egat[(int64_t)l * ne + k] = interior(fl, l) ? fc[l] : any;
}

// Null vector of G' in scaled variables: zy_f = dsq_f a_{K,f}, K the owner
// (C = +1) element of face f.
template <int D>
__global__ void __launch_bounds__(BS) k_zvec(int64_t nf, int64_t ne, const int32_t* __restrict__ fel,
                                             const int32_t* __restrict__ floc, const double* __restrict__ ecoord,
                                             const double* __restrict__ dsq, double* __restrict__ zy) {
  const int64_t f = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (f >= nf) return;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, fel[f], g);
  const int j = floc[f] & 0xff;
#pragma unroll
  for (int i = 0; i < D; ++i) zy[f * D + i] = dsq[f * D + i] * g.a[j][i];
}

// Divergence data eps of K0's row in the gauge-shifted system.  G W = S has
// no divergence row at K0, so eps is free; z^t S' = 0 (the consistency of
// G' W' = S', z the null vector of G') holds exactly when
// eps = -sum_{K != K0} e_K, the flux that K0 takes up.  Without boundary data
// eps = 0.  One workgroup, fixed summation order.
__global__ void __launch_bounds__(256) k_k0_eps(int64_t ne, int64_t k0, const double* __restrict__ ek,
                                                double* __restrict__ eps) {
  __shared__ double red[256];
  double v = 0.0;
  if (ek != nullptr)
    for (int64_t k = threadIdx.x; k < ne; k += 256) v += k == k0 ? 0.0 : ek[k];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) eps[0] = -red[0];
}

// Right-hand side of the element form: S' = S - u (l_K0^t R_K0 - eps) / B_K0,
// a change on the faces of K0 only (bs1 holds a copy of the scaled S).  One
// thread.
template <int D>
__global__ void k_k0_rhs(int64_t ne, int64_t k, const double* __restrict__ pack, const double* __restrict__ ecoord,
                         const int32_t* __restrict__ eface, const uint32_t* __restrict__ eflags,
                         const double* __restrict__ RK, const double* __restrict__ dsq, const double* __restrict__ eps,
                         double* __restrict__ bs1) {
  constexpr int N = D + 1;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  StokesFactors<D> F;
  load_stokes_pack<D>(pack, ne, k, F);
  const uint32_t fl = eflags[k];
  k0_schur<D>(ecoord, ne, k, fl, F);
  double rho = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < D; ++i)
      if (interior(fl, j)) rho += F.V[j][i] * RK[(int64_t)(j * D + i) * ne + k];
  rho -= eps[0];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (!interior(fl, j)) continue;
    const int64_t f = eface[(int64_t)j * ne + k];
#pragma unroll
    for (int i = 0; i < D; ++i) bs1[f * D + i] -= csign(fl, j) * F.V[j][i] * rho * F.invB / dsq[f * D + i];
  }
}

// Gauge shift: for a solution W' of G' W' = S', W = W' + t z solves G W = S
// with t = -P_K0(W'), P_K0(W') = (l^t (R - C W') - eps) / B at K0.  One
// thread writes t.
template <int D>
__global__ void k_k0_gauge(int64_t ne, int64_t k, const double* __restrict__ pack, const double* __restrict__ ecoord,
                           const int32_t* __restrict__ eface, const uint32_t* __restrict__ eflags,
                           const double* __restrict__ RK, const double* __restrict__ y,
                           const double* __restrict__ dsq, const double* __restrict__ eps, double* __restrict__ t) {
  constexpr int N = D + 1;
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  StokesFactors<D> F;
  load_stokes_pack<D>(pack, ne, k, F);
  const uint32_t fl = eflags[k];
  k0_schur<D>(ecoord, ne, k, fl, F);
  double p = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (!interior(fl, j)) continue;
    const int64_t f = eface[(int64_t)j * ne + k];
#pragma unroll
    for (int i = 0; i < D; ++i)
      p += F.V[j][i] * (RK[(int64_t)(j * D + i) * ne + k] - csign(fl, j) * y[f * D + i] / dsq[f * D + i]);
  }
  t[0] = -(p - eps[0]) * F.invB;
}

// ---------------------------------------------------------------------------
// Coarse correction of the element-form CG.  Columns of Z: the null vector z of
// G' restricted to the faces of one aggregate of elements (a constant pressure
// on the aggregate, seen through the faces it owns).  E = Z^t G' Z is summed
// element by element: entry (a, b) collects, for every element K and local
// faces j, l with faces in aggregates a and b, z_j^t G'_K[j, l] z_l =
// Sh_jl (z_j . z_l) - (Vh_j . z_j)(Vh_l . z_l) in the scaled variables.  One
// wavefront per nonzero, lanes over its entry list, a fixed-order reduction.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_coarse_E(int32_t npairs, const int32_t* __restrict__ pair_ptr,
                                                  const int32_t* __restrict__ pair_key,
                                                  const int32_t* __restrict__ pair_ent, int64_t ne,
                                                  const double* __restrict__ F, const int32_t* __restrict__ egat,
                                                  const double* __restrict__ zy, double* __restrict__ E) {
  using L = EfoLayout<D>;
  const int w = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= npairs) return;
  double acc = 0.0;
  for (int32_t e = pair_ptr[w] + lane; e < pair_ptr[w + 1]; e += 64) {
    const int32_t code = pair_ent[e];
    const int64_t k = code >> 4;
    const int j = (code >> 2) & 3, l = code & 3;
    const int64_t fj = egat[(int64_t)j * ne + k], fl = egat[(int64_t)l * ne + k];
    double zz = 0.0, vj = 0.0, vl = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double a = zy[fj * D + i], b = zy[fl * D + i];
      zz += a * b;
      vj += F[(int64_t)L::vh(j, i) * ne + k] * a;
      vl += F[(int64_t)L::vh(l, i) * ne + k] * b;
    }
    acc += F[(int64_t)L::sym(j, l) * ne + k] * zz - vj * vl;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) E[pair_key[w]] = acc;
}

// Inverse of E + s 1 1^t (s = trace(E) / m; E is positive semi-definite with
// null vector 1, since the columns of Z sum to z) by Gauss-Jordan without
// pivoting, for m a multiple of GJB = 32 (m > 128; the smaller ones are
// inverted in LDS below): in place, by 32 x 32 pivot blocks, on A = E + s 1 1^t
// (held in Einv).  For pivot block K, with P = A_KK^-1 (one workgroup, in LDS),
// T = P A_K* (the block row) and C = A_*K (the block column, copied first):
//   A_ij -= C_iK T_Kj (i, j not in K),  A_iK = -C_iK P,  A_Kj = T_Kj,  A_KK = P;
// after the last block A holds the inverse: m / 32 steps of three launches.  A
// pivot that is not positive sets the flag and leaves a zero inverse (the
// correction then does nothing).
constexpr int GJB = 32;

__global__ void __launch_bounds__(1024) k_gjb_init(int m, const double* __restrict__ E, double* __restrict__ A,
                                                   double* __restrict__ flag) {
  __shared__ double red[16];
  double tr = 0.0;
  for (int i = threadIdx.x; i < m; i += 1024) tr += E[(int64_t)i * m + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k];
    red[0] = t / m;
  }
  __syncthreads();
  const double sh = red[0];
  for (int64_t q = threadIdx.x; q < (int64_t)m * m; q += 1024) A[q] = E[q] + sh;
  if (threadIdx.x == 0) flag[0] = 0.0;
}

// P = A_KK^-1 by unblocked Gauss-Jordan in LDS; one workgroup of GJB * GJB threads
__global__ void __launch_bounds__(GJB * GJB) k_gjb_pivot(int m, int K0, const double* __restrict__ A,
                                                        double* __restrict__ P, double* __restrict__ flag) {
  __shared__ double B[GJB][GJB];
  __shared__ double fac[GJB];
  __shared__ int bad;
  const int r = threadIdx.x / GJB, c = threadIdx.x % GJB;
  B[r][c] = A[(int64_t)(K0 + r) * m + K0 + c];
  if (threadIdx.x == 0) bad = flag[0] != 0.0;
  __syncthreads();
  for (int k = 0; k < GJB; ++k) {
    const double piv = B[k][k];
    if (bad || !(piv > 0.0) || !isfinite(piv)) {
      if (threadIdx.x == 0) bad = 1;
      break;
    }
    if (c == 0) fac[r] = B[r][k];
    __syncthreads();
    const double ip = 1.0 / piv;
    if (r == k) B[k][c] = (c == k ? 1.0 : B[k][c]) * ip;
    __syncthreads();
    if (r != k) B[r][c] = (c == k ? 0.0 : B[r][c]) - fac[r] * B[k][c];
    __syncthreads();
  }
  __syncthreads();
  P[r * GJB + c] = B[r][c];
  if (threadIdx.x == 0 && bad) flag[0] = 1.0;
}

// T = P A_K* (GJB x m) and C = A_*K (m x GJB); one thread per entry of each
__global__ void __launch_bounds__(256) k_gjb_panel(int m, int K0, const double* __restrict__ A,
                                                   const double* __restrict__ P, double* __restrict__ T,
                                                   double* __restrict__ C) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)GJB * m;
  if (q < n) {
    const int l = (int)(q / m), j = (int)(q % m);
    double v = 0.0;
#pragma unroll 8
    for (int t = 0; t < GJB; ++t) v += P[l * GJB + t] * A[(int64_t)(K0 + t) * m + j];
    T[q] = v;
  } else if (q < 2 * n) {
    const int64_t u = q - n;
    const int i = (int)(u / GJB), l = (int)(u % GJB);
    C[u] = A[(int64_t)i * m + K0 + l];
  }
}

// the update of every entry of A for pivot block K; 16 x 16 tiles (a tile lies
// wholly inside or outside K in either direction), C and T (or P) staged in LDS
__global__ void __launch_bounds__(256) k_gjb_update(int m, int K0, double* __restrict__ A,
                                                    const double* __restrict__ P, const double* __restrict__ T,
                                                    const double* __restrict__ C, const double* __restrict__ flag) {
  __shared__ double Cs[16][GJB + 1];
  __shared__ double Ts[GJB][16 + 1];
  if (flag[0] != 0.0) return;
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int i = i0 + ti, j = j0 + tj;
  const bool rowK = i0 >= K0 && i0 < K0 + GJB, colK = j0 >= K0 && j0 < K0 + GJB;
  if (rowK) {
    A[(int64_t)i * m + j] = colK ? P[(i - K0) * GJB + (j - K0)] : T[(int64_t)(i - K0) * m + j];
    return;
  }
  for (int q = threadIdx.x; q < 16 * GJB; q += 256) {
    const int a = q / GJB, l = q % GJB;
    Cs[a][l] = C[(int64_t)(i0 + a) * GJB + l];
    const int lb = q / 16, b = q % 16;
    Ts[lb][b] = colK ? P[lb * GJB + (j0 - K0 + b)] : T[(int64_t)lb * m + j0 + b];
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll 8
  for (int l = 0; l < GJB; ++l) acc += Cs[ti][l] * Ts[l][tj];
  double* a = A + (int64_t)i * m + j;
  *a = colK ? -acc : *a - acc;
}

// zero inverse after a bad pivot; else make it exactly symmetric (the blocked
// updates leave a relative asymmetry near 1e-13, and CG wants a symmetric
// preconditioner): the thread of (i, j), i < j, writes the mean of the pair to
// both entries
__global__ void __launch_bounds__(256) k_gjb_final(int m, const double* __restrict__ flag, double* __restrict__ A) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (int64_t)m * m) return;
  if (flag[0] != 0.0) {
    A[q] = 0.0;
    return;
  }
  const int i = (int)(q / m), j = (int)(q % m);
  if (i >= j) return;
  const int64_t t = (int64_t)j * m + i;
  const double v = 0.5 * (A[q] + A[t]);
  A[q] = v;
  A[t] = v;
}

// The same inverse for m <= 128 with E held in LDS (m^2 doubles, at most
// 128 KB) and inverted in place: for each pivot k, row k is divided by the
// pivot (its diagonal entry becoming 1 / pivot) and eliminated from every
// other row (their column-k entries becoming -factor / pivot).
__global__ void __launch_bounds__(1024) k_coarse_inv_lds(int m, const double* __restrict__ E,
                                                         double* __restrict__ Einv) {
  extern __shared__ double A[];
  __shared__ double fac[128];
  __shared__ double s_tr;
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < m; ++i) tr += E[(int64_t)i * m + i];
    s_tr = tr / m;
    bad = 0;
  }
  __syncthreads();
  for (int q = t; q < m * m; q += 1024) A[q] = E[q] + s_tr;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const double piv = A[k * m + k];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (t == 0) bad = 1;
      break;
    }
    if (t < m) fac[t] = A[t * m + k];
    __syncthreads();
    const double ip = 1.0 / piv;
    if (t < m) A[k * m + t] = (t == k ? 1.0 : A[k * m + t]) * ip;
    __syncthreads();
    for (int q = t; q < m * m; q += 1024) {
      const int i = q / m, c = q % m;
      if (i == k) continue;
      const double rk = A[k * m + c];
      A[q] = (c == k ? 0.0 : A[q]) - fac[i] * rk;
    }
    __syncthreads();
  }
  __syncthreads();
  for (int q = t; q < m * m; q += 1024) Einv[q] = bad ? 0.0 : A[q];
}

__global__ void __launch_bounds__(BS) k_cast_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void __launch_bounds__(BS) k_gauge_axpy(int64_t n, const double* __restrict__ t,
                                                   const double* __restrict__ zy, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) y[i] += t[0] * zy[i];
}

// scale G by dsq on both sides and round a copy to FP32
template <int D>
__global__ void __launch_bounds__(BS) k_face_scale(int64_t nf, const int32_t* __restrict__ cols,
                                                   const double* __restrict__ dsq, double* __restrict__ G,
                                                   float* __restrict__ G32) {
  constexpr int DD = D * D;
  int64_t f = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (f >= nf) return;
  double rs[D];
#pragma unroll
  for (int i = 0; i < D; ++i) rs[i] = 1.0 / dsq[f * D + i];
#pragma unroll
  for (int s = 0; s <= 2 * D; ++s) {
    const int64_t c = s == 0 ? f : (int64_t)cols[(int64_t)(s - 1) * nf + f];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int ip = 0; ip < D; ++ip) {
        const int64_t idx = (int64_t)(s * DD + i * D + ip) * nf + f;
        const double v = G[idx] * rs[i] / dsq[c * D + ip];
        G[idx] = v;
        G32[idx] = (float)v;
      }
  }
}

// S re-gather for a new right-hand side (a6)
template <int D>
__global__ void __launch_bounds__(BS) k_face_rhs(int64_t nf, int64_t ne, const int32_t* __restrict__ fel,
                                                 const int32_t* __restrict__ floc, const double* __restrict__ sK,
                                                 const double* __restrict__ dsq, double* __restrict__ bs) {
  int64_t f = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (f >= nf) return;
  const int64_t K = fel[f], L = fel[nf + f];
  const int lc = floc[f];
  const int jK = lc & 0xff, jL = (lc >> 8) & 0xff;
#pragma unroll
  for (int i = 0; i < D; ++i)
    bs[f * D + i] = (sK[(int64_t)(jK * D + i) * ne + K] + sK[(int64_t)(jL * D + i) * ne + L]) / dsq[f * D + i];
}

// ---------------------------------------------------------------------------
// a5: recovery, one thread per element.  W_K from the resident scaled solution
// y = dsq * W.  P_K = r_K^t (R_K - C_K W_K) / B_K, U^_K = A^_K^{-1}(R_K - C_K W_K) - P_K l_K.
// The copy with C = +1 is written to U (canonical order); the other copy goes
// to Ujump for the mismatch diagnostic.
// ---------------------------------------------------------------------------
// One element of the recovery: its pressure p and the velocity copies u of
// its faces; fc[j] is the canonical id of local face j (-1: exterior).
template <int D, bool NSK>
__device__ __forceinline__ void recover_element(int64_t ne, int64_t k, uint32_t fl, const double* __restrict__ y,
                                                const double* __restrict__ dsq, const double* __restrict__ pack,
                                                const double* __restrict__ RK, const double* __restrict__ ek,
                                                const int32_t* __restrict__ eface,
                                                const int32_t* __restrict__ fcanon, double (&u)[D + 1][D],
                                                double& p, int (&fc)[D + 1]) {
  constexpr int N = D + 1;
  double rhs[N][D];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool in = interior(fl, j);
    const int64_t f = in ? eface[j * ne + k] : 0;
    fc[j] = in ? fcanon[f] : -1;
    const double c = csign(fl, j);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double w = in ? y[f * D + i] / dsq[f * D + i] : 0.0;
      rhs[j][i] = RK[(int64_t)(j * D + i) * ne + k] - c * w;
    }
  }
  p = 0.0;
  if constexpr (!NSK) {
    StokesFactors<D> F;
    load_stokes_pack<D>(pack, ne, k, F);
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < D; ++i) p += F.V[j][i] * rhs[j][i];
    if (ek != nullptr) p -= ek[k];
    p *= F.invB;
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) t += F.Si[j][l] * rhs[l][i];
        u[j][i] = t - p * F.V[j][i];
      }
  } else {
    // pack: A^{-1} [NU][NU], l [NU], r [NU], 1/B
    constexpr int NU = NsPack<D>::NU;
#pragma unroll
    for (int a = 0; a < NU; ++a) p += pack[(int64_t)(NU * NU + NU + a) * ne + k] * rhs[a / D][a % D];
    if (ek != nullptr) p -= ek[k];
    p *= pack[(int64_t)(NU * NU + 2 * NU) * ne + k];
#pragma unroll
    for (int a = 0; a < NU; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < NU; ++b) t += pack[(int64_t)(a * NU + b) * ne + k] * rhs[b / D][b % D];
      u[a / D][a % D] = t - p * pack[(int64_t)(NU * NU + a) * ne + k];
    }
  }
}

template <int D, bool NSK>
__global__ void __launch_bounds__(BS) k_recover(int64_t ne, const double* __restrict__ y,
                                                const double* __restrict__ dsq, const double* __restrict__ pack,
                                                const double* __restrict__ RK, const double* __restrict__ ek,
                                                const int32_t* __restrict__ eface,
                                                const uint32_t* __restrict__ eflags,
                                                const int32_t* __restrict__ ecaller,
                                                const int32_t* __restrict__ fcanon, double* __restrict__ U,
                                                double* __restrict__ P, double* __restrict__ Ujump) {
  constexpr int N = D + 1;
  int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (k >= ne) return;
  const uint32_t fl = eflags[k];
  double u[N][D], p;
  int fc[N];
  recover_element<D, NSK>(ne, k, fl, y, dsq, pack, RK, ek, eface, fcanon, u, p, fc);
  P[ecaller[k]] = p;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (fc[j] < 0) continue;
    double* dst = csign(fl, j) > 0.0 ? U : Ujump;
    if (dst == nullptr) continue;
#pragma unroll
    for (int i = 0; i < D; ++i) dst[(int64_t)fc[j] * D + i] = u[j][i];
  }
}

// Copy mismatch without a second velocity array: after k_recover has written
// the owner copies to U, each element recomputes its copies and adds the
// squared difference of its non-owner copies (C = -1) to U; one partial per
// workgroup, part[blockIdx.x].
template <int D, bool NSK>
__global__ void __launch_bounds__(BS) k_recover_mismatch(int64_t ne, const double* __restrict__ y,
                                                         const double* __restrict__ dsq,
                                                         const double* __restrict__ pack,
                                                         const double* __restrict__ RK,
                                                         const double* __restrict__ ek,
                                                         const int32_t* __restrict__ eface,
                                                         const uint32_t* __restrict__ eflags,
                                                         const int32_t* __restrict__ fcanon,
                                                         const double* __restrict__ U, double* __restrict__ part) {
  constexpr int N = D + 1;
  __shared__ double sh[BS];
  const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
  double s = 0.0;
  if (k < ne) {
    const uint32_t fl = eflags[k];
    double u[N][D], p;
    int fc[N];
    recover_element<D, NSK>(ne, k, fl, y, dsq, pack, RK, ek, eface, fcanon, u, p, fc);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (fc[j] < 0 || csign(fl, j) > 0.0) continue;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double t = u[j][i] - U[(int64_t)fc[j] * D + i];
        s += t * t;
      }
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// initial W from a caller array in canonical order: y = dsq * W (internal order)
__global__ void __launch_bounds__(BS) k_import_w(int64_t n, int d, const int32_t* __restrict__ fcanon,
                                                 const double* __restrict__ dsq, const double* __restrict__ w0,
                                                 double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t >= n * d) return;
  const int64_t f = t / d;
  const int i = (int)(t - f * d);
  y[t] = dsq[t] * w0[(int64_t)fcanon[f] * d + i];
}

// the resident W in canonical order: W = y / dsq (inverse of k_import_w)
__global__ void __launch_bounds__(BS) k_export_w(int64_t n, int d, const int32_t* __restrict__ fcanon,
                                                 const double* __restrict__ dsq, const double* __restrict__ y,
                                                 double* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t >= n * d) return;
  const int64_t f = t / d;
  const int i = (int)(t - f * d);
  w[(int64_t)fcanon[f] * d + i] = y[t] / dsq[t];
}

// deterministic sum of squared differences: per-block partials then one block
__global__ void __launch_bounds__(256) k_sqdiff_partial(int64_t n, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double t = a[i] - b[i];
    s += t * t;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_sqrt(int n, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0]);
}

// input permutation gathers
__global__ void k_gather_rows(int64_t n, int width, const int32_t* __restrict__ idx, const double* __restrict__ src,
                              double* __restrict__ dst) {
  int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * width) return;
  int64_t r = t / width;
  int c = (int)(t - r * width);
  dst[t] = src[(int64_t)idx[r] * width + c];
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static cr_status read_err(cr_system* s, const char* stage) {
  int32_t h[2];
  cr_status st = check_hip(hipMemcpyAsync(h, s->err, sizeof h, hipMemcpyDeviceToHost, s->stream), stage);
  if (st != CR_OK) return st;
  st = check_hip(hipStreamSynchronize(s->stream), stage);
  if (st != CR_OK) return st;
  if (h[0] == 0) return CR_OK;
  int64_t id = h[1];
  if (h[0] & ERR_NONFINITE) {
    set_error("%s: non-finite input at internal index %lld", stage, (long long)id);
    return CR_E_NONFINITE;
  }
  if (h[0] & ERR_ZERODIAG) {
    set_error("%s: zero or non-finite diagonal of G (internal face %lld)", stage, (long long)id);
    return CR_E_SINGULAR;
  }
  int64_t caller = (id >= 0 && id < s->ne) ? s->topo.elem_iperm[id] : id;
  set_error("%s: singular local system or B_K not positive at element %lld", stage, (long long)caller);
  return CR_E_SINGULAR;
}

static cr_status reset_err(cr_system* s) {
  int32_t h[2] = {0, INT32_MAX};
  return check_hip(hipMemcpyAsync(s->err, h, sizeof h, hipMemcpyHostToDevice, s->stream), "reset error word");
}

static cr_status gather_inputs(cr_system* s, const double* f_mean, const double* u_prev, const double* u_lin) {
  const int d = s->d;
  if (f_mean) {
    hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(s->ne * d, 256)), dim3(256), 0, s->stream, s->ne, d, s->ecaller,
                       f_mean, s->fbar);
  }
  if (u_prev) {
    hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(s->nf * d, 256)), dim3(256), 0, s->stream, s->nf, d, s->fcanon,
                       u_prev, s->uprev);
  }
  if (u_lin) {
    hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(s->nf * d, 256)), dim3(256), 0, s->stream, s->nf, d, s->fcanon,
                       u_lin, s->ulin);
  }
  return check_hip(hipGetLastError(), "gather inputs");
}

// S' of the element form from the current S
static cr_status k0_rhs(cr_system* s) {
  cr_status st = check_hip(hipMemcpyAsync(s->bs1, s->bs, sizeof(double) * s->nf * s->d, hipMemcpyDeviceToDevice,
                                          s->stream), "element-form right-hand side");
  if (st != CR_OK) return st;
  hipLaunchKernelGGL(k_k0_eps, dim3(1), dim3(256), 0, s->stream, s->ne, s->k0i, s->has_bnd ? s->ek : nullptr,
                     s->k0eps);
  if (s->d == 2)
    hipLaunchKernelGGL(k_k0_rhs<2>, dim3(1), dim3(64), 0, s->stream, s->ne, s->k0i, s->pack, s->ecoord, s->eface,
                       s->eflags, s->RK, s->dsq, s->k0eps, s->bs1);
  else
    hipLaunchKernelGGL(k_k0_rhs<3>, dim3(1), dim3(64), 0, s->stream, s->ne, s->k0i, s->pack, s->ecoord, s->eface,
                       s->eflags, s->RK, s->dsq, s->k0eps, s->bs1);
  return check_hip(hipGetLastError(), "element-form right-hand side");
}

cr_status enqueue_gauge_fix(cr_system* s, hipStream_t stream) {
  if (s->d == 2)
    hipLaunchKernelGGL(k_k0_gauge<2>, dim3(1), dim3(64), 0, stream, s->ne, s->k0i, s->pack, s->ecoord, s->eface,
                       s->eflags, s->RK, s->y, s->dsq, s->k0eps, s->k0t);
  else
    hipLaunchKernelGGL(k_k0_gauge<3>, dim3(1), dim3(64), 0, stream, s->ne, s->k0i, s->pack, s->ecoord, s->eface,
                       s->eflags, s->RK, s->y, s->dsq, s->k0eps, s->k0t);
  const int64_t n = s->nf * s->d;
  hipLaunchKernelGGL(k_gauge_axpy, dim3(nblocks(n, BS)), dim3(BS), 0, stream, n, s->k0t, s->zy, s->y);
  return check_hip(hipGetLastError(), "gauge shift");
}

// Face gather of step a3.  full: the block rows of G in FP64 and FP32 (the
// operator of the assembled form), allocated on first use.  Otherwise, where
// CG applies the element factors, only what the element form needs (the Jacobi
// scale from the diagonal blocks, S, the column table): the rows are built when
// an assembled-form call first asks for them (ensure_assembled), which saves
// their memory and a pass over 2(2d+1)d^2 numbers per face at each elimination.
template <int D, bool NSK>
static cr_status face_gather(cr_system* s, bool full) {
  const unsigned gf = nblocks(s->nf, BS);
  if (full) {
    const size_t n = (size_t)(2 * D + 1) * D * D * (size_t)s->nf;
    if (!s->G64) s->G64 = (double*)dev_alloc(s, sizeof(double) * n);
    if (!s->G32) s->G32 = (float*)dev_alloc(s, sizeof(float) * n);
    if (!s->G64 || !s->G32) return CR_E_NOMEM;
    hipLaunchKernelGGL((k_face_assemble<D, NSK, true>), dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel,
                       s->floc, s->eface, s->eflags, s->pack, s->sK, s->cols, s->G64, s->dsq, s->bs, s->err);
    hipLaunchKernelGGL(k_face_scale<D>, dim3(gf), dim3(BS), 0, s->stream, s->nf, s->cols, s->dsq, s->G64, s->G32);
  } else {
    hipLaunchKernelGGL((k_face_assemble<D, NSK, false>), dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel,
                       s->floc, s->eface, s->eflags, s->pack, s->sK, s->cols, nullptr, s->dsq, s->bs, s->err);
  }
  s->g_valid = full;
  return check_hip(hipGetLastError(), "face gather");
}

cr_status ensure_assembled(cr_system* s) {
  if (s->g_valid) return CR_OK;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  if (s->d == 2) return ns ? face_gather<2, true>(s, true) : face_gather<2, false>(s, true);
  return ns ? face_gather<3, true>(s, true) : face_gather<3, false>(s, true);
}

cr_status run_eliminate(cr_system* s, const double* f_mean, const double* u_prev, const double* u_lin) {
  const int d = s->d;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  const bool steady = s->params.mu == 0.0;
  cr_status st = reset_err(s);
  if (st != CR_OK) return st;
  st = gather_inputs(s, f_mean, u_prev, u_lin);
  if (st != CR_OK) return st;
  const double* up = u_prev ? s->uprev : nullptr;
  const unsigned ge = nblocks(s->ne, BS), gf = nblocks(s->nf, BS);
  const double lscale = s->params.lambda_scale > 0.0 ? s->params.lambda_scale : 2.0;
  const Bnd bnd{s->has_bnd ? s->ebf : nullptr, s->gbnd, s->has_bnd ? s->ek : nullptr};
  if (ns && d == 2) {
    if (steady)
      hipLaunchKernelGGL(k_ns_lambda, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface, s->ulin,
                         s->params.mu, s->params.nu, lscale, bnd, s->lam);
    hipLaunchKernelGGL(k_elim_ns, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface, s->enb,
                       steady ? s->lam : nullptr, s->fbar, up, s->ulin, s->params.mu, s->params.nu, bnd, s->pack,
                       s->RK, s->sK, s->err);
    st = face_gather<2, true>(s, true);
    if (st != CR_OK) return st;
  } else if (ns) {
    // 3D Newton step: the local 12 x 12 matrices live in LDS (72 KiB per workgroup)
    st = check_hip(hipFuncSetAttribute((const void*)k_elim_ns3, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)LDS_NS3), "Newton-step LDS size");
    if (st == CR_OK)
      st = check_hip(hipFuncSetAttribute((const void*)k_ns_lambda3, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)LDS_NS3), "Newton-step LDS size");
    if (st != CR_OK) return st;
    const unsigned g3 = nblocks(s->ne, BS_NS3);
    if (steady)
      hipLaunchKernelGGL(k_ns_lambda3, dim3(g3), dim3(BS_NS3), LDS_NS3, s->stream, s->ne, s->ecoord, s->eflags,
                         s->eface, s->ulin, s->params.mu, s->params.nu, lscale, bnd, s->lam);
    hipLaunchKernelGGL(k_elim_ns3, dim3(g3), dim3(BS_NS3), LDS_NS3, s->stream, s->ne, s->ecoord, s->eflags, s->eface,
                       s->enb, steady ? s->lam : nullptr, s->fbar, up, s->ulin, s->params.mu, s->params.nu, bnd,
                       s->pack, s->RK, s->sK, s->err);
    st = face_gather<3, true>(s, true);
    if (st != CR_OK) return st;
  } else if (d == 2) {
    if (steady)
      hipLaunchKernelGGL(k_stokes_lambda<2>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags,
                         s->params.mu, s->params.nu, lscale, s->lam);
    hipLaunchKernelGGL(k_elim_stokes<2>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface,
                       s->enb, steady ? s->lam : nullptr, s->fbar, up, s->params.mu, s->params.nu, bnd, s->pack,
                       s->RK, s->sK, s->err);
    st = face_gather<2, false>(s, s->efo64 == nullptr);
    if (st != CR_OK) return st;
    if (s->efo64)
      hipLaunchKernelGGL(k_efo_build<2>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->pack, s->ecoord, s->eface,
                         s->eflags, s->dsq, s->efo64, s->efo32, s->egat);
  } else {
    if (steady)
      hipLaunchKernelGGL(k_stokes_lambda<3>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags,
                         s->params.mu, s->params.nu, lscale, s->lam);
    hipLaunchKernelGGL(k_elim_stokes<3>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface,
                       s->enb, steady ? s->lam : nullptr, s->fbar, up, s->params.mu, s->params.nu, bnd, s->pack,
                       s->RK, s->sK, s->err);
    st = face_gather<3, false>(s, s->efo64 == nullptr);
    if (st != CR_OK) return st;
    if (s->efo64)
      hipLaunchKernelGGL(k_efo_build<3>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->pack, s->ecoord, s->eface,
                         s->eflags, s->dsq, s->efo64, s->efo32, s->egat);
  }
  st = check_hip(hipGetLastError(), "eliminate launch");
  if (st != CR_OK) return st;
  if (s->efo64) {
    if (d == 2)
      hipLaunchKernelGGL(k_zvec<2>, dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel, s->floc, s->ecoord,
                         s->dsq, s->zy);
    else
      hipLaunchKernelGGL(k_zvec<3>, dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel, s->floc, s->ecoord,
                         s->dsq, s->zy);
    st = k0_rhs(s);
    if (st != CR_OK) return st;
    if (s->nagg > 0) {
      const int m = s->nagg;
      st = check_hip(hipMemsetAsync(s->Ec, 0, sizeof(double) * m * m, s->stream), "coarse E");
      if (st != CR_OK) return st;
      const unsigned gp = (unsigned)(((int64_t)s->npairs * 64 + 255) / 256);
      if (d == 2)
        hipLaunchKernelGGL(k_coarse_E<2>, dim3(gp), dim3(256), 0, s->stream, s->npairs, s->pair_ptr, s->pair_key,
                           s->pair_ent, s->ne, s->efo64, s->egat, s->zy, s->Ec);
      else
        hipLaunchKernelGGL(k_coarse_E<3>, dim3(gp), dim3(256), 0, s->stream, s->npairs, s->pair_ptr, s->pair_key,
                           s->pair_ent, s->ne, s->efo64, s->egat, s->zy, s->Ec);
      if (m <= 128) {
        st = check_hip(hipFuncSetAttribute((const void*)k_coarse_inv_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(sizeof(double) * 128 * 128)),
                       "coarse inverse LDS size");
        if (st != CR_OK) return st;
        hipLaunchKernelGGL(k_coarse_inv_lds, dim3(1), dim3(1024), sizeof(double) * m * m, s->stream, m, s->Ec, s->Einv);
      } else if (m % GJB == 0) {
        // in place in Einv; scratch: P, T, C and the flag
        const size_t nscr = (size_t)GJB * GJB + (size_t)2 * GJB * m + 1;
        if (!s->gjbuf) s->gjbuf = (double*)dev_alloc(s, sizeof(double) * nscr);
        if (!s->gjbuf) return CR_E_NOMEM;
        double* P = s->gjbuf;
        double* T = P + (size_t)GJB * GJB;
        double* C = T + (size_t)GJB * m;
        double* flag = C + (size_t)GJB * m;
        hipLaunchKernelGGL(k_gjb_init, dim3(1), dim3(1024), 0, s->stream, m, s->Ec, s->Einv, flag);
        const unsigned gpan = (unsigned)(((int64_t)2 * GJB * m + 255) / 256);
        const dim3 gupd((unsigned)(m / 16), (unsigned)(m / 16));
        for (int K0 = 0; K0 < m; K0 += GJB) {
          hipLaunchKernelGGL(k_gjb_pivot, dim3(1), dim3(GJB * GJB), 0, s->stream, m, K0, s->Einv, P, flag);
          hipLaunchKernelGGL(k_gjb_panel, dim3(gpan), dim3(256), 0, s->stream, m, K0, s->Einv, P, T, C);
          hipLaunchKernelGGL(k_gjb_update, gupd, dim3(256), 0, s->stream, m, K0, s->Einv, P, T, C, flag);
        }
        hipLaunchKernelGGL(k_gjb_final, dim3((unsigned)(((int64_t)m * m + 255) / 256)), dim3(256), 0, s->stream, m,
                           flag, s->Einv);
      } else {
        // the aggregate rule makes m a power of 4 (2D) or 8 (3D) up to 512
        set_error("coarse setup: %d aggregates, neither at most 128 nor a multiple of %d", m, GJB);
        return CR_E_INVAL;
      }
      const int64_t n = s->nf * d;
      hipLaunchKernelGGL(k_cast_f32, dim3(nblocks(n, BS)), dim3(BS), 0, s->stream, n, s->zy, s->zy32);
      st = check_hip(hipGetLastError(), "coarse setup");
      if (st != CR_OK) return st;
    }
  }
  st = read_err(s, "cr_eliminate");
  if (st != CR_OK) return st;
  st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * d, s->stream), "zero W");
  if (st != CR_OK) return st;
  s->eliminated = true;
  s->has_solution = false;
  return CR_OK;
}

cr_status run_update_rhs(cr_system* s, const double* f_mean, const double* u_prev) {
  const int d = s->d;
  cr_status st = reset_err(s);
  if (st != CR_OK) return st;
  st = gather_inputs(s, f_mean, u_prev, nullptr);
  if (st != CR_OK) return st;
  const double* up = u_prev ? s->uprev : nullptr;
  const unsigned ge = nblocks(s->ne, BS), gf = nblocks(s->nf, BS);
  const Bnd bnd{s->has_bnd ? s->ebf : nullptr, s->gbnd, s->has_bnd ? s->ek : nullptr};
  if (d == 2) {
    hipLaunchKernelGGL(k_rhs_stokes<2>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface,
                       s->fbar, up, s->params.mu, s->params.nu, bnd, s->pack, s->RK, s->sK, s->err);
    hipLaunchKernelGGL(k_face_rhs<2>, dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel, s->floc, s->sK, s->dsq,
                       s->bs);
  } else {
    hipLaunchKernelGGL(k_rhs_stokes<3>, dim3(ge), dim3(BS), 0, s->stream, s->ne, s->ecoord, s->eflags, s->eface,
                       s->fbar, up, s->params.mu, s->params.nu, bnd, s->pack, s->RK, s->sK, s->err);
    hipLaunchKernelGGL(k_face_rhs<3>, dim3(gf), dim3(BS), 0, s->stream, s->nf, s->ne, s->fel, s->floc, s->sK, s->dsq,
                       s->bs);
  }
  st = check_hip(hipGetLastError(), "update_rhs launch");
  if (st == CR_OK && s->efo64) st = k0_rhs(s);
  return st;
}

cr_status enqueue_import_w(cr_system* s, const double* w0) {
  const int64_t n = s->nf;
  hipLaunchKernelGGL(k_import_w, dim3(nblocks(n * s->d, BS)), dim3(BS), 0, s->stream, n, s->d, s->fcanon, s->dsq, w0,
                     s->y);
  s->has_solution = true;
  return check_hip(hipGetLastError(), "import W launch");
}

cr_status enqueue_export_w(cr_system* s, double* w) {
  const int64_t n = s->nf;
  hipLaunchKernelGGL(k_export_w, dim3(nblocks(n * s->d, BS)), dim3(BS), 0, s->stream, n, s->d, s->fcanon, s->dsq,
                     s->y, w);
  return check_hip(hipGetLastError(), "export W launch");
}

cr_status run_recover(cr_system* s, double* U, double* P, double* jump) {
  const int d = s->d;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  double* Uj = nullptr;
  if (jump) {
    if (!s->ujump) s->ujump = (double*)dev_alloc(s, sizeof(double) * (s->nf * d + 1024));
    if (!s->ujump) return CR_E_NOMEM;
    Uj = s->ujump;
  }
  const unsigned ge = nblocks(s->ne, BS);
  if (ns && d == 2)
    hipLaunchKernelGGL((k_recover<2, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, Uj);
  else if (ns)
    hipLaunchKernelGGL((k_recover<3, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, Uj);
  else if (d == 2)
    hipLaunchKernelGGL((k_recover<2, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, Uj);
  else
    hipLaunchKernelGGL((k_recover<3, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, Uj);
  if (jump) {
    const int64_t n = s->nf * d;
    hipLaunchKernelGGL(k_sqdiff_partial, dim3(1024), dim3(256), 0, s->stream, n, U, Uj, Uj + n);
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s->stream, 1024, Uj + n, jump);
  }
  return check_hip(hipGetLastError(), "recover launch");
}

// Device address of the scratch array on each device, taken once per device
// with that device current.
namespace {
constexpr int SCRATCH_MAXDEV = 64;
std::mutex g_scratch_mu;
double* g_scratch[SCRATCH_MAXDEV] = {};

cr_status scratch_address(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= SCRATCH_MAXDEV) {
    set_error("device %d out of range for the allocation-free recovery", dev);
    return CR_E_INVAL;
  }
  if (!g_scratch[dev]) {
    int cur = -1;
    cr_status st = check_hip(hipGetDevice(&cur), "hipGetDevice");
    if (st != CR_OK) return st;
    if (cur != dev) {
      st = check_hip(hipSetDevice(dev), "hipSetDevice");
      if (st != CR_OK) return st;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const cr_status back = check_hip(hipSetDevice(cur), "hipSetDevice (restore)");
      if (back != CR_OK) return back;
    }
    st = check_hip(e, "hipGetSymbolAddress(scratch)");
    if (st != CR_OK) return st;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return CR_OK;
}
}  // namespace

cr_status run_recover_noalloc(cr_system* s, double* U, double* P, double* jump) {
  const int d = s->d;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  const unsigned ge = nblocks(s->ne, BS);
  double* part = nullptr;
  if (jump) {
    if ((int64_t)ge > NOALLOC_PARTIALS) {
      set_error("cr_recover_noalloc: %lld elements exceed its limit of %lld (one partial per %d elements)",
                (long long)s->ne, (long long)(NOALLOC_PARTIALS * BS), BS);
      return CR_E_INVAL;
    }
    const cr_status st = scratch_address(s->device, &part);
    if (st != CR_OK) return st;
  }
  if (ns && d == 2)
    hipLaunchKernelGGL((k_recover<2, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, nullptr);
  else if (ns)
    hipLaunchKernelGGL((k_recover<3, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, nullptr);
  else if (d == 2)
    hipLaunchKernelGGL((k_recover<2, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, nullptr);
  else
    hipLaunchKernelGGL((k_recover<3, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq, s->pack, s->RK,
                       s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->ecaller, s->fcanon, U, P, nullptr);
  if (jump) {
    if (ns && d == 2)
      hipLaunchKernelGGL((k_recover_mismatch<2, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq,
                         s->pack, s->RK, s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->fcanon, U, part);
    else if (ns)
      hipLaunchKernelGGL((k_recover_mismatch<3, true>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq,
                         s->pack, s->RK, s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->fcanon, U, part);
    else if (d == 2)
      hipLaunchKernelGGL((k_recover_mismatch<2, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq,
                         s->pack, s->RK, s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->fcanon, U, part);
    else
      hipLaunchKernelGGL((k_recover_mismatch<3, false>), dim3(ge), dim3(BS), 0, s->stream, s->ne, s->y, s->dsq,
                         s->pack, s->RK, s->has_bnd ? s->ek : nullptr, s->eface, s->eflags, s->fcanon, U, part);
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s->stream, (int)ge, part, jump);
  }
  return check_hip(hipGetLastError(), "recover launch");
}

}  // namespace crh
