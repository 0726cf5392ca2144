// Baseline: FP64 Krylov solve of the original coupled system (Section 3.1, eq. syslin)
//     [A  D^t] [U]   [R]
//     [D   0 ] [P] = [0]
// on the same GPU.  Stokes (A = S (x) I_d, symmetric): MINRES preconditioned by
// the positive diagonal diag(A) (+) diag(D diag(A)^{-1} D^t).  Newton step (A =
// the Jacobian of the convection form added to S (x) I_d, non-symmetric):
// BiCGStab on the system scaled symmetrically by the square root of the
// positive diagonal diag|A| (+) diag(D diag|A|^{-1} D^t).  This is the
// comparison the hybrid method is measured against; it is not on the hybrid
// path.
//
// Storage: A as scalar face-ELL (the same face stencil and column table as G,
// one value per face pair since A = S (x) I_d); D^t P at face row f is
// -a_{K,f} (P_K - P_L) with a_{K,f} of the owner K; D U at element K is
// -sum_j a_{K,j}.U_j over its interior faces (the K0 row is removed: its
// coefficients are zero and its preconditioner entry is zero, so P_K0 stays 0).
// Vector layout: [u (nf*d, internal face order) | p (ne, internal element order)].
//
// Preconditioned MINRES (Paige-Saunders recurrences), three kernels per
// iteration with the same partial-record reductions, parity-slotted scalars
// and device stop flag as the hybrid Krylov kernels; the three-term vector
// recurrences rotate through three buffers, so graphs hold multiples of six
// iterations.  Outer passes restart from the current iterate until the true
// FP64 residual meets the tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "convection.h"
#include "geometry.h"
#include "internal.h"
#include "rowkern.h"

namespace crh {
namespace {

struct CState {
  double beta[2], oldb[2], dbar[2], epsln[2], cs[2], sn[2], phibar[2], alfa[2];
  int it[2];
  int done;
  int iters;
  double beta1, tres2, bnorm2, thr;
  // host parameters
  double tol2;
  int maxit;
  int pad;
};

struct CDims {
  int64_t nf, ne;
  int nbf, nbe;        // blocks over face rows / element rows (multiples of 8)
  int64_t cf, ce;      // rows per block
};

__device__ __forceinline__ bool face_block(const CDims& C, int64_t& lo, int64_t& hi, int& lb) {
  int b = blockIdx.x;
  if (b < C.nbf) {
    lb = (b & 7) * (C.nbf >> 3) + (b >> 3);
    lo = (int64_t)lb * C.cf;
    hi = min(C.nf, lo + C.cf);
    return true;
  }
  b -= C.nbf;
  const int l = (b & 7) * (C.nbe >> 3) + (b >> 3);
  lb = C.nbf + l;
  lo = (int64_t)l * C.ce;
  hi = min(C.ne, lo + C.ce);
  return false;
}

// ---------------------------------------------------------------------------
// assembly: A values per face row (slot 0 = diagonal), owner face vectors, the
// per-element D coefficients, preconditioner, assembled R.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(128) k_coupled_faces(int64_t nf, int64_t ne, const double* __restrict__ ecoord,
                                                       const uint32_t* __restrict__ eflags,
                                                       const int32_t* __restrict__ fel,
                                                       const int32_t* __restrict__ floc, const double* __restrict__ RK,
                                                       double mu, double nu, double* __restrict__ Aval,
                                                       double* __restrict__ an, double* __restrict__ bvec,
                                                       double* __restrict__ dinv) {
  constexpr int N = D + 1;
  int64_t f = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (f >= nf) return;
  const int64_t e2[2] = {fel[f], fel[nf + f]};
  const int lc = floc[f];
  const int jj[2] = {lc & 0xff, (lc >> 8) & 0xff};
  double diag = 0.0;
  double R[D];
#pragma unroll
  for (int i = 0; i < D; ++i) R[i] = 0.0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t K = e2[side];
    const int j = jj[side];
    Geo<D> g;
    load_geometry<D>(ecoord, ne, K, g);
    const uint32_t fl = eflags[K];
    const double m = mu * g.vol / N, iv = nu / g.vol;
    int slot = 1 + side * D;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      double dot = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) dot += g.a[j][i] * g.a[l][i];
      const double v = iv * dot + (l == j ? m : 0.0);
      if (l == j) {
        diag += v;
      } else {
        Aval[(int64_t)slot * nf + f] = interior(fl, l) ? v : 0.0;
        ++slot;
      }
    }
    if (side == 0)
#pragma unroll
      for (int i = 0; i < D; ++i) an[f * D + i] = g.a[j][i];
#pragma unroll
    for (int i = 0; i < D; ++i) R[i] += RK[(int64_t)(j * D + i) * ne + K];
  }
  Aval[f] = diag;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    bvec[f * D + i] = R[i];
    dinv[f * D + i] = 1.0 / diag;
  }
}

template <int D>
__global__ void __launch_bounds__(128) k_coupled_elems(int64_t nf, int64_t ne, const double* __restrict__ ecoord,
                                                       const uint32_t* __restrict__ eflags,
                                                       const int32_t* __restrict__ eface,
                                                       const double* __restrict__ Aval, const double* __restrict__ ek,
                                                       double* __restrict__ ea, double* __restrict__ bvec,
                                                       double* __restrict__ dinv) {
  constexpr int N = D + 1;
  int64_t k = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (k >= ne) return;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  const bool k0 = fl & F_K0;
  double sch = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool in = interior(fl, j) && !k0;
    double a2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      ea[(int64_t)(j * D + i) * ne + k] = in ? g.a[j][i] : 0.0;
      a2 += g.a[j][i] * g.a[j][i];
    }
    if (in) sch += a2 / Aval[eface[j * ne + k]];
  }
  bvec[nf * D + k] = (ek != nullptr && !k0) ? ek[k] : 0.0;
  dinv[nf * D + k] = k0 ? 0.0 : 1.0 / sch;
}

// one row of y = M v for the coupled matrix M; In(c) gives v_u at face c,
// Pin(k) gives v_p at element k
template <int D, class In, class Pin>
__device__ __forceinline__ void coupled_face_row(const double* __restrict__ Aval, const int32_t* __restrict__ cols,
                                                 const double* __restrict__ an, const int32_t* __restrict__ fel,
                                                 int64_t nf, int64_t f, const In& in, const Pin& pin,
                                                 double (&y)[D]) {
  Vec<double, D> x0 = in(f);
#pragma unroll
  for (int i = 0; i < D; ++i) y[i] = Aval[f] * x0.v[i];
#pragma unroll
  for (int s = 1; s <= 2 * D; ++s) {
    const int64_t c = cols[(int64_t)(s - 1) * nf + f];
    const double a = Aval[(int64_t)s * nf + f];
    Vec<double, D> xc = in(c);
#pragma unroll
    for (int i = 0; i < D; ++i) y[i] += a * xc.v[i];
  }
  const double dp = pin(fel[f]) - pin(fel[nf + f]);
#pragma unroll
  for (int i = 0; i < D; ++i) y[i] -= an[f * D + i] * dp;
}

template <int D, class In>
__device__ __forceinline__ double coupled_elem_row(const double* __restrict__ ea, const int32_t* __restrict__ eface,
                                                   int64_t ne, int64_t k, const In& in) {
  double y = 0.0;
#pragma unroll
  for (int j = 0; j <= D; ++j) {
    const int f = eface[j * ne + k];
    if (f < 0) continue;
    Vec<double, D> x = in(f);
#pragma unroll
    for (int i = 0; i < D; ++i) y -= ea[(int64_t)(j * D + i) * ne + k] * x.v[i];
  }
  return y;
}

struct MatArgs {
  const double* Aval;
  const int32_t* cols;
  const double* an;
  const int32_t* fel;
  const double* ea;
  const int32_t* eface;
};

template <int D>
struct ScaledU {  // dinv * r / beta on the velocity part
  const double* __restrict__ r;
  const double* __restrict__ dinv;
  double sb;
  __device__ Vec<double, D> operator()(int64_t c) const {
    Vec<double, D> a = ldv<double, D>(r, c), w = ldv<double, D>(dinv, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] *= w.v[i] * sb;
    return a;
  }
};
struct ScaledP {
  const double* __restrict__ r;
  const double* __restrict__ dinv;
  double sb;
  __device__ double operator()(int64_t k) const { return r[k] * dinv[k] * sb; }
};
template <int D>
struct PlainU {
  const double* __restrict__ x;
  __device__ Vec<double, D> operator()(int64_t c) const { return ldv<double, D>(x, c); }
};
struct PlainP {
  const double* __restrict__ x;
  __device__ double operator()(int64_t k) const { return x[k]; }
};

// residual r = b - M x (FP64), r1 = r2 = r; partials [0] r.dinv.r, [1] r.r, [2] b.b
template <int D>
__global__ void __launch_bounds__(NT) k_mr_init(CDims C, MatArgs M, const double* __restrict__ b,
                                                const double* __restrict__ dinv, const double* __restrict__ x,
                                                double* __restrict__ r1, double* __restrict__ r2,
                                                double* __restrict__ w0, double* __restrict__ w1,
                                                double* __restrict__ pa, CState* __restrict__ st) {
  int64_t lo, hi;
  int lb;
  const bool fb = face_block(C, lo, hi, lb);
  const int64_t off = C.nf * D;
  double acc[3] = {0.0, 0.0, 0.0};
  if (fb) {
    for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
      double y[D];
      coupled_face_row<D>(M.Aval, M.cols, M.an, M.fel, C.nf, f, PlainU<D>{x}, PlainP{x + off}, y);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double bi = b[f * D + i], ri = bi - y[i];
        r1[f * D + i] = ri;
        r2[f * D + i] = ri;
        w0[f * D + i] = 0.0;
        w1[f * D + i] = 0.0;
        acc[0] += ri * ri * dinv[f * D + i];
        acc[1] += ri * ri;
        acc[2] += bi * bi;
      }
    }
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += NT) {
      // divergence rows: right-hand side e_K (boundary data), else zero
      const double bi = b[off + k], ri = bi - coupled_elem_row<D>(M.ea, M.eface, C.ne, k, PlainU<D>{x});
      r1[off + k] = ri;
      r2[off + k] = ri;
      w0[off + k] = 0.0;
      w1[off + k] = 0.0;
      acc[0] += ri * ri * dinv[off + k];
      acc[1] += ri * ri;
      acc[2] += bi * bi;
    }
  }
  block_sum<3>(acc);
  if (threadIdx.x == 0) {
    pa[(int64_t)lb * NPART] = acc[0];
    pa[(int64_t)lb * NPART + 1] = acc[1];
    pa[(int64_t)lb * NPART + 2] = acc[2];
  }
  if (lead()) {
    st->it[1] = 0;
    st->oldb[1] = 0.0;
    st->dbar[1] = 0.0;
    st->epsln[1] = 0.0;
    st->cs[1] = -1.0;
    st->sn[1] = 0.0;
    st->iters = 0;
    st->done = 0;
  }
}

// MA: v = dinv r2 / beta, y = M v - (beta/oldb) r1, partial v.y
template <int D>
__global__ void __launch_bounds__(NT) k_mr_a(CDims C, MatArgs M, const double* __restrict__ dinv,
                                             const double* __restrict__ r1, const double* __restrict__ r2,
                                             double* __restrict__ v, double* __restrict__ y,
                                             const double* __restrict__ pa, double* __restrict__ pb,
                                             CState* __restrict__ st, int q) {
  const int seen = st->done;
  const int p = q ^ 1;
  const int it = st->it[p];
  const bool first = it == 0;
  double beta, oldb;
  int done = 0;
  if (first) {
    double s[3];
    if (reduce_partials_stop<3>(pa, C.nbf + C.nbe, 0, s, seen)) return;
    beta = sqrt(s[0]);
    oldb = 0.0;
    const double thr = 0.1 * sqrt(st->tol2 * s[2]) * (s[1] > 0.0 ? beta / sqrt(s[1]) : 1.0);
    if (s[1] <= st->tol2 * s[2]) done = 2;
    else if (!(beta > 0.0) || !isfinite(beta)) done = isfinite(beta) ? 4 : 5;
    else if (it >= st->maxit) done = 3;
    if (lead()) {
      st->beta1 = beta;
      st->tres2 = s[1];
      st->bnorm2 = s[2];
      st->thr = thr;
      st->beta[p] = beta;
      st->phibar[p] = beta;
    }
  } else {
    // no reduction before the decision: a wave that saw the word set returns,
    // and the others reach the same decision from the same state and return
    if (seen) return;
    beta = st->beta[p];
    oldb = st->oldb[p];
    if (st->phibar[p] <= st->thr) done = 1;
    else if (it >= st->maxit) done = 3;
  }
  if (lead()) {
    st->it[q] = it + 1;
    st->iters = it;
    if (done) st->done = done;
  }
  if (done) return;
  const double sb = 1.0 / beta;
  const double c1 = first ? 0.0 : beta / oldb;
  int64_t lo, hi;
  int lb;
  const bool fb = face_block(C, lo, hi, lb);
  const int64_t off = C.nf * D;
  const ScaledU<D> inu{r2, dinv, sb};
  const ScaledP inp{r2 + off, dinv + off, sb};
  double acc[1] = {0.0};
  if (fb) {
    for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
      double yy[D];
      coupled_face_row<D>(M.Aval, M.cols, M.an, M.fel, C.nf, f, inu, inp, yy);
      Vec<double, D> vv = inu(f);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        yy[i] -= c1 * r1[f * D + i];
        v[f * D + i] = vv.v[i];
        y[f * D + i] = yy[i];
        acc[0] += vv.v[i] * yy[i];
      }
    }
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += NT) {
      const double yy = coupled_elem_row<D>(M.ea, M.eface, C.ne, k, inu) - c1 * r1[off + k];
      const double vv = inp(k);
      v[off + k] = vv;
      y[off + k] = yy;
      acc[0] += vv * yy;
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pb[(int64_t)lb * NPART] = acc[0];
}

// MB: alfa = v.y; y -= (alfa/beta) r2 (y becomes the new r2); partial y.dinv.y
__global__ void __launch_bounds__(NT) k_mr_b(CDims C, int64_t n, const double* __restrict__ dinv,
                                             const double* __restrict__ r2, double* __restrict__ y,
                                             const double* __restrict__ pb, double* __restrict__ pc,
                                             CState* __restrict__ st, int q) {
  if (st->done) return;
  double s[1];
  reduce_partials<1>(pb, C.nbf + C.nbe, 0, s);
  const double alfa = s[0];
  const double beta = st->beta[q ^ 1];
  const double c2 = alfa / beta;
  // flat partition of all n entries over the same number of blocks
  const int nb = C.nbf + C.nbe;
  const int lb = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int64_t per = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)lb * per, hi = min(n, lo + per);
  double acc[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    const double yy = y[i] - c2 * r2[i];
    y[i] = yy;
    acc[0] += yy * yy * dinv[i];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pc[(int64_t)lb * NPART] = acc[0];
  if (lead()) st->alfa[q] = alfa;
}

// MC: beta_new = sqrt(partials); plane rotations; w = (v - oldeps w1 - delta w2)/gamma; x += phi w
__global__ void __launch_bounds__(NT) k_mr_c(CDims C, int64_t n, const double* __restrict__ v,
                                             const double* __restrict__ w1, const double* __restrict__ w2,
                                             double* __restrict__ wn, double* __restrict__ x,
                                             const double* __restrict__ pc, CState* __restrict__ st, int q) {
  const int seen = st->done;
  double s[1];
  if (reduce_partials_stop<1>(pc, C.nbf + C.nbe, 0, s, seen)) return;
  const int p = q ^ 1;
  if (!(s[0] >= 0.0) || !isfinite(s[0])) {
    if (lead()) st->done = isfinite(s[0]) ? 4 : 5;
    return;
  }
  const double beta = sqrt(s[0]);
  const double oldb = st->beta[p];
  const double alfa = st->alfa[q];
  const double cs = st->cs[p], sn = st->sn[p], dbar = st->dbar[p], oldeps = st->epsln[p];
  const double delta = cs * dbar + sn * alfa;
  const double gbar = sn * dbar - cs * alfa;
  const double epsln = sn * beta;
  const double dbar_n = -cs * beta;
  const double gamma = fmax(hypot(gbar, beta), 1e-300);
  const double cs_n = gbar / gamma, sn_n = beta / gamma;
  const double phibar = st->phibar[p];
  const double phi = cs_n * phibar;
  const double phibar_n = sn_n * phibar;
  const double den = 1.0 / gamma;
  const int nb = C.nbf + C.nbe;
  const int lb = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int64_t per = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)lb * per, hi = min(n, lo + per);
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    const double w = (v[i] - oldeps * w1[i] - delta * w2[i]) * den;
    wn[i] = w;
    x[i] += phi * w;
  }
  if (lead()) {
    st->beta[q] = beta;
    st->oldb[q] = oldb;
    st->cs[q] = cs_n;
    st->sn[q] = sn_n;
    st->dbar[q] = dbar_n;
    st->epsln[q] = epsln;
    st->phibar[q] = phibar_n;
  }
}

// internal -> caller layouts
template <int D>
__global__ void k_mr_scatter(int64_t nf, int64_t ne, const double* __restrict__ x, const int32_t* __restrict__ fcanon,
                             const int32_t* __restrict__ ecaller, double* __restrict__ U, double* __restrict__ P) {
  int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < nf) {
#pragma unroll
    for (int i = 0; i < D; ++i) U[(int64_t)fcanon[t] * D + i] = x[t * D + i];
  } else if (t < nf + ne) {
    const int64_t k = t - nf;
    P[ecaller[k]] = x[nf * D + k];
  }
}

// ---------------------------------------------------------------------------
// Newton step: A in d x d blocks per face pair (block-ELL with the column table
// of G: slot 0 the diagonal block, slots 1..d the other faces of the owner
// element, d+1..2d those of the other element), from the element matrices
// A_K of the Jacobian (formed once per solve in a scratch array).
// ---------------------------------------------------------------------------
template <int D, class M>
__device__ __forceinline__ void ns_amat_elem(int64_t ne, int64_t k, const double* __restrict__ ecoord,
                                             const uint32_t* __restrict__ eflags, const int32_t* __restrict__ eface,
                                             const double* __restrict__ ulin, double mu, double nu, const Bnd& bnd,
                                             const M& A, double* __restrict__ amat) {
  constexpr int NU = NsPack<D>::NU;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  double Ub[D + 1][D], Nuu[D + 1][D], Gb[D + 1][D], Rb[D + 1][D];
  load_bnd<D>(bnd, fl, ne, k, Gb);
  load_ubar<D>(ulin, eface, fl, ne, k, Gb, Ub);
  ns_local<D>(g, fl, Ub, mu, nu, A, Nuu, Gb, Rb);
  for (int a = 0; a < NU; ++a)
    for (int b = 0; b < NU; ++b) amat[(int64_t)(a * NU + b) * ne + k] = A(a, b);
}

__global__ void __launch_bounds__(128) k_ns_amat2(int64_t ne, const double* __restrict__ ecoord,
                                                  const uint32_t* __restrict__ eflags,
                                                  const int32_t* __restrict__ eface, const double* __restrict__ ulin,
                                                  double mu, double nu, Bnd bnd, double* __restrict__ amat) {
  const int64_t k = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (k >= ne) return;
  double A[6][6];
  ns_amat_elem<2>(ne, k, ecoord, eflags, eface, ulin, mu, nu, bnd, RegMat<6>{A}, amat);
}

constexpr int BS_AM3 = 64;
__global__ void __launch_bounds__(BS_AM3) k_ns_amat3(int64_t ne, const double* __restrict__ ecoord,
                                                     const uint32_t* __restrict__ eflags,
                                                     const int32_t* __restrict__ eface,
                                                     const double* __restrict__ ulin, double mu, double nu, Bnd bnd,
                                                     double* __restrict__ amat) {
  extern __shared__ double lds_am[];
  const int64_t k = (int64_t)blockIdx.x * BS_AM3 + threadIdx.x;
  if (k >= ne) return;
  ns_amat_elem<3>(ne, k, ecoord, eflags, eface, ulin, mu, nu, bnd, LdsMat<12>{lds_am + threadIdx.x, BS_AM3}, amat);
}

// face rows of the Newton-step coupled matrix: blocks of A, owner face vector,
// assembled R, and the velocity part of the preconditioner 1/|A_(f,i),(f,i)|
template <int D>
__global__ void __launch_bounds__(128) k_coupled_faces_ns(int64_t nf, int64_t ne, const double* __restrict__ ecoord,
                                                          const uint32_t* __restrict__ eflags,
                                                          const int32_t* __restrict__ fel,
                                                          const int32_t* __restrict__ floc,
                                                          const double* __restrict__ RK,
                                                          const double* __restrict__ amat,
                                                          double* __restrict__ Ablk, double* __restrict__ an,
                                                          double* __restrict__ bvec, double* __restrict__ dinv) {
  constexpr int N = D + 1, DD = D * D, NU = N * D;
  const int64_t f = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (f >= nf) return;
  const int64_t e2[2] = {fel[f], fel[nf + f]};
  const int lc = floc[f];
  const int jj[2] = {lc & 0xff, (lc >> 8) & 0xff};
  double diag[D][D], R[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    R[i] = 0.0;
#pragma unroll
    for (int ip = 0; ip < D; ++ip) diag[i][ip] = 0.0;
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t K = e2[side];
    const int j = jj[side];
    const uint32_t fl = eflags[K];
    auto a = [&](int r, int c) { return amat[(int64_t)(r * NU + c) * ne + K]; };
#pragma unroll
    for (int i = 0; i < D; ++i) {
      R[i] += RK[(int64_t)(j * D + i) * ne + K];
#pragma unroll
      for (int ip = 0; ip < D; ++ip) diag[i][ip] += a(j * D + i, j * D + ip);
    }
    int slot = 1 + side * D;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      if (l == j) continue;
      const bool in = interior(fl, l);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int ip = 0; ip < D; ++ip)
          Ablk[(int64_t)(slot * DD + i * D + ip) * nf + f] = in ? a(j * D + i, l * D + ip) : 0.0;
      ++slot;
    }
    if (side == 0) {
      Geo<D> g;
      load_geometry<D>(ecoord, ne, K, g);
#pragma unroll
      for (int i = 0; i < D; ++i) an[f * D + i] = g.a[j][i];
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
#pragma unroll
    for (int ip = 0; ip < D; ++ip) Ablk[(int64_t)(i * D + ip) * nf + f] = diag[i][ip];
    bvec[f * D + i] = R[i];
    dinv[f * D + i] = 1.0 / fabs(diag[i][i]);
  }
}

// element rows (D U): coefficients and the pressure part of the
// preconditioner 1 / sum_{j,i} a_{K,j,i}^2 / |A_(f_j,i),(f_j,i)|
template <int D>
__global__ void __launch_bounds__(128) k_coupled_elems_ns(int64_t nf, int64_t ne, const double* __restrict__ ecoord,
                                                          const uint32_t* __restrict__ eflags,
                                                          const int32_t* __restrict__ eface,
                                                          const double* __restrict__ Ablk,
                                                          const double* __restrict__ ek, double* __restrict__ ea,
                                                          double* __restrict__ bvec, double* __restrict__ dinv) {
  constexpr int N = D + 1;
  const int64_t k = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (k >= ne) return;
  Geo<D> g;
  load_geometry<D>(ecoord, ne, k, g);
  const uint32_t fl = eflags[k];
  const bool k0 = fl & F_K0;
  double sch = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool in = interior(fl, j) && !k0;
    const int64_t f = interior(fl, j) ? eface[j * ne + k] : 0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      ea[(int64_t)(j * D + i) * ne + k] = in ? g.a[j][i] : 0.0;
      if (in) sch += g.a[j][i] * g.a[j][i] / fabs(Ablk[(int64_t)(i * D + i) * nf + f]);
    }
  }
  bvec[nf * D + k] = (ek != nullptr && !k0) ? ek[k] : 0.0;
  dinv[nf * D + k] = k0 ? 0.0 : 1.0 / sch;
}

// one velocity row of y = M v (Newton step): block row of A, then D^t P
template <int D, class In, class Pin>
__device__ __forceinline__ void coupled_face_row_ns(const double* __restrict__ Ablk, const int32_t* __restrict__ cols,
                                                    const double* __restrict__ an, const int32_t* __restrict__ fel,
                                                    int64_t nf, int64_t f, const In& in, const Pin& pin,
                                                    double (&y)[D]) {
  constexpr int DD = D * D;
#pragma unroll
  for (int i = 0; i < D; ++i) y[i] = 0.0;
#pragma unroll
  for (int s = 0; s <= 2 * D; ++s) {
    const int64_t c = s == 0 ? f : cols[(int64_t)(s - 1) * nf + f];
    Vec<double, D> xc = in(c);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) y[i] += Ablk[(int64_t)(s * DD + i * D + j) * nf + f] * xc.v[j];
  }
  const double dp = pin(fel[f]) - pin(fel[nf + f]);
#pragma unroll
  for (int i = 0; i < D; ++i) y[i] -= an[f * D + i] * dp;
}

// ---------------------------------------------------------------------------
// BiCGStab on the scaled coupled system K~ x~ = b~, K~ = Q K Q, b~ = Q b,
// x = Q x~, Q = diag(sqrt(dinv)); the iterate is kept unscaled (x += Q (alpha
// p + omega s)).  Three kernels per iteration, parity-slotted scalars, p and v
// double-buffered by parity (the product kernels gather the new direction
// p = r + beta (p_old - omega v_old) and s = r - alpha v at neighbouring rows
// on the fly).  Passes restart from the true residual b - K x until it meets
// the tolerance.
// ---------------------------------------------------------------------------
struct BState {
  double rho[2], alpha[2], omega[2];
  int it[2];
  int done;    // 1 pass converged, 3 limit, 4 breakdown, 5 non-finite
  int iters;
  double thr, tres2, bnorm2;
  // host parameters
  double tol2;
  int maxit;
  int pad;
};

template <int D>
struct QU {  // Q v at face c
  const double* __restrict__ v;
  const double* __restrict__ q;
  __device__ Vec<double, D> operator()(int64_t c) const {
    Vec<double, D> a = ldv<double, D>(v, c), w = ldv<double, D>(q, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] *= w.v[i];
    return a;
  }
};
struct QP {
  const double* __restrict__ v;
  const double* __restrict__ q;
  __device__ double operator()(int64_t k) const { return v[k] * q[k]; }
};
// Q (r + beta (p - omega v)) and Q (r - alpha v) at face c / element k
template <int D>
struct QPNewU {
  const double *r, *p, *v, *q;
  double beta, omega;
  __device__ Vec<double, D> operator()(int64_t c) const {
    Vec<double, D> a = ldv<double, D>(r, c), pp = ldv<double, D>(p, c), vv = ldv<double, D>(v, c),
                   w = ldv<double, D>(q, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] = w.v[i] * (a.v[i] + beta * (pp.v[i] - omega * vv.v[i]));
    return a;
  }
};
struct QPNewP {
  const double *r, *p, *v, *q;
  double beta, omega;
  __device__ double operator()(int64_t k) const { return q[k] * (r[k] + beta * (p[k] - omega * v[k])); }
};
template <int D>
struct QSNewU {
  const double *r, *v, *q;
  double alpha;
  __device__ Vec<double, D> operator()(int64_t c) const {
    Vec<double, D> a = ldv<double, D>(r, c), vv = ldv<double, D>(v, c), w = ldv<double, D>(q, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] = w.v[i] * (a.v[i] - alpha * vv.v[i]);
    return a;
  }
};
struct QSNewP {
  const double *r, *v, *q;
  double alpha;
  __device__ double operator()(int64_t k) const { return q[k] * (r[k] - alpha * v[k]); }
};

struct NsMat {
  const double* Ablk;
  const int32_t* cols;
  const double* an;
  const int32_t* fel;
  const double* ea;
  const int32_t* eface;
};

// pass start: res = b - K x (unscaled, true residual), r = rhat = Q res, p = v = 0.
// Partials: [0] rhat.r, [1] r.r, [2] res.res, [3] b.b
template <int D>
__global__ void __launch_bounds__(NT) k_cb_init(CDims C, NsMat M, const double* __restrict__ b,
                                                const double* __restrict__ q, const double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ rhat,
                                                double* __restrict__ p0, double* __restrict__ p1,
                                                double* __restrict__ v0, double* __restrict__ v1,
                                                double* __restrict__ pa, BState* __restrict__ st) {
  int64_t lo, hi;
  int lb;
  const bool fb = face_block(C, lo, hi, lb);
  const int64_t off = C.nf * D;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto put = [&](int64_t i, double res, double bi) {
    const double ri = q[i] * res;
    r[i] = ri;
    rhat[i] = ri;
    p0[i] = p1[i] = v0[i] = v1[i] = 0.0;
    acc[0] += ri * ri;
    acc[1] += ri * ri;
    acc[2] += res * res;
    acc[3] += bi * bi;
  };
  if (fb) {
    for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
      double y[D];
      coupled_face_row_ns<D>(M.Ablk, M.cols, M.an, M.fel, C.nf, f, PlainU<D>{x}, PlainP{x + off}, y);
#pragma unroll
      for (int i = 0; i < D; ++i) put(f * D + i, b[f * D + i] - y[i], b[f * D + i]);
    }
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += NT)
      put(off + k, b[off + k] - coupled_elem_row<D>(M.ea, M.eface, C.ne, k, PlainU<D>{x}), b[off + k]);
  }
  block_sum<4>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) pa[(int64_t)lb * NPART + m] = acc[m];
  if (lead()) {
    st->it[1] = 0;
    st->iters = 0;
    st->done = 0;
    st->rho[1] = 1.0;
    st->alpha[1] = 1.0;
    st->omega[1] = 1.0;
  }
}

// CB1 (parity par): rho = rhat.r; stopping; beta; v = K~ p with p = r + beta (p_old - omega v_old)
// formed at every gathered row; p stored; partial rhat.v
template <int D>
__global__ void __launch_bounds__(NT) k_cb_1(CDims C, NsMat M, const double* __restrict__ q,
                                             const double* __restrict__ r, const double* __restrict__ rhat,
                                             const double* __restrict__ pold, const double* __restrict__ vold,
                                             double* __restrict__ pnew, double* __restrict__ vnew,
                                             const double* __restrict__ pa, double* __restrict__ pb,
                                             BState* __restrict__ st, int par) {
  const int seen = st->done;
  const int it = st->it[par ^ 1];
  const bool first = it == 0;
  const double rho_old = st->rho[par ^ 1], alpha_old = st->alpha[par ^ 1], omega_old = st->omega[par ^ 1];
  double s[4];
  if (reduce_partials_stop<4>(pa, C.nbf + C.nbe, 0, s, seen)) return;
  const double rho = s[0], rr = s[1];
  int done = 0;
  if (first) {
    // pass start: the partials also hold the true residual and ||b||
    const double thr = 0.01 * st->tol2 * s[3] * (s[2] > 0.0 ? rr / s[2] : 1.0);
    if (lead()) {
      st->tres2 = s[2];
      st->bnorm2 = s[3];
      st->thr = thr;
    }
    if (s[2] <= st->tol2 * s[3]) done = 1;
  } else if (rr <= st->thr) {
    done = 1;
  }
  if (!done) {
    if (!isfinite(rho) || !isfinite(rr)) done = 5;
    else if (it >= st->maxit) done = 3;
    else if (!(fabs(rho) > 1e-300) || (!first && !(fabs(omega_old) > 0.0))) done = 4;
  }
  if (lead()) {
    st->iters = it;
    if (done) st->done = done;
  }
  if (done) return;
  const double beta = first ? 0.0 : (rho / rho_old) * (alpha_old / omega_old);
  if (lead()) {
    st->rho[par] = rho;
    st->it[par] = it + 1;
  }
  int64_t lo, hi;
  int lb;
  const bool fb = face_block(C, lo, hi, lb);
  const int64_t off = C.nf * D;
  const QPNewU<D> inu{r, pold, vold, q, beta, omega_old};
  const QPNewP inp{r + off, pold + off, vold + off, q + off, beta, omega_old};
  double acc[1] = {0.0};
  if (fb) {
    for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
      double y[D];
      coupled_face_row_ns<D>(M.Ablk, M.cols, M.an, M.fel, C.nf, f, inu, inp, y);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int64_t e = f * D + i;
        pnew[e] = r[e] + beta * (pold[e] - omega_old * vold[e]);
        const double vv = q[e] * y[i];
        vnew[e] = vv;
        acc[0] += rhat[e] * vv;
      }
    }
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += NT) {
      const int64_t e = off + k;
      pnew[e] = r[e] + beta * (pold[e] - omega_old * vold[e]);
      const double vv = q[e] * coupled_elem_row<D>(M.ea, M.eface, C.ne, k, inu);
      vnew[e] = vv;
      acc[0] += rhat[e] * vv;
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pb[(int64_t)lb * NPART] = acc[0];
}

// CB2: alpha = rho / rhat.v; t = K~ s with s = r - alpha v formed at gathered rows; s stored;
// partials t.s, t.t
template <int D>
__global__ void __launch_bounds__(NT) k_cb_2(CDims C, NsMat M, const double* __restrict__ q,
                                             const double* __restrict__ r, const double* __restrict__ v,
                                             double* __restrict__ sv, double* __restrict__ t,
                                             const double* __restrict__ pb, double* __restrict__ pc,
                                             BState* __restrict__ st, int par) {
  const int seen = st->done;
  const double rho = st->rho[par];
  double sm[1];
  if (reduce_partials_stop<1>(pb, C.nbf + C.nbe, 0, sm, seen)) return;
  const double rv = sm[0];
  if (!(fabs(rv) > 1e-300) || !isfinite(rv)) {
    if (lead()) st->done = isfinite(rv) ? 4 : 5;
    return;
  }
  const double alpha = rho / rv;
  if (lead()) st->alpha[par] = alpha;
  int64_t lo, hi;
  int lb;
  const bool fb = face_block(C, lo, hi, lb);
  const int64_t off = C.nf * D;
  const QSNewU<D> inu{r, v, q, alpha};
  const QSNewP inp{r + off, v + off, q + off, alpha};
  double acc[2] = {0.0, 0.0};
  if (fb) {
    for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
      double y[D];
      coupled_face_row_ns<D>(M.Ablk, M.cols, M.an, M.fel, C.nf, f, inu, inp, y);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int64_t e = f * D + i;
        const double si = r[e] - alpha * v[e], ti = q[e] * y[i];
        sv[e] = si;
        t[e] = ti;
        acc[0] += ti * si;
        acc[1] += ti * ti;
      }
    }
  } else {
    for (int64_t k = lo + threadIdx.x; k < hi; k += NT) {
      const int64_t e = off + k;
      const double si = r[e] - alpha * v[e], ti = q[e] * coupled_elem_row<D>(M.ea, M.eface, C.ne, k, inu);
      sv[e] = si;
      t[e] = ti;
      acc[0] += ti * si;
      acc[1] += ti * ti;
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    pc[(int64_t)lb * NPART] = acc[0];
    pc[(int64_t)lb * NPART + 1] = acc[1];
  }
}

// CB3: omega = t.s / t.t; x += Q (alpha p + omega s); r = s - omega t; partials rhat.r, r.r
__global__ void __launch_bounds__(NT) k_cb_3(CDims C, int64_t n, const double* __restrict__ q,
                                             const double* __restrict__ p, const double* __restrict__ sv,
                                             const double* __restrict__ t, const double* __restrict__ rhat,
                                             double* __restrict__ r, double* __restrict__ x,
                                             const double* __restrict__ pc, double* __restrict__ pa,
                                             BState* __restrict__ st, int par) {
  const int seen = st->done;
  const double alpha = st->alpha[par];
  double sm[2];
  if (reduce_partials_stop<2>(pc, C.nbf + C.nbe, 0, sm, seen)) return;
  const double omega = sm[1] > 0.0 ? sm[0] / sm[1] : 0.0;
  if (lead()) st->omega[par] = omega;
  const int nb = C.nbf + C.nbe;
  const int lb = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int64_t per = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)lb * per, hi = min(n, lo + per);
  double acc[2] = {0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
    x[i] += q[i] * (alpha * p[i] + omega * sv[i]);
    const double ri = sv[i] - omega * t[i];
    r[i] = ri;
    acc[0] += rhat[i] * ri;
    acc[1] += ri * ri;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    pa[(int64_t)lb * NPART] = acc[0];
    pa[(int64_t)lb * NPART + 1] = acc[1];
  }
}

struct CWs {
  CDims dims{};
  int64_t n = 0;
  double* Aval = nullptr;
  double* an = nullptr;
  double* ea = nullptr;
  double* b = nullptr;
  double* dinv = nullptr;
  double* x = nullptr;
  double* v = nullptr;
  double* R[3] = {};
  double* W[3] = {};
  double* pa = nullptr;
  double* pb = nullptr;
  double* pc = nullptr;
  CState* st = nullptr;
  CState* hst = nullptr;
  hipEvent_t ev[2] = {};
  bool assembled = false;
  // Newton step (BiCGStab): A blocks, element matrices, Q = sqrt(dinv), the
  // second direction buffer and the state; the other vectors reuse R and W
  double* Ablk = nullptr;
  double* amat = nullptr;
  double* q = nullptr;
  double* v1 = nullptr;
  BState* bst = nullptr;
  BState* hbst = nullptr;
};

CDims make_dims(int64_t nf, int64_t ne) {
  CDims C;
  C.nf = nf;
  C.ne = ne;
  auto part = [](int64_t rows, int& nb, int64_t& chunk) {
    const int64_t tiles = (rows + (int64_t)NT * (MAXBLK / 2) - 1) / ((int64_t)NT * (MAXBLK / 2));
    chunk = std::max<int64_t>(1, tiles) * NT;
    int64_t b = (rows + chunk - 1) / chunk;
    nb = (int)((b + 7) / 8 * 8);
  };
  part(nf, C.nbf, C.cf);
  part(ne, C.nbe, C.ce);
  return C;
}

cr_status ensure_cws(cr_system* s, CWs*& w) {
  w = (CWs*)s->cws;
  if (w) return CR_OK;
  w = new CWs();
  const int d = s->d;
  w->dims = make_dims(s->nf, s->ne);
  w->n = s->nf * d + s->ne;
  const size_t vb = sizeof(double) * w->n;
  w->Aval = (double*)dev_alloc(s, sizeof(double) * (2 * d + 1) * s->nf);
  w->an = (double*)dev_alloc(s, sizeof(double) * d * s->nf);
  w->ea = (double*)dev_alloc(s, sizeof(double) * (d + 1) * d * s->ne);
  w->b = (double*)dev_alloc(s, vb);
  w->dinv = (double*)dev_alloc(s, vb);
  w->x = (double*)dev_alloc(s, vb);
  w->v = (double*)dev_alloc(s, vb);
  for (auto& r : w->R) r = (double*)dev_alloc(s, vb);
  for (auto& r : w->W) r = (double*)dev_alloc(s, vb);
  const size_t pbytes = sizeof(double) * (w->dims.nbf + w->dims.nbe) * NPART;
  w->pa = (double*)dev_alloc(s, pbytes);
  w->pb = (double*)dev_alloc(s, pbytes);
  w->pc = (double*)dev_alloc(s, pbytes);
  w->st = (CState*)dev_alloc(s, sizeof(CState));
  if (!w->Aval || !w->an || !w->ea || !w->b || !w->dinv || !w->x || !w->v || !w->R[2] || !w->W[2] || !w->pc ||
      !w->st) {
    delete w;
    w = nullptr;
    return CR_E_NOMEM;
  }
  cr_status st = check_hip(hipHostMalloc((void**)&w->hst, 2 * sizeof(CState), hipHostMallocDefault), "pinned");
  for (auto& e : w->ev)
    if (st == CR_OK) st = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  if (st != CR_OK) {
    delete w;
    w = nullptr;
    return st;
  }
  s->cws = w;
  return CR_OK;
}

void free_cws(CWs* w) {
  if (!w) return;
  if (w->hbst) (void)hipHostFree(w->hbst);
  for (auto& e : w->ev)
    if (e) (void)hipEventDestroy(e);
  if (w->hst) (void)hipHostFree(w->hst);
  delete w;
}

template <int D>
void enqueue_mr(cr_system* s, CWs* w, int k0, int niter) {
  const CDims C = w->dims;
  const MatArgs M{w->Aval, s->cols, w->an, s->fel, w->ea, s->eface};
  const dim3 grid(C.nbf + C.nbe), blk(NT);
  for (int k = k0; k < k0 + niter; ++k) {
    const int q = k & 1;
    double* r1 = w->R[k % 3];
    double* r2 = w->R[(k + 1) % 3];
    double* y = w->R[(k + 2) % 3];
    double* w2old = w->W[k % 3];
    double* wold = w->W[(k + 1) % 3];
    double* wnew = w->W[(k + 2) % 3];
    hipLaunchKernelGGL(k_mr_a<D>, grid, blk, 0, s->stream, C, M, w->dinv, r1, r2, w->v, y, w->pa, w->pb, w->st, q);
    hipLaunchKernelGGL(k_mr_b, grid, blk, 0, s->stream, C, w->n, w->dinv, r2, y, w->pb, w->pc, w->st, q);
    hipLaunchKernelGGL(k_mr_c, grid, blk, 0, s->stream, C, w->n, w->v, w2old, wold, wnew, w->x, w->pc, w->st, q);
  }
}

// the coupled matrix, its right-hand side and the preconditioner, on the device
template <int D>
cr_status coupled_assemble(cr_system* s, CWs*& w) {
  cr_status st = ensure_cws(s, w);
  if (st != CR_OK) return st;
  hipLaunchKernelGGL(k_coupled_faces<D>, dim3((unsigned)((s->nf + 127) / 128)), dim3(128), 0, s->stream, s->nf, s->ne,
                     s->ecoord, s->eflags, s->fel, s->floc, s->RK, s->params.mu, s->params.nu, w->Aval, w->an, w->b,
                     w->dinv);
  hipLaunchKernelGGL(k_coupled_elems<D>, dim3((unsigned)((s->ne + 127) / 128)), dim3(128), 0, s->stream, s->nf, s->ne,
                     s->ecoord, s->eflags, s->eface, w->Aval, s->has_bnd ? s->ek : nullptr, w->ea, w->b, w->dinv);
  return check_hip(hipGetLastError(), "coupled assembly");
}

template <int D>
cr_status coupled_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info, double* U, double* P) {
  auto t0 = std::chrono::steady_clock::now();
  CWs* w = nullptr;
  cr_status st = coupled_assemble<D>(s, w);
  if (st != CR_OK) return st;
  const CDims C = w->dims;
  const MatArgs M{w->Aval, s->cols, w->an, s->fel, w->ea, s->eface};
  st = check_hip(hipMemsetAsync(w->x, 0, sizeof(double) * w->n, s->stream), "coupled x");
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  const int maxit = o->maxit > 0 ? o->maxit : 200000;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 20;
  int blk = o->check_every > 0 ? o->check_every : 48;
  blk = std::max(6, (blk + 5) / 6 * 6);
  int total = 0, outer = 0, reason = 0;
  double rel = -1.0;
  const dim3 grid(C.nbf + C.nbe), tb(NT);
  while (st == CR_OK) {
    const bool last = outer >= max_outer || total >= maxit;
    CState* h = &w->hst[1];
    h->tol2 = tol * tol;
    h->maxit = last ? 0 : maxit - total;
    const size_t off = offsetof(CState, tol2);
    st = check_hip(hipMemcpyAsync((char*)w->st + off, (char*)h + off, sizeof(CState) - off, hipMemcpyHostToDevice,
                                  s->stream), "coupled params");
    if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "coupled params");
    if (st != CR_OK) break;
    hipLaunchKernelGGL(k_mr_init<D>, grid, tb, 0, s->stream, C, M, w->b, w->dinv, w->x, w->R[0], w->R[1], w->W[0],
                       w->W[1], w->pa, w->st);
    ++outer;
    // iterate in blocks, polling the device flag after each
    int issued = 0;
    const int max_blocks = (last ? 0 : maxit - total) / blk + 2;
    CState ks{};
    for (;;) {
      enqueue_mr<D>(s, w, issued * blk, blk);
      ++issued;
      st = check_hip(hipGetLastError(), "coupled launch");
      if (st == CR_OK)
        st = check_hip(hipMemcpyAsync(&w->hst[0], w->st, sizeof(CState), hipMemcpyDeviceToHost, s->stream),
                       "coupled state copy");
      if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "coupled poll");
      if (st != CR_OK) break;
      ks = w->hst[0];
      if (ks.done || issued >= max_blocks) break;
    }
    if (st != CR_OK) break;
    total += ks.iters;
    rel = ks.bnorm2 > 0 ? std::sqrt(ks.tres2 / ks.bnorm2) : std::sqrt(ks.tres2);
    if (ks.done == 2) {
      reason = 1;
      break;
    }
    if (ks.done == 4 || ks.done == 5) {
      reason = ks.done;
      break;
    }
    if (last) {
      reason = 3;
      break;
    }
  }
  if (st == CR_OK) {
    hipLaunchKernelGGL(k_mr_scatter<D>, dim3((unsigned)((s->nf + s->ne + 255) / 256)), dim3(256), 0, s->stream, s->nf,
                       s->ne, w->x, s->fcanon, s->ecaller, U, P);
    st = check_hip(hipStreamSynchronize(s->stream), "coupled scatter");
  }
  if (st != CR_OK) return st;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->iters = total;
    info->outer_iters = outer;
    info->rel_residual = rel;
    info->t_solve_ms = ms;
    info->reason = reason;
  }
  if (reason == 1) return CR_OK;
  if (reason == 4 || reason == 5) {
    set_error("coupled MINRES breakdown after %d iterations", total);
    return reason == 4 ? CR_E_BREAKDOWN : CR_E_NONFINITE;
  }
  set_error("coupled MINRES: relative residual %.3e after %d iterations", rel, total);
  return CR_E_NOCONV;
}

__global__ void k_sqrt_vec(int64_t n, const double* __restrict__ a, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = sqrt(a[i]);
}

// the Newton-step coupled matrix, its right-hand side and the scaling, on the device
template <int D>
cr_status coupled_assemble_ns(cr_system* s, CWs*& w) {
  cr_status st = ensure_cws(s, w);
  if (st != CR_OK) return st;
  constexpr int NU = NsPack<D>::NU;
  const Bnd bnd{s->has_bnd ? s->ebf : nullptr, s->gbnd, nullptr};
  if (!w->Ablk) {
    w->Ablk = (double*)dev_alloc(s, sizeof(double) * (2 * D + 1) * D * D * s->nf);
    w->amat = (double*)dev_alloc(s, sizeof(double) * NU * NU * s->ne);
    w->q = (double*)dev_alloc(s, sizeof(double) * w->n);
    w->v1 = (double*)dev_alloc(s, sizeof(double) * w->n);
    w->bst = (BState*)dev_alloc(s, sizeof(BState));
    if (!w->Ablk || !w->amat || !w->q || !w->v1 || !w->bst) return CR_E_NOMEM;
    st = check_hip(hipHostMalloc((void**)&w->hbst, 2 * sizeof(BState), hipHostMallocDefault), "pinned");
    if (st != CR_OK) return st;
  }
  if constexpr (D == 2) {
    hipLaunchKernelGGL(k_ns_amat2, dim3((unsigned)((s->ne + 127) / 128)), dim3(128), 0, s->stream, s->ne, s->ecoord,
                       s->eflags, s->eface, s->ulin, s->params.mu, s->params.nu, bnd, w->amat);
  } else {
    const size_t lds = sizeof(double) * 144 * BS_AM3;
    st = check_hip(hipFuncSetAttribute((const void*)k_ns_amat3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                   "coupled Newton-step LDS size");
    if (st != CR_OK) return st;
    hipLaunchKernelGGL(k_ns_amat3, dim3((unsigned)((s->ne + BS_AM3 - 1) / BS_AM3)), dim3(BS_AM3), lds, s->stream,
                       s->ne, s->ecoord, s->eflags, s->eface, s->ulin, s->params.mu, s->params.nu, bnd, w->amat);
  }
  hipLaunchKernelGGL(k_coupled_faces_ns<D>, dim3((unsigned)((s->nf + 127) / 128)), dim3(128), 0, s->stream, s->nf,
                     s->ne, s->ecoord, s->eflags, s->fel, s->floc, s->RK, w->amat, w->Ablk, w->an, w->b, w->dinv);
  hipLaunchKernelGGL(k_coupled_elems_ns<D>, dim3((unsigned)((s->ne + 127) / 128)), dim3(128), 0, s->stream, s->nf,
                     s->ne, s->ecoord, s->eflags, s->eface, w->Ablk, s->has_bnd ? s->ek : nullptr, w->ea, w->b,
                     w->dinv);
  hipLaunchKernelGGL(k_sqrt_vec, dim3((unsigned)((w->n + 255) / 256)), dim3(256), 0, s->stream, w->n, w->dinv, w->q);
  return check_hip(hipGetLastError(), "coupled Newton-step assembly");
}

template <int D>
cr_status coupled_bicgstab(cr_system* s, const cr_solve_opts* o, cr_solve_info* info, double* U, double* P) {
  auto t0 = std::chrono::steady_clock::now();
  CWs* w = nullptr;
  cr_status st = coupled_assemble_ns<D>(s, w);
  if (st != CR_OK) return st;
  const CDims C = w->dims;
  const NsMat M{w->Ablk, s->cols, w->an, s->fel, w->ea, s->eface};
  double* r = w->R[0];
  double* rhat = w->R[1];
  double* sv = w->R[2];
  double* t = w->W[2];
  double* pv[2] = {w->W[0], w->W[1]};
  double* vv[2] = {w->v, w->v1};
  st = check_hip(hipMemsetAsync(w->x, 0, sizeof(double) * w->n, s->stream), "coupled x");
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  const int maxit = o->maxit > 0 ? o->maxit : 200000;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 50;
  const int blk = std::max(2, ((o->check_every > 0 ? o->check_every : 48) + 1) / 2 * 2);
  int total = 0, outer = 0, reason = 0, stuck = 0;
  double rel = -1.0;
  const dim3 grid(C.nbf + C.nbe), tb(NT);
  while (st == CR_OK) {
    const bool last = outer >= max_outer || total >= maxit;
    BState* h = &w->hbst[1];
    h->tol2 = tol * tol;
    h->maxit = last ? 0 : maxit - total;
    const size_t off = offsetof(BState, tol2);
    st = check_hip(hipMemcpyAsync((char*)w->bst + off, (char*)h + off, sizeof(BState) - off, hipMemcpyHostToDevice,
                                  s->stream), "coupled params");
    if (st != CR_OK) break;
    hipLaunchKernelGGL(k_cb_init<D>, grid, tb, 0, s->stream, C, M, w->b, w->q, w->x, r, rhat, pv[0], pv[1], vv[0],
                       vv[1], w->pa, w->bst);
    ++outer;
    int k = 0;
    const int max_iter_pass = (last ? 0 : maxit - total) + 2;
    BState ks{};
    for (;;) {
      for (int j = 0; j < blk; ++j, ++k) {
        const int par = k & 1;
        hipLaunchKernelGGL(k_cb_1<D>, grid, tb, 0, s->stream, C, M, w->q, r, rhat, pv[par ^ 1], vv[par ^ 1], pv[par],
                           vv[par], w->pa, w->pb, w->bst, par);
        hipLaunchKernelGGL(k_cb_2<D>, grid, tb, 0, s->stream, C, M, w->q, r, vv[par], sv, t, w->pb, w->pc, w->bst,
                           par);
        hipLaunchKernelGGL(k_cb_3, grid, tb, 0, s->stream, C, w->n, w->q, pv[par], sv, t, rhat, r, w->x, w->pc,
                           w->pa, w->bst, par);
      }
      st = check_hip(hipGetLastError(), "coupled launch");
      if (st == CR_OK)
        st = check_hip(hipMemcpyAsync(&w->hbst[0], w->bst, sizeof(BState), hipMemcpyDeviceToHost, s->stream),
                       "coupled state copy");
      if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "coupled poll");
      if (st != CR_OK) break;
      ks = w->hbst[0];
      if (ks.done || k >= max_iter_pass) break;
    }
    if (st != CR_OK) break;
    total += ks.iters;
    rel = ks.bnorm2 > 0 ? std::sqrt(ks.tres2 / ks.bnorm2) : std::sqrt(ks.tres2);
    if (ks.done == 1 && ks.iters == 0) {
      reason = 1;  // the true residual at the start of this pass meets the tolerance
      break;
    }
    if (ks.done == 5) {
      reason = 5;
      break;
    }
    if (ks.iters == 0 && ks.done == 4 && ++stuck >= 3) {
      reason = 4;
      break;
    }
    if (last || (ks.done == 3)) {
      reason = 3;
      if (!last) continue;  // one more pass evaluates the true residual of the final iterate
      break;
    }
  }
  if (st == CR_OK) {
    hipLaunchKernelGGL(k_mr_scatter<D>, dim3((unsigned)((s->nf + s->ne + 255) / 256)), dim3(256), 0, s->stream, s->nf,
                       s->ne, w->x, s->fcanon, s->ecaller, U, P);
    st = check_hip(hipStreamSynchronize(s->stream), "coupled scatter");
  }
  if (st != CR_OK) return st;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->iters = total;
    info->outer_iters = outer;
    info->rel_residual = rel;
    info->t_solve_ms = ms;
    info->reason = reason;
  }
  if (reason == 1) return CR_OK;
  if (reason == 4 || reason == 5) {
    set_error("coupled BiCGStab breakdown after %d iterations (relative residual %.3e)", total, rel);
    return reason == 4 ? CR_E_BREAKDOWN : CR_E_NONFINITE;
  }
  set_error("coupled BiCGStab: relative residual %.3e after %d iterations", rel, total);
  return CR_E_NOCONV;
}

}  // namespace

cr_status run_coupled_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info, double* U, double* P) {
  if (s->params.problem == CR_NS_NEWTON)
    return s->d == 2 ? coupled_bicgstab<2>(s, o, info, U, P) : coupled_bicgstab<3>(s, o, info, U, P);
  return s->d == 2 ? coupled_solve<2>(s, o, info, U, P) : coupled_solve<3>(s, o, info, U, P);
}

// The coupled matrix [A D^t; D 0] in canonical order as CSR: velocity rows
// (canonical face, component), then one pressure row per element in caller
// order without K0; columns sorted in each row.  Assembled by the coupled
// baseline's kernels, copied to the host and reordered there.
cr_status run_coupled_export(cr_system* s, int64_t* rowptr, int32_t* col, double* val, double* R) {
  CWs* w = nullptr;
  cr_status st = s->d == 2 ? coupled_assemble<2>(s, w) : coupled_assemble<3>(s, w);
  if (st != CR_OK) return st;
  const int d = s->d, d1 = d + 1;
  const int64_t nf = s->nf, ne = s->ne, nu = nf * d;
  std::vector<double> Aval((size_t)(2 * d + 1) * nf), an((size_t)d * nf), ea((size_t)d1 * d * ne),
      b((size_t)nf * d + ne);
  std::vector<int32_t> cols((size_t)2 * d * nf);
  auto get = [&](void* dst, const void* src, size_t bytes) {
    if (st == CR_OK) st = check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream), "export coupled");
  };
  get(Aval.data(), w->Aval, Aval.size() * 8);
  get(an.data(), w->an, an.size() * 8);
  get(ea.data(), w->ea, ea.size() * 8);
  get(b.data(), w->b, b.size() * 8);
  get(cols.data(), s->cols, cols.size() * 4);
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "export coupled");
  if (st != CR_OK) return st;
  const Topology& t = s->topo;
  const int32_t k0 = s->params.k0;
  auto pcol = [&](int32_t c) { return (int32_t)(nu + (c < k0 ? c : c - 1)); };
  // the rows in order; emit(r, rhs) receives each row's entries in `row`
  std::vector<std::pair<int32_t, double>> row;
  auto rows = [&](auto&& emit) {
    for (int64_t fc = 0; fc < nf; ++fc) {
      const int64_t f = t.face_perm[fc];
      const int32_t own = t.face_elem[2 * fc], oth = t.face_elem[2 * fc + 1];  // caller ids, owner (C = +1) first
      for (int i = 0; i < d; ++i) {
        row.clear();
        row.emplace_back((int32_t)(fc * d + i), Aval[f]);
        for (int sl = 1; sl <= 2 * d; ++sl) {
          const int64_t c = cols[(size_t)(sl - 1) * nf + f];
          if (c == f) continue;  // padding slot of an exterior face
          row.emplace_back((int32_t)(t.face_iperm[c] * d + i), Aval[(size_t)sl * nf + f]);
        }
        // D^t P at face f: -a_{K,f} (P_K - P_L), K the owner
        if (own != k0) row.emplace_back(pcol(own), -an[f * d + i]);
        if (oth != k0) row.emplace_back(pcol(oth), an[f * d + i]);
        emit(fc * d + i, b[f * d + i]);
      }
    }
    for (int32_t c = 0; c < (int32_t)ne; ++c) {
      if (c == k0) continue;
      const int64_t k = t.elem_perm[c];
      row.clear();
      // D U at element K: -sum_j a_{K,j} . U_j over its interior faces
      for (int j = 0; j < d1; ++j) {
        const int32_t fcan = t.elem_face[(int64_t)c * d1 + j];
        if (fcan < 0) continue;
        for (int i = 0; i < d; ++i) row.emplace_back((int32_t)(fcan * d + i), -ea[(size_t)(j * d + i) * ne + k]);
      }
      emit(pcol(c), b[(size_t)nu + k]);  // e_K (boundary data), else 0
    }
  };
  // count first: the caller's buffers hold coupled_nnz entries
  int64_t pos = 0;
  rows([&](int64_t, double) { pos += (int64_t)row.size(); });
  if (pos != coupled_nnz(s)) {
    set_error("coupled export: %lld entries where %lld are declared", (long long)pos, (long long)coupled_nnz(s));
    return CR_E_DEVICE;
  }
  pos = 0;
  rows([&](int64_t r, double rhs) {
    std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    if (rowptr) rowptr[r] = pos;
    for (auto& e : row) {
      if (col) col[pos] = e.first;
      if (val) val[pos] = e.second;
      ++pos;
    }
    if (R) R[r] = rhs;
  });
  if (rowptr) rowptr[nu + ne - 1] = pos;
  return CR_OK;
}

void free_coupled(cr_system* s) {
  free_cws((CWs*)s->cws);
  s->cws = nullptr;
}

}  // namespace crh
