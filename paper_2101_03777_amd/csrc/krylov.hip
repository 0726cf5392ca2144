// Step a4: Krylov solution of the hybridised system G W = S (Section 3.2, "hybrid
// method" step 2), HBM-bandwidth bound.
//
// Storage: G in block-ELL over interior faces (internal RCM order), one d x d
// block per slot, slot 0 the diagonal block, slots 1..2d the face's neighbours
// through its two elements; values as separate planes [slot][i][j][face] so
// that consecutive lanes read consecutive addresses.  Vectors are face-major
// [face][component].
//
// Jacobi preconditioning is folded into the matrix: the stored G is
// Ds G Ds with Ds = |diag G|^{-1/2}, and the solver works on y = W / Ds.
//
// Iterative refinement: the residual of the current FP64 y is computed with
// the FP64 plane; an inner Krylov solve (FP32 or FP64 plane) returns a
// correction; y += correction.  The FP64-only mode is the same loop with an
// FP64 inner solve.
//
// Kernel structure: every kernel processes a contiguous range of face rows per
// workgroup (remapped so that each XCD gets a contiguous eighth of the rows)
// and writes one partial sum per workgroup for each dot product it produces.
// The consuming kernel reduces the (few hundred) partials redundantly in every
// workgroup in a fixed order, so all workgroups see bit-identical scalars and
// no atomics or intra-kernel grid synchronisation are needed.  Per-iteration
// scalars alternate between two slots by iteration parity, which is a kernel
// argument, so an even number of iterations can be captured once in a hipGraph
// and replayed.  A device flag stops all later kernels once the iteration has
// converged or failed, so replays past convergence are no-ops.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace crh {
namespace {

constexpr int MAXBLK = 1024;   // upper bound on workgroups of the row kernels
constexpr int NPART = 4;       // doubles per partial record

struct KState {
  double rho[2];     // per parity: r.r (CG) or rhat.r (BiCGStab) at the start of the iteration
  double alpha[2];
  double omega[2];
  int it[2];         // iterations completed when the iteration of this parity started (+1)
  int done;          // 0 running, 1 inner converged, 2 outer converged, 3 limit, 4 breakdown, 5 non-finite
  int iters;         // iterations completed in the current inner solve
  double rr0, tres2, snorm2, thr2, last_rr;
  // parameters written by the host before each inner solve
  double inner_tol2, outer_tol2;
  int maxit;
  int pad;
};

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

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

template <typename T, int D>
struct Plain {
  const T* __restrict__ x;
  __device__ Vec<T, D> operator()(int64_t c) const { return ldv<T, D>(x, c); }
};

// ---------------------------------------------------------------------------
// refinement residual: r_s = bs - G64 y (FP64), inner right-hand side r = (T) r_s,
// inner iterate x = 0; partials: [0] r.r, [1] ||dsq r_s||^2 = ||S - G W||^2,
// [2] ||S||^2, [3] r.r (BiCGStab also takes rhat = r).
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ir_residual(Part P, const double* __restrict__ G64,
                                                    const int32_t* __restrict__ cols, const double* __restrict__ y,
                                                    const double* __restrict__ bs, const double* __restrict__ dsq,
                                                    T* __restrict__ r, T* __restrict__ x, T* __restrict__ rhat,
                                                    double* __restrict__ pa, KState* __restrict__ st) {
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<double, D> w = spmv_row<D, double>(G64, cols, P.nf, f, Plain<double, D>{y});
    Vec<T, D> rt, zero;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double b = bs[f * D + i], sq = dsq[f * D + i];
      const double rs = b - w.v[i];
      rt.v[i] = (T)rs;
      zero.v[i] = T(0);
      acc[0] += (double)rt.v[i] * (double)rt.v[i];
      acc[1] += (sq * rs) * (sq * rs);
      acc[2] += (sq * b) * (sq * b);
    }
    stv<T, D>(r, f, rt);
    stv<T, D>(x, f, zero);
    if (rhat) stv<T, D>(rhat, f, rt);
  }
  block_sum<3>(acc);
  if (threadIdx.x == 0) {
    pa[(int64_t)lb * NPART + 0] = acc[0];
    pa[(int64_t)lb * NPART + 1] = acc[1];
    pa[(int64_t)lb * NPART + 2] = acc[2];
    pa[(int64_t)lb * NPART + 3] = acc[0];
  }
  if (lead()) {
    st->it[1] = 0;
    st->rho[1] = 1.0;
    st->alpha[1] = 1.0;
    st->omega[1] = 1.0;
    st->iters = 0;
    st->done = 0;
  }
}

// common stopping logic of the first kernel of an iteration; rr = ||r||^2 of the
// inner system, v1/v2 = true residual / ||S||^2 partial sums (first iteration only)
__device__ __forceinline__ int stop_check(KState* st, int it, double rr, double v1, double v2, bool first,
                                          double& thr2) {
  if (first) {
    const double ratio = v1 > 0.0 ? v2 * rr / v1 : 0.0;
    thr2 = fmax(st->inner_tol2 * rr, 0.01 * st->outer_tol2 * ratio);
  } else {
    thr2 = st->thr2;
  }
  if (first && v1 <= st->outer_tol2 * v2) return 2;
  if (!isfinite(rr)) return 5;
  if (it >= st->maxit) return 3;
  if (rr <= thr2) return 1;
  return 0;
}

// ---------------------------------------------------------------------------
// CG on the scaled SPD system.  K1: w = G r, p = r + beta p, q = w + beta q
// (q = G p without a second product), partial p.q.  K2: alpha = rho / p.q,
// x += alpha p, r -= alpha q, partial r.r.
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_spmv(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                                const T* __restrict__ r, T* __restrict__ p, T* __restrict__ q,
                                                const double* __restrict__ pa, double* __restrict__ pb,
                                                KState* __restrict__ st, int par) {
  if (st->done) return;
  double v[3];
  reduce_partials<3>(pa, P.nblk, 0, v);
  const int it = st->it[par ^ 1];
  const bool first = it == 0;
  const double rr = v[0];
  double thr2;
  const int done = stop_check(st, it, rr, v[1], v[2], first, thr2);
  if (lead()) {
    if (first) {
      st->rr0 = rr;
      st->tres2 = v[1];
      st->snorm2 = v[2];
      st->thr2 = thr2;
    }
    st->rho[par] = rr;
    st->it[par] = it + 1;
    st->iters = it;
    st->last_rr = rr;
    if (done) st->done = done;
  }
  if (done) return;
  const T beta = first ? T(0) : (T)(rr / st->rho[par ^ 1]);
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> w = spmv_row<D, T>(G, cols, P.nf, f, Plain<T, D>{r});
    Vec<T, D> ri = ldv<T, D>(r, f), pi, qi;
    if (first) {
      pi = ri;
      qi = w;
    } else {
      pi = ldv<T, D>(p, f);
      qi = ldv<T, D>(q, f);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        pi.v[i] = ri.v[i] + beta * pi.v[i];
        qi.v[i] = w.v[i] + beta * qi.v[i];
      }
    }
    stv<T, D>(p, f, pi);
    stv<T, D>(q, f, qi);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[0] += (double)pi.v[i] * (double)qi.v[i];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pb[(int64_t)lb * NPART] = acc[0];
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_update(Part P, T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ p, const T* __restrict__ q,
                                                  const double* __restrict__ pb, double* __restrict__ pa,
                                                  KState* __restrict__ st, int par) {
  if (st->done) return;
  double v[1];
  reduce_partials<1>(pb, P.nblk, 0, v);
  const double pq = v[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead()) st->done = isfinite(pq) ? 4 : 5;
    return;
  }
  const double alpha = st->rho[par] / pq;
  const T ta = (T)alpha;
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> xi = ldv<T, D>(x, f), ri = ldv<T, D>(r, f), pi = ldv<T, D>(p, f), qi = ldv<T, D>(q, f);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xi.v[i] += ta * pi.v[i];
      ri.v[i] -= ta * qi.v[i];
      acc[0] += (double)ri.v[i] * (double)ri.v[i];
    }
    stv<T, D>(x, f, xi);
    stv<T, D>(r, f, ri);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pa[(int64_t)lb * NPART] = acc[0];
  if (lead()) st->alpha[par] = alpha;
}

// ---------------------------------------------------------------------------
// BiCGStab on the scaled system (non-symmetric G).  Three kernels per
// iteration; the direction p and the intermediate s are formed on the fly from
// double-buffered vectors inside the products that consume them:
//   B1: p_new = r + beta (p_old - omega v_old) gathered on the fly, v = G p_new,
//       partial rhat.v
//   B2: alpha = rho / rhat.v, s = r - alpha v gathered on the fly, t = G s,
//       partials t.s, t.t
//   B3: omega = t.s / t.t, x += alpha p + omega s, r = s - omega t,
//       partials rhat.r, r.r
// ---------------------------------------------------------------------------
template <typename T, int D>
struct PNew {
  const T* __restrict__ r;
  const T* __restrict__ p;
  const T* __restrict__ v;
  T beta, omega;
  bool first;
  __device__ Vec<T, D> operator()(int64_t c) const {
    Vec<T, D> a = ldv<T, D>(r, c);
    if (first) return a;
    Vec<T, D> b = ldv<T, D>(p, c), e = ldv<T, D>(v, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] += beta * (b.v[i] - omega * e.v[i]);
    return a;
  }
};

template <typename T, int D>
struct SNew {
  const T* __restrict__ r;
  const T* __restrict__ v;
  T alpha;
  __device__ Vec<T, D> operator()(int64_t c) const {
    Vec<T, D> a = ldv<T, D>(r, c), e = ldv<T, D>(v, c);
#pragma unroll
    for (int i = 0; i < D; ++i) a.v[i] -= alpha * e.v[i];
    return a;
  }
};

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_bicg_1(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                               const T* __restrict__ r, const T* __restrict__ rhat,
                                               const T* __restrict__ p_old, const T* __restrict__ v_old,
                                               T* __restrict__ p_new, T* __restrict__ v_new,
                                               const double* __restrict__ pa, double* __restrict__ pb,
                                               KState* __restrict__ st, int par) {
  if (st->done) return;
  double v[4];
  reduce_partials<4>(pa, P.nblk, 0, v);
  const int it = st->it[par ^ 1];
  const bool first = it == 0;
  const double rho = v[0], rr = v[3];
  double thr2;
  int done = stop_check(st, it, rr, v[1], v[2], first, thr2);
  if (!done && (!(rho != 0.0) || !isfinite(rho))) done = isfinite(rho) ? 4 : 5;
  if (lead()) {
    if (first) {
      st->rr0 = rr;
      st->tres2 = v[1];
      st->snorm2 = v[2];
      st->thr2 = thr2;
    }
    st->rho[par] = rho;
    st->it[par] = it + 1;
    st->iters = it;
    st->last_rr = rr;
    if (done) st->done = done;
  }
  if (done) return;
  const double beta = first ? 0.0 : (rho / st->rho[par ^ 1]) * (st->alpha[par ^ 1] / st->omega[par ^ 1]);
  const PNew<T, D> in{r, p_old, v_old, (T)beta, (T)st->omega[par ^ 1], first};
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> w = spmv_row<D, T>(G, cols, P.nf, f, in);
    Vec<T, D> pn = in(f), rh = ldv<T, D>(rhat, f);
    stv<T, D>(p_new, f, pn);
    stv<T, D>(v_new, f, w);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[0] += (double)rh.v[i] * (double)w.v[i];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) pb[(int64_t)lb * NPART] = acc[0];
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_bicg_2(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                               const T* __restrict__ r, const T* __restrict__ v_new,
                                               T* __restrict__ s, T* __restrict__ t, const double* __restrict__ pb,
                                               double* __restrict__ pc, KState* __restrict__ st, int par) {
  if (st->done) return;
  double v[1];
  reduce_partials<1>(pb, P.nblk, 0, v);
  const double rv = v[0];
  if (!(rv != 0.0) || !isfinite(rv)) {
    if (lead()) st->done = isfinite(rv) ? 4 : 5;
    return;
  }
  const double alpha = st->rho[par] / rv;
  const SNew<T, D> in{r, v_new, (T)alpha};
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[2] = {0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> w = spmv_row<D, T>(G, cols, P.nf, f, in);
    Vec<T, D> si = in(f);
    stv<T, D>(s, f, si);
    stv<T, D>(t, f, w);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      acc[0] += (double)w.v[i] * (double)si.v[i];
      acc[1] += (double)w.v[i] * (double)w.v[i];
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    pc[(int64_t)lb * NPART] = acc[0];
    pc[(int64_t)lb * NPART + 1] = acc[1];
  }
  if (lead()) st->alpha[par] = alpha;
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_bicg_3(Part P, T* __restrict__ x, T* __restrict__ r,
                                               const T* __restrict__ rhat, const T* __restrict__ p_new,
                                               const T* __restrict__ s, const T* __restrict__ t,
                                               const double* __restrict__ pc, double* __restrict__ pa,
                                               KState* __restrict__ st, int par) {
  if (st->done) return;
  double v[2];
  reduce_partials<2>(pc, P.nblk, 0, v);
  const double ts = v[0], tt = v[1];
  if (!(tt > 0.0) || !isfinite(tt) || !isfinite(ts)) {
    if (lead()) st->done = (isfinite(tt) && isfinite(ts)) ? 4 : 5;
    return;
  }
  const double omega = ts / tt;
  const T ta = (T)st->alpha[par], to = (T)omega;
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[2] = {0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> xi = ldv<T, D>(x, f), pi = ldv<T, D>(p_new, f), si = ldv<T, D>(s, f), ti = ldv<T, D>(t, f),
              rh = ldv<T, D>(rhat, f), ri;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xi.v[i] += ta * pi.v[i] + to * si.v[i];
      ri.v[i] = si.v[i] - to * ti.v[i];
      acc[0] += (double)rh.v[i] * (double)ri.v[i];
      acc[1] += (double)ri.v[i] * (double)ri.v[i];
    }
    stv<T, D>(x, f, xi);
    stv<T, D>(r, f, ri);
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    pa[(int64_t)lb * NPART] = acc[0];
    pa[(int64_t)lb * NPART + 3] = acc[1];
  }
  if (lead()) st->omega[par] = omega;
}

// y += x (FP64 accumulation of the inner correction)
template <typename T>
__global__ void __launch_bounds__(NT) k_ir_update(int64_t n, double* __restrict__ y, const T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) y[i] += (double)x[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct KWs {
  int64_t nf = 0;
  int d = 0;
  Part part{};
  void* vec[9] = {};          // x, r, rhat, p0, p1, v0, v1, s, t (each nf*d doubles)
  double* pa = nullptr;
  double* pb = nullptr;
  double* pc = nullptr;
  KState* st = nullptr;
  KState* hst = nullptr;      // pinned [3]
  hipEvent_t ev[2] = {};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[2][2] = {};  // [precision][method]
  int exec_m[2][2] = {};
  // scratch for kernel timing
  void* tvec[3] = {};
  double* tpart[2] = {};
  KState* tst = nullptr;
};

Part make_part(int64_t nf) {
  Part P;
  P.nf = nf;
  const int64_t tiles = (nf + (int64_t)NT * MAXBLK - 1) / ((int64_t)NT * MAXBLK);
  P.chunk = std::max<int64_t>(1, tiles) * NT;
  int64_t nb = (nf + P.chunk - 1) / P.chunk;
  nb = (nb + 7) / 8 * 8;
  P.nblk = (int)nb;
  return P;
}

cr_status ensure_ws(cr_system* s, KWs*& w) {
  w = (KWs*)s->kws;
  if (w) return CR_OK;
  w = new KWs();
  w->nf = s->nf;
  w->d = s->d;
  w->part = make_part(s->nf);
  const size_t vb = sizeof(double) * (size_t)s->nf * s->d;
  for (auto& v : w->vec) {
    v = dev_alloc(s, vb);
    if (!v) return CR_E_NOMEM;
  }
  const size_t pbytes = sizeof(double) * (size_t)w->part.nblk * NPART;
  w->pa = (double*)dev_alloc(s, pbytes);
  w->pb = (double*)dev_alloc(s, pbytes);
  w->pc = (double*)dev_alloc(s, pbytes);
  w->st = (KState*)dev_alloc(s, sizeof(KState));
  if (!w->pa || !w->pb || !w->pc || !w->st) return CR_E_NOMEM;
  cr_status st = check_hip(hipHostMalloc((void**)&w->hst, 3 * sizeof(KState), hipHostMallocDefault), "pinned state");
  if (st != CR_OK) return st;
  for (auto& e : w->ev) {
    st = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    if (st != CR_OK) return st;
  }
  st = check_hip(hipEventCreate(&w->t0), "event");
  if (st == CR_OK) st = check_hip(hipEventCreate(&w->t1), "event");
  if (st == CR_OK) st = check_hip(hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking), "capture stream");
  if (st != CR_OK) return st;
  s->kws = w;
  return CR_OK;
}

struct Launch {
  cr_system* s;
  KWs* w;
  int prec;    // CR_FP64 or CR_FP32_IR
  int method;  // CR_PCG or CR_BICGSTAB
};

template <int D, typename T>
void enqueue_iters(const Launch& L, hipStream_t stream, int npairs) {
  KWs* w = L.w;
  const Part P = w->part;
  const T* G = std::is_same<T, float>::value ? (const T*)L.s->G32 : (const T*)L.s->G64;
  T* x = (T*)w->vec[0];
  T* r = (T*)w->vec[1];
  T* rh = (T*)w->vec[2];
  T* pv[2] = {(T*)w->vec[3], (T*)w->vec[4]};
  T* vv[2] = {(T*)w->vec[5], (T*)w->vec[6]};
  T* s = (T*)w->vec[7];
  T* t = (T*)w->vec[8];
  const dim3 grid(P.nblk), blk(NT);
  for (int k = 0; k < npairs; ++k)
    for (int par = 0; par < 2; ++par) {
      if (L.method == CR_PCG) {
        hipLaunchKernelGGL((k_cg_spmv<D, T>), grid, blk, 0, stream, P, G, L.s->cols, r, pv[0], vv[0], w->pa, w->pb,
                           w->st, par);
        hipLaunchKernelGGL((k_cg_update<D, T>), grid, blk, 0, stream, P, x, r, pv[0], vv[0], w->pb, w->pa, w->st,
                           par);
      } else {
        hipLaunchKernelGGL((k_bicg_1<D, T>), grid, blk, 0, stream, P, G, L.s->cols, r, rh, pv[par ^ 1], vv[par ^ 1],
                           pv[par], vv[par], w->pa, w->pb, w->st, par);
        hipLaunchKernelGGL((k_bicg_2<D, T>), grid, blk, 0, stream, P, G, L.s->cols, r, vv[par], s, t, w->pb, w->pc,
                           w->st, par);
        hipLaunchKernelGGL((k_bicg_3<D, T>), grid, blk, 0, stream, P, x, r, rh, pv[par], s, t, w->pc, w->pa, w->st,
                           par);
      }
    }
}

void enqueue_iters_any(const Launch& L, hipStream_t stream, int npairs) {
  const bool f32 = L.prec == CR_FP32_IR;
  if (L.s->d == 2) {
    if (f32)
      enqueue_iters<2, float>(L, stream, npairs);
    else
      enqueue_iters<2, double>(L, stream, npairs);
  } else {
    if (f32)
      enqueue_iters<3, float>(L, stream, npairs);
    else
      enqueue_iters<3, double>(L, stream, npairs);
  }
}

void enqueue_residual(const Launch& L) {
  KWs* w = L.w;
  const Part P = w->part;
  const dim3 grid(P.nblk), blk(NT);
  void* rh = L.method == CR_BICGSTAB ? w->vec[2] : nullptr;
  const bool f32 = L.prec == CR_FP32_IR;
  cr_system* s = L.s;
#define CRH_RES(D, T)                                                                                        \
  hipLaunchKernelGGL((k_ir_residual<D, T>), grid, blk, 0, s->stream, P, s->G64, s->cols, s->y, s->bs, s->dsq, \
                     (T*)w->vec[1], (T*)w->vec[0], (T*)rh, w->pa, w->st)
  if (s->d == 2) {
    if (f32)
      CRH_RES(2, float);
    else
      CRH_RES(2, double);
  } else {
    if (f32)
      CRH_RES(3, float);
    else
      CRH_RES(3, double);
  }
#undef CRH_RES
}

void enqueue_update(const Launch& L) {
  const int64_t n = L.s->nf * L.s->d;
  const unsigned g = (unsigned)((n + NT - 1) / NT);
  if (L.prec == CR_FP32_IR)
    hipLaunchKernelGGL(k_ir_update<float>, dim3(g), dim3(NT), 0, L.s->stream, n, L.s->y, (const float*)L.w->vec[0]);
  else
    hipLaunchKernelGGL(k_ir_update<double>, dim3(g), dim3(NT), 0, L.s->stream, n, L.s->y, (const double*)L.w->vec[0]);
}

cr_status get_graph(const Launch& L, int npairs, hipGraphExec_t& out) {
  KWs* w = L.w;
  const int pi = L.prec == CR_FP32_IR ? 1 : 0, mi = L.method == CR_BICGSTAB ? 1 : 0;
  if (w->exec[pi][mi] && w->exec_m[pi][mi] == npairs) {
    out = w->exec[pi][mi];
    return CR_OK;
  }
  if (w->exec[pi][mi]) {
    hipGraphExecDestroy(w->exec[pi][mi]);
    w->exec[pi][mi] = nullptr;
  }
  hipGraph_t g = nullptr;
  cr_status st = check_hip(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st != CR_OK) return st;
  enqueue_iters_any(L, w->cap, npairs);
  hipError_t le = hipGetLastError();
  st = check_hip(hipStreamEndCapture(w->cap, &g), "end capture");
  if (st != CR_OK) return st;
  st = check_hip(le, "captured launch");
  if (st != CR_OK) {
    hipGraphDestroy(g);
    return st;
  }
  st = check_hip(hipGraphInstantiate(&w->exec[pi][mi], g, nullptr, nullptr, 0), "graph instantiate");
  hipGraphDestroy(g);
  if (st != CR_OK) return st;
  w->exec_m[pi][mi] = npairs;
  out = w->exec[pi][mi];
  return CR_OK;
}

// Runs inner iterations until the device flag is set; returns the final state.
cr_status run_inner(const Launch& L, int npairs, bool graph, int maxit, KState& out) {
  KWs* w = L.w;
  cr_system* s = L.s;
  hipGraphExec_t exec = nullptr;
  if (graph) {
    cr_status st = get_graph(L, npairs, exec);
    if (st != CR_OK) return st;
  }
  auto launch = [&]() {
    if (graph)
      hipGraphLaunch(exec, s->stream);
    else
      enqueue_iters_any(L, s->stream, npairs);
  };
  const int per = 2 * npairs;
  const int max_blocks = maxit / per + 3;
  int issued = 0, slot = 0;
  for (int k = 0; k < 2 && issued < max_blocks; ++k) {
    launch();
    hipMemcpyAsync(&w->hst[issued & 1], w->st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
    hipEventRecord(w->ev[issued & 1], s->stream);
    ++issued;
  }
  cr_status st = check_hip(hipGetLastError(), "inner launch");
  if (st != CR_OK) return st;
  for (;;) {
    st = check_hip(hipEventSynchronize(w->ev[slot]), "inner poll");
    if (st != CR_OK) return st;
    const int done = w->hst[slot].done;
    if (done || issued >= max_blocks) break;
    launch();
    hipMemcpyAsync(&w->hst[slot], w->st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
    hipEventRecord(w->ev[slot], s->stream);
    ++issued;
    slot ^= 1;
  }
  hipMemcpyAsync(&w->hst[2], w->st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
  st = check_hip(hipStreamSynchronize(s->stream), "inner sync");
  if (st != CR_OK) return st;
  out = w->hst[2];
  if (!out.done) out.done = 3;
  return CR_OK;
}

cr_status write_params(cr_system* s, KWs* w, double inner_tol, double tol, int maxit) {
  KState* h = &w->hst[2];
  // only the parameter fields are sent; the kernels own the others
  h->inner_tol2 = inner_tol * inner_tol;
  h->outer_tol2 = tol * tol;
  h->maxit = maxit;
  const size_t off = offsetof(KState, inner_tol2);
  cr_status st = check_hip(hipMemcpyAsync((char*)w->st + off, (char*)h + off, sizeof(KState) - off,
                                          hipMemcpyHostToDevice, s->stream),
                           "solver parameters");
  if (st != CR_OK) return st;
  // the staging slot is reused by the next poll: wait for the copy
  return check_hip(hipStreamSynchronize(s->stream), "solver parameters");
}

}  // namespace

cr_status run_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info) {
  auto t_start = std::chrono::steady_clock::now();
  KWs* w = nullptr;
  cr_status st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  Launch L{s, w, o->precision, o->method};
  const int blk = o->check_every > 0 ? o->check_every : 32;
  const int npairs = std::max(1, (blk + 1) / 2);
  const bool graph = o->use_graph != 0;
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  double inner_tol = o->inner_tol;
  if (!(inner_tol > 0)) inner_tol = o->precision == CR_FP32_IR ? 1e-4 : 0.0;
  const int maxit = o->maxit > 0 ? o->maxit : 100000;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 30;
  if (!o->warm_start || !s->has_solution) {
    st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * s->d, s->stream), "zero W");
    if (st != CR_OK) return st;
  }
  int total = 0, outer = 0, reason = 0;
  double rel = -1.0;
  for (;;) {
    const bool last = outer >= max_outer || total >= maxit;
    st = write_params(s, w, inner_tol, tol, last ? 0 : maxit - total);
    if (st != CR_OK) return st;
    enqueue_residual(L);
    ++outer;
    KState ks;
    st = run_inner(L, npairs, graph && !last, last ? 0 : maxit - total, ks);
    if (st != CR_OK) return st;
    total += ks.iters;
    rel = ks.snorm2 > 0 ? std::sqrt(ks.tres2 / ks.snorm2) : std::sqrt(ks.tres2);
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
    enqueue_update(L);
  }
  st = check_hip(hipStreamSynchronize(s->stream), "solve sync");
  if (st != CR_OK) return st;
  s->has_solution = true;
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (info) {
    info->iters = total;
    info->outer_iters = outer;
    info->rel_residual = rel;
    info->t_solve_ms = ms;
    info->reason = reason;
  }
  if (reason == 1) return CR_OK;
  if (reason == 4) {
    set_error("Krylov breakdown after %d iterations", total);
    return CR_E_BREAKDOWN;
  }
  if (reason == 5) {
    set_error("non-finite Krylov scalar after %d iterations", total);
    return CR_E_NONFINITE;
  }
  set_error("no convergence: relative residual %.3e after %d iterations, %d refinement passes", rel, total, outer);
  return CR_E_NOCONV;
}

cr_status run_time_spmv(cr_system* s, int precision, int reps, double* avg_ms, double* bytes) {
  KWs* w = nullptr;
  cr_status st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  const int d = s->d;
  const size_t vb = sizeof(double) * (size_t)s->nf * d;
  if (!w->tvec[0]) {
    for (auto& v : w->tvec) {
      v = dev_alloc(s, vb);
      if (!v) return CR_E_NOMEM;
    }
    for (auto& p : w->tpart) {
      p = (double*)dev_alloc(s, sizeof(double) * (size_t)w->part.nblk * NPART);
      if (!p) return CR_E_NOMEM;
    }
    w->tst = (KState*)dev_alloc(s, sizeof(KState));
    if (!w->tst) return CR_E_NOMEM;
  }
  // scratch state: one record with r.r = 1, iteration 1 in flight, no stopping
  std::vector<double> hp((size_t)w->part.nblk * NPART, 0.0);
  hp[0] = 1.0;
  KState ks{};
  ks.rho[1] = 1.0;
  ks.it[1] = 1;
  ks.thr2 = 0.0;
  ks.inner_tol2 = 0.0;
  ks.outer_tol2 = 0.0;
  ks.maxit = 1 << 30;
  st = check_hip(hipMemcpyAsync(w->tpart[0], hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, s->stream),
                 "timing partials");
  if (st == CR_OK) st = check_hip(hipMemcpyAsync(w->tst, &ks, sizeof ks, hipMemcpyHostToDevice, s->stream), "timing state");
  if (st == CR_OK) st = check_hip(hipMemsetAsync(w->tvec[1], 0, vb, s->stream), "timing p");
  if (st == CR_OK) st = check_hip(hipMemsetAsync(w->tvec[2], 0, vb, s->stream), "timing q");
  if (st != CR_OK) return st;
  const Part P = w->part;
  const bool f32 = precision == CR_FP32_IR;
  // input vector: the scaled right-hand side, rounded to the working type
  std::vector<double> hb((size_t)s->nf * d);
  st = check_hip(hipMemcpyAsync(hb.data(), s->bs, vb, hipMemcpyDeviceToHost, s->stream), "timing input");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "timing input");
  if (st != CR_OK) return st;
  if (f32) {
    std::vector<float> hf(hb.begin(), hb.end());
    st = check_hip(hipMemcpy(w->tvec[0], hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice), "timing input");
  } else {
    st = check_hip(hipMemcpy(w->tvec[0], hb.data(), vb, hipMemcpyHostToDevice), "timing input");
  }
  if (st != CR_OK) return st;
  const dim3 grid(P.nblk), blk(NT);
  auto launch = [&]() {
#define CRH_T(D, T)                                                                                               \
  hipLaunchKernelGGL((k_cg_spmv<D, T>), grid, blk, 0, s->stream, P, (const T*)(f32 ? (const void*)s->G32 : (const void*)s->G64), \
                     s->cols, (const T*)w->tvec[0], (T*)w->tvec[1], (T*)w->tvec[2], w->tpart[0], w->tpart[1], w->tst, 0)
    if (d == 2) {
      if (f32)
        CRH_T(2, float);
      else
        CRH_T(2, double);
    } else {
      if (f32)
        CRH_T(3, float);
      else
        CRH_T(3, double);
    }
#undef CRH_T
  };
  launch();  // warm-up
  hipEventRecord(w->t0, s->stream);
  for (int k = 0; k < reps; ++k) launch();
  hipEventRecord(w->t1, s->stream);
  st = check_hip(hipEventSynchronize(w->t1), "timing");
  if (st != CR_OK) return st;
  float ms = 0.f;
  hipEventElapsedTime(&ms, w->t0, w->t1);
  if (avg_ms) *avg_ms = (double)ms / reps;
  if (bytes) {
    const double vsz = f32 ? 4.0 : 8.0;
    const double nf = (double)s->nf;
    const double mat = nf * (2 * d + 1) * d * d * vsz + nf * 2 * d * 4.0;
    const double vec = nf * d * vsz * (1 /* r gathered once */ + 2 /* p r/w */ + 2 /* q r/w */);
    *bytes = mat + vec;
  }
  return CR_OK;
}

void free_krylov(cr_system* s) {
  KWs* w = (KWs*)s->kws;
  if (!w) return;
  for (auto& row : w->exec)
    for (auto& e : row)
      if (e) hipGraphExecDestroy(e);
  for (auto& e : w->ev)
    if (e) hipEventDestroy(e);
  if (w->t0) hipEventDestroy(w->t0);
  if (w->t1) hipEventDestroy(w->t1);
  if (w->cap) hipStreamDestroy(w->cap);
  if (w->hst) hipHostFree(w->hst);
  delete w;
  s->kws = nullptr;
}

}  // namespace crh
