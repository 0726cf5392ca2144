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
// Precision: the FP64 solution y is resident.  The Krylov recurrences run in
// FP32 (or FP64) on a correction x; whenever the recursive residual has fallen
// by a set factor since the last update, x is added to y and the residual is
// recomputed from y with the FP64 matrix plane ("reliable update" / residual
// replacement).  The search directions are kept across the update, so the
// Krylov space is not lost as it would be by restarting an inner solve.  The
// solve stops on the FP64 residual ||S - G W|| <= tol ||S||.
//
// CG (symmetric positive definite G) runs two kernels per iteration: the
// product w = G r fused with the direction updates p = r + beta p and
// q = w + beta q (q = G p without a second product) and the partial p.q; then
// alpha = rho / p.q, x += alpha p, r -= alpha q and the partial r.r.
// BiCGStab (non-symmetric G) uses three kernels per iteration.  A Krylov
// breakdown caused by rounding (p.q <= 0, rho = 0, ...) triggers a restart
// from the FP64 residual with a fresh direction.
//
// Reductions: every kernel processes a contiguous range of face rows per
// workgroup (remapped so that each XCD gets a contiguous eighth of the rows)
// and writes one partial sum per workgroup and dot product; the consuming
// kernel reduces the partials redundantly in every workgroup in a fixed order,
// so all workgroups see bit-identical scalars, without atomics.  Per-iteration
// scalars alternate between two slots by iteration parity, a kernel argument,
// so an even number of iterations is captured once in a hipGraph and replayed.
// A device flag stops all later kernels once the iteration has converged,
// needs a residual replacement or failed, so replays past it are no-ops.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.h"
#include "rowkern.h"

namespace crh {
namespace {

constexpr int NFIELD = 4;  // fields of a partial record

// done codes
enum : int { RUNNING = 0, REPLACE = 1, CONVERGED = 2, LIMIT = 3, BREAKDOWN = 4, NONFINITE = 5 };

struct KState {
  // per iteration parity
  double gam[2];   // CG: r.r; BiCGStab: rho = rhat.r
  double alp[2];
  double omg[2];   // BiCGStab omega
  int it[2];       // (index + 1) of the iteration run with this parity
  // control: each written by one kernel, read by later kernels
  int done;
  int iters;       // index of the iteration at which the last stop happened
  int it_rep;      // iteration index of the last residual replacement
  int it_first;    // iteration index that starts a new direction (beta = 0)
  int nrun;        // iterations executed since the start of the solve
  int pad0;
  double rr_rep, thr_rep, tgt, tres2, snorm2, last_rr;
  // parameters written by the host
  double rep_tol2, tol2;
  int maxit;
  int pad1;
};

template <typename T, int D>
struct Plain {
  const T* __restrict__ x;
  __device__ Vec<T, D> operator()(int64_t c) const { return ldv<T, D>(x, c); }
};

// ---------------------------------------------------------------------------
// Residual (replacement) kernel: r_s = bs - G64 y in FP64; r = (T) r_s; x = 0.
// Partial fields: 0 = r.r (CG) or rhat.r (BiCGStab), 1 = ||dsq r_s||^2 =
// ||S - G W||^2, 2 = ||S||^2, 3 = r.r.
// mode 0 (start): iteration counters reset, new direction, rhat = r.
// mode 1 (replacement): the iteration continues with its directions.
// mode 2 (restart after a finite-precision breakdown, or any stop at an odd
//   iteration): new direction from the next even iteration index, rhat = r.
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ir_residual(Part P, const double* __restrict__ G64,
                                                    const int32_t* __restrict__ cols, const double* __restrict__ y,
                                                    const double* __restrict__ bs, const double* __restrict__ dsq,
                                                    T* __restrict__ r, T* __restrict__ x, T* __restrict__ rhat,
                                                    double* __restrict__ part, KState* __restrict__ st, int mode,
                                                    int bicg) {
  // a replacement after a stop at an odd iteration (iteration limit) cannot
  // keep its directions at parity 0: it becomes a restart
  if (mode == 1 && (st->iters & 1)) mode = 2;
  const bool init = mode != 1;
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<double, D> w = spmv_row<D, double>(G64, cols, P.nf, f, Plain<double, D>{y});
    Vec<T, D> rt, zero, rh;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double b = bs[f * D + i], sq = dsq[f * D + i];
      const double rs = b - w.v[i];
      rt.v[i] = (T)rs;
      zero.v[i] = T(0);
      acc[1] += (sq * rs) * (sq * rs);
      acc[2] += (sq * b) * (sq * b);
      acc[3] += (double)rt.v[i] * (double)rt.v[i];
    }
    stv<T, D>(r, f, rt);
    stv<T, D>(x, f, zero);
    if (bicg) {
      if (init)
        rh = rt;
      else
        rh = ldv<T, D>(rhat, f);
      if (init) stv<T, D>(rhat, f, rt);
#pragma unroll
      for (int i = 0; i < D; ++i) acc[0] += (double)rh.v[i] * (double)rt.v[i];
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) acc[0] += (double)rt.v[i] * (double)rt.v[i];
    }
  }
  block_sum<4>(acc);
  if (threadIdx.x == 0) {
    part[lb] = acc[0];
    part[(int64_t)1 * P.nblk + lb] = acc[1];
    part[(int64_t)2 * P.nblk + lb] = acc[2];
    part[(int64_t)3 * P.nblk + lb] = acc[3];
  }
  if (lead()) {
    if (mode == 0) {
      st->it[1] = 0;
      st->iters = 0;
      st->it_first = 0;
      st->nrun = 0;
    } else if (mode == 2) {
      const int e = (st->iters + 1) & ~1;
      st->it[1] = e;
      st->iters = e;
      st->it_first = e;
    }
    st->it_rep = st->iters;
    st->done = RUNNING;
  }
}

// Stopping logic shared by the first kernel of each iteration.  rr is the
// squared norm of the recursive residual; at the first iteration after a
// replacement (fresh) the true residual and ||S|| come from partial fields 1, 2.
// Replacements are requested only at even iterations so that the next
// iteration starts a graph replay at parity 0.
struct Decision {
  int done;
  double rr_rep, thr_rep, tgt;
};

__device__ __forceinline__ Decision decide(const KState* st, int it, bool fresh, double rr, double tres2,
                                           double snorm2) {
  Decision d;
  d.done = RUNNING;
  if (fresh) {
    d.rr_rep = rr;
    d.thr_rep = st->rep_tol2 * rr;
    d.tgt = tres2 > 0.0 ? 0.01 * st->tol2 * snorm2 * rr / tres2 : 0.0;
    if (tres2 <= st->tol2 * snorm2) {
      d.done = CONVERGED;
      return d;
    }
  } else {
    d.rr_rep = st->rr_rep;
    d.thr_rep = st->thr_rep;
    d.tgt = st->tgt;
  }
  if (!isfinite(rr))
    d.done = NONFINITE;
  else if (it >= st->maxit)
    d.done = LIMIT;
  else if (!fresh && !(it & 1) && (rr <= d.thr_rep || rr <= d.tgt))
    d.done = REPLACE;
  return d;
}

__device__ __forceinline__ void record_decision(KState* st, const Decision& d, bool fresh, int it, double rr,
                                                double tres2, double snorm2) {
  if (fresh) {
    st->rr_rep = d.rr_rep;
    st->thr_rep = d.thr_rep;
    st->tgt = d.tgt;
    st->tres2 = tres2;
    st->snorm2 = snorm2;
  }
  st->iters = it;
  st->last_rr = rr;
  if (d.done) st->done = d.done;
}

// ---------------------------------------------------------------------------
// CG iteration, kernel 1 (parity par): partial fields of Pa: 0 = r.r (and
// 1, 2 after a replacement); w = G r, p = r + beta p, q = w + beta q; Pb field
// 0 = p.q.
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_spmv(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                                const T* __restrict__ r, T* __restrict__ p, T* __restrict__ q,
                                                const double* __restrict__ Pa, double* __restrict__ Pb,
                                                KState* __restrict__ st, int par) {
  if (st->done) return;
  const int it = st->it[par ^ 1];
  const bool first = it == st->it_first;
  const bool fresh = it == st->it_rep;
  double rr, tres2 = 0.0, snorm2 = 0.0;
  if (fresh) {
    const int fl[3] = {0, 1, 2};
    double v[3];
    reduce_fields<3>(Pa, P.nblk, fl, v);
    rr = v[0];
    tres2 = v[1];
    snorm2 = v[2];
  } else {
    const int fl[1] = {0};
    double v[1];
    reduce_fields<1>(Pa, P.nblk, fl, v);
    rr = v[0];
  }
  const Decision dec = decide(st, it, fresh, rr, tres2, snorm2);
  if (lead()) {
    record_decision(st, dec, fresh, it, rr, tres2, snorm2);
    if (!dec.done) {
      st->gam[par] = rr;
      st->it[par] = it + 1;
      st->nrun += 1;
    }
  }
  if (dec.done) return;
  const T beta = first ? T(0) : (T)(rr / st->gam[par ^ 1]);
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
  if (threadIdx.x == 0) Pb[lb] = acc[0];
}

// CG iteration, kernel 2: alpha = rho / p.q, x += alpha p, r -= alpha q; Pa field 0 = r.r
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_update(Part P, T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ p, const T* __restrict__ q,
                                                  const double* __restrict__ Pb, double* __restrict__ Pa,
                                                  KState* __restrict__ st, int par) {
  if (st->done) return;
  const int fl[1] = {0};
  double v[1];
  reduce_fields<1>(Pb, P.nblk, fl, v);
  const double pq = v[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (lead()) st->done = isfinite(pq) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double alpha = st->gam[par] / pq;
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
  if (threadIdx.x == 0) Pa[lb] = acc[0];
  if (lead()) st->alp[par] = alpha;
}

// ---------------------------------------------------------------------------
// BiCGStab on the scaled system (non-symmetric G), three kernels per
// iteration; the direction p and the intermediate s are formed on the fly from
// double-buffered vectors inside the products that consume them:
//   B1: p_new = r + beta (p_old - omega v_old), v = G p_new, partial rhat.v
//   B2: alpha = rho / rhat.v, s = r - alpha v, t = G s, partials t.s, t.t
//   B3: omega = t.s / t.t, x += alpha p + omega s, r = s - omega t,
//       partials rhat.r, r.r
// Partial arrays: B1 reads Pa (fields 0 rhat.r, 3 r.r, 1/2 after a
// replacement) and writes Pb; B2 reads Pb, writes Pc; B3 reads Pc, writes Pa.
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
                                               const double* __restrict__ Pa, double* __restrict__ Pb,
                                               KState* __restrict__ st, int par) {
  if (st->done) return;
  const int it = st->it[par ^ 1];
  const bool first = it == st->it_first;
  const bool fresh = it == st->it_rep;
  double rho, rr, tres2 = 0.0, snorm2 = 0.0;
  if (fresh) {
    const int fl[4] = {0, 3, 1, 2};
    double v[4];
    reduce_fields<4>(Pa, P.nblk, fl, v);
    rho = v[0];
    rr = v[1];
    tres2 = v[2];
    snorm2 = v[3];
  } else {
    const int fl[2] = {0, 3};
    double v[2];
    reduce_fields<2>(Pa, P.nblk, fl, v);
    rho = v[0];
    rr = v[1];
  }
  const Decision dec = decide(st, it, fresh, rr, tres2, snorm2);
  int done = dec.done;
  if (!done && (!(rho != 0.0) || !isfinite(rho))) done = isfinite(rho) ? BREAKDOWN : NONFINITE;
  const double beta = first ? 0.0 : (rho / st->gam[par ^ 1]) * (st->alp[par ^ 1] / st->omg[par ^ 1]);
  if (lead()) {
    record_decision(st, dec, fresh, it, rr, tres2, snorm2);
    if (done) {
      st->done = done;
    } else {
      st->gam[par] = rho;
      st->it[par] = it + 1;
      st->nrun += 1;
    }
  }
  if (done) return;
  const PNew<T, D> in{r, p_old, v_old, (T)beta, (T)st->omg[par ^ 1], first};
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
  if (threadIdx.x == 0) Pb[lb] = acc[0];
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_bicg_2(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                               const T* __restrict__ r, const T* __restrict__ v_new,
                                               T* __restrict__ s, T* __restrict__ t, const double* __restrict__ Pb,
                                               double* __restrict__ Pc, KState* __restrict__ st, int par) {
  if (st->done) return;
  const int fl[1] = {0};
  double v[1];
  reduce_fields<1>(Pb, P.nblk, fl, v);
  const double rv = v[0];
  if (!(rv != 0.0) || !isfinite(rv)) {
    if (lead()) st->done = isfinite(rv) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double alpha = st->gam[par] / rv;
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
    Pc[lb] = acc[0];
    Pc[(int64_t)P.nblk + lb] = acc[1];
  }
  if (lead()) st->alp[par] = alpha;
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_bicg_3(Part P, T* __restrict__ x, T* __restrict__ r,
                                               const T* __restrict__ rhat, const T* __restrict__ p_new,
                                               const T* __restrict__ s, const T* __restrict__ t,
                                               const double* __restrict__ Pc, double* __restrict__ Pa,
                                               KState* __restrict__ st, int par) {
  if (st->done) return;
  const int fl[2] = {0, 1};
  double v[2];
  reduce_fields<2>(Pc, P.nblk, fl, v);
  const double ts = v[0], tt = v[1];
  if (!(tt > 0.0) || !isfinite(tt) || !isfinite(ts)) {
    if (lead()) st->done = (isfinite(tt) && isfinite(ts)) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double omega = ts / tt;
  const T ta = (T)st->alp[par], to = (T)omega;
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
    Pa[lb] = acc[0];
    Pa[(int64_t)3 * P.nblk + lb] = acc[1];
  }
  if (lead()) st->omg[par] = omega;
}

// y += x (FP64 accumulation of the correction)
template <typename T>
__global__ void __launch_bounds__(NT) k_ir_update(int64_t n, double* __restrict__ y, const T* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) y[i] += (double)x[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// vector slots of the workspace
enum { V_X, V_P, V_R0, V_R1, V_W0, V_W1, V_S0, V_S1, V_RHAT, V_T, NVEC };

struct KWs {
  Part part{};
  void* vec[NVEC] = {};  // each nf*d doubles
  double* part3[3] = {};   // partial arrays, NFIELD x nblk each
  KState* st = nullptr;
  KState* hst = nullptr;   // pinned [3]
  hipEvent_t ev[2] = {};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[2][2] = {};  // [precision][method]
  int exec_m[2][2] = {};
  // scratch for kernel timing
  void* tvec[NVEC] = {};
  double* tpart[2] = {};
  KState* tst = nullptr;
};

int max_blocks_cfg() {
  static int v = [] {
    const char* e = std::getenv("CRH_MAXBLK");
    int m = e ? std::atoi(e) : MAXBLK / 2;
    m = std::max(8, std::min(4096, m));
    return m / 8 * 8;
  }();
  return v;
}

Part make_part(int64_t nf) {
  Part P;
  P.nf = nf;
  const int64_t mb = max_blocks_cfg();
  const int64_t tiles = (nf + (int64_t)NT * mb - 1) / ((int64_t)NT * mb);
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
  s->kws = w;
  w->part = make_part(s->nf);
  const size_t vb = sizeof(double) * (size_t)s->nf * s->d;
  for (auto& v : w->vec) {
    v = dev_alloc(s, vb);
    if (!v) return CR_E_NOMEM;
  }
  const size_t pbytes = sizeof(double) * (size_t)w->part.nblk * NFIELD;
  for (auto& p : w->part3) {
    p = (double*)dev_alloc(s, pbytes);
    if (!p) return CR_E_NOMEM;
  }
  w->st = (KState*)dev_alloc(s, sizeof(KState));
  if (!w->st) return CR_E_NOMEM;
  cr_status st = check_hip(hipHostMalloc((void**)&w->hst, 3 * sizeof(KState), hipHostMallocDefault), "pinned state");
  for (auto& e : w->ev)
    if (st == CR_OK) st = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  if (st == CR_OK) st = check_hip(hipEventCreate(&w->t0), "event");
  if (st == CR_OK) st = check_hip(hipEventCreate(&w->t1), "event");
  if (st == CR_OK) st = check_hip(hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking), "capture stream");
  return st;
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
  auto V = [&](int i) { return (T*)w->vec[i]; };
  const dim3 grid(P.nblk), blk(NT);
  for (int k = 0; k < npairs; ++k)
    for (int par = 0; par < 2; ++par) {
      if (L.method == CR_PCG) {
        hipLaunchKernelGGL((k_cg_spmv<D, T>), grid, blk, 0, stream, P, G, L.s->cols, V(V_R0), V(V_P), V(V_W0),
                           w->part3[0], w->part3[1], w->st, par);
        hipLaunchKernelGGL((k_cg_update<D, T>), grid, blk, 0, stream, P, V(V_X), V(V_R0), V(V_P), V(V_W0),
                           w->part3[1], w->part3[0], w->st, par);
      } else {
        T* pv[2] = {V(V_R1), V(V_W1)};  // p buffers
        T* vv[2] = {V(V_S0), V(V_S1)};  // v buffers
        hipLaunchKernelGGL((k_bicg_1<D, T>), grid, blk, 0, stream, P, G, L.s->cols, V(V_R0), V(V_RHAT), pv[par ^ 1],
                           vv[par ^ 1], pv[par], vv[par], w->part3[0], w->part3[1], w->st, par);
        hipLaunchKernelGGL((k_bicg_2<D, T>), grid, blk, 0, stream, P, G, L.s->cols, V(V_R0), vv[par], V(V_W0),
                           V(V_T), w->part3[1], w->part3[2], w->st, par);
        hipLaunchKernelGGL((k_bicg_3<D, T>), grid, blk, 0, stream, P, V(V_X), V(V_R0), V(V_RHAT), pv[par], V(V_W0),
                           V(V_T), w->part3[2], w->part3[0], w->st, par);
      }
    }
}

template <class F>
void dispatch(const cr_system* s, int prec, F&& f) {
  const bool f32 = prec == CR_FP32_IR;
  if (s->d == 2) {
    if (f32)
      f(std::integral_constant<int, 2>(), float());
    else
      f(std::integral_constant<int, 2>(), double());
  } else {
    if (f32)
      f(std::integral_constant<int, 3>(), float());
    else
      f(std::integral_constant<int, 3>(), double());
  }
}

void enqueue_iters_any(const Launch& L, hipStream_t stream, int npairs) {
  dispatch(L.s, L.prec, [&](auto dc, auto tc) {
    constexpr int D = decltype(dc)::value;
    using T = decltype(tc);
    enqueue_iters<D, T>(L, stream, npairs);
  });
}

// residual (replacement) kernel
void enqueue_residual(const Launch& L, int mode) {
  KWs* w = L.w;
  cr_system* s = L.s;
  const Part P = w->part;
  const dim3 grid(P.nblk), blk(NT);
  const bool bicg = L.method == CR_BICGSTAB;
  dispatch(s, L.prec, [&](auto dc, auto tc) {
    constexpr int D = decltype(dc)::value;
    using T = decltype(tc);
    hipLaunchKernelGGL((k_ir_residual<D, T>), grid, blk, 0, s->stream, P, s->G64, s->cols, s->y, s->bs, s->dsq,
                       (T*)w->vec[V_R0], (T*)w->vec[V_X], (T*)w->vec[V_RHAT], w->part3[0], w->st, mode,
                       bicg ? 1 : 0);
  });
}

void enqueue_update(const Launch& L) {
  const int64_t n = L.s->nf * L.s->d;
  const unsigned g = (unsigned)((n + NT - 1) / NT);
  if (L.prec == CR_FP32_IR)
    hipLaunchKernelGGL(k_ir_update<float>, dim3(g), dim3(NT), 0, L.s->stream, n, L.s->y, (const float*)L.w->vec[V_X]);
  else
    hipLaunchKernelGGL(k_ir_update<double>, dim3(g), dim3(NT), 0, L.s->stream, n, L.s->y,
                       (const double*)L.w->vec[V_X]);
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

// Replays iteration blocks until the device flag is set (at most max_blocks
// blocks, two in flight); returns the final state.
cr_status run_inner(const Launch& L, int npairs, bool graph, int max_blocks, KState& out) {
  KWs* w = L.w;
  cr_system* s = L.s;
  hipGraphExec_t exec = nullptr;
  if (graph) {
    cr_status st = get_graph(L, npairs, exec);
    if (st != CR_OK) return st;
  }
  auto launch = [&](int slot) {
    if (graph)
      hipGraphLaunch(exec, s->stream);
    else
      enqueue_iters_any(L, s->stream, npairs);
    hipMemcpyAsync(&w->hst[slot], w->st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
    hipEventRecord(w->ev[slot], s->stream);
  };
  int issued = 0, slot = 0;
  for (int k = 0; k < 2 && issued < max_blocks; ++k) launch(issued++ & 1);
  cr_status st = check_hip(hipGetLastError(), "inner launch");
  if (st != CR_OK) return st;
  for (;;) {
    st = check_hip(hipEventSynchronize(w->ev[slot]), "inner poll");
    if (st != CR_OK) return st;
    if (w->hst[slot].done || issued >= max_blocks) break;
    launch(slot);
    ++issued;
    slot ^= 1;
  }
  hipMemcpyAsync(&w->hst[2], w->st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
  st = check_hip(hipStreamSynchronize(s->stream), "inner sync");
  if (st != CR_OK) return st;
  out = w->hst[2];
  return CR_OK;
}

cr_status write_params(cr_system* s, KWs* w, double rep_tol, double tol, int maxit) {
  KState* h = &w->hst[2];
  h->rep_tol2 = rep_tol * rep_tol;
  h->tol2 = tol * tol;
  h->maxit = maxit;
  const size_t off = offsetof(KState, rep_tol2);
  cr_status st = check_hip(hipMemcpyAsync((char*)w->st + off, (char*)h + off, sizeof(KState) - off,
                                          hipMemcpyHostToDevice, s->stream),
                           "solver parameters");
  if (st != CR_OK) return st;
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
  const int per = 2 * npairs;
  const bool graph = o->use_graph != 0;
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  // reduction of the recursive residual between residual replacements
  double rep = o->inner_tol;
  if (!(rep > 0)) rep = o->precision == CR_FP32_IR ? 0.1 : 0.0;
  const int maxit = o->maxit > 0 ? o->maxit : 1000000;
  const int max_rep = o->max_outer > 0 ? o->max_outer : 400;
  if (!o->warm_start || !s->has_solution) {
    st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * s->d, s->stream), "zero W");
    if (st != CR_OK) return st;
  }
  st = write_params(s, w, rep, tol, maxit);
  if (st != CR_OK) return st;
  enqueue_residual(L, 0);
  int reps = 1, restarts = 0, reason = 0, iters = 0, fp32_iters = 0;
  double rel = -1.0, prev_true = -1.0;
  bool final_eval = false, fell_back = false;
  // FP32 intervals between replacements are capped; a stalled FP32 interval
  // or a replacement that does not halve the true residual switches the
  // remaining iterations to FP64 (FP32 Krylov cannot make progress once the
  // condition number times the FP32 unit roundoff approaches one).
  const int fp32_cap_blocks = std::max(8, 6000 / per);
  for (;;) {
    KState ks;
    const bool f32 = L.prec == CR_FP32_IR;
    const int cap = final_eval ? 1 : (f32 ? fp32_cap_blocks : maxit / per + 3);
    st = run_inner(L, npairs, graph && !final_eval, cap, ks);
    if (st != CR_OK) return st;
    if (f32) fp32_iters = ks.nrun;
    iters = ks.nrun;
    rel = ks.snorm2 > 0 ? std::sqrt(ks.tres2 / ks.snorm2) : std::sqrt(ks.tres2);
    if (ks.done == CONVERGED) {
      reason = 1;
      break;
    }
    if (ks.done == NONFINITE && !f32) {
      reason = ks.done;
      break;
    }
    if (ks.done == BREAKDOWN && !f32 && (final_eval || restarts >= 8)) {
      reason = ks.done;
      break;
    }
    if (final_eval) {
      reason = 3;
      break;
    }
    bool stall = false;
    if (f32) {
      stall = ks.done == RUNNING || ks.done == NONFINITE || (ks.done == BREAKDOWN && restarts >= 2) ||
              (prev_true > 0.0 && ks.tres2 > 0.25 * prev_true);
      prev_true = ks.tres2;
    }
    // fold the correction into y (unless it holds non-finite values) and
    // recompute the residual in FP64
    if (ks.done != NONFINITE) enqueue_update(L);
    if (stall) {
      L.prec = CR_FP64;
      fell_back = true;
      enqueue_residual(L, 2);
    } else if (ks.done == BREAKDOWN) {
      enqueue_residual(L, 2);
      ++restarts;
    } else {
      enqueue_residual(L, 1);
    }
    ++reps;
    if ((!stall && ks.done != REPLACE && ks.done != BREAKDOWN) || reps > max_rep || iters >= maxit) final_eval = true;
  }
  st = check_hip(hipStreamSynchronize(s->stream), "solve sync");
  if (st != CR_OK) return st;
  s->has_solution = true;
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (info) {
    info->iters = iters;
    info->outer_iters = reps;
    info->rel_residual = rel;
    info->t_solve_ms = ms;
    info->reason = reason;
    info->fp32_iters = o->precision == CR_FP32_IR ? fp32_iters : 0;
    info->fp64_fallback = fell_back ? 1 : 0;
  }
  if (reason == 1) return CR_OK;
  if (reason == BREAKDOWN) {
    set_error("Krylov breakdown after %d iterations", iters);
    return CR_E_BREAKDOWN;
  }
  if (reason == NONFINITE) {
    set_error("non-finite Krylov scalar after %d iterations", iters);
    return CR_E_NONFINITE;
  }
  set_error("no convergence: relative residual %.3e after %d iterations, %d residual evaluations", rel, iters, reps);
  return CR_E_NOCONV;
}

// Times the dominant kernel (SpMV fused with the CG direction updates) on
// scratch vectors; its input r is never written, so every launch does
// identical work.
cr_status run_time_spmv(cr_system* s, int precision, int reps, double* avg_ms, double* bytes) {
  KWs* w = nullptr;
  cr_status st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  const int d = s->d;
  const size_t vb = sizeof(double) * (size_t)s->nf * d;
  const Part P = w->part;
  if (!w->tvec[0]) {
    for (auto& v : w->tvec) {
      v = dev_alloc(s, vb);
      if (!v) return CR_E_NOMEM;
    }
    for (auto& p : w->tpart) {
      p = (double*)dev_alloc(s, sizeof(double) * (size_t)P.nblk * NFIELD);
      if (!p) return CR_E_NOMEM;
    }
    w->tst = (KState*)dev_alloc(s, sizeof(KState));
    if (!w->tst) return CR_E_NOMEM;
  }
  // scratch state: iteration 1 in flight (not first, not fresh), r.r = 1,
  // previous r.r = 1 (beta = 1), no stopping
  std::vector<double> hp((size_t)P.nblk * NFIELD, 0.0);
  hp[0] = 1.0;
  KState ks{};
  ks.gam[1] = 1.0;
  ks.it[1] = 1;
  ks.it_rep = -1;
  ks.it_first = -1;
  ks.maxit = 1 << 30;
  st = check_hip(hipMemcpyAsync(w->tpart[0], hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, s->stream),
                 "timing partials");
  if (st == CR_OK) st = check_hip(hipMemcpyAsync(w->tst, &ks, sizeof ks, hipMemcpyHostToDevice, s->stream), "timing state");
  for (int i = 0; i < NVEC && st == CR_OK; ++i)
    st = check_hip(hipMemsetAsync(w->tvec[i], 0, vb, s->stream), "timing vectors");
  if (st != CR_OK) return st;
  // input r: the scaled right-hand side rounded to the working type
  std::vector<double> hb((size_t)s->nf * d);
  st = check_hip(hipMemcpyAsync(hb.data(), s->bs, vb, hipMemcpyDeviceToHost, s->stream), "timing input");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "timing input");
  if (st != CR_OK) return st;
  const bool f32 = precision == CR_FP32_IR;
  std::vector<float> hf(hb.begin(), hb.end());
  st = check_hip(hipMemcpy(w->tvec[V_R0], f32 ? (const void*)hf.data() : (const void*)hb.data(),
                           f32 ? hf.size() * sizeof(float) : vb, hipMemcpyHostToDevice),
                 "timing input");
  if (st != CR_OK) return st;
  const dim3 grid(P.nblk), blk(NT);
  auto launch = [&]() {
    dispatch(s, precision, [&](auto dc, auto tc) {
      constexpr int D = decltype(dc)::value;
      using T = decltype(tc);
      const T* G = std::is_same<T, float>::value ? (const T*)s->G32 : (const T*)s->G64;
      auto V = [&](int i) { return (T*)w->tvec[i]; };
      hipLaunchKernelGGL((k_cg_spmv<D, T>), grid, blk, 0, s->stream, P, G, s->cols, V(V_R0), V(V_P), V(V_W0),
                         w->tpart[0], w->tpart[1], w->tst, 0);
    });
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
    // values and column indices of G, the gathered input r read once, p and q
    // read and written
    const double vsz = f32 ? 4.0 : 8.0;
    const double nf = (double)s->nf;
    const double mat = nf * (2 * d + 1) * d * d * vsz + nf * 2 * d * 4.0;
    const double vec = nf * d * vsz * (1 + 2 + 2);
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
