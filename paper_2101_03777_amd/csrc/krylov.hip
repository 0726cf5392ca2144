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
// Operator forms.  The assembled form reads the block-ELL rows of the scaled
// G.  The element form (transient Stokes) applies G = sum_K H_K G_K H_K^t
// from per-element factors of G_K (a symmetric (d+1)x(d+1) matrix and a
// (d+1) x d rank-one factor), about a fifth of the bytes of the assembled rows
// in 3D and two fifths in 2D.
//
// Pressure gauge in the element form.  G pins the pressure of one element K0
// by leaving out its Schur term; that leaves one eigenvalue of the scaled G
// about two orders of magnitude below the rest (the constant-pressure mode,
// eigenvector z with z_f = a_{K,f} for the owner K of f).  The element form
// keeps the Schur term of K0 too: G' = G - u u^t / B_K0 (u = C_K0 l_K0) is
// positive semi-definite with null vector z, and G' W' = S' with
// S' = S - u (l_K0^t R_K0) / B_K0 is consistent.  CG on it converges as if that
// eigenvalue were removed (about 20% fewer iterations at 512 x 512 x 2).  Its
// residual equals S - G W for W = W' + t z with t = -P_K0(W'), the shift applied
// after the solve, so the stopping test and the reported residual are those of
// G W = S, and W is the solution of G W = S.
//
// CG (symmetric positive definite G) runs two kernels per iteration.
// Assembled form: the product w = G r fused with the direction updates
// p = r + beta p and q = w + beta q (q = G p without a second product) and
// the partial p.q; then alpha = rho / p.q, x += alpha p, r -= alpha q and the
// partial r.r.  Element form: an element kernel forms p on the element's faces
// and its contribution G_K p_K (and p.Gp as a sum of element terms), a face
// kernel sums the two contributions of each face into q and updates x and r;
// q is never stored.
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
//
// The same CG kernel bodies run in batched form (one grid over the row ranges
// of many systems, per-system partials, scalars and flags) for serving.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <type_traits>
#include <vector>

#include <hip/hip_ext.h>

#include "internal.h"
#include "rowkern.h"

namespace crh {
namespace {

constexpr int NFIELD = 6;  // fields of a partial record
constexpr int KMAX = 4;    // aggregates a face block may touch (coarse restriction)

// done codes
enum : int { RUNNING = 0, REPLACE = 1, CONVERGED = 2, LIMIT = 3, BREAKDOWN = 4, NONFINITE = 5, STALL = 6, DIVERGED = 7 };

// growth of the recursive |r|^2 since the last residual evaluation that is
// treated as divergence (a factor 1e6 in norm)
constexpr double DIVERGE2 = 1e12;

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
  // BiCGStab(2) scalars of the iteration with each parity, each written by one
  // kernel and read by later ones: rho after the even and the odd BiCG step,
  // beta and alpha of both steps, omega_2 of the minimal-residual step
  double rho_a[2], beta1[2], alpha1[2], rho_b[2], beta2[2], alpha2[2], omega2[2];
  double bet[2];  // CG beta of the iteration with each parity
  // parameters written by the host
  double rep_tol2, tol2;
  int maxit;
  int interval_cap;  // > 0: at most this many iterations between replacements (FP32, and CG)
};

template <typename T, int D>
struct Plain {
  const T* __restrict__ x;
  __device__ Vec<T, D> operator()(int64_t c) const { return ldv<T, D>(x, c); }
};

// Everything one CG solve of one system touches; passed by value to the
// single-system kernels and read from a device table by the batched ones.
struct CgSys {
  Part P;                    // face rows
  Part PE;                   // elements (element-centric kernels)
  int boff;                  // first face block of this system in a batched grid
  int boffE;                 // first element block of this system in a batched grid
  const void* G;             // matrix plane of the iteration precision
  const int32_t* cols;
  const double* G64;         // FP64 plane (residual)
  double* y;                 // resident FP64 solution (scaled)
  const double* bs;
  const double* dsq;
  void* x;
  void* r;
  void* p;
  void* q;
  double* Pa;                // partials: fields 0 r.r, 1 true residual^2, 2 ||S||^2
  double* Pb;                // partials: field 0 p.q
  double* Pc;                // third partial array (MINRES)
  KState* st;
  // element-factor form (transient Stokes)
  void* p1;                  // second direction buffer (element-centric CG)
  void* tq;                  // [ne][d+1][d] element contributions w_K
  const uint32_t* eflags;
  const double* bs1;         // scaled right-hand side of the element form
  // coarse correction (nagg > 0): M^-1 = I + Z E^-1 Z^t
  int nagg;
  int boffC;                 // first coarse block of this system in a batched grid
  const int32_t* fagg;       // [nf] aggregate of each face
  const void* zT;            // [nf*d] columns of Z in the iteration precision
  double* Pr;                // [nblk][KMAX] restriction partials of face blocks
  const int32_t* ablk;       // [nblk] first aggregate of each face block
  const int32_t* bfa;        // [nagg] first face block of each aggregate
  const int32_t* bla;        // [nagg] last face block of each aggregate
  const double* Einv;        // [nagg*nagg]
  double* cvec;              // [nagg] c = Z^t r
  double* mu;                // [nagg] E^-1 c
  double* M2;                // [2][nagg] coarse part m of the direction, by parity
  const void* F;             // factors of the iteration precision
  const double* F64;         // FP64 factors (residual)
  const int32_t* egat;
  const int32_t* fel;
  const int32_t* floc;
  int64_t ne;
};

// One row of the scaled operator: OP 1 = element factors, OP 0 = assembled block-ELL rows.
template <int D, typename T, int OP, class In>
__device__ __forceinline__ Vec<T, D> op_row(const CgSys& S, const void* G, const void* F, int64_t f, const In& in) {
  if constexpr (OP == 1)
    return efo_row<D, T>(Efo<T>{(const T*)F, S.egat, S.fel, S.floc, S.ne}, S.P.nf, f, in);
  else
    return spmv_row<D, T>((const T*)G, S.cols, S.P.nf, f, in);
}

__device__ __forceinline__ int logical_of(int b, int nblk) { return (b & 7) * (nblk >> 3) + (b >> 3); }

// restriction partials of one face row: z_f . r_f into the slot of its aggregate
template <int D, typename T>
__device__ __forceinline__ void restrict_row(const CgSys& S, int64_t f, int a0, const Vec<T, D>& r,
                                             double (&acc)[KMAX]) {
  const Vec<T, D> z = ldv<T, D>((const T*)S.zT, f);
  double zr = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) zr += (double)z.v[i] * (double)r.v[i];
  const int a = S.fagg[f] - a0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k] += a == k ? zr : 0.0;
}

// ---------------------------------------------------------------------------
// Residual (replacement) kernel: r_s = bs - G64 y in FP64; r = (T) r_s; x = 0.
// Partial fields: 0 = r.r (CG) or rhat.r (BiCGStab), 1 = ||dsq r_s||^2 =
// ||S - G W||^2, 2 = ||S||^2, 3 = r.r.
// mode 0 (start): iteration counters reset, new direction, rhat = r.
// mode 1 (replacement): the iteration continues with its directions.
// mode 2 (restart after a finite-precision breakdown, or any stop at an odd
//   iteration): new direction from the next even iteration index, rhat = r.
// ---------------------------------------------------------------------------
template <int D, typename T, int OP>
__device__ __forceinline__ void ir_residual_body(const CgSys& S, int lb, T* __restrict__ rhat, int mode, int bicg) {
  const Part P = S.P;
  KState* st = S.st;
  // a replacement after a stop at an odd iteration (iteration limit) cannot
  // keep its directions at parity 0: it becomes a restart
  if (mode == 1 && (st->iters & 1)) mode = 2;
  const bool init = mode != 1;
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  T* __restrict__ r = (T*)S.r;
  T* __restrict__ x = (T*)S.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool crs = OP == 1 && S.nagg > 0;
  const int a0 = crs ? S.ablk[lb] : 0;
  double racc[KMAX] = {};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<double, D> w = op_row<D, double, OP>(S, S.G64, S.F64, f, Plain<double, D>{S.y});
    Vec<T, D> rt, zero, rh;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      // ||S|| always from the right-hand side of G W = S
      const double b = S.bs[f * D + i], sq = S.dsq[f * D + i];
      const double rs = (OP == 1 ? S.bs1[f * D + i] : b) - w.v[i];
      rt.v[i] = (T)rs;
      zero.v[i] = T(0);
      acc[1] += (sq * rs) * (sq * rs);
      acc[2] += (sq * b) * (sq * b);
      acc[3] += (double)rt.v[i] * (double)rt.v[i];
    }
    stv<T, D>(r, f, rt);
    stv<T, D>(x, f, zero);
    if (crs) restrict_row<D, T>(S, f, a0, rt, racc);
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
    S.Pa[lb] = acc[0];
    S.Pa[(int64_t)1 * P.nblk + lb] = acc[1];
    S.Pa[(int64_t)2 * P.nblk + lb] = acc[2];
    S.Pa[(int64_t)3 * P.nblk + lb] = acc[3];
  }
  if (crs) {
    block_sum<KMAX>(racc);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < KMAX; ++k) S.Pr[(int64_t)lb * KMAX + k] = racc[k];
  }
  if (threadIdx.x == 0 && lb == 0) {
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

template <int D, typename T, int OP>
__global__ void __launch_bounds__(NT) k_ir_residual(CgSys S, T* __restrict__ rhat, int mode, int bicg) {
  ir_residual_body<D, T, OP>(S, logical_block(S.P.nblk), rhat, mode, bicg);
}

// Stopping logic shared by the first kernel of each iteration.  rr is the
// squared norm of the recursive residual; at the first iteration after a
// replacement (fresh) the true residual and ||S|| come from partial fields 1, 2.
// Replacements are requested only at even iterations so that the next
// iteration starts at parity 0.
struct Decision {
  int done;
  double rr_rep, thr_rep, tgt;
};

// capped: the interval cap applies (FP32 iterations, and CG in either
// precision: a restart every interval_cap iterations bounds how long a run
// that no longer reaches a replacement can drift)
__device__ __forceinline__ Decision decide(const KState* st, int it, bool fresh, double rr, double tres2,
                                           double snorm2, bool capped) {
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
  else if (rr > DIVERGE2 * d.rr_rep)
    d.done = DIVERGED;
  else if (it >= st->maxit)
    d.done = LIMIT;
  else if (!fresh && !(it & 1) && (rr <= d.thr_rep || rr <= d.tgt))
    d.done = REPLACE;
  else if (capped && !fresh && !(it & 1) && st->interval_cap > 0 && it - st->it_rep >= st->interval_cap)
    d.done = STALL;
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
// CG iteration, kernel 1 (parity par): Pa fields 0 = r.r (and 1, 2 after a
// replacement); w = G r, p = r + beta p, q = w + beta q (q = G p without a
// second product); Pb field 0 = p.q.
// ---------------------------------------------------------------------------
// Start of a CG iteration (parity par), shared by both operator forms: reduces
// r.r (and after a replacement the true residual and ||S||) from the face
// partials Pa, with the coarse correction also c . mu over the aggregates
// (rho = r.M^-1 r = r.r + c.E^-1 c), applies the stopping logic (the
// workgroup with logical index 0 records it) and returns false if the
// iteration does not run; else sets beta and whether this iteration starts a
// new direction.  The state words and all the sums' inputs are requested
// before any is used, and one workgroup reduction forms every sum (each in the
// same order as its own reduction would).
__device__ __forceinline__ bool cg_head(const CgSys& S, int lb, int par, double& beta, bool& first,
                                        bool with_coarse = false) {
  KState* st = S.st;
  const int done = st->done;
  const int it = st->it[par ^ 1];
  const int it_first = st->it_first, it_rep = st->it_rep;
  const double gam_old = st->gam[par ^ 1];
  const int nblk = S.P.nblk;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += NT) {
    v[0] += S.Pa[i];
    v[1] += S.Pa[(int64_t)nblk + i];
    v[2] += S.Pa[(int64_t)2 * nblk + i];
  }
  if (with_coarse)
    for (int a = threadIdx.x; a < S.nagg; a += NT) v[3] += S.cvec[a] * S.mu[a];
  if (block_sum_stop<4>(v, done)) return false;
  first = it == it_first;
  const bool fresh = it == it_rep;
  const double rr = v[0], tres2 = fresh ? v[1] : 0.0, snorm2 = fresh ? v[2] : 0.0, coarse = v[3];
  const Decision dec = decide(st, it, fresh, rr, tres2, snorm2, true);
  if (threadIdx.x == 0 && lb == 0) record_decision(st, dec, fresh, it, rr, tres2, snorm2);
  beta = first ? 0.0 : (rr + coarse) / gam_old;
  if (threadIdx.x == 0 && lb == 0 && !dec.done) {
    st->gam[par] = rr + coarse;
    st->bet[par] = beta;
    st->it[par] = it + 1;
    st->nrun += 1;
  }
  if (dec.done) return false;
  return true;
}

template <int D, typename T, int OP>
__device__ __forceinline__ void cg_spmv_body(const CgSys& S, int lb, int par) {
  double beta_d;
  bool first;
  if (!cg_head(S, lb, par, beta_d, first)) return;
  const Part P = S.P;
  const T beta = (T)beta_d;
  const T* __restrict__ r = (const T*)S.r;
  T* __restrict__ p = (T*)S.p;
  T* __restrict__ q = (T*)S.q;
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> w = op_row<D, T, OP>(S, S.G, S.F, f, Plain<T, D>{r});
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
  if (threadIdx.x == 0) S.Pb[lb] = acc[0];
}

// CG iteration, kernel 2: alpha = rho / p.q, x += alpha p, r -= alpha q; Pa field 0 = r.r
template <int D, typename T>
__device__ __forceinline__ void cg_update_body(const CgSys& S, int lb, int par) {
  KState* st = S.st;
  const int seen = st->done;
  const Part P = S.P;
  const int fl[1] = {0};
  double v[1];
  if (reduce_fields_stop<1>(S.Pb, P.nblk, fl, v, seen)) return;
  const double pq = v[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (threadIdx.x == 0 && lb == 0) st->done = isfinite(pq) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double alpha = st->gam[par] / pq;
  const T ta = (T)alpha;
  T* __restrict__ x = (T*)S.x;
  T* __restrict__ r = (T*)S.r;
  const T* __restrict__ p = (const T*)S.p;
  const T* __restrict__ q = (const T*)S.q;
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
  if (threadIdx.x == 0) S.Pa[lb] = acc[0];
  if (threadIdx.x == 0 && lb == 0) st->alp[par] = alpha;
}

// y += x over the system's rows (FP64 accumulation of the correction)
template <int D, typename T>
__device__ __forceinline__ void ir_update_body(const CgSys& S, int lb) {
  const Part P = S.P;
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  const T* __restrict__ x = (const T*)S.x;
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT)
#pragma unroll
    for (int i = 0; i < D; ++i) S.y[f * D + i] += (double)x[f * D + i];
}

template <int D, typename T, int OP>
__global__ void __launch_bounds__(NT) k_cg_spmv(CgSys S, int par) {
  cg_spmv_body<D, T, OP>(S, logical_block(S.P.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_update(CgSys S, int par) {
  cg_update_body<D, T>(S, logical_block(S.P.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ir_update(CgSys S) {
  ir_update_body<D, T>(S, logical_block(S.P.nblk));
}

// Batched forms: one grid over the row ranges of all systems of a batch;
// bmap[block] is the table entry of the system that block belongs to.  Each
// system's blocks start at a multiple of 8, so the XCD mapping of a system's
// rows is the same as in its single-system launch.
template <int D, typename T, int OP>
__global__ void __launch_bounds__(NT) k_cg_spmv_b(const CgSys* __restrict__ tab, const int* __restrict__ bmap,
                                                  int par) {
  const CgSys S = tab[bmap[blockIdx.x]];
  cg_spmv_body<D, T, OP>(S, logical_of((int)blockIdx.x - S.boff, S.P.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_cg_update_b(const CgSys* __restrict__ tab, const int* __restrict__ bmap,
                                                    int par) {
  const CgSys S = tab[bmap[blockIdx.x]];
  cg_update_body<D, T>(S, logical_of((int)blockIdx.x - S.boff, S.P.nblk), par);
}

// ---------------------------------------------------------------------------
// CG with the element-factor operator, element-centric (two kernels per
// iteration, no stored q):
//   E1, one thread per element (parity par): after cg_head, the new direction
//     p = r + beta p_old on the element's d+1 faces (gathered; both elements of
//     a face compute bit-identical values), w_K = G~_K p_K (its contribution
//     to G~ p, stored per element), and the partial p.G~p = sum_K p_K.w_K
//     (each term >= 0 up to rounding: every G~_K is positive semi-definite);
//     the owner element (C = +1) of each face stores p there.
//   E2, one thread per face: q = w_K + w_L over the face's two elements (owner
//     first), alpha = rho / p.G~p, x += alpha p, r -= alpha q, partial r.r.
// p alternates between two buffers by parity.  w is stored [element][local
// face][component] so that E2 reads each side as one short vector.
// ---------------------------------------------------------------------------
// a * b + c with one rounding, the same in every kernel that forms the
// direction (the element kernel and, in 3D, the face kernel compute it for the
// same face and must agree bit for bit)
template <typename T>
__device__ __forceinline__ T mul_add(T a, T b, T c) {
  if constexpr (std::is_same<T, float>::value)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

// In 3D the face kernel stores the new direction (coalesced, one thread per
// face) and the element kernel does not scatter it to the owner faces: the
// scattered 12-byte stores cost as much as the element contributions' twice
// larger coalesced ones (measured on 64^3 x 6).  In 2D the scattered stores are
// cheap and the element kernel keeps them.
__host__ __device__ constexpr bool ec2_stores_direction(int d) { return d == 3; }

// Elements per thread whose loads are in flight together: four in 2D FP32
// (about 28 values each) where each thread has at least four elements, one
// elsewhere (measured on 512x512x2 and 64^3x6).
template <int D, typename T>
constexpr int ec1_batch() { return (D == 2 && sizeof(T) == 4) ? 4 : 1; }

// the element loop of E1 over [lo, hi) with EB elements per pass
template <int D, typename T, int EB>
__device__ __forceinline__ void ec1_pass(const CgSys& S, int par, int64_t lo, int64_t hi, double beta_d, bool first,
                                         double (&acc)[1]) {
  using L = EfoLayout<D>;
  constexpr int N = L::N;
  const T beta = (T)beta_d;
  const T* __restrict__ F = (const T*)S.F;
  const T* __restrict__ r = (const T*)S.r;
  const T* __restrict__ pold = (const T*)(par ? S.p : S.p1);
  T* __restrict__ pnew = (T*)(par ? S.p1 : S.p);
  T* __restrict__ tq = (T*)S.tq;
  const int64_t ne = S.ne;
  const double* __restrict__ mold = S.nagg > 0 ? S.M2 + (par ^ 1) * S.nagg : nullptr;
  // EB elements (stride NT) per pass: indices, flags, factors, and r and the
  // previous direction at their faces are all loaded before any is used;
  // indices past the range are clamped to its last element (ne >= 1), so the
  // loads carry no branches.  In 3D the element data (read once) is loaded
  // non-temporally, so that it does not push the gathered face vectors, which
  // neighbouring elements read again, out of the L2 (measured on 64^3 x 6:
  // 4.5% fewer bytes fetched, 7% faster; in 2D it is slower)
  for (int64_t Kb = lo + threadIdx.x; Kb < hi; Kb += (int64_t)EB * NT) {
    int32_t g[EB][N];
    uint32_t fl[EB];
    T fv[EB][L::NF];
    Vec<T, D> rv[EB][N], po[EB][N];
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int64_t K = min(Kb + (int64_t)e * NT, hi - 1);
      if constexpr (D == 3) {
        fl[e] = __builtin_nontemporal_load(S.eflags + K);
#pragma unroll
        for (int l = 0; l < N; ++l) g[e][l] = __builtin_nontemporal_load(S.egat + (int64_t)l * ne + K);
#pragma unroll
        for (int c = 0; c < L::NF; ++c) fv[e][c] = __builtin_nontemporal_load(F + (int64_t)c * ne + K);
      } else {
        fl[e] = S.eflags[K];
#pragma unroll
        for (int l = 0; l < N; ++l) g[e][l] = S.egat[(int64_t)l * ne + K];
#pragma unroll
        for (int c = 0; c < L::NF; ++c) fv[e][c] = F[(int64_t)c * ne + K];
      }
    }
#pragma unroll
    for (int e = 0; e < EB; ++e)
#pragma unroll
      for (int l = 0; l < N; ++l) {
        rv[e][l] = ldv<T, D>(r, g[e][l]);
        if (!first) po[e][l] = ldv<T, D>(pold, g[e][l]);
      }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int64_t K = Kb + (int64_t)e * NT;
      if (K >= hi) break;
      Vec<T, D> ph[N], pn[N];
#pragma unroll
      for (int l = 0; l < N; ++l) {
        ph[l] = rv[e][l];
        if (!first)
#pragma unroll
          for (int i = 0; i < D; ++i) ph[l].v[i] = mul_add(beta, po[e][l].v[i], ph[l].v[i]);
        pn[l] = ph[l];
      }
      // The direction is p = ph + Z m, with m = E^-1 Z^t r + beta m_old per
      // aggregate.  Where all faces of K lie in one aggregate, (Z m)_K is m_a
      // times the local null vector of G'_K: it changes neither G'_K p_K nor
      // p_K . G'_K p_K, so only elements on aggregate boundaries add it here.
      if (S.nagg > 0 && (fl[e] & F_AGGB)) {
#pragma unroll
        for (int l = 0; l < N; ++l) {
          const int a = S.fagg[g[e][l]];
          const T m = (T)(first ? S.mu[a] : S.mu[a] + beta_d * mold[a]);
          const Vec<T, D> z = ldv<T, D>((const T*)S.zT, g[e][l]);
#pragma unroll
          for (int i = 0; i < D; ++i) pn[l].v[i] += z.v[i] * m;
        }
      }
      T t = T(0);
#pragma unroll
      for (int l = 0; l < N; ++l)
#pragma unroll
        for (int i = 0; i < D; ++i) t += fv[e][L::vh(l, i)] * pn[l].v[i];
      Vec<T, D> w[N];
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < D; ++i) {
          T a = -fv[e][L::vh(j, i)] * t;
#pragma unroll
          for (int l = 0; l < N; ++l) a += fv[e][L::sym(j, l)] * pn[l].v[i];
          w[j].v[i] = a;
          acc[0] += (double)pn[j].v[i] * (double)a;
        }
#pragma unroll
      for (int j = 0; j < N; ++j) stv<T, D>(tq, K * N + j, w[j]);
      // the owner stores the direction without its coarse part
      if constexpr (!ec2_stores_direction(D))
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (((fl[e] >> j) & 1u) && !((fl[e] >> (8 + j)) & 1u)) stv<T, D>(pnew, g[e][j], ph[j]);
    }
  }
}

template <int D, typename T>
__device__ __forceinline__ void ec1_body(const CgSys& S, int lb, int par) {
  constexpr int EB = ec1_batch<D, T>();
  double beta_d;
  bool first;
  if (!cg_head(S, lb, par, beta_d, first, S.nagg > 0)) return;
  const int64_t lo = (int64_t)lb * S.PE.chunk, hi = min(S.ne, lo + S.PE.chunk);
  double acc[1] = {0.0};
  if (EB > 1 && S.PE.chunk >= (int64_t)EB * NT)
    ec1_pass<D, T, EB>(S, par, lo, hi, beta_d, first, acc);
  else
    ec1_pass<D, T, 1>(S, par, lo, hi, beta_d, first, acc);
  block_sum<1>(acc);
  if (threadIdx.x == 0) S.Pb[lb] = acc[0];
}

template <int D, typename T>
__device__ __forceinline__ void ec2_body(const CgSys& S, int lb, int par) {
  constexpr int N = D + 1;
  KState* st = S.st;
  // the state words, the partials of p.G~p and the coarse values of this
  // block's aggregates are all requested before any is used
  const int done = st->done;
  const double gam = st->gam[par], cbeta = st->bet[par];
  const bool cfirst = st->it[par] - 1 == st->it_first;
  const int a0 = S.nagg > 0 ? S.ablk[lb] : 0;
  const double* __restrict__ mold = S.nagg > 0 ? S.M2 + (par ^ 1) * S.nagg : nullptr;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < S.PE.nblk; i += NT) v[0] += S.Pb[i];
  double mu_k[KMAX], mo_k[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int a = min(a0 + k, S.nagg - 1);
    mu_k[k] = S.nagg > 0 ? S.mu[a] : 0.0;
    mo_k[k] = S.nagg > 0 ? mold[a] : 0.0;
  }
  if (block_sum_stop<1>(v, done)) return;
  const double pq = v[0];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (threadIdx.x == 0 && lb == 0) st->done = isfinite(pq) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double alpha = gam / pq;
  const T ta = (T)alpha;
  const Part P = S.P;
  T* __restrict__ x = (T*)S.x;
  T* __restrict__ r = (T*)S.r;
  // the direction without its coarse part: stored by the element kernel, or
  // (3D) formed here from r and the previous direction as the element kernel
  // formed it, and stored
  const T* __restrict__ p = (const T*)(par ? S.p1 : S.p);
  const T* __restrict__ pold = (const T*)(par ? S.p : S.p1);
  T* __restrict__ pnew = (T*)(par ? S.p1 : S.p);
  const T tbeta = (T)cbeta;
  const T* __restrict__ tq = (const T*)S.tq;
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  if (S.nagg > 0 && lb == 0)  // the coarse part m of this iteration's direction
    for (int a = threadIdx.x; a < S.nagg; a += NT)
      S.M2[par * S.nagg + a] = cfirst ? S.mu[a] : S.mu[a] + cbeta * mold[a];
  // m of the (at most KMAX) aggregates of this block's faces
  T mk[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) mk[k] = S.nagg > 0 ? (T)(cfirst ? mu_k[k] : mu_k[k] + cbeta * mo_k[k]) : T(0);
  double acc[1] = {0.0};
  double racc[KMAX] = {};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const int64_t K = S.fel[f], Lr = S.fel[P.nf + f];
    const int lc = S.floc[f];
    const Vec<T, D> wk = ldv<T, D>(tq, K * N + (lc & 0xff));
    const Vec<T, D> wl = ldv<T, D>(tq, Lr * N + ((lc >> 8) & 0xff));
    Vec<T, D> xi = ldv<T, D>(x, f), ri = ldv<T, D>(r, f), pi;
    if constexpr (ec2_stores_direction(D)) {
      pi = ri;
      if (!cfirst) {
        const Vec<T, D> po = ldv<T, D>(pold, f);
#pragma unroll
        for (int i = 0; i < D; ++i) pi.v[i] = mul_add(tbeta, po.v[i], ri.v[i]);
      }
      stv<T, D>(pnew, f, pi);
    } else {
      pi = ldv<T, D>(p, f);
    }
    Vec<T, D> zf;
    int ak = 0;
    if (S.nagg > 0) {
      zf = ldv<T, D>((const T*)S.zT, f);
      ak = S.fagg[f] - a0;
      T m = mk[0];
#pragma unroll
      for (int k = 1; k < KMAX; ++k) m = ak == k ? mk[k] : m;
#pragma unroll
      for (int i = 0; i < D; ++i) pi.v[i] += zf.v[i] * m;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const T qi = wk.v[i] + wl.v[i];
      xi.v[i] += ta * pi.v[i];
      ri.v[i] -= ta * qi;
      acc[0] += (double)ri.v[i] * (double)ri.v[i];
    }
    stv<T, D>(x, f, xi);
    stv<T, D>(r, f, ri);
    if (S.nagg > 0) {
      double zr = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) zr += (double)zf.v[i] * (double)ri.v[i];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) racc[k] += ak == k ? zr : 0.0;
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) S.Pa[lb] = acc[0];
  if (S.nagg > 0) {
    block_sum<KMAX>(racc);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < KMAX; ++k) S.Pr[(int64_t)lb * KMAX + k] = racc[k];
  }
  if (threadIdx.x == 0 && lb == 0) st->alp[par] = alpha;
}

// Coarse solve: c_a = sum of the restriction partials of the face blocks that
// hold aggregate a (fixed order), mu = E^-1 c; one wavefront per row.  Only
// in the first of those blocks can a be other than the block's first
// aggregate (its faces are contiguous), so bfa carries, with that block
// shifted left by two bits, a's slot in it, and every later block contributes
// its slot 0.
static_assert(KMAX == 4, "the slot of an aggregate in its first face block takes two bits");
__device__ __forceinline__ void coarse_body(const CgSys& S, int cb) {
  if (S.st->done) return;
  __shared__ double c[MAX_AGG];
  for (int a = threadIdx.x; a < S.nagg; a += NT) {
    const int pk = S.bfa[a], b1 = S.bla[a], b0 = pk >> 2;
    double v = 0.0;
    if (b0 <= b1) {
      v = S.Pr[(int64_t)b0 * KMAX + (pk & 3)];
      for (int b = b0 + 1; b <= b1; ++b) v += S.Pr[(int64_t)b * KMAX];
    }
    c[a] = v;
  }
  __syncthreads();
  const int row = cb * (NT / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= S.nagg) return;
  double v = 0.0;
  for (int j = lane; j < S.nagg; j += 64) v += S.Einv[(int64_t)row * S.nagg + j] * c[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) {
    S.mu[row] = v;
    S.cvec[row] = c[row];
  }
}

__global__ void __launch_bounds__(NT) k_coarse(CgSys S) { coarse_body(S, blockIdx.x); }

__global__ void __launch_bounds__(NT) k_coarse_b(const CgSys* __restrict__ tab, const int* __restrict__ bmap) {
  const CgSys S = tab[bmap[blockIdx.x]];
  coarse_body(S, (int)blockIdx.x - S.boffC);
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ec1(CgSys S, int par) {
  ec1_body<D, T>(S, logical_block(S.PE.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ec2(CgSys S, int par) {
  ec2_body<D, T>(S, logical_block(S.P.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ec1_b(const CgSys* __restrict__ tab, const int* __restrict__ bmap, int par) {
  const CgSys S = tab[bmap[blockIdx.x]];
  ec1_body<D, T>(S, logical_of((int)blockIdx.x - S.boffE, S.PE.nblk), par);
}
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_ec2_b(const CgSys* __restrict__ tab, const int* __restrict__ bmap, int par) {
  const CgSys S = tab[bmap[blockIdx.x]];
  ec2_body<D, T>(S, logical_of((int)blockIdx.x - S.boff, S.P.nblk), par);
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
  const int seen = st->done;
  const int it = st->it[par ^ 1];
  const bool first = it == st->it_first;
  const bool fresh = it == st->it_rep;
  double rho, rr, tres2 = 0.0, snorm2 = 0.0;
  if (fresh) {
    const int fl[4] = {0, 3, 1, 2};
    double v[4];
    if (reduce_fields_stop<4>(Pa, P.nblk, fl, v, seen)) return;
    rho = v[0];
    rr = v[1];
    tres2 = v[2];
    snorm2 = v[3];
  } else {
    const int fl[2] = {0, 3};
    double v[2];
    if (reduce_fields_stop<2>(Pa, P.nblk, fl, v, seen)) return;
    rho = v[0];
    rr = v[1];
  }
  const Decision dec = decide(st, it, fresh, rr, tres2, snorm2, std::is_same<T, float>::value);
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
  const int seen = st->done;
  const int fl[1] = {0};
  double v[1];
  if (reduce_fields_stop<1>(Pb, P.nblk, fl, v, seen)) return;
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
  const int seen = st->done;
  const int fl[2] = {0, 1};
  double v[2];
  if (reduce_fields_stop<2>(Pc, P.nblk, fl, v, seen)) return;
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

// ---------------------------------------------------------------------------
// BiCGStab(2) on the scaled non-symmetric system: per iteration two BiCG steps
// followed by a minimal-residual step over a polynomial of degree two, which
// (unlike the degree-one step of BiCGStab) can damp both signs of a real
// indefinite spectrum.  Five kernels per iteration, four products with G,
// each product fed on the fly with the linear combination it acts on:
//   E1: rho1 = rhat.r, beta1 = alpha rho1 / rho0 (rho0 = -omega2 rho_prev);
//       u1 = r - beta1 u, v = G u1; partial rhat.v
//   E2: alpha1 = rho1 / rhat.v; r1 = r - alpha1 v, s = G r1; x += alpha1 u1;
//       partial rhat.s
//   E3: beta2 = alpha1 rhat.s / rho1; v1 = s - beta2 v, w = G v1; partial rhat.w
//   E4: alpha2 = rhat.s / rhat.w; u2 = r1 - beta2 u1, r2 = r1 - alpha2 v1,
//       s2 = s - alpha2 w, t = G s2; partials r2.s2, s2.s2, s2.t, t.t, r2.t
//   E5: omega1, omega2 minimise |r2 - omega1 s2 - omega2 t|;
//       x += omega1 r2 + omega2 s2 + alpha2 u2, r = r2 - omega1 s2 - omega2 t,
//       u = u2 - omega1 v1 - omega2 w; partials rhat.r, r.r
// rhat is the fixed shadow residual (reset to r at a restart).
// ---------------------------------------------------------------------------
template <typename T, int D>
struct AxpyIn {
  const T* __restrict__ a;
  const T* __restrict__ b;
  T coef;
  bool only_a;
  __device__ Vec<T, D> operator()(int64_t c) const {
    Vec<T, D> x = ldv<T, D>(a, c);
    if (only_a) return x;
    const Vec<T, D> y = ldv<T, D>(b, c);
#pragma unroll
    for (int i = 0; i < D; ++i) x.v[i] -= coef * y.v[i];
    return x;
  }
};

struct B2Vecs {
  void* x;
  void* r;
  void* r1;
  void* u;
  void* u1;
  void* v;
  void* v1;
  void* s;
  void* s2;
  void* w;
  void* t;
  void* rhat;
};

template <int D, typename T>
__device__ __forceinline__ void rowrange(const Part& P, int& lb, int64_t& lo, int64_t& hi) {
  lb = logical_block(P.nblk);
  lo = (int64_t)lb * P.chunk;
  hi = min(P.nf, lo + P.chunk);
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_b2_1(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                             B2Vecs V, const double* __restrict__ Pa, double* __restrict__ Pb,
                                             KState* __restrict__ st, int par) {
  const int seen = st->done;
  const int it = st->it[par ^ 1];
  const bool first = it == st->it_first;
  const bool fresh = it == st->it_rep;
  double rho1, rr, tres2 = 0.0, snorm2 = 0.0;
  if (fresh) {
    const int fl[4] = {0, 3, 1, 2};
    double v[4];
    if (reduce_fields_stop<4>(Pa, P.nblk, fl, v, seen)) return;
    rho1 = v[0];
    rr = v[1];
    tres2 = v[2];
    snorm2 = v[3];
  } else {
    const int fl[2] = {0, 3};
    double v[2];
    if (reduce_fields_stop<2>(Pa, P.nblk, fl, v, seen)) return;
    rho1 = v[0];
    rr = v[1];
  }
  const Decision dec = decide(st, it, fresh, rr, tres2, snorm2, std::is_same<T, float>::value);
  int done = dec.done;
  if (!done && (!(rho1 != 0.0) || !isfinite(rho1))) done = isfinite(rho1) ? BREAKDOWN : NONFINITE;
  double beta1 = 0.0;
  if (!first) {
    const double rho0 = -st->omega2[par ^ 1] * st->rho_b[par ^ 1];
    beta1 = st->alpha2[par ^ 1] * rho1 / rho0;
  }
  if (lead()) {
    record_decision(st, dec, fresh, it, rr, tres2, snorm2);
    if (done) {
      st->done = done;
    } else {
      st->rho_a[par] = rho1;
      st->beta1[par] = beta1;
      st->it[par] = it + 1;
      st->nrun += 1;
    }
  }
  if (done) return;
  const AxpyIn<T, D> in{(const T*)V.r, (const T*)V.u, (T)beta1, first};
  int lb;
  int64_t lo, hi;
  rowrange<D, T>(P, lb, lo, hi);
  const T* __restrict__ rhat = (const T*)V.rhat;
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<T, D> vv = spmv_row<D, T>(G, cols, P.nf, f, in);
    stv<T, D>((T*)V.u1, f, in(f));
    stv<T, D>((T*)V.v, f, vv);
    const Vec<T, D> rh = ldv<T, D>(rhat, f);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[0] += (double)rh.v[i] * (double)vv.v[i];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) Pb[lb] = acc[0];
}

// E2 and E4 share the breakdown test of a denominator from one partial field
__device__ __forceinline__ bool b2_denominator(const double* __restrict__ part, int nblk, KState* st, int seen,
                                               double& val) {
  const int fl[1] = {0};
  double v[1];
  if (reduce_fields_stop<1>(part, nblk, fl, v, seen)) return false;
  val = v[0];
  if (!(val != 0.0) || !isfinite(val)) {
    if (lead()) st->done = isfinite(val) ? BREAKDOWN : NONFINITE;
    return false;
  }
  return true;
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_b2_2(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                             B2Vecs V, const double* __restrict__ Pb, double* __restrict__ Pc,
                                             KState* __restrict__ st, int par) {
  const int seen = st->done;
  double g1;
  if (!b2_denominator(Pb, P.nblk, st, seen, g1)) return;
  const double alpha1 = st->rho_a[par] / g1;
  const AxpyIn<T, D> in{(const T*)V.r, (const T*)V.v, (T)alpha1, false};
  int lb;
  int64_t lo, hi;
  rowrange<D, T>(P, lb, lo, hi);
  const T ta = (T)alpha1;
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<T, D> ss = spmv_row<D, T>(G, cols, P.nf, f, in);
    stv<T, D>((T*)V.r1, f, in(f));
    stv<T, D>((T*)V.s, f, ss);
    Vec<T, D> xi = ldv<T, D>((const T*)V.x, f);
    const Vec<T, D> ui = ldv<T, D>((const T*)V.u1, f), rh = ldv<T, D>((const T*)V.rhat, f);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xi.v[i] += ta * ui.v[i];
      acc[0] += (double)rh.v[i] * (double)ss.v[i];
    }
    stv<T, D>((T*)V.x, f, xi);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) Pc[lb] = acc[0];
  if (lead()) st->alpha1[par] = alpha1;
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_b2_3(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                             B2Vecs V, const double* __restrict__ Pc, double* __restrict__ Pb,
                                             KState* __restrict__ st, int par) {
  const int seen = st->done;
  double rho2;
  if (!b2_denominator(Pc, P.nblk, st, seen, rho2)) return;
  const double beta2 = st->alpha1[par] * rho2 / st->rho_a[par];
  const AxpyIn<T, D> in{(const T*)V.s, (const T*)V.v, (T)beta2, false};
  int lb;
  int64_t lo, hi;
  rowrange<D, T>(P, lb, lo, hi);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<T, D> ww = spmv_row<D, T>(G, cols, P.nf, f, in);
    stv<T, D>((T*)V.v1, f, in(f));
    stv<T, D>((T*)V.w, f, ww);
    const Vec<T, D> rh = ldv<T, D>((const T*)V.rhat, f);
#pragma unroll
    for (int i = 0; i < D; ++i) acc[0] += (double)rh.v[i] * (double)ww.v[i];
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) Pb[lb] = acc[0];
  if (lead()) {
    st->rho_b[par] = rho2;
    st->beta2[par] = beta2;
  }
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_b2_4(Part P, const T* __restrict__ G, const int32_t* __restrict__ cols,
                                             B2Vecs V, const double* __restrict__ Pb, double* __restrict__ Pc,
                                             KState* __restrict__ st, int par) {
  const int seen = st->done;
  double g2;
  if (!b2_denominator(Pb, P.nblk, st, seen, g2)) return;
  const double alpha2 = st->rho_b[par] / g2;
  const T ta = (T)alpha2, tb = (T)st->beta2[par];
  const AxpyIn<T, D> in{(const T*)V.s, (const T*)V.w, ta, false};
  int lb;
  int64_t lo, hi;
  rowrange<D, T>(P, lb, lo, hi);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<T, D> tt = spmv_row<D, T>(G, cols, P.nf, f, in);
    const Vec<T, D> s2 = in(f);
    Vec<T, D> r1 = ldv<T, D>((const T*)V.r1, f), u1 = ldv<T, D>((const T*)V.u1, f);
    const Vec<T, D> v1 = ldv<T, D>((const T*)V.v1, f);
    Vec<T, D> u2;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      u2.v[i] = r1.v[i] - tb * u1.v[i];
      r1.v[i] -= ta * v1.v[i];  // r2
      acc[0] += (double)r1.v[i] * (double)s2.v[i];
      acc[1] += (double)s2.v[i] * (double)s2.v[i];
      acc[2] += (double)s2.v[i] * (double)tt.v[i];
      acc[3] += (double)tt.v[i] * (double)tt.v[i];
      acc[4] += (double)r1.v[i] * (double)tt.v[i];
    }
    stv<T, D>((T*)V.u, f, u2);
    stv<T, D>((T*)V.r1, f, r1);
    stv<T, D>((T*)V.s2, f, s2);
    stv<T, D>((T*)V.t, f, tt);
  }
  block_sum<5>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < 5; ++m) Pc[(int64_t)m * P.nblk + lb] = acc[m];
  if (lead()) st->alpha2[par] = alpha2;
}

template <int D, typename T>
__global__ void __launch_bounds__(NT) k_b2_5(Part P, B2Vecs V, const double* __restrict__ Pc,
                                             double* __restrict__ Pa, KState* __restrict__ st, int par) {
  const int seen = st->done;
  const int fl[5] = {0, 1, 2, 3, 4};
  double v[5];
  if (reduce_fields_stop<5>(Pc, P.nblk, fl, v, seen)) return;
  const double rs = v[0], ss = v[1], stt = v[2], tt = v[3], rt = v[4];
  // minimise |r2 - omega1 s2 - omega2 t| (Gram-Schmidt of t against s2)
  const double tau = tt - stt * stt / ss;
  bool ok = ss > 0.0 && tau > 0.0 && isfinite(ss) && isfinite(tau) && isfinite(rs) && isfinite(rt);
  if (!ok) {
    if (lead()) st->done = (isfinite(ss) && isfinite(tt) && isfinite(rs) && isfinite(rt)) ? BREAKDOWN : NONFINITE;
    return;
  }
  const double om2 = (rt - stt * rs / ss) / tau;
  const double om1 = (rs - stt * om2) / ss;
  const T o1 = (T)om1, o2 = (T)om2, ta = (T)st->alpha2[par];
  int lb;
  int64_t lo, hi;
  rowrange<D, T>(P, lb, lo, hi);
  double acc[2] = {0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> xi = ldv<T, D>((const T*)V.x, f), u2 = ldv<T, D>((const T*)V.u, f);
    const Vec<T, D> r2 = ldv<T, D>((const T*)V.r1, f), s2 = ldv<T, D>((const T*)V.s2, f),
                    ti = ldv<T, D>((const T*)V.t, f), v1 = ldv<T, D>((const T*)V.v1, f),
                    wi = ldv<T, D>((const T*)V.w, f), rh = ldv<T, D>((const T*)V.rhat, f);
    Vec<T, D> rn;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      xi.v[i] += o1 * r2.v[i] + o2 * s2.v[i] + ta * u2.v[i];
      rn.v[i] = r2.v[i] - o1 * s2.v[i] - o2 * ti.v[i];
      u2.v[i] -= o1 * v1.v[i] + o2 * wi.v[i];
      acc[0] += (double)rh.v[i] * (double)rn.v[i];
      acc[1] += (double)rn.v[i] * (double)rn.v[i];
    }
    stv<T, D>((T*)V.x, f, xi);
    stv<T, D>((T*)V.r, f, rn);
    stv<T, D>((T*)V.u, f, u2);
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    Pa[lb] = acc[0];
    Pa[(int64_t)3 * P.nblk + lb] = acc[1];
  }
  if (lead()) st->omega2[par] = om2;
}

// ---------------------------------------------------------------------------
// MINRES (Paige-Saunders) on the scaled symmetric G, positive definite or not
// (steady Stokes: symmetric indefinite, Section 3.2 item 7).  The scaling
// Ds G Ds is the (positive) Jacobi preconditioner.  Refinement passes: each
// pass computes the FP64 residual r = bs - G64 y, runs MINRES in the working
// precision on G x = r from x = 0 until its residual estimate falls below the
// pass target, and adds x to y.  Three kernels per iteration; the Lanczos and
// direction vectors rotate through three buffers each.
// ---------------------------------------------------------------------------
template <typename T, int D>
struct ScaledIn {
  const T* __restrict__ a;
  T scale;
  __device__ Vec<T, D> operator()(int64_t c) const {
    Vec<T, D> x = ldv<T, D>(a, c);
#pragma unroll
    for (int i = 0; i < D; ++i) x.v[i] *= scale;
    return x;
  }
};

struct MState {
  double beta[2], oldb[2], dbar[2], epsln[2], cs[2], sn[2], phibar[2], alfa[2];
  int it[2];
  int done;   // 0 running, 1 pass target reached, 2 converged (true residual), 3 limit, 4 breakdown, 5 non-finite
  int iters;
  double tres2, bnorm2, thr;
  // parameters written by the host
  double tol2, rep;
  int maxit;
};

// init: r = bs - G64 y in FP64, r1 = r2 = (T) r, w = 0, x = 0;
// partials: 0 = r.r (working precision), 1 = |S - G W|^2, 2 = |S|^2
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_hm_init(CgSys S, T* __restrict__ r1, T* __restrict__ r2, T* __restrict__ w0,
                                                T* __restrict__ w1, MState* __restrict__ ms) {
  const Part P = S.P;
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  T* __restrict__ x = (T*)S.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<double, D> gy = spmv_row<D, double>(S.G64, S.cols, P.nf, f, Plain<double, D>{S.y});
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double b = S.bs[f * D + i], sq = S.dsq[f * D + i];
      const double rs = b - gy.v[i];
      const T rt = (T)rs;
      r1[f * D + i] = rt;
      r2[f * D + i] = rt;
      w0[f * D + i] = T(0);
      w1[f * D + i] = T(0);
      x[f * D + i] = T(0);
      acc[0] += (double)rt * (double)rt;
      acc[1] += (sq * rs) * (sq * rs);
      acc[2] += (sq * b) * (sq * b);
    }
  }
  block_sum<3>(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < 3; ++m) S.Pa[(int64_t)m * P.nblk + lb] = acc[m];
  if (lead()) {
    ms->it[1] = 0;
    ms->oldb[1] = 0.0;
    ms->dbar[1] = 0.0;
    ms->epsln[1] = 0.0;
    ms->cs[1] = -1.0;
    ms->sn[1] = 0.0;
    ms->iters = 0;
    ms->done = 0;
  }
}

// MA: v = r2 / beta, y = G v - (beta / oldb) r1, partial v.y
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_hm_a(CgSys S, const T* __restrict__ r1, const T* __restrict__ r2,
                                             T* __restrict__ v, T* __restrict__ y, MState* __restrict__ ms, int q) {
  const int seen = ms->done;
  const Part P = S.P;
  const int p = q ^ 1;
  const int it = ms->it[p];
  const bool first = it == 0;
  double beta, oldb;
  int done = 0;
  if (first) {
    const int fl[3] = {0, 1, 2};
    double sv[3];
    if (reduce_fields_stop<3>(S.Pa, P.nblk, fl, sv, seen)) return;
    beta = sqrt(sv[0]);
    oldb = 0.0;
    // pass target in the scaled norm: 0.1 of the tolerance, converted by the
    // ratio of the two norms of the same residual, and at most a reduction
    // by rep (precision of the working arithmetic)
    const double ratio = sv[1] > 0.0 ? beta / sqrt(sv[1]) : 1.0;
    const double thr = fmax(0.1 * sqrt(ms->tol2 * sv[2]) * ratio, ms->rep * beta);
    if (sv[1] <= ms->tol2 * sv[2]) done = 2;
    else if (!(beta > 0.0) || !isfinite(beta)) done = isfinite(beta) ? 4 : 5;
    else if (it >= ms->maxit) done = 3;
    if (lead()) {
      ms->tres2 = sv[1];
      ms->bnorm2 = sv[2];
      ms->thr = thr;
      ms->beta[p] = beta;
      ms->phibar[p] = beta;
    }
  } else {
    // no reduction before the decision: a wave that saw the word set returns,
    // and the others reach the same decision from the same state and return
    if (seen) return;
    beta = ms->beta[p];
    oldb = ms->oldb[p];
    if (ms->phibar[p] <= ms->thr) done = 1;
    else if (it >= ms->maxit) done = 3;
  }
  if (lead()) {
    ms->it[q] = it + 1;
    ms->iters = it;
    if (done) ms->done = done;
  }
  if (done) return;
  const T sb = (T)(1.0 / beta);
  const T c1 = first ? T(0) : (T)(beta / oldb);
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  const ScaledIn<T, D> in{r2, sb};
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> yy = spmv_row<D, T>((const T*)S.G, S.cols, P.nf, f, in);
    const Vec<T, D> vv = in(f), rr = ldv<T, D>(r1, f);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      yy.v[i] -= c1 * rr.v[i];
      acc[0] += (double)vv.v[i] * (double)yy.v[i];
    }
    stv<T, D>(v, f, vv);
    stv<T, D>(y, f, yy);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) S.Pb[lb] = acc[0];
}

// MB: alfa = v.y; y -= (alfa / beta) r2 (y becomes the next r2); partial y.y
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_hm_b(CgSys S, const T* __restrict__ r2, T* __restrict__ y,
                                             MState* __restrict__ ms, int q) {
  if (ms->done) return;
  const Part P = S.P;
  const int fl[1] = {0};
  double sv[1];
  reduce_fields<1>(S.Pb, P.nblk, fl, sv);
  const double alfa = sv[0];
  const T c2 = (T)(alfa / ms->beta[q ^ 1]);
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  double acc[1] = {0.0};
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    Vec<T, D> yy = ldv<T, D>(y, f);
    const Vec<T, D> rr = ldv<T, D>(r2, f);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      yy.v[i] -= c2 * rr.v[i];
      acc[0] += (double)yy.v[i] * (double)yy.v[i];
    }
    stv<T, D>(y, f, yy);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) S.Pc[lb] = acc[0];
  if (lead()) ms->alfa[q] = alfa;
}

// MC: beta_new = |y|; plane rotations; w = (v - oldeps w1 - delta w2) / gamma; x += phi w
template <int D, typename T>
__global__ void __launch_bounds__(NT) k_hm_c(CgSys S, const T* __restrict__ v, const T* __restrict__ w1,
                                             const T* __restrict__ w2, T* __restrict__ wn, MState* __restrict__ ms,
                                             int q) {
  const int seen = ms->done;
  const Part P = S.P;
  const int fl[1] = {0};
  double sv[1];
  if (reduce_fields_stop<1>(S.Pc, P.nblk, fl, sv, seen)) return;
  const int p = q ^ 1;
  if (!(sv[0] >= 0.0) || !isfinite(sv[0])) {
    if (lead()) ms->done = isfinite(sv[0]) ? 4 : 5;
    return;
  }
  const double beta = sqrt(sv[0]);
  const double oldb = ms->beta[p];
  const double alfa = ms->alfa[q];
  const double cs = ms->cs[p], sn = ms->sn[p], dbar = ms->dbar[p], oldeps = ms->epsln[p];
  const double delta = cs * dbar + sn * alfa;
  const double gbar = sn * dbar - cs * alfa;
  const double epsln = sn * beta;
  const double dbar_n = -cs * beta;
  const double gamma = fmax(hypot(gbar, beta), 1e-300);
  const double cs_n = gbar / gamma, sn_n = beta / gamma;
  const double phibar = ms->phibar[p];
  const T phi = (T)(cs_n * phibar);
  const T den = (T)(1.0 / gamma), te = (T)oldeps, td = (T)delta;
  const int lb = logical_block(P.nblk);
  const int64_t lo = (int64_t)lb * P.chunk, hi = min(P.nf, lo + P.chunk);
  T* __restrict__ x = (T*)S.x;
  for (int64_t f = lo + threadIdx.x; f < hi; f += NT) {
    const Vec<T, D> vv = ldv<T, D>(v, f), a = ldv<T, D>(w1, f), b = ldv<T, D>(w2, f);
    Vec<T, D> xi = ldv<T, D>(x, f), wv;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      wv.v[i] = (vv.v[i] - te * a.v[i] - td * b.v[i]) * den;
      xi.v[i] += phi * wv.v[i];
    }
    stv<T, D>(wn, f, wv);
    stv<T, D>(x, f, xi);
  }
  if (lead()) {
    ms->beta[q] = beta;
    ms->oldb[q] = oldb;
    ms->cs[q] = cs_n;
    ms->sn[q] = sn_n;
    ms->dbar[q] = dbar_n;
    ms->epsln[q] = epsln;
    ms->phibar[q] = sn_n * phibar;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// vector slots of the workspace
enum { V_X, V_P, V_R0, V_R1, V_W0, V_W1, V_S0, V_S1, V_RHAT, V_T, V_U2, V_V2, NVEC };

struct KWs {
  Part part{};           // face rows
  Part epart{};          // elements
  void* vec[NVEC] = {};  // each nf*d doubles
  void* tq = nullptr;    // element contributions, ne*(d+1)*d doubles
  // coarse correction: block/aggregate tables of this partition, restriction
  // partials, c and mu; use_coarse is set per solve
  bool coarse_ok = false, use_coarse = false;
  int32_t* ablk = nullptr;
  int32_t* bfa = nullptr;
  int32_t* bla = nullptr;
  double* Pr = nullptr;
  double* cvec = nullptr;
  double* mu = nullptr;
  double* M2 = nullptr;
  double* part3[3] = {};   // partial arrays, NFIELD x nblk each
  KState* st = nullptr;
  KState* hst = nullptr;   // pinned [3]
  hipEvent_t ev[2] = {};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec[2][3][3] = {};  // [precision][method][operator form, with coarse correction]
  int exec_m[2][3][3] = {};
  // scratch for kernel timing
  void* tvec[NVEC] = {};
  void* ttq = nullptr;
  double* tpart[2] = {};
  MState* mst = nullptr;    // MINRES state (device) and its pinned copy
  MState* mhst = nullptr;
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
  w->epart = make_part(s->ne);
  const size_t vb = sizeof(double) * (size_t)s->nf * s->d;
  for (auto& v : w->vec) {
    v = dev_alloc(s, vb);
    if (!v) return CR_E_NOMEM;
  }
  if (s->efo64) {
    w->tq = dev_alloc(s, sizeof(double) * (size_t)s->ne * (s->d + 1) * s->d);
    if (!w->tq) return CR_E_NOMEM;
  }
  if (s->nagg > 0) {
    // tables of the coarse restriction for this face partition: faces of an
    // aggregate are contiguous, so each face block holds a contiguous range of
    // aggregates (at most KMAX, else the correction is not used)
    const Part& P = w->part;
    const std::vector<int32_t>& fa = s->topo.face_agg;
    const int m = s->nagg;
    std::vector<int32_t> ablk(P.nblk, 0), bfa(m, 1), bla(m, 0);
    bool ok = true;
    for (int b = 0; b < P.nblk; ++b) {
      const int64_t lo = (int64_t)b * P.chunk, hi = std::min<int64_t>(s->nf, lo + P.chunk);
      if (lo >= hi) continue;
      ablk[b] = fa[lo];
      if (fa[hi - 1] - fa[lo] + 1 > KMAX) ok = false;
    }
    for (int64_t f = 0; f < s->nf; ++f) {
      const int a = fa[f], b = (int)(f / P.chunk);
      if (f == 0 || fa[f - 1] != a) bfa[a] = b;
      bla[a] = b;
    }
    // the first block of each aggregate, shifted, with the aggregate's slot in
    // that block's restriction partials (an empty aggregate keeps b0 > bla)
    for (int a = 0; a < m; ++a) {
      const int slot = bfa[a] <= bla[a] ? std::min(KMAX - 1, std::max(0, a - ablk[bfa[a]])) : 0;
      bfa[a] = (bfa[a] << 2) | slot;
    }
    w->coarse_ok = ok;
    auto up = [&](int32_t*& dst, const std::vector<int32_t>& src) {
      dst = (int32_t*)dev_alloc(s, sizeof(int32_t) * src.size());
      if (!dst) return CR_E_NOMEM;
      return check_hip(hipMemcpy(dst, src.data(), sizeof(int32_t) * src.size(), hipMemcpyHostToDevice), "coarse tables");
    };
    cr_status cs = up(w->ablk, ablk);
    if (cs == CR_OK) cs = up(w->bfa, bfa);
    if (cs == CR_OK) cs = up(w->bla, bla);
    if (cs != CR_OK) return cs;
    w->Pr = (double*)dev_alloc(s, sizeof(double) * (size_t)P.nblk * KMAX);
    w->cvec = (double*)dev_alloc(s, sizeof(double) * m);
    w->mu = (double*)dev_alloc(s, sizeof(double) * m);
    w->M2 = (double*)dev_alloc(s, sizeof(double) * 2 * m);
    if (!w->Pr || !w->cvec || !w->mu || !w->M2) return CR_E_NOMEM;
    cs = check_hip(hipMemset(w->cvec, 0, sizeof(double) * m), "coarse vectors");
    if (cs == CR_OK) cs = check_hip(hipMemset(w->mu, 0, sizeof(double) * m), "coarse vectors");
    if (cs == CR_OK) cs = check_hip(hipMemset(w->M2, 0, sizeof(double) * 2 * m), "coarse vectors");
    if (cs != CR_OK) return cs;
  }
  const size_t pbytes = sizeof(double) * (size_t)std::max(w->part.nblk, w->epart.nblk) * NFIELD;
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

CgSys make_sys(cr_system* s, KWs* w, int prec, KState* st) {
  CgSys S{};
  S.P = w->part;
  S.PE = w->epart;
  S.p1 = w->vec[V_W1];
  S.tq = w->tq;
  S.eflags = s->eflags;
  S.bs1 = s->bs1;
  if (w->use_coarse) {
    S.nagg = s->nagg;
    S.fagg = s->fagg;
    S.zT = prec == CR_FP32_IR ? (const void*)s->zy32 : (const void*)s->zy;
    S.Pr = w->Pr;
    S.ablk = w->ablk;
    S.bfa = w->bfa;
    S.bla = w->bla;
    S.Einv = s->Einv;
    S.cvec = w->cvec;
    S.mu = w->mu;
    S.M2 = w->M2;
  }
  S.G = prec == CR_FP32_IR ? (const void*)s->G32 : (const void*)s->G64;
  S.cols = s->cols;
  S.G64 = s->G64;
  S.y = s->y;
  S.bs = s->bs;
  S.dsq = s->dsq;
  S.x = w->vec[V_X];
  S.r = w->vec[V_R0];
  S.p = w->vec[V_P];
  S.q = w->vec[V_W0];
  S.Pa = w->part3[0];
  S.Pb = w->part3[1];
  S.Pc = w->part3[2];
  S.st = st;
  S.F = prec == CR_FP32_IR ? (const void*)s->efo32 : (const void*)s->efo64;
  S.F64 = s->efo64;
  S.egat = s->egat;
  S.fel = s->fel;
  S.floc = s->floc;
  S.ne = s->ne;
  return S;
}

// Operator form of a solve: the element factors (built for transient Stokes)
// serve CG; the assembled rows serve BiCGStab and explicit requests.
cr_status resolve_op(const cr_system* s, const cr_solve_opts* o, int& op) {
  // the element form carries K0's divergence row too (gauge-shifted system;
  // with boundary data K0's row takes up the net flux, so that the system
  // stays consistent)
  const bool have = s->efo64 != nullptr && o->method == CR_PCG;
  switch (o->operator_form) {
    case CR_OP_AUTO:
      op = have ? 1 : 0;
      return CR_OK;
    case CR_OP_ASSEMBLED:
      op = 0;
      return CR_OK;
    case CR_OP_ELEMENT:
      if (!have) {
        set_error("the element-factor operator needs CG on a transient Stokes system");
        return CR_E_INVAL;
      }
      op = 1;
      return CR_OK;
    default:
      set_error("unknown operator_form %d", o->operator_form);
      return CR_E_INVAL;
  }
}

template <class F>
void dispatch(int d, int prec, F&& f) {
  const bool f32 = prec == CR_FP32_IR;
  if (d == 2) {
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

// dispatch with the operator form as a third compile-time argument
template <class F>
void dispatch_op(int d, int prec, int op, F&& f) {
  dispatch(d, prec, [&](auto dc, auto tc) {
    if (op)
      f(dc, tc, std::integral_constant<int, 1>());
    else
      f(dc, tc, std::integral_constant<int, 0>());
  });
}

struct Launch {
  cr_system* s;
  KWs* w;
  int prec;    // CR_FP64 or CR_FP32_IR
  int method;  // CR_PCG, CR_BICGSTAB or CR_BICGSTAB2
  KState* st;  // device state of this solve
  int op;      // operator form (1: element factors)
};

void enqueue_iters(const Launch& L, hipStream_t stream, int npairs) {
  KWs* w = L.w;
  const Part P = w->part;
  const dim3 grid(P.nblk), blk(NT);
  dispatch_op(L.s->d, L.prec, L.op, [&](auto dc, auto tc, auto oc) {
    constexpr int D = decltype(dc)::value;
    constexpr int OP = decltype(oc)::value;
    using T = decltype(tc);
    auto V = [&](int i) { return (T*)w->vec[i]; };
    const T* G = std::is_same<T, float>::value ? (const T*)L.s->G32 : (const T*)L.s->G64;
    const CgSys S = make_sys(L.s, w, L.prec, L.st);
    for (int k = 0; k < npairs; ++k)
      for (int par = 0; par < 2; ++par) {
        if constexpr (OP == 1) {
          hipLaunchKernelGGL((k_ec1<D, T>), dim3(w->epart.nblk), blk, 0, stream, S, par);
          hipLaunchKernelGGL((k_ec2<D, T>), grid, blk, 0, stream, S, par);
          if (S.nagg > 0) hipLaunchKernelGGL(k_coarse, dim3((S.nagg + 3) / 4), blk, 0, stream, S);
        } else if (L.method == CR_PCG) {
          hipLaunchKernelGGL((k_cg_spmv<D, T, 0>), grid, blk, 0, stream, S, par);
          hipLaunchKernelGGL((k_cg_update<D, T>), grid, blk, 0, stream, S, par);
        } else if (L.method == CR_BICGSTAB2) {
          const B2Vecs BV{V(V_X), V(V_R0), V(V_R1), V(V_P), V(V_W1), V(V_W0), V(V_U2), V(V_S0), V(V_S1), V(V_V2),
                          V(V_T), V(V_RHAT)};
          hipLaunchKernelGGL((k_b2_1<D, T>), grid, blk, 0, stream, P, G, L.s->cols, BV, w->part3[0], w->part3[1],
                             L.st, par);
          hipLaunchKernelGGL((k_b2_2<D, T>), grid, blk, 0, stream, P, G, L.s->cols, BV, w->part3[1], w->part3[2],
                             L.st, par);
          hipLaunchKernelGGL((k_b2_3<D, T>), grid, blk, 0, stream, P, G, L.s->cols, BV, w->part3[2], w->part3[1],
                             L.st, par);
          hipLaunchKernelGGL((k_b2_4<D, T>), grid, blk, 0, stream, P, G, L.s->cols, BV, w->part3[1], w->part3[2],
                             L.st, par);
          hipLaunchKernelGGL((k_b2_5<D, T>), grid, blk, 0, stream, P, BV, w->part3[2], w->part3[0], L.st, par);
        } else {
          T* pv[2] = {V(V_R1), V(V_W1)};  // p buffers
          T* vv[2] = {V(V_S0), V(V_S1)};  // v buffers
          hipLaunchKernelGGL((k_bicg_1<D, T>), grid, blk, 0, stream, P, G, L.s->cols, V(V_R0), V(V_RHAT),
                             pv[par ^ 1], vv[par ^ 1], pv[par], vv[par], w->part3[0], w->part3[1], L.st, par);
          hipLaunchKernelGGL((k_bicg_2<D, T>), grid, blk, 0, stream, P, G, L.s->cols, V(V_R0), vv[par], V(V_W0),
                             V(V_T), w->part3[1], w->part3[2], L.st, par);
          hipLaunchKernelGGL((k_bicg_3<D, T>), grid, blk, 0, stream, P, V(V_X), V(V_R0), V(V_RHAT), pv[par],
                             V(V_W0), V(V_T), w->part3[2], w->part3[0], L.st, par);
        }
      }
  });
}

// residual (replacement) kernel for one system
void enqueue_residual(cr_system* s, KWs* w, int prec, int method, int op, KState* st, int mode,
                      hipStream_t stream) {
  const Part P = w->part;
  dispatch_op(s->d, prec, op, [&](auto dc, auto tc, auto oc) {
    constexpr int D = decltype(dc)::value;
    constexpr int OP = decltype(oc)::value;
    using T = decltype(tc);
    const CgSys S = make_sys(s, w, prec, st);
    hipLaunchKernelGGL((k_ir_residual<D, T, OP>), dim3(P.nblk), dim3(NT), 0, stream, S, (T*)w->vec[V_RHAT], mode,
                       method != CR_PCG ? 1 : 0);
    if (OP == 1 && S.nagg > 0) hipLaunchKernelGGL(k_coarse, dim3((S.nagg + 3) / 4), dim3(NT), 0, stream, S);
  });
}

void enqueue_update(cr_system* s, KWs* w, int prec, KState* st, hipStream_t stream) {
  const Part P = w->part;
  dispatch(s->d, prec, [&](auto dc, auto tc) {
    constexpr int D = decltype(dc)::value;
    using T = decltype(tc);
    hipLaunchKernelGGL((k_ir_update<D, T>), dim3(P.nblk), dim3(NT), 0, stream, make_sys(s, w, prec, st));
  });
}

cr_status get_graph(const Launch& L, int npairs, hipGraphExec_t& out) {
  KWs* w = L.w;
  const int pi = L.prec == CR_FP32_IR ? 1 : 0, mi = L.method, oi = L.op ? (L.w->use_coarse ? 2 : 1) : 0;
  hipGraphExec_t& ex = w->exec[pi][mi][oi];
  int& exm = w->exec_m[pi][mi][oi];
  if (ex && exm == npairs) {
    out = ex;
    return CR_OK;
  }
  if (ex) {
    (void)hipGraphExecDestroy(ex);
    ex = nullptr;
  }
  hipGraph_t g = nullptr;
  cr_status st = check_hip(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st != CR_OK) return st;
  enqueue_iters(L, w->cap, npairs);
  hipError_t le = hipGetLastError();
  st = check_hip(hipStreamEndCapture(w->cap, &g), "end capture");
  if (st != CR_OK) return st;
  st = check_hip(le, "captured launch");
  if (st != CR_OK) {
    (void)hipGraphDestroy(g);
    return st;
  }
  st = check_hip(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  if (st != CR_OK) return st;
  exm = npairs;
  out = ex;
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
  // one iteration block, then the copy of its state and the event the host polls
  auto launch = [&](int slot) {
    hipError_t e = hipSuccess;
    if (graph)
      e = hipGraphLaunch(exec, s->stream);
    else
      enqueue_iters(L, s->stream, npairs);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&w->hst[slot], L.st, sizeof(KState), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipEventRecord(w->ev[slot], s->stream);
    return check_hip(e, "inner launch");
  };
  int issued = 0, slot = 0;
  cr_status st = CR_OK;
  for (int k = 0; k < 2 && issued < max_blocks && st == CR_OK; ++k) st = launch(issued++ & 1);
  if (st != CR_OK) return st;
  for (;;) {
    st = check_hip(hipEventSynchronize(w->ev[slot]), "inner poll");
    if (st != CR_OK) return st;
    if (w->hst[slot].done || issued >= max_blocks) break;
    st = launch(slot);
    if (st != CR_OK) return st;
    ++issued;
    slot ^= 1;
  }
  st = check_hip(hipMemcpyAsync(&w->hst[2], L.st, sizeof(KState), hipMemcpyDeviceToHost, s->stream), "state copy");
  if (st != CR_OK) return st;
  st = check_hip(hipStreamSynchronize(s->stream), "inner sync");
  if (st != CR_OK) return st;
  out = w->hst[2];
  return CR_OK;
}

// parameters of one solve, written into its device state
void fill_params(KState& h, const cr_solve_opts* o, double& tol_out) {
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  // reduction of the recursive residual between residual replacements.  CG
  // takes them in FP64 too: near the attainable accuracy the recursive
  // residual of a long FP64 run drifts from the true one, and without
  // replacements a tight tolerance costs many restarts (64^3 x 6 tetrahedra
  // to 1e-13: 22,062 iterations without, 2,074 with).
  double rep = o->inner_tol;
  if (!(rep > 0)) rep = (o->precision == CR_FP32_IR || o->method == CR_PCG) ? 0.1 : 0.0;
  h.rep_tol2 = rep * rep;
  h.tol2 = tol * tol;
  h.maxit = o->maxit > 0 ? o->maxit : 1000000;
  // iterations between replacements are capped for FP32 iterations and for
  // CG (a stop that restarts the direction from the FP64 residual)
  h.interval_cap = 4000;
  tol_out = tol;
}

cr_status write_params(KState* dst, KState* staging, const cr_solve_opts* o, hipStream_t stream) {
  double tol;
  fill_params(*staging, o, tol);
  const size_t off = offsetof(KState, rep_tol2);
  cr_status st = check_hip(hipMemcpyAsync((char*)dst + off, (char*)staging + off, sizeof(KState) - off,
                                          hipMemcpyHostToDevice, stream),
                           "solver parameters");
  if (st != CR_OK) return st;
  return check_hip(hipStreamSynchronize(stream), "solver parameters");
}

// Host side of one solve: reacts to each stop of the device iteration
// (replacement, restart, FP32 stall -> FP64, limits) by enqueueing the FP64
// correction and residual kernels.  Shared by single and batched solves, so a
// system takes the same decisions at the same iterations in both.
struct Ctl {
  int prec = CR_FP64;
  int method = CR_PCG;
  int maxit = 0, max_rep = 400;
  int reps = 1, restarts = 0, reason = 0, iters = 0, fp32_iters = 0;
  double rel = -1.0, prev_true = -1.0;
  // FP64 iterations: smallest true residual seen at a replacement, and the
  // replacements since it last fell by half (stagnation at the attainable
  // accuracy ends the solve after STAGNANT of them)
  double best_true = -1.0;
  int stagnant = 0;
  static constexpr int STAGNANT = 8;
  bool fell_back = false, final_eval = false, stagnated = false;

  void init(const cr_solve_opts* o) {
    prec = o->precision;
    method = o->method;
    maxit = o->maxit > 0 ? o->maxit : 1000000;
    max_rep = o->max_outer > 0 ? o->max_outer : 400;
  }

  // returns true when the solve is finished (reason set)
  template <class Upd, class Res>
  bool step(const KState& ks, Upd&& update, Res&& residual) {
    const bool f32 = prec == CR_FP32_IR;
    if (f32) fp32_iters = ks.nrun;
    iters = ks.nrun;
    rel = ks.snorm2 > 0 ? std::sqrt(ks.tres2 / ks.snorm2) : std::sqrt(ks.tres2);
    if (ks.done == CONVERGED) {
      reason = 1;
      return true;
    }
    if (ks.done == NONFINITE && !f32) {
      reason = NONFINITE;
      return true;
    }
    if ((ks.done == BREAKDOWN || ks.done == DIVERGED) && !f32 && (final_eval || restarts >= 8)) {
      reason = BREAKDOWN;
      return true;
    }
    if (final_eval) {
      reason = 3;
      return true;
    }
    bool stall = false;
    if (f32) {
      stall = ks.done == STALL || ks.done == NONFINITE || ((ks.done == BREAKDOWN || ks.done == DIVERGED) && restarts >= 2) ||
              (ks.done == REPLACE && prev_true > 0.0 && ks.tres2 > 0.25 * prev_true);
      if (ks.done == REPLACE) prev_true = ks.tres2;
    }
    // fold the correction into y (unless it holds non-finite values) and
    // recompute the residual in FP64.  When the FP32 iterations of a
    // non-symmetric method stall, their last correction is discarded: without
    // CG's monotone error reduction it may have grown.
    if (ks.done != NONFINITE && ks.done != DIVERGED && !(stall && method != CR_PCG)) update(prec);
    if (stall) {
      prec = CR_FP64;
      fell_back = true;
      residual(prec, 2);
    } else if (ks.done == BREAKDOWN || ks.done == DIVERGED) {
      // restart from the FP64 residual with a fresh direction; a diverged
      // correction was discarded above
      residual(prec, 2);
      ++restarts;
    } else {
      residual(prec, ks.done == STALL ? 2 : 1);
    }
    ++reps;
    if (!f32 && (ks.done == REPLACE || ks.done == STALL)) {
      if (best_true < 0.0 || ks.tres2 < 0.25 * best_true) {
        best_true = ks.tres2;
        stagnant = 0;
      } else if (++stagnant >= STAGNANT) {
        stagnated = true;
      }
    }
    if ((!stall && ks.done != REPLACE && ks.done != STALL && ks.done != BREAKDOWN && ks.done != DIVERGED) ||
        reps > max_rep || stagnated ||
        iters >= maxit)
      final_eval = true;
    return false;
  }

  cr_status status() const {
    if (reason == 1) return CR_OK;
    if (reason == BREAKDOWN) {
      set_error("Krylov breakdown after %d iterations", iters);
      return CR_E_BREAKDOWN;
    }
    if (reason == NONFINITE) {
      set_error("non-finite Krylov scalar after %d iterations", iters);
      return CR_E_NONFINITE;
    }
    if (stagnated)
      set_error("no convergence: the residual stagnated at %.3e (the attainable accuracy) after %d iterations",
                rel, iters);
    else
      set_error("no convergence: relative residual %.3e after %d iterations, %d residual evaluations", rel, iters,
                reps);
    return CR_E_NOCONV;
  }

  void fill(cr_solve_info* info, double ms, int requested_prec) const {
    if (!info) return;
    info->iters = iters;
    info->outer_iters = reps;
    info->rel_residual = rel;
    info->t_solve_ms = ms;
    info->reason = reason;
    info->fp32_iters = requested_prec == CR_FP32_IR ? fp32_iters : 0;
    info->fp64_fallback = fell_back ? 1 : 0;
  }
};

}  // namespace

namespace {

template <int D, typename T>
void enqueue_minres(cr_system* s, KWs* w, const CgSys& S, int k0, int niter) {
  const dim3 grid(S.P.nblk), blk(NT);
  T* R[3] = {(T*)w->vec[V_R0], (T*)w->vec[V_R1], (T*)w->vec[V_W0]};
  T* W[3] = {(T*)w->vec[V_W1], (T*)w->vec[V_S0], (T*)w->vec[V_S1]};
  T* v = (T*)w->vec[V_P];
  for (int k = k0; k < k0 + niter; ++k) {
    const int q = k & 1;
    T* r1 = R[k % 3];
    T* r2 = R[(k + 1) % 3];
    T* y = R[(k + 2) % 3];
    hipLaunchKernelGGL((k_hm_a<D, T>), grid, blk, 0, s->stream, S, r1, r2, v, y, w->mst, q);
    hipLaunchKernelGGL((k_hm_b<D, T>), grid, blk, 0, s->stream, S, r2, y, w->mst, q);
    hipLaunchKernelGGL((k_hm_c<D, T>), grid, blk, 0, s->stream, S, v, W[k % 3], W[(k + 1) % 3], W[(k + 2) % 3],
                       w->mst, q);
  }
}

// MINRES with FP64 refinement passes (see the kernels above).  A pass in FP32
// that does not reduce the true residual by half switches the remaining passes
// to FP64.
cr_status run_minres(cr_system* s, KWs* w, const cr_solve_opts* o, cr_solve_info* info,
                     std::chrono::steady_clock::time_point t_start) {
  cr_status st = ensure_assembled(s);  // MINRES applies the assembled rows
  if (st != CR_OK) return st;
  if (!w->mst) {
    w->mst = (MState*)dev_alloc(s, sizeof(MState));
    if (!w->mst) return CR_E_NOMEM;
    st = check_hip(hipHostMalloc((void**)&w->mhst, sizeof(MState), hipHostMallocDefault), "pinned MINRES state");
    if (st != CR_OK) return st;
  }
  const double tol = o->tol > 0 ? o->tol : 1e-10;
  const int maxit = o->maxit > 0 ? o->maxit : 1000000;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 200;
  const int blk = std::max(6, ((o->check_every > 0 ? o->check_every : 48) + 5) / 6 * 6);
  int prec = o->precision;
  const double rep_f32 = o->inner_tol > 0 ? o->inner_tol : 1e-5;
  int total = 0, fp32_total = 0, outer = 0, reason = 0;
  double rel = -1.0, prev_t2 = -1.0;
  bool fell_back = false;
  if (o->precond < CR_PC_DEFAULT || o->precond > CR_PC_JACOBI) {
    set_error("MINRES takes CR_PC_DEFAULT or CR_PC_JACOBI (Jacobi scaling), not %d", o->precond);
    return CR_E_INVAL;
  }
  if (o->w0) {
    st = enqueue_import_w(s, o->w0);
    if (st != CR_OK) return st;
  } else if (!o->warm_start || !s->has_solution) {
    st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * s->d, s->stream), "zero W");
    if (st != CR_OK) return st;
  }
  for (;;) {
    const bool last = outer >= max_outer || total >= maxit;
    MState* h = w->mhst;
    h->tol2 = tol * tol;
    h->rep = prec == CR_FP32_IR ? rep_f32 : 0.0;
    // an FP32 pass is capped: its recurrences lose accuracy before a long pass
    // ends, and the next pass restarts from the FP64 residual
    const int pass_cap = prec == CR_FP32_IR ? 25000 : maxit;
    h->maxit = last ? 0 : std::min(maxit - total, pass_cap);
    const size_t off = offsetof(MState, tol2);
    st = check_hip(hipMemcpyAsync((char*)w->mst + off, (char*)h + off, sizeof(MState) - off, hipMemcpyHostToDevice,
                                  s->stream), "MINRES parameters");
    if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "MINRES parameters");
    if (st != CR_OK) return st;
    ++outer;
    MState ks{};
    dispatch(s->d, prec, [&](auto dc, auto tc) {
      constexpr int D = decltype(dc)::value;
      using T = decltype(tc);
      const CgSys S = make_sys(s, w, prec, w->st);
      hipLaunchKernelGGL((k_hm_init<D, T>), dim3(S.P.nblk), dim3(NT), 0, s->stream, S, (T*)w->vec[V_R0],
                         (T*)w->vec[V_R1], (T*)w->vec[V_W1], (T*)w->vec[V_S0], w->mst);
      int issued = 0;
      const int max_blocks = h->maxit / blk + 2;
      for (;;) {
        enqueue_minres<D, T>(s, w, S, issued * blk, blk);
        ++issued;
        st = check_hip(hipGetLastError(), "MINRES launch");
        if (st == CR_OK)
          st = check_hip(hipMemcpyAsync(w->mhst, w->mst, sizeof(MState), hipMemcpyDeviceToHost, s->stream),
                         "MINRES state copy");
        if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "MINRES poll");
        if (st != CR_OK) break;
        ks = *w->mhst;
        if (ks.done || issued >= max_blocks) break;
      }
      if (st == CR_OK && ks.done != 2 && ks.done != 5)
        hipLaunchKernelGGL((k_ir_update<D, T>), dim3(S.P.nblk), dim3(NT), 0, s->stream, S);
    });
    if (st != CR_OK) return st;
    st = check_hip(hipGetLastError(), "MINRES launch");
    if (st != CR_OK) return st;
    total += ks.iters;
    if (prec == CR_FP32_IR) fp32_total += ks.iters;
    rel = ks.bnorm2 > 0 ? std::sqrt(ks.tres2 / ks.bnorm2) : std::sqrt(ks.tres2);
    if (ks.done == 2) {
      reason = 1;
      break;
    }
    if (ks.done == 4 || ks.done == 5) {
      reason = ks.done == 4 ? BREAKDOWN : NONFINITE;
      break;
    }
    if (last || (prec != CR_FP32_IR && ks.done == 3)) {
      reason = 3;
      break;
    }
    if (prec == CR_FP32_IR && prev_t2 > 0.0 && ks.tres2 > 0.25 * prev_t2) {
      prec = CR_FP64;
      fell_back = true;
    }
    prev_t2 = ks.tres2;
  }
  st = check_hip(hipStreamSynchronize(s->stream), "MINRES sync");
  if (st != CR_OK) return st;
  s->has_solution = true;
  if (info) {
    info->iters = total;
    info->outer_iters = outer;
    info->rel_residual = rel;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    info->reason = reason;
    info->fp32_iters = o->precision == CR_FP32_IR ? fp32_total : 0;
    info->fp64_fallback = fell_back ? 1 : 0;
  }
  if (reason == 1) return CR_OK;
  if (reason == BREAKDOWN) {
    set_error("MINRES breakdown after %d iterations", total);
    return CR_E_BREAKDOWN;
  }
  if (reason == NONFINITE) {
    set_error("non-finite MINRES scalar after %d iterations", total);
    return CR_E_NONFINITE;
  }
  set_error("MINRES: relative residual %.3e after %d iterations, %d passes", rel, total, outer);
  return CR_E_NOCONV;
}

}  // namespace

// Whether this solve adds the aggregate coarse correction (opts.precond).
cr_status pick_coarse(cr_system* s, KWs* w, const cr_solve_opts* o, int op) {
  if (o->precond < CR_PC_DEFAULT || o->precond > CR_PC_COARSE) {
    set_error("unknown precond %d", o->precond);
    return CR_E_INVAL;
  }
  w->use_coarse = op == 1 && o->precond != CR_PC_JACOBI && w->coarse_ok;
  if (o->precond == CR_PC_COARSE && !w->use_coarse) {
    set_error("CR_PC_COARSE: the coarse correction exists only for CG with the element form on a mesh with "
              "aggregates (transient Stokes, at least 512 elements in 2D, 1024 in 3D)");
    return CR_E_INVAL;
  }
  return CR_OK;
}

cr_status run_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info) {
  auto t_start = std::chrono::steady_clock::now();
  KWs* w = nullptr;
  cr_status st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  if (o->method == CR_MINRES) {
    if (o->operator_form == CR_OP_ELEMENT) {
      set_error("MINRES applies the assembled G");
      return CR_E_INVAL;
    }
    return run_minres(s, w, o, info, t_start);
  }
  int op = 0;
  st = resolve_op(s, o, op);
  if (st == CR_OK && op == 0) st = ensure_assembled(s);
  if (st != CR_OK) return st;
  st = pick_coarse(s, w, o, op);
  if (st != CR_OK) return st;
  Ctl c;
  c.init(o);
  const int blk = o->check_every > 0 ? o->check_every : 32;
  const int npairs = std::max(1, (blk + 1) / 2);
  const int per = 2 * npairs;
  const bool graph = o->use_graph != 0;
  if (o->w0) {
    st = enqueue_import_w(s, o->w0);
    if (st != CR_OK) return st;
  } else if (!o->warm_start || !s->has_solution) {
    st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * s->d, s->stream), "zero W");
    if (st != CR_OK) return st;
  }
  st = write_params(w->st, &w->hst[2], o, s->stream);
  if (st != CR_OK) return st;
  enqueue_residual(s, w, c.prec, c.method, op, w->st, 0, s->stream);
  auto upd = [&](int prec) { enqueue_update(s, w, prec, w->st, s->stream); };
  auto res = [&](int prec, int mode) { enqueue_residual(s, w, prec, c.method, op, w->st, mode, s->stream); };
  for (;;) {
    KState ks;
    Launch L{s, w, c.prec, c.method, w->st, op};
    st = run_inner(L, npairs, graph && !c.final_eval, c.final_eval ? 1 : c.maxit / per + 3, ks);
    if (st != CR_OK) return st;
    if (ks.done == RUNNING) ks.done = LIMIT;  // host cap reached
    if (c.step(ks, upd, res)) break;
  }
  if (op == 1) {
    st = enqueue_gauge_fix(s, s->stream);
    if (st != CR_OK) return st;
  }
  st = check_hip(hipStreamSynchronize(s->stream), "solve sync");
  if (st != CR_OK) return st;
  s->has_solution = true;
  c.fill(info, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count(),
         o->precision);
  return c.status();
}

// Times the dominant kernel (SpMV fused with the CG direction updates) on
// scratch vectors; its input r is never written, so every launch does
// identical work.
cr_status run_time_spmv(cr_system* s, int precision, int form, int reps, double* avg_ms, double* bytes) {
  KWs* w = nullptr;
  cr_status st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  cr_solve_opts o{};
  o.method = CR_PCG;
  o.operator_form = form;
  int op = 0;
  st = resolve_op(s, &o, op);
  if (st == CR_OK && op == 0) st = ensure_assembled(s);
  if (st != CR_OK) return st;
  w->use_coarse = op == 1 && w->coarse_ok;
  const int d = s->d;
  const size_t vb = sizeof(double) * (size_t)s->nf * d;
  const Part P = w->part;
  if (!w->tvec[0]) {
    for (auto& v : w->tvec) {
      v = dev_alloc(s, vb);
      if (!v) return CR_E_NOMEM;
    }
    for (auto& p : w->tpart) {
      p = (double*)dev_alloc(s, sizeof(double) * (size_t)std::max(P.nblk, w->epart.nblk) * NFIELD);
      if (!p) return CR_E_NOMEM;
    }
    if (s->efo64) {
      w->ttq = dev_alloc(s, sizeof(double) * (size_t)s->ne * (d + 1) * d);
      if (!w->ttq) return CR_E_NOMEM;
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
  ks.rr_rep = 1.0;  // no divergence stop: r.r has not grown since the last evaluation
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
  CgSys S = make_sys(s, w, precision, w->tst);
  S.x = w->tvec[V_X];
  S.r = w->tvec[V_R0];
  S.p = w->tvec[V_P];
  S.q = w->tvec[V_W0];
  S.Pa = w->tpart[0];
  S.Pb = w->tpart[1];
  S.p1 = w->tvec[V_W1];
  S.tq = w->ttq;
  const dim3 grid(op ? w->epart.nblk : P.nblk), blk(NT);
  auto launch = [&]() {
    dispatch_op(d, precision, op, [&](auto dc, auto tc, auto oc) {
      constexpr int D = decltype(dc)::value;
      constexpr int OP = decltype(oc)::value;
      using T = decltype(tc);
      if constexpr (OP == 1)
        hipLaunchKernelGGL((k_ec1<D, T>), grid, blk, 0, s->stream, S, 0);
      else
        hipLaunchKernelGGL((k_cg_spmv<D, T, 0>), grid, blk, 0, s->stream, S, 0);
    });
  };
  float ms = 0.f;
  if (op && w->use_coarse) {
    // With the coarse correction the element kernel is timed inside the real
    // iteration sequence (element kernel, face kernel, coarse solve) on the
    // scratch state, with start and stop events attached to each of its
    // launches (recorded at the dispatch's start and end).
    ks.rr_rep = 1e300;
    st = check_hip(hipMemcpyAsync(w->tst, &ks, sizeof ks, hipMemcpyHostToDevice, s->stream), "timing state");
    if (st != CR_OK) return st;
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto& e : ev)
      if (st == CR_OK) st = check_hip(hipEventCreate(&e), "timing events");
    dispatch(d, precision, [&](auto dc, auto tc) {
      constexpr int D = decltype(dc)::value;
      using T = decltype(tc);
      for (int k = -2; k < reps && st == CR_OK; ++k) {
        const int par = k & 1;
        if (k >= 0)
          hipExtLaunchKernelGGL((k_ec1<D, T>), grid, blk, 0, s->stream, ev[2 * k], ev[2 * k + 1], 0, S, par);
        else
          hipLaunchKernelGGL((k_ec1<D, T>), grid, blk, 0, s->stream, S, par);
        hipLaunchKernelGGL((k_ec2<D, T>), dim3(P.nblk), blk, 0, s->stream, S, par);
        hipLaunchKernelGGL(k_coarse, dim3((S.nagg + 3) / 4), blk, 0, s->stream, S);
      }
    });
    if (st == CR_OK) st = check_hip(hipGetLastError(), "timing launch");
    if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "timing");
    double tot = 0.0;
    for (int k = 0; k < reps && st == CR_OK; ++k) {
      float e = 0.f;
      st = check_hip(hipEventElapsedTime(&e, ev[2 * k], ev[2 * k + 1]), "timing events");
      tot += e;
    }
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (st != CR_OK) return st;
    ms = (float)tot;
  } else {
    launch();  // warm-up
    st = check_hip(hipEventRecord(w->t0, s->stream), "timing");
    for (int k = 0; k < reps && st == CR_OK; ++k) launch();
    if (st == CR_OK) st = check_hip(hipGetLastError(), "timing launch");
    if (st == CR_OK) st = check_hip(hipEventRecord(w->t1, s->stream), "timing");
    if (st == CR_OK) st = check_hip(hipEventSynchronize(w->t1), "timing");
    if (st == CR_OK) st = check_hip(hipEventElapsedTime(&ms, w->t0, w->t1), "timing events");
    if (st != CR_OK) return st;
  }
  if (avg_ms) *avg_ms = (double)ms / reps;
  if (bytes) {
    const double vsz = f32 ? 4.0 : 8.0;
    const double nf = (double)s->nf, ne = (double)s->ne;
    const int d1 = d + 1;
    if (op) {
      // element-centric kernel: element factors, gather indices and flags read
      // once; r and the previous p read once (gathered); the new p written
      // once by the owner elements (2D; in 3D the face kernel writes it);
      // w_K written once
      *bytes = ne * (d1 * (d1 + 1) / 2 + d1 * d) * vsz + ne * (d1 + 1) * 4.0 +
               nf * d * vsz * (ec2_stores_direction(d) ? 2 : 3) + ne * d1 * d * vsz;
      // with the coarse correction: the aggregate of each face and the column
      // of Z there, read by the elements on aggregate boundaries
      if (w->use_coarse) *bytes += (double)s->nbnd * d1 * (4.0 + d * vsz);
    } else {
      // values and column indices of G read once, the gathered input r read
      // once, p and q read and written
      *bytes = nf * (2 * d + 1) * d * d * vsz + nf * 2 * d * 4.0 + nf * d * vsz * (1 + 2 + 2);
    }
  }
  return CR_OK;
}

void free_krylov(cr_system* s) {
  KWs* w = (KWs*)s->kws;
  if (!w) return;
  for (auto& a : w->exec)
    for (auto& b : a)
      for (auto& e : b)
        if (e) (void)hipGraphExecDestroy(e);
  for (auto& e : w->ev)
    if (e) (void)hipEventDestroy(e);
  if (w->t0) (void)hipEventDestroy(w->t0);
  if (w->t1) (void)hipEventDestroy(w->t1);
  if (w->cap) (void)hipStreamDestroy(w->cap);
  if (w->hst) (void)hipHostFree(w->hst);
  if (w->mhst) (void)hipHostFree(w->mhst);
  delete w;
  s->kws = nullptr;
}

}  // namespace crh

// ---------------------------------------------------------------------------
// Batched solves: the CG iterations of many resident systems advance in
// shared launches (block-diagonal batch).  Each launch covers the row ranges of
// all active systems of one precision; every system keeps its own partial
// sums, scalars and stop flag, so its iterates are bitwise those of a single
// solve.  Systems join (cr_batch_add) and leave (when finished) between
// iteration blocks; replacements and restarts of one system are serviced with
// that system's own single-system kernels.
// ---------------------------------------------------------------------------
namespace crh {
namespace {

struct BEntry {
  cr_system* s = nullptr;
  KWs* w = nullptr;
  cr_solve_opts o{};
  Ctl c;
  int op = 0;
  bool active = false;
  std::chrono::steady_clock::time_point t0;
  cr_status status = CR_OK;
  cr_solve_info info{};
};

}  // namespace
}  // namespace crh

struct cr_batch {
  hipStream_t stream = nullptr;
  int max_sys = 0;
  int d = 0;
  int op = -1;  // operator form shared by all systems of the batch
  crh::KState* dst = nullptr;  // device [max_sys]
  crh::KState* hst = nullptr;  // pinned [max_sys]
  std::vector<crh::BEntry> e;
  std::deque<int> finished;
  crh::CgSys* dtab[2] = {};
  int* dmap[2] = {};   // face block -> table entry
  int* dmapE[2] = {};  // element block -> table entry
  int* dmapC[2] = {};  // coarse block -> table entry
  crh::CgSys* htab[2] = {};
  int* hmap[2] = {};
  int* hmapE[2] = {};
  int* hmapC[2] = {};
  int nblocks[2] = {};
  int nblocksE[2] = {};
  int nblocksC[2] = {};
  // the iteration block of an advance, captured once per launch shape (block
  // counts and iteration count) and replayed; membership changes that keep
  // the shape only rewrite the device tables the graph reads
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  int exec_key[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int64_t map_cap = 0;
  bool dirty = true;
};

namespace crh {
namespace {

cr_status batch_rebuild(cr_batch* b) {
  for (int pi = 0; pi < 2; ++pi) {
    const int prec = pi ? CR_FP32_IR : CR_FP64;
    int n = 0, blocks = 0, eblocks = 0, cblocks = 0;
    for (int k = 0; k < b->max_sys; ++k) {
      BEntry& en = b->e[k];
      if (!en.active || en.c.prec != prec) continue;
      CgSys S = make_sys(en.s, en.w, prec, b->dst + k);
      S.boff = blocks;
      S.boffE = eblocks;
      S.boffC = cblocks;
      const int nc = S.nagg > 0 ? (S.nagg + 3) / 4 : 0;
      if (blocks + S.P.nblk > b->map_cap || eblocks + S.PE.nblk > b->map_cap) {
        set_error("batch block table full");
        return CR_E_NOMEM;
      }
      for (int j = 0; j < S.P.nblk; ++j) b->hmap[pi][blocks + j] = n;
      for (int j = 0; j < S.PE.nblk; ++j) b->hmapE[pi][eblocks + j] = n;
      for (int j = 0; j < nc; ++j) b->hmapC[pi][cblocks + j] = n;
      blocks += S.P.nblk;
      eblocks += S.PE.nblk;
      cblocks += nc;
      b->htab[pi][n++] = S;
    }
    b->nblocks[pi] = blocks;
    b->nblocksE[pi] = eblocks;
    b->nblocksC[pi] = cblocks;
    if (n) {
      cr_status st = check_hip(
          hipMemcpyAsync(b->dtab[pi], b->htab[pi], sizeof(CgSys) * n, hipMemcpyHostToDevice, b->stream), "batch table");
      if (st == CR_OK)
        st = check_hip(hipMemcpyAsync(b->dmap[pi], b->hmap[pi], sizeof(int) * blocks, hipMemcpyHostToDevice, b->stream),
                       "batch map");
      if (st == CR_OK)
        st = check_hip(
            hipMemcpyAsync(b->dmapE[pi], b->hmapE[pi], sizeof(int) * eblocks, hipMemcpyHostToDevice, b->stream),
            "batch map");
      if (st == CR_OK && cblocks)
        st = check_hip(
            hipMemcpyAsync(b->dmapC[pi], b->hmapC[pi], sizeof(int) * cblocks, hipMemcpyHostToDevice, b->stream),
            "batch map");
      if (st != CR_OK) return st;
    }
  }
  b->dirty = false;
  return CR_OK;
}

}  // namespace
}  // namespace crh

using namespace crh;

extern "C" {

cr_status cr_batch_create(void* hip_stream, int32_t max_systems, cr_batch** out) {
  clear_error();
  if (!out || max_systems < 1 || max_systems > 4096) {
    set_error("cr_batch_create: need an output pointer and 1 <= max_systems <= 4096");
    return CR_E_INVAL;
  }
  *out = nullptr;
  cr_batch* b = new cr_batch();
  b->stream = (hipStream_t)hip_stream;
  b->max_sys = max_systems;
  b->e.resize(max_systems);
  b->map_cap = (int64_t)max_systems * max_blocks_cfg() + 8;
  cr_status st = check_hip(hipMalloc((void**)&b->dst, sizeof(KState) * max_systems), "batch state");
  if (st == CR_OK) st = check_hip(hipHostMalloc((void**)&b->hst, sizeof(KState) * max_systems, hipHostMallocDefault), "batch state");
  for (int pi = 0; pi < 2 && st == CR_OK; ++pi) {
    st = check_hip(hipMalloc((void**)&b->dtab[pi], sizeof(CgSys) * max_systems), "batch table");
    if (st == CR_OK) st = check_hip(hipMalloc((void**)&b->dmap[pi], sizeof(int) * b->map_cap), "batch map");
    if (st == CR_OK) st = check_hip(hipMalloc((void**)&b->dmapE[pi], sizeof(int) * b->map_cap), "batch map");
    if (st == CR_OK) st = check_hip(hipMalloc((void**)&b->dmapC[pi], sizeof(int) * b->map_cap), "batch map");
    if (st == CR_OK) st = check_hip(hipHostMalloc((void**)&b->htab[pi], sizeof(CgSys) * max_systems, hipHostMallocDefault), "batch table");
    if (st == CR_OK) st = check_hip(hipHostMalloc((void**)&b->hmap[pi], sizeof(int) * b->map_cap, hipHostMallocDefault), "batch map");
    if (st == CR_OK) st = check_hip(hipHostMalloc((void**)&b->hmapE[pi], sizeof(int) * b->map_cap, hipHostMallocDefault), "batch map");
    if (st == CR_OK) st = check_hip(hipHostMalloc((void**)&b->hmapC[pi], sizeof(int) * b->map_cap, hipHostMallocDefault), "batch map");
  }
  if (st != CR_OK) {
    cr_batch_destroy(b);
    return st;
  }
  *out = b;
  return CR_OK;
}

cr_status cr_batch_add(cr_batch* b, cr_system* s, const cr_solve_opts* o) {
  clear_error();
  if (!b || !s || !o) {
    set_error("NULL argument");
    return CR_E_INVAL;
  }
  if (!s->eliminated || s->stream != b->stream) {
    set_error("cr_batch_add needs an eliminated system on the batch's stream");
    return CR_E_INVAL;
  }
  if (o->method != CR_PCG || !(s->params.mu > 0.0 && s->params.problem == CR_STOKES)) {
    set_error("batched solves run CG on transient Stokes systems");
    return CR_E_INVAL;
  }
  if (o->precision != CR_FP64 && o->precision != CR_FP32_IR) {
    set_error("unknown precision %d", o->precision);
    return CR_E_INVAL;
  }
  if (b->d && s->d != b->d) {
    set_error("all systems of a batch have the same dimension");
    return CR_E_INVAL;
  }
  for (const BEntry& en : b->e)
    if (en.active && en.s == s) {
      set_error("system already in the batch");
      return CR_E_INVAL;
    }
  int k = -1;
  for (int i = 0; i < b->max_sys; ++i)
    if (!b->e[i].active && !b->e[i].s) {
      k = i;
      break;
    }
  if (k < 0) {
    set_error("batch full (%d systems)", b->max_sys);
    return CR_E_NOMEM;
  }
  int op = 0;
  cr_status st = resolve_op(s, o, op);
  if (st == CR_OK && op == 0) st = ensure_assembled(s);
  if (st != CR_OK) return st;
  int n_act = 0;
  for (const BEntry& en : b->e) n_act += en.active ? 1 : 0;
  if (n_act && b->op >= 0 && op != b->op) {
    set_error("all systems of a batch use the same operator form");
    return CR_E_INVAL;
  }
  KWs* w = nullptr;
  st = ensure_ws(s, w);
  if (st != CR_OK) return st;
  BEntry& en = b->e[k];
  en = BEntry();
  en.s = s;
  en.w = w;
  en.o = *o;
  en.c.init(o);
  en.op = op;
  st = pick_coarse(s, w, o, op);
  if (st != CR_OK) return st;
  en.t0 = std::chrono::steady_clock::now();
  if (!o->warm_start || !s->has_solution) {
    st = check_hip(hipMemsetAsync(s->y, 0, sizeof(double) * s->nf * s->d, b->stream), "zero W");
    if (st != CR_OK) return st;
  }
  st = write_params(b->dst + k, b->hst + k, o, b->stream);
  if (st != CR_OK) return st;
  enqueue_residual(s, w, en.c.prec, CR_PCG, op, b->dst + k, 0, b->stream);
  st = check_hip(hipGetLastError(), "batch add");
  if (st != CR_OK) return st;
  en.active = true;
  b->d = s->d;
  b->op = op;
  b->dirty = true;
  return CR_OK;
}

cr_status cr_batch_advance(cr_batch* b, int32_t n_iters, int32_t* n_finished) {
  clear_error();
  if (!b || n_iters < 1) {
    set_error("cr_batch_advance: NULL batch or n_iters < 1");
    return CR_E_INVAL;
  }
  cr_status st = CR_OK;
  if (b->dirty) st = batch_rebuild(b);
  if (st != CR_OK) return st;
  const int npairs = (n_iters + 1) / 2;
  bool any = false;
  for (int pi = 0; pi < 2; ++pi) any = any || b->nblocks[pi] > 0;
  auto enqueue = [&](hipStream_t stream) {
    for (int k = 0; k < npairs; ++k)
      for (int par = 0; par < 2; ++par)
        for (int pi = 0; pi < 2; ++pi) {
          if (!b->nblocks[pi]) continue;
          dispatch_op(b->d, pi ? CR_FP32_IR : CR_FP64, b->op, [&](auto dc, auto tc, auto oc) {
            constexpr int D = decltype(dc)::value;
            constexpr int OP = decltype(oc)::value;
            using T = decltype(tc);
            if constexpr (OP == 1) {
              hipLaunchKernelGGL((k_ec1_b<D, T>), dim3(b->nblocksE[pi]), dim3(NT), 0, stream, b->dtab[pi],
                                 b->dmapE[pi], par);
              hipLaunchKernelGGL((k_ec2_b<D, T>), dim3(b->nblocks[pi]), dim3(NT), 0, stream, b->dtab[pi],
                                 b->dmap[pi], par);
              if (b->nblocksC[pi])
                hipLaunchKernelGGL(k_coarse_b, dim3(b->nblocksC[pi]), dim3(NT), 0, stream, b->dtab[pi], b->dmapC[pi]);
            } else {
              hipLaunchKernelGGL((k_cg_spmv_b<D, T, 0>), dim3(b->nblocks[pi]), dim3(NT), 0, stream, b->dtab[pi],
                                 b->dmap[pi], par);
              hipLaunchKernelGGL((k_cg_update_b<D, T>), dim3(b->nblocks[pi]), dim3(NT), 0, stream, b->dtab[pi],
                                 b->dmap[pi], par);
            }
          });
        }
  };
  if (any) {
    const int key[8] = {b->nblocks[0], b->nblocks[1], b->nblocksE[0], b->nblocksE[1],
                        b->nblocksC[0], b->nblocksC[1], npairs, b->op};
    if (!b->exec || !std::equal(key, key + 8, b->exec_key)) {
      if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
      }
      if (!b->cap) st = check_hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "batch capture stream");
      hipGraph_t g = nullptr;
      if (st == CR_OK) st = check_hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "batch capture");
      if (st == CR_OK) {
        enqueue(b->cap);
        const hipError_t le = hipGetLastError();
        st = check_hip(hipStreamEndCapture(b->cap, &g), "batch capture");
        if (st == CR_OK) st = check_hip(le, "batch captured launch");
        if (st == CR_OK) st = check_hip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "batch graph");
        if (g) (void)hipGraphDestroy(g);
      }
      if (st != CR_OK) return st;
      std::copy(key, key + 8, b->exec_key);
    }
    st = check_hip(hipGraphLaunch(b->exec, b->stream), "batch graph launch");
    if (st != CR_OK) return st;
  }
  st = check_hip(hipMemcpyAsync(b->hst, b->dst, sizeof(KState) * b->max_sys, hipMemcpyDeviceToHost, b->stream),
                 "batch state");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(b->stream), "batch advance");
  if (st != CR_OK) return st;
  int nfin = 0;
  for (int k = 0; k < b->max_sys; ++k) {
    BEntry& en = b->e[k];
    if (!en.active) continue;
    const KState ks = b->hst[k];
    if (ks.done == RUNNING) continue;
    const int prec0 = en.c.prec;
    auto upd = [&](int prec) { enqueue_update(en.s, en.w, prec, b->dst + k, b->stream); };
    auto res = [&](int prec, int mode) {
      enqueue_residual(en.s, en.w, prec, CR_PCG, en.op, b->dst + k, mode, b->stream);
    };
    if (en.c.step(ks, upd, res)) {
      if (en.op == 1) {
        st = enqueue_gauge_fix(en.s, b->stream);
        if (st != CR_OK) return st;
      }
      en.active = false;
      en.s->has_solution = true;
      en.c.fill(&en.info,
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - en.t0).count(),
                en.o.precision);
      en.status = en.c.status();
      b->finished.push_back(k);
      b->dirty = true;
      ++nfin;
    } else if (en.c.prec != prec0) {
      b->dirty = true;
    }
  }
  st = check_hip(hipGetLastError(), "batch service");
  if (n_finished) *n_finished = nfin;
  return st;
}

cr_status cr_batch_pop(cr_batch* b, cr_system** sys, cr_solve_info* info, int32_t* status) {
  clear_error();
  if (!b || !sys) {
    set_error("NULL argument");
    return CR_E_INVAL;
  }
  *sys = nullptr;
  if (b->finished.empty()) return CR_OK;
  const int k = b->finished.front();
  b->finished.pop_front();
  BEntry& en = b->e[k];
  *sys = en.s;
  if (info) *info = en.info;
  if (status) *status = en.status;
  en = BEntry();
  return CR_OK;
}

cr_status cr_batch_count(const cr_batch* b, int32_t* n_active, int32_t* n_finished) {
  clear_error();
  if (!b) {
    set_error("NULL batch");
    return CR_E_INVAL;
  }
  int a = 0;
  for (const BEntry& en : b->e) a += en.active ? 1 : 0;
  if (n_active) *n_active = a;
  if (n_finished) *n_finished = (int32_t)b->finished.size();
  return CR_OK;
}

void cr_batch_destroy(cr_batch* b) {
  if (!b) return;
  if (b->stream || b->dst) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dst) (void)hipFree(b->dst);
  if (b->hst) (void)hipHostFree(b->hst);
  for (int pi = 0; pi < 2; ++pi) {
    if (b->dtab[pi]) (void)hipFree(b->dtab[pi]);
    if (b->dmap[pi]) (void)hipFree(b->dmap[pi]);
    if (b->dmapE[pi]) (void)hipFree(b->dmapE[pi]);
    if (b->dmapC[pi]) (void)hipFree(b->dmapC[pi]);
    if (b->htab[pi]) (void)hipHostFree(b->htab[pi]);
    if (b->hmap[pi]) (void)hipHostFree(b->hmap[pi]);
    if (b->hmapE[pi]) (void)hipHostFree(b->hmapE[pi]);
    if (b->hmapC[pi]) (void)hipHostFree(b->hmapC[pi]);
  }
  delete b;
}

}  // extern "C"
