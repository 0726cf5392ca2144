// Internal declarations of the crhyb library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/crhyb.h"

namespace crh {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

// ---------------------------------------------------------------------------
// host topology (step a0)
// ---------------------------------------------------------------------------
struct Topology {
  int d = 0;
  int64_t ne = 0, nv = 0, nf = 0;
  // caller element order / canonical face order
  std::vector<int32_t> elem_face;      // [ne][d+1] canonical interior face of local face j, -1 exterior
  std::vector<int32_t> face_vertices;  // [nf][d] sorted vertex ids
  std::vector<int32_t> face_elem;      // [nf][2] caller element ids, K < L
  std::vector<int8_t> face_loc;        // [nf][2] local face index in K and in L
  std::vector<uint8_t> m1;             // [ne] element partition M1 (mu == 0 only)
  // exterior faces (one element), lexicographic in their sorted vertex ids
  int64_t nbf = 0;
  std::vector<int32_t> bface_vertices; // [nbf][d]
  std::vector<int32_t> elem_bface;     // [ne][d+1] exterior face of local face j, -1 interior
  // renumbering
  std::vector<int32_t> face_perm;      // canonical -> internal
  std::vector<int32_t> face_iperm;     // internal -> canonical
  std::vector<int32_t> elem_perm;      // caller -> internal
  std::vector<int32_t> elem_iperm;     // internal -> caller
  int64_t bw_internal = 0, bw_canonical = 0;
  // aggregates of elements for the coarse correction (0: none); face_agg is in
  // internal face order, and faces of one aggregate are contiguous there
  int32_t nagg = 0;
  std::vector<int32_t> face_agg;
};

// Returns CR_OK or an error (message set).  need_m1: compute the M1/M2 split.
// aggregate: group faces by element aggregates (the coarse correction of CG on
// transient Stokes); other problems keep the plain RCM order.
cr_status build_topology(const cr_mesh_desc* mesh, int renumber, bool need_m1, bool aggregate, Topology& t);

// element flag bits (device eflags)
constexpr uint32_t F_INTERIOR0 = 1u;        // bit j: local face j interior
constexpr uint32_t F_NEG0 = 1u << 8;        // bit 8+j: C_K = -1 on local face j
constexpr uint32_t F_K0 = 1u << 16;         // pinned pressure element
constexpr uint32_t F_M1 = 1u << 17;         // element in M1 (E_K = -lambda I)
constexpr uint32_t F_AGGB = 1u << 18;       // interior faces in more than one aggregate

constexpr int NT = 256;                     // threads per block of the row kernels
constexpr int MAX_AGG = 512;                // most aggregates of the coarse correction

}  // namespace crh

// ---------------------------------------------------------------------------
// the opaque system
// ---------------------------------------------------------------------------
struct CgState;

struct cr_system {
  int d = 0;
  int64_t ne = 0, nf = 0;
  cr_params params{};
  crh::Topology topo;
  hipStream_t stream = nullptr;
  int device = 0;
  cr_allocator alloc{};
  bool has_alloc = false;
  std::vector<void*> owned;

  // element data, internal element order, structure of arrays
  double* ecoord = nullptr;    // [(d+1)*d][ne] vertex coordinates
  int32_t* eface = nullptr;    // [d+1][ne] internal interior face or -1
  uint32_t* eflags = nullptr;  // [ne]
  int32_t* ecaller = nullptr;  // [ne] caller id
  int32_t* enb = nullptr;      // [d+1][ne] internal neighbour across local face j or -1
  // face data, internal face order
  int32_t* fel = nullptr;      // [2][nf] internal (owner K, other L)
  int32_t* floc = nullptr;     // [nf] jK | jL << 8
  int32_t* fcanon = nullptr;   // [nf] canonical id
  int32_t* cols = nullptr;     // [2d][nf] off-diagonal block columns (self if padded)
  // elimination products
  double* pack = nullptr;      // [npack][ne] element factors
  double* RK = nullptr;        // [(d+1)*d][ne] local right-hand side R_K
  double* sK = nullptr;        // [(d+1)*d][ne] local s_K
  double* lam = nullptr;       // [ne] lambda of M1 elements (mu == 0)
  double* G64 = nullptr;       // [(2d+1)*d*d][nf] scaled G, FP64
  float* G32 = nullptr;        // same, rounded to FP32
  double* dsq = nullptr;       // [nf*d] face scale sqrt(mean_i |G_(f,i),(f,i)|), same for all i
  // element-factor form of the scaled Stokes operator (layout in rowkern.h)
  double* efo64 = nullptr;     // [EfoLayout::NF][ne]
  float* efo32 = nullptr;      // same, rounded to FP32
  int32_t* egat = nullptr;     // [d+1][ne] face read for local face j (an interior one)
  // The element form carries the Schur term of K0 as well (pressure gauge
  // moved out of G, see krylov.hip): its right-hand side, the null vector of
  // that operator in scaled variables, and the gauge shift of the last solve.
  double* bs1 = nullptr;       // [nf*d]
  double* zy = nullptr;        // [nf*d]
  double* k0t = nullptr;       // [1]
  double* k0eps = nullptr;     // [1] divergence data of K0's row in the gauge-shifted system
  int64_t k0i = 0;             // internal id of K0
  // coarse correction of the element-form CG (nagg > 0): aggregate of each
  // face, the (element, j, l) entries of each nonzero of E = Z^t G' Z grouped
  // by (row, column) pair, E and its inverse (dense, nagg x nagg), and the
  // null-vector columns z in FP32
  int32_t nagg = 0;
  int32_t npairs = 0;
  int32_t* fagg = nullptr;     // [nf]
  int32_t* pair_ptr = nullptr; // [npairs + 1]
  int32_t* pair_key = nullptr; // [npairs] row * nagg + column
  int32_t* pair_ent = nullptr; // [entries] k * 16 + j * 4 + l
  double* Ec = nullptr;        // [nagg * nagg]
  double* Einv = nullptr;      // [nagg * nagg]
  double* gjbuf = nullptr;     // inversion scratch for nagg > 128
  float* zy32 = nullptr;       // [nf * d]
  int64_t nbnd = 0;            // elements with F_AGGB
  double* bs = nullptr;        // [nf*d] S / dsq
  double* y = nullptr;         // [nf*d] dsq * W (resident solution, scaled)
  double* fbar = nullptr;      // [ne*d] internal element order
  double* uprev = nullptr;     // [nf*d] internal face order
  double* ulin = nullptr;      // [nf*d] internal face order
  int32_t* err = nullptr;      // [4] device error word, first element
  // non-homogeneous Dirichlet data (cr_set_boundary): exterior face of each
  // local face, the data in canonical exterior order, and the right-hand side
  // e_K of the divergence rows
  bool has_bnd = false;
  int32_t* ebf = nullptr;      // [d+1][ne] internal element order, -1 interior
  double* gbnd = nullptr;      // [nbf*d]
  double* ek = nullptr;        // [ne]
  double* ujump = nullptr;     // [nf*d + 1024] non-owner copies for the mismatch diagnostic
  int npack = 0;
  bool eliminated = false;
  bool has_solution = false;
  // the block rows G64 / G32 hold the current G (built on first use where CG
  // applies the element factors)
  bool g_valid = false;

  // Krylov workspace (allocated on first solve), coupled-baseline workspace
  void* kws = nullptr;
  void* cws = nullptr;
};

namespace crh {

void* dev_alloc(cr_system* s, size_t bytes);
cr_status check_hip(hipError_t e, const char* what);

// element / face kernels (elements.hip)
cr_status run_eliminate(cr_system* s, const double* f_mean, const double* u_prev, const double* u_lin);
// builds the block rows of G (FP64, FP32) if the last elimination left them out
cr_status ensure_assembled(cr_system* s);
cr_status run_update_rhs(cr_system* s, const double* f_mean, const double* u_prev);
cr_status run_recover(cr_system* s, double* U, double* P, double* jump);
// y = dsq * w0 from a device array in canonical order (initial guess of a solve)
cr_status enqueue_import_w(cr_system* s, const double* w0);
// w = y / dsq into a device array in canonical order (the resident W)
cr_status enqueue_export_w(cr_system* s, double* w);
// cr_recover without device allocation: mismatch partials in a static device array
cr_status run_recover_noalloc(cr_system* s, double* U, double* P, double* jump);
// Maps a solution of the element-form system (with the K0 Schur term) to the
// solution of G W = S: y += t zy with t = -(K0 pressure of that solution).
cr_status enqueue_gauge_fix(cr_system* s, hipStream_t stream);

// Krylov (krylov.hip)
cr_status run_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info);
cr_status run_time_spmv(cr_system* s, int precision, int form, int reps, double* avg_ms, double* bytes);
void free_krylov(cr_system* s);

// coupled baseline (coupled.hip)
cr_status run_coupled_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info, double* U, double* P);
int64_t coupled_nnz(const cr_system* s);
cr_status run_coupled_export(cr_system* s, int64_t* rowptr, int32_t* col, double* val, double* R);
void free_coupled(cr_system* s);

}  // namespace crh
