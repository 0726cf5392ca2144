// C ABI of the crhyb library: system lifecycle, uploads, exports.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace crh {

const char* last_error_str();

cr_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return CR_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CR_E_NOMEM : CR_E_DEVICE;
}

void* dev_alloc(cr_system* s, size_t bytes) {
  void* p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (s->has_alloc) {
    p = s->alloc.alloc(bytes, s->alloc.ctx, (void*)s->stream);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p)
    s->owned.push_back(p);
  else
    set_error("device allocation of %zu bytes failed", bytes);
  return p;
}

namespace {

void release_all(cr_system* s) {
  free_krylov(s);
  free_coupled(s);
  for (void* p : s->owned) {
    if (s->has_alloc)
      s->alloc.release(p, s->alloc.ctx, (void*)s->stream);
    else
      (void)hipFree(p);
  }
  s->owned.clear();
}

template <typename T>
cr_status upload(cr_system* s, T*& dst, const std::vector<T>& src) {
  dst = (T*)dev_alloc(s, sizeof(T) * src.size());
  if (!dst) return CR_E_NOMEM;
  return check_hip(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s->stream), "upload");
}

template <typename T>
cr_status alloc_n(cr_system* s, T*& dst, size_t n) {
  dst = (T*)dev_alloc(s, sizeof(T) * n);
  return dst ? CR_OK : CR_E_NOMEM;
}

int64_t stencil_blocks(const Topology& t) {
  int64_t b = t.nf;
  const int d1 = t.d + 1;
  for (int64_t k = 0; k < t.ne; ++k) {
    int s = 0;
    for (int j = 0; j < d1; ++j) s += t.elem_face[k * d1 + j] >= 0;
    b += (int64_t)s * (s - 1);
  }
  return b;
}

cr_status build(cr_system* s) {
  const Topology& t = s->topo;
  const int d = t.d, d1 = d + 1;
  const int64_t ne = t.ne, nf = t.nf;
  s->d = d;
  s->ne = ne;
  s->nf = nf;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  // Newton step: A^_K^{-1} (NU x NU, NU = (d+1) d), l, r, 1/B; Stokes: S_K^{-1}
  // (symmetric), V = A^_K^{-1} D_K, 1/B
  const int nu_loc = d1 * d;
  s->npack = ns ? nu_loc * nu_loc + 2 * nu_loc + 1 : (d1 * (d1 + 1) / 2 + d1 * d + 1);
  return CR_OK;
}

}  // namespace
}  // namespace crh

using namespace crh;

namespace crh {

// Structural non-zeros of the coupled matrix [A D^t; D 0] (A: d x d blocks of
// the face stencil, or their diagonals for Stokes; D and D^t: d per interior
// face of every element but K0).
int64_t coupled_nnz(const cr_system* s) {
  const int d = s->d, d1 = d + 1;
  int64_t dcount = 0;
  for (int64_t k = 0; k < s->ne; ++k) {
    if (k == s->params.k0) continue;
    for (int j = 0; j < d1; ++j) dcount += s->topo.elem_face[k * d1 + j] >= 0 ? d : 0;
  }
  const int64_t blocks = stencil_blocks(s->topo);
  const int64_t a = s->params.problem == CR_NS_NEWTON ? blocks * d * d : blocks * d;
  return a + 2 * dcount;
}

// Host tables of a system in internal order, staged for upload.
struct Staging {
  std::vector<double> ecoord;
  std::vector<int32_t> eface, ecaller, enb, fel, floc, fcanon;
  std::vector<uint32_t> eflags;
  std::vector<int32_t> pair_ptr, pair_key, pair_ent;  // coarse correction
  bool coarse = false;
};

cr_status check_params(const cr_mesh_desc* mesh, const cr_params* p) {
  if (!mesh || !p) {
    set_error("NULL mesh or params");
    return CR_E_INVAL;
  }
  if (!(p->nu > 0.0) || !std::isfinite(p->nu) || !(p->mu >= 0.0) || !std::isfinite(p->mu)) {
    set_error("need nu > 0 and mu >= 0 (got mu=%g nu=%g)", p->mu, p->nu);
    return CR_E_INVAL;
  }
  if (p->lambda_scale > 0.0 && !(p->lambda_scale > 1.0)) {
    set_error("lambda_scale %g: lambda_K must exceed ||A_K||_inf (scale > 1, or <= 0 for the default 2)",
              p->lambda_scale);
    return CR_E_INVAL;
  }
  if (p->problem != CR_STOKES && p->problem != CR_NS_NEWTON) {
    set_error("unknown problem kind %d", p->problem);
    return CR_E_INVAL;
  }
  if (p->k0 < 0 || p->k0 >= mesh->n_elements) {
    set_error("k0=%d out of range", p->k0);
    return CR_E_INVAL;
  }
  return CR_OK;
}


// Host part of the coarse-correction setup: the aggregate of each face
// (internal order) and, for every nonzero (a, b) of E = Z^t G' Z, the list of
// element entries (element k, local faces j and l with faces in aggregates a
// and b) that sum to it, grouped by a counting sort on the pair key; flags the
// elements whose interior faces lie in more than one aggregate.
cr_status coarse_host(cr_system* s, Staging& h) {
  const Topology& t = s->topo;
  const int d1 = t.d + 1;
  const int64_t ne = t.ne;
  const int m = t.nagg;
  const std::vector<int32_t>& eface = h.eface;
  std::vector<int64_t> count((size_t)m * m + 1, 0);
  for (int64_t k = 0; k < ne; ++k)
    for (int j = 0; j < d1; ++j) {
      const int32_t fj = eface[(size_t)j * ne + k];
      if (fj < 0) continue;
      for (int l = 0; l < d1; ++l) {
        const int32_t fl = eface[(size_t)l * ne + k];
        if (fl < 0) continue;
        count[(size_t)t.face_agg[fj] * m + t.face_agg[fl] + 1]++;
      }
    }
  h.pair_key.clear();
  h.pair_ptr.assign(1, 0);
  std::vector<int64_t> start((size_t)m * m, -1);
  int64_t total = 0;
  for (int64_t q = 0; q < (int64_t)m * m; ++q) {
    if (!count[q + 1]) continue;
    start[q] = total;
    total += count[q + 1];
    h.pair_key.push_back((int32_t)q);
    h.pair_ptr.push_back((int32_t)total);
  }
  if (total >= INT32_MAX) {
    set_error("coarse correction: too many element entries");
    return CR_E_INVAL;
  }
  h.pair_ent.assign((size_t)total, 0);
  for (int64_t k = 0; k < ne; ++k)
    for (int j = 0; j < d1; ++j) {
      const int32_t fj = eface[(size_t)j * ne + k];
      if (fj < 0) continue;
      for (int l = 0; l < d1; ++l) {
        const int32_t fl = eface[(size_t)l * ne + k];
        if (fl < 0) continue;
        const int64_t q = (int64_t)t.face_agg[fj] * m + t.face_agg[fl];
        h.pair_ent[(size_t)start[q]++] = (int32_t)(k * 16 + j * 4 + l);
      }
    }
  int64_t nb = 0;
  for (int64_t k = 0; k < ne; ++k) {
    int a0 = -1;
    bool multi = false;
    for (int j = 0; j < d1; ++j) {
      const int32_t fj = eface[(size_t)j * ne + k];
      if (fj < 0) continue;
      if (a0 < 0) a0 = t.face_agg[fj];
      else if (t.face_agg[fj] != a0) multi = true;
    }
    if (multi) {
      h.eflags[k] |= F_AGGB;
      ++nb;
    }
  }
  s->nbnd = nb;
  s->nagg = m;
  s->npairs = (int32_t)h.pair_key.size();
  h.coarse = true;
  return CR_OK;
}

// Host part of cr_assemble (no device call): parameters, topology, and the
// element and face tables in internal order.
cr_status prepare_host(const cr_mesh_desc* mesh, const cr_params* params, cr_system*& out, Staging& h) {
  out = nullptr;
  cr_status st = check_params(mesh, params);
  if (st != CR_OK) return st;
  cr_system* s = new (std::nothrow) cr_system();
  if (!s) return CR_E_NOMEM;
  s->params = *params;
  st = build_topology(mesh, params->renumber, params->mu == 0.0,
                      params->mu > 0.0 && params->problem == CR_STOKES, s->topo);
  if (st == CR_OK) st = build(s);
  if (st != CR_OK) {
    delete s;
    return st;
  }
  const Topology& t = s->topo;
  const int d = t.d, d1 = d + 1;
  const int64_t ne = t.ne, nf = t.nf;
  h.ecoord.assign((size_t)d1 * d * ne, 0.0);
  h.eface.assign((size_t)d1 * ne, 0);
  h.ecaller.assign(ne, 0);
  h.enb.assign((size_t)d1 * ne, 0);
  h.eflags.assign(ne, 0u);
  for (int64_t k = 0; k < ne; ++k) {
    const int32_t c = t.elem_iperm[k];
    h.ecaller[k] = c;
    uint32_t fl = 0;
    for (int j = 0; j < d1; ++j) {
      const int32_t v = mesh->elem_vertices[(int64_t)c * d1 + j];
      for (int r = 0; r < d; ++r) h.ecoord[(size_t)(j * d + r) * ne + k] = mesh->coords[(int64_t)v * d + r];
      const int32_t fc = t.elem_face[(int64_t)c * d1 + j];
      if (fc >= 0) {
        h.eface[(size_t)j * ne + k] = t.face_perm[fc];
        fl |= F_INTERIOR0 << j;
        const bool owner = t.face_elem[2 * fc] == c;
        if (!owner) fl |= F_NEG0 << j;
        const int32_t other = owner ? t.face_elem[2 * fc + 1] : t.face_elem[2 * fc];
        h.enb[(size_t)j * ne + k] = t.elem_perm[other];
      } else {
        h.eface[(size_t)j * ne + k] = -1;
        h.enb[(size_t)j * ne + k] = -1;
      }
    }
    if (c == params->k0) {
      fl |= F_K0;
      s->k0i = k;
    }
    if (t.m1[c]) fl |= F_M1;
    h.eflags[k] = fl;
  }
  h.fel.assign((size_t)2 * nf, 0);
  h.floc.assign(nf, 0);
  h.fcanon.assign(nf, 0);
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t fc = t.face_iperm[f];
    h.fcanon[f] = fc;
    h.fel[f] = t.elem_perm[t.face_elem[2 * fc]];
    h.fel[nf + f] = t.elem_perm[t.face_elem[2 * fc + 1]];
    h.floc[f] = (int32_t)t.face_loc[2 * fc] | ((int32_t)t.face_loc[2 * fc + 1] << 8);
  }
  const bool ns = params->problem == CR_NS_NEWTON;
  if (!ns && params->mu > 0.0 && t.nagg > 0) st = coarse_host(s, h);
  if (st != CR_OK) {
    delete s;
    return st;
  }
  out = s;
  return CR_OK;
}

// Device part of cr_assemble: uploads the staged tables and allocates the
// system's device arrays on its stream; releases the system on failure.
cr_status finish_device(cr_system* s, Staging& h, const cr_allocator* alloc, void* hip_stream) {
  s->stream = (hipStream_t)hip_stream;
  if (alloc && alloc->alloc && alloc->release) {
    s->alloc = *alloc;
    s->has_alloc = true;
  }
  cr_status st = check_hip(hipGetDevice(&s->device), "hipGetDevice");
  const Topology& t = s->topo;
  const int d = t.d, d1 = d + 1;
  const int64_t ne = t.ne, nf = t.nf;
  const bool ns = s->params.problem == CR_NS_NEWTON;
  const size_t nslot = 2 * d + 1, nvec = (size_t)nf * d;
  if (st == CR_OK) st = upload(s, s->ecoord, h.ecoord);
  if (st == CR_OK) st = upload(s, s->eface, h.eface);
  if (st == CR_OK) st = upload(s, s->eflags, h.eflags);
  if (st == CR_OK) st = upload(s, s->ecaller, h.ecaller);
  if (st == CR_OK) st = upload(s, s->enb, h.enb);
  if (st == CR_OK) st = upload(s, s->fel, h.fel);
  if (st == CR_OK) st = upload(s, s->floc, h.floc);
  if (st == CR_OK) st = upload(s, s->fcanon, h.fcanon);
  if (st == CR_OK) st = alloc_n(s, s->cols, (size_t)2 * d * nf);
  if (st == CR_OK) st = alloc_n(s, s->pack, (size_t)s->npack * ne);
  if (st == CR_OK) st = alloc_n(s, s->RK, (size_t)d1 * d * ne);
  if (st == CR_OK) st = alloc_n(s, s->sK, (size_t)d1 * d * ne);
  if (st == CR_OK) st = alloc_n(s, s->lam, (size_t)ne);
  if (st == CR_OK) st = alloc_n(s, s->dsq, nvec);
  if (st == CR_OK && !ns && s->params.mu > 0.0) {
    // element-factor form of the scaled operator (transient Stokes CG)
    const size_t nplanes = (size_t)d1 * (d1 + 1) / 2 + (size_t)d1 * d;
    st = alloc_n(s, s->efo64, nplanes * ne);
    if (st == CR_OK) st = alloc_n(s, s->efo32, nplanes * ne);
    if (st == CR_OK) st = alloc_n(s, s->egat, (size_t)d1 * ne);
    if (st == CR_OK) st = alloc_n(s, s->bs1, nvec);
    if (st == CR_OK) st = alloc_n(s, s->zy, nvec);
    if (st == CR_OK) st = alloc_n(s, s->k0t, (size_t)1);
    if (st == CR_OK) st = alloc_n(s, s->k0eps, (size_t)1);
    if (st == CR_OK && h.coarse) {
      const size_t m = (size_t)s->nagg;
      st = upload(s, s->fagg, t.face_agg);
      if (st == CR_OK) st = upload(s, s->pair_ptr, h.pair_ptr);
      if (st == CR_OK) st = upload(s, s->pair_key, h.pair_key);
      if (st == CR_OK) st = upload(s, s->pair_ent, h.pair_ent);
      if (st == CR_OK) st = alloc_n(s, s->Ec, m * m);
      if (st == CR_OK) st = alloc_n(s, s->Einv, m * m);
      if (st == CR_OK) st = alloc_n(s, s->zy32, nvec);
    }
  }
  if (st == CR_OK) st = alloc_n(s, s->bs, nvec);
  if (st == CR_OK) st = alloc_n(s, s->y, nvec);
  if (st == CR_OK) st = alloc_n(s, s->fbar, (size_t)ne * d);
  if (st == CR_OK) st = alloc_n(s, s->uprev, nvec);
  if (st == CR_OK && ns) st = alloc_n(s, s->ulin, nvec);
  if (st == CR_OK) st = alloc_n(s, s->err, 4);
  // the staged host tables are read by the uploads until the stream drains
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "upload sync");
  if (st != CR_OK) {
    (void)hipStreamSynchronize(s->stream);
    release_all(s);
    delete s;
  }
  return st;
}

}  // namespace crh

extern "C" {

const char* cr_last_error(void) { return last_error_str(); }

const char* cr_version(void) { return "crhyb 0.1 (gfx950)"; }

cr_status cr_topology(const cr_mesh_desc* mesh, const cr_params* params, int64_t* n_int_faces, int32_t* perm,
                      int64_t* bw_int, int64_t* bw_can, int32_t* m1) {
  clear_error();
  cr_status st = check_params(mesh, params);
  if (st != CR_OK) return st;
  Topology t;
  st = build_topology(mesh, params->renumber, params->mu == 0.0,
                      params->mu > 0.0 && params->problem == CR_STOKES, t);
  if (st != CR_OK) return st;
  if (n_int_faces) *n_int_faces = t.nf;
  if (perm) std::copy(t.face_perm.begin(), t.face_perm.end(), perm);
  if (bw_int) *bw_int = t.bw_internal;
  if (bw_can) *bw_can = t.bw_canonical;
  if (m1)
    for (int64_t k = 0; k < t.ne; ++k) m1[k] = t.m1[k];
  return CR_OK;
}

cr_status cr_assemble(const cr_mesh_desc* mesh, const cr_params* params, const cr_allocator* alloc, void* hip_stream,
                      cr_system** out) {
  clear_error();
  if (!out) {
    set_error("NULL output pointer");
    return CR_E_INVAL;
  }
  *out = nullptr;
  cr_system* s = nullptr;
  Staging h;
  cr_status st = prepare_host(mesh, params, s, h);
  if (st == CR_OK) st = finish_device(s, h, alloc, hip_stream);
  if (st == CR_OK) *out = s;
  return st;
}

struct cr_prepared {
  cr_system* s = nullptr;
  crh::Staging h;
};

cr_status cr_prepare(const cr_mesh_desc* mesh, const cr_params* params, cr_prepared** out) {
  clear_error();
  if (!out) {
    set_error("NULL output pointer");
    return CR_E_INVAL;
  }
  *out = nullptr;
  cr_prepared* p = new (std::nothrow) cr_prepared();
  if (!p) return CR_E_NOMEM;
  const cr_status st = prepare_host(mesh, params, p->s, p->h);
  if (st != CR_OK) {
    delete p;
    return st;
  }
  *out = p;
  return CR_OK;
}

cr_status cr_assemble_prepared(cr_prepared* prep, const cr_allocator* alloc, void* hip_stream, cr_system** out) {
  clear_error();
  if (!prep || !out || !prep->s) {
    set_error("NULL prepared mesh or output pointer");
    delete prep;
    return CR_E_INVAL;
  }
  *out = nullptr;
  cr_system* s = prep->s;
  prep->s = nullptr;
  const cr_status st = finish_device(s, prep->h, alloc, hip_stream);
  delete prep;
  if (st == CR_OK) *out = s;
  return st;
}

void cr_prepared_destroy(cr_prepared* prep) {
  if (!prep) return;
  delete prep->s;
  delete prep;
}

cr_status cr_eliminate(cr_system* s, const double* f_mean, const double* u_prev, const double* u_lin) {
  clear_error();
  if (!s || !f_mean) {
    set_error("NULL system or f_mean");
    return CR_E_INVAL;
  }
  const bool ns = s->params.problem == CR_NS_NEWTON;
  if (ns && !u_lin) {
    set_error("the Newton step needs u_lin");
    return CR_E_INVAL;
  }
  if (!ns && u_lin) {
    set_error("u_lin given for a Stokes problem");
    return CR_E_INVAL;
  }
  return run_eliminate(s, f_mean, u_prev, u_lin);
}

cr_status cr_update_rhs(cr_system* s, const double* f_mean, const double* u_prev) {
  clear_error();
  if (!s || !f_mean) {
    set_error("NULL system or f_mean");
    return CR_E_INVAL;
  }
  if (!s->eliminated) {
    set_error("cr_update_rhs before cr_eliminate");
    return CR_E_INVAL;
  }
  if (s->params.problem != CR_STOKES) {
    set_error("cr_update_rhs is for the Stokes problem (a Newton step changes G)");
    return CR_E_INVAL;
  }
  return run_update_rhs(s, f_mean, u_prev);
}

cr_status cr_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info) {
  clear_error();
  if (!s || !o) {
    set_error("NULL system or options");
    return CR_E_INVAL;
  }
  if (!s->eliminated) {
    set_error("cr_solve before cr_eliminate");
    return CR_E_INVAL;
  }
  if (o->method < CR_PCG || o->method > CR_MINRES) {
    set_error("unknown method %d", o->method);
    return CR_E_INVAL;
  }
  if (o->precision != CR_FP64 && o->precision != CR_FP32_IR) {
    set_error("unknown precision %d", o->precision);
    return CR_E_INVAL;
  }
  if (o->method == CR_PCG && !(s->params.mu > 0.0 && s->params.problem == CR_STOKES)) {
    set_error("CG needs the symmetric positive definite case (mu > 0, Stokes); use BiCGStab");
    return CR_E_INVAL;
  }
  return run_solve(s, o, info);
}

cr_status cr_recover(cr_system* s, double* U, double* P, double* jump) {
  clear_error();
  if (!s || !U || !P) {
    set_error("NULL system or output");
    return CR_E_INVAL;
  }
  if (!s->eliminated) {
    set_error("cr_recover before cr_eliminate");
    return CR_E_INVAL;
  }
  return run_recover(s, U, P, jump);
}

cr_status cr_recover_noalloc(cr_system* s, double* U, double* P, double* jump) {
  clear_error();
  if (!s || !U || !P) {
    set_error("NULL system or output");
    return CR_E_INVAL;
  }
  if (!s->eliminated) {
    set_error("cr_recover_noalloc before cr_eliminate");
    return CR_E_INVAL;
  }
  return run_recover_noalloc(s, U, P, jump);
}

cr_status cr_query_sizes(const cr_system* s, int64_t* n_int_faces, int64_t* nnz_G, int64_t* nnz_coupled) {
  clear_error();
  if (!s) {
    set_error("NULL system");
    return CR_E_INVAL;
  }
  const int64_t blocks = stencil_blocks(s->topo);
  const int d = s->d;
  if (n_int_faces) *n_int_faces = s->nf;
  if (nnz_G) *nnz_G = blocks * d * d;
  if (nnz_coupled) *nnz_coupled = coupled_nnz(s);
  return CR_OK;
}

cr_status cr_export_G(const cr_system* s, int64_t* rowptr, int32_t* col, double* val, double* S) {
  clear_error();
  if (!s || !s->eliminated) {
    set_error("cr_export_G needs an eliminated system");
    return CR_E_INVAL;
  }
  // the block rows are a cache of the eliminated system: building them leaves
  // its state otherwise unchanged
  cr_status st0 = ensure_assembled(const_cast<cr_system*>(s));
  if (st0 != CR_OK) return st0;
  const int d = s->d, DD = d * d, ns = 2 * d + 1;
  const int64_t nf = s->nf;
  std::vector<double> G((size_t)ns * DD * nf), dsq((size_t)nf * d), bs((size_t)nf * d);
  std::vector<int32_t> cols((size_t)2 * d * nf);
  cr_status st = check_hip(hipMemcpyAsync(G.data(), s->G64, G.size() * 8, hipMemcpyDeviceToHost, s->stream), "export");
  if (st == CR_OK)
    st = check_hip(hipMemcpyAsync(cols.data(), s->cols, cols.size() * 4, hipMemcpyDeviceToHost, s->stream), "export");
  if (st == CR_OK)
    st = check_hip(hipMemcpyAsync(dsq.data(), s->dsq, dsq.size() * 8, hipMemcpyDeviceToHost, s->stream), "export");
  if (st == CR_OK)
    st = check_hip(hipMemcpyAsync(bs.data(), s->bs, bs.size() * 8, hipMemcpyDeviceToHost, s->stream), "export");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "export");
  if (st != CR_OK) return st;
  const Topology& t = s->topo;
  int64_t pos = 0;
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t fc = 0; fc < nf; ++fc) {
    const int64_t f = t.face_perm[fc];
    for (int i = 0; i < d; ++i) {
      if (rowptr) rowptr[fc * d + i] = pos;
      row.clear();
      for (int sl = 0; sl < ns; ++sl) {
        const int64_t c = sl == 0 ? f : cols[(size_t)(sl - 1) * nf + f];
        if (sl > 0 && c == f) continue;  // padding slot of an exterior face
        const int64_t cc = t.face_iperm[c];
        for (int j = 0; j < d; ++j) {
          const double v = G[(size_t)(sl * DD + i * d + j) * nf + f] * dsq[f * d + i] * dsq[c * d + j];
          row.emplace_back((int32_t)(cc * d + j), v);
        }
      }
      std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (auto& e : row) {
        if (col) col[pos] = e.first;
        if (val) val[pos] = e.second;
        ++pos;
      }
      if (S) S[fc * d + i] = bs[f * d + i] * dsq[f * d + i];
    }
  }
  if (rowptr) rowptr[nf * d] = pos;
  return CR_OK;
}

cr_status cr_export_W(const cr_system* s, double* W) {
  clear_error();
  if (!s || !W || !s->eliminated) {
    set_error("cr_export_W needs an eliminated system and a buffer");
    return CR_E_INVAL;
  }
  const int d = s->d;
  const int64_t nf = s->nf;
  std::vector<double> y((size_t)nf * d), dsq((size_t)nf * d);
  cr_status st = check_hip(hipMemcpyAsync(y.data(), s->y, y.size() * 8, hipMemcpyDeviceToHost, s->stream), "export W");
  if (st == CR_OK)
    st = check_hip(hipMemcpyAsync(dsq.data(), s->dsq, dsq.size() * 8, hipMemcpyDeviceToHost, s->stream), "export W");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "export W");
  if (st != CR_OK) return st;
  for (int64_t fc = 0; fc < nf; ++fc) {
    const int64_t f = s->topo.face_perm[fc];
    for (int i = 0; i < d; ++i) W[fc * d + i] = y[f * d + i] / dsq[f * d + i];
  }
  return CR_OK;
}

cr_status cr_export_W_device(cr_system* s, double* W) {
  clear_error();
  if (!s || !W || !s->eliminated) {
    set_error("cr_export_W_device needs an eliminated system and a device buffer");
    return CR_E_INVAL;
  }
  return enqueue_export_w(s, W);
}

cr_status cr_import_W(cr_system* s, const double* W) {
  clear_error();
  if (!s || !W || !s->eliminated) {
    set_error("cr_import_W needs an eliminated system and a host buffer");
    return CR_E_INVAL;
  }
  const int d = s->d;
  const int64_t nf = s->nf;
  std::vector<double> dsq((size_t)nf * d), y((size_t)nf * d);
  cr_status st = check_hip(hipMemcpyAsync(dsq.data(), s->dsq, dsq.size() * 8, hipMemcpyDeviceToHost, s->stream), "import W");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "import W");
  if (st != CR_OK) return st;
  for (int64_t fc = 0; fc < nf; ++fc) {
    const int64_t f = s->topo.face_perm[fc];
    for (int i = 0; i < d; ++i) y[f * d + i] = W[fc * d + i] * dsq[f * d + i];
  }
  st = check_hip(hipMemcpyAsync(s->y, y.data(), y.size() * 8, hipMemcpyHostToDevice, s->stream), "import W");
  if (st == CR_OK) st = check_hip(hipStreamSynchronize(s->stream), "import W");
  if (st == CR_OK) s->has_solution = true;
  return st;
}

cr_status cr_interior_faces(const cr_system* s, int32_t* face_vertices) {
  clear_error();
  if (!s || !face_vertices) {
    set_error("NULL system or buffer");
    return CR_E_INVAL;
  }
  std::copy(s->topo.face_vertices.begin(), s->topo.face_vertices.end(), face_vertices);
  return CR_OK;
}

cr_status cr_boundary_faces(const cr_system* s, int64_t* n_bnd_faces, int32_t* face_vertices) {
  clear_error();
  if (!s) {
    set_error("NULL system");
    return CR_E_INVAL;
  }
  if (n_bnd_faces) *n_bnd_faces = s->topo.nbf;
  if (face_vertices) std::copy(s->topo.bface_vertices.begin(), s->topo.bface_vertices.end(), face_vertices);
  return CR_OK;
}

cr_status cr_set_boundary(cr_system* s, const double* g) {
  clear_error();
  if (!s) {
    set_error("NULL system");
    return CR_E_INVAL;
  }
  if (!g) {
    s->has_bnd = false;
    return CR_OK;
  }
  const int d = s->d, d1 = d + 1;
  const int64_t ne = s->ne, nbf = s->topo.nbf;
  if (nbf == 0) {
    set_error("the mesh has no exterior face");
    return CR_E_INVAL;
  }
  cr_status st = CR_OK;
  if (!s->ebf) {
    // exterior face of each local face, internal element order
    std::vector<int32_t> h((size_t)d1 * ne);
    for (int64_t k = 0; k < ne; ++k) {
      const int64_t c = s->topo.elem_iperm[k];
      for (int j = 0; j < d1; ++j) h[(size_t)j * ne + k] = s->topo.elem_bface[(size_t)c * d1 + j];
    }
    st = upload(s, s->ebf, h);
    if (st == CR_OK) st = alloc_n(s, s->gbnd, (size_t)nbf * d);
    if (st == CR_OK) st = alloc_n(s, s->ek, (size_t)ne);
    if (st != CR_OK) return st;
  }
  st = check_hip(hipMemcpyAsync(s->gbnd, g, sizeof(double) * nbf * d, hipMemcpyDeviceToDevice, s->stream),
                 "boundary data");
  if (st != CR_OK) return st;
  s->has_bnd = true;
  return CR_OK;
}

cr_status cr_time_spmv(cr_system* s, int32_t precision, int32_t operator_form, int32_t reps, double* avg_ms,
                       double* bytes) {
  clear_error();
  if (!s || !s->eliminated || reps < 1) {
    set_error("cr_time_spmv needs an eliminated system and reps >= 1");
    return CR_E_INVAL;
  }
  if (precision != CR_FP64 && precision != CR_FP32_IR) {
    set_error("unknown precision %d", precision);
    return CR_E_INVAL;
  }
  return run_time_spmv(s, precision, operator_form, reps, avg_ms, bytes);
}

cr_status cr_export_coupled(cr_system* s, int64_t* rowptr, int32_t* col, double* val, double* R) {
  clear_error();
  if (!s || !s->eliminated) {
    set_error("cr_export_coupled needs an eliminated system");
    return CR_E_INVAL;
  }
  if (s->params.problem != CR_STOKES) {
    set_error("the coupled export is for the Stokes problem");
    return CR_E_INVAL;
  }
  return run_coupled_export(s, rowptr, col, val, R);
}

cr_status cr_coupled_solve(cr_system* s, const cr_solve_opts* o, cr_solve_info* info, double* U, double* P) {
  clear_error();
  if (!s || !o || !U || !P) {
    set_error("NULL argument");
    return CR_E_INVAL;
  }
  if (!s->eliminated) {
    set_error("cr_coupled_solve needs the element data of cr_eliminate");
    return CR_E_INVAL;
  }
  return run_coupled_solve(s, o, info, U, P);
}

void cr_destroy(cr_system* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  release_all(s);
  delete s;
}

}  // extern "C"
