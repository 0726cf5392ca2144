// Step a0: face topology, sign choice, reverse Cuthill-McKee face order, element
// order and the element partition M1/M2.  Host code only (no device calls).
//
// Paper: Section 2 item 1 (simplicial mesh, faces, M_sigma with one or two
// elements), Section 3.2 eq. propc (C_K = +-1, opposite on the two sides of a
// face), Section 3.2 item 7 (M1/M2 partition for mu = 0), Section 3.2 item 5
// (G has the block stencil of A, which the face adjacency below describes).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <queue>

#include "internal.h"

namespace crh {

namespace {

// Bisects idx[lo, hi) at the median of the longest centroid extent (ties by
// element id) and returns the split position.
size_t bisect(std::vector<int32_t>& idx, size_t lo, size_t hi, const std::vector<double>& cen, int d) {
  int ax = 0;
  double best = -1.0;
  for (int a = 0; a < d; ++a) {
    double mn = 1e300, mx = -1e300;
    for (size_t i = lo; i < hi; ++i) {
      const double c = cen[(size_t)idx[i] * d + a];
      mn = std::min(mn, c);
      mx = std::max(mx, c);
    }
    if (mx - mn > best) {
      best = mx - mn;
      ax = a;
    }
  }
  const size_t mid = lo + (hi - lo) / 2;
  std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [&](int32_t a, int32_t b) {
    const double ca = cen[(size_t)a * d + ax], cb = cen[(size_t)b * d + ax];
    return ca < cb || (ca == cb && a < b);
  });
  return mid;
}

// recursive coordinate bisection of idx[lo, hi) into `parts` (a power of two)
// groups; group ids in depth-first order, and idx ends up grouped in that order
void rcb(std::vector<int32_t>& idx, size_t lo, size_t hi, int parts, const std::vector<double>& cen, int d,
         int& next, std::vector<int32_t>& agg) {
  if (parts == 1 || hi - lo < 2) {
    for (size_t i = lo; i < hi; ++i) agg[idx[i]] = next;
    ++next;
    return;
  }
  const size_t mid = bisect(idx, lo, hi, cen, d);
  rcb(idx, lo, mid, parts / 2, cen, d, next, agg);
  rcb(idx, mid, hi, parts / 2, cen, d, next, agg);
}

// the same bisection continued down to `leaf` elements: a depth-first order in
// which elements that are close in the order are close in space
void rcb_order(std::vector<int32_t>& idx, size_t lo, size_t hi, const std::vector<double>& cen, int d, size_t leaf) {
  if (hi - lo <= leaf) return;
  const size_t mid = bisect(idx, lo, hi, cen, d);
  rcb_order(idx, lo, mid, cen, d, leaf);
  rcb_order(idx, mid, hi, cen, d, leaf);
}

struct LocalFace {
  uint32_t v[3];
  int32_t elem;
  int8_t loc;
};

bool key_less(const LocalFace& a, const LocalFace& b) {
  if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
  if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
  if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
  if (a.elem != b.elem) return a.elem < b.elem;
  return a.loc < b.loc;
}

bool key_eq(const LocalFace& a, const LocalFace& b) {
  return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
}

// BFS levels from `root` restricted to unvisited-in-component nodes; returns the
// last level and fills `depth` for the component.
int bfs_eccentricity(int root, const std::vector<int64_t>& ptr, const std::vector<int32_t>& adj,
                     std::vector<int32_t>& depth, std::vector<int32_t>& touched, std::vector<int32_t>& last) {
  for (int v : touched) depth[v] = -1;
  touched.clear();
  std::vector<int32_t> frontier{root};
  depth[root] = 0;
  touched.push_back(root);
  int level = 0;
  last = frontier;
  while (!frontier.empty()) {
    std::vector<int32_t> next;
    for (int v : frontier)
      for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
        int w = adj[e];
        if (depth[w] < 0) {
          depth[w] = level + 1;
          touched.push_back(w);
          next.push_back(w);
        }
      }
    if (!next.empty()) {
      last = next;
      ++level;
    }
    frontier.swap(next);
  }
  return level;
}

}  // namespace

cr_status build_topology(const cr_mesh_desc* mesh, int renumber, bool need_m1, bool aggregate, Topology& t) {
  const int d = mesh->dim;
  if (d != 2 && d != 3) {
    set_error("dim must be 2 or 3 (got %d)", d);
    return CR_E_INVAL;
  }
  const int d1 = d + 1;
  const int64_t ne = mesh->n_elements, nv = mesh->n_vertices;
  if (ne < 1 || nv < d1 || !mesh->coords || !mesh->elem_vertices) {
    set_error("empty mesh or NULL arrays");
    return CR_E_INVAL;
  }
  if (ne * d1 > INT32_MAX || nv > INT32_MAX) {
    set_error("mesh too large for 32-bit indices");
    return CR_E_INVAL;
  }
  t = Topology();
  t.d = d;
  t.ne = ne;
  t.nv = nv;
  const int32_t* ev = mesh->elem_vertices;
  const double* X = mesh->coords;

  // validate elements: ids in range, distinct, non-degenerate
  for (int64_t k = 0; k < ne; ++k) {
    const int32_t* e = ev + k * d1;
    for (int a = 0; a < d1; ++a) {
      if (e[a] < 0 || e[a] >= nv) {
        set_error("element %lld references vertex %d out of range", (long long)k, e[a]);
        return CR_E_MESH;
      }
      for (int b = 0; b < a; ++b)
        if (e[a] == e[b]) {
          set_error("element %lld repeats a vertex", (long long)k);
          return CR_E_MESH;
        }
    }
    double E[3][3] = {};
    double scale = 0.0;
    for (int c = 0; c < d; ++c)
      for (int r = 0; r < d; ++r) {
        E[r][c] = X[(int64_t)e[c + 1] * d + r] - X[(int64_t)e[0] * d + r];
        scale = std::max(scale, std::fabs(E[r][c]));
      }
    double det;
    if (d == 2)
      det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
    else
      det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
            E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (!(std::fabs(det) > 1e-14 * std::pow(scale, d)) || !std::isfinite(det)) {
      set_error("element %lld has zero volume", (long long)k);
      return CR_E_MESH;
    }
  }

  // local faces, face j opposite local vertex j, key = sorted vertex ids
  std::vector<LocalFace> lf((size_t)ne * d1);
  for (int64_t k = 0; k < ne; ++k) {
    const int32_t* e = ev + k * d1;
    for (int j = 0; j < d1; ++j) {
      LocalFace& f = lf[k * d1 + j];
      int n = 0;
      uint32_t v[3] = {0, 0, 0};
      for (int a = 0; a < d1; ++a)
        if (a != j) v[n++] = (uint32_t)e[a];
      std::sort(v, v + d);
      f.v[0] = v[0];
      f.v[1] = v[1];
      f.v[2] = d == 3 ? v[2] : 0u;
      f.elem = (int32_t)k;
      f.loc = (int8_t)j;
    }
  }
  std::sort(lf.begin(), lf.end(), key_less);

  t.elem_face.assign((size_t)ne * d1, -1);
  t.elem_bface.assign((size_t)ne * d1, -1);
  int64_t nf = 0;
  for (size_t i = 0; i < lf.size();) {
    size_t j = i + 1;
    while (j < lf.size() && key_eq(lf[i], lf[j])) ++j;
    if (j - i > 2) {
      set_error("a face is shared by %zu elements (element %d)", j - i, lf[i].elem);
      return CR_E_MESH;
    }
    if (j - i == 1) {
      // exterior face: canonical exterior id in the same lexicographic key order
      for (int a = 0; a < d; ++a) t.bface_vertices.push_back((int32_t)lf[i].v[a]);
      t.elem_bface[(size_t)lf[i].elem * d1 + lf[i].loc] = (int32_t)t.nbf;
      ++t.nbf;
    }
    if (j - i == 2) {
      // interior face: canonical id in lexicographic key order; K < L by caller id
      for (int a = 0; a < d; ++a) t.face_vertices.push_back((int32_t)lf[i].v[a]);
      t.face_elem.push_back(lf[i].elem);
      t.face_elem.push_back(lf[i + 1].elem);
      t.face_loc.push_back(lf[i].loc);
      t.face_loc.push_back(lf[i + 1].loc);
      t.elem_face[(size_t)lf[i].elem * d1 + lf[i].loc] = (int32_t)nf;
      t.elem_face[(size_t)lf[i + 1].elem * d1 + lf[i + 1].loc] = (int32_t)nf;
      ++nf;
    }
    i = j;
  }
  t.nf = nf;
  if (nf == 0) {
    set_error("mesh has no interior face");
    return CR_E_MESH;
  }
  for (int64_t k = 0; k < ne; ++k) {
    int s = 0;
    for (int j = 0; j < d1; ++j) s += t.elem_face[k * d1 + j] >= 0;
    if (s == 0) {
      set_error("element %lld has no interior face", (long long)k);
      return CR_E_MESH;
    }
  }

  // face adjacency through elements (the block stencil of A and of G)
  std::vector<int64_t> ptr(nf + 1, 0);
  for (int64_t k = 0; k < ne; ++k)
    for (int a = 0; a < d1; ++a) {
      int fa = t.elem_face[k * d1 + a];
      if (fa < 0) continue;
      for (int b = 0; b < d1; ++b)
        if (b != a && t.elem_face[k * d1 + b] >= 0) ptr[fa + 1]++;
    }
  for (int64_t f = 0; f < nf; ++f) ptr[f + 1] += ptr[f];
  std::vector<int32_t> adj(ptr[nf]);
  {
    std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t k = 0; k < ne; ++k)
      for (int a = 0; a < d1; ++a) {
        int fa = t.elem_face[k * d1 + a];
        if (fa < 0) continue;
        for (int b = 0; b < d1; ++b) {
          int fb = t.elem_face[k * d1 + b];
          if (b != a && fb >= 0) adj[pos[fa]++] = fb;
        }
      }
  }

  // face renumbering
  std::vector<int32_t> loc_elem_order;  // element order chosen with the aggregates (empty: none)
  t.face_perm.assign(nf, -1);
  t.face_iperm.assign(nf, -1);
  if (renumber == CR_NATURAL) {
    for (int64_t f = 0; f < nf; ++f) t.face_perm[f] = t.face_iperm[f] = (int32_t)f;
  } else if (renumber == CR_RCM) {
    // Reverse Cuthill-McKee: per connected component, start from a
    // pseudo-peripheral node (repeated BFS from a minimum-degree node of the
    // last level), visit neighbours by increasing degree, reverse at the end.
    std::vector<int32_t> deg(nf);
    for (int64_t f = 0; f < nf; ++f) deg[f] = (int32_t)(ptr[f + 1] - ptr[f]);
    std::vector<int32_t> order;
    order.reserve(nf);
    std::vector<uint8_t> seen(nf, 0);
    std::vector<int32_t> depth(nf, -1), touched, last;
    for (int64_t s0 = 0; s0 < nf; ++s0) {
      if (seen[s0]) continue;
      int root = (int)s0;
      int ecc = bfs_eccentricity(root, ptr, adj, depth, touched, last);
      for (int v : touched)  // minimum degree node of the component as the first guess
        if (deg[v] < deg[root] || (deg[v] == deg[root] && v < root)) root = v;
      ecc = bfs_eccentricity(root, ptr, adj, depth, touched, last);
      for (int it = 0; it < 8; ++it) {
        int cand = last[0];
        for (int v : last)
          if (deg[v] < deg[cand] || (deg[v] == deg[cand] && v < cand)) cand = v;
        int e2 = bfs_eccentricity(cand, ptr, adj, depth, touched, last);
        if (e2 <= ecc) break;
        ecc = e2;
        root = cand;
      }
      size_t head = order.size();
      order.push_back(root);
      seen[root] = 1;
      std::vector<int32_t> nb;
      while (head < order.size()) {
        int v = order[head++];
        nb.clear();
        for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
          if (!seen[adj[e]]) nb.push_back(adj[e]);
        std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
        for (int w : nb)
          if (!seen[w]) {
            seen[w] = 1;
            order.push_back(w);
          }
      }
    }
    std::reverse(order.begin(), order.end());
    // Aggregates for the coarse correction: recursive coordinate bisection of
    // the element centroids into nagg parts, numbered in bisection order so
    // that consecutive aggregates are neighbours.  nagg is a power of 4 in 2D
    // and of 8 in 3D (bisection alternates the axes on a square or a cube, so
    // the parts come out square or cubic: a power of two in between, with
    // elongated parts, takes about as many CG iterations as the power below
    // it), as many as the mesh has room for with at least 128 elements each,
    // at most 256 in 2D and MAX_AGG = 512 in 3D (the dense coarse inverse is
    // read at every iteration); none below 4 parts.  Smaller aggregates take
    // fewer iterations (2D, mu = 1000: 64x64x2 657 -> 260 with 4 -> 64
    // aggregates, 128x128x2 860 -> 439 with 16 -> 256; 3D 12^3 x 6: 340 -> 239
    // with 8 -> 64); 128 elements keep at least half a face block in each
    // aggregate, so that a face block of the solver touches at most 3 of them.
    // A face belongs to the aggregate of its owner element (the lower caller
    // id, C = +1).
    // With aggregates the element-form CG gathers its vectors element by
    // element, so the order is chosen for locality of those gathers rather
    // than for a narrow band: the bisection continues inside each aggregate
    // down to a few elements (elements close in the order are close in space;
    // the elements with faces in several aggregates come last within their
    // aggregate), and faces are numbered in the order the elements first touch
    // them, grouped by aggregate.  The two elements of most faces then fall in
    // the same workgroup pass, and the faces a wavefront gathers lie on few
    // cache lines.
    const int agg_base = d == 3 ? 8 : 4;
    const int agg_cap = d == 3 ? MAX_AGG : 256;
    const int64_t agg_min = 128;
    int nagg = 1;
    while (nagg * agg_base <= agg_cap && (int64_t)nagg * agg_base * agg_min <= ne) nagg *= agg_base;
    if (aggregate && nagg >= 4) {
      std::vector<double> cen((size_t)ne * d, 0.0);
      for (int64_t k = 0; k < ne; ++k)
        for (int j = 0; j < d1; ++j) {
          const int64_t v = mesh->elem_vertices[k * d1 + j];
          for (int a = 0; a < d; ++a) cen[k * d + a] += mesh->coords[v * d + a] / d1;
        }
      std::vector<int32_t> eagg(ne, 0), idx(ne);
      std::iota(idx.begin(), idx.end(), 0);
      int next = 0;
      rcb(idx, 0, (size_t)ne, nagg, cen, d, next, eagg);
      std::vector<int32_t> fagg(nf);
      for (int64_t f = 0; f < nf; ++f) fagg[f] = eagg[t.face_elem[2 * f]];
      // idx is grouped by aggregate in aggregate order; order each group
      for (size_t lo = 0; lo < (size_t)ne;) {
        size_t hi = lo;
        while (hi < (size_t)ne && eagg[idx[hi]] == eagg[idx[lo]]) ++hi;
        rcb_order(idx, lo, hi, cen, d, 4);
        lo = hi;
      }
      std::vector<uint8_t> multi(ne, 0);
      for (int64_t k = 0; k < ne; ++k) {
        int a0 = -1;
        for (int j = 0; j < d1; ++j) {
          const int f = t.elem_face[k * d1 + j];
          if (f < 0) continue;
          if (a0 < 0) a0 = fagg[f];
          else if (fagg[f] != a0) multi[k] = 1;
        }
      }
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        return eagg[a] != eagg[b] ? eagg[a] < eagg[b] : multi[a] < multi[b];
      });
      loc_elem_order = idx;
      order.clear();
      std::vector<uint8_t> seen(nf, 0);
      for (int64_t i = 0; i < ne; ++i)
        for (int j = 0; j < d1; ++j) {
          const int f = t.elem_face[(int64_t)idx[i] * d1 + j];
          if (f >= 0 && !seen[f]) {
            seen[f] = 1;
            order.push_back(f);
          }
        }
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fagg[a] < fagg[b]; });
      t.nagg = nagg;
      t.face_agg.resize(nf);
      for (int64_t i = 0; i < nf; ++i) t.face_agg[i] = fagg[order[i]];
    }
    for (int64_t i = 0; i < nf; ++i) {
      t.face_iperm[i] = order[i];
      t.face_perm[order[i]] = (int32_t)i;
    }
  } else {
    set_error("unknown renumbering %d", renumber);
    return CR_E_INVAL;
  }
  auto bandwidth = [&](const std::vector<int32_t>& pos) {
    int64_t bw = 0;
    for (int64_t f = 0; f < nf; ++f)
      for (int64_t e = ptr[f]; e < ptr[f + 1]; ++e) bw = std::max<int64_t>(bw, std::llabs((int64_t)pos[f] - pos[adj[e]]));
    return bw;
  };
  {
    std::vector<int32_t> ident(nf);
    std::iota(ident.begin(), ident.end(), 0);
    t.bw_canonical = bandwidth(ident);
    t.bw_internal = bandwidth(t.face_perm);
  }

  // element order: with aggregates, the locality order above (the elements
  // whose faces lie in more than one aggregate last within the range of their
  // aggregate, so that few wavefronts of the element kernel handle the coarse
  // term); otherwise by smallest internal face id, ties by caller id
  {
    std::vector<int64_t> key(ne);
    for (int64_t k = 0; k < ne; ++k) {
      int64_t m = INT64_MAX;
      int a0 = -1;
      bool multi = false;
      for (int j = 0; j < d1; ++j) {
        int f = t.elem_face[k * d1 + j];
        if (f < 0) continue;
        m = std::min<int64_t>(m, t.face_perm[f]);
        if (t.nagg > 0) {
          const int a = t.face_agg[t.face_perm[f]];
          if (a0 < 0) a0 = a;
          else if (a != a0) multi = true;
        }
      }
      key[k] = t.nagg > 0 ? (int64_t)t.face_agg[m] * 2 * nf + (multi ? nf : 0) + m : m;
    }
    t.elem_iperm.resize(ne);
    std::iota(t.elem_iperm.begin(), t.elem_iperm.end(), 0);
    if (!loc_elem_order.empty())
      t.elem_iperm = loc_elem_order;
    else
      std::stable_sort(t.elem_iperm.begin(), t.elem_iperm.end(), [&](int a, int b) { return key[a] < key[b]; });
    t.elem_perm.resize(ne);
    for (int64_t i = 0; i < ne; ++i) t.elem_perm[t.elem_iperm[i]] = (int32_t)i;
  }

  // M1: greedy maximal independent set in caller order (Section 3.2 item 7)
  t.m1.assign(ne, 0);
  if (need_m1) {
    for (int64_t k = 0; k < ne; ++k) {
      bool free_ = true;
      for (int j = 0; j < d1 && free_; ++j) {
        int f = t.elem_face[k * d1 + j];
        if (f < 0) continue;
        int other = t.face_elem[2 * f] == k ? t.face_elem[2 * f + 1] : t.face_elem[2 * f];
        if (t.m1[other]) free_ = false;
      }
      t.m1[k] = free_ ? 1 : 0;
    }
  }
  return CR_OK;
}

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

void clear_error() { g_err.clear(); }

const char* last_error_str() { return g_err.c_str(); }

}  // namespace crh
