// Host-side memory and undefined-behaviour check of the face topology, the
// renumbering and the aggregates (topology.cpp), built with g++ and
// -fsanitize=address,undefined by tests/test_host_sanitizers.py.  Runs
// build_topology on structured, jittered and shuffled meshes (2D and 3D, every
// combination of renumbering, M1/M2 split and aggregation) and on invalid
// meshes, and checks structural invariants of the result; exits non-zero on a
// failed invariant (the sanitizers abort on their own findings).
#include <algorithm>
#include <cstdio>
#include <numeric>
#include <random>
#include <vector>

#include "../../paper_2101_03777_amd/csrc/internal.h"

using namespace crh;

namespace {

int failures = 0;

void fail(const char* what, int d, int64_t ne) {
  std::printf("FAIL %s (dim %d, %lld elements)\n", what, d, (long long)ne);
  ++failures;
}

void shuffle_elements(int d, std::vector<int32_t>& e, std::mt19937& g) {
  const int nv = d + 1;
  const int ne = (int)e.size() / nv;
  std::vector<int> p(ne);
  std::iota(p.begin(), p.end(), 0);
  std::shuffle(p.begin(), p.end(), g);
  std::vector<int32_t> out;
  out.reserve(e.size());
  for (int k : p) {
    std::vector<int32_t> t(e.begin() + (size_t)k * nv, e.begin() + (size_t)(k + 1) * nv);
    std::shuffle(t.begin(), t.end(), g);
    out.insert(out.end(), t.begin(), t.end());
  }
  e.swap(out);
}

// n x n squares, two triangles each, interior vertices jittered by 0.2 h
void square(int n, std::vector<double>& c, std::vector<int32_t>& e, std::mt19937& g) {
  std::uniform_real_distribution<double> u(-0.2, 0.2);
  c.clear();
  e.clear();
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) {
      double x = (double)i / n, y = (double)j / n;
      if (i > 0 && i < n && j > 0 && j < n) {
        x += u(g) / n;
        y += u(g) / n;
      }
      c.push_back(x);
      c.push_back(y);
    }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const int a = j * (n + 1) + i, b = a + 1, q = a + n + 1, r = q + 1;
      e.insert(e.end(), {a, b, r});
      e.insert(e.end(), {a, r, q});
    }
}

// n^3 cubes, six Kuhn tetrahedra each
void cube(int n, std::vector<double>& c, std::vector<int32_t>& e) {
  c.clear();
  e.clear();
  auto id = [n](int i, int j, int k) { return (k * (n + 1) + j) * (n + 1) + i; };
  for (int k = 0; k <= n; ++k)
    for (int j = 0; j <= n; ++j)
      for (int i = 0; i <= n; ++i) {
        c.push_back((double)i / n);
        c.push_back((double)j / n);
        c.push_back((double)k / n);
      }
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (const auto& p : perms) {
          int x[3] = {i, j, k};
          int32_t t[4];
          t[0] = id(x[0], x[1], x[2]);
          for (int s = 0; s < 3; ++s) {
            ++x[p[s]];
            t[s + 1] = id(x[0], x[1], x[2]);
          }
          e.insert(e.end(), t, t + 4);
        }
}

bool is_permutation(const std::vector<int32_t>& p, int64_t n) {
  if ((int64_t)p.size() != n) return false;
  std::vector<char> seen(n, 0);
  for (int32_t v : p) {
    if (v < 0 || v >= n || seen[v]) return false;
    seen[v] = 1;
  }
  return true;
}

// every combination of the options; expect_ok: a valid mesh, and its interior
// face count when known (-1: not known)
void check_mesh(int d, const std::vector<double>& c, const std::vector<int32_t>& e, bool expect_ok, int64_t nf_expect) {
  cr_mesh_desc m{};
  m.dim = d;
  m.n_vertices = (int64_t)c.size() / d;
  m.coords = c.data();
  m.n_elements = (int64_t)e.size() / (d + 1);
  m.elem_vertices = e.data();
  const int64_t ne = m.n_elements;
  for (int ren = 0; ren < 2; ++ren)
    for (int m1 = 0; m1 < 2; ++m1)
      for (int ag = 0; ag < 2; ++ag) {
        Topology t;
        const cr_status st = build_topology(&m, ren, m1 != 0, ag != 0, t);
        if (!expect_ok) {
          if (st == CR_OK) fail("invalid mesh accepted", d, ne);
          continue;
        }
        if (st != CR_OK) {
          fail("valid mesh refused", d, ne);
          continue;
        }
        if (nf_expect >= 0 && t.nf != nf_expect) fail("interior face count", d, ne);
        if (2 * t.nf + t.nbf != ne * (d + 1)) fail("face slots", d, ne);
        if (!is_permutation(t.face_perm, t.nf) || !is_permutation(t.face_iperm, t.nf)) fail("face permutation", d, ne);
        if (!is_permutation(t.elem_perm, ne) || !is_permutation(t.elem_iperm, ne)) fail("element permutation", d, ne);
        for (int64_t f = 0; f < t.nf && failures == 0; ++f) {
          if (t.face_iperm[t.face_perm[f]] != f) fail("face inverse permutation", d, ne);
          const int32_t K = t.face_elem[2 * f], L = t.face_elem[2 * f + 1];
          if (!(0 <= K && K < L && L < ne)) fail("face elements", d, ne);
          for (int s = 0; s < 2; ++s) {
            const int32_t el = t.face_elem[2 * f + s];
            const int j = t.face_loc[2 * f + s];
            if (j < 0 || j > d || t.elem_face[(size_t)el * (d + 1) + j] != f) fail("element-face table", d, ne);
            // the face is the element's facet opposite local vertex j
            for (int q = 0; q < d; ++q) {
              const int32_t v = t.face_vertices[(size_t)f * d + q];
              bool in = false;
              for (int r = 0; r <= d; ++r)
                if (r != j && e[(size_t)el * (d + 1) + r] == v) in = true;
              if (!in) fail("face vertices", d, ne);
            }
          }
        }
        for (int64_t k = 0; k < ne; ++k)
          if (t.elem_iperm[t.elem_perm[k]] != k) fail("element inverse permutation", d, ne);
        if (ag && t.nagg > 0) {
          if (t.nagg > MAX_AGG || (int64_t)t.face_agg.size() != t.nf) fail("aggregate table", d, ne);
          for (int64_t f = 0; f < t.nf; ++f) {
            if (t.face_agg[f] < 0 || t.face_agg[f] >= t.nagg) fail("aggregate id", d, ne);
            if (f > 0 && t.face_agg[f] < t.face_agg[f - 1]) fail("aggregates not contiguous", d, ne);
          }
        }
      }
}

}  // namespace

int main() {
  std::mt19937 g(7);
  std::vector<double> c;
  std::vector<int32_t> e;
  for (int n : {1, 2, 3, 8, 24, 64, 100, 128}) {
    square(n, c, e, g);
    check_mesh(2, c, e, true, 3LL * n * n - 2LL * n);
    shuffle_elements(2, e, g);
    check_mesh(2, c, e, true, 3LL * n * n - 2LL * n);
  }
  for (int n : {1, 2, 5, 12, 24}) {
    cube(n, c, e);
    check_mesh(3, c, e, true, 12LL * n * n * n - 6LL * n * n);
    shuffle_elements(3, e, g);
    check_mesh(3, c, e, true, 12LL * n * n * n - 6LL * n * n);
  }
  square(4, c, e, g);
  {
    std::vector<int32_t> bad = e;  // a face shared by three elements
    bad.insert(bad.end(), e.begin(), e.begin() + 3);
    check_mesh(2, c, bad, false, -1);
  }
  {
    std::vector<int32_t> bad = e;  // repeated vertex
    bad[1] = bad[0];
    check_mesh(2, c, bad, false, -1);
  }
  {
    std::vector<int32_t> bad = e;  // vertex ids out of range
    bad[2] = 1000;
    check_mesh(2, c, bad, false, -1);
    bad[2] = -1;
    check_mesh(2, c, bad, false, -1);
  }
  {
    std::vector<int32_t> none;
    check_mesh(2, c, none, false, -1);
  }
  cube(2, c, e);
  {
    std::vector<int32_t> bad = e;  // a flat tetrahedron: four vertices of the plane z = 0
    const int32_t flat[4] = {0, 1, 3, 4};
    std::copy(flat, flat + 4, bad.begin());
    check_mesh(3, c, bad, false, -1);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
