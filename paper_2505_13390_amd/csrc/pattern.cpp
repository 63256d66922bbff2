// Host construction of the fixed sparsity pattern of A (Sec. 4.2: the matrix
// structure depends on the topology only, so it is built once). Row c and
// row d are coupled iff their constraints share a vertex; the pattern keeps
// such entries even when their value is zero (a shared pinned vertex).
// Built with one std::thread per hardware thread over row ranges.
#include <algorithm>
#include <thread>

#include "xpbd.hpp"

namespace mgpbd {

namespace {

template <class F>
void parallel_rows(int64_t m, F f) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (m < 4096) nt = 1;
  std::vector<std::thread> th;
  int64_t per = (m + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t lo = t * per, hi = std::min<int64_t>(m, lo + per);
    if (lo >= hi) break;
    th.emplace_back([=, &f] { f(lo, hi); });
  }
  for (auto &x : th) x.join();
}

}  // namespace

void build_topology(int64_t n_verts, int64_t n_tets, const int32_t *tets, int64_t n_edges,
                    const int32_t *edges, int64_t n_vols, const int32_t *vol_tet,
                    int64_t n_arap, const int32_t *arap_tet, Topology &t) {
  MG_REQUIRE(n_verts > 0 && n_verts < (int64_t)INT32_MAX, MGPBD_E_INVALID_ARG, "n_verts out of range");
  MG_REQUIRE(n_edges >= 0 && n_vols >= 0 && n_arap >= 0 && n_tets >= 0, MGPBD_E_INVALID_ARG,
             "negative size");
  t.n_verts = n_verts;
  t.n_edges = n_edges;
  t.n_vols = n_vols;
  t.n_arap = n_arap;
  t.m = n_edges + n_vols + n_arap;
  const int64_t m = t.m;
  MG_REQUIRE(m < (int64_t)INT32_MAX, MGPBD_E_INVALID_ARG, "too many constraint rows");
  t.rv.assign(4 * (size_t)m, -1);
  for (int64_t e = 0; e < n_edges; ++e) {
    int32_t i = edges[2 * e], j = edges[2 * e + 1];
    MG_REQUIRE(i >= 0 && j < n_verts && i < j, MGPBD_E_INVALID_ARG,
               "edge " + std::to_string(e) + " not (i < j) in range");
    if (e > 0) {
      int32_t pi = edges[2 * e - 2], pj = edges[2 * e - 1];
      MG_REQUIRE(pi < i || (pi == i && pj < j), MGPBD_E_INVALID_ARG,
                 "edges not strictly ascending at " + std::to_string(e));
    }
    t.rv[4 * e] = i;
    t.rv[4 * e + 1] = j;
  }
  // tet rows: the volume rows, then the ARAP rows
  for (int64_t q = 0; q < n_vols + n_arap; ++q) {
    const bool vol = q < n_vols;
    int32_t tt = vol ? vol_tet[q] : arap_tet[q - n_vols];
    MG_REQUIRE(tt >= 0 && tt < n_tets, MGPBD_E_INVALID_ARG,
               vol ? "vol_tet index out of range" : "arap_tet index out of range");
    int64_t r = n_edges + q;
    for (int k = 0; k < 4; ++k) {
      int32_t v = tets[4 * (int64_t)tt + k];
      MG_REQUIRE(v >= 0 && v < n_verts, MGPBD_E_INVALID_ARG, "tet vertex out of range");
      t.rv[4 * r + k] = v;
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        MG_REQUIRE(t.rv[4 * r + a] != t.rv[4 * r + b], MGPBD_E_INVALID_ARG, "degenerate tet");
  }
  auto arity = [&](int64_t r) { return r < n_edges ? 2 : 4; };
  // vertex -> (row, slot), rows ascending
  t.vptr.assign(n_verts + 1, 0);
  for (int64_t r = 0; r < m; ++r)
    for (int k = 0; k < arity(r); ++k) t.vptr[t.rv[4 * r + k] + 1]++;
  for (int64_t v = 0; v < n_verts; ++v) t.vptr[v + 1] += t.vptr[v];
  t.vrow.resize(t.vptr[n_verts]);
  t.vslot.resize(t.vptr[n_verts]);
  {
    std::vector<int64_t> cur(t.vptr.begin(), t.vptr.end() - 1);
    for (int64_t r = 0; r < m; ++r)
      for (int k = 0; k < arity(r); ++k) {
        int32_t v = t.rv[4 * r + k];
        t.vrow[cur[v]] = (int32_t)r;
        t.vslot[cur[v]] = (int8_t)k;
        cur[v]++;
      }
  }
  // pattern rows: neighbour rows through each vertex, sorted and unique
  auto row_neighbours = [&](int64_t r, std::vector<int32_t> &buf) {
    buf.clear();
    for (int k = 0; k < arity(r); ++k) {
      int32_t v = t.rv[4 * r + k];
      for (int64_t e = t.vptr[v]; e < t.vptr[v + 1]; ++e) buf.push_back(t.vrow[e]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
  };
  std::vector<int64_t> cnt(m + 1, 0);
  parallel_rows(m, [&](int64_t lo, int64_t hi) {
    std::vector<int32_t> buf;
    for (int64_t r = lo; r < hi; ++r) {
      row_neighbours(r, buf);
      cnt[r + 1] = (int64_t)buf.size();
    }
  });
  t.rowptr.assign(m + 1, 0);
  for (int64_t r = 0; r < m; ++r) t.rowptr[r + 1] = t.rowptr[r] + cnt[r + 1];
  t.nnz = t.rowptr[m];
  t.col.resize(t.nnz);
  t.meta.resize(t.nnz);
  parallel_rows(m, [&](int64_t lo, int64_t hi) {
    std::vector<int32_t> buf;
    for (int64_t c = lo; c < hi; ++c) {
      row_neighbours(c, buf);
      int kc = arity(c);
      // slots of c in ascending vertex id
      int ord[4] = {0, 1, 2, 3};
      for (int a = 1; a < kc; ++a)
        for (int q = a; q > 0 && t.rv[4 * c + ord[q - 1]] > t.rv[4 * c + ord[q]]; --q)
          std::swap(ord[q], ord[q - 1]);
      int64_t e = t.rowptr[c];
      for (int32_t d : buf) {
        uint32_t code = 0;
        if (d != c) {
          int kd = arity(d), nsh = 0;
          for (int a = 0; a < kc; ++a) {
            int sc = ord[a];
            int32_t v = t.rv[4 * c + sc];
            for (int sd = 0; sd < kd; ++sd)
              if (t.rv[4 * (int64_t)d + sd] == v) {
                code |= (uint32_t)(sc | (sd << 2)) << (3 + 4 * nsh);
                ++nsh;
              }
          }
          code |= (uint32_t)nsh;
        }
        t.col[e] = d;
        t.meta[e] = code;
        ++e;
      }
    }
  });
}

}  // namespace mgpbd
