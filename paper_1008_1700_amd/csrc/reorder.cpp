// Host-side preparation of general sparse matrices for the banded block
// path: reverse Cuthill-McKee ordering, the symmetric permutation of a CSR
// matrix, its half-bandwidth, and the equal-slab row partition that
// ddps_setup accepts.  Plain C++; no GPU work.
//
// Reverse Cuthill-McKee (Cuthill & McKee 1969, reversed as George proposed):
// a breadth-first numbering of the graph of A + A^T in which the neighbours
// of each node are numbered in increasing degree, started from a
// pseudo-peripheral node (George & Liu 1979: repeat a breadth-first search
// from a node of least degree in the last level while that raises the
// eccentricity), then read backwards.  The levels of the search become
// contiguous index ranges, so every edge joins the same or adjacent levels
// and the bandwidth is bounded by two level widths.
#include "../../include/ddps.h"

#include <algorithm>
#include <cstdint>
#include <vector>

namespace {

struct Graph {
  std::vector<int64_t> ptr;   // n + 1
  std::vector<int64_t> adj;   // neighbours, sorted, no self loops, no repeats
  int64_t deg(int64_t v) const { return ptr[v + 1] - ptr[v]; }
};

// Adjacency of the symmetric pattern A + A^T without the diagonal.
bool build_graph(int64_t n, const int64_t* row_ptr, const int32_t* col, Graph& g) {
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int64_t j = col[q];
      if (j < 0 || j >= n) return false;
      if (j == i) continue;
      ++cnt[i];
      ++cnt[j];
    }
  std::vector<int64_t> ptr(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] = ptr[i] + cnt[i];
  std::vector<int64_t> adj(ptr[n]);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int64_t j = col[q];
      if (j == i) continue;
      adj[fill[i]++] = j;
      adj[fill[j]++] = i;
    }
  // sort and drop repeats (an entry present in both A and A^T)
  g.ptr.assign(n + 1, 0);
  g.adj.clear();
  g.adj.reserve(adj.size());
  for (int64_t i = 0; i < n; ++i) {
    auto b = adj.begin() + ptr[i], e = adj.begin() + ptr[i + 1];
    std::sort(b, e);
    e = std::unique(b, e);
    g.adj.insert(g.adj.end(), b, e);
    g.ptr[i + 1] = (int64_t)g.adj.size();
  }
  return true;
}

// Breadth-first level structure from r inside the unmarked part of the
// graph: returns the nodes in visiting order and the start of each level.
void levels_from(const Graph& g, int64_t r, const std::vector<char>& done, std::vector<int64_t>& order,
                 std::vector<int64_t>& level_start, std::vector<int64_t>& stamp, int64_t mark) {
  order.clear();
  level_start.clear();
  order.push_back(r);
  stamp[r] = mark;
  size_t head = 0;
  while (head < order.size()) {
    level_start.push_back((int64_t)head);
    const size_t end = order.size();
    for (; head < end; ++head) {
      const int64_t v = order[head];
      for (int64_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q) {
        const int64_t w = g.adj[q];
        if (!done[w] && stamp[w] != mark) {
          stamp[w] = mark;
          order.push_back(w);
        }
      }
    }
  }
}

}  // namespace

extern "C" {

int ddps_rcm(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* perm) {
  if (n < 0) return DDPS_E_ARG;
  if (n == 0) return DDPS_OK;
  if (!row_ptr || !perm || (row_ptr[n] > 0 && !col)) return DDPS_E_ARG;
  Graph g;
  if (!build_graph(n, row_ptr, col, g)) return DDPS_E_ARG;
  std::vector<char> done(n, 0);
  std::vector<int64_t> stamp(n, -1), order, level_start, cm;
  cm.reserve(n);
  int64_t mark = 0;
  std::vector<int64_t> nbr;
  for (int64_t s0 = 0; s0 < n; ++s0) {
    if (done[s0]) continue;
    // the component of s0, and a node of least degree in it
    levels_from(g, s0, done, order, level_start, stamp, mark++);
    int64_t r = order[0];
    for (int64_t v : order)
      if (g.deg(v) < g.deg(r) || (g.deg(v) == g.deg(r) && v < r)) r = v;
    // pseudo-peripheral node: move to a least-degree node of the last level
    // while the eccentricity grows
    levels_from(g, r, done, order, level_start, stamp, mark++);
    int64_t ecc = (int64_t)level_start.size();
    for (;;) {
      int64_t x = -1;
      for (size_t q = (size_t)level_start.back(); q < order.size(); ++q) {
        const int64_t v = order[q];
        if (x < 0 || g.deg(v) < g.deg(x) || (g.deg(v) == g.deg(x) && v < x)) x = v;
      }
      levels_from(g, x, done, order, level_start, stamp, mark++);
      const int64_t ecc_x = (int64_t)level_start.size();
      if (ecc_x > ecc) {
        r = x;
        ecc = ecc_x;
      } else {
        break;
      }
    }
    // Cuthill-McKee numbering from r: neighbours in increasing degree
    const size_t base = cm.size();
    cm.push_back(r);
    done[r] = 1;
    for (size_t head = base; head < cm.size(); ++head) {
      const int64_t v = cm[head];
      nbr.clear();
      for (int64_t q = g.ptr[v]; q < g.ptr[v + 1]; ++q)
        if (!done[g.adj[q]]) nbr.push_back(g.adj[q]);
      std::sort(nbr.begin(), nbr.end(), [&](int64_t a, int64_t b) {
        return g.deg(a) != g.deg(b) ? g.deg(a) < g.deg(b) : a < b;
      });
      for (int64_t w : nbr) {
        done[w] = 1;
        cm.push_back(w);
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) perm[i] = cm[n - 1 - i];
  return DDPS_OK;
}

int ddps_bandwidth(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* b) {
  if (n < 0 || !b || (n > 0 && !row_ptr) || (n > 0 && row_ptr[n] > 0 && !col)) return DDPS_E_ARG;
  int64_t bw = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      const int64_t j = col[q];
      if (j < 0 || j >= n) return DDPS_E_ARG;
      bw = std::max(bw, j > i ? j - i : i - j);
    }
  *b = bw;
  return DDPS_OK;
}

int ddps_permute_csr(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                     const int64_t* perm, int64_t* out_row_ptr, int32_t* out_col, double* out_val) {
  if (n < 0 || (n > 0 && (!row_ptr || !perm || !out_row_ptr))) return DDPS_E_ARG;
  if (n == 0) {
    if (out_row_ptr) out_row_ptr[0] = 0;
    return DDPS_OK;
  }
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && (!col || !out_col)) return DDPS_E_ARG;
  std::vector<int64_t> inv(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = perm[i];
    if (o < 0 || o >= n || inv[o] >= 0) return DDPS_E_ARG;   // not a permutation
    inv[o] = i;
  }
  out_row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = perm[i];
    out_row_ptr[i + 1] = out_row_ptr[i] + (row_ptr[o + 1] - row_ptr[o]);
  }
  std::vector<std::pair<int64_t, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t o = perm[i];
    row.clear();
    for (int64_t q = row_ptr[o]; q < row_ptr[o + 1]; ++q) {
      const int64_t j = col[q];
      if (j < 0 || j >= n) return DDPS_E_ARG;
      row.emplace_back(inv[j], val ? val[q] : 0.0);
    }
    std::sort(row.begin(), row.end(),
              [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
    int64_t w = out_row_ptr[i];
    for (const auto& e : row) {
      out_col[w] = (int32_t)e.first;
      if (out_val) out_val[w] = e.second;
      ++w;
    }
  }
  return DDPS_OK;
}

int ddps_partition_rows(int64_t n, int64_t b, int32_t p_max, int64_t* part_ptr, int32_t* p) {
  if (n < 1 || b < 0 || p_max < 1 || !part_ptr || !p) return DDPS_E_ARG;
  const int64_t t = std::max<int64_t>(64, (b + 63) / 64 * 64);
  const int64_t np = std::max<int64_t>(1, std::min<int64_t>(p_max, n / (2 * t)));
  const int64_t q = n / np, rem = n % np;
  part_ptr[0] = 0;
  for (int64_t i = 0; i < np; ++i) part_ptr[i + 1] = part_ptr[i] + q + (i < rem ? 1 : 0);
  *p = (int32_t)np;
  return DDPS_OK;
}

}  // extern "C"
