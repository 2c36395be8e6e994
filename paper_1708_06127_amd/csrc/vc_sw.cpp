// Host exact minimum cut of the small remaining ("kernel") graph by
// Stoer-Wagner maximum-adjacency phases, with fixed tie rules so that the
// chosen side is unique:
//   * every phase starts at the smallest surviving vertex id;
//   * the next vertex is the one most tightly connected to the set built so
//     far, ties to the smallest id;
//   * s = second-to-last, t = last vertex of the phase; the cut-of-the-phase
//     is t's connection weight; t is merged into s (s keeps its id);
//   * the side is the set of kernel vertices merged into t at the first phase
//     whose cut-of-the-phase is strictly smaller than all before.
// Adjacency lists are merged lazily: an entry's endpoint is resolved through
// the merge forest when read, and entries that resolve to the vertex itself
// are skipped. Connection weights live in an indexed binary max-heap with
// increase-key.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "vc_internal.h"

namespace vc {
namespace {

struct MaxHeap {  // keys (conn, -id): larger conn first, then smaller id
  std::vector<int32_t> heap, pos;
  const std::vector<int64_t> *conn = nullptr;
  bool before(int32_t a, int32_t b) const {
    int64_t ca = (*conn)[a], cb = (*conn)[b];
    return ca > cb || (ca == cb && a < b);
  }
  void reset(int32_t n) { heap.clear(); pos.assign(n, -1); }
  void swap_at(size_t i, size_t j) {
    std::swap(heap[i], heap[j]);
    pos[heap[i]] = (int32_t)i;
    pos[heap[j]] = (int32_t)j;
  }
  void up(size_t i) {
    while (i > 0) {
      size_t p = (i - 1) / 2;
      if (!before(heap[i], heap[p])) break;
      swap_at(i, p);
      i = p;
    }
  }
  void down(size_t i) {
    while (true) {
      size_t l = 2 * i + 1, r = l + 1, b = i;
      if (l < heap.size() && before(heap[l], heap[b])) b = l;
      if (r < heap.size() && before(heap[r], heap[b])) b = r;
      if (b == i) break;
      swap_at(i, b);
      i = b;
    }
  }
  void push(int32_t v) {
    pos[v] = (int32_t)heap.size();
    heap.push_back(v);
    up(heap.size() - 1);
  }
  void increased(int32_t v) { up((size_t)pos[v]); }
  bool contains(int32_t v) const { return pos[v] >= 0; }
  int32_t pop() {
    int32_t top = heap[0];
    swap_at(0, heap.size() - 1);
    heap.pop_back();
    pos[top] = -1;
    if (!heap.empty()) down(0);
    return top;
  }
};

}  // namespace

int64_t stoer_wagner_host(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w, uint8_t *side) {
  struct Arc { int32_t to; int64_t w; };
  std::vector<std::vector<Arc>> adj(n);
  for (int32_t v = 0; v < n; v++) {
    adj[v].reserve(row_ptr[v + 1] - row_ptr[v]);
    for (int32_t i = row_ptr[v]; i < row_ptr[v + 1]; i++) adj[v].push_back({col[i], (int64_t)w[i]});
  }
  std::vector<int32_t> up(n);  // merge forest: up[v] == v for surviving vertices
  for (int32_t v = 0; v < n; v++) up[v] = v;
  auto find = [&](int32_t x) {
    while (up[x] != x) { up[x] = up[up[x]]; x = up[x]; }
    return x;
  };
  std::vector<int64_t> conn(n, 0);
  std::vector<uint8_t> added(n, 0);
  std::vector<size_t> clean(n, 0);  // list length after the last compaction
  MaxHeap hp;
  hp.conn = &conn;
  std::vector<std::pair<int32_t, int32_t>> merges;  // (s, t) per phase
  int64_t best = INT64_MAX;
  int32_t best_phase = -1, best_t = -1;
  int32_t alive = n;
  int32_t first_alive = 0;
  while (alive > 1) {
    while (up[first_alive] != first_alive) first_alive++;
    hp.reset(n);
    for (int32_t v = first_alive; v < n; v++) {
      if (up[v] != v) continue;
      conn[v] = 0;
      added[v] = 0;
      if (v != first_alive) hp.push(v);
    }
    auto add = [&](int32_t x) {
      added[x] = 1;
      for (const Arc &a : adj[x]) {
        int32_t y = find(a.to);
        if (y == x || added[y]) continue;
        conn[y] += a.w;
        hp.increased(y);
      }
    };
    int32_t s = first_alive, t = first_alive;
    add(first_alive);
    int64_t cut_of_phase = 0;
    while (!hp.heap.empty()) {
      int32_t x = hp.pop();
      s = t;
      t = x;
      cut_of_phase = conn[x];
      add(x);
    }
    if (cut_of_phase < best) {
      best = cut_of_phase;
      best_phase = (int32_t)merges.size();
      best_t = t;
    }
    // merge t into s: s inherits t's adjacency (resolved lazily)
    up[t] = s;
    if (adj[t].size() > adj[s].size()) adj[s].swap(adj[t]);
    adj[s].insert(adj[s].end(), adj[t].begin(), adj[t].end());
    std::vector<Arc>().swap(adj[t]);
    // compact s's list when it has doubled since its last compaction (amortised)
    if (adj[s].size() > 2 * clean[s] + 64) {
      std::vector<Arc> &L = adj[s];
      for (Arc &a : L) a.to = find(a.to);
      std::sort(L.begin(), L.end(), [](const Arc &a, const Arc &b) { return a.to < b.to; });
      size_t o = 0;
      for (size_t i = 0; i < L.size(); i++) {
        if (L[i].to == s) continue;
        if (o > 0 && L[o - 1].to == L[i].to) L[o - 1].w += L[i].w;
        else L[o++] = L[i];
      }
      L.resize(o);
      clean[s] = o;
    }
    merges.push_back({s, t});
    alive--;
  }
  // side: vertices merged into best_t by the merges before the best phase
  std::vector<int32_t> rep(n);
  for (int32_t v = 0; v < n; v++) rep[v] = v;
  auto rfind = [&](int32_t x) {
    while (rep[x] != x) { rep[x] = rep[rep[x]]; x = rep[x]; }
    return x;
  };
  for (int32_t i = 0; i < best_phase; i++) rep[merges[i].second] = merges[i].first;
  for (int32_t v = 0; v < n; v++) side[v] = (best_t >= 0 && rfind(v) == best_t) ? 1 : 0;
  return best;
}

}  // namespace vc
