// CPU ORACLE - TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU implementation of the synchronous
// inexact minimum-cut method (label-propagation cluster contraction,
// Padberg-Rinaldi contraction, minimum-degree upper bound, exact
// Stoer-Wagner solve on the remaining kernel graph, solution transfer).
// It exists only so that tests, the smoke check and the benchmark's CPU
// baseline can check and time the GPU library against it. It shares no code,
// header or table with the GPU library, and nothing in the GPU library may
// call it.
//
// Paper references are to Henzinger, Noe, Schulz, Strash, "Practical Minimum
// Cut Algorithms" (arXiv 1708.06127):
//   * problem statement, cut capacity, lambda, trivial cut bound:  Section 3
//     "Preliminaries";
//   * upper bound lambda-hat = minimum weighted degree, lowered after every
//     contraction:  Section 4 (introduction);
//   * label propagation clustering, iterations capped at l:  Section 4.1;
//   * cluster contraction, Lemma 1:  Section 4.1;
//   * Padberg-Rinaldi conditions 1-4:  Lemma "Padberg-Rinaldi", Section 4.1;
//   * union-find contraction of marked edges:  Section 4.1;
//   * isolated vertex => lambda = 0:  Section 4.1 and the proof of Lemma 3;
//   * the outer loop and solution transfer:  Algorithm 1 (appendix A).
//
// Readings taken where the paper leaves the method open (each one the same
// in the GPU library, which implements them independently):
//   * LP is synchronous: iteration t reads only the labels of iteration t-1;
//     every round starts again from singleton labels.
//   * LP tie-break: keep the current label if it attains the maximum;
//     otherwise take the maximiser x with the smallest (prio(x), x), where
//     prio(x) = fmix32(uint32(x) XOR low32(s)), fmix32 is MurmurHash3's
//     32-bit finaliser (Appleby) and s is output number r*l + t of a SplitMix64
//     generator (Steele, Lea, Flood 2014) started at the seed.
//   * PR conditions 2 and 3 are tested with strict '<' (all marked edges are
//     contracted at once); 1 and 4 keep '>= lambda-hat'. Conditions 3 and 4 are
//     tested on every edge against its full common neighbourhood. The
//     "only edge" guard of the lemma is not applied.
//   * lambda-hat is lowered only on a strictly smaller minimum degree; the
//     witness is the smallest vertex id attaining it at the earliest level.
//   * The correcting step (fixing misplaced vertices; Section 4.1 and
//     Algorithm 1's fixMisplacedVertices) runs only when asked for (flag 1).
//     Reading: after label propagation, a cluster C with
//     2 <= |C| <= floor(log2 n) (n: vertices of the current graph) loses at
//     most one vertex: the member v whose removal leaves C minus {v} with the
//     smallest weighted degree in the contracted graph (smallest v on ties),
//     and only if that degree is strictly below the minimum weighted degree of
//     the contracted graph without any correction. The removed vertex becomes
//     a singleton cluster with label n + v, so coarse ids follow the ordinary
//     labels first and then the corrected vertices in ascending id.
//   * Label-propagation variants (Section 4.1 and appendix D, "Algorithm
//     Configuration"), each only when asked for:
//     - convergence stop (flag 2): iteration t is the last one when at most
//       floor(n / 10000) vertices (n: vertices of the current graph) got a
//       label different from the one they had before iteration t, else the
//       iterations run on up to l;
//     - first-iteration restriction (flag 4), a synchronous reading of the
//       rule that a vertex may not leave its block once another vertex has
//       moved into it: after the first iteration of a round, every vertex
//       that some other vertex chose (as its new label) keeps its own label;
//       the others keep their choice. Unlike the sequential rule this does
//       not bound the cluster count by n / 2 (two vertices that choose each
//       other both stay).
//   * The exact solve is Stoer-Wagner: every phase starts at the smallest
//     surviving id, maximum-adjacency ties go to the smallest id, the last
//     vertex t is merged into the second-to-last s (s keeps its id), and the
//     first phase attaining a strictly smaller cut-of-the-phase gives the side
//     (the original kernel vertices merged into t).
//   * The returned side bitmap never contains vertex 0.
//
// Built with g++ -O2 (optionally -fopenmp: the per-vertex label-propagation
// loop is a parallel for whose result does not depend on the thread count).

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <map>
#include <queue>
#include <tuple>
#include <vector>

namespace {

enum {
  OK = 0, E_INVAL = -1, E_WEIGHT = -2, E_OVERFLOW = -3, E_NOTSYM = -6
};
enum { ST_COLLAPSED = 1, ST_DISCONNECTED = 2, ST_NO_PROGRESS = 4, ST_MAX_ROUNDS = 8 };
enum { EV_LP = 1, EV_CONTRACT = 2, EV_BOUND = 3, EV_PR = 4, EV_UF = 5, EV_FIX = 6 };
enum { F_CORRECT = 1, F_CONVERGE = 2, F_RESTRICT = 4 };

}  // namespace

extern "C" {
// One trace record; which arrays are set depends on `kind`:
//   EV_LP       a = labels[n] after iteration `iter` of round `round`
//   EV_CONTRACT a = row_ptr[n+1], b = col[nnz], c = w[nnz], d = deg[n] of the
//               new graph at `level`; e = cl[n_prev] (old vertex -> new vertex)
//   EV_BOUND    lam_hat, witness vertex and level after the update at `level`
//   EV_PR       a = mark[nnz] (1 on both arcs of a marked edge) on the graph at `level`
//   EV_UF       a = rep[n] (smallest vertex id of the marked-edge component)
//   EV_FIX      a = labels[n] after the correcting step of round `round`
typedef struct {
  int32_t kind, round, iter, level;
  int32_t n, n_prev;
  int64_t nnz;
  int64_t lam_hat;
  int32_t witness_vertex, witness_level;
  const int32_t *a, *b, *c;
  const int64_t *d;
  const int32_t *e;
} oracle_event;
typedef void (*oracle_trace_fn)(void *user, const oracle_event *ev);
}

namespace {

struct Graph {            // symmetric CSR, rows sorted by column
  int32_t n = 0;
  std::vector<int64_t> row;  // n+1
  std::vector<int32_t> col;
  std::vector<int64_t> w;
  int64_t arcs() const { return row[n]; }
};

// SplitMix64 (Steele, Lea, Flood 2014): the state advances by the golden
// gamma and each output is the state passed through the variant-13 mixer.
// Output number i (i >= 1) is the i-th value returned after starting at `seed`.
uint64_t splitmix64_output(uint64_t seed, uint64_t i) {
  uint64_t state = seed, z = 0;
  for (uint64_t k = 0; k < i; k++) {
    state += 0x9E3779B97F4A7C15ULL;
    z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
  }
  return z;
}

// MurmurHash3 32-bit finaliser (Appleby).
uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6BU;
  h ^= h >> 13;
  h *= 0xC2B2AE35U;
  h ^= h >> 16;
  return h;
}

uint32_t prio(uint64_t s, int32_t x) { return fmix32((uint32_t)x ^ (uint32_t)(s & 0xFFFFFFFFULL)); }

// Weighted degree c(v): sum of the weights of v's incident edges (Section 3, Preliminaries).
std::vector<int64_t> degrees(const Graph &g) {
  std::vector<int64_t> deg(g.n, 0);
  for (int32_t v = 0; v < g.n; v++)
    for (int64_t i = g.row[v]; i < g.row[v + 1]; i++) deg[v] += g.w[i];
  return deg;
}

// Synchronous label propagation (Section 4.1): l iterations, each computing
// every vertex's new label from the previous iteration's labels only; the
// variants of the flags as read in the file header.
std::vector<int32_t> label_propagation(const Graph &g, int32_t iters, uint64_t seed, int32_t round, uint32_t flags,
                                       oracle_trace_fn cb, void *user) {
  std::vector<int32_t> L(g.n), Lnew(g.n);
  for (int32_t v = 0; v < g.n; v++) L[v] = v;  // every vertex starts in its own cluster
  for (int32_t t = 1; t <= iters; t++) {
    uint64_t s = splitmix64_output(seed, (uint64_t)round * (uint64_t)iters + (uint64_t)t);
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t v = 0; v < g.n; v++) {
      if (g.row[v] == g.row[v + 1]) { Lnew[v] = L[v]; continue; }
      // S(x): total weight from v to neighbours currently labelled x
      std::map<int32_t, int64_t> S;
      for (int64_t i = g.row[v]; i < g.row[v + 1]; i++) S[L[g.col[i]]] += g.w[i];
      int64_t maxS = 0;
      for (const auto &kv : S) maxS = std::max(maxS, kv.second);
      auto own = S.find(L[v]);
      if (own != S.end() && own->second == maxS) { Lnew[v] = L[v]; continue; }
      int32_t best = -1;
      for (const auto &kv : S) {
        if (kv.second != maxS) continue;
        if (best < 0 || std::make_pair(prio(s, kv.first), kv.first) < std::make_pair(prio(s, best), best))
          best = kv.first;
      }
      Lnew[v] = best;
    }
    if (t == 1 && (flags & F_RESTRICT)) {
      // a vertex chosen by another vertex stays where it is
      std::vector<char> chosen(g.n, 0);
      for (int32_t u = 0; u < g.n; u++)
        if (Lnew[u] != L[u]) chosen[Lnew[u]] = 1;  // L is the identity here
      for (int32_t v = 0; v < g.n; v++)
        if (chosen[v]) Lnew[v] = L[v];
    }
    int64_t changed = 0;
    for (int32_t v = 0; v < g.n; v++) changed += Lnew[v] != L[v];
    L.swap(Lnew);
    if (cb) {
      oracle_event ev{};
      ev.kind = EV_LP; ev.round = round; ev.iter = t; ev.n = g.n; ev.a = L.data();
      cb(user, &ev);
    }
    if ((flags & F_CONVERGE) && changed <= g.n / 10000) break;
  }
  return L;
}

// The correcting step (Section 4.1, "correcting algorithm": a misplaced
// vertex is one whose removal from its cluster improves the minimum weighted
// degree of the contracted graph; only clusters of up to log2(n) vertices are
// checked), with the reading in the file header. Weighted degrees of clusters
// are recounted from the arcs for every candidate.
std::vector<int32_t> fix_misplaced(const Graph &g, const std::vector<int32_t> &L) {
  std::map<int32_t, std::vector<int32_t>> members;  // label -> vertices, ascending
  for (int32_t v = 0; v < g.n; v++) members[L[v]].push_back(v);
  // weighted degree of each cluster in the contracted graph
  std::map<int32_t, int64_t> cut;
  for (const auto &kv : members) cut[kv.first] = 0;
  for (int32_t v = 0; v < g.n; v++)
    for (int64_t i = g.row[v]; i < g.row[v + 1]; i++)
      if (L[g.col[i]] != L[v]) cut[L[v]] += g.w[i];
  int64_t delta_c = INT64_MAX;
  for (const auto &kv : cut) delta_c = std::min(delta_c, kv.second);
  int32_t limit = 0;  // floor(log2(n))
  while (((int64_t)1 << (limit + 1)) <= (int64_t)g.n) limit++;
  std::vector<int32_t> out(L);
  for (const auto &kv : members) {
    const std::vector<int32_t> &mem = kv.second;
    if (mem.size() < 2 || (int64_t)mem.size() > limit) continue;
    int64_t best = INT64_MAX;
    int32_t best_v = -1;
    for (int32_t v : mem) {
      // weighted degree of the cluster without v: its edges to every vertex
      // outside it, v included
      int64_t c = 0;
      for (int32_t x : mem) {
        if (x == v) continue;
        for (int64_t i = g.row[x]; i < g.row[x + 1]; i++) {
          const int32_t u = g.col[i];
          if (L[u] != kv.first || u == v) c += g.w[i];
        }
      }
      if (c < best) { best = c; best_v = v; }
    }
    if (best < delta_c) out[best_v] = g.n + best_v;
  }
  return out;
}

// Contract the partition given by `label` (any int32 values): each block
// becomes one vertex, numbered by ascending label value; inter-block weights
// are summed and intra-block edges dropped (Section 4.1, "contract it").
Graph contract(const Graph &g, const std::vector<int32_t> &label, std::vector<int32_t> &cl) {
  std::vector<int32_t> used(label.begin(), label.end());
  std::sort(used.begin(), used.end());
  used.erase(std::unique(used.begin(), used.end()), used.end());
  cl.assign(g.n, 0);
  for (int32_t v = 0; v < g.n; v++)
    cl[v] = (int32_t)(std::lower_bound(used.begin(), used.end(), label[v]) - used.begin());
  int32_t k = (int32_t)used.size();
  std::vector<std::tuple<int32_t, int32_t, int64_t>> t;
  for (int32_t v = 0; v < g.n; v++)
    for (int64_t i = g.row[v]; i < g.row[v + 1]; i++)
      if (cl[v] != cl[g.col[i]]) t.emplace_back(cl[v], cl[g.col[i]], g.w[i]);
  std::sort(t.begin(), t.end());
  Graph h;
  h.n = k;
  h.row.assign(k + 1, 0);
  for (size_t i = 0; i < t.size(); i++) {
    if (!h.col.empty() && i > 0 && std::get<0>(t[i]) == std::get<0>(t[i - 1]) &&
        std::get<1>(t[i]) == std::get<1>(t[i - 1])) {
      h.w.back() += std::get<2>(t[i]);
    } else {
      h.col.push_back(std::get<1>(t[i]));
      h.w.push_back(std::get<2>(t[i]));
      h.row[std::get<0>(t[i]) + 1]++;
    }
  }
  for (int32_t i = 0; i < k; i++) h.row[i + 1] += h.row[i];
  return h;
}

// Padberg-Rinaldi conditions (Lemma "Padberg-Rinaldi"), tested on every edge
// {v, x} with the readings in the file header. Returns a mark per arc,
// set on both arcs of a marked edge.
std::vector<int32_t> pr_marks(const Graph &g, const std::vector<int64_t> &deg, int64_t lam) {
  std::vector<int32_t> mark(g.arcs(), 0);
  for (int32_t v = 0; v < g.n; v++) {
    for (int64_t i = g.row[v]; i < g.row[v + 1]; i++) {
      int32_t x = g.col[i];
      if (x < v) continue;
      int64_t c = g.w[i];
      bool pr1 = c >= lam;
      bool pr2 = deg[v] < 2 * c || deg[x] < 2 * c;
      bool pr3 = false;
      int64_t sum4 = c;
      // common neighbourhood N(v) ∩ N(x) by merging the two sorted rows
      int64_t a = g.row[v], b = g.row[x];
      while (a < g.row[v + 1] && b < g.row[x + 1]) {
        if (g.col[a] < g.col[b]) a++;
        else if (g.col[a] > g.col[b]) b++;
        else {
          int64_t cvu = g.w[a], cxu = g.w[b];
          if (deg[v] < 2 * (c + cvu) && deg[x] < 2 * (c + cxu)) pr3 = true;
          sum4 += std::min(cvu, cxu);
          a++; b++;
        }
      }
      bool pr4 = sum4 >= lam;
      if (pr1 || pr2 || pr3 || pr4) {
        mark[i] = 1;
        for (int64_t j = g.row[x]; j < g.row[x + 1]; j++)
          if (g.col[j] == v) mark[j] = 1;
      }
    }
  }
  return mark;
}

// Connected components of the marked edges; each vertex gets the smallest
// vertex id of its component (graph search, Section 4.1 "union-find").
std::vector<int32_t> marked_components(const Graph &g, const std::vector<int32_t> &mark) {
  std::vector<int32_t> rep(g.n, -1), stack;
  for (int32_t s = 0; s < g.n; s++) {
    if (rep[s] >= 0) continue;
    rep[s] = s;  // ascending scan: s is the smallest id of its component
    stack.push_back(s);
    while (!stack.empty()) {
      int32_t v = stack.back(); stack.pop_back();
      for (int64_t i = g.row[v]; i < g.row[v + 1]; i++)
        if (mark[i] && rep[g.col[i]] < 0) { rep[g.col[i]] = s; stack.push_back(g.col[i]); }
    }
  }
  return rep;
}

// Stoer-Wagner exact minimum cut with the tie rules in the file header.
// Returns the value and a 0/1 flag per vertex of g for the chosen side.
int64_t stoer_wagner(const Graph &g, std::vector<uint8_t> &side) {
  int32_t n = g.n;
  std::vector<std::map<int32_t, int64_t>> adj(n);
  for (int32_t v = 0; v < n; v++)
    for (int64_t i = g.row[v]; i < g.row[v + 1]; i++) adj[v][g.col[i]] += g.w[i];
  std::vector<std::vector<int32_t>> members(n);
  for (int32_t v = 0; v < n; v++) members[v] = {v};
  std::vector<uint8_t> alive(n, 1), in_a(n, 0);
  std::vector<int64_t> conn(n, 0);
  int64_t best = INT64_MAX;
  std::vector<int32_t> best_side;
  int32_t remaining = n;
  while (remaining > 1) {
    int32_t start = 0;
    while (!alive[start]) start++;
    std::priority_queue<std::pair<int64_t, int32_t>> pq;  // (conn, -id): max conn, then min id
    for (int32_t v = 0; v < n; v++) {
      conn[v] = 0;
      in_a[v] = 0;
    }
    in_a[start] = 1;
    for (const auto &kv : adj[start]) conn[kv.first] += kv.second;
    for (int32_t v = 0; v < n; v++)
      if (alive[v] && v != start) pq.push({conn[v], -v});
    int32_t s = start, t = start;
    int64_t cut_of_phase = 0;
    for (int32_t added = 1; added < remaining; added++) {
      int32_t x;
      while (true) {
        auto top = pq.top();
        pq.pop();
        x = -top.second;
        if (!in_a[x] && conn[x] == top.first) break;
      }
      in_a[x] = 1;
      s = t;
      t = x;
      cut_of_phase = conn[x];
      for (const auto &kv : adj[x])
        if (!in_a[kv.first]) { conn[kv.first] += kv.second; pq.push({conn[kv.first], -kv.first}); }
    }
    if (cut_of_phase < best) { best = cut_of_phase; best_side = members[t]; }
    // merge t into s
    for (const auto &kv : adj[t]) {
      int32_t u = kv.first;
      if (u == s) continue;
      adj[s][u] += kv.second;
      adj[u][s] += kv.second;
      adj[u].erase(t);
    }
    adj[s].erase(t);
    adj[t].clear();
    members[s].insert(members[s].end(), members[t].begin(), members[t].end());
    members[t].clear();
    alive[t] = 0;
    remaining--;
  }
  side.assign(n, 0);
  for (int32_t v : best_side) side[v] = 1;
  return best;
}

int validate(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w, bool check_sym) {
  if (n < 2 || !row_ptr) return E_INVAL;
  if (row_ptr[0] != 0) return E_INVAL;
  for (int32_t v = 0; v < n; v++)
    if (row_ptr[v + 1] < row_ptr[v]) return E_INVAL;
  int64_t total = 0;
  for (int32_t v = 0; v < n; v++)
    for (int64_t i = row_ptr[v]; i < row_ptr[v + 1]; i++) {
      if (col[i] < 0 || col[i] >= n || col[i] == v) return E_INVAL;
      if (i > row_ptr[v] && col[i] <= col[i - 1]) return E_INVAL;
      if (w[i] < 1) return E_WEIGHT;
      total += w[i];
    }
  if (total / 2 > INT32_MAX) return E_OVERFLOW;
  if (check_sym) {
    for (int32_t v = 0; v < n; v++)
      for (int64_t i = row_ptr[v]; i < row_ptr[v + 1]; i++) {
        int32_t u = col[i];
        const int32_t *b = col + row_ptr[u], *e = col + row_ptr[u + 1];
        const int32_t *p = std::lower_bound(b, e, v);
        if (p == e || *p != v || w[p - col] != w[i]) return E_NOTSYM;
      }
  }
  return OK;
}

void emit_graph(oracle_trace_fn cb, void *user, int32_t level, const Graph &h, const std::vector<int64_t> &deg,
                const std::vector<int32_t> &cl) {
  if (!cb) return;
  std::vector<int32_t> rp(h.n + 1), w(h.arcs());
  for (int32_t i = 0; i <= h.n; i++) rp[i] = (int32_t)h.row[i];
  for (int64_t i = 0; i < h.arcs(); i++) w[i] = (int32_t)h.w[i];
  oracle_event ev{};
  ev.kind = EV_CONTRACT; ev.level = level; ev.n = h.n; ev.n_prev = (int32_t)cl.size(); ev.nnz = h.arcs();
  ev.a = rp.data(); ev.b = h.col.data(); ev.c = w.data(); ev.d = deg.data(); ev.e = cl.data();
  cb(user, &ev);
}

}  // namespace

extern "C" {

uint64_t oracle_splitmix64_output(uint64_t seed, uint64_t i) { return splitmix64_output(seed, i); }
uint32_t oracle_fmix32(uint32_t h) { return fmix32(h); }
uint32_t oracle_prio(uint64_t s, int32_t x) { return prio(s, x); }

// The correcting step alone on given labels (values in [0, n)); out_labels
// receives the corrected labels (a removed vertex v gets n + v).
int oracle_fix_misplaced(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                         const int32_t *labels, int32_t *out_labels) {
  int rc = validate(n, row_ptr, col, w, true);
  if (rc) return rc;
  for (int32_t v = 0; v < n; v++)
    if (labels[v] < 0 || labels[v] >= n) return E_INVAL;
  Graph g;
  g.n = n;
  g.row.assign(row_ptr, row_ptr + n + 1);
  g.col.assign(col, col + row_ptr[n]);
  g.w.assign(w, w + row_ptr[n]);
  std::vector<int32_t> out = fix_misplaced(g, std::vector<int32_t>(labels, labels + n));
  std::memcpy(out_labels, out.data(), sizeof(int32_t) * (size_t)n);
  return OK;
}

// Exact minimum cut of a CSR graph by Stoer-Wagner (tie rules above).
// side: one byte per vertex, 1 on the returned side (vertex-0 normalisation
// is NOT applied here). Returns 0 or a negative error code.
int oracle_stoer_wagner(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w, int64_t *out_cut,
                        uint8_t *out_side) {
  int rc = validate(n, row_ptr, col, w, true);
  if (rc) return rc;
  Graph g;
  g.n = n;
  g.row.assign(row_ptr, row_ptr + n + 1);
  g.col.assign(col, col + row_ptr[n]);
  g.w.assign(w, w + row_ptr[n]);
  std::vector<uint8_t> side;
  *out_cut = stoer_wagner(g, side);
  std::memcpy(out_side, side.data(), n);
  return OK;
}

// The whole method (Algorithm 1 with the readings above).
// out_side: ceil(n/64) words; bit (u & 63) of word (u >> 6) is 1 iff input
// vertex u is on the side that does not contain vertex 0.
// out_info[0..3] = rounds, kernel_n, witness_level (-1: exact solve), status bits.
int oracle_mincut(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w, int32_t lp_iters,
                  int32_t n0, int32_t max_rounds, uint64_t seed, uint32_t flags, int64_t *out_cut,
                  uint64_t *out_side, int32_t *out_info, oracle_trace_fn cb, void *user) {
  if (lp_iters < 0 || n0 < 0 || max_rounds < 0) return E_INVAL;
  int rc = validate(n, row_ptr, col, w, true);
  if (rc) return rc;
  Graph g;
  g.n = n;
  g.row.assign(row_ptr, row_ptr + n + 1);
  g.col.assign(col, col + row_ptr[n]);
  g.w.assign(w, w + row_ptr[n]);

  std::vector<int32_t> map(n);  // input vertex -> vertex of the current graph
  for (int32_t u = 0; u < n; u++) map[u] = u;
  int32_t level = 0, rounds = 0;
  uint32_t status = 0;

  // lambda-hat starts at the minimum weighted degree (trivial cut bound)
  std::vector<int64_t> deg = degrees(g);
  int64_t lam = INT64_MAX;
  int32_t wit_v = -1, wit_level = 0;
  std::vector<uint8_t> witness(n, 0);
  auto bound_update = [&](int32_t lvl) {
    int64_t mn = INT64_MAX;
    int32_t arg = -1;
    for (int32_t v = 0; v < g.n; v++)
      if (deg[v] < mn) { mn = deg[v]; arg = v; }
    if (mn < lam) {
      lam = mn; wit_v = arg; wit_level = lvl;
      for (int32_t u = 0; u < n; u++) witness[u] = map[u] == arg;
    }
    if (cb) {
      oracle_event ev{};
      ev.kind = EV_BOUND; ev.level = lvl; ev.n = g.n; ev.lam_hat = lam;
      ev.witness_vertex = wit_v; ev.witness_level = wit_level;
      cb(user, &ev);
    }
  };
  bound_update(0);
  bool done = false;
  if (lam == 0) { status |= ST_DISCONNECTED; done = true; }

  auto apply_contraction = [&](const std::vector<int32_t> &label) -> bool {
    std::vector<int32_t> cl;
    Graph h = contract(g, label, cl);
    for (int32_t u = 0; u < n; u++) map[u] = cl[map[u]];
    g = std::move(h);
    level++;
    deg = degrees(g);
    emit_graph(cb, user, level, g, deg, cl);
    if (g.n == 1) { status |= ST_COLLAPSED; return true; }
    bound_update(level);
    if (lam == 0) { status |= ST_DISCONNECTED; return true; }
    return false;
  };

  while (!done && g.n > n0) {
    if (rounds >= max_rounds) { status |= ST_MAX_ROUNDS; break; }
    int32_t r = rounds++;
    int32_t n_start = g.n;
    if (lp_iters > 0) {
      std::vector<int32_t> L = label_propagation(g, lp_iters, seed, r, flags, cb, user);
      if (flags & F_CORRECT) {
        L = fix_misplaced(g, L);
        if (cb) {
          oracle_event ev{};
          ev.kind = EV_FIX; ev.round = r; ev.n = g.n; ev.a = L.data();
          cb(user, &ev);
        }
      }
      if (apply_contraction(L)) { done = true; break; }
    }
    std::vector<int32_t> mark = pr_marks(g, deg, lam);
    if (cb) {
      oracle_event ev{};
      ev.kind = EV_PR; ev.round = r; ev.level = level; ev.n = g.n; ev.nnz = g.arcs(); ev.lam_hat = lam;
      ev.a = mark.data();
      cb(user, &ev);
    }
    bool any = false;
    for (int32_t m : mark) any = any || m;
    if (any) {
      std::vector<int32_t> rep = marked_components(g, mark);
      if (cb) {
        oracle_event ev{};
        ev.kind = EV_UF; ev.round = r; ev.level = level; ev.n = g.n; ev.a = rep.data();
        cb(user, &ev);
      }
      if (apply_contraction(rep)) { done = true; break; }
    }
    if (g.n == n_start) { status |= ST_NO_PROGRESS; break; }
  }

  int64_t cut = lam;
  std::vector<uint8_t> side = witness;
  int32_t out_level = wit_level;
  if (!(status & (ST_COLLAPSED | ST_DISCONNECTED)) && g.n >= 2) {
    std::vector<uint8_t> kside;
    int64_t lk = stoer_wagner(g, kside);
    if (lk < lam) {
      cut = lk;
      out_level = -1;
      for (int32_t u = 0; u < n; u++) side[u] = kside[map[u]];
    }
  }
  if (side[0])
    for (int32_t u = 0; u < n; u++) side[u] ^= 1;
  int32_t words = (n + 63) / 64;
  for (int32_t i = 0; i < words; i++) out_side[i] = 0;
  for (int32_t u = 0; u < n; u++)
    if (side[u]) out_side[u >> 6] |= 1ULL << (u & 63);
  *out_cut = cut;
  out_info[0] = rounds;
  out_info[1] = g.n;
  out_info[2] = out_level;
  out_info[3] = (int32_t)status;
  return OK;
}

}  // extern "C"
