// Seeded synthetic graph generators for the minimum-cut workloads.
//
// These produce the inputs that both the CPU oracle and the GPU library are
// run on. They contain none of the minimum-cut method's arithmetic: only
// random graph models and the instance-preparation steps that the paper
// applies before measuring (k-core, largest connected component).
//
// Output format: a symmetric CSR with int32 row pointers, int32 column ids
// (strictly increasing per row, no self loops) and int32 weights (>= 1,
// w(u,v) == w(v,u)).
//
// Models:
//  * planted cut: two random blocks, each a random Hamiltonian cycle plus
//    uniformly random distinct pairs, joined by a few random cross pairs;
//  * random hyperbolic graph (threshold model, power-law exponent gamma,
//    Section "Random Hyperbolic Graphs" of the paper's instance appendix);
//  * R-MAT with a/b/c/d quadrant probabilities, duplicates merged into the
//    weight, followed by the k-core on distinct-neighbour degree and the
//    largest connected component (the paper's real-world-graph recipe).
//
// Randomness: every random draw comes from a counter-keyed stream
// (xoshiro256** state seeded by splitmix64 from (seed, stream id)), so
// results do not depend on the number of OpenMP threads.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- RNG ----
inline uint64_t sm64_next(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct Rng {  // xoshiro256** (Blackman & Vigna)
  uint64_t s[4];
  Rng(uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ (stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL);
    for (auto &v : s) v = sm64_next(x);
  }
  static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  inline uint64_t next() {
    uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]; s[2] ^= t; s[3] = rotl(s[3], 45);
    return r;
  }
  inline double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }  // [0,1)
  inline uint64_t below(uint64_t b) {  // unbiased in [0,b)
    if (b <= 1) return 0;
    uint64_t lim = (~0ULL) - ((~0ULL) % b);
    uint64_t x;
    do { x = next(); } while (x >= lim);
    return x % b;
  }
};

struct Edge { int32_t u, v, w; };

// --------------------------------------------------------------- CSR -----
struct Csr {
  int32_t n = 0;
  std::vector<int64_t> rp;  // n+1
  std::vector<int32_t> col, w;
};

// Symmetrise an undirected edge list (u != v) into a CSR; duplicate pairs
// (in either orientation) are merged by summing their weights.
Csr build_csr(int32_t n, const std::vector<Edge> &edges) {
  Csr g;
  g.n = n;
  std::vector<int64_t> cnt(n + 1, 0);
  for (const Edge &e : edges) { cnt[e.u + 1]++; cnt[e.v + 1]++; }
  for (int32_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  std::vector<int32_t> col(cnt[n]), w(cnt[n]);
  std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
  for (const Edge &e : edges) {
    int64_t a = cur[e.u]++; col[a] = e.v; w[a] = e.w;
    int64_t b = cur[e.v]++; col[b] = e.u; w[b] = e.w;
  }
  std::vector<int64_t> len(n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < n; v++) {
    int64_t b = cnt[v], e = cnt[v + 1];
    std::vector<std::pair<int32_t, int32_t>> row;
    row.reserve(e - b);
    for (int64_t i = b; i < e; i++) row.push_back({col[i], w[i]});
    std::sort(row.begin(), row.end());
    int64_t o = b;
    for (size_t i = 0; i < row.size(); i++) {
      if (o > b && col[o - 1] == row[i].first) { w[o - 1] += row[i].second; }
      else { col[o] = row[i].first; w[o] = row[i].second; o++; }
    }
    len[v] = o - b;
  }
  g.rp.assign(n + 1, 0);
  for (int32_t v = 0; v < n; v++) g.rp[v + 1] = g.rp[v] + len[v];
  g.col.resize(g.rp[n]);
  g.w.resize(g.rp[n]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < n; v++) {
    std::copy(col.begin() + cnt[v], col.begin() + cnt[v] + len[v], g.col.begin() + g.rp[v]);
    std::copy(w.begin() + cnt[v], w.begin() + cnt[v] + len[v], g.w.begin() + g.rp[v]);
  }
  return g;
}

// Induced subgraph on vertices with keep[v] != 0, renumbered compactly in
// ascending original id.
Csr induced(const Csr &g, const std::vector<uint8_t> &keep) {
  std::vector<int32_t> nid(g.n, -1);
  int32_t k = 0;
  for (int32_t v = 0; v < g.n; v++) if (keep[v]) nid[v] = k++;
  Csr h;
  h.n = k;
  h.rp.assign(k + 1, 0);
  for (int32_t v = 0; v < g.n; v++) {
    if (!keep[v]) continue;
    int64_t c = 0;
    for (int64_t i = g.rp[v]; i < g.rp[v + 1]; i++) c += keep[g.col[i]] ? 1 : 0;
    h.rp[nid[v] + 1] = c;
  }
  for (int32_t i = 0; i < k; i++) h.rp[i + 1] += h.rp[i];
  h.col.resize(h.rp[k]);
  h.w.resize(h.rp[k]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t v = 0; v < g.n; v++) {
    if (!keep[v]) continue;
    int64_t o = h.rp[nid[v]];
    for (int64_t i = g.rp[v]; i < g.rp[v + 1]; i++)
      if (keep[g.col[i]]) { h.col[o] = nid[g.col[i]]; h.w[o] = g.w[i]; o++; }
  }
  return h;
}

// Largest connected component (ties: the component containing the smallest id).
std::vector<uint8_t> lcc_mask(const Csr &g, const std::vector<uint8_t> *alive) {
  std::vector<int32_t> comp(g.n, -1);
  std::vector<int32_t> stack;
  int32_t best = -1, ncomp = 0;
  int64_t best_size = 0;
  for (int32_t s = 0; s < g.n; s++) {
    if (comp[s] >= 0 || (alive && !(*alive)[s])) continue;
    int64_t size = 0;
    comp[s] = ncomp;
    stack.push_back(s);
    while (!stack.empty()) {
      int32_t v = stack.back(); stack.pop_back(); size++;
      for (int64_t i = g.rp[v]; i < g.rp[v + 1]; i++) {
        int32_t u = g.col[i];
        if (comp[u] < 0 && (!alive || (*alive)[u])) { comp[u] = ncomp; stack.push_back(u); }
      }
    }
    if (size > best_size) { best_size = size; best = ncomp; }
    ncomp++;
  }
  std::vector<uint8_t> keep(g.n, 0);
  for (int32_t v = 0; v < g.n; v++) keep[v] = (best >= 0 && comp[v] == best) ? 1 : 0;
  return keep;
}

// k-core on distinct-neighbour degree (peeling).
std::vector<uint8_t> kcore_mask(const Csr &g, int32_t k) {
  std::vector<int64_t> deg(g.n);
  std::vector<uint8_t> alive(g.n, 1);
  std::vector<int32_t> q;
  for (int32_t v = 0; v < g.n; v++) {
    deg[v] = g.rp[v + 1] - g.rp[v];
    if (deg[v] < k) { alive[v] = 0; q.push_back(v); }
  }
  while (!q.empty()) {
    int32_t v = q.back(); q.pop_back();
    for (int64_t i = g.rp[v]; i < g.rp[v + 1]; i++) {
      int32_t u = g.col[i];
      if (alive[u] && --deg[u] < k) { alive[u] = 0; q.push_back(u); }
    }
  }
  return alive;
}

// ------------------------------------------------------------- planted ----
// Distinct random pairs inside `members` (excluding those already present),
// appended until the block holds `target` pairs. Deterministic for a seed.
void add_random_pairs(const std::vector<int32_t> &members, int64_t target, std::vector<uint64_t> &keys,
                      Rng &rng) {
  int64_t nb = (int64_t)members.size();
  int64_t maxp = nb * (nb - 1) / 2;
  if (target > maxp) target = maxp;
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  while ((int64_t)keys.size() < target) {
    int64_t need = target - (int64_t)keys.size();
    std::vector<uint64_t> batch;
    batch.reserve(need);
    for (int64_t i = 0; i < need; i++) {
      int32_t a = members[rng.below(nb)], b = members[rng.below(nb)];
      if (a == b) { i--; continue; }
      if (a > b) std::swap(a, b);
      batch.push_back(((uint64_t)(uint32_t)a << 32) | (uint32_t)b);
    }
    std::sort(batch.begin(), batch.end());
    batch.erase(std::unique(batch.begin(), batch.end()), batch.end());
    std::vector<uint64_t> fresh;
    std::set_difference(batch.begin(), batch.end(), keys.begin(), keys.end(), std::back_inserter(fresh));
    if ((int64_t)fresh.size() > need) fresh.resize(need);  // keep the smallest keys: deterministic
    std::vector<uint64_t> merged;
    merged.reserve(keys.size() + fresh.size());
    std::merge(keys.begin(), keys.end(), fresh.begin(), fresh.end(), std::back_inserter(merged));
    keys.swap(merged);
  }
}

Csr planted(int32_t n, double d, int32_t kx, int32_t wlo, int32_t whi, uint64_t seed) {
  Rng rng(seed, 1);
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  for (int32_t i = n - 1; i > 0; i--) std::swap(perm[i], perm[rng.below(i + 1)]);
  int32_t n0 = n / 2;
  std::vector<int32_t> blk[2] = {std::vector<int32_t>(perm.begin(), perm.begin() + n0),
                                 std::vector<int32_t>(perm.begin() + n0, perm.end())};
  std::vector<uint64_t> all;
  for (int b = 0; b < 2; b++) {
    const std::vector<int32_t> &m = blk[b];
    int64_t nb = (int64_t)m.size();
    if (nb < 2) continue;
    std::vector<uint64_t> keys;
    // Hamiltonian cycle in the (random) block order; a 2-vertex block gets one edge.
    int64_t cyc = nb >= 3 ? nb : 1;
    for (int64_t i = 0; i < cyc; i++) {
      int32_t a = m[i], c = m[(i + 1) % nb];
      if (a > c) std::swap(a, c);
      keys.push_back(((uint64_t)(uint32_t)a << 32) | (uint32_t)c);
    }
    int64_t target = std::llround(nb * d / 2.0);
    if (target < (int64_t)keys.size()) target = (int64_t)keys.size();
    add_random_pairs(m, target, keys, rng);
    all.insert(all.end(), keys.begin(), keys.end());
  }
  // distinct cross pairs
  std::vector<uint64_t> cross;
  int64_t maxc = (int64_t)blk[0].size() * (int64_t)blk[1].size();
  int64_t want = std::min<int64_t>(kx, maxc);
  while ((int64_t)cross.size() < want) {
    int32_t a = blk[0][rng.below(blk[0].size())], c = blk[1][rng.below(blk[1].size())];
    if (a > c) std::swap(a, c);
    uint64_t key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)c;
    if (std::find(cross.begin(), cross.end(), key) == cross.end()) cross.push_back(key);
  }
  all.insert(all.end(), cross.begin(), cross.end());
  std::sort(all.begin(), all.end());
  std::vector<Edge> edges;
  edges.reserve(all.size());
  Rng wr(seed, 2);
  for (uint64_t key : all) {
    int32_t w = wlo + (int32_t)wr.below((uint64_t)(whi - wlo + 1));
    edges.push_back({(int32_t)(key >> 32), (int32_t)(key & 0xffffffffu), w});
  }
  return build_csr(n, edges);
}

// ------------------------------------------------------ clustered ER ----
// Clustered Erdos-Renyi graph (the paper's appendix on instances): every
// unordered pair is an edge with probability d / 100 (so m has mean
// n (n - 1) / 2 * d / 100), its weight is uniform in [1, 100] and multiplied
// by n when both ends are in the same cluster. The k clusters are balanced:
// a seeded random permutation deals the vertices round-robin.
Csr clustered_er(int32_t n, double d, int32_t k, uint64_t seed) {
  Rng rng(seed, 1);
  std::vector<int32_t> perm(n), cluster(n);
  std::iota(perm.begin(), perm.end(), 0);
  for (int32_t i = n - 1; i > 0; i--) std::swap(perm[i], perm[rng.below(i + 1)]);
  for (int32_t i = 0; i < n; i++) cluster[perm[i]] = k > 0 ? i % k : 0;
  const double p = d / 100.0;
  Rng er(seed, 2), wr(seed, 3);
  std::vector<Edge> edges;
  for (int32_t u = 0; u < n; u++)
    for (int32_t v = u + 1; v < n; v++) {
      if (er.uniform() >= p) continue;
      int64_t w = 1 + (int64_t)wr.below(100);
      if (cluster[u] == cluster[v]) w *= n;
      edges.push_back({u, v, (int32_t)std::min<int64_t>(w, INT32_MAX)});
    }
  return build_csr(n, edges);
}

// ----------------------------------------------------------------- RHG ----
// Threshold random hyperbolic graph: points in a disk of radius R, angle
// uniform, radius with density alpha*sinh(alpha r)/(cosh(alpha R)-1),
// alpha = (gamma-1)/2; an edge joins every pair at hyperbolic distance <= R.
struct RhgModel {
  double alpha, R, coshR;
  // largest angular difference at which radii (r1, r2) are still adjacent
  double dtheta_max(double r1, double r2) const {
    double s = std::sinh(r1) * std::sinh(r2);
    double num = coshR - std::cosh(r1 - r2);
    if (num <= 0) return 0.0;
    if (s <= 0) return M_PI;
    double x = num / (2.0 * s);
    if (x >= 1.0) return M_PI;
    return 2.0 * std::asin(std::sqrt(x));
  }
  double radius_at(double u) const {  // inverse CDF
    return std::acosh(1.0 + u * (std::cosh(alpha * R) - 1.0)) / alpha;
  }
  // expected degree of a vertex (n-1 others), by equal-probability midpoint quadrature
  double expected_avg_degree(int64_t n, int M = 700) const {
    std::vector<double> r(M);
    for (int i = 0; i < M; i++) r[i] = radius_at((i + 0.5) / M);
    double acc = 0;
    for (int i = 0; i < M; i++)
      for (int j = 0; j < M; j++) acc += dtheta_max(r[i], r[j]);
    return (double)(n - 1) * acc / ((double)M * M * M_PI);
  }
};

Csr rhg_once(int32_t n, const RhgModel &md, int32_t wlo, int32_t whi, uint64_t seed, double *avg_out) {
  std::vector<double> rr(n), th(n);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; i++) {
    Rng rng(seed, 1000003ULL + (uint64_t)i);
    th[i] = rng.uniform() * 2.0 * M_PI;
    rr[i] = md.radius_at(rng.uniform());
  }
  // angular order defines the vertex ids
  std::vector<int32_t> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return th[a] < th[b] || (th[a] == th[b] && a < b); });
  std::vector<double> r(n), t(n);
  for (int32_t i = 0; i < n; i++) { r[i] = rr[ord[i]]; t[i] = th[ord[i]]; }
  // radial bands
  std::vector<double> bnd;
  bnd.push_back(0.0);
  {
    double lo = std::max(0.0, md.R - 16.0);
    if (lo > 0) bnd.push_back(lo);
    double x = lo;
    while (x < md.R - 8.0) { x = std::min(md.R - 8.0, x + 2.0); if (x > bnd.back()) bnd.push_back(x); }
    while (x < md.R) { x = std::min(md.R, x + 0.5); if (x > bnd.back()) bnd.push_back(x); }
    if (bnd.back() < md.R) bnd.push_back(md.R);
  }
  int nb = (int)bnd.size() - 1;
  std::vector<std::vector<int32_t>> band(nb);
  std::vector<std::vector<double>> bth(nb);
  for (int32_t i = 0; i < n; i++) {
    int j = (int)(std::upper_bound(bnd.begin(), bnd.end(), r[i]) - bnd.begin()) - 1;
    j = std::max(0, std::min(nb - 1, j));
    band[j].push_back(i);
    bth[j].push_back(t[i]);
  }
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  std::vector<std::vector<Edge>> local(nthreads);
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<Edge> &out = local[tid];
#pragma omp for schedule(dynamic, 2048)
    for (int32_t p = 0; p < n; p++) {
      double rp = r[p], tp = t[p];
      double shp = std::sinh(rp);
      for (int j = 0; j < nb; j++) {
        if (bnd[j + 1] < rp || band[j].empty()) continue;
        double lower = std::max(bnd[j], rp);
        double dt = md.dtheta_max(rp, lower);
        if (dt <= 0) continue;
        const std::vector<double> &bt = bth[j];
        auto scan = [&](double a, double b) {
          size_t lo = std::lower_bound(bt.begin(), bt.end(), a) - bt.begin();
          size_t hi = std::upper_bound(bt.begin(), bt.end(), b) - bt.begin();
          for (size_t x = lo; x < hi; x++) {
            int32_t q = band[j][x];
            if (q == p) continue;
            double rq = r[q];
            if (!(rq > rp || (rq == rp && q > p))) continue;
            double dth = std::fabs(tp - t[q]);
            if (dth > M_PI) dth = 2 * M_PI - dth;
            double sh = std::sin(0.5 * dth);
            double cd = std::cosh(rp - rq) + 2.0 * sh * sh * shp * std::sinh(rq);
            if (cd <= md.coshR) out.push_back({std::min(p, q), std::max(p, q), 1});
          }
        };
        if (dt >= M_PI) { scan(-1.0, 7.0); continue; }
        double a = tp - dt, b = tp + dt;
        if (a < 0) { scan(0.0, b); scan(a + 2 * M_PI, 7.0); }
        else if (b >= 2 * M_PI) { scan(a, 7.0); scan(-1.0, b - 2 * M_PI); }
        else scan(a, b);
      }
    }
  }
  std::vector<Edge> edges;
  size_t tot = 0;
  for (auto &l : local) tot += l.size();
  edges.reserve(tot);
  for (auto &l : local) { edges.insert(edges.end(), l.begin(), l.end()); std::vector<Edge>().swap(l); }
  // weights from a per-pair stream: independent of the discovery order
  if (whi > wlo || wlo != 1) {
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < edges.size(); i++) {
      Rng wr(seed ^ 0x5bd1e995ULL, ((uint64_t)(uint32_t)edges[i].u << 32) | (uint32_t)edges[i].v);
      edges[i].w = wlo + (int32_t)wr.below((uint64_t)(whi - wlo + 1));
    }
  }
  if (avg_out) *avg_out = 2.0 * (double)edges.size() / (double)n;
  return build_csr(n, edges);
}

Csr rhg(int32_t n, double avg_deg, double gamma, int32_t wlo, int32_t whi, uint64_t seed, double *R_out,
        double *avg_out) {
  RhgModel md;
  md.alpha = (gamma - 1.0) / 2.0;
  // bisection of R on the expected average degree (decreasing in R)
  double lo = 0.5, hi = 2.0 * std::log((double)n) + 40.0;
  for (int it = 0; it < 50; it++) {
    md.R = 0.5 * (lo + hi);
    md.coshR = std::cosh(md.R);
    if (md.expected_avg_degree(n, 400) > avg_deg) lo = md.R; else hi = md.R;
  }
  md.R = 0.5 * (lo + hi);
  md.coshR = std::cosh(md.R);
  double avg = 0;
  Csr g;
  for (int attempt = 0; attempt < 6; attempt++) {
    g = rhg_once(n, md, wlo, whi, seed, &avg);
    if (std::fabs(avg - avg_deg) <= 0.01 * avg_deg) break;
    // the average degree scales like exp(-R/2): correct R and regenerate
    md.R += 2.0 * std::log(avg / avg_deg);
    md.coshR = std::cosh(md.R);
  }
  if (R_out) *R_out = md.R;
  if (avg_out) *avg_out = avg;
  return g;
}

// ---------------------------------------------------------------- RMAT ----
Csr rmat(int32_t scale, int64_t ef, double a, double b, double c, uint64_t seed) {
  int32_t n = 1 << scale;
  int64_t m = ef * (int64_t)n;
  std::vector<Edge> edges(m);
  std::vector<uint8_t> keepe(m);
  double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static, 65536)
  for (int64_t i = 0; i < m; i++) {
    Rng rng(seed, 7000000000ULL + (uint64_t)i);
    uint32_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; l++) {
      double x = rng.uniform();
      uint32_t bu = 0, bv = 0;
      if (x < a) {} else if (x < ab) { bv = 1; } else if (x < abc) { bu = 1; } else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    keepe[i] = u != v;
    edges[i] = {(int32_t)std::min(u, v), (int32_t)std::max(u, v), 1};
  }
  int64_t o = 0;
  for (int64_t i = 0; i < m; i++) if (keepe[i]) edges[o++] = edges[i];
  edges.resize(o);
  std::vector<uint8_t>().swap(keepe);
  return build_csr(n, edges);
}

struct Out {
  int32_t n;
  int32_t pad;
  int64_t nnz;
  int32_t *row_ptr, *col, *w;
  double info[8];
};

Out *export_csr(Csr &&g, const double *info, int ninfo) {
  Out *o = (Out *)std::calloc(1, sizeof(Out));
  o->n = g.n;
  o->nnz = g.rp[g.n];
  o->row_ptr = (int32_t *)std::malloc(sizeof(int32_t) * (g.n + 1));
  o->col = (int32_t *)std::malloc(sizeof(int32_t) * std::max<int64_t>(1, o->nnz));
  o->w = (int32_t *)std::malloc(sizeof(int32_t) * std::max<int64_t>(1, o->nnz));
  for (int32_t i = 0; i <= g.n; i++) o->row_ptr[i] = (int32_t)g.rp[i];
  std::memcpy(o->col, g.col.data(), sizeof(int32_t) * o->nnz);
  std::memcpy(o->w, g.w.data(), sizeof(int32_t) * o->nnz);
  for (int i = 0; i < ninfo && i < 8; i++) o->info[i] = info[i];
  return o;
}

}  // namespace

extern "C" {

// planted cut, see file header; info[0] = number of cross pairs
void *gg_planted(int32_t n, double d, int32_t kx, int32_t wlo, int32_t whi, uint64_t seed) {
  double info[1] = {(double)kx};
  return export_csr(planted(n, d, kx, wlo, whi, seed), info, 1);
}

// clustered Erdos-Renyi graph; info = {number of clusters}
void *gg_clustered_er(int32_t n, double d, int32_t k, uint64_t seed) {
  double info[1] = {(double)k};
  return export_csr(clustered_er(n, d, k, seed), info, 1);
}

// random hyperbolic graph; info = {R, realised average degree, n before LCC}
void *gg_rhg(int32_t n, double avg_deg, double gamma, int32_t wlo, int32_t whi, uint64_t seed, int32_t keep_lcc) {
  double R = 0, avg = 0;
  Csr g = rhg(n, avg_deg, gamma, wlo, whi, seed, &R, &avg);
  double info[3] = {R, avg, (double)g.n};
  if (keep_lcc) {
    std::vector<uint8_t> keep = lcc_mask(g, nullptr);
    g = induced(g, keep);
  }
  return export_csr(std::move(g), info, 3);
}

// R-MAT, symmetrised with duplicates merged into weights, then (if kcore > 0)
// the k-core on distinct-neighbour degree, then (if keep_lcc) its largest
// connected component. info = {n, nnz after merge, n after core}
void *gg_rmat(int32_t scale, int64_t ef, double a, double b, double c, uint64_t seed, int32_t kcore, int32_t keep_lcc) {
  Csr g = rmat(scale, ef, a, b, c, seed);
  double info[3] = {(double)g.n, (double)g.rp[g.n], 0};
  std::vector<uint8_t> alive(g.n, 1);
  if (kcore > 0) alive = kcore_mask(g, kcore);
  if (keep_lcc) {
    std::vector<uint8_t> keep = lcc_mask(g, &alive);
    alive.swap(keep);
  }
  g = induced(g, alive);
  info[2] = (double)g.n;
  return export_csr(std::move(g), info, 3);
}

// CSR from an undirected edge list (u != v); duplicates are summed.
void *gg_from_edges(int32_t n, int64_t m, const int32_t *u, const int32_t *v, const int32_t *w) {
  std::vector<Edge> e(m);
  for (int64_t i = 0; i < m; i++) e[i] = {u[i], v[i], w ? w[i] : 1};
  return export_csr(build_csr(n, e), nullptr, 0);
}

// k-core (distinct-neighbour degree) + LCC of a CSR
void *gg_kcore_lcc(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w, int32_t kcore,
                   int32_t keep_lcc) {
  Csr g;
  g.n = n;
  g.rp.assign(row_ptr, row_ptr + n + 1);
  g.col.assign(col, col + row_ptr[n]);
  g.w.assign(w, w + row_ptr[n]);
  std::vector<uint8_t> alive(n, 1);
  if (kcore > 0) alive = kcore_mask(g, kcore);
  if (keep_lcc) { std::vector<uint8_t> keep = lcc_mask(g, &alive); alive.swap(keep); }
  return export_csr(induced(g, alive), nullptr, 0);
}

double gg_rhg_expected_degree(int64_t n, double R, double gamma) {
  RhgModel md;
  md.alpha = (gamma - 1.0) / 2.0;
  md.R = R;
  md.coshR = std::cosh(R);
  return md.expected_avg_degree(n);
}

void gg_free(void *p) {
  Out *o = (Out *)p;
  if (!o) return;
  std::free(o->row_ptr);
  std::free(o->col);
  std::free(o->w);
  std::free(o);
}

}  // extern "C"
