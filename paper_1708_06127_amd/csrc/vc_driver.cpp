// Host driver of the inexact minimum-cut method (Algorithm 1 of the paper
// with synchronous label propagation): workspace carving, the round loop
// (label propagation -> cluster contraction -> bound -> Padberg-Rinaldi
// marking -> union-find contraction -> bound), the exact solve on the
// remaining graph and the transfer of its side to the input vertices.
// Device work is enqueued on the caller's stream; the host reads the small
// status block back at the points where sizes or stop decisions are needed.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/viecut.h"
#include "vc_internal.h"

namespace vc {

// SplitMix64 (Steele, Lea, Flood 2014): output number `index` (1-based) of the
// generator whose state starts at `seed` is mix(seed + index * golden gamma).
uint64_t splitmix64_at(uint64_t seed, uint64_t index) {
  uint64_t z = seed + index * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------ kernel timing
// Process-wide and off by default. While on, each timed launch gets an event
// pair on its stream, and its kernel writes the level's tile totals (rows,
// arcs: 16 bytes) into a page-locked record; prof_collect() folds completed
// records into per-kernel totals of duration and algorithmic bytes.
namespace {
struct ProfRec {
  int kind;
  int32_t ntiles;
  hipEvent_t a, b;
  double bytes = -1;  // >= 0: set by the host (spans); < 0: from the kernel's tile totals
};
struct ProfState {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int32_t *slots = nullptr;  // 4 int32 per record: tile rows, big tiles, tile arcs (u64)
  int32_t *dslots = nullptr;  // the same memory's device address
  int32_t cap = 0;
  int64_t launches[PROF_KINDS] = {0};
  double ms[PROF_KINDS] = {0}, bytes[PROF_KINDS] = {0};
};
ProfState &prof() {
  static ProfState p;
  return p;
}
const char *kProfNames[PROF_KINDS] = {"k_first_tile", "k_first_tile_level0", "k_lp_tile", "lp_contract_sweep"};
// algorithmic bytes per arc and per row of each timed kernel (spans carry their own)
const double kProfPerArc[PROF_KINDS] = {8, 8, 12, 0};   // col, w (+ the label gather Lin[col])
const double kProfPerRow[PROF_KINDS] = {8, 16, 12, 0};  // rp + label out (+ degree, + own label)
hipEvent_t prof_event(ProfState &p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ProfScope::ProfScope(ProfKind kind, hipStream_t stream, const Status *st_, int32_t ntiles) : s(stream), st(st_) {
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.on || !p.slots || (int32_t)p.pending.size() >= p.cap) return;
  ProfRec r;
  r.kind = kind;
  r.ntiles = ntiles;
  r.a = prof_event(p);
  r.b = prof_event(p);
  if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) return;
  slot = (int)p.pending.size();
  p.pending.push_back(r);
  dev = p.dslots + 4 * slot;
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (slot >= (int)p.pending.size()) return;
  (void)hipEventRecord(p.pending[slot].b, s);
}

int prof_span_begin(ProfKind kind, hipStream_t s) {
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.on || !p.slots || (int32_t)p.pending.size() >= p.cap) return -1;
  ProfRec r;
  r.kind = kind;
  r.ntiles = 0;
  r.a = prof_event(p);
  r.b = prof_event(p);
  if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) return -1;
  r.bytes = 0;
  p.pending.push_back(r);
  return (int)p.pending.size() - 1;
}

void prof_span_end(int id, hipStream_t s) {
  if (id < 0) return;
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (id < (int)p.pending.size()) (void)hipEventRecord(p.pending[id].b, s);
}

void prof_span_bytes(int id, double bytes) {
  if (id < 0) return;
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (id < (int)p.pending.size()) p.pending[id].bytes = bytes;
}

void prof_collect() {
  ProfState &p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  for (size_t i = 0; i < p.pending.size(); i++) {
    ProfRec &r = p.pending[i];
    float ms = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p.launches[r.kind]++;
      p.ms[r.kind] += ms;
      if (r.bytes >= 0) {
        p.bytes[r.kind] += r.bytes;
      } else {
        const int32_t rows = p.slots[4 * i];
        uint64_t arcs;
        std::memcpy(&arcs, &p.slots[4 * i + 2], 8);
        p.bytes[r.kind] += kProfPerArc[r.kind] * (double)arcs + kProfPerRow[r.kind] * rows + 16.0 * r.ntiles;
      }
    }
    p.pool.push_back(r.a);
    p.pool.push_back(r.b);
  }
  p.pending.clear();
}

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t off[40];
  int cnt = 0;
  size_t total = 0;
  size_t add(size_t bytes) {
    off[cnt++] = total;
    total += align256(bytes);
    return off[cnt - 1];
  }
};

// state words of the single-pass scan: one per 2048-element tile
int64_t scan_tiles_max(int64_t count) { return (count + 2047) / 2048 + 1; }

// map_n: entries of the input -> current vertex map (n for a single solve,
// 64 per word of the padded input index space for a batched one); extra:
// rows of the gather staging beyond n (one per graph in a batch).
Layout make_layout(int32_t n, int64_t nnz, int64_t map_n, int64_t extra) {
  Layout L;
  const int64_t tiles = (nnz + kRsTile - 1) / kRsTile + 1;
  const int64_t huge_rows = nnz / (kHugeChunk + 1) + 1;
  const int64_t ntiles = (nnz + n) / kTile + 2;
  const int64_t nseg = ntiles + 4 * (nnz / kTile + 1) + 2;
  int64_t maxscan = std::max<int64_t>({nnz, 2 * (int64_t)n + 1, 256 * tiles, nseg});
  L.add(sizeof(Status));                       // 0 st
  for (int b = 0; b < 2; b++) {
    L.add(4 * ((size_t)n + 1));                // rp
    L.add(4 * (size_t)std::max<int64_t>(nnz, 1));  // col
    L.add(4 * (size_t)std::max<int64_t>(nnz, 1));  // w
  }                                            // 1..6
  L.add(8 * (size_t)n + 8);                    // 7 deg
  L.add(4 * (size_t)n + 4);                    // 8 La
  L.add(4 * (size_t)n + 4);                    // 9 Lb
  L.add(4 * (2 * (size_t)n + 1));              // 10 ids (label range up to 2n with the correcting step)
  L.add(4 * (size_t)n + 4);                    // 11 cl
  L.add(4 * (size_t)map_n + 4);                // 12 map
  L.add(8 * (((size_t)map_n + 63) / 64) + 8);  // 13 witness
  L.add(4 * (size_t)kBins * n + 4);            // 14 bins
  L.add(4 * ((size_t)n + (size_t)extra + 1));  // 15 cnt (batched: gather staging rows)
  L.add(8 * (size_t)std::max<int64_t>(nnz, 1));  // 16 keys0
  L.add(8 * (size_t)std::max<int64_t>(nnz, 1));  // 17 keys1
  L.add(4 * (size_t)std::max<int64_t>(nnz, 1));  // 18 vals0
  L.add(4 * (size_t)std::max<int64_t>(nnz, 1));  // 19 vals1
  L.add(4 * 256 * (size_t)tiles);              // 20 hist
  L.add(8 * (size_t)scan_tiles_max(maxscan) + 64);  // 21 scan state words + ticket
  L.add((size_t)std::max<int64_t>(nnz, 1));    // 22 mark
  L.add(4 * (size_t)n + 4);                    // 23 parent
  L.add(4 * 4 * (size_t)std::max<int64_t>(nnz, 1));  // 24 huge keys (4 slots per arc)
  L.add(4 * 4 * (size_t)std::max<int64_t>(nnz, 1));  // 25 huge vals
  L.add(8 * (size_t)huge_rows);                // 26 huge best
  L.add(12 * (size_t)huge_rows);               // 27 huge meta
  L.add((size_t)n + 1);                        // 28 flags8
  L.add(16 * (size_t)ntiles);                  // 29 tile_meta
  L.add(24 * (2 * (size_t)ntiles + 1 + kLongParts));  // 30 part
  L.add(8 * (size_t)nseg);                     // 31 seg
  L.add(4 * (size_t)nseg + 4);                 // 32 seg_cnt
  L.add(4 * (size_t)ntiles);                   // 33 big_tiles
  L.add(4 * (size_t)n + 4);                    // 34 fix_cnt
  L.add(4 * (size_t)n + 4);                    // 35 fix_out
  L.add(8 * (size_t)n + 8);                    // 36 fix_cut
  L.add(8 * (size_t)n + 8);                    // 37 fix_key
  return L;
}

}  // namespace

size_t work_bytes(int32_t n, int64_t nnz, int64_t map_n, int64_t extra) {
  return make_layout(n, nnz, map_n < 0 ? n : map_n, extra).total + 256;
}

bool carve(void *ws, size_t bytes, int32_t n, int64_t nnz, Work &w, int64_t map_n, int64_t extra) {
  Layout L = make_layout(n, nnz, map_n < 0 ? n : map_n, extra);
  uintptr_t base = ((uintptr_t)ws + 255) & ~uintptr_t(255);
  if (base + L.total > (uintptr_t)ws + bytes) return false;
  auto at = [&](int i) { return (void *)(base + L.off[i]); };
  w.n_in = n;
  w.nnz_in = nnz;
  w.st = (Status *)at(0);
  for (int b = 0; b < 2; b++) {
    w.rp[b] = (int32_t *)at(1 + 3 * b);
    w.col[b] = (int32_t *)at(2 + 3 * b);
    w.w[b] = (int32_t *)at(3 + 3 * b);
  }
  w.deg = (long long *)at(7);
  w.La = (int32_t *)at(8);
  w.Lb = (int32_t *)at(9);
  w.ids = (int32_t *)at(10);
  w.cl = (int32_t *)at(11);
  w.map = (int32_t *)at(12);
  w.witness = (unsigned long long *)at(13);
  w.bins = (int32_t *)at(14);
  w.cnt = (int32_t *)at(15);
  w.keys[0] = (unsigned long long *)at(16);
  w.keys[1] = (unsigned long long *)at(17);
  w.vals[0] = (int32_t *)at(18);
  w.vals[1] = (int32_t *)at(19);
  w.hist = (int32_t *)at(20);
  {
    const int64_t tiles = (nnz + kRsTile - 1) / kRsTile + 1;
    const int64_t nseg = (nnz + n) / kTile + 2 + 4 * (nnz / kTile + 1) + 2;
    w.lb_tiles = scan_tiles_max(std::max<int64_t>({nnz, 2 * (int64_t)n + 1, 256 * tiles, nseg}));
    w.lb_state = (unsigned long long *)at(21);
    w.lb_ticket = (uint32_t *)(w.lb_state + w.lb_tiles);
    w.lb_epoch = 0;
  }
  w.mark = (uint8_t *)at(22);
  w.parent = (int32_t *)at(23);
  w.huge_tab_key = (int32_t *)at(24);
  w.huge_tab_val = (uint32_t *)at(25);
  w.huge_best = (unsigned long long *)at(26);
  w.huge_meta = (int32_t *)at(27);
  w.huge_cap = 4 * std::max<int64_t>(nnz, 1);
  w.flags8 = (uint8_t *)at(28);
  w.tile_meta = (int4 *)at(29);
  w.part = (unsigned long long *)at(30);
  w.seg = (int32_t *)at(31);
  w.seg_cnt = (int32_t *)at(32);
  w.big_tiles = (int32_t *)at(33);
  w.fix_cnt = (int32_t *)at(34);
  w.fix_out = (uint32_t *)at(35);
  w.fix_cut = (unsigned long long *)at(36);
  w.fix_key = (unsigned long long *)at(37);
  return true;
}

namespace {

inline int bits_for_host(int32_t k) {
  int b = 0;
  while (b < 31 && (1 << b) < k) b++;
  return b;
}

struct Tracer {
  viecut_trace_fn fn = nullptr;
  void *user = nullptr;
};

#define VC_TRY(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return VIECUT_EDEVICE; \
  } while (0)

struct Solver {
  Work &w;
  hipStream_t s;
  const viecut_params &p;
  Tracer tr;
  Status st{};  // host copy
  // false: no page-locked host buffers (the allocation-free entry point);
  // status reads and the kernel-graph hand-off use pageable host memory
  bool pinned = true;
  // kernel timer span of round 1's label propagation and cluster contraction
  // (from the solve's first launch to the coarse CSR), -1 when not timed
  int sweep = -1;

  Solver(Work &w_, hipStream_t s_, const viecut_params &p_) : w(w_), s(s_), p(p_) {}

  // Page-locked landing buffer for the status copies, one per host thread
  // (a thread's solves run one after another), allocated on first use and
  // kept for the life of the process: a copy into pageable memory goes
  // through the runtime's staging buffer and a host copy after the wait.
  static Status *pinned_status() {
    static thread_local Status *h = nullptr;
    if (!h) {
      void *q = nullptr;
      if (hipHostMalloc(&q, sizeof(Status), 0) == hipSuccess) h = (Status *)q;
    }
    return h;
  }

  // Page-locked staging for the kernel graph's hand-off to the host solve
  // (and the side flags back), one per host thread, grown on demand up to
  // 16 MiB and kept; larger hand-offs use pageable copies. Every use ends
  // with a stream wait before the buffer is touched again.
  static char *pinned_stage(size_t bytes) {
    static thread_local void *buf = nullptr;
    static thread_local size_t cap = 0;
    if (bytes > ((size_t)16 << 20)) return nullptr;
    if (bytes > cap) {
      if (buf) (void)hipHostFree(buf);
      buf = nullptr;
      cap = 0;
      size_t want = (size_t)1 << 16;
      while (want < bytes) want <<= 1;
      if (hipHostMalloc(&buf, want, 0) != hipSuccess) {
        buf = nullptr;
        return nullptr;
      }
      cap = want;
    }
    return (char *)buf;
  }

  // A status read that lets work enqueued after it run while the host waits:
  // status_begin queues the copy (into the page-locked buffer) and an event,
  // status_end waits for the event only.
  static hipEvent_t status_event() {
    static thread_local hipEvent_t ev = nullptr;
    static thread_local int ev_dev = -1;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (ev && ev_dev != dev) {
      (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
    ev_dev = ev ? dev : -1;
    return ev;
  }
  int status_begin(hipEvent_t ev) {
    VC_TRY(hipMemcpyAsync(pinned_status(), w.st, sizeof(Status), hipMemcpyDeviceToHost, s));
    VC_TRY(hipEventRecord(ev, s));
    return VIECUT_OK;
  }
  int status_end(hipEvent_t ev) {
    VC_TRY(hipEventSynchronize(ev));
    st = *pinned_status();
    if (st.err & ERR_DEVICE) return VIECUT_EDEVICE;
    return VIECUT_OK;
  }

  int sync_status() {
    Status *h = pinned ? pinned_status() : nullptr;
    VC_TRY(hipMemcpyAsync(h ? h : &st, w.st, sizeof(Status), hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    if (h) st = *h;
    if (st.err & ERR_DEVICE) return VIECUT_EDEVICE;
    return VIECUT_OK;
  }

  uint32_t salt(int32_t round, int32_t iter) const {
    return (uint32_t)(splitmix64_at(p.seed, (uint64_t)round * (uint64_t)p.lp_iters + (uint64_t)iter) & 0xFFFFFFFFull);
  }

  // ---- tracing helpers (host copies)
  template <class T>
  std::vector<T> d2h(const T *d, int64_t count) {
    std::vector<T> h((size_t)std::max<int64_t>(count, 0));
    if (count > 0) {
      (void)hipMemcpyAsync(h.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost, s);
      (void)hipStreamSynchronize(s);
    }
    return h;
  }
  void trace_labels(int32_t round, int32_t iter, const int32_t *L, int32_t n, int32_t kind = 1) {
    if (!tr.fn) return;
    std::vector<int32_t> h = d2h(L, n);
    viecut_event ev{};
    ev.kind = kind; ev.round = round; ev.iter = iter; ev.n = n; ev.a = h.data();
    tr.fn(tr.user, &ev);
  }
  void trace_graph(int32_t level, const DGraph &G, int32_t n_prev) {
    if (!tr.fn) return;
    std::vector<int32_t> rp = d2h(G.row_ptr, (int64_t)G.n + 1), col = d2h(G.col, G.nnz), ww = d2h(G.w, G.nnz),
                         cl = d2h(w.cl, n_prev);
    std::vector<long long> deg = d2h(w.deg, G.n);
    std::vector<int64_t> d64(deg.begin(), deg.end());
    viecut_event ev{};
    ev.kind = 2; ev.level = level; ev.n = G.n; ev.n_prev = n_prev; ev.nnz = G.nnz;
    ev.a = rp.data(); ev.b = col.data(); ev.c = ww.data(); ev.d = d64.data(); ev.e = cl.data();
    tr.fn(tr.user, &ev);
  }
  void trace_bound(int32_t level, int32_t n) {
    if (!tr.fn) return;
    viecut_event ev{};
    ev.kind = 3; ev.level = level; ev.n = n; ev.lam_hat = st.lam_hat;
    ev.witness_vertex = st.wit_v; ev.witness_level = st.wit_level;
    tr.fn(tr.user, &ev);
  }
  void trace_pr(int32_t round, int32_t level, const DGraph &G) {
    if (!tr.fn) return;
    std::vector<uint8_t> m8 = d2h(w.mark, G.nnz);
    std::vector<int32_t> m(m8.begin(), m8.end());
    viecut_event ev{};
    ev.kind = 4; ev.round = round; ev.level = level; ev.n = G.n; ev.nnz = G.nnz; ev.lam_hat = st.lam_hat;
    ev.a = m.data();
    tr.fn(tr.user, &ev);
  }
  void trace_rep(int32_t round, int32_t level, const int32_t *rep, int32_t n) {
    if (!tr.fn) return;
    std::vector<int32_t> h = d2h(rep, n);
    viecut_event ev{};
    ev.kind = 5; ev.round = round; ev.level = level; ev.n = n; ev.a = h.data();
    tr.fn(tr.user, &ev);
  }

  // Contract the partition `L` of G into the other CSR buffer. Returns the
  // new graph in G/cur; reads the status (k, ax, then nnz / stop / bins).
  // Contract the partition `L` of G into the other CSR buffer; G/cur become
  // the new graph, whose arc tiles and long-row lists are built here.
  // `known` holds the host copy of G's long-row counts (nullptr: unknown) and
  // is invalidated for the new graph.
  int contract(const int32_t *L, DGraph &G, int &cur, int32_t &level, const int32_t *&known,
               int64_t lspace = -1) {
    VC_TRY(relabel(L, G.n, w, s, nullptr, nullptr, lspace));
    VC_TRY(contract_emit(G, w, known, s));
    int rc = sync_status();
    if (rc) return rc;
    const int32_t k = st.k;
    const int64_t ax = st.ax;
    const int kb = bits_for_host(k);
    const int dst = cur == 0 ? 1 : 0;
    if (k == 1) {  // one cluster: no inter-cluster arc (ax = 0), the graph collapses
      level++;
      VC_TRY(contract_collapse(w, dst, s));
    } else {
      int which = 1;  // the emission leaves the packed triples in buffer 1
      VC_TRY(radix_sort(w, ax, 2 * kb, which, s));
      level++;
      VC_TRY(contract_build(w, which, ax, kb, k, dst, level, s));
    }
    if (sweep >= 0) prof_span_end(sweep, s);
    rc = sync_status();
    if (rc) return rc;
    if (sweep >= 0) {
      // algorithmic bytes of the sweep: LP iteration 1 with the level-0 degrees
      // (8A + 16n), iteration 2 (12A + 12n), relabel and map (24n), contraction
      // (8A + 4 A_x + 8 A' + 8n): 28A + 4A_x + 8A' + 60n, plus 12A + 12n per
      // further LP iteration
      const double A = (double)w.nnz_in, n = (double)w.n_in;
      const double extra = (double)std::max(p.lp_iters - 2, 0) * (12 * A + 12 * n) -
                           (p.lp_iters < 2 ? 12 * A + 12 * n : 0.0);
      prof_span_bytes(sweep, 28 * A + 4 * (double)ax + 8 * (double)st.nnz + 60 * n + extra);
      sweep = -1;
    }
    DGraph H;
    H.n = k;
    H.nnz = st.nnz;
    H.row_ptr = w.rp[dst];
    H.col = w.col[dst];
    H.w = w.w[dst];
    const int32_t n_prev = G.n;
    G = H;
    cur = dst;
    if (!(st.stop & ST_COLLAPSED)) {  // (a collapsed graph ends the rounds: no tiles needed)
      VC_TRY(reset_bins(w, s));
      VC_TRY(build_tiles(G, w, s));
    }
    known = nullptr;
    trace_graph(level, G, n_prev);
    if (!(st.stop & ST_COLLAPSED)) trace_bound(level, G.n);
    return VIECUT_OK;
  }

  int run(const viecut_csr &g, viecut_result *out, uint64_t *side) {
    auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point a) {
      return std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - a).count();
    };
    float t_ms[8] = {0};
    DGraph G;
    G.n = g.n;
    G.nnz = g.nnz;
    G.row_ptr = g.row_ptr;
    G.col = g.col;
    G.w = g.w;
    const bool do_lp = p.lp_iters > 0 && g.n > p.n0;
    if (do_lp && !tr.fn) sweep = prof_span_begin(PROF_SWEEP, s);
    VC_TRY(status_reset(w.st, s));
    VC_TRY(init_map(w, s));
    VC_TRY(check_rowptr(G, w.st, s));
    VC_TRY(build_tiles(G, w, s));
    VC_TRY(lp_first(G, w, nullptr, w.La, salt(0, 1), true, s));
    if (p.flags & VIECUT_F_VALIDATE) VC_TRY(validate_sym(G, w.st, s));
    VC_TRY(bound_level0(w, s));
    // the arc tiles of LP iteration 2 need neither the level-0 status nor the
    // long-row counts, so they run while the host waits for the status (they
    // exit at once on an input error)
    hipEvent_t ev = nullptr;
    const bool early = pinned && !tr.fn && do_lp && p.lp_iters >= 2 &&
                       !(p.flags & (VIECUT_F_RESTRICT | VIECUT_F_CONVERGE)) && pinned_status() &&
                       (ev = status_event()) != nullptr;
    int rc;
    if (early) {
      rc = status_begin(ev);
      if (rc) return rc;
      VC_TRY(lp_iter(G, w, nullptr, w.La, w.Lb, salt(0, 2), s, nullptr, 1));
      rc = status_end(ev);
    } else {
      rc = sync_status();
    }
    if (rc) return rc;
    if (st.err & (ERR_ROWPTR | ERR_COL | ERR_SELF)) return VIECUT_EINVAL;
    if (st.err & ERR_WEIGHT) return VIECUT_EWEIGHT;
    if (st.wsum / 2 > (unsigned long long)INT32_MAX) return VIECUT_EOVERFLOW;
    if (st.err & (ERR_NOTSYM | ERR_UNSORTED)) return VIECUT_ENOTSYM;
    t_ms[0] = ms_since(t0);
    trace_bound(0, G.n);

    int32_t known_buf[8];
    std::memcpy(known_buf, st.bin_cnt, sizeof(known_buf));
    const int32_t *known = known_buf;
    auto refresh_known = [&]() {
      std::memcpy(known_buf, st.bin_cnt, sizeof(known_buf));
      known = known_buf;
    };
    uint32_t status = 0;
    int32_t level = 0, rounds = 0, cur = -1;
    bool done = false;
    if (st.lam_hat == 0) { status |= ST_DISCONNECTED; done = true; }
    while (!done && G.n > p.n0) {
      if (rounds >= p.max_rounds) { status |= ST_MAX_ROUNDS; break; }
      const int32_t r = rounds++;
      const int32_t n_start = G.n;
      if (p.lp_iters > 0) {
        auto tl = std::chrono::steady_clock::now();
        int32_t *Lc = w.La, *Lo = w.Lb;
        if (!(r == 0 && do_lp)) VC_TRY(lp_first(G, w, known, Lc, salt(r, 1), false, s));
        if (p.flags & VIECUT_F_RESTRICT) VC_TRY(restrict_first(G, w, Lc, s));
        trace_labels(r, 1, Lc, G.n);
        // convergence stop: the iterations end after one that changed at
        // most floor(n / 10000) labels
        const bool conv = (p.flags & VIECUT_F_CONVERGE) != 0;
        auto converged = [&](const int32_t *prev, const int32_t *cur, bool &stop) -> int {
          stop = false;
          if (!conv) return VIECUT_OK;
          VC_TRY(count_changed(prev, cur, G.n, w, s));
          const int rc2 = sync_status();
          if (rc2) return rc2;
          stop = st.lp_changed <= G.n / 10000;
          return VIECUT_OK;
        };
        bool stop_lp = false;
        rc = converged(nullptr, Lc, stop_lp);
        if (rc) return rc;
        for (int32_t t = 2; t <= p.lp_iters && !stop_lp; t++) {
          // (round 0, iteration 2 with the early tiles: only the long rows are left)
          VC_TRY(lp_iter(G, w, known, Lc, Lo, salt(r, t), s, nullptr, (early && r == 0 && t == 2) ? 2 : 0));
          std::swap(Lc, Lo);
          trace_labels(r, t, Lc, G.n);
          rc = converged(Lo, Lc, stop_lp);
          if (rc) return rc;
        }
        int64_t lspace = -1;
        if (p.flags & VIECUT_F_CORRECT) {  // misplaced vertices become singletons (labels n + v)
          VC_TRY(fix_misplaced(G, w, Lc, s));
          trace_labels(r, 0, Lc, G.n, 6);
          lspace = 2ll * G.n;
        }
        t_ms[1] += ms_since(tl);  // enqueue time: the LP kernels finish inside the contraction's first sync
        auto tc = std::chrono::steady_clock::now();
        rc = contract(Lc, G, cur, level, known, lspace);
        if (rc) return rc;
        t_ms[2] += ms_since(tc);
        if (st.stop) { status |= (uint32_t)st.stop; done = true; break; }
      }
      auto tp = std::chrono::steady_clock::now();
      VC_TRY(pr_mark(G, w, known, s));
      rc = sync_status();
      if (rc) return rc;
      refresh_known();
      trace_pr(r, level, G);
      if (st.nmarked > 0) {
        int32_t *rep = w.Lb;
        VC_TRY(union_find(G, w, known, rep, s));
        trace_rep(r, level, rep, G.n);
        rc = contract(rep, G, cur, level, known);
        if (rc) return rc;
        if (st.stop) { status |= (uint32_t)st.stop; done = true; t_ms[3] += ms_since(tp); break; }
      }
      t_ms[3] += ms_since(tp);
      if (G.n == n_start) { status |= ST_NO_PROGRESS; break; }
    }

    // exact solve on the remaining graph, transfer of the side
    auto te = std::chrono::steady_clock::now();
    int64_t cut = st.lam_hat;
    int32_t out_level = st.wit_level;
    bool from_kernel = false;
    if (!done && !(status & (ST_COLLAPSED | ST_DISCONNECTED)) && G.n >= 2 && G.n <= kDenseMax) {
      // small kernel graph: solved on the device, no hand-off to the host
      VC_TRY(exact_dense(G, w, side, s));
      rc = sync_status();
      if (rc) return rc;
      if (st.sw_cut < cut) {
        cut = st.sw_cut;
        out_level = -1;
      }
      from_kernel = true;  // the side is written
    } else if (!done && !(status & (ST_COLLAPSED | ST_DISCONNECTED)) && G.n >= 2) {
      const size_t b_rp = sizeof(int32_t) * ((size_t)G.n + 1), b_arc = sizeof(int32_t) * (size_t)G.nnz;
      char *stg = pinned ? pinned_stage(b_rp + 2 * b_arc) : nullptr;
      std::vector<int32_t> rp, col, ww;
      if (stg) {  // three copies, one wait
        rp.resize((size_t)G.n + 1);
        col.resize((size_t)G.nnz);
        ww.resize((size_t)G.nnz);
        VC_TRY(hipMemcpyAsync(stg, G.row_ptr, b_rp, hipMemcpyDeviceToHost, s));
        if (b_arc) {
          VC_TRY(hipMemcpyAsync(stg + b_rp, G.col, b_arc, hipMemcpyDeviceToHost, s));
          VC_TRY(hipMemcpyAsync(stg + b_rp + b_arc, G.w, b_arc, hipMemcpyDeviceToHost, s));
        }
        VC_TRY(hipStreamSynchronize(s));
        std::memcpy(rp.data(), stg, b_rp);
        if (b_arc) {
          std::memcpy(col.data(), stg + b_rp, b_arc);
          std::memcpy(ww.data(), stg + b_rp + b_arc, b_arc);
        }
      } else {
        rp = d2h(G.row_ptr, (int64_t)G.n + 1);
        col = d2h(G.col, G.nnz);
        ww = d2h(G.w, G.nnz);
      }
      std::vector<uint8_t> kside((size_t)G.n);
      int64_t lk = stoer_wagner_host(G.n, rp.data(), col.data(), ww.data(), kside.data());
      if (lk < cut) {
        cut = lk;
        out_level = -1;
        from_kernel = true;
        const uint8_t *src = kside.data();
        if (stg) {  // n flag bytes fit in the row-pointer part of the stage
          std::memcpy(stg, kside.data(), (size_t)G.n);
          src = (const uint8_t *)stg;
        }
        VC_TRY(hipMemcpyAsync(w.flags8, src, (size_t)G.n, hipMemcpyHostToDevice, s));
        VC_TRY(side_from_flags(w, w.flags8, side, s));
      }
    }
    if (!from_kernel) VC_TRY(side_from_witness(w, side, s));
    VC_TRY(hipStreamSynchronize(s));
    t_ms[4] = ms_since(te);
    t_ms[5] = ms_since(t0);
    out->cut = cut;
    out->rounds = rounds;
    out->kernel_n = G.n;
    out->witness_level = out_level;
    out->status_bits = status;
    out->levels = level;
    out->reserved = 0;
    std::memcpy(out->t_ms, t_ms, sizeof(t_ms));
    return VIECUT_OK;
  }
};

}  // namespace

int check_args(const viecut_csr *g, const viecut_params *p) {
  if (!g || !p) return VIECUT_EINVAL;
  if (g->n < 2 || g->nnz < 0 || !g->row_ptr) return VIECUT_EINVAL;
  if (g->n > kMaxVertices) return VIECUT_EOVERFLOW;
  if (g->nnz > 0 && (!g->col || !g->w)) return VIECUT_EINVAL;
  if (p->lp_iters < 0 || p->n0 < 0 || p->max_rounds < 0) return VIECUT_EINVAL;
  return VIECUT_OK;
}

int solve_one(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
              viecut_result *out, uint64_t *side, viecut_trace_fn fn, void *user) {
  int rc = check_args(g, p);
  if (rc) return rc;
  if (!out || !side) return VIECUT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  void *own = nullptr;
  size_t need = work_bytes(g->n, g->nnz);
  if (!ws) {
    if (hipMalloc(&own, need) != hipSuccess) return VIECUT_ENOMEM;
    ws = own;
    ws_bytes = need;
  }
  Work w;
  if (!carve(ws, ws_bytes, g->n, g->nnz, w)) {
    if (own) (void)hipFree(own);
    return VIECUT_ENOMEM;
  }
  Solver sv(w, s, *p);
  sv.tr.fn = fn;
  sv.tr.user = user;
  viecut_result res{};
  rc = sv.run(*g, &res, side);
  if (rc != VIECUT_OK) (void)hipStreamSynchronize(s);
  prof_collect();
  if (own) (void)hipFree(own);
  if (rc == VIECUT_OK) *out = res;
  return rc;
}

// The allocation-free single solve: the workspace is the calling device's
// static scratch array. One call at a time per device: a lock per device
// serialises the calls of this process, which all share that device's array
// (it keeps the last call's contents; every buffer that must start cleared is
// cleared by the solve itself).
int solve_noalloc(const viecut_csr *g, const viecut_params *p, void *stream, viecut_result *out,
                  uint64_t *side) {
  int rc = check_args(g, p);
  if (rc) return rc;
  if (!out || !side) return VIECUT_EINVAL;
  if (work_bytes(g->n, g->nnz) > kScratchBytes) return VIECUT_ETOOBIG;
  hipStream_t s = (hipStream_t)stream;
  int dev = -1;
  VC_TRY(hipGetDevice(&dev));
  if (s) {
    hipDevice_t sdev = -1;
    VC_TRY(hipStreamGetDevice(s, &sdev));
    if (sdev != dev) return VIECUT_EINVAL;  // the stream must belong to the current device
  }
  if (dev < 0 || dev >= kMaxScratchDevices) return VIECUT_EDEVICE;
  static std::mutex locks[kMaxScratchDevices];
  std::lock_guard<std::mutex> lk(locks[dev]);
  void *base = nullptr;
  VC_TRY(scratch_address(dev, &base));
  Work w;
  if (!carve(base, kScratchBytes, g->n, g->nnz, w)) return VIECUT_ETOOBIG;
  Solver sv(w, s, *p);
  sv.pinned = false;
  viecut_result res{};
  rc = sv.run(*g, &res, side);
  if (rc != VIECUT_OK) (void)hipStreamSynchronize(s);
  prof_collect();
  if (rc == VIECUT_OK) *out = res;
  return rc;
}

}  // namespace vc

// ============================================================ C ABI
extern "C" {

void viecut_default_params(viecut_params *p) {
  if (!p) return;
  p->lp_iters = 2;
  p->n0 = 10000;
  p->max_rounds = 64;
  p->flags = 0;
  p->seed = 0;
}

size_t viecut_workspace_bytes(int32_t n, int32_t nnz, const viecut_params *p) {
  (void)p;
  if (n < 2 || nnz < 0 || n > vc::kMaxVertices) return 0;
  return vc::work_bytes(n, nnz);
}

int viecut_mincut(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
                  viecut_result *out, uint64_t *side) {
  return vc::solve_one(g, p, ws, ws_bytes, stream, out, side, nullptr, nullptr);
}

int viecut_mincut_trace(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
                        viecut_result *out, uint64_t *side, viecut_trace_fn fn, void *user) {
  return vc::solve_one(g, p, ws, ws_bytes, stream, out, side, fn, user);
}

int viecut_mincut_noalloc(const viecut_csr *g, const viecut_params *p, void *stream, viecut_result *out,
                          uint64_t *side) {
  return vc::solve_noalloc(g, p, stream, out, side);
}

int viecut_validate(const viecut_csr *g, uint32_t flags, void *stream) {
  viecut_params p;
  viecut_default_params(&p);
  p.flags = flags;
  int rc = vc::check_args(g, &p);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  void *ws = nullptr;
  size_t need = vc::work_bytes(g->n, g->nnz);
  if (hipMalloc(&ws, need) != hipSuccess) return VIECUT_ENOMEM;
  vc::Work w;
  vc::carve(ws, need, g->n, g->nnz, w);
  vc::DGraph G;
  G.n = g->n; G.nnz = g->nnz; G.row_ptr = g->row_ptr; G.col = g->col; G.w = g->w;
  vc::Status st{};
  rc = VIECUT_OK;
  if (vc::status_reset(w.st, s) != hipSuccess || vc::check_rowptr(G, w.st, s) != hipSuccess ||
      vc::build_tiles(G, w, s) != hipSuccess || vc::lp_first(G, w, nullptr, w.La, 0u, true, s) != hipSuccess ||
      ((flags & VIECUT_F_VALIDATE) && vc::validate_sym(G, w.st, s) != hipSuccess) ||
      hipMemcpyAsync(&st, w.st, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = VIECUT_EDEVICE;
  (void)hipFree(ws);
  if (rc) return rc;
  if (st.err & (vc::ERR_ROWPTR | vc::ERR_COL | vc::ERR_SELF)) return VIECUT_EINVAL;
  if (st.err & vc::ERR_WEIGHT) return VIECUT_EWEIGHT;
  if (st.wsum / 2 > (unsigned long long)INT32_MAX) return VIECUT_EOVERFLOW;
  if (st.err & (vc::ERR_NOTSYM | vc::ERR_UNSORTED)) return VIECUT_ENOTSYM;
  return VIECUT_OK;
}

int viecut_profile_enable(int on) {
  vc::ProfState &p = vc::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (on) {
    if (!p.slots) {
      const int32_t cap = 1 << 16;
      if (hipHostMalloc((void **)&p.slots, 16 * (size_t)cap, 0) != hipSuccess) {
        p.slots = nullptr;
        return VIECUT_ENOMEM;
      }
      if (hipHostGetDevicePointer((void **)&p.dslots, p.slots, 0) != hipSuccess) {
        (void)hipHostFree(p.slots);
        p.slots = nullptr;
        return VIECUT_EDEVICE;
      }
      p.cap = cap;
    }
    for (int k = 0; k < vc::PROF_KINDS; k++) {
      p.launches[k] = 0;
      p.ms[k] = 0;
      p.bytes[k] = 0;
    }
  }
  p.on = on != 0;
  return VIECUT_OK;
}

int viecut_profile_read(viecut_kernel_stat *out, int32_t max) {
  if (max < 0 || (max > 0 && !out)) return VIECUT_EINVAL;
  vc::prof_collect();
  vc::ProfState &p = vc::prof();
  std::lock_guard<std::mutex> lk(p.mu);
  const int32_t k = std::min<int32_t>(max, vc::PROF_KINDS);
  for (int32_t i = 0; i < k; i++) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::strncpy(out[i].name, vc::kProfNames[i], sizeof(out[i].name) - 1);
    out[i].launches = p.launches[i];
    out[i].total_ms = p.ms[i];
    out[i].bytes = p.bytes[i];
  }
  return k;
}

const char *viecut_strerror(int code) {
  switch (code) {
    case VIECUT_OK: return "ok";
    case VIECUT_EINVAL: return "invalid argument or malformed CSR";
    case VIECUT_EWEIGHT: return "edge weight < 1";
    case VIECUT_EOVERFLOW: return "total edge weight exceeds INT32_MAX, or too many arcs or vertices";
    case VIECUT_ENOMEM: return "workspace too small or device allocation failed";
    case VIECUT_EDEVICE: return "HIP runtime error";
    case VIECUT_ENOTSYM: return "graph not symmetric or rows not strictly increasing";
    case VIECUT_EBUDGET: return "request exceeds the session memory budget";
    case VIECUT_ETOOBIG: return "graph needs more workspace than the static scratch of viecut_mincut_noalloc";
    default: return "unknown error";
  }
}

}  // extern "C"
