// Batched and served execution of the inexact minimum-cut method.
//
// Many graphs are solved as ONE disjoint union held in device memory: every
// phase of a round (label propagation, relabelling, emission, sort, coarse
// CSR build, Padberg-Rinaldi marking, union-find) is one launch over the
// arc tiles of all graphs at once, and the host synchronisations a round
// needs (sizes for the sort and the next level) are shared by the whole
// union. Each graph still follows its own loop (Algorithm 1 of the paper):
// per-graph state (GStat) on the device holds its level, round, bound,
// witness and stop bits, and small per-graph kernels apply the stop rules
// (<= n0 vertices, round cap, collapse, degree 0, no progress) exactly as
// the single-graph driver does. A graph that leaves the loop is dropped from
// the union at the next relabelling, its last level is copied out for the
// exact solve on the host, and its side bitmap is written through its own
// frozen input -> kernel map.
//
// The engine also serves a request stream (continuous batching): requests
// are admitted between rounds while the union has room (vertex, arc, word
// and slot capacities derived from the device-memory budget), are appended
// at the end of the union at level 0, and from then on advance one round
// per step together with graphs that are rounds ahead of them.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/viecut.h"
#include "vc_internal.h"

namespace vc {
namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
inline int bits_for_host(int32_t k) {
  int b = 0;
  while (b < 31 && (1 << b) < k) b++;
  return b;
}

// First-fit allocator over a range of 64-vertex words of the input index
// space (each admitted graph owns ceil(n/64) consecutive words).
class WordAlloc {
 public:
  void reset(int32_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int32_t alloc(int32_t len) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const int32_t start = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest > 0) free_[start + len] = rest;
        return start;
      }
    }
    return -1;
  }
  void release(int32_t start, int32_t len) {
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        prev->second += len;
        return;
      }
    }
    free_[start] = len;
  }

 private:
  std::map<int32_t, int32_t> free_;  // start -> length
};

// Page-locked host buffer, grown on demand.
struct Pinned {
  void *p = nullptr;
  size_t bytes = 0;
  Pinned() = default;
  Pinned(const Pinned &) = delete;
  Pinned &operator=(const Pinned &) = delete;
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
  bool ensure(size_t b) {
    if (b <= bytes) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, b, 0) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = b;
    return true;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

struct ReqRec {
  viecut_csr g{};
  uint64_t *side = nullptr;
  int64_t id = 0;
  int32_t slot = -1, woff = -1, words = 0;
  double t_submit = 0, t_admit = 0;
};

struct DoneRec {
  int64_t id;
  viecut_result res;
  double t_submit;
};

// Capacities of one engine workspace.
struct Caps {
  int32_t n = 0;   // union vertices
  int64_t a = 0;   // union arcs
  int32_t w = 0;   // 64-vertex words of the input index space
  int32_t s = 0;   // graph slots
};

struct Extras {
  size_t gv0, gv1, gs, ring, wg, desc, gdesc, sdesc, total;
};
Extras extras_layout(const Caps &c) {
  Extras e{};
  size_t off = 0;
  auto add = [&](size_t b) {
    size_t o = off;
    off += al256(b);
    return o;
  };
  e.gv0 = add(4 * (size_t)c.n + 4);
  e.gv1 = add(4 * (size_t)c.n + 4);
  e.gs = add(sizeof(GStat) * (size_t)c.s);
  e.ring = add(sizeof(GStat) * (size_t)c.s);
  e.wg = add(4 * (size_t)c.w + 4);
  e.desc = add(sizeof(GDesc) * (size_t)c.s);
  e.gdesc = add(sizeof(GatherDesc) * (size_t)c.s);
  e.sdesc = add(sizeof(SideDesc) * (size_t)c.s);
  e.total = off;
  return e;
}

size_t engine_bytes(const Caps &c) {
  return al256(work_bytes(std::max(c.n, 2), std::max<int64_t>(c.a, 1), 64ll * c.w, c.s)) + extras_layout(c).total +
         256;
}

#define VC_TRY(x)                                \
  do {                                           \
    hipError_t e_ = (x);                         \
    if (e_ != hipSuccess) return VIECUT_EDEVICE; \
  } while (0)

// input error bits of a graph -> status code (same precedence as a single solve)
int error_code(const GStat &e) {
  if (e.err & (ERR_ROWPTR | ERR_COL | ERR_SELF)) return VIECUT_EINVAL;
  if (e.err & ERR_WEIGHT) return VIECUT_EWEIGHT;
  if (e.wsum / 2 > (unsigned long long)INT32_MAX) return VIECUT_EOVERFLOW;
  if (e.err & (ERR_NOTSYM | ERR_UNSORTED)) return VIECUT_ENOTSYM;
  return VIECUT_EINVAL;
}

struct Engine {
  viecut_params p{};
  hipStream_t s = nullptr;
  Caps cap;
  void *ws = nullptr;
  bool own_ws = false;
  Work w;
  int32_t *gvb[2] = {nullptr, nullptr};
  GStat *gs = nullptr, *ring = nullptr;
  int32_t *wg = nullptr;
  GDesc *d_desc = nullptr;
  GatherDesc *d_gdesc = nullptr;
  SideDesc *d_sdesc = nullptr;
  Pinned h_st, h_ring, h_desc, h_gdesc, h_sdesc, h_rp, h_col, h_w, h_flags;
  // the union
  int32_t N = 0;
  int64_t A = 0;
  int cur = 1, gvc = 0;
  bool tiles_valid = false;
  int32_t known_buf[8] = {0};
  const int32_t *known = nullptr;
  // graphs
  int32_t n_active = 0, drained = 0;
  WordAlloc words;
  std::vector<int32_t> free_slots;
  // slots of finished graphs whose rows may still be in the union: a graph
  // that leaves the loop keeps its rows until the next relabelling drops
  // them (it does so for every graph not in the loop), and a slot reused
  // before that would make those rows count as the new graph's
  std::vector<int32_t> zombie_slots;
  std::vector<ReqRec> slot_req;
  std::deque<ReqRec> pending;
  std::vector<DoneRec> staged, ready;
  unsigned n_threads = 1;
  // phase times (host clock, ms) for VIECUT_LOG=1 diagnostics
  bool verbose = false;
  double t_sync = 0, t_drain_read = 0, t_gather = 0, t_solve = 0, t_side = 0, t_admit = 0, t_init = 0;
  int64_t n_syncs = 0, n_steps = 0, n_solved = 0;

  Engine(const Engine &) = delete;
  Engine &operator=(const Engine &) = delete;
  Engine() = default;
  ~Engine() {
    if (own_ws && ws) (void)hipFree(ws);
  }

  Status *hst() { return h_st.as<Status>(); }

  int init(const Caps &c, const viecut_params &prm, hipStream_t stream, void *buf, size_t bytes) {
    p = prm;
    s = stream;
    cap = c;
    cap.n = std::max(cap.n, 2);
    cap.a = std::max<int64_t>(cap.a, 1);
    cap.s = std::max(cap.s, 1);
    cap.w = std::max(cap.w, 1);
    if (cap.a >= INT32_MAX || (int64_t)cap.n + cap.s > kMaxVertices || 64ll * cap.w >= INT32_MAX)
      return VIECUT_EOVERFLOW;
    const size_t need = engine_bytes(cap);
    if (!buf) {
      if (hipMalloc(&buf, need) != hipSuccess) return VIECUT_ENOMEM;
      own_ws = true;
      bytes = need;
    }
    ws = buf;
    if (bytes < need) return VIECUT_ENOMEM;
    const size_t core = al256(work_bytes(cap.n, cap.a, 64ll * cap.w, cap.s));
    if (!carve(ws, core, cap.n, cap.a, w, 64ll * cap.w, cap.s)) return VIECUT_ENOMEM;
    const uintptr_t base = (((uintptr_t)ws + 255) & ~uintptr_t(255)) + core;
    const Extras e = extras_layout(cap);
    gvb[0] = (int32_t *)(base + e.gv0);
    gvb[1] = (int32_t *)(base + e.gv1);
    gs = (GStat *)(base + e.gs);
    ring = (GStat *)(base + e.ring);
    wg = (int32_t *)(base + e.wg);
    d_desc = (GDesc *)(base + e.desc);
    d_gdesc = (GatherDesc *)(base + e.gdesc);
    d_sdesc = (SideDesc *)(base + e.sdesc);
    if (!h_st.ensure(sizeof(Status)) || !h_ring.ensure(sizeof(GStat) * cap.s) ||
        !h_desc.ensure(sizeof(GDesc) * cap.s) || !h_gdesc.ensure(sizeof(GatherDesc) * cap.s) ||
        !h_sdesc.ensure(sizeof(SideDesc) * cap.s))
      return VIECUT_ENOMEM;
    VC_TRY(status_reset(w.st, s));
    VC_TRY(fill_i32((int32_t *)gs, 0, (int64_t)sizeof(GStat) / 4 * cap.s, s));  // all slots GS_FREE
    VC_TRY(fill_i32(wg, -1, cap.w, s));
    VC_TRY(hipStreamSynchronize(s));
    words.reset(cap.w);
    free_slots.clear();
    for (int32_t i = cap.s - 1; i >= 0; i--) free_slots.push_back(i);
    slot_req.assign(cap.s, ReqRec{});
    n_threads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const char *lg = getenv("VIECUT_LOG");
    verbose = lg && lg[0] == '1';
    return VIECUT_OK;
  }

  // whether a graph of this size can ever be admitted
  bool fits_ever(const viecut_csr &g) const {
    return g.n <= cap.n && (int64_t)g.nnz <= cap.a && (g.n + 63) / 64 <= cap.w;
  }

  void submit(const viecut_csr &g, uint64_t *side, int64_t id, double t) {
    ReqRec r;
    r.g = g;
    r.side = side;
    r.id = id;
    r.t_submit = t;
    pending.push_back(r);
  }

  int sync_status() {
    const double t0 = now_ms();
    VC_TRY(hipMemcpyAsync(hst(), w.st, sizeof(Status), hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    t_sync += now_ms() - t0;
    n_syncs++;
    if (hst()->err & ERR_DEVICE) return VIECUT_EDEVICE;
    return VIECUT_OK;
  }

  // ------------------------------------------------------------ admission
  // Pending requests (in order) join the union at its end while they fit.
  int admit(int32_t &n_fresh, int32_t &N0) {
    n_fresh = 0;
    if (n_active == 0) {  // nothing in the loop and everything drained: restart the union
      N = 0;
      A = 0;
      free_slots.insert(free_slots.end(), zombie_slots.begin(), zombie_slots.end());
      zombie_slots.clear();
    }
    N0 = N;
    std::vector<GDesc> fd;
    int32_t rch = 0, ach = 0;
    const double t = now_ms();
    while (!pending.empty()) {
      ReqRec &r = pending.front();
      if (free_slots.empty()) break;
      if ((int64_t)N + r.g.n > cap.n || A + r.g.nnz > cap.a) break;
      const int32_t nw = (r.g.n + 63) / 64;
      const int32_t woff = words.alloc(nw);
      if (woff < 0) break;
      const int32_t slot = free_slots.back();
      free_slots.pop_back();
      GDesc d{};
      d.rp = r.g.row_ptr;
      d.col = r.g.col;
      d.w = r.g.w;
      d.n = r.g.n;
      d.nnz = r.g.nnz;
      d.voff = N;
      d.aoff = (int32_t)A;
      d.woff = woff;
      d.words = nw;
      d.slot = slot;
      d.rchunk0 = rch;
      d.achunk0 = ach;
      rch += (int32_t)((64ll * nw + kPackRows - 1) / kPackRows);
      ach += (int32_t)(((int64_t)r.g.nnz + kPackArcs - 1) / kPackArcs);
      N += r.g.n;
      A += r.g.nnz;
      r.slot = slot;
      r.woff = woff;
      r.words = nw;
      r.t_admit = t;
      slot_req[slot] = r;
      pending.pop_front();
      fd.push_back(d);
    }
    if (fd.empty()) return VIECUT_OK;
    n_fresh = (int32_t)fd.size();
    std::memcpy(h_desc.p, fd.data(), sizeof(GDesc) * fd.size());
    VC_TRY(hipMemcpyAsync(d_desc, h_desc.p, sizeof(GDesc) * fd.size(), hipMemcpyHostToDevice, s));
    VC_TRY(b_gs_init(gs, d_desc, n_fresh, cur, s));
    VC_TRY(b_pack(d_desc, n_fresh, rch, ach, gvb[gvc], w.map, wg, w.rp[cur], w.col[cur], w.w[cur], gs, s));
    tiles_valid = false;
    return VIECUT_OK;
  }

  // ------------------------------------------------------------ finished graphs
  // Reads the ring entries pushed since the last drain, runs the exact solve
  // on the graphs that need it, writes every side bitmap and records the
  // results (readable once the stream has passed the side kernel).
  int drain() {
    const int32_t cnt = hst()->ring_cnt;
    n_active = hst()->active_cnt;
    if (cnt == drained) return VIECUT_OK;
    const int32_t m = cnt - drained;
    if (m > cap.s) return VIECUT_EDEVICE;  // cannot happen: one entry per admitted graph between drains
    const int32_t first = drained % cap.s;
    const int32_t n1 = std::min(m, cap.s - first);
    double t0 = now_ms();
    GStat *he = h_ring.as<GStat>();
    VC_TRY(hipMemcpyAsync(he, ring + first, sizeof(GStat) * n1, hipMemcpyDeviceToHost, s));
    if (m > n1) VC_TRY(hipMemcpyAsync(he + n1, ring, sizeof(GStat) * (m - n1), hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    drained = cnt;
    t_drain_read += now_ms() - t0;

    // exact solve on the last level of graphs that left the loop unsolved:
    // kernel graphs of at most kDenseMax vertices on the device, one wave
    // each, in place; larger ones gathered and solved on host threads
    std::vector<int32_t> solve, dense;
    for (int32_t i = 0; i < m; i++)
      if (he[i].fin == FIN_SOLVE && he[i].k >= 2 && he[i].lam_hat > 0)
        (he[i].k <= kDenseMax ? dense : solve).push_back(i);
    std::vector<int64_t> lk(m, INT64_MAX);
    std::vector<int64_t> foff(m, -1);
    int64_t fdev = 0;  // flags written by the device solve come first
    if (!dense.empty()) {
      static_assert(sizeof(SwDesc) <= sizeof(GatherDesc), "descriptor staging");
      static_assert(sizeof(long long) <= sizeof(SideDesc), "cut staging");
      t0 = now_ms();
      SwDesc *sd = h_gdesc.as<SwDesc>();
      int32_t kmax = 2;
      for (size_t j = 0; j < dense.size(); j++) {
        const GStat &e = he[dense[j]];
        SwDesc d{};
        d.rp = w.rp[e.buf];
        d.col = w.col[e.buf];
        d.w = w.w[e.buf];
        d.base = e.base;
        d.k = e.k;
        d.foff = (int32_t)fdev;
        fdev += e.k;
        kmax = std::max(kmax, e.k);
        sd[j] = d;
      }
      if (fdev > (int64_t)cap.n + 1) return VIECUT_EDEVICE;  // one level holds them all
      // the side descriptors' buffers are free until the side step below
      long long *dcut = (long long *)d_sdesc, *hcut = h_sdesc.as<long long>();
      VC_TRY(hipMemcpyAsync(d_gdesc, sd, sizeof(SwDesc) * dense.size(), hipMemcpyHostToDevice, s));
      VC_TRY(exact_dense_batch((const SwDesc *)d_gdesc, (int32_t)dense.size(), kmax, w.flags8, dcut, s));
      VC_TRY(hipMemcpyAsync(hcut, dcut, sizeof(long long) * dense.size(), hipMemcpyDeviceToHost, s));
      VC_TRY(hipStreamSynchronize(s));
      for (size_t j = 0; j < dense.size(); j++) {
        const int32_t i = dense[j];
        lk[i] = hcut[j];
        if (hcut[j] < he[i].lam_hat) foff[i] = sd[j].foff;
      }
      n_solved += (int64_t)dense.size();
      t_solve += now_ms() - t0;
    }
    std::vector<uint8_t> flags;
    size_t pos = 0;
    while (pos < solve.size()) {  // in groups that fit the staging buffers
      GatherDesc *gd = h_gdesc.as<GatherDesc>();
      int64_t rows = 0, arcs = 0;
      int32_t rch = 0, ach = 0, cnt_g = 0;
      const int64_t row_cap = (int64_t)cap.n + cap.s + 1, arc_cap = cap.a;
      size_t end = pos;
      while (end < solve.size()) {
        const GStat &e = he[solve[end]];
        if (cnt_g > 0 && (rows + e.k + 1 > row_cap || arcs + e.nnz > arc_cap)) break;
        GatherDesc d{};
        d.rp = w.rp[e.buf];
        d.col = w.col[e.buf];
        d.w = w.w[e.buf];
        d.base = e.base;
        d.k = e.k;
        d.aoff = e.aoff;
        d.nnz = e.nnz;
        d.drp = (int32_t)rows;
        d.darc = (int32_t)arcs;
        d.rchunk0 = rch;
        d.achunk0 = ach;
        rch += (e.k + 1 + kPackRows - 1) / kPackRows;
        ach += (e.nnz + kPackArcs - 1) / kPackArcs;
        rows += e.k + 1;
        arcs += e.nnz;
        gd[cnt_g++] = d;
        end++;
      }
      if (!h_rp.ensure(4 * (size_t)rows) || !h_col.ensure(4 * (size_t)std::max<int64_t>(arcs, 1)) ||
          !h_w.ensure(4 * (size_t)std::max<int64_t>(arcs, 1)))
        return VIECUT_ENOMEM;
      t0 = now_ms();
      int32_t *srp = w.cnt, *scol = (int32_t *)w.keys[0], *sw = w.vals[0];  // free at every drain point
      VC_TRY(hipMemcpyAsync(d_gdesc, gd, sizeof(GatherDesc) * cnt_g, hipMemcpyHostToDevice, s));
      VC_TRY(b_gather(d_gdesc, cnt_g, rch, ach, srp, scol, sw, s));
      VC_TRY(hipMemcpyAsync(h_rp.p, srp, 4 * (size_t)rows, hipMemcpyDeviceToHost, s));
      if (arcs > 0) {
        VC_TRY(hipMemcpyAsync(h_col.p, scol, 4 * (size_t)arcs, hipMemcpyDeviceToHost, s));
        VC_TRY(hipMemcpyAsync(h_w.p, sw, 4 * (size_t)arcs, hipMemcpyDeviceToHost, s));
      }
      VC_TRY(hipStreamSynchronize(s));
      t_gather += now_ms() - t0;
      t0 = now_ms();
      // solve the group on host threads
      std::vector<std::vector<uint8_t>> kside(cnt_g);
      std::vector<int64_t> kcut(cnt_g);
      std::atomic<int32_t> next{0};
      auto work = [&]() {
        for (int32_t j; (j = next.fetch_add(1)) < cnt_g;) {
          const GatherDesc &d = gd[j];
          kside[j].assign((size_t)d.k, 0);
          kcut[j] = stoer_wagner_host(d.k, h_rp.as<int32_t>() + d.drp, h_col.as<int32_t>() + d.darc,
                                      h_w.as<int32_t>() + d.darc, kside[j].data());
        }
      };
      const unsigned nt = std::min<unsigned>(n_threads, (unsigned)cnt_g);
      if (nt <= 1 || arcs < 20000) {
        work();
      } else {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; t++) th.emplace_back(work);
        for (auto &t : th) t.join();
      }
      t_solve += now_ms() - t0;
      n_solved += cnt_g;
      for (int32_t j = 0; j < cnt_g; j++) {
        const int32_t i = solve[pos + j];
        lk[i] = kcut[j];
        if (kcut[j] < he[i].lam_hat) {
          foff[i] = fdev + (int64_t)flags.size();
          flags.insert(flags.end(), kside[j].begin(), kside[j].end());
        }
      }
      pos = end;
    }

    // sides and results
    t0 = now_ms();
    if (!flags.empty()) {
      if (fdev + flags.size() > (size_t)cap.n + 1) return VIECUT_EDEVICE;  // one level holds them all
      if (!h_flags.ensure(flags.size())) return VIECUT_ENOMEM;
      std::memcpy(h_flags.p, flags.data(), flags.size());
      VC_TRY(hipMemcpyAsync(w.flags8 + fdev, h_flags.p, flags.size(), hipMemcpyHostToDevice, s));
    }
    SideDesc *sd = h_sdesc.as<SideDesc>();
    int32_t wsum = 0;
    for (int32_t i = 0; i < m; i++) {
      const GStat &e = he[i];
      ReqRec &r = slot_req[e.slot];
      SideDesc d{};
      d.side = (unsigned long long *)r.side;
      d.woff = r.woff;
      d.n = r.g.n;
      d.wchunk0 = wsum;
      viecut_result res{};
      if (e.fin == FIN_ERROR) {
        d.mode = 2;
        res.status_bits = 0x80000000u | (uint32_t)(-error_code(e));
      } else {
        res.cut = e.lam_hat;
        res.rounds = e.rounds;
        res.kernel_n = e.k;
        res.witness_level = e.wit_level;
        res.status_bits = (uint32_t)e.status;
        res.levels = e.level;
        d.mode = 0;
        if (foff[i] >= 0) {
          res.cut = lk[i];
          res.witness_level = -1;
          d.mode = 1;
          d.foff = (int32_t)foff[i];
          d.fbase = e.base;
        }
      }
      res.t_ms[6] = (float)(r.t_admit - r.t_submit);
      sd[i] = d;
      wsum += r.words;
      staged.push_back(DoneRec{r.id, res, r.t_submit});
      words.release(r.woff, r.words);
      zombie_slots.push_back(e.slot);
    }
    VC_TRY(hipMemcpyAsync(d_sdesc, sd, sizeof(SideDesc) * m, hipMemcpyHostToDevice, s));
    VC_TRY(b_side(d_sdesc, m, wsum, w.map, w.witness, w.flags8, wg, s));
    // the descriptors in pinned memory must not change before the copies ran
    VC_TRY(hipStreamSynchronize(s));
    t_side += now_ms() - t0;
    return VIECUT_OK;
  }

  void report(const char *what) const {
    if (!verbose) return;
    fprintf(stderr,
            "[viecut] %s: init %.2f ms, steps %lld syncs %lld (%.2f ms) ring read %.2f ms, gather %.2f ms, exact "
            "solves %lld (%.2f ms), sides %.2f ms, admission %.2f ms\n",
            what, t_init, (long long)n_steps, (long long)n_syncs, t_sync, t_drain_read, t_gather, (long long)n_solved,
            t_solve, t_side, t_admit);
  }

  // results whose side kernels have completed become readable; t_ms[5] is
  // the latency from submission
  void publish() {
    const double t = now_ms();
    for (auto &d : staged) {
      d.res.t_ms[5] = (float)(t - d.t_submit);
      ready.push_back(d);
    }
    staged.clear();
  }

  // ------------------------------------------------------------ contraction
  // mode 0: clusters of the labels L; mode 1: components of marked edges
  int contract(const int32_t *L, int mode, DGraph &G) {
    BatchView bv{gvb[gvc], gs, cap.s};
    // this relabelling drops the rows of every graph already finished: their
    // slots can be reused by admissions after it (in stream order)
    std::vector<int32_t> release;
    release.swap(zombie_slots);
    VC_TRY(relabel(L, G.n, w, s, &bv, gvb[gvc ^ 1]));
    free_slots.insert(free_slots.end(), release.begin(), release.end());
    VC_TRY(b_gsizes(gs, cap.s, w.ids, mode, w.st, s));
    VC_TRY(b_compose(w.map, w.cl, 64ll * cap.w, wg, gs, s));
    VC_TRY(contract_emit(G, w, known, s, &bv));
    int rc = sync_status();
    if (rc) return rc;
    rc = drain();
    if (rc) return rc;
    const int32_t K = hst()->k;
    const int64_t ax = hst()->ax;
    if (K == 0) {  // every graph has left the loop
      N = 0;
      A = 0;
      G = DGraph{};
      tiles_valid = false;
      return VIECUT_OK;
    }
    // keys: (new vertex) << lb | (neighbour minus its graph's first new vertex)
    const int kb = bits_for_host(K), lb = bits_for_host(hst()->kloc);
    int which = 1;
    VC_TRY(radix_sort(w, ax, kb + lb, which, s));
    const int dst = cur ^ 1;
    VC_TRY(contract_build(w, which, ax, lb, K, dst, 0, s, false, gvb[gvc ^ 1], gs));
    gvc ^= 1;
    cur = dst;
    VC_TRY(b_gdeg(w.deg, 0, K, gvb[gvc], gs, false, s));
    VC_TRY(b_gbound(gs, cap.s, w.rp[cur], cur, w.st, ring, cap.s, s));
    VC_TRY(b_gwitness(w.map, wg, gs, cap.w, w.witness, s));
    rc = sync_status();
    if (rc) return rc;
    rc = drain();
    if (rc) return rc;
    G.n = K;
    G.nnz = hst()->nnz;
    G.row_ptr = w.rp[cur];
    G.col = w.col[cur];
    G.w = w.w[cur];
    N = K;
    A = G.nnz;
    VC_TRY(reset_bins(w, s));
    VC_TRY(build_tiles(G, w, s));
    known = nullptr;
    tiles_valid = true;
    return VIECUT_OK;
  }

  // ------------------------------------------------------------ one round
  // Admits what fits, then runs one round for every graph in the loop.
  int step() {
    int32_t n_fresh = 0, N0 = 0;
    const double ta = now_ms();
    int rc = admit(n_fresh, N0);
    t_admit += now_ms() - ta;
    if (rc) return rc;
    if (n_active == 0 && n_fresh == 0) return VIECUT_OK;
    n_steps++;
    DGraph G;
    G.n = N;
    G.nnz = A;
    G.row_ptr = w.rp[cur];
    G.col = w.col[cur];
    G.w = w.w[cur];
    if (!tiles_valid) {
      VC_TRY(reset_bins(w, s));
      VC_TRY(build_tiles(G, w, s));
      known = nullptr;
      tiles_valid = true;
    }
    const BatchView bv{gvb[gvc], gs, cap.s};
    // first LP iteration; at level 0 of fresh graphs it also validates and
    // yields the weighted degrees
    VC_TRY(b_salts(gs, cap.s, p.seed, p.lp_iters, 1, true, s));
    VC_TRY(lp_first(G, w, known, w.La, 0u, n_fresh > 0, s, &bv));
    if (n_fresh > 0) {
      if (p.flags & VIECUT_F_VALIDATE) VC_TRY(validate_sym(G, w.st, s, &bv));
      VC_TRY(b_gdeg(w.deg, N0, N, gvb[gvc], gs, true, s));
      VC_TRY(b_gbound0(gs, cap.s, w.st, ring, cap.s, s));
      VC_TRY(b_gwitness(w.map, wg, gs, cap.w, w.witness, s));
    }
    VC_TRY(b_step_top(gs, cap.s, p.n0, p.max_rounds, w.st, ring, cap.s, s));
    int32_t *Lc = w.La, *Lo = w.Lb;
    for (int32_t t = 2; t <= p.lp_iters; t++) {
      VC_TRY(b_salts(gs, cap.s, p.seed, p.lp_iters, t, false, s));
      VC_TRY(lp_iter(G, w, known, Lc, Lo, 0u, s, &bv));
      std::swap(Lc, Lo);
    }
    if (p.lp_iters > 0) {
      rc = contract(Lc, 0, G);
      if (rc) return rc;
    }
    if (G.n > 0) {
      const BatchView bv2{gvb[gvc], gs, cap.s};
      VC_TRY(pr_mark(G, w, known, s, &bv2));
      rc = sync_status();
      if (rc) return rc;
      rc = drain();
      if (rc) return rc;
      std::memcpy(known_buf, hst()->bin_cnt, sizeof(known_buf));
      known = known_buf;
      if (hst()->nmarked > 0) {
        VC_TRY(union_find(G, w, known, w.Lb, s));
        rc = contract(w.Lb, 1, G);
        if (rc) return rc;
      }
    }
    VC_TRY(b_step_end(gs, cap.s, w.st, ring, cap.s, s));
    rc = sync_status();
    if (rc) return rc;
    rc = drain();
    if (rc) return rc;
    if (tiles_valid && known == nullptr) {
      std::memcpy(known_buf, hst()->bin_cnt, sizeof(known_buf));
      known = known_buf;
    }
    publish();
    prof_collect();
    return VIECUT_OK;
  }

  int32_t in_flight() const { return n_active + (int32_t)pending.size(); }
};

// Capacities for a device-memory budget: arcs and vertices in a 4 : 1
// ratio (average degree >= 4), slots for up to 4096 graphs in flight.
Caps caps_for_budget(size_t budget) {
  Caps c;
  c.s = 4096;
  int64_t lo = 0, hi = INT32_MAX - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    Caps t;
    t.a = mid;
    t.n = (int32_t)std::max<int64_t>(2, mid / 4);
    t.s = c.s;
    t.w = t.n / 64 + t.s;
    if (engine_bytes(t) <= budget) lo = mid; else hi = mid - 1;
  }
  c.a = lo;
  c.n = (int32_t)std::max<int64_t>(2, lo / 4);
  c.w = c.n / 64 + c.s;
  return c;
}

}  // namespace
}  // namespace vc

// ============================================================ serving lanes
namespace vc {
namespace {
// A session serves requests in two lanes, each an Engine with its own union,
// workspace and stream: requests of up to kSmallLaneArcs arcs go to the small
// lane, which the caller's thread steps, and larger ones to the large lane,
// which a worker thread steps on its own stream. A round of large graphs
// (tens of milliseconds) then no longer holds the rounds of small requests
// that arrive meanwhile (they overlap on the device), and each lane's host
// work (admission, exact solves) overlaps the other lane's kernels. Every
// request's arithmetic is that of a solo solve in either lane.
constexpr int64_t kSmallLaneArcs = 1 << 20;
}  // namespace
}  // namespace vc

struct viecut_session {
  vc::Engine small, large;
  size_t budget = 0;
  hipStream_t large_stream = nullptr;
  std::thread worker;
  std::mutex mu;                       // guards everything below
  std::condition_variable cv_work;     // worker: new large requests or stop
  std::condition_variable cv_done;     // caller: the large lane finished a step
  std::deque<vc::ReqRec> large_in;     // submitted, not yet handed to the large lane
  std::vector<vc::DoneRec> large_ready;
  int32_t large_in_flight = 0;
  int64_t large_steps = 0;
  int large_err = VIECUT_OK;
  bool stop = false;
  bool two_lanes = false;  // false: a budget too small to split, every request in the one lane

  void run_large() {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      cv_work.wait(lk, [&] { return stop || !large_in.empty() || large_in_flight > 0; });
      if (stop) return;
      while (!large_in.empty()) {
        const vc::ReqRec &r = large_in.front();
        large.submit(r.g, r.side, r.id, r.t_submit);
        large_in.pop_front();
      }
      lk.unlock();
      const int rc = large.step();
      lk.lock();
      if (rc && large_err == VIECUT_OK) large_err = rc;
      for (const auto &d : large.ready) large_ready.push_back(d);
      large.ready.clear();
      large_in_flight = rc ? 0 : large.in_flight();
      large_steps++;
      cv_done.notify_all();
      if (rc) {
        large_in.clear();
        cv_work.wait(lk, [&] { return stop; });
        return;
      }
    }
  }
};

extern "C" {

size_t viecut_batch_workspace_bytes(const viecut_csr *gs, int32_t count, const viecut_params *p) {
  if (!gs || !p || count < 0) return 0;
  vc::Caps c;
  for (int32_t i = 0; i < count; i++) {
    if (vc::check_args(&gs[i], p)) continue;
    c.n += gs[i].n;
    c.a += gs[i].nnz;
    c.w += (gs[i].n + 63) / 64;
    c.s += 1;
  }
  if (c.a >= INT32_MAX || (int64_t)c.n + c.s > vc::kMaxVertices || 64ll * c.w >= INT32_MAX) return 0;
  return vc::engine_bytes(c);
}

int viecut_mincut_batch(const viecut_csr *gs, int32_t count, const viecut_params *p, void *ws, size_t ws_bytes,
                        void *stream, viecut_result *outs, uint64_t *const *sides) {
  if (!gs || !p || !outs || !sides || count < 0) return VIECUT_EINVAL;
  viecut_params q = *p;
  if (q.lp_iters < 0 || q.n0 < 0 || q.max_rounds < 0) return VIECUT_EINVAL;
  // the correcting step and the label-propagation variants run on the single path only
  if (q.flags & (VIECUT_F_CORRECT | VIECUT_F_CONVERGE | VIECUT_F_RESTRICT)) return VIECUT_EINVAL;
  vc::Caps c;
  for (int32_t i = 0; i < count; i++) {
    const int rc = vc::check_args(&gs[i], p);
    if (rc || !sides[i]) {
      outs[i] = viecut_result{};
      outs[i].status_bits = 0x80000000u | (uint32_t)(-(rc ? rc : VIECUT_EINVAL));
      continue;
    }
    c.n += gs[i].n;
    c.a += gs[i].nnz;
    c.w += (gs[i].n + 63) / 64;
    c.s += 1;
  }
  if (c.s == 0) return VIECUT_OK;
  if (c.a >= INT32_MAX || (int64_t)c.n + c.s > vc::kMaxVertices || 64ll * c.w >= INT32_MAX) return VIECUT_EOVERFLOW;
  vc::Engine eng;
  const double ti = vc::now_ms();
  int rc = eng.init(c, q, (hipStream_t)stream, ws, ws_bytes);
  eng.t_init = vc::now_ms() - ti;
  if (rc) return rc;
  const double t0 = vc::now_ms();
  for (int32_t i = 0; i < count; i++)
    if (vc::check_args(&gs[i], p) == VIECUT_OK && sides[i]) eng.submit(gs[i], sides[i], i, t0);
  while (eng.in_flight() > 0) {
    rc = eng.step();
    if (rc) {
      (void)hipStreamSynchronize((hipStream_t)stream);
      return rc;
    }
  }
  for (const auto &d : eng.ready) outs[d.id] = d.res;
  eng.report("batch");
  return VIECUT_OK;
}

int viecut_session_create(size_t hbm_budget, const viecut_params *p, void *stream, viecut_session **out) {
  if (!p || !out) return VIECUT_EINVAL;
  if (p->lp_iters < 0 || p->n0 < 0 || p->max_rounds < 0) return VIECUT_EINVAL;
  // the correcting step and the label-propagation variants run on the single path only
  if (p->flags & (VIECUT_F_CORRECT | VIECUT_F_CONVERGE | VIECUT_F_RESTRICT)) return VIECUT_EINVAL;
  // a quarter of the budget for the small lane, the rest for the large one;
  // a budget whose quarter cannot hold a small-lane request keeps one lane
  vc::Caps cs = vc::caps_for_budget(hbm_budget / 4);
  vc::Caps cl = vc::caps_for_budget(hbm_budget - hbm_budget / 4);
  const bool two = cs.a >= vc::kSmallLaneArcs && cl.a >= 1;
  if (!two) cs = vc::caps_for_budget(hbm_budget);
  if (cs.a < 1) return VIECUT_EBUDGET;
  viecut_session *ss = new (std::nothrow) viecut_session;
  if (!ss) return VIECUT_ENOMEM;
  ss->budget = hbm_budget;
  ss->two_lanes = two;
  if (two && hipStreamCreateWithFlags(&ss->large_stream, hipStreamNonBlocking) != hipSuccess) {
    delete ss;
    return VIECUT_EDEVICE;
  }
  int rc = ss->small.init(cs, *p, (hipStream_t)stream, nullptr, 0);
  if (!rc && two) rc = ss->large.init(cl, *p, ss->large_stream, nullptr, 0);
  if (rc) {
    hipStream_t ls = ss->large_stream;
    if (ls) (void)hipStreamSynchronize(ls);
    delete ss;
    if (ls) (void)hipStreamDestroy(ls);
    return rc;
  }
  if (two) ss->worker = std::thread([ss] { ss->run_large(); });
  *out = ss;
  return VIECUT_OK;
}

int viecut_session_submit(viecut_session *s, const viecut_csr *g, uint64_t *side, int64_t request_id) {
  if (!s || !g || !side) return VIECUT_EINVAL;
  const int rc = vc::check_args(g, &s->small.p);
  if (rc) return rc;
  const double t = vc::now_ms();
  if (!s->two_lanes || ((int64_t)g->nnz <= vc::kSmallLaneArcs && s->small.fits_ever(*g))) {
    if (!s->small.fits_ever(*g)) return VIECUT_EBUDGET;
    s->small.submit(*g, side, request_id, t);
    return VIECUT_OK;
  }
  if (!s->large.fits_ever(*g)) return VIECUT_EBUDGET;
  vc::ReqRec r;
  r.g = *g;
  r.side = side;
  r.id = request_id;
  r.t_submit = t;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->large_in.push_back(r);
  }
  s->cv_work.notify_one();
  return VIECUT_OK;
}

int viecut_session_step(viecut_session *s, int32_t *n_active) {
  if (!s) return VIECUT_EINVAL;
  int rc = VIECUT_OK;
  if (s->small.in_flight() > 0) {
    rc = s->small.step();
  } else {
    // nothing for the small lane: wait up to a millisecond for the large
    // lane to finish a step instead of returning at once (a caller that
    // loops over step and its own arrivals then neither spins nor delays a
    // new arrival by more than that)
    std::unique_lock<std::mutex> lk(s->mu);
    const int64_t seen = s->large_steps;
    if (!s->large_in.empty() || s->large_in_flight > 0)
      s->cv_done.wait_for(lk, std::chrono::milliseconds(1),
                          [&] { return s->large_steps != seen || s->large_err != VIECUT_OK; });
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!rc && s->large_err) rc = s->large_err;
  if (n_active) *n_active = s->small.in_flight() + s->large_in_flight + (int32_t)s->large_in.size();
  return rc;
}

int viecut_session_poll(viecut_session *s, int64_t *ids, viecut_result *outs, int32_t max) {
  if (!s || max < 0 || (max > 0 && (!ids || !outs))) return VIECUT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  for (auto *r : {&s->small.ready, &s->large_ready}) {
    const int32_t take = std::min<int32_t>(max - k, (int32_t)r->size());
    for (int32_t i = 0; i < take; i++) {
      ids[k + i] = (*r)[i].id;
      outs[k + i] = (*r)[i].res;
    }
    r->erase(r->begin(), r->begin() + take);
    k += take;
  }
  return k;
}

void viecut_session_destroy(viecut_session *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->small.s);
  if (s->large_stream) (void)hipStreamSynchronize(s->large_stream);
  s->small.report("session small lane");
  if (s->two_lanes) s->large.report("session large lane");
  hipStream_t ls = s->large_stream;
  delete s;
  if (ls) (void)hipStreamDestroy(ls);
}

}  // extern "C"
