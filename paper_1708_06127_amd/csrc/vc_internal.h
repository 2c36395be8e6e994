// Internal declarations of the HIP min-cut library (device status block,
// workspace views, kernel launchers). Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/viecut.h"

namespace vc {

constexpr int kBlock = 256;   // threads per workgroup everywhere (4 wave64)
// Largest vertex count of a graph or a batch union: label gathers address the
// label array with 32-bit byte offsets (4 * x < 2^32).
constexpr int32_t kMaxVertices = VIECUT_MAX_VERTICES;
// Static device scratch of the allocation-free single solve (one per GPU).
constexpr size_t kScratchBytes = VIECUT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;
constexpr int kBins = 8;      // degree classes for per-vertex work
constexpr int kHugeChunk = 4096;  // arcs per work item of a huge row
// Largest grids of the per-row launches of the long classes and of the huge
// rows' chunk kernel; the level-0 statistics of their workgroups take that
// many entries of Work::part beyond the tile kernels' (kLongParts).
constexpr unsigned kRowsGridMax = 8192;
constexpr unsigned kHugeChunksGrid = 4096;
constexpr int64_t kLongParts = 3 * (int64_t)kRowsGridMax + kHugeChunksGrid;
constexpr int kPartSlots = 16384;  // LDS table slots of one huge-row label partition (128 KB)
constexpr int kPartDistinct = 4;   // pass 1 plans room for d / kPartDistinct distinct labels of a huge row
constexpr int kPartProbe = 64;     // pass 1: a longer probe run sends the row to pass 2
// Row-aligned arc tiles: tile t holds the rows v with rp[v] + v in
// [t*kTile, (t+1)*kTile). A row with d >= kTile arcs is always the last row of
// its tile and is left to the long-row kernels; the short rows of a tile then
// hold at most kTile rows and fewer than 2*kTile arcs.
constexpr int kTB = 64;       // threads of a tile workgroup (one wave: barriers are cheap)
constexpr int kTile = 256;
constexpr int kRsTile = 1024;  // elements per workgroup of a radix sort pass
constexpr int kTileArcs = 2 * kTile;
constexpr int kPerThread = kTileArcs / kTB;  // up to 8 consecutive arcs per thread

// Degree classes (by arc count d of the row). Only the long classes are
// listed per level: 4: kTile <= d < 512 and 5: 512 <= d < 1024 (a wave per
// row, LDS tables of 1024 / 2048 slots: the smaller table keeps more waves
// resident), 6: 1024 <= d <= 4096 (a workgroup per row, LDS table), 7: d >
// 4096 (rows split into kHugeChunk-arc chunks sharing a global table).
// Shorter rows are handled by the arc tiles.
constexpr int kBinHuge = 7;
__host__ __device__ inline int degree_bin(int32_t d) {
  return d <= 8 ? 0 : d <= 16 ? 1 : d <= 32 ? 2 : d <= 64 ? 3 : d < 512 ? 4 : d < 1024 ? 5 : d <= 4096 ? 6 : 7;
}

enum : int32_t {
  ERR_ROWPTR = 1, ERR_COL = 2, ERR_SELF = 4, ERR_WEIGHT = 8, ERR_NOTSYM = 16, ERR_UNSORTED = 32,
  ERR_DEVICE = 64  // a bounded wait between workgroups expired (results of the call are void)
};
enum : int32_t { ST_COLLAPSED = 1, ST_DISCONNECTED = 2, ST_NO_PROGRESS = 4, ST_MAX_ROUNDS = 8 };

// Device-resident status of one solve. Read back to the host once per round.
struct Status {
  unsigned long long minkey;   // min over the level of (deg << 32 | v)
  unsigned long long wsum;     // sum of the input's arc weights
  long long lam_hat;           // current upper bound
  long long pad0;
  int32_t err;                 // ERR_* bits
  int32_t k;                   // vertices of the graph being built (relabel total)
  int32_t ax;                  // emitted inter-cluster arcs
  int32_t nnz;                 // arcs of the graph being built
  int32_t nmarked;             // PR-marked edges
  int32_t wit_v, wit_level;    // witness vertex / level of lam_hat
  int32_t updated;             // lam_hat lowered at the last bound update
  int32_t stop;                // ST_COLLAPSED / ST_DISCONNECTED
  int32_t dmax;                // largest row length of the current level
  int32_t huge_items;          // work items (chunks) of the huge bin
  int32_t huge_slots;          // table slots of the huge bin
  int32_t bin_cnt[8];          // vertices per degree class
  int32_t ring_cnt;            // (batched) finished graphs pushed to the ring so far
  int32_t active_cnt;          // (batched) graphs still in the round loop
  int32_t big_tiles;           // tiles of more than 256 arcs (listed in Work::big_tiles)
  int32_t pad1;
  unsigned long long tile_tot;  // (rows << 32) | arcs covered by the arc tiles of the current level
  int32_t pr_rows[2];          // rows marked with an LDS table of their row (short / long tables)
  unsigned long long fix_delta;  // correcting step: minimum weighted degree of the contracted graph
  long long sw_cut;            // device exact solve: the kernel graph's minimum cut
  int32_t lp_changed;          // labels changed by the last counted LP iteration
  int32_t huge_ticket;         // next work item of the huge-row label partitions
  int32_t huge_overflow;       // a huge-row label partition of pass 1 overflowed (its row runs again)
  int32_t huge_fallback;       // a pass-2 partition filled its table (the global-table path runs)
  int32_t kloc;                // (batched) largest vertex count of one graph at the level being built
  int32_t pad2;
};

// Kernel graphs of at most this many vertices are solved on the device (dense
// Stoer-Wagner in LDS, one wave per graph) instead of on the host.
constexpr int kDenseMax = 128;

// ------------------------------------------------------------ batched solves
// Many graphs are solved as one disjoint union: their CSRs are concatenated
// (graph g owns the vertex range [base, base + k) and the arc range
// [aoff, aoff + nnz) of the current level), every phase is one launch over
// the union, and a per-vertex graph index `gv` gives the kernels each row's
// graph. What makes the result of a graph independent of its neighbours in
// the union: label priorities use graph-local ids and a per-graph salt,
// relabelling by prefix sum keeps every graph's clusters contiguous and in
// the same order, and bounds, witnesses, marks and stop rules are kept per
// graph (GStat).
enum : int32_t { GS_FREE = 0, GS_FRESH = 1, GS_ACTIVE = 2, GS_DONE = 3 };
enum : int32_t { FIN_NONE = 0, FIN_SOLVE = 1, FIN_STOP = 2, FIN_ERROR = 3 };

struct GStat {
  unsigned long long minkey;   // min over the graph's vertices of (deg << 32 | local v)
  unsigned long long wsum;     // arc weight sum of the input
  long long lam_hat;           // current upper bound
  int32_t err;                 // ERR_* bits of the input
  int32_t wit_v, wit_level;    // witness vertex (local id) and its level
  int32_t updated;             // lam_hat lowered at the last bound update
  int32_t status;              // ST_* bits
  int32_t nmarked;             // some edge of the graph was PR-marked in this round
  int32_t base, k;             // first vertex and vertex count at the current level
  int32_t aoff, nnz;           // first arc and arc count at the current level
  int32_t level, rounds;       // contractions performed, rounds started
  int32_t n_start;             // vertices at the start of the current round
  int32_t state;               // GS_*
  int32_t fin;                 // FIN_*: how the graph left the loop
  int32_t buf;                 // CSR buffer holding its current level
  int32_t contracted;          // contracted by the current contraction step
  int32_t slot;                // own index
  uint32_t salt;               // tie-break salt of the current LP iteration
  int32_t pad;
};
static_assert(sizeof(GStat) == 104, "GStat layout");

// Static descriptor of an admitted graph (device copy).
struct GDesc {
  const int32_t *rp, *col, *w; // the caller's CSR (device)
  int32_t n, nnz;
  int32_t voff, aoff;          // its vertex / arc offset in the union at admission
  int32_t woff, words;         // its range of 64-vertex words in the input index space
  int32_t slot;
  int32_t rchunk0, achunk0;    // first row chunk / arc chunk of the packing work
  int32_t pad;
};

// Copy of a finished graph's last level out of the union (for the exact solve).
struct GatherDesc {
  const int32_t *rp, *col, *w;   // union buffer holding that level
  int32_t base, k, aoff, nnz;    // its vertex and arc ranges there
  int32_t drp, darc;             // destination offsets in the staging arrays
  int32_t rchunk0, achunk0;      // first row chunk / arc chunk of the copy work
};

// A finished graph's last level for the device exact solve (read in place).
struct SwDesc {
  const int32_t *rp, *col, *w;   // union buffer holding that level
  int32_t base, k;               // its vertex range there
  int32_t foff;                  // its side flags at flags + foff
  int32_t pad;
};

// Side bitmap of a finished graph.
struct SideDesc {
  unsigned long long *side;      // caller's array, ceil(n/64) words
  int32_t woff, n;               // its words in the input index space, vertex count
  int32_t mode;                  // 0: witness bitmap, 1: kernel-graph flags through the map, 2: release only
  int32_t foff, fbase;           // flags of kernel vertex (map - fbase) at foff + (map - fbase)
  int32_t wchunk0;               // first output word of this graph in the launch
};

// Device views used by the kernels in batched mode (all nullptr for a single solve).
struct BatchView {
  const int32_t *gv = nullptr;   // graph index per vertex of the current level
  GStat *gs = nullptr;           // per-graph state, indexed by slot
  int32_t slots = 0;
};

// One graph level in device memory. Rows may be unsorted only for the input.
struct DGraph {
  int32_t n = 0;
  int64_t nnz = 0;
  const int32_t *row_ptr = nullptr;
  const int32_t *col = nullptr;
  const int32_t *w = nullptr;
};

// Per-solve device buffers (carved from one workspace).
struct Work {
  int32_t n_in = 0;
  int64_t nnz_in = 0;
  Status *st = nullptr;
  // two ping-pong CSR buffers for coarse levels
  int32_t *rp[2] = {nullptr, nullptr};
  int32_t *col[2] = {nullptr, nullptr};
  int32_t *w[2] = {nullptr, nullptr};
  long long *deg = nullptr;      // degrees of the current level
  int32_t *La = nullptr, *Lb = nullptr;   // LP labels (ping-pong)
  int32_t *ids = nullptr;        // relabel flags / prefix sums, n+1
  int32_t *cl = nullptr;         // old vertex -> new vertex
  int32_t *map = nullptr;        // input vertex -> current vertex
  unsigned long long *witness = nullptr;  // ceil(n_in/64) words
  int32_t *bins = nullptr;       // kBins lists of capacity n
  int32_t *cnt = nullptr;        // per-vertex counts (n+1)
  unsigned long long *keys[2] = {nullptr, nullptr};  // sort keys (nnz each)
  int32_t *vals[2] = {nullptr, nullptr};             // sort values
  int32_t *hist = nullptr;       // radix histogram, 256 * tiles
  // single-pass scans: one state word per tile (epoch, flag, value) and the
  // tile ticket; lb_epoch == 0 means the words have not been cleared yet
  unsigned long long *lb_state = nullptr;
  uint32_t *lb_ticket = nullptr;
  int64_t lb_tiles = 0;          // state words available
  uint32_t lb_epoch = 0;         // host-side: epoch of the last scan launched
  uint8_t *mark = nullptr;       // PR mark per arc
  int32_t *parent = nullptr;     // union-find
  int32_t *huge_tab_key = nullptr;  // global hash tables of the huge bin
  uint32_t *huge_tab_val = nullptr;
  unsigned long long *huge_best = nullptr;  // per huge vertex best key
  int32_t *huge_meta = nullptr;  // per huge vertex: chunk offset, table offset, table size
  int64_t huge_cap = 0;          // table slots available
  uint8_t *flags8 = nullptr;     // side flags of the kernel graph (n)
  int4 *tile_meta = nullptr;     // per arc tile: first row, short rows, first arc, arcs
  int32_t *big_tiles = nullptr;  // ids of the tiles of more than 256 arcs (any order)
  int32_t ntiles = 0;            // tiles of the current level
  unsigned long long *part = nullptr;  // per-block partial results (3 per tile)
  int32_t *seg = nullptr;        // emission segments: first arc of each
  int32_t *seg_cnt = nullptr;    // their counts, then exclusive offsets
  // correcting step (per label of the current level): member counts, the
  // cluster's weighted degree in the contracted graph, the best removal key;
  // per vertex: weight of its edges to other clusters
  int32_t *fix_cnt = nullptr;
  uint32_t *fix_out = nullptr;
  unsigned long long *fix_cut = nullptr;
  unsigned long long *fix_key = nullptr;
};

size_t work_bytes(int32_t n, int64_t nnz, int64_t map_n = -1, int64_t extra = 0);
bool carve(void *ws, size_t bytes, int32_t n, int64_t nnz, Work &w, int64_t map_n = -1, int64_t extra = 0);

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return hipSuccess or the launch error.
hipError_t fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s);
hipError_t status_reset(Status *st, hipStream_t s);
// exclusive scan of int32 counts (in-place capable); *total (optional) gets the sum
hipError_t scan_exclusive(Work &w, const int32_t *in, int32_t *out, int64_t count, int32_t *total, hipStream_t s);

hipError_t check_rowptr(const DGraph &g, Status *st, hipStream_t s);
hipError_t reset_bins(Work &w, hipStream_t s);
// per level: arc tiles (w.ntiles set from g.nnz, which must be host-known) and long-row lists
hipError_t build_tiles(const DGraph &g, Work &w, hipStream_t s);
// `known`: host copy of the bin counts, or nullptr when they are only on the device
// iteration 1 of LP (labels are the identity): row argmax, at level 0 fused
// with validation, the weighted degree and the minimum-degree key
hipError_t lp_first(const DGraph &g, Work &w, const int32_t *known, int32_t *L, uint32_t salt, bool level0,
                    hipStream_t s, const BatchView *bv = nullptr);
// iteration t >= 2: neighbour-label weight sums in hash tables; part 0: the
// whole iteration, 1: only the arc tiles (rows of fewer than 256 arcs), 2:
// only the long and huge rows
hipError_t lp_iter(const DGraph &g, Work &w, const int32_t *known, const int32_t *Lin, int32_t *Lout, uint32_t salt,
                   hipStream_t s, const BatchView *bv = nullptr, int part = 0);
hipError_t validate_sym(const DGraph &g, Status *st, hipStream_t s, const BatchView *bv = nullptr);
// relabel: ids = prefix sum of used label values, cl[v] = ids[L[v]], k -> st->k;
// a single solve also composes map[u] <- cl[map[u]] in the same pass
// (batched: only graphs in the round loop keep their vertices; gv_new receives
// the graph index of every new vertex; the map is composed separately)
// lspace: size of the label value range (n, or 2n after the correcting step)
hipError_t relabel(const int32_t *L, int32_t n, Work &w, hipStream_t s, const BatchView *bv = nullptr,
                   int32_t *gv_new = nullptr, int64_t lspace = -1);
// correcting step on the labels L of the graph g (single solve): a misplaced
// vertex v gets label n + v (labels then range over [0, 2n))
hipError_t fix_misplaced(const DGraph &g, Work &w, int32_t *L, hipStream_t s);
// first-iteration restriction: vertices chosen by another vertex keep their
// own label (L holds iteration 1's labels; uses flags8 as scratch)
hipError_t restrict_first(const DGraph &g, Work &w, int32_t *L, hipStream_t s);
// st->lp_changed = #{v : cur[v] != prev[v]} (prev == nullptr: the identity)
hipError_t count_changed(const int32_t *prev, const int32_t *cur, int32_t n, Work &w, hipStream_t s);
hipError_t init_map(Work &w, hipStream_t s);
// contraction: inter-cluster triples packed into buffer 1 (count -> st->ax, key bits from st->k)
hipError_t contract_emit(const DGraph &g, Work &w, const int32_t *known, hipStream_t s,
                         const BatchView *bv = nullptr);
// sorts the `count` triples held in buffer `which` (in/out: the buffer holding the result)
hipError_t radix_sort(Work &w, int64_t count, int total_bits, int &which, hipStream_t s);
// sorted triples -> CSR buffer `dst` with k rows, degrees, bound update at `level`, witness
// key_bits: width of the keys' low part; gv_new / gs (batched): the low part
// is the neighbour relative to the first vertex of its graph at the new level
hipError_t contract_build(Work &w, int which, int64_t count, int key_bits, int32_t k, int dst, int32_t level,
                          hipStream_t s, bool single_bound = true, const int32_t *gv_new = nullptr,
                          const GStat *gs = nullptr);
hipError_t bound_level0(Work &w, hipStream_t s);
// The contracted graph of a partition into one cluster: one vertex, no arcs
// (row pointers and degree zero, nnz = 0, the stop flag ST_COLLAPSED), in one
// launch instead of the segment passes and the bound update.
hipError_t contract_collapse(Work &w, int dst, hipStream_t s);
// PR marks on the v < x arcs (st->nmarked != 0 iff some edge was marked)
hipError_t pr_mark(const DGraph &g, Work &w, const int32_t *known, hipStream_t s, const BatchView *bv = nullptr);
hipError_t union_find(const DGraph &g, Work &w, const int32_t *known, int32_t *rep, hipStream_t s);
hipError_t side_from_flags(Work &w, const uint8_t *flags, uint64_t *side, hipStream_t s);
hipError_t side_from_witness(Work &w, uint64_t *side, hipStream_t s);
// exact solve of the graph g (g.n <= kDenseMax) on the device: the cut into
// st->sw_cut, the kernel side flags into w.flags8; then the input side: the
// kernel side through the map if it beats lambda-hat, else the witness
hipError_t exact_dense(const DGraph &g, Work &w, uint64_t *side, hipStream_t s);
// batched: one wave per listed graph (every k <= kmax <= kDenseMax); cuts[i]
// and the flags of graph i at flags + d[i].foff
hipError_t exact_dense_batch(const SwDesc *d, int32_t count, int32_t kmax, uint8_t *flags, long long *cuts,
                             hipStream_t s);

// ---- batched-solve launchers (see the kernels for what each does)
hipError_t b_gs_init(GStat *gs, const GDesc *d, int32_t count, int32_t buf, hipStream_t s);
hipError_t b_pack(const GDesc *d, int32_t count, int32_t rchunks, int32_t achunks, int32_t *gv, int32_t *map,
                  int32_t *wg, int32_t *rpu, int32_t *colu, int32_t *wu, GStat *gs, hipStream_t s);
hipError_t b_salts(GStat *gs, int32_t slots, uint64_t seed, int32_t lp_iters, int32_t t, bool pre, hipStream_t s);
hipError_t b_gdeg(const long long *deg, int32_t v0, int32_t v1, const int32_t *gv, GStat *gs, bool with_sum,
                  hipStream_t s);
hipError_t b_gbound0(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap, hipStream_t s);
hipError_t b_step_top(GStat *gs, int32_t slots, int32_t n0, int32_t max_rounds, Status *st, GStat *ring,
                      int32_t ring_cap, hipStream_t s);
hipError_t b_step_end(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap, hipStream_t s);
hipError_t b_gsizes(GStat *gs, int32_t slots, const int32_t *ids, int mode, Status *st, hipStream_t s);
hipError_t b_gbound(GStat *gs, int32_t slots, const int32_t *rp, int32_t buf, Status *st, GStat *ring,
                    int32_t ring_cap, hipStream_t s);
hipError_t b_gwitness(const int32_t *map, const int32_t *wg, const GStat *gs, int32_t words,
                      unsigned long long *wit, hipStream_t s);
hipError_t b_compose(int32_t *map, const int32_t *cl, int64_t entries, const int32_t *wg, const GStat *gs,
                     hipStream_t s);
hipError_t b_gather(const GatherDesc *d, int32_t count, int32_t rchunks, int32_t achunks, int32_t *orp,
                    int32_t *ocol, int32_t *ow, hipStream_t s);
hipError_t b_side(const SideDesc *d, int32_t count, int32_t words, const int32_t *map,
                  const unsigned long long *wit, const uint8_t *flags, int32_t *wg, hipStream_t s);
constexpr int kPackRows = 2048;  // rows (input index entries) per chunk of the packing and gather work
constexpr int kPackArcs = 8192;  // arcs per chunk of the packing and gather work

// ---- optional kernel timing (viecut_profile_*): an event pair around a
// launch plus a copy of the level's tile totals for its algorithmic bytes
enum ProfKind : int { PROF_FIRST_TILE = 0, PROF_FIRST_TILE_L0 = 1, PROF_LP_TILE = 2, PROF_SWEEP = 3, PROF_KINDS = 4 };
struct ProfScope {
  int slot = -1;
  hipStream_t s;
  const Status *st;
  // device address of the record's 16-byte snapshot of (tile rows, big
  // tiles, tile arcs) in page-locked host memory, or nullptr: the first launch of
  // the scope writes it from one thread (no copy is queued)
  int32_t *dev = nullptr;
  ProfScope(ProfKind kind, hipStream_t stream, const Status *st, int32_t ntiles);
  ~ProfScope();
};
void prof_collect();  // after a synchronisation: fold finished records into the totals
// An event-timed span on a stream whose algorithmic bytes the host knows only
// later (label propagation + contraction of the first contraction round): begin returns a
// record id (-1 when timing is off), end records the closing event, and
// prof_span_bytes sets the record's bytes once they are known.
int prof_span_begin(ProfKind kind, hipStream_t s);
void prof_span_end(int id, hipStream_t s);
void prof_span_bytes(int id, double bytes);

// host driver entry points shared by the single, batched and session paths
int check_args(const viecut_csr *g, const viecut_params *p);
int solve_one(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
              viecut_result *out, uint64_t *side, viecut_trace_fn fn, void *user);

// device address of the static scratch on `device` (which must be current);
// looked up on the first call per device and kept
hipError_t scratch_address(int device, void **ptr);

// Launch-shape choices that change no result, per size bucket (arcs of the
// level): read at load time from the tuning file, else these defaults.
struct Tuning {
  int64_t radix_large_from = 1 << 22;    // sort elements from which radix blocks hold 4096 elements
  int64_t compact_direct_max = 1 << 20;  // segments up to which each output element searches all offsets
  int64_t pr_merge_tiles = 16384;        // batch unions: tiles from which short rows merge from global memory
  int64_t long_split = 512;              // long rows below this many arcs take the 1024-slot LDS class
  int64_t emit_wave = 1;                 // rows of 256..1023 arcs emitted by a wave per row (0: a workgroup)
  int64_t lp_group = 2;                  // tiles of at most 256 arcs per LP workgroup (1..4)
  int64_t emit_group = 2;                // tiles of at most 256 arcs per emission workgroup (1..2)
  int64_t huge_part = 1;                 // LP t >= 2 on rows of more than 4096 arcs: 1 = label partitions in LDS,
                                         // 0 = one global hash table per row
  int64_t first_group = 1;               // LP iteration 1: 1 = a workgroup per tile, 2 = two short-row tiles per
                                         // workgroup plus a persistent kernel for the others
};
Tuning tuning_for(int64_t arcs);

// host helpers
uint64_t splitmix64_at(uint64_t seed, uint64_t index);
int64_t stoer_wagner_host(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *w,
                          uint8_t *side);

}  // namespace vc
