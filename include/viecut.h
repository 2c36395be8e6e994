/*
 * viecut.h - C ABI of the MI355X (gfx950) inexact minimum-cut library.
 *
 * The library computes a cut of an undirected graph with positive integer
 * edge weights, G = (V, E, c), following the method of Henzinger, Noe,
 * Schulz and Strash, "Practical Minimum Cut Algorithms" (arXiv 1708.06127):
 * rounds of label-propagation clustering and cluster contraction
 * (Section 4.1), Padberg-Rinaldi contraction tests applied through a
 * union-find (Lemma "Padberg-Rinaldi", Section 4.1), a running upper bound
 * equal to the minimum weighted degree (Section 4, introduction), an exact
 * solve on the small remaining graph and a transfer of its cut back to the
 * input (Algorithm 1, appendix A).
 *
 * What is returned follows the problem statement (Section 3, Preliminaries): a cut
 * (A, V \ A) with both sides non-empty and its capacity c(A) = the summed
 * weight of the edges between A and V \ A. The value is never below the
 * minimum cut lambda(G) (contraction only removes cuts) and never above the
 * minimum weighted degree delta(G); it is not guaranteed to equal lambda(G)
 * (the method is a heuristic).
 *
 * Determinism: label propagation is synchronous (every vertex reads the
 * previous iteration's labels) with a seeded, hash-based tie-break, so the
 * result (value and side) is a pure function of (graph, params). It does not
 * depend on thread timing, launch configuration or batch composition.
 *
 * Arithmetic: int32 weights, sums in int64 (or in uint32 where the sum is
 * bounded by the total weight, which is checked to be <= INT32_MAX).
 *
 * All graph pointers are DEVICE pointers unless stated otherwise. A stream
 * argument is a hipStream_t passed as void* (NULL = the default stream).
 * Passes whose long rows carry much of the work also queue those rows'
 * kernels on a second stream that the calling host thread borrows per device
 * from a pool the library keeps for the life of the process (default
 * priority; a thread gives its streams back when it exits); it is
 * ordered after the work already on the caller's stream, and the caller's
 * stream waits for it (events) before the next pass: whatever is queued on
 * the caller's stream after a call, or waits for that stream, also comes
 * after the call's work on the second stream.
 * No function throws; every function that can fail returns a status code
 * (VIECUT_OK = 0 or a negative VIECUT_E* value). On error no output is
 * written and the library stays usable.
 */
#ifndef VIECUT_H
#define VIECUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
  VIECUT_OK = 0,
  VIECUT_EINVAL = -1,    /* bad argument: n < 2, bad row_ptr, column out of range or a self loop, bad params */
  VIECUT_EWEIGHT = -2,   /* an edge weight < 1 */
  VIECUT_EOVERFLOW = -3, /* total weight (sum over edges) > INT32_MAX, nnz >= 2^31, or more than
                            VIECUT_MAX_VERTICES vertices (per graph, and summed over a batch) */
  VIECUT_ENOMEM = -4,    /* workspace too small, or device allocation failed */
  VIECUT_EDEVICE = -5,   /* a HIP runtime call failed */
  VIECUT_ENOTSYM = -6,   /* (with VIECUT_F_VALIDATE) not symmetric, or a row not strictly increasing */
  VIECUT_EBUDGET = -7,   /* (sessions) a request larger than the whole memory budget */
  VIECUT_ETOOBIG = -8    /* (viecut_mincut_noalloc) the graph's workspace exceeds the static scratch */
};

/* status_bits of a result */
enum {
  VIECUT_ST_COLLAPSED = 1,    /* a contraction left one vertex: the result is the upper bound */
  VIECUT_ST_DISCONNECTED = 2, /* a vertex of degree 0 was found: the minimum cut is 0 */
  VIECUT_ST_NO_PROGRESS = 4,  /* a round did not shrink the graph; the exact solve ran on what remained */
  VIECUT_ST_MAX_ROUNDS = 8    /* max_rounds reached before the graph got to n0 vertices */
};

/* Largest vertex count the library accepts: one graph of at most 2^30 vertices, and at most
 * 2^30 vertices plus graphs summed over the graphs of one batch (label gathers address the
 * label array with 32-bit byte offsets). Larger inputs return VIECUT_EOVERFLOW before any
 * device work. */
#define VIECUT_MAX_VERTICES (1 << 30)

/* params.flags */
enum {
  VIECUT_F_VALIDATE = 1, /* check symmetry (w(u,v) == w(v,u)) and strictly increasing rows (O(nnz log d)) */
  VIECUT_F_CORRECT = 2,  /* the correcting step after label propagation (Section 4.1's correcting algorithm,
                            fixMisplacedVertices in Algorithm 1): in every cluster of 2 to floor(log2 n)
                            vertices, the vertex whose removal leaves the cluster the smallest weighted
                            degree in the contracted graph becomes a singleton if that degree is below the
                            contracted graph's minimum weighted degree. Single-graph calls only: batches and
                            sessions return VIECUT_EINVAL. */
  VIECUT_F_CONVERGE = 4, /* label-propagation convergence stop (appendix D, "Algorithm Configuration"): the
                            iterations of a round end after the first one in which at most floor(n / 10000)
                            vertices (n: vertices of the current graph) changed their label, else after
                            lp_iters. Costs one status read per iteration. Single-graph calls only. */
  VIECUT_F_RESTRICT = 8  /* first-iteration restriction (Section 4.1), read synchronously: after the first
                            label-propagation iteration of a round, every vertex chosen by another vertex
                            keeps its own label. Unlike the sequential rule it does not bound the cluster
                            count by n / 2. Single-graph calls only. */
};

/* Input graph: a symmetric CSR. Row v lists the neighbours of v.
 * Layout: row_ptr[n+1] (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz),
 * col[nnz] (0 <= col < n, no self loops, strictly increasing within a row),
 * w[nnz] (w >= 1, w(u,v) == w(v,u), total weight sum(w)/2 <= INT32_MAX).
 * nnz = 2|E| arcs. The arrays are owned by the caller, read-only, and must
 * stay valid until the call returns (or, for sessions, until the request is
 * reported done). */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t *row_ptr;
  const int32_t *col;
  const int32_t *w;
} viecut_csr;

/* Method parameters (label propagation bounded to l iterations and the loop down to n0
 * vertices: Section 4.1 and Algorithm 1 in appendix A; the defaults are the paper's
 * configuration in Section 5):
 *   lp_iters   - label-propagation iterations per round (the paper's l; 2). 0 disables clustering.
 *   n0         - bound for the exact solve: rounds run while more than n0 vertices remain (10000).
 *   max_rounds - safety cap on rounds (64).
 *   flags      - VIECUT_F_* bits.
 *   seed       - seed of the tie-break priorities (0). */
typedef struct {
  int32_t lp_iters;
  int32_t n0;
  int32_t max_rounds;
  uint32_t flags;
  uint64_t seed;
} viecut_params;

/* Result of one solve.
 *   cut           - capacity of the returned cut
 *   rounds        - rounds started
 *   kernel_n      - vertices of the graph the loop stopped at
 *   witness_level - contraction level whose minimum-degree vertex gave the cut, or -1 when the
 *                   exact solve on the remaining graph gave it
 *   status_bits   - VIECUT_ST_* bits
 *   levels        - contractions performed
 *   t_ms          - host-measured phase times: [0] validate+first LP iteration, [1] enqueueing the
 *                   remaining LP iterations (their kernels finish within [2]), [2] cluster
 *                   contraction, [3] PR marking+union-find+contraction, [4] exact solve + transfer,
 *                   [5] total; [6],[7] unused. */
typedef struct {
  int64_t cut;
  int32_t rounds;
  int32_t kernel_n;
  int32_t witness_level;
  uint32_t status_bits;
  int32_t levels;
  int32_t reserved;
  float t_ms[8];
} viecut_result;

/* Fills *p with the defaults above (lp_iters 2, n0 10000, max_rounds 64, flags 0, seed 0). */
void viecut_default_params(viecut_params *p);

/* Device workspace (bytes) that viecut_mincut needs for a graph of n vertices
 * and nnz arcs: two coarse CSR levels, labels, the contraction's sort buffers
 * and the Padberg-Rinaldi marks (about 73 bytes per arc plus 80 per vertex).
 * Returns 0 for invalid sizes (n < 2, nnz < 0, n > VIECUT_MAX_VERTICES). */
size_t viecut_workspace_bytes(int32_t n, int32_t nnz, const viecut_params *p);

/* Solves one graph with the whole method (Algorithm 1 in appendix A: label
 * propagation and cluster contraction of Section 4.1, the Padberg-Rinaldi
 * contraction of Section 4.1, the minimum-degree bound of Section 4, the
 * exact solve of the remaining graph and the transfer of its cut).
 * g: device CSR as above. p: parameters (host). ws: device workspace of at least viecut_workspace_bytes()
 * bytes (NULL: the library allocates and frees it inside the call). side:
 * device array of ceil(n/64) uint64 words; on success bit (u & 63) of word
 * (u >> 6) is 1 iff vertex u is on the side NOT containing vertex 0 (padding
 * bits 0). out: host struct. The call returns when the result is final
 * (the exact solve runs on the host). One call at a time per workspace.
 * The calling thread keeps a small page-locked host buffer (the status
 * reads, and kernel-graph hand-offs up to 16 MiB) for the rest of the
 * process; larger hand-offs use pageable copies. */
int viecut_mincut(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
                  viecut_result *out, uint64_t *side);

/* Trace record for viecut_mincut_trace. Array pointers are HOST copies valid
 * only during the callback.
 *   kind 1 (LP):       a = labels[n] after iteration `iter` of round `round`
 *   kind 2 (CONTRACT): a = row_ptr[n+1], b = col[nnz], c = w[nnz], d = deg[n] of the new graph at
 *                      `level`, e = cl[n_prev] (old vertex -> new vertex). Rows are sorted.
 *   kind 3 (BOUND):    lam_hat, witness_vertex, witness_level after the update at `level`
 *   kind 4 (PR):       a = mark[nnz] on the graph at `level`: 1 on the arc (v, x), v < x, of
 *                      every marked edge, 0 elsewhere
 *   kind 5 (UF):       a = rep[n], the smallest vertex id of each marked-edge component
 *   kind 6 (FIX):      a = labels[n] after the correcting step of round `round` (a vertex v made a
 *                      singleton has label n + v) */
typedef struct {
  int32_t kind, round, iter, level;
  int32_t n, n_prev;
  int64_t nnz;
  int64_t lam_hat;
  int32_t witness_vertex, witness_level;
  const int32_t *a, *b, *c;
  const int64_t *d;
  const int32_t *e;
} viecut_event;
typedef void (*viecut_trace_fn)(void *user, const viecut_event *ev);

/* Size of the static device scratch array that serves as the workspace of
 * viecut_mincut_noalloc: 64 MiB, held by every GPU the library runs on for the
 * life of the process. A graph fits if viecut_workspace_bytes(n, nnz) is at
 * most this (about 73 bytes per arc plus 80 per vertex: e.g. 8192 vertices of
 * average degree 64). */
#define VIECUT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* viecut_mincut for callers that cannot allocate (tight serving loops,
 * harnesses that forbid allocation): the same solve with the same results,
 * without a workspace argument and without allocating anything on the
 * device or in page-locked host memory (no hipMalloc, hipHostMalloc or
 * their frees; nothing through torch). Its workspace is a static device array
 * of VIECUT_NOALLOC_SCRATCH_BYTES per GPU; status reads and the exact solve's
 * hand-off use ordinary (pageable) host memory. g, p, out and side are as for
 * viecut_mincut; stream must belong to the current device (NULL: its default
 * stream). Returns VIECUT_ETOOBIG, before any device work, if
 * viecut_workspace_bytes(g->n, g->nnz) exceeds the scratch.
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (the solve clears what must start at zero). Calls that overlapped
 * on one GPU would race on it, so the library serialises the calls of a
 * process per device with a lock: a second call waits until the first has
 * returned. Other processes have arrays of their own. */
int viecut_mincut_noalloc(const viecut_csr *g, const viecut_params *p, void *stream, viecut_result *out,
                          uint64_t *side);

/* viecut_mincut (same method and arguments) with a host callback receiving every intermediate state
 * (for parity checking and debugging; it synchronises and copies at every
 * step, so it is slow). */
int viecut_mincut_trace(const viecut_csr *g, const viecut_params *p, void *ws, size_t ws_bytes, void *stream,
                        viecut_result *out, uint64_t *side, viecut_trace_fn fn, void *user);

/* Checks g on the device against the input contract of the problem statement
 * (Section 3: an undirected graph with positive integer edge weights, stored as
 * a symmetric CSR): row_ptr, column range, self loops, weights, total weight;
 * with VIECUT_F_VALIDATE in flags also symmetry and sorted rows. Does not
 * solve. Allocates a temporary workspace of viecut_workspace_bytes() and frees
 * it before returning. Returns VIECUT_OK or the error code viecut_mincut would. */
int viecut_validate(const viecut_csr *g, uint32_t flags, void *stream);

/* ------------------------------------------------------------ batching */
/* Device workspace (bytes) for solving the `count` graphs of gs together with
 * viecut_mincut_batch (the union of their CSRs and per-graph state; the method
 * is Algorithm 1 per graph). Graphs that fail the host argument checks are not
 * counted. Returns 0 if the union exceeds VIECUT_MAX_VERTICES vertices or
 * 2^31 - 1 arcs. */
size_t viecut_batch_workspace_bytes(const viecut_csr *gs, int32_t count, const viecut_params *p);

/* Solves `count` independent graphs in one batched execution, each with the
 * method of viecut_mincut (Algorithm 1; the paper motivates many small cut
 * problems with the separation step of branch-and-cut solvers, Section 1) (all graphs
 * advance round by round together; each graph's arithmetic and result are
 * identical to viecut_mincut on it alone). gs: host array of descriptors
 * (device pointers inside). outs: host array of count results. sides: host
 * array of count device pointers (ceil(n_i/64) words each). Returns
 * VIECUT_OK, or the first error; per-graph input errors are reported in
 * outs[i].status_bits as 0x80000000 | (-code) and do not stop the others. */
int viecut_mincut_batch(const viecut_csr *gs, int32_t count, const viecut_params *p, void *ws, size_t ws_bytes,
                        void *stream, viecut_result *outs, uint64_t *const *sides);

/* ------------------------------------------------------------ serving */
/* Serving of the same method (Algorithm 1 per request; applications in
 * Section 1). A session keeps admitted graphs resident and advances them by
 * batched rounds (continuous batching): requests submitted while others are
 * in flight join at the next round once their workspace fits in the budget;
 * finished requests release their workspace. Requests of up to 2^20 arcs go
 * to a small-request lane (a quarter of the budget) that the caller's thread
 * advances one round per viecut_session_step; larger ones go to a second lane
 * that a worker thread of the session advances on a stream of its own, so a
 * round of large graphs does not hold back small requests. One thread drives
 * a session (its calls are not to be made concurrently). */
typedef struct viecut_session viecut_session;

/* Creates a session (Algorithm 1 per request). hbm_budget: bytes of device
 * memory the session allocates once here for the workspaces of its two lanes
 * (vertices and arcs in a 1 : 4 ratio, up to 4096 requests in flight per
 * lane). p: parameters of every request (host, copied). stream: the stream
 * of the small-request lane; the large lane creates one of its own (default
 * priority). A budget whose quarter cannot hold a 2^20-arc request keeps one
 * lane for every request. *out receives the handle. Returns VIECUT_EBUDGET if
 * the budget holds no graph at all, VIECUT_ENOMEM if an allocation fails. */
int viecut_session_create(size_t hbm_budget, const viecut_params *p, void *stream, viecut_session **out);
/* Queues a request (a graph as in viecut_mincut; Section 3's input). g's
 * arrays and side (ceil(n/64) device words) are owned by the caller and must
 * stay valid until the request is polled. request_id is returned by poll.
 * Host argument errors return the viecut_mincut code; device-detected input
 * errors are reported per request by poll. Returns VIECUT_EBUDGET if it can
 * never fit in the session's workspace. */
int viecut_session_submit(viecut_session *s, const viecut_csr *g, uint64_t *side, int64_t request_id);
/* Admits queued small requests that fit, runs one round of the method (label
 * propagation, cluster contraction, Padberg-Rinaldi contraction, bounds:
 * Section 4.1) for every active small request, exact-solves and finishes
 * those that left the loop (Algorithm 1's last steps); the large lane runs its
 * rounds meanwhile on its own. With no small request in flight it waits up to
 * a millisecond for the large lane to finish a round. Returns an error of
 * either lane. *n_active receives the number of requests still in flight or
 * queued in both lanes. */
int viecut_session_step(viecut_session *s, int32_t *n_active);
/* Retrieves up to max finished requests into the host arrays ids and outs
 * (results as viecut_mincut's; an input error shows as status_bits
 * 0x80000000 | -code). Returns how many, or VIECUT_EINVAL. */
int viecut_session_poll(viecut_session *s, int64_t *ids, viecut_result *outs, int32_t max);
/* Waits for the session's stream and frees its workspace; requests not yet
 * polled are dropped. */
void viecut_session_destroy(viecut_session *s);

/* ------------------------------------------------------------ kernel timing */
/* Optional measurement aid, off by default and process-wide. While enabled,
 * every launch of the arc-tile label-propagation kernels (first iteration,
 * first iteration at level 0, iterations >= 2) is timed with a pair of HIP
 * events on the stream it runs on, and its algorithmic bytes are counted from
 * the exact row and arc totals of the tiles it sweeps:
 *   k_first_tile        8 B per arc (col, w) + 8 B per row (row_ptr, label) + 16 B per tile
 *   k_first_tile_level0 8 B per arc + 16 B per row (also the weighted degree) + 16 B per tile
 *   k_lp_tile           12 B per arc (col, w, neighbour label) + 12 B per row (row_ptr, own
 *                       label, new label) + 16 B per tile
 * Timing adds two event records per timed launch; the launch's kernel writes
 * the tile totals (16 bytes) into page-locked host memory itself. */
typedef struct {
  char name[32];     /* kernel name */
  int64_t launches;  /* timed launches since viecut_profile_enable(1) */
  double total_ms;   /* summed event-to-event durations */
  double bytes;      /* summed algorithmic bytes */
} viecut_kernel_stat;

/* on != 0: start timing and clear the totals; on == 0: stop. Returns VIECUT_OK or VIECUT_ENOMEM. */
int viecut_profile_enable(int on);
/* Copies up to max totals into out (host array); returns how many, or VIECUT_EINVAL. Totals cover
 * the solves that have returned (batched: the rounds completed). */
int viecut_profile_read(viecut_kernel_stat *out, int32_t max);

/* ------------------------------------------------------------ launch-shape tuning */
/* Measurement aid for the project's tuner (paper_1708_06127_amd/autotune.py),
 * process-wide. Some launch shapes change no result, only speed: the sort
 * elements from which radix blocks hold 4096 elements (radix_large_from), the
 * segment count up to which the compaction searches all segment offsets per
 * element (compact_direct_max), the union tile count from which batched PR
 * marking of short rows merges rows from global memory (pr_merge_tiles), the
 * row length splitting the 1024- and 2048-slot long-row LP classes
 * (long_split, 256..768), the long-row emission variant (emit_wave, 0/1),
 * and the tiles of at most 256 arcs that one label-propagation workgroup
 * takes (lp_group, 1..4) and one emission workgroup takes (emit_group, 1..2),
 * and the launch shape of label-propagation iteration 1 (first_group: 1 = a
 * workgroup per tile, 2 = two short-row tiles per workgroup plus a
 * persistent kernel for the tiles of more than 256 arcs), and the table of
 * label propagation on rows of more than 4096 arcs (huge_part: 1 = label
 * partitions in LDS, 0 = a global hash table per row).
 * The library keeps one set per size bucket (arcs of the level being worked
 * on, at most max_arcs; max_arcs < 0: no bound) and reads the table at load
 * time from the file named by the environment variable VIECUT_TUNING, else
 * viecut_tuning.txt beside the library; lines read
 *   bucket <max_arcs> key=value ...
 * viecut_tuning_set sets one key of one bucket (creating it with defaults);
 * returns VIECUT_EINVAL for an unknown key or a value out of range. */
int viecut_tuning_set(int64_t max_arcs, const char *key, int64_t value);
/* Drops every bucket (back to the defaults; the file is not read again). */
int viecut_tuning_clear(void);
/* Writes the table in the file format into buf (len bytes, NUL-terminated);
 * with buf == NULL returns the length needed. Returns the bytes written. */
int viecut_tuning_get(char *buf, size_t len);

/* Static message for a status code. */
const char *viecut_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* VIECUT_H */
