// HIP kernels for gfx950 (wave64) of the inexact minimum-cut method:
//  * synchronous label propagation (Section 4.1 of the paper): every vertex
//    picks the neighbouring label of largest connection weight, reading only
//    the previous iteration's labels; ties keep the own label when it is
//    maximal, else go to the smallest (prio, label) with
//    prio(x) = fmix32(x ^ salt) (MurmurHash3's finaliser, a bijection on
//    32-bit words, so labels never tie on prio);
//  * relabelling by prefix sum and cluster contraction (Section 4.1): the
//    inter-cluster arcs are emitted as (cl(u), cl(v), w) triples, radix
//    sorted on the packed key and reduced into a coarse CSR;
//  * the minimum weighted degree as upper bound (Section 4);
//  * Padberg-Rinaldi conditions 1-4 tested edge-parallel (Lemma
//    "Padberg-Rinaldi") and a lock-free union-find over marked edges;
//  * transfer of a side back to the input vertices as a bitmap.
//
// Work is cut by arc count: rows of fewer than 256 arcs are processed on
// row-aligned arc tiles (tile t holds the rows v with row_ptr[v] + v in
// [256 t, 256 (t + 1)), one 64-lane wave per tile, each row owning a region
// of an LDS hash table keyed by neighbour label). Longer rows are listed per
// level: a wave per row with an LDS table up to 1023 arcs, a workgroup per
// row with an LDS table up to 4096 arcs, and beyond that 4096-arc chunks
// (label propagation's first iteration, emission) or label partitions of the
// row, each summed in its own 128 KB LDS table (later LP iterations).
#include <mutex>
#include <utility>
#include <vector>

#include "vc_internal.h"

namespace vc {
namespace {

// ------------------------------------------------------------ primitives
__device__ __forceinline__ uint32_t fmix32_dev(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}
// inverse of fmix32: undo each xorshift and multiply by the modular inverse
__device__ __forceinline__ uint32_t fmix32_inv_dev(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7ED1B41Du;
  h ^= (h >> 13) ^ (h >> 26);
  h *= 0xA5CB9243u;
  h ^= h >> 16;
  return h;
}
// Candidate key: larger connection weight first, then smaller prio.
__device__ __forceinline__ unsigned long long cand_key(uint32_t S, int32_t x, uint32_t salt) {
  return ((unsigned long long)S << 32) | (unsigned long long)(~fmix32_dev((uint32_t)x ^ salt));
}
// Candidate key with the own-label flag between the sum and the prio:
// (S, own, -prio(x)); S < 2^31.
__device__ __forceinline__ unsigned long long own_key(uint32_t S, bool own, int32_t x, uint32_t salt) {
  return ((unsigned long long)S << 33) | ((unsigned long long)own << 32) |
         (unsigned long long)(~fmix32_dev((uint32_t)x ^ salt));
}
__device__ __forceinline__ int32_t key_label(unsigned long long key, uint32_t salt) {
  return (int32_t)(fmix32_inv_dev(~(uint32_t)(key & 0xFFFFFFFFull)) ^ salt);
}
__device__ __forceinline__ uint32_t slot_hash(int32_t x) { return (uint32_t)x * 2654435761u; }
// Low 32 bits of the product of the low 24 bits of x and the golden-ratio
// constant 0x9E3779, as the full-rate 24-bit multiply: written out because
// the compiler otherwise prefers the quarter-rate 32-bit multiply when only
// the low product bits are used.
__device__ __forceinline__ uint32_t mul24_golden(uint32_t x) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, 0x9e3779, %1" : "=v"(r) : "v"(x));
  return r;
}
// Slot in [0, size) for size < 2^9, from 24-bit multiplies only (full rate):
// a 16-bit hash scaled by size. Every product stays below 2^31 (hipcc turns a
// logical right shift of a 24-bit product into an arithmetic one).
__device__ __forceinline__ uint32_t region_slot(int32_t x, uint32_t size) {
  const uint32_t h = (mul24_golden((uint32_t)x ^ ((uint32_t)x >> 16)) >> 8) & 0xFFFFu;
  return __umul24(h, size) >> 16;
}
// Element i of an array addressed with a 32-bit byte offset from its base,
// so that the base stays in scalar registers; needs i * sizeof(T) < 2^32.
template <class T>
__device__ __forceinline__ const T &at32(const T *base, uint32_t i) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}
__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
  return a < b ? a : b;
}

// Full-wave reductions in DPP moves: quad_perm [1,0,3,2] and [2,3,0,1],
// row_half_mirror and row_mirror leave every lane of a 16-lane row with the
// row's result; the broadcasts of lane 15 (to rows 1 and 3) and lane 31 (to
// rows 2 and 3) then fold the rows into lane 63, which is read back into
// every lane. ID is the identity of the operation (what a lane of a row
// that a broadcast skips contributes).
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v, unsigned long long id) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)id, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(id >> 32), (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}
template <class Op>
__device__ __forceinline__ unsigned long long wave_reduce64(unsigned long long v, unsigned long long id, Op op) {
  v = op(v, dpp64<0xB1, 0xF>(v, id));
  v = op(v, dpp64<0x4E, 0xF>(v, id));
  v = op(v, dpp64<0x141, 0xF>(v, id));
  v = op(v, dpp64<0x140, 0xF>(v, id));
  v = op(v, dpp64<0x142, 0xA>(v, id));
  v = op(v, dpp64<0x143, 0xC>(v, id));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Reductions over aligned groups of G lanes (G <= 64 stays inside a wave;
// result in every lane of the group; called by whole waves).
template <int G>
__device__ __forceinline__ unsigned long long grp_max(unsigned long long v) {
  if constexpr (G == 64) return wave_reduce64(v, 0ull, [](unsigned long long a, unsigned long long b) { return umax64(a, b); });
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v = umax64(v, __shfl_xor(v, off, G));
  return v;
}
template <int G>
__device__ __forceinline__ unsigned long long grp_min(unsigned long long v) {
  if constexpr (G == 64) return wave_reduce64(v, ~0ull, [](unsigned long long a, unsigned long long b) { return umin64(a, b); });
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v = umin64(v, __shfl_xor(v, off, G));
  return v;
}
template <int G>
__device__ __forceinline__ unsigned long long grp_sum(unsigned long long v) {
  if constexpr (G == 64) return wave_reduce64(v, 0ull, [](unsigned long long a, unsigned long long b) { return a + b; });
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}
template <int G>
__device__ __forceinline__ int grp_or(int v) {
  if constexpr (G == 64)
    return (int)wave_reduce64((unsigned long long)(uint32_t)v, 0ull,
                              [](unsigned long long a, unsigned long long b) { return a | b; });
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v |= __shfl_xor(v, off, G);
  return v;
}

// Block-wide reductions (all threads call; result valid in every thread).
__device__ __forceinline__ unsigned long long block_max(unsigned long long v, unsigned long long *sh) {
  v = grp_max<64>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long r = sh[0];
  for (int i = 1; i < kBlock / 64; i++) r = umax64(r, sh[i]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ unsigned long long block_min(unsigned long long v, unsigned long long *sh) {
  v = grp_min<64>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long r = sh[0];
  for (int i = 1; i < kBlock / 64; i++) r = umin64(r, sh[i]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long *sh) {
  v = grp_sum<64>(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long r = 0;
  for (int i = 0; i < kBlock / 64; i++) r += sh[i];
  __syncthreads();
  return r;
}
__device__ __forceinline__ int block_or(int v, unsigned long long *sh) {
  return (int)block_max((unsigned long long)grp_or<64>(v), sh) | 0;
}

__device__ __forceinline__ int bits_for(int32_t k) {  // bits to hold values 0..k-1
  int b = 0;
  while (b < 31 && (1 << b) < k) b++;
  return b;
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// ------------------------------------------------------------ basic kernels
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

__global__ void k_status_reset(Status *st) {
  if (threadIdx.x == 0) {
    st->minkey = ~0ull;
    st->wsum = 0;
    st->lam_hat = 0x7FFFFFFFFFFFFFFFll;
    st->err = 0;
    st->k = 0;
    st->ax = 0;
    st->nnz = 0;
    st->nmarked = 0;
    st->wit_v = -1;
    st->wit_level = 0;
    st->updated = 0;
    st->stop = 0;
    st->dmax = 0;
    st->huge_items = 0;
    st->huge_slots = 0;
    st->ring_cnt = 0;
    st->active_cnt = 0;
    st->tile_tot = 0;
    st->big_tiles = 0;
  }
  if (threadIdx.x < 8) st->bin_cnt[threadIdx.x] = 0;
}

// row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz, all within [0, nnz]
__global__ void k_check_rowptr(const int32_t *rp, int32_t n, int64_t nnz, Status *st) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    int32_t a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || (int64_t)b > nnz) bad = 1;
    if (i == 0 && a != 0) bad = 1;
    if (i == n - 1 && (int64_t)b != nnz) bad = 1;
  }
  if (bad) atomicOr(&st->err, ERR_ROWPTR);
}

// Arc tiles: tile t starts at the first row v with rp[v] + v >= t * kTile.
// meta[t] = {first row, short rows, first arc, arcs of the short rows}; a
// trailing row with >= kTile arcs is excluded (the long-row kernels take it).
// The first row of tile t is the smallest v in [0, n] with rp[v] + v >= 256 t.
// As f(v) = rp[v] + v grows strictly, row v is the first row of exactly the
// tiles t with f(v - 1) < 256 t <= f(v): one pass over the rows (k_row_pass)
// writes every tile's first row into meta[t].x, with no search.
// Tiles of more than 4 * 64 arcs (a long row closes them) are also listed in
// `big`, in any order, for the LP kernel that runs them with 8 arcs per thread.
// Device-scope atomics on one cache line are serialized (about 11 ns each on
// this GPU), so a workgroup takes kTilesPer tiles per thread (all their loads
// in flight together) and makes one reservation for its big tiles and one
// 64-bit addition of its (rows, arcs) totals.
constexpr int kTilesPer = 8;
__global__ __launch_bounds__(kBlock) void k_tiles(const int32_t *rp, int32_t n, int32_t ntiles, int4 *meta, Status *st,
                                                   int32_t *big) {
  __shared__ unsigned long long sh[kBlock / 64];
  __shared__ int32_t s_off[kBlock / 64][kTilesPer];
  __shared__ int32_t s_base;
  if (st->err) return;  // k_row_pass built no first rows
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int64_t kSpan = (int64_t)kBlock * kTilesPer;
  unsigned long long tot = 0;  // (rows << 32) + arcs: the arcs of all tiles stay below 2^31
  for (int64_t b0 = blockIdx.x * kSpan; b0 < ntiles; b0 += (int64_t)gridDim.x * kSpan) {
    // first rows from k_row_pass (this pass rewrites meta[t].x unchanged)
    int32_t r0[kTilesPer], r1[kTilesPer];
#pragma unroll
    for (int k = 0; k < kTilesPer; k++) {
      const int64_t t = b0 + (int64_t)k * kBlock + threadIdx.x;
      r0[k] = t < ntiles ? meta[t].x : 0;
      r1[k] = t < ntiles ? (t + 1 == ntiles ? n : meta[t + 1].x) : 0;
    }
    int32_t a0[kTilesPer], a1[kTilesPer], am[kTilesPer];
#pragma unroll
    for (int k = 0; k < kTilesPer; k++) {  // row ids lie in [0, n]
      a0[k] = rp[r0[k]];
      a1[k] = rp[r1[k]];
      am[k] = rp[max(r1[k] - 1, 0)];
    }
    unsigned long long bal[kTilesPer];
#pragma unroll
    for (int k = 0; k < kTilesPer; k++) {
      const int64_t t = b0 + (int64_t)k * kBlock + threadIdx.x;
      bool is_big = false;
      if (t < ntiles) {
        int32_t e = r1[k], ae = a1[k];
        if (e > r0[k] && ae - am[k] >= kTile) {  // a trailing long row is left to the long-row kernels
          e--;
          ae = am[k];
        }
        const int32_t acnt = ae - a0[k];
        meta[t] = make_int4(r0[k], e - r0[k], a0[k], acnt);
        tot += ((unsigned long long)(uint32_t)(e - r0[k]) << 32) + (uint32_t)acnt;
        is_big = acnt > 4 * kTB;
      }
      bal[k] = __ballot(is_big);
      if (lane == 0) s_off[wid][k] = __popcll(bal[k]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // offsets of the (wave, k) groups, one global reservation
      int32_t sum = 0;
      for (int q = 0; q < kBlock / 64; q++)
        for (int k = 0; k < kTilesPer; k++) {
          const int32_t c = s_off[q][k];
          s_off[q][k] = sum;
          sum += c;
        }
      s_base = sum ? atomicAdd(&st->big_tiles, sum) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTilesPer; k++)
      if ((bal[k] >> lane) & 1)
        big[s_base + s_off[wid][k] + __popcll(bal[k] & ((1ull << lane) - 1))] =
            (int32_t)(b0 + (int64_t)k * kBlock + threadIdx.x);
    __syncthreads();
  }
  // totals over the tiles (the algorithmic size of a tile sweep)
  tot = block_sum(tot, sh);
  if (threadIdx.x == 0 && tot) atomicAdd(&st->tile_tot, tot);
}

// largest j in [0, rows) with s_rp[j] <= i (the row holding local arc i)
__device__ __forceinline__ int32_t row_of(const int32_t *s_rp, int32_t rows, int32_t i) {
  int32_t lo = 0, hi = rows - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (s_rp[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One pass over the rows of a level: the first row of every arc tile (into
// meta[t].x, see above) and the lists of long rows (classes 4-7 of
// degree_bin), appended per workgroup: LDS counters, then one global
// reservation per pair of classes and workgroup (a 64-bit addition on two
// adjacent 32-bit counts: a class never holds 2^31 rows, so no carry crosses
// into the other count). A workgroup of kRowBlock threads takes kRowsPer rows
// per thread, which keeps the serialized reservations few.
constexpr int kRowBlock = 1024;
constexpr int kRowsPer = 4;
static_assert(offsetof(Status, bin_cnt) % 8 == 0, "bin_cnt pairs are added as 64-bit words");
__global__ __launch_bounds__(kRowBlock) void k_row_pass(const int32_t *rp, int32_t n, int32_t ntiles, int4 *meta,
                                                        int64_t stride, int32_t *bins, Status *st,
                                                        int32_t long_split) {
  constexpr int kLong = kBins - 4;  // long classes 4 .. kBins - 1
  static_assert(kLong == 4, "two pairs of long classes");
  __shared__ int32_t cnt[kLong], base[kLong];
  // an invalid row_ptr (flagged by k_check_rowptr, earlier on the stream)
  // could name tiles outside [0, ntiles): nothing is built from it
  if (st->err) return;
  constexpr int64_t kSpan = (int64_t)kRowBlock * kRowsPer;
  for (int64_t b0 = blockIdx.x * kSpan; b0 <= n; b0 += (int64_t)gridDim.x * kSpan) {
    if (threadIdx.x < kLong) cnt[threadIdx.x] = 0;
    int32_t lo[kRowsPer], mid[kRowsPer], hi[kRowsPer];
#pragma unroll
    for (int k = 0; k < kRowsPer; k++) {  // rp[v - 1], rp[v], rp[v + 1] where they exist
      const int64_t v = b0 + (int64_t)k * kRowBlock + threadIdx.x;
      lo[k] = v >= 1 && v <= n ? rp[v - 1] : 0;
      mid[k] = v <= n ? rp[v] : 0;
      hi[k] = v < n ? rp[v + 1] : 0;
    }
    __syncthreads();
    int cls[kRowsPer], pos[kRowsPer];
#pragma unroll
    for (int k = 0; k < kRowsPer; k++) {
      const int64_t v = b0 + (int64_t)k * kRowBlock + threadIdx.x;
      if (v <= n) {
        const int64_t t_lo = v == 0 ? 0 : ((int64_t)lo[k] + v - 1) / kTile + 1;
        const int64_t t_hi = min(((int64_t)mid[k] + v) / kTile, (int64_t)ntiles - 1);
        for (int64_t t = t_lo; t <= t_hi; t++) meta[t].x = (int32_t)v;
      }
      const int32_t d = v < n ? hi[k] - mid[k] : 0;
      // classes 4 and 5 split at long_split (256..768) instead of degree_bin's 512
      cls[k] = d < kTile ? -1 : d < long_split ? 0 : d < 1024 ? 1 : degree_bin(d) - 4;
      pos[k] = cls[k] >= 0 ? atomicAdd(&cnt[cls[k]], 1) : 0;
    }
    __syncthreads();
    if (threadIdx.x < kLong / 2) {
      const int c = 2 * threadIdx.x;
      const unsigned long long add = (uint32_t)cnt[c] | ((unsigned long long)(uint32_t)cnt[c + 1] << 32);
      const unsigned long long old =
          add ? atomicAdd(reinterpret_cast<unsigned long long *>(&st->bin_cnt[4 + c]), add) : 0ull;
      base[c] = (int32_t)(uint32_t)old;
      base[c + 1] = (int32_t)(old >> 32);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRowsPer; k++) {
      const int64_t v = b0 + (int64_t)k * kRowBlock + threadIdx.x;
      if (cls[k] >= 0) bins[(int64_t)(4 + cls[k]) * stride + base[cls[k]] + pos[k]] = (int32_t)v;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ XCD-aware tile order
// Workgroup i runs on XCD i mod 8, and each XCD has its own L2. The LP tile
// kernel, with many tiles, deals them to the XCDs in chunks of 64 consecutive
// tiles (chunk c to XCD c mod 8), and the workgroups of an XCD walk its chunks
// in order: the neighbour-label gathers of a tile, which mostly hit ids close
// to its own rows in locality-ordered inputs, then find lines that the XCD's
// L2 already holds for the neighbouring tiles, while at least 32 chunks per
// XCD keep the work balanced on skewed inputs. Fewer tiles are dealt one by
// one. (The union-find tiles keep the plain order: neighbouring tiles at once
// link into the same components and contend.) Grids are multiples of 8.
constexpr int kXcds = 8;
constexpr int kXcdChunkLog = 6;
constexpr int32_t kXcdChunkMin = kXcds * 32 << kXcdChunkLog;  // tiles for chunked dealing
struct XcdWalk {
  int32_t x, l, step, ntiles, cl;
  __device__ __forceinline__ explicit XcdWalk(int32_t n) : ntiles(n) {
    x = (int32_t)(blockIdx.x % kXcds);
    l = (int32_t)(blockIdx.x / kXcds);
    step = (int32_t)(gridDim.x / kXcds);
    cl = n >= kXcdChunkMin ? kXcdChunkLog : 0;
  }
  // increasing in l, so the walk ends at the first tile past the range
  __device__ __forceinline__ int32_t tile() const {
    return (((l >> cl) * kXcds + x) << cl) + (l & ((1 << cl) - 1));
  }
  __device__ __forceinline__ bool ok() const { return tile() < ntiles; }
  __device__ __forceinline__ void next() { l += step; }
};

// Per-lane loops over a long row load kLoadBatch arcs (and their gathers)
// before using any of them, so that one memory latency covers the batch.
constexpr int kLoadBatch = 8;

// ------------------------------------------------------------ LP iteration 1
// Identity labels: S(x) = w(v, x), so the new label is the row's argmax of
// (w, -prio). At level 0 the same pass validates the row and computes the
// weighted degree and the minimum-degree key.
// Up to three long-row classes in one launch: workgroups [first[c],
// first[c + 1]) take class c (its list, count and, for emission, its segment
// region), so classes with few or no rows cost no launch of their own.
struct RowClasses {
  const int32_t *list[3];
  const int32_t *cnt[3];
  int32_t *seg[3];
  int32_t *seg_cnt[3];
  int32_t first[4];
};
__device__ __forceinline__ int row_class(const RowClasses &rc) {
  int c = 0;
  if ((int32_t)blockIdx.x >= rc.first[1]) c = 1;
  if ((int32_t)blockIdx.x >= rc.first[2]) c = 2;
  return c;
}

// Level-0 statistics of one workgroup, (minimum-degree key, weight sum, error
// bits), into its own entry of `part` (combined by k_reduce_parts): device
// atomics on the status words from every workgroup would be serialized.
__device__ __forceinline__ void part_write(unsigned long long *part, unsigned long long key, unsigned long long sum,
                                           int err) {
  unsigned long long *p = part + 3 * (int64_t)blockIdx.x;
  p[0] = key;
  p[1] = sum;
  p[2] = (unsigned long long)(uint32_t)err;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_lp_first(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                      const int32_t *__restrict__ w, int32_t n, RowClasses rc,
                                                      int32_t *__restrict__ L, long long *__restrict__ deg,
                                                      uint32_t salt, int level0, Status *st,
                                                      const int32_t *__restrict__ gv, GStat *gs,
                                                      unsigned long long *part) {
  __shared__ unsigned long long sh[kBlock / 64];
  const int cls = row_class(rc);
  const int32_t *__restrict__ list = rc.list[cls];
  const int32_t bid = (int32_t)blockIdx.x - rc.first[cls], nblk = rc.first[cls + 1] - rc.first[cls];
  const bool stats = level0 && !gv;  // the workgroup's (min-degree key, weight sum, errors) go to part
  if (!gv && st->err) {
    if (stats && threadIdx.x == 0) part_write(part, ~0ull, 0, 0);
    return;
  }
  constexpr int NG = kBlock / G;
  const int gi = threadIdx.x / G, lane = threadIdx.x % G;
  const int32_t cnt = *rc.cnt[cls];
  unsigned long long mykey = ~0ull, mysum = 0;
  int myerr = 0;
  for (int64_t base = bid * (int64_t)NG; base < cnt; base += (int64_t)nblk * NG) {
    int64_t idx = base + gi;
    bool act = idx < cnt;
    int32_t v = act ? list[idx] : 0;
    int32_t beg = act ? rp[v] : 0, end = act ? rp[v + 1] : 0;
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv && act) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    unsigned long long best = 0, sum = 0;
    int err = 0;
    for (int32_t i0 = beg + lane; i0 < end; i0 += G * kLoadBatch) {
      int32_t xs[kLoadBatch], cs[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {  // the batch's loads first (clamped into the row)
        const int32_t i = min(i0 + u * G, end - 1);
        xs[u] = col[i];
        cs[u] = w[i];
      }
      bool bad = false;  // (level 0) an arc of this batch fails an input check
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {
        if (i0 + u * G >= end) break;
        const int32_t x = xs[u], c = cs[u];
        if (level0) bad |= ((uint32_t)x >= (uint32_t)n) | (x == v) | (c < 1);
        sum += (unsigned long long)(uint32_t)c;
        best = umax64(best, cand_key((uint32_t)c, x - b0, sl));
      }
      if (bad) {  // invalid input (rare): the error bits of the batch
#pragma unroll
        for (int u = 0; u < kLoadBatch; u++) {
          if (i0 + u * G >= end) break;
          const int32_t x = xs[u], c = cs[u];
          if (x < 0 || x >= n) err |= ERR_COL;
          if (x == v) err |= ERR_SELF;
          if (c < 1) err |= ERR_WEIGHT;
        }
      }
    }
    best = grp_max<G>(best);
    sum = grp_sum<G>(sum);
    err = grp_or<G>(err);
    if (act && lane == 0) {
      L[v] = end > beg ? key_label(best, sl) + b0 : v;
      if (level0) {
        deg[v] = (long long)sum;
        if (gv) {
          if (err) atomicOr(&gs[gv[v]].err, err);
        } else {
          unsigned long long s32 = sum > 0xFFFFFFFFull ? 0xFFFFFFFFull : sum;
          mykey = umin64(mykey, (s32 << 32) | (uint32_t)v);
          mysum += sum;
          myerr |= err;
        }
      }
    }
  }
  if (stats) {
    unsigned long long k = block_min(mykey, sh);
    unsigned long long s = block_sum(mysum, sh);
    int e = (int)block_max((unsigned long long)myerr, sh);
    if (threadIdx.x == 0) part_write(part, k, s, e);
  }
}

// ------------------------------------------------------------ LP iteration t >= 2
// Long rows (256..4096 arcs), G lanes per row: S(x) = sum of w(v,u) over
// neighbours u with Lin[u] == x, accumulated in an open-addressing LDS table
// (int32 key, uint32 sum; sums are bounded by the total weight <= INT32_MAX)
// of T = the power of two >= 2 d slots (d the row's arcs), so that probing
// ends and only T slots are cleared. Each weight is added with a returning
// atomic: the returned partial sum plus the weight is a lower bound of the
// label's final sum, and the last update of a label sees the final sum, so
// the row maximum of the keys (S, own, -prio) over all updates is the maximum
// over the labels' final sums; no pass over the table is needed. The own-label
// bit sits between S and prio: the maximum has it set exactly when the own
// label attains the maximum sum, which keeps the own label.
template <int G, int TBL>
__global__ __launch_bounds__(kBlock) void k_lp_tab(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ w, const int32_t *__restrict__ Lin,
                                                    int32_t *__restrict__ Lout, const int32_t *__restrict__ list,
                                                    const int32_t *cnt_p, uint32_t salt, const Status *st,
                                                    const int32_t *__restrict__ gv, const GStat *gs) {
  constexpr int NG = kBlock / G;
  __shared__ int32_t tkey[NG][TBL];
  __shared__ uint32_t tval[NG][TBL];
  __shared__ unsigned long long red[kBlock / 64];
  if (!gv && st->err) return;
  const int gi = threadIdx.x / G, lane = threadIdx.x % G;
  const int32_t cnt = *cnt_p;
  for (int64_t base = blockIdx.x * (int64_t)NG; base < cnt; base += (int64_t)gridDim.x * NG) {
    const int64_t idx = base + gi;
    const bool act = idx < cnt;
    const int32_t v = act ? list[idx] : 0;
    const int32_t beg = act ? rp[v] : 0, end = act ? rp[v + 1] : 0;
    const int32_t own = act ? Lin[v] : -1;
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv && act) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    uint32_t T = 2 * G;  // power of two >= 2 d, at most TBL (d <= TBL / 2 for the rows of this class)
    while (T < 2u * (uint32_t)(end - beg) && T < (uint32_t)TBL) T <<= 1;
    const uint32_t mask = T - 1;
    for (uint32_t e = lane; e < T; e += G) {
      tkey[gi][e] = -1;
      tval[gi][e] = 0;
    }
    __syncthreads();
    unsigned long long best = 0;
    for (int32_t i0 = beg + lane; i0 < end; i0 += G * kLoadBatch) {
      int32_t xs[kLoadBatch], cs[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {  // the batch's loads and gathers first
        const int32_t i = min(i0 + u * G, end - 1);
        xs[u] = col[i];
        cs[u] = w[i];
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) xs[u] = Lin[xs[u]];
      uint32_t hs[kLoadBatch];
      int32_t old[kLoadBatch];
      bool real[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {  // claims first, all in flight
        real[u] = i0 + u * G < end;
        hs[u] = (mul24_golden((uint32_t)xs[u] ^ ((uint32_t)xs[u] >> 16)) >> 8) & mask;
        old[u] = real[u] ? atomicCAS(&tkey[gi][hs[u]], -1, xs[u]) : -1;
      }
      bool coll = false;
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) coll |= real[u] && old[u] != -1 && old[u] != xs[u];
      if (__ballot(coll)) {  // (rare: one wave-wide test skips the probing code)
#pragma unroll
        for (int u = 0; u < kLoadBatch; u++) {
          if (!real[u]) continue;
          while (old[u] != -1 && old[u] != xs[u]) {  // taken by another label: probe on
            hs[u] = (hs[u] + 1) & mask;
            old[u] = atomicCAS(&tkey[gi][hs[u]], -1, xs[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++)
        old[u] = real[u] ? (int32_t)atomicAdd(&tval[gi][hs[u]], (uint32_t)cs[u]) : 0;
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++)
        if (real[u])
          best = umax64(best, own_key((uint32_t)old[u] + (uint32_t)cs[u], xs[u] == own, xs[u] - b0, sl));
    }
    if constexpr (G <= 64) {
      best = grp_max<G>(best);
    } else {
      best = block_max(best, red);  // G == kBlock: one group per block
    }
    if (act && lane == 0) Lout[v] = (end == beg || ((best >> 32) & 1)) ? own : key_label(best, sl) + b0;
    __syncthreads();
  }
}

// Kernel timing: one thread copies the level's tile totals into the timing
// record, a page-locked host buffer, as (rows, big tiles, arcs: 64 bits).
__device__ __forceinline__ void prof_snapshot(int32_t *prof, const Status *st) {
  if (prof && blockIdx.x == 0 && threadIdx.x == 0) {
    const unsigned long long t = st->tile_tot;
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(prof);
    dst[0] = (t >> 32) | ((unsigned long long)(uint32_t)st->big_tiles << 32);
    dst[1] = t & 0xFFFFFFFFull;
  }
}

// ------------------------------------------------------------ tiled LP (short rows)
// A tile's arcs are split into 64 runs of q = ceil(arcs/64) <= 8 consecutive
// arcs, one per lane of the tile's single wave. Every global load of a lane's
// run is issued before the barrier that publishes the tile's row offsets in
// LDS; the row of each arc is then found by one binary search and a forward
// walk.

// combine per-block (min key, weight sum, error bits) into the status
__global__ void k_reduce_parts(const unsigned long long *part, int32_t count, Status *st) {
  __shared__ unsigned long long red[kBlock / 64];
  unsigned long long k = ~0ull, sm = 0, e = 0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) {
    k = umin64(k, part[3 * i]);
    sm += part[3 * i + 1];
    e |= part[3 * i + 2];
  }
  k = block_min(k, red);
  sm = block_sum(sm, red);
  e = block_max(e, red);  // error bits are few: the maximum is nonzero iff any bit is set
  if (threadIdx.x == 0) {
    if (k != ~0ull) atomicMin(&st->minkey, k);
    if (sm) atomicAdd(&st->wsum, sm);
    if (e) atomicOr(&st->err, (int)e);
  }
}

// Iteration t >= 2 on a tile. Lane l takes the tile's arcs [NQ l, NQ l + NQ)
// (NQ = 4 on tiles of at most 256 arcs, 8 on the others), so the arcs of a
// row sit in one lane or a few. Loads use clamped indices instead of
// branches, so all arc loads, and then all label gathers, are in flight
// together. The row data stays in registers (lane j: row j's first arc; the
// next lane's register gives its end), and the row of each arc comes from a
// running maximum over row-start marks (lane_rows). Row j owns the hash
// region [2 first_j, 2 end_j) of the tile's LDS table (twice its arc count,
// so probing always ends), keyed by neighbour label and summing weights.
// Runs of adjacent arcs of equal (row, label) within a lane are folded
// first; the claims of a lane are all issued before any result is used.
// Each run then adds its weight with a returning atomic, and the candidate
// keys (sum, own, -prio) of a lane's runs are folded per row piece into one
// maximum update per piece, so no pass over the table is needed.
// Inclusive maximum over lanes 0..lane of the wave, in DPP moves: shifts
// by 1, 2, 4 and 8 within the 16-lane rows, then the broadcasts of lane 15
// (to rows 1 and 3) and lane 31 (to rows 2 and 3). Lanes without a source
// keep 0, the identity of the unsigned maximum.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false));  // row_shr:1
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false));  // row_shr:2
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false));  // row_shr:4
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false));  // row_shr:8
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return x;
}


// Row-start marks of a tile's arcs: one byte per arc, lane l's NQ arcs in
// its own word.
template <int NQ>
struct MarkWord;
template <>
struct MarkWord<4> {
  using T = uint32_t;
};
template <>
struct MarkWord<8> {
  using T = unsigned long long;
};

// Row (tile-local index) of each of a lane's NQ arcs: the running maximum of
// the marks within the lane's word, then the maximum over all earlier lanes
// (a DPP scan), since a row's index is marked at its first arc and rows
// grow with the arc position.
template <int NQ>
__device__ __forceinline__ void lane_rows(typename MarkWord<NQ>::T v, int32_t (&rw)[NQ]) {
  uint32_t b[NQ], run = 0;
#pragma unroll
  for (int k = 0; k < NQ; k++) {
    run = max(run, (uint32_t)(v >> (8 * k)) & 0xFFu);
    b[k] = run;
  }
  const uint32_t carry =
      (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wave_incl_max(run), 0x138, 0xF, 0xF, false);  // wave_shr:1
#pragma unroll
  for (int k = 0; k < NQ; k++) rw[k] = (int32_t)max(b[k], carry);
}

// LDS of one tile whose threads take NQ arcs each. Row j: (first arc |
// arc count << 16, own label) and its best key; the hash table interleaves
// (label, weight sum) and holds two slots per arc of the tile.
template <int NQ>
struct alignas(16) LpTileShared {
  static constexpr int kSlots = 2 * NQ * kTB;
  // 8-arc tiles: a sink slot per lane takes the updates of inactive lanes
  // (no branches); the 4-arc kernel masks them instead and keeps its LDS
  // small enough for more resident workgroups
  static constexpr int kSinks = NQ == kPerThread ? kTB : 0;
  uint2 row[kTile];
  unsigned long long best[kTile + kSinks];
  uint2 slot[kSlots + kSinks];
  typename MarkWord<NQ>::T mark[kTB];
};

// Registers of one tile, fetched ahead of its processing: per thread NQ arcs
// (neighbour, then its label, and weight) and the tile's row data, one entry
// per 64 rows (only the entries below the tile's row count are loaded).
constexpr int kRowRegs = kTile / kTB;  // row-offset registers per lane (rows <= kTile)

template <bool B, int NQ>
struct LpFetch {
  int4 m;
  int32_t xs[NQ], cs[NQ];
  int32_t rpv[kRowRegs + 1];
  int32_t ownv[kRowRegs];
  int32_t basev[B ? kRowRegs : 1];
  uint32_t saltv[B ? kRowRegs : 1];
};

// Lane l takes the tile's arcs [NQ l, NQ l + NQ) (clamped loads: lanes past
// the end repeat the last arc and are masked later).
template <bool B, int NQ>
__device__ __forceinline__ void lp_fetch_loads(LpFetch<B, NQ> &f, int4 m, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ col, const int32_t *__restrict__ w,
                                               const int32_t *__restrict__ Lin, const int32_t *__restrict__ gv,
                                               const GStat *gs) {
  const int lane = threadIdx.x;
  f.m = m;
  const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
#pragma unroll
  for (int k = 0; k < NQ; k++) f.xs[k] = f.cs[k] = 0;
  if (acnt > 0) {
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      const uint32_t i = (uint32_t)min(NQ * lane + k, acnt - 1);
      f.xs[k] = at32(col + a0, i);
      f.cs[k] = at32(w + a0, i);
    }
  }
#pragma unroll
  for (int r = 0; r <= kRowRegs; r++) {
    f.rpv[r] = 0;
    if (r == 0 || kTB * r <= rows) f.rpv[r] = at32(rp + r0, (uint32_t)min(lane + kTB * r, rows));
  }
  if (rows > 0) {
#pragma unroll
    for (int r = 0; r < kRowRegs; r++) {
      if (r > 0 && kTB * r >= rows) break;
      const uint32_t j = (uint32_t)min(lane + kTB * r, rows - 1);
      f.ownv[r] = at32(Lin + r0, j);
      if constexpr (B) {
        const GStat &g = gs[at32(gv + r0, j)];
        f.basev[r] = g.base;
        f.saltv[r] = g.salt;
      }
    }
  }
}
template <bool B, int NQ>
__device__ __forceinline__ void lp_fetch_gather(LpFetch<B, NQ> &f, const int32_t *__restrict__ Lin) {
  if (f.m.w > 0) {
#pragma unroll
    for (int k = 0; k < NQ; k++) f.xs[k] = at32(Lin, (uint32_t)f.xs[k]);
  }
}

// The LDS phases of one tile whose registers were fetched; `hook` runs after
// the table updates (the caller issues the next tile's gathers there).
template <bool B, int NQ, class Hook>
__device__ __forceinline__ void lp_tile_run(const LpFetch<B, NQ> &f, int32_t *__restrict__ Lout, uint32_t salt,
                                            LpTileShared<NQ> &sh, int32_t *s_base, uint32_t *s_salt, Hook hook) {
  const int lane = threadIdx.x;
  const int32_t r0 = f.m.x, rows = f.m.y, a0 = f.m.z, acnt = f.m.w;
  uint8_t *s_mark = reinterpret_cast<uint8_t *>(sh.mark);
  sh.mark[lane] = 0;
  // rows: packed (first arc, count) and own label; marks at first arcs
  int32_t cnt[kRowRegs];
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    cnt[r] = 0;
    if (r > 0 && kTB * r >= rows) break;
    const int j = lane + kTB * r;
    // row j + 1 starts where lane + 1 holds it; lane 63 takes lane 0 of the next register
    const int32_t nxt = r + 1 <= kRowRegs ? __builtin_amdgcn_readlane(f.rpv[r + 1], 0) : 0;
    const int32_t hi = __builtin_amdgcn_update_dpp(nxt, f.rpv[r], 0x130, 0xF, 0xF, false) - a0;  // wave_shl:1
    const int32_t lo = f.rpv[r] - a0;
    cnt[r] = hi - lo;
    if (j < rows) {
      sh.row[j] = make_uint2((uint32_t)lo | ((uint32_t)cnt[r] << 16), (uint32_t)f.ownv[r]);
      sh.best[j] = 0;
      if constexpr (B) {
        s_base[j] = f.basev[r];
        s_salt[j] = f.saltv[r];
      }
      if (cnt[r] > 0) s_mark[lo] = (uint8_t)j;
    }
  }
  // the table: two slots per arc, cleared 16 bytes (two slots) per lane and store
#pragma unroll
  for (int i = 0; i < NQ; i++) {
    if (kTB * i >= acnt) break;
    const int e = lane + kTB * i;
    if (e < acnt) reinterpret_cast<uint4 *>(sh.slot)[e] = make_uint4(~0u, 0u, ~0u, 0u);
  }
  __syncthreads();
  if (acnt > 0) {
    int32_t rw[NQ], hb[NQ], hsz[NQ], ow[NQ], bj[NQ];
    uint32_t sj[NQ], hh[NQ], cc[NQ], old[NQ];
    bool real[NQ], ok[NQ];
    lane_rows<NQ>(sh.mark[lane], rw);
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      real[k] = NQ * lane + k < acnt;
      const uint2 ri = sh.row[rw[k]];
      hb[k] = 2 * (int32_t)(ri.x & 0xFFFFu);
      hsz[k] = 2 * (int32_t)(ri.x >> 16);
      ow[k] = (int32_t)ri.y;
      bj[k] = 0;
      sj[k] = salt;
      if constexpr (B) { bj[k] = s_base[rw[k]]; sj[k] = s_salt[rw[k]]; }
    }
    // fold runs of adjacent arcs of equal (row, label) into their first arc
    // (register work instead of LDS atomics)
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      cc[k] = (uint32_t)f.cs[k];
      ok[k] = real[k] && !(k > 0 && real[k - 1] && rw[k] == rw[k - 1] && f.xs[k] == f.xs[k - 1]);
    }
#pragma unroll
    for (int k = NQ - 1; k > 0; k--)
      if (real[k] && !ok[k]) cc[k - 1] += cc[k];
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      hh[k] = region_slot(f.xs[k], (uint32_t)hsz[k]);
      if constexpr (LpTileShared<NQ>::kSinks > 0)
        old[k] = atomicCAS(&sh.slot[ok[k] ? hb[k] + (int32_t)hh[k] : LpTileShared<NQ>::kSlots + lane].x, ~0u,
                           (uint32_t)f.xs[k]);
      else
        old[k] = ok[k] ? atomicCAS(&sh.slot[hb[k] + (int32_t)hh[k]].x, ~0u, (uint32_t)f.xs[k]) : ~0u;
    }
    // collisions are rare (the table is at most half full): one wave-wide
    // test skips the probing code when no lane has one
    bool coll = false;
#pragma unroll
    for (int k = 0; k < NQ; k++) coll |= ok[k] && old[k] != ~0u && old[k] != (uint32_t)f.xs[k];
    if (__ballot(coll)) {
#pragma unroll
      for (int k = 0; k < NQ; k++) {
        if (!ok[k]) continue;
        while (old[k] != ~0u && old[k] != (uint32_t)f.xs[k]) {  // taken by another label
          hh[k] = (hh[k] + 1 == (uint32_t)hsz[k]) ? 0 : hh[k] + 1;
          old[k] = atomicCAS(&sh.slot[hb[k] + (int32_t)hh[k]].x, ~0u, (uint32_t)f.xs[k]);
        }
      }
    }
    // add the run weights: the returned partial sum plus the run's weight is
    // a lower bound of the label's final sum, and the last update of a label
    // sees the final sum, so the maximum of (partial sum, -prio) over all
    // updates of a row is the maximum over its labels' final sums
    // The key (S, own, -prio) orders by sum, then the own label first, then
    // the smaller prio, so the row maximum decides the update rule at once.
#pragma unroll
    for (int k = 0; k < NQ; k++)
      if constexpr (LpTileShared<NQ>::kSinks > 0)
        old[k] = atomicAdd(&sh.slot[ok[k] ? hb[k] + (int32_t)hh[k] : LpTileShared<NQ>::kSlots + lane].y, cc[k]);
      else
        old[k] = ok[k] ? atomicAdd(&sh.slot[hb[k] + (int32_t)hh[k]].y, cc[k]) : 0u;
    // running maximum per row piece of this thread, one update per piece
    unsigned long long run = 0;
    int32_t cur = rw[0];
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      if (!real[k]) break;
      if (rw[k] != cur) {
        atomicMax(&sh.best[cur], run);
        run = 0;
        cur = rw[k];
      }
      if (ok[k]) run = umax64(run, own_key(old[k] + cc[k], f.xs[k] == ow[k], f.xs[k] - bj[k], sj[k]));
    }
    if (real[0]) atomicMax(&sh.best[cur], run);
  }
  hook();
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    if (r > 0 && kTB * r >= rows) break;
    const int j = lane + kTB * r;
    if (j < rows) {
      const int32_t own = f.ownv[r];
      int32_t out = own;
      if (cnt[r] > 0) {
        const unsigned long long b = sh.best[j];
        int32_t bjj = 0;
        uint32_t sjj = salt;
        if constexpr (B) { bjj = f.basev[r]; sjj = f.saltv[r]; }
        if (!((b >> 32) & 1)) out = key_label(b, sjj) + bjj;
      }
      Lout[r0 + j] = out;
    }
  }
  __syncthreads();
}

// The tiles of at most 4 * 64 arcs, 4 arcs per thread. A workgroup (one
// wave) takes TP consecutive tiles of the XCD-aware order: it issues the
// loads of all of them, then all their label gathers, and only then runs
// their LDS phases one after the other, so TP tiles' memory latency is
// paid once (the kernel is bound by the latency of these dependent loads
// times the number of resident waves, not by bytes). Short-lived
// workgroups leave the balancing to the hardware. The tiles of more than
// 256 arcs are left to k_lp_tile_big.
template <bool B, int TP>
__global__ __launch_bounds__(kTB) void k_lp_tile(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ w, const int32_t *__restrict__ Lin,
                                                     int32_t *__restrict__ Lout, const int4 *__restrict__ meta,
                                                     int32_t ntiles, uint32_t salt, const Status *st,
                                                     const int32_t *__restrict__ gv, const GStat *gs, int32_t *prof) {
  __shared__ LpTileShared<4> sh;
  __shared__ int32_t s_base[B ? kTile : 1];
  __shared__ uint32_t s_salt[B ? kTile : 1];
  prof_snapshot(prof, st);
  if (!B && st->err) return;
  constexpr int32_t kSmall = 4 * kTB;
  XcdWalk xw((ntiles + TP - 1) / TP);
  for (; xw.ok(); xw.next()) {
    const int32_t t0 = xw.tile() * TP;
    int4 m[TP];
    bool use[TP];
#pragma unroll
    for (int u = 0; u < TP; u++) {
      m[u] = t0 + u < ntiles ? meta[t0 + u] : make_int4(0, 0, 0, 0);
      use[u] = m[u].w <= kSmall && (m[u].y > 0 || m[u].w > 0);
      if (!use[u]) m[u] = make_int4(m[u].x, 0, 0, 0);  // nothing to load beyond row pointer r0
    }
    LpFetch<B, 4> f[TP];
#pragma unroll
    for (int u = 0; u < TP; u++) lp_fetch_loads(f[u], m[u], rp, col, w, Lin, gv, gs);
#pragma unroll
    for (int u = 0; u < TP; u++) lp_fetch_gather(f[u], Lin);
#pragma unroll
    for (int u = 0; u < TP; u++)
      if (use[u]) lp_tile_run<B, 4>(f[u], Lout, salt, sh, s_base, s_salt, []() {});
  }
}

// The listed tiles of more than 256 arcs, 8 arcs per thread. Persistent
// (as many workgroups as fit, striding over the list): the next tile's arcs
// and row data are loaded before this tile's LDS phases and its label
// gathers are issued after this tile's table updates, so the memory latency
// of one tile overlaps the LDS work of the previous one.
template <bool B>
__global__ __launch_bounds__(kTB) void k_lp_tile_big(const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ w,
                                                         const int32_t *__restrict__ Lin, int32_t *__restrict__ Lout,
                                                         const int4 *__restrict__ meta,
                                                         const int32_t *__restrict__ big, uint32_t salt,
                                                         const Status *st, const int32_t *__restrict__ gv,
                                                         const GStat *gs) {
  __shared__ LpTileShared<kPerThread> sh;
  __shared__ int32_t s_base[B ? kTile : 1];
  __shared__ uint32_t s_salt[B ? kTile : 1];
  if (!B && st->err) return;
  const int32_t cnt = st->big_tiles;
  const int32_t G = (int32_t)gridDim.x;
  int32_t i = (int32_t)blockIdx.x;
  if (i >= cnt) return;
  LpFetch<B, kPerThread> cur;
  lp_fetch_loads(cur, meta[big[i]], rp, col, w, Lin, gv, gs);
  lp_fetch_gather(cur, Lin);
  while (true) {
    const int32_t in = i + G;
    const bool more = in < cnt;
    LpFetch<B, kPerThread> nxt;
    if (more) lp_fetch_loads(nxt, meta[big[in]], rp, col, w, Lin, gv, gs);
    lp_tile_run<B, kPerThread>(cur, Lout, salt, sh, s_base, s_salt, [&]() {
      if (more) lp_fetch_gather(nxt, Lin);
    });
    if (!more) break;
    i = in;
    cur = nxt;
  }
}

// ------------------------------------------------------------ LP iteration 1 on tiles
// Identity labels: S(x) = w(v, x), so a row's new label is the argmax of
// (w, -prio) over its arcs, and no label is gathered. At level 0 the same
// pass validates every arc and sums the weighted degree, and each workgroup
// leaves its minimum-degree key, weight sum and error bits in `part`.
// Lane l takes the tile's arcs [NQ l, NQ l + NQ); rows come from the marks
// (lane_rows); each thread folds its keys and sums per row piece and makes
// one LDS update per piece.
template <bool L0, bool B, int NQ>
struct alignas(16) FirstShared {
  unsigned long long best[kTile];
  unsigned long long sum[L0 ? kTile : 1];
  int32_t base[B ? kTile : 1];
  uint32_t salt[B ? kTile : 1];
  typename MarkWord<NQ>::T mark[kTB];
};

template <bool B, int NQ>
struct FirstFetch {
  int4 m;
  int32_t xs[NQ], cs[NQ];
  int32_t rpv[kRowRegs + 1];
  int32_t basev[B ? kRowRegs : 1];
  uint32_t saltv[B ? kRowRegs : 1];
};

template <bool B, int NQ>
__device__ __forceinline__ void first_fetch(FirstFetch<B, NQ> &f, int4 m, const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ col, const int32_t *__restrict__ w,
                                            const int32_t *__restrict__ gv, const GStat *gs) {
  const int lane = threadIdx.x;
  f.m = m;
  const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
#pragma unroll
  for (int k = 0; k < NQ; k++) f.xs[k] = f.cs[k] = 0;
  if (acnt > 0) {
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      const uint32_t i = (uint32_t)min(NQ * lane + k, acnt - 1);
      f.xs[k] = at32(col + a0, i);
      f.cs[k] = at32(w + a0, i);
    }
  }
#pragma unroll
  for (int r = 0; r <= kRowRegs; r++) {
    f.rpv[r] = 0;
    if (r == 0 || kTB * r <= rows) f.rpv[r] = at32(rp + r0, (uint32_t)min(lane + kTB * r, rows));
  }
  if constexpr (B) {
    if (rows > 0) {
#pragma unroll
      for (int r = 0; r < kRowRegs; r++) {
        if (r > 0 && kTB * r >= rows) break;
        const GStat &g = gs[at32(gv + r0, (uint32_t)min(lane + kTB * r, rows - 1))];
        f.basev[r] = g.base;
        f.saltv[r] = g.salt;
      }
    }
  }
}

// Level-0 accumulators of a workgroup (single solves only).
struct FirstAcc {
  unsigned long long key = ~0ull, sum = 0;
  int err = 0;
};

template <bool L0, bool B, int NQ>
__device__ __forceinline__ void first_tile_run(const FirstFetch<B, NQ> &f, int32_t n, int32_t *__restrict__ L,
                                               long long *__restrict__ deg, uint32_t salt,
                                               const int32_t *__restrict__ gv, GStat *gs, FirstShared<L0, B, NQ> &sh,
                                               FirstAcc &acc) {
  using MW = typename MarkWord<NQ>::T;
  const int lane = threadIdx.x;
  const int32_t r0 = f.m.x, rows = f.m.y, a0 = f.m.z, acnt = f.m.w;
  uint8_t *s_mark = reinterpret_cast<uint8_t *>(sh.mark);
  sh.mark[lane] = 0;
  int32_t cnt[kRowRegs];
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    cnt[r] = 0;
    if (r > 0 && kTB * r >= rows) break;
    const int j = lane + kTB * r;
    const int32_t nxt = __builtin_amdgcn_readlane(f.rpv[r + 1], 0);
    cnt[r] = __builtin_amdgcn_update_dpp(nxt, f.rpv[r], 0x130, 0xF, 0xF, false) - f.rpv[r];  // wave_shl:1
    if (j < rows) {
      sh.best[j] = 0;
      if constexpr (L0) sh.sum[j] = 0;
      if constexpr (B) {
        sh.base[j] = f.basev[r];
        sh.salt[j] = f.saltv[r];
      }
      if (cnt[r] > 0) s_mark[f.rpv[r] - a0] = (uint8_t)j;
    }
  }
  __syncthreads();
  if (acnt > 0) {
    int32_t rw[NQ];
    lane_rows<NQ>(sh.mark[lane], rw);
    // running maximum and weight sum per row piece, one LDS update per piece
    unsigned long long best = 0, sum = 0;
    int32_t cur = rw[0], bj = 0;
    uint32_t sj = salt;
    bool bad = false;  // (level 0) an arc of this lane fails an input check
    if constexpr (B) { bj = sh.base[cur]; sj = sh.salt[cur]; }
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      if (NQ * lane + k >= acnt) break;
      if (rw[k] != cur) {
        atomicMax(&sh.best[cur], best);
        if constexpr (L0) atomicAdd(&sh.sum[cur], sum);
        best = sum = 0;
        cur = rw[k];
        if constexpr (B) { bj = sh.base[cur]; sj = sh.salt[cur]; }
      }
      const int32_t x = f.xs[k], c = f.cs[k];
      best = umax64(best, cand_key((uint32_t)c, x - bj, sj));
      if constexpr (L0) {
        sum += (unsigned long long)(uint32_t)c;
        bad |= ((uint32_t)x >= (uint32_t)n) | (x == r0 + cur) | (c < 1);
      }
    }
    if (NQ * lane < acnt) {
      atomicMax(&sh.best[cur], best);
      if constexpr (L0) atomicAdd(&sh.sum[cur], sum);
    }
    if constexpr (L0) {
      if (__ballot(bad)) {  // invalid input (rare): the error bits of this lane's arcs
#pragma unroll
        for (int k = 0; k < NQ; k++) {
          if (NQ * lane + k >= acnt) break;
          const int32_t x = f.xs[k], c = f.cs[k];
          int e = 0;
          if (x < 0 || x >= n) e |= ERR_COL;
          if (x == r0 + rw[k]) e |= ERR_SELF;
          if (c < 1) e |= ERR_WEIGHT;
          if constexpr (B) {
            if (e) atomicOr(&gs[gv[r0 + rw[k]]].err, e);  // straight to the graph's flags
          } else {
            acc.err |= e;
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    if (r > 0 && kTB * r >= rows) break;
    const int j = lane + kTB * r;
    if (j < rows) {
      const int32_t v = r0 + j;
      int32_t bj = 0;
      uint32_t sj = salt;
      if constexpr (B) { bj = f.basev[r]; sj = f.saltv[r]; }
      L[v] = cnt[r] > 0 ? key_label(sh.best[j], sj) + bj : v;
      if constexpr (L0) {
        const unsigned long long d = sh.sum[j];
        const unsigned long long dd = cnt[r] > 0 ? d : 0ull;
        deg[v] = (long long)dd;
        if constexpr (!B) {
          acc.key = umin64(acc.key, ((dd > 0xFFFFFFFFull ? 0xFFFFFFFFull : dd) << 32) | (uint32_t)v);
          acc.sum += dd;
        }
      }
    }
  }
  __syncthreads();
}

template <bool L0, bool B>
__device__ __forceinline__ void first_acc_flush(const FirstAcc &acc, unsigned long long *part, int32_t slot) {
  if constexpr (L0 && !B) {
    const unsigned long long k = grp_min<64>(acc.key);
    const unsigned long long sm = grp_sum<64>(acc.sum);
    const int e = grp_or<64>(acc.err);
    if (threadIdx.x == 0) {
      part[3 * (int64_t)slot] = k;
      part[3 * (int64_t)slot + 1] = sm;
      part[3 * (int64_t)slot + 2] = (unsigned long long)e;
    }
  }
}

// Tiles of at most 256 arcs, TP consecutive tiles per workgroup step (all
// their loads in flight together); tiles of more than 256 arcs are left to
// k_first_tile_big. Workgroup i writes part entry i.
template <bool L0, bool B, int TP>
__global__ __launch_bounds__(kTB) void k_first_tile(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ w, int32_t n,
                                                        const int4 *__restrict__ meta, int32_t ntiles,
                                                        int32_t *__restrict__ L, long long *__restrict__ deg,
                                                        uint32_t salt, const Status *st,
                                                        unsigned long long *__restrict__ part,
                                                        const int32_t *__restrict__ gv, GStat *gs, int32_t *prof) {
  __shared__ FirstShared<L0, B, 4> sh;
  prof_snapshot(prof, st);
  FirstAcc acc;
  if (B || !st->err) {
    const int32_t groups = (ntiles + TP - 1) / TP;
    for (int32_t g = blockIdx.x; g < groups; g += gridDim.x) {
      int4 m[TP];
      bool use[TP];
#pragma unroll
      for (int u = 0; u < TP; u++) {
        const int32_t t = g * TP + u;
        m[u] = t < ntiles ? meta[t] : make_int4(0, 0, 0, 0);
        use[u] = t < ntiles && m[u].w <= 4 * kTB;
        if (!use[u]) m[u] = make_int4(m[u].x, 0, 0, 0);
      }
      FirstFetch<B, 4> f[TP];
#pragma unroll
      for (int u = 0; u < TP; u++) first_fetch(f[u], m[u], rp, col, w, gv, gs);
#pragma unroll
      for (int u = 0; u < TP; u++)
        if (use[u]) first_tile_run<L0, B, 4>(f[u], n, L, deg, salt, gv, gs, sh, acc);
    }
  }
  first_acc_flush<L0, B>(acc, part, (int32_t)blockIdx.x);
}

// Every tile, one per workgroup (4 or 8 arcs per lane by the tile's size):
// the hardware keeps many of these short-lived workgroups in flight instead
// of a workgroup holding several tiles' loads. Workgroup i writes part
// entry i.
template <bool L0, bool B>
__global__ __launch_bounds__(kTB) void k_first_tile_each(const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col,
                                                             const int32_t *__restrict__ w, int32_t n,
                                                             const int4 *__restrict__ meta, int32_t ntiles,
                                                             int32_t *__restrict__ L, long long *__restrict__ deg,
                                                             uint32_t salt, const Status *st,
                                                             unsigned long long *__restrict__ part,
                                                             const int32_t *__restrict__ gv, GStat *gs,
                                                             int32_t *prof) {
  __shared__ FirstShared<L0, B, kPerThread> sh8;
  prof_snapshot(prof, st);
  FirstAcc acc;
  if (B || !st->err) {
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
      const int4 m = meta[t];
      if (m.w <= 4 * kTB) {
        FirstFetch<B, 4> f;
        first_fetch(f, m, rp, col, w, gv, gs);
        first_tile_run<L0, B, 4>(f, n, L, deg, salt, gv, gs, *reinterpret_cast<FirstShared<L0, B, 4> *>(&sh8),
                                 acc);
      } else {
        FirstFetch<B, kPerThread> f;
        first_fetch(f, m, rp, col, w, gv, gs);
        first_tile_run<L0, B, kPerThread>(f, n, L, deg, salt, gv, gs, sh8, acc);
      }
    }
  }
  first_acc_flush<L0, B>(acc, part, (int32_t)blockIdx.x);
}

// The listed tiles of more than 256 arcs, 8 arcs per lane. Persistent (as
// many workgroups as fit, striding over the list), with the next tile's
// loads issued before this tile's LDS phases; workgroup i writes part entry
// part_base + i.
template <bool L0, bool B>
__global__ __launch_bounds__(kTB) void k_first_tile_big(const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const int32_t *__restrict__ w, int32_t n,
                                                            const int4 *__restrict__ meta,
                                                            const int32_t *__restrict__ big,
                                                            int32_t *__restrict__ L, long long *__restrict__ deg,
                                                            uint32_t salt, const Status *st,
                                                            unsigned long long *__restrict__ part, int32_t part_base,
                                                            const int32_t *__restrict__ gv, GStat *gs) {
  __shared__ FirstShared<L0, B, kPerThread> sh;
  FirstAcc acc;
  if (B || !st->err) {
    const int32_t nb = st->big_tiles;
    int32_t i = (int32_t)blockIdx.x;
    if (i < nb) {
      FirstFetch<B, kPerThread> cur;
      first_fetch(cur, meta[big[i]], rp, col, w, gv, gs);
      while (true) {
        const int32_t in = i + (int32_t)gridDim.x;
        FirstFetch<B, kPerThread> nxt;
        if (in < nb) first_fetch(nxt, meta[big[in]], rp, col, w, gv, gs);
        first_tile_run<L0, B, kPerThread>(cur, n, L, deg, salt, gv, gs, sh, acc);
        if (in >= nb) break;
        i = in;
        cur = nxt;
      }
    }
  }
  first_acc_flush<L0, B>(acc, part, part_base + (int32_t)blockIdx.x);
}

// ------------------------------------------------------------ huge rows
// Rows longer than 4096 arcs: split into chunks; one workgroup per chunk.
// plan, per huge vertex i by mode:
//  0: meta[3i] = first chunk (chunks of kHugeChunk arcs);
//  1: the same plus meta[3i+1] = table offset, meta[3i+2] = table size
//     (power of two >= 2 d) of the global-table path (runs only when
//     huge_fallback is set);
//  2: label partitions: meta[3i] = first work item, meta[3i+1] = parts
//     P = ceil(2 d / (kPartDistinct kPartSlots)) (room for d / kPartDistinct
//     distinct labels at load 1/2), meta[3i+2] = 0 (the row's overflow flag);
//  3: (only when huge_overflow is set) the rows whose flag is set get
//     P = ceil(2 d / kPartSlots) (room for d distinct labels) and a cleared
//     best key; the others get no item and keep their key.
// (deg_zero, at level 0: the huge rows' degree accumulators, zeroed here)
__global__ void k_huge_plan(const int32_t *rp, const int32_t *list, const int32_t *cnt_p, int32_t *meta,
                            unsigned long long *best, int with_table, int64_t cap, Status *st,
                            long long *deg_zero) {
  __shared__ int64_t sh_c[kBlock], sh_t[kBlock];
  __shared__ int64_t carry_c, carry_t;
  if (st->err) return;
  if (with_table == 1 && !st->huge_fallback) return;  // the global-table path is the fallback only
  if (with_table == 3 && !st->huge_overflow) return;  // no partition overflowed
  const int32_t cnt = *cnt_p;
  if (threadIdx.x == 0) { carry_c = 0; carry_t = 0; }
  __syncthreads();
  for (int32_t base = 0; base < cnt; base += kBlock) {
    int32_t i = base + threadIdx.x;
    int64_t c = 0, t = 0;
    if (i < cnt) {
      int32_t v = list[i];
      int32_t d = rp[v + 1] - rp[v];
      c = (d + kHugeChunk - 1) / kHugeChunk;
      if (with_table == 1) { t = 1; while (t < 2 * (int64_t)d) t <<= 1; }
      if (with_table == 2) {
        constexpr int64_t room = (int64_t)kPartDistinct * kPartSlots;
        c = t = (2 * (int64_t)d + room - 1) / room;
      }
      if (with_table == 3) c = t = meta[3 * (int64_t)i + 2] ? (2 * (int64_t)d + kPartSlots - 1) / kPartSlots : 0;
      if (with_table != 3 || c > 0) best[i] = 0;
      if (deg_zero) deg_zero[v] = 0;
    }
    sh_c[threadIdx.x] = c;
    sh_t[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {  // inclusive scan (Hillis-Steele)
      int64_t ac = threadIdx.x >= off ? sh_c[threadIdx.x - off] : 0;
      int64_t at = threadIdx.x >= off ? sh_t[threadIdx.x - off] : 0;
      __syncthreads();
      sh_c[threadIdx.x] += ac;
      sh_t[threadIdx.x] += at;
      __syncthreads();
    }
    if (i < cnt) {
      meta[3 * (int64_t)i] = (int32_t)(carry_c + sh_c[threadIdx.x] - c);
      meta[3 * (int64_t)i + 1] = with_table >= 2 ? (int32_t)t : (int32_t)(carry_t + sh_t[threadIdx.x] - t);
      if (with_table != 3) meta[3 * (int64_t)i + 2] = with_table == 2 ? 0 : (int32_t)t;
    }
    __syncthreads();
    if (threadIdx.x == kBlock - 1) { carry_c += sh_c[kBlock - 1]; carry_t += sh_t[kBlock - 1]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->huge_items = (int32_t)carry_c;
    if (with_table >= 2) {  // the partition count of row i sits in meta[3i + 1]
      st->huge_ticket = 0;
      if (with_table == 2) {
        st->huge_overflow = 0;
        st->huge_fallback = 0;
      }
    } else {
      st->huge_slots = (int32_t)carry_t;
      if (carry_t > cap) atomicOr(&st->err, ERR_ROWPTR);  // cannot happen: sum of 2^ceil(log2 2d) <= 4 nnz
    }
  }
}

__device__ __forceinline__ int32_t huge_find(const int32_t *meta, int32_t cnt, int32_t p, int field) {
  int32_t lo = 0, hi = cnt - 1;  // last i with meta[3i+field] <= p
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (meta[3 * (int64_t)mid + field] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_huge_clear(int32_t *tk, uint32_t *tv, const Status *st) {
  if (st->err || !st->huge_fallback) return;  // fallback only
  const int64_t slots = st->huge_slots;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < slots; i += (int64_t)gridDim.x * kBlock) {
    tk[i] = -1;
    tv[i] = 0;
  }
}

// one chunk per block iteration: the first-iteration argmax of (w, -prio),
// at level 0 (mode 2) also validation and degree
__global__ __launch_bounds__(kBlock) void k_huge_chunks(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ w, int32_t n,
                                                        const int32_t *list, const int32_t *cnt_p,
                                                        const int32_t *meta, unsigned long long *part,
                                                        unsigned long long *best, long long *deg, uint32_t salt,
                                                        int mode, Status *st, const int32_t *__restrict__ gv,
                                                        GStat *gs) {
  __shared__ unsigned long long sh[kBlock / 64];
  const bool stats = mode == 2 && !gv;  // the workgroup's weight sum and errors go to part
  if (!gv && st->err) {
    if (stats && threadIdx.x == 0) part_write(part, ~0ull, 0, 0);
    return;
  }
  const int32_t cnt = *cnt_p;
  const int32_t items = st->huge_items;
  unsigned long long wsum = 0;
  int werr = 0;
  for (int32_t p = blockIdx.x; p < items; p += gridDim.x) {
    int32_t i = huge_find(meta, cnt, p, 0);
    int32_t v = list[i];
    int32_t beg = rp[v] + (p - meta[3 * (int64_t)i]) * kHugeChunk;
    int32_t end = min(rp[v + 1], beg + kHugeChunk);
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    unsigned long long b = 0, sum = 0;
    int err = 0;
    for (int32_t a0 = beg + threadIdx.x; a0 < end; a0 += kBlock * kLoadBatch) {
      int32_t xs[kLoadBatch], cs[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {
        const int32_t a = min(a0 + u * kBlock, end - 1);
        xs[u] = col[a];
        cs[u] = w[a];
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {
        if (a0 + u * kBlock >= end) break;
        const int32_t x = xs[u], c = cs[u];
        if (mode == 2) {
          if (x < 0 || x >= n) err |= ERR_COL;
          if (x == v) err |= ERR_SELF;
          if (c < 1) err |= ERR_WEIGHT;
        }
        sum += (unsigned long long)(uint32_t)c;
        b = umax64(b, cand_key((uint32_t)c, x - b0, sl));
      }
    }
    b = block_max(b, sh);
    sum = block_sum(sum, sh);
    err = (int)block_max((unsigned long long)err, sh);
    if (threadIdx.x == 0) {
      atomicMax(&best[i], b);
      if (mode == 2) {
        atomicAdd((unsigned long long *)&deg[v], sum);
        if (gv) {
          if (err) atomicOr(&gs[gv[v]].err, err);
        } else {
          wsum += sum;
          werr |= err;
        }
      }
    }
  }
  if (stats && threadIdx.x == 0) part_write(part, ~0ull, wsum, werr);
}

// Table insertion for LP iterations t >= 2 on huge rows, one chunk of
// kHugeChunk arcs per block iteration: the chunk's (label, weight) pairs are
// first summed in an LDS table, then each distinct label of the chunk makes
// one insertion into the row's global table (neighbour labels of a huge row
// repeat a lot, so this removes most global atomics).
constexpr int kHugeLocal = 2 * kHugeChunk;  // LDS slots: load <= 1/2
__global__ __launch_bounds__(kBlock) void k_huge_insert(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ w, const int32_t *list,
                                                        const int32_t *cnt_p, const int32_t *meta,
                                                        const int32_t *__restrict__ Lin, int32_t *tk, uint32_t *tv,
                                                        unsigned long long *best, uint32_t salt, const Status *st,
                                                        const int32_t *__restrict__ gv, const GStat *gs) {
  __shared__ int32_t lk[kHugeLocal];
  __shared__ uint32_t lv[kHugeLocal];
  __shared__ unsigned long long red[kBlock / 64];
  if ((!gv && st->err) || !st->huge_fallback) return;  // fallback only
  const int32_t cnt = *cnt_p;
  const int32_t items = st->huge_items;
  constexpr uint32_t lmask = kHugeLocal - 1;
  for (int32_t p = blockIdx.x; p < items; p += gridDim.x) {
    const int32_t i = huge_find(meta, cnt, p, 0);
    const int32_t v = list[i];
    const int32_t beg = rp[v] + (p - meta[3 * (int64_t)i]) * kHugeChunk;
    const int32_t end = min(rp[v + 1], beg + kHugeChunk);
    for (int e = threadIdx.x; e < kHugeLocal; e += kBlock) {
      lk[e] = -1;
      lv[e] = 0;
    }
    __syncthreads();
    for (int32_t a0 = beg + threadIdx.x; a0 < end; a0 += kBlock * kLoadBatch) {
      int32_t xs[kLoadBatch], cs[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {
        const int32_t a = min(a0 + u * kBlock, end - 1);
        xs[u] = col[a];
        cs[u] = w[a];
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) xs[u] = Lin[xs[u]];
#pragma unroll
      for (int u = 0; u < kLoadBatch; u++) {
        if (a0 + u * kBlock >= end) break;
        const int32_t x = xs[u];
        uint32_t h = slot_hash(x) & lmask;
        while (true) {
          const int32_t old = atomicCAS(&lk[h], -1, x);
          if (old == -1 || old == x) break;
          h = (h + 1) & lmask;
        }
        atomicAdd(&lv[h], (uint32_t)cs[u]);
      }
    }
    __syncthreads();
    int32_t *K = tk + meta[3 * (int64_t)i + 1];
    uint32_t *V = tv + meta[3 * (int64_t)i + 1];
    const uint32_t mask = (uint32_t)meta[3 * (int64_t)i + 2] - 1;
    const int32_t own = Lin[v];
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    // one insertion per distinct label; a thread's first probes are all in
    // flight before any of their results is looked at. The returned partial
    // sum plus the chunk's sum bounds the label's final sum from below and the
    // row's last update of the label sees it: the row's best key is the
    // maximum over these updates (no pass over the table).
    constexpr int kPer = kHugeLocal / kBlock;
    int32_t xs[kPer], old[kPer];
    uint32_t hs[kPer], add[kPer];
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      xs[u] = lk[u * kBlock + threadIdx.x];
      add[u] = lv[u * kBlock + threadIdx.x];
      hs[u] = slot_hash(xs[u]) & mask;
    }
#pragma unroll
    for (int u = 0; u < kPer; u++) old[u] = xs[u] >= 0 ? atomicCAS(&K[hs[u]], -1, xs[u]) : -1;
#pragma unroll
    for (int u = 0; u < kPer; u++) {
      if (xs[u] < 0) continue;
      while (old[u] != -1 && old[u] != xs[u]) {  // taken by another label: probe on
        hs[u] = (hs[u] + 1) & mask;
        old[u] = atomicCAS(&K[hs[u]], -1, xs[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; u++) old[u] = xs[u] >= 0 ? (int32_t)atomicAdd(&V[hs[u]], add[u]) : 0;
    unsigned long long key = 0;
#pragma unroll
    for (int u = 0; u < kPer; u++)
      if (xs[u] >= 0) key = umax64(key, own_key((uint32_t)old[u] + add[u], xs[u] == own, xs[u] - b0, sl));
    key = block_max(key, red);
    if (threadIdx.x == 0 && key) atomicMax(&best[i], key);
    __syncthreads();
  }
}

// LP iterations t >= 2 on huge rows without a global table: the labels of
// row i are split into P_i parts by a hash (as planned by k_huge_plan modes 2
// and 3), and one work item (row, part) sums the weights of its part's labels
// in an LDS table of kPartSlots slots, so every label's whole sum is in one
// table. Each item reads the whole row (neighbour and its
// label, 8 arcs per thread in flight) and loads the weight only for the arcs
// of its part. The returned
// partial sum plus the weight bounds the label's final sum from below and
// the last update sees it, so the item's best key (S, own, -prio) is the
// maximum over its updates; one atomicMax per wave merges the items of a
// row. Items are taken by ticket. Pass 1 plans room for a quarter of the
// arcs as distinct labels; a probe run longer than kPartProbe flags the row
// and sets huge_overflow, and pass 2 redoes the flagged rows with room for
// every arc. A table that fills up in pass 2 sets huge_fallback, and the
// global-table kernels (which otherwise exit at once) redo the whole bin.
constexpr int kPartThreads = 1024;
constexpr int kPartBatch = 8;
__device__ __forceinline__ uint32_t part_of(int32_t x, uint32_t parts) {
  uint32_t h = ((uint32_t)x ^ 0x5BD1E995u) * 0x2C1B3C6Du;
  h ^= h >> 15;
  return __umulhi(h, parts);
}
__global__ __launch_bounds__(kPartThreads) void k_huge_part(const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ col,
                                                            const int32_t *__restrict__ w, const int32_t *list,
                                                            const int32_t *cnt_p, const int32_t *meta,
                                                            const int32_t *__restrict__ Lin,
                                                            unsigned long long *best, uint32_t salt, Status *st,
                                                            const int32_t *__restrict__ gv, const GStat *gs,
                                                            int32_t *row_flag, int pass) {
  extern __shared__ uint32_t part_lds[];
  int32_t *tk = reinterpret_cast<int32_t *>(part_lds);
  uint32_t *tv = part_lds + kPartSlots;
  __shared__ int32_t s_item;
  if (!gv && st->err) return;
  if (pass == 2 && !st->huge_overflow) return;
  const int32_t max_probe = pass == 1 ? kPartProbe : kPartSlots;
  const int32_t cnt = *cnt_p;
  const int32_t items = st->huge_items;
  constexpr uint32_t mask = kPartSlots - 1;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(&st->huge_ticket, 1);
    __syncthreads();
    const int32_t p = s_item;
    if (p >= items) break;
    const int32_t i = huge_find(meta, cnt, p, 0);
    const int32_t v = list[i];
    const uint32_t parts = (uint32_t)meta[3 * (int64_t)i + 1];
    const uint32_t mine = (uint32_t)(p - meta[3 * (int64_t)i]);
    const int32_t beg = rp[v], end = rp[v + 1];
    const int32_t own = Lin[v];
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    for (int e = threadIdx.x; e < kPartSlots; e += kPartThreads) {
      tk[e] = -1;
      tv[e] = 0;
    }
    __syncthreads();
    unsigned long long key = 0;
    bool full = false;
    for (int32_t a0 = beg + threadIdx.x; a0 < end; a0 += kPartThreads * kPartBatch) {
      int32_t xs[kPartBatch], cs[kPartBatch], h[kPartBatch], old[kPartBatch];
      bool m[kPartBatch];
#pragma unroll
      for (int u = 0; u < kPartBatch; u++) xs[u] = col[min(a0 + u * kPartThreads, end - 1)];
#pragma unroll
      for (int u = 0; u < kPartBatch; u++) xs[u] = Lin[xs[u]];
#pragma unroll
      for (int u = 0; u < kPartBatch; u++) {
        m[u] = a0 + u * kPartThreads < end && (parts == 1 || part_of(xs[u], parts) == mine);
        cs[u] = m[u] ? w[a0 + u * kPartThreads] : 0;
      }
#pragma unroll
      for (int u = 0; u < kPartBatch; u++) {
        h[u] = (int32_t)((mul24_golden((uint32_t)xs[u] ^ ((uint32_t)xs[u] >> 16)) >> 8) & mask);
        old[u] = m[u] ? atomicCAS(&tk[h[u]], -1, xs[u]) : -1;
      }
#pragma unroll
      for (int u = 0; u < kPartBatch; u++) {
        if (!m[u]) continue;
        int32_t probes = 0;
        while (old[u] != -1 && old[u] != xs[u]) {  // taken by another label: probe on
          if (++probes >= max_probe) {             // too full for this row's parts
            full = true;
            m[u] = false;
            break;
          }
          h[u] = (h[u] + 1) & (int32_t)mask;
          old[u] = atomicCAS(&tk[h[u]], -1, xs[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < kPartBatch; u++)
        if (m[u]) {
          const uint32_t S = atomicAdd(&tv[h[u]], (uint32_t)cs[u]) + (uint32_t)cs[u];
          key = umax64(key, own_key(S, xs[u] == own, xs[u] - b0, sl));
        }
    }
    if (full) {
      if (pass == 1) {
        row_flag[3 * (int64_t)i + 2] = 1;
        st->huge_overflow = 1;
      } else {
        st->huge_fallback = 1;
      }
    }
    key = grp_max<64>(key);
    if ((threadIdx.x & 63) == 0 && key) atomicMax(&best[i], key);
    __syncthreads();
  }
}

// final decision per huge vertex
__global__ void k_huge_final(const int32_t *rp, const int32_t *list, const int32_t *cnt_p, const int32_t *meta,
                             const unsigned long long *best, const int32_t *Lin, int32_t *Lout, long long *deg,
                             uint32_t salt, int mode, Status *st, const int32_t *__restrict__ gv,
                             const GStat *gs) {
  if (!gv && st->err) return;
  const int32_t cnt = *cnt_p;
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < cnt; i += gridDim.x * kBlock) {
    int32_t v = list[i];
    unsigned long long b = best[i];
    int32_t b0 = 0;
    uint32_t sl = salt;
    if (gv) {
      const GStat &g = gs[gv[v]];
      b0 = g.base;
      sl = g.salt;
    }
    if (mode == 1) {
      // the best key (S, own, -prio) of k_huge_insert: its own bit is set
      // exactly when the own label attains the maximum sum
      Lout[v] = ((b >> 32) & 1) ? Lin[v] : key_label(b, sl) + b0;
    } else {
      Lout[v] = key_label(b, sl) + b0;
      if (mode == 2 && !gv) {
        unsigned long long s = (unsigned long long)deg[v];
        unsigned long long s32 = s > 0xFFFFFFFFull ? 0xFFFFFFFFull : s;
        atomicMin(&st->minkey, (s32 << 32) | (uint32_t)v);
      }
    }
  }
}


// ------------------------------------------------------------ validation (flag)
// every arc (v,u,c) has its reverse (u,v,c); rows strictly increasing
__global__ void k_validate_sym(const int32_t *rp, const int32_t *col, const int32_t *w, int32_t n, Status *st,
                               const int32_t *gv, GStat *gs) {
  if (!gv && st->err) return;
  int bad = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    if (gv) {  // batched: only graphs still at level 0 are checked, each into its own flags
      GStat &g = gs[gv[v]];
      if (g.state != GS_FRESH) continue;
      int e = 0;
      for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
        int32_t u = col[i];
        if (i > rp[v] && col[i - 1] >= u) e |= ERR_UNSORTED;
        int32_t lo = rp[u], hi = rp[u + 1];
        while (lo < hi) {
          int32_t mid = (lo + hi) >> 1;
          if (col[mid] < v) lo = mid + 1; else hi = mid;
        }
        if (lo >= rp[u + 1] || col[lo] != v || w[lo] != w[i]) e |= ERR_NOTSYM;
      }
      if (e) atomicOr(&g.err, e);
      continue;
    }
    for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
      int32_t u = col[i];
      if (i > rp[v] && col[i - 1] >= u) bad |= ERR_UNSORTED;
      int32_t lo = rp[u], hi = rp[u + 1];
      while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (lo >= rp[u + 1] || col[lo] != v || w[lo] != w[i]) bad |= ERR_NOTSYM;
    }
  }
  if (bad) atomicOr(&st->err, bad);
}

// ------------------------------------------------------------ scan
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

// exclusive scan of one value per thread across the block; returns the block total
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t &total, int32_t *sh) {
  int32_t inc = wave_incl_scan(x);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  int32_t off = 0;
  total = 0;
  for (int i = 0; i < kBlock / 64; i++) {
    if (i < wid) off += sh[i];
    total += sh[i];
  }
  __syncthreads();
  return off + inc - x;
}

// ---- single-pass scan with decoupled look-back (Merrill & Garland 2016)
// Workgroups take tiles in ticket order, so every predecessor of a tile has
// started. A tile publishes its aggregate, then wave 0 reads the state words
// of up to 64 predecessors at once, newest first, and adds them up to the
// first one holding an inclusive prefix. Each state word packs (epoch, flag,
// value) into one 64-bit atomic, so a value is never seen without its flag,
// and words of earlier launches (older epochs) read as "not ready": the array
// is cleared once, not per launch. The wait is bounded by the wall clock: on
// expiry the status gets ERR_DEVICE and missing aggregates count as 0, which
// keeps every offset at or below its true value (in bounds for consumers).
constexpr uint32_t kLbAgg = 1, kLbInc = 2;
constexpr uint64_t kLbWaitTicks = 1ull << 26;  // ~0.67 s of the 100 MHz wall clock

__device__ __forceinline__ unsigned long long lb_word(uint32_t epoch, uint32_t flag, uint32_t v) {
  return ((unsigned long long)((epoch << 2) | flag) << 32) | v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// wave-uniform; call from one whole wave. Returns the sum of the values of
// tiles [0, t) published under `epoch`.
__device__ unsigned long long lb_lookback(const unsigned long long *state, int64_t t, uint32_t epoch, Status *st) {
  const int lane = threadIdx.x & 63;
  unsigned long long excl = 0;
  int64_t j = t - 1;  // newest predecessor not yet accounted for
  const uint64_t t0 = wall_clock64();
  while (j >= 0) {
    const int64_t idx = j - lane;
    unsigned long long wd, need, ib;
    bool ready;
    while (true) {
      wd = idx >= 0 ? __hip_atomic_load(&state[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : lb_word(epoch, kLbInc, 0u);
      const uint32_t hi = (uint32_t)(wd >> 32);
      ready = (hi >> 2) == epoch && (hi & 3u) != 0;
      ib = __ballot(ready && (hi & 3u) == kLbInc);
      const unsigned long long nr = __ballot(!ready);
      need = ib ? (((ib & (~ib + 1)) << 1) - 1) : ~0ull;  // lanes up to the first inclusive one
      if ((nr & need) == 0) break;
      if (wall_clock64() - t0 > kLbWaitTicks) {
        if (lane == 0) atomicOr(&st->err, ERR_DEVICE);
        ib = ~0ull;  // stop after this window
        break;
      }
    }
    const bool take = ((need >> lane) & 1ull) && ready;
    excl += wave_sum_u64(take ? (unsigned long long)(uint32_t)wd : 0ull);
    if (ib) break;
    j -= 64;
  }
  return excl;
}

__device__ __forceinline__ int lb_pad(int e) { return e + (e >> 5); }

// ITEMS elements per thread; all global loads are issued before any is used
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_scan_lb(const int32_t *in, int32_t *out, int64_t count, int32_t *total,
                                                     unsigned long long *state, uint32_t *ticket, uint32_t epoch,
                                                     int32_t ntiles, Status *st) {
  constexpr int TILE = kBlock * ITEMS;
  __shared__ int32_t tile[TILE + TILE / 32];  // one pad word per 32: conflict-free rows
  __shared__ int32_t sh[kBlock / 64];
  __shared__ int32_t s_t, s_excl;
  if (threadIdx.x == 0) {
    const int32_t t = (int32_t)atomicAdd(ticket, 1u);
    if (t == ntiles - 1) atomicExch(ticket, 0u);  // the last ticket of the launch: rearm
    s_t = t;
  }
  __syncthreads();
  const int32_t t = s_t;
  const int64_t base = t * (int64_t)TILE;
  int32_t v[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; j++) {
    const int64_t i = base + j * kBlock + threadIdx.x;
    v[j] = in[i < count ? i : count - 1];
  }
#pragma unroll
  for (int j = 0; j < ITEMS; j++) {
    const int64_t i = base + j * kBlock + threadIdx.x;
    tile[lb_pad(j * kBlock + threadIdx.x)] = i < count ? v[j] : 0;
  }
  __syncthreads();
  int32_t acc = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; j++) {
    v[j] = acc;
    acc += tile[lb_pad(threadIdx.x * ITEMS + j)];
  }
  int32_t tot;
  const int32_t off = block_excl_scan(acc, tot, sh);
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0)
      __hip_atomic_store(&state[t], lb_word(epoch, t == 0 ? kLbInc : kLbAgg, (uint32_t)tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long ex = t > 0 ? lb_lookback(state, t, epoch, st) : 0ull;
    if (threadIdx.x == 0) {
      if (t > 0)
        __hip_atomic_store(&state[t], lb_word(epoch, kLbInc, (uint32_t)(ex + (uint32_t)tot)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      s_excl = (int32_t)ex;
    }
  }
  __syncthreads();
  const int32_t add = s_excl;
#pragma unroll
  for (int j = 0; j < ITEMS; j++) tile[lb_pad(threadIdx.x * ITEMS + j)] = add + off + v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; j++) {
    const int64_t i = base + j * kBlock + threadIdx.x;
    if (i < count) out[i] = tile[lb_pad(j * kBlock + threadIdx.x)];
  }
  if (total && threadIdx.x == 0 && t == ntiles - 1) *total = add + tot;
}

__global__ void k_lb_clear(unsigned long long *state, int64_t words, uint32_t *ticket) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlock)
    state[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;
}

// one tile (count <= kScanTile), one workgroup; in-place capable
__global__ void k_scan_tile(const int32_t *in, int32_t *out, int64_t count, int32_t *total) {
  __shared__ int32_t tile[kScanTile + kScanTile / 32];
  __shared__ int32_t sh[kBlock / 64];
  int32_t v[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    const int64_t i = j * kBlock + threadIdx.x;
    v[j] = in[i < count ? i : count - 1];
  }
#pragma unroll
  for (int j = 0; j < kScanItems; j++)
    tile[lb_pad(j * kBlock + threadIdx.x)] = j * kBlock + threadIdx.x < count ? v[j] : 0;
  __syncthreads();
  int32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = acc;
    acc += tile[lb_pad(threadIdx.x * kScanItems + j)];
  }
  int32_t tot;
  const int32_t off = block_excl_scan(acc, tot, sh);
#pragma unroll
  for (int j = 0; j < kScanItems; j++) tile[lb_pad(threadIdx.x * kScanItems + j)] = off + v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    const int64_t i = j * kBlock + threadIdx.x;
    if (i < count) out[i] = tile[lb_pad(j * kBlock + threadIdx.x)];
  }
  if (total && threadIdx.x == 0) *total = tot;
}

// ------------------------------------------------------------ relabel / map
// Batched: vertices of graphs that left the round loop are dropped here
// (cl = -1); their rows then emit nothing, as both ends of each of their
// arcs map to -1.
__global__ void k_flag_labels(const int32_t *L, int32_t n, int32_t *flags, const int32_t *gv, const GStat *gs) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    if (!gv || gs[gv[v]].state == GS_ACTIVE) flags[L[v]] = 1;
}
__global__ void k_apply_ids(const int32_t *L, const int32_t *ids, int32_t n, int32_t *cl, const int32_t *gv,
                            const GStat *gs, int32_t *gv_new) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    if (!gv) {
      cl[v] = ids[L[v]];
      continue;
    }
    const int32_t g = gv[v];
    if (gs[g].state == GS_ACTIVE) {
      const int32_t c = ids[L[v]];
      cl[v] = c;
      gv_new[c] = g;  // every member of a cluster writes the same graph index
    } else {
      cl[v] = -1;
    }
  }
}
// ------------------------------------------------------------ correcting step
// Section 4.1's correcting algorithm (fixMisplacedVertices of Algorithm 1):
// a vertex of a cluster C with 2 <= |C| <= floor(log2 n) is misplaced if its
// removal lowers the minimum weighted degree of the contracted graph; per
// cluster at most one, the one leaving C - {v} the smallest degree (smallest
// v on ties). With out(v) the weight from v to other clusters and c(v) its
// degree, C - {v} has degree cut(C) - out(v) + (c(v) - out(v)).
__global__ void k_fix_clear(int32_t *cnt, unsigned long long *cut, unsigned long long *key, int32_t n, Status *st) {
  for (int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock) {
    cnt[x] = 0;
    cut[x] = 0;
    key[x] = ~0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->fix_delta = ~0ull;
}
// one wave per row: out(v), the member count and the cluster's degree
__global__ void k_fix_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ w, const int32_t *__restrict__ L, int32_t n, int32_t *cnt,
                           uint32_t *out, unsigned long long *cut) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t v = wave; v < n; v += nw) {
    const int32_t lv = L[v];
    const int32_t beg = rp[v], end = rp[v + 1];
    unsigned long long o = 0;
    for (int32_t i = beg + lane; i < end; i += 64)
      if (L[col[i]] != lv) o += (uint32_t)w[i];
    o = grp_sum<64>(o);
    if (lane == 0) {
      out[v] = (uint32_t)o;  // <= the total weight <= INT32_MAX
      atomicAdd(&cnt[lv], 1);
      if (o) atomicAdd(&cut[lv], o);
    }
  }
}
// minimum weighted degree of the contracted graph (every cluster)
__global__ void k_fix_delta(const int32_t *cnt, const unsigned long long *cut, int32_t n, Status *st) {
  unsigned long long m = ~0ull;
  for (int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock)
    if (cnt[x] > 0) m = umin64(m, cut[x]);
  m = grp_min<64>(m);
  if ((threadIdx.x & 63) == 0 && m != ~0ull) atomicMin(&st->fix_delta, m);
}
// candidate removals: (degree of C - {v}) << 32 | v, minimum per cluster
__global__ void k_fix_cand(const int32_t *__restrict__ L, const long long *__restrict__ deg, const int32_t *cnt,
                           const unsigned long long *cut, const uint32_t *out, int32_t n, int32_t limit,
                           const Status *st, unsigned long long *key) {
  const unsigned long long delta = st->fix_delta;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int32_t lv = L[v];
    const int32_t c = cnt[lv];
    if (c < 2 || c > limit) continue;
    const unsigned long long rest = cut[lv] + (unsigned long long)deg[v] - 2ull * out[v];
    if (rest < delta) atomicMin(&key[lv], (rest << 32) | (uint32_t)v);
  }
}
// the chosen vertex of each cluster becomes a singleton with label n + v
__global__ void k_fix_apply(int32_t *L, const unsigned long long *key, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const unsigned long long k = key[L[v]];
    if (k != ~0ull && (int32_t)(uint32_t)k == (int32_t)v) L[v] = n + (int32_t)v;
  }
}

// single solve: cl[v] = ids[L[v]] and, in the same pass, map[u] <- ids[L[map[u]]]
// (the composed map reads the ids directly, so it need not wait for cl)
__global__ void k_apply_compose(const int32_t *L, const int32_t *ids, int32_t n, int32_t *cl, int32_t *map,
                                int32_t n_in) {
  const int64_t m = n > n_in ? n : n_in;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < m; v += (int64_t)gridDim.x * kBlock) {
    if (v < n) cl[v] = ids[L[v]];
    if (v < n_in) map[v] = ids[L[map[v]]];
  }
}
// map[u] <- cl[map[u]]. Batched: u runs over the padded input index space
// (64 entries per word, word -> slot in wg; padding entries hold -1), and
// graphs out of the loop keep the map of their last level.
__global__ void k_compose(int32_t *map, const int32_t *cl, int32_t n_in, const int32_t *wg, const GStat *gs) {
  for (int64_t u = blockIdx.x * (int64_t)kBlock + threadIdx.x; u < n_in; u += (int64_t)gridDim.x * kBlock) {
    if (wg) {
      const int32_t slot = wg[u >> 6];
      const int32_t m = map[u];
      if (slot < 0 || m < 0 || gs[slot].state != GS_ACTIVE) continue;
      map[u] = cl[m];
    } else {
      map[u] = cl[map[u]];
    }
  }
}
__global__ void k_iota(int32_t *p, int32_t n) {
  for (int64_t u = blockIdx.x * (int64_t)kBlock + threadIdx.x; u < n; u += (int64_t)gridDim.x * kBlock)
    p[u] = (int32_t)u;
}

// ------------------------------------------------------------ contraction
// Inter-cluster arcs, written compacted (in arc order) into the source
// segment's own arc range of the triple buffer: segment s = tile s, or long
// row (class 4 to 6) after the tiles: first[s] = its first arc, cnt[s] = the
// pairs written. A scan over the counts and k_compact then pack the segments.
__device__ __forceinline__ void emit_chunk(const int32_t *xs, const int32_t *cus, const int32_t *cs, int q,
                                           int32_t i0, int32_t acnt, const int32_t *s_rp, int32_t rows,
                                           const int32_t *s_cl, int32_t cl_row, int32_t cl_base, int key_bits,
                                           int64_t out0, unsigned long long *keys, int32_t *vals, int32_t *sh,
                                           int32_t &total) {
  unsigned long long k[kPerThread];
  uint32_t fl = 0;
  if (i0 < acnt) {
    int32_t j = s_rp ? row_of(s_rp, rows, i0) : 0;
#pragma unroll
    for (int m = 0; m < kPerThread; m++) {
      const int32_t i = i0 + m;
      k[m] = 0;
      if (m < q && i < acnt) {
        if (s_rp)
          while (i >= s_rp[j + 1]) j++;
        const int32_t cv = s_rp ? s_cl[j] : cl_row;
        if (cus[m] != cv) {
          k[m] = ((unsigned long long)(uint32_t)cv << key_bits) | (uint32_t)(cus[m] - cl_base);
          fl |= 1u << m;
        }
      }
    }
  }
  const int32_t off = block_excl_scan(__popc(fl), total, sh);
#pragma unroll
  for (int m = 0; m < kPerThread; m++)
    if (fl & (1u << m)) {
      const int64_t o = out0 + off + __popc(fl & ((1u << m) - 1));
      keys[o] = k[m];
      vals[o] = cs[m];
    }
  (void)xs;
}

// Tile emission with a combiner: the tile's inter-cluster arcs are summed per
// (cl(u), cl(v)) pair in an LDS hash table, and only the distinct pairs are
// written (the sort and the final segmented sum do not depend on how a
// pair's weight is split). Thread l takes q consecutive arcs as in the LP
// tile kernel: clamped loads, so loads and cluster gathers are in flight
// together; rows from the prefix maximum of row-start marks; runs of equal
// pairs folded in registers; all claims issued before any result is used.
// The occupied slots are then written in slot order, 64 at a time.
// Emission keys: (cluster of the row) << lo | low, where low is the
// neighbour's cluster minus the first cluster of the row's graph in a batch
// union (its clusters are contiguous and both ends lie in one graph, so lo =
// bits of the largest graph's cluster count), or the neighbour's cluster
// itself in a single solve (lo = bits of the cluster count).
__device__ __forceinline__ int emit_lo_bits(const Status *st, const int32_t *gv) {
  return bits_for(gv ? st->kloc : st->k);
}

constexpr int kCombSlots = kTileArcs;  // > arcs of a tile, so probing ends
constexpr unsigned long long kNoPair = ~0ull;
template <bool B>
struct alignas(16) EmitTileShared {
  int32_t rcl[kTile];                  // cluster of each row
  int32_t rbase[B ? kTile : 1];        // (batched) first cluster of the row's graph
  unsigned long long tkey[kCombSlots];
  uint32_t tval[kCombSlots];
  unsigned long long mark[kTB];        // row-start marks, NQ bytes per lane
};

// Registers of one emission tile: lane l's arcs [NQ l, NQ l + NQ) (their
// neighbours' clusters) and the rows' first arcs and clusters, one entry per
// 64 rows (only entries below the row count are loaded). Weights are loaded
// later, for the arcs between clusters only (about 30 % of the arcs of the
// random hyperbolic graph after two LP iterations).
template <bool B, int NQ>
struct EmitFetch {
  int4 m;
  int32_t cus[NQ];
  int32_t rpv[kRowRegs + 1];
  int32_t clv[kRowRegs];
  int32_t basev[B ? kRowRegs : 1];
};

template <bool B, int NQ>
__device__ __forceinline__ void emit_fetch_loads(EmitFetch<B, NQ> &f, int4 m, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const int32_t *__restrict__ w,
                                                 const int32_t *__restrict__ cl, const int32_t *__restrict__ gv,
                                                 const GStat *gs) {
  const int lane = threadIdx.x;
  f.m = m;
  const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
#pragma unroll
  for (int k = 0; k < NQ; k++) f.cus[k] = 0;
  if (acnt > 0) {
#pragma unroll
    for (int k = 0; k < NQ; k++) f.cus[k] = at32(col + a0, (uint32_t)min(NQ * lane + k, acnt - 1));
  }
#pragma unroll
  for (int r = 0; r <= kRowRegs; r++) {
    f.rpv[r] = 0;
    if (r == 0 || kTB * r <= rows) f.rpv[r] = at32(rp + r0, (uint32_t)min(lane + kTB * r, rows));
  }
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    f.clv[r] = 0;
    if constexpr (B) f.basev[r] = 0;
    if (rows > 0 && (r == 0 || kTB * r < rows)) {
      const uint32_t j = (uint32_t)min(lane + kTB * r, rows - 1);
      f.clv[r] = at32(cl + r0, j);
      if constexpr (B) f.basev[r] = gs[at32(gv + r0, j)].base;
    }
  }
}
template <bool B, int NQ>
__device__ __forceinline__ void emit_fetch_gather(EmitFetch<B, NQ> &f, const int32_t *__restrict__ cl) {
  if (f.m.w > 0) {
#pragma unroll
    for (int k = 0; k < NQ; k++) f.cus[k] = at32(cl, (uint32_t)f.cus[k]);
  }
}

// Emission of one tile: its arcs between different clusters become (cluster
// of the row, cluster of the neighbour) pairs, summed per distinct pair in
// an LDS table sized for the tile's inter-cluster arcs (twice their count,
// a power of two), and written in slot order into the tile's arc range.
// Tiles with no such arc write an empty segment and skip the table.
template <bool B, int NQ>
__device__ __forceinline__ void emit_tile_run(const EmitFetch<B, NQ> &f, const int32_t *__restrict__ w, int32_t t,
                                              int key_bits, unsigned long long *__restrict__ keys,
                                              int32_t *__restrict__ vals, int32_t *__restrict__ first,
                                              int32_t *__restrict__ cnt, EmitTileShared<B> &sh) {
  using MW = typename MarkWord<NQ>::T;
  const int lane = threadIdx.x;
  const int32_t rows = f.m.y, a0 = f.m.z, acnt = f.m.w;
  MW *mark = reinterpret_cast<MW *>(sh.mark);
  uint8_t *s_mark = reinterpret_cast<uint8_t *>(sh.mark);
  mark[lane] = 0;
#pragma unroll
  for (int r = 0; r < kRowRegs; r++) {
    if (r > 0 && kTB * r >= rows) break;
    const int j = lane + kTB * r;
    const int32_t nxt = __builtin_amdgcn_readlane(f.rpv[r + 1], 0);
    const int32_t hi = __builtin_amdgcn_update_dpp(nxt, f.rpv[r], 0x130, 0xF, 0xF, false);  // wave_shl:1
    if (j < rows) {
      sh.rcl[j] = f.clv[r];
      if constexpr (B) sh.rbase[j] = f.basev[r];
      if (hi > f.rpv[r]) s_mark[f.rpv[r] - a0] = (uint8_t)j;
    }
  }
  __syncthreads();
  int32_t rw[NQ];
  lane_rows<NQ>(mark[lane], rw);
  bool ok[NQ];
  uint32_t cc[NQ];
  unsigned long long key[NQ];
#pragma unroll
  for (int k = 0; k < NQ; k++) {
    const int32_t cv = sh.rcl[rw[k]];
    int32_t cb = 0;
    if constexpr (B) cb = sh.rbase[rw[k]];
    ok[k] = NQ * lane + k < acnt && f.cus[k] != cv;
    key[k] = ((unsigned long long)(uint32_t)cv << key_bits) | (uint32_t)(f.cus[k] - cb);
  }
#pragma unroll
  for (int k = 0; k < NQ; k++) cc[k] = ok[k] ? (uint32_t)at32(w + a0, (uint32_t)(NQ * lane + k)) : 0u;
  // fold runs of equal pairs into their first arc
#pragma unroll
  for (int k = NQ - 1; k > 0; k--)
    if (ok[k] && ok[k - 1] && key[k] == key[k - 1]) {
      cc[k - 1] += cc[k];
      ok[k] = false;
    }
  int32_t e = 0;
#pragma unroll
  for (int k = 0; k < NQ; k++) e += __popcll(__ballot(ok[k]));
  int32_t tot = 0;
  if (e > 0) {
    // table of T = pow2 >= 2e slots (64 .. kCombSlots)
    int32_t tb = 6;
    while ((1 << tb) < 2 * e && (1 << tb) < kCombSlots) tb++;
    const int32_t T = 1 << tb;
    const uint32_t msk = (uint32_t)T - 1;
    for (int i = lane; i < T; i += kTB) {
      sh.tkey[i] = kNoPair;
      sh.tval[i] = 0;
    }
    __syncthreads();
    uint32_t hh[NQ];
    unsigned long long old[NQ];
#pragma unroll
    for (int k = 0; k < NQ; k++) {
      const uint32_t fold = (uint32_t)key[k] ^ (uint32_t)(key[k] >> 32);
      hh[k] = (mul24_golden(fold ^ (fold >> 16)) >> 8) & msk;
      old[k] = ok[k] ? atomicCAS(&sh.tkey[hh[k]], kNoPair, key[k]) : kNoPair;
    }
    bool coll = false;
#pragma unroll
    for (int k = 0; k < NQ; k++) coll |= ok[k] && old[k] != kNoPair && old[k] != key[k];
    if (__ballot(coll)) {  // (rare: one wave-wide test skips the probing code)
#pragma unroll
      for (int k = 0; k < NQ; k++) {
        if (!ok[k]) continue;
        while (old[k] != kNoPair && old[k] != key[k]) {  // taken by another pair
          hh[k] = (hh[k] + 1) & msk;
          old[k] = atomicCAS(&sh.tkey[hh[k]], kNoPair, key[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NQ; k++)
      if (ok[k]) atomicAdd(&sh.tval[hh[k]], cc[k]);
    __syncthreads();
    // write the distinct pairs into the tile's region, in slot order
    for (int i0 = 0; i0 < T; i0 += kTB) {
      const int i = i0 + lane;
      const unsigned long long kk = sh.tkey[i];
      const uint32_t vv = sh.tval[i];
      const bool occ = kk != kNoPair;
      const unsigned long long bal = __ballot(occ);
      if (occ) {
        const int32_t pos = tot + __popcll(bal & ((1ull << lane) - 1));
        keys[(int64_t)a0 + pos] = kk;
        vals[(int64_t)a0 + pos] = (int32_t)vv;
      }
      tot += __popcll(bal);
    }
  }
  if (lane == 0) {
    first[t] = a0;
    cnt[t] = tot;
  }
  __syncthreads();
}

// Tiles of at most 256 arcs, TP consecutive tiles per workgroup (one wave):
// the loads and cluster gathers of all of them are issued before any is
// processed. Tiles of more than 256 arcs are left to k_emit_tile_big.
template <bool B, int TP>
__global__ __launch_bounds__(kTB) void k_emit_tile(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ w, const int32_t *__restrict__ cl,
                                                       const int4 *__restrict__ meta, int32_t ntiles,
                                                       const Status *st, unsigned long long *__restrict__ keys,
                                                       int32_t *__restrict__ vals, int32_t *__restrict__ first,
                                                       int32_t *__restrict__ cnt, const int32_t *__restrict__ gv,
                                                       const GStat *gs) {
  __shared__ EmitTileShared<B> sh;
  const int key_bits = emit_lo_bits(st, gv);
  const int32_t groups = (ntiles + TP - 1) / TP;
  for (int32_t g = blockIdx.x; g < groups; g += gridDim.x) {
    int4 m[TP];
    bool use[TP];
#pragma unroll
    for (int u = 0; u < TP; u++) {
      const int32_t t = g * TP + u;
      m[u] = t < ntiles ? meta[t] : make_int4(0, 0, 0, 0);
      use[u] = t < ntiles && m[u].w <= 4 * kTB;
      if (!use[u]) m[u] = make_int4(m[u].x, 0, 0, 0);
    }
    EmitFetch<B, 4> f[TP];
#pragma unroll
    for (int u = 0; u < TP; u++) emit_fetch_loads(f[u], m[u], rp, col, w, cl, gv, gs);
#pragma unroll
    for (int u = 0; u < TP; u++) emit_fetch_gather(f[u], cl);
#pragma unroll
    for (int u = 0; u < TP; u++)
      if (use[u]) emit_tile_run<B, 4>(f[u], w, g * TP + u, key_bits, keys, vals, first, cnt, sh);
  }
}

// The listed tiles of more than 256 arcs, 8 arcs per lane. Persistent (as
// many workgroups as fit, striding over the list), with the next tile's
// loads and gathers issued before this tile's LDS phases.
template <bool B>
__global__ __launch_bounds__(kTB) void k_emit_tile_big(const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ col,
                                                           const int32_t *__restrict__ w,
                                                           const int32_t *__restrict__ cl,
                                                           const int4 *__restrict__ meta,
                                                           const int32_t *__restrict__ big, const Status *st,
                                                           unsigned long long *__restrict__ keys,
                                                           int32_t *__restrict__ vals, int32_t *__restrict__ first,
                                                           int32_t *__restrict__ cnt, const int32_t *__restrict__ gv,
                                                           const GStat *gs) {
  __shared__ EmitTileShared<B> sh;
  const int key_bits = emit_lo_bits(st, gv);
  const int32_t nb = st->big_tiles;
  int32_t i = (int32_t)blockIdx.x;
  if (i >= nb) return;
  int32_t t = big[i];
  EmitFetch<B, kPerThread> cur;
  emit_fetch_loads(cur, meta[t], rp, col, w, cl, gv, gs);
  emit_fetch_gather(cur, cl);
  while (true) {
    const int32_t in = i + (int32_t)gridDim.x;
    const int32_t tn = in < nb ? big[in] : 0;
    EmitFetch<B, kPerThread> nxt;
    if (in < nb) {
      emit_fetch_loads(nxt, meta[tn], rp, col, w, cl, gv, gs);
      emit_fetch_gather(nxt, cl);
    }
    emit_tile_run<B, kPerThread>(cur, w, t, key_bits, keys, vals, first, cnt, sh);
    if (in >= nb) break;
    i = in;
    t = tn;
    cur = nxt;
  }
}

// Exclusive prefix sum over the 64 lanes of a wave; *total gets the sum.
__device__ __forceinline__ int32_t wave_excl_scan(int32_t x, int32_t &total) {
  const int lane = threadIdx.x & 63;
  int32_t v = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(v, d, 64);
    if (lane >= d) v += y;
  }
  total = __shfl(v, 63, 64);
  return v - x;
}

// rows of 256..1023 arcs: one wave per row, 8 arcs per lane per pass with
// consecutive lanes on consecutive arcs; the wave's inter-cluster arcs are
// appended in order with a wave prefix sum (no workgroup barriers)
__global__ __launch_bounds__(kBlock) void k_emit_wave(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ w, const int32_t *__restrict__ cl,
                                                       RowClasses rc, const Status *st,
                                                       unsigned long long *__restrict__ keys,
                                                       int32_t *__restrict__ vals, const int32_t *__restrict__ gv,
                                                       const GStat *gs) {
  constexpr int kPer = 8;
  const int cls = row_class(rc);
  const int32_t *list = rc.list[cls];
  int32_t *__restrict__ first = rc.seg[cls];
  int32_t *__restrict__ seg_cnt = rc.seg_cnt[cls];
  const int32_t bid = (int32_t)blockIdx.x - rc.first[cls], nblk = rc.first[cls + 1] - rc.first[cls];
  const int key_bits = emit_lo_bits(st, gv);
  const int32_t cnt = *rc.cnt[cls];
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = ((int64_t)nblk * kBlock) >> 6;
  for (int64_t r = (bid * (int64_t)kBlock + threadIdx.x) >> 6; r < cnt; r += nwaves) {
    const int32_t v0 = list[r];
    const int32_t cv = cl[v0];
    const int32_t cb = gv ? gs[gv[v0]].base : 0;
    const int32_t beg = rp[v0], end = rp[v0 + 1];
    int64_t out = beg;
    for (int32_t c0 = beg; c0 < end; c0 += 64 * kPer) {
      int32_t cus[kPer], cs[kPer];
#pragma unroll
      for (int k = 0; k < kPer; k++) {  // clamped loads, all issued before use
        const int32_t a = min(c0 + lane + 64 * k, end - 1);
        cus[k] = col[a];
        cs[k] = w[a];
      }
#pragma unroll
      for (int k = 0; k < kPer; k++) cus[k] = cl[cus[k]];
      uint32_t fl = 0;
#pragma unroll
      for (int k = 0; k < kPer; k++)
        if (c0 + lane + 64 * k < end && cus[k] != cv) fl |= 1u << k;
      int32_t tot;
      const int32_t off = wave_excl_scan(__popc(fl), tot);
      int32_t o = 0;
#pragma unroll
      for (int k = 0; k < kPer; k++)
        if (fl & (1u << k)) {
          keys[out + off + o] = ((unsigned long long)(uint32_t)cv << key_bits) | (uint32_t)(cus[k] - cb);
          vals[out + off + o] = cs[k];
          o++;
        }
      out += tot;
    }
    if (lane == 0) {
      first[r] = beg;
      seg_cnt[r] = (int32_t)(out - beg);
    }
  }
}

// long rows: one workgroup per row, chunks of kBlock * kPerThread arcs
__global__ __launch_bounds__(kBlock) void k_emit_long(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ w, const int32_t *__restrict__ cl,
                                                       const int32_t *list, const int32_t *cnt_p, const Status *st,
                                                       unsigned long long *__restrict__ keys,
                                                       int32_t *__restrict__ vals, int32_t *__restrict__ first,
                                                       int32_t *__restrict__ seg_cnt, const int32_t *__restrict__ gv,
                                                       const GStat *gs) {
  __shared__ int32_t sh[kBlock / 64];
  const int key_bits = emit_lo_bits(st, gv);
  const int32_t cnt = *cnt_p;
  for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
    const int32_t v0 = list[r];
    const int32_t cv = cl[v0];
    const int32_t cb = gv ? gs[gv[v0]].base : 0;
    const int32_t beg = rp[v0], end = rp[v0 + 1];
    int64_t out = beg;
    for (int32_t c0 = beg; c0 < end; c0 += kBlock * kPerThread) {
      const int32_t acnt = min(kBlock * kPerThread, end - c0);
      const int32_t i0 = threadIdx.x * kPerThread;
      int32_t cus[kPerThread], cs[kPerThread];
#pragma unroll
      for (int k = 0; k < kPerThread; k++) {  // clamped loads, all issued before use
        const int32_t a = c0 + min(i0 + k, acnt - 1);
        cus[k] = col[a];
        cs[k] = w[a];
      }
#pragma unroll
      for (int k = 0; k < kPerThread; k++) cus[k] = cl[cus[k]];
      int32_t tot;
      emit_chunk(cus, cus, cs, kPerThread, i0, acnt, nullptr, 0, nullptr, cv, cb, key_bits, out, keys, vals, sh, tot);
      out += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      first[r] = beg;
      seg_cnt[r] = (int32_t)(out - beg);
    }
  }
}

// huge rows (more than 4096 arcs): one workgroup per 4096-arc chunk (the
// chunk offsets of k_huge_plan), one segment per chunk, so that a hub row is
// spread over many workgroups instead of one
__global__ __launch_bounds__(kBlock) void k_emit_huge(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       const int32_t *__restrict__ w, const int32_t *__restrict__ cl,
                                                       const int32_t *list, const int32_t *cnt_p, const int32_t *meta,
                                                       const Status *st, unsigned long long *__restrict__ keys,
                                                       int32_t *__restrict__ vals, int32_t *__restrict__ first,
                                                       int32_t *__restrict__ seg_cnt, const int32_t *__restrict__ gv,
                                                       const GStat *gs) {
  __shared__ int32_t sh[kBlock / 64];
  const int key_bits = emit_lo_bits(st, gv);
  const int32_t cnt = *cnt_p;
  const int32_t items = st->huge_items;
  for (int32_t p = blockIdx.x; p < items; p += gridDim.x) {
    const int32_t i = huge_find(meta, cnt, p, 0);
    const int32_t v0 = list[i];
    const int32_t cv = cl[v0];
    const int32_t cb = gv ? gs[gv[v0]].base : 0;
    const int32_t beg = rp[v0] + (p - meta[3 * (int64_t)i]) * kHugeChunk;
    const int32_t end = min(rp[v0 + 1], beg + kHugeChunk);
    int64_t out = beg;
    for (int32_t c0 = beg; c0 < end; c0 += kBlock * kPerThread) {
      const int32_t acnt = min(kBlock * kPerThread, end - c0);
      const int32_t i0 = threadIdx.x * kPerThread;
      int32_t cus[kPerThread], cs[kPerThread];
#pragma unroll
      for (int k = 0; k < kPerThread; k++) {  // clamped loads, all issued before use
        const int32_t a = c0 + min(i0 + k, acnt - 1);
        cus[k] = col[a];
        cs[k] = w[a];
      }
#pragma unroll
      for (int k = 0; k < kPerThread; k++) cus[k] = cl[cus[k]];
      int32_t tot;
      emit_chunk(cus, cus, cs, kPerThread, i0, acnt, nullptr, 0, nullptr, cv, cb, key_bits, out, keys, vals, sh, tot);
      out += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      first[p] = beg;
      seg_cnt[p] = (int32_t)(out - beg);
    }
  }
}

// pack the segments into buffer 1: output element e comes from the last
// segment s with off[s] <= e (binary search of the exclusive offsets), so the
// work is balanced whatever the segment lengths
// A workgroup takes kCompactItems * 256 consecutive output elements. The
// first wave finds the segments of the range's first and last element, each
// half-wave by a 32-way search (a probe per lane, the ballot's count narrows
// the span 32-fold per step); the offsets in between are staged in LDS (at
// most kCompactWin of them) and every element searches only there. A wider
// span (long runs of empty segments) searches the global offsets between the
// two bounds.
constexpr int kCompactItems = 4;
constexpr int kCompactWin = 2048;

// Last segment s in [0, nseg) with off[s] <= t, by the 32 lanes of one half
// of wave 0 (off nondecreasing, off[0] = 0 <= t). Every lane of the wave calls
// it; the loop ends when both halves are done.
__device__ int32_t compact_bound(const int32_t *off, int32_t nseg, int64_t t) {
  const int half = threadIdx.x >> 5, k = threadIdx.x & 31;
  int32_t lo = 0, hi = nseg - 1;
  bool done = false;
  for (;;) {
    const int32_t stride = done ? 0 : (hi - lo + 32) >> 5;
    const int32_t p = lo + k * stride;
    const bool le = !done && p <= hi && off[p] <= t;
    const int c = __popc((uint32_t)(__ballot(le) >> (32 * half)));
    if (!done) {
      if (stride == 1) {
        lo += c - 1;
        done = true;
      } else {
        const int32_t nlo = lo + (c - 1) * stride;
        hi = min(hi, nlo + stride - 1);
        lo = nlo;
      }
    }
    if (__ballot(!done) == 0) break;
  }
  return lo;
}

// Few segments (their offsets stay in L2): every element searches all the
// offsets itself, with no barrier or dependent bound search in between.
__global__ void k_compact_direct(const int32_t *first, const int32_t *off, int32_t nseg, const Status *st,
                                 const unsigned long long *kin, const int32_t *vin, unsigned long long *kout,
                                 int32_t *vout) {
  const int64_t total = st->ax;
  for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int64_t src = first[lo] + (e - off[lo]);
    kout[e] = kin[src];
    vout[e] = vin[src];
  }
}

__global__ __launch_bounds__(kBlock) void k_compact(const int32_t *first, const int32_t *off, int32_t nseg,
                                                    const Status *st, const unsigned long long *kin,
                                                    const int32_t *vin, unsigned long long *kout, int32_t *vout) {
  __shared__ int32_t s_off[kCompactWin];
  __shared__ int32_t s_bound[2];
  constexpr int kSpan = kBlock * kCompactItems;
  const int64_t total = st->ax;
  for (int64_t e0 = blockIdx.x * (int64_t)kSpan; e0 < total; e0 += (int64_t)gridDim.x * kSpan) {
    if (threadIdx.x < 64) {
      const int64_t t = threadIdx.x < 32 ? e0 : min<int64_t>(e0 + kSpan, total) - 1;
      const int32_t b = compact_bound(off, nseg, t);
      if ((threadIdx.x & 31) == 0) s_bound[threadIdx.x >> 5] = b;
    }
    __syncthreads();
    const int32_t slo = s_bound[0], shi = s_bound[1];
    const bool win = shi - slo < kCompactWin;
    if (win)
      for (int i = threadIdx.x; i <= shi - slo; i += kBlock) s_off[i] = off[slo + i];
    __syncthreads();
    int64_t src[kCompactItems];
#pragma unroll
    for (int it = 0; it < kCompactItems; it++) {
      const int64_t e = e0 + it * kBlock + threadIdx.x;
      src[it] = -1;
      if (e < total) {
        int32_t seg, o;
        if (win) {
          int32_t lo = 0, hi = shi - slo;
          while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= e) lo = mid; else hi = mid - 1;
          }
          seg = slo + lo;
          o = s_off[lo];
        } else {
          int32_t lo = slo, hi = shi;
          while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (off[mid] <= e) lo = mid; else hi = mid - 1;
          }
          seg = lo;
          o = off[lo];
        }
        src[it] = first[seg] + (e - o);
      }
    }
    unsigned long long kv[kCompactItems];
    int32_t vv[kCompactItems];
#pragma unroll
    for (int it = 0; it < kCompactItems; it++) {
      const int64_t sc = src[it] < 0 ? 0 : src[it];
      kv[it] = kin[sc];
      vv[it] = vin[sc];
    }
#pragma unroll
    for (int it = 0; it < kCompactItems; it++) {
      if (src[it] < 0) continue;
      const int64_t e = e0 + it * kBlock + threadIdx.x;
      kout[e] = kv[it];
      vout[e] = vv[it];
    }
    __syncthreads();
  }
}

// ---- LSD radix sort of (u64 key, i32 value), 8-bit digits, stable
// ITEMS elements per thread: small sorts use kRsTile-element blocks (more
// blocks than CUs), large ones 4x larger blocks (a 4x smaller digit-by-block
// matrix to scan, longer runs per digit in the scatter).
constexpr int kRsItemsSmall = kRsTile / kBlock;
constexpr int kRsItemsLarge = 4 * kRsItemsSmall;

template <int kRsItems>
__global__ __launch_bounds__(kBlock) void k_rs_hist(const unsigned long long *keys, int64_t count, int shift, int32_t *hist, int32_t tiles) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = blockIdx.x * (int64_t)(kBlock * kRsItems) + (int64_t)wid * 64 * kRsItems;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int dg[kRsItems];
#pragma unroll
  for (int j = 0; j < kRsItems; j++) {  // all loads first (clamped in range), then the ranking
    const int64_t i = base + j * 64 + lane;
    dg[j] = (int)((keys[i < count ? i : count - 1] >> shift) & 255);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRsItems; j++) {
    const bool ok = base + j * 64 + lane < count;
    const int d = ok ? dg[j] : 0;
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const unsigned long long bb = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bb : ~bb;
    }
    if (ok && (peers & lt) == 0) atomicAdd(&h[d], __popcll(peers));
  }
  __syncthreads();
  hist[threadIdx.x * (int64_t)tiles + blockIdx.x] = h[threadIdx.x];
}

// The block ranks its elements per digit (wave match by ballots), stages them
// in LDS in digit order, and then writes each digit's run to its global
// position with consecutive threads on consecutive elements, so that the
// writes of a run are coalesced instead of one scattered line per element.
template <int kRsItems>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const unsigned long long *__restrict__ kin,
                                                        const int32_t *__restrict__ vin,
                                                        unsigned long long *__restrict__ kout,
                                                        int32_t *__restrict__ vout, int64_t count, int shift,
                                                        const int32_t *__restrict__ offs, int32_t tiles) {
  __shared__ int32_t wcnt[kBlock / 64][256];
  __shared__ int32_t dstart[256];  // block-local start of each digit's run
  __shared__ int32_t goff[256];    // global position of a run minus its block-local start
  __shared__ int32_t sh[kBlock / 64];
  __shared__ unsigned long long skey[kBlock * kRsItems];
  __shared__ int32_t sval[kBlock * kRsItems];
  static_assert(kBlock == 256, "one thread per digit");
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < 256 * (kBlock / 64); d += kBlock) (&wcnt[0][0])[d] = 0;
  __syncthreads();
  const int64_t blk0 = blockIdx.x * (int64_t)(kBlock * kRsItems);
  const int64_t base = blk0 + (int64_t)wid * 64 * kRsItems;
  unsigned long long key[kRsItems];
  int32_t val[kRsItems], rank[kRsItems], dig[kRsItems];
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int j = 0; j < kRsItems; j++) {  // all loads first (clamped in range), then the ranking
    const int64_t i = base + j * 64 + lane;
    const int64_t ic = i < count ? i : count - 1;
    key[j] = kin[ic];
    val[j] = vin[ic];
  }
  for (int j = 0; j < kRsItems; j++) {
    const int64_t i = base + j * 64 + lane;
    const bool ok = i < count;
    const int d = ok ? (int)((key[j] >> shift) & 255) : 0;
    dig[j] = ok ? d : -1;
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const unsigned long long bb = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bb : ~bb;
    }
    const int r = __popcll(peers & lt);
    const int old = ok ? wcnt[wid][d] : 0;
    __builtin_amdgcn_wave_barrier();
    if (ok && r == 0) wcnt[wid][d] = old + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[j] = old + r;
  }
  __syncthreads();
  {  // thread d: offsets of digit d across the block's waves, then the digit's run start
    const int d = threadIdx.x;
    int acc = 0;
    for (int q = 0; q < kBlock / 64; q++) {
      const int t = wcnt[q][d];
      wcnt[q][d] = acc;
      acc += t;
    }
    int32_t total;
    const int32_t start = block_excl_scan(acc, total, sh);
    dstart[d] = start;
    goff[d] = offs[d * (int64_t)tiles + blockIdx.x] - start;
  }
  __syncthreads();
  for (int j = 0; j < kRsItems; j++) {
    if (dig[j] < 0) continue;
    const int d = dig[j];
    const int32_t l = dstart[d] + wcnt[wid][d] + rank[j];
    skey[l] = key[j];
    sval[l] = val[j];
  }
  __syncthreads();
  const int32_t nvalid = (int32_t)min<int64_t>(kBlock * kRsItems, count - blk0);
  for (int e = threadIdx.x; e < nvalid; e += kBlock) {
    const unsigned long long k = skey[e];
    const int64_t pos = (int64_t)goff[(int)((k >> shift) & 255)] + e;
    kout[pos] = k;
    vout[pos] = sval[e];
  }
}

// sorted triples -> coarse CSR: segment heads, column, summed weight per segment
// The same pass zeroes the accumulators of the coarse graph being built (row
// counts, int64 degrees as 32-bit words, weights) and, when given, resets the
// minimum-degree key.
__global__ void k_seg_heads(const unsigned long long *keys, int64_t count, int32_t *head, int32_t *rowcnt,
                            int64_t nrow, int32_t *degw, int64_t ndeg, int32_t *wsum,
                            unsigned long long *minkey) {
  const int64_t m = max(count, max(nrow, ndeg));
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
    if (i < count) {
      head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
      wsum[i] = 0;
    }
    if (i < nrow) rowcnt[i] = 0;
    if (i < ndeg) degw[i] = 0;
  }
  if (minkey && blockIdx.x == 0 && threadIdx.x == 0) *minkey = ~0ull;
}
// seg = exclusive scan of head; each element adds its weight to its segment.
// Within a wave, a segmented scan keyed by segment leaves one weight
// contribution per segment piece, and a second one keyed by row leaves one
// degree and one column-count contribution per row piece, so the atomics
// are few and rarely on the same address.
__global__ void k_seg_write(const unsigned long long *keys, const int32_t *vals, int64_t count, const int32_t *seg,
                            const int32_t *head, int key_bits, int32_t *colo, int32_t *wo, int32_t *rowcnt,
                            unsigned long long *degu, const int32_t *__restrict__ gv_new, const GStat *gs) {
  const int lane = threadIdx.x & 63;
  const unsigned long long mask_lo = (1ull << key_bits) - 1;
  for (int64_t base = blockIdx.x * (int64_t)kBlock; base < count; base += (int64_t)gridDim.x * kBlock) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < count;
    const unsigned long long k = ok ? keys[i] : ~0ull;
    const int32_t h = ok ? head[i] : 1;
    const int32_t s = ok ? seg[i] + h - 1 : -1;  // segment index of element i
    unsigned long long x = ok ? (unsigned long long)(uint32_t)vals[i] : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long y = __shfl_up(x, off, 64);
      const int32_t sy = __shfl_up(s, off, 64);
      if (lane >= off && sy == s) x += y;
    }
    const int32_t s_next = __shfl_down(s, 1, 64);
    const bool last = (lane == 63) || (s_next != s);
    if (ok && last) atomicAdd((uint32_t *)&wo[s], (uint32_t)x);
    if (ok && h) {  // batched keys hold the neighbour relative to its graph's first vertex
      const int32_t lo = (int32_t)(k & mask_lo);
      colo[s] = gv_new ? lo + gs[gv_new[(int64_t)(k >> key_bits)]].base : lo;
    }
    // per row piece: degree (sum of the segment pieces) and new columns (heads)
    const long long row = ok ? (long long)(k >> key_bits) : -1;
    unsigned long long dsum = (ok && last) ? x : 0;
    int32_t hsum = (ok && h) ? 1 : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned long long y = __shfl_up(dsum, off, 64);
      const int32_t hy = __shfl_up(hsum, off, 64);
      const long long ry = __shfl_up(row, off, 64);
      if (lane >= off && ry == row) {
        dsum += y;
        hsum += hy;
      }
    }
    const long long r_next = __shfl_down(row, 1, 64);
    if (ok && (lane == 63 || r_next != row)) {
      if (dsum) atomicAdd(&degu[row], dsum);
      if (hsum) atomicAdd(&rowcnt[row], hsum);
    }
  }
}

// counters of the PR pass
__global__ void k_pr_reset(Status *st) {
  if (threadIdx.x == 0) {
    st->nmarked = 0;
    st->huge_items = 0;
    st->pr_rows[0] = 0;
    st->pr_rows[1] = 0;
  }
}
__global__ void k_reset_bins(Status *st) {
  if (threadIdx.x < 8) st->bin_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    st->dmax = 0;
    st->tile_tot = 0;
    st->big_tiles = 0;
  }
}

__global__ void k_min_degree(const unsigned long long *degu, int32_t n, Status *st) {
  __shared__ unsigned long long sh[kBlock / 64];
  unsigned long long m = ~0ull;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    unsigned long long d = degu[v];
    d = d > 0xFFFFFFFFull ? 0xFFFFFFFFull : d;
    m = umin64(m, (d << 32) | (uint32_t)v);
  }
  m = block_min(m, sh);
  if (threadIdx.x == 0 && m != ~0ull) atomicMin(&st->minkey, m);
}

// lam_hat update after a contraction to a graph of k vertices (one thread)
__global__ void k_bound(Status *st, int32_t level, int32_t k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->updated = 0;
  if (k == 1) { st->stop |= ST_COLLAPSED; return; }
  long long d = (long long)(st->minkey >> 32);
  int32_t v = (int32_t)(st->minkey & 0xFFFFFFFFull);
  if (d < st->lam_hat) {
    st->lam_hat = d;
    st->wit_v = v;
    st->wit_level = level;
    st->updated = 1;
  }
  if (st->lam_hat == 0) st->stop |= ST_DISCONNECTED;
}

// witness bitmap {u : map[u] == wit_v} when lam_hat was just lowered
__global__ void k_witness(const int32_t *map, int32_t n_in, const Status *st, unsigned long long *wit) {
  if (!st->updated) return;
  const int32_t x = st->wit_v;
  for (int64_t base = blockIdx.x * (int64_t)kBlock; base < n_in; base += (int64_t)gridDim.x * kBlock) {
    int64_t u = base + threadIdx.x;
    bool b = u < n_in && map[u] == x;
    unsigned long long bal = __ballot(b);
    if ((threadIdx.x & 63) == 0 && (base + (threadIdx.x & ~63)) < n_in) wit[(base + threadIdx.x) >> 6] = bal;
  }
}

// ------------------------------------------------------------ Padberg-Rinaldi
// Conditions 1-4 of the lemma (2 and 3 strict) on every edge {v, x}. Each
// edge is decided once, by its OWNER: the endpoint with the longer row (ties:
// the smaller id). The mark goes on the owner's arc; the other arc gets 0
// (the union-find takes an edge from either arc). Conditions 1 and 2 need
// only the weight and the two degrees; 3 and 4 need the common
// neighbourhood N(v) & N(x), and the scan stops as soon as condition 3 holds
// or the condition-4 sum reaches lambda-hat, which does not change the
// decision. Who intersects:
//  * rows shorter than kPrRow arcs, in the tiles: the owner's thread merges
//    the two short rows;
//  * rows of kPrRow..kPrLds arcs: a workgroup per row holds the row in an LDS
//    hash table (neighbour -> weight); a 16-lane group per owned arc scans
//    the other (not longer) row and probes the table;
//  * rows longer than kPrLds: owned arcs that the cheap tests leave open are
//    queued; a wave per arc binary-searches the long row for the other row's
//    entries, 64 at a time.
constexpr int kPrRow = 32;
constexpr int kPrSmallMax = 512;   // rows up to this length use the small table
constexpr int kPrLds = 4096;

__device__ __forceinline__ bool pr_cheap(long long c, long long dv, long long dx, long long lam) {
  return c >= lam || dv < 2 * c || dx < 2 * c;
}
__device__ __forceinline__ bool pr_owner(int32_t v, int32_t lv, int32_t x, int32_t lx) {
  return lv > lx || (lv == lx && v < x);
}
// batched: bound of the row's graph, or -1 when it is out of the loop
__device__ __forceinline__ long long graph_lam(const GStat &g) { return g.state == GS_ACTIVE ? g.lam_hat : -1; }
// batched: record that graph g has a marked edge (once per thread and graph)
__device__ __forceinline__ void flag_marked(GStat *gs, int32_t g, int32_t &flagged) {
  if (g == flagged) return;
  flagged = g;
  if (__hip_atomic_load(&gs[g].nmarked, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    atomicExch(&gs[g].nmarked, 1);
}

// conditions 3 and 4 for the owned arc (v, x) of a short row: v's sorted row
// is in LDS ([vb, ve) of s_col / s_w), x's row (not longer) is read from
// global memory 8 entries at a time, all loads first, and merged with v's
// row by a pointer that only moves forward. The decision does not depend on
// the order in which the common neighbours are met.
__device__ bool pr_probe(const int32_t *s_col, const int32_t *s_w, int32_t vb, int32_t ve,
                         const int32_t *__restrict__ col, const int32_t *__restrict__ w, int32_t xb, int32_t xe,
                         long long c, long long dv, long long dx, long long lam) {
  long long sum4 = c;
  int32_t p = vb;
  for (int32_t j0 = xb; j0 < xe && p < ve; j0 += kLoadBatch) {
    int32_t us[kLoadBatch], cx[kLoadBatch];
#pragma unroll
    for (int k = 0; k < kLoadBatch; k++) {
      const int32_t jj = min(j0 + k, xe - 1);
      us[k] = col[jj];
      cx[k] = w[jj];
    }
#pragma unroll
    for (int k = 0; k < kLoadBatch; k++) {
      if (j0 + k >= xe) break;
      while (p < ve && s_col[p] < us[k]) p++;
      if (p == ve) break;  // v's row is exhausted: no further common neighbour
      if (s_col[p] == us[k]) {
        const long long cvu = s_w[p], cxu = cx[k];
        if (dv < 2 * (c + cvu) && dx < 2 * (c + cxu)) return true;
        sum4 += cvu < cxu ? cvu : cxu;
        if (sum4 >= lam) return true;
      }
    }
  }
  return sum4 >= lam;
}

// conditions 3 and 4 by merging two short sorted rows
__device__ bool pr_merge(const int32_t *col, const int32_t *w, int32_t vb, int32_t ve, int32_t xb, int32_t xe,
                         long long c, long long dv, long long dx, long long lam) {
  long long sum4 = c;
  int32_t i = vb, j = xb;
  while (i < ve && j < xe) {
    const int32_t a = col[i], b = col[j];
    if (a < b) {
      i++;
    } else if (b < a) {
      j++;
    } else {
      const long long cvu = w[i], cxu = w[j];
      if (dv < 2 * (c + cvu) && dx < 2 * (c + cxu)) return true;
      sum4 += cvu < cxu ? cvu : cxu;
      if (sum4 >= lam) return true;
      i++;
      j++;
    }
  }
  return sum4 >= lam;
}

// Short rows on the tiles. Rows of kPrRow arcs or more are left to k_pr_rows.
// Small PR graphs (a single solve's coarse graphs): a tile takes a workgroup
// of TB threads (kTileArcs / TB arcs each at most), which keeps enough waves
// in flight, and the owner's row is read from LDS.
template <bool B, int TB>
__global__ __launch_bounds__(TB) void k_pr_tile(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ w,
                                                     const unsigned long long *__restrict__ degu,
                                                     const int4 *__restrict__ meta, int32_t ntiles,
                                                     uint8_t *__restrict__ mark, Status *st,
                                                     const int32_t *__restrict__ gv, GStat *gs) {
  __shared__ int32_t s_rp[kTile + 1];
  __shared__ int32_t s_col[kTileArcs], s_w[kTileArcs];  // the tile's arcs
  __shared__ int s_any;
  __shared__ long long s_lam[B ? kTile : 1];
  __shared__ int32_t s_g[B ? kTile : 1];
  const long long lam0 = B ? 0 : st->lam_hat;
  int32_t flagged = -1;
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 m = meta[t];
    const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
    const int32_t q = (acnt + TB - 1) / TB;
    const int32_t i0 = threadIdx.x * q;
    for (int j = threadIdx.x; j <= rows; j += TB) s_rp[j] = rp[r0 + j] - a0;
    for (int e = threadIdx.x; e < acnt; e += TB) {
      s_col[e] = col[a0 + e];
      s_w[e] = w[a0 + e];
    }
    if constexpr (B) {
      for (int j = threadIdx.x; j < rows; j += TB) {
        const int32_t g = gv[r0 + j];
        s_g[j] = g;
        s_lam[j] = graph_lam(gs[g]);
      }
    }
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    bool any = false;
    if (i0 < acnt) {
      const int32_t iend = min(i0 + q, acnt);
      // the other ends' row bounds and degrees, all loads first (clamped)
      int32_t xs[(kTileArcs / TB)], xbs[(kTileArcs / TB)], xes[(kTileArcs / TB)];
      unsigned long long dxs[(kTileArcs / TB)];
#pragma unroll
      for (int k = 0; k < (kTileArcs / TB); k++) xs[k] = s_col[min(i0 + k, iend - 1)];
#pragma unroll
      for (int k = 0; k < (kTileArcs / TB); k++) {
        xbs[k] = rp[xs[k]];
        xes[k] = rp[xs[k] + 1];
        dxs[k] = degu[xs[k]];
      }
      int32_t j = row_of(s_rp, rows, i0);
#pragma unroll
      for (int k = 0; k < (kTileArcs / TB); k++) {
        const int32_t i = i0 + k;
        if (i >= iend) break;
        while (i >= s_rp[j + 1]) j++;
        const int32_t lv = s_rp[j + 1] - s_rp[j];
        if (lv >= kPrRow) continue;  // k_pr_rows
        const int32_t v = r0 + j, a = a0 + i;
        const int32_t x = xs[k], xb = xbs[k], xe = xes[k];
        const long long lam = B ? s_lam[j] : lam0;
        bool mk = false;
        if (pr_owner(v, lv, x, xe - xb) && lam >= 0) {
          const long long c = s_w[i];
          const long long dv = (long long)degu[v], dx = (long long)dxs[k];
          mk = pr_cheap(c, dv, dx, lam) ||
               pr_probe(s_col, s_w, s_rp[j], s_rp[j + 1], col, w, xb, xe, c, dv, dx, lam);
        }
        mark[a] = mk ? 1 : 0;
        if (mk) {
          any = true;
          if constexpr (B) flag_marked(gs, s_g[j], flagged);
        }
      }
    }
    if (any) s_any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_any && st->nmarked == 0) atomicExch(&st->nmarked, 1);
    __syncthreads();
  }
}

// The same on the large PR graphs of batched unions: one wave per tile, each
// owned edge merged from the two rows in global memory, which measured
// faster there than staging the tile's rows in LDS.
template <bool B>
__global__ __launch_bounds__(kTB) void k_pr_tile_merge(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ w,
                                                     const unsigned long long *__restrict__ degu,
                                                     const int4 *__restrict__ meta, int32_t ntiles,
                                                     uint8_t *__restrict__ mark, Status *st,
                                                     const int32_t *__restrict__ gv, GStat *gs) {
  __shared__ int32_t s_rp[kTile + 1];
  __shared__ int s_any;
  __shared__ long long s_lam[B ? kTile : 1];
  __shared__ int32_t s_g[B ? kTile : 1];
  const long long lam0 = B ? 0 : st->lam_hat;
  int32_t flagged = -1;
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 m = meta[t];
    const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
    const int32_t q = (acnt + kTB - 1) / kTB;
    const int32_t i0 = threadIdx.x * q;
    for (int j = threadIdx.x; j <= rows; j += kTB) s_rp[j] = rp[r0 + j] - a0;
    if constexpr (B) {
      for (int j = threadIdx.x; j < rows; j += kTB) {
        const int32_t g = gv[r0 + j];
        s_g[j] = g;
        s_lam[j] = graph_lam(gs[g]);
      }
    }
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    bool any = false;
    if (i0 < acnt) {
      int32_t j = row_of(s_rp, rows, i0);
      const int32_t iend = min(i0 + q, acnt);
      for (int32_t i = i0; i < iend; i++) {
        while (i >= s_rp[j + 1]) j++;
        const int32_t lv = s_rp[j + 1] - s_rp[j];
        if (lv >= kPrRow) continue;  // k_pr_rows
        const int32_t v = r0 + j, a = a0 + i;
        const int32_t x = col[a];
        const int32_t xb = rp[x], xe = rp[x + 1];
        const long long lam = B ? s_lam[j] : lam0;
        bool mk = false;
        if (pr_owner(v, lv, x, xe - xb) && lam >= 0) {
          const long long c = w[a];
          const long long dv = (long long)degu[v], dx = (long long)degu[x];
          mk = pr_cheap(c, dv, dx, lam) || pr_merge(col, w, a0 + s_rp[j], a0 + s_rp[j + 1], xb, xe, c, dv, dx, lam);
        }
        mark[a] = mk ? 1 : 0;
        if (mk) {
          any = true;
          if constexpr (B) flag_marked(gs, s_g[j], flagged);
        }
      }
    }
    if (any) s_any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_any && st->nmarked == 0) atomicExch(&st->nmarked, 1);
    __syncthreads();
  }
}

// rows of kPrRow..kPrSmallMax arcs from the front of `list`, longer ones up
// to kPrLds from the back
__global__ void k_pr_list(const int32_t *rp, int32_t n, int32_t *list, Status *st) {
  __shared__ int32_t cnt[2], base[2];
  for (int64_t b0 = blockIdx.x * (int64_t)kBlock; b0 < n; b0 += (int64_t)gridDim.x * kBlock) {
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t v = b0 + threadIdx.x;
    const int32_t d = v < n ? rp[v + 1] - rp[v] : 0;
    const int cls = (d >= kPrRow && d <= kPrSmallMax) ? 0 : (d > kPrSmallMax && d <= kPrLds) ? 1 : -1;
    const int pos = cls >= 0 ? atomicAdd(&cnt[cls], 1) : 0;
    __syncthreads();
    if (threadIdx.x < 2) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&st->pr_rows[threadIdx.x], cnt[threadIdx.x]) : 0;
    __syncthreads();
    if (cls == 0) list[base[0] + pos] = (int32_t)v;
    if (cls == 1) list[n - 1 - (base[1] + pos)] = (int32_t)v;
    __syncthreads();
  }
}

// A workgroup per listed row v: v's row in an LDS hash table of 2-4 |row|
// slots; one 16-lane group per owned arc (v, x) scans x's row against it,
// 16 entries at a time (4 arcs in flight per wave, loads still coalesced).
// Partial sums are 32-bit: c + sum <= deg(v) <= total weight <= INT32_MAX.
constexpr int kPrGroup = 16;  // lanes per owned arc in k_pr_rows
constexpr int kPrBuckets = 8;  // length classes of the other row: < 16, 16-31, ..., 512-1023, >= 1024

// Sum / or over each aligned row of 16 lanes with DPP moves (no LDS): after
// the two quad permutations a lane holds its quad's value, row_half_mirror
// pairs the quads of each half row, row_mirror the two halves. Every lane of
// a row must be active.
__device__ __forceinline__ uint32_t row16_sum(uint32_t v) {
  static_assert(kPrGroup == 16, "PR groups are DPP rows");
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  return v;
}
__device__ __forceinline__ int row16_or(int v) {
  v |= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  v |= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  v |= __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
  v |= __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
  return v;
}
// Slot of key u in a power-of-two table (24-bit multiplies: full rate).
__device__ __forceinline__ uint32_t pr_slot(int32_t u, uint32_t mask) {
  return (mul24_golden((uint32_t)u ^ ((uint32_t)u >> 16)) >> 8) & mask;
}
__device__ __forceinline__ int32_t clamp_i32(long long x) {
  return x > INT32_MAX ? INT32_MAX : x < -1 ? -1 : (int32_t)x;
}
template <int TBL, bool B>
__global__ __launch_bounds__(kBlock) void k_pr_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const int32_t *__restrict__ w,
                                                     const unsigned long long *__restrict__ degu,
                                                     const int32_t *__restrict__ list, int which, int32_t n,
                                                     uint8_t *__restrict__ mark, Status *st,
                                                     const int32_t *__restrict__ gv, GStat *gs) {
  __shared__ int32_t tkey[TBL];
  __shared__ int32_t tval[TBL];
  __shared__ int s_any;
  // owned arcs of the current chunk that need the common neighbourhood
  __shared__ int32_t s_nwork;
  __shared__ int32_t s_bcnt[kPrBuckets], s_bbase[kPrBuckets];
  __shared__ int32_t s_wi[kBlock], s_wb[kBlock], s_we[kBlock], s_wc[kBlock];
  __shared__ long long s_wd[kBlock];
  constexpr int G = kPrGroup;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int32_t cnt = st->pr_rows[which];
  int32_t flagged = -1;
  for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
    const int32_t v = which == 0 ? list[r] : list[n - 1 - r];
    const int32_t vb = rp[v], ve = rp[v + 1], lv = ve - vb;
    // power-of-two table of 4 |row| slots or TBL, whichever is smaller (TBL
    // is a power of two >= 2 |row|): load factor at most 1/2, mostly 1/4, so
    // a miss (most probes) rarely takes a second slot
    uint32_t size = 64;
    while (size < 4u * (uint32_t)lv && size < (uint32_t)TBL) size <<= 1;
    const uint32_t mask = size - 1;
    const int32_t g = B ? gv[v] : 0;
    const long long lam = B ? graph_lam(gs[g]) : st->lam_hat;
    for (int e = threadIdx.x; e < (int)size; e += kBlock) tkey[e] = -1;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    for (int32_t i = vb + threadIdx.x; i < ve; i += kBlock) {  // distinct keys: one free slot each
      const int32_t u = col[i];
      uint32_t h = pr_slot(u, mask);
      while (atomicCAS(&tkey[h], -1, u) != -1) h = (h + 1) & mask;
      tval[h] = w[i];
    }
    __syncthreads();
    const long long dv = (long long)degu[v];
    bool any = false;
    // The row's arcs in chunks of kBlock: every thread decides the cheap
    // cases of one arc and lists the owned arcs that need the common
    // neighbourhood, grouped by the length class of the other row, so that
    // the four groups of a wave scan rows of similar length together; the
    // groups then share that list evenly.
    for (int32_t c0 = vb; c0 < ve; c0 += kBlock) {
      if (threadIdx.x < kPrBuckets) s_bcnt[threadIdx.x] = 0;
      __syncthreads();
      const int32_t i = c0 + (int32_t)threadIdx.x;
      int32_t xb = 0, xe = 0, c = 0, bk = -1, rank = 0;
      long long dx = 0;
      if (i < ve) {
        const int32_t x = col[i];
        xb = rp[x];
        xe = rp[x + 1];
        bool mk = false;
        if (pr_owner(v, lv, x, xe - xb) && lam >= 0) {
          c = w[i];
          dx = (long long)degu[x];
          mk = pr_cheap(c, dv, dx, lam);
          if (!mk) {
            bk = min(kPrBuckets - 1, max(0, 28 - __clz(xe - xb)));  // floor(log2 length) - 3, clamped
            rank = atomicAdd(&s_bcnt[bk], 1);
          }
        }
        mark[i] = mk ? 1 : 0;
        if (mk) {
          any = true;
          if constexpr (B) flag_marked(gs, g, flagged);
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int b = 0; b < kPrBuckets; b++) {
          s_bbase[b] = acc;
          acc += s_bcnt[b];
        }
        s_nwork = acc;
      }
      __syncthreads();
      if (bk >= 0) {
        const int32_t k = s_bbase[bk] + rank;
        s_wi[k] = i;
        s_wb[k] = xb;
        s_we[k] = xe;
        s_wc[k] = c;
        s_wd[k] = dx;
      }
      __syncthreads();
      const int32_t nwork = s_nwork;
      for (int32_t wi = grp; wi < nwork; wi += kBlock / G) {
        const int32_t ia = s_wi[wi], xb = s_wb[wi], xe = s_we[wi];
        const long long c = s_wc[wi], dx = s_wd[wi];
        bool mk;
        {
          // condition 3 for a common neighbour u: w(v,u) > dv/2 - c and w(x,u) > dx/2 - c
          // (dv < 2(c + a) <=> a > floor(dv/2) - c); the thresholds are clamped to
          // int32 (weights are positive int32), so the comparisons stay 32-bit
          const int32_t tv = clamp_i32(dv / 2 - c), tx = clamp_i32(dx / 2 - c);
          // x's row in blocks of U chunks of G entries: the next block's
          // loads are issued before this block is probed (first probes, then
          // the rare longer ones); one reduction per block. The decision is
          // the same as entry by entry: the sums only grow.
          constexpr int U = 4;
          long long sum4 = c;
          int pr3 = 0;
          int32_t uu[U], wx[U];
#pragma unroll
          for (int q = 0; q < U; q++) {
            const int32_t j = min(xb + q * G + lane, xe - 1);
            uu[q] = col[j];
            wx[q] = w[j];
          }
          for (int32_t j0 = xb; j0 < xe; j0 += U * G) {
            int32_t nu[U] = {}, nw[U] = {}, kk[U];
            uint32_t hh[U];
            if (j0 + U * G < xe) {
#pragma unroll
              for (int q = 0; q < U; q++) {
                const int32_t j = min(j0 + U * G + q * G + lane, xe - 1);
                nu[q] = col[j];
                nw[q] = w[j];
              }
            }
#pragma unroll
            for (int q = 0; q < U; q++) {
              hh[q] = pr_slot(uu[q], mask);
              kk[q] = tkey[hh[q]];
            }
            uint32_t part = 0;
            int p3 = 0;
#pragma unroll
            for (int q = 0; q < U; q++) {
              if (j0 + q * G + lane >= xe) continue;
              while (kk[q] != uu[q] && kk[q] != -1) {
                hh[q] = (hh[q] + 1) & mask;
                kk[q] = tkey[hh[q]];
              }
              if (kk[q] == uu[q]) {
                const int32_t cvu = tval[hh[q]], cxu = wx[q];
                if (cvu > tv && cxu > tx) p3 = 1;
                part += (uint32_t)(cvu < cxu ? cvu : cxu);
              }
            }
            part = row16_sum(part);  // the groups are the 16-lane DPP rows
            p3 = row16_or(p3);
            sum4 += part;
            pr3 |= p3;
            if (pr3 || sum4 >= lam) break;  // decided
#pragma unroll
            for (int q = 0; q < U; q++) {
              uu[q] = nu[q];
              wx[q] = nw[q];
            }
          }
          mk = pr3 || sum4 >= lam;
        }
        if (lane == 0) mark[ia] = mk ? 1 : 0;
        if (mk) {
          any = true;
          if constexpr (B)
            if (lane == 0) flag_marked(gs, g, flagged);
        }
      }
      __syncthreads();
    }
    if (any && lane == 0) s_any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_any && st->nmarked == 0) atomicExch(&st->nmarked, 1);
    __syncthreads();
  }
}

// rows longer than kPrLds: cheap tests per owned arc, the rest queued
__global__ void k_pr_long(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ w, const unsigned long long *__restrict__ degu,
                          const int32_t *list, const int32_t *cnt_p, uint8_t *__restrict__ mark, int32_t *heavy,
                          Status *st, const int32_t *__restrict__ gv, GStat *gs) {
  __shared__ int s_any;
  const int32_t cnt = *cnt_p;
  int32_t flagged = -1;
  for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
    const int32_t v = list[r];
    const int32_t vb = rp[v], ve = rp[v + 1], lv = ve - vb;
    const int32_t g = gv ? gv[v] : 0;
    const long long lam = gv ? graph_lam(gs[g]) : st->lam_hat;
    const long long dv = (long long)degu[v];
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    bool any = false;
    for (int32_t i = vb + threadIdx.x; i < ve; i += kBlock) {
      const int32_t x = col[i];
      bool mk = false;
      if (pr_owner(v, lv, x, rp[x + 1] - rp[x]) && lam >= 0) {
        const long long c = w[i];
        mk = pr_cheap(c, dv, (long long)degu[x], lam);
        if (!mk) heavy[atomicAdd(&st->huge_items, 1)] = i;  // decided by k_pr_heavy
      }
      mark[i] = mk ? 1 : 0;
      if (mk) {
        any = true;
        if (gv) flag_marked(gs, g, flagged);
      }
    }
    if (any) s_any = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_any && st->nmarked == 0) atomicExch(&st->nmarked, 1);
    __syncthreads();
  }
}

// queued arcs (v, x) of rows longer than kPrLds: one wave each; the lanes
// take 64 entries of x's row at a time and binary-search v's row
__global__ void k_pr_heavy(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ w, const unsigned long long *__restrict__ degu, int32_t n,
                           const int32_t *heavy, uint8_t *__restrict__ mark, Status *st,
                           const int32_t *__restrict__ gv, GStat *gs) {
  const long long lam_single = gv ? 0 : st->lam_hat;
  const int32_t cnt = st->huge_items;
  const int lane = threadIdx.x & 63;
  for (int64_t h = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6; h < cnt; h += ((int64_t)gridDim.x * kBlock) >> 6) {
    const int32_t i = heavy[h];
    // the row of arc i: largest v with rp[v] <= i
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (rp[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const int32_t v = lo, x = col[i];
    const long long lam = gv ? gs[gv[v]].lam_hat : lam_single;  // queued arcs belong to graphs in the loop
    const long long c = w[i];
    const long long dv = (long long)degu[v], dx = (long long)degu[x];
    const int32_t vb = rp[v], ve = rp[v + 1], xb = rp[x], xe = rp[x + 1];
    long long sum4 = c;
    int pr3 = 0;
    for (int32_t j0 = xb; j0 < xe; j0 += 64) {
      const int32_t j = j0 + lane;
      unsigned long long part = 0;
      int p3 = 0;
      if (j < xe) {
        const int32_t u = col[j];
        int32_t a = vb, b = ve;
        while (a < b) {
          int32_t mid = (a + b) >> 1;
          if (col[mid] < u) a = mid + 1; else b = mid;
        }
        if (a < ve && col[a] == u) {
          const long long cvu = w[a], cxu = w[j];
          if (dv < 2 * (c + cvu) && dx < 2 * (c + cxu)) p3 = 1;
          part = (unsigned long long)(cvu < cxu ? cvu : cxu);
        }
      }
      sum4 += (long long)grp_sum<64>(part);
      pr3 |= grp_or<64>(p3);
      if (pr3 || sum4 >= lam) break;
    }
    const bool m = pr3 || sum4 >= lam;
    if (lane == 0) {
      mark[i] = m ? 1 : 0;
      if (m && st->nmarked == 0) atomicExch(&st->nmarked, 1);
      if (m && gv && gs[gv[v]].nmarked == 0) atomicExch(&gs[gv[v]].nmarked, 1);
    }
  }
}

// ------------------------------------------------------------ union-find
// Root of x with path halving. Only non-roots are rewritten, and always to
// one of their ancestors, so concurrent halving and linking stay consistent.
__device__ __forceinline__ int32_t uf_root(int32_t *parent, int32_t x) {
  while (true) {
    int32_t p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    int32_t gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp != p) __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}
// link the larger root under the smaller one: each component's root ends as
// its smallest vertex id, independent of the order of the links
__device__ __forceinline__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_root(parent, a);
    b = uf_root(parent, b);
    if (a == b) return;
    if (a > b) { int32_t t = a; a = b; b = t; }
    if (atomicCAS(&parent[b], b, a) == b) return;
  }
}
// The same union-find on a tile's rows in LDS (local ids 0 .. rows - 1),
// for the marked edges with both ends in the tile.
__device__ __forceinline__ int32_t lds_root(int32_t *lp, int32_t x) {
  while (true) {
    const int32_t p = __hip_atomic_load(&lp[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    const int32_t gp = __hip_atomic_load(&lp[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (gp != p) __hip_atomic_store(&lp[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = gp;
  }
}
__device__ __forceinline__ void lds_union(int32_t *lp, int32_t a, int32_t b) {
  while (true) {
    a = lds_root(lp, a);
    b = lds_root(lp, b);
    if (a == b) return;
    if (a > b) { const int32_t t = a; a = b; b = t; }
    if (atomicCAS(&lp[b], b, a) == b) return;
  }
}
// One wave per tile (wider workgroups ran more unions at once and lost more
// time to failed root links than they gained). Most marked edges join two
// rows of the same tile (on the RHG graph's first coarse graph: 95 %, with
// 99 % of its edges marked), so they are first united in LDS; then every
// row that is not its local root is linked under it in the global forest
// (one CAS, or a full union if another tile linked the row first), and only
// the edges that leave the tile run full unions, from the local root. Links
// always go to a smaller id, so each component's root stays its smallest
// vertex, as with unions in any order.
__global__ __launch_bounds__(kTB) void k_uf_tile(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const uint8_t *__restrict__ mark, const int4 *__restrict__ meta, int32_t ntiles,
                          int32_t *parent) {
  __shared__ int32_t s_rp[kTile + 1];
  __shared__ int32_t lp[kTile];
  for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int4 m = meta[t];
    const int32_t r0 = m.x, rows = m.y, a0 = m.z, acnt = m.w;
    const int32_t q = (acnt + kTB - 1) / kTB;
    const int32_t i0 = threadIdx.x * q;
    for (int j = threadIdx.x; j <= rows; j += kTB) {
      s_rp[j] = rp[r0 + j] - a0;
      if (j < rows) lp[j] = j;
    }
    __syncthreads();
    uint8_t mk[kPerThread];
    int32_t xs[kPerThread], js[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; k++) {  // the lane's marks first (clamped), then the marked columns
      mk[k] = k < q && i0 + k < acnt ? mark[a0 + i0 + k] : 0;
      js[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < kPerThread; k++) xs[k] = mk[k] ? col[a0 + i0 + k] : 0;
    if (i0 < acnt) {
      int32_t j = row_of(s_rp, rows, i0);
#pragma unroll
      for (int k = 0; k < kPerThread; k++) {
        const int32_t i = i0 + k;
        if (k >= q || i >= acnt) break;
        while (i >= s_rp[j + 1]) j++;
        js[k] = j;
      }
    }
    // edges inside the tile, in LDS
#pragma unroll
    for (int k = 0; k < kPerThread; k++) {
      const uint32_t xl = (uint32_t)(xs[k] - r0);
      if (mk[k] && xl < (uint32_t)rows) {
        lds_union(lp, js[k], (int32_t)xl);
        mk[k] = 0;
      }
    }
    // rows under their local roots in the global forest
    for (int j = threadIdx.x; j < rows; j += kTB) {
      const int32_t rj = lds_root(lp, j);
      if (rj != j) {
        const int32_t v = r0 + j, a = r0 + rj;
        if (atomicCAS(&parent[v], v, a) != v) uf_union(parent, v, a);
      }
    }
    // edges that leave the tile
#pragma unroll
    for (int k = 0; k < kPerThread; k++)
      if (mk[k]) uf_union(parent, r0 + lds_root(lp, js[k]), xs[k]);
    __syncthreads();
  }
}
__global__ void k_uf_long(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                          const uint8_t *__restrict__ mark, const int32_t *list, const int32_t *cnt_p,
                          int32_t *parent) {
  const int32_t cnt = *cnt_p;
  for (int32_t r = blockIdx.x; r < cnt; r += gridDim.x) {
    const int32_t v = list[r];
    for (int32_t i = rp[v] + threadIdx.x; i < rp[v + 1]; i += kBlock)
      if (mark[i]) uf_union(parent, v, col[i]);
  }
}
__global__ void k_uf_compress(int32_t *parent, int32_t n, int32_t *rep) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    rep[v] = uf_root(parent, (int32_t)v);
}

// ------------------------------------------------------------ side transfer
// bit u = flag[map[u]] (kernel side) XOR flag[map[0]]: vertex 0 ends on side 0
__global__ void k_side_flags(const int32_t *map, const uint8_t *flags, int32_t n_in, unsigned long long *side) {
  const uint8_t f0 = flags[map[0]];
  for (int64_t base = blockIdx.x * (int64_t)kBlock; base < n_in; base += (int64_t)gridDim.x * kBlock) {
    int64_t u = base + threadIdx.x;
    bool b = u < n_in && (flags[map[u]] != f0);
    unsigned long long bal = __ballot(b);
    if ((threadIdx.x & 63) == 0 && (base + (threadIdx.x & ~63)) < n_in) side[(base + threadIdx.x) >> 6] = bal;
  }
}
__global__ void k_side_witness(const unsigned long long *wit, int32_t n_in, unsigned long long *side) {
  const bool flip = wit[0] & 1ull;
  const int32_t words = (n_in + 63) / 64;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlock) {
    unsigned long long x = wit[i] ^ (flip ? ~0ull : 0ull);
    int32_t rem = n_in - (int32_t)i * 64;
    if (rem < 64) x &= (1ull << rem) - 1;
    side[i] = x;
  }
}

// ------------------------------------------------------------ device exact solve
// Stoer-Wagner on a kernel graph of k <= kDenseMax vertices with the tie
// rules of the host solver (every phase starts at the smallest surviving id;
// the most tightly connected vertex is added next, ties to the smallest id;
// the last vertex t of a phase is merged into the second-to-last s, which
// keeps its id; the side is the set of vertices merged into t at the first
// phase whose cut-of-the-phase is strictly smaller than all before). One wave
// per graph: the weight matrix sits in LDS (rows of odd stride, so column
// walks hit distinct banks), lane l holds vertices l and l + 64 (connection
// weight, membership as a 128-bit set), and each step's selection is one
// wave maximum of (1, conn, 255 - id).
__device__ __forceinline__ unsigned long long sw_key(bool cand, unsigned long long conn, int32_t v) {
  return cand ? (1ull << 62) | (conn << 8) | (uint64_t)(255 - v) : 0ull;
}
// rp: the k + 1 row pointers of the graph (absolute arc indices into col
// and w); columns are vertex ids + cbase. Returns the cut, writes the side
// flags of the k vertices.
__device__ unsigned long long sw_dense_solve(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                             const int32_t *__restrict__ w, int32_t k, int32_t cbase, uint32_t *A,
                                             uint8_t *flags) {
  const int lane = threadIdx.x;
  const int32_t P = k | 1;
  for (int32_t i = lane; i < k * P; i += 64) A[i] = 0;
  __syncthreads();
  for (int32_t v = 0; v < k; v++)
    for (int32_t a = rp[v] + lane; a < rp[v + 1]; a += 64) A[v * P + col[a] - cbase] = (uint32_t)w[a];
  __syncthreads();
  const int32_t v0 = lane, v1 = lane + 64;
  bool alive0 = v0 < k, alive1 = v1 < k;
  unsigned long long m0lo = v0 < k ? 1ull << v0 : 0ull, m0hi = 0ull;
  unsigned long long m1lo = 0ull, m1hi = v1 < k ? 1ull << (v1 - 64) : 0ull;
  unsigned long long best = ~0ull, blo = 0ull, bhi = 0ull;
  for (int32_t remaining = k; remaining > 1; remaining--) {
    const unsigned long long b0 = __ballot(alive0), b1 = __ballot(alive1);
    const int32_t start = b0 ? __ffsll((long long)b0) - 1 : 64 + __ffsll((long long)b1) - 1;
    bool in0 = v0 == start, in1 = v1 == start;
    unsigned long long c0 = alive0 && !in0 ? A[start * P + v0] : 0ull;
    unsigned long long c1 = alive1 && !in1 ? A[start * P + v1] : 0ull;
    int32_t s = start, t = start;
    unsigned long long cut_phase = 0;
    for (int32_t added = 1; added < remaining; added++) {
      const unsigned long long key =
          umax64(sw_key(alive0 && !in0, c0, v0), sw_key(alive1 && !in1, c1, v1));
      const unsigned long long top = grp_max<64>(key);
      const int32_t x = 255 - (int32_t)(top & 0xFFull);
      s = t;
      t = x;
      cut_phase = (top >> 8) & ((1ull << 54) - 1);
      in0 = in0 || v0 == x;
      in1 = in1 || v1 == x;
      if (alive0 && !in0) c0 += A[x * P + v0];
      if (alive1 && !in1) c1 += A[x * P + v1];
    }
    // members of t (from the lane that holds it)
    const int32_t tl = t & 63;
    const unsigned long long tlo = t < 64 ? __shfl(m0lo, tl, 64) : __shfl(m1lo, tl, 64);
    const unsigned long long thi = t < 64 ? __shfl(m0hi, tl, 64) : __shfl(m1hi, tl, 64);
    if (cut_phase < best) {
      best = cut_phase;
      blo = tlo;
      bhi = thi;
    }
    // merge t into s: row and column s gain t's weights (diagonal left 0)
    __syncthreads();
    if (alive0 && v0 != s && v0 != t) {
      A[s * P + v0] += A[t * P + v0];
      A[v0 * P + s] += A[v0 * P + t];
    }
    if (alive1 && v1 != s && v1 != t) {
      A[s * P + v1] += A[t * P + v1];
      A[v1 * P + s] += A[v1 * P + t];
    }
    __syncthreads();
    if (v0 == s) { m0lo |= tlo; m0hi |= thi; }
    if (v1 == s) { m1lo |= tlo; m1hi |= thi; }
    if (v0 == t) alive0 = false;
    if (v1 == t) alive1 = false;
  }
  if (v0 < k) flags[v0] = (uint8_t)((blo >> v0) & 1ull);
  if (v1 < k) flags[v1] = (uint8_t)((bhi >> (v1 - 64)) & 1ull);
  return best;
}
__global__ __launch_bounds__(64) void k_sw_dense(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  const int32_t *__restrict__ w, int32_t k, Status *st,
                                                  uint8_t *flags) {
  extern __shared__ uint32_t A[];
  const unsigned long long best = sw_dense_solve(rp, col, w, k, 0, A, flags);
  if (threadIdx.x == 0) st->sw_cut = (long long)best;
}
// batched: one wave per finished graph, read in place from the union's level
__global__ __launch_bounds__(64) void k_sw_dense_batch(const SwDesc *d, uint8_t *flags, long long *cuts) {
  extern __shared__ uint32_t A[];
  const SwDesc &g = d[blockIdx.x];
  const unsigned long long best = sw_dense_solve(g.rp + g.base, g.col, g.w, g.k, g.base, A, flags + g.foff);
  if (threadIdx.x == 0) cuts[blockIdx.x] = (long long)best;
}
// input side after the device exact solve: the kernel side through the map
// when it beats lambda-hat (ties keep lambda-hat), else the witness
__global__ void k_side_exact(const int32_t *map, const uint8_t *flags, const unsigned long long *wit, int32_t n_in,
                             const Status *st, unsigned long long *side) {
  const bool use_flags = st->sw_cut < st->lam_hat;
  if (use_flags) {
    const uint8_t f0 = flags[map[0]];
    for (int64_t base = blockIdx.x * (int64_t)kBlock; base < n_in; base += (int64_t)gridDim.x * kBlock) {
      const int64_t u = base + threadIdx.x;
      const bool b = u < n_in && (flags[map[u]] != f0);
      const unsigned long long bal = __ballot(b);
      if ((threadIdx.x & 63) == 0 && (base + (threadIdx.x & ~63)) < n_in) side[(base + threadIdx.x) >> 6] = bal;
    }
  } else {
    const bool flip = wit[0] & 1ull;
    const int32_t words = (n_in + 63) / 64;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < words; i += (int64_t)gridDim.x * kBlock) {
      unsigned long long x = wit[i] ^ (flip ? ~0ull : 0ull);
      const int32_t rem = n_in - (int32_t)i * 64;
      if (rem < 64) x &= (1ull << rem) - 1;
      side[i] = x;
    }
  }
}

// ------------------------------------------------------------ batched solves
// SplitMix64 output number `index` (1-based) for a state starting at `seed`
// (Steele, Lea, Flood 2014), as on the host.
__device__ __forceinline__ uint64_t splitmix64_at_dev(uint64_t seed, uint64_t index) {
  uint64_t z = seed + index * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// A graph leaves the round loop: its state is frozen and a snapshot is
// pushed to the ring the host drains at its next status read.
__device__ void finish_graph(GStat &g, int fin, Status *st, GStat *ring, int32_t ring_cap) {
  if (g.state == GS_ACTIVE) atomicSub(&st->active_cnt, 1);
  g.state = GS_DONE;
  g.fin = fin;
  const int32_t idx = atomicAdd(&st->ring_cnt, 1);
  ring[idx % ring_cap] = g;
}

// fresh slots: state at admission
__global__ void k_gs_init(GStat *gs, const GDesc *d, int32_t count, int32_t buf) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    GStat g;
    g.minkey = ~0ull;
    g.wsum = 0;
    g.lam_hat = 0x7FFFFFFFFFFFFFFFll;
    g.err = 0;
    g.wit_v = -1;
    g.wit_level = 0;
    g.updated = 0;
    g.status = 0;
    g.nmarked = 0;
    g.base = d[i].voff;
    g.k = d[i].n;
    g.aoff = d[i].aoff;
    g.nnz = d[i].nnz;
    g.level = 0;
    g.rounds = 0;
    g.n_start = d[i].n;
    g.state = GS_FRESH;
    g.fin = FIN_NONE;
    g.buf = buf;
    g.contracted = 0;
    g.slot = d[i].slot;
    g.salt = 0;
    g.pad = 0;
    gs[d[i].slot] = g;
  }
}

// last descriptor whose chunk offset (field at byte offset `off` of the
// struct) is <= c
template <class D>
__device__ __forceinline__ int32_t desc_find(const D *d, int32_t count, int32_t c, int32_t D::*field) {
  int32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (d[mid].*field <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Packing pass 1, per input row of the fresh graphs: graph index, identity
// map over the padded index range, word owners, row pointer checks.
__global__ void k_pack_rows1(const GDesc *d, int32_t count, int32_t chunks, int32_t *gv, int32_t *map, int32_t *wg,
                             GStat *gs) {
  for (int32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const GDesc &g = d[desc_find(d, count, c, &GDesc::rchunk0)];
    const int64_t v0 = (int64_t)(c - g.rchunk0) * kPackRows;
    const int64_t lim = 64ll * g.words;
    int bad = 0;
    for (int64_t v = v0 + threadIdx.x; v < v0 + kPackRows && v < lim; v += kBlock) {
      const int64_t pu = 64ll * g.woff + v;
      if (v < g.n) {
        gv[g.voff + v] = g.slot;
        map[pu] = g.voff + (int32_t)v;
        const int32_t a = g.rp[v], b = g.rp[v + 1];
        if (a < 0 || b < a || b > g.nnz) bad = 1;
        if (v == 0 && a != 0) bad = 1;
        if (v == g.n - 1 && b != g.nnz) bad = 1;
      } else {
        map[pu] = -1;
      }
      if ((v & 63) == 0) wg[g.woff + (v >> 6)] = g.slot;
    }
    if (bad) atomicOr(&gs[g.slot].err, ERR_ROWPTR);
  }
}

// Packing pass 2: union row pointers (a graph with a malformed row pointer
// gets empty rows but its last, which holds all its arcs).
__global__ void k_pack_rows2(const GDesc *d, int32_t count, int32_t chunks, int32_t *rpu, const GStat *gs) {
  for (int32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const GDesc &g = d[desc_find(d, count, c, &GDesc::rchunk0)];
    const bool bad = (gs[g.slot].err & ERR_ROWPTR) != 0;
    const int64_t v0 = (int64_t)(c - g.rchunk0) * kPackRows;
    for (int64_t v = v0 + threadIdx.x; v < v0 + kPackRows && v < g.n; v += kBlock) {
      rpu[g.voff + v] = g.aoff + (bad ? 0 : g.rp[v]);
      if (v == g.n - 1) rpu[g.voff + g.n] = g.aoff + g.nnz;
    }
  }
}

// Packing of the arcs: columns shifted to union ids (out-of-range columns are
// flagged and replaced by the graph's vertex 0, so no arc leaves its graph).
__global__ void k_pack_arcs(const GDesc *d, int32_t count, int32_t chunks, int32_t *colu, int32_t *wu, GStat *gs) {
  for (int32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const GDesc &g = d[desc_find(d, count, c, &GDesc::achunk0)];
    const int64_t a0 = (int64_t)(c - g.achunk0) * kPackArcs;
    int e = 0;
    for (int64_t a = a0 + threadIdx.x; a < a0 + kPackArcs && a < g.nnz; a += kBlock) {
      int32_t x = g.col[a];
      const int32_t c2 = g.w[a];
      if (x < 0 || x >= g.n) { e |= ERR_COL; x = 0; }
      if (c2 < 1) e |= ERR_WEIGHT;
      colu[g.aoff + a] = g.voff + x;
      wu[g.aoff + a] = c2;
    }
    if (e) atomicOr(&gs[g.slot].err, e);
  }
}

// salt of LP iteration t of each graph's current round (pre: before the
// round counter is advanced at the top of the round)
__global__ void k_salts(GStat *gs, int32_t slots, uint64_t seed, int32_t lp_iters, int32_t t, int32_t pre) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    if (g.state != GS_ACTIVE && g.state != GS_FRESH) continue;
    const int64_t r = pre ? g.rounds : g.rounds - 1;
    g.salt = (uint32_t)(splitmix64_at_dev(seed, (uint64_t)r * (uint64_t)lp_iters + (uint64_t)t) & 0xFFFFFFFFull);
  }
}

// Per-graph minimum-degree key (and weight sum) over vertices [v0, v1).
// Lanes hold consecutive vertices, so a wave mostly covers one graph: then
// one atomic per wave, else one per lane.
__global__ void k_gdeg(const unsigned long long *degu, int32_t v0, int32_t v1, const int32_t *gv, GStat *gs,
                       int with_sum) {
  const int lane = threadIdx.x & 63;
  for (int64_t base = v0 + blockIdx.x * (int64_t)kBlock; base < v1; base += (int64_t)gridDim.x * kBlock) {
    const int64_t v = base + threadIdx.x;
    const bool ok = v < v1;
    const int32_t g = ok ? gv[v] : -1;
    unsigned long long key = ~0ull, sum = 0;
    if (ok) {
      const unsigned long long d = degu[v];
      sum = d;
      key = ((d > 0xFFFFFFFFull ? 0xFFFFFFFFull : d) << 32) | (uint32_t)((int32_t)v - gs[g].base);
    }
    const int32_t g0 = __shfl(g, 0, 64);
    if (__all(g == g0)) {
      if (g0 < 0) continue;
      key = grp_min<64>(key);
      sum = grp_sum<64>(sum);
      if (lane == 0) {
        atomicMin(&gs[g0].minkey, key);
        if (with_sum && sum) atomicAdd(&gs[g0].wsum, sum);
      }
    } else if (ok) {
      atomicMin(&gs[g].minkey, key);
      if (with_sum && sum) atomicAdd(&gs[g].wsum, sum);
    }
  }
}

// level 0 of the fresh graphs: input errors, then the bound from the minimum
// weighted degree; the graph enters the round loop
__global__ void k_gbound0(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    if (g.state != GS_FRESH) continue;
    g.updated = 0;
    if (g.err || g.wsum / 2 > 0x7FFFFFFFull) {
      finish_graph(g, FIN_ERROR, st, ring, ring_cap);
      continue;
    }
    g.state = GS_ACTIVE;
    atomicAdd(&st->active_cnt, 1);
    g.lam_hat = (long long)(g.minkey >> 32);
    g.wit_v = (int32_t)(g.minkey & 0xFFFFFFFFull);
    g.wit_level = 0;
    g.updated = 1;
    if (g.lam_hat == 0) {
      g.status |= ST_DISCONNECTED;
      finish_graph(g, FIN_STOP, st, ring, ring_cap);
    }
  }
}

// top of a round: leave the loop at <= n0 vertices or at the round cap,
// else start the round
__global__ void k_step_top(GStat *gs, int32_t slots, int32_t n0, int32_t max_rounds, Status *st, GStat *ring,
                           int32_t ring_cap) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    g.nmarked = 0;
    if (g.state != GS_ACTIVE) continue;
    if (g.k <= n0) {
      finish_graph(g, FIN_SOLVE, st, ring, ring_cap);
    } else if (g.rounds >= max_rounds) {
      g.status |= ST_MAX_ROUNDS;
      finish_graph(g, FIN_SOLVE, st, ring, ring_cap);
    } else {
      g.rounds++;
      g.n_start = g.k;
    }
  }
}

// end of a round: a round that did not shrink the graph ends its loop
__global__ void k_step_end(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    if (g.state == GS_ACTIVE && g.k == g.n_start) {
      g.status |= ST_NO_PROGRESS;
      finish_graph(g, FIN_SOLVE, st, ring, ring_cap);
    }
  }
}

// after the relabelling scan: each graph's vertex range at the new level
// (mode 0: cluster contraction, every graph in the loop is contracted; mode
// 1: marked-edge contraction, only graphs with a marked edge are)
__global__ void k_gsizes(GStat *gs, int32_t slots, const int32_t *ids, int mode, Status *st) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    if (g.state != GS_ACTIVE) continue;
    const int32_t nb = ids[g.base];
    g.k = ids[g.base + g.k] - nb;
    g.base = nb;
    atomicMax(&st->kloc, g.k);  // (the emission keys' low part holds a graph-local vertex)
    g.minkey = ~0ull;
    g.contracted = mode == 0 ? 1 : (g.nmarked != 0);
  }
}

// after a contraction: arc range, level count, collapse, bound update
__global__ void k_gbound(GStat *gs, int32_t slots, const int32_t *rp, int32_t buf, Status *st, GStat *ring,
                         int32_t ring_cap) {
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < slots; i += gridDim.x * kBlock) {
    GStat &g = gs[i];
    g.updated = 0;
    if (g.state != GS_ACTIVE) continue;
    g.aoff = rp[g.base];
    g.nnz = rp[g.base + g.k] - g.aoff;
    g.buf = buf;
    if (!g.contracted) continue;
    g.level++;
    if (g.k == 1) {
      g.status |= ST_COLLAPSED;
      finish_graph(g, FIN_STOP, st, ring, ring_cap);
      continue;
    }
    const long long d = (long long)(g.minkey >> 32);
    if (d < g.lam_hat) {
      g.lam_hat = d;
      g.wit_v = (int32_t)(g.minkey & 0xFFFFFFFFull);
      g.wit_level = g.level;
      g.updated = 1;
    }
    if (g.lam_hat == 0) {
      g.status |= ST_DISCONNECTED;
      finish_graph(g, FIN_STOP, st, ring, ring_cap);
    }
  }
}

// witness words of the graphs whose bound was just lowered: one wave per
// word of the padded input index space
__global__ void k_gwitness(const int32_t *map, const int32_t *wg, const GStat *gs, int32_t words,
                           unsigned long long *wit) {
  const int lane = threadIdx.x & 63;
  for (int64_t q = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6; q < words;
       q += ((int64_t)gridDim.x * kBlock) >> 6) {
    const int32_t slot = wg[q];
    if (slot < 0 || !gs[slot].updated) continue;
    const int32_t target = gs[slot].base + gs[slot].wit_v;
    const unsigned long long bal = __ballot(map[q * 64 + lane] == target);
    if (lane == 0) wit[q] = bal;
  }
}

// kernel graphs of finished graphs, rebased to local ids, into staging
__global__ void k_gather(const GatherDesc *d, int32_t count, int32_t rchunks, int32_t chunks, int32_t *orp,
                         int32_t *ocol, int32_t *ow) {
  for (int32_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    if (c < rchunks) {
      const GatherDesc &g = d[desc_find(d, count, c, &GatherDesc::rchunk0)];
      const int64_t v0 = (int64_t)(c - g.rchunk0) * kPackRows;
      for (int64_t v = v0 + threadIdx.x; v < v0 + kPackRows && v <= g.k; v += kBlock)
        orp[g.drp + v] = g.rp[g.base + v] - g.aoff;
    } else {
      const int32_t ca = c - rchunks;
      const GatherDesc &g = d[desc_find(d, count, ca, &GatherDesc::achunk0)];
      const int64_t a0 = (int64_t)(ca - g.achunk0) * kPackArcs;
      for (int64_t a = a0 + threadIdx.x; a < a0 + kPackArcs && a < g.nnz; a += kBlock) {
        ocol[g.darc + a] = g.col[g.aoff + a] - g.base;
        ow[g.darc + a] = g.w[g.aoff + a];
      }
    }
  }
}

// Side bitmaps of finished graphs, one wave per output word; the word is
// released (wg = -1) once written. mode 0: the witness bitmap; mode 1:
// flags of the kernel graph's vertices, through the frozen map; mode 2: no
// output (failed input), release only. Vertex 0 ends on side 0.
__global__ void k_side_batch(const SideDesc *d, int32_t count, int32_t words, const int32_t *map,
                             const unsigned long long *wit, const uint8_t *flags, int32_t *wg) {
  const int lane = threadIdx.x & 63;
  for (int64_t q = (blockIdx.x * (int64_t)kBlock + threadIdx.x) >> 6; q < words;
       q += ((int64_t)gridDim.x * kBlock) >> 6) {
    const SideDesc &g = d[desc_find(d, count, (int32_t)q, &SideDesc::wchunk0)];
    const int32_t j = (int32_t)q - g.wchunk0;
    const int64_t word = (int64_t)g.woff + j;
    if (g.mode == 2) {  // failed graph: release only
      if (lane == 0) wg[word] = -1;
      continue;
    }
    unsigned long long x;
    if (g.mode == 0) {
      const bool flip = wit[g.woff] & 1ull;
      x = wit[word] ^ (flip ? ~0ull : 0ull);
    } else {
      const uint8_t f0 = flags[g.foff + (map[64ll * g.woff] - g.fbase)];
      const int32_t u = j * 64 + lane;
      const bool b = u < g.n && flags[g.foff + (map[word * 64 + lane] - g.fbase)] != f0;
      x = __ballot(b);
    }
    if (lane == 0) {
      const int32_t rem = g.n - j * 64;
      if (rem < 64) x &= (1ull << rem) - 1;
      g.side[j] = x;
      wg[word] = -1;
    }
  }
}

// grid of a tile kernel walking XcdWalk: a multiple of the XCD count
inline unsigned xcd_grid(unsigned g) { return (g + kXcds - 1) / kXcds * kXcds; }

inline unsigned grid_for(int64_t items, int per_block = kBlock, unsigned cap = 8192) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ============================================================ launchers
// ------------------------------------------------------------ side stream
// Work on disjoint rows (the long-row kernels beside the arc tiles) is queued
// on a second stream of the calling host thread, so that the two run side by
// side on the device instead of one after the other. side_fork makes the side
// stream wait for the work queued on s so far and returns it; side_join makes
// s wait for the side stream. side_mark records the fork point on s without
// waiting, for a later side_after_mark. Without a side stream (its creation
// failed) every call returns s and the work stays in order on s. The streams
// have the default priority and live until the process ends; a host thread
// borrows one per device on first use and gives it back to a shared pool when
// it exits, so the streams number at most the threads that use the library at
// once (session workers come and go).
namespace {
struct SideStream {
  int dev;
  hipStream_t s2;
  hipEvent_t fork, join;
};
std::mutex side_mu;
std::vector<SideStream> side_pool;
struct SideLease {
  std::vector<SideStream> held;
  ~SideLease() {
    std::lock_guard<std::mutex> lk(side_mu);
    for (const auto &e : held)
      if (e.s2) side_pool.push_back(e);
  }
};
SideStream *side_stream() {
  thread_local SideLease lease;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  for (auto &e : lease.held)
    if (e.dev == dev) return e.s2 ? &e : nullptr;
  SideStream e{dev, nullptr, nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(side_mu);
    for (size_t i = 0; i < side_pool.size(); i++)
      if (side_pool[i].dev == dev) {
        e = side_pool[i];
        side_pool.erase(side_pool.begin() + (int64_t)i);
        break;
      }
  }
  if (!e.s2) {
    if (hipStreamCreateWithFlags(&e.s2, hipStreamNonBlocking) != hipSuccess) {
      e.s2 = nullptr;
    } else if (hipEventCreateWithFlags(&e.fork, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&e.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(e.s2);
      e.s2 = nullptr;
    }
  }
  lease.held.push_back(e);
  return lease.held.back().s2 ? &lease.held.back() : nullptr;
}
hipStream_t side_after_mark(hipStream_t s) {
  SideStream *ss = side_stream();
  if (!ss || hipStreamWaitEvent(ss->s2, ss->fork, 0) != hipSuccess) return s;
  return ss->s2;
}
void side_mark(hipStream_t s) {
  SideStream *ss = side_stream();
  if (ss) (void)hipEventRecord(ss->fork, s);
}
hipStream_t side_fork(hipStream_t s) {
  SideStream *ss = side_stream();
  if (!ss || hipEventRecord(ss->fork, s) != hipSuccess) return s;
  return side_after_mark(s);
}
hipError_t side_join(hipStream_t s, hipStream_t s2) {
  if (s2 == s) return hipSuccess;
  SideStream *ss = side_stream();
  if (!ss) return hipErrorInvalidValue;
  const hipError_t e = hipEventRecord(ss->join, s2);
  return e != hipSuccess ? e : hipStreamWaitEvent(s, ss->join, 0);
}
}  // namespace

hipError_t fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_i32<<<grid_for(count), kBlock, 0, s>>>(p, v, count);
  return hipGetLastError();
}

hipError_t status_reset(Status *st, hipStream_t s) {
  k_status_reset<<<1, 64, 0, s>>>(st);
  return hipGetLastError();
}

hipError_t scan_exclusive(Work &w, const int32_t *in, int32_t *out, int64_t count, int32_t *total, hipStream_t s) {
  if (count <= 0) {
    if (total) return fill_i32(total, 0, 1, s);
    return hipSuccess;
  }
  if (count <= kScanTile) {
    k_scan_tile<<<1, kBlock, 0, s>>>(in, out, count, total);
    return hipGetLastError();
  }
  // up to 256 tiles of 2048 elements (at most 4 look-back windows of 64
  // predecessors); longer arrays: 8192-element tiles, which keeps the
  // look-back at a few windows
  const bool big = count > 256ll * kScanTile;
  const int64_t tile = big ? 4 * kScanTile : kScanTile;
  const int64_t tiles = (count + tile - 1) / tile;
  if (tiles > w.lb_tiles) return hipErrorInvalidValue;
  if (w.lb_epoch == 0 || w.lb_epoch + 1 >= (1u << 30)) {
    k_lb_clear<<<grid_for(w.lb_tiles, kBlock, 256), kBlock, 0, s>>>(w.lb_state, w.lb_tiles, w.lb_ticket);
    w.lb_epoch = 0;
  }
  w.lb_epoch++;
  if (big)
    k_scan_lb<4 * kScanItems><<<(unsigned)tiles, kBlock, 0, s>>>(in, out, count, total, w.lb_state, w.lb_ticket,
                                                                 w.lb_epoch, (int32_t)tiles, w.st);
  else
    k_scan_lb<kScanItems><<<(unsigned)tiles, kBlock, 0, s>>>(in, out, count, total, w.lb_state, w.lb_ticket,
                                                             w.lb_epoch, (int32_t)tiles, w.st);
  return hipGetLastError();
}

hipError_t check_rowptr(const DGraph &g, Status *st, hipStream_t s) {
  k_check_rowptr<<<grid_for(g.n), kBlock, 0, s>>>(g.row_ptr, g.n, g.nnz, st);
  return hipGetLastError();
}

hipError_t build_tiles(const DGraph &g, Work &w, hipStream_t s) {
  w.ntiles = (int32_t)((g.nnz + g.n + kTile - 1) / kTile);
  k_row_pass<<<grid_for((int64_t)g.n + 1, kRowBlock * kRowsPer, 2048), kRowBlock, 0, s>>>(
      g.row_ptr, g.n, w.ntiles, w.tile_meta, w.n_in, w.bins, w.st, (int32_t)tuning_for(g.nnz).long_split);
  k_tiles<<<grid_for(w.ntiles, kBlock * kTilesPer, 1u << 16), kBlock, 0, s>>>(g.row_ptr, g.n, w.ntiles, w.tile_meta,
                                                                             w.st, w.big_tiles);
  return hipGetLastError();
}

namespace {
// items of bin b: host-known count (>= 0) or -1 when only the device knows it
inline int64_t bin_items(const int32_t *known, int b, int64_t fallback) { return known ? known[b] : fallback; }
inline int64_t long_rows_bound(const DGraph &g) { return g.nnz / kTile + 1; }
// grid of a per-row launch: sized to the rows when the host knows them, else
// about one resident wave per SIMD slot (the kernels stride over the list)
inline unsigned rows_grid(int64_t items, int per_block, const int32_t *known) {
  return grid_for(items, per_block, known ? kRowsGridMax : 2048u);
}
// The side stream costs a wait across hardware queues at the fork and at the
// join (several microseconds each): it pays only when the long rows hold much
// of a pass's work. With the class counts known their arcs are bounded from
// below by the class minimums; without them (the first pass of a solve) the
// average degree stands in.
inline bool side_worth(const DGraph &g, const int32_t *known) {
  if (!known) return g.nnz >= 64 * (int64_t)g.n;
  const int64_t lb = 256ll * known[4] + (int64_t)tuning_for(g.nnz).long_split * known[5] + 1024ll * known[6] +
                     4097ll * known[7];
  return lb >= std::max<int64_t>(1 << 22, g.nnz / 8);
}

template <int G, int TBL>
void launch_tab(const DGraph &g, Work &w, int b, const int32_t *known, const int32_t *Lin, int32_t *Lout,
                uint32_t salt, hipStream_t s, const int32_t *gv, const GStat *gs) {
  const int64_t items = bin_items(known, b, long_rows_bound(g));
  if (items <= 0) return;
  const int32_t *list = w.bins + (int64_t)b * w.n_in;
  k_lp_tab<G, TBL><<<rows_grid(items, kBlock / G, known), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, Lin, Lout, list,
                                                                       &w.st->bin_cnt[b], salt, w.st, gv, gs);
}
}  // namespace

// Grid of a persistent kernel: as many workgroups as fit on the device at
// once (at least one), capped by the work items.
// (the occupancy query is made once per kernel and device and kept: it costs
// host time on every launch otherwise)
template <class K>
unsigned resident_grid(K kernel, int block, int64_t items) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void *, int>, int64_t>> known;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  const std::pair<const void *, int> key((const void *)kernel, dev * 4096 + block);
  int64_t full = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (const auto &e : known)
      if (e.first == key) full = e.second;
  }
  if (full == 0) {
    int per_cu = 0, cus = 0;
    if (dev < 0 || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      per_cu = cus = 1;
    full = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
    std::lock_guard<std::mutex> lk(mu);
    known.push_back({key, full});
  }
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(items, full));
}

namespace {
// Dynamic LDS above 64 KB must be allowed per kernel; the attribute is set
// once per kernel and device, under a lock (several host threads may launch).
hipError_t allow_lds(const void *fn, int bytes) {
  static std::mutex mu;
  static std::vector<std::pair<const void *, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  for (const auto &d : done)
    if (d.first == fn && d.second == dev) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.push_back({fn, dev});
  return e;
}
}  // namespace

hipError_t lp_first(const DGraph &g, Work &w, const int32_t *known, int32_t *L, uint32_t salt, bool level0,
                    hipStream_t s, const BatchView *bv) {
  const int l0 = level0 ? 1 : 0;
  const int32_t *gv = bv ? bv->gv : nullptr;
  GStat *gs = bv ? bv->gs : nullptr;
  constexpr int kTP = 2;  // tiles per workgroup step of the small-tile kernel
  const bool each = tuning_for(g.nnz).first_group == 1;
  const unsigned tg = each ? grid_for(w.ntiles, 1, 1u << 20) : grid_for((w.ntiles + kTP - 1) / kTP, 1, 1u << 20);
  const unsigned tb = each ? 0u : resident_grid(k_first_tile_big<true, false>, kTB, w.ntiles);
  // the long and huge rows on the side stream, beside the arc tiles
  const hipStream_t s2 = side_worth(g, known) ? side_fork(s) : s;
  if (each) {
    ProfScope ps(level0 ? PROF_FIRST_TILE_L0 : PROF_FIRST_TILE, s, w.st, w.ntiles);
    if (bv) {
      if (level0)
        k_first_tile_each<true, true><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                         w.deg, salt, w.st, w.part, gv, gs, ps.dev);
      else
        k_first_tile_each<false, true><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                          w.deg, salt, w.st, w.part, gv, gs, ps.dev);
    } else if (level0) {
      k_first_tile_each<true, false><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                        w.deg, salt, w.st, w.part, nullptr, nullptr, ps.dev);
    } else {
      k_first_tile_each<false, false><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                         w.deg, salt, w.st, w.part, nullptr, nullptr, ps.dev);
    }
  } else {
    ProfScope ps(level0 ? PROF_FIRST_TILE_L0 : PROF_FIRST_TILE, s, w.st, w.ntiles);
    if (bv) {
      if (level0) {
        k_first_tile<true, true, kTP><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                         w.deg, salt, w.st, w.part, gv, gs, ps.dev);
        k_first_tile_big<true, true><<<tb, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.big_tiles, L,
                                                        w.deg, salt, w.st, w.part, (int32_t)tg, gv, gs);
      } else {
        k_first_tile<false, true, kTP><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                          w.deg, salt, w.st, w.part, gv, gs, ps.dev);
        k_first_tile_big<false, true><<<tb, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.big_tiles, L,
                                                         w.deg, salt, w.st, w.part, (int32_t)tg, gv, gs);
      }
    } else if (level0) {
      k_first_tile<true, false, kTP><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                        w.deg, salt, w.st, w.part, nullptr, nullptr, ps.dev);
      k_first_tile_big<true, false><<<tb, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.big_tiles, L,
                                                       w.deg, salt, w.st, w.part, (int32_t)tg, nullptr, nullptr);
    } else {
      k_first_tile<false, false, kTP><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.ntiles, L,
                                                         w.deg, salt, w.st, w.part, nullptr, nullptr, ps.dev);
      k_first_tile_big<false, false><<<tb, kTB, 0, s>>>(g.row_ptr, g.col, g.w, g.n, w.tile_meta, w.big_tiles, L,
                                                        w.deg, salt, w.st, w.part, (int32_t)tg, nullptr, nullptr);
    }
  }
  // Level-0 statistics of a single solve: every workgroup of the tile, long-row
  // and huge-chunk kernels leaves (key, sum, errors) in its own part entry,
  // combined by one k_reduce_parts at the end.
  static_assert(kBinHuge - 4 == 3 && kLongParts >= 3 * (int64_t)kRowsGridMax + kHugeChunksGrid, "part entries");
  const bool stats = !bv && level0;
  int64_t np = (int64_t)tg + tb;
  // long rows: a wave per row up to 4096 arcs (the three classes in one launch), chunked beyond
  RowClasses rc = {};
  rc.first[0] = 0;
  for (int c = 0; c < 3; c++) {
    const int b = 4 + c;
    const int64_t items = known ? known[b] : g.nnz / kTile + 1;
    rc.list[c] = w.bins + (int64_t)b * w.n_in;
    rc.cnt[c] = &w.st->bin_cnt[b];
    rc.first[c + 1] = rc.first[c] + (items > 0 ? (int32_t)rows_grid(items, kBlock / 64, known) : 0);
  }
  if (rc.first[3] > 0) {
    k_lp_first<64><<<rc.first[3], kBlock, 0, s2>>>(g.row_ptr, g.col, g.w, g.n, rc, L, w.deg, salt, l0, w.st, gv, gs,
                                                   w.part + 3 * np);
    if (stats) np += rc.first[3];
  }
  if (bin_items(known, kBinHuge, 1) > 0) {
    // huge rows: chunked
    const int32_t *list6 = w.bins + (int64_t)kBinHuge * w.n_in;
    const int32_t *cnt6 = &w.st->bin_cnt[kBinHuge];
    k_huge_plan<<<1, kBlock, 0, s2>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, 0, w.huge_cap, w.st,
                                      level0 ? w.deg : nullptr);
    const unsigned gh = grid_for(g.nnz, kHugeChunk, kHugeChunksGrid);
    k_huge_chunks<<<gh, kBlock, 0, s2>>>(g.row_ptr, g.col, g.w, g.n, list6, cnt6, w.huge_meta, w.part + 3 * np,
                                         w.huge_best, w.deg, salt, level0 ? 2 : 0, w.st, gv, gs);
    if (stats) np += gh;
    k_huge_final<<<64, kBlock, 0, s2>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, nullptr, L, w.deg, salt,
                                        level0 ? 2 : 0, w.st, gv, gs);
  }
  hipError_t e = hipGetLastError();
  const hipError_t ej = side_join(s, s2);
  if (e == hipSuccess) e = ej;
  if (e != hipSuccess) return e;
  if (stats) k_reduce_parts<<<grid_for(np, kBlock, 64), kBlock, 0, s>>>(w.part, (int32_t)np, w.st);
  return hipGetLastError();
}


template <bool B>
void launch_lp_small(int tp, const DGraph &g, Work &w, const int32_t *Lin, int32_t *Lout, uint32_t salt,
                     const int32_t *gv, const GStat *gs, int32_t *prof, hipStream_t s) {
  const int64_t groups = (w.ntiles + tp - 1) / tp;
  const unsigned grid = xcd_grid(grid_for(groups, 1, 1u << 20));
  switch (tp) {
    case 2:
      k_lp_tile<B, 2><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.ntiles, salt, w.st, gv,
                                           gs, prof);
      break;
    case 3:
      k_lp_tile<B, 3><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.ntiles, salt, w.st, gv,
                                           gs, prof);
      break;
    case 4:
      k_lp_tile<B, 4><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.ntiles, salt, w.st, gv,
                                           gs, prof);
      break;
    default:
      k_lp_tile<B, 1><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.ntiles, salt, w.st, gv,
                                           gs, prof);
  }
}

namespace {
hipError_t lp_long_rows(const DGraph &g, Work &w, const int32_t *known, const int32_t *Lin, int32_t *Lout,
                        uint32_t salt, hipStream_t s, const int32_t *gv, GStat *gs);
}  // namespace

hipError_t lp_iter(const DGraph &g, Work &w, const int32_t *known, const int32_t *Lin, int32_t *Lout, uint32_t salt,
                   hipStream_t s, const BatchView *bv, int part) {
  const int32_t *gv = bv ? bv->gv : nullptr;
  GStat *gs = bv ? bv->gs : nullptr;
  // the long and huge rows on the side stream, beside the arc tiles (part 1
  // marks the fork point before its tiles, part 2 starts from that mark)
  hipStream_t s2 = s;
  if (part == 0 && side_worth(g, known)) s2 = side_fork(s);
  if (part == 1 && side_worth(g, nullptr)) side_mark(s);
  if (part == 2 && side_worth(g, nullptr)) s2 = side_after_mark(s);
  if (part != 2) {
    ProfScope ps(PROF_LP_TILE, s, w.st, w.ntiles);
    const int tp = (int)tuning_for(g.nnz).lp_group;
    if (bv) {
      launch_lp_small<true>(tp, g, w, Lin, Lout, salt, gv, gs, ps.dev, s);
      k_lp_tile_big<true><<<resident_grid(k_lp_tile_big<true>, kTB, w.ntiles), kTB, 0, s>>>(
          g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.big_tiles, salt, w.st, gv, gs);
    } else {
      launch_lp_small<false>(tp, g, w, Lin, Lout, salt, nullptr, nullptr, ps.dev, s);
      k_lp_tile_big<false><<<resident_grid(k_lp_tile_big<false>, kTB, w.ntiles), kTB, 0, s>>>(
          g.row_ptr, g.col, g.w, Lin, Lout, w.tile_meta, w.big_tiles, salt, w.st, nullptr, nullptr);
    }
  }
  if (part == 1) return hipGetLastError();
  hipError_t e = lp_long_rows(g, w, known, Lin, Lout, salt, s2, gv, gs);
  const hipError_t ej = side_join(s, s2);
  return e != hipSuccess ? e : ej;
}

namespace {
// LP iteration t >= 2 on the long and huge rows (the classes of at least
// 256 arcs), queued on stream s
hipError_t lp_long_rows(const DGraph &g, Work &w, const int32_t *known, const int32_t *Lin, int32_t *Lout,
                        uint32_t salt, hipStream_t s, const int32_t *gv, GStat *gs) {
  launch_tab<64, 1024>(g, w, 4, known, Lin, Lout, salt, s, gv, gs);
  launch_tab<64, 2048>(g, w, 5, known, Lin, Lout, salt, s, gv, gs);
  launch_tab<256, 8192>(g, w, 6, known, Lin, Lout, salt, s, gv, gs);
  if (bin_items(known, kBinHuge, 1) <= 0) return hipGetLastError();
  const int32_t *list6 = w.bins + (int64_t)kBinHuge * w.n_in;
  const int32_t *cnt6 = &w.st->bin_cnt[kBinHuge];
  // label partitions in LDS; the global-table kernels run only if a partition overflowed
  k_huge_plan<<<1, kBlock, 0, s>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, 2, w.huge_cap, w.st, nullptr);
  if (!tuning_for(g.nnz).huge_part) {  // the global-table path for every huge row
    const hipError_t e = fill_i32(&w.st->huge_fallback, 1, 1, s);
    if (e != hipSuccess) return e;
  } else {
    const hipError_t e = allow_lds((const void *)k_huge_part, (int)(8 * kPartSlots));
    if (e != hipSuccess) return e;
    const unsigned pg = resident_grid(k_huge_part, kPartThreads, 1 << 20);
    k_huge_part<<<pg, kPartThreads, 8 * kPartSlots, s>>>(g.row_ptr, g.col, g.w, list6, cnt6, w.huge_meta, Lin,
                                                         w.huge_best, salt, w.st, gv, gs, w.huge_meta, 1);
    // flagged rows again with room for every arc (both launches exit at once without a flag)
    k_huge_plan<<<1, kBlock, 0, s>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, 3, w.huge_cap, w.st, nullptr);
    k_huge_part<<<pg, kPartThreads, 8 * kPartSlots, s>>>(g.row_ptr, g.col, g.w, list6, cnt6, w.huge_meta, Lin,
                                                         w.huge_best, salt, w.st, gv, gs, w.huge_meta, 2);
  }
  k_huge_plan<<<1, kBlock, 0, s>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, 1, w.huge_cap, w.st, nullptr);
  k_huge_clear<<<2048, kBlock, 0, s>>>(w.huge_tab_key, w.huge_tab_val, w.st);
  k_huge_insert<<<grid_for(g.nnz, kHugeChunk, 4096), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, list6, cnt6,
                                                                     w.huge_meta, Lin, w.huge_tab_key,
                                                                     w.huge_tab_val, w.huge_best, salt, w.st, gv,
                                                                     gs);
  k_huge_final<<<64, kBlock, 0, s>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, Lin, Lout, nullptr, salt, 1,
                                     w.st, gv, gs);
  return hipGetLastError();
}
}  // namespace

hipError_t validate_sym(const DGraph &g, Status *st, hipStream_t s, const BatchView *bv) {
  k_validate_sym<<<grid_for(g.n), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, g.n, st, bv ? bv->gv : nullptr,
                                                  bv ? bv->gs : nullptr);
  return hipGetLastError();
}

hipError_t relabel(const int32_t *L, int32_t n, Work &w, hipStream_t s, const BatchView *bv, int32_t *gv_new,
                   int64_t lspace) {
  const int32_t *gv = bv ? bv->gv : nullptr;
  const GStat *gs = bv ? bv->gs : nullptr;
  if (lspace < 0) lspace = n;
  hipError_t e = fill_i32(w.ids, 0, lspace + 1, s);
  if (e != hipSuccess) return e;
  k_flag_labels<<<grid_for(n), kBlock, 0, s>>>(L, n, w.ids, gv, gs);
  // batched: ids[n] = total too, the end of the last graph's range
  e = scan_exclusive(w, w.ids, w.ids, bv ? lspace + 1 : lspace, &w.st->k, s);
  if (e != hipSuccess) return e;
  if (bv) {
    k_apply_ids<<<grid_for(n), kBlock, 0, s>>>(L, w.ids, n, w.cl, gv, gs, gv_new);
  } else {
    k_apply_compose<<<grid_for(std::max(n, w.n_in)), kBlock, 0, s>>>(L, w.ids, n, w.cl, w.map, w.n_in);
  }
  return hipGetLastError();
}

// map = identity; the same launch clears the scans' look-back state, so the
// first scan of the solve needs no clearing launch of its own
__global__ void k_init_map(int32_t *map, int32_t n, unsigned long long *lb_state, int64_t lb_words,
                           uint32_t *lb_ticket) {
  const int64_t m = max((int64_t)n, lb_words);
  for (int64_t u = blockIdx.x * (int64_t)kBlock + threadIdx.x; u < m; u += (int64_t)gridDim.x * kBlock) {
    if (u < n) map[u] = (int32_t)u;
    if (u < lb_words) lb_state[u] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *lb_ticket = 0;
}

// ------------------------------------------------------------ LP variants
// First-iteration restriction (Section 4.1, read synchronously): a vertex
// that another vertex chose in iteration 1 keeps its own label.
__global__ void k_restrict_clear(uint8_t *chosen, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    chosen[v] = 0;
}
__global__ void k_restrict_mark(const int32_t *__restrict__ L, int32_t n, uint8_t *chosen) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int32_t x = L[v];
    if (x != (int32_t)v) chosen[x] = 1;  // iteration 1 starts from the identity
  }
}
__global__ void k_restrict_apply(int32_t *L, int32_t n, const uint8_t *chosen) {
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    if (chosen[v]) L[v] = (int32_t)v;
}
// Labels that differ between two iterations (prev == nullptr: the identity).
__global__ void k_count_changed(const int32_t *__restrict__ prev, const int32_t *__restrict__ cur, int32_t n,
                                Status *st) {
  __shared__ unsigned long long sh[kBlock / 64];
  unsigned long long c = 0;
  for (int64_t v = blockIdx.x * (int64_t)kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock)
    c += cur[v] != (prev ? prev[v] : (int32_t)v);
  c = block_sum(c, sh);
  if (threadIdx.x == 0 && c) atomicAdd(&st->lp_changed, (int32_t)c);
}

hipError_t restrict_first(const DGraph &g, Work &w, int32_t *L, hipStream_t s) {
  if (g.n <= 0) return hipSuccess;
  const unsigned grid = grid_for(g.n);
  k_restrict_clear<<<grid, kBlock, 0, s>>>(w.flags8, g.n);
  k_restrict_mark<<<grid, kBlock, 0, s>>>(L, g.n, w.flags8);
  k_restrict_apply<<<grid, kBlock, 0, s>>>(L, g.n, w.flags8);
  return hipGetLastError();
}

hipError_t count_changed(const int32_t *prev, const int32_t *cur, int32_t n, Work &w, hipStream_t s) {
  hipError_t e = fill_i32(&w.st->lp_changed, 0, 1, s);
  if (e != hipSuccess || n <= 0) return e;
  k_count_changed<<<grid_for(n), kBlock, 0, s>>>(prev, cur, n, w.st);
  return hipGetLastError();
}

hipError_t fix_misplaced(const DGraph &g, Work &w, int32_t *L, hipStream_t s) {
  const int32_t n = g.n;
  if (n <= 0) return hipSuccess;
  int32_t limit = 0;  // floor(log2 n)
  while (((int64_t)1 << (limit + 1)) <= (int64_t)n) limit++;
  k_fix_clear<<<grid_for(n), kBlock, 0, s>>>(w.fix_cnt, w.fix_cut, w.fix_key, n, w.st);
  k_fix_rows<<<grid_for(64ll * n, kBlock, 1u << 16), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, L, n, w.fix_cnt,
                                                                     w.fix_out, w.fix_cut);
  k_fix_delta<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(w.fix_cnt, w.fix_cut, n, w.st);
  k_fix_cand<<<grid_for(n), kBlock, 0, s>>>(L, w.deg, w.fix_cnt, w.fix_cut, w.fix_out, n, limit, w.st, w.fix_key);
  k_fix_apply<<<grid_for(n), kBlock, 0, s>>>(L, w.fix_key, n);
  return hipGetLastError();
}

hipError_t init_map(Work &w, hipStream_t s) {
  k_init_map<<<grid_for(std::max<int64_t>(w.n_in, w.lb_tiles)), kBlock, 0, s>>>(w.map, w.n_in, w.lb_state,
                                                                               w.lb_tiles, w.lb_ticket);
  w.lb_epoch = 1;  // cleared: the next scan takes epoch 2
  return hipGetLastError();
}

namespace {
template <bool B>
void launch_emit_tiles(const DGraph &g, Work &w, const int32_t *gv, const GStat *gs, hipStream_t s) {
  const int tp = (int)tuning_for(g.nnz).emit_group;
  const unsigned grid = grid_for((w.ntiles + tp - 1) / tp, 1, 1u << 20);
  if (tp == 2)
    k_emit_tile<B, 2><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, w.cl, w.tile_meta, w.ntiles, w.st, w.keys[0],
                                           w.vals[0], w.seg, w.seg_cnt, gv, gs);
  else
    k_emit_tile<B, 1><<<grid, kTB, 0, s>>>(g.row_ptr, g.col, g.w, w.cl, w.tile_meta, w.ntiles, w.st, w.keys[0],
                                           w.vals[0], w.seg, w.seg_cnt, gv, gs);
  k_emit_tile_big<B><<<resident_grid(k_emit_tile_big<B>, kTB, w.ntiles), kTB, 0, s>>>(
      g.row_ptr, g.col, g.w, w.cl, w.tile_meta, w.big_tiles, w.st, w.keys[0], w.vals[0], w.seg, w.seg_cnt, gv, gs);
}
}  // namespace

namespace {
hipError_t emit_long_rows(const DGraph &g, Work &w, const int32_t *known, hipStream_t s, const int32_t *gv,
                          const GStat *gs, int64_t long_max);
}  // namespace

hipError_t contract_emit(const DGraph &g, Work &w, const int32_t *known, hipStream_t s, const BatchView *bv) {
  const int32_t *gv = bv ? bv->gv : nullptr;
  const GStat *gs = bv ? bv->gs : nullptr;
  const int64_t long_max = g.nnz / kTile + 1;
  constexpr int kLong = kBins - 4;  // one region of long_max segments per long class
  const int64_t nseg = w.ntiles + kLong * long_max;
  // the long and huge rows on the side stream, beside the arc tiles
  const hipStream_t s2 = side_worth(g, known) ? side_fork(s) : s;
  if (bv)
    launch_emit_tiles<true>(g, w, gv, gs, s);
  else
    launch_emit_tiles<false>(g, w, nullptr, nullptr, s);
  hipError_t e = emit_long_rows(g, w, known, s2, gv, gs, long_max);
  const hipError_t ej = side_join(s, s2);
  if (e == hipSuccess) e = ej;
  if (e != hipSuccess) return e;
  e = scan_exclusive(w, w.seg_cnt, w.seg_cnt, nseg, &w.st->ax, s);
  if (e != hipSuccess) return e;
  if (nseg <= tuning_for(g.nnz).compact_direct_max)
    k_compact_direct<<<grid_for(g.nnz, kBlock, 4096), kBlock, 0, s>>>(w.seg, w.seg_cnt, (int32_t)nseg, w.st,
                                                                       w.keys[0], w.vals[0], w.keys[1], w.vals[1]);
  else
    k_compact<<<grid_for(g.nnz, kBlock * kCompactItems, 4096), kBlock, 0, s>>>(
        w.seg, w.seg_cnt, (int32_t)nseg, w.st, w.keys[0], w.vals[0], w.keys[1], w.vals[1]);
  return hipGetLastError();
}

namespace {
// Emission of the long and huge rows into their segment regions (beyond the
// tiles' segments), queued on stream s
hipError_t emit_long_rows(const DGraph &g, Work &w, const int32_t *known, hipStream_t s, const int32_t *gv,
                          const GStat *gs, int64_t long_max) {
  constexpr int kLong = kBins - 4;  // one region of long_max segments per long class
  // long-row segments beyond the device-side row counts stay empty
  hipError_t e = fill_i32(w.seg_cnt + w.ntiles, 0, kLong * long_max, s);
  if (e != hipSuccess) return e;
  // rows of fewer than 1024 arcs: a wave per row (both classes in one launch)
  RowClasses rc = {};
  const bool wave = tuning_for(g.nnz).emit_wave != 0;
  for (int c = 0; c < 3; c++) rc.first[c + 1] = rc.first[c];
  for (int b = 4; b < kBinHuge; b++) {
    const int64_t items = known ? known[b] : long_max;
    if (items <= 0) continue;
    const int64_t s0 = w.ntiles + (b - 4) * long_max;
    if (b < 6 && wave) {
      const int c = b - 4;
      rc.list[c] = w.bins + (int64_t)b * w.n_in;
      rc.cnt[c] = &w.st->bin_cnt[b];
      rc.seg[c] = w.seg + s0;
      rc.seg_cnt[c] = w.seg_cnt + s0;
      const int32_t gb = (int32_t)grid_for(items, kBlock / 64, 8192);
      for (int c2 = c + 1; c2 < 4; c2++) rc.first[c2] += gb;
    } else {
      k_emit_long<<<grid_for(items, 1, 4096), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, w.cl,
                                                              w.bins + (int64_t)b * w.n_in, &w.st->bin_cnt[b], w.st,
                                                              w.keys[0], w.vals[0], w.seg + s0, w.seg_cnt + s0, gv,
                                                              gs);
    }
  }
  if (rc.first[3] > 0)
    k_emit_wave<<<rc.first[3], kBlock, 0, s>>>(g.row_ptr, g.col, g.w, w.cl, rc, w.st, w.keys[0], w.vals[0], gv, gs);
  if (bin_items(known, kBinHuge, 1) > 0) {
    // chunks of the huge rows (at most long_max of them: one segment each)
    const int32_t *list6 = w.bins + (int64_t)kBinHuge * w.n_in;
    const int32_t *cnt6 = &w.st->bin_cnt[kBinHuge];
    const int64_t s0 = w.ntiles + (kBinHuge - 4) * long_max;
    k_huge_plan<<<1, kBlock, 0, s>>>(g.row_ptr, list6, cnt6, w.huge_meta, w.huge_best, 0, w.huge_cap, w.st, nullptr);
    k_emit_huge<<<grid_for(g.nnz, kHugeChunk, 4096), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, w.cl, list6, cnt6,
                                                                      w.huge_meta, w.st, w.keys[0], w.vals[0],
                                                                      w.seg + s0, w.seg_cnt + s0, gv, gs);
  }
  return hipGetLastError();
}
}  // namespace

namespace {
template <int ITEMS>
hipError_t radix_passes(Work &w, int64_t count, int total_bits, int &which, hipStream_t s) {
  constexpr int64_t tile = (int64_t)kBlock * ITEMS;
  const int32_t tiles = (int32_t)((count + tile - 1) / tile);
  for (int shift = 0; shift < total_bits; shift += 8) {
    k_rs_hist<ITEMS><<<tiles, kBlock, 0, s>>>(w.keys[which], count, shift, w.hist, tiles);
    hipError_t e = scan_exclusive(w, w.hist, w.hist, 256ll * tiles, nullptr, s);
    if (e != hipSuccess) return e;
    k_rs_scatter<ITEMS><<<tiles, kBlock, 0, s>>>(w.keys[which], w.vals[which], w.keys[which ^ 1],
                                                 w.vals[which ^ 1], count, shift, w.hist, tiles);
    which ^= 1;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t radix_sort(Work &w, int64_t count, int total_bits, int &which, hipStream_t s) {
  if (count <= 1) return hipSuccess;
  return count >= tuning_for(count).radix_large_from ? radix_passes<kRsItemsLarge>(w, count, total_bits, which, s)
                               : radix_passes<kRsItemsSmall>(w, count, total_bits, which, s);
}

hipError_t contract_build(Work &w, int which, int64_t count, int key_bits, int32_t k, int dst, int32_t level,
                          hipStream_t s, bool single_bound, const int32_t *gv_new, const GStat *gs) {
  int32_t *rowcnt = w.rp[dst];
  unsigned long long *degu = (unsigned long long *)w.deg;
  // free scratch while the sorted triples sit in buffer `which`
  int32_t *head = w.vals[which ^ 1];
  int32_t *seg = (int32_t *)w.keys[which ^ 1];
  hipError_t e = hipSuccess;
  k_seg_heads<<<grid_for(std::max<int64_t>(count, 2ll * k + 1)), kBlock, 0, s>>>(
      w.keys[which], count, head, rowcnt, (int64_t)k + 1, (int32_t *)degu, 2ll * k, w.w[dst],
      single_bound ? &w.st->minkey : nullptr);
  if (count > 0) {
    e = scan_exclusive(w, head, seg, count, &w.st->nnz, s);
    if (e != hipSuccess) return e;
    k_seg_write<<<grid_for(count), kBlock, 0, s>>>(w.keys[which], w.vals[which], count, seg, head, key_bits,
                                                   w.col[dst], w.w[dst], rowcnt, degu, gv_new, gs);
  } else {
    e = fill_i32(&w.st->nnz, 0, 1, s);
    if (e != hipSuccess) return e;
  }
  e = scan_exclusive(w, rowcnt, rowcnt, (int64_t)k + 1, nullptr, s);
  if (e != hipSuccess) return e;
  if (!single_bound) return hipGetLastError();
  k_min_degree<<<grid_for(k, kBlock, 1024), kBlock, 0, s>>>(degu, k, w.st);
  k_bound<<<1, 64, 0, s>>>(w.st, level, k);
  k_witness<<<grid_for(w.n_in), kBlock, 0, s>>>(w.map, w.n_in, w.st, w.witness);
  return hipGetLastError();
}

__global__ void k_collapse(int32_t *rp, long long *deg, Status *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  rp[0] = 0;
  rp[1] = 0;
  deg[0] = 0;
  st->nnz = 0;
  st->updated = 0;
  st->stop |= ST_COLLAPSED;
}

hipError_t contract_collapse(Work &w, int dst, hipStream_t s) {
  k_collapse<<<1, 64, 0, s>>>(w.rp[dst], w.deg, w.st);
  return hipGetLastError();
}

hipError_t bound_level0(Work &w, hipStream_t s) {
  k_bound<<<1, 64, 0, s>>>(w.st, 0, w.n_in);
  k_witness<<<grid_for(w.n_in), kBlock, 0, s>>>(w.map, w.n_in, w.st, w.witness);
  return hipGetLastError();
}

hipError_t reset_bins(Work &w, hipStream_t s) {
  k_reset_bins<<<1, 64, 0, s>>>(w.st);
  return hipGetLastError();
}

hipError_t pr_mark(const DGraph &g, Work &w, const int32_t *known, hipStream_t s, const BatchView *bv) {
  const int32_t *gv = bv ? bv->gv : nullptr;
  GStat *gs = bv ? bv->gs : nullptr;
  k_pr_reset<<<1, 64, 0, s>>>(w.st);
  const unsigned long long *degu = (const unsigned long long *)w.deg;
  int32_t *heavy = (int32_t *)w.keys[0];  // free between contractions
  int32_t *list = w.parent;               // free until the union-find
  const unsigned tg = grid_for(w.ntiles, 1, 1u << 20);
  // single solves always take the LDS variant; the merge variant is for the
  // large unions of a batch
  const bool wide = !bv || w.ntiles < tuning_for(g.nnz).pr_merge_tiles;
  if (bv) {
    if (wide)
      k_pr_tile<true, kBlock><<<tg, kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu, w.tile_meta, w.ntiles, w.mark, w.st,
                                                    gv, gs);
    else
      k_pr_tile_merge<true><<<tg, kTB, 0, s>>>(g.row_ptr, g.col, g.w, degu, w.tile_meta, w.ntiles, w.mark, w.st, gv,
                                               gs);
  } else {
    k_pr_tile<false, kBlock><<<tg, kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu, w.tile_meta, w.ntiles, w.mark, w.st,
                                                   nullptr, nullptr);
  }
  k_pr_list<<<grid_for(g.n, kBlock, 2048), kBlock, 0, s>>>(g.row_ptr, g.n, list, w.st);
  const unsigned rg = grid_for(g.nnz / kPrRow + 1, 1, 4096);
  if (bv) {
    k_pr_rows<4 * kPrSmallMax, true><<<rg, kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu, list, 0, g.n, w.mark, w.st,
                                                            gv, gs);
    k_pr_rows<2 * kPrLds, true><<<grid_for(g.nnz / kPrSmallMax + 1, 1, 1024), kBlock, 0, s>>>(
        g.row_ptr, g.col, g.w, degu, list, 1, g.n, w.mark, w.st, gv, gs);
  } else {
    k_pr_rows<4 * kPrSmallMax, false><<<rg, kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu, list, 0, g.n, w.mark,
                                                             w.st, nullptr, nullptr);
    k_pr_rows<2 * kPrLds, false><<<grid_for(g.nnz / kPrSmallMax + 1, 1, 1024), kBlock, 0, s>>>(
        g.row_ptr, g.col, g.w, degu, list, 1, g.n, w.mark, w.st, nullptr, nullptr);
  }
  const int64_t items6 = known ? known[kBinHuge] : g.nnz / kHugeChunk + 1;
  if (items6 > 0) {
    k_pr_long<<<grid_for(items6, 1, 4096), kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu,
                                                          w.bins + (int64_t)kBinHuge * w.n_in,
                                                          &w.st->bin_cnt[kBinHuge], w.mark, heavy, w.st, gv, gs);
    k_pr_heavy<<<1024, kBlock, 0, s>>>(g.row_ptr, g.col, g.w, degu, g.n, heavy, w.mark, w.st, gv, gs);
  }
  return hipGetLastError();
}

hipError_t union_find(const DGraph &g, Work &w, const int32_t *known, int32_t *rep, hipStream_t s) {
  k_iota<<<grid_for(g.n), kBlock, 0, s>>>(w.parent, g.n);
  k_uf_tile<<<grid_for(w.ntiles, 1, 1u << 20), kTB, 0, s>>>(g.row_ptr, g.col, w.mark, w.tile_meta, w.ntiles,
                                                               w.parent);
  for (int b = 4; b <= kBinHuge; b++) {
    const int64_t items = known ? known[b] : g.nnz / kTile + 1;
    if (items <= 0) continue;
    k_uf_long<<<grid_for(items, 1, 4096), kBlock, 0, s>>>(g.row_ptr, g.col, w.mark, w.bins + (int64_t)b * w.n_in,
                                                          &w.st->bin_cnt[b], w.parent);
  }
  k_uf_compress<<<grid_for(g.n), kBlock, 0, s>>>(w.parent, g.n, rep);
  return hipGetLastError();
}

hipError_t side_from_flags(Work &w, const uint8_t *flags, uint64_t *side, hipStream_t s) {
  k_side_flags<<<grid_for(w.n_in), kBlock, 0, s>>>(w.map, flags, w.n_in, (unsigned long long *)side);
  return hipGetLastError();
}

hipError_t side_from_witness(Work &w, uint64_t *side, hipStream_t s) {
  k_side_witness<<<grid_for((w.n_in + 63) / 64), kBlock, 0, s>>>(w.witness, w.n_in, (unsigned long long *)side);
  return hipGetLastError();
}

namespace {
// the largest matrix (128 x 129 words) needs more than 64 KB of LDS
hipError_t allow_dense_lds() {
  const int bytes = (int)(sizeof(uint32_t) * kDenseMax * (kDenseMax | 1));
  hipError_t e = allow_lds((const void *)k_sw_dense, bytes);
  return e != hipSuccess ? e : allow_lds((const void *)k_sw_dense_batch, bytes);
}
}  // namespace

hipError_t exact_dense_batch(const SwDesc *d, int32_t count, int32_t kmax, uint8_t *flags, long long *cuts,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (kmax < 2 || kmax > kDenseMax) return hipErrorInvalidValue;
  hipError_t e = allow_dense_lds();
  if (e != hipSuccess) return e;
  k_sw_dense_batch<<<count, 64, sizeof(uint32_t) * (size_t)kmax * (size_t)(kmax | 1), s>>>(d, flags, cuts);
  return hipGetLastError();
}

hipError_t exact_dense(const DGraph &g, Work &w, uint64_t *side, hipStream_t s) {
  if (g.n < 2 || g.n > kDenseMax) return hipErrorInvalidValue;
  const int32_t P = g.n | 1;
  const size_t lds = sizeof(uint32_t) * (size_t)g.n * (size_t)P;
  hipError_t e = allow_dense_lds();
  if (e != hipSuccess) return e;
  k_sw_dense<<<1, 64, lds, s>>>(g.row_ptr, g.col, g.w, g.n, w.st, w.flags8);
  k_side_exact<<<grid_for(w.n_in), kBlock, 0, s>>>(w.map, w.flags8, w.witness, w.n_in, w.st,
                                                   (unsigned long long *)side);
  return hipGetLastError();
}

// ------------------------------------------------------------ batched launchers
hipError_t b_gs_init(GStat *gs, const GDesc *d, int32_t count, int32_t buf, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_gs_init<<<grid_for(count), kBlock, 0, s>>>(gs, d, count, buf);
  return hipGetLastError();
}

hipError_t b_pack(const GDesc *d, int32_t count, int32_t rchunks, int32_t achunks, int32_t *gv, int32_t *map,
                  int32_t *wg, int32_t *rpu, int32_t *colu, int32_t *wu, GStat *gs, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (rchunks > 0) {
    k_pack_rows1<<<grid_for(rchunks, 1, 1u << 16), kBlock, 0, s>>>(d, count, rchunks, gv, map, wg, gs);
    k_pack_rows2<<<grid_for(rchunks, 1, 1u << 16), kBlock, 0, s>>>(d, count, rchunks, rpu, gs);
  }
  if (achunks > 0) k_pack_arcs<<<grid_for(achunks, 1, 1u << 16), kBlock, 0, s>>>(d, count, achunks, colu, wu, gs);
  return hipGetLastError();
}

hipError_t b_salts(GStat *gs, int32_t slots, uint64_t seed, int32_t lp_iters, int32_t t, bool pre, hipStream_t s) {
  k_salts<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, seed, lp_iters, t, pre ? 1 : 0);
  return hipGetLastError();
}

hipError_t b_gdeg(const long long *deg, int32_t v0, int32_t v1, const int32_t *gv, GStat *gs, bool with_sum,
                  hipStream_t s) {
  if (v1 <= v0) return hipSuccess;
  k_gdeg<<<grid_for(v1 - v0, kBlock, 4096), kBlock, 0, s>>>((const unsigned long long *)deg, v0, v1, gv, gs,
                                                             with_sum ? 1 : 0);
  return hipGetLastError();
}

hipError_t b_gbound0(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap, hipStream_t s) {
  k_gbound0<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, st, ring, ring_cap);
  return hipGetLastError();
}

hipError_t b_step_top(GStat *gs, int32_t slots, int32_t n0, int32_t max_rounds, Status *st, GStat *ring,
                      int32_t ring_cap, hipStream_t s) {
  k_step_top<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, n0, max_rounds, st, ring, ring_cap);
  return hipGetLastError();
}

hipError_t b_step_end(GStat *gs, int32_t slots, Status *st, GStat *ring, int32_t ring_cap, hipStream_t s) {
  k_step_end<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, st, ring, ring_cap);
  return hipGetLastError();
}

hipError_t b_gsizes(GStat *gs, int32_t slots, const int32_t *ids, int mode, Status *st, hipStream_t s) {
  const hipError_t e = fill_i32(&st->kloc, 0, 1, s);
  if (e != hipSuccess) return e;
  k_gsizes<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, ids, mode, st);
  return hipGetLastError();
}

hipError_t b_gbound(GStat *gs, int32_t slots, const int32_t *rp, int32_t buf, Status *st, GStat *ring,
                    int32_t ring_cap, hipStream_t s) {
  k_gbound<<<grid_for(slots), kBlock, 0, s>>>(gs, slots, rp, buf, st, ring, ring_cap);
  return hipGetLastError();
}

hipError_t b_gwitness(const int32_t *map, const int32_t *wg, const GStat *gs, int32_t words,
                      unsigned long long *wit, hipStream_t s) {
  if (words <= 0) return hipSuccess;
  k_gwitness<<<grid_for(64ll * words, kBlock, 8192), kBlock, 0, s>>>(map, wg, gs, words, wit);
  return hipGetLastError();
}

hipError_t b_compose(int32_t *map, const int32_t *cl, int64_t entries, const int32_t *wg, const GStat *gs,
                     hipStream_t s) {
  if (entries <= 0) return hipSuccess;
  k_compose<<<grid_for(entries), kBlock, 0, s>>>(map, cl, (int32_t)entries, wg, gs);
  return hipGetLastError();
}

hipError_t b_gather(const GatherDesc *d, int32_t count, int32_t rchunks, int32_t achunks, int32_t *orp,
                    int32_t *ocol, int32_t *ow, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_gather<<<grid_for(rchunks + achunks, 1, 1u << 16), kBlock, 0, s>>>(d, count, rchunks, rchunks + achunks, orp,
                                                                        ocol, ow);
  return hipGetLastError();
}

hipError_t b_side(const SideDesc *d, int32_t count, int32_t words, const int32_t *map,
                  const unsigned long long *wit, const uint8_t *flags, int32_t *wg, hipStream_t s) {
  if (count <= 0 || words <= 0) return hipSuccess;
  k_side_batch<<<grid_for(64ll * words, kBlock, 8192), kBlock, 0, s>>>(d, count, words, map, wit, flags, wg);
  return hipGetLastError();
}

// ------------------------------------------------------------ static scratch
// Workspace of viecut_mincut_noalloc: a file-scope device array, so that the
// call needs no allocation. Every GPU the library runs on holds its own copy
// for the life of the process. In host code `scratch` names a host-side
// stand-in, never the device memory: kernels and copies get the address that
// hipGetSymbolAddress returns for the device (scratch_address).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **ptr) {
  static std::mutex mu;
  static void *addr[kMaxScratchDevices] = {};
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {  // once per device, with that device current
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

}  // namespace vc
