// HIP kernels of one DDQMC step on gfx950 (wave64).
//
//   scan      one thread per occupied configuration: the cheap test whether any
//             clone/death or spawning event happens (most entries: none); the
//             others are staged in LDS and appended to one dense list (large
//             populations to the heavy list)
//   loud      the entries with events, densely, in 256-entry chunks handed out
//             by a counter: counts, multinomial splits and records
//             (model.hpp), staged in LDS and flushed into 64 segments that
//             each have their own counter
//   heavy     the entries with large populations, one wave each (for large
//             lists on a second stream, beside the loud kernel)
//   sort      LSD radix sort of the records by key, 8-bit digits: per pass the
//             digit counts of every tile (the first pass also seals the
//             segments), their prefixes over the tiles with the digit totals,
//             then tiles ranked in LDS with wave ballots and scattered
//   merge     merge-path join of the sorted list with the sorted records: sums
//             every run of equal keys (annihilation) applying the initiator
//             rule, drops empty entries; a count pass, the tile offsets, and a
//             write pass that compacts and emits estimator sums
//   finalize  one block: reduces the estimator sums per solve, updates the shift
//             and the accumulators, and arms the next step
//
// Same-address device atomics serialise (about 11 ns each on MI355X), so no
// kernel here issues more than a few per block or chunk: compaction inside a
// block uses LDS, and record output is spread over 64 counters.
//
// Counts live in device memory (Ctrl) so the host never waits between steps; a
// step that overflows a buffer sets a flag and every later kernel returns at
// once, leaving the list of the last completed step untouched.
#pragma once

#include "model.hpp"

namespace ddqmc {

constexpr int NT = 256;              // threads per block
// Tile shapes are compiled for a few sizes and chosen per handle (and per list
// size, from the tuner's table): records per thread in a sort tile, merged
// positions per thread in a merge tile.  Buffers are laid out for the smallest.
constexpr int SORT_IT_MIN = 4, SORT_IT_DEFAULT = 8;   // 4, 8 or 16
constexpr int MERGE_IT_MIN = 4, MERGE_IT_DEFAULT = 8; // 4 or 8
constexpr int MIN_SORT_TILE = NT * SORT_IT_MIN;
constexpr int MIN_MERGE_TILE = NT * MERGE_IT_MIN;
constexpr int STAGE = 2048;          // spawn records staged in LDS per block iteration
// member trees queued per loud chunk (an entry finding no room takes the
// general path): as many as keep three loud blocks per CU in LDS
template <typename K>
constexpr uint32_t tree_jobs() {
  return sizeof(K) == 4 ? 1024u : 768u;
}
constexpr int MAX_PASSES = 8;
constexpr int NSEG = 64;             // spawn-record segments
constexpr int COUNT_W = 5;           // per-step counts: in, records, out, loud, heavy
constexpr int SEG_STRIDE = 16;       // their 64-bit counters sit 128 bytes apart
constexpr int32_t NON_INIT = INT32_MIN;  // marks the unused part of a non-initiator record
constexpr int MAX_SLOTS = 512;
constexpr int SERIES_W = 3 + S_NSUM;

enum : uint32_t {
  F_SPAWN_CAP = 1u,  // spawn records exceed their buffer
  F_MAIN_CAP = 2u,   // the new list exceeds its buffer
  F_INT_OVF = 4u,    // a walker count left int32
  F_EXTINCT = 8u,    // a solve lost all walkers / its diagonal weight
  F_RNG = 16u,       // a random stream ran dry
  F_ORDER = 64u,     // merge cuts out of order: the list or the records are not sorted
};

struct Ctrl {
  uint32_t n_main;      // entries of the current list
  uint32_t n_new;       // entries of the list being built
  uint32_t n_spawn;     // records requested this step (may exceed the buffer)
  uint32_t abort;       // set by finalize when a step fails
  uint32_t flags;       // F_* of the current step
  uint32_t fail_flags;  // flags of the failed step
  uint32_t committed;   // steps completed since the host last looked
  uint32_t series_pos;  // rows in the series buffer
  uint32_t epoch;       // bumped every step
  uint32_t n_inject;    // records waiting to enter the list
  uint32_t extinct_slot;
  uint32_t last_spawn;  // records of the last completed step
  uint32_t pad0;
  unsigned long long seg_need;  // largest segment fill of a failed step (64-bit: the
                                // attempted records of a step may exceed 2^32)
  uint32_t n_heavy;     // loud entries that need the general sampling path (scan)
  uint32_t n_late;      // loud entries the light path passed on (loud kernel)
  uint32_t n_loud;      // entries with some event this step
  uint32_t loud_next;   // next chunk of loud entries to hand out
  uint32_t seg_prefix[NSEG + 1];  // record offsets of the segments
};

// The merge's estimator sums go to SUM_BUCKETS buckets per solve, tile t
// into bucket t mod SUM_BUCKETS (with int64 atomics: exact, in any order), so
// that no address takes more than a few hundred adds per step and the
// finalize kernel reads SUM_BUCKETS x S_NSUM words per solve.
constexpr int SUM_BUCKETS = 64;

// ---- small helpers --------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive scan over the block (NT threads); *total = sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds4, uint32_t *total) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const uint32_t x = lds4[i];
    before += (i < w) ? x : 0u;
    all += x;
  }
  *total = all;
  __syncthreads();
  return before + inc - v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive prefix of row[0, n) in place by a block of NTB threads (all of
// them call it; wsum holds NTB / 64 words of LDS); returns the total, in every
// thread.  Up to 8 NTB values each thread takes a run of at most eight
// consecutive values (one wave scan).  Beyond, in rounds of 16 NTB values,
// wave w takes 16 x 64 consecutive values, loaded 64 at a time (coalesced),
// the waves' totals give each wave its offset, then each group of 64 is
// scanned across the lanes: runs of consecutive values per thread would be
// read 64 lanes apart (a 42,500-value prefix took 74 us that way).
template <int NTB>
__device__ uint32_t block_prefix_inplace(uint32_t *row, uint32_t n, uint32_t *wsum) {
  constexpr int NW = NTB / 64;
  constexpr int C = 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (n <= 8u * NTB) {
    const uint32_t per = (n + NTB - 1) / NTB;
    const uint32_t b0 = tid * per < n ? tid * per : n;
    const uint32_t b1 = (b0 + per < n) ? b0 + per : n;
    uint32_t local = 0;
    for (uint32_t b = b0; b < b1; ++b) local += row[b];
    const uint32_t inc = wave_incl_scan(local);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t x = wsum[i];
      before += i < w ? x : 0u;
      all += x;
    }
    uint32_t run = before + inc - local;
    for (uint32_t b = b0; b < b1; ++b) {
      const uint32_t c = row[b];
      row[b] = run;
      run += c;
    }
    __syncthreads();
    return all;
  }
  uint32_t carry = 0;  // the earlier rounds' total (the same in every thread)
  for (uint32_t r0 = 0; r0 < n; r0 += (uint32_t)NTB * C) {
    const uint32_t wb = r0 + (uint32_t)w * 64u * C;
    uint32_t v[C];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const uint32_t b = wb + (uint32_t)k * 64u + (uint32_t)lane;
      v[k] = b < n ? row[b] : 0u;
      sum += v[k];
    }
    const uint32_t wt = wave_sum(sum);
    if (lane == 0) wsum[w] = wt;
    __syncthreads();
    uint32_t off = carry, rt = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t x = wsum[i];
      off += i < w ? x : 0u;
      rt += x;
    }
    __syncthreads();  // (wsum is written again in the next round)
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const uint32_t inc = wave_incl_scan(v[k]);
      const uint32_t b = wb + (uint32_t)k * 64u + (uint32_t)lane;
      if (b < n) row[b] = off + inc - v[k];
      off += __shfl(inc, 63, 64);
    }
    carry += rt;
  }
  return carry;
}

template <typename K>
__device__ __forceinline__ uint32_t lower_bound(const K *a, uint32_t n, K key) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// number of A elements among the first `diag` merged (ties: A first)
template <typename K>
__device__ __forceinline__ uint32_t merge_path(const K *A, uint32_t na, const K *B, uint32_t nb,
                                               uint32_t diag) {
  uint32_t lo = diag > nb ? diag - nb : 0;
  uint32_t hi = diag < na ? diag : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (A[mid] <= B[diag - 1 - mid])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Position pos of the concatenated segments -> index in the segmented buffer.
__device__ __forceinline__ size_t seg_addr(const uint32_t *pre, uint32_t pos, uint32_t segcap) {
  int lo = 0, hi = NSEG;  // pre[lo] <= pos < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= pos)
      lo = mid;
    else
      hi = mid;
  }
  return (size_t)lo * segcap + (pos - pre[lo]);
}

// contiguous range of entries of scan block b
__device__ __forceinline__ uint32_t scan_chunk(uint32_t n, uint32_t nblocks) {
  const uint32_t per = (n + nblocks - 1) / nblocks;
  return (per + NT - 1) / NT * NT;
}

template <typename K>
__device__ __forceinline__ uint32_t slot_of(K key, int SB) {
  return (SB >= (int)(8 * sizeof(K))) ? 0u : (uint32_t)(key >> SB);
}
template <typename K>
__device__ __forceinline__ K low_mask(int SB) {
  return (SB >= (int)(8 * sizeof(K))) ? ~(K)0 : (((K)1 << SB) - 1);
}

// ---- spawn ----------------------------------------------------------------
// Pass 1: the quiet test of every entry (one Philox block).  Block b owns the
// entries [b*chunk, (b+1)*chunk).  The loud ones whose channels can all be
// drawn by inversion are staged in LDS with their key and value and appended
// to one dense list (entry index, key, value) of ctrl->n_loud entries; a block
// reserves its room with one atomic per flush, so the list's order varies
// between runs (nothing downstream depends on it).  The other loud entries
// (large populations, a few hundred) go straight to the heavy list.
constexpr uint32_t LOUD_STAGE = 1024;  // staged loud entries per block (>= 2 NT)

template <typename K, bool GENERAL = false>
__global__ __launch_bounds__(NT) void k_spawn_scan(const K *__restrict__ keys,
                                                   const int2 *__restrict__ vals, Ctrl *ctrl,
                                                   const SlotParams *__restrict__ sp,
                                                   const SlotState *__restrict__ ss,
                                                   uint32_t *__restrict__ lidx,
                                                   K *__restrict__ lkey, int2 *__restrict__ lval,
                                                   uint32_t *__restrict__ heavy, int SB,
                                                   bool split = false) {
  if (ctrl->abort) return;
  __shared__ uint32_t lcount, lbase;
  __shared__ uint32_t s_i[LOUD_STAGE];
  __shared__ K s_k[LOUD_STAGE];
  __shared__ int2 s_v[LOUD_STAGE];
  const uint32_t n = ctrl->n_main;
  const uint32_t chunk = scan_chunk(n, gridDim.x);
  const uint32_t b0 = blockIdx.x * chunk;
  const uint32_t b1 = (b0 + chunk < n) ? b0 + chunk : n;
  const K lowm = low_mask<K>(SB);
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  if (threadIdx.x == 0) lcount = 0;
  __syncthreads();
  // called by the whole block: the staged entries go to the dense list
  auto flush = [&]() {
    const uint32_t c = lcount;
    if (threadIdx.x == 0) lbase = c ? atomicAdd(&ctrl->n_loud, c) : 0u;
    __syncthreads();
    const uint32_t b = lbase;
    for (uint32_t q = threadIdx.x; q < c; q += NT) {
      lidx[b + q] = s_i[q];
      lkey[b + q] = s_k[q];
      lval[b + q] = s_v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) lcount = 0;
    __syncthreads();
  };
  // block-uniform trip count: every thread reaches the ballots and barriers
  for (uint32_t base = b0; base < b1; base += NT) {
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < b1;
    K key = 0;
    int2 v = make_int2(0, 0);
    uint32_t slot = 0;
    if (valid) {
      key = keys[i];
      v = vals[i];
      slot = slot_of<K>(key, SB);
    }
    auto kind_of = [&](const SlotParams &P, double S, uint32_t step) {
      const uint64_t cfg = (uint64_t)(key & lowm);
      const uint32_t N = P.N;
      const uint32_t l = (uint32_t)(cfg >> N);
      const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
      // (a handle with the field sends every entry with events to the loud
      // list, sampled by k_spawn_listed; with split, every solve has the field
      // and the entries whose draws are not all small go to the heavy list)
      if (GENERAL) {
        const int k = P.field ? entry_kind_field(P, S, step, l, m, v.x, v.y, split)
                              : entry_kind(P, S, step, l, m, v.x, v.y);
        return k == ENTRY_QUIET                 ? (int)ENTRY_QUIET
               : (split && k == ENTRY_HEAVY) ? (int)ENTRY_HEAVY
                                               : (int)ENTRY_LIGHT;
      }
      return entry_kind(P, S, step, l, m, v.x, v.y);
    };
    int kind = ENTRY_QUIET;
    // the wave's entries almost always belong to one solve: its parameters are
    // then loaded once, into scalar registers
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(slot);
    if (__ballot(valid && slot != s0) == 0) {
      if (ss[s0].status == 1) {
        const SlotParams &P = sp[s0];
        const double S = ss[s0].S;
        const uint32_t step = (uint32_t)ss[s0].step;
        if (valid) kind = kind_of(P, S, step);
      }
    } else if (valid && ss[slot].status == 1) {
      kind = kind_of(sp[slot], ss[slot].S, (uint32_t)ss[slot].step);
    }
    const uint64_t hmask = __ballot(kind == ENTRY_HEAVY);
    if (hmask) {
      const int leader = __builtin_ctzll(hmask);
      uint32_t hb = 0;
      if (lane == leader) hb = atomicAdd(&ctrl->n_heavy, (uint32_t)__popcll(hmask));
      hb = __shfl(hb, leader, 64);
      if (kind == ENTRY_HEAVY) heavy[hb + (uint32_t)__popcll(hmask & lt)] = i;
    }
    const bool is_loud = kind == ENTRY_LIGHT;
    const uint64_t mask = __ballot(is_loud);
    if (mask) {
      const int leader = __builtin_ctzll(mask);
      uint32_t qbase = 0;
      if (lane == leader) qbase = atomicAdd(&lcount, (uint32_t)__popcll(mask));
      qbase = __shfl(qbase, leader, 64);
      if (is_loud) {
        const uint32_t pos = qbase + (uint32_t)__popcll(mask & lt);
        s_i[pos] = i;
        s_k[pos] = key;
        s_v[pos] = v;
      }
    }
    __syncthreads();
    // room for the next iteration's NT entries
    if (lcount > LOUD_STAGE - NT) flush();
  }
  flush();
}

// Append records to segment seg (its counter is segcnt[seg * SEG_STRIDE]).
template <typename K>
__device__ __forceinline__ void seg_flush(const K *sk, const int2 *sv, uint32_t c, int seg,
                                          unsigned long long *segcnt, K *ok, int2 *ov,
                                          uint32_t segcap, unsigned long long *sbase) {
  if (threadIdx.x == 0)
    *sbase = c ? atomicAdd(&segcnt[seg * SEG_STRIDE], (unsigned long long)c) : 0ull;
  __syncthreads();
  const unsigned long long b = *sbase;
  const size_t off = (size_t)seg * segcap;
  for (uint32_t q = threadIdx.x; q < c; q += NT)
    if (b + q < segcap) {
      ok[off + b + q] = sk[q];
      ov[off + b + q] = sv[q];
    }
  __syncthreads();
}

// seg_flush for a 64-thread block.
template <typename K>
__device__ __forceinline__ void seg_flush64(const K *sk, const int2 *sv, uint32_t c, int seg,
                                            unsigned long long *segcnt, K *ok, int2 *ov,
                                            uint32_t segcap, unsigned long long *sbase) {
  if (threadIdx.x == 0)
    *sbase = c ? atomicAdd(&segcnt[seg * SEG_STRIDE], (unsigned long long)c) : 0ull;
  __syncthreads();
  const unsigned long long b = *sbase;
  const size_t off = (size_t)seg * segcap;
  for (uint32_t q = threadIdx.x; q < c; q += blockDim.x)
    if (b + q < segcap) {
      ok[off + b + q] = sk[q];
      ov[off + b + q] = sv[q];
    }
  __syncthreads();
}

// Emitter shared by the loud kernels: record (key, contribution) into the
// block's LDS stage, or straight into its segment when the stage is full.
template <typename K, uint32_t CAP = STAGE>
struct RecordSink {
  K *sk;
  int2 *sv;
  uint32_t *scount;
  unsigned long long *segcnt;
  K *ok;
  int2 *ov;
  uint32_t segcap;
  int seg;
  bool *int_ovf;
  __device__ void operator()(K ck, int64_t dr, int64_t di, bool keep) const {
    if (dr > 2147483647LL || dr < -2147483647LL || di > 2147483647LL || di < -2147483647LL)
      *int_ovf = true;
    int2 rv = make_int2((int)dr, (int)di);
    if (!keep) {
      if (dr != 0)
        rv.y = NON_INIT;
      else
        rv.x = NON_INIT;
    }
    const uint32_t s = atomicAdd(scount, 1u);
    if (s < CAP) {
      sk[s] = ck;
      sv[s] = rv;
    } else {
      const unsigned long long g = atomicAdd(&segcnt[seg * SEG_STRIDE], 1ull);
      if (g < segcap) {
        ok[(size_t)seg * segcap + g] = ck;
        ov[(size_t)seg * segcap + g] = rv;
      }
    }
  }
};

// The loud kernel's queue of member trees in LDS: an entry reserves places
// for all of its trees at once (reserve fails when the queue is full; the
// entry then takes the general path, having emitted nothing), pushes its
// trees into them, and marks the places it did not use as empty.  Every
// place below min(*count, cap) is thus written by the entry that took
// it before the block's barrier.
static_assert(sizeof(TreeJob) == 24, "tree jobs are sized for the LDS queue");
struct TreeQueue {
  TreeJob *jobs;
  uint32_t *count;
  uint32_t cap;
  uint32_t slot;
  uint32_t at, end;
  __device__ bool reserve(int k) {
    const uint32_t b = atomicAdd(count, (uint32_t)k);
    if (b + (uint32_t)k > cap) {
      // the places below the end of the queue that this failed reservation
      // took are read by the walk: mark them empty
      for (uint32_t i = b; i < cap; ++i) jobs[i].M = 0;
      return false;
    }
    at = b;
    end = b + (uint32_t)k;
    return true;
  }
  __device__ void push(TreeJob t) {
    t.slot = (uint16_t)slot;
    jobs[at++] = t;
  }
  __device__ void close() {
    for (; at < end; ++at) jobs[at].M = 0;
  }
};

// Pass 2: the loud entries, densely (the list the scan wrote).  Entries whose
// draws all take the inversion branch are done here; the few whose channel
// search finds a spawn count too large for it are appended to late[*nlate]
// for k_spawn_heavy.  The initiator rule is applied in
// the merge: a record from a non-initiator parent carries NON_INIT in its
// unused (re or im) part.
template <typename K>
__global__ __launch_bounds__(NT, 3) void k_spawn_loud(
    Ctrl *ctrl, const SlotParams *__restrict__ sp, const SlotState *__restrict__ ss,
    const uint32_t *__restrict__ lidx, const K *__restrict__ lkey, const int2 *__restrict__ lval,
    uint32_t *__restrict__ late, uint32_t *nlate, K *__restrict__ ok, int2 *__restrict__ ov,
    unsigned long long *segcnt, uint32_t segcap, uint32_t tree_cap, int dyn, int SB) {
  if (ctrl->abort) return;
  __shared__ K sk[STAGE];
  __shared__ int2 sv[STAGE];
  __shared__ uint32_t scount;
  __shared__ unsigned long long sbase;
  // the chunk's member trees, walked after its entries (see below)
  constexpr uint32_t TREE_JOBS = tree_jobs<K>();
  __shared__ TreeJob s_jobs[TREE_JOBS];
  __shared__ uint32_t s_njobs;
  const uint32_t tcap = tree_cap < TREE_JOBS ? tree_cap : TREE_JOBS;
  const uint32_t nl = ctrl->n_loud;
  const int seg = blockIdx.x % NSEG;
  const K lowm = low_mask<K>(SB);
  int rng_err = 0, tree_dry = 0;
  bool int_ovf = false;
  const RecordSink<K> sink{sk, sv, &scount, segcnt, ok, ov, segcap, seg, &int_ovf};
  // chunks of NT entries: with dyn, handed out by a counter to blocks that
  // stay resident (blocks that drew cheap chunks take more of them; the next
  // chunk is claimed while the current one is sampled); otherwise block b
  // takes chunks b, b + gridDim.x, ..., and a grid of about one block per
  // chunk retires block by block, which lets the heavy kernel beside it in
  __shared__ uint32_t s_chunk, s_next;
  if (threadIdx.x == 0) s_chunk = dyn ? atomicAdd(&ctrl->loud_next, 1u) : blockIdx.x;
  __syncthreads();
  for (;;) {
    const uint32_t base = s_chunk * NT;
    if (base >= nl) break;
    if (threadIdx.x == 0) {
      scount = 0;
      s_njobs = 0;
    }
    __syncthreads();
    // the last wave claims the next chunk (its wait overlaps the other waves' sampling)
    if (threadIdx.x == NT - 64) s_next = dyn ? atomicAdd(&ctrl->loud_next, 1u) : s_chunk + gridDim.x;
    const uint32_t q = base + threadIdx.x;
    if (q < nl) {
      const K key = lkey[q];
      const int2 v = lval[q];
      const uint32_t slot = slot_of<K>(key, SB);
      const SlotParams &P = sp[slot];
      const K hibits = key & ~lowm;
      const uint64_t cfg = (uint64_t)(key & lowm);
      const uint32_t N = P.N;
      const uint32_t l = (uint32_t)(cfg >> N);
      const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
      const uint32_t step = (uint32_t)ss[slot].step;
      auto rec = [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
        sink(hibits | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
      };
      TreeQueue tq{s_jobs, &s_njobs, tcap, slot, 0, 0};
      const bool done = entry_events_small(P, ss[slot].S, step, l, m, v.x, v.y, &rng_err, rec, tq);
      if (!done) late[atomicAdd(nlate, 1u)] = lidx[q];
      tq.close();
    }
    __syncthreads();
    // The member trees (entries spawning two or more walkers into one class:
    // a few per wave, each a chain of binomial draws) are walked here, one per
    // thread, instead of by their entry's lane while its 63 neighbours wait.
    {
      const uint32_t nj = s_njobs < tcap ? s_njobs : tcap;
      // job r * NT + 4 i + w goes to lane i of wave w: the jobs spread over
      // the block's four waves (and SIMDs) instead of filling the first one
      const uint32_t jt = (threadIdx.x & 63u) * (NT / 64) + (threadIdx.x >> 6);
      for (uint32_t jq = jt; jq < nj; jq += NT) {
        const TreeJob t = s_jobs[jq];
        if (t.M == 0) continue;  // a reserved place the entry did not use
        const SlotParams &P = sp[t.slot];
        const uint32_t N = P.N;
        const K hib = (SB >= (int)(8 * sizeof(K))) ? (K)0 : (K)((K)t.slot << SB);
        run_tree_job(P, (uint32_t)ss[t.slot].step, t, tree_dry,
                     [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
                       sink(hib | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
                     });
      }
    }
    __syncthreads();
    seg_flush(sk, sv, scount < (uint32_t)STAGE ? scount : (uint32_t)STAGE, seg, segcnt, ok, ov,
              segcap, &sbase);
    // seg_flush ends with a barrier: every thread has read s_chunk
    if (threadIdx.x == 0) s_chunk = s_next;
    __syncthreads();
  }
  if (rng_err || tree_dry) atomicOr(&ctrl->flags, F_RNG);
  if (int_ovf) atomicOr(&ctrl->flags, F_INT_OVF);
}

// Pass 3: the entries with large populations, one 64-lane block (one wave) per
// entry, for the list heavy[0, *nheavy).  For a large list it runs on a second
// stream next to the loud kernel (the scan's heavy list) and again after it
// (the loud kernel's late list); for a small one, once after the loud kernel,
// which then appends to the scan's list.  Lanes 0..7 draw the eight channel counts at once; lanes 0 and 1 split
// the two hop channels over their classes; then the binomial trees of all
// classes are walked level by level from an LDS frontier, one node per lane.
// Every draw uses the stream of the same (channel, class, node) as in
// entry_events, so the records are the same.
// A level of a tree has at most as many nodes as the tree has members, so a
// frontier never holds more than the two jump trees (N <= 32 members each)
// plus the twelve hop classes (per part and side the three classes are
// disjoint sets of the 2N <= 64 bonds): 64 + 2 * 2 * 64 = 320 nodes.
constexpr int HEAVY_FRONT = 320;     // tree nodes per frontier level
constexpr uint32_t HEAVY_STAGE = 512;  // records staged in LDS per entry (the rest go direct)

// MINW: waves per SIMD the kernel is compiled for.  1 leaves the compiler its
// registers (two waves per SIMD): the most entries per second, for long
// lists.  3 holds it to 168 VGPRs (with spills): beside the loud kernel its
// waves then find room sooner, which shortens the spawn stage when the list
// is short.  The draws, and so the records, are the same.
template <typename K, int MINW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MINW))) void k_spawn_heavy(
    const K *__restrict__ keys, const int2 *__restrict__ vals, Ctrl *ctrl,
    const SlotParams *__restrict__ sp, const SlotState *__restrict__ ss,
    const uint32_t *__restrict__ heavy, const uint32_t *__restrict__ nheavy, K *__restrict__ ok,
    int2 *__restrict__ ov, unsigned long long *segcnt, uint32_t segcap, int SB) {
  if (ctrl->abort) return;
  __shared__ K sk[HEAVY_STAGE];
  __shared__ int2 sv[HEAVY_STAGE];
  __shared__ uint32_t scount, fcount[2];
  __shared__ unsigned long long sbase;
  __shared__ uint32_t fnode[2][HEAVY_FRONT];  // tree | lo << 5 | hi << 12 | h << 19
  __shared__ int64_t fM[2][HEAVY_FRONT];
  __shared__ uint32_t s_cr[6], s_cu[6];  // class bond masks (right, up) and signs, so
  __shared__ int s_cs[6];                // that a per-lane class index reads LDS
  __shared__ EntryProbs s_e;             // the entry's probabilities, read from LDS by
                                         // every lane instead of held in its registers
  const uint32_t nh = *nheavy;
  const int lane = threadIdx.x;
  const int seg = (blockIdx.x + 17) % NSEG;
  const K lowm = low_mask<K>(SB);
  bool int_ovf = false;
  int dry = 0;
  const RecordSink<K, HEAVY_STAGE> sink{sk, sv, &scount, segcnt, ok, ov, segcap, seg, &int_ovf};
  for (uint32_t q = blockIdx.x; q < nh; q += gridDim.x) {
    const uint32_t i = heavy[q];
    const K key = keys[i];
    const int2 v = vals[i];
    const uint32_t slot = slot_of<K>(key, SB);
    const SlotParams &P = sp[slot];
    const K hibits = key & ~lowm;
    const uint64_t cfg = (uint64_t)(key & lowm);
    const uint32_t N = P.N;
    const uint32_t l = (uint32_t)(cfg >> N);
    const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
    if (lane == 0) {
      s_e = entry_probs(P, ss[slot].S, (uint32_t)ss[slot].step, l, m, v.x, v.y);
      scount = 0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        s_cr[c] = s_e.hc.r[c];
        s_cu[c] = s_e.hc.u[c];
        s_cs[c] = s_e.hc.sgn[c];
      }
    }
    __syncthreads();
    const EntryProbs &e = s_e;
    EntryCounter cnt = s_e.cnt;  // per lane: the draws set its dry flag
    auto out = [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
      sink(hibits | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
    };

    // which channels fire (the primary stream's search, the same on every lane),
    // then lanes 0..7 draw the firing channels' counts at once: each count has
    // its own stream, so the order of the draws does not matter
    bool split_all;
    const uint32_t ev = event_channels(e.p8, e.n8, cnt, &split_all);
    int64_t x = 0;
    if (lane < 8 && ((ev >> lane) & 1u)) {
      double pl = e.p8[0];
      int64_t nl = e.n8[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        pl = lane == k ? e.p8[k] : pl;
        nl = lane == k ? e.n8[k] : nl;
      }
      x = cnt.inl(draw_channel((uint32_t)lane + 1u), nl, pl, split_all ? DRAW_SPLIT : DRAW_POS);
    }
    int64_t X[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) X[c] = __shfl(x, c, 64);
    if (lane == 0) {
      const int64_t dR = e.sR * sgnd(e.d_r) * X[0] - e.sI * sgnd(e.d_i) * X[5];
      const int64_t dI = e.sI * sgnd(e.d_r) * X[4] + e.sR * sgnd(e.d_i) * X[1];
      if (dR != 0 || dI != 0) out(l, m, dR, dI, true);
    }

    // class splits of the two hop channels (lane 0: real walkers, lane 1:
    // imaginary); a single walker is placed at once
    int64_t Mc[6] = {0, 0, 0, 0, 0, 0};
    if (lane < 2) {
      const int part = lane;
      const int ch = part ? 8 : 4;
      int64_t rem = part ? X[7] : X[3];
      const int64_t sg = part ? e.sI : e.sR;
      if (rem == 1) {
        int c, j;
        pick_hop(cnt, draw_channel(ch) + DRAW_PICK, e.Sc, e.hc.n, c, j);
        const uint32_t bm = class_member_mask(P, s_cr[c], s_cu[c], j);
        const uint32_t cl = c < 3 ? (l ^ bm) : l;
        const uint32_t cm = c < 3 ? m : (m ^ bm);
        const int64_t val = sg * (int64_t)s_cs[c];
        out(cl, cm, part ? -val : 0, part ? 0 : val, e.init || cl == cm);
        rem = 0;
      }
      int last = -1;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (e.hc.W[c] > 0.0) last = c;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (rem == 0 || e.hc.W[c] == 0.0) continue;
        const int64_t mc = (c == last) ? rem
                                       : cnt.inl(draw_channel(ch) + 1u + (uint32_t)c, rem,
                                                   e.hc.W[c] / e.Sc[c], DRAW_BIN);
        Mc[c] = mc;
        rem -= mc;
      }
    }
    // the roots: tree 0/1 = jumps of the real/imaginary walkers (nJ members),
    // tree 2 + 6 part + c = hop class c of that part; single jump walkers placed
    if (lane == 0) {
      uint32_t nf = 0;
      const int64_t rootM[2] = {X[2], X[6]};
      for (int part = 0; part < 2; ++part) {
        if (rootM[part] == 1) {
          const int j = pick_member(cnt, draw_channel(part ? 7 : 3) + DRAW_PICK, e.nJ);
          const uint32_t bit = 1u << nth_bit(e.jm, j);
          const int64_t val = part ? e.sI : e.sR;
          out(l & ~bit, m & ~bit, part ? 0 : val, part ? val : 0, e.init);
        } else if (rootM[part] > 1) {
          fnode[0][nf] = (uint32_t)part | (uint32_t)e.nJ << 12 | 1u << 19;
          fM[0][nf++] = rootM[part];
        }
      }
      fcount[0] = nf;
    }
    __syncthreads();
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int64_t mc = __shfl(Mc[c], part, 64);
        if (lane == 0 && mc > 0) {
          const uint32_t f = fcount[0]++;
          fnode[0][f] = (uint32_t)(2 + 6 * part + c) | (uint32_t)e.hc.n[c] << 12 | 1u << 19;
          fM[0][f] = mc;
        }
      }
    __syncthreads();

    // level by level
    int cur = 0;
    while (fcount[cur] > 0) {
      const uint32_t nf = fcount[cur];
      if (lane == 0) fcount[cur ^ 1] = 0;
      __syncthreads();
      for (uint32_t b = 0; b < nf; b += 64) {
        const uint32_t f = b + (uint32_t)lane;
        uint32_t child[2] = {0, 0};
        int64_t childM[2] = {0, 0};
        int nchild = 0;
        if (f < nf) {
          const uint32_t w = fnode[cur][f];
          const int64_t M = fM[cur][f];
          const int t = (int)(w & 31u), lo = (int)((w >> 5) & 127u),
                    hi = (int)((w >> 12) & 127u), h = (int)(w >> 19);
          const int part = t < 2 ? t : (t - 2) / 6;
          const int c = t < 2 ? 0 : (t - 2) % 6;
          const uint32_t base = t < 2 ? draw_channel(part ? 7 : 3) + 64u
                                      : draw_channel(part ? 8 : 4) + 64u + 64u * (uint32_t)c;
          if (hi - lo == 1) {
            const int64_t sg = part ? e.sI : e.sR;
            if (t < 2) {
              const uint32_t bit = 1u << nth_bit(e.jm, lo);
              const int64_t val = sg * M;
              out(l & ~bit, m & ~bit, part ? 0 : val, part ? val : 0, e.init);
            } else {
              const uint32_t cr = s_cr[c], cu = s_cu[c];
              const int nr = popc(cr);
              uint32_t bm;
              if (lo < nr) {
                const uint32_t s = nth_bit(cr, lo);
                bm = (1u << s) | (1u << right_site(P, s));
              } else {
                const uint32_t s = nth_bit(cu, lo - nr);
                bm = (1u << s) | (1u << up_site(P, s));
              }
              const uint32_t cl = c < 3 ? (l ^ bm) : l;
              const uint32_t cm = c < 3 ? m : (m ^ bm);
              const int64_t val = sg * (int64_t)s_cs[c] * M;
              out(cl, cm, part ? -val : 0, part ? 0 : val, e.init || cl == cm);
            }
          } else {
            const int mid = lo + (hi - lo) / 2;
            const int64_t ML = cnt.inl(base + (uint32_t)h, M,
                                         (double)(mid - lo) / (double)(hi - lo), DRAW_BIN);
            if (ML > 0) {
              child[nchild] = (uint32_t)t | (uint32_t)lo << 5 | (uint32_t)mid << 12 |
                              (uint32_t)(2 * h) << 19;
              childM[nchild++] = ML;
            }
            if (M - ML > 0) {
              child[nchild] = (uint32_t)t | (uint32_t)mid << 5 | (uint32_t)hi << 12 |
                              (uint32_t)(2 * h + 1) << 19;
              childM[nchild++] = M - ML;
            }
          }
        }
        // append the children to the next level
        const uint32_t inc = wave_incl_scan((uint32_t)nchild);
        const uint32_t tot = __shfl(inc, 63, 64);
        const uint32_t nbase = fcount[cur ^ 1];
        const uint32_t pos = nbase + inc - (uint32_t)nchild;
        for (int cc = 0; cc < nchild; ++cc)
          if (pos + cc < HEAVY_FRONT) {
            fnode[cur ^ 1][pos + cc] = child[cc];
            fM[cur ^ 1][pos + cc] = childM[cc];
          }
        __syncthreads();
        if (lane == 0) fcount[cur ^ 1] = nbase + tot;
        __syncthreads();
      }
      cur ^= 1;
      __syncthreads();
    }
    dry |= cnt.dry;
    __syncthreads();
    seg_flush64(sk, sv, scount < HEAVY_STAGE ? scount : HEAVY_STAGE, seg, segcnt, ok, ov, segcap,
                &sbase);
  }
  if (dry) atomicOr(&ctrl->flags, F_RNG);
  if (int_ovf) atomicOr(&ctrl->flags, F_INT_OVF);
}

// Entries with events in a handle with the field, one thread each: *count
// of them, entry q = idx ? idx[q] : q of (skey, sval).  FIELD_ONLY (every
// solve of the handle has the field): the call-free routine, which takes the
// entries whose draws are all small, the others' indices in (skey, sval) to
// the late list (late, ctrl->n_late), and so do those with limit or more
// spawns in one part; else entry_events_field for the solves with the field
// and entry_events for the others.  Records are staged in LDS
// per block iteration and flushed into the block's segment.
template <typename K, bool FIELD_ONLY>
__global__ __launch_bounds__(NT, 2) void k_spawn_listed(Ctrl *ctrl,
                                                     const SlotParams *__restrict__ sp,
                                                     const SlotState *__restrict__ ss,
                                                     const K *__restrict__ skey,
                                                     const int2 *__restrict__ sval,
                                                     const uint32_t *__restrict__ idx,
                                                     const uint32_t *count,
                                                     uint32_t *__restrict__ late,
                                                     K *__restrict__ ok, int2 *__restrict__ ov,
                                                     unsigned long long *segcnt, uint32_t segcap,
                                                     int SB, int limit) {
  if (ctrl->abort) return;
  __shared__ K sk[STAGE];
  __shared__ int2 sv[STAGE];
  __shared__ uint32_t scount;
  __shared__ unsigned long long sbase;
  // With the field's call-free routine, and for a list through idx (the
  // field's large entries), the parts with two or more walkers (class splits
  // and member trees) are queued, then sampled one per thread once NT of them
  // wait (or at the end), so that a wave's lanes walk them together instead
  // of idling beside the few that have them.
  constexpr uint32_t JOBS = 4 * NT;
  __shared__ uint32_t jq[JOBS];    // entry index in (skey, sval)
  __shared__ uint32_t jrem[JOBS];  // walkers of the part
  __shared__ uint8_t jinfo[JOBS];  // el | par << 1
  __shared__ uint32_t jcount;
  if (threadIdx.x == 0) jcount = 0;
  const uint32_t n = *count;
  const bool queued = FIELD_ONLY || idx != nullptr;
  const int seg = blockIdx.x % NSEG;
  const K lowm = low_mask<K>(SB);
  int rng_err = 0;
  bool int_ovf = false;
  const RecordSink<K> sink{sk, sv, &scount, segcnt, ok, ov, segcap, seg, &int_ovf};
  // a list through idx (the large entries, few and each a long chain of
  // draws) is dealt one entry per wave first, so that they spread over the
  // SIMDs; the loud list goes in contiguous runs of NT
  const bool spread = idx != nullptr;
  const uint32_t waves = gridDim.x * (NT / 64);
  const uint32_t wave = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  for (uint32_t base = 0; base < n; base += gridDim.x * NT) {
    if (threadIdx.x == 0) scount = 0;
    __syncthreads();
    const uint32_t i = base + (spread ? (threadIdx.x & 63) * waves + wave
                                      : blockIdx.x * NT + threadIdx.x);
    if (i < n) {
      const uint32_t q = idx ? idx[i] : i;
      const K key = skey[q];
      const int2 v = sval[q];
      const uint32_t slot = slot_of<K>(key, SB);
      const SlotParams &P = sp[slot];
      const K hibits = key & ~lowm;
      const uint64_t cfg = (uint64_t)(key & lowm);
      const uint32_t N = P.N;
      const uint32_t l = (uint32_t)(cfg >> N);
      const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
      const uint32_t step = (uint32_t)ss[slot].step;
      auto rec = [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
        sink(hibits | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
      };
      auto queue = [&](int el, int par, int64_t rem) {
        if (!queued) return false;
        const uint32_t at = atomicAdd(&jcount, 1u);
        if (at >= JOBS) return false;
        jq[at] = q;
        jrem[at] = (uint32_t)rem;
        jinfo[at] = (uint8_t)(el | (par << 1));
        return true;
      };
      if constexpr (FIELD_ONLY) {
        if (!entry_events_field_small(P, ss[slot].S, step, l, m, v.x, v.y, &rng_err, rec, queue,
                                      (int64_t)limit))
          late[atomicAdd(&ctrl->n_late, 1u)] = q;
      } else {
        if (P.field)
          entry_events_field(P, ss[slot].S, step, l, m, v.x, v.y, &rng_err, rec, queue);
        else
          entry_events(P, ss[slot].S, step, l, m, v.x, v.y, &rng_err, rec);
      }
    }
    __syncthreads();
    if (queued) {
      // (block-uniform: jcount and the last iteration are the same for all)
      const uint32_t nj = jcount < JOBS ? jcount : JOBS;
      if (nj >= NT || (nj > 0 && base + gridDim.x * NT >= n)) {
        for (uint32_t t = threadIdx.x; t < nj; t += NT) {
          const uint32_t q = jq[t];
          const uint32_t info = jinfo[t];
          const K key = skey[q];
          const int2 v = sval[q];
          const uint32_t slot = slot_of<K>(key, SB);
          const SlotParams &P = sp[slot];
          const K hibits = key & ~lowm;
          const uint64_t cfg = (uint64_t)(key & lowm);
          const uint32_t N = P.N;
          const uint32_t l = (uint32_t)(cfg >> N);
          const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
          auto rec = [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
            sink(hibits | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
          };
          field_part_job<FIELD_ONLY>(P, ss[slot].S, (uint32_t)ss[slot].step, l, m, v.x, v.y,
                                     (int)(info & 1u), (int)((info >> 1) & 1u),
                                     (int64_t)jrem[t], &rng_err, rec);
        }
        __syncthreads();
        if (threadIdx.x == 0) jcount = 0;
      }
    }
    __syncthreads();
    seg_flush(sk, sv, scount < (uint32_t)STAGE ? scount : (uint32_t)STAGE, seg, segcnt, ok, ov,
              segcap, &sbase);
  }
  if (rng_err) atomicOr(&ctrl->flags, F_RNG);
  if (int_ovf) atomicOr(&ctrl->flags, F_INT_OVF);
}

// ---- per-walker sampling (ablation of the per-entry scheme) ----------------
// k_pw_prefix: walkers of each entry (|re| + |im| of running solves), their
// exclusive prefix within the block of NT entries (pre) and the block totals
// (btot); k_pw_scan: the blocks' offsets in place, the total in btot[nblk];
// k_pw_walk: one thread per walker (grid-stride), its entry found by binary
// search over the block offsets and then over the block's prefixes.
template <typename K>
__global__ __launch_bounds__(NT) void k_pw_prefix(const K *__restrict__ keys,
                                                  const int2 *__restrict__ vals, Ctrl *ctrl,
                                                  const SlotState *__restrict__ ss,
                                                  unsigned long long *__restrict__ pre,
                                                  unsigned long long *__restrict__ btot, int SB) {
  if (ctrl->abort) return;
  __shared__ unsigned long long w4[NT / 64];
  const uint32_t n = ctrl->n_main;
  const uint32_t nblk = (n + NT - 1) / NT;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const uint32_t q = b * NT + threadIdx.x;
    unsigned long long c = 0;
    if (q < n) {
      const int2 v = vals[q];
      if (ss[slot_of<K>(keys[q], SB)].status == 1)
        c = (unsigned long long)(v.x < 0 ? -(int64_t)v.x : v.x) +
            (unsigned long long)(v.y < 0 ? -(int64_t)v.y : v.y);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned long long inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    __syncthreads();
    if (lane == 63) w4[w] = inc;
    __syncthreads();
    unsigned long long before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
      before += i < w ? w4[i] : 0ull;
      all += w4[i];
    }
    if (q < n) pre[q] = before + inc - c;
    if (threadIdx.x == 0) btot[b] = all;
  }
}

__global__ __launch_bounds__(1024) void k_pw_scan(Ctrl *ctrl, unsigned long long *btot) {
  if (ctrl->abort) return;
  __shared__ unsigned long long wsum[16];
  const uint32_t n = ctrl->n_main;
  const uint32_t nblk = (n + NT - 1) / NT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t per = (nblk + 1023) / 1024;
  const uint32_t b0 = tid * per < nblk ? tid * per : nblk;
  const uint32_t b1 = (b0 + per < nblk) ? b0 + per : nblk;
  unsigned long long local = 0;
  for (uint32_t b = b0; b < b1; ++b) local += btot[b];
  unsigned long long inc = local;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  unsigned long long before = 0;
  for (int i = 0; i < w; ++i) before += wsum[i];
  unsigned long long run = before + inc - local;
  for (uint32_t b = b0; b < b1; ++b) {
    const unsigned long long c = btot[b];
    btot[b] = run;
    run += c;
  }
  __syncthreads();
  if (tid == 1023) btot[nblk] = before + inc;
}

template <typename K>
__global__ __launch_bounds__(NT) void k_pw_walk(const K *__restrict__ keys,
                                                const int2 *__restrict__ vals, Ctrl *ctrl,
                                                const SlotParams *__restrict__ sp,
                                                const SlotState *__restrict__ ss,
                                                const unsigned long long *__restrict__ pre,
                                                const unsigned long long *__restrict__ boff,
                                                K *__restrict__ ok, int2 *__restrict__ ov,
                                                unsigned long long *segcnt, uint32_t segcap,
                                                int SB) {
  if (ctrl->abort) return;
  __shared__ K sk[STAGE];
  __shared__ int2 sv[STAGE];
  __shared__ uint32_t scount;
  __shared__ unsigned long long sbase;
  const uint32_t n = ctrl->n_main;
  const uint32_t nblk = (n + NT - 1) / NT;
  const unsigned long long total = boff[nblk];
  const int seg = blockIdx.x % NSEG;
  const K lowm = low_mask<K>(SB);
  int rng_err = 0;
  bool int_ovf = false;
  const RecordSink<K> sink{sk, sv, &scount, segcnt, ok, ov, segcap, seg, &int_ovf};
  const unsigned long long stride = (unsigned long long)gridDim.x * NT;
  for (unsigned long long base = (unsigned long long)blockIdx.x * NT; base < total;
       base += stride) {
    if (threadIdx.x == 0) scount = 0;
    __syncthreads();
    const unsigned long long g = base + threadIdx.x;
    if (g < total) {
      // the block of entries holding walker g, then the entry
      uint32_t lo = 0, hi = nblk;  // the last b with boff[b] <= g
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (boff[mid] <= g) lo = mid; else hi = mid;
      }
      const unsigned long long r = g - boff[lo];
      uint32_t qlo = lo * NT, qhi = (lo + 1) * NT < n ? (lo + 1) * NT : n;
      while (qhi - qlo > 1) {
        const uint32_t mid = (qlo + qhi) >> 1;
        if (pre[mid] <= r) qlo = mid; else qhi = mid;
      }
      // (an entry without walkers shares its prefix with the next one: the
      // search ends on the last entry of the run, which holds the walker)
      const uint32_t q = qlo;
      const unsigned long long k = r - pre[q];
      const K key = keys[q];
      const int2 v = vals[q];
      const uint32_t slot = slot_of<K>(key, SB);
      const SlotParams &P = sp[slot];
      const unsigned long long nR = (unsigned long long)(v.x < 0 ? -(int64_t)v.x : v.x);
      const int part = k < nR ? 0 : 1;
      const unsigned long long w = part ? k - nR : k;
      if (w >= (unsigned long long)PW_MAX_WALKERS) {
        rng_err = 1;
      } else {
        const K hibits = key & ~lowm;
        const uint64_t cfg = (uint64_t)(key & lowm);
        const uint32_t N = P.N;
        const uint32_t l = (uint32_t)(cfg >> N);
        const uint32_t m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
        walker_events(P, ss[slot].S, (uint32_t)ss[slot].step, l, m, v.x, v.y, part,
                      (uint32_t)w, &rng_err,
                      [&](uint32_t cl, uint32_t cm, int64_t dr, int64_t di, bool keep) {
                        sink(hibits | (K)(((uint64_t)cl << N) | cm), dr, di, keep);
                      });
      }
    }
    __syncthreads();
    seg_flush(sk, sv, scount < (uint32_t)STAGE ? scount : (uint32_t)STAGE, seg, segcnt, ok, ov,
              segcap, &sbase);
  }
  if (rng_err) atomicOr(&ctrl->flags, F_RNG);
  if (int_ovf) atomicOr(&ctrl->flags, F_INT_OVF);
}

// Records of solves entering the list this step (serving admissions).
template <typename K>
__global__ void k_inject(const K *__restrict__ ik, const int2 *__restrict__ iv, Ctrl *ctrl,
                         K *__restrict__ ok, int2 *__restrict__ ov,
                         unsigned long long *segcnt, uint32_t segcap) {
  if (ctrl->abort) return;
  __shared__ uint32_t cnt;
  __shared__ unsigned long long base;
  if (threadIdx.x == 0) {
    cnt = ctrl->n_inject;
    base = cnt ? atomicAdd(&segcnt[0], (unsigned long long)cnt) : 0ull;
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < cnt; q += blockDim.x) {
    if (base + q < segcap) {
      ok[base + q] = ik[q];
      ov[base + q] = iv[q];
    }
  }
  // n_inject is cleared when the step commits (k_finalize): a step that fails
  // and is run again after the buffers grow injects the same records again
}

// ---- radix sort -------------------------------------------------------------
// One LSD pass over an 8-bit digit, reduce-then-scan: k_sort_count writes the
// digit counts of every tile (digit-major), k_sort_rowscan turns each digit's
// row into exclusive prefixes over the tiles (and records the row's total),
// and k_sort_pass ranks each tile in LDS and scatters it to (global start of
// the digit, from the totals) + (its row prefix).
// No tile waits on another.  Pass 0 reads the segmented spawn buffer
// (segcap > 0), later passes read a contiguous array (segcap == 0).
template <typename K, int SORT_IT>
__global__ __launch_bounds__(NT) void k_sort_count(const K *__restrict__ ik, Ctrl *ctrl,
                                                   uint32_t *__restrict__ cnt, int pass,
                                                   uint32_t segcap,
                                                   const unsigned long long *__restrict__ segcnt) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  __shared__ uint32_t h[256];
  __shared__ uint32_t pre[NSEG + 1];
  __shared__ unsigned long long s_over;
  if (pass == 0) {
    // the records' segment offsets (every block computes them; block 0 also
    // publishes them, the record count and a segment overflow for the later
    // kernels).  A segment's counter holds the records its step attempted,
    // which may exceed its capacity (then the step is redone with larger
    // buffers, and the offsets below are not used).
    if (threadIdx.x < NSEG) {
      const unsigned long long c64 = segcnt[threadIdx.x * SEG_STRIDE];
      const uint32_t c = c64 < segcap ? (uint32_t)c64 : segcap;
      const uint32_t inc = wave_incl_scan(c);
      pre[threadIdx.x] = inc - c;
      if (threadIdx.x == NSEG - 1) pre[NSEG] = inc;
      unsigned long long mx = c64;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
      }
      if (threadIdx.x == 0) s_over = mx > segcap ? mx : 0ull;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
      if (threadIdx.x <= NSEG) ctrl->seg_prefix[threadIdx.x] = pre[threadIdx.x];
      if (threadIdx.x == 0) {
        ctrl->n_spawn = pre[NSEG];
        if (s_over) {
          ctrl->seg_need = s_over;
          atomicOr(&ctrl->flags, F_SPAWN_CAP);
        }
      }
    }
    if (s_over) return;
  } else {
    if (threadIdx.x <= NSEG) pre[threadIdx.x] = ctrl->seg_prefix[threadIdx.x];
  }
  __syncthreads();
  constexpr uint32_t SORT_TILE = NT * SORT_IT;
  const uint32_t n = pre[NSEG];
  const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
  const uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  h[threadIdx.x] = 0;
  __syncthreads();
  const int shift = 8 * pass;
  // the thread's keys are all loaded before the first is counted
  K key[SORT_IT];
#pragma unroll
  for (int k = 0; k < SORT_IT; ++k) {
    const uint32_t pos = t * SORT_TILE + (uint32_t)k * NT + threadIdx.x;
    if (pos < n) key[k] = ik[segcap ? seg_addr(pre, pos, segcap) : (size_t)pos];
  }
#pragma unroll
  for (int k = 0; k < SORT_IT; ++k) {
    const uint32_t pos = t * SORT_TILE + (uint32_t)k * NT + threadIdx.x;
    if (pos < n) atomicAdd(&h[(uint32_t)((key[k] >> shift) & 255u)], 1u);
  }
  __syncthreads();
  cnt[(size_t)threadIdx.x * ntiles + t] = h[threadIdx.x];
}

// Exclusive prefix over the tiles of digit blockIdx.x's row of counts, in place;
// the row's total (the digit's count over all records) goes to
// hist[pass * 256 + digit].
__global__ __launch_bounds__(NT) void k_sort_rowscan(Ctrl *ctrl, uint32_t *cnt, uint32_t *hist,
                                                     int pass, uint32_t sort_tile) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  const uint32_t n = ctrl->n_spawn;
  const uint32_t ntiles = (n + sort_tile - 1) / sort_tile;
  if (ntiles == 0) {
    if (threadIdx.x == 0) hist[pass * 256 + blockIdx.x] = 0;
    return;
  }
  __shared__ uint32_t scan4[NT / 64];
  uint32_t *row = cnt + (size_t)blockIdx.x * ntiles;
  const uint32_t tot = block_prefix_inplace<NT>(row, ntiles, scan4);
  if (threadIdx.x == 0) hist[pass * 256 + blockIdx.x] = tot;
}

template <typename K, int SORT_IT>
__global__ __launch_bounds__(NT) void k_sort_pass(const K *__restrict__ ik,
                                                  const int2 *__restrict__ iv,
                                                  K *__restrict__ okk, int2 *__restrict__ ov,
                                                  Ctrl *ctrl, const uint32_t *__restrict__ hist,
                                                  const uint32_t *__restrict__ cnt, int pass,
                                                  uint32_t segcap) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  constexpr uint32_t SORT_TILE = NT * SORT_IT;
  const uint32_t n = ctrl->n_spawn;
  if (n == 0) return;
  const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
  const uint32_t t = blockIdx.x;
  if (t >= ntiles) return;
  const int shift = 8 * pass;

  __shared__ K tk[SORT_TILE];
  __shared__ int2 tv[SORT_TILE];
  __shared__ uint32_t wcnt[NT / 64][256];
  __shared__ uint32_t gstart[256], lstart[256], goff[256];
  __shared__ uint32_t scan4[NT / 64];
  __shared__ uint32_t pre[NSEG + 1];

  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  if (threadIdx.x <= NSEG) pre[threadIdx.x] = ctrl->seg_prefix[threadIdx.x];
  {
    uint32_t tot;
    const uint32_t h = hist[pass * 256 + threadIdx.x];
    gstart[threadIdx.x] = block_excl_scan(h, scan4, &tot);
  }
  // this tile's place for each digit: the digit's start plus the counts of the
  // digit in the tiles before
  goff[threadIdx.x] = gstart[threadIdx.x] + cnt[(size_t)threadIdx.x * ntiles + t];
  for (int i = threadIdx.x; i < (NT / 64) * 256; i += NT) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  {
    const uint32_t tbase = t * SORT_TILE;
    const uint32_t wbase = tbase + (uint32_t)w * 64u * SORT_IT;
    K key[SORT_IT];
    int2 val[SORT_IT];
    uint32_t rank[SORT_IT];
    // all of the lane's records are loaded before the first is ranked, so
    // that their loads are in flight together
#pragma unroll
    for (int k = 0; k < SORT_IT; ++k) {
      const uint32_t pos = wbase + (uint32_t)k * 64u + (uint32_t)lane;
      if (pos < n) {
        const size_t a = segcap ? seg_addr(pre, pos, segcap) : (size_t)pos;
        key[k] = ik[a];
        val[k] = iv[a];
      }
    }
#pragma unroll
    for (int k = 0; k < SORT_IT; ++k) {
      const uint32_t pos = wbase + (uint32_t)k * 64u + (uint32_t)lane;
      const bool valid = pos < n;
      const uint32_t d = valid ? (uint32_t)((key[k] >> shift) & 255u) : 0u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bb : ~bb;
      }
      if (valid) {
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t old = wcnt[w][d];
        rank[k] = old + below;
        __builtin_amdgcn_wave_barrier();
        if (below == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
      } else {
        __builtin_amdgcn_wave_barrier();
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: wave prefixes and the tile-local start
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int ww = 0; ww < NT / 64; ++ww) {
      const uint32_t x = wcnt[ww][d];
      wcnt[ww][d] = c;
      c += x;
    }
    uint32_t tot;
    lstart[d] = block_excl_scan(c, scan4, &tot);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_IT; ++k) {
      const uint32_t pos = wbase + (uint32_t)k * 64u + (uint32_t)lane;
      if (pos < n) {
        const uint32_t dd = (uint32_t)((key[k] >> shift) & 255u);
        const uint32_t lp = lstart[dd] + wcnt[w][dd] + rank[k];
        tk[lp] = key[k];
        tv[lp] = val[k];
      }
    }
    __syncthreads();
    const uint32_t tn = (n - tbase) < (uint32_t)SORT_TILE ? (n - tbase) : (uint32_t)SORT_TILE;
    for (uint32_t q = threadIdx.x; q < tn; q += NT) {
      const K kq = tk[q];
      const uint32_t dd = (uint32_t)((kq >> shift) & 255u);
      const uint32_t g = goff[dd] + (q - lstart[dd]);
      okk[g] = kq;
      ov[g] = tv[q];
    }
  }
}

// ---- merge ----------------------------------------------------------------
// Sum of a run of records: all of them, and those from initiator parents.
struct RunSum {
  int64_t aR, aI, iR, iI;
};
// (selects rather than branches, so the sums stay in registers)
__device__ __forceinline__ void run_add(RunSum &s, int2 v) {
  const bool nx = v.x == NON_INIT;         // non-initiator record, imaginary part only
  const bool ny = !nx && v.y == NON_INIT;  // non-initiator record, real part only
  const int64_t x = nx ? 0 : (int64_t)v.x;
  const int64_t y = ny ? 0 : (int64_t)v.y;
  const bool ini = !nx && !ny;
  s.aR += x;
  s.aI += y;
  s.iR += ini ? x : 0;
  s.iI += ini ? y : 0;
}

// Tile boundaries of the merge: part[t] = A elements among the first t*TILE of
// the merged sequence (all tiles in parallel; the merge reads them).
template <typename K>
__global__ __launch_bounds__(NT) void k_merge_partition(const K *__restrict__ Ak,
                                                        const K *__restrict__ Bk, Ctrl *ctrl,
                                                        uint32_t *__restrict__ part,
                                                        uint32_t merge_tile) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  const uint32_t na = ctrl->n_main, nb = ctrl->n_spawn;
  const uint32_t total = na + nb;
  const uint32_t ntiles = (total + merge_tile - 1) / merge_tile;
  for (uint32_t t = blockIdx.x * NT + threadIdx.x; t <= ntiles; t += gridDim.x * NT) {
    const uint32_t d = t * merge_tile < total ? t * merge_tile : total;
    part[t] = merge_path(Ak, na, Bk, nb, d);
  }
}

// Merge of the step-start list A (unique keys) with the sorted records B (runs
// of equal keys).  Every key of A gets its post-step value A + (sum of its run);
// a run without a key in A becomes a new entry with the sum of all its records
// if the configuration is diagonal, else of its initiator records only
// (Sec. IV.A).  Empty entries are dropped, the rest compacted in order.
// Two launches over the same tiles (the merge path cut into MERGE_TILE merged
// positions): COUNT writes each tile's number of survivors, k_merge_offsets
// turns them into output offsets, WRITE stores the survivors there and the
// tile's estimator sums.  Both decide survival with the same code, so their
// counts agree; no tile waits on another.
// Inside a tile, the runs whose first record lies in the tile are summed once
// (one thread per record, the run's head does the work): a run on an occupied
// configuration patches that entry, any other run becomes a candidate entry.
// The entry that ends a tile and whose run starts in the next one is patched
// by the tile that holds the entry.  The write pass then walks the merged
// order with two compares per position and sums the estimators over the
// compacted survivors.
// Tiles per CU: with 32-bit keys and 2048 positions a count tile's LDS is
// 27 KB and six fit; a write tile also holds the survivors' places (31 KB) and
// five fit, at 74 VGPRs.  (The write pass used to stage the survivors' keys
// and values in registers: at the bound's 96 VGPRs it spilled 76 bytes a
// lane, and its launch took 139 instead of 102 us on the 4x4 step.  A count
// pass that read the record values from HBM, with 10 KB of LDS and eight
// tiles per CU, was slower too: 88 against 70 us.)  With 64-bit keys and 2048
// positions the write tile's 39 KB allow four.
template <typename K, bool WRITE, int MERGE_IT>
__global__ __launch_bounds__(NT, sizeof(K) == 4 ? (MERGE_IT == 4 ? 8 : 5) : (MERGE_IT == 4 ? 6 : 4)) void k_merge(
    const K *__restrict__ Ak, const int2 *__restrict__ Av, const K *__restrict__ Bk,
    const int2 *__restrict__ Bv, K *__restrict__ Ck, int2 *__restrict__ Cv, uint32_t capC,
    Ctrl *ctrl, const SlotParams *__restrict__ sp, const SlotState *__restrict__ ss,
    unsigned long long *__restrict__ spill,
    uint32_t *__restrict__ tile_cnt, const uint32_t *__restrict__ part, int SB) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  constexpr uint32_t MERGE_TILE = NT * MERGE_IT;
  const uint32_t na = ctrl->n_main;
  const uint32_t nb = ctrl->n_spawn;
  const uint32_t total = na + nb;
  const uint32_t ntiles = (total + MERGE_TILE - 1) / MERGE_TILE;
  const K lowm = low_mask<K>(SB);

  // A tile holds nA entries and nB records with nA + nB <= MERGE_TILE: both
  // live in one set of arrays, the entries first, the records after them
  // (half the LDS of separate arrays, so more tiles per CU).
  __shared__ K sK[MERGE_TILE];
  __shared__ int2 sV[MERGE_TILE];
  __shared__ uint8_t sF[MERGE_TILE];  // entries: annihilated by their records;
                                      // records: run heads that become new entries
  __shared__ uint16_t sIdx[WRITE ? MERGE_TILE : 1];  // survivors' places in sK / sV, in order
  __shared__ uint32_t s_i0, s_i1;
  __shared__ K s_aprev, s_bprev, s_bnext;  // the keys just outside the tile
  __shared__ uint32_t scan4[NT / 64];
  __shared__ int64_t red[WRITE ? NT / 64 : 1][S_NSUM];
  bool int_ovf = false;

  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    __syncthreads();
    const uint32_t d0 = t * MERGE_TILE;
    const uint32_t d1 = (d0 + MERGE_TILE < total) ? d0 + MERGE_TILE : total;
    if (threadIdx.x == 0) s_i0 = part[t];
    if (threadIdx.x == 64) s_i1 = part[t + 1];
    __syncthreads();
    const uint32_t i0 = s_i0, i1 = s_i1, j0 = d0 - i0, j1 = d1 - i1;
    // the cuts of a sorted list and sorted records are monotone; anything else
    // (a list whose order was broken) fails the step instead of being read
    if (i1 < i0 || i1 > na || i0 > d0 || i1 > d1 || j1 < j0 || j1 > nb) {
      if (threadIdx.x == 0) {
        atomicOr(&ctrl->flags, F_ORDER);
        if (!WRITE) tile_cnt[t] = 0;
      }
      continue;
    }
    const uint32_t nA = i1 - i0, nB = j1 - j0;
    K *const sAk = sK, *const sBk = sK + nA;
    int2 *const sAv = sV, *const sBv = sV + nA;
    uint8_t *const sAdel = sF, *const sBout = sF + nA;
    for (uint32_t q = threadIdx.x; q < nA; q += NT) {
      sAk[q] = Ak[i0 + q];
      if (WRITE) sAv[q] = Av[i0 + q];
      sAdel[q] = 0;
    }
    for (uint32_t q = threadIdx.x; q < nB; q += NT) {
      sBk[q] = Bk[j0 + q];
      sBv[q] = Bv[j0 + q];
    }
    if (threadIdx.x == NT - 1) {
      s_aprev = i0 > 0 ? Ak[i0 - 1] : (K)0;
      s_bprev = j0 > 0 ? Bk[j0 - 1] : (K)0;
      s_bnext = j1 < nb ? Bk[j1] : (K)0;
    }
    __syncthreads();
    // keys and values by global record index; callers pass indices < nb
    auto bkey = [&](uint32_t j) -> K {
      if (j >= j0 && j < j1) return sBk[j - j0];
      if (j == j1) return s_bnext;
      return Bk[j];
    };
    auto bval = [&](uint32_t j) -> int2 { return (j >= j0 && j < j1) ? sBv[j - j0] : Bv[j]; };
    // the run of key k from record j on, whose first value v0 the caller read
    auto run_from = [&](uint32_t j, K k, int2 v0) -> RunSum {
      RunSum s{0, 0, 0, 0};
      run_add(s, v0);
      for (++j; j < nb && bkey(j) == k; ++j) run_add(s, bval(j));
      return s;
    };
    // the tile's first solve: its parameters once, in registers
    const uint32_t s0 = slot_of<K>((nA > 0 && (nB == 0 || sAk[0] <= sBk[0])) ? sAk[0] : sBk[0], SB);
    const SlotParams P0 = sp[s0];
    const bool leaving0 = ss[s0].status == 3;
    auto leaving = [&](uint32_t slot) { return slot == s0 ? leaving0 : ss[slot].status == 3; };
    auto ket_bra = [&](K k, uint32_t N, uint32_t &l, uint32_t &m) {
      const uint64_t cfg = (uint64_t)(k & lowm);
      l = (uint32_t)(cfg >> N);
      m = (uint32_t)(cfg & ((N == 32) ? 0xffffffffull : ((1ull << N) - 1)));
    };
    auto fits = [](int64_t R, int64_t I) {
      return R <= 2147483647LL && R >= -2147483647LL && I <= 2147483647LL && I >= -2147483647LL;
    };
    // an occupied entry (value av) and the sums of its run: annihilated, or
    // its new value
    auto patch = [&](uint32_t p, int2 av, const RunSum &rs) {
      const int64_t R = (int64_t)av.x + rs.aR;
      const int64_t I = (int64_t)av.y + rs.aI;
      if (R == 0 && I == 0) {
        sAdel[p] = 1;
      } else if (WRITE) {
        if (!fits(R, I)) int_ovf = true;
        sAv[p] = make_int2((int)R, (int)I);
      }
    };

    // runs whose first record is in this tile
    for (uint32_t j = threadIdx.x; j < nB; j += NT) {
      const K k = sBk[j];
      const uint32_t gj = j0 + j;
      const bool head = j > 0 ? sBk[j - 1] != k : (gj == 0 || s_bprev != k);
      uint8_t out = 0;
      // an entry right before the tile with this key already took the run
      if (head && !(i0 > 0 && s_aprev == k)) {
        const int2 v0 = sBv[j];
        const uint32_t p = lower_bound(sAk, nA, k);
        const bool hit = p < nA && sAk[p] == k;
        const int2 av = !hit ? make_int2(0, 0) : WRITE ? sAv[p] : Av[i0 + p];
        const RunSum rs = run_from(gj, k, v0);
        if (hit) {
          patch(p, av, rs);
        } else {
          const uint32_t slot = slot_of<K>(k, SB);
          uint32_t l, m;
          ket_bra(k, slot == s0 ? P0.N : sp[slot].N, l, m);
          // new configuration: every record if diagonal, else initiator records only
          const int64_t R = (l == m) ? rs.aR : rs.iR;
          const int64_t I = (l == m) ? rs.aI : rs.iI;
          if ((R != 0 || I != 0) && !leaving(slot)) {
            out = 1;
            if (WRITE) {
              if (!fits(R, I)) int_ovf = true;
              sBv[j] = make_int2((int)R, (int)I);
            }
          }
        }
      }
      sBout[j] = out;
    }
    // the tile's last entry, when its run starts right after the tile
    if (threadIdx.x == 0 && nA > 0 && j1 < nb && s_bnext == sAk[nA - 1] &&
        (nB == 0 || sBk[nB - 1] != s_bnext))
      patch(nA - 1, WRITE ? sAv[nA - 1] : Av[i0 + nA - 1], run_from(j1, s_bnext, Bv[j1]));
    __syncthreads();

    if (!WRITE) {
      uint32_t c = 0;
      for (uint32_t q = threadIdx.x; q < nA; q += NT)
        c += (!sAdel[q] && !leaving(slot_of<K>(sAk[q], SB))) ? 1u : 0u;
      for (uint32_t q = threadIdx.x; q < nB; q += NT) c += sBout[q];
      const uint32_t v = wave_sum(c);
      if ((threadIdx.x & 63) == 0) scan4[threadIdx.x >> 6] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += scan4[w];
        tile_cnt[t] = s;
      }
      continue;
    }

    // this thread's merged positions [dd, dd + MERGE_IT): survivors in order
    const uint32_t len = nA + nB;
    const uint32_t dd = (uint32_t)threadIdx.x * MERGE_IT < len ? (uint32_t)threadIdx.x * MERGE_IT
                                                               : len;
    uint32_t a, b;
    {
      uint32_t lo = dd > nB ? dd - nB : 0, hi = dd < nA ? dd : nA;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sAk[mid] <= sBk[dd - 1 - mid])
          lo = mid + 1;
        else
          hi = mid;
      }
      a = lo;
      b = dd - lo;
    }
    // each merged position's place in sK / sV (entries at a, records at
    // nA + b < MERGE_TILE), 16 bits each, two to a register, and a mask of
    // the survivors
    static_assert(MERGE_IT % 2 == 0 && NT * MERGE_IT <= 65536, "16-bit places");
    uint32_t src[MERGE_IT / 2];
#pragma unroll
    for (int i = 0; i < MERGE_IT / 2; ++i) src[i] = 0;
    uint32_t okm = 0, nsurv = 0;
#pragma unroll
    for (int it = 0; it < MERGE_IT; ++it) {
      if (dd + (uint32_t)it >= len) continue;
      uint32_t at;
      bool ok;
      if (a < nA && (b >= nB || sAk[a] <= sBk[b])) {
        ok = !sAdel[a] && !leaving(slot_of<K>(sAk[a], SB));
        at = a;
        ++a;
      } else {
        ok = sBout[b] != 0;
        at = nA + b;
        ++b;
      }
      src[it >> 1] |= at << (16 * (it & 1));
      if (ok) {
        okm |= 1u << it;
        ++nsurv;
      }
    }
    uint32_t ttot;
    const uint32_t lpos = block_excl_scan(nsurv, scan4, &ttot);
    const uint32_t gbase = tile_cnt[t];
    // the survivors' places in merged order, then the barrier (sK and sV
    // stay as they are)
    {
      uint32_t q = lpos;
#pragma unroll
      for (int it = 0; it < MERGE_IT; ++it)
        if (okm & (1u << it)) {
          sIdx[q] = (uint16_t)(src[it >> 1] >> (16 * (it & 1)));
          ++q;
        }
    }
    __syncthreads();
    // write them coalesced, and their estimator sums (Sec. III.A, V.A)
    int64_t acc[S_NSUM];
#pragma unroll
    for (int s = 0; s < S_NSUM; ++s) acc[s] = 0;
    for (uint32_t q = threadIdx.x; q < ttot; q += NT) {
      const uint32_t at = sIdx[q];
      const K k = sK[at];
      const int2 v = sV[at];
      const uint32_t g = gbase + q;
      if (g < capC) {
        Ck[g] = k;
        Cv[g] = v;
      }
      const uint32_t slot = slot_of<K>(k, SB);
      uint32_t l, m;
      if (slot == s0) {
        ket_bra(k, P0.N, l, m);
        entry_sums(P0, l, m, v.x, v.y, [&](int s, int64_t x) { acc[s] += x; });
      } else {
        const SlotParams &P = sp[slot];
        ket_bra(k, P.N, l, m);
        unsigned long long *const sums =
            spill + ((size_t)slot * SUM_BUCKETS + t % SUM_BUCKETS) * S_NSUM;
        entry_sums(P, l, m, v.x, v.y, [&](int s, int64_t x) {
          if (x) atomicAdd(&sums[s], (unsigned long long)x);
        });
      }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < S_NSUM; ++s) {
      const int64_t v = wave_sum(acc[s]);
      if (lane == 0) red[w][s] = v;
    }
    __syncthreads();
    if (threadIdx.x < S_NSUM) {
      int64_t v = 0;
#pragma unroll
      for (int ww = 0; ww < NT / 64; ++ww) v += red[ww][threadIdx.x];
      if (v)
        atomicAdd(&spill[((size_t)s0 * SUM_BUCKETS + t % SUM_BUCKETS) * S_NSUM + threadIdx.x],
                  (unsigned long long)v);
    }
  }
  if (int_ovf) atomicOr(&ctrl->flags, F_INT_OVF);
}

// Output offsets of the merge tiles, in place: cnt[t] <- survivors of tiles
// < t; the new list size goes to ctrl->n_new.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void k_merge_offsets(Ctrl *ctrl, uint32_t *cnt,
                                                       uint32_t merge_tile) {
  if (ctrl->abort || (ctrl->flags & F_SPAWN_CAP)) return;
  __shared__ uint32_t wsum[16];
  const uint32_t total = ctrl->n_main + ctrl->n_spawn;
  const uint32_t n = (total + merge_tile - 1) / merge_tile;
  const uint32_t all = block_prefix_inplace<1024>(cnt, n, wsum);
  if (threadIdx.x == 0) ctrl->n_new = all;
}

// ---- finalize (one block) ---------------------------------------------------
__global__ __launch_bounds__(1024) void k_finalize(Ctrl *ctrl, const SlotParams *__restrict__ sp,
                                                   SlotState *ss, unsigned long long *spill,
                                                   int nslots,
                                                   uint32_t *hist, int passes, uint32_t capC,
                                                   unsigned long long *segcnt, int64_t *series,
                                                   uint32_t *counts, uint32_t series_cap,
                                                   uint32_t merge_tile) {
  if (ctrl->abort) return;
  __shared__ unsigned long long sums[MAX_SLOTS * S_NSUM];
  __shared__ uint32_t s_bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  // a spawn overflow means the merge did not run: its sums are not valid
  if (ctrl->flags & F_SPAWN_CAP) {
    if (tid == 0) {
      ctrl->fail_flags = ctrl->flags | F_SPAWN_CAP;
      ctrl->abort = 1;
    }
    return;
  }
  for (int i = tid; i < nslots * S_NSUM; i += nt) sums[i] = 0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  // every solve's buckets (a thread per bucket), cleared for the next step
  for (int i = tid; i < nslots * SUM_BUCKETS; i += nt) {
    unsigned long long *const b = spill + (size_t)i * S_NSUM;
    unsigned long long v[S_NSUM];
#pragma unroll
    for (int k = 0; k < S_NSUM; ++k) v[k] = b[k];
#pragma unroll
    for (int k = 0; k < S_NSUM; ++k) {
      b[k] = 0;
      if (v[k]) atomicAdd(&sums[(i / SUM_BUCKETS) * S_NSUM + k], v[k]);
    }
  }
  __syncthreads();
  const uint32_t total = ctrl->n_main + ctrl->n_spawn;
  const uint32_t ntiles = (total + merge_tile - 1) / merge_tile;
  uint32_t flags = ctrl->flags;
  const uint32_t n_new = ntiles ? ctrl->n_new : 0u;
  if (n_new > capC) flags |= F_MAIN_CAP;
  // extinction check before anything is committed
  for (int s = tid; s < nslots; s += nt) {
    const SlotState &st = ss[s];
    if (st.status != 1) continue;
    const int64_t nw = (int64_t)sums[s * S_NSUM + S_NW];
    const int64_t ne = (int64_t)sums[s * S_NSUM + S_NENT];
    bool bad = (ne == 0);
    if (st.mode == 1 && (nw == 0 || st.nw_prev == 0)) bad = true;
    if (bad) {
      atomicOr(&s_bad, 1u);
      ctrl->extinct_slot = (uint32_t)s;
    }
  }
  __syncthreads();
  if (s_bad) flags |= F_EXTINCT;
  if (flags) {
    if (tid == 0) {
      ctrl->fail_flags = flags;
      ctrl->abort = 1;
    }
    return;
  }
  const uint32_t row = ctrl->series_pos;
  for (int s = tid; s < nslots; s += nt) {
    SlotState st = ss[s];
    const SlotParams &P = sp[s];
    int64_t v[S_NSUM];
    for (int i = 0; i < S_NSUM; ++i) v[i] = (int64_t)sums[s * S_NSUM + i];
    if (row < series_cap && st.status != 1) series[((size_t)row * nslots + s) * SERIES_W] = -1;
    if (st.status == 0) continue;
    if (st.status == 3) {
      st.status = 0;
      ss[s] = st;
      continue;
    }
    if (st.status == 2) {  // entered this step: its step 0
      st.status = 1;
      st.step = 0;
      st.S = P.shift_init;
      st.mode = 0;
      st.nw_prev = v[S_NW];
      st.n_accum = 0;
      for (int i = 0; i < S_NSUM; ++i) {
        st.last[i] = v[i];
        st.acc[i] = 0;
      }
      ss[s] = st;
      continue;
    }
    const int64_t nw = v[S_NW];
    if (st.mode == 0) {
      if (nw >= P.target) st.mode = 1;
    } else {
      st.S = st.S + P.delta_over_dt * dlog((double)nw / (double)st.nw_prev);
    }
    st.nw_prev = nw;
    st.step += 1;
    for (int i = 0; i < S_NSUM; ++i) st.last[i] = v[i];
    if (st.step > P.n_equil) {
      for (int i = 0; i < S_NSUM; ++i) st.acc[i] += v[i];
      st.n_accum += 1;
    }
    ss[s] = st;
    if (row < series_cap) {
      int64_t *r = series + ((size_t)row * nslots + s) * SERIES_W;
      r[0] = st.step;
      r[1] = __builtin_bit_cast(int64_t, st.S);
      r[2] = st.mode;
      for (int i = 0; i < S_NSUM; ++i) r[3 + i] = v[i];
    }
  }
  for (int i = tid; i < passes * 256; i += nt) hist[i] = 0;
  for (int i = tid; i < NSEG; i += nt) segcnt[i * SEG_STRIDE] = 0;
  if (tid == 0) {
    if (row < series_cap) {
      counts[COUNT_W * row + 0] = ctrl->n_main;
      counts[COUNT_W * row + 1] = ctrl->n_spawn;
      counts[COUNT_W * row + 2] = n_new;
      counts[COUNT_W * row + 3] = ctrl->n_loud;
      counts[COUNT_W * row + 4] = ctrl->n_heavy + ctrl->n_late;
    }
    ctrl->n_main = n_new;
    ctrl->last_spawn = ctrl->n_spawn;
    ctrl->n_spawn = 0;
    ctrl->n_inject = 0;
    ctrl->n_heavy = 0;
    ctrl->n_late = 0;
    ctrl->n_loud = 0;
    ctrl->loud_next = 0;
    ctrl->epoch += 1;
    ctrl->committed += 1;
    ctrl->series_pos = row + 1;
  }
}

// After a failed step: re-arm the counters (the list is untouched).
__global__ void k_rearm(Ctrl *ctrl, uint32_t *hist, int passes, unsigned long long *spill,
                        int nspill, unsigned long long *segcnt) {
  for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) hist[i] = 0;
  for (int i = threadIdx.x; i < nspill; i += blockDim.x) spill[i] = 0;
  for (int i = threadIdx.x; i < NSEG; i += blockDim.x) segcnt[i * SEG_STRIDE] = 0;
  if (threadIdx.x == 0) {
    ctrl->n_spawn = 0;
    ctrl->n_heavy = 0;
    ctrl->n_late = 0;
    ctrl->n_loud = 0;
    ctrl->loud_next = 0;
    ctrl->n_new = 0;
    ctrl->flags = 0;
    ctrl->abort = 0;
    ctrl->epoch += 1;
  }
}

// Start of a chunk of steps: the host reads these two counters at its end.
__global__ void k_chunk_begin(Ctrl *ctrl) {
  ctrl->committed = 0;
  ctrl->series_pos = 0;
}

// ---- self-check kernels ---------------------------------------------------
__global__ void k_dev_uniforms(uint64_t seed, uint32_t solve, uint64_t cfg, uint32_t step,
                               uint32_t draw, int64_t count, double *out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Stream st(seed, solve, cfg, step, draw, nullptr);
    for (int64_t i = 0; i < count; ++i) out[i] = st.next();
  }
}

// Fill count words with v (a kernel rather than a memset, so that a captured
// sequence holds no memset node).
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint32_t count) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_dev_binom(int64_t n, double p, int mode, uint64_t seed, int64_t count,
                            int64_t *out, int *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int e = 0;
  Stream st(seed, 0, (uint64_t)i, 0, 1, &e);
  int64_t x;
  if (mode == 0)
    x = binomial(n, p, st);
  else if (mode == 1)
    x = binomial_positive(n, p, st);
  else
    x = binomial_split(n, p, st);
  out[i] = x;
  if (e) atomicOr(err, 1);
}

__global__ void k_dev_quiet(const double *p4, const int64_t *n2, const double *u, int64_t count,
                            int32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double p8[8];
  int64_t n8[8];
  for (int k = 0; k < 4; ++k) {
    p8[k] = p8[k + 4] = p4[4 * i + k];
    n8[k] = n2[2 * i];
    n8[k + 4] = n2[2 * i + 1];
  }
  out[i] = quiet_test(p8, n8, u[i]);
}

__global__ void k_dev_math(const double *x, int64_t count, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double v = x[i];
  out[4 * i + 0] = dlog(v);
  out[4 * i + 1] = dexp(v);
  out[4 * i + 2] = __builtin_sqrt(v);
  out[4 * i + 3] = 1.0 / v;
}

}  // namespace ddqmc
