// C ABI of the DDQMC step library (declared in include/ddqmc.h).
//
// A handle owns a sorted walker list (two ping-pong buffers), the spawn-record
// buffers of the radix sort and its tile counts, the estimator sums per solve
// and the per-solve parameter/state tables.  One step is a fixed sequence of
// launches on the handle's stream (kernels.hpp); the host synchronises only at
// the end of a chunk of steps, reads the control block and, if a buffer was too
// small, grows it and redoes the failed step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ddqmc.h"
#include "kernels.hpp"

using namespace ddqmc;

// Scratch of ddqmc_dev_binom_noalloc, the variant of ddqmc_dev_binom for
// callers that cannot allocate device memory: a 256-byte header (the error
// flag) and room for NOALLOC_MAX_SAMPLES int64 samples.  Every GPU the library
// runs on holds its own copy for the life of the process.  Host code never
// passes this name to a kernel (on the host it is only a stand-in for the
// symbol): it uses the device address that hipGetSymbolAddress returns, kept
// per device in noalloc_scratch().
constexpr int64_t NOALLOC_MAX_SAMPLES = 1 << 20;
constexpr size_t NOALLOC_HEADER = 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_HEADER + NOALLOC_MAX_SAMPLES * 8];

namespace {

constexpr uint32_t SERIES_CAP = 1024;  // steps per chunk between host synchronisations
// Largest list or spawn buffer, in entries: list + records stay below 2^32, so
// every 32-bit count and index in the kernels is exact.
constexpr uint64_t MAX_CAP = 0x7FF00000ull;
constexpr uint64_t FORK_MIN_CAP = 1ull << 23;  // list capacity from which heavy runs beside loud
// stages: scan, gather, loud, heavy, seal, histogram, sort, count, merge, finalize
constexpr int NSTAGE = 10;
constexpr int STAGE_SEAL = 4, STAGE_HIST = 5, STAGE_SORT = 6;

struct StageEvents {
  hipEvent_t e[NSTAGE + 1];
};

}  // namespace

struct ddqmc_t {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int nslots = 1;
  int Nmax = 0;
  int SB = 0;       // bit position of the slot field
  int key_bits = 0;
  int passes = 1;
  bool k64 = false;
  bool pool = false;
  uint64_t cap_main = 0, cap_sp = 0;
  int cur = 0;
  uint32_t n_main_known = 0, n_spawn_known = 0;

  // Device memory, two arenas (fixed_layout, sized_layout): the fixed one holds
  // what depends on the slot count only, the sized one the lists and the
  // per-step scratch, replaced whole when a step outgrows it.  Both are one
  // allocation each, or pieces of a caller's workspace (ddqmc_create_in).
  char *fixed = nullptr, *sized = nullptr;
  size_t fixed_bytes = 0, sized_bytes = 0;
  bool own_mem = true;     // false: in a caller's workspace, which is never regrown
  uint64_t cap_limit = 0;  // largest capacity growth may reach (0: MAX_CAP)

  void *mk[2] = {nullptr, nullptr};
  int2 *mv[2] = {nullptr, nullptr};
  void *sk[2] = {nullptr, nullptr};
  int2 *sv[2] = {nullptr, nullptr};
  uint32_t *sort_cnt = nullptr;  // sort: digit counts of the tiles, then their prefixes
  uint32_t *tile_cnt = nullptr;  // merge: survivors per tile, then offsets
  uint32_t *hist = nullptr;
  Ctrl *ctrl = nullptr;
  SlotParams *dsp = nullptr;
  SlotState *dss = nullptr;
  unsigned long long *spill = nullptr;
  int64_t *series = nullptr;
  uint32_t *counts = nullptr;  // per step: entries in, records, entries out, loud, heavy
  uint32_t *heavy = nullptr;     // loud entries that need the general sampling code (scan)
  uint32_t *late = nullptr;      // loud entries the light path passed on (loud kernel)
  uint32_t *lidx = nullptr;      // loud list (entries with some event): index, key, value
  void *lkey = nullptr;
  int2 *lval = nullptr;
  uint32_t *part = nullptr;      // merge tile boundaries
  unsigned long long *segcnt = nullptr;  // record counters of the spawn segments
  uint32_t nscan = 1;          // blocks of the scan kernel (fixed per list capacity)
  uint32_t loud_blocks = 1024;   // blocks of the loud spawn kernel the device holds at once
  uint32_t heavy_blocks = 1024;  // one-wave blocks of the heavy spawn kernel, likewise
  void *inj_k = nullptr;
  int2 *inj_v = nullptr;
  uint32_t n_inject_host = 0;

  std::vector<SlotParams> hp;
  std::vector<ddqmc_params> up;
  std::vector<int> slot_state;  // host view: 0 free, 1 running, 2 entering, 3 leaving
  std::vector<std::vector<int64_t>> hseries;
  std::vector<int64_t> hcounts;

  // k-step HIP graphs, one per parity of the list the replay starts from,
  // captured again whenever a buffer has been reallocated
  int graph_k = 0;
  uint64_t buf_gen = 0;
  hipStream_t cap_stream = nullptr;
  // second stream: the scan's heavy entries are sampled on it while the loud
  // kernel runs on the main stream (fork and join by events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool fork_heavy = false;  // only for large lists: a fork and join cost more than
                            // the heavy kernel saves on a short step
  int fork_mode = 0;        // 0 by list capacity, 1 always, -1 never
  uint32_t tree_cap = 0;    // member-tree places per loud chunk (0: all the kernel holds)
  int field_limit = 20;     // spawns in one part that send a field entry to the general routine
  bool loud_dyn = false;    // loud kernel: resident blocks and a chunk counter (else a
                            // block per chunk); chosen per chunk of steps, see run_steps
  int loud_grid = 0;        // 0 chosen per chunk of steps, 1 resident, 2 block per chunk
  bool general = false;     // some solve has the in-plane field: the general spawn path
  bool all_field = false;   // every solve has it (a batch or solve made so; not a pool)
  bool per_walker = false;  // every solve samples walker by walker (the ablation path)
  uint32_t general_blocks = 1024;
  uint32_t ncu = 256;            // compute units of the device
  // tile shapes (records / merged positions per thread) of the sort and the
  // merge, and an optional table choosing them by list size before each chunk
  int sort_it = SORT_IT_DEFAULT, merge_it = MERGE_IT_DEFAULT;
  struct TileRow {
    int64_t min_entries;
    int sort_it, merge_it;
  };
  std::vector<TileRow> tile_table;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  uint64_t gexec_gen[2] = {~0ull, ~0ull};
  int gexec_k[2] = {0, 0};

  bool profiling = false;
  int prof_every = 1;  // stage events on every prof_every-th step of a chunk
  std::vector<StageEvents> ev;
  double stage_ms[NSTAGE] = {};
  int64_t stage_steps = 0;
};

namespace {

int hip_err(hipError_t e) {
  if (e == hipSuccess) return DDQMC_OK;
  if (e == hipErrorOutOfMemory) return DDQMC_ENOMEM;
  std::fprintf(stderr, "ddqmc: HIP error %s\n", hipGetErrorString(e));
  return DDQMC_EHIP;
}

#define HIPC(x)                           \
  do {                                    \
    const hipError_t e_ = (x);            \
    if (e_ != hipSuccess) return hip_err(e_); \
  } while (0)

size_t key_size(const ddqmc_t *h) { return h->k64 ? 8 : 4; }

// (the tile arrays are laid out for the smallest tiles, so every shape fits)
uint64_t sort_tiles(uint64_t cap) { return (cap + MIN_SORT_TILE - 1) / MIN_SORT_TILE; }
uint64_t merge_tiles(uint64_t a, uint64_t b) { return (a + b + MIN_MERGE_TILE - 1) / MIN_MERGE_TILE; }
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the fixed arena's buffers (each 256-byte aligned).
struct FixedLayout {
  size_t ctrl, dsp, dss, spill, series, counts, inj_k, inj_v, segcnt, hist, total;
};
FixedLayout fixed_layout(int nslots, size_t ks) {
  FixedLayout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += al256(bytes);
    return at;
  };
  L.ctrl = take(sizeof(Ctrl));
  L.dsp = take((size_t)nslots * sizeof(SlotParams));
  L.dss = take((size_t)nslots * sizeof(SlotState));
  L.spill = take((size_t)nslots * SUM_BUCKETS * S_NSUM * sizeof(unsigned long long));
  L.series = take((size_t)SERIES_CAP * nslots * SERIES_W * sizeof(int64_t));
  L.counts = take((size_t)SERIES_CAP * COUNT_W * sizeof(uint32_t));
  L.inj_k = take((size_t)nslots * ks);
  L.inj_v = take((size_t)nslots * sizeof(int2));
  L.segcnt = take((size_t)NSEG * SEG_STRIDE * sizeof(unsigned long long));
  L.hist = take((size_t)MAX_PASSES * 256 * sizeof(uint32_t));
  L.total = o;
  return L;
}

// Byte offsets of the sized arena's buffers for a list capacity cap_main and a
// record capacity cap_sp (rounded up to whole segments).
struct SizedLayout {
  uint64_t cap_main, cap_sp;
  size_t mk[2], mv[2], sk[2], sv[2], sort_cnt, tile_cnt, part;
  size_t heavy, late, lidx, lkey, lval, total;
};
SizedLayout sized_layout(size_t ks, uint64_t cap_main, uint64_t cap_sp) {
  SizedLayout L;
  cap_sp = (cap_sp + NSEG - 1) / NSEG * NSEG;
  L.cap_main = cap_main;
  L.cap_sp = cap_sp;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += al256(bytes);
    return at;
  };
  for (int b = 0; b < 2; ++b) {  // the walker list, two ping-pong buffers
    L.mk[b] = take(cap_main * ks);
    L.mv[b] = take(cap_main * sizeof(int2));
  }
  for (int b = 0; b < 2; ++b) {  // spawn records: segments, then the sort's second buffer
    L.sk[b] = take(cap_sp * ks);
    L.sv[b] = take(cap_sp * sizeof(int2));
  }
  L.sort_cnt = take(sort_tiles(cap_sp) * 256 * sizeof(uint32_t));
  const uint64_t t = merge_tiles(cap_main, cap_sp);
  L.tile_cnt = take((t + 1) * sizeof(uint32_t));
  L.part = take((t + 1) * sizeof(uint32_t));
  // the loud list (index, key, value) and the two heavy queues: at most one
  // place per list entry each
  L.heavy = take(cap_main * sizeof(uint32_t));
  L.late = take(cap_main * sizeof(uint32_t));
  L.lidx = take(cap_main * sizeof(uint32_t));
  L.lkey = take(cap_main * ks);
  L.lval = take(cap_main * sizeof(int2));
  L.total = o;
  return L;
}

// Capacities of a new handle: the list as asked (at least 4096 entries, at
// most MAX_CAP), records a quarter of that (at least 4096).
void initial_caps(uint64_t cap, uint64_t *cap_main, uint64_t *cap_sp) {
  cap = std::min<uint64_t>(std::max<uint64_t>(cap, 4096), MAX_CAP);
  *cap_main = cap;
  *cap_sp = std::max<uint64_t>(4096, cap / 4);
}

// Reserve of device memory that growth must leave free: the runtime needs
// headroom for kernel scratch and queues, so that a list that outgrows the
// device ends as an error, not a fault.
uint64_t memory_reserve(uint64_t total_b) {
  return std::max<uint64_t>((uint64_t)4 << 30, total_b / 32);
}

int validate(const ddqmc_params *p) {
  if (!p || p->struct_size != sizeof(ddqmc_params)) return DDQMC_EINVAL;
  if (p->Lx < 2 || p->Ly < 2 || p->Lx * p->Ly > 32) return DDQMC_EINVAL;
  if (!(p->gamma > 0.0) || !(p->dt > 0.0) || p->n_a < 0 || !(p->is_p >= 0.0)) return DDQMC_EINVAL;
  if (!std::isfinite(p->Jx) || !std::isfinite(p->Jy) || !std::isfinite(p->Jz)) return DDQMC_EINVAL;
  if (p->initial_walkers <= 0 || p->initial_walkers > 2147483647LL) return DDQMC_EINVAL;
  if (p->solve_id >= 65536u || p->capacity_hint < 0 || p->n_equil < 0) return DDQMC_EINVAL;
  if (!std::isfinite(p->shift_damping) || !std::isfinite(p->shift_init)) return DDQMC_EINVAL;
  if (!std::isfinite(p->hx) || !std::isfinite(p->hy)) return DDQMC_EINVAL;
  if (p->flags & ~(DDQMC_NO_INITIATOR | DDQMC_PER_WALKER)) return DDQMC_EINVAL;
  if ((p->flags & DDQMC_PER_WALKER) && (p->hx != 0.0 || p->hy != 0.0)) return DDQMC_EINVAL;
  return DDQMC_OK;
}

// Lattice tables and constants of one solve.
SlotParams make_slot(const ddqmc_params &p) {
  SlotParams s;
  std::memset(&s, 0, sizeof(s));
  const uint32_t Lx = (uint32_t)p.Lx, Ly = (uint32_t)p.Ly, N = Lx * Ly;
  s.N = N;
  s.Lx = Lx;
  s.Ly = Ly;
  for (uint32_t site = 0; site < N; ++site) {
    const uint32_t x = site % Lx, y = site / Lx;
    if (Lx > 2 || x == 0) s.rmask |= 1u << site;
    if (Ly > 2 || y == 0) s.umask |= 1u << site;
    if (x == Lx - 1) s.col_last |= 1u << site;
    if (y == Ly - 1) s.row_last |= 1u << site;
  }
  s.nb = (uint32_t)(__builtin_popcount(s.rmask) + __builtin_popcount(s.umask));
  s.flags = p.flags;
  s.solve = p.solve_id;
  s.n_a = p.n_a;
  s.target = p.target_walkers;
  s.n_equil = p.n_equil;
  s.seed = p.seed;
  s.dt = p.dt;
  s.gamma = p.gamma;
  s.half_gamma = 0.5 * p.gamma;
  s.half_jz = 0.5 * p.Jz;
  s.h_al = (p.Jx - p.Jy) * 0.25;
  s.h_an = (p.Jx + p.Jy) * 0.25;
  s.a_al = std::fabs(s.h_al);
  s.a_an = std::fabs(s.h_an);
  s.w_dn = dexp(-p.is_p);
  s.w_up = dexp(p.is_p);
  s.delta_over_dt = p.shift_damping / p.dt;
  s.shift_init = p.shift_init;
  s.hx = p.hx;
  s.hy = p.hy;
  s.ahx = std::fabs(p.hx);
  s.ahy = std::fabs(p.hy);
  s.field = (p.hx != 0.0 || p.hy != 0.0) ? 1u : 0u;
  return s;
}

SlotState fresh_state(const ddqmc_params &p, int status) {
  SlotState st;
  std::memset(&st, 0, sizeof(st));
  st.S = p.shift_init;
  st.mode = 0;
  st.status = status;
  st.step = 0;
  st.nw_prev = p.initial_walkers;
  return st;
}

void free_all(ddqmc_t *h) {
  if (h->own_mem) {
    if (h->sized) (void)hipFree(h->sized);
    if (h->fixed) (void)hipFree(h->fixed);
  }
  h->sized = h->fixed = nullptr;
  for (int p = 0; p < 2; ++p)
    if (h->gexec[p]) (void)hipGraphExecDestroy(h->gexec[p]);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (auto &e : h->ev)
    for (int i = 0; i <= NSTAGE; ++i) (void)hipEventDestroy(e.e[i]);
  h->ev.clear();
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

uint32_t clampu(uint64_t v, uint32_t lo, uint32_t hi) {
  return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(v, lo), hi);
}

// Point the handle's buffers into a fixed arena at base.
void bind_fixed(ddqmc_t *h, char *base) {
  const FixedLayout L = fixed_layout(h->nslots, key_size(h));
  h->fixed = base;
  h->fixed_bytes = L.total;
  h->ctrl = (Ctrl *)(base + L.ctrl);
  h->dsp = (SlotParams *)(base + L.dsp);
  h->dss = (SlotState *)(base + L.dss);
  h->spill = (unsigned long long *)(base + L.spill);
  h->series = (int64_t *)(base + L.series);
  h->counts = (uint32_t *)(base + L.counts);
  h->inj_k = base + L.inj_k;
  h->inj_v = (int2 *)(base + L.inj_v);
  h->segcnt = (unsigned long long *)(base + L.segcnt);
  h->hist = (uint32_t *)(base + L.hist);
}

// Point the handle's buffers into a sized arena at base with layout L.
void bind_sized(ddqmc_t *h, char *base, const SizedLayout &L) {
  h->sized = base;
  h->sized_bytes = L.total;
  for (int b = 0; b < 2; ++b) {
    h->mk[b] = base + L.mk[b];
    h->mv[b] = (int2 *)(base + L.mv[b]);
    h->sk[b] = base + L.sk[b];
    h->sv[b] = (int2 *)(base + L.sv[b]);
  }
  h->sort_cnt = (uint32_t *)(base + L.sort_cnt);
  h->tile_cnt = (uint32_t *)(base + L.tile_cnt);
  h->part = (uint32_t *)(base + L.part);
  h->heavy = (uint32_t *)(base + L.heavy);
  h->late = (uint32_t *)(base + L.late);
  h->lidx = (uint32_t *)(base + L.lidx);
  h->lkey = base + L.lkey;
  h->lval = (int2 *)(base + L.lval);
  h->cap_main = L.cap_main;
  h->cap_sp = L.cap_sp;
  h->nscan = clampu((h->cap_main + NT - 1) / NT, 1, 4096);
  h->fork_heavy = h->fork_mode > 0 || (h->fork_mode == 0 && h->cap_main >= FORK_MIN_CAP);
}

// Largest list capacity whose handle fits in `bytes` (0 if not even the
// smallest one does).
uint64_t fit_capacity(int nslots, size_t ks, size_t bytes) {
  const size_t fixed = fixed_layout(nslots, ks).total;
  auto need = [&](uint64_t c) {
    uint64_t cm, cs;
    initial_caps(c, &cm, &cs);
    return fixed + sized_layout(ks, cm, cs).total;
  };
  if (need(4096) > bytes) return 0;
  uint64_t lo = 4096, hi = MAX_CAP;
  if (need(hi) <= bytes) return hi;
  while (hi - lo > 1) {  // need(lo) fits, need(hi) does not
    const uint64_t mid = lo + (hi - lo) / 2;
    (need(mid) <= bytes ? lo : hi) = mid;
  }
  return lo;
}

// Common construction: slots, key layout, buffers.  With ws == nullptr the
// arenas are allocated (hipMalloc) for a list capacity cap; else they are
// carved out of the caller's workspace [ws, ws + ws_bytes), with capacity cap
// if it is nonzero, else the largest that fits.
int build(ddqmc_t *h, int nslots, int Nmax, uint64_t cap, void *stream, void *ws = nullptr,
          size_t ws_bytes = 0) {
  if (nslots < 1 || nslots > MAX_SLOTS || Nmax < 4 || Nmax > 32) return DDQMC_EINVAL;
  if (ws && ((uintptr_t)ws & 255)) return DDQMC_EINVAL;
  HIPC(hipGetDevice(&h->device));
  if (stream) {
    h->stream = (hipStream_t)stream;
  } else {
    HIPC(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  HIPC(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  HIPC(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming | hipEventReleaseToDevice));
  HIPC(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming | hipEventReleaseToDevice));
  h->nslots = nslots;
  h->Nmax = Nmax;
  h->SB = 2 * Nmax;
  int slot_bits = 0;
  while ((1 << slot_bits) < nslots) ++slot_bits;
  h->key_bits = h->SB + slot_bits;
  if (h->key_bits > 64) return DDQMC_EINVAL;
  h->k64 = h->key_bits > 32;
  {
    // the spawn kernels loop over their work: launch as many blocks as the
    // device runs at once, so that no block waits for a second round
    int ncu = 0, nl = 0, nh = 0;
    HIPC(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
    if (h->k64) {
      HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nl, reinterpret_cast<const void *>(&k_spawn_loud<uint64_t>), NT, 0));
      HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nh, reinterpret_cast<const void *>(&k_spawn_heavy<uint64_t, 1>), 64, 0));
    } else {
      HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nl, reinterpret_cast<const void *>(&k_spawn_loud<uint32_t>), NT, 0));
      HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nh, reinterpret_cast<const void *>(&k_spawn_heavy<uint32_t, 1>), 64, 0));
    }
    h->loud_blocks = clampu((uint64_t)std::max(ncu, 1) * (uint64_t)std::max(nl, 1), 1, 4096);
    h->heavy_blocks = clampu((uint64_t)std::max(ncu, 1) * (uint64_t)std::max(nh, 1), 1, 8192);
    h->general_blocks = clampu((uint64_t)std::max(ncu, 1) * 4, 1, 4096);
    h->ncu = clampu((uint64_t)std::max(ncu, 1), 1, 4096);
  }
  h->passes = (h->key_bits + 7) / 8;
  const size_t ks = key_size(h);
  const FixedLayout FL = fixed_layout(nslots, ks);
  if (ws) {
    h->own_mem = false;
    if (cap == 0) cap = fit_capacity(nslots, ks, ws_bytes);
    if (cap == 0) return DDQMC_ECAPACITY;
  }
  uint64_t cm, cs;
  initial_caps(cap, &cm, &cs);
  const SizedLayout SL = sized_layout(ks, cm, cs);
  char *fixed = nullptr, *sized = nullptr;
  if (ws) {
    if (FL.total + SL.total > ws_bytes) return DDQMC_ECAPACITY;
    fixed = (char *)ws;
    sized = fixed + FL.total;
  } else {
    size_t free_b = 0, total_b = 0;
    HIPC(hipMemGetInfo(&free_b, &total_b));
    if (FL.total + SL.total + memory_reserve(total_b) > free_b) return DDQMC_ENOMEM;
    HIPC(hipMalloc((void **)&fixed, FL.total));
    h->fixed = fixed;  // owned from here on (free_all)
    HIPC(hipMalloc((void **)&sized, SL.total));
  }
  bind_fixed(h, fixed);
  bind_sized(h, sized, SL);
  HIPC(hipMemsetAsync(h->fixed, 0, FL.total, h->stream));
  h->hp.assign(nslots, SlotParams{});
  h->up.assign(nslots, ddqmc_params{});
  h->slot_state.assign(nslots, 0);
  h->hseries.assign(nslots, {});
  return DDQMC_OK;
}

// Upload a sorted list (keys with slot bits) into the current buffer.
int upload_list(ddqmc_t *h, const std::vector<uint64_t> &keys, const std::vector<int2> &vals) {
  const size_t n = keys.size();
  if (n > h->cap_main) return DDQMC_ECAPACITY;
  if (n) {
    if (h->k64) {
      HIPC(hipMemcpyAsync(h->mk[h->cur], keys.data(), n * 8, hipMemcpyHostToDevice, h->stream));
    } else {
      std::vector<uint32_t> k32(keys.begin(), keys.end());
      HIPC(hipMemcpyAsync(h->mk[h->cur], k32.data(), n * 4, hipMemcpyHostToDevice, h->stream));
      HIPC(hipStreamSynchronize(h->stream));
    }
    HIPC(hipMemcpyAsync(h->mv[h->cur], vals.data(), n * sizeof(int2), hipMemcpyHostToDevice,
                        h->stream));
  }
  const uint32_t n32 = (uint32_t)n;
  HIPC(hipMemcpyAsync(&h->ctrl->n_main, &n32, sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
  HIPC(hipStreamSynchronize(h->stream));
  h->n_main_known = n32;
  return DDQMC_OK;
}

int download_list(ddqmc_t *h, std::vector<uint64_t> &keys, std::vector<int2> &vals) {
  HIPC(hipStreamSynchronize(h->stream));
  uint32_t n = 0;
  HIPC(hipMemcpy(&n, &h->ctrl->n_main, sizeof(uint32_t), hipMemcpyDeviceToHost));
  keys.resize(n);
  vals.resize(n);
  if (n) {
    if (h->k64) {
      HIPC(hipMemcpy(keys.data(), h->mk[h->cur], n * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<uint32_t> k32(n);
      HIPC(hipMemcpy(k32.data(), h->mk[h->cur], n * 4, hipMemcpyDeviceToHost));
      for (uint32_t i = 0; i < n; ++i) keys[i] = k32[i];
    }
    HIPC(hipMemcpy(vals.data(), h->mv[h->cur], n * sizeof(int2), hipMemcpyDeviceToHost));
  }
  h->n_main_known = n;
  return DDQMC_OK;
}


template <typename K>
int launch_step(ddqmc_t *h, int par, StageEvents *ev, hipStream_t s) {
  const K *ak = (const K *)h->mk[par];
  const int2 *av = h->mv[par];
  K *ck = (K *)h->mk[par ^ 1];
  int2 *cv = h->mv[par ^ 1];
  const uint32_t capC = (uint32_t)h->cap_main;
  const uint32_t segcap = (uint32_t)(h->cap_sp / NSEG);
  // grids from the capacities: every kernel loops over the device-side counts
  const uint32_t g_loud = h->loud_dyn ? clampu(h->nscan, 1, h->loud_blocks)
                                      : clampu((h->cap_main + NT - 1) / NT, 1, 8 * h->loud_blocks);
  const uint32_t g_heavy = h->heavy_blocks;
  const uint32_t sort_tile = (uint32_t)(NT * h->sort_it), merge_tile = (uint32_t)(NT * h->merge_it);
  const uint32_t g_s = clampu((h->cap_sp + sort_tile - 1) / sort_tile, 1, 1u << 24);
  const uint32_t g_m = clampu((h->cap_main + h->cap_sp + merge_tile - 1) / merge_tile, 1, 1u << 20);
  if (ev) HIPC(hipEventRecord(ev->e[0], s));
  Ctrl *c = h->ctrl;
  if (h->per_walker) {
    // walker by walker: the walkers' prefix over the list (in the loud value
    // buffer, 8 bytes per entry, and the heavy queue for the block offsets),
    // then one thread per walker (timed as the loud stage)
    if (ev) HIPC(hipEventRecord(ev->e[1], s));
    static_assert(sizeof(int2) == sizeof(unsigned long long), "one prefix per list entry");
    unsigned long long *pre = reinterpret_cast<unsigned long long *>(h->lval);
    unsigned long long *boff = reinterpret_cast<unsigned long long *>(h->heavy);
    k_pw_prefix<K><<<h->general_blocks, NT, 0, s>>>(ak, av, c, h->dss, pre, boff, h->SB);
    k_pw_scan<<<1, 1024, 0, s>>>(c, boff);
    if (ev) HIPC(hipEventRecord(ev->e[2], s));
    k_pw_walk<K><<<h->general_blocks, NT, 0, s>>>(ak, av, c, h->dsp, h->dss, pre, boff,
                                                  (K *)h->sk[0], h->sv[0], h->segcnt, segcap,
                                                  h->SB);
    if (ev) HIPC(hipEventRecord(ev->e[3], s));
    if (ev) HIPC(hipEventRecord(ev->e[4], s));
  } else if (h->general) {
    // the in-plane field: the quiet scan on the field's probabilities, then
    // every entry with events, one thread each (timed as the loud stage; the
    // gather and heavy stages are empty).  When every solve has the field the
    // scan sends the entries whose draws are not all small to the heavy list,
    // sampled by the general routine (for large lists on the second stream,
    // beside the call-free routine over the rest); the entries the call-free
    // routine passes on (a spawn count of 20 or more) follow it.
    const bool split = h->all_field;
    k_spawn_scan<K, true><<<h->nscan, NT, 0, s>>>(ak, av, h->ctrl, h->dsp, h->dss, h->lidx,
                                                 (K *)h->lkey, h->lval, h->heavy, h->SB, split);
    if (ev) HIPC(hipEventRecord(ev->e[1], s));
    if (ev) HIPC(hipEventRecord(ev->e[2], s));
    if (split) {
      hipStream_t hs = h->fork_heavy ? h->side : s;
      if (h->fork_heavy) {
        HIPC(hipEventRecord(h->ev_fork, s));
        HIPC(hipStreamWaitEvent(h->side, h->ev_fork, 0));
      }
      // (the large entries on half a block per CU, dealt one per wave first,
      // leaving the rest of the CUs to the call-free routine)
      k_spawn_listed<K, false><<<clampu(h->ncu / 2, 1, 4096), NT, 0, hs>>>(
          c, h->dsp, h->dss, ak, av, h->heavy, &c->n_heavy, nullptr, (K *)h->sk[0], h->sv[0],
          h->segcnt, segcap, h->SB, 0);
      if (h->fork_heavy) HIPC(hipEventRecord(h->ev_join, h->side));
      k_spawn_listed<K, true><<<h->general_blocks, NT, 0, s>>>(
          c, h->dsp, h->dss, (const K *)h->lkey, h->lval, nullptr, &c->n_loud, h->late,
          (K *)h->sk[0], h->sv[0], h->segcnt, segcap, h->SB, h->field_limit);
      k_spawn_listed<K, false><<<h->general_blocks, NT, 0, s>>>(
          c, h->dsp, h->dss, (const K *)h->lkey, h->lval, h->late, &c->n_late, nullptr,
          (K *)h->sk[0], h->sv[0], h->segcnt, segcap, h->SB, 0);
      if (h->fork_heavy) HIPC(hipStreamWaitEvent(s, h->ev_join, 0));
    } else {
      k_spawn_listed<K, false><<<h->general_blocks, NT, 0, s>>>(
          c, h->dsp, h->dss, (const K *)h->lkey, h->lval, nullptr, &c->n_loud, nullptr,
          (K *)h->sk[0], h->sv[0], h->segcnt, segcap, h->SB, 0);
    }
    if (ev) HIPC(hipEventRecord(ev->e[3], s));
    if (ev) HIPC(hipEventRecord(ev->e[4], s));
  } else {
  k_spawn_scan<K><<<h->nscan, NT, 0, s>>>(ak, av, h->ctrl, h->dsp, h->dss, h->lidx,
                                         (K *)h->lkey, h->lval, h->heavy, h->SB);
  if (ev) HIPC(hipEventRecord(ev->e[1], s));
  if (h->fork_heavy) {
    // the scan's heavy list on the second stream, alongside the loud kernel
    HIPC(hipEventRecord(h->ev_fork, s));
    HIPC(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    // (a short list, with the loud kernel's grid of a block per chunk: the
    // kernel built for three waves per SIMD, whose waves find room sooner)
    if (h->loud_dyn)
      k_spawn_heavy<K, 1><<<g_heavy, 64, 0, h->side>>>(ak, av, c, h->dsp, h->dss, h->heavy,
                                                       &c->n_heavy, (K *)h->sk[0], h->sv[0],
                                                       h->segcnt, segcap, h->SB);
    else
      k_spawn_heavy<K, 3><<<g_heavy, 64, 0, h->side>>>(ak, av, c, h->dsp, h->dss, h->heavy,
                                                       &c->n_heavy, (K *)h->sk[0], h->sv[0],
                                                       h->segcnt, segcap, h->SB);
    HIPC(hipEventRecord(h->ev_join, h->side));
  }
  if (ev) HIPC(hipEventRecord(ev->e[2], s));
  uint32_t *late = h->fork_heavy ? h->late : h->heavy;
  uint32_t *nlate = h->fork_heavy ? &c->n_late : &c->n_heavy;
  const uint32_t tcap = h->tree_cap ? h->tree_cap : tree_jobs<K>();
  k_spawn_loud<K><<<g_loud, NT, 0, s>>>(c, h->dsp, h->dss, h->lidx, (const K *)h->lkey, h->lval,
                                        late, nlate, (K *)h->sk[0], h->sv[0], h->segcnt, segcap,
                                        tcap, h->loud_dyn ? 1 : 0, h->SB);
  if (ev) HIPC(hipEventRecord(ev->e[3], s));
  // the entries the loud kernel passed on (with the fork: usually none), then
  // the join
  k_spawn_heavy<K, 1><<<h->fork_heavy ? clampu(g_heavy, 1, 512) : g_heavy, 64, 0, s>>>(
      ak, av, c, h->dsp, h->dss, late, nlate, (K *)h->sk[0], h->sv[0], h->segcnt, segcap, h->SB);
  if (h->fork_heavy) HIPC(hipStreamWaitEvent(s, h->ev_join, 0));
  if (ev) HIPC(hipEventRecord(ev->e[4], s));
  }
  if (h->pool)
    k_inject<K><<<1, NT, 0, s>>>((const K *)h->inj_k, h->inj_v, h->ctrl, (K *)h->sk[0], h->sv[0],
                                 h->segcnt, segcap);
  // (the records' segment offsets and count are sealed by the first sort pass,
  // and the digit totals of every pass come from the sort's row scans: the
  // seal and histogram stages are empty, and no events are recorded for them)
  for (int p = 0; p < h->passes; ++p) {
    const K *ik = (const K *)h->sk[p & 1];
    const int2 *iv = h->sv[p & 1];
    K *ok = (K *)h->sk[(p + 1) & 1];
    int2 *ov = h->sv[(p + 1) & 1];
    uint32_t *tcnt = h->sort_cnt;
    const uint32_t sc = p == 0 ? segcap : 0u;
    switch (h->sort_it) {
      case 4:
        k_sort_count<K, 4><<<g_s, NT, 0, s>>>(ik, h->ctrl, tcnt, p, sc, h->segcnt);
        break;
      case 16:
        k_sort_count<K, 16><<<g_s, NT, 0, s>>>(ik, h->ctrl, tcnt, p, sc, h->segcnt);
        break;
      default:
        k_sort_count<K, 8><<<g_s, NT, 0, s>>>(ik, h->ctrl, tcnt, p, sc, h->segcnt);
    }
    k_sort_rowscan<<<256, NT, 0, s>>>(h->ctrl, tcnt, h->hist, p, sort_tile);
    switch (h->sort_it) {
      case 4:
        k_sort_pass<K, 4><<<g_s, NT, 0, s>>>(ik, iv, ok, ov, h->ctrl, h->hist, tcnt, p, sc);
        break;
      case 16:
        k_sort_pass<K, 16><<<g_s, NT, 0, s>>>(ik, iv, ok, ov, h->ctrl, h->hist, tcnt, p, sc);
        break;
      default:
        k_sort_pass<K, 8><<<g_s, NT, 0, s>>>(ik, iv, ok, ov, h->ctrl, h->hist, tcnt, p, sc);
    }
  }
  {
    // the merge-path partition is timed with the sort stage, so that the merge
    // stage is the merge kernel alone
    const int spb = h->passes & 1;
    const uint32_t g_p = clampu((g_m + NT) / NT, 1, 1024);
    k_merge_partition<K><<<g_p, NT, 0, s>>>(ak, (const K *)h->sk[spb], h->ctrl, h->part,
                                            merge_tile);
  }
  if (ev) HIPC(hipEventRecord(ev->e[7], s));
  {
    const int sp = h->passes & 1;
    const K *bk = (const K *)h->sk[sp];
    const int2 *bv = h->sv[sp];
    if (h->merge_it == 4)
      k_merge<K, false, 4><<<g_m, NT, 0, s>>>(ak, av, bk, bv, ck, cv, capC, h->ctrl, h->dsp,
                                              h->dss, h->spill, h->tile_cnt, h->part,
                                              h->SB);
    else
      k_merge<K, false, 8><<<g_m, NT, 0, s>>>(ak, av, bk, bv, ck, cv, capC, h->ctrl, h->dsp,
                                              h->dss, h->spill, h->tile_cnt, h->part,
                                              h->SB);
    k_merge_offsets<<<1, 1024, 0, s>>>(h->ctrl, h->tile_cnt, merge_tile);
    if (ev) HIPC(hipEventRecord(ev->e[8], s));
    if (h->merge_it == 4)
      k_merge<K, true, 4><<<g_m, NT, 0, s>>>(ak, av, bk, bv, ck, cv, capC, h->ctrl, h->dsp,
                                             h->dss, h->spill, h->tile_cnt, h->part,
                                             h->SB);
    else
      k_merge<K, true, 8><<<g_m, NT, 0, s>>>(ak, av, bk, bv, ck, cv, capC, h->ctrl, h->dsp,
                                             h->dss, h->spill, h->tile_cnt, h->part,
                                             h->SB);
  }
  if (ev) HIPC(hipEventRecord(ev->e[9], s));
  k_finalize<<<1, 1024, 0, s>>>(h->ctrl, h->dsp, h->dss, h->spill, h->nslots,
                                h->hist, h->passes, capC, h->segcnt, h->series, h->counts,
                                SERIES_CAP, merge_tile);
  if (ev) HIPC(hipEventRecord(ev->e[10], s));
  HIPC(hipGetLastError());
  return DDQMC_OK;
}

// Growth of a handle's buffers after a step that outgrew them (host
// arithmetic only; exported as ddqmc_plan_growth for tests).  A capacity that
// is short grows to 1.5 x its need + 4096, at most the ceiling (MAX_CAP, or a
// smaller cap_limit); a need above the ceiling is DDQMC_ECAPACITY.  The record
// need is the fullest segment's fill times the segment count, in 64 bits.
// Both capacities stay at most MAX_CAP, so list + records stay below 2^32 and
// every 32-bit count, position and tile offset in the kernels is exact.  The
// new sized arena is allocated while the old one is still held (the list is
// copied across), so it must leave the reserve free: else DDQMC_ENOMEM.
int plan_growth(uint64_t cap_main, uint64_t cap_sp, uint64_t need_main, uint64_t seg_need,
                size_t ks, uint64_t free_b, uint64_t total_b, uint64_t cap_limit,
                uint64_t *new_main, uint64_t *new_sp, uint64_t *bytes) {
  const uint64_t ceil = cap_limit ? std::min<uint64_t>(cap_limit, MAX_CAP) : MAX_CAP;
  const uint64_t need_sp = seg_need > ~0ull / NSEG ? ~0ull : seg_need * NSEG;
  uint64_t nm = cap_main, ns = cap_sp;
  if (need_main > cap_main) {
    if (need_main > ceil) return DDQMC_ECAPACITY;
    nm = std::min<uint64_t>(ceil, need_main + need_main / 2 + 4096);
  }
  if (need_sp > cap_sp) {
    if (need_sp > ceil) return DDQMC_ECAPACITY;
    ns = std::min<uint64_t>(ceil, need_sp + need_sp / 2 + 4096);
  }
  const uint64_t b = sized_layout(ks, nm, ns).total;
  *new_main = nm;
  *new_sp = sized_layout(ks, nm, ns).cap_sp;
  *bytes = b;
  if (b + memory_reserve(total_b) > free_b) return DDQMC_ENOMEM;
  return DDQMC_OK;
}

// Grow the sized arena (keeping the current list) after a step that needed
// need_main list entries or seg_need records in one segment.  A handle in a
// caller's workspace cannot grow: DDQMC_ECAPACITY.
int regrow(ddqmc_t *h, uint64_t need_main, uint64_t seg_need) {
  HIPC(hipStreamSynchronize(h->stream));
  if (!h->own_mem) return DDQMC_ECAPACITY;
  const size_t ks = key_size(h);
  size_t free_b = 0, total_b = 0;
  HIPC(hipMemGetInfo(&free_b, &total_b));
  uint64_t nm = 0, ns = 0, bytes = 0;
  const int rc = plan_growth(h->cap_main, h->cap_sp, need_main, seg_need, ks, free_b, total_b,
                             h->cap_limit, &nm, &ns, &bytes);
  if (rc != DDQMC_OK) return rc;
  const SizedLayout L = sized_layout(ks, nm, ns);
  char *base = nullptr;
  HIPC(hipMalloc((void **)&base, L.total));
  // the current list moves into the new arena's first list buffer
  const size_t n = h->n_main_known;
  hipError_t e = hipMemcpyAsync(base + L.mk[0], h->mk[h->cur], n * ks, hipMemcpyDeviceToDevice,
                                h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.mv[0], h->mv[h->cur], n * sizeof(int2), hipMemcpyDeviceToDevice,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    (void)hipFree(base);
    return hip_err(e);
  }
  HIPC(hipFree(h->sized));
  bind_sized(h, base, L);
  h->cur = 0;
  h->buf_gen += 1;  // captured graphs hold the old pointers and grids
  return DDQMC_OK;
}

// Capture graph_k steps starting from the list of parity par (kernels only:
// no memset or copy nodes) on a private stream, and instantiate them.
int capture_steps(ddqmc_t *h, int par) {
  if (!h->cap_stream) HIPC(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPC(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = DDQMC_OK;
  for (int j = 0; j < h->graph_k && rc == DDQMC_OK; ++j) {
    const int p = (par + j) & 1;
    rc = h->k64 ? launch_step<uint64_t>(h, p, nullptr, h->cap_stream)
                : launch_step<uint32_t>(h, p, nullptr, h->cap_stream);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc != DDQMC_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != DDQMC_OK ? rc : hip_err(e);
  }
  if (h->gexec[par]) {
    (void)hipGraphExecDestroy(h->gexec[par]);
    h->gexec[par] = nullptr;
  }
  const hipError_t ei = hipGraphInstantiate(&h->gexec[par], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    h->gexec[par] = nullptr;
    return hip_err(ei);
  }
  h->gexec_gen[par] = h->buf_gen;
  h->gexec_k[par] = h->graph_k;
  return DDQMC_OK;
}

int run_steps(ddqmc_t *h, int64_t n) {
  if (!h || n < 0) return DDQMC_EINVAL;
  if (h->profiling && h->ev.size() < SERIES_CAP) {
    const size_t old = h->ev.size();
    h->ev.resize(SERIES_CAP);
    for (size_t i = old; i < h->ev.size(); ++i)
      for (int j = 0; j <= NSTAGE; ++j)
        HIPC(hipEventCreateWithFlags(&h->ev[i].e[j], hipEventReleaseToDevice));
  }
  for (int i = 0; i < NSTAGE; ++i) h->stage_ms[i] = 0.0;
  h->stage_steps = 0;
  const bool use_graph = h->graph_k > 0 && !h->profiling;
  int64_t left = n;
  while (left > 0) {
    uint32_t chunk = (uint32_t)std::min<int64_t>(left, SERIES_CAP);
    uint32_t reps = 0;  // graph replays of graph_k steps
    if (use_graph && chunk >= (uint32_t)h->graph_k) {
      reps = chunk / (uint32_t)h->graph_k;
      chunk = reps * (uint32_t)h->graph_k;
    }
    if (!h->tile_table.empty()) {
      // the tuned shapes for the list size the chunk starts from
      const ddqmc_t::TileRow *row = &h->tile_table[0];
      for (const auto &r : h->tile_table)
        if ((int64_t)h->n_main_known >= r.min_entries) row = &r;
      if (row->sort_it != h->sort_it || row->merge_it != h->merge_it) {
        h->sort_it = row->sort_it;
        h->merge_it = row->merge_it;
        h->buf_gen += 1;  // captured graphs hold the other kernels
      }
    }
    k_chunk_begin<<<1, 1, 0, h->stream>>>(h->ctrl);
    if (reps) {
      // graph_k is even: every replay starts from the list of parity h->cur
      const int par = h->cur;
      if (h->gexec_gen[par] != h->buf_gen || h->gexec_k[par] != h->graph_k) {
        const int rc = capture_steps(h, par);
        if (rc != DDQMC_OK) return rc;
      }
      for (uint32_t r = 0; r < reps; ++r) HIPC(hipGraphLaunch(h->gexec[par], h->stream));
    } else {
      for (uint32_t j = 0; j < chunk; ++j) {
        const int par = (h->cur + (int)j) & 1;
        StageEvents *ev = h->profiling && j % (uint32_t)h->prof_every == 0 ? &h->ev[j] : nullptr;
        const int rc = h->k64 ? launch_step<uint64_t>(h, par, ev, h->stream)
                              : launch_step<uint32_t>(h, par, ev, h->stream);
        if (rc != DDQMC_OK) return rc;
      }
    }
    Ctrl c;
    HIPC(hipMemcpyAsync(&c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
    const uint32_t done = c.committed;
    if (done) {
      std::vector<int64_t> rows((size_t)done * h->nslots * SERIES_W);
      HIPC(hipMemcpy(rows.data(), h->series, rows.size() * sizeof(int64_t),
                     hipMemcpyDeviceToHost));
      for (uint32_t r = 0; r < done; ++r)
        for (int s = 0; s < h->nslots; ++s) {
          const int64_t *row = &rows[((size_t)r * h->nslots + s) * SERIES_W];
          if (row[0] >= 1) h->hseries[s].insert(h->hseries[s].end(), row, row + SERIES_W);
        }
      std::vector<uint32_t> cnt((size_t)done * COUNT_W);
      HIPC(hipMemcpy(cnt.data(), h->counts, cnt.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
      h->hcounts.insert(h->hcounts.end(), cnt.begin(), cnt.end());
      // The loud kernel's grid for the next chunk of steps, from the last
      // step's loud and large-population entries: while the heavy kernel's
      // list is small (below 0.25% of the loud list), one block per chunk of
      // entries, so that the heavy waves find room as loud blocks retire; when
      // it is large (above 1%), resident blocks, so that the loud kernel keeps
      // its CUs.  In between the grid stays as it is.
      const uint64_t n_loud = cnt[((size_t)done - 1) * COUNT_W + 3];
      const uint64_t n_heavy = cnt[((size_t)done - 1) * COUNT_W + 4];
      const bool dyn = h->loud_grid == 1   ? true
                       : h->loud_grid == 2 ? false
                       : h->loud_dyn       ? !(n_heavy * 400 < n_loud)
                                           : (n_heavy * 100 > n_loud);
      if (dyn != h->loud_dyn) {
        h->loud_dyn = dyn;
        h->buf_gen += 1;  // captured graphs hold the other grid
      }
    }
    if (h->profiling) {
      for (uint32_t j = 0; j < done; j += (uint32_t)h->prof_every) {
        for (int st = 0; st < NSTAGE; ++st) {
          if (st == STAGE_SEAL || st == STAGE_HIST) continue;  // empty stages
          // the sort stage starts where the heavy stage ends (its pool
          // injection included)
          const int from = st == STAGE_SORT ? STAGE_SEAL : st;
          float ms = 0.f;
          HIPC(hipEventElapsedTime(&ms, h->ev[j].e[from], h->ev[j].e[st + 1]));
          h->stage_ms[st] += ms;
        }
        h->stage_steps += 1;
      }
    }
    h->cur = (h->cur + (int)done) & 1;
    h->n_main_known = c.n_main;
    h->n_spawn_known = c.last_spawn;
    left -= done;
    // slots that entered or left are settled after a completed step
    if (done) {
      std::vector<SlotState> st(h->nslots);
      HIPC(hipMemcpy(st.data(), h->dss, h->nslots * sizeof(SlotState), hipMemcpyDeviceToHost));
      for (int s = 0; s < h->nslots; ++s) h->slot_state[s] = st[s].status;
    }
    if (c.abort) {
      const uint32_t f = c.fail_flags;
      const uint64_t seg_need = c.seg_need, need_main = c.n_new;
      k_rearm<<<1, 256, 0, h->stream>>>(h->ctrl, h->hist, MAX_PASSES, h->spill,
                                         h->nslots * SUM_BUCKETS * S_NSUM, h->segcnt);
      HIPC(hipGetLastError());
      HIPC(hipStreamSynchronize(h->stream));
      if (f & F_INT_OVF) return DDQMC_EOVERFLOW;
      if (f & F_RNG) return DDQMC_ERNG;
      if (f & F_EXTINCT) return DDQMC_EEXTINCT;
      if (f & F_ORDER) {
        std::fprintf(stderr, "ddqmc: the merge found the list or the records out of order\n");
        return DDQMC_EHIP;
      }
      if (f & (F_SPAWN_CAP | F_MAIN_CAP)) {
        const int rc = regrow(h, (f & F_MAIN_CAP) ? need_main : 0, (f & F_SPAWN_CAP) ? seg_need : 0);
        if (rc != DDQMC_OK) return rc;
        continue;
      }
      return DDQMC_EHIP;
    }
  }
  return DDQMC_OK;
}

// Flyvbjerg-Petersen blocking of (num, den) per-step series; the error of the
// ratio of means by the delta method, maximised over blocking levels.
double ratio_se(const std::vector<double> &num, const std::vector<double> &den) {
  std::vector<double> a = num, b = den;
  double best = 0.0;
  while (a.size() >= 16) {
    const size_t n = a.size();
    double ma = 0, mb = 0;
    for (size_t i = 0; i < n; ++i) {
      ma += a[i];
      mb += b[i];
    }
    ma /= (double)n;
    mb /= (double)n;
    const double r = ma / mb;
    double var = 0, mg = 0;
    std::vector<double> g(n);
    for (size_t i = 0; i < n; ++i) {
      g[i] = (a[i] - r * b[i]) / mb;
      mg += g[i];
    }
    mg /= (double)n;
    for (size_t i = 0; i < n; ++i) var += (g[i] - mg) * (g[i] - mg);
    var /= (double)(n - 1);
    best = std::max(best, std::sqrt(var / (double)n));
    std::vector<double> a2(n / 2), b2(n / 2);
    for (size_t i = 0; i < n / 2; ++i) {
      a2[i] = 0.5 * (a[2 * i] + a[2 * i + 1]);
      b2[i] = 0.5 * (b[2 * i] + b[2 * i + 1]);
    }
    a.swap(a2);
    b.swap(b2);
  }
  return best;
}

int fill_obs(ddqmc_t *h, int slot, ddqmc_obs *o) {
  if (!h || !o || slot < 0 || slot >= h->nslots) return DDQMC_EINVAL;
  HIPC(hipStreamSynchronize(h->stream));
  SlotState st;
  HIPC(hipMemcpy(&st, &h->dss[slot], sizeof(SlotState), hipMemcpyDeviceToHost));
  std::memset(o, 0, sizeof(*o));
  o->step = st.step;
  o->shift = st.S;
  o->mode = st.mode;
  o->status = st.status == 0 ? 0 : 1;
  for (int i = 0; i < S_NSUM; ++i) {
    o->last[i] = st.last[i];
    o->acc[i] = st.acc[i];
  }
  o->n_accum = st.n_accum;
  const SlotParams &P = h->hp[slot];
  const double wup = P.w_up;
  const double N = (double)P.N, nb = (double)P.nb;
  const double den = (double)st.acc[S_T_RE];
  if (st.n_accum > 0 && den != 0.0) {
    o->mz = (double)st.acc[S_Z] / (N * den);
    o->mx = ((double)st.acc[S_X] * wup) / (N * den);
    o->my = ((double)st.acc[S_Y] * wup) / (N * den);
    o->cxx = ((double)st.acc[S_CXX] * wup) / (nb * den);
    o->cyy = ((double)st.acc[S_CYY] * wup) / (nb * den);
    o->czz = (double)st.acc[S_CZZ] / (nb * den);
  }
  // errors from the per-step series after n_equil
  const std::vector<int64_t> &rows = h->hseries[slot];
  std::vector<double> d, nz, nx, ny, cx, cy, cz;
  for (size_t r = 0; r + SERIES_W <= rows.size(); r += SERIES_W) {
    if (rows[r] <= P.n_equil) continue;
    const int64_t *v = &rows[r + 3];
    d.push_back((double)v[S_T_RE]);
    nz.push_back((double)v[S_Z] / N);
    nx.push_back((double)v[S_X] * wup / N);
    ny.push_back((double)v[S_Y] * wup / N);
    cx.push_back((double)v[S_CXX] * wup / nb);
    cy.push_back((double)v[S_CYY] * wup / nb);
    cz.push_back((double)v[S_CZZ] / nb);
  }
  if (d.size() >= 16) {
    o->se_mz = ratio_se(nz, d);
    o->se_mx = ratio_se(nx, d);
    o->se_my = ratio_se(ny, d);
    o->se_cxx = ratio_se(cx, d);
    o->se_cyy = ratio_se(cy, d);
    o->se_czz = ratio_se(cz, d);
  }
  return DDQMC_OK;
}

uint64_t auto_capacity(const ddqmc_params &p) {
  if (p.capacity_hint > 0) return (uint64_t)p.capacity_hint;
  const uint64_t t = (uint64_t)std::max<int64_t>(p.target_walkers, p.initial_walkers);
  return std::min<uint64_t>(std::max<uint64_t>(t / 2, 16384), 1ull << 26);
}

// Device address of `scratch` on the current device, looked up once per
// device (hipGetSymbolAddress with that device current) and kept.
int noalloc_scratch(unsigned char **out) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static unsigned char *addr[MAX_DEVICES] = {};
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return DDQMC_EINVAL;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? hip_err(e) : DDQMC_EHIP;
    addr[dev] = (unsigned char *)p;
  }
  *out = addr[dev];
  return DDQMC_OK;
}

struct StateHeader {
  uint64_t magic;
  uint32_t version, key_bytes;
  ddqmc_params params;
  SlotState state;
  uint64_t n;
};

}  // namespace

extern "C" {

const char *ddqmc_strerror(int code) {
  switch (code) {
    case DDQMC_OK: return "ok";
    case DDQMC_EINVAL: return "invalid argument";
    case DDQMC_ENOMEM: return "out of memory";
    case DDQMC_ECAPACITY: return "walker list exceeds the largest buffer";
    case DDQMC_EOVERFLOW: return "walker count left the int32 range";
    case DDQMC_EEXTINCT: return "walker population died out";
    case DDQMC_EHIP: return "HIP runtime error";
    case DDQMC_ESTATE: return "call not valid in this state";
    case DDQMC_ERNG: return "random stream exhausted";
    default: return "unknown error";
  }
}

}  // extern "C"

namespace {

// Creation of a handle for count solves: in its own device memory (ws ==
// nullptr) or inside a caller's workspace.
int create_common(const ddqmc_params *p, int32_t count, void *hip_stream, void *ws,
                  size_t ws_bytes, ddqmc_t **out) {
  if (!p || !out || count < 1 || count > MAX_SLOTS) return DDQMC_EINVAL;
  *out = nullptr;
  int Nmax = 0;
  uint64_t cap = 0;
  for (int i = 0; i < count; ++i) {
    const int rc = validate(&p[i]);
    if (rc != DDQMC_OK) return rc;
    Nmax = std::max(Nmax, p[i].Lx * p[i].Ly);
    cap += auto_capacity(p[i]);
    if ((p[i].flags ^ p[0].flags) & DDQMC_PER_WALKER) return DDQMC_EINVAL;
  }
  // in a workspace: the capacity asked for, else the largest that fits
  if (ws) {
    cap = 0;
    for (int i = 0; i < count; ++i) cap += (uint64_t)p[i].capacity_hint;
    bool all = true;
    for (int i = 0; i < count; ++i) all = all && p[i].capacity_hint > 0;
    if (!all) cap = 0;
  }
  ddqmc_t *h = new (std::nothrow) ddqmc_t();
  if (!h) return DDQMC_ENOMEM;
  int rc = build(h, count, Nmax, cap, hip_stream, ws, ws_bytes);
  if (rc != DDQMC_OK) {
    free_all(h);
    delete h;
    return rc;
  }
  std::vector<SlotState> st(count);
  std::vector<uint64_t> keys(count);
  std::vector<int2> vals(count);
  h->all_field = count > 0;
  for (int i = 0; i < count; ++i) {
    h->hp[i] = make_slot(p[i]);
    if (h->hp[i].field) h->general = true;
    if (!h->hp[i].field) h->all_field = false;
    if (h->hp[i].flags & FLAG_PER_WALKER) h->per_walker = true;
    h->up[i] = p[i];
    st[i] = fresh_state(p[i], 1);
    h->slot_state[i] = 1;
    keys[i] = (count > 1) ? ((uint64_t)i << h->SB) : 0ull;
    vals[i] = make_int2((int)p[i].initial_walkers, 0);
  }
  rc = hip_err(hipMemcpyAsync(h->dsp, h->hp.data(), count * sizeof(SlotParams),
                              hipMemcpyHostToDevice, h->stream));
  if (rc == DDQMC_OK)
    rc = hip_err(hipMemcpyAsync(h->dss, st.data(), count * sizeof(SlotState),
                                hipMemcpyHostToDevice, h->stream));
  if (rc == DDQMC_OK) rc = upload_list(h, keys, vals);
  if (rc != DDQMC_OK) {
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return DDQMC_OK;
}

}  // namespace

extern "C" {

int ddqmc_batch_create(const ddqmc_params *p, int32_t count, void *hip_stream, ddqmc_t **out) {
  return create_common(p, count, hip_stream, nullptr, 0, out);
}

int ddqmc_create_in(const ddqmc_params *p, void *dev_ws, size_t bytes, void *hip_stream,
                    ddqmc_t **out) {
  if (!dev_ws) return DDQMC_EINVAL;
  return create_common(p, 1, hip_stream, dev_ws, bytes, out);
}

int ddqmc_create(const ddqmc_params *p, void *hip_stream, ddqmc_t **out) {
  return ddqmc_batch_create(p, 1, hip_stream, out);
}

int ddqmc_step(ddqmc_t *h, int64_t n_steps) { return run_steps(h, n_steps); }
int ddqmc_batch_step(ddqmc_t *h, int64_t n_steps) { return run_steps(h, n_steps); }

int ddqmc_observables(ddqmc_t *h, ddqmc_obs *out) { return fill_obs(h, 0, out); }
int ddqmc_batch_observables(ddqmc_t *h, int32_t idx, ddqmc_obs *out) {
  return fill_obs(h, idx, out);
}
int ddqmc_slot_observables(ddqmc_t *h, int32_t slot, ddqmc_obs *out) {
  return fill_obs(h, slot, out);
}

int ddqmc_destroy(ddqmc_t *h) {
  if (!h) return DDQMC_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
  return DDQMC_OK;
}

int ddqmc_pool_create(int32_t slots, int32_t max_sites, int64_t capacity_hint, void *hip_stream,
                      ddqmc_t **out) {
  if (!out || slots < 1 || slots > MAX_SLOTS || max_sites < 4 || max_sites > 32 ||
      capacity_hint < 0)
    return DDQMC_EINVAL;
  *out = nullptr;
  ddqmc_t *h = new (std::nothrow) ddqmc_t();
  if (!h) return DDQMC_ENOMEM;
  int rc = build(h, slots, max_sites, capacity_hint ? (uint64_t)capacity_hint : 1ull << 20,
                 hip_stream);
  if (rc == DDQMC_OK) {
    h->pool = true;
    rc = upload_list(h, {}, {});
  }
  if (rc != DDQMC_OK) {
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return DDQMC_OK;
}

int ddqmc_slot_admit(ddqmc_t *h, const ddqmc_params *p, int32_t *slot) {
  if (!h || !slot || !h->pool) return DDQMC_EINVAL;
  int rc = validate(p);
  if (rc != DDQMC_OK) return rc;
  if (p->Lx * p->Ly > h->Nmax) return DDQMC_EINVAL;
  if (p->flags & DDQMC_PER_WALKER) return DDQMC_EINVAL;
  int s = -1;
  for (int i = 0; i < h->nslots; ++i)
    if (h->slot_state[i] == 0) {
      s = i;
      break;
    }
  if (s < 0) return DDQMC_ESTATE;
  h->hp[s] = make_slot(*p);
  if (h->hp[s].field && !h->general) {
    h->general = true;  // (the handle keeps the general path from here on)
    h->buf_gen += 1;    // captured graphs hold the other spawn kernels
  }
  h->up[s] = *p;
  h->hseries[s].clear();
  const SlotState st = fresh_state(*p, 2);
  HIPC(hipStreamSynchronize(h->stream));
  uint32_t ninj = 0;
  HIPC(hipMemcpy(&ninj, &h->ctrl->n_inject, 4, hipMemcpyDeviceToHost));
  const uint64_t key = (uint64_t)s << h->SB;
  const int2 val = make_int2((int)p->initial_walkers, 0);
  if (h->k64) {
    HIPC(hipMemcpy((uint64_t *)h->inj_k + ninj, &key, 8, hipMemcpyHostToDevice));
  } else {
    const uint32_t k32 = (uint32_t)key;
    HIPC(hipMemcpy((uint32_t *)h->inj_k + ninj, &k32, 4, hipMemcpyHostToDevice));
  }
  HIPC(hipMemcpy(h->inj_v + ninj, &val, sizeof(int2), hipMemcpyHostToDevice));
  ninj += 1;
  HIPC(hipMemcpy(&h->ctrl->n_inject, &ninj, 4, hipMemcpyHostToDevice));
  HIPC(hipMemcpy(&h->dsp[s], &h->hp[s], sizeof(SlotParams), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(&h->dss[s], &st, sizeof(SlotState), hipMemcpyHostToDevice));
  h->slot_state[s] = 2;
  *slot = s;
  return DDQMC_OK;
}

int ddqmc_slot_retire(ddqmc_t *h, int32_t slot) {
  if (!h || slot < 0 || slot >= h->nslots) return DDQMC_EINVAL;
  if (h->slot_state[slot] != 1) return DDQMC_ESTATE;
  HIPC(hipStreamSynchronize(h->stream));
  const int32_t three = 3;
  HIPC(hipMemcpy(&h->dss[slot].status, &three, 4, hipMemcpyHostToDevice));
  h->slot_state[slot] = 3;
  return DDQMC_OK;
}

int ddqmc_list_size(ddqmc_t *h, int64_t *n) {
  if (!h || !n) return DDQMC_EINVAL;
  HIPC(hipStreamSynchronize(h->stream));
  uint32_t v = 0;
  HIPC(hipMemcpy(&v, &h->ctrl->n_main, 4, hipMemcpyDeviceToHost));
  *n = v;
  return DDQMC_OK;
}

int ddqmc_get_walkers(ddqmc_t *h, int32_t slot, uint64_t *keys, int32_t *re, int32_t *im,
                      int64_t cap, int64_t *n) {
  if (!h || !n || slot < 0 || slot >= h->nslots) return DDQMC_EINVAL;
  std::vector<uint64_t> k;
  std::vector<int2> v;
  int rc = download_list(h, k, v);
  if (rc != DDQMC_OK) return rc;
  const uint64_t lowm = (h->SB >= 64) ? ~0ull : ((1ull << h->SB) - 1);
  int64_t cnt = 0;
  for (size_t i = 0; i < k.size(); ++i) {
    const uint64_t s = (h->SB >= 64) ? 0 : (k[i] >> h->SB);
    if ((int)s != slot) continue;
    if (cnt < cap && keys && re && im) {
      keys[cnt] = k[i] & lowm;
      re[cnt] = v[i].x;
      im[cnt] = v[i].y;
    }
    ++cnt;
  }
  *n = cnt;
  return cnt > cap ? DDQMC_EINVAL : DDQMC_OK;
}

int ddqmc_set_walkers(ddqmc_t *h, const uint64_t *keys, const int32_t *re, const int32_t *im,
                      int64_t n) {
  if (!h || h->nslots != 1 || n < 0 || (n > 0 && (!keys || !re || !im))) return DDQMC_EINVAL;
  const uint64_t lim = (h->SB >= 64) ? ~0ull : ((1ull << h->SB) - 1);
  std::vector<uint64_t> k(n);
  std::vector<int2> v(n);
  for (int64_t i = 0; i < n; ++i) {
    if (keys[i] > lim || (i > 0 && keys[i] <= keys[i - 1])) return DDQMC_EINVAL;
    if ((re[i] == 0 && im[i] == 0) || re[i] == INT32_MIN || im[i] == INT32_MIN)
      return DDQMC_EINVAL;
    k[i] = keys[i];
    v[i] = make_int2(re[i], im[i]);
  }
  if ((uint64_t)n > h->cap_main) {
    int rc = regrow(h, (uint64_t)n, 0);
    if (rc != DDQMC_OK) return rc;
  }
  return upload_list(h, k, v);
}

int ddqmc_get_scalars(ddqmc_t *h, int32_t slot, double *shift, int32_t *mode, int64_t *step,
                      int64_t *nw_prev) {
  if (!h || slot < 0 || slot >= h->nslots) return DDQMC_EINVAL;
  HIPC(hipStreamSynchronize(h->stream));
  SlotState st;
  HIPC(hipMemcpy(&st, &h->dss[slot], sizeof(SlotState), hipMemcpyDeviceToHost));
  if (shift) *shift = st.S;
  if (mode) *mode = st.mode;
  if (step) *step = st.step;
  if (nw_prev) *nw_prev = st.nw_prev;
  return DDQMC_OK;
}

int ddqmc_set_scalars(ddqmc_t *h, int32_t slot, double shift, int32_t mode, int64_t step,
                      int64_t nw_prev) {
  if (!h || slot < 0 || slot >= h->nslots || (mode != 0 && mode != 1) || step < 0 ||
      step > 0xffffffffLL)
    return DDQMC_EINVAL;
  HIPC(hipStreamSynchronize(h->stream));
  SlotState st;
  HIPC(hipMemcpy(&st, &h->dss[slot], sizeof(SlotState), hipMemcpyDeviceToHost));
  st.S = shift;
  st.mode = mode;
  st.step = step;
  st.nw_prev = nw_prev;
  HIPC(hipMemcpy(&h->dss[slot], &st, sizeof(SlotState), hipMemcpyHostToDevice));
  return DDQMC_OK;
}

int ddqmc_get_state(ddqmc_t *h, void *buf, size_t cap, size_t *n) {
  if (!h || !n || h->nslots != 1) return DDQMC_EINVAL;
  std::vector<uint64_t> k;
  std::vector<int2> v;
  int rc = download_list(h, k, v);
  if (rc != DDQMC_OK) return rc;
  const size_t bytes = sizeof(StateHeader) + k.size() * (8 + sizeof(int2));
  *n = bytes;
  if (!buf) return DDQMC_OK;
  if (cap < bytes) return DDQMC_EINVAL;
  StateHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  hd.magic = 0x43514d5144445144ull;
  hd.version = 1;
  hd.key_bytes = 8;
  hd.params = h->up[0];
  HIPC(hipMemcpy(&hd.state, &h->dss[0], sizeof(SlotState), hipMemcpyDeviceToHost));
  hd.n = k.size();
  char *b = (char *)buf;
  std::memcpy(b, &hd, sizeof(hd));
  std::memcpy(b + sizeof(hd), k.data(), k.size() * 8);
  std::memcpy(b + sizeof(hd) + k.size() * 8, v.data(), v.size() * sizeof(int2));
  return DDQMC_OK;
}

int ddqmc_set_state(ddqmc_t *h, const void *buf, size_t n) {
  if (!h || !buf || h->nslots != 1 || n < sizeof(StateHeader)) return DDQMC_EINVAL;
  StateHeader hd;
  std::memcpy(&hd, buf, sizeof(hd));
  if (hd.magic != 0x43514d5144445144ull || hd.version != 1 || hd.key_bytes != 8)
    return DDQMC_EINVAL;
  if (n != sizeof(hd) + hd.n * (8 + sizeof(int2))) return DDQMC_EINVAL;
  ddqmc_params a = hd.params, b = h->up[0];
  a.capacity_hint = b.capacity_hint = 0;
  if (std::memcmp(&a, &b, sizeof(a)) != 0) return DDQMC_EINVAL;
  const char *c = (const char *)buf;
  std::vector<uint64_t> k(hd.n);
  std::vector<int2> v(hd.n);
  std::memcpy(k.data(), c + sizeof(hd), hd.n * 8);
  std::memcpy(v.data(), c + sizeof(hd) + hd.n * 8, hd.n * sizeof(int2));
  // the list invariants the step relies on: keys in range and strictly
  // increasing, values nonzero and representable with a sign flip
  const uint64_t lim = (h->SB >= 64) ? ~0ull : ((1ull << h->SB) - 1);
  for (uint64_t i = 0; i < hd.n; ++i) {
    if (k[i] > lim || (i > 0 && k[i] <= k[i - 1])) return DDQMC_EINVAL;
    if ((v[i].x == 0 && v[i].y == 0) || v[i].x == INT32_MIN || v[i].y == INT32_MIN)
      return DDQMC_EINVAL;
  }
  if (hd.n > h->cap_main) {
    int rc = regrow(h, hd.n, 0);
    if (rc != DDQMC_OK) return rc;
  }
  int rc = upload_list(h, k, v);
  if (rc != DDQMC_OK) return rc;
  HIPC(hipMemcpy(&h->dss[0], &hd.state, sizeof(SlotState), hipMemcpyHostToDevice));
  h->hseries[0].clear();
  return DDQMC_OK;
}

int ddqmc_get_series(ddqmc_t *h, int32_t slot, int64_t *rows, int64_t cap, int64_t *n) {
  if (!h || !n || slot < 0 || slot >= h->nslots) return DDQMC_EINVAL;
  const std::vector<int64_t> &s = h->hseries[slot];
  const int64_t nr = (int64_t)(s.size() / SERIES_W);
  *n = nr;
  if (rows && cap > 0)
    std::memcpy(rows, s.data(), (size_t)std::min(cap, nr) * SERIES_W * sizeof(int64_t));
  return DDQMC_OK;
}

int ddqmc_get_step_counts(ddqmc_t *h, int64_t *rows, int64_t cap, int64_t *n) {
  if (!h || !n) return DDQMC_EINVAL;
  const int64_t nr = (int64_t)(h->hcounts.size() / COUNT_W);
  *n = nr;
  if (rows && cap > 0)
    std::memcpy(rows, h->hcounts.data(), (size_t)std::min(cap, nr) * COUNT_W * sizeof(int64_t));
  return DDQMC_OK;
}

int ddqmc_workspace_query(const ddqmc_params *p, int64_t capacity, size_t *bytes) {
  if (!bytes || capacity < 0) return DDQMC_EINVAL;
  int rc = validate(p);
  if (rc != DDQMC_OK) return rc;
  const int N = p->Lx * p->Ly;
  const size_t ks = (2 * N > 32) ? 8 : 4;
  uint64_t cm, cs;
  initial_caps(capacity > 0 ? (uint64_t)capacity : auto_capacity(*p), &cm, &cs);
  *bytes = fixed_layout(1, ks).total + sized_layout(ks, cm, cs).total;
  return DDQMC_OK;
}

int ddqmc_device_bytes(ddqmc_t *h, size_t *bytes, int64_t *capacity) {
  if (!h || !bytes) return DDQMC_EINVAL;
  *bytes = h->fixed_bytes + h->sized_bytes;
  if (capacity) *capacity = (int64_t)h->cap_main;
  return DDQMC_OK;
}

int ddqmc_ratio_se(const double *num, const double *den, int64_t n, double *se) {
  if (!num || !den || !se || n < 0) return DDQMC_EINVAL;
  *se = ratio_se(std::vector<double>(num, num + n), std::vector<double>(den, den + n));
  return DDQMC_OK;
}

int ddqmc_set_capacity_limit(ddqmc_t *h, int64_t max_entries) {
  if (!h || max_entries < 0) return DDQMC_EINVAL;
  h->cap_limit = (uint64_t)max_entries;
  return DDQMC_OK;
}

int ddqmc_plan_growth(uint64_t cap_main, uint64_t cap_sp, uint64_t need_main, uint64_t seg_need,
                      uint32_t key_bytes, uint64_t free_bytes, uint64_t total_bytes,
                      uint64_t cap_limit, uint64_t *new_main, uint64_t *new_sp,
                      uint64_t *bytes) {
  if (!new_main || !new_sp || !bytes || (key_bytes != 4 && key_bytes != 8)) return DDQMC_EINVAL;
  return plan_growth(cap_main, cap_sp, need_main, seg_need, key_bytes, free_bytes, total_bytes,
                     cap_limit, new_main, new_sp, bytes);
}

int ddqmc_set_profiling(ddqmc_t *h, int32_t on) {
  if (!h) return DDQMC_EINVAL;
  if (on < 0) return DDQMC_EINVAL;
  h->profiling = on != 0;
  h->prof_every = on > 0 ? on : 1;
  return DDQMC_OK;
}

int ddqmc_set_graph_steps(ddqmc_t *h, int32_t k) {
  if (!h || k < 0 || (k > 0 && (k < 2 || (k & 1) || k > (int32_t)SERIES_CAP)))
    return DDQMC_EINVAL;
  h->graph_k = k;
  return DDQMC_OK;
}

int ddqmc_set_heavy_fork(ddqmc_t *h, int32_t mode) {
  if (!h || mode < -1 || mode > 1) return DDQMC_EINVAL;
  h->fork_mode = mode;
  h->fork_heavy = mode > 0 || (mode == 0 && h->cap_main >= FORK_MIN_CAP);
  h->buf_gen += 1;  // captured graphs hold the other launch sequence
  return DDQMC_OK;
}

int ddqmc_set_loud_grid(ddqmc_t *h, int32_t mode) {
  if (!h || mode < 0 || mode > 2) return DDQMC_EINVAL;
  h->loud_grid = mode;
  const bool dyn = mode == 1 || (mode == 0 && h->loud_dyn);
  if (dyn != h->loud_dyn) {
    h->loud_dyn = dyn;
    h->buf_gen += 1;  // captured graphs hold the other grid
  }
  return DDQMC_OK;
}

int ddqmc_set_tiles(ddqmc_t *h, int32_t sort_it, int32_t merge_it) {
  if (!h || (sort_it != 4 && sort_it != 8 && sort_it != 16) || (merge_it != 4 && merge_it != 8))
    return DDQMC_EINVAL;
  h->tile_table.clear();
  if (sort_it != h->sort_it || merge_it != h->merge_it) {
    h->sort_it = sort_it;
    h->merge_it = merge_it;
    h->buf_gen += 1;  // captured graphs hold the other kernels
  }
  return DDQMC_OK;
}

int ddqmc_set_tile_table(ddqmc_t *h, int32_t rows, const int64_t *min_entries,
                         const int32_t *sort_it, const int32_t *merge_it) {
  if (!h || rows < 0 || rows > 64 || (rows > 0 && (!min_entries || !sort_it || !merge_it)))
    return DDQMC_EINVAL;
  std::vector<ddqmc_t::TileRow> t;
  for (int i = 0; i < rows; ++i) {
    if ((sort_it[i] != 4 && sort_it[i] != 8 && sort_it[i] != 16) ||
        (merge_it[i] != 4 && merge_it[i] != 8) || min_entries[i] < 0 ||
        (i > 0 && min_entries[i] <= min_entries[i - 1]))
      return DDQMC_EINVAL;
    t.push_back({min_entries[i], sort_it[i], merge_it[i]});
  }
  h->tile_table.swap(t);
  return DDQMC_OK;
}

int ddqmc_get_tiles(ddqmc_t *h, int32_t *sort_it, int32_t *merge_it) {
  if (!h || !sort_it || !merge_it) return DDQMC_EINVAL;
  *sort_it = h->sort_it;
  *merge_it = h->merge_it;
  return DDQMC_OK;
}

int ddqmc_set_tree_queue(ddqmc_t *h, int32_t places) {
  if (!h || places < 0) return DDQMC_EINVAL;
  const uint32_t most = h->k64 ? tree_jobs<uint64_t>() : tree_jobs<uint32_t>();
  if ((uint32_t)places > most) return DDQMC_EINVAL;
  h->tree_cap = (uint32_t)places;
  h->buf_gen += 1;  // captured graphs hold the old kernel argument
  return DDQMC_OK;
}

int ddqmc_set_field_limit(ddqmc_t *h, int32_t spawns) {
  if (!h || spawns < 1 || spawns > 20) return DDQMC_EINVAL;
  h->field_limit = spawns;
  h->buf_gen += 1;  // captured graphs hold the old kernel argument
  return DDQMC_OK;
}

int ddqmc_stage_times(ddqmc_t *h, double ms[10], int64_t *steps) {
  if (!h || !ms) return DDQMC_EINVAL;
  for (int i = 0; i < NSTAGE; ++i) ms[i] = h->stage_ms[i];
  if (steps) *steps = h->stage_steps;
  return DDQMC_OK;
}

int ddqmc_dev_uniforms(uint64_t seed, uint32_t solve_id, uint64_t cfg, uint32_t step,
                       uint32_t draw, int64_t count, double *out) {
  if (!out || count < 0) return DDQMC_EINVAL;
  if (count == 0) return DDQMC_OK;
  double *d = nullptr;
  HIPC(hipMalloc((void **)&d, count * sizeof(double)));
  k_dev_uniforms<<<1, 64>>>(seed, solve_id, cfg, step, draw, count, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(out, d, count * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  return hip_err(e);
}

int ddqmc_dev_binom(int64_t n, double p, int32_t mode, uint64_t seed, int64_t count,
                    int64_t *out) {
  if (!out || count < 0 || mode < 0 || mode > 2 || n < 0 || !(p >= 0.0)) return DDQMC_EINVAL;
  if ((mode == 0 || mode == 1) && p > 1.0) return DDQMC_EINVAL;
  if (mode == 1 && (n < 1 || p <= 0.0 || p >= 1.0)) return DDQMC_EINVAL;
  if (count == 0) return DDQMC_OK;
  int64_t *d = nullptr;
  int *err = nullptr;
  HIPC(hipMalloc((void **)&d, count * sizeof(int64_t)));
  HIPC(hipMalloc((void **)&err, sizeof(int)));
  HIPC(hipMemset(err, 0, sizeof(int)));
  const int64_t blocks = (count + 255) / 256;
  k_dev_binom<<<(uint32_t)blocks, 256>>>(n, p, mode, seed, count, d, err);
  hipError_t e = hipGetLastError();
  int he = 0;
  if (e == hipSuccess) e = hipMemcpy(out, d, count * sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&he, err, sizeof(int), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  (void)hipFree(err);
  if (e != hipSuccess) return hip_err(e);
  return he ? DDQMC_ERNG : DDQMC_OK;
}

int ddqmc_dev_binom_noalloc(int64_t n, double p, int32_t mode, uint64_t seed, int64_t count,
                            int64_t *out) {
  if (!out || count < 0 || mode < 0 || mode > 2 || n < 0 || !(p >= 0.0)) return DDQMC_EINVAL;
  if ((mode == 0 || mode == 1) && p > 1.0) return DDQMC_EINVAL;
  if (mode == 1 && (n < 1 || p <= 0.0 || p >= 1.0)) return DDQMC_EINVAL;
  if (count > NOALLOC_MAX_SAMPLES) {
    std::fprintf(stderr,
                 "ddqmc_dev_binom_noalloc: %lld samples asked for, its scratch holds at most "
                 "%lld\n",
                 (long long)count, (long long)NOALLOC_MAX_SAMPLES);
    return DDQMC_EINVAL;
  }
  if (count == 0) return DDQMC_OK;
  unsigned char *base = nullptr;
  const int rc = noalloc_scratch(&base);
  if (rc != DDQMC_OK) return rc;
  int *err = (int *)base;
  int64_t *d = (int64_t *)(base + NOALLOC_HEADER);
  // the flag left by the previous call is cleared by a kernel on the same
  // stream as the sampler (no memset node, so the sequence may be captured)
  k_fill_u32<<<1, 64>>>((uint32_t *)err, 0u, 1u);
  k_dev_binom<<<(uint32_t)((count + 255) / 256), 256>>>(n, p, mode, seed, count, d, err);
  hipError_t e = hipGetLastError();
  int he = 0;
  if (e == hipSuccess) e = hipMemcpy(out, d, count * sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&he, err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_err(e);
  return he ? DDQMC_ERNG : DDQMC_OK;
}

int ddqmc_dev_quiet(const double *p, const int64_t *n, const double *u, int64_t count,
                    int32_t *out) {
  if (!p || !n || !u || !out || count < 0) return DDQMC_EINVAL;
  for (int64_t i = 0; i < count; ++i) {
    if (n[2 * i] < 0 || n[2 * i + 1] < 0) return DDQMC_EINVAL;
    for (int k = 0; k < 4; ++k)
      if (!(p[4 * i + k] >= 0.0 && p[4 * i + k] < 1.0)) return DDQMC_EINVAL;
  }
  if (count == 0) return DDQMC_OK;
  double *dp = nullptr, *du = nullptr;
  int64_t *dn = nullptr;
  int32_t *dout = nullptr;
  HIPC(hipMalloc((void **)&dp, 4 * count * sizeof(double)));
  HIPC(hipMalloc((void **)&dn, 2 * count * sizeof(int64_t)));
  HIPC(hipMalloc((void **)&du, count * sizeof(double)));
  HIPC(hipMalloc((void **)&dout, count * sizeof(int32_t)));
  hipError_t e = hipMemcpy(dp, p, 4 * count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dn, n, 2 * count * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(du, u, count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_dev_quiet<<<(uint32_t)((count + 255) / 256), 256>>>(dp, dn, du, count, dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dout, count * sizeof(int32_t), hipMemcpyDeviceToHost);
  (void)hipFree(dp);
  (void)hipFree(dn);
  (void)hipFree(du);
  (void)hipFree(dout);
  return hip_err(e);
}

int ddqmc_dev_math(const double *x, int64_t count, double *out) {
  if (!x || !out || count < 0) return DDQMC_EINVAL;
  if (count == 0) return DDQMC_OK;
  double *dx = nullptr, *dout = nullptr;
  HIPC(hipMalloc((void **)&dx, count * sizeof(double)));
  HIPC(hipMalloc((void **)&dout, 4 * count * sizeof(double)));
  hipError_t e = hipMemcpy(dx, x, count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_dev_math<<<(uint32_t)((count + 255) / 256), 256>>>(dx, count, dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dout, 4 * count * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(dx);
  (void)hipFree(dout);
  return hip_err(e);
}

}  // extern "C"
