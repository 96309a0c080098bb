/*
 * ddqmc.h -- C ABI of the MI355X (gfx950) library for the driven-dissipative
 * quantum Monte Carlo propagation step of Nagy & Savona, arXiv:1802.05931.
 *
 * One step advances a complex integer walker population over density-matrix
 * configurations |ket><bra| by the rules of Sec. III.C (spawning along the
 * off-diagonal Liouvillian elements by the multinomial formalism of Sec. III.B,
 * clone/death on the diagonal element, annihilation), with the initiator rule of
 * Sec. IV.A, the importance-sampling weights of Sec. IV.B, the shift update of
 * Sec. III.C and the estimators of Sec. III.A / V.A, for the dissipative 2D XYZ
 * model of Sec. V.  Every stage runs in hand-written HIP kernels on the device.
 *
 * Conventions
 *   site s = x + Lx*y; bit s of a bitstring = 1 <=> spin up;
 *   configuration key = (ket << N) | bra, N = Lx*Ly <= 32 (a 64-bit value);
 *   H = sum over unique nearest-neighbour bonds of the periodic Lx x Ly lattice of
 *       Jx SxSx + Jy SySy + Jz SzSz with S = sigma/2, plus hx sigma^x + hy sigma^y
 *       per site (the in-plane field of Sec. V.B); jump S^- per site, rate gamma;
 *   walkers are int32 (re, im) per configuration; all estimator sums are int64.
 *
 * Return codes: 0 on success, a negative DDQMC_E* code otherwise (see
 * ddqmc_strerror).  On any error a handle is left at its last completed step.
 * Calls on one handle are not thread-safe; distinct handles are independent.
 * Host pointers are borrowed for the duration of a call only.
 */
#ifndef DDQMC_H
#define DDQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDQMC_OK 0
#define DDQMC_EINVAL (-1)     /* bad argument or parameter                          */
#define DDQMC_ENOMEM (-2)     /* host or device allocation failed                   */
#define DDQMC_ECAPACITY (-3)  /* list exceeds the allowed capacity after regrowing  */
#define DDQMC_EOVERFLOW (-4)  /* a configuration's walker count left int32 range    */
#define DDQMC_EEXTINCT (-5)   /* no walkers left / diagonal weight N_w reached zero  */
#define DDQMC_EHIP (-6)       /* HIP runtime error                                  */
#define DDQMC_ESTATE (-7)     /* call not valid in the handle's current state       */
#define DDQMC_ERNG (-8)       /* a random stream ran out of counter blocks          */

/* flags */
#define DDQMC_NO_INITIATOR 1u /* every parent counts as an initiator                */
/* Spawning and clone/death walker by walker, by the rules of Sec. II: each
 * walker dies / clones along the diagonal element with probability dt |d|,
 * and makes one attempt per element part (real: jumps, imaginary: hops) at a
 * connection chosen uniformly, with success probability n_conn dt |element|
 * (importance-sampled).  Same expectation as the default per-entry sampling,
 * which draws all of an entry's walkers at once; kept as its ablation.  All
 * solves of a handle carry the flag or none does (DDQMC_EINVAL otherwise); not
 * with the in-plane field, not in a serving pool (DDQMC_EINVAL); at most 2^27
 * walkers on one part of one entry (DDQMC_ERNG beyond). */
#define DDQMC_PER_WALKER 2u

/* Parameters of one steady-state solve (Sec. V model; Sec. III.C shift;
 * Sec. IV.A initiator threshold; Sec. IV.B importance-sampling parameter). */
typedef struct {
  uint32_t struct_size;     /* = sizeof(ddqmc_params)                              */
  int32_t Lx, Ly;           /* 2 <= Lx, Ly and Lx*Ly <= 32, periodic               */
  double Jx, Jy, Jz;        /* couplings                                           */
  double gamma;             /* > 0, rate of the S^- jump on every site             */
  double dt;                /* > 0, Euler time step                                */
  int32_t n_a;              /* >= 0, initiator threshold I_limit on |re|+|im|      */
  int64_t target_walkers;   /* N_w (diagonal real weight) that ends the growth phase */
  int64_t initial_walkers;  /* 1 .. 2^31-1 real walkers on |dn..dn><dn..dn|         */
  double is_p;              /* >= 0, weight e^{-p} on off-diagonal configurations  */
  double shift_damping;     /* delta of the shift update                           */
  double shift_init;        /* shift held while N_w < target_walkers               */
  uint64_t seed;            /* Philox key (with solve_id)                          */
  uint32_t solve_id;        /* < 65536; distinct solves draw distinct streams       */
  int64_t n_equil;          /* steps before estimator accumulation starts          */
  int64_t capacity_hint;    /* initial list capacity in entries; 0 = automatic     */
  uint32_t flags;           /* DDQMC_NO_INITIATOR | DDQMC_PER_WALKER                */
  double hx, hy;            /* in-plane field sum_i hx sigma^x_i + hy sigma^y_i, i.e.
                               h (cos theta, sin theta) of Sec. V.B; 0, 0 = none.
                               In a handle with a field on, every solve's
                               entries with events are sampled one thread
                               each by the general routine (same results)     */
} ddqmc_params;

/* Sums over the walker list after a step (Sec. III.A numerators/denominators):
 * t_re/t_im = Re/Im Tr rho; n_w = sum |Re rho_ii|; z = sum_i Re rho_ii (2 n_up(i) - N);
 * x, y = sum over single-flip configurations of the sigma^x / sigma^y element
 * (real part); cxx, cyy, czz = the same for nearest-neighbour pairs (czz on the
 * diagonal); w_tot = sum |re| + |im|; n_entries = occupied configurations. */
enum {
  DDQMC_T_RE = 0, DDQMC_T_IM, DDQMC_NW, DDQMC_Z, DDQMC_X, DDQMC_Y, DDQMC_CXX, DDQMC_CYY,
  DDQMC_CZZ, DDQMC_WTOT, DDQMC_NENT, DDQMC_NSUM
};

typedef struct {
  int64_t step;             /* steps done by this solve                            */
  double shift;             /* current shift S                                     */
  int32_t mode;             /* 0 growth (S held), 1 shift varies                   */
  int32_t status;           /* 1 running, 0 slot empty                             */
  int64_t last[DDQMC_NSUM]; /* sums after the last step                            */
  int64_t n_accum;          /* steps accumulated (those with step > n_equil)       */
  int64_t acc[DDQMC_NSUM];  /* sums over the accumulated steps                     */
  /* ratios of the accumulated sums: M_alpha = num / (N acc[T_RE]),
   * C_alpha = num / (n_bonds acc[T_RE]); off-diagonal numerators times e^{p}    */
  double mx, my, mz, cxx, cyy, czz;
  /* standard errors: blocking of the per-step series + delta method            */
  double se_mx, se_my, se_mz, se_cxx, se_cyy, se_czz;
} ddqmc_obs;

typedef struct ddqmc_t ddqmc_t;

/* ---- one solve -------------------------------------------------------------
 * ddqmc_create: validates *p, allocates device buffers (hipMalloc), places
 *   initial_walkers real walkers on key 0 and sets S = shift_init.  stream may be
 *   NULL (the handle creates its own) or a hipStream_t owned by the caller, which
 *   must outlive the handle.  EINVAL on bad parameters, ENOMEM, EHIP.
 * ddqmc_step: advances n_steps steps on the stream; returns after they finished.
 *   Lists that outgrow their buffers are regrown and the step is redone (the
 *   random streams are counter based, so the result is unchanged).  EOVERFLOW,
 *   EEXTINCT, ECAPACITY, ERNG or EHIP leave the handle at its last good step.
 * ddqmc_observables: sums, ratios and standard errors of solve 0.
 * ddqmc_destroy: frees everything; NULL is accepted.                          */
int ddqmc_create(const ddqmc_params *p, void *hip_stream, ddqmc_t **out);
int ddqmc_step(ddqmc_t *h, int64_t n_steps);
int ddqmc_observables(ddqmc_t *h, ddqmc_obs *out);
int ddqmc_destroy(ddqmc_t *h);

/* ---- one solve inside a caller-owned device workspace ------------------------
 * ddqmc_create_in: as ddqmc_create, but every device buffer of the handle lies
 *   in [dev_ws, dev_ws + bytes), device memory the caller allocated (e.g. a
 *   torch tensor) and keeps alive, unmoved, until ddqmc_destroy; the library
 *   allocates no device memory for it and never frees it.  dev_ws must be
 *   256-byte aligned (EINVAL otherwise, or when it is NULL).  The list capacity
 *   is p->capacity_hint if it is nonzero (ECAPACITY if that handle does not fit
 *   in bytes), else the largest that fits (ECAPACITY if not even the smallest,
 *   4096 entries, does; ddqmc_workspace_query gives the bytes a capacity
 *   needs).  The buffers never grow: a step that would outgrow them returns
 *   ECAPACITY and leaves the handle at its last completed step. */
int ddqmc_create_in(const ddqmc_params *p, void *dev_ws, size_t bytes, void *hip_stream,
                    ddqmc_t **out);

/* ---- many independent solves in one launch per stage (batched) --------------
 * The solves share one sorted list whose keys carry the slot number above the
 * configuration bits; each solve keeps its own parameters, shift and step count
 * and draws exactly the random numbers it would draw alone.
 * ddqmc_batch_create: count solves, parameters p[0..count-1], all started.
 * ddqmc_batch_step == ddqmc_step.  ddqmc_batch_observables: solve idx.        */
int ddqmc_batch_create(const ddqmc_params *p, int32_t count, void *hip_stream, ddqmc_t **out);
int ddqmc_batch_step(ddqmc_t *h, int64_t n_steps);
int ddqmc_batch_observables(ddqmc_t *h, int32_t idx, ddqmc_obs *out);

/* ---- continuous batching (serving) ------------------------------------------
 * ddqmc_pool_create: an empty handle with `slots` slots for lattices of up to
 *   max_sites sites (<= 32; with the slot bits the key must fit 64 bits).
 * ddqmc_slot_admit: puts a new solve in a free slot; its initial walkers enter the
 *   list during the next step, after which it steps like a fresh ddqmc_create
 *   handle.  Writes the slot index; ESTATE if no slot is free.
 * ddqmc_slot_retire: the slot's walkers leave the list during the next step.
 * ddqmc_slot_observables: as ddqmc_observables for one slot.
 * ddqmc_list_size: occupied configurations over all slots (last synchronised). */
int ddqmc_pool_create(int32_t slots, int32_t max_sites, int64_t capacity_hint, void *hip_stream,
                      ddqmc_t **out);
int ddqmc_slot_admit(ddqmc_t *h, const ddqmc_params *p, int32_t *slot);
int ddqmc_slot_retire(ddqmc_t *h, int32_t slot);
int ddqmc_slot_observables(ddqmc_t *h, int32_t slot, ddqmc_obs *out);
int ddqmc_list_size(ddqmc_t *h, int64_t *n);

/* ---- state access (tests, checkpoints) ---------------------------------------
 * Keys cross the ABI as uint64 (ket << N) | bra without slot bits, ascending.
 * ddqmc_get_walkers: copies slot's list; cap in entries; *n = its length
 *   (EINVAL, with *n set, if cap is too small).
 * ddqmc_set_walkers: replaces slot's list (keys strictly ascending, no (0,0),
 *   |values| < 2^31); only on a handle with one slot.
 * ddqmc_get_scalars / ddqmc_set_scalars: shift, mode, step, N_w of the previous
 *   step of one slot.
 * ddqmc_get_state / ddqmc_set_state: checkpoint of a one-slot handle as an opaque
 *   byte string (list, scalars, accumulators); set_state requires the same
 *   parameters.  get_state with buf == NULL reports the size in *n.           */
int ddqmc_get_walkers(ddqmc_t *h, int32_t slot, uint64_t *keys, int32_t *re, int32_t *im,
                      int64_t cap, int64_t *n);
int ddqmc_set_walkers(ddqmc_t *h, const uint64_t *keys, const int32_t *re, const int32_t *im,
                      int64_t n);
int ddqmc_get_scalars(ddqmc_t *h, int32_t slot, double *shift, int32_t *mode, int64_t *step,
                      int64_t *nw_prev);
int ddqmc_set_scalars(ddqmc_t *h, int32_t slot, double shift, int32_t mode, int64_t step,
                      int64_t nw_prev);
int ddqmc_get_state(ddqmc_t *h, void *buf, size_t cap, size_t *n);
int ddqmc_set_state(ddqmc_t *h, const void *buf, size_t n);

/* Per-step series of one slot since creation: rows of (step, shift bit pattern,
 * mode, the DDQMC_NSUM sums), int64.  *n = rows available; copies min(cap, n). */
int ddqmc_get_series(ddqmc_t *h, int32_t slot, int64_t *rows, int64_t cap, int64_t *n);

/* Per step since creation, over all slots: rows of five int64 (entries at the
 * start of the step, spawn records produced, entries after the step, entries
 * with some event, of those the ones sampled one wave each).  These size the
 * memory traffic of each kernel launch (bytes per launch for a roofline).
 * rows holds cap rows (5 cap int64); *n receives the number of steps. */
int ddqmc_get_step_counts(ddqmc_t *h, int64_t *rows, int64_t cap, int64_t *n);

/* Device bytes of a one-slot handle with list capacity `capacity` entries
 * (0: the capacity ddqmc_create would choose for *p): exactly what ddqmc_create
 * allocates for it and what ddqmc_create_in needs, from the same layout of its
 * buffers (the walker list twice, the spawn records twice at a quarter of the
 * list capacity, the sort and merge tile arrays, the loud and heavy lists, and
 * the fixed per-solve tables, each 256-byte aligned).  Serving admission sizes
 * requests with it.  EINVAL on bad parameters or a negative capacity.
 * ddqmc_device_bytes: the device bytes a handle holds now (both arenas) and its
 *   current list capacity (capacity may be NULL). */
int ddqmc_workspace_query(const ddqmc_params *p, int64_t capacity, size_t *bytes);
int ddqmc_device_bytes(ddqmc_t *h, size_t *bytes, int64_t *capacity);

/* Growth of a handle's buffers (host arithmetic only, no device call; the step
 * uses it after a step outgrew its buffers).  Given the current list and record
 * capacities, the entries the failed step needed (need_main, 0 if the list fit),
 * the records its fullest spawn segment needed (seg_need, 0 if they fit; the
 * record need is seg_need x 64 segments, taken in 64 bits), the key size (4 or
 * 8 bytes), the device's free and total bytes and a capacity ceiling (0: the
 * largest buffer, 0x7FF00000 entries): a short capacity grows to 1.5 x its need
 * + 4096, at most the ceiling.  Writes the new capacities and the bytes of the
 * new list and scratch arena.  Returns 0, ECAPACITY (a need above the
 * ceiling), ENOMEM (the new arena would leave less than max(4 GiB, total/32)
 * free; the old arena is still held while the list is copied) or EINVAL.
 * ddqmc_set_capacity_limit: a ceiling (entries) for one handle's growth, 0 = the
 *   largest buffer; a step that needs more returns ECAPACITY with the handle at
 *   its last completed step. */
int ddqmc_plan_growth(uint64_t cap_main, uint64_t cap_sp, uint64_t need_main, uint64_t seg_need,
                      uint32_t key_bytes, uint64_t free_bytes, uint64_t total_bytes,
                      uint64_t cap_limit, uint64_t *new_main, uint64_t *new_sp,
                      uint64_t *bytes);
int ddqmc_set_capacity_limit(ddqmc_t *h, int64_t max_entries);

/* Standard error of the ratio of means of a per-step (numerator, denominator)
 * series, as ddqmc_observables computes it (host arithmetic only): the series
 * is blocked by successive halving (Flyvbjerg-Petersen) while at least 16
 * blocks remain; at each level the error of mean(num) / mean(den) follows from
 * the block means by the delta method, sqrt(var(num_b - r den_b) / n_b) /
 * mean(den); the largest over the levels is returned (0 for fewer than 16
 * points).  EINVAL on NULL pointers or n < 0. */
int ddqmc_ratio_se(const double *num, const double *den, int64_t n, double *se);

/* Wall time of the kernels of the last ddqmc_step call, per stage, from HIP
 * events on the handle's stream when profiling is on (ddqmc_set_profiling);
 * ms[10] = quiet scan (which also writes the list of loud entries), loud
 * gather (kept for the layout of ms: the scan writes that list; with the
 * second stream on, the fork to it),
 * loud spawn (the spawn kernel alone), heavy spawn (the entries the loud
 * kernel passed on, and the wait for the heavy kernel that ran on a second
 * stream next to the loud one), record seal and histogram (both kept for the
 * layout and empty: the first sort pass seals the records, and the sort's
 * row scans give the digit totals),
 * sort (the radix passes and the merge-path partition), merge count
 * (survivors per tile and their offsets), merge (the merge kernel that writes
 * the new list), finalize, summed over the steps that carried events;
 * *steps receives their number.  ddqmc_set_profiling(h, k): k = 0 off, k >= 1
 * events on every k-th step of each chunk of steps (an event costs a few
 * microseconds of the step it is in, so sampling keeps the other steps
 * undisturbed).  EINVAL for k < 0. */
int ddqmc_set_profiling(ddqmc_t *h, int32_t on);

/* Launch the kernels of k consecutive steps as one HIP graph (k even,
 * 2 <= k <= 1024); k = 0 (the default) launches them one by one.  A graph is
 * captured on first use for each parity of the list it starts from, and again
 * after the handle's buffers grow; steps that do not fill a whole graph run
 * one by one.  Graphs are not used while profiling is on.  The results are the
 * same either way: a graph holds the same kernels with the same grids, and
 * each kernel reads its counts from device memory.  EINVAL for other k. */
int ddqmc_set_graph_steps(ddqmc_t *h, int32_t k);

/* Where the entries with large populations are sampled.  They are known after
 * the quiet scan; with the fork on, their kernel runs on a second stream of
 * the handle, next to the kernel that samples the other loud entries, and the
 * main stream waits for it before the records are sorted.  mode 0 (default):
 * on when the list capacity is at least 2^23 entries (below that a fork and
 * join cost more than they save), 1: always, -1: never.  The results are the
 * same either way.  EINVAL for other modes. */
int ddqmc_set_heavy_fork(ddqmc_t *h, int32_t mode);
/* Places in the loud kernel's per-chunk queue of member trees (the binomial
 * trees that spread two or more walkers over the members of a class,
 * Sec. III.B): an entry whose trees find no room takes the general path,
 * and the results are the same either way.  0 (default): the most the
 * kernel holds, 1024 with 32-bit keys and 768 with 64-bit keys.  EINVAL
 * below 0 or above that. */
int ddqmc_set_tree_queue(ddqmc_t *h, int32_t places);
/* With the in-plane field in every solve of a handle, the entries whose
 * draws are all small are sampled by a routine that draws by inversion
 * only; an entry with `spawns` or more walkers spawned along one element part
 * by one part of its walkers is passed on to the general routine, and the
 * results are the same either way.  Default and most 20 (the inversion
 * sampler then covers every split); smaller values are for tests of the
 * passing on.  EINVAL outside 1..20. */
int ddqmc_set_field_limit(ddqmc_t *h, int32_t spawns);
/* Grid of the loud spawn kernel.  0 (default): chosen per chunk of steps from
 * the last step's counts (one block per 256-entry chunk while the list of
 * large-population entries is small beside the loud list, resident blocks
 * taking chunks from a counter when it is large); 1: always resident blocks;
 * 2: always a block per chunk.  The results are the same either way.  EINVAL
 * for other modes. */
int ddqmc_set_loud_grid(ddqmc_t *h, int32_t mode);
/* Tile shapes of the annihilation stage (Sec. III.C rule (iii)): records per
 * thread of a radix-sort tile (sort_it: 4, 8 or 16; a tile is 256 sort_it
 * records) and merged positions per thread of a merge-path tile (merge_it: 4
 * or 8).  Default 8 and 8.  The results are the same for every shape.
 * ddqmc_set_tiles: one shape for every step (it clears a table).
 * ddqmc_set_tile_table: rows (min_entries ascending, strictly; shapes as
 *   above): before each chunk of steps the handle takes the shape of the last
 *   row whose min_entries is at most its current list size (the first row
 *   below all of them).  rows = 0 clears the table.  Written by the tuner,
 *   which times every shape per key width and list-size bucket.
 * ddqmc_get_tiles: the shape in use.  EINVAL for other values. */
int ddqmc_set_tiles(ddqmc_t *h, int32_t sort_it, int32_t merge_it);
int ddqmc_set_tile_table(ddqmc_t *h, int32_t rows, const int64_t *min_entries,
                         const int32_t *sort_it, const int32_t *merge_it);
int ddqmc_get_tiles(ddqmc_t *h, int32_t *sort_it, int32_t *merge_it);
int ddqmc_stage_times(ddqmc_t *h, double ms[10], int64_t *steps);

/* ---- device self-checks of the sampling primitives --------------------------
 * Same streams as the step (Philox4x32-10, key (seed_lo, seed_hi ^ solve),
 * counter (cfg_lo, cfg_hi, step, draw << 16 | block), 53-bit uniforms).
 * ddqmc_dev_uniforms: count uniforms of one stream, computed on the device.
 * ddqmc_dev_binom: sample i uses stream (seed, 0, cfg = i, 0, draw 1);
 *   mode 0 Bin(n,p), 1 Bin(n,p | >= 1), 2 integer part + Bin(n, fraction).
 * ddqmc_dev_math: out[4i..4i+3] = det_log(x_i), det_exp(x_i), sqrt(x_i), 1/x_i.
 * ddqmc_dev_quiet: the spawn scan's test of whether an entry spawns nothing in
 *   a step (Sec. III.B: every channel count zero).  Entry i has the channel
 *   probabilities p[4i..4i+3] (diagonal real, diagonal imaginary, jump, hop),
 *   the same for its real and its imaginary walkers, walker counts
 *   n[2i] = |R|, n[2i+1] = |I|, and primary uniform u[i].  Bit 0 of out[i] is
 *   1 iff u[i] < prod over the four channels and both parts of (1 - p)^n,
 *   the product taken in fp64 in that order by binary powers; bit 1 is 1 when
 *   the scan's single-precision estimate decided it without the product.
 *   EINVAL for p outside [0, 1) or negative n.
 * All pointers are host memory.                                               */
int ddqmc_dev_uniforms(uint64_t seed, uint32_t solve_id, uint64_t cfg, uint32_t step,
                       uint32_t draw, int64_t count, double *out);
int ddqmc_dev_binom(int64_t n, double p, int32_t mode, uint64_t seed, int64_t count,
                    int64_t *out);
int ddqmc_dev_math(const double *x, int64_t count, double *out);
/* ddqmc_dev_binom_noalloc: ddqmc_dev_binom for callers that cannot allocate
 *   device memory (code under HIP graph capture, tight serving loops, harnesses
 *   that forbid hipMalloc): the same samples, staged in a static device
 *   scratch array of the library (8 MiB + 256 bytes, held by every GPU the
 *   library runs on until the process ends) instead of a buffer allocated per
 *   call; it calls no hipMalloc or hipFree.  count <= 2^20 (EINVAL beyond, with
 *   a message on stderr); other arguments and errors as ddqmc_dev_binom.  The
 *   scratch keeps the last call's contents; calls that overlap on one GPU (from
 *   several host threads) race on it and must be serialised by the caller. */
int ddqmc_dev_binom_noalloc(int64_t n, double p, int32_t mode, uint64_t seed, int64_t count,
                            int64_t *out);
int ddqmc_dev_quiet(const double *p, const int64_t *n, const double *u, int64_t count,
                    int32_t *out);

const char *ddqmc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
