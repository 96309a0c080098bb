/*
 * CPU oracle for one DDQMC propagation step (Nagy & Savona, arXiv:1802.05931).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded reference of
 * the walker step that the GPU library implements.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * Conventions (each side implements them on its own):
 *   site s = x + Lx*y, bit s of a bitstring set <=> spin up;
 *   configuration |ket><bra| has key (ket << N) | bra, N = Lx*Ly <= 32;
 *   bonds = unique nearest-neighbour pairs of the periodic Lx x Ly torus, ordered
 *   "right" bonds (origin site ascending) then "up" bonds (origin ascending);
 *   H = sum_bonds Jx SxSx + Jy SySy + Jz SzSz with S = sigma/2 (Sec. V, model
 *   Hamiltonian) + sum_sites hx sigma^x + hy sigma^y (the in-plane field of
 *   Sec. V.B); one jump operator S^- per site with rate gamma.
 */
#ifndef DDQMC_ORACLE_H
#define DDQMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-4)
#define ORC_EEXTINCT (-5)
#define ORC_ERNG (-8)

#define ORC_NO_INITIATOR 1u
#define ORC_PER_WALKER 2u   /* spawning and clone/death walker by walker (Sec. II)  */

typedef struct {
  int32_t Lx, Ly;
  double Jx, Jy, Jz, gamma, dt;
  int32_t n_a;              /* initiator threshold I_limit (Sec. IV.A)            */
  int64_t target_walkers;   /* N_w at which the shift starts to vary              */
  int64_t initial_walkers;  /* real walkers placed on |dn..dn><dn..dn|            */
  double is_p;              /* importance-sampling parameter p (Sec. IV.B)        */
  double shift_damping;     /* delta of the shift update (Sec. III.C)             */
  double shift_init;        /* S held during the growth phase                     */
  uint64_t seed;
  uint32_t solve_id;
  int64_t n_equil;          /* steps after which estimators are accumulated       */
  uint32_t flags;
  double hx, hy;            /* in-plane field sum_i (hx sigma^x_i + hy sigma^y_i),
                               h (cos theta, sin theta) of Sec. V.B               */
} orc_params;

enum { ORC_T_RE, ORC_T_IM, ORC_NW, ORC_Z, ORC_X, ORC_Y, ORC_CXX, ORC_CYY, ORC_CZZ,
       ORC_WTOT, ORC_NENT, ORC_NSUM };

typedef struct orc_t orc_t;

int orc_create(const orc_params *p, orc_t **out);
void orc_destroy(orc_t *h);
int orc_step(orc_t *h, int64_t n_steps);
int64_t orc_size(const orc_t *h);
int orc_get_list(const orc_t *h, uint64_t *keys, int32_t *re, int32_t *im, int64_t cap);
int orc_set_list(orc_t *h, const uint64_t *keys, const int32_t *re, const int32_t *im,
                 int64_t n);
int orc_get_scalars(const orc_t *h, double *S, int32_t *mode, int64_t *step, int64_t *nw_prev);
int orc_set_scalars(orc_t *h, double S, int32_t mode, int64_t step, int64_t nw_prev);
int orc_get_last(const orc_t *h, int64_t out[ORC_NSUM]);
int orc_get_acc(const orc_t *h, int64_t out[ORC_NSUM], int64_t *n_accum);
/* one row per step: step, S (as its bit pattern), mode, then ORC_NSUM sums */
int64_t orc_series_len(const orc_t *h);
int orc_get_series(const orc_t *h, int64_t *rows, int64_t cap_rows);

/* ---- pieces exposed for the pin tests ---- */
/* The step's annihilation: contributions (any order, repeated keys) summed per
 * configuration and merged with a list of sorted unique keys whose values
 * (int64) already carry their clone/death; zero totals dropped.  nk/nre/nim
 * hold n + ncon entries; *nout receives the new list's length.  ORC_EOVERFLOW
 * when a total leaves the int32 range. */
int orc_annihilate(const uint64_t *ckeys, const int64_t *cre, const int64_t *cim, int64_t ncon,
                   const uint64_t *keys, const int64_t *pr, const int64_t *pi, int64_t n,
                   uint64_t *nk, int64_t *nre, int64_t *nim, int64_t *nout);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_det_log(double x);
double orc_det_exp(double x);
void orc_uniforms(uint64_t seed, uint32_t solve_id, uint64_t cfg, uint32_t step, uint32_t draw,
                  int64_t count, double *out);
/* mode 0: Bin(n,p); 1: Bin(n,p) conditioned on >= 1; 2: Bsplit(n,p).
 * Sample i uses the stream (seed, solve 0, cfg = i, step 0, draw 1). */
int orc_binom_many(int64_t n, double p, int mode, uint64_t seed, int64_t count, int64_t *out);
/* Probability that no channel fires: prod_k (1 - p_k)^n_k in fp64, k = 0..7,
 * each factor by binary powers (Sec. III.B). */
double orc_no_event_prob(const double p[8], const int64_t n[8]);
/* entry-level channel sampler on its own: probabilities p[8], counts n[8];
 * sample i uses cfg = i.  out is count x 8. */
int orc_channels_many(const double p[8], const int64_t n[8], uint64_t seed, int64_t count,
                      int64_t *out);
int orc_bonds(int32_t Lx, int32_t Ly, int32_t *s1, int32_t *s2);
/* the placement of X walkers of one spawning channel (3/7 jumps, 4/8 hops) of
 * the entry key over its connections, by the step's code; sample i at step i.
 * Rows of N (jumps, by site) or 2 nb (hops: ket bonds, then bra bonds) counts;
 * returns the row width or a negative code. */
int orc_split_many(const orc_params *p, uint64_t key, int channel, int64_t X, int64_t count,
                   int64_t *out);
/* off-diagonal elements of the shifted, importance-sampled Liouvillian seen from
 * the parent (ket, bra): child configuration and element (re, im); plus diagonal. */
int orc_connections(const orc_params *p, uint64_t ket, uint64_t bra, double S, uint64_t *cket,
                    uint64_t *cbra, double *re, double *im, int32_t cap, double *d_re,
                    double *d_im);

#ifdef __cplusplus
}
#endif
#endif
