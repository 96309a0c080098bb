/*
 * CPU oracle for one DDQMC propagation step (Nagy & Savona, arXiv:1802.05931).
 *
 * TEST INFRASTRUCTURE ONLY -- see ddqmc_oracle.h.  Plain C, one thread, fp64
 * with IEEE round-to-nearest, built with -ffp-contract=off so that every
 * product and sum is rounded on its own.  Nothing here is tuned.
 *
 * What one step computes (Sec. III.C, the numbered list "Spawning / Clone-Death /
 * Annihilation", on top of the Euler map of eq. (Euler) for the shifted
 * Liouvillian of eq. (lindShift), in the element form of eq. (eq:elmeq)):
 *   for every occupied configuration |l><m| with complex walker number R + iI
 *     - clone/death on the diagonal element L_{lm}^{lm} (Sec. II rule (ii),
 *       Sec. III.C rule (ii)),
 *     - spawning along the off-diagonal elements, Re and Im parts in turn, each
 *       by the multinomial formalism of Sec. III.B: N_sp ~ Bin(n, P_tot), then a
 *       multinomial split over the connected configurations,
 *     - the initiator rule of Sec. IV.A on the progeny,
 *   then annihilation: all contributions to one configuration are summed.
 * Importance sampling (Sec. IV.B) multiplies each off-diagonal element by
 * w_child / w_parent with w = e^{-p} off the diagonal and 1 on it.
 * The shift follows the update of Sec. III.C on the diagonal real weight N_w.
 * Estimators are the numerator/denominator sums of Sec. III.A.
 *
 * The paper leaves the sampling details open (it cites binomial generators);
 * the choices fixed here -- counter-based streams, BINV/BTRD, the entry-level
 * "first event" decomposition and the split order -- are exact in law and are
 * pinned by the tests against exact pmfs and the exact one-step expectation.
 */
#include "ddqmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).                                                 */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  int round;
  for (round = 0; round < 10; round++) {
    uint64_t p0, p1;
    uint32_t n0, n1, n2, n3;
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    n1 = (uint32_t)p1;
    n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of uniforms for one draw: key = (seed_lo, seed_hi ^ solve_id),
 * counter = (cfg_lo, cfg_hi, step, draw << 16 | block).  Each block yields two
 * 53-bit uniforms, from (x0, x1) and then (x2, x3). */
typedef struct {
  uint32_t key[2];
  uint32_t c0, c1, c2;
  uint32_t draw;
  uint32_t block;
  int has_spare;
  double spare;
  int *err;
} stream_t;

static void stream_init(stream_t *s, uint64_t seed, uint32_t solve_id, uint64_t cfg,
                        uint32_t step, uint32_t draw, int *err) {
  s->key[0] = (uint32_t)seed;
  s->key[1] = (uint32_t)(seed >> 32) ^ solve_id;
  s->c0 = (uint32_t)cfg;
  s->c1 = (uint32_t)(cfg >> 32);
  s->c2 = step;
  s->draw = draw;
  s->block = 0;
  s->has_spare = 0;
  s->spare = 0.0;
  s->err = err;
}

static double u53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

static int stream_exhausted(const stream_t *s) { return s->block >= 65536u && !s->has_spare; }

static double stream_next(stream_t *s) {
  uint32_t ctr[4], out[4];
  if (s->has_spare) {
    s->has_spare = 0;
    return s->spare;
  }
  if (s->block >= 65536u) {
    if (s->err) *s->err = ORC_ERNG;
    return 0.0;
  }
  ctr[0] = s->c0; ctr[1] = s->c1; ctr[2] = s->c2; ctr[3] = (s->draw << 16) | s->block;
  s->block++;
  orc_philox4x32_10(ctr, s->key, out);
  s->spare = u53(out[2], out[3]);
  s->has_spare = 1;
  return u53(out[0], out[1]);
}

void orc_uniforms(uint64_t seed, uint32_t solve_id, uint64_t cfg, uint32_t step, uint32_t draw,
                  int64_t count, double *out) {
  stream_t s;
  int err = 0;
  int64_t i;
  stream_init(&s, seed, solve_id, cfg, step, draw, &err);
  for (i = 0; i < count; i++) out[i] = stream_next(&s);
}

/* ------------------------------------------------------------------------ */
/* Deterministic log and exp from +, -, *, / only, so that both sides of the */
/* parity check round identically.                                           */
/* ------------------------------------------------------------------------ */
static const double LN2_HI = 0x1.62e42p-1;          /* ln 2 with 21 significant bits */
static const double LN2_LO = 0x1.fdf473de6af28p-22; /* ln 2 - LN2_HI                 */
static const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

static uint64_t dbits(double x) { uint64_t b; memcpy(&b, &x, 8); return b; }
static double bitsd(uint64_t b) { double x; memcpy(&x, &b, 8); return x; }

/* ln x = e ln 2 + ln m with m in [sqrt(1/2), sqrt(2)), and
 * ln m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^25/25), s = (m-1)/(m+1). */
double orc_det_log(double x) {
  uint64_t b;
  int e;
  double m, s, z, poly, lnm, ed;
  int k;
  if (x != x) return x;
  if (x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (x == INFINITY) return x;
  b = dbits(x);
  e = (int)((b >> 52) & 0x7ff);
  if (e == 0) { /* subnormal: scale by 2^54 */
    x = x * 18014398509481984.0;
    b = dbits(x);
    e = (int)((b >> 52) & 0x7ff) - 54;
  }
  e = e - 1022;
  m = bitsd((b & 0x000fffffffffffffull) | 0x3fe0000000000000ull); /* [0.5, 1) */
  if (m < SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  s = (m - 1.0) / (m + 1.0);
  z = s * s;
  poly = 1.0 / 25.0;
  for (k = 23; k >= 1; k -= 2) poly = poly * z + 1.0 / (double)k;
  lnm = (2.0 * s) * poly;
  ed = (double)e;
  return ed * LN2_HI + (ed * LN2_LO + lnm);
}

/* e^x = 2^k e^r, r = x - k ln 2 (two-part reduction), e^r by its Taylor series
 * to r^16/16! evaluated by Horner. */
double orc_det_exp(double x) {
  double kd, r, poly;
  int k, i;
  if (x != x) return x;
  if (x > 709.0) return INFINITY;
  if (x < -708.0) return 0.0;
  kd = floor(x / (LN2_HI + LN2_LO) + 0.5);
  k = (int)kd;
  r = (x - kd * LN2_HI) - kd * LN2_LO;
  poly = 1.0;
  for (i = 16; i >= 1; i--) poly = poly * (r / (double)i) + 1.0;
  return poly * bitsd((uint64_t)(k + 1023) << 52);
}

/* ------------------------------------------------------------------------ */
/* Binomial generators (the paper cites Kachitvichyanukul & Schmeiser 1988    */
/* and Hormann 1993 for these, Sec. III.B).                                  */
/* ------------------------------------------------------------------------ */
static double powi(double b, int64_t e) {
  double r = 1.0;
  while (e > 0) {
    if (e & 1) r = r * b;
    e >>= 1;
    if (e > 0) b = b * b;
  }
  return r;
}

/* Stirling remainder fc(k) = ln k! - (k + 1/2) ln(k+1) + (k+1) - ln(2 pi)/2. */
static double fc_table[10];
static int fc_ready = 0;
static void fc_init(void) {
  int k;
  double fact = 1.0;
  double half_ln_2pi = 0.5 * orc_det_log(0x1.921fb54442d18p+2);
  for (k = 0; k <= 9; k++) {
    double kk = (double)k;
    if (k > 0) fact = fact * kk;
    fc_table[k] = orc_det_log(fact) - (kk + 0.5) * orc_det_log(kk + 1.0) + (kk + 1.0) - half_ln_2pi;
  }
  fc_ready = 1;
}
static double fc(int64_t k) {
  double ikp1, ik2;
  if (k <= 9) return fc_table[k];
  ikp1 = 1.0 / ((double)k + 1.0);
  ik2 = ikp1 * ikp1;
  return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * ik2) * ik2) * ikp1;
}

/* Inversion (BINV).  trunc != 0 samples X conditioned on X >= 1. */
static int64_t binv(int64_t n, double p, stream_t *s, int trunc) {
  double q = 1.0 - p;
  double sr = p / q;
  double a = ((double)n + 1.0) * sr;
  double r0 = powi(q, n);
  int64_t lim = n < 110 ? n : 110;
  for (;;) {
    double u, r;
    int64_t x;
    if (stream_exhausted(s)) return 0;
    u = stream_next(s);
    if (trunc) {
      u = u * (1.0 - r0);
      x = 1;
      r = r0 * (a - sr);
    } else {
      x = 0;
      r = r0;
    }
    for (;;) {
      if (u < r) return x;
      u = u - r;
      x = x + 1;
      if (x > lim) break;
      r = r * (a / (double)x - sr);
    }
  }
}

/* Transformed rejection with decomposition (BTRD), for p <= 1/2, n p >= 10. */
static int64_t btrd(int64_t n, double p, stream_t *s) {
  double nd = (double)n;
  double q = 1.0 - p;
  double md = floor((nd + 1.0) * p);
  int64_t m = (int64_t)md;
  double r = p / q;
  double nr = (nd + 1.0) * r;
  double npq = nd * p * q;
  double spq = sqrt(npq);
  double b = 1.15 + 2.53 * spq;
  double a = -0.0873 + 0.0248 * b + 0.01 * p;
  double c = nd * p + 0.5;
  double alpha = (2.83 + 5.1 / b) * spq;
  double vr = 0.92 - 4.2 / b;
  double urvr = 0.86 * vr;
  for (;;) {
    double v, u, us, kd, kmd, rho, t, nm, h, nk;
    int64_t k, km;
    if (stream_exhausted(s)) return 0;
    v = stream_next(s);
    if (v <= urvr) {
      u = v / vr - 0.43;
      kd = floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
      if (kd < 0.0 || kd > nd) continue;
      return (int64_t)kd;
    }
    if (v >= vr) {
      u = stream_next(s) - 0.5;
    } else {
      u = v / vr - 0.93;
      u = (u < 0.0 ? -0.5 : 0.5) - u;
      v = stream_next(s) * vr;
    }
    us = 0.5 - fabs(u);
    kd = floor((2.0 * a / us + b) * u + c);
    if (kd < 0.0 || kd > nd) continue;
    k = (int64_t)kd;
    v = v * alpha / (a / (us * us) + b);
    km = k > m ? k - m : m - k;
    if (km <= 15) {
      double f = 1.0;
      int64_t i;
      if (m < k) {
        for (i = m + 1; i <= k; i++) f = f * (nr / (double)i - r);
      } else if (m > k) {
        for (i = k + 1; i <= m; i++) v = v * (nr / (double)i - r);
      }
      if (v <= f) return k;
      continue;
    }
    v = orc_det_log(v);
    kmd = (double)km;
    rho = (kmd / npq) * (((kmd / 3.0 + 0.625) * kmd + 1.0 / 6.0) / npq + 0.5);
    t = -kmd * kmd / (2.0 * npq);
    if (v < t - rho) return k;
    if (v > t + rho) continue;
    nm = nd - md + 1.0;
    h = (md + 0.5) * orc_det_log((md + 1.0) / (r * nm)) + fc(m) + fc(n - m);
    nk = nd - kd + 1.0;
    if (v <= h + (nd + 1.0) * orc_det_log(nm / nk) +
                  (kd + 0.5) * orc_det_log(nk * r / (kd + 1.0)) - fc(k) - fc(n - k))
      return k;
  }
}

static int64_t binom_half(int64_t n, double p, stream_t *s) {
  if ((double)n * p < 10.0) return binv(n, p, s, 0);
  return btrd(n, p, s);
}

/* X ~ Bin(n, p), 0 <= p <= 1. */
static int64_t binom(int64_t n, double p, stream_t *s) {
  if (n <= 0 || p <= 0.0) return 0;
  if (p > 0.5) return n - binom_half(n, 1.0 - p, s);
  return binom_half(n, p, s);
}

/* X ~ Bin(n, p) conditioned on X >= 1; n >= 1, 0 < p < 1. */
static int64_t binom_trunc(int64_t n, double p, stream_t *s) {
  if (p > 0.5) {
    for (;;) {
      int64_t y = binom_half(n, 1.0 - p, s);
      if (y < n) return n - y;
      if (stream_exhausted(s)) return 1;
    }
  }
  if ((double)n * p < 10.0) return binv(n, p, s, 1);
  for (;;) {
    int64_t x = btrd(n, p, s);
    if (x >= 1) return x;
    if (stream_exhausted(s)) return 1;
  }
}

/* n walkers, each producing floor(P) events plus one more with probability
 * P - floor(P) (Sec. II rule (i): integer part deterministic, fraction drawn). */
static int64_t bsplit(int64_t n, double P, stream_t *s) {
  double f;
  if (n <= 0 || P <= 0.0) return 0;
  if (P < 1.0) return binom(n, P, s);
  f = floor(P);
  return n * (int64_t)f + binom(n, P - f, s);
}

int orc_binom_many(int64_t n, double p, int mode, uint64_t seed, int64_t count, int64_t *out) {
  int64_t i;
  int err = 0;
  if (!fc_ready) fc_init();
  for (i = 0; i < count; i++) {
    stream_t s;
    stream_init(&s, seed, 0, (uint64_t)i, 0, 1, &err);
    if (mode == 0) out[i] = binom(n, p, &s);
    else if (mode == 1) out[i] = binom_trunc(n, p, &s);
    else out[i] = bsplit(n, p, &s);
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* Entry-level sampling of the eight independent channel counts.             */
/* Channel k (1..8) draws X_k ~ Bsplit(n_k, p_k); k = 1..4 act on the real    */
/* walkers (death-re, death-im, spawn along Re elements, spawn along Im),     */
/* k = 5..8 on the imaginary walkers in the same order.  When every p_k < 1,  */
/* successive uniforms of the primary stream (draw 0) locate the nonzero      */
/* channels one after the other: starting at channel `start`, a uniform u is  */
/* compared by inversion with the running products of the zero probabilities  */
/* from `start` on; u below the last product means no further channel fires,  */
/* otherwise the first product u exceeds names the next nonzero channel,      */
/* which is drawn conditioned on >= 1; the search resumes after it.  The      */
/* joint law is that of eight independent counts.                             */
/* ------------------------------------------------------------------------ */
#define DRAW_CH(k) ((uint32_t)(k) << 10)
#define DRAW_PICK 7u /* within a channel: the single-walker categorical draw */

typedef struct {
  uint64_t seed;
  uint32_t solve_id;
  uint64_t cfg;
  uint32_t step;
  int *err;
} ectx_t;

static void channel_stream(const ectx_t *c, stream_t *s, uint32_t draw) {
  stream_init(s, c->seed, c->solve_id, c->cfg, c->step, draw, c->err);
}
/* G[k] = prod over j = start..k of (1 - p_j)^n_j (Sec. III.B): the
 * probability that none of the channels start..k fires; channels with no
 * walkers or zero probability contribute 1. */
static void no_event_products(const double p[8], const int64_t n[8], int start, double G[8]) {
  double g = 1.0;
  int k;
  for (k = start; k < 8; k++) {
    if (n[k] > 0 && p[k] > 0.0) g = g * powi(1.0 - p[k], n[k]);
    G[k] = g;
  }
}

double orc_no_event_prob(const double p[8], const int64_t n[8]) {
  double G[8];
  no_event_products(p, n, 0, G);
  return G[7];
}


static void sample_channels(const ectx_t *c, const double p[8], const int64_t n[8], int64_t X[8]) {
  int k, loud = 0, start;
  stream_t prim, s;
  for (k = 0; k < 8; k++) {
    X[k] = 0;
    if (n[k] > 0 && p[k] >= 1.0) loud = 1;
  }
  if (loud) {
    for (k = 0; k < 8; k++) {
      channel_stream(c, &s, DRAW_CH(k + 1));
      X[k] = bsplit(n[k], p[k], &s);
    }
    return;
  }
  channel_stream(c, &prim, 0);
  start = 0;
  while (start < 8) {
    double G[8], u;
    int first;
    no_event_products(p, n, start, G);
    u = stream_next(&prim);
    if (u < G[7]) break;
    first = start;
    while (u < G[first]) first++;
    channel_stream(c, &s, DRAW_CH(first + 1));
    X[first] = binom_trunc(n[first], p[first], &s);
    start = first + 1;
  }
}

int orc_channels_many(const double p[8], const int64_t n[8], uint64_t seed, int64_t count,
                      int64_t *out) {
  int64_t i;
  int err = 0;
  if (!fc_ready) fc_init();
  for (i = 0; i < count; i++) {
    ectx_t c;
    c.seed = seed; c.solve_id = 0; c.cfg = (uint64_t)i; c.step = 0; c.err = &err;
    sample_channels(&c, p, n, out + 8 * i);
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* Model: lattice, bonds, Liouvillian elements (Sec. V model; Sec. III.C     */
/* Kronecker form; Sec. IV.B weights).                                       */
/* ------------------------------------------------------------------------ */
int orc_bonds(int32_t Lx, int32_t Ly, int32_t *s1, int32_t *s2) {
  int nb = 0, s;
  int N = Lx * Ly;
  if (Lx < 2 || Ly < 2 || N > 32) return ORC_EINVAL;
  for (s = 0; s < N; s++) { /* right bonds */
    int x = s % Lx, y = s / Lx;
    if (Lx > 2 || x == 0) {
      s1[nb] = s;
      s2[nb] = (x + 1) % Lx + Lx * y;
      nb++;
    }
  }
  for (s = 0; s < N; s++) { /* up bonds */
    int x = s % Lx, y = s / Lx;
    if (Ly > 2 || y == 0) {
      s1[nb] = s;
      s2[nb] = x + Lx * ((y + 1) % Ly);
      nb++;
    }
  }
  return nb;
}

typedef struct {
  int N, nb;
  int s1[64], s2[64];
  uint64_t bmask[64];
  double h_al, h_an, a_al, a_an, w_dn, w_up, half_gamma, half_jz;
  int field;            /* the in-plane field is on */
  double hx, hy, ahx, ahy;
} model_t;

static int model_init(model_t *md, const orc_params *p) {
  int b;
  md->N = p->Lx * p->Ly;
  md->nb = orc_bonds(p->Lx, p->Ly, md->s1, md->s2);
  if (md->nb < 0) return md->nb;
  for (b = 0; b < md->nb; b++) md->bmask[b] = (1ull << md->s1[b]) | (1ull << md->s2[b]);
  md->h_al = (p->Jx - p->Jy) * 0.25;
  md->h_an = (p->Jx + p->Jy) * 0.25;
  md->a_al = fabs(md->h_al);
  md->a_an = fabs(md->h_an);
  md->w_dn = orc_det_exp(-p->is_p);
  md->w_up = orc_det_exp(p->is_p);
  md->half_gamma = 0.5 * p->gamma;
  md->half_jz = 0.5 * p->Jz;
  md->hx = p->hx;
  md->hy = p->hy;
  md->ahx = fabs(p->hx);
  md->ahy = fabs(p->hy);
  md->field = (p->hx != 0.0 || p->hy != 0.0);
  return ORC_OK;
}

static int bit(uint64_t x, int s) { return (int)((x >> s) & 1u); }
static int aligned(const model_t *md, uint64_t x, int b) {
  return bit(x, md->s1[b]) == bit(x, md->s2[b]);
}
static int n_aligned(const model_t *md, uint64_t x) {
  int b, c = 0;
  for (b = 0; b < md->nb; b++) c += aligned(md, x, b);
  return c;
}
static int popc(uint64_t x) {
  int c = 0;
  while (x) {
    c += (int)(x & 1u);
    x >>= 1;
  }
  return c;
}
static int64_t sgn64(int64_t x) { return (x > 0) - (x < 0); }
static int sgnd(double x) { return (x > 0.0) - (x < 0.0); }

/* Hop classes seen from parent (l, m), in the fixed order
 *   0 ket-aligned, 1 ket-anti, 2 ket to-diagonal, 3 bra-aligned, 4 bra-anti,
 *   5 bra to-diagonal.
 * "to-diagonal" is the one bond b (if any) with l ^ m == mask_b: flipping it on
 * either side makes the child diagonal.  Members are kept in bond order. */
typedef struct {
  int n[6];
  int mem[6][64];
  double W[6];   /* n_c * |element| * w_child / w_parent */
  int sgn[6];    /* sign of Im of the element */
} hop_classes_t;

static void hop_classes(const model_t *md, uint64_t l, uint64_t m, hop_classes_t *hc) {
  int T = -1, b, c, side;
  int diag = (l == m);
  for (b = 0; b < md->nb; b++)
    if ((l ^ m) == md->bmask[b]) T = b;
  for (c = 0; c < 6; c++) hc->n[c] = 0;
  for (side = 0; side < 2; side++) {
    uint64_t x = side ? m : l;
    for (b = 0; b < md->nb; b++) {
      c = 3 * side + (b == T ? 2 : (aligned(md, x, b) ? 0 : 1));
      hc->mem[c][hc->n[c]++] = b;
    }
  }
  for (c = 0; c < 6; c++) {
    int al = (c % 3 == 2) ? (T >= 0 ? aligned(md, l, T) : 1) : (c % 3 == 0);
    double amp = al ? md->a_al : md->a_an;
    double h = al ? md->h_al : md->h_an;
    double w = diag ? md->w_dn : (c % 3 == 2 ? md->w_up : 1.0);
    /* ket side: -i h  -> Im = -h ; bra side: +i h -> Im = +h (eq. for L-tilde) */
    hc->sgn[c] = (c < 3) ? -sgnd(h) : sgnd(h);
    hc->W[c] = ((double)hc->n[c] * amp) * w;
  }
}

int orc_connections(const orc_params *p, uint64_t ket, uint64_t bra, double S, uint64_t *cket,
                    uint64_t *cbra, double *re, double *im, int32_t cap, double *d_re,
                    double *d_im) {
  model_t md;
  hop_classes_t hc;
  int c, j, k, cnt = 0;
  if (model_init(&md, p) != ORC_OK) return ORC_EINVAL;
  hop_classes(&md, ket, bra, &hc);
  for (c = 0; c < 6; c++) {
    for (j = 0; j < hc.n[c]; j++) {
      int b = hc.mem[c][j];
      int al = (c % 3 == 2) ? aligned(&md, ket, b) : (c % 3 == 0);
      double w = (ket == bra) ? md.w_dn : (c % 3 == 2 ? md.w_up : 1.0);
      if (cnt >= cap) return ORC_ENOMEM;
      re[cnt] = 0.0;
      im[cnt] = (double)hc.sgn[c] * ((al ? md.a_al : md.a_an) * w);
      cket[cnt] = c < 3 ? (ket ^ md.bmask[b]) : ket;
      cbra[cnt] = c < 3 ? bra : (bra ^ md.bmask[b]);
      cnt++;
    }
  }
  for (k = 0; k < md.N; k++) {
    if (bit(ket, k) && bit(bra, k)) {
      if (cnt >= cap) return ORC_ENOMEM;
      cket[cnt] = ket & ~(1ull << k);
      cbra[cnt] = bra & ~(1ull << k);
      re[cnt] = p->gamma;
      im[cnt] = 0.0;
      cnt++;
    }
  }
  if (md.field) {
    /* single flips of the in-plane field: Re part hy (-1 for a flip up, +1 for a
     * flip down), Im part hx (-1 on the ket, +1 on the bra), times the IS weight */
    uint64_t d = ket ^ bra;
    int side;
    for (side = 0; side < 2; side++)
      for (k = 0; k < md.N; k++) {
        uint64_t x = side ? bra : ket;
        int to_diag = d == (1ull << k);
        double w = (ket == bra) ? md.w_dn : (to_diag ? md.w_up : 1.0);
        if (cnt >= cap) return ORC_ENOMEM;
        cket[cnt] = side ? ket : (ket ^ (1ull << k));
        cbra[cnt] = side ? (bra ^ (1ull << k)) : bra;
        re[cnt] = (bit(x, k) ? md.hy : -md.hy) * w;
        im[cnt] = (side ? md.hx : -md.hx) * w;
        cnt++;
      }
  }
  *d_re = -(md.half_gamma * (double)(popc(ket) + popc(bra))) - S;
  *d_im = md.half_jz * (double)(n_aligned(&md, bra) - n_aligned(&md, ket));
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* The walker state and one step.                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  int64_t re, im;
} contrib_t;

struct orc_t {
  orc_params p;
  model_t md;
  double delta_over_dt;
  int64_t n, cap;
  uint64_t *keys;
  int32_t *re, *im;
  double S;
  int32_t mode; /* 0 grow (S held), 1 vary */
  int64_t step, nw_prev;
  int64_t last[ORC_NSUM], acc[ORC_NSUM], n_accum;
  int64_t *series;
  int64_t series_len, series_cap;
  contrib_t *con;
  int64_t ncon, capcon;
};

#define SERIES_W (3 + ORC_NSUM)

static int reserve_list(orc_t *h, int64_t need) {
  if (need <= h->cap) return ORC_OK;
  {
    int64_t nc = h->cap ? h->cap : 64;
    uint64_t *k;
    int32_t *r, *i;
    while (nc < need) nc *= 2;
    k = (uint64_t *)realloc(h->keys, (size_t)nc * sizeof(uint64_t));
    if (!k) return ORC_ENOMEM;
    h->keys = k;
    r = (int32_t *)realloc(h->re, (size_t)nc * sizeof(int32_t));
    if (!r) return ORC_ENOMEM;
    h->re = r;
    i = (int32_t *)realloc(h->im, (size_t)nc * sizeof(int32_t));
    if (!i) return ORC_ENOMEM;
    h->im = i;
    h->cap = nc;
  }
  return ORC_OK;
}

static int push_contrib(orc_t *h, uint64_t key, int64_t re, int64_t im) {
  if (h->ncon == h->capcon) {
    int64_t nc = h->capcon ? 2 * h->capcon : 1024;
    contrib_t *c = (contrib_t *)realloc(h->con, (size_t)nc * sizeof(contrib_t));
    if (!c) return ORC_ENOMEM;
    h->con = c;
    h->capcon = nc;
  }
  h->con[h->ncon].key = key;
  h->con[h->ncon].re = re;
  h->con[h->ncon].im = im;
  h->ncon++;
  return ORC_OK;
}

static int in_list(const orc_t *h, uint64_t key) {
  int64_t lo = 0, hi = h->n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (h->keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo < h->n && h->keys[lo] == key;
}

typedef struct {
  orc_t *h;
  int init;    /* parent is an initiator */
  int rc;
} emit_t;

/* Progeny of a non-initiator survives only on a configuration occupied at the
 * start of the step or on the diagonal (Sec. IV.A). */
static void emit(emit_t *em, uint64_t cl, uint64_t cm, int64_t re, int64_t im) {
  int N = em->h->md.N;
  uint64_t key = (cl << N) | cm;
  if (!em->init && cl != cm && !in_list(em->h, key)) return;
  if (push_contrib(em->h, key, re, im) != ORC_OK) em->rc = ORC_ENOMEM;
}

/* Multinomial split of M walkers over members [lo, hi) of one class, equal
 * weights, by a balanced binary tree of binomials; node h of the heap. */
typedef struct {
  const ectx_t *ec;
  uint32_t draw_base; /* channel and class part of the draw id */
  int64_t *out;       /* per-member counts */
} tree_t;

static void tree_split(const tree_t *t, int lo, int hi, int hnode, int64_t M) {
  int mid;
  int64_t ML;
  stream_t s;
  if (M == 0) return;
  if (hi - lo == 1) {
    t->out[lo] += M;
    return;
  }
  mid = lo + (hi - lo) / 2;
  channel_stream(t->ec, &s, t->draw_base + (uint32_t)hnode);
  ML = binom(M, (double)(mid - lo) / (double)(hi - lo), &s);
  tree_split(t, lo, mid, 2 * hnode, ML);
  tree_split(t, mid, hi, 2 * hnode + 1, M - ML);
}

/* The in-plane field of Sec. V.B, h (cos theta sigma^x + sin theta sigma^y) per
 * site = hx sigma^x + hy sigma^y, flips one spin of the ket (-iH rho) or of the
 * bra (+i rho H).  With sigma^y |dn> = -i |up> the element from |l><m| to the
 * configuration with site s flipped has
 *   Re part hy (-1 if the flipped bit was 0, +1 if it was 1), on either side,
 *   Im part hx (-1 on the ket, +1 on the bra).
 * With the field on, each element part gets four classes of equal-weight
 * members: ket flips, the ket flip that makes the child diagonal (l ^ m one
 * bit), bra flips, the bra flip to the diagonal; their IS weights are those of
 * the hop classes.  The real part's classes come after the jump class, the
 * imaginary part's after the six hop classes.  Each member carries its child
 * and the sign of its element part. */
#define FMAX 10
typedef struct {
  int ncls;
  int n[FMAX];
  double W[FMAX];            /* n_c |element part| w_child / w_parent */
  double Sc[FMAX + 1];       /* suffix sums of W, Sc[ncls] = 0 */
  uint64_t cl[FMAX][64], cm[FMAX][64];
  int sgn[FMAX][64];         /* sign of the element part of each member */
} fclasses_t;

/* one class of single flips: side 0 ket, 1 bra; to_diag selects the flip of
 * site T (if any) or all the others */
static void field_class(const model_t *md, uint64_t l, uint64_t m, int side, int to_diag, int T,
                        int re_part, fclasses_t *f) {
  int c = f->ncls++, s;
  int diag = (l == m);
  double w = diag ? md->w_dn : (to_diag ? md->w_up : 1.0);
  f->n[c] = 0;
  for (s = 0; s < md->N; s++) {
    uint64_t x = side ? m : l;
    int k;
    if ((s == T) != (to_diag != 0)) continue;
    k = f->n[c]++;
    f->cl[c][k] = side ? l : (l ^ (1ull << s));
    f->cm[c][k] = side ? (m ^ (1ull << s)) : m;
    if (re_part)
      f->sgn[c][k] = sgnd(md->hy) * (bit(x, s) ? 1 : -1);
    else
      f->sgn[c][k] = sgnd(md->hx) * (side ? 1 : -1);
  }
  f->W[c] = ((double)f->n[c] * (re_part ? md->ahy : md->ahx)) * w;
}

/* The classes of the real element part with the field on: the jumps (weight
 * gamma each, sign +1), then the four field classes. */
static void field_re_classes(const model_t *md, double gamma, uint64_t l, uint64_t m,
                             fclasses_t *f) {
  int k, c, T = -1;
  uint64_t d = l ^ m;
  if (popc(d) == 1)
    for (k = 0; k < md->N; k++)
      if (d == (1ull << k)) T = k;
  f->ncls = 1;
  f->n[0] = 0;
  for (k = 0; k < md->N; k++)
    if (bit(l, k) && bit(m, k)) {
      int j = f->n[0]++;
      f->cl[0][j] = l & ~(1ull << k);
      f->cm[0][j] = m & ~(1ull << k);
      f->sgn[0][j] = 1;
    }
  f->W[0] = (double)f->n[0] * gamma;
  field_class(md, l, m, 0, 0, T, 1, f);
  field_class(md, l, m, 0, 1, T, 1, f);
  field_class(md, l, m, 1, 0, T, 1, f);
  field_class(md, l, m, 1, 1, T, 1, f);
  f->Sc[f->ncls] = 0.0;
  f->Sc[f->ncls - 1] = f->W[f->ncls - 1];
  for (c = f->ncls - 2; c >= 0; c--) f->Sc[c] = f->W[c] + f->Sc[c + 1];
}

/* The classes of the imaginary element part with the field on: the six hop
 * classes, then the four field classes. */
static void field_im_classes(const model_t *md, const hop_classes_t *hc, uint64_t l, uint64_t m,
                             fclasses_t *f) {
  int k, c, j, T = -1;
  uint64_t d = l ^ m;
  if (popc(d) == 1)
    for (k = 0; k < md->N; k++)
      if (d == (1ull << k)) T = k;
  f->ncls = 6;
  for (c = 0; c < 6; c++) {
    f->n[c] = hc->n[c];
    f->W[c] = hc->W[c];
    for (j = 0; j < hc->n[c]; j++) {
      int b = hc->mem[c][j];
      f->cl[c][j] = c < 3 ? (l ^ md->bmask[b]) : l;
      f->cm[c][j] = c < 3 ? m : (m ^ md->bmask[b]);
      f->sgn[c][j] = hc->sgn[c];
    }
  }
  field_class(md, l, m, 0, 0, T, 0, f);
  field_class(md, l, m, 0, 1, T, 0, f);
  field_class(md, l, m, 1, 0, T, 0, f);
  field_class(md, l, m, 1, 1, T, 0, f);
  f->Sc[f->ncls] = 0.0;
  f->Sc[f->ncls - 1] = f->W[f->ncls - 1];
  for (c = f->ncls - 2; c >= 0; c--) f->Sc[c] = f->W[c] + f->Sc[c + 1];
}

/* Draw id, within a channel, of the class split of class c (the ids below 16
 * keep their meaning of the field-free step; the pick is DRAW_PICK). */
static uint32_t class_split_draw(int c) { return c < 6 ? 1u + (uint32_t)c : 16u + (uint32_t)c; }

/* Placement of rem walkers of one channel over field-on classes (Sec. III.B):
 * one walker by one categorical pick (class by inversion on the suffix sums,
 * then a uniform member); more walkers by sequential conditional binomials over
 * the classes (the last class with weight takes the rest) and the balanced tree
 * inside each class.  cnt[c][j] receives member j of class c. */
static void place_field(const ectx_t *ec, int ch, int64_t rem, const fclasses_t *f,
                        int64_t cnt[FMAX][64]) {
  int c, j, last = -1;
  for (c = 0; c < f->ncls; c++)
    for (j = 0; j < f->n[c]; j++) cnt[c][j] = 0;
  if (rem == 0) return;
  if (rem == 1) {
    stream_t s;
    double u1, u2, T;
    int jj;
    channel_stream(ec, &s, DRAW_CH(ch) + DRAW_PICK);
    u1 = stream_next(&s);
    u2 = stream_next(&s);
    T = f->Sc[0] * (1.0 - u1);
    c = 0;
    while (!(f->Sc[c + 1] < T)) c++;
    jj = (int)floor(u2 * (double)f->n[c]);
    if (jj > f->n[c] - 1) jj = f->n[c] - 1;
    cnt[c][jj] = 1;
    return;
  }
  for (c = 0; c < f->ncls; c++)
    if (f->W[c] > 0.0) last = c;
  for (c = 0; c < f->ncls && rem > 0; c++) {
    int64_t Mc;
    tree_t t;
    stream_t s;
    if (f->W[c] == 0.0) continue;
    if (c == last) {
      Mc = rem;
    } else {
      channel_stream(ec, &s, DRAW_CH(ch) + class_split_draw(c));
      Mc = binom(rem, f->W[c] / f->Sc[c], &s);
    }
    rem -= Mc;
    if (Mc == 0) continue;
    t.ec = ec; t.draw_base = DRAW_CH(ch) + 64u + 64u * (uint32_t)c; t.out = cnt[c];
    tree_split(&t, 0, f->n[c], 1, Mc);
  }
}

/* Placement of the Xs walkers a real-element (jump) channel spawns over the
 * nJ sites where ket and bra are both up (Sec. III.B: the multinomial over
 * equally weighted connections): one walker takes a uniform site, more are
 * split by the balanced binomial tree.  cnt[j] receives site j's count. */
static void place_jumps(const ectx_t *ec, int ch, int64_t Xs, int nJ, int64_t *cnt) {
  int j;
  for (j = 0; j < nJ; j++) cnt[j] = 0;
  if (Xs == 0) return;
  if (Xs == 1) {
    stream_t s;
    int jj;
    channel_stream(ec, &s, DRAW_CH(ch) + DRAW_PICK);
    jj = (int)floor(stream_next(&s) * (double)nJ);
    if (jj > nJ - 1) jj = nJ - 1;
    cnt[jj] = 1;
  } else {
    tree_t t;
    t.ec = ec; t.draw_base = DRAW_CH(ch) + 64u; t.out = cnt;
    tree_split(&t, 0, nJ, 1, Xs);
  }
}

/* Placement of the rem walkers an imaginary-element (hop) channel spawns over
 * the hop classes and their members (Sec. III.B: the multinomial over the
 * connections with weights |element| x IS weight): one walker by one
 * categorical pick (its class by inversion on the suffix sums Sc of the class
 * weights, then a uniform member); more walkers by sequential conditional
 * binomials over the classes (the last class with weight takes the rest), then
 * the balanced binomial tree inside each class.  cnt[c][j] receives member j
 * of class c. */
static void place_hops(const ectx_t *ec, int ch, int64_t rem, const hop_classes_t *hc,
                       const double Sc[6], int64_t cnt[6][64]) {
  int c, j, last = -1;
  for (c = 0; c < 6; c++)
    for (j = 0; j < hc->n[c]; j++) cnt[c][j] = 0;
  if (rem == 0) return;
  if (rem == 1) {
    stream_t s;
    double u1, u2, T;
    int jj;
    channel_stream(ec, &s, DRAW_CH(ch) + DRAW_PICK);
    u1 = stream_next(&s);
    u2 = stream_next(&s);
    T = Sc[0] * (1.0 - u1);
    c = 0;
    while (!((c < 5 ? Sc[c + 1] : 0.0) < T)) c++;
    jj = (int)floor(u2 * (double)hc->n[c]);
    if (jj > hc->n[c] - 1) jj = hc->n[c] - 1;
    cnt[c][jj] = 1;
    return;
  }
  for (c = 0; c < 6; c++)
    if (hc->W[c] > 0.0) last = c;
  for (c = 0; c < 6 && rem > 0; c++) {
    int64_t Mc;
    tree_t t;
    stream_t s;
    if (hc->W[c] == 0.0) continue;
    if (c == last) {
      Mc = rem;
    } else {
      channel_stream(ec, &s, DRAW_CH(ch) + 1u + (uint32_t)c);
      Mc = binom(rem, hc->W[c] / Sc[c], &s);
    }
    rem -= Mc;
    if (Mc == 0) continue;
    t.ec = ec; t.draw_base = DRAW_CH(ch) + 64u + 64u * (uint32_t)c; t.out = cnt[c];
    tree_split(&t, 0, hc->n[c], 1, Mc);
  }
}

/* Per-walker sampling, the rules of Sec. II taken walker by walker (the
 * alternative to the multinomial formalism of Sec. III.B): each walker of the
 * entry's real or imaginary part
 *   - dies / clones along the diagonal element's real part (probability
 *     dt |d_r|) and transfers along its imaginary part (dt |d_i|), each an
 *     integer part realised for sure plus a Bernoulli draw of the fraction;
 *   - makes one spawning attempt along the real element part: a jump site chosen
 *     uniformly among the nJ connections, success probability nJ dt gamma;
 *   - makes one along the imaginary element part: a hop chosen uniformly among
 *     the nh hop connections (all six classes), success probability
 *     nh dt |element| w_child / w_parent; a probability above 1 realises its
 *     integer part for sure and draws the fraction.
 * Walker w of part q draws its six uniforms from the stream with draw id
 * 0x8000 + q * 2^13 + (w >> 14), blocks 4 (w mod 2^14) .. + 2 (so at most 2^27
 * walkers per part of an entry).  The expectation is the Euler map, as with
 * the multinomial scheme; the law of the spawned counts differs (a uniform
 * choice of connection instead of one proportional to the element). */
#define PW_MAX_WALKERS (1ll << 27)
static double pw_frac_count(double p, double u, int64_t *c) {
  double f = floor(p);
  *c = (int64_t)f + ((u < p - f) ? 1 : 0);
  return f;
}

static void per_walker_entry(orc_t *h, uint64_t key, uint64_t l, uint64_t m, int32_t R, int32_t I,
                             double d_r, double d_i, double p_r, double p_i,
                             const hop_classes_t *hc, const int *jsite, int nJ, emit_t *em,
                             int64_t *dR, int64_t *dI, int *err) {
  const model_t *md = &h->md;
  int part, c;
  int nh = 0;
  uint64_t diag = (l == m);
  for (c = 0; c < 6; c++) nh += hc->n[c];
  *dR = 0;
  *dI = 0;
  for (part = 0; part < 2; part++) {
    int64_t n = part ? (I < 0 ? -(int64_t)I : I) : (R < 0 ? -(int64_t)R : R);
    int64_t sg = part ? sgn64(I) : sgn64(R);
    int64_t w;
    if (n > PW_MAX_WALKERS) {
      *err = ORC_ERNG;
      return;
    }
    for (w = 0; w < n; w++) {
      stream_t s;
      double u[6];
      int64_t cr, ci, cs;
      int k;
      stream_init(&s, h->p.seed, h->p.solve_id, key, (uint32_t)h->step,
                  0x8000u + ((uint32_t)part << 13) + (uint32_t)(w >> 14), err);
      s.block = 4u * (uint32_t)(w & 0x3FFF);
      for (k = 0; k < 6; k++) u[k] = stream_next(&s);
      /* clone/death: (R + iI)(d_r + i d_i) dt, walker by walker */
      pw_frac_count(p_r, u[0], &cr);
      pw_frac_count(p_i, u[1], &ci);
      if (part == 0) {
        *dR += sg * sgnd(d_r) * cr;
        *dI += sg * sgnd(d_i) * ci;
      } else {
        *dI += sg * sgnd(d_r) * cr;
        *dR -= sg * sgnd(d_i) * ci;
      }
      /* one attempt along the real part: a uniform jump site */
      if (nJ > 0) {
        int j = (int)floor(u[2] * (double)nJ);
        uint64_t bitk;
        if (j > nJ - 1) j = nJ - 1;
        pw_frac_count(h->p.dt * ((double)nJ * h->p.gamma), u[3], &cs);
        bitk = 1ull << jsite[j];
        if (cs) {
          if (part == 0) emit(em, l & ~bitk, m & ~bitk, sg * cs, 0);
          else emit(em, l & ~bitk, m & ~bitk, 0, sg * cs);
        }
      }
      /* one attempt along the imaginary part: a uniform hop among all classes */
      if (nh > 0) {
        int j = (int)floor(u[4] * (double)nh), b, al, T = -1, bb;
        double amp, wgt;
        uint64_t cl, cm;
        if (j > nh - 1) j = nh - 1;
        c = 0;
        while (j >= hc->n[c]) j -= hc->n[c++];
        b = hc->mem[c][j];
        for (bb = 0; bb < md->nb; bb++)
          if ((l ^ m) == md->bmask[bb]) T = bb;
        al = (c % 3 == 2) ? (T >= 0 ? aligned(md, l, T) : 1) : (c % 3 == 0);
        amp = al ? md->a_al : md->a_an;
        wgt = diag ? md->w_dn : (c % 3 == 2 ? md->w_up : 1.0);
        pw_frac_count(h->p.dt * (((double)nh * amp) * wgt), u[5], &cs);
        cl = c < 3 ? (l ^ md->bmask[b]) : l;
        cm = c < 3 ? m : (m ^ md->bmask[b]);
        if (cs) {
          int64_t v = sg * (int64_t)hc->sgn[c] * cs;
          if (part == 0) emit(em, cl, cm, 0, v);
          else emit(em, cl, cm, -v, 0);
        }
      }
    }
  }
}

static void process_entry(orc_t *h, uint64_t key, int32_t R, int32_t I, int64_t *dR, int64_t *dI,
                          int *err) {
  const model_t *md = &h->md;
  int N = md->N;
  uint64_t mask = (N == 32) ? 0xffffffffull : ((1ull << N) - 1);
  uint64_t l = key >> N, m = key & mask;
  int diag = (l == m);
  int64_t nR = R < 0 ? -(int64_t)R : R, nI = I < 0 ? -(int64_t)I : I;
  int64_t sR = sgn64(R), sI = sgn64(I);
  double d_r, d_i, p_r, p_i, Sc[6], P_im, P_re;
  hop_classes_t hc;
  int jsite[64], nJ = 0, k, c;
  double p[8];
  int64_t n[8], X[8];
  ectx_t ec;
  emit_t em;

  ec.seed = h->p.seed; ec.solve_id = h->p.solve_id; ec.cfg = key;
  ec.step = (uint32_t)h->step; ec.err = err;
  em.h = h;
  em.init = diag || (nR + nI > (int64_t)h->p.n_a) || (h->p.flags & ORC_NO_INITIATOR);
  em.rc = ORC_OK;

  /* diagonal element: Re = -(gamma/2)(n_up(l) + n_up(m)) - S, Im = -(E_l - E_m) */
  d_r = -(md->half_gamma * (double)(popc(l) + popc(m))) - h->S;
  d_i = md->half_jz * (double)(n_aligned(md, m) - n_aligned(md, l));
  p_r = h->p.dt * fabs(d_r);
  p_i = h->p.dt * fabs(d_i);

  hop_classes(md, l, m, &hc);
  Sc[5] = hc.W[5];
  for (c = 4; c >= 0; c--) Sc[c] = hc.W[c] + Sc[c + 1];
  P_im = h->p.dt * Sc[0];

  for (k = 0; k < N; k++)
    if (bit(l, k) && bit(m, k)) jsite[nJ++] = k;
  P_re = h->p.dt * ((double)nJ * h->p.gamma);

  if (h->p.flags & ORC_PER_WALKER) {
    per_walker_entry(h, key, l, m, R, I, d_r, d_i, p_r, p_i, &hc, jsite, nJ, &em, dR, dI, err);
    if (em.rc != ORC_OK) *err = em.rc;
    return;
  }

  if (md->field) {
    /* the in-plane field adds single-flip classes to both element parts */
    static fclasses_t fre, fim; /* (large; the oracle is single-threaded) */
    int64_t fcnt[FMAX][64];
    field_re_classes(md, h->p.gamma, l, m, &fre);
    field_im_classes(md, &hc, l, m, &fim);
    P_re = h->p.dt * fre.Sc[0];
    P_im = h->p.dt * fim.Sc[0];
    p[0] = p_r; p[1] = p_i; p[2] = P_re; p[3] = P_im;
    p[4] = p_r; p[5] = p_i; p[6] = P_re; p[7] = P_im;
    for (k = 0; k < 4; k++) { n[k] = nR; n[k + 4] = nI; }
    sample_channels(&ec, p, n, X);
    *dR = sR * sgnd(d_r) * X[0] - sI * sgnd(d_i) * X[5];
    *dI = sI * sgnd(d_r) * X[4] + sR * sgnd(d_i) * X[1];
    for (k = 0; k < 4; k++) {
      int ch = (k & 1) ? (k < 2 ? 7 : 8) : (k < 2 ? 3 : 4); /* 3, 7, 4, 8 */
      int im_el = k >= 2;           /* element part: 0 Re (channels 3, 7), 1 Im (4, 8) */
      int im_par = (k & 1) != 0;    /* parent part: 0 real walkers, 1 imaginary */
      const fclasses_t *f = im_el ? &fim : &fre;
      int64_t sg = im_par ? sI : sR;
      int j;
      if (X[ch - 1] == 0) continue;
      place_field(&ec, ch, X[ch - 1], f, fcnt);
      for (c = 0; c < f->ncls; c++)
        for (j = 0; j < f->n[c]; j++) {
          int64_t v;
          if (fcnt[c][j] == 0) continue;
          v = sg * (int64_t)f->sgn[c][j] * fcnt[c][j];
          /* (R + iI) x element part: Re x R -> re, Re x I -> im, Im x R -> im,
           * Im x I -> -re (Sec. III.C rule (i)) */
          if (!im_el && !im_par) emit(&em, f->cl[c][j], f->cm[c][j], v, 0);
          else if (!im_el) emit(&em, f->cl[c][j], f->cm[c][j], 0, v);
          else if (!im_par) emit(&em, f->cl[c][j], f->cm[c][j], 0, v);
          else emit(&em, f->cl[c][j], f->cm[c][j], -v, 0);
        }
    }
    if (em.rc != ORC_OK) *err = em.rc;
    return;
  }

  p[0] = p_r; p[1] = p_i; p[2] = P_re; p[3] = P_im;
  p[4] = p_r; p[5] = p_i; p[6] = P_re; p[7] = P_im;
  for (k = 0; k < 4; k++) { n[k] = nR; n[k + 4] = nI; }
  sample_channels(&ec, p, n, X);

  /* clone/death: (R + iI)(d_r + i d_i) dt, one count per (part, Re/Im) */
  *dR = sR * sgnd(d_r) * X[0] - sI * sgnd(d_i) * X[5];
  *dI = sI * sgnd(d_r) * X[4] + sR * sgnd(d_i) * X[1];

  /* spawning along the real elements (jumps gamma S^- rho S^+) */
  for (k = 0; k < 2; k++) {
    int ch = k ? 7 : 3; /* 1-based channel number */
    int64_t cnt[64];
    int64_t sg = k ? sI : sR;
    int j;
    if (X[ch - 1] == 0) continue;
    place_jumps(&ec, ch, X[ch - 1], nJ, cnt);
    for (j = 0; j < nJ; j++) {
      if (cnt[j] == 0) continue;
      {
        uint64_t bitk = 1ull << jsite[j];
        if (k == 0) emit(&em, l & ~bitk, m & ~bitk, sg * cnt[j], 0);
        else emit(&em, l & ~bitk, m & ~bitk, 0, sg * cnt[j]);
      }
    }
  }

  /* spawning along the imaginary elements (hops -iH on the ket, +iH on the bra):
   * the channel's walkers placed over the classes and their members */
  for (k = 0; k < 2; k++) {
    int ch = k ? 8 : 4;
    int64_t sg = k ? sI : sR;
    int64_t cnt[6][64];
    if (X[ch - 1] == 0) continue;
    place_hops(&ec, ch, X[ch - 1], &hc, Sc, cnt);
    for (c = 0; c < 6; c++) {
      int j;
      for (j = 0; j < hc.n[c]; j++) {
        int b = hc.mem[c][j];
        int64_t v;
        uint64_t cl, cm;
        if (cnt[c][j] == 0) continue;
        v = sg * (int64_t)hc.sgn[c] * cnt[c][j];
        cl = c < 3 ? (l ^ md->bmask[b]) : l;
        cm = c < 3 ? m : (m ^ md->bmask[b]);
        /* real parent x Im element -> imaginary child; imaginary parent x Im
         * element -> real child with a minus sign (Sec. III.C, rule (i)) */
        if (k == 0) emit(&em, cl, cm, 0, v);
        else emit(&em, cl, cm, -v, 0);
      }
    }
  }
  if (em.rc != ORC_OK) *err = em.rc;
}

static int cmp_contrib(const void *a, const void *b) {
  uint64_t x = ((const contrib_t *)a)->key, y = ((const contrib_t *)b)->key;
  return (x > y) - (x < y);
}

/* Annihilation (Sec. III.C, the third rule): every contribution summed per
 * configuration, the sums added to the step-start list (sorted unique keys,
 * values already moved by their own clone/death), and every configuration whose
 * total is zero dropped.  con is sorted and compacted in place; the new list,
 * sorted, goes to nk/nre/nim, which must hold n + ncon entries; *nout is its
 * length.  ORC_EOVERFLOW when a total leaves the int32 range. */
static int annihilate(contrib_t *con, int64_t ncon, const uint64_t *keys, const int64_t *pr,
                      const int64_t *pi, int64_t n, uint64_t *nk, int64_t *nre, int64_t *nim,
                      int64_t *nout) {
  int64_t i, a = 0, u = 0, nu = 0, j = 0;
  qsort(con, (size_t)ncon, sizeof(contrib_t), cmp_contrib);
  for (i = 0; i < ncon; i++) {
    if (nu > 0 && con[nu - 1].key == con[i].key) {
      con[nu - 1].re += con[i].re;
      con[nu - 1].im += con[i].im;
    } else {
      con[nu++] = con[i];
    }
  }
  while (a < n || u < nu) {
    uint64_t key;
    int64_t R, I;
    if (u >= nu || (a < n && keys[a] < con[u].key)) {
      key = keys[a]; R = pr[a]; I = pi[a]; a++;
    } else if (a >= n || con[u].key < keys[a]) {
      key = con[u].key; R = con[u].re; I = con[u].im; u++;
    } else {
      key = keys[a]; R = pr[a] + con[u].re; I = pi[a] + con[u].im; a++; u++;
    }
    if (R == 0 && I == 0) continue;
    if (R > 2147483647LL || R < -2147483647LL || I > 2147483647LL || I < -2147483647LL)
      return ORC_EOVERFLOW;
    nk[j] = key; nre[j] = R; nim[j] = I; j++;
  }
  *nout = j;
  return ORC_OK;
}

int orc_annihilate(const uint64_t *ckeys, const int64_t *cre, const int64_t *cim, int64_t ncon,
                   const uint64_t *keys, const int64_t *pr, const int64_t *pi, int64_t n,
                   uint64_t *nk, int64_t *nre, int64_t *nim, int64_t *nout) {
  int64_t i;
  int rc;
  contrib_t *con;
  if (ncon < 0 || n < 0 || !nout) return ORC_EINVAL;
  con = (contrib_t *)malloc((size_t)(ncon ? ncon : 1) * sizeof(contrib_t));
  if (!con) return ORC_ENOMEM;
  for (i = 0; i < ncon; i++) {
    con[i].key = ckeys[i];
    con[i].re = cre[i];
    con[i].im = cim[i];
  }
  rc = annihilate(con, ncon, keys, pr, pi, n, nk, nre, nim, nout);
  free(con);
  return rc;
}

static void estimator_sums(const orc_t *h, const uint64_t *keys, const int64_t *re,
                           const int64_t *im, int64_t n, int64_t out[ORC_NSUM]) {
  const model_t *md = &h->md;
  int N = md->N, b;
  uint64_t mask = (N == 32) ? 0xffffffffull : ((1ull << N) - 1);
  int64_t i;
  for (b = 0; b < ORC_NSUM; b++) out[b] = 0;
  for (i = 0; i < n; i++) {
    uint64_t l = keys[i] >> N, m = keys[i] & mask, d = l ^ m;
    int64_t R = re[i], I = im[i];
    out[ORC_WTOT] += (R < 0 ? -R : R) + (I < 0 ? -I : I);
    out[ORC_NENT] += 1;
    if (l == m) {
      out[ORC_T_RE] += R;
      out[ORC_T_IM] += I;
      out[ORC_NW] += R < 0 ? -R : R;
      out[ORC_Z] += R * (int64_t)(2 * popc(l) - N);
      out[ORC_CZZ] += R * (int64_t)(2 * n_aligned(md, l) - md->nb);
    }
    if (popc(d) == 1) {
      /* Tr(rho sigma^x_k) and Tr(rho sigma^y_k), real parts */
      out[ORC_X] += R;
      out[ORC_Y] += (l & d) ? -I : I;
    }
    for (b = 0; b < md->nb; b++) {
      if (d == md->bmask[b]) {
        out[ORC_CXX] += R;
        out[ORC_CYY] += aligned(md, l, b) ? -R : R;
      }
    }
  }
}

static int one_step(orc_t *h) {
  int64_t i, j, nn;
  int err = ORC_OK;
  int64_t *pr = (int64_t *)malloc((size_t)(h->n ? h->n : 1) * sizeof(int64_t));
  int64_t *pi = (int64_t *)malloc((size_t)(h->n ? h->n : 1) * sizeof(int64_t));
  uint64_t *nk = NULL;
  int64_t *nre = NULL, *nim = NULL, sums[ORC_NSUM];
  if (!pr || !pi) { free(pr); free(pi); return ORC_ENOMEM; }
  h->ncon = 0;

  /* spawning and clone/death, entry by entry */
  for (i = 0; i < h->n; i++) {
    int64_t dR, dI;
    process_entry(h, h->keys[i], h->re[i], h->im[i], &dR, &dI, &err);
    pr[i] = (int64_t)h->re[i] + dR;
    pi[i] = (int64_t)h->im[i] + dI;
  }
  if (err != ORC_OK) { free(pr); free(pi); return err; }

  /* annihilation: sum every contribution per configuration, merge with the list */
  nn = h->n + h->ncon;
  nk = (uint64_t *)malloc((size_t)(nn ? nn : 1) * sizeof(uint64_t));
  nre = (int64_t *)malloc((size_t)(nn ? nn : 1) * sizeof(int64_t));
  nim = (int64_t *)malloc((size_t)(nn ? nn : 1) * sizeof(int64_t));
  if (!nk || !nre || !nim) { err = ORC_ENOMEM; goto done; }
  err = annihilate(h->con, h->ncon, h->keys, pr, pi, h->n, nk, nre, nim, &j);
  if (err != ORC_OK) goto done;
  estimator_sums(h, nk, nre, nim, j, sums);
  if (j == 0) { err = ORC_EEXTINCT; goto done; }

  /* population control on the diagonal real weight N_w (Sec. III.C) */
  {
    double S = h->S;
    int32_t mode = h->mode;
    int64_t nw = sums[ORC_NW];
    if (mode == 0) {
      if (nw >= h->p.target_walkers) mode = 1;
    } else {
      if (nw == 0 || h->nw_prev == 0) { err = ORC_EEXTINCT; goto done; }
      S = S + h->delta_over_dt * orc_det_log((double)nw / (double)h->nw_prev);
    }
    /* commit */
    if ((err = reserve_list(h, j)) != ORC_OK) goto done;
    for (i = 0; i < j; i++) {
      h->keys[i] = nk[i];
      h->re[i] = (int32_t)nre[i];
      h->im[i] = (int32_t)nim[i];
    }
    h->n = j;
    h->S = S;
    h->mode = mode;
    h->nw_prev = nw;
    h->step += 1;
    memcpy(h->last, sums, sizeof(sums));
    if (h->step > h->p.n_equil) {
      for (i = 0; i < ORC_NSUM; i++) h->acc[i] += sums[i];
      h->n_accum += 1;
    }
    if (h->series_len == h->series_cap) {
      int64_t nc = h->series_cap ? 2 * h->series_cap : 1024;
      int64_t *s = (int64_t *)realloc(h->series, (size_t)(nc * SERIES_W) * sizeof(int64_t));
      if (!s) { err = ORC_ENOMEM; goto done; }
      h->series = s;
      h->series_cap = nc;
    }
    {
      int64_t *row = h->series + h->series_len * SERIES_W;
      uint64_t sb = dbits(S);
      row[0] = h->step;
      memcpy(&row[1], &sb, 8);
      row[2] = mode;
      for (i = 0; i < ORC_NSUM; i++) row[3 + i] = sums[i];
      h->series_len++;
    }
  }
done:
  free(pr); free(pi); free(nk); free(nre); free(nim);
  return err;
}

int orc_create(const orc_params *p, orc_t **out) {
  orc_t *h;
  int rc;
  if (!p || !out) return ORC_EINVAL;
  /* the per-walker sampler covers the field-free model only */
  if ((p->flags & ORC_PER_WALKER) && (p->hx != 0.0 || p->hy != 0.0)) return ORC_EINVAL;
  if (p->Lx < 2 || p->Ly < 2 || p->Lx * p->Ly > 32 || !(p->gamma > 0.0) || !(p->dt > 0.0) ||
      p->n_a < 0 || p->initial_walkers <= 0 || p->initial_walkers > 2147483647LL ||
      p->is_p < 0.0 || p->solve_id >= 65536u)
    return ORC_EINVAL;
  if (!fc_ready) fc_init();
  h = (orc_t *)calloc(1, sizeof(orc_t));
  if (!h) return ORC_ENOMEM;
  h->p = *p;
  if ((rc = model_init(&h->md, p)) != ORC_OK) { free(h); return rc; }
  h->delta_over_dt = p->shift_damping / p->dt;
  if ((rc = reserve_list(h, 1)) != ORC_OK) { orc_destroy(h); return rc; }
  h->keys[0] = 0;
  h->re[0] = (int32_t)p->initial_walkers;
  h->im[0] = 0;
  h->n = 1;
  h->S = p->shift_init;
  h->mode = 0;
  h->step = 0;
  h->nw_prev = p->initial_walkers;
  *out = h;
  return ORC_OK;
}

void orc_destroy(orc_t *h) {
  if (!h) return;
  free(h->keys); free(h->re); free(h->im); free(h->series); free(h->con);
  free(h);
}

int orc_step(orc_t *h, int64_t n_steps) {
  int64_t i;
  for (i = 0; i < n_steps; i++) {
    int rc = one_step(h);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

int64_t orc_size(const orc_t *h) { return h->n; }

int orc_get_list(const orc_t *h, uint64_t *keys, int32_t *re, int32_t *im, int64_t cap) {
  if (cap < h->n) return ORC_EINVAL;
  memcpy(keys, h->keys, (size_t)h->n * sizeof(uint64_t));
  memcpy(re, h->re, (size_t)h->n * sizeof(int32_t));
  memcpy(im, h->im, (size_t)h->n * sizeof(int32_t));
  return ORC_OK;
}

int orc_set_list(orc_t *h, const uint64_t *keys, const int32_t *re, const int32_t *im,
                 int64_t n) {
  int64_t i;
  int rc;
  for (i = 0; i < n; i++) {
    if (i > 0 && keys[i] <= keys[i - 1]) return ORC_EINVAL;
    if (re[i] == 0 && im[i] == 0) return ORC_EINVAL;
    if (re[i] == INT32_MIN || im[i] == INT32_MIN) return ORC_EINVAL;
  }
  if ((rc = reserve_list(h, n)) != ORC_OK) return rc;
  memcpy(h->keys, keys, (size_t)n * sizeof(uint64_t));
  memcpy(h->re, re, (size_t)n * sizeof(int32_t));
  memcpy(h->im, im, (size_t)n * sizeof(int32_t));
  h->n = n;
  return ORC_OK;
}

int orc_get_scalars(const orc_t *h, double *S, int32_t *mode, int64_t *step, int64_t *nw_prev) {
  *S = h->S; *mode = h->mode; *step = h->step; *nw_prev = h->nw_prev;
  return ORC_OK;
}

int orc_set_scalars(orc_t *h, double S, int32_t mode, int64_t step, int64_t nw_prev) {
  h->S = S; h->mode = mode; h->step = step; h->nw_prev = nw_prev;
  return ORC_OK;
}

int orc_get_last(const orc_t *h, int64_t out[ORC_NSUM]) {
  memcpy(out, h->last, sizeof(h->last));
  return ORC_OK;
}

int orc_get_acc(const orc_t *h, int64_t out[ORC_NSUM], int64_t *n_accum) {
  memcpy(out, h->acc, sizeof(h->acc));
  *n_accum = h->n_accum;
  return ORC_OK;
}

int64_t orc_series_len(const orc_t *h) { return h->series_len; }

int orc_get_series(const orc_t *h, int64_t *rows, int64_t cap_rows) {
  if (cap_rows < h->series_len) return ORC_EINVAL;
  memcpy(rows, h->series, (size_t)(h->series_len * SERIES_W) * sizeof(int64_t));
  return ORC_OK;
}

/* Test entry point: X walkers of spawning channel `channel` of the entry `key`
 * placed over its connections by the step's own code (place_jumps /
 * place_hops), count times, sample i drawing at step i.  Channels 3 and 7
 * (jumps): rows of N counts by site (0 where ket and bra are not both up).
 * Channels 4 and 8 (hops): rows of 2 nb counts, ket bond b at column b and bra
 * bond b at column nb + b.  Returns the row width, or a negative code. */
int orc_split_many(const orc_params *p, uint64_t key, int channel, int64_t X, int64_t count,
                   int64_t *out) {
  model_t md;
  int N, rc, width, k, err = 0;
  uint64_t mask, l, m;
  int64_t i;
  if (!p || !out || X < 0 || count < 0) return ORC_EINVAL;
  if (channel != 3 && channel != 4 && channel != 7 && channel != 8) return ORC_EINVAL;
  rc = model_init(&md, p);
  if (rc != ORC_OK) return rc;
  N = md.N;
  mask = (N == 32) ? 0xffffffffull : ((1ull << N) - 1);
  l = key >> N;
  m = key & mask;
  width = (channel == 3 || channel == 7) ? N : 2 * md.nb;
  for (i = 0; i < count; i++) {
    ectx_t ec;
    int64_t *row = out + i * width;
    ec.seed = p->seed; ec.solve_id = p->solve_id; ec.cfg = key; ec.step = (uint32_t)i;
    ec.err = &err;
    for (k = 0; k < width; k++) row[k] = 0;
    if (channel == 3 || channel == 7) {
      int jsite[64], nJ = 0, j;
      int64_t cnt[64];
      for (k = 0; k < N; k++)
        if (bit(l, k) && bit(m, k)) jsite[nJ++] = k;
      if (nJ == 0) return ORC_EINVAL;
      place_jumps(&ec, channel, X, nJ, cnt);
      for (j = 0; j < nJ; j++) row[jsite[j]] = cnt[j];
    } else {
      hop_classes_t hc;
      double Sc[6];
      int64_t cnt[6][64];
      int c, j;
      hop_classes(&md, l, m, &hc);
      Sc[5] = hc.W[5];
      for (c = 4; c >= 0; c--) Sc[c] = hc.W[c] + Sc[c + 1];
      if (!(Sc[0] > 0.0)) return ORC_EINVAL;
      place_hops(&ec, channel, X, &hc, Sc, cnt);
      for (c = 0; c < 6; c++)
        for (j = 0; j < hc.n[c]; j++) row[(c < 3 ? 0 : md.nb) + hc.mem[c][j]] += cnt[c][j];
    }
  }
  return err ? err : width;
}
