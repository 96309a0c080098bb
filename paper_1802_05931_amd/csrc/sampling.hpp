// Counter-based random streams and exact binomial samplers for the DDQMC step.
//
// The multinomial formalism (arXiv:1802.05931, Sec. III.B) draws the number of
// spawning events of an occupied configuration as Bin(N_i, P_tot) and splits
// them over the connected configurations by a multinomial; clone/death
// (Sec. II rule (ii), Sec. III.C rule (ii)) is a binomial count as well.  The
// paper points to BINV- and BTRD-type generators for these.  Everything below
// uses fp64 +, -, *, / (and floor / fabs / sqrt, which round exactly) in a fixed
// order; the translation unit is built with -ffp-contract=off so no product is
// fused into an add.  The same arithmetic runs in host code (constants) and on
// the device (the step).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DQ_HD __host__ __device__ __forceinline__

namespace ddqmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplies with the round keys bumped by the Weyl constants.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x0, x1, x2, x3;
};

DQ_HD U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)0xD2511F53u * c0;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t y0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    const uint32_t y2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = y0;
    c2 = y2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// 53-bit uniform on [0, 1): 27 high bits of a, 26 high bits of b.
DQ_HD double unit53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// One draw's stream: key (seed_lo, seed_hi ^ solve), counter
// (cfg_lo, cfg_hi, step, draw << 16 | block); two uniforms per block.
struct Stream {
  uint32_t k0, k1, c0, c1, c2, hi;  // hi = draw << 16
  uint32_t block;
  bool spare_ok;
  double spare;
  int *err;

  DQ_HD Stream(uint64_t seed, uint32_t solve, uint64_t cfg, uint32_t step, uint32_t draw,
               int *e)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32) ^ solve), c0((uint32_t)cfg),
        c1((uint32_t)(cfg >> 32)), c2(step), hi(draw << 16), block(0), spare_ok(false),
        spare(0.0), err(e) {}

  DQ_HD bool dry() const { return block >= 65536u && !spare_ok; }

  DQ_HD double next() {
    if (spare_ok) {
      spare_ok = false;
      return spare;
    }
    if (block >= 65536u) {
      if (err) *err = 1;
      return 0.0;
    }
    const U4 o = philox10(c0, c1, c2, hi | block, k0, k1);
    ++block;
    spare = unit53(o.x2, o.x3);
    spare_ok = true;
    return unit53(o.x0, o.x1);
  }
};

// Draw-id layout: 0 = the entry's primary uniform; channel k (1..8) owns ids
// k*1024 + [0, 1024): +0 its count, +1+c the class split of class c,
// +64+64c+h node h of the member tree of class c.
DQ_HD uint32_t draw_channel(int k) { return (uint32_t)k << 10; }

// ---------------------------------------------------------------------------
// Deterministic logarithm and exponential from +, -, *, /.
// ---------------------------------------------------------------------------
DQ_HD double ln2_hi() { return 0x1.62e42p-1; }
DQ_HD double ln2_lo() { return 0x1.fdf473de6af28p-22; }

DQ_HD double dlog(double x) {
  if (!(x == x)) return x;
  if (x < 0.0) return __builtin_nan("");
  if (x == 0.0) return -__builtin_inf();
  if (x == __builtin_inf()) return x;
  uint64_t b = __builtin_bit_cast(uint64_t, x);
  int e = (int)((b >> 52) & 0x7ffu);
  if (e == 0) {  // subnormal input: scale by 2^54 first
    x = x * 18014398509481984.0;
    b = __builtin_bit_cast(uint64_t, x);
    e = (int)((b >> 52) & 0x7ffu) - 54;
  }
  e -= 1022;
  double m = __builtin_bit_cast(double, (b & 0x000fffffffffffffull) | 0x3fe0000000000000ull);
  if (m < 0x1.6a09e667f3bcdp-1) {  // bring m into [sqrt(1/2), sqrt(2))
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = 1.0 / 25.0;  // 2 atanh(s) = 2 s sum_k s^{2k} / (2k + 1)
  for (int k = 23; k >= 1; k -= 2) q = q * z + 1.0 / (double)k;
  const double lnm = (2.0 * s) * q;
  const double ed = (double)e;
  return ed * ln2_hi() + (ed * ln2_lo() + lnm);
}

DQ_HD double dexp(double x) {
  if (!(x == x)) return x;
  if (x > 709.0) return __builtin_inf();
  if (x < -708.0) return 0.0;
  const double kd = __builtin_floor(x / (ln2_hi() + ln2_lo()) + 0.5);
  const int k = (int)kd;
  const double r = (x - kd * ln2_hi()) - kd * ln2_lo();
  double q = 1.0;  // e^r by Horner on its Taylor series to r^16 / 16!
  for (int i = 16; i >= 1; --i) q = q * (r / (double)i) + 1.0;
  return q * __builtin_bit_cast(double, (uint64_t)(k + 1023) << 52);
}

// b^e by squaring over the bits of e, low to high.  The low four bits (all of
// e for the small populations that dominate) without a loop: squaring b after
// the last set bit is never used, so the products are those of the plain loop.
DQ_HD double ipow(double b, int64_t e) {
  double r = 1.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r = (e & 1) ? r * b : r;
    e >>= 1;
    b = b * b;
  }
  while (e > 0) {
    if (e & 1) r = r * b;
    e >>= 1;
    if (e > 0) b = b * b;
  }
  return r;
}

// Stirling remainder: ln k! - (k + 1/2) ln(k + 1) + (k + 1) - ln(2 pi) / 2.
DQ_HD double stirling_fc(int64_t k) {
  if (k <= 9) {
    double fact = 1.0;
    for (int64_t i = 1; i <= k; ++i) fact = fact * (double)i;
    const double kk = (double)k;
    const double half_ln_2pi = 0.5 * dlog(0x1.921fb54442d18p+2);
    return dlog(fact) - (kk + 0.5) * dlog(kk + 1.0) + (kk + 1.0) - half_ln_2pi;
  }
  const double t = 1.0 / ((double)k + 1.0);
  const double t2 = t * t;
  return (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * t2) * t2) * t;
}

// ---------------------------------------------------------------------------
// Binomial generators.
// ---------------------------------------------------------------------------

// Sequential inversion (BINV, Kachitvichyanukul & Schmeiser 1988).  With
// `positive` the search starts at 1 over the mass 1 - q^n (X | X >= 1).
DQ_HD int64_t bin_inversion(int64_t n, double p, Stream &st, bool positive) {
  const double q = 1.0 - p;
  const double ratio = p / q;
  const double a = ((double)n + 1.0) * ratio;
  const double p0 = ipow(q, n);
  const int64_t cut = n < 110 ? n : 110;
  for (;;) {
    if (st.dry()) return 0;
    double u = st.next();
    int64_t x;
    double f;
    if (positive) {
      u = u * (1.0 - p0);
      x = 1;
      f = p0 * (a - ratio);
    } else {
      x = 0;
      f = p0;
    }
    while (true) {
      if (u < f) return x;
      u = u - f;
      ++x;
      if (x > cut) break;
      f = f * (a / (double)x - ratio);
    }
  }
}

// Transformed rejection with decomposition (BTRD, Hormann 1993); p <= 1/2 and
// n p >= 10.  Out of line: only entries with many walkers get here.
__host__ __device__ __attribute__((noinline)) int64_t bin_btrd(int64_t n, double p, Stream &st) {
  const double nd = (double)n;
  const double q = 1.0 - p;
  const double md = __builtin_floor((nd + 1.0) * p);
  const int64_t mode = (int64_t)md;
  const double r = p / q;
  const double nr = (nd + 1.0) * r;
  const double npq = nd * p * q;
  const double spq = __builtin_sqrt(npq);
  const double b = 1.15 + 2.53 * spq;
  const double a = -0.0873 + 0.0248 * b + 0.01 * p;
  const double c = nd * p + 0.5;
  const double alpha = (2.83 + 5.1 / b) * spq;
  const double vr = 0.92 - 4.2 / b;
  const double urvr = 0.86 * vr;
  for (;;) {
    if (st.dry()) return 0;
    double v = st.next();
    double u;
    if (v <= urvr) {  // inside the box: immediate acceptance
      u = v / vr - 0.43;
      const double kd = __builtin_floor((2.0 * a / (0.5 - __builtin_fabs(u)) + b) * u + c);
      if (kd < 0.0 || kd > nd) continue;
      return (int64_t)kd;
    }
    if (v >= vr) {
      u = st.next() - 0.5;
    } else {
      u = v / vr - 0.93;
      u = (u < 0.0 ? -0.5 : 0.5) - u;
      v = st.next() * vr;
    }
    const double us = 0.5 - __builtin_fabs(u);
    const double kd = __builtin_floor((2.0 * a / us + b) * u + c);
    if (kd < 0.0 || kd > nd) continue;
    const int64_t k = (int64_t)kd;
    v = v * alpha / (a / (us * us) + b);
    const int64_t km = k > mode ? k - mode : mode - k;
    if (km <= 15) {  // exact ratio of pmfs by recursion from the mode
      double f = 1.0;
      if (mode < k) {
        for (int64_t i = mode + 1; i <= k; ++i) f = f * (nr / (double)i - r);
      } else if (mode > k) {
        for (int64_t i = k + 1; i <= mode; ++i) v = v * (nr / (double)i - r);
      }
      if (v <= f) return k;
      continue;
    }
    v = dlog(v);  // squeeze, then the final test with Stirling terms
    const double kmd = (double)km;
    const double rho = (kmd / npq) * (((kmd / 3.0 + 0.625) * kmd + 1.0 / 6.0) / npq + 0.5);
    const double t = -kmd * kmd / (2.0 * npq);
    if (v < t - rho) return k;
    if (v > t + rho) continue;
    const double nm = nd - md + 1.0;
    const double h = (md + 0.5) * dlog((md + 1.0) / (r * nm)) + stirling_fc(mode) +
                     stirling_fc(n - mode);
    const double nk = nd - kd + 1.0;
    if (v <= h + (nd + 1.0) * dlog(nm / nk) + (kd + 0.5) * dlog(nk * r / (kd + 1.0)) -
                 stirling_fc(k) - stirling_fc(n - k))
      return k;
  }
}

DQ_HD int64_t bin_low(int64_t n, double p, Stream &st) {
  if ((double)n * p < 10.0) return bin_inversion(n, p, st, false);
  return bin_btrd(n, p, st);
}

// X ~ Bin(n, p), 0 <= p <= 1 (p > 1/2 through n - Bin(n, 1 - p)).
DQ_HD int64_t binomial(int64_t n, double p, Stream &st) {
  if (n <= 0 || p <= 0.0) return 0;
  if (p > 0.5) return n - bin_low(n, 1.0 - p, st);
  return bin_low(n, p, st);
}

// X ~ Bin(n, p) given X >= 1; n >= 1, 0 < p < 1.
DQ_HD int64_t binomial_positive(int64_t n, double p, Stream &st) {
  if (p > 0.5) {
    for (;;) {
      const int64_t y = bin_low(n, 1.0 - p, st);
      if (y < n) return n - y;
      if (st.dry()) return 1;
    }
  }
  if ((double)n * p < 10.0) return bin_inversion(n, p, st, true);
  for (;;) {
    const int64_t x = bin_btrd(n, p, st);
    if (x >= 1) return x;
    if (st.dry()) return 1;
  }
}

// floor(P) events per walker for sure, one more with probability P - floor(P).
DQ_HD int64_t binomial_split(int64_t n, double P, Stream &st) {
  if (n <= 0 || P <= 0.0) return 0;
  if (P < 1.0) return binomial(n, P, st);
  const double f = __builtin_floor(P);
  return n * (int64_t)f + binomial(n, P - f, st);
}

// The same law as binomial() / binomial_positive() for draws where those use
// inversion only: (double)n * min(p, 1 - p) < 10 and p < 1.  Inlined: the
// callers keep one copy of it per loop.
DQ_HD int64_t binomial_small(uint64_t seed, uint32_t solve, uint64_t cfg, uint32_t step,
                             uint32_t draw, int64_t n, double p, bool positive, int &dry) {
  int e = 0;
  Stream st(seed, solve, cfg, step, draw, &e);
  int64_t x;
  if (p > 0.5) {
    if (!positive) {
      x = n - bin_inversion(n, 1.0 - p, st, false);
    } else {
      for (;;) {
        const int64_t y = bin_inversion(n, 1.0 - p, st, false);
        if (y < n) {
          x = n - y;
          break;
        }
        if (st.dry()) {
          x = 1;
          break;
        }
      }
    }
  } else {
    x = bin_inversion(n, p, st, positive);
  }
  dry |= e;
  return x;
}

// True if binomial(n, p) (or its positive variant) takes the inversion branch
// for every p in the argument's reflection, i.e. binomial_small applies.
DQ_HD bool small_draw(int64_t n, double p) {
  if (n <= 0 || p <= 0.0) return true;
  if (p >= 1.0) return false;
  const double q = p > 0.5 ? 1.0 - p : p;
  return (double)n * q < 10.0;
}

// One count drawn from its own stream (draw id `draw` of the entry's counter):
// mode 0 Bin(n, p), 1 Bin(n, p) given >= 1, 2 integer part + Bin(n, fraction).
// Out of line, so the generators exist once in a kernel however many call
// sites it has.  Sets bit 0 of *err if the stream ran dry.
struct Count {
  int64_t x;
  int dry;
};
enum { DRAW_BIN = 0, DRAW_POS = 1, DRAW_SPLIT = 2 };

__host__ __device__ __attribute__((always_inline)) inline Count draw_count_inline(
    uint64_t seed, uint32_t solve, uint64_t cfg, uint32_t step, uint32_t draw, int64_t n, double p,
    int mode) {
  int e = 0;
  Stream st(seed, solve, cfg, step, draw, &e);
  int64_t x;
  if (mode == DRAW_BIN)
    x = binomial(n, p, st);
  else if (mode == DRAW_POS)
    x = binomial_positive(n, p, st);
  else
    x = binomial_split(n, p, st);
  return Count{x, e};
}

__host__ __device__ __attribute__((noinline)) Count draw_count(uint64_t seed, uint32_t solve,
                                                               uint64_t cfg, uint32_t step,
                                                               uint32_t draw, int64_t n, double p,
                                                               int mode) {
  return draw_count_inline(seed, solve, cfg, step, draw, n, p, mode);
}

struct EntryCounter {
  uint64_t seed, cfg;
  uint32_t solve, step;
  int dry;
  DQ_HD int64_t operator()(uint32_t draw, int64_t n, double p, int mode) {
    const Count c = draw_count(seed, solve, cfg, step, draw, n, p, mode);
    dry |= c.dry;
    return c.x;
  }
  // the same draw inline, for a chain of dependent draws where a call would
  // spill the caller's live registers to scratch memory around every draw
  DQ_HD int64_t inl(uint32_t draw, int64_t n, double p, int mode) {
    const Count c = draw_count_inline(seed, solve, cfg, step, draw, n, p, mode);
    dry |= c.dry;
    return c.x;
  }
};

// Draw id, within a channel, of the single-walker categorical pick.
constexpr uint32_t DRAW_PICK = 7u;

// The eight channel counts of one entry (real walkers: death-re, death-im,
// spawn along Re elements, spawn along Im elements; then the same for the
// imaginary walkers) are independent Bsplit(n_k, p_k).  When all p_k < 1,
// successive uniforms of the primary stream (draw 0) locate the nonzero
// channels one after the other: from channel `start` on, u is inverted against
// the running products of the zero probabilities; below the last product no
// further channel fires, otherwise the first product u exceeds names the next
// nonzero channel, drawn given >= 1, and the search resumes after it.
//
// event_channels: which channels fire (bit k for channel k), from the search
// alone, which needs only the primary stream.  *all is set when some p_k >= 1;
// then every channel is drawn as integer part + Bin(n, fraction).
DQ_HD uint32_t event_channels(const double p[8], const int64_t n[8], const EntryCounter &cnt,
                              bool *all) {
  bool loud = false;
#pragma unroll
  for (int k = 0; k < 8; ++k) loud = loud || (n[k] > 0 && p[k] >= 1.0);
  *all = loud;
  if (loud) return 0xffu;
  // each channel's zero probability once (1 for a channel that cannot fire:
  // multiplying by it leaves the running product as it is)
  double f[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) f[k] = (n[k] > 0 && p[k] > 0.0) ? ipow(1.0 - p[k], n[k]) : 1.0;
  Stream prim(cnt.seed, cnt.solve, cnt.cfg, cnt.step, 0, nullptr);
  uint32_t ev = 0;
  int start = 0;
  while (start < 8) {
    double G[8];
    double g = 1.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= start) g = g * f[k];
      G[k] = g;
    }
    const double u = prim.next();
    if (u < G[7]) break;
    int first = 8;
#pragma unroll
    for (int k = 7; k >= 0; --k)
      if (k >= start && u >= G[k]) first = k;
    ev |= 1u << first;
    start = first + 1;
  }
  return ev;
}

// The counts of the firing channels, each from its own stream (so the draws do
// not depend on the order they are taken in).
DQ_HD void channel_counts(const double p[8], const int64_t n[8], EntryCounter &cnt,
                          int64_t X[8]) {
  bool all;
  const uint32_t ev = event_channels(p, n, cnt, &all);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    X[k] = ((ev >> k) & 1u) ? cnt(draw_channel(k + 1), n[k], p[k], all ? DRAW_SPLIT : DRAW_POS)
                            : 0;
}

}  // namespace ddqmc
