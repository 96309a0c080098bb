// Dissipative XYZ lattice (arXiv:1802.05931, Sec. V) and the Liouvillian
// elements seen from one occupied configuration |l><m| (Sec. III.C, Kronecker
// form, element form eq. (eq:elmeq); Sec. IV.B weights), evaluated with bit
// arithmetic on the two bitstrings.
//
// Bonds are the unique nearest-neighbour pairs of the periodic Lx x Ly lattice.
// A bond is named by its origin site and direction: "right" bonds (s, s+x) and
// "up" bonds (s, s+y).  Bond order is: right bonds by origin, then up bonds by
// origin.  Masks of origins (rmask, umask) drop the duplicate wrap-around pair
// on a length-2 dimension.
#pragma once

#include "sampling.hpp"

namespace ddqmc {

enum { S_T_RE = 0, S_T_IM, S_NW, S_Z, S_X, S_Y, S_CXX, S_CYY, S_CZZ, S_WTOT, S_NENT, S_NSUM };

enum : uint32_t { FLAG_NO_INITIATOR = 1u, FLAG_PER_WALKER = 2u };

// Per-solve constants (device, read-only during a step).
struct SlotParams {
  uint32_t N, nb, Lx, Ly;
  uint32_t rmask, umask;       // origins of right / up bonds
  uint32_t col_last, row_last; // sites with x == Lx-1 / y == Ly-1
  uint32_t flags, solve;
  int64_t n_a, target, n_equil;
  uint64_t seed;
  double dt, gamma, half_gamma, half_jz;
  double h_al, h_an, a_al, a_an;  // signed / absolute hop amplitude, aligned / anti
  double w_dn, w_up;              // e^{-p}, e^{+p}
  double delta_over_dt, shift_init;
  // in-plane field hx sigma^x + hy sigma^y per site (Sec. V.B); field = 1 if on
  double hx, hy, ahx, ahy;
  uint32_t field, pad;
};

// Per-solve evolving state (device, written by the step's last kernel).
struct SlotState {
  double S;
  int32_t mode;    // 0 growth (S held), 1 shift varies
  int32_t status;  // 0 empty, 1 running, 2 entering this step, 3 leaving this step
  int64_t step, nw_prev;
  int64_t n_accum;
  int64_t last[S_NSUM];
  int64_t acc[S_NSUM];
};

DQ_HD int popc(uint32_t x) { return __builtin_popcount(x); }

// bit s of the result = bit of x at the right (resp. up) neighbour of s
DQ_HD uint32_t right_of(const SlotParams &P, uint32_t x) {
  return ((x >> 1) & ~P.col_last) | ((uint32_t)((uint64_t)x << (P.Lx - 1)) & P.col_last);
}
DQ_HD uint32_t up_of(const SlotParams &P, uint32_t x) {
  return ((x >> P.Lx) & ~P.row_last) |
         ((uint32_t)((uint64_t)x << (P.Lx * (P.Ly - 1))) & P.row_last);
}
DQ_HD uint32_t right_site(const SlotParams &P, uint32_t s) {
  return ((P.col_last >> s) & 1u) ? s - (P.Lx - 1) : s + 1;
}
DQ_HD uint32_t up_site(const SlotParams &P, uint32_t s) {
  return ((P.row_last >> s) & 1u) ? s - P.Lx * (P.Ly - 1) : s + P.Lx;
}

// position of the j-th set bit of x (j < popcount(x))
DQ_HD uint32_t nth_bit(uint32_t x, int j) {
  for (int i = 0; i < j; ++i) x &= x - 1;
  return (uint32_t)__builtin_ctz(x);
}

struct Geometry {
  uint32_t al_r[2], al_u[2];  // aligned right / up bonds (by origin) of l and m
  int al[2];                  // their counts
  uint32_t Tr, Tu;            // the bond b with l ^ m == mask_b, if any
  bool T_aligned;             // its alignment (same in l and m)
};

DQ_HD Geometry geometry(const SlotParams &P, uint32_t l, uint32_t m) {
  Geometry g;
  const uint32_t x[2] = {l, m};
  for (int s = 0; s < 2; ++s) {
    g.al_r[s] = ~(x[s] ^ right_of(P, x[s])) & P.rmask;
    g.al_u[s] = ~(x[s] ^ up_of(P, x[s])) & P.umask;
    g.al[s] = popc(g.al_r[s]) + popc(g.al_u[s]);
  }
  const uint32_t d = l ^ m;
  g.Tr = 0;
  g.Tu = 0;
  if (popc(d) == 2) {
    g.Tr = d & right_of(P, d) & P.rmask;
    g.Tu = d & up_of(P, d) & P.umask;
  }
  g.T_aligned = ((g.Tr | g.Tu) == 0) || ((g.al_r[0] & g.Tr) | (g.al_u[0] & g.Tu)) != 0;
  return g;
}

// Hop classes seen from (l, m): 0 ket-aligned, 1 ket-anti, 2 ket to-diagonal,
// 3 bra-aligned, 4 bra-anti, 5 bra to-diagonal.  Each is a set of bonds given by
// origin masks; members are ordered right bonds then up bonds, by origin.
struct HopClasses {
  uint32_t r[6], u[6];
  int n[6];
  double W[6];  // n_c |element| w_child / w_parent
  int sgn[6];   // sign of Im of the element
};

DQ_HD HopClasses hop_classes(const SlotParams &P, const Geometry &g, uint32_t l, uint32_t m) {
  HopClasses hc;
  const bool diag = (l == m);
  for (int side = 0; side < 2; ++side) {
    const int c0 = 3 * side;
    hc.r[c0] = g.al_r[side] & ~g.Tr;
    hc.u[c0] = g.al_u[side] & ~g.Tu;
    hc.r[c0 + 1] = ~g.al_r[side] & P.rmask & ~g.Tr;
    hc.u[c0 + 1] = ~g.al_u[side] & P.umask & ~g.Tu;
    hc.r[c0 + 2] = g.Tr;
    hc.u[c0 + 2] = g.Tu;
  }
  for (int c = 0; c < 6; ++c) {
    const int kind = c % 3;
    const bool al = (kind == 2) ? g.T_aligned : (kind == 0);
    const double amp = al ? P.a_al : P.a_an;
    const double h = al ? P.h_al : P.h_an;
    const double w = diag ? P.w_dn : (kind == 2 ? P.w_up : 1.0);
    const int sh = (h > 0.0) - (h < 0.0);
    hc.sgn[c] = c < 3 ? -sh : sh;  // ket: -i h, bra: +i h
    hc.n[c] = popc(hc.r[c]) + popc(hc.u[c]);
    hc.W[c] = ((double)hc.n[c] * amp) * w;
  }
  return hc;
}

// Multinomial split of M walkers over the n members of one class (equal
// weights) by a balanced binary tree of binomials; node h of the heap draws the
// left share Bin(M, |left| / |node|).  emit(member, count) for nonzero leaves.
template <typename F>
DQ_HD void tree_split(int n, int64_t M, EntryCounter &cnt, uint32_t draw_base, F &&emit) {
  struct Node {
    int lo, hi, h;
    int64_t M;
  };
  Node stack[8];
  int sp = 0;
  stack[sp++] = Node{0, n, 1, M};
  while (sp > 0) {
    const Node nd = stack[--sp];
    if (nd.M == 0) continue;
    if (nd.hi - nd.lo == 1) {
      emit(nd.lo, nd.M);
      continue;
    }
    const int mid = nd.lo + (nd.hi - nd.lo) / 2;
    const int64_t ML = cnt(draw_base + (uint32_t)nd.h, nd.M,
                           (double)(mid - nd.lo) / (double)(nd.hi - nd.lo), DRAW_BIN);
    stack[sp++] = Node{mid, nd.hi, 2 * nd.h + 1, nd.M - ML};
    stack[sp++] = Node{nd.lo, mid, 2 * nd.h, ML};
  }
}

// tree_split for n <= 64 members without an array: the same draws and leaves,
// by a depth-first walk that goes left first and keeps the right child's
// count of each split in the register of its depth (depths 1..6), read and
// written through select chains; a waiting child is found again from the
// current heap index, its range rebuilt from the root.
// (draw(id, n, p) draws node id's Bin(n, p))
template <typename D, typename F>
DQ_HD void tree_split_flat_with(int n, int64_t M, uint32_t draw_base, D &&draw, F &&emit) {
  int64_t q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q6 = 0;  // waiting right children
  uint32_t wait = 0;                                         // bit d: depth d has one
  int lo = 0, hi = n, depth = 0;
  uint32_t h = 1;
  int64_t Mn = M;
#pragma unroll 1
  for (;;) {
    if (Mn > 0) {
      if (hi - lo == 1) {
        emit(lo, Mn);
      } else {
        const int mid = lo + (hi - lo) / 2;
        const int64_t ML = draw(draw_base + h, Mn, (double)(mid - lo) / (double)(hi - lo));
        ++depth;
        const int64_t MR = Mn - ML;
        if (MR > 0) {
          q1 = depth == 1 ? MR : q1;
          q2 = depth == 2 ? MR : q2;
          q3 = depth == 3 ? MR : q3;
          q4 = depth == 4 ? MR : q4;
          q5 = depth == 5 ? MR : q5;
          q6 = depth == 6 ? MR : q6;
          wait |= 1u << depth;
        }
        hi = mid;  // the left child next
        h = 2 * h;
        Mn = ML;
        continue;
      }
    }
    if (wait == 0) break;
    const int d = 31 - __builtin_clz(wait);  // the deepest waiting child
    wait &= ~(1u << d);
    Mn = d == 1 ? q1 : d == 2 ? q2 : d == 3 ? q3 : d == 4 ? q4 : d == 5 ? q5 : q6;
    h = (h >> (depth - d)) | 1u;  // right sibling of the path's node at depth d
    depth = d;
    lo = 0;
    hi = n;
#pragma unroll 1
    for (int k = d - 1; k >= 0; --k) {
      const int mid = lo + (hi - lo) / 2;
      if ((h >> k) & 1u)
        lo = mid;
      else
        hi = mid;
    }
  }
}

template <typename F>
DQ_HD void tree_split_flat(int n, int64_t M, EntryCounter &cnt, uint32_t draw_base, F &&emit) {
  tree_split_flat_with(
      n, M, draw_base,
      [&](uint32_t id, int64_t nn, double p) { return cnt.inl(id, nn, p, DRAW_BIN); }, emit);
}

DQ_HD int64_t sgn64(int64_t x) { return (x > 0) - (x < 0); }
DQ_HD int64_t sgnd(double x) { return (x > 0.0) - (x < 0.0); }

// Select element c of a 6-array (keeps the arrays in registers inside loops
// that are not unrolled).
template <typename T>
DQ_HD T pick6(const T *a, int c) {
  T v = a[0];
#pragma unroll
  for (int i = 1; i < 6; ++i) v = (c == i) ? a[i] : v;
  return v;
}

// Element c of six values held in registers (a select chain on values, so no
// array has to live in memory to be indexed).
template <typename T>
DQ_HD T sel6(int c, T a0, T a1, T a2, T a3, T a4, T a5) {
  T v = a0;
  v = c == 1 ? a1 : v;
  v = c == 2 ? a2 : v;
  v = c == 3 ? a3 : v;
  v = c == 4 ? a4 : v;
  v = c == 5 ? a5 : v;
  return v;
}

// One spawned walker among n equal members: a uniform member from the pick
// stream of the channel.
DQ_HD int pick_member(const EntryCounter &c, uint32_t draw, int n) {
  Stream st(c.seed, c.solve, c.cfg, c.step, draw, nullptr);
  int j = (int)__builtin_floor(st.next() * (double)n);
  return j > n - 1 ? n - 1 : j;
}

// One spawned walker among the hop classes: class c with probability W_c / S_0
// (inversion: the smallest c with S_{c+1} < S_0 (1 - u1)), then a uniform
// member j of it from u2.
DQ_HD void pick_hop(const EntryCounter &cn, uint32_t draw, const double *Sc, const int *ncls,
                    int &c, int &j) {
  Stream st(cn.seed, cn.solve, cn.cfg, cn.step, draw, nullptr);
  const double u1 = st.next();
  const double u2 = st.next();
  const double T = Sc[0] * (1.0 - u1);
  c = 5;
#pragma unroll
  for (int k = 4; k >= 0; --k)
    if (Sc[k + 1] < T) c = k;
  int n = ncls[0];
#pragma unroll
  for (int k = 1; k < 6; ++k) n = c == k ? ncls[k] : n;
  j = (int)__builtin_floor(u2 * (double)n);
  j = j > n - 1 ? n - 1 : j;
}

// Bond mask of member j of hop class c (right bonds of the class first).
DQ_HD uint32_t class_member_mask(const SlotParams &P, uint32_t cr, uint32_t cu, int j) {
  const int nr = popc(cr);
  if (j < nr) {
    const uint32_t s = nth_bit(cr, j);
    return (1u << s) | (1u << right_site(P, s));
  }
  const uint32_t s = nth_bit(cu, j - nr);
  return (1u << s) | (1u << up_site(P, s));
}

// Everything the channel counts of one entry depend on.
struct EntryProbs {
  bool init;
  int64_t sR, sI;
  double d_r, d_i;
  Geometry g;
  HopClasses hc;
  double Sc[6];
  uint32_t jm;
  int nJ;
  double p8[8];
  int64_t n8[8];
  EntryCounter cnt;
};

DQ_HD EntryProbs entry_probs(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                             int32_t R, int32_t I) {
  EntryProbs e;
  const bool diag = (l == m);
  const int64_t nR = R < 0 ? -(int64_t)R : (int64_t)R;
  const int64_t nI = I < 0 ? -(int64_t)I : (int64_t)I;
  e.sR = sgn64(R);
  e.sI = sgn64(I);
  e.init = diag || (nR + nI > P.n_a) || (P.flags & FLAG_NO_INITIATOR);
  e.g = geometry(P, l, m);
  // diagonal element: Re = -(gamma/2)(n_up(l) + n_up(m)) - S, Im = -(E_l - E_m)
  e.d_r = -(P.half_gamma * (double)(popc(l) + popc(m))) - S;
  e.d_i = P.half_jz * (double)(e.g.al[1] - e.g.al[0]);
  const double p_r = P.dt * __builtin_fabs(e.d_r);
  const double p_i = P.dt * __builtin_fabs(e.d_i);
  e.hc = hop_classes(P, e.g, l, m);
  e.Sc[5] = e.hc.W[5];
  for (int c = 4; c >= 0; --c) e.Sc[c] = e.hc.W[c] + e.Sc[c + 1];
  const double P_im = P.dt * e.Sc[0];
  e.jm = l & m;  // jump sites: up in both ket and bra
  e.nJ = popc(e.jm);
  const double P_re = P.dt * ((double)e.nJ * P.gamma);
  const double pp[4] = {p_r, p_i, P_re, P_im};
  for (int k = 0; k < 4; ++k) {
    e.p8[k] = pp[k];
    e.p8[k + 4] = pp[k];
    e.n8[k] = nR;
    e.n8[k + 4] = nI;
  }
  e.cnt = EntryCounter{P.seed, ((uint64_t)l << P.N) | m, P.solve, step, 0};
  return e;
}

enum { ENTRY_QUIET = 0, ENTRY_LIGHT = 1, ENTRY_HEAVY = 2 };

// The quiet test u < g, g = prod_k (1 - p_k)^n_k, where g is the fp64 product
// of the k = 0..7 factors, each by ipow.  Decided from a single-precision
// estimate where possible: with every p_k <= 1/2 and n = n_R + n_I <= 1024,
// ga = 2^(n_R sum_k<4 log2(1 - p_k) + n_I sum_k>=4 ...) computed in float
// differs from the exact product by a relative error below 2e-7 + 2e-6 n: per
// channel, the float rounding of p_k and of 1 - p_k (6e-8 together, times at
// most 2.9 through log2) and 2 ulps of log2 give 3e-7 in the logarithm; the
// two four-term sums add 7e-7 and the products and their sum 5e-7 n; ln 2
// turns 2.4e-6 n in the exponent into 1.7e-6 n, and exp2 adds 2 ulps.  The
// fp64 product itself is within (n + 100) 2^-52 of the real value.  With the
// margin mg = 1e-5 (1 + n), u < ga (1 - mg) implies u < g and u >= ga (1 + mg)
// implies u >= g; only a u inside the band, or ga below 2^-30, takes the
// exact product.  Returns 1 (quiet), 0 (not quiet) or -1 (undecided).  The
// counts are those of an entry: n8[0..3] = n_R and n8[4..7] = n_I (anything
// else is left undecided).
DQ_HD int quiet_estimate(const double p8[8], const int64_t n8[8], double u) {
  const int64_t nR = n8[0], nI = n8[4];
  if (nR + nI > 1024) return -1;
  if (n8[1] != nR || n8[2] != nR || n8[3] != nR || n8[5] != nI || n8[6] != nI || n8[7] != nI)
    return -1;
  float lr = 0.0f, li = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!(p8[k] <= 0.5) || !(p8[k + 4] <= 0.5)) return -1;
    lr += log2f(1.0f - (float)p8[k]);
    li += log2f(1.0f - (float)p8[k + 4]);
  }
  const float E = (float)nR * lr + (float)nI * li;
  if (!(E > -30.0f)) return -1;
  const double ga = (double)exp2f(E);
  const double mg = 1e-5 * (double)(1 + nR + nI);
  if (u < ga * (1.0 - mg)) return 1;
  if (u >= ga * (1.0 + mg)) return 0;
  return -1;
}

// u < g exactly, by the estimate where it decides, else by the fp64 product.
// Bit 0: quiet; bit 1: the estimate decided.
DQ_HD int quiet_test(const double p8[8], const int64_t n8[8], double u) {
  const int q = quiet_estimate(p8, n8, u);
  if (q >= 0) return q | 2;
  double g = 1.0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (n8[k] > 0 && p8[k] > 0.0) g = g * ipow(1.0 - p8[k], n8[k]);
  return u < g ? 1 : 0;
}

// What the step does with an entry: 0 (quiet) when all eight channel counts
// are zero (decided by the primary uniform exactly as channel_counts decides
// it); otherwise 2 when some channel may be too large to draw by inversion
// (max(n_R, n_I) max_k p_k >= 10, or some p_k >= 1: a superset of the entries
// the light path refuses, which tests n_k min(p_k, 1 - p_k) per channel),
// else 1.  Either path gives the same counts; this only routes
// the large populations to the general path early.
DQ_HD int entry_kind(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                     int32_t R, int32_t I) {
  const EntryProbs e = entry_probs(P, S, step, l, m, R, I);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (e.n8[k] > 0 && e.p8[k] >= 1.0) return ENTRY_HEAVY;
  Stream prim(e.cnt.seed, e.cnt.solve, e.cnt.cfg, e.cnt.step, 0, nullptr);
  if (quiet_test(e.p8, e.n8, prim.next()) & 1) return ENTRY_QUIET;
  const double pm = __builtin_fmax(__builtin_fmax(e.p8[0], e.p8[1]),
                                   __builtin_fmax(e.p8[2], e.p8[3]));
  const int64_t nm = e.n8[0] > e.n8[4] ? e.n8[0] : e.n8[4];
  return (double)nm * pm >= 10.0 ? ENTRY_HEAVY : ENTRY_LIGHT;
}

// One occupied configuration |l><m| with walkers R + iI: draw its clone/death
// and spawning counts and hand every nonzero contribution to
// emit(child_l, child_m, d_re, d_im, survives_filter_unconditionally).
// The caller applies the initiator rule (Sec. IV.A) to contributions flagged
// false: they survive only on configurations occupied at the start of the step.
template <typename Emit>
DQ_HD void entry_events(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                        int32_t R, int32_t I, int *err, Emit &&emit) {
  EntryProbs e = entry_probs(P, S, step, l, m, R, I);
  const bool init = e.init;
  const int64_t sR = e.sR, sI = e.sI;
  EntryCounter &cnt = e.cnt;
  int64_t X[8];
  channel_counts(e.p8, e.n8, cnt, X);

  // clone/death: dt (R + iI)(d_r + i d_i)
  const int64_t dR = sR * sgnd(e.d_r) * X[0] - sI * sgnd(e.d_i) * X[5];
  const int64_t dI = sI * sgnd(e.d_r) * X[4] + sR * sgnd(e.d_i) * X[1];
  if (dR != 0 || dI != 0) emit(l, m, dR, dI, true);

  // spawning along the real elements: the jump gamma S^-_k rho S^+_k
  const uint32_t jm = e.jm;
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const int ch = part ? 7 : 3;
    const int64_t c = X[ch - 1];
    if (c == 0) continue;
    const int64_t sg = part ? sI : sR;
    auto leaf = [&](int j, int64_t M) {
      const uint32_t bit = 1u << nth_bit(jm, j);
      if (part == 0)
        emit(l & ~bit, m & ~bit, sg * M, 0, init);
      else
        emit(l & ~bit, m & ~bit, 0, sg * M, init);
    };
    if (c == 1)
      leaf(pick_member(cnt, draw_channel(ch) + DRAW_PICK, e.nJ), 1);
    else
      tree_split(e.nJ, c, cnt, draw_channel(ch) + 64u, leaf);
  }

  // spawning along the imaginary elements: -iH on the ket, +iH on the bra;
  // classes by sequential conditional binomials, members by the tree
  const HopClasses &hc = e.hc;
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    const int ch = part ? 8 : 4;
    int64_t rem = X[ch - 1];
    if (rem == 0) continue;
    const int64_t sg = part ? sI : sR;
    if (rem == 1) {  // one walker: class by inversion on the weights, then a member
      int c, j;
      pick_hop(cnt, draw_channel(ch) + DRAW_PICK, e.Sc, hc.n, c, j);
      const uint32_t bm = class_member_mask(P, pick6(hc.r, c), pick6(hc.u, c), j);
      const uint32_t cl = c < 3 ? (l ^ bm) : l;
      const uint32_t cm = c < 3 ? m : (m ^ bm);
      const int64_t v = sg * (int64_t)pick6(hc.sgn, c);
      if (part == 0)
        emit(cl, cm, 0, v, init || cl == cm);
      else
        emit(cl, cm, -v, 0, init || cl == cm);
      continue;
    }
    int last = -1;
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (hc.W[c] > 0.0) last = c;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (rem == 0 || hc.W[c] == 0.0) continue;
      int64_t Mc;
      if (c == last)
        Mc = rem;
      else
        Mc = cnt(draw_channel(ch) + 1u + (uint32_t)c, rem, hc.W[c] / e.Sc[c], DRAW_BIN);
      rem -= Mc;
      if (Mc == 0) continue;
      const uint32_t cr = hc.r[c], cu = hc.u[c];
      const int nr = popc(cr);
      const int64_t sv = sg * (int64_t)hc.sgn[c];
      tree_split(hc.n[c], Mc, cnt, draw_channel(ch) + 64u + 64u * (uint32_t)c,
                 [&](int j, int64_t M) {
                   uint32_t bm;
                   if (j < nr) {
                     const uint32_t s = nth_bit(cr, j);
                     bm = (1u << s) | (1u << right_site(P, s));
                   } else {
                     const uint32_t s = nth_bit(cu, j - nr);
                     bm = (1u << s) | (1u << up_site(P, s));
                   }
                   const uint32_t cl = c < 3 ? (l ^ bm) : l;
                   const uint32_t cm = c < 3 ? m : (m ^ bm);
                   const int64_t v = sv * M;
                   // real parent x Im element -> imaginary child; imaginary parent
                   // x Im element -> real child, negative (Sec. III.C rule (i))
                   if (part == 0)
                     emit(cl, cm, 0, v, init || cl == cm);
                   else
                     emit(cl, cm, -v, 0, init || cl == cm);
                 });
    }
  }
  if (cnt.dry) *err = 1;
}

// ---- the in-plane field (Sec. V.B) -----------------------------------------
// hx sigma^x + hy sigma^y per site flips one spin of the ket (-iH rho) or of the
// bra (+i rho H).  With sigma^y |dn> = -i |up>, the element from |l><m| to the
// configuration with site s flipped has Re part hy (-1 for a flip up, +1 for a
// flip down), on either side, and Im part hx (-1 on the ket, +1 on the bra).
// Each element part gets four classes of single flips: ket, ket to the
// diagonal (the flip of the one site where l and m differ, if they differ in
// one), bra, bra to the diagonal, members by ascending site, with the hop
// classes' importance-sampling weights.  The real part's classes follow the
// jump class; the imaginary part's follow the six hop classes.
// the draw id, within a channel, of the class split of class c
DQ_HD uint32_t class_split_draw(int c) { return c < 6 ? 1u + (uint32_t)c : 16u + (uint32_t)c; }

// The geometry and class weights of an entry |l><m| of a solve with the
// field, as values (a struct of scalars, no arrays, so that they stay in
// registers): aligned bonds, the bond l ^ m if it is one, the hop classes
// (0 ket-aligned, 1 ket-anti, 2 ket to-diagonal, 3-5 the bra's) and the field
// classes (flips of the sites where l and m agree, A, and of the one where
// they differ if only one, B; each element part's four field classes are ket
// A, ket B, bra A, bra B, with the hop classes' importance-sampling weights).
// The hop classes' expressions are hop_classes'.
struct FieldGeom {
  uint32_t r0, u0, r1, u1, r3, u3, r4, u4, Tr, Tu;  // hop classes' bond origins
  int hn0, hn1, hn2, hn3, hn4;                       // their members (class 5 as 2)
  int sh_al, sh_an, sh2;                             // sign of h: aligned, anti, class 2
  double Wh0, Wh1, Wh2, Wh3, Wh4, Wh5;               // hop class weights
  uint32_t fA, fB, jm;                               // field flip sites; jump sites
  int nA, nB, nJ;
  double WyA, WyB, WxA, WxB, WJ;                     // field and jump class weights
  double d_r, d_i;                                   // the diagonal element
};

DQ_HD FieldGeom field_geom(const SlotParams &P, double S, uint32_t l, uint32_t m) {
  FieldGeom g;
  const bool diag = (l == m);
  const uint32_t al_r0 = ~(l ^ right_of(P, l)) & P.rmask;
  const uint32_t al_u0 = ~(l ^ up_of(P, l)) & P.umask;
  const uint32_t al_r1 = ~(m ^ right_of(P, m)) & P.rmask;
  const uint32_t al_u1 = ~(m ^ up_of(P, m)) & P.umask;
  const int al0 = popc(al_r0) + popc(al_u0);
  const int al1 = popc(al_r1) + popc(al_u1);
  const uint32_t d = l ^ m;
  uint32_t Tr = 0, Tu = 0;
  if (popc(d) == 2) {
    Tr = d & right_of(P, d) & P.rmask;
    Tu = d & up_of(P, d) & P.umask;
  }
  const bool T_al = ((Tr | Tu) == 0) || ((al_r0 & Tr) | (al_u0 & Tu)) != 0;
  g.d_r = -(P.half_gamma * (double)(popc(l) + popc(m))) - S;
  g.d_i = P.half_jz * (double)(al1 - al0);
  g.Tr = Tr;
  g.Tu = Tu;
  g.r0 = al_r0 & ~Tr, g.u0 = al_u0 & ~Tu;
  g.r1 = ~al_r0 & P.rmask & ~Tr, g.u1 = ~al_u0 & P.umask & ~Tu;
  g.r3 = al_r1 & ~Tr, g.u3 = al_u1 & ~Tu;
  g.r4 = ~al_r1 & P.rmask & ~Tr, g.u4 = ~al_u1 & P.umask & ~Tu;
  g.hn0 = popc(g.r0) + popc(g.u0), g.hn1 = popc(g.r1) + popc(g.u1);
  g.hn2 = popc(Tr) + popc(Tu), g.hn3 = popc(g.r3) + popc(g.u3), g.hn4 = popc(g.r4) + popc(g.u4);
  const double w_al = diag ? P.w_dn : 1.0;    // weight ratio off the diagonal target
  const double w_td = diag ? P.w_dn : P.w_up;  // ... onto it
  const double amp2 = T_al ? P.a_al : P.a_an;
  g.Wh0 = ((double)g.hn0 * P.a_al) * w_al, g.Wh1 = ((double)g.hn1 * P.a_an) * w_al;
  g.Wh2 = ((double)g.hn2 * amp2) * w_td;
  g.Wh3 = ((double)g.hn3 * P.a_al) * w_al, g.Wh4 = ((double)g.hn4 * P.a_an) * w_al;
  g.Wh5 = ((double)g.hn2 * amp2) * w_td;
  g.sh_al = (P.h_al > 0.0) - (P.h_al < 0.0), g.sh_an = (P.h_an > 0.0) - (P.h_an < 0.0);
  g.sh2 = T_al ? g.sh_al : g.sh_an;
  const uint32_t all = P.N == 32 ? 0xffffffffu : ((1u << P.N) - 1u);
  const uint32_t tbit = popc(d) == 1 ? d : 0u;
  g.fA = all & ~tbit, g.fB = tbit;
  g.nA = popc(g.fA), g.nB = popc(g.fB);
  g.WyA = ((double)g.nA * P.ahy) * w_al, g.WyB = ((double)g.nB * P.ahy) * w_td;
  g.WxA = ((double)g.nA * P.ahx) * w_al, g.WxB = ((double)g.nB * P.ahx) * w_td;
  g.jm = l & m;
  g.nJ = popc(g.jm);
  g.WJ = (double)g.nJ * P.gamma;
  return g;
}

// The four channel probabilities of an entry of a solve with the field
// (dt |d_r| and dt |d_i| along the diagonal element, dt x the total weight of
// the real and of the imaginary element part's classes, each total the
// classes' suffix sum from the last class down), for both parts' walkers.
struct FieldProbs {
  double p_r, p_i, P_re, P_im;
};
DQ_HD FieldProbs field_probs(const SlotParams &P, const FieldGeom &g) {
  const double S0re = g.WJ + (g.WyA + (g.WyB + (g.WyA + g.WyB)));
  const double S0im =
      g.Wh0 + (g.Wh1 + (g.Wh2 + (g.Wh3 + (g.Wh4 + (g.Wh5 + (g.WxA + (g.WxB + (g.WxA + g.WxB))))))));
  return FieldProbs{P.dt * __builtin_fabs(g.d_r), P.dt * __builtin_fabs(g.d_i), P.dt * S0re,
                    P.dt * S0im};
}

// small_draw for both parts' walkers (nR, nI) and the four channel
// probabilities: every count of the entry by inversion.  With every p at most
// 1/2 (the usual case) the largest n p decides it, in three instructions.
DQ_HD bool all_small(int64_t nR, int64_t nI, double p0, double p1, double p2, double p3) {
  const double pm = __builtin_fmax(__builtin_fmax(p0, p1), __builtin_fmax(p2, p3));
  if (pm <= 0.5) return (double)(nR > nI ? nR : nI) * pm < 10.0;
  return small_draw(nR, p0) && small_draw(nI, p0) && small_draw(nR, p1) && small_draw(nI, p1) &&
         small_draw(nR, p2) && small_draw(nI, p2) && small_draw(nR, p3) && small_draw(nI, p3);
}

// The scan's decision for an entry of a solve with the field: quiet when the
// primary uniform says that none of its eight channels fires (the test
// channel_counts makes on the same probabilities), else sampled.  With
// heavy_ok, a sampled entry whose channel probabilities are not all small for
// both parts' walkers (entry_events_field_small would refuse it) is
// ENTRY_HEAVY.
DQ_HD int entry_kind_field(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                           int32_t R, int32_t I, bool heavy_ok = false) {
  const int64_t nR = R < 0 ? -(int64_t)R : (int64_t)R;
  const int64_t nI = I < 0 ? -(int64_t)I : (int64_t)I;
  const FieldProbs fp = field_probs(P, field_geom(P, S, l, m));
  const double p8[8] = {fp.p_r, fp.p_i, fp.P_re, fp.P_im, fp.p_r, fp.p_i, fp.P_re, fp.P_im};
  const int64_t n8[8] = {nR, nR, nR, nR, nI, nI, nI, nI};
  // (a probability of 1 or more is not small)
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (n8[k] > 0 && p8[k] >= 1.0) return heavy_ok ? ENTRY_HEAVY : ENTRY_LIGHT;
  Stream prim(P.seed, P.solve, ((uint64_t)l << P.N) | m, step, 0, nullptr);
  if (quiet_test(p8, n8, prim.next()) & 1) return ENTRY_QUIET;
  if (heavy_ok && !all_small(nR, nI, p8[0], p8[1], p8[2], p8[3])) return ENTRY_HEAVY;
  return ENTRY_LIGHT;
}

// Element c of ten values held in registers (a select chain on values).
template <typename T>
DQ_HD T sel10(int c, T a0, T a1, T a2, T a3, T a4, T a5, T a6, T a7, T a8, T a9) {
  T v = a0;
  v = c == 1 ? a1 : v;
  v = c == 2 ? a2 : v;
  v = c == 3 ? a3 : v;
  v = c == 4 ? a4 : v;
  v = c == 5 ? a5 : v;
  v = c == 6 ? a6 : v;
  v = c == 7 ? a7 : v;
  v = c == 8 ? a8 : v;
  v = c == 9 ? a9 : v;
  return v;
}

// The walkers one parent part (par: 0 real, 1 imaginary, sign sg) sends along
// element part el (0 Re: jump and field classes, 1 Im: hop and field
// classes), rem >= 1 of them: one by one categorical pick, else the class
// split (sequential conditional binomials, the last class with weight taking
// the rest) and the member trees.  The part's classes are values (the real
// part's five padded with empty ones to the imaginary part's ten, which
// leaves its suffix sums as they are); a class chosen at run time is read
// through select chains.  SMALL: every split by the inline inversion sampler
// (rem < 20, so each is small).
template <bool SMALL, typename Emit>
DQ_HD void field_part(const SlotParams &P, const FieldGeom &g, EntryCounter &cnt, int &dry,
                      uint32_t l, uint32_t m, bool init, int el, int par, int64_t sg, int64_t rem,
                      Emit &&emit) {
  const int nc = el ? 10 : 5;
  const int ch = el ? (par ? 8 : 4) : (par ? 7 : 3);
  const double W0 = el ? g.Wh0 : g.WJ, W1 = el ? g.Wh1 : g.WyA, W2 = el ? g.Wh2 : g.WyB;
  const double W3 = el ? g.Wh3 : g.WyA, W4 = el ? g.Wh4 : g.WyB, W5 = el ? g.Wh5 : 0.0;
  const double W6 = el ? g.WxA : 0.0, W7 = el ? g.WxB : 0.0, W8 = el ? g.WxA : 0.0;
  const double W9 = el ? g.WxB : 0.0;
  const double Sc9 = W9, Sc8 = W8 + Sc9, Sc7 = W7 + Sc8, Sc6 = W6 + Sc7, Sc5 = W5 + Sc6;
  const double Sc4 = W4 + Sc5, Sc3 = W3 + Sc4, Sc2 = W2 + Sc3, Sc1 = W1 + Sc2;
  const double Sc0 = W0 + Sc1;
  const int n0 = el ? g.hn0 : g.nJ, n1 = el ? g.hn1 : g.nA, n2 = el ? g.hn2 : g.nB;
  const int n3 = el ? g.hn3 : g.nA, n4 = el ? g.hn4 : g.nB, n5 = el ? g.hn2 : 0;
  const int n6 = el ? g.nA : 0, n7 = el ? g.nB : 0, n8 = el ? g.nA : 0, n9 = el ? g.nB : 0;
  const int64_t sgx = sgnd(P.hx), sgy = sgnd(P.hy);
  // member j of class c: its child and the sign of its element part
  auto leaf = [&](int c, int j, int64_t M) {
    uint32_t cl = l, cm = m;
    int64_t sgn = 1;
    bool keep = init;
    if (el == 0 && c == 0) {  // a jump: down in both ket and bra
      const uint32_t bit = 1u << nth_bit(g.jm, j);
      cl = l & ~bit;
      cm = m & ~bit;
    } else if (el == 1 && c < 6) {  // a hop of one bond
      const uint32_t bm = class_member_mask(P, sel6(c, g.r0, g.r1, g.Tr, g.r3, g.r4, g.Tr),
                                            sel6(c, g.u0, g.u1, g.Tu, g.u3, g.u4, g.Tu), j);
      const int shc = sel6(c, g.sh_al, g.sh_an, g.sh2, g.sh_al, g.sh_an, g.sh2);
      cl = c < 3 ? (l ^ bm) : l;
      cm = c < 3 ? m : (m ^ bm);
      sgn = c < 3 ? -shc : shc;  // ket: -i h, bra: +i h
      keep = init || cl == cm;
    } else {  // a field flip: ket (k = 0, 1) or bra (2, 3), sites A (k even) or B
      const int fk = el ? c - 6 : c - 1;
      const bool bra = fk >= 2;
      const uint32_t site = nth_bit((fk & 1) ? g.fB : g.fA, j);
      const uint32_t x = bra ? m : l;
      if (bra)
        cm = m ^ (1u << site);
      else
        cl = l ^ (1u << site);
      sgn = el ? (bra ? sgx : -sgx) : (((x >> site) & 1u) ? sgy : -sgy);
      keep = init || cl == cm;
    }
    const int64_t v = sg * sgn * M;
    // (R + iI) x element part: Re x R -> re, Re x I -> im, Im x R -> im,
    // Im x I -> -re (Sec. III.C rule (i))
    if (!el && !par)
      emit(cl, cm, v, 0, keep);
    else if (!el || !par)
      emit(cl, cm, 0, v, keep);
    else
      emit(cl, cm, -v, 0, keep);
  };
  if (rem == 1) {
    Stream st(cnt.seed, cnt.solve, cnt.cfg, cnt.step, draw_channel(ch) + DRAW_PICK, nullptr);
    const double u_1 = st.next();
    const double u_2 = st.next();
    const double T = Sc0 * (1.0 - u_1);
    // the first class c with Sc[c + 1] < T (the suffix sums fall, and
    // Sc[nc] = 0 < T), and its member count
    int c = 0, nmem = n0;
    if (!(Sc1 < T)) c = 1, nmem = n1;
    if (!(Sc2 < T)) c = 2, nmem = n2;
    if (!(Sc3 < T)) c = 3, nmem = n3;
    if (!(Sc4 < T)) c = 4, nmem = n4;
    if (nc > 5) {
      if (!(Sc5 < T)) c = 5, nmem = n5;
      if (!(Sc6 < T)) c = 6, nmem = n6;
      if (!(Sc7 < T)) c = 7, nmem = n7;
      if (!(Sc8 < T)) c = 8, nmem = n8;
      if (!(Sc9 < T)) c = 9, nmem = n9;
    }
    int j = (int)__builtin_floor(u_2 * (double)nmem);
    j = j > nmem - 1 ? nmem - 1 : j;
    leaf(c, j, 1);
    return;
  }
  // one split's Bin(n, p) from draw id `id` of the entry's counter
  auto draw = [&](uint32_t id, int64_t n, double p) -> int64_t {
    if constexpr (SMALL)
      return binomial_small(cnt.seed, cnt.solve, cnt.cfg, cnt.step, id, n, p, false, dry);
    else
      return cnt.inl(id, n, p, DRAW_BIN);
  };
  int last = -1;
  last = W0 > 0.0 ? 0 : last;
  last = W1 > 0.0 ? 1 : last;
  last = W2 > 0.0 ? 2 : last;
  last = W3 > 0.0 ? 3 : last;
  last = W4 > 0.0 ? 4 : last;
  last = W5 > 0.0 ? 5 : last;
  last = W6 > 0.0 ? 6 : last;
  last = W7 > 0.0 ? 7 : last;
  last = W8 > 0.0 ? 8 : last;
  last = W9 > 0.0 ? 9 : last;
#pragma unroll 1
  for (int c = 0; c < nc; ++c) {
    const double Wc = sel10(c, W0, W1, W2, W3, W4, W5, W6, W7, W8, W9);
    if (rem == 0 || Wc == 0.0) continue;
    int64_t Mc;
    if (c == last) {
      Mc = rem;
    } else {
      const double Scc = sel10(c, Sc0, Sc1, Sc2, Sc3, Sc4, Sc5, Sc6, Sc7, Sc8, Sc9);
      Mc = draw(draw_channel(ch) + class_split_draw(c), rem, Wc / Scc);
    }
    rem -= Mc;
    if (Mc == 0) continue;
    // (at most 64 members: bonds, jump and field sites of N <= 32 sites)
    const int nm = sel10(c, n0, n1, n2, n3, n4, n5, n6, n7, n8, n9);
    tree_split_flat_with(nm, Mc, draw_channel(ch) + 64u + 64u * (uint32_t)c, draw,
                         [&](int j, int64_t M) { leaf(c, j, M); });
  }
}

// entry_events with the field on (the slot's P.field): the same clone/death,
// the real element part's jumps and field flips, the imaginary part's hops
// and field flips (field_part), on the probabilities the scan's quiet test
// used (field_probs).
// SMALL: every draw by inversion (binomial_small, the same values), with no
// out-of-line call, for entries whose channel probabilities are all small for
// both parts' walkers and whose spawn counts stay below limit (at most 20, so
// that every class and tree split is small too); false, before anything is
// emitted, for an entry that is not such (the caller hands it to the general
// routine).
// A part with two or more walkers may be handed to queue(el, par, rem),
// which returns true when it takes it (field_part_job samples it later).
template <bool SMALL, typename Emit, typename Queue>
DQ_HD bool entry_events_field_impl(const SlotParams &P, double S, uint32_t step, uint32_t l,
                                   uint32_t m, int32_t R, int32_t I, int *err, Emit &&emit,
                                   Queue &&queue, int64_t limit = 20) {
  const bool diag = (l == m);
  const int64_t nR = R < 0 ? -(int64_t)R : (int64_t)R;
  const int64_t nI = I < 0 ? -(int64_t)I : (int64_t)I;
  const int64_t sR = sgn64(R), sI = sgn64(I);
  const bool init = diag || (nR + nI > P.n_a) || (P.flags & FLAG_NO_INITIATOR);
  const FieldGeom g = field_geom(P, S, l, m);
  const FieldProbs fp = field_probs(P, g);
  const double p_r = fp.p_r, p_i = fp.p_i, P_re = fp.P_re, P_im = fp.P_im;
  EntryCounter cnt{P.seed, ((uint64_t)l << P.N) | m, P.solve, step, 0};
  int dry = 0;
  int64_t X0 = 0, X1 = 0, X2 = 0, X3 = 0, X4 = 0, X5 = 0, X6 = 0, X7 = 0;
  if constexpr (SMALL) {
    if (!all_small(nR, nI, p_r, p_i, P_re, P_im)) return false;
    // successive primary uniforms locate the channels with events (as
    // event_channels), each count then drawn from its own stream
    const double pk[4] = {p_r, p_i, P_re, P_im};
    double f[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t nk = k < 4 ? nR : nI;
      f[k] = (nk > 0 && pk[k & 3] > 0.0) ? ipow(1.0 - pk[k & 3], nk) : 1.0;
    }
    Stream prim(cnt.seed, cnt.solve, cnt.cfg, cnt.step, 0, nullptr);
    int start = 0;
#pragma unroll 1
    while (start < 8) {
      double G[8];
      double gg = 1.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k >= start) gg = gg * f[k];
        G[k] = gg;
      }
      const double u = prim.next();
      if (u < G[7]) break;
      int first = 8;
#pragma unroll
      for (int k = 7; k >= 0; --k)
        if (k >= start && u >= G[k]) first = k;
      const int64_t nk = first < 4 ? nR : nI;
      double p = pk[0];
      p = (first & 3) == 1 ? pk[1] : p;
      p = (first & 3) == 2 ? pk[2] : p;
      p = (first & 3) == 3 ? pk[3] : p;
      const int64_t x = binomial_small(cnt.seed, cnt.solve, cnt.cfg, cnt.step,
                                       draw_channel(first + 1), nk, p, true, dry);
      X0 = first == 0 ? x : X0;
      X1 = first == 1 ? x : X1;
      X2 = first == 2 ? x : X2;
      X3 = first == 3 ? x : X3;
      X4 = first == 4 ? x : X4;
      X5 = first == 5 ? x : X5;
      X6 = first == 6 ? x : X6;
      X7 = first == 7 ? x : X7;
      start = first + 1;
    }
    if (X2 >= limit || X3 >= limit || X6 >= limit || X7 >= limit) return false;
  } else {
    const double p8[8] = {p_r, p_i, P_re, P_im, p_r, p_i, P_re, P_im};
    const int64_t n8[8] = {nR, nR, nR, nR, nI, nI, nI, nI};
    int64_t X[8];
    channel_counts(p8, n8, cnt, X);
    X0 = X[0], X1 = X[1], X2 = X[2], X3 = X[3], X4 = X[4], X5 = X[5], X6 = X[6], X7 = X[7];
  }
  const int64_t dR = sR * sgnd(g.d_r) * X0 - sI * sgnd(g.d_i) * X5;
  const int64_t dI = sI * sgnd(g.d_r) * X4 + sR * sgnd(g.d_i) * X1;
  if (dR != 0 || dI != 0) emit(l, m, dR, dI, true);
#pragma unroll 1
  for (int el = 0; el < 2; ++el)  // element part: 0 Re (channels 3, 7), 1 Im (4, 8)
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {  // parent part: 0 real walkers, 1 imaginary
      const int64_t rem = el ? (par ? X7 : X3) : (par ? X6 : X2);
      if (rem == 0 || (rem >= 2 && queue(el, par, rem))) continue;
      field_part<SMALL>(P, g, cnt, dry, l, m, init, el, par, par ? sI : sR, rem, emit);
    }
  if (cnt.dry || dry) *err = 1;
  return true;
}

template <typename Emit, typename Queue>
DQ_HD void entry_events_field(const SlotParams &P, double S, uint32_t step, uint32_t l,
                              uint32_t m, int32_t R, int32_t I, int *err, Emit &&emit,
                              Queue &&queue) {
  (void)entry_events_field_impl<false>(P, S, step, l, m, R, I, err, emit, queue);
}

template <typename Emit>
DQ_HD void entry_events_field(const SlotParams &P, double S, uint32_t step, uint32_t l,
                              uint32_t m, int32_t R, int32_t I, int *err, Emit &&emit) {
  entry_events_field(P, S, step, l, m, R, I, err, emit, [](int, int, int64_t) { return false; });
}

// entry_events_field for an entry whose draws are all small and whose spawn
// counts stay below limit (see above); false, with nothing emitted, for any
// other.  queue as above.
template <typename Emit, typename Queue>
DQ_HD bool entry_events_field_small(const SlotParams &P, double S, uint32_t step, uint32_t l,
                                    uint32_t m, int32_t R, int32_t I, int *err, Emit &&emit,
                                    Queue &&queue, int64_t limit) {
  return entry_events_field_impl<true>(P, S, step, l, m, R, I, err, emit, queue, limit);
}

// A part that entry_events_field_impl<SMALL> queued: rem walkers of parent
// part par along element part el of the entry |l><m| with walkers R + iI.
template <bool SMALL, typename Emit>
DQ_HD void field_part_job(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                          int32_t R, int32_t I, int el, int par, int64_t rem, int *err,
                          Emit &&emit) {
  const int64_t nR = R < 0 ? -(int64_t)R : (int64_t)R;
  const int64_t nI = I < 0 ? -(int64_t)I : (int64_t)I;
  const bool init = (l == m) || (nR + nI > P.n_a) || (P.flags & FLAG_NO_INITIATOR);
  const FieldGeom g = field_geom(P, S, l, m);
  EntryCounter cnt{P.seed, ((uint64_t)l << P.N) | m, P.solve, step, 0};
  int dry = 0;
  field_part<SMALL>(P, g, cnt, dry, l, m, init, el, par, par ? sgn64(I) : sgn64(R), rem, emit);
  if (cnt.dry || dry) *err = 1;
}

// ---- per-walker sampling (the rules of Sec. II, walker by walker) ----------
// Walker w of part q (0 real, 1 imaginary walkers) of the entry |l><m| with
// walkers R + iI: its clone/death along the diagonal element (dt |d_r| on its
// own part, dt |d_i| across), and one spawning attempt per element part at a
// uniformly chosen connection (a jump site among nJ; a hop among all nh hop
// connections) with success probability n_conn dt |element| w_child/w_parent;
// each probability's integer part is realised for sure and its fraction
// drawn.  Six uniforms from the stream with draw id 0x8000 + q 2^13 +
// (w >> 14), blocks 4 (w mod 2^14) on.  emit as in entry_events.
constexpr int64_t PW_MAX_WALKERS = 1ll << 27;

DQ_HD int64_t pw_count(double p, double u) {
  const double f = __builtin_floor(p);
  return (int64_t)f + ((u < p - f) ? 1 : 0);
}

template <typename Emit>
DQ_HD void walker_events(const SlotParams &P, double S, uint32_t step, uint32_t l, uint32_t m,
                         int32_t R, int32_t I, int part, uint32_t w, int *err, Emit &&emit) {
  const bool diag = (l == m);
  const int64_t nR = R < 0 ? -(int64_t)R : (int64_t)R;
  const int64_t nI = I < 0 ? -(int64_t)I : (int64_t)I;
  const bool init = diag || (nR + nI > P.n_a) || (P.flags & FLAG_NO_INITIATOR);
  const int64_t sg = part ? sgn64(I) : sgn64(R);
  const Geometry g = geometry(P, l, m);
  const double d_r = -(P.half_gamma * (double)(popc(l) + popc(m))) - S;
  const double d_i = P.half_jz * (double)(g.al[1] - g.al[0]);
  const double p_r = P.dt * __builtin_fabs(d_r);
  const double p_i = P.dt * __builtin_fabs(d_i);
  Stream st(P.seed, P.solve, ((uint64_t)l << P.N) | m, step,
            0x8000u + ((uint32_t)part << 13) + (w >> 14), err);
  st.block = 4u * (w & 0x3FFFu);
  double u[6];
  for (int k = 0; k < 6; ++k) u[k] = st.next();
  const int64_t cr = pw_count(p_r, u[0]);
  const int64_t ci = pw_count(p_i, u[1]);
  const int64_t dR = part ? -sg * sgnd(d_i) * ci : sg * sgnd(d_r) * cr;
  const int64_t dI = part ? sg * sgnd(d_r) * cr : sg * sgnd(d_i) * ci;
  if (dR != 0 || dI != 0) emit(l, m, dR, dI, true);
  // one attempt along the real element part: a uniform jump site
  const uint32_t jm = l & m;
  const int nJ = popc(jm);
  if (nJ > 0) {
    int j = (int)__builtin_floor(u[2] * (double)nJ);
    j = j > nJ - 1 ? nJ - 1 : j;
    const int64_t c = pw_count(P.dt * ((double)nJ * P.gamma), u[3]);
    if (c) {
      const uint32_t bit = 1u << nth_bit(jm, j);
      emit(l & ~bit, m & ~bit, part ? 0 : sg * c, part ? sg * c : 0, init);
    }
  }
  // one attempt along the imaginary element part: a uniform hop
  const HopClasses hc = hop_classes(P, g, l, m);
  int nh = 0;
  for (int c = 0; c < 6; ++c) nh += hc.n[c];
  if (nh > 0) {
    int j = (int)__builtin_floor(u[4] * (double)nh);
    j = j > nh - 1 ? nh - 1 : j;
    int c = 0;
    while (j >= hc.n[c]) j -= hc.n[c++];
    const int kind = c % 3;
    const bool al = (kind == 2) ? g.T_aligned : (kind == 0);
    const double amp = al ? P.a_al : P.a_an;
    const double wgt = diag ? P.w_dn : (kind == 2 ? P.w_up : 1.0);
    const int64_t cs = pw_count(P.dt * (((double)nh * amp) * wgt), u[5]);
    if (cs) {
      const uint32_t bm = class_member_mask(P, hc.r[c], hc.u[c], j);
      const uint32_t cl = c < 3 ? (l ^ bm) : l;
      const uint32_t cm = c < 3 ? m : (m ^ bm);
      const int64_t v = sg * (int64_t)hc.sgn[c] * cs;
      if (part == 0)
        emit(cl, cm, 0, v, init || cl == cm);
      else
        emit(cl, cm, -v, 0, init || cl == cm);
    }
  }
}

// Tree split for small counts (M < 32, n <= 64): the same draws and leaves as
// tree_split, by a depth-first walk without a stack.  The walk goes left
// first; the right child of a split waits as a 5-bit count in the field of its
// depth (at most one per depth), and is found again from the current heap
// index, its range rebuilt from the root.  Inversion-only draws.
template <typename F>
DQ_HD void tree_split_small(int n, int64_t M, const EntryCounter &c, uint32_t draw_base,
                            int &dry, F &&emit) {
  uint64_t pend = 0;  // bits [5d, 5d + 5): count of the right child waiting at depth d
  int lo = 0, hi = n, depth = 0;
  uint32_t h = 1;
  int64_t Mn = M;
#pragma unroll 1
  for (;;) {
    if (Mn > 0) {
      if (hi - lo == 1) {
        emit(lo, Mn);
      } else {
        const int mid = lo + (hi - lo) / 2;
        const int64_t ML = binomial_small(c.seed, c.solve, c.cfg, c.step, draw_base + h, Mn,
                                          (double)(mid - lo) / (double)(hi - lo), false, dry);
        ++depth;
        pend |= (uint64_t)(Mn - ML) << (5 * depth);
        hi = mid;  // the left child next
        h = 2 * h;
        Mn = ML;
        continue;
      }
    }
    if (pend == 0) break;
    const int d = (63 - __builtin_clzll(pend)) / 5;  // the deepest waiting child
    Mn = (int64_t)((pend >> (5 * d)) & 31u);
    pend &= ~(31ull << (5 * d));
    h = (h >> (depth - d)) | 1u;  // right sibling of the path's node at depth d
    depth = d;
    lo = 0;
    hi = n;
#pragma unroll 1
    for (int k = d - 1; k >= 0; --k) {
      const int mid = lo + (hi - lo) / 2;
      if ((h >> k) & 1u)
        lo = mid;
      else
        hi = mid;
    }
  }
}

// A member tree of the light path, handed to the caller instead of walked in
// place: the caller walks it later with run_tree_job (the same streams, so
// the same records), next to the trees of other entries.  The caller's queue
// has trees.reserve(k) (room for k more trees of this entry, or false) and
// trees.push(job).
struct TreeJob {
  uint32_t l, m;    // the parent configuration
  uint32_t cr, cu;  // hop: the class's right / up bond origins; jump: cr = jump sites
  uint16_t slot;    // the parent's solve (set by the caller)
  uint8_t n, M;     // members; walkers to place (M < 32)
  uint8_t flags;    // TJ_* below
  uint8_t cls;      // hop class (its tree's streams)
  uint16_t pad;
};
enum : uint8_t { TJ_IM = 1, TJ_HOP = 2, TJ_KET = 4, TJ_INIT = 8, TJ_NEG = 16 };

// Walk tree job t of solve P (at step `step`): each leaf goes to
// emit(child_l, child_m, d_re, d_im, survives_filter_unconditionally).
template <typename Emit>
DQ_HD void run_tree_job(const SlotParams &P, uint32_t step, const TreeJob &t, int &dry,
                        Emit &&emit) {
  const EntryCounter cnt{P.seed, ((uint64_t)t.l << P.N) | t.m, P.solve, step, 0};
  const int64_t sg = (t.flags & TJ_NEG) ? -1 : 1;
  const bool part = (t.flags & TJ_IM) != 0;
  // the root's stream: jumps of channel 3 / 7, hops of channel 4 / 8 by class
  const uint32_t draw_base = (t.flags & TJ_HOP)
                                 ? draw_channel(part ? 8 : 4) + 64u + 64u * (uint32_t)t.cls
                                 : draw_channel(part ? 7 : 3) + 64u;
  const bool init = (t.flags & TJ_INIT) != 0;
  const uint32_t l = t.l, m = t.m;
  if (!(t.flags & TJ_HOP)) {
    const uint32_t jm = t.cr;
    tree_split_small(t.n, t.M, cnt, draw_base, dry, [&](int j, int64_t M) {
      const uint32_t bit = 1u << nth_bit(jm, j);
      const int64_t v = sg * M;
      emit(l & ~bit, m & ~bit, part ? 0 : v, part ? v : 0, init);
    });
    return;
  }
  const uint32_t cr = t.cr, cu = t.cu;
  const int nr = popc(cr);
  const bool ket = (t.flags & TJ_KET) != 0;
  tree_split_small(t.n, t.M, cnt, draw_base, dry, [&](int j, int64_t M) {
    uint32_t bm;
    if (j < nr) {
      const uint32_t s = nth_bit(cr, j);
      bm = (1u << s) | (1u << right_site(P, s));
    } else {
      const uint32_t s = nth_bit(cu, j - nr);
      bm = (1u << s) | (1u << up_site(P, s));
    }
    const uint32_t cl = ket ? (l ^ bm) : l;
    const uint32_t cm = ket ? m : (m ^ bm);
    const int64_t v = sg * M;
    // Re parent x Im element -> Im child; Im parent -> -Re child
    emit(cl, cm, part ? -v : 0, part ? 0 : v, init || cl == cm);
  });
}

// entry_events for entries whose every draw uses inversion; returns false
// (having emitted nothing) when the entry needs the general path.  The draws,
// and so the contributions, are identical to entry_events'.
template <typename Emit, typename Trees>
DQ_HD bool entry_events_small(const SlotParams &P, double S, uint32_t step, uint32_t l,
                              uint32_t m, int32_t R, int32_t I, int *err, Emit &&emit,
                              Trees &trees) {
  const EntryProbs e = entry_probs(P, S, step, l, m, R, I);
  const double pk[4] = {e.p8[0], e.p8[1], e.p8[2], e.p8[3]};
  const int64_t nR = e.n8[0], nI = e.n8[4];
  if (!all_small(nR, nI, pk[0], pk[1], pk[2], pk[3])) return false;
  // successive primary uniforms locate the channels with events
  Stream prim(e.cnt.seed, e.cnt.solve, e.cnt.cfg, e.cnt.step, 0, nullptr);
  int64_t X0 = 0, X1 = 0, X2 = 0, X3 = 0, X4 = 0, X5 = 0, X6 = 0, X7 = 0;
  int dry = 0;
  int start = 0;
  // each channel's zero probability once (1 for an empty channel: multiplying
  // by it leaves the running product as it is)
  double f[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int64_t nk = k < 4 ? nR : nI;
    f[k] = (nk > 0 && pk[k & 3] > 0.0) ? ipow(1.0 - pk[k & 3], nk) : 1.0;
  }
#pragma unroll 1
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
    const int64_t nk = first < 4 ? nR : nI;
    double p = pk[0];
    p = (first & 3) == 1 ? pk[1] : p;
    p = (first & 3) == 2 ? pk[2] : p;
    p = (first & 3) == 3 ? pk[3] : p;
    const int64_t x = binomial_small(e.cnt.seed, e.cnt.solve, e.cnt.cfg, e.cnt.step,
                                     draw_channel(first + 1), nk, p, true, dry);
    X0 = first == 0 ? x : X0;
    X1 = first == 1 ? x : X1;
    X2 = first == 2 ? x : X2;
    X3 = first == 3 ? x : X3;
    X4 = first == 4 ? x : X4;
    X5 = first == 5 ? x : X5;
    X6 = first == 6 ? x : X6;
    X7 = first == 7 ? x : X7;
    start = first + 1;
  }
  // larger spawn counts can need the rejection sampler in their splits
  if (X2 >= 20 || X3 >= 20 || X6 >= 20 || X7 >= 20) return false;
  // room for the entry's member trees (one per jump part with two or more
  // walkers, one per hop class reached by a part with two or more), else the
  // general path takes the entry
  const int ntree = (X2 >= 2 ? 1 : 0) + (X6 >= 2 ? 1 : 0) + (X3 >= 2 ? (X3 < 6 ? (int)X3 : 6) : 0) +
                    (X7 >= 2 ? (X7 < 6 ? (int)X7 : 6) : 0);
  if (ntree > 0 && !trees.reserve(ntree)) return false;
  if (dry) *err = 1;

  // the hop classes again, after the channel search, so that their tables are
  // not held in registers through it (the opaque copy of l, m keeps the
  // compiler from reusing the first computation)
  uint32_t lo = l, mo = m;
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(lo), "+v"(mo));
#endif
  const HopClasses hc = hop_classes(P, geometry(P, lo, mo), lo, mo);
  const uint32_t cr0 = hc.r[0], cr1 = hc.r[1], cr2 = hc.r[2], cr3 = hc.r[3], cr4 = hc.r[4],
                 cr5 = hc.r[5];
  const uint32_t cu0 = hc.u[0], cu1 = hc.u[1], cu2 = hc.u[2], cu3 = hc.u[3], cu4 = hc.u[4],
                 cu5 = hc.u[5];
  const int cn0 = hc.n[0], cn1 = hc.n[1], cn2 = hc.n[2], cn3 = hc.n[3], cn4 = hc.n[4],
            cn5 = hc.n[5];
  const int cs0 = hc.sgn[0], cs1 = hc.sgn[1], cs2 = hc.sgn[2], cs3 = hc.sgn[3], cs4 = hc.sgn[4],
            cs5 = hc.sgn[5];
  const double cw0 = hc.W[0], cw1 = hc.W[1], cw2 = hc.W[2], cw3 = hc.W[3], cw4 = hc.W[4],
               cw5 = hc.W[5];
  // suffix sums of the class weights, in entry_probs' order
  const double sc5 = cw5, sc4 = cw4 + sc5, sc3 = cw3 + sc4, sc2 = cw2 + sc3, sc1 = cw1 + sc2,
               sc0 = cw0 + sc1;

  const int64_t sR = e.sR, sI = e.sI;
  const int64_t dR = sR * sgnd(e.d_r) * X0 - sI * sgnd(e.d_i) * X5;
  const int64_t dI = sI * sgnd(e.d_r) * X4 + sR * sgnd(e.d_i) * X1;
  if (dR != 0 || dI != 0) emit(l, m, dR, dI, true);
  const bool init = e.init;

  // jumps, then hops; part 0 = real walkers, part 1 = imaginary walkers
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    const int64_t cj = part ? X6 : X2;
    const int64_t sg = part ? sI : sR;
    if (cj > 0) {
      const uint32_t jm = e.jm;
      auto leaf = [&](int j, int64_t M) {
        const uint32_t bit = 1u << nth_bit(jm, j);
        const int64_t v = sg * M;
        emit(l & ~bit, m & ~bit, part ? 0 : v, part ? v : 0, init);
      };
      if (cj == 1)
        leaf(pick_member(e.cnt, draw_channel(part ? 7 : 3) + DRAW_PICK, e.nJ), 1);
      else
        trees.push(TreeJob{l, m, jm, 0u, 0, (uint8_t)e.nJ, (uint8_t)cj,
                           (uint8_t)((part ? TJ_IM : 0) | (init ? TJ_INIT : 0) |
                                     (sg < 0 ? TJ_NEG : 0)),
                           0, 0});
    }
    int64_t rem = part ? X7 : X3;
    if (rem == 0) continue;
    const int ch = part ? 8 : 4;
    if (rem == 1) {  // one walker: class by inversion on the weights, then a member
      // class by inversion on the weights (the smallest c with S_{c+1} < S_0 (1 - u1)),
      // then a uniform member from u2, as pick_hop
      Stream st(e.cnt.seed, e.cnt.solve, e.cnt.cfg, e.cnt.step, draw_channel(ch) + DRAW_PICK,
                nullptr);
      const double u1 = st.next();
      const double u2 = st.next();
      const double T = sc0 * (1.0 - u1);
      int c = 5;
      c = sc5 < T ? 4 : c;
      c = sc4 < T ? 3 : c;
      c = sc3 < T ? 2 : c;
      c = sc2 < T ? 1 : c;
      c = sc1 < T ? 0 : c;
      const int nc = sel6(c, cn0, cn1, cn2, cn3, cn4, cn5);
      int j = (int)__builtin_floor(u2 * (double)nc);
      j = j > nc - 1 ? nc - 1 : j;
      const uint32_t bm = class_member_mask(P, sel6(c, cr0, cr1, cr2, cr3, cr4, cr5),
                                            sel6(c, cu0, cu1, cu2, cu3, cu4, cu5), j);
      const uint32_t cl = c < 3 ? (l ^ bm) : l;
      const uint32_t cm = c < 3 ? m : (m ^ bm);
      const int64_t v = sg * (int64_t)sel6(c, cs0, cs1, cs2, cs3, cs4, cs5);
      emit(cl, cm, part ? -v : 0, part ? 0 : v, init || cl == cm);
      continue;
    }
    int last = -1;
    last = cw0 > 0.0 ? 0 : last;
    last = cw1 > 0.0 ? 1 : last;
    last = cw2 > 0.0 ? 2 : last;
    last = cw3 > 0.0 ? 3 : last;
    last = cw4 > 0.0 ? 4 : last;
    last = cw5 > 0.0 ? 5 : last;
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
      const double Wc = sel6(c, cw0, cw1, cw2, cw3, cw4, cw5);
      if (rem == 0 || Wc == 0.0) continue;
      int64_t Mc = rem;
      if (c != last)
        Mc = binomial_small(e.cnt.seed, e.cnt.solve, e.cnt.cfg, e.cnt.step,
                            draw_channel(ch) + 1u + (uint32_t)c, rem,
                            Wc / sel6(c, sc0, sc1, sc2, sc3, sc4, sc5), false, dry);
      rem -= Mc;
      if (Mc == 0) continue;
      const uint32_t cr = sel6(c, cr0, cr1, cr2, cr3, cr4, cr5);
      const uint32_t cu = sel6(c, cu0, cu1, cu2, cu3, cu4, cu5);
      const int64_t sv = sg * (int64_t)sel6(c, cs0, cs1, cs2, cs3, cs4, cs5);
      trees.push(TreeJob{l, m, cr, cu, 0, (uint8_t)sel6(c, cn0, cn1, cn2, cn3, cn4, cn5),
                         (uint8_t)Mc,
                         (uint8_t)(TJ_HOP | (part ? TJ_IM : 0) | (c < 3 ? TJ_KET : 0) |
                                   (init ? TJ_INIT : 0) | (sv < 0 ? TJ_NEG : 0)),
                         (uint8_t)c, 0});
    }
  }
  if (dry) *err = 1;
  return true;
}

// Estimator contributions of one entry of the new list (Sec. III.A, V.A),
// each handed to add(sum index, value).
template <class Add>
DQ_HD void entry_sums(const SlotParams &P, uint32_t l, uint32_t m, int64_t R, int64_t I,
                      Add &&add) {
  const int64_t aR = R < 0 ? -R : R, aI = I < 0 ? -I : I;
  add(S_WTOT, aR + aI);
  add(S_NENT, 1);
  if (l == m) {
    const uint32_t alr = ~(l ^ right_of(P, l)) & P.rmask;
    const uint32_t alu = ~(l ^ up_of(P, l)) & P.umask;
    add(S_T_RE, R);
    add(S_T_IM, I);
    add(S_NW, aR);
    add(S_Z, R * (int64_t)(2 * popc(l) - (int)P.N));
    add(S_CZZ, R * (int64_t)(2 * (popc(alr) + popc(alu)) - (int)P.nb));
    return;
  }
  const uint32_t d = l ^ m;
  const int pd = popc(d);
  if (pd == 1) {
    add(S_X, R);
    add(S_Y, (l & d) ? -I : I);
  } else if (pd == 2) {
    const uint32_t tr = d & right_of(P, d) & P.rmask;
    const uint32_t tu = d & up_of(P, d) & P.umask;
    if (tr | tu) {
      const bool al = ((~(l ^ right_of(P, l)) & tr) | (~(l ^ up_of(P, l)) & tu)) != 0;
      add(S_CXX, R);
      add(S_CYY, al ? -R : R);
    }
  }
}

}  // namespace ddqmc
