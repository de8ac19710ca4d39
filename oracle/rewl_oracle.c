/*
 * Reference oracle for replica-exchange Wang-Landau sampling.
 * TEST INFRASTRUCTURE ONLY -- see rewl_oracle.h for scope and the paper
 * passages followed.  Plain single-threaded C, FP64 unless the FP32
 * compensated mode is selected; built with -O2 -ffp-contract=off and no
 * fast-math so every floating-point operation is the one written here.
 *
 * Parity status per function (what pins it, see tests/):
 *   philox            pinned: rocRAND's host-compiled philox4x32_10
 *   exp_spec/expf     pinned: libm exp / mpmath, ulp bound
 *   energy            pinned: brute-force enumeration, incremental-vs-full
 *   windows           pinned: closed-form edges, overlap fraction
 *   WL + REWL cycle   pinned: converged ln g vs exact Ising DOS (brute force,
 *                     Kaufman torus formula) and Potts sum rules; exchange
 *                     with frozen exact ln g accepts every in-range swap
 *   stitch/normalise  pinned: exact ln g with per-window offsets recovered
 *   thermo            pinned: closed-form 2-level / independent sums
 *   two-float ops     pinned: against FP64 / exact rational arithmetic
 */
#include "rewl_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of a   */
/* 4x32 Feistel-like network; each round multiplies counter words 0 and */
/* 2 by fixed 32-bit constants, mixes the high halves with words 1 and  */
/* 3 and the round key, and the key is bumped by two Weyl constants.    */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* RNG streams: the fourth counter word carries tag | instance << 8. */
enum { TAG_MC = 0, TAG_PERM = 1, TAG_ACC = 2, TAG_WARM = 3, TAG_INIT = 4 };

static void draw(const orc_sim* s, uint64_t idx, uint32_t word2, uint32_t tag, uint32_t out[4]);

/* ------------------------------------------------------------------ */
/* Deterministic exponential.  exp(x) = 2^n exp(r), n = nearest integer */
/* to x/ln2, r = x - n ln2 by a two-constant (Cody-Waite) split of ln2, */
/* exp(r) by its Taylor series to degree 13 (|r| <= ln2/2, truncation  */
/* < 2^-57) in Horner form with fused multiply-adds.                   */
/* ------------------------------------------------------------------ */
double orc_exp_spec(double x) {
  const double inv_ln2 = 0x1.71547652b82fep+0;
  const double ln2_hi = 0x1.62e42feep-1;        /* 32 significant bits */
  const double ln2_lo = 0x1.a39ef35793c76p-33;  /* ln2 - ln2_hi */
  double n = rint(x * inv_ln2);
  double r = fma(-n, ln2_hi, x);
  r = fma(-n, ln2_lo, r);
  /* 1/k!, k = 13 .. 0 */
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

/* Single-precision counterpart: Taylor degree 8 (truncation < 2^-31). */
float orc_expf_spec(float x) {
  const float inv_ln2 = 0x1.715476p+0f;
  const float ln2_hi = 0x1.62e000p-1f;          /* 12 significant bits */
  const float ln2_lo = 0x1.0bfbe8p-15f;         /* ln2 - ln2_hi */
  float n = rintf(x * inv_ln2);
  float r = fmaf(-n, ln2_hi, x);
  r = fmaf(-n, ln2_lo, r);
  float p = 1.0f / 40320.0f;
  p = fmaf(p, r, 1.0f / 5040.0f);
  p = fmaf(p, r, 1.0f / 720.0f);
  p = fmaf(p, r, 1.0f / 120.0f);
  p = fmaf(p, r, 1.0f / 24.0f);
  p = fmaf(p, r, 1.0f / 6.0f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

/* Acceptance min[1, exp(delta)] (Sec. 2) with u = u53 * 2^-53 in [0,1).
 * For delta < -40, exp(delta) < 2^-53, so u < exp(delta) iff u == 0. */
int orc_accept64(uint64_t u53, double delta) {
  if (delta >= 0.0) return 1;
  if (delta < -40.0) return u53 == 0;
  return (double)u53 * 0x1p-53 < orc_exp_spec(delta);
}

/* Same with a 24-bit uniform; exp(-17) < 2^-24. */
int orc_accept32(uint32_t u24, float delta) {
  if (delta >= 0.0f) return 1;
  if (delta < -17.0f) return u24 == 0;
  return (float)u24 * 0x1p-24f < orc_expf_spec(delta);
}

static uint64_t u53_of(uint32_t hi, uint32_t lo) {
  return (((uint64_t)hi << 32) | lo) >> 11;
}

/* ------------------------------------------------------------------ */
/* Two-float arithmetic (Knuth's TwoSum, Dekker's FastTwoSum).          */
/* ------------------------------------------------------------------ */
static void two_sum(float a, float b, float* s, float* e) {
  float ss = a + b;
  float bb = ss - a;
  *e = (a - (ss - bb)) + (b - bb);
  *s = ss;
}
static void fast_two_sum(float a, float b, float* s, float* e) {
  float ss = a + b;
  *e = b - (ss - a);
  *s = ss;
}
void orc_df_add1(float ah, float al, float b, float* rh, float* rl) {
  float s, e;
  two_sum(ah, b, &s, &e);
  e = e + al;
  fast_two_sum(s, e, rh, rl);
}
void orc_df_add(float ah, float al, float bh, float bl, float* rh, float* rl) {
  float s, e;
  two_sum(ah, bh, &s, &e);
  e = e + (al + bl);
  fast_two_sum(s, e, rh, rl);
}
void orc_df_div_int(float ah, float al, int32_t m, float* rh, float* rl) {
  float fm = (float)m;
  float qh = ah / fm;
  float rem = fmaf(-qh, fm, ah);   /* exact remainder of the rounded quotient */
  float ql = (rem + al) / fm;
  fast_two_sum(qh, ql, rh, rl);
}

/* ------------------------------------------------------------------ */
/* Lattice models.  Ising: E = -sum_<ij> s_i s_j, s = +-1.              */
/* Potts: E = -sum_<ij> delta(s_i, s_j), s in 0..q-1.  Periodic L x L.  */
/* ------------------------------------------------------------------ */
int32_t orc_energy(int32_t model, int32_t L, int32_t q, const int8_t* sp) {
  (void)q;
  int32_t e = 0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int s0 = sp[y * L + x];
      int sr = sp[y * L + (x + 1) % L];
      int sd = sp[((y + 1) % L) * L + x];
      if (model == ORC_ISING) e -= s0 * sr + s0 * sd;
      else e -= (s0 == sr) + (s0 == sd);
    }
  return e;
}

/* Equal-size windows with overlap o = on/od over bins 0..nbins-1
 * (Fig. 1a): real width W = S/(1+(h-1)(1-o)), lo_i = round(i(1-o)W),
 * hi_i = round((i(1-o)+1)W), rounding half up, all in integers. */
int orc_equal_windows(int32_t nbins, int32_t h, int32_t on, int32_t od, int32_t* lo, int32_t* hi) {
  if (h < 1 || od <= 0 || on < 0 || on >= od || nbins < 2) return -1;
  int64_t S = nbins - 1;
  int64_t d = od - on;
  int64_t D = od + (int64_t)(h - 1) * d;
  for (int i = 0; i < h; ++i) {
    lo[i] = (int32_t)((2 * i * d * S + D) / (2 * D));
    hi[i] = (int32_t)((2 * (i * d + od) * S + D) / (2 * D));
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Simulation state                                                     */
/* ------------------------------------------------------------------ */
#define MAX_STAGES 64
struct orc_sim {
  orc_params p;
  int32_t N, L, q, model, binw, nbins, emin, h, m, W, max_nb;
  int32_t *lo, *hi, *nb;
  int8_t** spins;      /* per slot: the configuration it carries */
  int32_t* cfg_id;     /* per slot: identity of that configuration */
  int32_t* E;
  uint64_t *att, *watt;
  double** lng;        /* FP64 mode */
  float **lhi, **llo;  /* FP32 compensated mode */
  uint32_t** H;
  uint8_t** U;         /* per window */
  double* lnf;
  int32_t *stage, *frozen, *phase;
  double** pieces;     /* per slot: ln g captured before the freezing merge */
  int64_t* stage_merge;  /* [h][MAX_STAGES] */
  uint64_t *ex_try, *ex_acc, *ex_inr;
  int64_t merges;
  uint64_t rounds;
  int32_t done;
  int64_t done_merge;
  int32_t warm_fail;
};

static void draw(const orc_sim* s, uint64_t idx, uint32_t word2, uint32_t tag, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), word2,
                     tag | ((uint32_t)s->p.instance << 8)};
  uint32_t key[2] = {(uint32_t)s->p.seed, (uint32_t)(s->p.seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

static int bin_of(const orc_sim* s, int32_t E) { return (E - s->emin) / s->binw; }

/* Neighbour spins of a site (right, left, down, up). */
static void neighbours(const orc_sim* s, const int8_t* sp, int site, int nb[4]) {
  int L = s->L, x = site % L, y = site / L;
  nb[0] = sp[y * L + (x + 1) % L];
  nb[1] = sp[y * L + (x + L - 1) % L];
  nb[2] = sp[((y + 1) % L) * L + x];
  nb[3] = sp[((y + L - 1) % L) * L + x];
}

/* Proposal from one Philox block: site from word 0, Potts target value
 * from word 1 (uniform over the q-1 other values); returns dE. */
static int propose(const orc_sim* s, const int8_t* sp, const uint32_t r[4], int* site, int* newv) {
  int st = (int)(((uint64_t)r[0] * (uint32_t)s->N) >> 32);
  int nb[4];
  neighbours(s, sp, st, nb);
  int old = sp[st];
  int dE;
  if (s->model == ORC_ISING) {
    *newv = -old;
    dE = 2 * old * (nb[0] + nb[1] + nb[2] + nb[3]);
  } else {
    int nv = (old + 1 + (int)(((uint64_t)r[1] * (uint32_t)(s->q - 1)) >> 32)) % s->q;
    int eq_old = (nb[0] == old) + (nb[1] == old) + (nb[2] == old) + (nb[3] == old);
    int eq_new = (nb[0] == nv) + (nb[1] == nv) + (nb[2] == nv) + (nb[3] == nv);
    *newv = nv;
    dE = eq_old - eq_new;
  }
  *site = st;
  return dE;
}

static int32_t dist_to(int32_t E, int32_t elo, int32_t ehi) {
  if (E < elo) return elo - E;
  if (E > ehi) return E - ehi;
  return 0;
}

/* Warm-up: greedy moves that never increase the distance of E to the
 * window, budget 1000 N attempts; on failure restart once from an extreme
 * state (ground state below the middle of the range, checkerboard above). */
static int warm_up(orc_sim* s, int slot) {
  int w = slot / s->m;
  int32_t elo = s->emin + s->lo[w] * s->binw, ehi = s->emin + s->hi[w] * s->binw;
  int8_t* sp = s->spins[slot];
  int32_t E = orc_energy(s->model, s->L, s->q, sp);
  for (int phase = 0; phase < 2; ++phase) {
    int64_t budget = 1000LL * s->N;
    for (int64_t it = 0; it < budget && dist_to(E, elo, ehi) > 0; ++it) {
      uint32_t r[4];
      draw(s, s->watt[slot]++, (uint32_t)slot, TAG_WARM, r);
      int site, nv;
      int dE = propose(s, sp, r, &site, &nv);
      if (dist_to(E + dE, elo, ehi) <= dist_to(E, elo, ehi)) {
        sp[site] = (int8_t)nv;
        E += dE;
      }
    }
    if (dist_to(E, elo, ehi) == 0) break;
    if (phase == 0) {
      uint32_t r[4];
      draw(s, s->watt[slot]++, (uint32_t)slot, TAG_WARM, r);
      int below = (s->lo[w] + s->hi[w]) < (s->nbins - 1);
      int a, b;
      if (s->model == ORC_ISING) {
        a = (r[0] >> 31) ? 1 : -1;
        b = -a;
      } else {
        a = (int)(((uint64_t)r[0] * (uint32_t)s->q) >> 32);
        b = (a + 1 + (int)(((uint64_t)r[1] * (uint32_t)(s->q - 1)) >> 32)) % s->q;
      }
      for (int y = 0; y < s->L; ++y)
        for (int x = 0; x < s->L; ++x)
          sp[y * s->L + x] = (int8_t)((below || ((x + y) & 1) == 0) ? a : b);
      E = orc_energy(s->model, s->L, s->q, sp);
    }
  }
  s->E[slot] = E;
  return dist_to(E, elo, ehi) == 0 ? 0 : -1;
}

static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

orc_sim* orc_new(const orc_params* p, const int32_t* win_lo, const int32_t* win_hi) {
  if (!p) return NULL;
  if (p->model != ORC_ISING && p->model != ORC_POTTS) return NULL;
  if (p->L < 2 || p->L > 4096) return NULL;
  if (p->model == ORC_POTTS && (p->q < 2 || p->q > 127)) return NULL;
  if (p->n_windows < 1 || p->walkers_per_window < 1) return NULL;
  if (p->flat_den <= 0 || p->flat_num < 0 || p->flat_num > p->flat_den) return NULL;
  if (p->flips_per_exchange < 0) return NULL;
  if (p->precision != ORC_FP64 && p->precision != ORC_FP32C) return NULL;
  if (p->schedule != ORC_HALVING && p->schedule != ORC_ONE_OVER_T) return NULL;
  if (!(p->lnf_init > 0.0) || !(p->lnf_final > 0.0)) return NULL;
  if ((win_lo == NULL) != (win_hi == NULL)) return NULL;

  orc_sim* s = (orc_sim*)xcalloc(1, sizeof(orc_sim));
  s->p = *p;
  s->L = p->L;
  s->N = p->L * p->L;
  s->model = p->model;
  s->q = p->model == ORC_POTTS ? p->q : 2;
  s->emin = -2 * s->N;
  if (s->model == ORC_ISING) s->binw = 4;
  else s->binw = (s->q == 2) ? 2 : 1;
  int32_t emax = (s->model == ORC_ISING) ? 2 * s->N : 0;
  s->nbins = (emax - s->emin) / s->binw + 1;
  s->h = p->n_windows;
  s->m = p->walkers_per_window;
  s->W = s->h * s->m;

  s->lo = (int32_t*)xcalloc(s->h, 4);
  s->hi = (int32_t*)xcalloc(s->h, 4);
  s->nb = (int32_t*)xcalloc(s->h, 4);
  int bad = 0;
  if (win_lo) {
    memcpy(s->lo, win_lo, 4 * (size_t)s->h);
    memcpy(s->hi, win_hi, 4 * (size_t)s->h);
  } else if (orc_equal_windows(s->nbins, s->h, p->overlap_num, p->overlap_den, s->lo, s->hi)) {
    bad = 1;
  }
  for (int w = 0; w < s->h && !bad; ++w) {
    if (s->lo[w] < 0 || s->hi[w] >= s->nbins || s->hi[w] - s->lo[w] < 4) bad = 1;
    if (w > 0 && (s->lo[w] <= s->lo[w - 1] || s->hi[w] <= s->hi[w - 1] || s->lo[w] > s->hi[w - 1])) bad = 1;
    s->nb[w] = s->hi[w] - s->lo[w] + 1;
    if (s->nb[w] > s->max_nb) s->max_nb = s->nb[w];
  }
  if (bad) { orc_free(s); return NULL; }

  s->spins = (int8_t**)xcalloc(s->W, sizeof(int8_t*));
  s->cfg_id = (int32_t*)xcalloc(s->W, 4);
  s->E = (int32_t*)xcalloc(s->W, 4);
  s->att = (uint64_t*)xcalloc(s->W, 8);
  s->watt = (uint64_t*)xcalloc(s->W, 8);
  s->H = (uint32_t**)xcalloc(s->W, sizeof(uint32_t*));
  if (p->precision == ORC_FP64) s->lng = (double**)xcalloc(s->W, sizeof(double*));
  else {
    s->lhi = (float**)xcalloc(s->W, sizeof(float*));
    s->llo = (float**)xcalloc(s->W, sizeof(float*));
  }
  for (int slot = 0; slot < s->W; ++slot) {
    int w = slot / s->m;
    s->spins[slot] = (int8_t*)xcalloc(s->N, 1);
    s->cfg_id[slot] = slot;
    s->H[slot] = (uint32_t*)xcalloc(s->nb[w], 4);
    if (s->lng) s->lng[slot] = (double*)xcalloc(s->nb[w], 8);
    else {
      s->lhi[slot] = (float*)xcalloc(s->nb[w], 4);
      s->llo[slot] = (float*)xcalloc(s->nb[w], 4);
    }
  }
  s->U = (uint8_t**)xcalloc(s->h, sizeof(uint8_t*));
  for (int w = 0; w < s->h; ++w) s->U[w] = (uint8_t*)xcalloc(s->nb[w], 1);
  s->lnf = (double*)xcalloc(s->h, 8);
  s->stage = (int32_t*)xcalloc(s->h, 4);
  s->frozen = (int32_t*)xcalloc(s->h, 4);
  s->phase = (int32_t*)xcalloc(s->h, 4);
  s->pieces = (double**)xcalloc(s->W, sizeof(double*));
  for (int slot = 0; slot < s->W; ++slot) s->pieces[slot] = (double*)xcalloc(s->nb[slot / s->m], 8);
  s->stage_merge = (int64_t*)xcalloc((size_t)s->h * MAX_STAGES, 8);
  s->ex_try = (uint64_t*)xcalloc(s->h, 8);
  s->ex_acc = (uint64_t*)xcalloc(s->h, 8);
  s->ex_inr = (uint64_t*)xcalloc(s->h, 8);
  for (size_t i = 0; i < (size_t)s->h * MAX_STAGES; ++i) s->stage_merge[i] = -1;
  for (int w = 0; w < s->h; ++w) {
    s->lnf[w] = p->lnf_init;
    s->frozen[w] = p->lnf_init <= p->lnf_final;
  }
  s->done_merge = -1;

  /* Random initial spins: one INIT block per 4 sites. */
  for (int slot = 0; slot < s->W; ++slot) {
    for (int site = 0; site < s->N; ++site) {
      uint32_t r[4];
      draw(s, (uint64_t)(site / 4), (uint32_t)slot, TAG_INIT, r);
      uint32_t v = r[site % 4];
      if (s->model == ORC_ISING) s->spins[slot][site] = (int8_t)((v >> 31) ? 1 : -1);
      else s->spins[slot][site] = (int8_t)(((uint64_t)v * (uint32_t)s->q) >> 32);
    }
    if (warm_up(s, slot)) s->warm_fail = -1;
  }
  int all = 1;
  for (int w = 0; w < s->h; ++w) all &= s->frozen[w];
  if (all) { s->done = 1; s->done_merge = -1; }
  return s;
}

void orc_free(orc_sim* s) {
  if (!s) return;
  for (int slot = 0; s->spins && slot < s->W; ++slot) {
    free(s->spins[slot]);
    if (s->H) free(s->H[slot]);
    if (s->lng) free(s->lng[slot]);
    if (s->lhi) { free(s->lhi[slot]); free(s->llo[slot]); }
  }
  for (int w = 0; s->U && w < s->h; ++w) free(s->U[w]);
  for (int slot = 0; s->pieces && slot < s->W; ++slot) free(s->pieces[slot]);
  free(s->pieces); free(s->phase);
  free(s->spins); free(s->cfg_id); free(s->E); free(s->att); free(s->watt);
  free(s->H); free(s->lng); free(s->lhi); free(s->llo); free(s->U);
  free(s->lnf); free(s->stage); free(s->frozen); free(s->stage_merge);
  free(s->ex_try); free(s->ex_acc); free(s->ex_inr); free(s->lo); free(s->hi); free(s->nb);
  free(s);
}

int orc_get_info(const orc_sim* s, orc_info* o) {
  if (!s || !o) return -1;
  o->N = s->N; o->nbins = s->nbins; o->binw = s->binw; o->emin = s->emin;
  o->h = s->h; o->m = s->m; o->W = s->W; o->max_nb = s->max_nb;
  return 0;
}

int orc_get_windows(const orc_sim* s, int32_t* lo, int32_t* hi) {
  if (!s) return -1;
  for (int w = 0; w < s->h; ++w) { if (lo) lo[w] = s->lo[w]; if (hi) hi[w] = s->hi[w]; }
  return 0;
}

int orc_warm_status(const orc_sim* s) { return s ? s->warm_fail : -1; }

/* ------------------------------------------------------------------ */
/* One Wang-Landau attempt for one walker (Sec. 2).                     */
/* ------------------------------------------------------------------ */
static void wl_attempt(orc_sim* s, int slot) {
  int w = slot / s->m;
  int8_t* sp = s->spins[slot];
  uint32_t r[4];
  draw(s, s->att[slot]++, (uint32_t)slot, TAG_MC, r);
  int site, nv;
  int dE = propose(s, sp, r, &site, &nv);
  int b = bin_of(s, s->E[slot]);
  int bn = b + dE / s->binw;
  int lo = s->lo[w];
  int accept = 0;
  if (bn >= lo && bn <= s->hi[w]) {
    if (s->lng) {
      /* ln[g(E_old)/g(E_new)] */
      double delta = s->lng[slot][b - lo] - s->lng[slot][bn - lo];
      accept = orc_accept64(u53_of(r[2], r[3]), delta);
    } else {
      float* hi = s->lhi[slot];
      float* lw = s->llo[slot];
      float delta = (hi[b - lo] - hi[bn - lo]) + (lw[b - lo] - lw[bn - lo]);
      accept = orc_accept32(r[2] >> 8, delta);
    }
  }
  if (accept) {
    sp[site] = (int8_t)nv;
    s->E[slot] += dE;
    b = bn;
  }
  if (!s->frozen[w]) {
    /* g(E) -> f g(E) and H(E) += 1 at the walker's current energy */
    if (s->lng) s->lng[slot][b - lo] += s->lnf[w];
    else orc_df_add1(s->lhi[slot][b - lo], s->llo[slot][b - lo], (float)s->lnf[w],
                     &s->lhi[slot][b - lo], &s->llo[slot][b - lo]);
    s->H[slot][b - lo] += 1u;
  }
}

int orc_sweep(orc_sim* s, int64_t flips) {
  if (!s) return -1;
  if (s->done) return 0;
  for (int slot = 0; slot < s->W; ++slot)
    for (int64_t t = 0; t < flips; ++t) wl_attempt(s, slot);
  return 0;
}

/* Pairwise sum by levels: adjacent pairs are added, an odd last element is
 * carried up unchanged, until one value remains. */
static double tree_sum64(double* v, int n) {
  while (n > 1) {
    int k = 0;
    for (int i = 0; i + 1 < n; i += 2) v[k++] = v[i] + v[i + 1];
    if (n & 1) v[k++] = v[n - 1];
    n = k;
  }
  return v[0];
}
static void tree_sum32(float* vh, float* vl, int n, float* rh, float* rl) {
  while (n > 1) {
    int k = 0;
    for (int i = 0; i + 1 < n; i += 2) {
      float a, b;
      orc_df_add(vh[i], vl[i], vh[i + 1], vl[i + 1], &a, &b);
      vh[k] = a; vl[k] = b; ++k;
    }
    if (n & 1) { vh[k] = vh[n - 1]; vl[k] = vl[n - 1]; ++k; }
    n = k;
  }
  *rh = vh[0]; *rl = vl[0];
}

static double lng_at(const orc_sim* s, int slot, int j);

/* Average the m walkers' ln g of window w bin by bin (geometric mean of g),
 * redistribute, reset H. */
static void merge_window(orc_sim* s, int w, double* t64, float* th, float* tl) {
  int m = s->m;
  for (int j = 0; j < s->nb[w]; ++j) {
    if (s->lng) {
      for (int k = 0; k < m; ++k) t64[k] = s->lng[w * m + k][j];
      double mean = tree_sum64(t64, m) / (double)m;
      for (int k = 0; k < m; ++k) s->lng[w * m + k][j] = mean;
    } else {
      for (int k = 0; k < m; ++k) { th[k] = s->lhi[w * m + k][j]; tl[k] = s->llo[w * m + k][j]; }
      float sh, sl, mh, ml;
      tree_sum32(th, tl, m, &sh, &sl);
      orc_df_div_int(sh, sl, m, &mh, &ml);
      for (int k = 0; k < m; ++k) { s->lhi[w * m + k][j] = mh; s->llo[w * m + k][j] = ml; }
    }
    for (int k = 0; k < m; ++k) s->H[w * m + k][j] = 0;
  }
}

/* Flatness check for every non-frozen window (Sec. 2).
 * Halving schedule: when all m walkers of a window are flat at the same
 * check, their ln g are averaged and redistributed, H is reset and
 * ln f -> ln f / 2 (f -> sqrt f).
 * 1/t schedule (Belardinelli-Pereyra, which Sec. 2 names as compatible):
 * phase A halves ln f, with the same merge, once every walker has visited
 * every bin of the window's visited union; when ln f <= 1/t (t = attempts
 * per walker / visited bins) the window enters phase B, where every check
 * sets ln f = 1/t and merges.
 * A window freezes when ln f <= ln f_final; the walkers' ln g just before
 * that merge are kept for the jackknife. */
int orc_merge(orc_sim* s) {
  if (!s) return -1;
  if (s->done) return 0;
  int m = s->m;
  double* t64 = (double*)xcalloc(m, 8);
  float* th = (float*)xcalloc(m, 4);
  float* tl = (float*)xcalloc(m, 4);
  for (int w = 0; w < s->h; ++w) {
    if (s->frozen[w]) continue;
    int nbw = s->nb[w];
    for (int j = 0; j < nbw; ++j)
      for (int k = 0; k < m; ++k)
        if (s->H[w * m + k][j] > 0) s->U[w][j] = 1;
    uint64_t cnt = 0;
    for (int j = 0; j < nbw; ++j) cnt += s->U[w][j];
    int ready = cnt > 0;
    int phase_b = s->p.schedule == ORC_ONE_OVER_T && s->phase[w] == 1;
    for (int k = 0; k < m && ready && !phase_b; ++k) {
      const uint32_t* H = s->H[w * m + k];
      uint64_t mn = UINT64_MAX, sum = 0;
      for (int j = 0; j < nbw; ++j) {
        sum += H[j];
        if (s->U[w][j] && H[j] < mn) mn = H[j];
      }
      if (s->p.schedule == ORC_HALVING) {
        if ((uint64_t)s->p.flat_den * cnt * mn < (uint64_t)s->p.flat_num * sum) ready = 0;
      } else if (mn == 0) {
        ready = 0;
      }
    }
    if (!ready) continue;
    /* new ln f and phase of this window */
    double tinv = (double)cnt / (double)s->att[w * m];
    double next = phase_b ? tinv : 0.5 * s->lnf[w];
    int to_b = s->p.schedule == ORC_ONE_OVER_T && !phase_b && next <= tinv;
    if (to_b) next = tinv;
    if (next <= s->p.lnf_final)
      for (int k = 0; k < m; ++k)
        for (int j = 0; j < nbw; ++j) s->pieces[w * m + k][j] = lng_at(s, w * m + k, j);
    merge_window(s, w, t64, th, tl);
    if (!phase_b) {
      if (s->stage[w] < MAX_STAGES) s->stage_merge[(size_t)w * MAX_STAGES + s->stage[w]] = s->merges;
      s->stage[w] += 1;
    }
    s->lnf[w] = next;
    if (to_b) s->phase[w] = 1;
    if (next <= s->p.lnf_final) s->frozen[w] = 1;
  }
  free(t64); free(th); free(tl);
  int all = 1;
  for (int w = 0; w < s->h; ++w) all &= s->frozen[w];
  if (all) { s->done = 1; s->done_merge = s->merges; }
  s->merges += 1;
  return 0;
}

static double lng_at(const orc_sim* s, int slot, int j) {
  if (s->lng) return s->lng[slot][j];
  return (double)s->lhi[slot][j] + (double)s->llo[slot][j];
}

/* Replica exchange round t (Sec. 2, Eq. 1): window pairs (w, w+1) with
 * w = t mod 2; walker k of window w is paired with walker pi(k) of window
 * w+1, pi a uniform random permutation (Fisher-Yates); pairs are drawn
 * without looking at energies; a pair with an energy outside the other
 * window is disregarded; otherwise accept with
 * min[1, g_i(E_X)/g_i(E_Y) * g_j(E_Y)/g_j(E_X)] and swap configurations. */
/* Partner choice of Sec. 2 (a walker picks a random partner in the
 * neighbouring window): a uniformly random permutation pi of 0..m-1 by the
 * Fisher-Yates shuffle.  For i = m-1 down to 1, j is uniform in 0..i,
 * j = (r (i+1)) >> 32 with r the next 32-bit word of the EXCH_PERM stream
 * (counter: round, (w << 8) | call, instance tag; four words per call), and
 * pi[i], pi[j] are swapped.  Walker k of window w meets walker pi[k] of
 * window w+1. */
int orc_exchange_pairing(uint64_t seed, int32_t instance, uint64_t round, int32_t w, int32_t m,
                         int32_t* pi) {
  if (!pi || m < 1 || w < 0 || instance < 0) return -1;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int k = 0; k < m; ++k) pi[k] = k;
  uint32_t r[4];
  int used = 4, call = 0;
  for (int i = m - 1; i >= 1; --i) {
    if (used == 4) {
      uint32_t ctr[4] = {(uint32_t)round, (uint32_t)(round >> 32), ((uint32_t)w << 8) | (uint32_t)call++,
                         TAG_PERM | ((uint32_t)instance << 8)};
      orc_philox4x32_10(ctr, key, r);
      used = 0;
    }
    int j = (int)(((uint64_t)r[used++] * (uint32_t)(i + 1)) >> 32);
    int32_t tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
  }
  return 0;
}

int orc_exchange(orc_sim* s) {
  if (!s) return -1;
  if (s->done) return 0;
  int m = s->m;
  uint64_t t = s->rounds;
  int32_t* pi = (int32_t*)xcalloc(m, sizeof(int32_t));
  for (int w = (int)(t & 1); w + 1 < s->h; w += 2) {
    uint32_t r[4];
    orc_exchange_pairing(s->p.seed, s->p.instance, t, w, m, pi);
    for (int k = 0; k < m; ++k) {
      int si = w * m + k, sj = (w + 1) * m + pi[k];
      int bx = bin_of(s, s->E[si]), by = bin_of(s, s->E[sj]);
      s->ex_try[w] += 1;
      if (by < s->lo[w] || by > s->hi[w] || bx < s->lo[w + 1] || bx > s->hi[w + 1]) continue;
      s->ex_inr[w] += 1;
      int ix = bx - s->lo[w], iy = by - s->lo[w];
      int jx = bx - s->lo[w + 1], jy = by - s->lo[w + 1];
      draw(s, t, (uint32_t)si, TAG_ACC, r);
      int accept;
      if (s->lng) {
        double lnP = (s->lng[si][ix] - s->lng[si][iy]) + (s->lng[sj][jy] - s->lng[sj][jx]);
        accept = orc_accept64(u53_of(r[2], r[3]), lnP);
      } else {
        float a = (s->lhi[si][ix] - s->lhi[si][iy]) + (s->llo[si][ix] - s->llo[si][iy]);
        float b = (s->lhi[sj][jy] - s->lhi[sj][jx]) + (s->llo[sj][jy] - s->llo[sj][jx]);
        accept = orc_accept32(r[2] >> 8, a + b);
      }
      if (accept) {
        int8_t* tp = s->spins[si]; s->spins[si] = s->spins[sj]; s->spins[sj] = tp;
        int32_t te = s->E[si]; s->E[si] = s->E[sj]; s->E[sj] = te;
        int32_t tc = s->cfg_id[si]; s->cfg_id[si] = s->cfg_id[sj]; s->cfg_id[sj] = tc;
        s->ex_acc[w] += 1;
      }
    }
  }
  free(pi);
  s->rounds += 1;
  return 0;
}

int64_t orc_run(orc_sim* s, int64_t max_cycles) {
  if (!s) return -1;
  int64_t c = 0;
  for (; c < max_cycles && !s->done; ++c) {
    orc_sweep(s, s->p.flips_per_exchange);
    orc_merge(s);
    if (!s->done) orc_exchange(s);
  }
  return c;
}

int orc_status(const orc_sim* s, orc_status_t* o) {
  if (!s || !o) return -1;
  o->done = s->done; o->pad = 0; o->done_merge = s->done_merge;
  o->merges = s->merges; o->rounds = s->rounds;
  return 0;
}

int orc_get_walker(const orc_sim* s, int32_t slot, int8_t* spins, int32_t* E, uint32_t* H,
                   double* lng64, uint64_t* attempts, int32_t* config_id) {
  if (!s || slot < 0 || slot >= s->W) return -1;
  int w = slot / s->m;
  if (spins) memcpy(spins, s->spins[slot], (size_t)s->N);
  if (E) *E = s->E[slot];
  if (H) memcpy(H, s->H[slot], 4 * (size_t)s->nb[w]);
  if (lng64) for (int j = 0; j < s->nb[w]; ++j) lng64[j] = lng_at(s, slot, j);
  if (attempts) *attempts = s->att[slot];
  if (config_id) *config_id = s->cfg_id[slot];
  return 0;
}

int orc_set_walker_lng(orc_sim* s, int32_t slot, const double* lng64) {
  if (!s || slot < 0 || slot >= s->W || !lng64) return -1;
  int w = slot / s->m;
  for (int j = 0; j < s->nb[w]; ++j) {
    if (s->lng) s->lng[slot][j] = lng64[j];
    else {
      float h = (float)lng64[j];
      s->lhi[slot][j] = h;
      s->llo[slot][j] = (float)(lng64[j] - (double)h);
    }
  }
  return 0;
}

int orc_get_walker_f32(const orc_sim* s, int32_t slot, float* hi, float* lo) {
  if (!s || slot < 0 || slot >= s->W || !s->lhi) return -1;
  int w = slot / s->m;
  if (hi) memcpy(hi, s->lhi[slot], 4 * (size_t)s->nb[w]);
  if (lo) memcpy(lo, s->llo[slot], 4 * (size_t)s->nb[w]);
  return 0;
}

int orc_get_phase(const orc_sim* s, int32_t w) {
  if (!s || w < 0 || w >= s->h) return -1;
  return s->phase[w];
}

int orc_get_piece(const orc_sim* s, int32_t slot, double* out) {
  if (!s || !out || slot < 0 || slot >= s->W) return -1;
  memcpy(out, s->pieces[slot], sizeof(double) * (size_t)s->nb[slot / s->m]);
  return 0;
}

int orc_get_window(const orc_sim* s, int32_t w, double* lnf, int32_t* stage, int32_t* frozen,
                   uint8_t* U, int64_t* stage_merge) {
  if (!s || w < 0 || w >= s->h) return -1;
  if (lnf) *lnf = s->lnf[w];
  if (stage) *stage = s->stage[w];
  if (frozen) *frozen = s->frozen[w];
  if (U) memcpy(U, s->U[w], (size_t)s->nb[w]);
  if (stage_merge) memcpy(stage_merge, s->stage_merge + (size_t)w * MAX_STAGES, 8 * MAX_STAGES);
  return 0;
}

int orc_get_exchange_stats(const orc_sim* s, uint64_t* tries, uint64_t* in_range, uint64_t* accepts) {
  if (!s) return -1;
  for (int w = 0; w < s->h; ++w) {
    if (tries) tries[w] = s->ex_try[w];
    if (in_range) in_range[w] = s->ex_inr[w];
    if (accepts) accepts[w] = s->ex_acc[w];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Joining (Sec. 3, Eq. 2).                                             */
/* ------------------------------------------------------------------ */
static double beta5(const double* l, int j) {
  /* five-point first derivative in bin units */
  return (((l[j - 2] - 8.0 * l[j - 1]) + 8.0 * l[j + 1]) - l[j + 2]) / 12.0;
}

int orc_stitch(int32_t h, const int32_t* lo, const int32_t* hi, const double* const* l,
               const uint8_t* const* U, int32_t nbins, double* R, int32_t* joins) {
  if (h < 1) return -1;
  for (int b = 0; b < nbins; ++b) R[b] = -INFINITY;
  for (int b = lo[0]; b <= hi[0]; ++b)
    if (U[0][b - lo[0]]) R[b] = l[0][b - lo[0]];
  double shift = 0.0;
  for (int w = 1; w < h; ++w) {
    const double* la = l[w - 1];
    const double* lb = l[w];
    int oa = lo[w - 1], ob = lo[w];
    int best = -1;
    double bestd = 0.0;
    for (int b = lo[w] + 2; b <= hi[w - 1] - 2; ++b) {
      int ok = 1;
      for (int d = -2; d <= 2 && ok; ++d) ok = U[w - 1][b + d - oa] && U[w][b + d - ob];
      if (!ok) continue;
      double db = fabs(beta5(la, b - oa) - beta5(lb, b - ob));
      if (best < 0 || db < bestd) { best = b; bestd = db; }
    }
    if (best < 0) best = (lo[w] + hi[w - 1]) / 2;
    shift = (la[best - oa] + shift) - lb[best - ob];
    if (joins) joins[w - 1] = best;
    for (int b = best; b <= hi[w]; ++b) R[b] = U[w][b - ob] ? lb[b - ob] + shift : -INFINITY;
  }
  return 0;
}

/* Ising: sum_E g(E) = 2^N.  Potts: g(ground) = q. */
int orc_normalise(int32_t model, int32_t N, int32_t q, int32_t nbins, double* R) {
  double c;
  if (model == ORC_ISING) {
    double mx = -INFINITY;
    for (int b = 0; b < nbins; ++b) if (R[b] > mx) mx = R[b];
    if (!isfinite(mx)) return -1;
    double acc = 0.0;
    for (int b = 0; b < nbins; ++b) if (isfinite(R[b])) acc += exp(R[b] - mx);
    double lse = mx + log(acc);
    c = (double)N * log(2.0) - lse;
  } else {
    if (!isfinite(R[0])) return -1;
    c = log((double)q) - R[0];
  }
  for (int b = 0; b < nbins; ++b) if (isfinite(R[b])) R[b] += c;
  return 0;
}

static int window_rep(const orc_sim* s, int w, double* out) {
  int m = s->m;
  if (s->lng) {
    double* t = (double*)xcalloc(m, 8);
    for (int j = 0; j < s->nb[w]; ++j) {
      for (int k = 0; k < m; ++k) t[k] = s->lng[w * m + k][j];
      out[j] = tree_sum64(t, m) / (double)m;
    }
    free(t);
  } else {
    float* th = (float*)xcalloc(m, 4);
    float* tl = (float*)xcalloc(m, 4);
    for (int j = 0; j < s->nb[w]; ++j) {
      for (int k = 0; k < m; ++k) { th[k] = s->lhi[w * m + k][j]; tl[k] = s->llo[w * m + k][j]; }
      float sh, sl, mh, ml;
      tree_sum32(th, tl, m, &sh, &sl);
      orc_df_div_int(sh, sl, m, &mh, &ml);
      out[j] = (double)mh + (double)ml;
    }
    free(th); free(tl);
  }
  return 0;
}

int orc_join_raw(const orc_sim* s, double* out, int32_t* joins) {
  if (!s || !out) return -1;
  double** reps = (double**)xcalloc(s->h, sizeof(double*));
  for (int w = 0; w < s->h; ++w) {
    reps[w] = (double*)xcalloc(s->nb[w], 8);
    window_rep(s, w, reps[w]);
  }
  int rc = orc_stitch(s->h, s->lo, s->hi, (const double* const*)reps,
                      (const uint8_t* const*)s->U, s->nbins, out, joins);
  for (int w = 0; w < s->h; ++w) free(reps[w]);
  free(reps);
  return rc;
}

int orc_jackknife(const orc_sim* s, double* mean, double* err) {
  if (!s || !mean || !err || s->m < 2 || !s->done) return -1;
  int m = s->m;
  double** reps = (double**)xcalloc(s->h, sizeof(double*));
  for (int w = 0; w < s->h; ++w) reps[w] = (double*)xcalloc(s->nb[w], 8);
  double* Rk = (double*)xcalloc((size_t)m * s->nbins, 8);
  double* t = (double*)xcalloc(m, 8);
  int rc = 0;
  for (int k = 0; k < m && !rc; ++k) {
    for (int w = 0; w < s->h; ++w)
      for (int j = 0; j < s->nb[w]; ++j) {
        int n = 0;
        for (int i = 0; i < m; ++i)
          if (i != k) t[n++] = s->pieces[w * m + i][j];
        reps[w][j] = tree_sum64(t, n) / (double)n;
      }
    double* R = Rk + (size_t)k * s->nbins;
    rc = orc_stitch(s->h, s->lo, s->hi, (const double* const*)reps,
                    (const uint8_t* const*)s->U, s->nbins, R, NULL);
    if (!rc) rc = orc_normalise(s->model, s->N, s->q, s->nbins, R);
  }
  for (int b = 0; b < s->nbins && !rc; ++b) {
    int fin = 1;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
      fin &= isfinite(Rk[(size_t)k * s->nbins + b]) != 0;
      acc += Rk[(size_t)k * s->nbins + b];
    }
    if (!fin) { mean[b] = -INFINITY; err[b] = 0.0; continue; }
    double mu = acc / (double)m, v = 0.0;
    for (int k = 0; k < m; ++k) {
      double d = Rk[(size_t)k * s->nbins + b] - mu;
      v += d * d;
    }
    mean[b] = mu;
    err[b] = sqrt((double)(m - 1) / (double)m * v);
  }
  for (int w = 0; w < s->h; ++w) free(reps[w]);
  free(reps); free(Rk); free(t);
  return rc;
}

int orc_join(const orc_sim* s, double* out, int32_t* joins) {
  int rc = orc_join_raw(s, out, joins);
  if (rc) return rc;
  return orc_normalise(s->model, s->N, s->q, s->nbins, out);
}

/* Canonical averages from g(E) (Sec. 5, Eqs. 7-8, k_B = 1): weights
 * g(E) exp(-E/T) by log-sum-exp, variance by a second pass. */
int orc_thermo(const double* lng, int32_t nbins, int32_t emin, int32_t binw,
               const double* T, int32_t nT, double* Emean, double* Cv) {
  for (int i = 0; i < nT; ++i) {
    double t = T[i];
    double mx = -INFINITY;
    for (int b = 0; b < nbins; ++b) {
      if (!isfinite(lng[b])) continue;
      double a = lng[b] - (double)(emin + b * binw) / t;
      if (a > mx) mx = a;
    }
    double z = 0.0, e1 = 0.0;
    for (int b = 0; b < nbins; ++b) {
      if (!isfinite(lng[b])) continue;
      double E = (double)(emin + b * binw);
      double wgt = exp(lng[b] - E / t - mx);
      z += wgt;
      e1 += wgt * E;
    }
    double em = e1 / z;
    double v = 0.0;
    for (int b = 0; b < nbins; ++b) {
      if (!isfinite(lng[b])) continue;
      double E = (double)(emin + b * binw);
      double wgt = exp(lng[b] - E / t - mx);
      v += wgt * (E - em) * (E - em);
    }
    if (Emean) Emean[i] = em;
    if (Cv) Cv[i] = (v / z) / (t * t);
  }
  return 0;
}
