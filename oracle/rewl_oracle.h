/*
 * Reference oracle for replica-exchange Wang-Landau (REWL) sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, single-threaded, deliberately
 * slow CPU implementation of the method of Li, Vogel, Wuest and Landau,
 * "A new paradigm for petascale Monte Carlo simulation: Replica exchange
 * Wang-Landau sampling" (arXiv:1402.2328).  It exists so that the GPU
 * library can be checked against something written straight from the paper.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the GPU library.
 *
 * Paper passages followed (by section / equation):
 *   Sec. 2, standard WL: accept with min[1, g(E_old)/g(E_new)], g -> f g,
 *           histogram H, flat -> reset H and f -> sqrt(f), stop at f_final.
 *   Sec. 2, REWL: h overlapping windows (Fig. 1a, overlap o), m walkers per
 *           window each with its own g and H, replica exchange between
 *           neighbouring windows with acceptance Eq. (1), out-of-range
 *           exchanges disregarded, merge (average g) when all m walkers of a
 *           window are flat, per-window f, end when every window reaches
 *           f_final.
 *   Sec. 3, joining: beta = d log g / dE, join where |beta_i - beta_j| is
 *           smallest, rescale g_j at E_join, piecewise Eq. (2); 5-point
 *           derivative stencil (Fig. 2 caption).
 *   Sec. 2, the "1/t" rule named as compatible with REWL: ln f halves while
 *           every walker visits every level, then follows 1/t.
 *   Sec. 3, statistical errors by the jackknife over the m pieces per window.
 *   Sec. 5, Eqs. (7)-(8): <E>, C_V from g(E).
 * Points the paper leaves open (window edges, RNG streams, warm-up,
 * flatness mask, merge order, exchange pairing, normalisation) are fixed
 * where each is implemented, and the comments there state the choice.
 *
 * Every function here is pinned by the tests against results that do not
 * come from this file: brute-force enumeration, exact densities of states
 * (transfer matrix, Kaufman's torus formula), closed forms, invariants and
 * planted mistakes.  One quantity has no exact reference: ln g of q >= 3
 * Potts beyond L = 6 (exact tables exist up to q = 3, L = 6), checked only
 * statistically (sum rule, exact low-energy counts) -- parity unpinned for
 * that quantity.
 *
 * Error convention: functions returning int give 0 on success and a negative
 * value on error; orc_new returns NULL on invalid parameters.
 */
#ifndef REWL_ORACLE_H
#define REWL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ISING = 0, ORC_POTTS = 1 };
enum { ORC_FP64 = 0, ORC_FP32C = 1 };

typedef struct {
  int32_t model;              /* ORC_ISING or ORC_POTTS */
  int32_t L;                  /* periodic L x L lattice, L >= 2 */
  int32_t q;                  /* Potts states (ignored for Ising) */
  int32_t n_windows;          /* h */
  int32_t overlap_num, overlap_den;   /* o = num/den */
  int32_t walkers_per_window; /* m */
  int32_t flat_num, flat_den; /* flatness p = num/den */
  double lnf_init, lnf_final;
  int64_t flips_per_exchange; /* F: attempts per walker per cycle */
  uint64_t seed;              /* Philox key */
  int32_t precision;          /* ORC_FP64 or ORC_FP32C */
  int32_t instance;           /* instance index folded into RNG counters */
  int32_t schedule;           /* ORC_HALVING (flatness + f -> sqrt f) or ORC_ONE_OVER_T */
  int32_t reserved;
} orc_params;

enum { ORC_HALVING = 0, ORC_ONE_OVER_T = 1 };

typedef struct {
  int32_t N, nbins, binw, emin, h, m, W;
  int32_t max_nb;             /* largest window, in bins */
} orc_info;

typedef struct orc_sim orc_sim;

/* Creation runs initialisation and warm-up.  win_lo/win_hi (both NULL or
 * both of length n_windows, global bin indices, inclusive) override the
 * equal-size window split. */
orc_sim* orc_new(const orc_params* p, const int32_t* win_lo, const int32_t* win_hi);
void orc_free(orc_sim* s);
int orc_get_info(const orc_sim* s, orc_info* out);
int orc_get_windows(const orc_sim* s, int32_t* lo, int32_t* hi);
int orc_warm_status(const orc_sim* s);   /* 0 all walkers inside, <0 a walker failed */

/* One cycle = sweeps (F attempts per walker), flatness/merge, exchange.
 * Returns number of cycles executed (stops early once every window froze). */
int64_t orc_run(orc_sim* s, int64_t max_cycles);
/* The three phases separately. */
int orc_sweep(orc_sim* s, int64_t flips);
int orc_merge(orc_sim* s);
int orc_exchange(orc_sim* s);

typedef struct {
  int32_t done;          /* every window frozen */
  int32_t pad;
  int64_t done_merge;    /* merge index (0-based) at which the last window froze, -1 */
  int64_t merges;        /* merge calls executed */
  uint64_t rounds;       /* exchange rounds executed */
} orc_status_t;
int orc_status(const orc_sim* s, orc_status_t* out);

/* Per-walker state.  Any pointer may be NULL.  lng64 gets ln g in FP64
 * (for FP32C it is hi + lo widened); spins length N, H/lng length nb_w. */
int orc_get_walker(const orc_sim* s, int32_t slot, int8_t* spins, int32_t* E,
                   uint32_t* H, double* lng64, uint64_t* attempts, int32_t* config_id);
/* Overwrite a walker's ln g (test hook; FP32C splits into hi + lo). */
int orc_set_walker_lng(orc_sim* s, int32_t slot, const double* lng64);
int orc_get_walker_f32(const orc_sim* s, int32_t slot, float* hi, float* lo);
/* Per-window state: U (visited union, length nb_w), stage completion merges
 * (length 64, -1 when not reached). */
int orc_get_window(const orc_sim* s, int32_t w, double* lnf, int32_t* stage,
                   int32_t* frozen, uint8_t* U, int64_t* stage_merge);
/* Per lower window w of a pair (w, w+1): proposals, proposals with both
 * energies inside the partner window, accepted swaps. */
/* Statistical errors of the joined, normalised ln g by the jackknife over
 * the m walkers of every window (Sec. 3): piece k of window w is the
 * average of the walkers' ln g captured just before the merge that froze the
 * window, leaving walker k out; the m leave-one-out joins give mean and
 * error per bin.  Needs every window frozen and m >= 2; -1 otherwise. */
int orc_jackknife(const orc_sim* s, double* mean, double* err);
/* Schedule phase of window w (0 halving, 1 ln f = 1/t), -1 on bad input. */
int orc_get_phase(const orc_sim* s, int32_t w);
/* ln g of walker `slot` captured before its window's freezing merge. */
int orc_get_piece(const orc_sim* s, int32_t slot, double* out);
int orc_get_exchange_stats(const orc_sim* s, uint64_t* tries, uint64_t* in_range, uint64_t* accepts);

/* Joined and normalised ln g over all nbins (-inf where no window visited);
 * joins receives the h-1 join bins (may be NULL). */
int orc_join(const orc_sim* s, double* out, int32_t* joins);
/* Joined, not normalised. */
int orc_join_raw(const orc_sim* s, double* out, int32_t* joins);

/* Stand-alone pieces, exposed so each can be pinned on its own. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_exp_spec(double x);          /* x in [-40, 0) */
float orc_expf_spec(float x);           /* x in [-17, 0) */
/* Exchange partners of round `round` between windows w and w+1 (Sec. 2):
 * pi (m entries) receives a uniform random permutation; walker k of window
 * w is paired with walker pi[k] of window w+1. */
int orc_exchange_pairing(uint64_t seed, int32_t instance, uint64_t round, int32_t w, int32_t m,
                         int32_t* pi);
int orc_accept64(uint64_t u53, double delta);
int orc_accept32(uint32_t u24, float delta);
int32_t orc_energy(int32_t model, int32_t L, int32_t q, const int8_t* spins);
int orc_equal_windows(int32_t nbins, int32_t h, int32_t on, int32_t od, int32_t* lo, int32_t* hi);
int orc_stitch(int32_t h, const int32_t* lo, const int32_t* hi,
               const double* const* l, const uint8_t* const* U,
               int32_t nbins, double* R, int32_t* joins);
int orc_normalise(int32_t model, int32_t N, int32_t q, int32_t nbins, double* R);
int orc_thermo(const double* lng, int32_t nbins, int32_t emin, int32_t binw,
               const double* T, int32_t nT, double* Emean, double* Cv);
/* Two-float helpers (FP32 compensated mode), exposed for pinning. */
void orc_df_add1(float ah, float al, float b, float* rh, float* rl);
void orc_df_add(float ah, float al, float bh, float bl, float* rh, float* rl);
void orc_df_div_int(float ah, float al, int32_t m, float* rh, float* rl);

#ifdef __cplusplus
}
#endif
#endif
