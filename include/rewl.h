/*
 * librewl -- replica-exchange Wang-Landau (REWL) sampling on one MI355X.
 *
 * Method: Li, Vogel, Wuest, Landau, "A new paradigm for petascale Monte Carlo
 * simulation: Replica exchange Wang-Landau sampling" (arXiv:1402.2328).
 *   Sec. 2  standard Wang-Landau: a trial move is accepted with
 *           min[1, g(E_old)/g(E_new)]; after every attempt g(E) -> f g(E) and
 *           H(E) += 1 at the current energy; when H is flat, H is reset and
 *           f -> sqrt(f); the run ends at f_final.
 *   Sec. 2  REWL: the energy range is split into h overlapping windows
 *           (Fig. 1a, overlap o); m walkers per window, each with its own g
 *           and H; every so many MC steps a walker swaps configurations with a
 *           random walker of a neighbouring window with probability Eq. (1),
 *           min[1, g_i(E(X))/g_i(E(Y)) * g_j(E(Y))/g_j(E(X))]; a pair with an
 *           energy outside the other's window is disregarded; when all m
 *           walkers of a window are flat their g are averaged and
 *           redistributed; each window has its own f; the run ends when every
 *           window reached f_final.
 *   Sec. 3  the h pieces are joined where the slopes d ln g/dE agree best
 *           (Eq. 2), using a 5-point derivative (Fig. 2).
 *   Sec. 5  Eqs. (7)-(8): <E> and C_V from g(E).
 *
 * Models: 2D Ising (E = -sum s_i s_j, s = +-1) and q-state Potts
 * (E = -sum delta(s_i, s_j)) on a periodic L x L lattice, single-site moves.
 * Energies are binned: bin b = (E - E_min)/binw with E_min = -2N, binw 4
 * (Ising), 2 (Potts q = 2) or 1 (Potts q >= 3).
 *
 * Conventions
 *   - Every function returns 0 (REWL_OK) or a negative REWL_E_* code and never
 *     throws.  rewl_strerror() names a code.
 *   - Device memory: the caller allocates one device buffer of
 *     rewl_workspace_bytes() bytes (any allocator, e.g. a torch tensor) and
 *     keeps it alive until rewl_destroy().  The library writes all simulation
 *     state into it and allocates no device memory of its own.  The library
 *     owns only the host-side context object.
 *   - Streams: run/merge/exchange/init calls only enqueue work on the
 *     hipStream_t given to rewl_init (a null pointer means the legacy default
 *     stream) and return without synchronising.  When a batch holds
 *     instances of more than one sweep kernel class, the sweeps of the other
 *     classes run on two streams the library owns, forked from that stream
 *     and joined back to it by events, so work enqueued on the caller's
 *     stream afterwards still sees finished sweeps.  rewl_status, rewl_get_*,
 *     rewl_thermo, rewl_checkpoint and rewl_restore synchronise that stream.
 *   - Calls on one context are not thread-safe.  Per cycle the call order is
 *     rewl_run_sweeps -> rewl_merge -> rewl_exchange.
 *   - A batch of n_instances independent REWL instances shares one context;
 *     instance i draws its random numbers from counters that carry i, so an
 *     instance gives bit-identical results alone or inside any batch.
 */
#ifndef REWL_H
#define REWL_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  REWL_OK = 0,
  REWL_E_INVAL = -1,     /* invalid argument or parameter set */
  REWL_E_NOMEM = -2,     /* workspace too small / host allocation failed */
  REWL_E_HIP = -3,       /* a HIP runtime call failed */
  REWL_E_NONFINITE = -4, /* a non-finite ln g value was found */
  REWL_E_OVERFLOW = -5,  /* a histogram counter reached 2^31 */
  REWL_E_STATE = -6,     /* call not valid in the current state */
  REWL_E_WARMUP = -7,    /* a walker could not be brought into its window */
  REWL_E_FORMAT = -8     /* checkpoint blob does not match this context */
};

enum { REWL_ISING = 0, REWL_POTTS = 1 };
enum { REWL_FP64 = 0, REWL_FP32C = 1 };
/* ln f schedules.  HALVING (Sec. 2): when all m walkers of a window are flat
 * their ln g are merged, H is reset and ln f halves.  ONE_OVER_T, the "1/t"
 * rule (Belardinelli and Pereyra) that Sec. 2 names as compatible with REWL:
 * phase A halves ln f, with the same merge, once every walker of the window
 * has visited every bin of the window's visited union; once halving would
 * bring ln f to or below 1/t, t = MC attempts per walker / visited bins, the
 * window switches to phase B, where every check sets ln f = 1/t and merges. */
enum { REWL_HALVING = 0, REWL_ONE_OVER_T = 1 };

/* One REWL instance.  All instances of one context must share `precision`. */
typedef struct {
  int32_t model;              /* REWL_ISING or REWL_POTTS */
  int32_t L;                  /* periodic L x L lattice, 2 <= L <= 64 */
  int32_t q;                  /* Potts states, 2..127 (ignored for Ising) */
  int32_t n_windows;          /* h >= 1 */
  int32_t overlap_num;        /* overlap o = num/den of the equal-size split */
  int32_t overlap_den;
  int32_t walkers_per_window; /* m >= 1 */
  int32_t flat_num;           /* flatness: min H >= (num/den) mean H */
  int32_t flat_den;
  int32_t precision;          /* REWL_FP64, or REWL_FP32C: two-float ln g */
  double lnf_init;            /* ln f_0 > 0 */
  double lnf_final;           /* window frozen once ln f <= lnf_final */
  int64_t flips_per_exchange; /* F: attempts per walker per cycle (informative) */
  uint64_t seed;              /* Philox4x32-10 key */
  int32_t schedule;           /* REWL_HALVING or REWL_ONE_OVER_T */
  int32_t reserved;           /* must be 0 */
} rewl_params;

typedef struct rewl_ctx rewl_ctx;

/* Device bytes needed for `n` instances.  win_lo/win_hi: NULL for the
 * equal-size split of every instance, or arrays concatenating, instance by
 * instance, n_windows inclusive global-bin edges (explicit windows, e.g. a
 * run-time balanced split, Fig. 1b).  Returns 0 for invalid input. */
size_t rewl_workspace_bytes(const rewl_params* params, int32_t n_instances,
                            const int32_t* win_lo, const int32_t* win_hi);

/* Builds the context, lays out the workspace and enqueues initialisation:
 * random spins, full energies, warm-up of every walker into its window
 * (greedy moves, restart from an extreme state), ln g = 0, H = 0,
 * ln f = lnf_init.  params: n_instances entries.  d_workspace: device
 * pointer to >= rewl_workspace_bytes() bytes.  stream: hipStream_t or NULL.
 * Errors: INVAL (bad parameters), NOMEM (workspace too small), HIP. */
int rewl_init(const rewl_params* params, int32_t n_instances,
              const int32_t* win_lo, const int32_t* win_hi,
              void* d_workspace, size_t workspace_bytes, void* stream, rewl_ctx** out);

/* Enqueues `flips` Wang-Landau attempts for every walker of every instance
 * that is not finished (Sec. 2).  Frozen windows keep moving without updating
 * ln g or H.  Errors: INVAL (flips < 0), HIP. */
int rewl_run_sweeps(rewl_ctx* ctx, int64_t flips);

/* Launch shape of the sweep.  Walkers are grouped by kernel class:
 * 0 = Ising L <= 32, 1 = Ising 32 < L <= 64, 2 = Potts.  For class cls (-1:
 * all classes) keep page_bins ln g bins of each walker's window in LDS (the
 * rest stays in device memory; the page follows the walker) and put
 * walkers_per_group walkers in each workgroup; 0 picks the default (the
 * largest page that lets four workgroups share a compute unit).  page_bins
 * is rounded up to a power of two, at least 16 (32 for a class with q >= 3
 * Potts instances) and at most the power of two that holds the class's
 * largest window.  rng_producer: 1 gives each workgroup a second
 * wavefront that computes the walkers' random numbers ahead of them (for
 * launches with few walkers, whose time is the walkers' serial chain), 0
 * none, -1 the default (a producer when the class has no more workgroups
 * than the GPU has compute units).  potts_nibbles (Potts class, every
 * q <= 16): 1 keeps spins in LDS as 4-bit nibbles (half the lattice, more
 * workgroups per compute unit) together with a table of every site's four
 * neighbours (8 bytes per site, shared by the workgroup: no row, column or
 * wrap arithmetic per attempt), 2 as nibbles without the table, 0 as bytes
 * (shorter chain per attempt), -1 the default (form 1 when the class has
 * more workgroups than compute units, else bytes); ignored where it does
 * not apply.  Results do not depend on the
 * shape, only speed does.  out: NULL
 * or 21 entries: per class {page_bins, walkers_per_group, LDS bytes per
 * workgroup, workgroups, rng_producer, potts_nibbles}, then the batch's
 * {fused, splits, order} (rewl_set_batching).  A fused batch whose classes
 * no longer share one rng_producer setting returns to per-class launches.
 * Synchronises.  Errors: INVAL (shape does not fit in LDS), HIP. */
int rewl_set_launch(rewl_ctx* ctx, int32_t cls, int32_t page_bins, int32_t walkers_per_group,
                    int32_t rng_producer, int32_t potts_nibbles, int32_t* out);

/* How a batch's sweep is launched.  fused = 0: one launch per kernel class,
 * classes side by side on forked streams; fused = 1: every class in one
 * launch (each workgroup runs the loop of its class, all in the LDS size
 * of the largest class; needs one rng_producer setting for all classes).
 * splits: a sweep of F attempts runs as that many consecutive launches
 * (1..64; the workgroups are placed afresh for each).  order (fused only):
 * order of the workgroups in the launch, i.e. which the hardware starts
 * first: 0 by class (Ising L <= 32, Ising L <= 64, Potts), 1 classes
 * reversed, 2 classes interleaved one workgroup at a time.  Results do not
 * depend on any of these.  out: as for rewl_set_launch.  Synchronises.
 * Errors: INVAL (out of range, or fused with differing producer
 * settings), HIP. */
int rewl_set_batching(rewl_ctx* ctx, int32_t fused, int32_t splits, int32_t order, int32_t* out);

/* Chooses the launch shape of every class and the batching
 * (rewl_set_batching) by timing sweeps of `flips` attempts (median of
 * `repeats` sweeps per candidate) on the whole batch: classes sweep side by
 * side and share the compute units, so a candidate replaces the best plan
 * only when the batch is faster with it.  Candidates are first one page
 * size for all classes (with and without the RNG producer, Potts spins as
 * bytes or nibbles, with or without the neighbour table; for batches of
 * several classes both per-class launches
 * and the fused launch in each workgroup order), then, in two passes over
 * the classes, every shape of one class with the others at their best so
 * far, then on the best shapes the sweep in 1, 2 or 4 launches and the
 * other batching forms.  The five best plans (with the best per-class and
 * the best fused plan when none of the five has that form) are then timed
 * as a run uses them: `repeats` whole cycles (sweep, merge, exchange)
 * queued back to back from the saved state, interleaved four times, and
 * the plan with the lowest mean plus standard deviation of its cycle times
 * is kept (a plan whose time swings with the placement of concurrent
 * kernels pays for the swings).
 * The plan in force before the call is the first candidate.
 * The simulation state is saved to host memory first and restored
 * afterwards, so tuning changes nothing but the launch shape.  out: as for
 * rewl_set_launch.  Synchronises.
 * Errors: INVAL, HIP. */
int rewl_autotune(rewl_ctx* ctx, int64_t flips, int32_t repeats, int32_t* out);

/* Enqueues the flatness test and in-window merge for every non-frozen window
 * (Sec. 2): when all m walkers of a window are flat at this check, their ln g
 * are averaged (pairwise sum in walker order, divided by m), H is reset and
 * ln f halves; the window freezes once ln f <= lnf_final.  Under the 1/t
 * schedule the readiness test and the new ln f follow REWL_ONE_OVER_T.  The
 * walkers' ln g just before the merge that freezes a window are kept as the
 * window's m pieces (rewl_get_piece, rewl_jackknife).  An instance whose
 * windows are all frozen is finished.  Errors: HIP. */
int rewl_merge(rewl_ctx* ctx);

/* Enqueues one replica-exchange round (Eq. 1) for every unfinished instance:
 * round t pairs windows (w, w+1) with w = t mod 2; walker k of window w is
 * paired with walker pi(k) of window w+1, pi uniform; configurations are
 * swapped by exchanging configuration indices.  Errors: HIP. */
int rewl_exchange(rewl_ctx* ctx);

/* Enqueues `cycles` x (run_sweeps(flips) -> merge -> exchange).  With
 * use_graph != 0 the sequence is captured once into a hipGraph and replayed.
 * Errors: INVAL, HIP. */
int rewl_run_cycles(rewl_ctx* ctx, int64_t cycles, int64_t flips, int32_t use_graph);

typedef struct {
  int32_t done;          /* every window frozen */
  int32_t error;         /* 0 or a REWL_E_* code raised on the device */
  int64_t done_merge;    /* merge index at which the last window froze, -1 */
  int64_t merges;        /* merge calls executed while unfinished */
  uint64_t rounds;       /* exchange rounds executed */
  uint64_t attempts;     /* MC attempts summed over the instance's walkers */
} rewl_instance_status;

/* Synchronises.  out: one entry.  stage_per_window / frozen_per_window /
 * lnf_per_window: NULL or n_windows entries. */
int rewl_status(rewl_ctx* ctx, int32_t instance, rewl_instance_status* out,
                int32_t* stage_per_window, int32_t* frozen_per_window, double* lnf_per_window);

/* Synchronises.  Number of instances neither finished nor failed. */
int rewl_running(rewl_ctx* ctx, int32_t* n_running);

/* Synchronises.  which = 0: ln g joined over all windows (Sec. 3, Eq. 2) in
 * FP64 and normalised (Ising: sum g = 2^N; Potts: g(E_min) = q); which = 1:
 * joined, not normalised.  host_out: capacity doubles, receives nbins values
 * (-inf where no walker of the supplying window visited); joins: NULL or
 * n_windows-1 join bins.  Errors: INVAL (capacity too small), HIP. */
int rewl_get_lng(rewl_ctx* ctx, int32_t instance, int32_t which, double* host_out,
                 int32_t capacity, int32_t* n_bins_out, int32_t* joins);

/* Synchronises.  Geometry of an instance: N, nbins, binw, E_min, h, m, first
 * global walker slot, and the window edges (NULL allowed). */
int rewl_get_geometry(rewl_ctx* ctx, int32_t instance, int32_t* N, int32_t* nbins,
                      int32_t* binw, int32_t* emin, int32_t* h, int32_t* m,
                      int32_t* first_slot, int32_t* win_lo, int32_t* win_hi);

/* Synchronises.  State of one walker (instance-local slot = w*m + k): the
 * spins of the configuration it carries (N int8), its energy, H and ln g over
 * its window (FP64; FP32C gives hi + lo widened), its attempt counter and
 * the identity (index) of the configuration.  Any pointer may be NULL. */
int rewl_get_walker(rewl_ctx* ctx, int32_t instance, int32_t slot, int8_t* spins,
                    int32_t* energy, uint32_t* H, double* lng, uint64_t* attempts,
                    int32_t* config_id);
/* Host only.  Where a walker's state sits in the workspace (byte offsets
 * from its start): its energy (one int32), its histogram row (n_bins uint32)
 * and its ln g row (n_bins FP64, or for FP32C the n_bins floats of the high
 * parts).  For inspection tools and tests that inject faults (a non-finite
 * ln g, a histogram near 2^31, an energy outside the window); the layout is
 * otherwise private.  Any pointer may be NULL.  Errors: INVAL. */
int rewl_locate_walker(rewl_ctx* ctx, int32_t instance, int32_t slot, size_t* energy_off,
                       size_t* H_off, size_t* lng_off, int32_t* n_bins);
/* FP32C only: the two-float parts of a walker's ln g. */
int rewl_get_walker_f32(rewl_ctx* ctx, int32_t instance, int32_t slot, float* hi, float* lo);
/* Synchronises.  Visited-union mask of a window (nb_w bytes). */
int rewl_get_visited(rewl_ctx* ctx, int32_t instance, int32_t window, uint8_t* mask);
/* Synchronises.  Per lower window w of pair (w, w+1): proposals, proposals
 * with both energies inside the partner window, accepted swaps (h entries). */
int rewl_get_exchange_stats(rewl_ctx* ctx, int32_t instance, uint64_t* tries,
                            uint64_t* in_range, uint64_t* accepts);

/* Synchronises.  phase: NULL or n_windows entries (0 = halving phase, 1 =
 * ln f = 1/t phase); stage_merge: NULL or n_windows * 64 entries, entry
 * w * 64 + s = merge index at which window w finished WL iteration s (-1 if
 * not yet).  Errors: INVAL, HIP. */
int rewl_get_schedule(rewl_ctx* ctx, int32_t instance, int32_t* phase, int64_t* stage_merge);

/* Synchronises.  ln g (FP64; FP32C hi + lo widened) of walker `slot`
 * (w*m + k) just before the merge that froze its window: nb_w doubles, zero
 * while the window is not frozen.  Errors: INVAL, HIP. */
int rewl_get_piece(rewl_ctx* ctx, int32_t instance, int32_t slot, double* host_lng);

/* Synchronises.  Jackknife error bars of the joined, normalised ln g over
 * the m pieces per window (Sec. 3): for k = 0..m-1 each window's
 * representative is the mean of its pieces without walker k (pairwise sum in
 * walker order, divided by m-1); the h representatives are joined and
 * normalised as in rewl_get_lng, giving R_k.  Per bin: mean = sum R_k / m,
 * err = sqrt((m-1)/m * sum (R_k - mean)^2); where any R_k is -inf, mean =
 * -inf and err = 0.  The pieces of a window share everything up to its last
 * merge, so these errors see only the spread since then and can be far
 * below the true error (halving, Ising L = 8: about 7e-4 against 0.18;
 * 1/t to ln f = 1e-7 with m = 64, Ising L = 32: a median of 3e-6 per bin
 * against a spread of 2e-3 between instances); error bars must come from
 * independent instances (a batch).  mean, err: capacity doubles each,
 * nbins used.  Errors: INVAL (capacity), STATE (instance not
 * finished, or m < 2), HIP. */
int rewl_jackknife(rewl_ctx* ctx, int32_t instance, double* host_mean, double* host_err,
                   int32_t capacity, int32_t* n_bins_out);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid it): rewl_jackknife with the
 * same arguments, results and errors, whose leave-one-out rows and window
 * representatives live in a device array of the library instead of the
 * workspace.  It calls no allocator.  Limit: the instance's
 * (m + 2) * nbins + (sum of its window sizes, rounded up to 32) doubles
 * must fit in 2^19 doubles (4 MiB), else NOMEM (every Ising instance,
 * and Potts up to L = 60, fits for any m <= 64).  Every GPU holds one such array for the life of the
 * process and every call on that GPU uses it (it keeps the last call's
 * contents, which no call reads), so calls that overlap on one GPU, from
 * any context or thread, race. */
int rewl_jackknife_noalloc(rewl_ctx* ctx, int32_t instance, double* host_mean, double* host_err,
                           int32_t capacity, int32_t* n_bins_out);

/* Synchronises.  Canonical <E> and C_V (Sec. 5, Eqs. 7-8, k_B = 1) from the joined,
 * normalised ln g of an instance, evaluated on the GPU in FP64 for nT
 * temperatures.  Errors: INVAL, HIP. */
int rewl_thermo(rewl_ctx* ctx, int32_t instance, const double* T, int32_t nT,
                double* E_mean, double* C_v);

/* Synchronises.  Serialises the whole simulation state into host_buf
 * (capacity cap bytes); *used receives the size (call with host_buf = NULL
 * to query).  rewl_restore loads such a blob into a context built with the
 * same parameters; a restored run continues bit-identically.  Errors: NOMEM
 * (cap too small), FORMAT (blob from another configuration), HIP. */
int rewl_checkpoint(rewl_ctx* ctx, void* host_buf, size_t cap, size_t* used);
int rewl_restore(rewl_ctx* ctx, const void* host_buf, size_t n);

/* Host only (no device, no context).  Run-time balanced split (Fig. 1b):
 * h window edges over bins 0..nbins-1 such that every window should finish
 * its first WL iteration after about the same number of MC steps, from a
 * pre-run with pre_h windows [pre_lo[v], pre_hi[v]] whose first iteration
 * took pre_steps[v] MC steps per walker (e.g. (stage_merge[v][0] + 1) x
 * flips_per_exchange from rewl_get_schedule, averaged over instances).
 * Model: a window that took S steps has cost width S^(1/alpha) (alpha = 2
 * for a diffusive walk), spread evenly over its bins; a bin's cost density
 * is the mean over the pre-run windows containing it; the new windows are
 * the equal split with overlap num/den done in the cumulative-cost
 * coordinate of the bin centres, edges at the nearest bin centre (ties to
 * the higher bin); then every window is widened to >= 5 bins and every
 * neighbour overlap to >= 5 bins, keeping edges strictly increasing.
 * lo, hi: h entries each, usable as win_lo / win_hi of rewl_init.
 * Errors: INVAL (bad input, a bin no pre-run window covers, or h too large
 * for nbins). */
int rewl_balanced_windows(int32_t nbins, int32_t h, int32_t overlap_num, int32_t overlap_den,
                          int32_t pre_h, const int32_t* pre_lo, const int32_t* pre_hi,
                          const double* pre_steps, double alpha, int32_t* lo, int32_t* hi);

/* Frees the host context (the caller frees the workspace). */
int rewl_destroy(rewl_ctx* ctx);

const char* rewl_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
