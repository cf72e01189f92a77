/*
 * hfqmc.h -- C ABI of the MI355X (gfx950) Hirsch-Fye QMC impurity engine.
 *
 * What it solves.  Real-space DMFT for the trapped Hubbard model (Bluemer &
 * Gorelik, arXiv:1006.2716, Eq. (1)) maps the lattice, through the local
 * self-energy assumption stated after Eq. (2), onto one Anderson impurity
 * problem per inequivalent site.  Each impurity is given by its Weiss function
 * G0_sigma(tau) and is solved with the Hirsch-Fye QMC algorithm that the
 * paper's "Model and Methods" paragraph names, on L = beta/dtau imaginary-time
 * slices; the impurity solves are independent, which the paper's parallel
 * strategy paragraph (after Eq. (2)) exploits by solving all of them at once.
 * This library runs those solves batched on one GPU.
 *
 * Conventions (the paper states none of them; these are the library's):
 *   - g(tau) = <T c(tau) c^dag(0)> > 0; G[l][l] = g(0+) = 1 - n.
 *   - Weiss input: L samples g(tau_k), tau_k = k*beta/L, k = 0..L-1, k = 0 is
 *     tau = 0+.  The L x L matrix is G0[i][j] = g(tau_{i-j}) (i >= j) and
 *     -g(tau_{i-j+L}) (i < j).  Inputs are expected to be Hartree shifted
 *     (one-body level includes +U/2), as the HS decoupling requires.
 *   - lambda: cosh(lambda) = exp(dtau U / 2); V_sigma,l = sigma lambda s_l,
 *     sigma = +1 (up, index 0), -1 (down, index 1).
 *   - Metropolis acceptance u < R_up R_dn with u from Philox4x64-10 keyed by
 *     (seed, site_id); slice l of sweep w uses word (l >> 6) of the block at
 *     counter (l & 63, w + sweep_offset, 2, 0); u = (x >> 11) 2^-53.  Drawn
 *     initial fields use the top bit of word (l >> 6) at counter (l & 63, 0, 1, 0)
 *     (0 -> +1).  Counter word 3 is the chain index (0 for a single chain).
 *     Results therefore depend only on the problem, never on the batch it
 *     runs in.
 *   - The Dyson equation G = [1 + (1 - G0)(e^V - 1)]^{-1} G0 is solved from
 *     scratch at the start and after every `recompute_every` sweeps; measured
 *     sweeps (after n_warmup) contribute g_sigma(tau_k) (k = 0..L, with
 *     g(tau_L) = n_sigma), n_sigma and d = <n_up n_dn> to n_bins consecutive
 *     bins (measured sweep m goes to bin floor(m n_bins / n_measure)).
 *   - Checkpoints: a chain's whole state between sweeps is its fields and
 *     its sweep count w.  A run given init_fields = the final fields of a
 *     run of w sweeps and sweep_offset = w (plus that run's own offset)
 *     continues that chain with the same random numbers; when w is a multiple of recompute_every (and no drift
 *     over the limit shortened the interval) both rebuild G from scratch at
 *     sweep w and the continuation is bit-exact.
 *
 * Memory ownership.  The caller owns every host buffer and ALL device memory:
 * the workspace of hfqmc_solve and the pool of the site/serving calls are
 * caller allocations passed as raw device pointers.  The library allocates
 * only small pinned host staging buffers inside its context.  Inputs are
 * copied during the call; outputs are written before the call returns (or,
 * for hfqmc_poll, when it returns HFQMC_OK).
 *
 * Errors.  Every call returns an hfqmc_status; no C++ exception crosses the
 * ABI.  HFQMC_EINVAL: invalid argument, nothing changed.  HFQMC_ENOMEM:
 * workspace or pool too small.  HFQMC_EDEVICE: a HIP call failed, the context
 * must be destroyed.  HFQMC_EAGAIN: not admissible now / not finished yet.
 * HFQMC_ENUMERIC: a non-finite ratio or Green function was seen.
 * HFQMC_ENOTFOUND: unknown ticket or site.  hfqmc_last_error() describes the
 * most recent failure on the calling thread.
 */
#ifndef HFQMC_H
#define HFQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HFQMC_OK = 0,
    HFQMC_EINVAL = -1,
    HFQMC_ENOMEM = -2,
    HFQMC_EDEVICE = -3,
    HFQMC_EAGAIN = -4,
    HFQMC_ENUMERIC = -5,
    HFQMC_ENOTFOUND = -6
} hfqmc_status;

/* FP64: everything in fp64.  MIXED: the rank-k products of the window or
 * delayed updates in fp32, added into the fp64 G; ratios, the decisions of a
 * window and the Dyson recompute stay fp64.  Classes with no fp32-product
 * kernel (the window kernel at 128 slices, G in device memory) run fp64. */
typedef enum { HFQMC_FP64 = 0, HFQMC_MIXED = 1 } hfqmc_precision;

typedef struct hfqmc_ctx hfqmc_ctx;   /* opaque; one per device and stream */
typedef struct hfqmc_site hfqmc_site; /* opaque device-resident impurity state */

/* One impurity problem.  1 <= L <= 160, beta > 0, U >= 0, n_bins >= 2,
 * n_measure >= n_bins per chain, recompute_every >= 1, Weiss samples finite
 * with g(0+) in (0, 1). */
typedef struct {
    int32_t L;
    double beta;
    double U;
    const double *weiss[2];     /* host: [0] up, [1] down, L samples each */
    int64_t n_warmup;
    int64_t n_measure;
    int32_t recompute_every;    /* sweeps between from-scratch Dyson solves */
    int32_t n_bins;
    uint64_t seed;              /* Philox key word 0 */
    uint64_t site_id;           /* Philox key word 1 */
    int64_t sweep_offset;       /* added to the sweep index in the Philox counter */
    const int8_t *init_fields;  /* host, L entries (+1/-1), or NULL to draw them */
    int32_t delay;              /* 0: library choice (the autotuned shape -- rank-one,
                                   delayed or window updates -- else the untuned
                                   default for L);
                                   1: rank-one Sherman-Morrison updates;
                                   2..32: delayed rank-k updates, flushed into G
                                   every k accepted flips (fp32 products when
                                   the context precision is HFQMC_MIXED).
                                   L > 128 keeps G in device memory, fp64 in
                                   either precision: delay 0 runs window
                                   updates where that kernel is compiled
                                   (padded L 144 and 160), else delayed updates
                                   of depth 16; 1..16 delayed updates of that
                                   depth; more is EINVAL */
    int32_t n_chains;           /* independent Markov chains for this impurity
                                   (0 or 1: one).  Chain j draws with Philox
                                   counter word 3 = j, runs the full warm-up and
                                   n_measure / n_chains measured sweeps (the first
                                   n_measure % n_chains chains one more); bin b of
                                   the result pools all chains' bin b.  At most
                                   64; n_measure >= n_chains * n_bins. */
} hfqmc_problem;

/* Result of one impurity.  Pointer members are caller-owned and may be NULL. */
typedef struct {
    double *g[2];               /* L+1 bin-averaged g_sigma(tau_k), k = 0..L */
    double *g_err[2];           /* L+1 errors std(bins)/sqrt(n_bins) */
    double *bins;               /* n_bins x (2(L+1)+3) bin means:
                                   g_up[0..L], g_dn[0..L], n_up, n_dn, d */
    int8_t *final_fields;       /* L entries: fields after the last sweep */
    double n[2], n_err[2];
    double docc, docc_err;
    double accept_rate;
    double max_drift;           /* max |G_updated - G_from_scratch| seen */
    int64_t proposals;          /* attempted single-field flips, warm-up included */
    int64_t accepts;
    int64_t nonpositive;        /* proposals rejected because R <= 0 */
    int32_t status;             /* hfqmc_status of this impurity */
    int32_t recoveries;         /* sweeps repeated after a ratio that was not a
                                   positive number (see numeric recovery below) */
} hfqmc_result;

/* lambda from cosh(lambda) = exp(dtau U / 2) (paper: HF discretisation of
 * the interval 0 <= tau <= 1/T, "Model and Methods").  EINVAL unless dtau > 0
 * and U >= 0. */
hfqmc_status hfqmc_lambda(double dtau, double U, double *lambda_out);

/* Create a context on HIP device `device` that launches on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `tune_cache` may be NULL or a
 * path to a JSON autotune cache.  *out is owned by the caller until
 * hfqmc_destroy. */
hfqmc_status hfqmc_create(int device, void *hip_stream, hfqmc_precision precision, const char *tune_cache,
                          hfqmc_ctx **out);
void hfqmc_destroy(hfqmc_ctx *ctx);
const char *hfqmc_last_error(const hfqmc_ctx *ctx);

/* Bytes of device workspace hfqmc_solve needs for these n problems. */
hfqmc_status hfqmc_workspace_size(hfqmc_ctx *ctx, const hfqmc_problem *problems, int32_t n, size_t *bytes);

/* Solve n independent impurity problems in one batch (blocking).
 * d_ws: caller-owned device memory of ws_bytes >= hfqmc_workspace_size.
 * out: n caller-owned results.  Equivalent to stage + run + collect.  n = 0
 * is an empty batch: HFQMC_OK, nothing run (problems, d_ws, out may be NULL);
 * n < 0 is HFQMC_EINVAL. */
hfqmc_status hfqmc_solve(hfqmc_ctx *ctx, const hfqmc_problem *problems, int32_t n, void *d_ws, size_t ws_bytes,
                         hfqmc_result *out);

/* ---- numeric recovery and drift control ----
 * Every Metropolis sweep checks its ratios R = R_up R_dn (Eq. (1)); in exact
 * arithmetic they are positive.  A sweep that meets one that is not a
 * positive number (R <= 0, NaN, a non-finite G) is undone -- fields,
 * counters -- and repeated once from a from-scratch fp64 Dyson solve
 * (Eq. (2)) of its starting fields; the result's `recoveries` counts these.
 * If the repeat fails too, the impurity's status is HFQMC_ENUMERIC.  A
 * recovered sweep takes the decisions of an undisturbed one, so results
 * agree with a run that never failed up to rounding.
 *
 * Drift limit (per context; HFQMC_FP64 default 0 = off, HFQMC_MIXED default
 * 1e-3): a scheduled from-scratch recompute that finds max |G_updated -
 * G_recomputed| over the diagonal 16 x 16 blocks above the limit halves the
 * interval to the next recompute (kept across the launches of a chain); if
 * the interval is already 1 sweep, the impurity ends HFQMC_ENUMERIC.  EINVAL
 * unless 0 <= limit < inf.  Applies to problems staged afterwards. */
hfqmc_status hfqmc_set_drift_limit(hfqmc_ctx *ctx, double limit);

/* Test hook for the numeric recovery: the Metropolis ratios of sweep
 * `sweep_a` (first attempt) and of the repeated attempt of sweep `sweep_b`
 * are formed from a NaN-poisoned copy of G's diagonal (blocks), as a
 * non-finite G would give; -1 disables either.  Global sweep indices
 * (warm-up included) of every chain of problems staged afterwards. */
hfqmc_status hfqmc_debug_poison(hfqmc_ctx *ctx, int64_t sweep_a, int64_t sweep_b);

/* Bytes of the library's own device array used by hfqmc_solve_static. */
#define HFQMC_STATIC_BYTES ((size_t)64 << 20)

/* hfqmc_solve on the library's own device array of HFQMC_STATIC_BYTES per
 * device instead of a caller workspace.  For callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc): it allocates and creates nothing (the context's events
 * exist from hfqmc_create; the kernel classes run one after another on the
 * context stream, not forked onto auxiliary streams).  HFQMC_EINVAL, with nothing run,
 * if hfqmc_workspace_size of the batch exceeds HFQMC_STATIC_BYTES (at L = 64
 * about 390 impurities fit).  Every call on a device uses the same array, so
 * calls that overlap on one device (from several contexts or threads) race;
 * a call leaves the array holding its batch, and the next call restages
 * every input and clears every accumulator it reads.  Results, and the
 * empty batch, as hfqmc_solve. */
hfqmc_status hfqmc_solve_static(hfqmc_ctx *ctx, const hfqmc_problem *problems, int32_t n, hfqmc_result *out);

/* Split form of hfqmc_solve.  stage: validate, plan, copy inputs to d_ws
 * (blocking).  run: enqueue the whole device pass (field initialisation,
 * Dyson, sweeps, measurement) on the context stream, asynchronous; may be
 * called repeatedly -- every call recomputes the same deterministic result
 * from the staged inputs.  collect: wait, copy bins/status back, finalise
 * results (bin means and errors).  The staged d_ws must stay valid between
 * the three calls.  stage needs n >= 1 (HFQMC_EINVAL otherwise). */
hfqmc_status hfqmc_stage(hfqmc_ctx *ctx, const hfqmc_problem *problems, int32_t n, void *d_ws, size_t ws_bytes);
hfqmc_status hfqmc_run(hfqmc_ctx *ctx);
hfqmc_status hfqmc_collect(hfqmc_ctx *ctx, hfqmc_result *out);

/* Same pass as hfqmc_run, replayed from a hipGraph captured on the first
 * call after each hfqmc_stage (kernel classes are graph branches that run
 * concurrently; the pass contains no memset and no host copy).  Results are
 * identical to hfqmc_run. */
hfqmc_status hfqmc_run_graph(hfqmc_ctx *ctx);

/* Device time in milliseconds of the whole last pass (hfqmc_run or
 * hfqmc_run_graph), from HIP events recorded on the context stream around
 * it; *n_launches receives the number of kernel classes. */
hfqmc_status hfqmc_last_run_ms(hfqmc_ctx *ctx, double *sweep_ms, int32_t *n_launches);

/* Duration of class kernel i of the last eager hfqmc_run, from HIP events
 * recorded on the stream it ran on, with its padded slice count and item
 * count (pointers may be NULL).  Classes run largest L first, concurrently
 * on up to four streams. */
hfqmc_status hfqmc_last_launch_ms(hfqmc_ctx *ctx, int32_t i, double *ms, int32_t *L_padded, int32_t *n_items);

/* ---- autotuning (kernel shape per padded slice count) ----
 * For every padded L present in `problems`, time each compiled kernel shape
 * (tile-rows per wave; window updates (k = 0: the decisions of 16 slices
 * taken on the 16 x 16 diagonal blocks of G, then one rank-|accepted|
 * matrix-core update of G), rank-one, or delayed with k in {4, 8, 16, 32};
 * fp32 products in the context precision HFQMC_MIXED) on those problems
 * shortened to `sweeps` (>= 4) and to 2 `sweeps` sweeps, the rate taken
 * from the difference of the two times (so per-launch costs do not count);
 * every timing run holds the whole shortened batch, the other classes in
 * their current shapes, so a shape is timed beside the classes it shares
 * the GPU with.  Keep the fastest unless the class's untuned default comes
 * within 5 % of it, and write the table to the context's tune cache (JSON,
 * if a path was given to hfqmc_create).  Problems with delay 0 then use the
 * tuned shape.  d_ws must hold hfqmc_workspace_size(problems); any staged
 * batch is discarded (stage again). */
hfqmc_status hfqmc_tune(hfqmc_ctx *ctx, const hfqmc_problem *problems, int32_t n, void *d_ws, size_t ws_bytes,
                        int32_t sweeps);
/* The shape a problem with L slices and this delay would run with:
 * tile-rows per wave, delay depth (1 = rank-one, 0 = window updates) and the tuned rate in
 * proposals/s (0 if untuned).  Pointers may be NULL. */
hfqmc_status hfqmc_plan(hfqmc_ctx *ctx, int32_t L, int32_t delay, int32_t *rt, int32_t *k, double *tuned_rate);

/* ---- device-resident sites (state kept across DMFT iterations) ---- */

/* Give the context caller-owned device memory for site state and serving. */
hfqmc_status hfqmc_attach_pool(hfqmc_ctx *ctx, void *d_pool, size_t bytes);
/* Bytes of pool one site of L slices and n_chains chains (0 or 1: one)
 * occupies (per chain: fields, G, bins, Weiss). */
hfqmc_status hfqmc_site_bytes(int32_t L, int32_t n_bins, int32_t n_chains, size_t *bytes);
/* Open a site; its problems must have this L, n_bins and n_chains.  The test
 * hooks below act on chain 0. */
hfqmc_status hfqmc_site_open(hfqmc_ctx *ctx, int32_t L, int32_t n_bins, int32_t n_chains, hfqmc_site **out);
hfqmc_status hfqmc_site_close(hfqmc_ctx *ctx, hfqmc_site *site);
/* Upload the problem (Weiss, U, beta, seeds) without sweeping. */
hfqmc_status hfqmc_site_define(hfqmc_ctx *ctx, hfqmc_site *site, const hfqmc_problem *problem);

/* Deterministic test hooks (blocking).  set_fields: fields (L x +-1) and a
 * fresh Dyson solve, on every chain of the site.  The others act on chain 0.
 * force_flips: flip the listed slices in order, each
 * accepted unconditionally via Sherman-Morrison; ratios (n, may be NULL)
 * receive R_up R_dn of each flip.  get_green: G_spin as L x L row-major.
 * recompute: fresh Dyson solve; *drift (may be NULL) receives
 * max |G_before - G_after|. */
hfqmc_status hfqmc_site_set_fields(hfqmc_ctx *ctx, hfqmc_site *site, const int8_t *fields);
hfqmc_status hfqmc_site_force_flips(hfqmc_ctx *ctx, hfqmc_site *site, const int32_t *slices, int32_t n,
                                    double *ratios);
hfqmc_status hfqmc_site_get_green(hfqmc_ctx *ctx, hfqmc_site *site, int32_t spin, double *LxL_row_major);
hfqmc_status hfqmc_site_get_fields(hfqmc_ctx *ctx, hfqmc_site *site, int8_t *fields);
hfqmc_status hfqmc_site_recompute(hfqmc_ctx *ctx, hfqmc_site *site, double *drift);

/* ---- serving: continuous batching of impurity solves on sites ----
 * A library thread admits submitted requests while the CU shares of the
 * admitted ones (n_chains / resident workgroups per CU of the site's kernel)
 * fit the capacity, and advances all admitted requests together in steps: a
 * step launches every chain of every admitted request once (one workgroup
 * per chain), each kernel class on its own
 * stream (classes run concurrently), with a per-class sweep count sized from
 * the class's time per proposal (a cost model of the kernel shape, measured
 * on MI355X) so that the step takes about `step_ms`.  Requests that arrive
 * while a step runs join the next step.
 * Field and G state stay on the device: a request without init_fields on a
 * site that already ran starts from the site's last fields with a fresh
 * Dyson solve (the next DMFT iteration), otherwise from init_fields or drawn
 * fields.  A request's result is bitwise the result of hfqmc_solve on the
 * same problem with delay 0, whatever else runs beside it and however it is
 * split into steps: a site runs the kernel shape its L had (tuned or
 * default) when it was opened, whatever the request's delay field.  The
 * site must not be used by the test hooks while it has a request (EAGAIN). */

/* step_ms > 0 (default 8) sets the target step duration; quantum_proposals
 * > 0 instead fixes the proposals per request per step (0: timed steps);
 * capacity_cus > 0 sets the admission capacity in CUs (0: all CUs). */
hfqmc_status hfqmc_serve_config(hfqmc_ctx *ctx, double step_ms, int64_t quantum_proposals, double capacity_cus);
/* Queue a request on a site (problem L, n_bins and n_chains must match the
 * site's).
 * Inputs are copied before the call returns.  EAGAIN: the site has a
 * request in progress, or the queue is full.  *ticket identifies it. */
hfqmc_status hfqmc_submit(hfqmc_ctx *ctx, hfqmc_site *site, const hfqmc_problem *problem, uint64_t *ticket);
/* EAGAIN while the request runs; OK (or its error status) once done, with
 * `out` filled like hfqmc_collect does; the ticket is then released.
 * ENOTFOUND: unknown, released or cancelled ticket. */
hfqmc_status hfqmc_poll(hfqmc_ctx *ctx, uint64_t ticket, hfqmc_result *out);
/* Drop a request (queued: at once; running: when its launch ends).  The
 * site keeps the fields of its last completed launch. */
hfqmc_status hfqmc_cancel(hfqmc_ctx *ctx, uint64_t ticket);

typedef struct {
    int64_t submitted, completed, cancelled, launches, steps;
    int32_t pending;        /* queued, not admitted */
    int32_t active;         /* admitted, waiting for or in a launch */
    double capacity_used;   /* CU shares held by admitted requests */
    double capacity;
    double step_ms_avg;     /* wall time of a step, launch to retirement */
    double launch_ms_avg;   /* device time of one class launch (HIP events) */
} hfqmc_serve_stats_t;
hfqmc_status hfqmc_serve_stats(hfqmc_ctx *ctx, hfqmc_serve_stats_t *out);

/* ---- dtau -> 0: removal of the discretisation error ----
 * The discretised problem's observables are even in dtau (the paper removes
 * the Trotter error by extrapolating dtau -> 0; see the sentence on the
 * discretisation after Eq. (2)).  Weighted least-squares fit of
 * value_i = sum_k coef_k dtau_i^(2k), k = 0 .. order (0 <= order <= 3), over
 * n >= order + 1 runs (host arrays), weights 1 / err_i^2 (err may be NULL:
 * unweighted).  coef_0 is the dtau -> 0 estimate.  coef_err (may be NULL)
 * receives sqrt of the diagonal of (A^T W A)^-1, NaN without err.  Pure host
 * arithmetic (Householder QR); EINVAL for dtau <= 0, non-finite input or too
 * few distinct dtau. */
hfqmc_status hfqmc_extrapolate(int32_t n, const double *dtau, const double *value, const double *err, int32_t order,
                               double *coef, double *coef_err);

/* ---- entropy from dS/dmu = dN/dT ----
 * Sampling gives no entropy directly; the paper integrates the temperature
 * derivative of the densities over the chemical potential from the empty
 * system (mu -> -inf, S = 0): see the entropy discussion after the
 * magnetization results.  For every site i (host arrays, [k][i] layout):
 * dn_i/dT at mu_k = (n_hi - n_lo) / (T_hi - T_lo) (central difference, for
 * T = (T_lo + T_hi) / 2) and s[k][i] = trapezoid integral of it over
 * mu_0 .. mu_k, the lowest grid point taken as empty (s = 0).  mu strictly
 * ascending, n_mu >= 2, 0 < T_lo < T_hi.  Pure host arithmetic. */
hfqmc_status hfqmc_entropy(int32_t n_mu, int32_t n_sites, const double *mu, const double *n_lo, const double *n_hi,
                           double T_lo, double T_hi, double *s);

/* ---- real-space DMFT self-consistency around the solver ----
 * The lattice Dyson equation, Eq. (2) (site-diagonal self-energy, one inverse
 * per Matsubara frequency and spin), the impurity Dyson equation linking the
 * local Green function, self-energy and Weiss function of each site, and the
 * transforms between Matsubara frequencies w_n = (2n + 1) pi / beta
 * (n < n_freq) and the solver's time slices.
 *
 * Conventions.  Spin s = 0 (up), 1 (down).  The one-body matrix of spin s is
 * hop + diag(eps_s): hop real symmetric (hopping amplitudes; the paper's
 * t_ij enters with the opposite sign), eps_s the site energies (trap
 * potential, seed fields).  mu is the chemical potential of the
 * Hartree-shifted levels the solver takes (mu - U/2 in the paper's
 * notation) and sigma the self-energy relative to them (Sigma - U/2), so that
 * sigma = 0 gives the U = 0 lattice.  Complex arrays are interleaved (re, im)
 * doubles; a "spin-frequency-site" array holds element (s, n, i) at
 * (s * n_freq + n) * n_sites + i.  Every array argument named d_* is device
 * memory owned by the caller; all calls are asynchronous on the context's
 * stream and allocate no device memory.
 *
 * Lattice structure.  Sites are numbered layer by layer (n_sites = n_layers x
 * layer, 1 <= layer <= 64); hop may couple sites inside a layer arbitrarily,
 * and site j of layer k only with site j of layers k +- 1 (a square lattice
 * numbered row by row, with the row as the layer).  Anything else is EINVAL. */
typedef struct hfqmc_lattice hfqmc_lattice; /* opaque: hopping blocks on the device */

/* Device memory a lattice needs: its hopping blocks and a site-list buffer
 * of n_sites entries. */
hfqmc_status hfqmc_lattice_bytes(int32_t n_sites, int32_t layer, size_t *bytes);
/* Validates hop (host, n_sites x n_sites row-major) and uploads its blocks
 * into d_mem (caller-owned device memory of hfqmc_lattice_bytes, kept until
 * destroy); the handle is library-owned.  Blocks until the upload is done. */
hfqmc_status hfqmc_lattice_create(hfqmc_ctx *ctx, int32_t n_sites, int32_t layer, const double *hop, void *d_mem,
                                  size_t mem_bytes, hfqmc_lattice **out);
/* Waits for the context's stream, then frees the handle.  A lattice is used
 * only with the context that created it (EINVAL otherwise). */
hfqmc_status hfqmc_lattice_destroy(hfqmc_ctx *ctx, hfqmc_lattice *lat);
/* Device workspace of hfqmc_lattice_green for n_freq frequencies
 * (1 <= n_freq <= 2048): 2 n_freq n_layers P^2 complex doubles, P the layer
 * width padded to 16, 32, 48 or 64. */
hfqmc_status hfqmc_lattice_workspace(const hfqmc_lattice *lat, int32_t n_freq, size_t *bytes);
/* Eq. (2): d_gloc(s, n, i) = [(i w_n + mu) 1 - hop - diag(eps_s) -
 * diag(sigma_s(i w_n))]^-1_ii.  d_eps: 2 x n_sites; d_sigma, d_gloc:
 * spin-frequency-site.  Needs Im sigma(i w_n) < w_n (true of a causal
 * self-energy), which keeps every eliminated block invertible. */
hfqmc_status hfqmc_lattice_green(hfqmc_ctx *ctx, hfqmc_lattice *lat, int32_t n_freq, double beta, double mu,
                                 const double *d_eps, const double *d_sigma, double *d_gloc, void *d_ws,
                                 size_t ws_bytes);
/* Weiss functions of the n_sel sites listed in `sites` (host, indices
 * checked): W = (G_loc^-1 + sigma)^-1 into d_weiss_iw ([s][n][j], complex),
 * and the solver's samples g(tau_l) = -W(tau_l), tau_l = l beta / L, l < L,
 * into d_weiss_tau ([j][s][l]): the level 1 / (i w - e), e = eps_s,i - mu,
 * transformed exactly, the rest summed over the n_freq frequencies and their
 * negatives.  2 <= L <= 160.  The site list (at most n_sites entries) is
 * copied into the lattice's buffer in stream order; the call returns once
 * that copy is done. */
hfqmc_status hfqmc_lattice_weiss(hfqmc_ctx *ctx, hfqmc_lattice *lat, int32_t n_freq, double beta, double mu,
                                 int32_t L, const double *d_eps, const double *d_gloc, const double *d_sigma,
                                 const int32_t *sites, int32_t n_sel, double *d_weiss_iw, double *d_weiss_tau);
/* New self-energy of the listed sites (distinct; host list) from the solver's
 * g(tau_k), k = 0 .. L, in d_gimp_tau ([j][s][k]) and densities d_density
 * ([j][s]), given the Weiss functions d_weiss_iw of hfqmc_lattice_weiss:
 * with sigma_inf = U (n_other spin - 1/2) and W_H = (W^-1 - sigma_inf)^-1,
 * G_imp = W_H - int exp(i w tau) (g - g_H) dtau over the piecewise-linear
 * interpolant, sigma_new = W^-1 - G_imp^-1 for n < max(1, L / 4), and
 * sigma_inf + U^2 n_other (1 - n_other) / (i w_n) above.  Then
 * sigma <- mix sigma_new + (1 - mix) sigma (0 < mix <= 1) at those sites;
 * other sites keep theirs. */
hfqmc_status hfqmc_lattice_sigma(hfqmc_ctx *ctx, hfqmc_lattice *lat, int32_t n_freq, double beta, double mu,
                                 double U, int32_t L, const double *d_eps, const int32_t *sites, int32_t n_sel,
                                 const double *d_weiss_iw, const double *d_gimp_tau, const double *d_density,
                                 double mix, double *d_sigma);

#ifdef __cplusplus
}
#endif

#endif /* HFQMC_H */
