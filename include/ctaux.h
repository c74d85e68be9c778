/*
 * ctaux.h — C ABI of the MI355X (gfx950) CT-AUX submatrix-update library.
 *
 * The library runs Markov chains of the continuous-time auxiliary-field
 * (CT-AUX) Monte Carlo method of Gull et al., "Submatrix updates for the
 * Continuous-Time Auxiliary Field algorithm" (arXiv:1010.3690), on one GPU.
 * Per chain and per block of k proposals it:
 *   - draws the proposals from a counter-based Philox4x32-10 stream and
 *     pre-inserts the block's insertion candidates as spin-0 vertices
 *     (Sec. IV, "Preparation steps");
 *   - evaluates insert / remove / spin-flip proposals as spin changes
 *     0 -> +-1, +-1 -> 0, +-1 -> -+1 with determinant ratios from a growing
 *     Gamma^{-1} (Sec. III B 2, inversion by partitioning, Eq. ratS);
 *   - applies the accepted changes with one rank-k update of
 *     N_sigma = [e^{V_sigma} - G0_sigma (e^{V_sigma} - 1)]^{-1}  (Eq. Nmatrix)
 *     per spin sector (Eq. Nshermanmorrison) and deletes spin-0 rows and
 *     columns (Sec. IV C);
 *   - measures at the end of a block (Sec. IV D) and periodically refines N
 *     against its definition in FP64.
 *
 * Conventions for every entry point:
 *   - Return value 0 (CTAUX_OK) or a negative CTAUX_E* code.  No exception
 *     crosses the ABI.  ctaux_last_error() describes the last failure of a
 *     handle (or of creation, with a NULL handle).
 *   - Host pointers are read during the call only; the caller keeps them.
 *   - Device memory: the caller passes one device workspace of at least
 *     ctaux_workspace_bytes() bytes (256-byte aligned) that must stay valid
 *     until ctaux_destroy(); the library allocates no device memory itself.
 *   - Streams: the block kernels and every copy run on the caller's HIP
 *     stream (NULL = the default stream).  The measurement kernels run on a
 *     stream the library creates at ctaux_create (default priority,
 *     non-blocking), ordered against the caller's stream with two events per
 *     block; ctaux_destroy releases them.  Entry points return after both
 *     streams have drained, except where stated.
 *   - Handles are not thread-safe; distinct handles may be used concurrently
 *     on distinct streams.
 *   - Chains are independent: chain c draws from the stream keyed by
 *     (opts.seed, c).  Vertex order is canonical: ascending vertex id, ids
 *     assigned in order of accepted insertions.
 */
#ifndef CTAUX_H
#define CTAUX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTAUX_OK 0
#define CTAUX_EINVAL (-1)     /* invalid argument or state                        */
#define CTAUX_ENOMEM (-2)     /* workspace too small / host allocation failed     */
#define CTAUX_EDEVICE (-3)    /* HIP runtime error                                */
#define CTAUX_ENUMERIC (-4)   /* NaN/Inf in a ratio or in N, or refinement failed */
#define CTAUX_ECAPACITY (-5)  /* an insertion would exceed n_cap                  */

#define CTAUX_FP64 0          /* N stored and updated in FP64 (FP64 MFMA)               */
#define CTAUX_FP32 1          /* N stored in FP32, rank-k update on FP32 MFMA, FP64 Gamma */
#define CTAUX_BF16X3 2        /* N stored in FP32, rank-k update as split-BF16x3: each FP32
                                 operand split into two BF16 terms (hi + lo), the product taken
                                 as hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation
                                 (~2^-16 relative per product); FP64 Gamma                    */

/* Model of one chain (Sec. II A).  U >= 0, K > 0, beta > 0.
 * gamma is fixed by cosh(gamma) = 1 + beta*U*n_sites/(2K)  (Eq. gamma; the
 * factor n_sites is the cluster form of the decoupling).
 * The bare propagator of the pair of sites (x, y) is table site_disp[x*n_sites+y]:
 * g0_sigma[d*n_tau + m] = G0_sigma,d(tau_m), tau_m = m*beta/(n_tau-1),
 * with G0(tau) = <T c_x(tau) c_y^dagger(0)>_0 (entry 0 = tau -> 0+, last = beta-).
 * Between grid points G0 is interpolated linearly; G0(tau - beta) = -G0(tau). */
typedef struct {
    double beta, U, K;
    int32_t n_sites;          /* Nc >= 1                                       */
    int32_t n_tau;            /* >= 2                                          */
    int32_t n_disp;           /* number of tables per sector                   */
    const int32_t *site_disp; /* host, [n_sites*n_sites], values in [0, n_disp) */
    const double *g0_up;      /* host, [n_disp*n_tau], finite                  */
    const double *g0_dn;      /* host, [n_disp*n_tau], finite                  */
    const double *site_pos;   /* host, [n_sites*3] site positions r_x (lattice units), or NULL;
                                 needed when opts.n_matsubara > 0                          */
    const double *kvecs;      /* host, [n_k*3] cluster momenta K                             */
    int32_t n_k;              /* number of momenta, 1..512 when site_pos is given           */
} ctaux_model;

/* Run options shared by all chains of a batch. */
typedef struct {
    int32_t k_max;            /* proposals per block, 1..128                                  */
    int32_t k_cap;            /* accepted changes per block (size of Gamma), 1..64; a block
                                 ends early once Gamma is full (does not change the chain)     */
    double p_flip;            /* P(flip); P(insert) = P(remove) = (1 - p_flip - p_pair)/2     */
    int32_t recompute_every;  /* most blocks between FP64 refinements of N (0 = never).  Each
                                 chain has its own interval, a power of two between 1 and the
                                 largest power of two <= recompute_every, starting at 1
                                 and counted in blocks of the batch (chain c
                                 is refined after block b when b is a multiple of its
                                 interval).  After each refinement of a chain its interval is
                                 quartered when the drift exceeded drift_target and doubled
                                 when the drift stayed below drift_target / 16              */
    int32_t precision;        /* CTAUX_FP64, CTAUX_FP32 or CTAUX_BF16X3                       */
    int32_t meas_every;       /* measure after every meas_every proposals ...                 */
    int64_t n_therm;          /* ... once more than n_therm proposals are done                */
    int32_t n_tau_out;        /* G(tau) output points tau_j = (j+1/2) beta / n_tau_out (0: none;
                                 densities and double occupancy are measured regardless)     */
    int32_t n_cap;            /* maximum order per chain                                      */
    uint64_t seed;
    int64_t log_cap;          /* decisions of proposals with index < log_cap are recorded     */
    double gamma_tol;         /* Gamma^{-1} for the N update: the growth inverse X0 (built
                                 while proposing, Sec. IV C) is used when
                                 max|(I - Gamma X0)_ij| <= gamma_tol (1e-8 is a good value),
                                 with one Newton step when that residual lies above its own
                                 FP64 rounding floor; otherwise, and always when
                                 gamma_tol < 0, a Gauss-Jordan elimination with partial
                                 pivoting of Gamma.                                           */
    double drift_tol;         /* a refinement whose drift exceeds drift_tol stops the chain
                                 with CTAUX_ENUMERIC (N no longer represents the inverse of
                                 its definition); <= 0 disables the check                     */
    int32_t rankk_tile;       /* output tile edge of the rank-k update: 64, 32, or 0 for 64;
                                 smaller tiles waste less of the ragged edge at small orders  */
    double drift_target;      /* N error a chain should carry at most between refinements (the
                                 refinement drift, see ctaux_recompute); 0 selects 1e-10 for
                                 FP64 storage and 1e-4 for FP32 storage                       */
    int32_t n_matsubara;      /* 0..32: also measure in cluster momenta and the first
                                 n_matsubara fermionic frequencies (ctaux_get_obs_kw);
                                 n_sites * n_matsubara <= 2048                               */
    int32_t recompute_mode;   /* periodic refinements: 0 = a Newton step from the current N,
                                 recomputed from scratch when the step cannot recover it (see
                                 ctaux_recompute); 1 = always from scratch
                                 (ctaux_recompute_from_scratch)                               */
    double p_pair;            /* pair updates (Sec. IV B: Gamma grows by two rows and columns):
                                 two vertices inserted together with probability p_pair/2,
                                 two removed together with p_pair/2; 0 <= p_pair <= 1 - p_flip
                                 (0: single-vertex moves only).  Acceptance ratios
                                 K^2/((n+1)(n+2)) and n(n-1)/K^2 times the two sectors'
                                 determinant ratios.  The second vertex of a pair insertion
                                 takes u_spin2 (second word pair of Philox tag 2) and u_tau2,
                                 u_pick2 (tag 3); a pair removal picks ranks floor(n u_pick)
                                 and floor((n-1) u_pick2), the second skipping the first, in
                                 ascending id order, and is rejected (and counted) at n < 2.
                                 Requires k_max >= 2 and k_cap >= 2.  A block ends before a
                                 pair proposal that could overfill Gamma or the block's
                                 k_max insertion candidates; like every block boundary this
                                 leaves the chain unchanged                                  */
} ctaux_opts;

/* Per-chain counters. */
typedef struct {
    int64_t proposals;        /* proposals processed                         */
    int64_t accepted;         /* accepted proposals                          */
    int64_t blocks;           /* blocks (outer iterations) completed          */
    int64_t sum_ka;           /* sum over blocks of accepted changes          */
    int64_t next_id;          /* next vertex id                              */
    int32_t order;            /* current expansion order n                    */
    int32_t status;           /* 0 or the CTAUX_E* code that stopped the chain */
    double sign;              /* sign of the current configuration weight    */
    double max_drift;         /* largest refinement drift seen (see ctaux_recompute) */
    double rankk_flops;       /* algorithmic flops of the rank-k updates so far (both sectors:
                                 2 n'^2 k_a + 2 k_a^2 n' each, n' = order after the block)   */
    double rankk_bytes;       /* algorithmic HBM bytes of the rank-k updates so far (read and
                                 write n'^2 entries of N, read the n' x k_a operands)          */
    double sum_order;         /* sum over blocks of the order after the block                */
    int64_t gj_fallbacks;     /* sector-blocks whose Gamma^{-1} came from the pivoted
                                 elimination instead of the growth inverse                */
    double prep_flops;        /* algorithmic flops of the preparation products: per sector
                                 4 n^2 k_ins (YT, Rt) + 2 k_ins^2 n (Gnn)                      */
    double prep_bytes;        /* their algorithmic HBM bytes: N read twice, X, ZT, YT, Rt once */
    double meas_flops;        /* algorithmic flops of the measurements: per sector
                                 2 n^2 nc (W) + 2 nc^2 (n_out+1) n (G)                         */
    double meas_bytes;        /* their algorithmic bytes: N read once, gL written and read,
                                 two table reads per gL entry, gR                              */
    int64_t scratch_recomputes; /* refinements that recomputed N from scratch                  */
    int32_t refine_interval;  /* the chain's current refinement interval in blocks (0: none)    */
} ctaux_stats;

/* One vertex of a configuration (tau in [0, beta), site in [0, n_sites), s = +-1). */
typedef struct {
    int64_t id;
    double tau;
    int32_t site;
    int32_t s;
} ctaux_vertex;

typedef struct ctaux_batch ctaux_batch;

/* Device bytes needed for n_chains chains with these models and options
 * (0 if the arguments are invalid). */
size_t ctaux_workspace_bytes(const ctaux_model *models, int32_t n_chains, const ctaux_opts *opts);

/* Create a batch of n_chains chains, all starting at order 0.  models is a
 * host array [n_chains].  The workspace is device memory owned by the caller. */
int ctaux_create(const ctaux_model *models, int32_t n_chains, const ctaux_opts *opts,
                 void *dev_workspace, size_t ws_bytes, void *hip_stream, ctaux_batch **out);

/* Advance every chain by n_proposals proposals (propose/accept batch).  Stops
 * a chain early on CTAUX_ECAPACITY / CTAUX_ENUMERIC and returns that code. */
int ctaux_run(ctaux_batch *b, int64_t n_proposals);

/* Refine N of every chain against its definition in FP64 and return the
 * largest relative drift of the first step, ||N_before - N_after||_F / ||N_after||_F,
 * over the chains (the N error the chain carried, to first order).
 * A step is one Newton iteration N <- N + N (I - M N) with M = e^V - G0(e^V - 1)
 * built from the tables (Eq. Nmatrix); a chain whose drift exceeded 1e-9 with
 * FP64 storage (1e-4 with FP32) gets another step, up to three in all.  N is
 * recomputed from scratch instead (as by ctaux_recompute_from_scratch) when a
 * step measures a drift above 1e-2 or a non-finite N, when a further step does
 * not reduce the drift fourfold, or after the third step.  A drift above
 * opts.drift_tol (> 0) stops the chain with CTAUX_ENUMERIC.
 * Also runs automatically on the schedule of opts.recompute_every. */
int ctaux_recompute(ctaux_batch *b, double *max_drift_out);

/* Recompute N of every chain from scratch: M = e^V - G0(e^V - 1) from the
 * tables, inverted in FP64 by a blocked Gauss-Jordan elimination (32 columns
 * per step, pivot rows chosen by tournament pivoting, the trailing updates on
 * FP64 MFMA; 2 n^3 flops per sector).  Returns the largest relative difference
 * ||N_before - N_after||_F / ||N_after||_F over the chains.  A singular or
 * non-finite M stops the chain with CTAUX_ENUMERIC. */
int ctaux_recompute_from_scratch(ctaux_batch *b, double *max_drift_out);

/* Observable accumulators of a chain (doubles, len >= ctaux_obs_len()):
 *   [0] measurements   [1] sum sign       [2] sum sign*order   [3] sum sign*order^2
 *   [4] sum sign*[order==0]               [5] sum sign*D (double occupancy per site)
 *   [6] sum sign*n_up per site            [7] sum sign*n_dn per site
 *   [8 ...] sum sign*G_up[d][j]; then sum sign*G_dn[d][j]  (d < n_disp, j < n_tau_out),
 * G_sigma[d][j] = average of G_sigma(x, tau_j; y, 0) over pairs with table d. */
int32_t ctaux_obs_len(const ctaux_batch *b);
/* Measurement in cluster momenta and Matsubara frequencies (Sec. IV D), with
 * n_matsubara > 0.  With M = (e^V - 1) N, every measurement adds sign * S(K, w_n),
 *   S(K, w) = sum_{l,k} exp(i w tau_l - i K.r_{x_l}) M_lk exp(-i w tau_k + i K.r_{x_k}),
 * w_n = (2n + 1) pi / beta, so that the estimate of the Green's function is
 *   G(K, i w_n) = G0(K, i w_n) + G0(K, i w_n)^2 (sum sign S / sum sign) / (beta n_sites)
 * (sum sign is entry [1] of ctaux_get_obs), with
 *   G0(K, i w_n) = (1/n_sites) sum_{x,y} exp(-i K.(r_x - r_y)) int_0^beta exp(i w_n s) G0_xy(s) ds
 * for the linear interpolant of the tables (computed at ctaux_create).
 * s_out receives the accumulated sign * S and g0_out (may be NULL) G0, both as
 * [sector][k][n][re, im] doubles; len >= 4 n_k n_matsubara. */
int ctaux_get_obs_kw(ctaux_batch *b, int32_t chain, double *s_out, double *g0_out, int32_t len);
int ctaux_get_obs(ctaux_batch *b, int32_t chain, double *out, int32_t len);
int ctaux_reset_obs(ctaux_batch *b);

int ctaux_get_stats(ctaux_batch *b, int32_t chain, ctaux_stats *out);
/* Configuration in canonical order; *n_out = order; at most cap vertices copied. */
int ctaux_get_config(ctaux_batch *b, int32_t chain, int32_t cap, ctaux_vertex *out, int32_t *n_out);
/* N of one sector (0 up, 1 down) as FP64, row-major with leading dimension ld >= order.
 * With out == NULL only *n_out is set. */
int ctaux_get_N(ctaux_batch *b, int32_t chain, int32_t sector, double *out, int32_t ld,
                int32_t *n_out);
/* Decisions of proposals [first, first+count) (count <= log_cap - first):
 * acc[i] = 1 if accepted, R[i] = signed acceptance ratio (0 for a removal or
 * flip proposed at order 0). */
int ctaux_get_decisions(ctaux_batch *b, int32_t chain, int64_t first, int64_t count,
                        uint8_t *acc, double *R);
/* Per-kernel device time (ms) accumulated since the last reset, measured with
 * HIP events around the launches selected by ctaux_set_timing(b, mask): bit i
 * of mask selects entry i of the names ctaux_get_timing reports (-1: all,
 * 0: off; every event pair adds a little time to the stream).  names[i] are
 * static strings; returns the number of entries written (<= cap). */
int ctaux_set_timing(ctaux_batch *b, int32_t mask);
/* Time only one launch in `every` of each selected kernel (default 1), which
 * keeps the events' own device time out of most launches. */
int ctaux_set_timing_every(ctaux_batch *b, int32_t every);
/* Replay windows of `blocks` blocks (0: off, or a power of two <= 64) from a
 * HIP graph captured at the first window: ctaux_run then launches one graph
 * per window instead of the window's kernels one by one (the same kernels in
 * the same order, so the chains' results are unchanged).  A window is used
 * where at least one more block of the run follows it, it starts at a
 * multiple of `blocks` blocks, and every chain's refinement interval is at
 * least `blocks` (refinements, which synchronise with the host, then fall
 * between windows); elsewhere blocks are launched one by one.  No event
 * timing runs inside a window.  Waits for the batch's streams; CTAUX_EINVAL
 * for an invalid size. */
int ctaux_set_graph(ctaux_batch *b, int32_t blocks);
/* Number of graph windows launched so far (-1 for b == NULL). */
int64_t ctaux_graph_launches(const ctaux_batch *b);
int32_t ctaux_get_timing(ctaux_batch *b, const char **names, double *ms, int64_t *launches,
                         int32_t cap);

/* Checkpoint / resume of one chain (the chain state the method carries from
 * block to block, Sec. IV C: the vertex configuration and N of both sectors,
 * plus the proposal counter that keys the random stream and the measurement
 * accumulators).
 *   ctaux_checkpoint: with buf == NULL stores the needed size in *len; else
 *     *len is the capacity of buf on entry (CTAUX_EINVAL if too small) and the
 *     bytes written on return.  The blob is a host byte string of the same
 *     build (native endianness).
 *   ctaux_restore: loads a blob into `chain` of this batch, which must have the
 *     same precision, n_sites, n_tau, beta, K, coupling and observable layout
 *     (CTAUX_EINVAL otherwise) and n_cap >= the stored order.  The FP64
 *     refinement schedule belongs to the batch; a one-chain batch with the same
 *     recompute_every also takes over that schedule, so continuing with the
 *     same seed and chain index reproduces the uninterrupted chain bit for bit.
 *     In a larger batch the refinement phase may differ, which changes N by
 *     rounding only.  The decision log of the target is not restored. */
int ctaux_checkpoint(ctaux_batch *b, int32_t chain, void *buf, size_t *len);
int ctaux_restore(ctaux_batch *b, int32_t chain, const void *buf, size_t len);

/* N of one spin sector (0 up, 1 down) of a configuration, from its definition
 * N = [e^V - G0 (e^V - 1)]^{-1} (Eq. Nmatrix) with G0 interpolated from the
 * model's tables as the chains do, inverted in FP64 by the elimination of
 * ctaux_recompute_from_scratch.  Stateless; independent of any batch.
 *   model:   host, as for ctaux_create (one chain).
 *   config:  host, n vertices (0 <= tau < beta, 0 <= site < n_sites, s = +-1;
 *            id is ignored); row and column i of N belong to config[i].
 *   dev_out: device, n rows of ld_out >= n doubles (row-major), written.
 *   dev_workspace: device, >= ctaux_build_N_workspace_bytes(model, n) bytes,
 *            256-byte aligned, used during the call only.
 *   hip_stream: the stream every copy and kernel runs on (NULL: default).
 * Returns after the stream has drained.  0 <= n <= 32768 (n = 0 does nothing).
 * Errors (ctaux_last_error(NULL) describes them): CTAUX_EINVAL (arguments),
 * CTAUX_ENOMEM (workspace too small), CTAUX_ENUMERIC (M singular or not
 * finite; dev_out then holds NaN), CTAUX_EDEVICE. */
size_t ctaux_build_N_workspace_bytes(const ctaux_model *model, int32_t n);
int ctaux_build_N(const ctaux_model *model, const ctaux_vertex *config, int32_t n, int32_t sector, double *dev_out,
                  int32_t ld_out, void *dev_workspace, size_t ws_bytes, void *hip_stream);

/* ctaux_build_N without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * ctaux_build_N; allocates nothing.  Its scratch is a fixed 24 MiB array in
 * device memory that each GPU the library runs on holds until the process
 * ends; n is limited to 1024 and the model's tables of one sector plus
 * 8 n^2 bytes must fit in it (CTAUX_EINVAL otherwise).  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (other host threads,
 * other streams) race and must be serialised by the caller. */
int ctaux_build_N_noalloc(const ctaux_model *model, const ctaux_vertex *config, int32_t n, int32_t sector,
                          double *dev_out, int32_t ld_out, void *hip_stream);

const char *ctaux_last_error(const ctaux_batch *b);
void ctaux_destroy(ctaux_batch *b);

#ifdef __cplusplus
}
#endif
#endif
