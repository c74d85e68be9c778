/*
 * ctaux_cpu.h — the CT-AUX submatrix update on the host CPU (one chain per
 * object, FP64, single-threaded).
 *
 * The same method as the GPU library (Gull et al., arXiv:1010.3690, Sec. IV):
 * per block of k proposals the insertion candidates are pre-inserted as spin-0
 * vertices (Sec. IV A), the proposals are evaluated from a growing Gamma^{-1}
 * (Sec. III B 2, Eq. ratS) and the accepted changes are applied to
 * N = [e^V - G0 (e^V - 1)]^{-1} (Eq. Nmatrix) in one rank-k update per spin
 * sector (Eq. Nshermanmorrison) followed by the deletion of spin-0 rows and
 * columns (Sec. IV C).  The O(n^2 k) products run as cache-blocked loops
 * (matrix-matrix work that replaces the memory-bound rank-1 updates, the
 * paper's point).  It draws the same counter-based proposal stream as the GPU
 * library for the same (seed, chain), so it takes the same decisions.
 *
 * Conventions: as include/ctaux.h (0 or a negative CTAUX_E* code; host
 * pointers are read during the call only).  Options used: k_max, p_flip,
 * meas_every, n_therm, n_tau_out, n_cap, seed, log_cap (k_cap, precision,
 * recompute_every, gamma_tol, drift_tol, rankk_tile, drift_target,
 * n_matsubara, recompute_mode are ignored: FP64, Gamma as large as k_max).
 * Pair updates are not built here: p_pair must be 0 (CTAUX_EINVAL otherwise).
 */
#ifndef CTAUX_CPU_H
#define CTAUX_CPU_H

#include "ctaux.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctaux_cpu_chain ctaux_cpu_chain;

/* One chain at order 0, drawing from the stream keyed by (opts.seed, chain_id). */
int ctaux_cpu_create(const ctaux_model *model, const ctaux_opts *opts, int32_t chain_id, ctaux_cpu_chain **out);
/* Process the next n_proposals proposals. */
int ctaux_cpu_run(ctaux_cpu_chain *c, int64_t n_proposals);
/* Counters: proposals done, accepted, blocks, current order and sign. */
int ctaux_cpu_get_state(const ctaux_cpu_chain *c, int64_t *proposals, int64_t *accepted, int64_t *blocks,
                        int32_t *order, double *sign);
/* Configuration in canonical order (cap entries at most); *n_out = order. */
int ctaux_cpu_get_config(const ctaux_cpu_chain *c, int32_t cap, ctaux_vertex *out, int32_t *n_out);
/* N of a sector, row-major with leading dimension ld >= order. */
int ctaux_cpu_get_N(const ctaux_cpu_chain *c, int32_t sector, double *out, int32_t ld);
/* Decisions of proposals [first, first + count) within opts.log_cap (as ctaux_get_decisions). */
int ctaux_cpu_get_decisions(const ctaux_cpu_chain *c, int64_t first, int64_t count, uint8_t *acc, double *R);
/* Observable accumulators in the layout of ctaux_get_obs; len >= 8 + 2 n_disp n_tau_out. */
int ctaux_cpu_get_obs(const ctaux_cpu_chain *c, double *out, int32_t len);
/* Replace the configuration (ascending ids) and continue the stream at proposal
 * index `proposals_done` with the given next id and sign; N is computed from its
 * definition by Gauss-Jordan elimination with partial pivoting. */
int ctaux_cpu_set_config(ctaux_cpu_chain *c, int32_t n, const ctaux_vertex *config, int64_t proposals_done,
                         int64_t next_id, double sign);
/* How Gamma grows inside a block (Sec. III B): mode 0 keeps its inverse by
 * partitioning (Eq. ratS; the default), mode 1 an LU factorisation grown by two
 * triangular solves per proposal (Eqs. lineq1, lineq2, detrat, betagammak),
 * re-factorised after an accepted repeated change of a vertex.  Both give the
 * same ratios up to rounding and the same N (Gamma's inverse for the update is
 * taken from Gamma itself at the end of the block either way).  Applies from
 * the next block; CTAUX_EINVAL for another mode. */
int ctaux_cpu_set_growth(ctaux_cpu_chain *c, int32_t mode);
const char *ctaux_cpu_last_error(const ctaux_cpu_chain *c);
void ctaux_cpu_destroy(ctaux_cpu_chain *c);

#ifdef __cplusplus
}
#endif
#endif
