/*
 * CT-AUX oracle: a plain, slow, FP64 CPU implementation of the continuous-time
 * auxiliary-field Monte Carlo walk with rank-1 ("fast update") bookkeeping.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for
 * the GPU submatrix path.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; no product code path calls it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (Gull et al., "Submatrix updates for the Continuous-Time
 * Auxiliary Field algorithm", Sec. II):
 *   - weights of auxiliary-spin configurations {(tau_i, site_i, s_i)} through
 *     N_sigma = [e^{V_sigma} - G0_sigma (e^{V_sigma} - 1)]^{-1}   (Eq. Nmatrix)
 *     with e^{V_sigma} = diag(exp(gamma * sigma * s_i)), sigma = +1 (up) / -1 (down)
 *     and cosh(gamma) = 1 + beta*U*Nc/(2K)                         (Eq. gamma,
 *     with the cluster factor Nc);
 *   - Metropolis insert / remove / spin-flip proposals with acceptance
 *     ratios of Eq. (insprob) and Sec. II B;
 *   - the matrix N kept current by rank-1 updates after every accepted move
 *     (bordering for insertion, Schur complement for removal, the Dyson
 *     relation of Eq. (DysonG) normalised by the ratio for a flip);
 *   - measurements of the order, sign, densities, double occupancy and
 *     G(tau) from the complete N (Sec. IV D).
 * Random numbers follow a counter-based stream (Philox4x32-10, Salmon et al.,
 * SC'11) keyed by (seed, chain) with counter (proposal index, chain, tag).
 *
 * All functions return 0 on success or a negative OC_E* code; oc_error()
 * gives a message.  Matrices are row-major, leading dimension = order n.
 */
#ifndef CTAUX_ORACLE_H
#define CTAUX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OC_OK 0
#define OC_EINVAL (-1)
#define OC_ENOMEM (-2)
#define OC_ENUMERIC (-4)
#define OC_ECAPACITY (-5)

typedef struct oc_chain oc_chain;

/* Observable accumulator layout (doubles), every entry summed over
 * measurements and weighted by the configuration sign where noted:
 *   [0] number of measurements      [1] sum sign
 *   [2] sum sign*order              [3] sum sign*order^2
 *   [4] sum sign*[order==0]         [5] sum sign*D (double occupancy per site)
 *   [6] sum sign*n_up per site      [7] sum sign*n_dn per site
 *   [8 ...]                         sum sign*G_up[d][j], d < n_disp, j < n_tau_out
 *   [8 + n_disp*n_tau_out ...]      sum sign*G_dn[d][j]
 * G_sigma[d][j] averages G_sigma(x, tau_j; y, 0) over site pairs whose table
 * index is d, at tau_j = (j + 1/2) * beta / n_tau_out.                       */
#define OC_OBS_HEADER 8

oc_chain *oc_create(double beta, double U, double K, int32_t n_sites, int32_t n_tau,
                    int32_t n_disp, const int32_t *site_disp, const double *g0_up,
                    const double *g0_dn, uint64_t seed, uint32_t chain_id, double p_flip,
                    int32_t meas_every, int64_t n_therm, int32_t n_tau_out, int32_t n_cap);
void oc_destroy(oc_chain *c);
const char *oc_error(const oc_chain *c);

/* Process the next n_proposals proposals of the stream. */
int oc_run(oc_chain *c, int64_t n_proposals);

/* Record decisions of proposals with global index < cap (0 disables). */
int oc_set_log(oc_chain *c, int64_t cap);
/* Copy logged decisions [first, first+count): acc (0/1) and the signed ratio R. */
int oc_get_log(const oc_chain *c, int64_t first, int64_t count, uint8_t *acc, double *R);

int32_t oc_order(const oc_chain *c);
int64_t oc_proposals_done(const oc_chain *c);
double oc_sign(const oc_chain *c);
double oc_gamma_value(const oc_chain *c);

/* Current configuration in canonical (ascending id) order. */
int oc_get_config(const oc_chain *c, int64_t *id, double *tau, int32_t *site, int32_t *s);
/* N of a sector (0 = up, 1 = down), n x n row-major into out (ld = n). */
int oc_get_N(const oc_chain *c, int32_t sector, double *out);
/* M = N^{-1} of the current configuration built from its definition (Eq. Nmatrix). */
int oc_build_Minv(const oc_chain *c, int32_t sector, double *out);
/* The same definition for a configuration given by its arrays (the chain only
 * supplies the model); O(n^2), no inversion. */
int oc_build_M_of(const oc_chain *c, int32_t sector, int32_t n, const double *tau,
                  const int32_t *site, const int32_t *s, double *out);

/* Replace the configuration (used for restore and for brute-force pins);
 * N is rebuilt by successive bordering.  log|det N_sigma^{-1}| and its sign
 * are returned per sector (either pointer may be NULL). */
int oc_set_config(oc_chain *c, int32_t n, const int64_t *id, const double *tau,
                  const int32_t *site, const int32_t *s, double *logabsdet, double *sgn);
/* Checkpoint scalars: proposal counter, next id, sign. */
int oc_get_state(const oc_chain *c, int64_t *proposals_done, int64_t *next_id, double *sign);
int oc_set_state(oc_chain *c, int64_t proposals_done, int64_t next_id, double sign);

/* Last processed proposal: type (0 ins, 1 rem, 2 flip, 3 pair insertion,
 * 4 pair removal), vertex position p (insert: n before insertion), tau, site,
 * new spin, signed ratio, accepted.  For a pair these describe its first
 * vertex and oc_last_pair its second (position n + 1 for a pair insertion;
 * -1 for other types). */
int oc_last_proposal(const oc_chain *c, int32_t *type, int32_t *p, double *tau,
                     int32_t *site, int32_t *s_new, double *R, int32_t *acc);
int oc_last_pair(const oc_chain *c, int32_t *p2, double *tau2, int32_t *site2, int32_t *s2);

/* Pair updates (Sec. IV B: Gamma grows by two rows and columns): insertion and
 * removal of two vertices at once, each with probability p_pair/2, in place
 * of single insertions and removals (which keep (1 - p_flip - p_pair)/2 each).
 * Requires 0 <= p_pair <= 1 - p_flip; 0 (the default) leaves the walk as it is.
 * A pair insertion draws its second vertex from oc_pair_draws; a pair removal
 * picks ranks r1 = floor(n u_pick) and r2 = floor((n - 1) u_pick2), the second
 * skipping r1 (r2 >= r1 -> r2 + 1), in ascending id order; at n < 2 it is
 * rejected and counted. */
int oc_set_pair(oc_chain *c, double p_pair);

/* Observables. */
int32_t oc_obs_len(const oc_chain *c);
int oc_get_obs(const oc_chain *c, double *out);
int oc_reset_obs(oc_chain *c);
/* Measurement estimator for the current configuration, without accumulating:
 * G_sigma(x, tau; y, 0) for 0 <= tau < beta (tau = 0 means 0+). */
int oc_estimate_G(const oc_chain *c, int32_t sector, int32_t x, int32_t y, double tau,
                  double *out);

/* Measurement in cluster momenta and Matsubara frequencies (Sec. IV D).  With
 * M = (e^V - 1) N, site positions r_x and momenta K, every measurement adds
 * sign * S_sigma(K, w_n) with
 *   S(K, w) = sum_{l,k} exp(i w tau_l - i K.r_{x_l}) M_lk exp(-i w tau_k + i K.r_{x_k}),
 * w_n = (2n + 1) pi / beta, so that
 *   G(K, i w_n) = G0(K, i w_n) + G0(K, i w_n)^2 <S(K, w_n)> / (beta Nc).
 * site_pos [n_sites*3], kvecs [n_k*3]; n_matsubara frequencies.  Layout of the
 * accumulator (oc_get_obs_kw): [sector][k][n][re, im]. */
int oc_set_momentum(oc_chain *c, int32_t n_k, const double *kvecs, const double *site_pos,
                    int32_t n_matsubara);
int oc_get_obs_kw(const oc_chain *c, double *out);
/* G0(K, i w_n) = (1/Nc) sum_{x,y} exp(-i K.(r_x - r_y)) int_0^beta exp(i w_n s) G0_xy(s) ds
 * with G0_xy the linear interpolant of the tables; out = [re, im]. */
int oc_g0_matsubara(const oc_chain *c, int32_t sector, int32_t k, int32_t n, double *out);

/* Building blocks exposed for the pins. */
double oc_g0_lookup(const oc_chain *c, int32_t sector, int32_t x, int32_t y, double dtau);
void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* The five uniforms of proposal `index`: u_type, u_acc, u_tau, u_pick, u_spin. */
void oc_draws(uint64_t seed, uint32_t chain_id, uint64_t index, double out[5]);
double oc_gamma_of(double beta, double U, double K, int32_t n_sites);
/* The extra uniforms of a pair proposal: u_spin2 (the second word pair of tag
 * 2), u_tau2 and u_pick2 (tag 3). */
void oc_pair_draws(uint64_t seed, uint32_t chain_id, uint64_t index, double out[3]);

#ifdef __cplusplus
}
#endif
#endif
