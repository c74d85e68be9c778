// Internal structures of the gfx950 CT-AUX submatrix library.
//
// One "chain" is an independent Markov chain.  Every per-chain buffer lives
// in the caller's device workspace; ChainDesc holds the pointers (fixed at
// creation) and ChainState the evolving scalars.  All kernels take the batch
// arrays and find their chain from the grid, so one launch serves every
// chain of a batch (the batched form) and a single chain alike.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctaux {

constexpr int kMaxKcap = 64;    // Gamma capacity per block (Gamma^{-1} of both sectors in LDS)
constexpr int kMaxKmax = 128;   // proposals per block


enum Precision : int32_t { kFP64 = 0, kFP32 = 1, kBF16X3 = 2 };   // storage of N: FP64, FP32, FP32

struct ChainDesc {
  // ---- model (Sec. II A) ----
  double beta, K, gamma, inv_h, p_flip;
  double gamma_tol;        // growth inverse of Gamma (Newton-refined where that gains) accepted below this residual
  double drift_tol;        // refinement drift above this stops the chain (<= 0: no check)
  double evd[2][5];        // exp(gamma*sigma*d), d = -2..2 (index d+2); sigma = +1 up, -1 down
  int32_t nc, n_tau, n_disp;
  int32_t lda;             // leading dimension of Ac rows (k_cap rounded up to 8)
  const double *g0[2];     // tables [n_disp*n_tau] per sector
  const int32_t *site_disp;  // [nc*nc]
  // ---- geometry of the per-chain buffers ----
  int32_t n_cap;           // max order
  int32_t ld;              // leading dimension of N, X, ZT, YT, Rt, Bc (>= n_cap)
  int32_t kmax, kcap;
  int32_t meas_every, n_out;
  int64_t n_therm;
  uint32_t seed_lo, seed_hi, chain_id;
  int32_t precision;
  int64_t log_cap;
  // ---- buffers ----
  void *N[2][2];           // [parity][sector], ld x ld, double or float
  double *tau[2];          // [parity][n_cap]
  int32_t *site[2];
  int32_t *s0[2];
  int64_t *id[2];
  // block proposals (decoded)
  int32_t *ptype;          // [kmax] 0 ins, 1 rem, 2 flip, 3 pair insertion, 4 pair removal
  int32_t *pspin;          // [kmax] spin of an insertion (+-1; first vertex of a pair)
  double *pacc;            // [kmax] u_acc
  double *ppick;           // [kmax] u_pick
  double *ctau;            // [kmax] candidate times
  int32_t *csite;          // [kmax] candidate sites
  int64_t *cid;            // [kmax] ids given to accepted candidates
  // preparation products, FP64, per sector
  double *X[2];            // X_ji = G0(tau_j^new - tau_i)(e^{V_i} - 1), kmax x ld in cand_offset order
  double *ZT[2];           // ZT_ji = G0(tau_i - tau_j^new), the same layout
  double *G0nn[2];         // [kmax][kmax]
  double *YT[2];           // [kmax][ld]  (N Z)^T: G of old rows, new columns
  double *Rt[2];           // [kmax][ld]  X N: rows of the augmented N for new vertices
  double *Gnn[2];          // [kmax][kmax] X Y + G0nn: G of new rows, new columns
  // Gamma bookkeeping of the block
  int32_t *P;              // [kcap] augmented index of each accepted change
  double *ghat[2];         // [kcap]
  double *Gam[2];          // [kcap][kcap] entries of the column-scaled Gamma~ of the accepted changes
  double *Ginv[2];         // [kcap][kcap] Gamma~^{-1} for the rank-k update
  double *Rg[2];           // [kcap][kcap] residual I - Gamma~ X0 of the growth inverse
  int32_t *map;            // [n_cap] new canonical index -> augmented index
  // rank-k operands (storage type of N)
  void *Ac[2];             // ((G - I) D^{-1})_{map, P}, n' x lda in ac_offset order (ld x lda allocated)
  void *Bc[2];             // [lda][ld]       Gamma~^{-1} N_a(P, map)
  // measurement
  double *W[2];            // [n_cap][nc]  N gR
  double *gR[2];           // G0_{x_k y}(tau_k), nc x n_cap in cand_offset order (rows y)
  double *Gxy[2];          // [(n_out+1)][nc*nc]  row 0 = equal time
  const int32_t *cls_off;  // [n_disp+1] pairs (x*nc+y) of each table, CSR offsets
  const int32_t *cls_pairs;  // [nc*nc]
  double *obs;             // accumulators
  int32_t obs_len;
  int32_t pad1;
  // measurement in cluster momenta and Matsubara frequencies (n_mats = 0: off)
  int32_t n_k, n_mats;
  double *kw_pos;          // [nc*3] site positions
  double *kw_k;            // [n_k*3] cluster momenta
  double *kw_g0;           // [2][n_k][n_mats][2] G0(K, i w_n), set at creation
  int32_t *kw_off;         // [nc+1] vertices of each site (CSR offsets into kw_list)
  int32_t *kw_list;        // [n_cap] vertex indices sorted by site (ascending within a site)
  double *kw_ph;           // [n_cap][n_mats][2] exp(-i w_n tau_k)
  double *kw_C;            // [2][nc][nc][n_mats][2] sum_{l in x, k in x'} e^{i w tau_l} M_lk e^{-i w tau_k}
  double *obs_kw;          // [2][n_k][n_mats][2] sum of sign * S(K, w_n)
  // decision log
  uint8_t *log_acc;        // [log_cap]
  double *log_R;           // [log_cap]
  // measurement of batches of fewer than 8 chains (null otherwise)
  double *gL[2];           // [nc*(n_out+1)][ld]  G0_{x x_l}(tau_j - tau_l)(e^{V_l} - 1), row (j, x)
  // measurement of batches of 8 chains or more: vertices in order of their time
  // (stable by 128 time buckets), so that the interpolations of gL for
  // consecutive vertices read neighbouring table entries
  int32_t *mpos;           // [n_cap] position of vertex l in that order
  double *mtau;            // [n_cap] tau of the vertex at each position
  int32_t *msite;          // [n_cap] its site
  double *mfac;            // [n_cap] e^{V} - 1 of its sector 0 and 1 ([2][n_cap])
  // pair proposals (Sec. IV B; the fields above keep their offsets without them)
  double p_pair;           // pair insertions and removals, p_pair / 2 each
  int32_t *pspin2;         // [kmax] spin of a pair insertion's second vertex
  double *ppick2;          // [kmax] u_pick2 of a pair removal
};

struct ChainState {
  int32_t n;           // order at block start
  int32_t k_ins;       // insertion candidates drawn for this block
  int32_t L;           // proposals drawn for this block
  int32_t L_eff;       // proposals processed in this block
  int32_t k_a;         // accepted changes (size of Gamma)
  int32_t n_new;       // order after the block
  int32_t parity;      // current buffer set
  int32_t status;      // 0 or negative error code
  int32_t meas_now;    // 1: measure after this block
  int32_t active;      // 1: the chain runs this block
  int64_t done;        // proposals processed
  int64_t target;      // run until done == target
  int64_t next_id;
  int64_t accepted;
  int64_t blocks;
  int64_t sum_ka;
  double sign;
  double max_drift;
  double last_drift;
  double pass_drift;       // drift measured by the latest refinement pass
  int64_t err_index;   // proposal index of a failure
  double rk_flops;     // algorithmic flops of operand assembly + rank-k update, summed over blocks
  double rk_bytes;     // algorithmic HBM bytes of the rank-k update (read N_a, write N', read Ac, Bc)
  double sum_order;    // sum over blocks of the order after the block
  int64_t gj_fallbacks;  // sector-blocks whose Gamma^{-1} needed the pivoted elimination
  double prep_flops, prep_bytes;   // algorithmic work of the preparation products
  double meas_flops, meas_bytes;   // algorithmic work of the measurements
  int64_t scratch_recomputes;      // refinements that recomputed N from scratch (pivoted elimination)
};

// Kernel launchers (each .hip file owns its kernels).
struct Batch;
void launch_block_begin(const Batch &b, hipStream_t s);
void launch_interp(const Batch &b, hipStream_t s);
void launch_prep(const Batch &b, hipStream_t s);
void launch_propose(const Batch &b, hipStream_t s);
void launch_assemble(const Batch &b, hipStream_t s);
void launch_rankk(const Batch &b, hipStream_t s);
void launch_block_end(const Batch &b, hipStream_t s);
void launch_block_turn(const Batch &b, hipStream_t s);   // block end + next block begin
void launch_measure(const Batch &b, hipStream_t s);
void launch_kw_g0(const Batch &b, hipStream_t s);   // G0(K, i w_n) of every chain, once at creation
// Refinement of a group of chains: each item names a chain, its order and the
// offset (in doubles) of its scratch in the refinement pool.
struct RefineItem {
  int32_t chain;
  int32_t n;
  int64_t off;
};
int refine_slots(int precision);           // n x n scratch blocks per sector
size_t refine_red_doubles(int n_chains);   // partial sums for the drift of a batch of n_chains chains
// pool doubles one chain of order n needs for a refinement (Newton slots of both
// sectors, then the from-scratch elimination's scratch of both sectors)
size_t refine_need_doubles(int n, int precision);
void launch_refine_group(const Batch &b, hipStream_t s, const RefineItem *items, int n_items, int pass);
// From-scratch recompute of the chains of a group: M from the tables, inverted
// by the blocked Gauss-Jordan elimination (k_invert.hip); inv = 2 items per
// chain (sector 0, 1) whose pointers the host has carved from the pool.
struct InvItem;
void launch_scratch_group(const Batch &b, hipStream_t s, const RefineItem *items, const InvItem *inv, int n_items,
                          int n_max, int pass);

// ---- blocked Gauss-Jordan inversion (k_invert.hip) ----
constexpr int kInvNB = 32;   // columns eliminated per step
constexpr int kBuildMaxOrder = 32768;   // largest configuration of the stateless N builder
struct InvItem {
  double *W;        // [n][ldw] the matrix, eliminated in place
  double *T;        // [kInvNB][n]   A11^{-1} W[p, :] of the current step
  double *Lp;       // [n][kInvNB]   W[:, J] of the current step
  double *Ainv;     // [kInvNB][kInvNB]
  int32_t *cand;    // [ceil(n/256) * kInvNB] tournament candidate lists
  int32_t *blk;     // [n] step at which a row became a pivot (-1: not yet)
  int32_t *slot;    // [n] its place within that step
  int32_t *perm;    // [n] pivot row of each position
  int32_t *flag;    // [1] set when a pivot block is singular or not finite
  int32_t n, ldw;
};
size_t inv_scratch_doubles(int n);   // T, Lp, Ainv and the index arrays of one n x n elimination
void inv_item_carve(InvItem &it, double *W, int n, int ldw, double *scratch);
int setup_invert(int max_items);     // 0 or -1 (attribute call failed)
void launch_invert(hipStream_t s, const InvItem *items, int n_items, int n_max, int n_cu);
void launch_inv_gather(hipStream_t s, const InvItem *items, double *out, int ldo, int n);
void launch_set_target(const Batch &b, hipStream_t s, int64_t n_proposals);
// per-batch kernel attributes (dynamic LDS limits), once at creation; 0 or -1
int setup_propose(const Batch &b);
int setup_refine(const Batch &b);
// LDS of the proposal kernel: dynamic bytes for these options, and the bound
// on its static LDS that validation adds to them
size_t propose_lds_bytes(int kcap, int kmax, int n_cap);
constexpr size_t kProposeStaticLds = 8192;
constexpr size_t kLdsPerWorkgroup = 160 * 1024;   // gfx950

// Host-side view of a batch used by the launchers.
struct Batch {
  int32_t n_chains;
  int32_t kmax, kcap, n_cap, ld, nc_max, n_out_max, n_tau_max;
  int32_t n_mats, n_k_max;   // momentum / Matsubara measurement (n_mats = 0: off)
  int32_t precision;
  int32_t grid_per_chain;    // workgroups per chain for per-chain streaming kernels
  int32_t rankk_tile;        // rank-k output tile edge, 64 or 32
  int32_t pairs;             // 1: pair proposals are drawn (p_pair > 0)
  ChainDesc *d_desc;         // device [n_chains]
  ChainState *d_state;       // device [n_chains]
  ChainState *d_mstate;      // device [n_chains]: the state as the last block left it, read by
                             // the measurement, which runs beside the next block
  int32_t n_cu;
  // refinement: scratch pool for a group of chains, the group's items, drift partial sums
  double *r_pool;
  size_t r_pool_doubles;
  RefineItem *r_items;       // [n_chains]
  double *r_red;             // [refine_red_doubles(n_chains)]
  InvItem *r_inv;            // [2 n_chains] from-scratch elimination items
};

// Grid of a per-chain streaming kernel and its xcd_g argument (chain_block):
// XCD-aware one-dimensional for batches of 8 chains or more, (G, C) otherwise.
inline dim3 chain_grid(const Batch &b) {
  if (b.n_chains >= 8) return dim3(8u * b.grid_per_chain * ((b.n_chains + 7) / 8));
  return dim3(b.grid_per_chain, b.n_chains);
}
inline int chain_grid_arg(const Batch &b) { return b.n_chains >= 8 ? b.grid_per_chain : 0; }

}  // namespace ctaux
