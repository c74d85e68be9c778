// The inner loop of a block (Sec. IV B): k sequential insert / remove / flip
// proposals, each a spin change of one vertex of the augmented configuration.
//
// For a change of vertex p from spin s_old to s_new (block-start spin s0),
//   gh = exp(V(s_new) - V(s0)) - exp(V(s_old) - V(s0))        (per sector)
// Gamma (Eq. Gamma, repeated changes allowed) has the entries
// Gamma_ab = (G - I)_{P_a P_b} - delta_ab / gh_b with G the block-start Green's
// function.  The loop works with the column-scaled Gamma~ = Gamma D^{-1},
// D_b = e^{V_b} / (e^{V_b} - 1) for an old vertex P_b (block-start V) and 1 for
// a candidate: by Eq. (NfromG) the scaled old columns are plain entries of the
// augmented N, (G - I)_{i b} / D_b = (N_a - I)_{i b}, so Gamma~ has O(1) entries
// where Gamma's columns span factors e^{+-gamma} (whose cancellation in the
// update cost FP64 digits).  The new column and row are
//   s_a = Gamma_{P_a p} / D_p,  w_b = Gamma_{p P_b} / D_b,  d = Gamma_pp / D_p,
// and inversion by partitioning (Sec. III B 2) gives
//   beta~ = d - w^T Gamma~^{-1} s = beta / D_p,
//   det ratio of the sector = -gh * beta = -gh * D_p * beta~   (Eq. ratS);
// on acceptance Gamma~^{-1} grows by one row and column.  The N update uses
// (G - I)_{:,P} Gamma^{-1} = [(G - I)_{:,P} D^{-1}] Gamma~^{-1}.
//
// Repeated changes of one vertex within a block (the modification the paper
// asks for, Sec. III B): P holds every changed vertex once, with its net
// change gh = exp(V(s) - V(s0)) - 1 from the block-start spin.  A further
// change of a vertex in P (slot a) only replaces gh_a, i.e. the diagonal entry
// Gamma~_aa = (.)_pp - 1/(gh_a D_p), so the sector's determinant ratio is
//   (gh_new / gh_old) (1 + delta X_aa),  delta = (1/gh_old - 1/gh_new) / D_p,
// with X = Gamma~^{-1} (matrix determinant lemma), and on acceptance
// X <- X - delta/(1 + delta X_aa) X_{:,a} X_{a,:} (Sherman-Morrison).  A change
// back to the block-start spin (gh_new = 0) removes slot a: the ratio is
// X_aa / (-gh_old D_p) (the cofactor) and X loses row and column a by the
// Schur complement X_{-a,-a} - X_{-a,a} X_{a,-a} / X_aa.  Without this, a vertex
// changed twice contributes two almost equal columns to Gamma (condition
// numbers of 1e6 - 1e8), and the update loses FP64 digits.
// R = {K/(n+1), n/K, 1} * r_up * r_dn (Eq. insprob and Sec. II B); accept iff u < |R|.
//
// Below, Gamma stands for the column-scaled Gamma~.
//
// One workgroup (4 waves) per chain.  X = Gamma~^{-1} lives in registers:
// waves 0 and 2 hold the rows of the up and down sector's X (lane a: row a),
// waves 1 and 3 its columns (lane b: column b), zero beyond k_a.  Every wave
// gathers both s and w of its sector (one load each per lane, in flight
// together); a row wave forms v = X s and beta~ = d - w.v, a column wave
// u = X^T w, each from registers and its own vector read across lanes.  One
// barrier per proposal publishes the two sectors' beta~ (and v, u for the
// growth); it orders LDS only, so the global stores of the loop (the recorded
// Gamma entries, the decision log) stay in flight until the full barrier
// after the loop.  The growth after an acceptance is deferred to the next
// proposal with gathers, where it runs while those loads are in flight:
//   X' = [[X + v u^T / beta~, -v / beta~], [-u^T / beta~, 1 / beta~]]
//      = [[X, 0], [0, 0]] + (vt / beta~) ut^T,  vt = [v; -1], ut = [u; -1],
// a rank-1 update of the zero-padded X (the two copies round its terms in a
// different order; the row copy is the one written out, and a column copy
// that is read back from it takes its values).
// v, u and the beta~ are double-buffered by the parity of the proposals with
// gathers.  A repeated change (rare) and the end of the loop write the rows to
// LDS, where the code that follows works as before.  Bookkeeping that the next
// proposal reads (P, the spins) is written by every thread with the same value
// and each thread reads back only what it wrote itself or what precedes a
// barrier, so every wave selects the vertex of a removal or flip on its own.
//
// Everything the loop reads from the chain descriptor is copied to registers
// or LDS first: the loop stores to global memory, so reads through the
// descriptor could not be hoisted and would sit on the latency-critical path.
#include "ctaux_device.h"

namespace ctaux {

// Entry (i, j) of the column-scaled (G - I) D^{-1} of the augmented configuration
// (old vertices 0..n-1, candidates n..):
//   old column j:       (N_a - I)_ij, N_a,ij = N_ij (old row) or Rt_{i-n, j}
//   candidate column j: (G - I)_ij, G_ij = (N Z)_{i, j-n} (old row) or (X Y + G0nn)_{i-n, j-n}.

// Calls f with a compile-time even count of k-steps, the smallest that covers ns
// (ns <= 16: k_a <= 64).
template <int V>
struct StepCount {
  static constexpr int value = V;
};
template <typename F>
__device__ __forceinline__ void with_even_steps(int ns, F &f) {
  if (ns <= 2) f(StepCount<2>{});
  else if (ns <= 4) f(StepCount<4>{});
  else if (ns <= 6) f(StepCount<6>{});
  else if (ns <= 8) f(StepCount<8>{});
  else if (ns <= 10) f(StepCount<10>{});
  else if (ns <= 12) f(StepCount<12>{});
  else if (ns <= 14) f(StepCount<14>{});
  else f(StepCount<16>{});
}

// PAIRS: the instantiation that also takes pair proposals (p_pair > 0); their
// path is compiled only there, so that the loop without it keeps its register
// allocation.
template <typename T, bool PAIRS>
__global__ __launch_bounds__(256) void k_propose(const ChainDesc *descs, ChainState *states) {
  const int c = blockIdx.x;
  const ChainDesc &d = descs[c];
  ChainState &st = states[c];
  if (!st.active) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int sec = tid >> 7, loc = tid & 127;
  const int n = st.n, kins = st.k_ins, L = st.L;
  const int par = st.parity;
  const int64_t done0 = st.done;
  // descriptor fields used in the loop
  const int kcap = d.kcap, n_cap = d.n_cap, kmax = d.kmax, ld = d.ld;
  // LDS layout per sector: kp = 64 rows of lg = 65 entries whatever k_cap is, so
  // that every offset into the written-out X is a compile-time constant
  constexpr int kp = kMaxKcap, lg = kMaxKcap + 1;
  const double Kc = d.K, gtol = d.gamma_tol;
  const bool gz = (d.gamma == 0.0);
  const auto Nsec = gview(static_cast<const T *>(d.N[par][sec]));
  const auto Rts = gview(d.Rt[sec]), YTs = gview(d.YT[sec]), Gnns = gview(d.Gnn[sec]);
  const auto gam = gview_w(d.Gam[sec]);
  const auto log_acc = gview_w(d.log_acc);
  const auto log_R = gview_w(d.log_R);
  const int64_t log_cap = d.log_cap;

  extern __shared__ double smem[];
  double *Gi = smem;                         // [2][kp][lg]  X written out (repeated changes, block end)
  double *vs = Gi + 2 * kp * lg;             // [2][kp]   s vectors (row waves)
  double *vw = vs + 2 * kp;                  // [2][kp]   w vectors (column waves)
  double *vv = vw + 2 * kp;                  // [2][2][kp] v = X s, [parity][sector]
  double *vu = vv + 4 * kp;                  // [2][2][kp] u = X^T w
  int *P = reinterpret_cast<int *>(vu + 4 * kp);   // [kcap]
  int8_t *scur = reinterpret_cast<int8_t *>(P + kcap);  // [n + kmax] current spins
  int8_t *s0l = scur + (n_cap + kmax);                      // [n + kmax] block-start spins
  double *Gis = Gi + sec * kp * lg;
  __shared__ double sh_ev[2][5];                   // exp(gamma*sigma*d), d = -2..2
  __shared__ double sh_dsc[2][5];                  // D = e^V / (e^V - 1) for block-start spin d = +-1
  __shared__ double sh_igd[2][27];                 // 1 / (gh D) by (s0 + 1, s_old + 1, s_new + 1)
  __shared__ double sh_beta[2][2];                 // [parity][sector]
  __shared__ double sh_pr[2], sh_bt[2];            // pair proposals: sector ratio, beta~ of a new slot
  __shared__ double sh_S[2][4];                    // pair proposals: 2x2 Schur complement per sector
  __shared__ double sh_gh[2][kMaxKcap];
  __shared__ double sh_pacc[kMaxKmax], sh_ppick[kMaxKmax];
  __shared__ int8_t sh_ptype[kMaxKmax], sh_pspin[kMaxKmax];
  __shared__ int sh_bad, sh_nnew;
  __shared__ int sh_fallback[2];
  __shared__ unsigned sh_mx[4][3];                 // per wave: max|R|, max|Gamma|, max|X0| (high words)
  __shared__ int sh_perm[2][kMaxKcap];
  __shared__ int64_t sh_cid[kMaxKmax];

  int ka = 0, nchg = 0, ncur = n, ndead = 0, next_cand = 0;   // nchg: accepted changes (== ka unless U = 0)
  int64_t next_id = st.next_id, accepted = st.accepted;
  double sign = st.sign;
  int status = 0, L_eff = L;
  int64_t err_index = -1;
  // growth of Gamma^{-1} owed by the last accepted proposal: it runs while the
  // next proposal's gathers are in flight
  bool pend = false;
  int pk = 0;
  double pbeta = 1.0;
  bool had_repeat = false;   // an accepted repeated change rewrote Gamma~ (rebuilt at block end)

  // the written-out X (with the padding rows) and the vectors start at zero
  for (int i = tid; i < static_cast<int>(reinterpret_cast<double *>(P) - Gi); i += 256) Gi[i] = 0.0;
  for (int i = tid; i < n + kins; i += 256) {
    const int8_t v = (i < n) ? static_cast<int8_t>(d.s0[par][i]) : 0;
    scur[i] = v;
    s0l[i] = v;
  }
  if (tid == 0) {
    sh_bad = 0;
    sh_fallback[0] = 0;
    sh_fallback[1] = 0;
  }
  if (tid < 10) {
    const double e = d.evd[tid / 5][tid % 5];
    sh_ev[tid / 5][tid % 5] = e;
    sh_dsc[tid / 5][tid % 5] = (tid % 5 == 2) ? 1.0 : e / (e - 1.0);
  }
  if (tid >= 64 && tid < 64 + 54) {   // entries whose s_new equals s_old never occur in the loop
    const int sc = (tid - 64) / 27, e = (tid - 64) % 27;
    const int s0 = e / 9 - 1, so = (e / 3) % 3 - 1, sn = e % 3 - 1;
    const double ev_new = d.evd[sc][sn - s0 + 2], ev_old = d.evd[sc][so - s0 + 2];
    const double dv = (s0 == 0) ? 1.0 : d.evd[sc][s0 + 2] / (d.evd[sc][s0 + 2] - 1.0);
    sh_igd[sc][e] = (sn != so) ? 1.0 / ((ev_new - ev_old) * dv) : 0.0;
  }
  for (int t = tid; t < L; t += 256) {
    sh_ptype[t] = static_cast<int8_t>(d.ptype[t]);
    sh_pspin[t] = static_cast<int8_t>(d.pspin[t]);
    sh_pacc[t] = d.pacc[t];
    sh_ppick[t] = d.ppick[t];
  }
  __syncthreads();

  // The proposals' draws live in registers (proposal t in lane t % 64 of slot
  // t / 64) and are read with readlane; lane b of each wave holds P_b and the
  // b-th removed old vertex, and two 64-bit masks the live candidates.  The
  // loop then reads them without LDS round trips.
  double r_pacc[2], r_ppick[2];
  int r_tspin[2];   // type | (spin + 1) << 8
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int t = 64 * j + lane;
    r_pacc[j] = (t < L) ? sh_pacc[t] : 0.0;
    r_ppick[j] = (t < L) ? sh_ppick[t] : 0.0;
    r_tspin[j] = (t < L) ? (static_cast<int>(sh_ptype[t]) | ((static_cast<int>(sh_pspin[t]) + 1) << 8)) : 0;
  }
  int myP = 0, myDead = 0x7fffffff;

  // ---- X = Gamma~^{-1} in registers (row or column copy, see the top) ----
  const int role = wave & 1;   // 0: rows, 1: columns
  double xr[kMaxKcap];
#pragma unroll
  for (int i = 0; i < kMaxKcap; ++i) xr[i] = 0.0;
  double *bcast = (role == 0 ? vs : vw) + sec * kp;   // this wave's vector buffer (pair proposals)
  double myv = 0.0;   // v_a (rows) or u_b (columns) of the last proposal with gathers
  int q = 0;          // parity of the proposals with gathers
  int pq = 0;         // parity of the proposal whose growth is owed

  auto chunks = [&](const double *src, int nent, auto &&body) {
#pragma unroll
    for (int c = 0; c < kMaxKcap; c += 8) {
      if (c < nent) {
        double o[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = src[c + i];
        body(c, o);
      }
    }
  };
  // owed growth of X from k to k + 1 slots with Schur complement beta~ (the
  // vectors of the proposal of parity bq)
  auto growth = [&](int k, double beta, int bq) {
    const double ib = 1.0 / beta;
    const double mine = (lane < k) ? myv : (lane == k ? -1.0 : 0.0);
    const double *other = (role == 0 ? vu : vv) + (bq * 2 + sec) * kp;
    // rows: X_ab += (vt_a / beta~) ut_b; columns: X_ab += (ut_b / beta~) vt_a
    const double f = mine * ib;
    chunks(other, k + 1, [&](int c, const double *o) {
#pragma unroll
      for (int i = 0; i < 8; ++i) xr[c + i] = fma(f, o[i], xr[c + i]);
    });
  };
  // row a . s (rows) or column b . w (columns) over k entries, four
  // accumulators; the vector is held by the wave itself, entry b in lane b, and
  // read with readlane, eight entries at a time (no LDS round trip)
  auto matvec_lanes = [&](double vec, int k) -> double {
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < kMaxKcap; c += 8) {
      if (c < k) {
        double o[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = readlane_f64(vec, c + i);
#pragma unroll
        for (int i = 0; i < 8; ++i) a4[i & 3] = fma(xr[c + i], o[i], a4[i & 3]);
      }
    }
    return (a4[0] + a4[1]) + (a4[2] + a4[3]);
  };
  // the same from an LDS vector, and the rank-2 growth of a pair:
  // X_ab += f1 o1_b + f2 o2_b over the first nent entries
  auto matvec_from = [&](const double *src, int k) -> double {
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    chunks(src, k, [&](int c, const double *o) {
#pragma unroll
      for (int i = 0; i < 8; ++i) a4[i & 3] = fma(xr[c + i], o[i], a4[i & 3]);
    });
    return (a4[0] + a4[1]) + (a4[2] + a4[3]);
  };
  auto growth2 = [&](int nent, double f1, const double *o1, double f2, const double *o2) {
#pragma unroll
    for (int c = 0; c < kMaxKcap; c += 8) {
      if (c < nent) {
        double a[8], b[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          a[i] = o1[c + i];
          b[i] = o2[c + i];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) xr[c + i] = fma(f1, a[i], fma(f2, b[i], xr[c + i]));
      }
    }
  };
  // X to LDS (the rows; the LDS code of repeated changes and of the block end
  // reads it there) and back
  auto write_out = [&]() {
    if (role == 0) {
#pragma unroll
      for (int b = 0; b < kMaxKcap; ++b) Gis[lane * lg + b] = xr[b];
    }
  };
  auto read_back = [&]() {
    if (role == 0) {
      const double *row = Gis + lane * lg;
#pragma unroll
      for (int i = 0; i < kMaxKcap; ++i) xr[i] = row[i];
    } else {
      const double *col = Gis + lane;
#pragma unroll
      for (int i = 0; i < kMaxKcap; ++i) xr[i] = col[i * lg];
    }
  };
  // entry (i, j) of the block-start G - I, column-scaled (see the top)
  auto gat = [&](int gi, int gj) -> double {
    if (gj < n) return (gi < n) ? static_cast<double>(Nsec[static_cast<size_t>(gi) * ld + gj])
                                : Rts[static_cast<size_t>(gi - n) * ld + gj];
    return (gi < n) ? YTs[static_cast<size_t>(gj - n) * ld + gi]
                    : Gnns[static_cast<size_t>(gi - n) * kmax + (gj - n)];
  };

  // Accepted repeated change of slot a (k = k_a slots), on the X written out to
  // LDS: snapshots of X's column and row a (and of its last row and column) in
  // the vector buffers, then every thread rewrites the entries it owns (thread
  // (cp = loc % 32, rg = loc / 32) of the sector: columns 2cp, 2cp + 1 of rows
  // rg + 4i).  remove: slot a is deleted by the Schur complement and the last
  // slot takes its place (its row and column then zero, keeping the zero
  // padding beyond k_a); otherwise the Sherman-Morrison update of the diagonal
  // change.
  auto repeat_update = [&](int a, bool remove, double gn, double dp) {
    const int k = ka, last = ka - 1;
    double *cv = vv + sec * kp, *rv = vu + sec * kp, *lrw = vs + sec * kp, *lcl = vw + sec * kp;
    for (int i = loc; i < k; i += 128) {
      cv[i] = Gis[i * lg + a];
      rv[i] = Gis[a * lg + i];
      lrw[i] = Gis[last * lg + i];
      lcl[i] = Gis[i * lg + last];
    }
    const double xaa = Gis[a * lg + a], go = sh_gh[sec][a];
    lds_barrier();
    const int cp = loc & 31, rg = loc >> 5;
    if (!remove) {
      const double del = (1.0 / go - 1.0 / gn) / dp;
      const double coef = del / (1.0 + del * xaa);
      for (int r = rg; r < k; r += 4)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int c = 2 * cp + h2;
          if (c < k) Gis[r * lg + c] -= coef * cv[r] * rv[c];
        }
    } else {
      const double ixa = 1.0 / xaa;
      for (int r = rg; r < k; r += 4)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int c = 2 * cp + h2;
          if (c >= k) continue;
          double x = 0.0;
          if (r != last && c != last) {
            const int sr = (r == a) ? last : r, sc = (c == a) ? last : c;
            double base;
            if (sr == last && sc == last) base = lrw[last];
            else if (sr == last) base = lrw[sc];
            else if (sc == last) base = lcl[sr];
            else base = Gis[r * lg + c];
            x = base - cv[sr] * rv[sc] * ixa;
          }
          Gis[r * lg + c] = x;
        }
    }
    lds_barrier();
  };

  // One change of vertex p (spin s_old -> s_new) of a pair proposal, applied to
  // the X written out to LDS: multiplies sh_pr[sector] by the sector's
  // determinant ratio and leaves X, P, gh and ka as Gamma with the change has
  // them.  A vertex in P takes the repeated-change formulas (as above); any
  // other vertex a new slot by partitioning, with its s, w and d gathered here:
  // v = X s (threads 0-63 of the sector), u = X^T w (threads 64-127),
  // beta~ = d - w.v, ratio -gh D_p beta~, then X grows by the rank-1 form of
  // the inner loop.  The caller has checked that Gamma has room (ka < 64).
  auto lds_change = [&](int p, int s_old, int s_new) {
    int a = -1;
    for (int b = 0; b < ka; ++b)
      if (P[b] == p) {
        a = b;
        break;
      }
    if (a >= 0) {
      const int s0p = s0l[p];
      const double gh0 = sh_ev[0][s_new - s0p + 2] - 1.0, gh1 = sh_ev[1][s_new - s0p + 2] - 1.0;
      const double dp = sh_dsc[sec][s0p + 2], gn = sec == 0 ? gh0 : gh1;
      const bool remove = (s_new == s0p);
      if (loc == 0) {
        const double xaa = Gis[a * lg + a], go = sh_gh[sec][a];
        sh_pr[sec] *= remove ? xaa / (-go * dp) : (gn / go) * (1.0 + (1.0 / go - 1.0 / gn) / dp * xaa);
      }
      repeat_update(a, remove, gn, dp);   // its first barrier follows every read above
      if (!remove) {
        if (tid == 0) {
          sh_gh[0][a] = gh0;
          sh_gh[1][a] = gh1;
        }
      } else {
        const int last = ka - 1;
        if (a != last) {   // the last slot moves into slot a (every thread writes the same value)
          P[a] = P[last];
          if (tid == 0) {
            sh_gh[0][a] = sh_gh[0][last];
            sh_gh[1][a] = sh_gh[1][last];
          }
        }
        ka -= 1;
      }
      lds_barrier();
      return;
    }
    const int k = ka;
    const int s0p = s_old;   // outside P: the block-start spin (0 for a candidate)
    const double gh0 = sh_ev[0][s_new - s0p + 2] - 1.0, gh1 = sh_ev[1][s_new - s0p + 2] - 1.0;
    double *sv = vs + sec * kp, *wv = vw + sec * kp, *cv = vv + sec * kp, *rw = vu + sec * kp;
    if (loc < 64) {
      if (loc < k) sv[loc] = gat(P[loc], p);
    } else if (loc - 64 < k) {
      wv[loc - 64] = gat(p, P[loc - 64]);
    }
    lds_barrier();
    if (loc < 64) {
      double acc = 0.0;
      if (loc < k)
        for (int b = 0; b < k; ++b) acc = fma(Gis[loc * lg + b], sv[b], acc);
      cv[loc] = acc;
    } else {
      const int b = loc - 64;
      double acc = 0.0;
      if (b < k)
        for (int a2 = 0; a2 < k; ++a2) acc = fma(wv[a2], Gis[a2 * lg + b], acc);
      rw[b] = acc;
    }
    lds_barrier();
    if (loc < 64) {
      const double sum = wave_sum((loc < k) ? wv[loc] * cv[loc] : 0.0);
      if (loc == 0) {
        const double igd = sh_igd[sec][(s0p + 1) * 9 + (s_old + 1) * 3 + (s_new + 1)];   // 1 / (gh D_p)
        const double beta = gat(p, p) - 1.0 - igd - sum;
        sh_bt[sec] = beta;
        sh_pr[sec] *= -(sec == 0 ? gh0 : gh1) * sh_dsc[sec][s0p + 2] * beta;
      }
    }
    lds_barrier();
    const double ib = 1.0 / sh_bt[sec];
    // X' = [[X, 0], [0, 0]] + (vt / beta~) ut^T, vt = [v; -1], ut = [u; -1]; each
    // entry is read and written by one thread
    for (int e = loc; e < (k + 1) * (k + 1); e += 128) {
      const int r = e / (k + 1), c2 = e - r * (k + 1);
      const double vr = (r < k) ? cv[r] : -1.0, uc = (c2 < k) ? rw[c2] : -1.0;
      const double base = (r < k && c2 < k) ? Gis[r * lg + c2] : 0.0;
      Gis[r * lg + c2] = fma(vr * ib, uc, base);
    }
    P[k] = p;   // every thread writes the same value
    if (tid == 0) {
      sh_gh[0][k] = gh0;
      sh_gh[1][k] = gh1;
    }
    ka = k + 1;
    lds_barrier();
  };

  unsigned long long alive_lo = 0ull, alive_hi = 0ull;   // live candidates (bit j of candidates 0-63, 64-127)
  // the vertex of rank r among the interacting ones in canonical (augmented-index)
  // order, or -1; every wave computes it from the bookkeeping all threads wrote
  // identically (pair removals; the inner loop has its own copy of these lines,
  // which keeps the register allocation of the loop as it is without pairs)
  auto select_rank = [&](int r) -> int {
    if (r < n - ndead) {
      // old vertex: least idx with idx = r + #{dead <= idx}
      int idx = r;
      while (true) {
        const bool le = myDead <= idx;   // lanes past the list hold INT_MAX
        const int nw = r + __popcll(__ballot(le));
        if (nw == idx) break;
        idx = nw;
      }
      return idx;
    }
    // the r2-th live candidate in index order
    int r2 = r - (n - ndead);
    const int c0 = __popcll(alive_lo);
    const int wsel = (r2 < c0) ? 0 : 1;
    const unsigned long long m = wsel ? alive_hi : alive_lo;
    if (wsel == 1) r2 -= c0;
    const bool hitl = ((m >> lane) & 1ull) && __popcll(m & ((1ull << lane) - 1ull)) == r2;
    const unsigned long long hit = __ballot(hitl);
    return hit ? n + 64 * wsel + __ffsll(static_cast<long long>(hit)) - 1 : -1;
  };
  int why = 0;   // why the inner loop stopped: 1 capacity, 2 bookkeeping, 3 non-finite ratio, 4 Gamma full
  // The proposals run in an inner loop that handles insertions, removals and
  // flips of vertices outside P; a repeated change of a vertex in P, and a pair
  // proposal, leave it and are handled once below (X written out, updated in
  // LDS, read back), so that the inner loop keeps X in registers without those
  // paths' demands.
  int t = 0;
  while (t < L) {
    int rp = -1, p = -1, s_old = 0, s_new = 0, type = 0;
    double u_acc = 0.0, fpre = 0.0;
    for (; t < L; ++t) {
      const int tj = t >> 6, tl = t & 63;
      const int tspin = __builtin_amdgcn_readlane(tj ? r_tspin[1] : r_tspin[0], tl);
      type = tspin & 0xff;
      u_acc = readlane_f64(tj ? r_pacc[1] : r_pacc[0], tl);
      if (PAIRS && type >= 3) {
        why = 5;
        break;   // a pair proposal: handled after this loop
      }
      p = -1;
      s_old = 0;
      s_new = 0;
      int skip = 0;
      if (type == 0) {
        if (ncur + 1 > n_cap) {
          why = 1;
          break;
        }
        p = n + next_cand;
        s_new = (tspin >> 8) - 1;
      } else if (ncur == 0) {
        skip = 1;
      } else {
        // rank r among interacting vertices in canonical order (as select_rank)
        int r = static_cast<int>(floor(static_cast<double>(ncur) * readlane_f64(tj ? r_ppick[1] : r_ppick[0], tl)));
        if (r > ncur - 1) r = ncur - 1;
        if (r < n - ndead) {
          // old vertex: least idx with idx = r + #{dead <= idx}
          int idx = r;
          while (true) {
            const bool le = myDead <= idx;   // lanes past the list hold INT_MAX
            const int nw = r + __popcll(__ballot(le));
            if (nw == idx) break;
            idx = nw;
          }
          p = idx;
        } else {
          // the r2-th live candidate in index order
          int r2 = r - (n - ndead);
          const int c0 = __popcll(alive_lo);
          const int wsel = (r2 < c0) ? 0 : 1;
          const unsigned long long m = wsel ? alive_hi : alive_lo;
          if (wsel == 1) r2 -= c0;
          const bool hitl = ((m >> lane) & 1ull) && __popcll(m & ((1ull << lane) - 1ull)) == r2;
          const unsigned long long hit = __ballot(hitl);
          if (hit) p = n + 64 * wsel + __ffsll(static_cast<long long>(hit)) - 1;
        }
        if (p < 0 || p >= n + next_cand) {   // cannot happen unless bookkeeping is broken
          why = 2;
          break;
        }
      }

      // The gathers go out first; the spins, the liveness check and the
      // prefactor are worked out while they are in flight.
      double gh0 = 0.0, gh1 = 0.0, dp0 = 1.0, dp1 = 1.0;
      double raw_s, raw_w;   // set (and read) only on the path with gathers
      const bool gath = !skip && !gz;
      if (gath) {
        if (type != 0) {
          const unsigned long long hit = __ballot(lane < ka && myP == p);
          if (hit) rp = __ffsll(static_cast<long long>(hit)) - 1;   // a repeated change: handled after this loop
        }
        if (rp < 0) {
          // ---- issue the gathers: lane b < k_a takes s_b = G(P_b, p) and
          // w_b = G(p, P_b), lane 63 (never a slot while proposing) G_pp ----
          if constexpr (std::is_same<T, double>::value) {
            // every lane loads (lanes past k_a other than 63 take G_pp and drop
            // it): with i = P_b (or p) and j = p, the four blocks of the
            // augmented G are N[i][j], Rt[i-n][j], YT[j-n][i] and Gnn[i-n][j-n];
            // p decides (for the whole wave) which pair of blocks a gather
            // reads, i < n (per lane) which of the two
            const int gi = (lane < ka) ? myP : p;
            const bool ic = gi < n;
            const unsigned gl = static_cast<unsigned>(ic ? gi : gi - n);
            std::remove_const_t<decltype(Rts)> sb0, sb1, wb0, wb1;
            unsigned sm0, sm1, wm1;
            if (p < n) {
              sb0 = Nsec + p;                                    // N[i][p]
              sb1 = Rts + p;                                     // Rt[i-n][p]
              sm0 = ld;
              sm1 = ld;
              wb0 = Nsec + static_cast<size_t>(p) * ld;          // N[p][i]
              wb1 = YTs + p;                                     // YT[i-n][p]
              wm1 = ld;
            } else {
              sb0 = YTs + static_cast<size_t>(p - n) * ld;       // YT[p-n][i]
              sb1 = Gnns + (p - n);                              // Gnn[i-n][p-n]
              sm0 = 1;
              sm1 = kmax;
              wb0 = Rts + static_cast<size_t>(p - n) * ld;       // Rt[p-n][i]
              wb1 = Gnns + static_cast<size_t>(p - n) * kmax;    // Gnn[p-n][i-n]
              wm1 = 1;
            }
            raw_s = *((ic ? sb0 : sb1) + static_cast<uint64_t>(gl) * (ic ? sm0 : sm1));
            raw_w = *((ic ? wb0 : wb1) + static_cast<uint64_t>(gl) * (ic ? 1u : wm1));
          } else {
            int si = -1, sj = -1, wi = -1, wj = -1;
            if (lane < ka) {
              si = myP; sj = p; wi = p; wj = myP;
            } else if (lane == 63) {
              si = p; sj = p;
            }
            raw_s = (si >= 0) ? gat(si, sj) : 0.0;
            raw_w = (wi >= 0) ? gat(wi, wj) : 0.0;
          }
        }
      }
      if (type != 0 && !skip) {
        const int sc = scur[p];
        if (sc == 0) {   // cannot happen unless bookkeeping is broken
          why = 2;
          break;
        }
        s_old = sc;
        s_new = (type == 1) ? 0 : -s_old;
      }
      // prefactor of the acceptance ratio (Eq. insprob)
      fpre = (type == 0) ? Kc / static_cast<double>(ncur + 1)
                         : (type == 1 ? static_cast<double>(ncur) / Kc : 1.0);
      if (rp >= 0) break;
      if (gath) {
        // outside P an old vertex still has its block-start spin, a candidate 0
        const int s0p = s_old;
        gh0 = sh_ev[0][s_new - s0p + 2] - sh_ev[0][s_old - s0p + 2];
        gh1 = sh_ev[1][s_new - s0p + 2] - sh_ev[1][s_old - s0p + 2];
        dp0 = sh_dsc[0][s0p + 2];   // 1 for a candidate (s0 = 0)
        dp1 = sh_dsc[1][s0p + 2];
        // ---- owed growth of X (registers only) ----
        if (pend) {
          growth(pk, pbeta, pq);
          pend = false;
        }
        // ---- entries of Gamma~ (the raw entry minus the identity; P_b != p) ----
        const double igd = sh_igd[sec][(s0p + 1) * 9 + (s_old + 1) * 3 + (s_new + 1)];   // 1 / (gh D_p)
        const double dd = raw_s - 1.0 - igd;   // d, in lane 63
        const double sv = (lane < ka) ? raw_s : 0.0, wv = (lane < ka) ? raw_w : 0.0;
        // record row / column ka of Gamma~ for the inversion at block end (a
        // rejected proposal's entries are overwritten by the next one)
        if (role == 0) {
          if (lane < ka) gam[lane * kcap + ka] = sv;
          else if (lane == 63) gam[ka * kcap + ka] = dd;
        } else if (lane < ka) {
          gam[ka * kcap + lane] = wv;
        }
        myv = matvec_lanes((role == 0) ? sv : wv, ka);
        if (role == 0) {
          const double beta = readlane_f64(dd, 63) - wave_sum_dpp(wv * myv);
          if (lane == 0) sh_beta[q][sec] = beta;
        }
        double *mv = (role == 0 ? vv : vu) + (q * 2 + sec) * kp;
        mv[lane] = (lane == ka) ? -1.0 : myv;
        lds_barrier();
      }

      double R = 0.0;
      if (!skip) {
        double r0 = 1.0, r1 = 1.0;
        if (!gz) {
          r0 = -gh0 * dp0 * sh_beta[q][0];
          r1 = -gh1 * dp1 * sh_beta[q][1];
        }
        R = fpre * r0 * r1;
      }
      if (!isfinite(R)) {
        why = 3;
        break;
      }
      const int acc = (!skip && u_acc < fabs(R)) ? 1 : 0;
      if (tid == 0) {
        const int64_t idx = done0 + t;
        if (idx < log_cap) {
          log_acc[idx] = static_cast<uint8_t>(acc);
          log_R[idx] = R;
        }
      }
      if (acc) {
        accepted += 1;
        nchg += 1;
        if (R < 0.0) sign = -sign;
        if (!gz) {
          pend = true;
          pk = ka;
          pbeta = sh_beta[q][sec];
          pq = q;
          P[ka] = p;           // every thread writes the same value
          if (lane == ka) myP = p;
          if (tid == 0) {
            sh_gh[0][ka] = gh0;
            sh_gh[1][ka] = gh1;
          }
          ka += 1;
        }
        scur[p] = static_cast<int8_t>(s_new);   // every thread writes the same value
        if (type == 0) {
          const int j = p - n;
          if (j < 64) alive_lo |= 1ull << j;
          else alive_hi |= 1ull << (j - 64);
          if (tid == 0) sh_cid[next_cand] = next_id;
          next_id += 1;
          ncur += 1;
        } else if (type == 1) {
          ncur -= 1;
          if (p < n) {
            if (lane == ndead) myDead = p;
            ndead += 1;
          } else {
            const int j = p - n;
            if (j < 64) alive_lo &= ~(1ull << j);
            else alive_hi &= ~(1ull << (j - 64));
          }
        }
      }
      if (!skip && !gz) q ^= 1;
      if (type == 0) next_cand += 1;
      // with U = 0 there are no gather barriers; without one here a wave could run
      // ahead and overwrite spins another wave still has to read
      if (gz) lds_barrier();
      // Gamma full: the block ends here (with U = 0 the removed-vertex list, whose
      // length never exceeds that of P otherwise, bounds the block)
      if ((gz ? nchg : ka) == kcap) {
        why = 4;
        break;
      }
    }
    if constexpr (PAIRS) {
      if (why == 5) {
        // ---- a pair insertion (type 3) or removal (type 4) at proposal t ----
        why = 0;
        const int tj = t >> 6, tl = t & 63;
        // Gamma gains up to two slots: the block ends before a pair that could overfill it
        if ((gz ? nchg : ka) + 2 > kcap) {
          L_eff = t;
          break;
        }
        int pa0 = -1, pa1 = -1, so0 = 0, so1 = 0, sn0 = 0, sn1 = 0;
        bool skip = false;
        double fpre2 = 0.0;
        if (type == 3) {
          if (ncur + 2 > n_cap) {
            status = -5;   // CTAUX_ECAPACITY
            L_eff = t;
            err_index = done0 + t;
            break;
          }
          pa0 = n + next_cand;
          pa1 = pa0 + 1;
          sn0 = (__builtin_amdgcn_readlane(tj ? r_tspin[1] : r_tspin[0], tl) >> 8) - 1;
          sn1 = gview(d.pspin2)[t];
          fpre2 = Kc * Kc / (static_cast<double>(ncur + 1) * static_cast<double>(ncur + 2));
        } else if (ncur < 2) {
          skip = true;   // rejected, still counted
        } else {
          int r1 = static_cast<int>(floor(static_cast<double>(ncur) * readlane_f64(tj ? r_ppick[1] : r_ppick[0], tl)));
          if (r1 > ncur - 1) r1 = ncur - 1;
          int r2 = static_cast<int>(floor(static_cast<double>(ncur - 1) * gview(d.ppick2)[t]));
          if (r2 > ncur - 2) r2 = ncur - 2;
          if (r2 >= r1) r2 += 1;
          pa0 = select_rank(r1);
          pa1 = select_rank(r2);
          if (pa0 < 0 || pa0 >= n + next_cand || pa1 < 0 || pa1 >= n + next_cand || pa0 == pa1 || scur[pa0] == 0 ||
              scur[pa1] == 0) {   // cannot happen unless bookkeeping is broken
            status = -4;   // CTAUX_ENUMERIC
            L_eff = t;
            err_index = -3;
            break;
          }
          so0 = scur[pa0];
          so1 = scur[pa1];
          fpre2 = static_cast<double>(ncur) * static_cast<double>(ncur - 1) / (Kc * Kc);
        }
        const int ka0 = ka;
        // Both vertices outside P (every pair insertion; a pair removal of two
        // vertices unchanged in this block): the two new slots at once, from X
        // in registers.  With s1, w1 (s2, w2) the new column and row of the first
        // (second) vertex and the 2x2 corner of Gamma~,
        //   S = [[d1, G12], [G21, d2]] - [w1 w2]^T X [s1 s2]   (Schur complement),
        // the sector ratio is (-gh1 D1)(-gh2 D2) det S, and on acceptance
        //   X'' = [[X, 0], [0, 0]] + Vt S^{-1} Ut^T,  Vt = [[X s1, X s2], [-I]],
        //   Ut = [[X^T w1, X^T w2], [-I]]   (inversion by partitioning, two rows at once).
        // A rejected pair leaves X as it was.  Otherwise (a vertex in P) the LDS path
        // below applies the two changes in turn.
        const bool fresh = !skip && !gz && __ballot(lane < ka && (myP == pa0 || myP == pa1)) == 0ull;
        const bool lds_path = !skip && !gz && !fresh;
        int *Psv = reinterpret_cast<int *>(vu + 2 * kp);   // parity-1 vector buffers: free here
        double *ghsv = vv + 2 * kp;
        const auto xsv = gview_w(d.Rg[sec]);   // the residual's buffer, free until block end
        double R = skip ? 0.0 : fpre2;
        double rs1 = 0.0, rw1 = 0.0, rs2 = 0.0, rw2 = 0.0, m1 = 0.0, m2 = 0.0;
        if (fresh) {
          if (lane < ka) {
            rs1 = gat(myP, pa0);
            rw1 = gat(pa0, myP);
            rs2 = gat(myP, pa1);
            rw2 = gat(pa1, myP);
          }
          const double g00 = gat(pa0, pa0), g01 = gat(pa0, pa1), g10 = gat(pa1, pa0), g11 = gat(pa1, pa1);
          if (pend) {   // while the gathers are in flight
            growth(pk, pbeta, pq);
            pend = false;
          }
          lds_barrier();   // every wave's growth has read the vector buffers
          double *b1 = bcast, *b2 = (role == 0 ? vv : vu) + sec * kp;
          b1[lane] = role == 0 ? rs1 : rw1;
          b2[lane] = role == 0 ? rs2 : rw2;
          __builtin_amdgcn_wave_barrier();
          m1 = matvec_from(b1, ka);   // rows: (X s1)_a; columns: (X^T w1)_b
          m2 = matvec_from(b2, ka);
          __builtin_amdgcn_wave_barrier();   // the wave's reads of b1, b2 before it overwrites them
          b1[lane] = (lane == ka) ? -1.0 : m1;       // vt1 (rows), ut1 (columns)
          b2[lane] = (lane == ka + 1) ? -1.0 : m2;   // vt2, ut2
          if (role == 0) {
            const double t11 = wave_sum_dpp(rw1 * m1), t12 = wave_sum_dpp(rw1 * m2);
            const double t21 = wave_sum_dpp(rw2 * m1), t22 = wave_sum_dpp(rw2 * m2);
            if (lane == 0) {
              sh_S[sec][0] = g00 - 1.0 - sh_igd[sec][(so0 + 1) * 9 + (so0 + 1) * 3 + (sn0 + 1)] - t11;
              sh_S[sec][1] = g01 - t12;
              sh_S[sec][2] = g10 - t21;
              sh_S[sec][3] = g11 - 1.0 - sh_igd[sec][(so1 + 1) * 9 + (so1 + 1) * 3 + (sn1 + 1)] - t22;
              // Gamma~ entries of the two slots, for the inversion at block end
              // (a rejected pair's are overwritten later)
              gam[ka * kcap + ka] = g00 - 1.0 - sh_igd[sec][(so0 + 1) * 9 + (so0 + 1) * 3 + (sn0 + 1)];
              gam[ka * kcap + ka + 1] = g01;
              gam[(ka + 1) * kcap + ka] = g10;
              gam[(ka + 1) * kcap + ka + 1] = g11 - 1.0 - sh_igd[sec][(so1 + 1) * 9 + (so1 + 1) * 3 + (sn1 + 1)];
            }
            if (lane < ka) {
              gam[lane * kcap + ka] = rs1;
              gam[lane * kcap + ka + 1] = rs2;
            }
          } else if (lane < ka) {
            gam[ka * kcap + lane] = rw1;
            gam[(ka + 1) * kcap + lane] = rw2;
          }
          lds_barrier();
          double rr[2];
#pragma unroll
          for (int sc = 0; sc < 2; ++sc) {
            const double det = sh_S[sc][0] * sh_S[sc][3] - sh_S[sc][1] * sh_S[sc][2];
            const double f0 = -(sh_ev[sc][sn0 - so0 + 2] - 1.0) * sh_dsc[sc][so0 + 2];
            const double f1 = -(sh_ev[sc][sn1 - so1 + 2] - 1.0) * sh_dsc[sc][so1 + 2];
            rr[sc] = f0 * f1 * det;
          }
          R = fpre2 * rr[0] * rr[1];
        } else if (pend) {
          growth(pk, pbeta, pq);
          pend = false;
        }
        if (lds_path) {
          write_out();
          lds_barrier();   // also ends every read of the vector buffers by the growth
          // X, P and gh as they are, for a rejected pair (X goes to global memory;
          // both outcomes then read X back, so the registers need not hold it)
          for (int e = loc; e < ka0 * ka0; e += 128) xsv[e] = Gis[(e / ka0) * lg + e % ka0];
          for (int i = tid; i < ka0; i += 256) {
            Psv[i] = P[i];
            ghsv[i] = sh_gh[0][i];
            ghsv[kp + i] = sh_gh[1][i];
          }
          if (tid < 2) sh_pr[tid] = 1.0;
          __syncthreads();   // the saved X is visible to the whole workgroup
          lds_change(pa0, so0, sn0);
          lds_change(pa1, so1, sn1);
          R = fpre2 * sh_pr[0] * sh_pr[1];
          if (!(u_acc < fabs(R))) {   // rejected (or not finite): P, gh, ka and X as they were
            for (int i = tid; i < ka0; i += 256) {
              P[i] = Psv[i];
              sh_gh[0][i] = ghsv[i];
              sh_gh[1][i] = ghsv[kp + i];
            }
            ka = ka0;
            // the changes touched rows and columns below ka0 + 2 at most
            const int m = ka0 + 2 < kp ? ka0 + 2 : kp;
            for (int e = loc; e < m * m; e += 128) {
              const int r = e / m, c2 = e - r * m;
              Gis[r * lg + c2] = (r < ka0 && c2 < ka0) ? xsv[r * ka0 + c2] : 0.0;
            }
          }
          lds_barrier();
          // X back to registers within this branch: between write_out and here the
          // registers hold nothing live
          read_back();
          myP = (lane < ka) ? P[lane] : 0;
        }
        if (!isfinite(R)) {
          status = -4;   // CTAUX_ENUMERIC
          L_eff = t;
          err_index = done0 + t;
          break;
        }
        const int acc = (!skip && u_acc < fabs(R)) ? 1 : 0;
        if (tid == 0) {
          const int64_t idx = done0 + t;
          if (idx < log_cap) {
            log_acc[idx] = static_cast<uint8_t>(acc);
            log_R[idx] = R;
          }
        }
        if (acc) {
          accepted += 1;
          nchg += 2;
          if (R < 0.0) sign = -sign;
          if (lds_path) had_repeat = true;   // Gamma~ is gathered again at block end
          if (fresh) {
            const double S0 = sh_S[sec][0], S1 = sh_S[sec][1], S2 = sh_S[sec][2], S3 = sh_S[sec][3];
            const double id = 1.0 / (S0 * S3 - S1 * S2);
            const double i00 = S3 * id, i01 = -S1 * id, i10 = -S2 * id, i11 = S0 * id;   // S^{-1}
            const double e1 = (lane == ka) ? -1.0 : m1, e2 = (lane == ka + 1) ? -1.0 : m2;
            if (role == 0) {   // row a: X''_ab += (vt_a S^{-1})_j ut_j,b
              growth2(ka + 2, e1 * i00 + e2 * i10, vw + sec * kp, e1 * i01 + e2 * i11, vu + sec * kp);
            } else {           // column b: X''_ab += vt_i,a (S^{-1} ut_b)_i
              growth2(ka + 2, i00 * e1 + i01 * e2, vs + sec * kp, i10 * e1 + i11 * e2, vv + sec * kp);
            }
            P[ka] = pa0;   // every thread writes the same values
            P[ka + 1] = pa1;
            if (lane == ka) myP = pa0;
            if (lane == ka + 1) myP = pa1;
            if (tid == 0) {
#pragma unroll
              for (int sc = 0; sc < 2; ++sc) {
                sh_gh[sc][ka] = sh_ev[sc][sn0 - so0 + 2] - 1.0;
                sh_gh[sc][ka + 1] = sh_ev[sc][sn1 - so1 + 2] - 1.0;
              }
            }
            ka += 2;
          }
          scur[pa0] = static_cast<int8_t>(sn0);   // every thread writes the same value
          scur[pa1] = static_cast<int8_t>(sn1);
          if (type == 3) {
  #pragma unroll
            for (int i = 0; i < 2; ++i) {
              const int j = pa0 - n + i;
              if (j < 64) alive_lo |= 1ull << j;
              else alive_hi |= 1ull << (j - 64);
              if (tid == 0) sh_cid[j] = next_id + i;
            }
            next_id += 2;
            ncur += 2;
          } else {
  #pragma unroll
            for (int i = 0; i < 2; ++i) {
              const int pi = i ? pa1 : pa0;
              if (pi < n) {
                if (lane == ndead) myDead = pi;
                ndead += 1;
              } else {
                const int j = pi - n;
                if (j < 64) alive_lo &= ~(1ull << j);
                else alive_hi &= ~(1ull << (j - 64));
              }
            }
            ncur -= 2;
          }
        }
        if (type == 3) next_cand += 2;
        lds_barrier();   // the bookkeeping above before the next proposal reads it
        ++t;
        if ((gz ? nchg : ka) >= kcap) {   // Gamma full: the block ends here
          L_eff = t;
          break;
        }
        continue;
      }
    }
    if (why != 0) {
      L_eff = (why == 4) ? t + 1 : t;
      if (why != 4) {
        status = (why == 1) ? -5 : -4;   // CTAUX_ECAPACITY, CTAUX_ENUMERIC
        err_index = (why == 2) ? -3 : done0 + t;
      }
      break;
    }
    if (rp < 0) break;

    // ---- a repeated change of slot rp at proposal t (a removal or a flip) ----
    {
      const int s0p = s0l[p];
      // net change from the block-start spin
      const double gh0 = sh_ev[0][s_new - s0p + 2] - 1.0, gh1 = sh_ev[1][s_new - s0p + 2] - 1.0;
      const double dp0 = sh_dsc[0][s0p + 2], dp1 = sh_dsc[1][s0p + 2];
      if (pend) {
        growth(pk, pbeta, pq);
        pend = false;
      }
      write_out();
      lds_barrier();
      if (loc == 0) {   // the sector ratio from X_aa
        const double xaa = Gis[rp * lg + rp], go = sh_gh[sec][rp];
        const double gn = sec == 0 ? gh0 : gh1, dp = sec == 0 ? dp0 : dp1;
        sh_beta[q][sec] = (s_new == s0p) ? xaa / (-go * dp)
                                         : (gn / go) * (1.0 + (1.0 / go - 1.0 / gn) / dp * xaa);
      }
      lds_barrier();
      const double R = fpre * sh_beta[q][0] * sh_beta[q][1];
      if (!isfinite(R)) {
        status = -4;  // CTAUX_ENUMERIC
        L_eff = t;
        err_index = done0 + t;
        break;
      }
      const int acc = (u_acc < fabs(R)) ? 1 : 0;
      if (tid == 0) {
        const int64_t idx = done0 + t;
        if (idx < log_cap) {
          log_acc[idx] = static_cast<uint8_t>(acc);
          log_R[idx] = R;
        }
      }
      if (acc) {
        accepted += 1;
        nchg += 1;
        if (R < 0.0) sign = -sign;
        had_repeat = true;
        repeat_update(rp, s_new == s0p, sec == 0 ? gh0 : gh1, sec == 0 ? dp0 : dp1);
        if (s_new != s0p) {
          if (tid == 0) {
            sh_gh[0][rp] = gh0;
            sh_gh[1][rp] = gh1;
          }
        } else {
          // slot rp is removed: the last slot moves into it (every thread writes the same values)
          const int last = ka - 1, pl = P[last];
          if (rp != last) {
            P[rp] = pl;
            if (lane == rp) myP = pl;
            if (tid == 0) {
              sh_gh[0][rp] = sh_gh[0][last];
              sh_gh[1][rp] = sh_gh[1][last];
            }
          }
          ka -= 1;
        }
        scur[p] = static_cast<int8_t>(s_new);   // every thread writes the same value
        if (type == 1) {
          ncur -= 1;
          if (p < n) {
            if (lane == ndead) myDead = p;
            ndead += 1;
          } else {
            const int j = p - n;
            if (j < 64) alive_lo &= ~(1ull << j);
            else alive_hi &= ~(1ull << (j - 64));
          }
        }
      }
      read_back();   // X as written out and, on acceptance, updated
      q ^= 1;
      ++t;
    }
  }
  __syncthreads();
  // the growth owed by the last acceptance; X then goes to LDS, the starting
  // point of the refinement below
  if (pend) growth(pk, pbeta, pq);
  write_out();
  lds_barrier();
  // Gamma~ as recorded while proposing is stale once a repeated change rewrote
  // a slot: gather it again for the final P and net changes
  if (had_repeat && ka > 0) {
    for (int e = loc; e < ka * ka; e += 128) {
      const int a = e / ka, b = e - a * ka;
      const int pa = P[a], pb = P[b];
      double raw;
      if (pb < n) raw = (pa < n) ? static_cast<double>(Nsec[static_cast<size_t>(pa) * ld + pb])
                                 : Rts[static_cast<size_t>(pa - n) * ld + pb];
      else raw = (pa < n) ? YTs[static_cast<size_t>(pb - n) * ld + pa]
                          : Gnns[static_cast<size_t>(pa - n) * kmax + (pb - n)];
      double v = raw - (a == b ? 1.0 : 0.0);
      if (a == b) v -= 1.0 / (sh_gh[sec][b] * sh_dsc[sec][s0l[pb] + 2]);
      gam[a * kcap + b] = v;
    }
  }
  __syncthreads();

  if (wave == 1) {
    // ---- compaction map: interacting vertices in augmented order (one wave,
    // ballot scan over the spins in LDS).  The times, sites and ids follow the
    // map in k_operands, whose wide grid copies them off this kernel's path;
    // the ids given to accepted candidates go out in cid ----
    const int na = n + kins;
    int32_t *s0_n = d.s0[par ^ 1];
    int *map = d.map;
    int running = 0;
    for (int base = 0; base < na; base += 64) {
      const int i = base + lane;
      const int sv = i < na ? static_cast<int>(scur[i]) : 0;
      const unsigned long long m = __ballot(sv != 0);
      if (sv != 0) {
        const int pos = running + __popcll(m & ((1ull << lane) - 1ull));
        map[pos] = i;
        s0_n[pos] = sv;
      }
      running += __popcll(m);
    }
    for (int j = lane; j < kins; j += 64) d.cid[j] = sh_cid[j];
    if (lane == 0) sh_nnew = running;
  }
  if (ka > 0) {
    // ---- Gamma^{-1} for the rank-k update ----
    // The ratios above came from the unpivoted growth, whose inverse X0 loses
    // accuracy when an intermediate Schur complement of Gamma is small
    // (repeated changes of one vertex give condition numbers of 1e6-1e8).  The
    // residual R = I - Gamma X0 on the recorded Gamma decides:
    //  * max|R_ij| > gamma_tol: Gamma^{-1} comes from an in-place Gauss-Jordan
    //    elimination with partial pivoting of the recorded Gamma;
    //  * max|R_ij| above the FP64 rounding floor of the residual itself,
    //    rho = 16 k_a eps max|Gamma| max|X0|: one Newton step X1 = X0 + X0 R
    //    makes X0 accurate to |R|^2 + rounding;
    //  * otherwise X0 is used as it is: a Newton step would add rounding of
    //    order rho |X0| (on strongly coupled models Gamma^{-1} has entries of
    //    1e6 that the update cancels, and that rounding then dominates N's error).
    // Two waves per sector (waves 0, 1: up; 2, 3: down; wave 1 has built the
    // compaction map first).  The products run on MFMA 16x16x4 tiles: wave h of
    // a sector takes the residual's row tiles and the Newton step's column tiles
    // h and h + 2, with their global operands loaded up front; the number of
    // k-steps is a compile-time count of at least k_a / 4 (the steps beyond k_a
    // add exact zeros).  The elimination runs on the sector's first wave, lane r
    // owning row r.
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int h = wave & 1;
    const int nt = (ka + 15) >> 4, lr = lane & 15, lk = lane >> 4;
    const auto Rg = gview_w(d.Rg[sec]);
    const auto gi = gview_w(d.Ginv[sec]);
    bool bad = false;
    double rmax = 0.0, gmax = 0.0, xmax = 0.0;
    auto residual = [&](auto nsc) {
      constexpr int NS = decltype(nsc)::value;
      double a[2][NS];   // Gamma[16 ti + lr][4 s4 + lk], ti = h, h + 2
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int row = (h + 2 * u) * 16 + lr;
#pragma unroll
        for (int s4 = 0; s4 < NS; ++s4) {
          const int k = 4 * s4 + lk;
          a[u][s4] = (row < ka && k < ka) ? gam[row * kcap + k] : 0.0;
          gmax = fmax(gmax, fabs(a[u][s4]));
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int ti = h + 2 * u;
        if (ti >= nt) break;
        for (int tj = 0; tj < nt; ++tj) {
          const int col = tj * 16 + lr;
          v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < NS; ++s4) {
            const int k = 4 * s4 + lk;
            const double b = (k < ka && col < ka) ? Gis[k * lg + col] : 0.0;
            if (ti == 0) xmax = fmax(xmax, fabs(b));   // tile row 0 reads all of X0
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][s4], b, acc, 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = ti * 16 + lk + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
            if (r < ka && col < ka) {
              const double x = (r == col ? 1.0 : 0.0) - acc[q];
              Rg[r * kcap + col] = x;
              const double ax = fabs(x);
              rmax = (ax != ax) ? INFINITY : (ax > rmax ? ax : rmax);
            }
          }
        }
      }
    };
    auto newton_step = [&](auto nsc) {
      constexpr int NS = decltype(nsc)::value;
      double b[2][NS];   // R[4 s4 + lk][16 tj + lr], tj = h, h + 2
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int col = (h + 2 * u) * 16 + lr;
#pragma unroll
        for (int s4 = 0; s4 < NS; ++s4) {
          const int k = 4 * s4 + lk;
          b[u][s4] = (k < ka && col < ka) ? Rg[k * kcap + col] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tj = h + 2 * u;
        if (tj >= nt) break;
        const int col = tj * 16 + lr;
        for (int ti = 0; ti < nt; ++ti) {
          const int row = ti * 16 + lr;
          v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < NS; ++s4) {
            const int k = 4 * s4 + lk;
            const double a = (row < ka && k < ka) ? Gis[row * lg + k] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[u][s4], acc, 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = ti * 16 + lk + 4 * q;
            if (r < ka && col < ka) {
              const double x = Gis[r * lg + col] + acc[q];
              bad |= !isfinite(x);
              gi[r * kcap + col] = x;
            }
          }
        }
      }
    };
    const int ns = (ka + 3) >> 2;   // k-steps of four
    with_even_steps(ns, residual);
    // maxima of the sector's two waves (high words of non-negative doubles order
    // like the values); the barrier also publishes R to the other wave
    {
      const unsigned mr = wave_max_u32(static_cast<unsigned>(__double_as_longlong(rmax) >> 32));
      const unsigned mg = wave_max_u32(static_cast<unsigned>(__double_as_longlong(gmax) >> 32));
      const unsigned mx = wave_max_u32(static_cast<unsigned>(__double_as_longlong(xmax) >> 32));
      if (lane == 0) {
        sh_mx[wave][0] = mr;
        sh_mx[wave][1] = mg;
        sh_mx[wave][2] = mx;
      }
    }
    __syncthreads();
    const int w0 = wave & ~1;
    const unsigned rhi = max(sh_mx[w0][0], sh_mx[w0 + 1][0]);
    const bool growth_ok = gtol >= 0.0 && rhi <= static_cast<unsigned>(__double_as_longlong(gtol) >> 32);
    // rounding floor (maxima to within a factor 2 from the high words; NaN/inf in
    // Gamma or X0 already make rmax infinite)
    const double gm = __longlong_as_double(static_cast<long long>(max(sh_mx[w0][1], sh_mx[w0 + 1][1])) << 32);
    const double xm = __longlong_as_double(static_cast<long long>(max(sh_mx[w0][2], sh_mx[w0 + 1][2])) << 32);
    const double rho = 16.0 * ka * 2.220446049250313e-16 * gm * xm;
    const bool newton = growth_ok && __longlong_as_double(static_cast<long long>(rhi) << 32) > rho;
    if (growth_ok && !newton) {
      for (int e = loc; e < ka * ka; e += 128) {
        const int r = e / ka, col = e - r * ka;
        const double x = Gis[r * lg + col];
        bad |= !isfinite(x);
        gi[r * kcap + col] = x;
      }
    } else if (newton) {
      with_even_steps(ns, newton_step);
    } else if (h == 0) {
      if (lane == 0) sh_fallback[sec] = 1;
      double *A = Gis;   // the growth inverse is no longer needed
      // Gamma was written by this workgroup before the full barrier after the
      // loop (workgroup-scope visibility); all loads are issued before the first store
      for (int r0 = 0; r0 < ka; r0 += 16) {
        double g[16];
  #pragma unroll
        for (int i = 0; i < 16; ++i) g[i] = (r0 + i < ka && lane < ka) ? gam[(r0 + i) * kcap + lane] : 0.0;
  #pragma unroll
        for (int i = 0; i < 16; ++i)
          if (r0 + i < ka && lane < ka) A[(r0 + i) * lg + lane] = g[i];
      }
      __builtin_amdgcn_wave_barrier();
      const bool mine = lane < ka;
      double *row = A + lane * lg;
      bool used = false;
      int mypos = 0;
      double f = mine ? row[0] : 0.0;   // this row's entry in the pivot column
      for (int col = 0; col < ka; ++col) {
        // pivot: largest |A[r][col]| among unused rows; the high word of |x| orders
        // like |x| to 13 mantissa bits, bit 6 marks a candidate, bits 0-5 carry the row
        unsigned key = 0u;
        if (mine && !used) {
          const unsigned hi = static_cast<unsigned>(__double_as_longlong(fabs(f)) >> 32);
          key = (hi & ~127u) | 64u | static_cast<unsigned>(lane);
        }
        const int p = static_cast<int>(wave_max_u32(key) & 63u);   // uniform
        const double ip = 1.0 / readlane_f64(f, p);
        const bool piv = (lane == p);
        if (lane == 0) sh_perm[sec][col] = p;
        if (piv) {
          used = true;
          mypos = col;
        }
        // pivot row: A[p][j] *= ip, A[p][col] = ip; other rows: A[r][j] -= f ip A[p][j],
        // A[r][col] = -f ip
        const double scale = piv ? ip : 1.0;
        const double fi = piv ? 0.0 : f * ip;
        const double xc = piv ? ip : -fi;
        const double *prow = A + p * lg;
        // entry of the next pivot column, from the values before this step
        double fnext = 0.0;
        if (mine && col + 1 < ka) fnext = row[col + 1] * scale - fi * prow[col + 1];
        if (mine) {
          int j1 = 0;
          for (; j1 + 16 <= ka; j1 += 16) {   // full batches: loads in flight together, then stores
            double rv[16], pr[16];
  #pragma unroll
            for (int i = 0; i < 16; ++i) {
              rv[i] = row[j1 + i];
              pr[i] = prow[j1 + i];
            }
  #pragma unroll
            for (int i = 0; i < 16; ++i) row[j1 + i] = (j1 + i == col) ? xc : rv[i] * scale - fi * pr[i];
          }
          if (j1 < ka) {   // last partial batch; loads clamped to the row
            double rv[16], pr[16];
  #pragma unroll
            for (int i = 0; i < 16; ++i) {
              const int j = min(j1 + i, ka - 1);
              rv[i] = row[j];
              pr[i] = prow[j];
            }
  #pragma unroll
            for (int i = 0; i < 16; ++i)
              if (j1 + i < ka) row[j1 + i] = (j1 + i == col) ? xc : rv[i] * scale - fi * pr[i];
          }
        }
        f = fnext;
        __builtin_amdgcn_wave_barrier();
      }
      // store Gamma^{-1}: row pos(r) of the inverse is row r of A with column m
      // moved to column perm[m]
      if (mine) {
        for (int m = 0; m < ka; ++m) {
          const double x = row[m];
          bad |= !isfinite(x);
          gi[mypos * kcap + sh_perm[sec][m]] = x;
        }
      }
    }
    if (__ballot(bad) != 0ull && lane == 0) sh_bad = 1;   // singular Gamma
  }
  __syncthreads();
  if (sh_bad && status == 0) {
    status = -4;
    err_index = -4;
  }
  // ---- P and gh for the rank-k update (Gamma itself was recorded on acceptance) ----
  for (int a = tid; a < ka; a += 256) {
    d.P[a] = P[a];
    d.ghat[0][a] = sh_gh[0][a];
    d.ghat[1][a] = sh_gh[1][a];
  }
  if (tid == 0) {
    st.k_a = ka;
    st.n_new = sh_nnew;
    st.L_eff = L_eff;
    st.sign = sign;
    st.next_id = next_id;
    st.accepted = accepted;
    st.gj_fallbacks += sh_fallback[0] + sh_fallback[1];
    if (status != 0) {   // never clears a status set elsewhere (a refinement between blocks)
      st.status = status;
      st.err_index = err_index;
    }
    if (sh_nnew != ncur && status == 0) {
      st.status = -4;
      st.err_index = -2;   // bookkeeping mismatch
    }
  }
}

// LDS: X of both sectors written out as 64 rows of 65 entries, the s and w
// vectors, v and u by parity, P and the current and block-start spins.
size_t propose_lds_bytes(int kcap, int kmax, int n_cap) {
  const size_t kp = kMaxKcap;
  return sizeof(double) * (2 * kp * (kp + 1) + 12 * kp) + sizeof(int) * static_cast<size_t>(kcap) +
         2ull * static_cast<size_t>(n_cap + kmax) + 16;
}

static size_t propose_lds_bytes(const Batch &b) { return propose_lds_bytes(b.kcap, b.kmax, b.n_cap); }

// Dynamic LDS limits are set once per batch: the call costs host time that would
// otherwise sit between the launches of every block.  Returns -1 if the runtime
// refuses the size (the options were validated against the LDS of a workgroup,
// so this signals a device that has less).
int setup_propose(const Batch &b) {
  const int lds = static_cast<int>(propose_lds_bytes(b));
  const void *fns[4] = {reinterpret_cast<const void *>(k_propose<double, false>),
                        reinterpret_cast<const void *>(k_propose<float, false>),
                        reinterpret_cast<const void *>(k_propose<double, true>),
                        reinterpret_cast<const void *>(k_propose<float, true>)};
  for (const void *f : fns) {
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) return -1;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) != hipSuccess || fa.sharedSizeBytes > kProposeStaticLds) return -1;
  }
  return 0;
}

void launch_propose(const Batch &b, hipStream_t s) {
  const size_t lds = propose_lds_bytes(b);
  const dim3 grid(b.n_chains), block(256);
  if (b.precision == kFP64) {
    if (b.pairs) hipLaunchKernelGGL((k_propose<double, true>), grid, block, lds, s, b.d_desc, b.d_state);
    else hipLaunchKernelGGL((k_propose<double, false>), grid, block, lds, s, b.d_desc, b.d_state);
  } else {
    if (b.pairs) hipLaunchKernelGGL((k_propose<float, true>), grid, block, lds, s, b.d_desc, b.d_state);
    else hipLaunchKernelGGL((k_propose<float, false>), grid, block, lds, s, b.d_desc, b.d_state);
  }
}

}  // namespace ctaux
