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
// One workgroup (4 waves) per chain; Gamma^{-1} of both sectors lives in LDS.
// Threads 0..127 serve the up sector, 128..255 the down sector.
//
// Synchronisation: two barriers per proposal (after the gathers, after
// Gamma^{-1} s and w^T Gamma^{-1}); they also keep the waves within one
// proposal of each other.  They order LDS only: the global stores of the loop
// (the recorded Gamma entries, the decision log) are read only after the
// full barrier that ends the loop, so they stay in flight.  Bookkeeping that the next proposal reads
// (P, the spins, the removed list) is written by every thread with the same
// value and each thread reads back only what it wrote itself or what precedes
// a barrier, so every wave selects the vertex of a removal or flip on its own;
// the per-proposal scalars are double-buffered by proposal parity.  The
// growth of Gamma^{-1} after an acceptance is deferred to the next proposal and
// runs while that proposal's gathers are in flight.
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

template <typename T>
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
  // LDS layout per sector: k_cap rounded up to 8 (kp) rows of lg = kp + 1 entries
  const int kp = (kcap + 7) & ~7, lg = kp + 1;
  const double Kc = d.K, gtol = d.gamma_tol;
  const bool gz = (d.gamma == 0.0);
  const auto Nsec = gview(static_cast<const T *>(d.N[par][sec]));
  const auto Rts = gview(d.Rt[sec]), YTs = gview(d.YT[sec]), Gnns = gview(d.Gnn[sec]);
  const auto gam = gview_w(d.Gam[sec]);
  const auto log_acc = gview_w(d.log_acc);
  const auto log_R = gview_w(d.log_R);
  const int64_t log_cap = d.log_cap;

  extern __shared__ double smem[];
  double *Gi = smem;                         // [2][kp][lg]
  double *vs = Gi + 2 * kp * lg;             // [2][kp]   s vectors
  double *vw = vs + 2 * kp;                  // [2][kp]   w vectors
  double *vv = vw + 2 * kp;                  // [2][kp]   Gamma^{-1} s
  double *vu = vv + 2 * kp;                  // [2][kp]   w^T Gamma^{-1}
  int *P = reinterpret_cast<int *>(vu + 2 * kp);   // [kcap]
  int8_t *scur = reinterpret_cast<int8_t *>(P + kcap);  // [n + kmax] current spins
  int8_t *s0l = scur + (n_cap + kmax);                      // [n + kmax] block-start spins
  int8_t *slot_of = s0l + (n_cap + kmax);                   // [n + kmax] slot of a vertex in P (-1: none)
  double *Gis = Gi + sec * kp * lg;
  __shared__ double sh_ev[2][5];                   // exp(gamma*sigma*d), d = -2..2
  __shared__ double sh_dsc[2][5];                  // D = e^V / (e^V - 1) for block-start spin d = +-1
  __shared__ double sh_gpp[2][2], sh_beta[2][2];   // [proposal parity][sector]
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

  // Gamma^{-1} of both sectors (with the padding rows) and the s, w vectors start
  // at zero: entries beyond k_a stay zero for the whole block, so the
  // matrix-vector products below can read whole batches of 8 without masks.
  for (int i = tid; i < static_cast<int>(vv - Gi); i += 256) Gi[i] = 0.0;
  for (int i = tid; i < n + kins; i += 256) {
    const int8_t v = (i < n) ? static_cast<int8_t>(d.s0[par][i]) : 0;
    scur[i] = v;
    s0l[i] = v;
    slot_of[i] = -1;
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
  for (int t = tid; t < L; t += 256) {
    sh_ptype[t] = static_cast<int8_t>(d.ptype[t]);
    sh_pspin[t] = static_cast<int8_t>(d.pspin[t]);
    sh_pacc[t] = d.pacc[t];
    sh_ppick[t] = d.ppick[t];
  }
  __syncthreads();

  // The proposals' draws live in registers (proposal t in lane t % 64 of slot
  // t / 64) and are read with readlane; lane b of each wave holds P_b and the
  // b-th removed old vertex.  The loop then reads them without LDS round trips.
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

  // Gamma^{-1} of size k grows to k + 1 after an acceptance with Schur
  // complement beta, from v = Gamma^{-1} s and u = w^T Gamma^{-1}:
  //   [[X + v u^T / beta, -v / beta], [-u^T / beta, 1 / beta]].
  // Thread (cp = loc % 32, rg = loc / 32) of the sector owns columns 2cp, 2cp+1
  // (adjacent doubles: paired LDS accesses) of rows rg + 4i; batches of four
  // rows are loaded before they are stored.  Load addresses are clamped into the
  // matrix and values beyond k never used, so the loads need no branch.
  auto grow = [&](int k, double beta) {
    const double ib = 1.0 / beta;
    const double *v = vv + sec * kp, *u = vu + sec * kp;
    const int cp = loc & 31, rg = loc >> 5, b0 = 2 * cp, b1 = b0 + 1;
    if (b0 <= k) {
      const double ub0 = (b0 < k) ? u[b0] * ib : 0.0;
      const double ub1 = (b1 < k) ? u[b1] * ib : 0.0;
      for (int a1 = rg; a1 <= k; a1 += 16) {
        double va[4], g0[4], g1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ac = min(a1 + 4 * i, kcap - 1);
          va[i] = v[ac];
          g0[i] = Gis[ac * lg + b0];
          g1[i] = Gis[ac * lg + b1];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = a1 + 4 * i;
          if (a <= k) {
            Gis[a * lg + b0] = (a < k) ? ((b0 < k) ? g0[i] + va[i] * ub0 : -va[i] * ib) : ((b0 < k) ? -ub0 : ib);
            if (b1 <= k)
              Gis[a * lg + b1] = (a < k) ? ((b1 < k) ? g1[i] + va[i] * ub1 : -va[i] * ib) : ((b1 < k) ? -ub1 : ib);
          }
        }
      }
    }
  };

  // Accepted repeated change of slot a (k = k_a slots): snapshots of X's column
  // and row a (and of its last row and column) in the vector buffers, then every
  // thread rewrites the entries it owns in grow's layout.  remove: slot a is
  // deleted by the Schur complement and the last slot takes its place (its row
  // and column then zero, keeping the zero padding beyond k_a); otherwise the
  // Sherman-Morrison update of the diagonal change.
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

  for (int t = 0; t < L; ++t) {
    const int tp = t & 1, tj = t >> 6, tl = t & 63;
    const int tspin = __builtin_amdgcn_readlane(tj ? r_tspin[1] : r_tspin[0], tl);
    const int type = tspin & 0xff;
    const double u_acc = readlane_f64(tj ? r_pacc[1] : r_pacc[0], tl);
    int p = -1, s_old = 0, s_new = 0, skip = 0;
    if (type == 0) {
      if (ncur + 1 > n_cap) {
        status = -5;  // CTAUX_ECAPACITY
        L_eff = t;
        err_index = done0 + t;
        break;
      }
      p = n + next_cand;
      s_new = (tspin >> 8) - 1;
    } else if (ncur == 0) {
      skip = 1;
    } else {
      // rank r among interacting vertices in canonical (augmented-index) order;
      // every wave computes it from the bookkeeping all threads wrote identically
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
        int r2 = r - (n - ndead);
        for (int base = 0; base < next_cand; base += 64) {
          const int j = base + lane;
          const bool alive = (j < next_cand) && scur[n + j] != 0;
          const unsigned long long m = __ballot(alive);
          const int cnt = __popcll(m);
          if (r2 < cnt) {
            const unsigned long long hit = __ballot(alive && __popcll(m & ((1ull << lane) - 1ull)) == r2);
            p = n + base + __ffsll(static_cast<long long>(hit)) - 1;
            break;
          }
          r2 -= cnt;
        }
      }
      if (p < 0 || p >= n + next_cand || scur[p] == 0) {   // cannot happen unless bookkeeping is broken
        status = -4;
        L_eff = t;
        err_index = -3;
        break;
      }
      s_old = scur[p];
      s_new = (type == 1) ? 0 : -s_old;
    }

    // prefactor of the acceptance ratio (Eq. insprob), computed while the
    // gathers below are in flight
    const double fpre = (type == 0) ? Kc / static_cast<double>(ncur + 1)
                                    : (type == 1 ? static_cast<double>(ncur) / Kc : 1.0);
    double gh0 = 0.0, gh1 = 0.0, dp0 = 1.0, dp1 = 1.0;
    const int rp = (!skip && !gz) ? static_cast<int>(slot_of[p]) : -1;   // slot of a repeated change
    if (rp >= 0) {
      // ---- repeated change: ratio from X_aa (the owed growth first) ----
      const int s0p = s0l[p];
      gh0 = sh_ev[0][s_new - s0p + 2] - 1.0;   // net change from the block-start spin
      gh1 = sh_ev[1][s_new - s0p + 2] - 1.0;
      dp0 = sh_dsc[0][s0p + 2];
      dp1 = sh_dsc[1][s0p + 2];
      if (pend) {
        grow(pk, pbeta);
        pend = false;
      }
      lds_barrier();
      if (loc == 0) {
        const double xaa = Gis[rp * lg + rp], go = sh_gh[sec][rp];
        const double gn = sec == 0 ? gh0 : gh1, dp = sec == 0 ? dp0 : dp1;
        sh_beta[tp][sec] = (s_new == s0p) ? xaa / (-go * dp)
                                          : (gn / go) * (1.0 + (1.0 / go - 1.0 / gn) / dp * xaa);
      }
      lds_barrier();
    } else if (!skip && !gz) {
      // ---- issue the gathers: thread loc < 64 takes s_loc = G(P_loc, p) (loc == 63: G_pp),
      // thread 64 + b takes w_b = G(p, P_b) ----
      int gi = -1, gj = -1;
      if (loc < 64) {
        if (loc < ka) { gi = myP; gj = p; }
        else if (loc == 63) { gi = p; gj = p; }
      } else if (loc - 64 < ka) {
        gi = p;
        gj = myP;
      }
      double raw = 0.0;
      if (gi >= 0) {
        if (gj < n) raw = (gi < n) ? static_cast<double>(Nsec[static_cast<size_t>(gi) * ld + gj])
                                   : Rts[static_cast<size_t>(gi - n) * ld + gj];
        else raw = (gi < n) ? YTs[static_cast<size_t>(gj - n) * ld + gi]
                            : Gnns[static_cast<size_t>(gi - n) * kmax + (gj - n)];
      }
      {
        const int s0p = s0l[p];
        gh0 = sh_ev[0][s_new - s0p + 2] - sh_ev[0][s_old - s0p + 2];
        gh1 = sh_ev[1][s_new - s0p + 2] - sh_ev[1][s_old - s0p + 2];
        dp0 = sh_dsc[0][s0p + 2];   // 1 for a candidate (s0 = 0)
        dp1 = sh_dsc[1][s0p + 2];
      }
      // ---- owed growth of Gamma^{-1} by partitioning (Sec. III B 2), LDS only ----
      if (pend) {
        grow(pk, pbeta);
        pend = false;
      }
      // ---- finish the gathers (entries of Gamma~: the raw entry minus the identity);
      // each thread also records its entry as row / column ka of Gamma~ for the
      // pivoted inversion at block end (a rejected proposal's entries are
      // overwritten by the next one) ----
      const double gh = sec == 0 ? gh0 : gh1, dp = sec == 0 ? dp0 : dp1;
      if (gi >= 0) {
        const double v = raw - (gi == gj ? 1.0 : 0.0);
        if (loc == 63 && gi == gj && loc >= ka) {
          const double dd = v - 1.0 / (gh * dp);
          sh_gpp[tp][sec] = dd;
          gam[ka * kcap + ka] = dd;
        } else if (loc < 64) {
          vs[sec * kp + loc] = v;
          gam[loc * kcap + ka] = v;
        } else {
          vw[sec * kp + loc - 64] = v;
          gam[ka * kcap + loc - 64] = v;
        }
      }
      lds_barrier();
      // v = Gamma^{-1} s and beta = d - w.v (waves 0 and 2), u = w^T Gamma^{-1} (waves 1 and 3);
      // four accumulators, loads of eight terms in flight together
      if (loc < 64) {
        double acc = 0.0;
        if (loc < ka) {
          const double *row = Gis + loc * lg;
          const double *sv = vs + sec * kp;
          double a4[4] = {0.0, 0.0, 0.0, 0.0};
          for (int b0 = 0; b0 < ka; b0 += 8) {   // whole batches of 8: entries beyond k_a are zero
            double x[8], y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              x[i] = row[b0 + i];
              y[i] = sv[b0 + i];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) a4[i & 3] = fma(x[i], y[i], a4[i & 3]);
          }
          acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
          vv[sec * kp + loc] = acc;
        }
        const double x = (loc < ka) ? vw[sec * kp + loc] * acc : 0.0;
        const double s = wave_sum_dpp(x);
        if (lane == 0) sh_beta[tp][sec] = sh_gpp[tp][sec] - s;
      } else {
        const int b = loc - 64;
        if (b < ka) {
          const double *wv = vw + sec * kp;
          double a4[4] = {0.0, 0.0, 0.0, 0.0};
          for (int a0 = 0; a0 < ka; a0 += 8) {   // whole batches of 8: entries beyond k_a are zero
            double x[8], y[8];
            const double *col = Gis + a0 * lg + b;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              x[i] = wv[a0 + i];
              y[i] = col[i * lg];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) a4[i & 3] = fma(x[i], y[i], a4[i & 3]);
          }
          vu[sec * kp + b] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
      }
      lds_barrier();
    }

    double R;
    if (skip) {
      R = 0.0;
    } else {
      double r0 = 1.0, r1 = 1.0;
      if (rp >= 0) {   // the sector ratios themselves
        r0 = sh_beta[tp][0];
        r1 = sh_beta[tp][1];
      } else if (!gz) {
        r0 = -gh0 * dp0 * sh_beta[tp][0];
        r1 = -gh1 * dp1 * sh_beta[tp][1];
      }
      R = fpre * r0 * r1;
    }
    if (!isfinite(R)) {
      status = -4;  // CTAUX_ENUMERIC
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
      nchg += 1;
      if (R < 0.0) sign = -sign;
      if (rp >= 0) {
        had_repeat = true;
        repeat_update(rp, s_new == s0l[p], sec == 0 ? gh0 : gh1, sec == 0 ? dp0 : dp1);
        if (s_new != s0l[p]) {
          if (tid == 0) {
            sh_gh[0][rp] = gh0;
            sh_gh[1][rp] = gh1;
          }
        } else {
          // slot rp is removed: the last slot moves into it (every thread writes the same values)
          const int last = ka - 1, pl = P[last];
          if (rp != last) {
            P[rp] = pl;
            slot_of[pl] = static_cast<int8_t>(rp);
            if (lane == rp) myP = pl;
            if (tid == 0) {
              sh_gh[0][rp] = sh_gh[0][last];
              sh_gh[1][rp] = sh_gh[1][last];
            }
          }
          slot_of[p] = -1;
          ka -= 1;
        }
      } else if (!gz) {
        pend = true;
        pk = ka;
        pbeta = sh_beta[tp][sec];
        P[ka] = p;           // every thread writes the same value
        slot_of[p] = static_cast<int8_t>(ka);
        if (lane == ka) myP = p;
        if (tid == 0) {
          sh_gh[0][ka] = gh0;
          sh_gh[1][ka] = gh1;
        }
        ka += 1;
      }
      scur[p] = static_cast<int8_t>(s_new);   // every thread writes the same value
      if (type == 0) {
        if (tid == 0) sh_cid[next_cand] = next_id;
        next_id += 1;
        ncur += 1;
      } else if (type == 1) {
        ncur -= 1;
        if (p < n) {
          if (lane == ndead) myDead = p;
          ndead += 1;
        }
      }
    }
    if (type == 0) next_cand += 1;
    // with U = 0 there are no gather barriers; without one here a wave could run
    // ahead and overwrite spins another wave still has to read
    if (gz) lds_barrier();
    // Gamma full: the block ends here (with U = 0 the removed-vertex list, whose
    // length never exceeds that of P otherwise, bounds the block)
    if ((gz ? nchg : ka) == kcap) {
      L_eff = t + 1;
      break;
    }
  }
  __syncthreads();
  // the growth owed by the last acceptance: Gamma^{-1} of the growth is the
  // starting point of the refinement below
  if (pend) grow(pk, pbeta);
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

// LDS: Gamma^{-1} of both sectors as k_cap rounded up to 8 rows (the
// matrix-vector products read whole batches of 8) of that many plus one
// entries, the four vectors, P, the spins and the slots.
size_t propose_lds_bytes(int kcap, int kmax, int n_cap) {
  const size_t kp = (static_cast<size_t>(kcap) + 7) & ~size_t{7};
  return sizeof(double) * (2 * kp * (kp + 1) + 8 * kp) + sizeof(int) * static_cast<size_t>(kcap) +
         3ull * static_cast<size_t>(n_cap + kmax) + 16;
}

static size_t propose_lds_bytes(const Batch &b) { return propose_lds_bytes(b.kcap, b.kmax, b.n_cap); }

// Dynamic LDS limits are set once per batch: the call costs host time that would
// otherwise sit between the launches of every block.  Returns -1 if the runtime
// refuses the size (the options were validated against the LDS of a workgroup,
// so this signals a device that has less).
int setup_propose(const Batch &b) {
  const int lds = static_cast<int>(propose_lds_bytes(b));
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_propose<double>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
      hipFuncSetAttribute(reinterpret_cast<const void *>(k_propose<float>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return -1;
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_propose<double>)) != hipSuccess ||
      fa.sharedSizeBytes > kProposeStaticLds)
    return -1;
  return 0;
}

void launch_propose(const Batch &b, hipStream_t s) {
  const size_t lds = propose_lds_bytes(b);
  if (b.precision == kFP64)
    hipLaunchKernelGGL(k_propose<double>, dim3(b.n_chains), dim3(256), lds, s, b.d_desc, b.d_state);
  else
    hipLaunchKernelGGL(k_propose<float>, dim3(b.n_chains), dim3(256), lds, s, b.d_desc, b.d_state);
}

}  // namespace ctaux
