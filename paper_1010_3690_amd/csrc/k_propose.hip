// The inner loop of a block (Sec. IV B): k sequential insert / remove / flip
// proposals, each a spin change of one vertex of the augmented configuration.
//
// For a change of vertex p from spin s_old to s_new (block-start spin s0),
//   gh = exp(V(s_new) - V(s0)) - exp(V(s_old) - V(s0))        (per sector)
// the new row/column of Gamma are s_a = G_{P_a p} - delta, w_b = G_{p P_b} - delta,
// d = G_pp - 1 - 1/gh, with G the block-start Green's function (Eq. Gamma with
// repeated changes allowed).  Inversion by partitioning (Sec. III B 2):
//   beta = d - w^T Gamma^{-1} s,   det ratio of the sector = -gh * beta  (Eq. ratS),
// and on acceptance Gamma^{-1} grows by one row and column.
// R = {K/(n+1), n/K, 1} * r_up * r_dn (Eq. insprob and Sec. II B); accept iff u < |R|.
//
// One workgroup (4 waves) per chain; Gamma^{-1} of both sectors lives in LDS.
// Threads 0..127 serve the up sector, 128..255 the down sector.
//
// Synchronisation: an insertion costs two barriers (after the gathers, after
// Gamma^{-1} s and w^T Gamma^{-1}), a removal or flip three (the rank
// selection first).  Bookkeeping that the next proposal reads (P, the spins,
// the removed list) is written by every thread with the same value, each
// thread reads back only what it wrote itself or what precedes a barrier, and
// the per-proposal scalars are double-buffered by proposal parity, so no
// barrier is needed at the end of a proposal.
#include "ctaux_device.h"

namespace ctaux {

// G entry with the block-start spins taken from LDS.
template <typename T>
__device__ __forceinline__ double g_entry_l(const ChainDesc &d, const T *N, const int8_t *s0l, int n, int sec,
                                            int i, int j) {
  if (j < n) {
    const double e = d.evd[sec][s0l[j] + 2];
    const double nij = (i < n) ? static_cast<double>(N[static_cast<size_t>(i) * d.ld + j])
                               : d.Rt[sec][static_cast<size_t>(i - n) * d.ld + j];
    return (nij * e - (i == j ? 1.0 : 0.0)) / (e - 1.0);
  }
  const int jj = j - n;
  return (i < n) ? d.YT[sec][static_cast<size_t>(jj) * d.ld + i]
                 : d.Gnn[sec][static_cast<size_t>(i - n) * d.kmax + jj];
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
  const int kcap = d.kcap, lg = kcap + 1;
  const int par = st.parity;
  const T *Nsec = static_cast<const T *>(d.N[par][sec]);
  const bool gz = (d.gamma == 0.0);
  const int64_t done0 = st.done;

  extern __shared__ double smem[];
  double *Gi = smem;                         // [2][kcap][lg]
  double *vs = Gi + 2 * kcap * lg;           // [2][kcap]   s vectors
  double *vw = vs + 2 * kcap;                // [2][kcap]   w vectors
  double *vv = vw + 2 * kcap;                // [2][kcap]   Gamma^{-1} s
  double *vu = vv + 2 * kcap;                // [2][kcap]   w^T Gamma^{-1}
  int *P = reinterpret_cast<int *>(vu + 2 * kcap);   // [kcap]
  int *dead = P + kcap;                      // [kcap] removed old vertices
  int8_t *scur = reinterpret_cast<int8_t *>(dead + kcap);  // [n + kmax] current spins
  int8_t *s0l = scur + (d.n_cap + d.kmax);                  // [n + kmax] block-start spins
  double *Gis = Gi + sec * kcap * lg;
  __shared__ double sh_gpp[2][2], sh_beta[2][2];   // [proposal parity][sector]
  __shared__ double sh_gh[2][kMaxKcap];
  __shared__ double sh_pacc[kMaxKmax], sh_ppick[kMaxKmax];
  __shared__ int8_t sh_ptype[kMaxKmax], sh_pspin[kMaxKmax];
  __shared__ int sh_p;
  __shared__ int64_t sh_cid[kMaxKmax];
  __shared__ int sh_scan[256];

  int ka = 0, nchg = 0, ncur = n, ndead = 0, next_cand = 0;   // nchg: accepted changes (== ka unless U = 0)
  int64_t next_id = st.next_id, accepted = st.accepted;
  double sign = st.sign;
  int status = 0, L_eff = L;
  int64_t err_index = -1;

  for (int i = tid; i < n + kins; i += 256) {
    const int8_t v = (i < n) ? static_cast<int8_t>(d.s0[par][i]) : 0;
    scur[i] = v;
    s0l[i] = v;
  }
  for (int t = tid; t < L; t += 256) {
    sh_ptype[t] = static_cast<int8_t>(d.ptype[t]);
    sh_pspin[t] = static_cast<int8_t>(d.pspin[t]);
    sh_pacc[t] = d.pacc[t];
    sh_ppick[t] = d.ppick[t];
  }
  __syncthreads();

  for (int t = 0; t < L; ++t) {
    const int tp = t & 1;
    const int type = sh_ptype[t];
    const double u_acc = sh_pacc[t];
    int p = -1, s_old = 0, s_new = 0, skip = 0;
    if (type == 0) {
      if (ncur + 1 > d.n_cap) {
        status = -5;  // CTAUX_ECAPACITY
        L_eff = t;
        err_index = done0 + t;
        break;
      }
      p = n + next_cand;
      s_new = sh_pspin[t];
    } else if (ncur == 0) {
      skip = 1;
    } else {
      int r = static_cast<int>(floor(static_cast<double>(ncur) * sh_ppick[t]));
      if (r > ncur - 1) r = ncur - 1;
      if (wave == 0) {
        if (lane == 0) sh_p = -1;
        // rank r among interacting vertices in canonical (augmented-index) order
        if (r < n - ndead) {
          // old vertex: least idx with idx = r + #{dead <= idx}
          int idx = r;
          while (true) {
            const bool le = (lane < ndead) && (dead[lane] <= idx);
            const int nw = r + __popcll(__ballot(le));
            if (nw == idx) break;
            idx = nw;
          }
          if (lane == 0) sh_p = idx;
        } else {
          int r2 = r - (n - ndead);
          for (int base = 0; base < next_cand; base += 64) {
            const int j = base + lane;
            const bool alive = (j < next_cand) && scur[n + j] != 0;
            const unsigned long long m = __ballot(alive);
            const int cnt = __popcll(m);
            if (r2 < cnt) {
              if (alive && __popcll(m & ((1ull << lane) - 1ull)) == r2) sh_p = n + j;
              break;
            }
            r2 -= cnt;
          }
        }
      }
      __syncthreads();
      p = sh_p;
      if (p < 0 || p >= n + next_cand || scur[p] == 0) {   // cannot happen unless bookkeeping is broken
        status = -4;
        L_eff = t;
        err_index = -3;
        break;
      }
      s_old = scur[p];
      s_new = (type == 1) ? 0 : -s_old;
    }

    double gh0 = 0.0, gh1 = 0.0;
    if (!skip && !gz) {
      const int s0p = s0l[p];
      gh0 = d.evd[0][s_new - s0p + 2] - d.evd[0][s_old - s0p + 2];
      gh1 = d.evd[1][s_new - s0p + 2] - d.evd[1][s_old - s0p + 2];
      const double gh = sec == 0 ? gh0 : gh1;
      // gather the new row / column of Gamma and G_pp; each thread also records
      // its entry as row / column ka of Gamma for the pivoted inversion at block
      // end (a rejected proposal's entries are overwritten by the next one)
      double *gam = d.Gam[sec];
      if (loc < ka) {
        const int pa = P[loc];
        const double v = g_entry_l<T>(d, Nsec, s0l, n, sec, pa, p) - (pa == p ? 1.0 : 0.0);
        vs[sec * kcap + loc] = v;
        gam[loc * kcap + ka] = v;
      } else if (loc < 2 * ka) {
        const int b = loc - ka, pb = P[b];
        const double v = g_entry_l<T>(d, Nsec, s0l, n, sec, p, pb) - (pb == p ? 1.0 : 0.0);
        vw[sec * kcap + b] = v;
        gam[ka * kcap + b] = v;
      } else if (loc == 2 * ka) {
        const double gpp = g_entry_l<T>(d, Nsec, s0l, n, sec, p, p);
        sh_gpp[tp][sec] = gpp;
        gam[ka * kcap + ka] = gpp - 1.0 - 1.0 / gh;
      }
      __syncthreads();
      // v = Gamma^{-1} s and beta = d - w.v (waves 0 and 2), u = w^T Gamma^{-1} (waves 1 and 3)
      if (loc < 64) {
        double acc = 0.0;
        if (loc < ka) {
          const double *row = Gis + loc * lg;
          const double *sv = vs + sec * kcap;
          for (int b = 0; b < ka; ++b) acc += row[b] * sv[b];
          vv[sec * kcap + loc] = acc;
        }
        const double x = (loc < ka) ? vw[sec * kcap + loc] * acc : 0.0;
        const double s = wave_sum(x);
        if (lane == 0) sh_beta[tp][sec] = (sh_gpp[tp][sec] - 1.0 - 1.0 / gh) - s;
      } else {
        const int b = loc - 64;
        if (b < ka) {
          double acc = 0.0;
          const double *wv = vw + sec * kcap;
          for (int a = 0; a < ka; ++a) acc += wv[a] * Gis[a * lg + b];
          vu[sec * kcap + b] = acc;
        }
      }
      __syncthreads();
    }

    double R;
    if (skip) {
      R = 0.0;
    } else {
      double r0 = 1.0, r1 = 1.0;
      if (!gz) {
        r0 = -gh0 * sh_beta[tp][0];
        r1 = -gh1 * sh_beta[tp][1];
      }
      const double f = (type == 0) ? d.K / static_cast<double>(ncur + 1)
                                   : (type == 1 ? static_cast<double>(ncur) / d.K : 1.0);
      R = f * r0 * r1;
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
      if (idx < d.log_cap) {
        d.log_acc[idx] = static_cast<uint8_t>(acc);
        d.log_R[idx] = R;
      }
    }
    if (acc) {
      accepted += 1;
      nchg += 1;
      if (R < 0.0) sign = -sign;
      if (!gz) {
        // Gamma^{-1} grows by partitioning; thread (b = loc % 64, a = loc / 64 + 2i)
        const int k = ka;
        const double beta = sh_beta[tp][sec];
        const double ib = 1.0 / beta;
        const double *v = vv + sec * kcap, *u = vu + sec * kcap;
        const int b = loc & 63, a0 = loc >> 6;
        if (b <= k) {
          // batches of 8 rows: loads first (in flight together), then stores
          const double ub = (b < k) ? u[b] * ib : 0.0;
          for (int a1 = a0; a1 <= k; a1 += 16) {
            double va[8], ga[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int a = a1 + 2 * i;
              va[i] = (a < k) ? v[a] : 0.0;
              ga[i] = (a < k && b < k) ? Gis[a * lg + b] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int a = a1 + 2 * i;
              if (a < k) Gis[a * lg + b] = (b < k) ? ga[i] + va[i] * ub : -va[i] * ib;
              else if (a == k) Gis[k * lg + b] = (b < k) ? -ub : ib;
            }
          }
        }
        P[k] = p;           // every thread writes the same value
        if (tid == 0) {
          sh_gh[0][k] = gh0;
          sh_gh[1][k] = gh1;
        }
        ka = k + 1;
      }
      scur[p] = static_cast<int8_t>(s_new);   // every thread writes the same value
      if (type == 0) {
        if (tid == 0) sh_cid[next_cand] = next_id;
        next_id += 1;
        ncur += 1;
      } else if (type == 1) {
        ncur -= 1;
        if (p < n) {
          dead[ndead] = p;   // every thread writes the same value
          ndead += 1;
        }
      }
    }
    if (type == 0) next_cand += 1;
    if (gz) __syncthreads();   // U = 0 has no gather barriers; keep the selection scalar safe
    if (nchg == kcap) {   // Gamma (and the removed-vertex list) is full: the block ends here
      L_eff = t + 1;
      break;
    }
  }
  __syncthreads();

  // ---- compaction map: interacting vertices in augmented order ----
  const int na = n + kins;
  const int chunk = (na + 255) / 256;
  const int b0 = tid * chunk, b1 = min(b0 + chunk, na);
  int cnt = 0;
  for (int i = b0; i < b1; ++i) cnt += (scur[i] != 0);
  sh_scan[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = (tid >= off) ? sh_scan[tid - off] : 0;
    __syncthreads();
    sh_scan[tid] += v;
    __syncthreads();
  }
  int pos = sh_scan[tid] - cnt;
  const int np = par ^ 1;
  for (int i = b0; i < b1; ++i) {
    if (scur[i] == 0) continue;
    d.map[pos] = i;
    if (i < n) {
      d.tau[np][pos] = d.tau[par][i];
      d.site[np][pos] = d.site[par][i];
      d.id[np][pos] = d.id[par][i];
    } else {
      d.tau[np][pos] = d.ctau[i - n];
      d.site[np][pos] = d.csite[i - n];
      d.id[np][pos] = sh_cid[i - n];
    }
    d.s0[np][pos] = scur[i];
    ++pos;
  }
  // ---- P and gh for the rank-k update (Gamma itself was recorded on acceptance) ----
  for (int a = tid; a < ka; a += 256) {
    d.P[a] = P[a];
    d.ghat[0][a] = sh_gh[0][a];
    d.ghat[1][a] = sh_gh[1][a];
  }
  if (tid == 0) {
    st.k_a = ka;
    st.n_new = sh_scan[255];
    st.L_eff = L_eff;
    st.sign = sign;
    st.next_id = next_id;
    st.accepted = accepted;
    st.status = status;
    if (status != 0) st.err_index = err_index;
    if (sh_scan[255] != ncur && status == 0) {
      st.status = -4;
      st.err_index = -2;   // bookkeeping mismatch
    }
  }
}

size_t propose_lds_bytes(const Batch &b) {
  return sizeof(double) * (2ull * b.kcap * (b.kcap + 1) + 8ull * b.kcap) + sizeof(int) * 2ull * b.kcap +
         2ull * static_cast<size_t>(b.n_cap + b.kmax) + 16;
}

void launch_propose(const Batch &b, hipStream_t s) {
  const size_t lds = propose_lds_bytes(b);
  if (b.precision == kFP64) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_propose<double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    hipLaunchKernelGGL(k_propose<double>, dim3(b.n_chains), dim3(256), lds, s, b.d_desc, b.d_state);
  } else {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_propose<float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    hipLaunchKernelGGL(k_propose<float>, dim3(b.n_chains), dim3(256), lds, s, b.d_desc, b.d_state);
  }
}

}  // namespace ctaux
