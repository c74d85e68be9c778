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
#include "ctaux_device.h"

namespace ctaux {

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
  const int32_t *s0 = d.s0[par];
  const bool gz = (d.gamma == 0.0);

  extern __shared__ double smem[];
  double *Gi = smem;                         // [2][kcap][lg]
  double *vs = Gi + 2 * kcap * lg;           // [2][kcap]   s vectors
  double *vw = vs + 2 * kcap;                // [2][kcap]   w vectors
  double *vv = vw + 2 * kcap;                // [2][kcap]   Gamma^{-1} s
  double *vu = vv + 2 * kcap;                // [2][kcap]   w^T Gamma^{-1}
  int *P = reinterpret_cast<int *>(vu + 2 * kcap);   // [kcap]
  int *dead = P + kcap;                      // [kcap] removed old vertices
  int8_t *scur = reinterpret_cast<int8_t *>(dead + kcap);  // [n + kmax] current spins
  double *Gis = Gi + sec * kcap * lg;
  __shared__ double sh_gpp[2], sh_beta[2];
  __shared__ double sh_gh[2][kMaxKcap];
  __shared__ int sh_p;
  __shared__ int64_t sh_cid[kMaxKmax];
  __shared__ int sh_scan[256];

  int ka = 0, nchg = 0, ncur = n, ndead = 0, next_cand = 0;   // nchg: accepted changes (== ka unless U = 0)
  int64_t next_id = st.next_id, accepted = st.accepted;
  double sign = st.sign;
  int status = 0, L_eff = L;
  int64_t err_index = -1;

  for (int i = tid; i < n + kins; i += 256) scur[i] = (i < n) ? static_cast<int8_t>(s0[i]) : 0;
  __syncthreads();

  for (int t = 0; t < L; ++t) {
    const int type = d.ptype[t];
    const double u_acc = d.pacc[t];
    int p = -1, s_old = 0, s_new = 0, skip = 0;
    if (type == 0) {
      if (ncur + 1 > d.n_cap) {
        status = -5;  // CTAUX_ECAPACITY
        L_eff = t;
        err_index = st.done + t;
        break;
      }
      p = n + next_cand;
      s_new = d.pspin[t];
    } else if (ncur == 0) {
      skip = 1;
    } else {
      int r = static_cast<int>(floor(static_cast<double>(ncur) * d.ppick[t]));
      if (r > ncur - 1) r = ncur - 1;
      if (tid == 0) sh_p = -1;
      __syncthreads();
      if (wave == 0) {
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
      const int s0p = (p < n) ? s0[p] : 0;
      gh0 = d.evd[0][s_new - s0p + 2] - d.evd[0][s_old - s0p + 2];
      gh1 = d.evd[1][s_new - s0p + 2] - d.evd[1][s_old - s0p + 2];
      // gather the new row / column of Gamma and G_pp
      if (loc < ka) {
        const int pa = P[loc];
        vs[sec * kcap + loc] = g_entry<T>(d, Nsec, s0, n, sec, pa, p) - (pa == p ? 1.0 : 0.0);
      } else if (loc < 2 * ka) {
        const int b = loc - ka, pb = P[b];
        vw[sec * kcap + b] = g_entry<T>(d, Nsec, s0, n, sec, p, pb) - (pb == p ? 1.0 : 0.0);
      } else if (loc == 2 * ka) {
        sh_gpp[sec] = g_entry<T>(d, Nsec, s0, n, sec, p, p);
      }
      __syncthreads();
      // v = Gamma^{-1} s (threads loc < 64), u = w^T Gamma^{-1} (threads loc >= 64)
      if (loc < 64) {
        if (loc < ka) {
          double acc = 0.0;
          const double *row = Gis + loc * lg;
          const double *sv = vs + sec * kcap;
          for (int b = 0; b < ka; ++b) acc += row[b] * sv[b];
          vv[sec * kcap + loc] = acc;
        }
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
      if ((wave & 1) == 0) {   // waves 0 (up) and 2 (down)
        const double x = (lane < ka) ? vw[sec * kcap + lane] * vv[sec * kcap + lane] : 0.0;
        const double s = wave_sum(x);
        if (lane == 0) {
          const double gh = sec == 0 ? gh0 : gh1;
          sh_beta[sec] = (sh_gpp[sec] - 1.0 - 1.0 / gh) - s;
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
        r0 = -gh0 * sh_beta[0];
        r1 = -gh1 * sh_beta[1];
      }
      const double f = (type == 0) ? d.K / static_cast<double>(ncur + 1)
                                   : (type == 1 ? static_cast<double>(ncur) / d.K : 1.0);
      R = f * r0 * r1;
    }
    if (!isfinite(R)) {
      status = -4;  // CTAUX_ENUMERIC
      L_eff = t;
      err_index = st.done + t;
      break;
    }
    const int acc = (!skip && u_acc < fabs(R)) ? 1 : 0;
    if (tid == 0) {
      const int64_t idx = st.done + t;
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
        // Gamma^{-1} grows by partitioning
        const int k = ka;
        const double ib = 1.0 / sh_beta[sec];
        const double *v = vv + sec * kcap, *u = vu + sec * kcap;
        for (int e = loc; e < (k + 1) * (k + 1); e += 128) {
          const int a = e / (k + 1), b = e - a * (k + 1);
          if (a < k && b < k) Gis[a * lg + b] += v[a] * u[b] * ib;
          else if (a < k) Gis[a * lg + k] = -v[a] * ib;
          else if (b < k) Gis[k * lg + b] = -u[b] * ib;
          else Gis[k * lg + k] = ib;
        }
        // record the new row and column of Gamma for the pivoted inversion at block end
        double *gam = d.Gam[sec];
        for (int e = loc; e < 2 * k + 1; e += 128) {
          if (e < k) gam[e * kcap + k] = vs[sec * kcap + e];
          else if (e < 2 * k) gam[k * kcap + (e - k)] = vw[sec * kcap + (e - k)];
          else gam[k * kcap + k] = sh_gpp[sec] - 1.0 - 1.0 / (sec == 0 ? gh0 : gh1);
        }
        if (tid == 0) {
          P[k] = p;
          sh_gh[0][k] = gh0;
          sh_gh[1][k] = gh1;
        }
        ka = k + 1;
      }
      if (tid == 0) {
        scur[p] = static_cast<int8_t>(s_new);
        if (type == 0) sh_cid[next_cand] = next_id;
        if (type == 1 && p < n) dead[ndead] = p;
      }
      if (type == 0) {
        next_id += 1;
        ncur += 1;
      } else if (type == 1) {
        ncur -= 1;
        if (p < n) ndead += 1;
      }
    }
    if (type == 0) next_cand += 1;
    __syncthreads();
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
         static_cast<size_t>(b.n_cap + b.kmax) + 16;
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
