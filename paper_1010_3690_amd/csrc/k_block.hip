// Block set-up and tear-down: proposal draws, pre-insertion of the block's
// insertion candidates, G0 interpolation for the candidates (Sec. IV A), and
// the end-of-block bookkeeping.
#include "ctaux_device.h"

namespace ctaux {

__global__ void k_set_target(ChainState *states, int n_chains, int64_t n_proposals) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n_chains) states[c].target = states[c].done + n_proposals;
}

void launch_set_target(const Batch &b, hipStream_t s, int64_t n_proposals) {
  hipLaunchKernelGGL(k_set_target, dim3((b.n_chains + 255) / 256), dim3(256), 0, s, b.d_state,
                     b.n_chains, n_proposals);
}

// One workgroup per chain.  Decides the block length (at most k_max, never
// past a measurement point, and short enough that its insertion candidates -
// two for a pair insertion - number at most k_max), decodes the block's
// proposals and collects the insertion candidates in proposal order.
// Proposal mix: insertion and removal (1 - p_flip - p_pair)/2 each, pair
// insertion and pair removal p_pair/2 each, flip p_flip.
__device__ void block_begin_chain(const ChainDesc &d, ChainState &st) {
  __shared__ int sh_L, sh_active, sh_cut;
  __shared__ int scan[256];
  if (threadIdx.x == 0) {
    int active = (st.status == 0 && st.done < st.target) ? 1 : 0;
    int64_t L = 0;
    if (active) {
      L = st.target - st.done;
      if (L > d.kmax) L = d.kmax;
      int64_t m = (st.done / d.meas_every + 1) * d.meas_every;
      if (m <= d.n_therm) m = (d.n_therm / d.meas_every + 1) * d.meas_every;
      if (m - st.done < L) L = m - st.done;
    }
    st.active = active;
    st.L = static_cast<int>(L);
    st.L_eff = 0;
    st.k_a = 0;
    st.meas_now = 0;
    sh_L = static_cast<int>(L);
    sh_active = active;
    sh_cut = static_cast<int>(L);
  }
  __syncthreads();
  if (!sh_active) {
    if (threadIdx.x == 0) st.k_ins = 0;
    return;
  }
  const int L = sh_L;
  const int t = threadIdx.x;
  int ncand = 0;
  double tau = 0.0, tau2 = 0.0;
  int site = 0, site2 = 0;
  if (t < L) {
    double u[5];
    const uint64_t index = static_cast<uint64_t>(st.done + t);
    proposal_uniforms(d, index, u);
    const double p_one = 0.5 * (1.0 - d.p_flip - d.p_pair);
    int type;
    if (u[0] < p_one) type = 0;
    else if (u[0] < 2.0 * p_one) type = 1;
    else if (u[0] < 2.0 * p_one + 0.5 * d.p_pair) type = 3;
    else if (u[0] < 2.0 * p_one + d.p_pair) type = 4;
    else type = 2;
    d.ptype[t] = type;
    d.pacc[t] = u[1];
    d.ppick[t] = u[3];
    if (type == 0 || type == 3) {
      tau = d.beta * u[2];
      site = static_cast<int>(floor(static_cast<double>(d.nc) * u[3]));
      if (site > d.nc - 1) site = d.nc - 1;
      d.pspin[t] = u[4] < 0.5 ? -1 : 1;
      ncand = 1;
    } else {
      d.pspin[t] = 0;
    }
    if (type >= 3) {
      double v[3];
      pair_uniforms(d, index, v);
      d.ppick2[t] = v[2];
      if (type == 3) {
        tau2 = d.beta * v[1];
        site2 = static_cast<int>(floor(static_cast<double>(d.nc) * v[2]));
        if (site2 > d.nc - 1) site2 = d.nc - 1;
        d.pspin2[t] = v[0] < 0.5 ? -1 : 1;
        ncand = 2;
      }
    }
  }
  // inclusive prefix sum of the candidate counts (Hillis-Steele over 256 lanes)
  scan[t] = ncand;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int v = (t >= off) ? scan[t - off] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  // the block ends before the first proposal whose candidates would exceed k_max
  if (t < L && scan[t] > d.kmax) atomicMin(&sh_cut, t);
  __syncthreads();
  const int Lc = sh_cut;
  if (t < Lc && ncand > 0) {
    const int j = scan[t] - ncand;
    d.ctau[j] = tau;
    d.csite[j] = site;
    if (ncand == 2) {
      d.ctau[j + 1] = tau2;
      d.csite[j + 1] = site2;
    }
  }
  if (t == 0) {
    st.L = Lc;
    st.k_ins = Lc > 0 ? scan[Lc - 1] : 0;
  }
}

__global__ __launch_bounds__(256) void k_block_begin(const ChainDesc *descs, ChainState *states) {
  block_begin_chain(descs[blockIdx.x], states[blockIdx.x]);
}

void launch_block_begin(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_block_begin, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
}

// G0 products for the candidates (Sec. IV A, "Preparation steps"), per sector:
//   X_ji  = G0(tau_j^new - tau_i)(e^{V_i} - 1)   (so that Rt = X N)
//   ZT_ji = G0(tau_i - tau_j^new)                 (so that YT = (N Z)^T)
// (both in the blocked order of cand_offset)
//   G0nn_jj' = G0(tau_j^new - tau_j'^new)          (0+ on the diagonal)
__global__ __launch_bounds__(256) void k_interp(const ChainDesc *descs, const ChainState *states, int n_chains,
                                                int xcd_g) {
  const ChainBlock cb = chain_block(xcd_g);
  const int c = cb.c;
  if (c >= n_chains) return;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active) return;
  const int n = st.n, k = st.k_ins;
  const int par = st.parity;
  const double *tau = d.tau[par];
  const int32_t *site = d.site[par];
  const int32_t *s0 = d.s0[par];
  // 32-bit index arithmetic: 2 (2 k n + k^2) < 2^31 for k <= 128, n <= 8192
  const int kn = k * n, per_sec = 2 * kn + k * k, total = 2 * per_sec;
  const int rt = (d.kmax + 15) >> 4;   // candidate tiles of the X, ZT layout (cand_offset)
  for (int e = cb.sub * 256 + threadIdx.x; e < total; e += cb.g * 256) {
    const int sec = e >= per_sec ? 1 : 0;
    int r = e - sec * per_sec;
    if (r < 2 * kn) {
      const int which = r >= kn ? 1 : 0;
      r -= which * kn;
      const int j = r / n, i = r - j * n;
      if (which == 0) {
        const double ev = d.evd[sec][s0[i] + 2];
        d.X[sec][cand_offset(j, i, rt)] =
            g0_interp(d, sec, d.csite[j], site[i], d.ctau[j] - tau[i]) * (ev - 1.0);
      } else {
        d.ZT[sec][cand_offset(j, i, rt)] =
            g0_interp(d, sec, site[i], d.csite[j], tau[i] - d.ctau[j]);
      }
    } else {
      r -= 2 * kn;
      const int j = r / k, jj = r - j * k;
      d.G0nn[sec][static_cast<size_t>(j) * d.kmax + jj] =
          g0_interp(d, sec, d.csite[j], d.csite[jj], d.ctau[j] - d.ctau[jj]);
    }
  }
}

void launch_interp(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_interp, chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_state, b.n_chains,
                     chain_grid_arg(b));
}

// Ends a block and leaves a copy of the chain's state for the measurement
// (mstates), which runs on a stream of its own beside the next block.
__device__ void block_end_chain(const ChainDesc &d, ChainState &st, ChainState &mst) {
  if (!st.active) {
    mst = st;
    return;
  }
  // algorithmic work of the update per sector: Bc = Gamma^{-1} N_P (2 k^2 n') and
  // N' = N - Ac Bc (2 n'^2 k); bytes: read and write n'^2 entries of N plus Ac and Bc
  const double np = st.n_new, ka = st.k_a;
  const double es = d.precision == kFP64 ? 8.0 : 4.0;
  st.rk_flops += 2.0 * (2.0 * np * np * ka + 2.0 * ka * ka * np);
  st.rk_bytes += 2.0 * es * (2.0 * np * np + 2.0 * np * ka);
  st.sum_order += np;
  // preparation of this block (per sector): YT = ZT N^T and Rt = X N read N once
  // each (2 n^2 k_ins flops each), Gnn = X YT^T + G0nn (2 k_ins^2 n)
  {
    const double n0 = st.n, ki = st.k_ins;
    st.prep_flops += 2.0 * (4.0 * n0 * n0 * ki + 2.0 * ki * ki * n0);
    st.prep_bytes += 2.0 * (2.0 * es * n0 * n0 + 8.0 * 4.0 * ki * n0);
  }
  st.n = st.n_new;
  st.parity ^= 1;
  st.done += st.L_eff;
  st.blocks += 1;
  st.sum_ka += st.k_a;
  st.meas_now = (st.done % d.meas_every == 0 && st.done > d.n_therm) ? 1 : 0;
  if (st.meas_now) {
    // measurement (per sector): W = N gR reads N once (2 n^2 nc flops), gR is
    // written and read once; G = G0 + gL W (2 nc (n_out + 1) n nc flops) with the
    // nc (n_out + 1) n entries of gL interpolated in the product, two table reads
    // each (counted as loads, though they mostly hit the L2)
    const double m = static_cast<double>(d.nc) * (d.n_out + 1), nc = d.nc;
    st.meas_flops += 2.0 * (2.0 * np * np * nc + 2.0 * m * np * nc);
    st.meas_bytes += 2.0 * (es * np * np + 8.0 * 2.0 * m * np + 8.0 * 2.0 * np * nc);
  }
  mst = st;
}

__global__ void k_block_end(const ChainDesc *descs, ChainState *states, ChainState *mstates, int n_chains) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n_chains) block_end_chain(descs[c], states[c], mstates[c]);
}

// The end of one block and the start of the next in one launch (one workgroup
// per chain): saves a kernel, and its launch gap, on the critical path of every
// block but the last of a run.
__global__ __launch_bounds__(256) void k_block_turn(const ChainDesc *descs, ChainState *states, ChainState *mstates) {
  const int c = blockIdx.x;
  if (threadIdx.x == 0) block_end_chain(descs[c], states[c], mstates[c]);
  __syncthreads();   // the state thread 0 wrote is read by the whole workgroup below
  block_begin_chain(descs[c], states[c]);
}

void launch_block_end(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_block_end, dim3((b.n_chains + 63) / 64), dim3(64), 0, s, b.d_desc, b.d_state,
                     b.d_mstate, b.n_chains);
}

void launch_block_turn(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_block_turn, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state, b.d_mstate);
}

}  // namespace ctaux
