// Gamma^{-1} for the rank-k update, recomputed at the end of the block from
// the recorded entries of Gamma by Gauss-Jordan elimination with partial
// pivoting in FP64.  The O(k^2) growth by partitioning (Sec. III B 2) gives
// the acceptance ratios during the block; with repeated changes of a vertex
// Gamma can be ill-conditioned (condition numbers 1e6-1e8 are common), and the
// unpivoted growth then loses several digits that a pivoted inversion keeps.
//
// One workgroup per (chain, sector) on the augmented [Gamma | I] in LDS:
// thread (row r = tid % 64, column group tid / 64) updates every fourth column
// of its row, three barriers per eliminated column.
#include "ctaux_device.h"

namespace ctaux {

__global__ __launch_bounds__(256) void k_gamma_inv(const ChainDesc *descs, ChainState *states) {
  const int c = blockIdx.y, sec = blockIdx.x;
  const ChainDesc &d = descs[c];
  ChainState &st = states[c];
  if (!st.active) return;
  const int ka = st.k_a;
  if (ka == 0) return;
  const int w2 = 2 * ka, kcap = d.kcap;
  __shared__ double M[kMaxKcap][2 * kMaxKcap + 1];
  __shared__ double prow[2 * kMaxKcap], oldc[2 * kMaxKcap], f[kMaxKcap];
  __shared__ int sh_piv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane, cg = wave;
  const double *gam = d.Gam[sec];
  if (r < ka)
    for (int j = cg; j < w2; j += 4) M[r][j] = j < ka ? gam[r * kcap + j] : ((j - ka) == r ? 1.0 : 0.0);
  __syncthreads();
  for (int col = 0; col < ka; ++col) {
    if (wave == 0) {
      double v = (lane >= col && lane < ka) ? fabs(M[lane][col]) : -1.0;
      int idx = lane;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
      }
      if (lane == 0) sh_piv = idx;
    }
    __syncthreads();
    const int p = sh_piv;
    const double pv = M[p][col];
    if (tid < w2) {
      prow[tid] = M[p][tid] / pv;
      oldc[tid] = M[col][tid];
    } else if (tid >= 128 && tid - 128 < ka) {
      f[tid - 128] = M[tid - 128][col];
    }
    __syncthreads();
    if (r < ka) {
      // loads first, then arithmetic, then stores: the LDS loads of all the
      // thread's columns are in flight together
      const double fr = (r == p) ? f[col] : f[r];
      for (int j1 = cg; j1 < w2; j1 += 32) {   // batches of 8 columns
        double mv[8], pr[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = j1 + 4 * i;
          pr[i] = (j < w2) ? prow[j] : 0.0;
          mv[i] = (j < w2) ? ((r == p) ? oldc[j] : M[r][j]) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = j1 + 4 * i;
          if (j < w2) M[r][j] = (r == col) ? pr[i] : mv[i] - fr * pr[i];
        }
      }
    }
    __syncthreads();
  }
  bool bad = false;
  if (r < ka) {
    for (int j = cg; j < ka; j += 4) {
      const double v = M[r][ka + j];
      bad |= !isfinite(v);
      d.Ginv[sec][r * kcap + j] = v;
    }
  }
  if (bad) {
    st.status = -4;   // singular Gamma
    st.err_index = -4;
  }
}

void launch_gamma_inv(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_gamma_inv, dim3(2, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
}

}  // namespace ctaux
