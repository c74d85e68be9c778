// Gamma^{-1} for the rank-k update, recomputed at the end of the block from
// the recorded entries of Gamma by Gauss-Jordan elimination with partial
// pivoting in FP64.  The O(k^2) growth by partitioning (Sec. III B 2) gives
// the acceptance ratios during the block; with repeated changes of a vertex
// Gamma can be ill-conditioned (condition numbers 1e6-1e8 are common), and the
// unpivoted growth then loses several digits that a pivoted inversion keeps.
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
  const double *gam = d.Gam[sec];
  for (int e = tid; e < ka * w2; e += 256) {
    const int r = e / w2, j = e - r * w2;
    M[r][j] = j < ka ? gam[r * kcap + j] : ((j - ka) == r ? 1.0 : 0.0);
  }
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
    for (int j = tid; j < w2; j += 256) {
      prow[j] = M[p][j] / pv;
      oldc[j] = M[col][j];
    }
    if (tid < ka) f[tid] = M[tid][col];
    __syncthreads();
    for (int e = tid; e < ka * w2; e += 256) {
      const int r = e / w2, j = e - r * w2;
      if (r == col) M[r][j] = prow[j];
      else if (r == p) M[r][j] = oldc[j] - f[col] * prow[j];
      else M[r][j] -= f[r] * prow[j];
    }
    __syncthreads();
  }
  bool bad = false;
  for (int e = tid; e < ka * ka; e += 256) {
    const int r = e / ka, j = e - r * ka;
    const double v = M[r][ka + j];
    bad |= !isfinite(v);
    d.Ginv[sec][r * kcap + j] = v;
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
