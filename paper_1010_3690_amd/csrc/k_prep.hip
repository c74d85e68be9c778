// Preparation products of a block (Sec. IV A): for the k_ins candidates,
//   YT = (N Z)^T   (G of old rows, candidate columns),
//   Rt = X N       (candidate rows of the augmented N, the paper's R~),
//   Gnn = X Y + G0nn (G of candidate rows and columns).
// Each of YT and Rt reads N once.  One workgroup owns a 64-wide panel of the
// output for all candidates, so no cross-workgroup reduction is needed and the
// summation order is fixed.
#include "ctaux_device.h"

namespace ctaux {

constexpr int kPanel = 64;
constexpr int kChunk = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_prep(const ChainDesc *descs, const ChainState *states,
                                              int panels_cap) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active) return;
  const int n = st.n, k = st.k_ins;
  if (n == 0 || k == 0) return;
  const int panels = (n + kPanel - 1) / kPanel;
  // blockIdx.x = (role * 2 + sec) * panels_cap + panel
  const int panel = blockIdx.x % panels_cap;
  const int rs = blockIdx.x / panels_cap;
  const int role = rs >> 1, sec = rs & 1;
  if (panel >= panels) return;
  const T *N = static_cast<const T *>(d.N[st.parity][sec]);
  const double *A = role == 0 ? d.ZT[sec] : d.X[sec];
  double *out = role == 0 ? d.YT[sec] : d.Rt[sec];
  __shared__ double nt[kPanel][kChunk + 1];     // role 0: [row i][k]; role 1: [k][col i] (transposed store)
  __shared__ double at[kMaxKmax][kChunk + 1];   // A[j][k0 + q]
  const int tid = threadIdx.x;
  const int ti = tid & 63, tg = tid >> 6;
  const int i0 = panel * kPanel;
  double acc[kMaxKmax / 4];
#pragma unroll
  for (int q = 0; q < kMaxKmax / 4; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < n; k0 += kChunk) {
    // stage the N panel chunk
    for (int e = tid; e < kPanel * kChunk; e += 256) {
      double v = 0.0;
      if (role == 0) {
        const int r = e / kChunk, q = e % kChunk;      // row i0+r, column k0+q
        if (i0 + r < n && k0 + q < n) v = static_cast<double>(N[static_cast<size_t>(i0 + r) * d.ld + k0 + q]);
        nt[r][q] = v;
      } else {
        const int q = e / kPanel, r = e % kPanel;      // row k0+q, column i0+r
        if (i0 + r < n && k0 + q < n) v = static_cast<double>(N[static_cast<size_t>(k0 + q) * d.ld + i0 + r]);
        nt[r][q] = v;
      }
    }
    for (int e = tid; e < k * kChunk; e += 256) {
      const int j = e / kChunk, q = e % kChunk;
      at[j][q] = (k0 + q < n) ? A[static_cast<size_t>(j) * d.ld + k0 + q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < kMaxKmax / 4; ++jj) {
      const int j = tg + 4 * jj;
      if (j < k) {
        double s = acc[jj];
#pragma unroll 8
        for (int q = 0; q < kChunk; ++q) s += at[j][q] * nt[ti][q];
        acc[jj] = s;
      }
    }
    __syncthreads();
  }
  if (i0 + ti < n) {
#pragma unroll
    for (int jj = 0; jj < kMaxKmax / 4; ++jj) {
      const int j = tg + 4 * jj;
      if (j < k) out[static_cast<size_t>(j) * d.ld + i0 + ti] = acc[jj];
    }
  }
}

// Gnn_jj' = sum_i X_ji YT_j'i + G0nn_jj'.  One workgroup per (candidate j, sector).
__global__ __launch_bounds__(256) void k_gnn(const ChainDesc *descs, const ChainState *states) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active) return;
  const int n = st.n, k = st.k_ins;
  const int j = blockIdx.x >> 1, sec = blockIdx.x & 1;
  if (j >= k) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double *x = d.X[sec] + static_cast<size_t>(j) * d.ld;
  for (int jj = wave; jj < k; jj += 4) {
    const double *y = d.YT[sec] + static_cast<size_t>(jj) * d.ld;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += x[i] * y[i];
    s = wave_sum(s);
    if (lane == 0)
      d.Gnn[sec][static_cast<size_t>(j) * d.kmax + jj] = s + d.G0nn[sec][static_cast<size_t>(j) * d.kmax + jj];
  }
}

void launch_prep(const Batch &b, hipStream_t s) {
  const int panels_cap = (b.n_cap + kPanel - 1) / kPanel;
  dim3 grid(4 * panels_cap, b.n_chains);
  if (b.precision == kFP64)
    hipLaunchKernelGGL(k_prep<double>, grid, dim3(256), 0, s, b.d_desc, b.d_state, panels_cap);
  else
    hipLaunchKernelGGL(k_prep<float>, grid, dim3(256), 0, s, b.d_desc, b.d_state, panels_cap);
  hipLaunchKernelGGL(k_gnn, dim3(2 * b.kmax, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
}

}  // namespace ctaux
