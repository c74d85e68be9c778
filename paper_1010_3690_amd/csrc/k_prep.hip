// Preparation products of a block (Sec. IV A): for the k_ins candidates,
//   YT = (N Z)^T   (G of old rows, candidate columns),
//   Rt = X N       (candidate rows of the augmented N, the paper's R~),
//   Gnn = X Y + G0nn (G of candidate rows and columns).
// Each of YT and Rt reads N once; both run as skinny MFMA products (k_skinny.hip).
// Gnn has only 2 k_ins^2 outputs: for a few chains it runs as one wave per
// output (a length-n dot product of two contiguous rows), which spreads its
// short work over the whole GPU; for many chains as a skinny product.
#include "ctaux_device.h"

namespace ctaux {

void launch_skinny(const Batch &b, hipStream_t s, int kind);

// Gnn[sec][m][c] = sum_k X[sec][m][k] YT[sec][c][k] + G0nn[sec][m][c], one wave
// per output; lanes take k = lane + 64 i, summed in a fixed order.
__global__ __launch_bounds__(256) void k_gnn_dot(const ChainDesc *descs, const ChainState *states) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active) return;
  const int n = st.n, ki = st.k_ins, ld = d.ld, km = d.kmax, rt = (km + 15) >> 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per = ki * ki;
  for (int w = blockIdx.x * 4 + wave; w < 2 * per; w += gridDim.x * 4) {
    const int sec = w >= per ? 1 : 0, r = w - sec * per, m = r / ki, cc = r - m * ki;
    const auto X = gview(d.X[sec]);
    const auto YT = gview(d.YT[sec] + static_cast<size_t>(cc) * ld);
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 64 * 8) {   // eight loads of each row in flight
      double x[8], y[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + 64 * i + lane;
        x[i] = k < n ? X[cand_offset(m, k, rt)] : 0.0;
        y[i] = k < n ? YT[k] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i & 3] += x[i] * y[i];
    }
    const double s = wave_sum_dpp((a[0] + a[1]) + (a[2] + a[3]));
    if (lane == 0)
      gview_w(d.Gnn[sec])[static_cast<size_t>(m) * km + cc] = s + gview(d.G0nn[sec])[static_cast<size_t>(m) * km + cc];
  }
}

void launch_prep(const Batch &b, hipStream_t s) {
  launch_skinny(b, s, 0);   // YT = ZT N^T, Rt = X N
  if (b.n_chains < 8)
    hipLaunchKernelGGL(k_gnn_dot, dim3(512, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
  else
    launch_skinny(b, s, 1);   // Gnn = X YT^T + G0nn
}

}  // namespace ctaux
