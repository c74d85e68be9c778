// Measurement at the end of a block (Sec. IV D), from the complete N.
// With T = (e^V - 1) N the Green's function in the field of the auxiliary
// spins is
//   G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k),
// evaluated as W = N gR (gR_ky = G0_{x_k y}(tau_k), stored transposed), then
// G = G0 + gL W with gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l) (e^{V_l} - 1).
// Accumulated per chain: order, sign, densities and double occupancy from the
// equal-time G (tau = 0+), and G(tau_j) averaged over the site pairs of each table.
#include "ctaux_device.h"

namespace ctaux {

void launch_skinny(const Batch &b, hipStream_t s, int kind);

__global__ __launch_bounds__(256) void k_meas_gR(const ChainDesc *descs, const ChainState *states) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int n = st.n, nc = d.nc, par = st.parity;
  const int64_t per = static_cast<int64_t>(n) * nc;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < 2 * per; e += gridDim.x * 256ll) {
    const int sec = static_cast<int>(e / per);
    const int64_t r = e - sec * per;
    const int k = static_cast<int>(r / nc), y = static_cast<int>(r - static_cast<int64_t>(k) * nc);
    d.gR[sec][static_cast<size_t>(y) * d.n_cap + k] = g0_interp(d, sec, d.site[par][k], y, d.tau[par][k]);
  }
}

// Accumulate the observables of one measurement (one workgroup per chain).
__global__ __launch_bounds__(256) void k_meas_acc(const ChainDesc *descs, const ChainState *states) {
  const int c = blockIdx.x;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int nc = d.nc, no = d.n_out, nd = d.n_disp;
  const double w = st.sign;
  double *o = d.obs;
  const int tid = threadIdx.x;
  if (tid == 0) {
    double dsum = 0.0, nu = 0.0, ndn = 0.0;
    for (int x = 0; x < nc; ++x) {
      const double a = 1.0 - d.Gxy[0][x * nc + x];
      const double b = 1.0 - d.Gxy[1][x * nc + x];
      nu += a;
      ndn += b;
      dsum += a * b;
    }
    const double n = static_cast<double>(st.n);
    o[0] += 1.0;
    o[1] += w;
    o[2] += w * n;
    o[3] += w * n * n;
    o[4] += (st.n == 0) ? w : 0.0;
    o[5] += w * dsum / nc;
    o[6] += w * nu / nc;
    o[7] += w * ndn / nc;
  }
  for (int e = tid; e < 2 * nd * no; e += 256) {
    const int sec = e / (nd * no), r = e - sec * nd * no;
    const int dd = r / no, j = r - dd * no;
    const int b0 = d.cls_off[dd], b1 = d.cls_off[dd + 1];
    double s = 0.0;
    for (int q = b0; q < b1; ++q) s += d.Gxy[sec][static_cast<size_t>(j + 1) * nc * nc + d.cls_pairs[q]];
    if (b1 > b0) o[8 + e] += w * s / (b1 - b0);
  }
}

void launch_measure(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_gR, dim3(b.grid_per_chain, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
  launch_skinny(b, s, 2);   // W = N gR
  launch_skinny(b, s, 3);   // Gxy = G0 + gL W, gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l)(e^{V_l} - 1)
  hipLaunchKernelGGL(k_meas_acc, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
}

}  // namespace ctaux
