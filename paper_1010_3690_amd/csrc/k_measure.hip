// Measurement at the end of a block (Sec. IV D), from the complete N.
// With T = (e^V - 1) N the Green's function in the field of the auxiliary
// spins is
//   G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k),
// evaluated as W = N gR (gR_ky = G0_{x_k y}(tau_k), stored transposed), then
// G = G0 + gL W with gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l) (e^{V_l} - 1)
// tabulated by its own kernel (every entry an independent interpolation).
// Accumulated per chain: order, sign, densities and double occupancy from the
// equal-time G (tau = 0+), and G(tau_j) averaged over the site pairs of each table.
#include "ctaux_device.h"

namespace ctaux {

void launch_skinny(const Batch &b, hipStream_t s, int kind);

__global__ __launch_bounds__(256) void k_meas_gR(const ChainDesc *descs, const ChainState *states, int n_chains,
                                                 int xcd_g) {
  const ChainBlock cb = chain_block(xcd_g);
  const int c = cb.c;
  if (c >= n_chains) return;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int n = st.n, nc = d.nc, par = st.parity;
  // rows y, columns k (consecutive threads write consecutive k); 32-bit indices
  const int per = n * nc;
  for (int e = cb.sub * 256 + threadIdx.x; e < 2 * per; e += cb.g * 256) {
    const int sec = e >= per ? 1 : 0;
    const int r = e - sec * per;
    const int y = r / n, k = r - y * n;
    gview_w(d.gR[sec])[static_cast<size_t>(y) * d.n_cap + k] =
        g0_interp(d, sec, gview(d.site[par])[k], y, gview(d.tau[par])[k]);
  }
}

// gL_{(j, x), l} = G0_{x x_l}(tau_j - tau_l) (e^{V_l} - 1) for the output times
// tau_0 = 0+ and tau_j = (j - 1/2) beta / n_out, j >= 1 (row j*nc + x).
__global__ __launch_bounds__(256) void k_meas_gL(const ChainDesc *descs, const ChainState *states, int n_chains,
                                                 int xcd_g) {
  const ChainBlock cb = chain_block(xcd_g);
  const int c = cb.c;
  if (c >= n_chains) return;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int n = st.n, nc = d.nc, par = st.parity, ld = d.ld;
  const int rows = nc * (d.n_out + 1);
  const double dt = d.beta / d.n_out;
  const int per = rows * n;   // 32-bit indices: 2 (n_out + 1) nc n < 2^31
  const auto tau = gview(d.tau[par]);
  const auto site = gview(d.site[par]), s0 = gview(d.s0[par]);
  for (int e = cb.sub * 256 + threadIdx.x; e < 2 * per; e += cb.g * 256) {
    const int sec = e >= per ? 1 : 0;
    const int r = e - sec * per;
    const int m = r / n, l = r - m * n;
    const int j = m / nc, x = m - j * nc;
    const double tj = j == 0 ? 0.0 : (static_cast<double>(j - 1) + 0.5) * dt;
    gview_w(d.gL[sec])[static_cast<size_t>(m) * ld + l] =
        g0_interp(d, sec, x, site[l], tj - tau[l]) * (gview(d.evd[sec])[s0[l] + 2] - 1.0);
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
  if (tid < 64) {
    // equal-time densities n_sigma(x) = 1 - G_sigma(x 0+; x 0) and their product, lanes over x
    double nu = 0.0, ndn = 0.0, dsum = 0.0;
    for (int x = tid; x < nc; x += 64) {
      const double a = 1.0 - d.Gxy[0][x * nc + x];
      const double b = 1.0 - d.Gxy[1][x * nc + x];
      nu += a;
      ndn += b;
      dsum += a * b;
    }
    nu = wave_sum_dpp(nu);
    ndn = wave_sum_dpp(ndn);
    dsum = wave_sum_dpp(dsum);
    if (tid == 0) {
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
  }
  // G(tau_j) averaged over the site pairs of each table; member loads eight at a time
  for (int e = tid; e < 2 * nd * no; e += 256) {
    const int sec = e / (nd * no), r = e - sec * nd * no;
    const int dd = r / no, j = r - dd * no;
    const int b0 = d.cls_off[dd], b1 = d.cls_off[dd + 1];
    const double *g = d.Gxy[sec] + static_cast<size_t>(j + 1) * nc * nc;
    double s = 0.0;
    for (int q0 = b0; q0 < b1; q0 += 8) {
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (q0 + i < b1) ? g[d.cls_pairs[q0 + i]] : 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) s += v[i];
    }
    if (b1 > b0) o[8 + e] += w * s / (b1 - b0);
  }
}

void launch_measure(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_gR, chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_mstate, b.n_chains, chain_grid_arg(b));
  hipLaunchKernelGGL(k_meas_gL, chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_mstate, b.n_chains, chain_grid_arg(b));
  launch_skinny(b, s, 2);   // W = N gR
  launch_skinny(b, s, 3);   // Gxy = G0 + gL W, gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l)(e^{V_l} - 1)
  hipLaunchKernelGGL(k_meas_acc, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate);
}

}  // namespace ctaux
