// Measurement at the end of a block (Sec. IV D), from the complete N.
// With T = (e^V - 1) N the Green's function in the field of the auxiliary
// spins is
//   G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k),
// evaluated as W = (e^V - 1) N gR (gR_ky = G0_{x_k y}(tau_k)), then
// G = G0 + gL W with gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l).
// Accumulated per chain: order, sign, densities and double occupancy from the
// equal-time G (tau = 0+), and G(tau_j) averaged over the site pairs of each table.
#include "ctaux_device.h"

namespace ctaux {

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
    d.gR[sec][r] = g0_interp(d, sec, d.site[par][k], y, d.tau[par][k]);
  }
}

constexpr int kMRows = 64, kMChunk = 32, kMaxNc = 128;

// W[l][y] = (e^{V_l} - 1) sum_k N[l][k] gR[k][y]; one workgroup per 64 rows and sector.
template <typename T>
__global__ __launch_bounds__(256) void k_meas_W(const ChainDesc *descs, const ChainState *states,
                                                int blocks_cap) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int n = st.n, nc = d.nc, par = st.parity;
  const int sec = blockIdx.x / blocks_cap, rb = blockIdx.x % blocks_cap;
  const int l0 = rb * kMRows;
  if (l0 >= n) return;
  const T *N = static_cast<const T *>(d.N[par][sec]);
  const double *gR = d.gR[sec];
  __shared__ double nt[kMRows][kMChunk + 1];
  __shared__ double gt[kMChunk][kMaxNc];
  const int tid = threadIdx.x, ti = tid & 63, tg = tid >> 6;
  double acc[kMaxNc / 4];
#pragma unroll
  for (int q = 0; q < kMaxNc / 4; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < n; k0 += kMChunk) {
    for (int e = tid; e < kMRows * kMChunk; e += 256) {
      const int r = e / kMChunk, q = e % kMChunk;
      nt[r][q] = (l0 + r < n && k0 + q < n) ? static_cast<double>(N[static_cast<size_t>(l0 + r) * d.ld + k0 + q]) : 0.0;
    }
    for (int e = tid; e < kMChunk * nc; e += 256) {
      const int q = e / nc, y = e % nc;
      gt[q][y] = (k0 + q < n) ? gR[static_cast<size_t>(k0 + q) * nc + y] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int yy = 0; yy < kMaxNc / 4; ++yy) {
      const int y = tg + 4 * yy;
      if (y < nc) {
        double s = acc[yy];
        for (int q = 0; q < kMChunk; ++q) s += nt[ti][q] * gt[q][y];
        acc[yy] = s;
      }
    }
    __syncthreads();
  }
  const int l = l0 + ti;
  if (l < n) {
    const double f = d.evd[sec][d.s0[par][l] + 2] - 1.0;
#pragma unroll
    for (int yy = 0; yy < kMaxNc / 4; ++yy) {
      const int y = tg + 4 * yy;
      if (y < nc) d.W[sec][static_cast<size_t>(l) * nc + y] = f * acc[yy];
    }
  }
}

// Gxy[row][x*nc + y], row 0: tau = 0+, row j+1: tau_j.  One workgroup per (sector, x, row).
__global__ __launch_bounds__(256) void k_meas_G(const ChainDesc *descs, const ChainState *states,
                                                int x_cap, int rows_cap) {
  const int c = blockIdx.y;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int nc = d.nc, n = st.n, par = st.parity;
  int b = blockIdx.x;
  const int row = b % rows_cap; b /= rows_cap;
  const int x = b % x_cap;
  const int sec = b / x_cap;
  if (x >= nc || row > d.n_out) return;
  const double tau = row == 0 ? 0.0 : (static_cast<double>(row - 1) + 0.5) * d.beta / d.n_out;
  __shared__ double gl[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int l0 = 0; l0 < n; l0 += 256) {
    const int l = l0 + tid;
    gl[tid] = (l < n) ? g0_interp(d, sec, x, d.site[par][l], tau - d.tau[par][l]) : 0.0;
    __syncthreads();
    if (tid < nc) {
      const int lim = min(256, n - l0);
      const double *w = d.W[sec] + static_cast<size_t>(l0) * nc + tid;
      for (int q = 0; q < lim; ++q) acc += gl[q] * w[static_cast<size_t>(q) * nc];
    }
    __syncthreads();
  }
  if (tid < nc)
    d.Gxy[sec][static_cast<size_t>(row) * nc * nc + x * nc + tid] = g0_interp(d, sec, x, tid, tau) + acc;
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
  const int blocks_cap = (b.n_cap + kMRows - 1) / kMRows;
  if (b.precision == kFP64)
    hipLaunchKernelGGL(k_meas_W<double>, dim3(2 * blocks_cap, b.n_chains), dim3(256), 0, s, b.d_desc,
                       b.d_state, blocks_cap);
  else
    hipLaunchKernelGGL(k_meas_W<float>, dim3(2 * blocks_cap, b.n_chains), dim3(256), 0, s, b.d_desc,
                       b.d_state, blocks_cap);
  const int rows_cap = b.n_out_max + 1;
  hipLaunchKernelGGL(k_meas_G, dim3(2 * b.nc_max * rows_cap, b.n_chains), dim3(256), 0, s, b.d_desc,
                     b.d_state, b.nc_max, rows_cap);
  hipLaunchKernelGGL(k_meas_acc, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_state);
}

}  // namespace ctaux
