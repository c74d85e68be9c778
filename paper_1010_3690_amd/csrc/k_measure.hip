// Measurement at the end of a block (Sec. IV D), from the complete N.
// With T = (e^V - 1) N the Green's function in the field of the auxiliary
// spins is
//   G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k),
// evaluated as W = N gR (gR_ky = G0_{x_k y}(tau_k), stored transposed), then
// G = G0 + gL W with gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l) (e^{V_l} - 1)
// (the output times are tau = 0+ and tau_j = (j - 1/2) beta / n_out, j >= 1,
// row j*nc + x), tabulated first for a few chains and interpolated inside the
// product for many.
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
  const int n = st.n, nc = d.nc, par = st.parity, rt = (nc + 15) >> 4;
  // rows y, columns k, stored in the blocked order of cand_offset (the W product's
  // operand order); 32-bit indices
  const int per = n * nc;
  for (int e = cb.sub * 256 + threadIdx.x; e < 2 * per; e += cb.g * 256) {
    const int sec = e >= per ? 1 : 0;
    const int r = e - sec * per;
    const int y = r / n, k = r - y * n;
    gview_w(d.gR[sec])[cand_offset(y, k, rt)] =
        g0_interp(d, sec, gview(d.site[par])[k], y, gview(d.tau[par])[k]);
  }
}

// gL_{(j, x), l} = G0_{x x_l}(tau_j - tau_l) (e^{V_l} - 1) for the output times
// tau_0 = 0+ and tau_j = (j - 1/2) beta / n_out, j >= 1 (row j*nc + x), as a
// table: batches of fewer than 8 chains, whose G product splits K over the
// waves of a workgroup and has too few items to hide interpolations in its k
// loop (many chains interpolate gL inside the product instead).
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

// Time order of the vertices for the measurement of many chains (one workgroup
// per chain): a stable sort into 128 buckets of tau (ascending index within a
// bucket, so the order does not depend on thread timing); records the position
// of every vertex and, per position, its tau, site and e^{V} - 1 of both
// sectors.  The G product then interpolates consecutive vertices from
// neighbouring table entries.
constexpr int kTauBuckets = 128;
__global__ __launch_bounds__(256) void k_meas_tsort(const ChainDesc *descs, const ChainState *states) {
  __shared__ int cnt[kTauBuckets], run[kTauBuckets], chunk_b[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now) return;
  const int n = st.n, par = st.parity;
  const auto tau = gview(d.tau[par]);
  const auto site = gview(d.site[par]), s0 = gview(d.s0[par]);
  const double scale = kTauBuckets / d.beta;
  auto bucket = [&](int i) { return min(kTauBuckets - 1, static_cast<int>(tau[i] * scale)); };
  for (int b = tid; b < kTauBuckets; b += 256) cnt[b] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += 256) atomicAdd(&cnt[bucket(i)], 1);   // integer counts: any order
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b < kTauBuckets; ++b) {
      run[b] = acc;
      acc += cnt[b];
    }
  }
  __syncthreads();
  for (int base = 0; base < n; base += 256) {
    const int i = base + tid;
    const int bi = i < n ? bucket(i) : -1;
    chunk_b[tid] = bi;
    __syncthreads();
    if (i < n) {
      int r = 0;
      for (int j = 0; j < tid; ++j) r += chunk_b[j] == bi;
      const int pos = run[bi] + r;
      gview_w(d.mpos)[i] = pos;
      gview_w(d.mtau)[pos] = tau[i];
      gview_w(d.msite)[pos] = site[i];
      gview_w(d.mfac)[pos] = gview(d.evd[0])[s0[i] + 2] - 1.0;
      gview_w(d.mfac)[d.n_cap + pos] = gview(d.evd[1])[s0[i] + 2] - 1.0;
    }
    __syncthreads();
    if (tid < kTauBuckets) {
      int add = 0;
      for (int j = 0; j < 256; ++j) add += chunk_b[j] == tid;
      run[tid] += add;
    }
    __syncthreads();
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

// ---- measurement in cluster momenta and Matsubara frequencies (Sec. IV D) ----
// The real-space estimator, transformed in both of its arguments (time and
// site), gives G(K, i w) = G0(K, i w) + G0(K, i w)^2 S(K, w) / (beta Nc) with
//   S(K, w) = sum_{l,k} e^{i w tau_l - i K.r_l} M_lk e^{-i w tau_k + i K.r_k},  M = (e^V - 1) N.
// With the vertices grouped by site, S(K, w) = sum_{x,x'} e^{-i K.r_x} e^{i K.r_x'} C_xx'(w),
//   C_xx'(w) = sum_{l at x} e^{i w tau_l} (e^{V_l} - 1) sum_{k at x'} N_lk e^{-i w tau_k},
// which reads N once and costs 4 n^2 N_w flops per sector (not n^2 N_K N_w).

__device__ __forceinline__ double matsubara(const ChainDesc &d, int m) {
  return (2.0 * m + 1.0) * 3.14159265358979323846 / d.beta;
}

// Vertices sorted by site (stable: ascending index within a site) and the
// phases e^{-i w_n tau_k}; one workgroup per chain.
__global__ __launch_bounds__(256) void k_meas_kw_sort(const ChainDesc *descs, const ChainState *states) {
  __shared__ int cnt[128], run[128], chunk_site[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now || d.n_mats == 0) return;
  const int n = st.n, nc = d.nc, nm = d.n_mats, par = st.parity;
  const auto site = gview(d.site[par]);
  const auto tau = gview(d.tau[par]);
  for (int x = tid; x < nc; x += 256) cnt[x] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += 256) atomicAdd(&cnt[site[i]], 1);   // integer counts: any order
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int x = 0; x < nc; ++x) {
      gview_w(d.kw_off)[x] = acc;
      run[x] = acc;
      acc += cnt[x];
    }
    gview_w(d.kw_off)[nc] = acc;
  }
  __syncthreads();
  for (int base = 0; base < n; base += 256) {
    const int i = base + tid;
    const int sx = i < n ? site[i] : -1;
    chunk_site[tid] = sx;
    __syncthreads();
    if (i < n) {
      int r = 0;
      for (int j = 0; j < tid; ++j) r += chunk_site[j] == sx;
      gview_w(d.kw_list)[run[sx] + r] = i;
    }
    __syncthreads();
    if (tid < nc) {
      int add = 0;
      for (int j = 0; j < 256; ++j) add += chunk_site[j] == tid;
      run[tid] += add;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * nm; e += 256) {
    const int k = e / nm, m = e - k * nm;
    double sn, cs;
    sincos(matsubara(d, m) * tau[k], &sn, &cs);
    gview_w(d.kw_ph)[2 * e] = cs;
    gview_w(d.kw_ph)[2 * e + 1] = -sn;
  }
}

// C_xx'(w) for one (chain, sector, site x) per workgroup:
//   C_xx'(w) = sum_{l in x} e^{i w tau_l} (e^{V_l} - 1) sum_{k in x'} N_lk e^{-i w tau_k}.
// Wave w takes the sites x' = w, w + 4, ...; lane (r, m) takes frequency m and
// row r of a pass over up to 16 rows of site x, so the lanes of one row read
// the same N entry (one transaction for all frequencies) and each N entry of
// the pass is loaded once.  The rows' partial sums are added in a fixed order
// through LDS: deterministic, no atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_meas_kw_C(const ChainDesc *descs, const ChainState *states, int nc_max) {
  __shared__ double red[4][64][2];
  const int c = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now || d.n_mats == 0) return;
  const int sec = blockIdx.x >= nc_max ? 1 : 0, x = blockIdx.x - sec * nc_max;
  const int nc = d.nc, nm = d.n_mats, par = st.parity, ld = d.ld;
  if (x >= nc) return;
  const auto N = gview(static_cast<const T *>(d.N[par][sec]));
  const auto s0 = gview(d.s0[par]);
  const auto off = gview(d.kw_off);
  const auto list = gview(d.kw_list);
  const auto ph = gview(d.kw_ph);
  const auto evd = gview(d.evd[sec]);
  int mp = 1;   // frequencies padded to a power of two (n_matsubara <= 32)
  while (mp < nm) mp <<= 1;
  const int rows = min(16, 64 / mp);           // rows of site x per pass
  const int r = lane / mp, m = lane - r * mp;  // lane's row in the pass, frequency
  const bool mine = m < nm && r < rows;
  const int l0 = off[x], l1 = off[x + 1], nb = nc * nm;
  double *C = d.kw_C + 2 * (static_cast<size_t>(sec) * nc + x) * nb;
  for (int xp = wave; xp < nc; xp += 4) {
    const int k0 = off[xp], k1 = off[xp + 1];
    double cre = 0.0, cim = 0.0;
    for (int lb = l0; lb < l1; lb += rows) {
      const bool on = mine && lb + r < l1;
      const int l = on ? list[lb + r] : list[l0];   // an in-range row for idle lanes (value unused)
      const auto nrow = N + static_cast<size_t>(l) * ld;
      const int mm = m < nm ? m : 0;
      double yre = 0.0, yim = 0.0;
      int ki = k0;
      for (; ki + 4 <= k1; ki += 4) {   // four independent loads in flight
        const int ka = list[ki], kb = list[ki + 1], kc = list[ki + 2], kd = list[ki + 3];
        const double na = static_cast<double>(nrow[ka]), nb2 = static_cast<double>(nrow[kb]);
        const double nc2 = static_cast<double>(nrow[kc]), nd = static_cast<double>(nrow[kd]);
        const auto pa = ph + 2 * (ka * nm + mm), pb = ph + 2 * (kb * nm + mm);
        const auto pc = ph + 2 * (kc * nm + mm), pd = ph + 2 * (kd * nm + mm);
        yre = fma(na, pa[0], yre);
        yim = fma(na, pa[1], yim);
        yre = fma(nb2, pb[0], yre);
        yim = fma(nb2, pb[1], yim);
        yre = fma(nc2, pc[0], yre);
        yim = fma(nc2, pc[1], yim);
        yre = fma(nd, pd[0], yre);
        yim = fma(nd, pd[1], yim);
      }
      for (; ki < k1; ++ki) {
        const int k = list[ki];
        const double nlk = static_cast<double>(nrow[k]);
        yre = fma(nlk, ph[2 * (k * nm + mm)], yre);
        yim = fma(nlk, ph[2 * (k * nm + mm) + 1], yim);
      }
      if (on) {
        const double evl = evd[s0[l] + 2] - 1.0;
        // e^{+i w tau_l} = conj(ph_l)
        const double pr = ph[2 * (l * nm + m)], pi = -ph[2 * (l * nm + m) + 1];
        cre += evl * (pr * yre - pi * yim);
        cim += evl * (pr * yim + pi * yre);
      }
    }
    // rows of the pass in a fixed order: lane m collects lanes m, m + mp, ...
    red[wave][lane][0] = cre;
    red[wave][lane][1] = cim;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    if (lane < nm) {
      double sre = 0.0, sim = 0.0;
      for (int q = 0; q < rows; ++q) {
        sre += red[wave][q * mp + lane][0];
        sim += red[wave][q * mp + lane][1];
      }
      gview_w(C)[2 * (xp * nm + lane)] = sre;
      gview_w(C)[2 * (xp * nm + lane) + 1] = sim;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();   // red is reused for the next site
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }
}

// S(K, w) = sum_x e^{-i K.r_x} sum_x' e^{i K.r_x'} C_xx'(w), accumulated with the
// configuration's sign; one workgroup per (chain, K).
__global__ __launch_bounds__(256) void k_meas_kw_S(const ChainDesc *descs, const ChainState *states) {
  __shared__ double P[128][2];
  __shared__ double Tsh[2048][2];   // n_sites * n_matsubara <= 2048
  const int c = blockIdx.y, q = blockIdx.x, tid = threadIdx.x;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active || !st.meas_now || d.n_mats == 0 || q >= d.n_k) return;
  const int nc = d.nc, nm = d.n_mats;
  const double *K = d.kw_k + 3 * q;
  for (int x = tid; x < nc; x += 256) {
    const double *r = d.kw_pos + 3 * x;
    double sn, cs;
    sincos(K[0] * r[0] + K[1] * r[1] + K[2] * r[2], &sn, &cs);
    P[x][0] = cs;   // e^{i K.r_x}
    P[x][1] = sn;
  }
  __syncthreads();
  const double w = st.sign;
  for (int sec = 0; sec < 2; ++sec) {
    const double *C = d.kw_C + 2 * static_cast<size_t>(sec) * nc * nc * nm;
    for (int e = tid; e < nc * nm; e += 256) {
      const int x = e / nm, m = e - x * nm;
      double tr = 0.0, ti = 0.0;
      for (int xp = 0; xp < nc; ++xp) {
        const double *cv = C + 2 * ((static_cast<size_t>(x) * nc + xp) * nm + m);
        tr += P[xp][0] * cv[0] - P[xp][1] * cv[1];
        ti += P[xp][0] * cv[1] + P[xp][1] * cv[0];
      }
      Tsh[e][0] = tr;
      Tsh[e][1] = ti;
    }
    __syncthreads();
    for (int m = tid; m < nm; m += 256) {
      double sr = 0.0, si = 0.0;
      for (int x = 0; x < nc; ++x) {   // e^{-i K.r_x} = conj(P_x)
        const double *tv = Tsh[x * nm + m];
        sr += P[x][0] * tv[0] + P[x][1] * tv[1];
        si += P[x][0] * tv[1] - P[x][1] * tv[0];
      }
      double *o = d.obs_kw + 2 * ((static_cast<size_t>(sec) * d.n_k + q) * nm + m);
      o[0] += w * sr;
      o[1] += w * si;
    }
    __syncthreads();
  }
}

// G0(K, i w_n) = (1/Nc) sum_{x,y} e^{-i K.(r_x - r_y)} g_{d(x,y)}(i w_n), where
// g_d(i w) = int_0^beta e^{i w s} g_d(s) ds for the linear interpolant of table d
// on the grid s_m = m h:  sum_m e^{i w s_m} (g_m A + g_{m+1} B) with
//   A = int_0^h e^{i w u} (1 - u/h) du,  B = int_0^h e^{i w u} (u/h) du
// (power series in i w h below w h = 1, closed forms above).  One workgroup
// per chain; the table transforms are staged in kw_C.
__device__ void seg_weights(double theta, double h, double *A, double *B) {
  if (theta < 1.0) {
    // A = h sum_j (i theta)^j / (j! (j+1)(j+2)),  B = h sum_j (i theta)^j / (j! (j+2))
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    double pr = 1.0, pi = 0.0;   // (i theta)^j / j!
    for (int j = 0; j < 24; ++j) {
      const double fa = 1.0 / ((j + 1.0) * (j + 2.0)), fb = 1.0 / (j + 2.0);
      ar += pr * fa; ai += pi * fa;
      br += pr * fb; bi += pi * fb;
      const double nr = -pi * theta / (j + 1.0), ni = pr * theta / (j + 1.0);
      pr = nr;
      pi = ni;
    }
    A[0] = h * ar; A[1] = h * ai; B[0] = h * br; B[1] = h * bi;
  } else {
    double sn, cs;
    sincos(theta, &sn, &cs);
    // E - 1 with E = e^{i theta};  int_0^1 e^{i theta t} dt = (E - 1)/(i theta)
    const double er = cs - 1.0, ei = sn;
    const double ir = ei / theta, ii = -er / theta;                 // (E - 1)/(i theta)
    // int_0^1 t e^{i theta t} dt = E/(i theta) + (E - 1)/theta^2
    const double tr = sn / theta + er / (theta * theta), ti = -cs / theta + ei / (theta * theta);
    B[0] = h * tr; B[1] = h * ti;
    A[0] = h * (ir - tr); A[1] = h * (ii - ti);
  }
}

__global__ __launch_bounds__(256) void k_kw_g0(const ChainDesc *descs) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const ChainDesc &d = descs[c];
  if (d.n_mats == 0) return;
  const int nm = d.n_mats, nd = d.n_disp, nt = d.n_tau, nc = d.nc;
  const double h = d.beta / (nt - 1);
  double *gt = d.kw_C;   // [2][nd][nm][2]
  for (int e = tid; e < 2 * nd * nm; e += 256) {
    const int sec = e / (nd * nm), r = e - sec * nd * nm, dd = r / nm, m = r - dd * nm;
    const double om = matsubara(d, m);
    double A[2], B[2];
    seg_weights(om * h, h, A, B);
    const double *tab = d.g0[sec] + static_cast<size_t>(dd) * nt;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j + 1 < nt; ++j) {
      double sn, cs;
      sincos(om * (j * h), &sn, &cs);
      const double vr = tab[j] * A[0] + tab[j + 1] * B[0], vi = tab[j] * A[1] + tab[j + 1] * B[1];
      sr += cs * vr - sn * vi;
      si += cs * vi + sn * vr;
    }
    gt[2 * e] = sr;
    gt[2 * e + 1] = si;
  }
  __syncthreads();
  for (int e = tid; e < 2 * d.n_k * nm; e += 256) {
    const int sec = e / (d.n_k * nm), r = e - sec * d.n_k * nm, q = r / nm, m = r - q * nm;
    const double *K = d.kw_k + 3 * q;
    double sr = 0.0, si = 0.0;
    for (int x = 0; x < nc; ++x)
      for (int y = 0; y < nc; ++y) {
        const double *rx = d.kw_pos + 3 * x, *ry = d.kw_pos + 3 * y;
        double sn, cs;
        sincos(-(K[0] * (rx[0] - ry[0]) + K[1] * (rx[1] - ry[1]) + K[2] * (rx[2] - ry[2])), &sn, &cs);
        const double *g = gt + 2 * ((static_cast<size_t>(sec) * nd + d.site_disp[x * nc + y]) * nm + m);
        sr += cs * g[0] - sn * g[1];
        si += cs * g[1] + sn * g[0];
      }
    d.kw_g0[2 * e] = sr / nc;
    d.kw_g0[2 * e + 1] = si / nc;
  }
}

void launch_kw_g0(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_kw_g0, dim3(b.n_chains), dim3(256), 0, s, b.d_desc);
}

void launch_measure(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL(k_meas_gR, chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_mstate, b.n_chains, chain_grid_arg(b));
  if (b.n_chains < 8)
    hipLaunchKernelGGL(k_meas_gL, chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_mstate, b.n_chains,
                       chain_grid_arg(b));
  else
    hipLaunchKernelGGL(k_meas_tsort, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate);
  launch_skinny(b, s, 2);   // W = N gR
  launch_skinny(b, s, 3);   // Gxy = G0 + gL W, gL_{(x,tau), l} = G0_{x x_l}(tau - tau_l)(e^{V_l} - 1)
  hipLaunchKernelGGL(k_meas_acc, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate);
  if (b.n_mats > 0) {
    hipLaunchKernelGGL(k_meas_kw_sort, dim3(b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate);
    if (b.precision == kFP64)
      hipLaunchKernelGGL(k_meas_kw_C<double>, dim3(2 * b.nc_max, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate,
                         b.nc_max);
    else
      hipLaunchKernelGGL(k_meas_kw_C<float>, dim3(2 * b.nc_max, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate,
                         b.nc_max);
    hipLaunchKernelGGL(k_meas_kw_S, dim3(b.n_k_max, b.n_chains), dim3(256), 0, s, b.d_desc, b.d_mstate);
  }
}

}  // namespace ctaux
