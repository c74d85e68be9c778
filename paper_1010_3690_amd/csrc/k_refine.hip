// FP64 refinement of N against its definition (Eq. Nmatrix):
//   M = e^V - G0 (e^V - 1) built from the tables (n^2 interpolations),
//   R = I - M N,  N <- N + N R   (one Newton-Schulz step, two FP64 MFMA GEMMs),
//   drift = ||N R||_F / ||N + N R||_F.
// The step squares the relative error of N, so it restores the FP64 inverse of
// the current configuration from an updated N whose error is small (FP64
// rounding drift, or the ~1e-7 error of FP32 storage), and the drift is the
// relative error N had before the step, to first order.
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_build_M(const ChainDesc *descs, const ChainState *states, int c,
                                                 int sec, double *M) {
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  const int n = st.n, par = st.parity;
  const double *tau = d.tau[par];
  const int32_t *site = d.site[par], *s0 = d.s0[par];
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    const double evj = d.evd[sec][s0[j] + 2];
    double v = -g0_interp(d, sec, site[i], site[j], tau[i] - tau[j]) * (evj - 1.0);
    if (i == j) v += d.evd[sec][s0[i] + 2];
    M[static_cast<size_t>(i) * d.ld + j] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_to_f64(const ChainDesc *descs, const ChainState *states, int c,
                                                int sec, double *out) {
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  const int n = st.n;
  const T *N = static_cast<const T *>(d.N[st.parity][sec]);
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    out[static_cast<size_t>(i) * d.ld + j] = static_cast<double>(N[static_cast<size_t>(i) * d.ld + j]);
  }
}

// C = alpha * A B + diag * I   (n x n, leading dimension ld), FP64 MFMA 16x16x4,
// 64x64 tile per workgroup, K staged through LDS in chunks of 16.
constexpr int kGK = 16;
__global__ __launch_bounds__(256) void k_gemm_f64(const ChainState *states, int c, int ld, const double *A,
                                                  const double *B, double *C, double alpha, double diag) {
  const int n = states[c].n;
  const int tiles = (n + 63) / 64;
  const int tti = blockIdx.y, tj = blockIdx.x;
  if (tti >= tiles || tj >= tiles) return;
  __shared__ double As[64][kGK + 1];
  __shared__ double Bs[kGK][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, lr = lane & 15, lk = lane >> 4;
  const int r0 = tti * 64, c0 = tj * 64;
  v4d acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += kGK) {
    for (int e = tid; e < 64 * kGK; e += 256) {
      const int r = e / kGK, q = e % kGK;
      As[r][q] = (r0 + r < n && k0 + q < n) ? A[static_cast<size_t>(r0 + r) * ld + k0 + q] : 0.0;
      const int qb = e / 64, cb = e % 64;
      Bs[qb][cb] = (k0 + qb < n && c0 + cb < n) ? B[static_cast<size_t>(k0 + qb) * ld + c0 + cb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[wr * 32 + i * 16 + lr][kk + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[kk + lk][wc * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr * 32 + i * 16 + lk + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
        const int cc = c0 + wc * 32 + j * 16 + lr;
        if (r < n && cc < n) C[static_cast<size_t>(r) * ld + cc] = alpha * acc[i][j][q] + (r == cc ? diag : 0.0);
      }
}

// N <- N + T (T = N R held in `t`), and per-workgroup partial sums of T^2 and N'^2.
template <typename T>
__global__ __launch_bounds__(256) void k_refine_apply(const ChainDesc *descs, const ChainState *states, int c,
                                                      int sec, const double *nd, const double *t, double *red) {
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  const int n = st.n;
  T *N = static_cast<T *>(d.N[st.parity][sec]);
  const int64_t total = static_cast<int64_t>(n) * n;
  double s_t = 0.0, s_n = 0.0;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    const size_t o = static_cast<size_t>(i) * d.ld + j;
    const double tv = t[o];
    const double nv = nd[o] + tv;
    N[o] = static_cast<T>(nv);
    s_t += tv * tv;
    s_n += nv * nv;
  }
  __shared__ double sh[2][4];
  s_t = wave_sum(s_t);
  s_n = wave_sum(s_n);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = s_t; sh[1][threadIdx.x >> 6] = s_n; }
  __syncthreads();
  if (threadIdx.x == 0) {
    red[2 * (sec * gridDim.x + blockIdx.x)] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    red[2 * (sec * gridDim.x + blockIdx.x) + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

__global__ void k_refine_reduce(ChainState *states, int c, const double *red, int nblk) {
  if (threadIdx.x != 0) return;
  ChainState &st = states[c];
  double drift = 0.0;
  for (int sec = 0; sec < 2; ++sec) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nblk; ++i) {
      a += red[2 * (sec * nblk + i)];
      b += red[2 * (sec * nblk + i) + 1];
    }
    const double dr = (b > 0.0) ? sqrt(a / b) : 0.0;
    if (!isfinite(dr)) drift = INFINITY;
    else if (dr > drift) drift = dr;
  }
  st.last_drift = drift;
  if (!(drift <= st.max_drift)) st.max_drift = drift;
  if (!isfinite(drift) && st.status == 0) st.status = -4;
}

constexpr int kApplyBlocks = 512;

void launch_refine(const Batch &b, hipStream_t s, int32_t c) {
  const int tiles = (b.n_cap + 63) / 64;
  const dim3 ggrid(tiles, tiles);
  const int eblocks = 1024;
  for (int sec = 0; sec < 2; ++sec) {
    hipLaunchKernelGGL(k_build_M, dim3(eblocks), dim3(256), 0, s, b.d_desc, b.d_state, c, sec, b.r_M);
    // N (current parity, known only on the device) is copied into r_N as the FP64 GEMM
    // operand: n^2 traffic, negligible next to the two n^3 products.
    const double *nd;
    if (b.precision == kFP64) {
      hipLaunchKernelGGL(k_to_f64<double>, dim3(eblocks), dim3(256), 0, s, b.d_desc, b.d_state, c, sec, b.r_N);
    } else {
      hipLaunchKernelGGL(k_to_f64<float>, dim3(eblocks), dim3(256), 0, s, b.d_desc, b.d_state, c, sec, b.r_N);
    }
    nd = b.r_N;
    // R = I - M N
    hipLaunchKernelGGL(k_gemm_f64, ggrid, dim3(256), 0, s, b.d_state, c, b.ld, b.r_M, nd, b.r_R, -1.0, 1.0);
    // T = N R  (into r_M)
    hipLaunchKernelGGL(k_gemm_f64, ggrid, dim3(256), 0, s, b.d_state, c, b.ld, nd, b.r_R, b.r_M, 1.0, 0.0);
    if (b.precision == kFP64)
      hipLaunchKernelGGL(k_refine_apply<double>, dim3(kApplyBlocks), dim3(256), 0, s, b.d_desc, b.d_state, c,
                         sec, nd, b.r_M, b.r_red);
    else
      hipLaunchKernelGGL(k_refine_apply<float>, dim3(kApplyBlocks), dim3(256), 0, s, b.d_desc, b.d_state, c,
                         sec, nd, b.r_M, b.r_red);
  }
  hipLaunchKernelGGL(k_refine_reduce, dim3(1), dim3(64), 0, s, b.d_state, c, b.r_red, kApplyBlocks);
}

}  // namespace ctaux
