// Skinny products with few rows and long K on MFMA f64 16x16x4:
//   C[m][c] = sum_k A(m, k) * B(k, c) (+ D[m][c]),  m < M <= 128 per job, k < K, c < Ncols,
//   B(k, c) = B[k][c] or, transposed, B[c][k].
// They are the preparation products of a block (Sec. IV A): YT = ZT N^T,
// Rt = X N (both read N once), Gnn = X YT^T + G0nn; and the measurement
// (Sec. IV D): W = N gR, then G(x tau_j; y 0) = G0 + gL W with the rows of gL
// evaluated from the G0 tables inside the loop.  One workgroup owns a
// 16-column output tile; its 8 waves split K and their partial tiles are
// summed in LDS in a fixed order (deterministic).
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kSkWaves = 8;
constexpr int kSkMaxRt = kMaxKmax / 16;   // row tiles per job (M <= 128)
constexpr int kSkUnroll = 2;
constexpr int kSkThreads = kSkWaves * 64;
constexpr int kMeasGRows = 16;           // rows of gL per measurement work item

enum SkinnyKind : int { kSkPrep = 0, kSkGnn = 1, kSkMeasW = 2, kSkMeasG = 3 };

template <typename T>
__device__ __forceinline__ double b_load(const T *B, int ldb, int trans, int k, int c) {
  return trans ? static_cast<double>(B[static_cast<size_t>(c) * ldb + k])
               : static_cast<double>(B[static_cast<size_t>(k) * ldb + c]);
}

// Partial products of this workgroup's waves, reduced into red[nrt*256].
template <typename T, typename AF>
__device__ void skinny_core(AF afn, const T *B, int ldb, int trans, int M, int K, int Ncols, int c0,
                            double *red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nrt = (M + 15) >> 4;
  v4d acc[kSkMaxRt];
#pragma unroll
  for (int r = 0; r < kSkMaxRt; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
  const int c = c0 + lr;
  const bool cok = c < Ncols;
  for (int k0 = wave * 4; k0 < K; k0 += kSkWaves * 4 * kSkUnroll) {
    double bv[kSkUnroll], av[kSkUnroll][kSkMaxRt];
#pragma unroll
    for (int u = 0; u < kSkUnroll; ++u) {
      const int k = k0 + u * kSkWaves * 4 + lk;
      const bool kok = k < K;
      bv[u] = (cok && kok) ? b_load<T>(B, ldb, trans, k, c) : 0.0;
#pragma unroll
      for (int r = 0; r < kSkMaxRt; ++r) {
        const int m = r * 16 + lr;
        av[u][r] = (r < nrt && m < M && kok) ? afn(m, k) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kSkUnroll; ++u)
#pragma unroll
      for (int r = 0; r < kSkMaxRt; ++r)
        if (r < nrt) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][r], bv[u], acc[r], 0, 0, 0);
  }
  for (int w = 0; w < kSkWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < kSkMaxRt; ++r) {
        if (r < nrt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double *p = red + (r * 64 + lane) * 4 + q;
            *p = (w == 0) ? acc[r][q] : *p + acc[r][q];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Element e of red (after skinny_core) is output row m, column cc.
__device__ __forceinline__ void red_index(int e, int c0, int &m, int &cc) {
  const int r = e >> 8, l = (e >> 2) & 63, q = e & 3;
  m = r * 16 + (l >> 4) + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
  cc = c0 + (l & 15);
}

// Work items of one chain for a kind (0 when the chain does not take part).
__device__ __forceinline__ int skinny_items(const ChainDesc &d, const ChainState &st, int kind) {
  if (!st.active) return 0;
  const int n = st.n;
  if (kind == kSkPrep) return st.k_ins > 0 ? 4 * ((n + 15) >> 4) : 0;
  if (kind == kSkGnn) return st.k_ins > 0 ? 2 * ((st.k_ins + 15) >> 4) : 0;
  if (!st.meas_now) return 0;
  if (kind == kSkMeasW) return 2 * ((n + 15) >> 4);
  const int mtot = d.nc * (d.n_out + 1);
  return 2 * ((mtot + kMeasGRows - 1) / kMeasGRows) * ((d.nc + 15) >> 4);
}

// Persistent over the work items of all chains: every workgroup builds the
// per-chain prefix of work items in LDS (no separate scan launch), then takes
// items blockIdx.x, blockIdx.x + gridDim.x, ...
template <typename T>
__global__ __launch_bounds__(kSkThreads) void k_skinny(const ChainDesc *descs, const ChainState *states, int kind,
                                                        int n_chains) {
  extern __shared__ int pre[];   // [n_chains + 1]
  __shared__ int scan[kSkThreads];
  __shared__ int carry;
  __shared__ double red[kSkMaxRt * 256];
  const int tid = threadIdx.x;
  if (tid == 0) { carry = 0; pre[0] = 0; }
  __syncthreads();
  for (int base = 0; base < n_chains; base += kSkThreads) {
    const int cc = base + tid;
    scan[tid] = cc < n_chains ? skinny_items(descs[cc], states[cc], kind) : 0;
    __syncthreads();
    for (int off = 1; off < kSkThreads; off <<= 1) {
      const int v = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    if (cc < n_chains) pre[cc + 1] = carry + scan[tid];
    __syncthreads();
    if (tid == 0) carry += scan[kSkThreads - 1];
    __syncthreads();
  }
  const int total = pre[n_chains];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int lo = 0, hi = n_chains;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= item) lo = mid; else hi = mid;
    }
    const int c = lo, local = item - pre[c];
    const ChainDesc &d = descs[c];
    const ChainState &st = states[c];
    const int n = st.n, par = st.parity;
    if (kind == kSkMeasG) {
      // rows m = j*nc + x (j = 0: tau = 0+, j >= 1: tau_{j-1}); group g holds rows [16 g, 16 g + 16)
      const int nc = d.nc, Mtot = nc * (d.n_out + 1);
      const int ngroups = (Mtot + kMeasGRows - 1) / kMeasGRows, ntiles = (nc + 15) >> 4;
      const int sec = local / (ngroups * ntiles), rem = local - sec * ngroups * ntiles;
      const int g = rem / ntiles, c0 = (rem - g * ntiles) * 16;
      const int m0 = g * kMeasGRows, M = min(kMeasGRows, Mtot - m0);
      const double *tau = d.tau[par];
      const int32_t *site = d.site[par], *s0 = d.s0[par];
      const double dt = d.beta / d.n_out;
      auto afn = [&](int m, int l) -> double {
        const int mm = m0 + m, j = mm / nc, x = mm - j * nc;
        const double tj = j == 0 ? 0.0 : (static_cast<double>(j - 1) + 0.5) * dt;
        return g0_interp(d, sec, x, site[l], tj - tau[l]) * (d.evd[sec][s0[l] + 2] - 1.0);
      };
      skinny_core<double>(afn, d.W[sec], nc, 0, M, n, nc, c0, red);
      for (int e = tid; e < ((M + 15) >> 4) * 256; e += kSkThreads) {
        int m, cc;
        red_index(e, c0, m, cc);
        if (m < M && cc < nc) {
          const int mm = m0 + m, j = mm / nc, x = mm - j * nc;
          const double tj = j == 0 ? 0.0 : (static_cast<double>(j - 1) + 0.5) * dt;
          d.Gxy[sec][static_cast<size_t>(j) * nc * nc + x * nc + cc] = g0_interp(d, sec, x, cc, tj) + red[e];
        }
      }
      __syncthreads();
      continue;
    }
    int M, K = n, Ncols, lda, ldb, ldc, ldd = 0, trans, out_trans = 0, job, c0;
    const double *A, *D = nullptr;
    const void *B;
    double *C;
    if (kind == kSkPrep) {
      // job 0,1: YT[sec] = ZT N^T ; job 2,3: Rt[sec] = X N
      const int nt = (n + 15) >> 4;
      job = local / nt; c0 = (local - job * nt) * 16;
      const int sec = job & 1;
      M = st.k_ins; Ncols = n;
      A = (job < 2) ? d.ZT[sec] : d.X[sec];
      B = d.N[par][sec];
      C = (job < 2) ? d.YT[sec] : d.Rt[sec];
      lda = d.ld; ldb = d.ld; ldc = d.ld;
      trans = (job < 2);
    } else if (kind == kSkGnn) {
      // Gnn[sec] = X YT^T + G0nn  (B = YT is FP64; K = 0 still writes C = D)
      const int nt = (st.k_ins + 15) >> 4;
      job = local / nt; c0 = (local - job * nt) * 16;
      const int sec = job;
      M = st.k_ins; Ncols = st.k_ins;
      A = d.X[sec]; B = d.YT[sec]; C = d.Gnn[sec]; D = d.G0nn[sec];
      lda = d.ld; ldb = d.ld; ldc = d.kmax; ldd = d.kmax;
      trans = 1;
    } else {
      // W[sec] = N gR, computed as (gRT N^T)^T: C[l][y]
      const int nt = (n + 15) >> 4;
      job = local / nt; c0 = (local - job * nt) * 16;
      const int sec = job;
      M = d.nc; Ncols = n;
      A = d.gR[sec]; B = d.N[par][sec]; C = d.W[sec];
      lda = d.n_cap; ldb = d.ld; ldc = d.nc;
      trans = 1; out_trans = 1;
    }
    auto afn = [&](int m, int k) -> double { return A[static_cast<size_t>(m) * lda + k]; };
    if (kind == kSkGnn)
      skinny_core<double>(afn, static_cast<const double *>(B), ldb, trans, M, K, Ncols, c0, red);
    else
      skinny_core<T>(afn, static_cast<const T *>(B), ldb, trans, M, K, Ncols, c0, red);
    for (int e = tid; e < ((M + 15) >> 4) * 256; e += kSkThreads) {
      int m, cc;
      red_index(e, c0, m, cc);
      if (m < M && cc < Ncols) {
        double v = red[e];
        if (D) v += D[static_cast<size_t>(m) * ldd + cc];
        if (out_trans) C[static_cast<size_t>(cc) * ldc + m] = v;
        else C[static_cast<size_t>(m) * ldc + cc] = v;
      }
    }
    __syncthreads();   // red is reused by the next item
  }
}

void launch_skinny(const Batch &b, hipStream_t s, int kind) {
  const dim3 grid(b.n_cu * 2);
  const size_t lds = sizeof(int) * (b.n_chains + 1);
  if (b.precision == kFP32)
    hipLaunchKernelGGL(k_skinny<float>, grid, dim3(kSkThreads), lds, s, b.d_desc, b.d_state, kind, b.n_chains);
  else
    hipLaunchKernelGGL(k_skinny<double>, grid, dim3(kSkThreads), lds, s, b.d_desc, b.d_state, kind, b.n_chains);
}

}  // namespace ctaux
