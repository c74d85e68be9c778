// From-scratch FP64 inverse of N^{-1} = M = e^V - G0 (e^V - 1)  (Eq. Nmatrix).
//
// Blocked Gauss-Jordan elimination in place ("sweep" form), kInvNB columns per
// step, with the pivot rows of each step chosen by tournament pivoting
// (Grigori, Demmel and Xiang, "CALU: a communication optimal LU factorization
// algorithm", SIAM J. Matrix Anal. Appl. 32 (2011)): every workgroup selects
// kInvNB candidate rows of a 256-row chunk by partial pivoting on the step's
// panel columns, and the candidates are merged eight lists at a time by the
// same selection until one list remains.  With the step's pivot rows p and
// columns J, A11 = W[p, J] is inverted (partial pivoting inside the block) and
//   W[p, c]  <- A11^{-1} W[p, c]           (c outside J),   W[p, J] <- A11^{-1},
//   W[i, c]  <- W[i, c] - W[i, J] A11^{-1} W[p, c]   (other rows i),
//   W[i, J]  <- -W[i, J] A11^{-1},
// i.e. W <- base - Lp T with Lp = W[:, J] and T = A11^{-1} W[p, :] (T[:, J] =
// A11^{-1}), a rank-kInvNB update on FP64 MFMA.  Rows are never exchanged:
// row perm[q] of W ends as row q of (P M)^{-1}, where P moves the pivot row of
// position q to row q, so that M^{-1}[i][j] = W[perm[i]][pos(j)], pos(j) = the
// position at which row j became a pivot.  Cost 2 n^3 flops.
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));

size_t inv_scratch_doubles(int n) {
  const size_t nn = static_cast<size_t>(n);
  const size_t nch = (nn + 255) / 256;
  const size_t ints = kInvNB * nch + 3 * nn + 8;
  auto r8 = [](size_t x) { return (x + 7) / 8 * 8; };
  return r8(kInvNB * nn) + r8(kInvNB * nn) + r8(kInvNB * kInvNB) + r8((ints + 1) / 2);
}

void inv_item_carve(InvItem &it, double *W, int n, int ldw, double *scratch) {
  auto r8 = [](size_t x) { return (x + 7) / 8 * 8; };
  const size_t nn = static_cast<size_t>(n);
  it.W = W;
  it.n = n;
  it.ldw = ldw;
  it.T = scratch;
  it.Lp = it.T + r8(kInvNB * nn);
  it.Ainv = it.Lp + r8(kInvNB * nn);
  int32_t *ip = reinterpret_cast<int32_t *>(it.Ainv + r8(kInvNB * kInvNB));
  it.cand = ip;
  ip += kInvNB * ((nn + 255) / 256);
  it.blk = ip;
  ip += nn;
  it.slot = ip;
  ip += nn;
  it.perm = ip;
  ip += nn;
  it.flag = ip;
}

// Rows start unpivoted; the singularity flag starts clear.
__global__ __launch_bounds__(256) void k_inv_init(const InvItem *items) {
  const InvItem it = items[blockIdx.y];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) it.blk[i] = -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) it.flag[0] = 0;
}

// Selection by partial pivoting among the rows held by the 256 threads of the
// workgroup (row < 0: none) on the panel columns [j0, j0 + nbe) of W: for each
// column in turn the remaining row of largest magnitude (ties: lowest thread)
// is taken, and the other remaining rows are eliminated against it.  The
// selected rows go to out[0 .. kInvNB) in order (-1 when no row is left).
__device__ void select_pivots(const InvItem &it, int j0, int nbe, int row, int32_t *out) {
  __shared__ double sh_v[4];
  __shared__ int sh_i[4];
  __shared__ double prow[kInvNB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const auto W = gview(it.W);
  double a[kInvNB];
#pragma unroll
  for (int k = 0; k < kInvNB; ++k)
    a[k] = (row >= 0 && k < nbe) ? W[static_cast<size_t>(row) * it.ldw + j0 + k] : 0.0;
  bool live = row >= 0;
#pragma unroll
  for (int j = 0; j < kInvNB; ++j) {
    if (j >= nbe) {   // uniform
      if (tid == 0) out[j] = -1;
      continue;
    }
    double v = live ? fabs(a[j]) : -1.0;
    if (v != v) v = INFINITY;   // a NaN is taken first (and flagged by the pivot block)
    int ix = live ? tid : 0x7fffffff;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(ix, off, 64);
      if (ov > v || (ov == v && oi < ix)) { v = ov; ix = oi; }
    }
    if (lane == 0) { sh_v[wave] = v; sh_i[wave] = ix; }
    __syncthreads();
    double bv = sh_v[0];
    int bi = sh_i[0];
#pragma unroll
    for (int w = 1; w < 4; ++w)
      if (sh_v[w] > bv || (sh_v[w] == bv && sh_i[w] < bi)) { bv = sh_v[w]; bi = sh_i[w]; }
    if (bv < 0.0) {   // no row left (uniform)
      if (tid == 0) out[j] = -1;
      __syncthreads();
      continue;
    }
    if (tid == bi) {
#pragma unroll
      for (int k = 0; k < kInvNB; ++k) prow[k] = a[k];
      out[j] = row;
      live = false;
    }
    __syncthreads();
    const double pj = prow[j];
    if (live && pj != 0.0) {
      const double f = a[j] / pj;
#pragma unroll
      for (int k = j + 1; k < kInvNB; ++k) a[k] -= f * prow[k];
    }
  }
  __syncthreads();
}

// First tournament level: chunk blockIdx.x of 256 rows.
__global__ __launch_bounds__(256) void k_inv_tourn1(const InvItem *items, int j0) {
  const InvItem it = items[blockIdx.y];
  const int n = it.n;
  if (j0 >= n || blockIdx.x * 256 >= n) return;   // uniform over the workgroup
  const int nbe = min(kInvNB, n - j0);
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int row = (r < n && it.blk[r] < 0) ? r : -1;
  select_pivots(it, j0, nbe, row, it.cand + blockIdx.x * kInvNB);
}

// Further levels: lists of kInvNB candidates merged eight at a time (one
// workgroup per item) until list 0 holds the step's pivot rows.
__global__ __launch_bounds__(256) void k_inv_tourn2(const InvItem *items, int j0) {
  const InvItem it = items[blockIdx.x];
  const int n = it.n;
  if (j0 >= n) return;
  const int nbe = min(kInvNB, n - j0);
  int lists = (n + 255) / 256;
  while (lists > 1) {
    const int groups = (lists + 7) / 8;
    for (int g = 0; g < groups; ++g) {
      const int l = 8 * g + threadIdx.x / kInvNB, q = threadIdx.x % kInvNB;
      const int row = (l < lists) ? it.cand[l * kInvNB + q] : -1;
      __syncthreads();   // list g is read above before the selection overwrites it
      select_pivots(it, j0, nbe, row, it.cand + g * kInvNB);
    }
    lists = groups;
  }
}

// The step's pivot block A11 = W[p, J]: in-place Gauss-Jordan with partial
// pivoting on one wave (lane r owns row r), A11^{-1} to Ainv (kInvNB square,
// zero beyond nbe), and the pivot bookkeeping.
__global__ __launch_bounds__(64) void k_inv_pivot(const InvItem *items, int j0) {
  __shared__ double A[kInvNB][kInvNB + 1];
  __shared__ int perm_l[kInvNB];
  const InvItem it = items[blockIdx.x];
  const int n = it.n;
  if (j0 >= n) return;
  const int m = min(kInvNB, n - j0);
  const int lane = threadIdx.x;
  const auto W = gview(it.W);
  // the tournament leaves m rows whenever m rows are unpivoted; a missing one
  // (cannot happen) is flagged and replaced by row 0 to keep every access in range
  int myrow = lane < m ? it.cand[lane] : 0;
  bool bad = false;
  if (myrow < 0 || myrow >= n) {
    bad = true;
    myrow = 0;
  }
  for (int r = 0; r < m; ++r) {
    const int pr = __shfl(myrow, r, 64);
    if (lane < m) A[r][lane] = W[static_cast<size_t>(pr) * it.ldw + j0 + lane];
  }
  __syncthreads();
  const bool mine = lane < m;
  bool used = false;
  int mypos = 0;
  for (int col = 0; col < m; ++col) {
    double f = mine ? A[lane][col] : 0.0;
    double v = (mine && !used) ? fabs(f) : -1.0;
    if (v != v) v = INFINITY;
    int ix = (mine && !used) ? lane : 0x7fffffff;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(ix, off, 64);
      if (ov > v || (ov == v && oi < ix)) { v = ov; ix = oi; }
    }
    const int p = ix;   // uniform; a row is always left while col < m
    const double pv = __shfl(f, p, 64);
    if (!(pv != 0.0) || !isfinite(pv)) bad = true;
    const double ip = 1.0 / pv;
    const bool piv = lane == p;
    if (piv) { used = true; mypos = col; }
    if (lane == 0) perm_l[col] = p;
    const double scale = piv ? ip : 1.0;
    const double fi = piv ? 0.0 : f * ip;
    const double xc = piv ? ip : -fi;
    double rv[kInvNB], pr[kInvNB];
#pragma unroll
    for (int j = 0; j < kInvNB; ++j) {
      rv[j] = (mine && j < m) ? A[lane][j] : 0.0;
      pr[j] = (j < m) ? A[p][j] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    if (mine) {
#pragma unroll
      for (int j = 0; j < kInvNB; ++j)
        if (j < m) A[lane][j] = (j == col) ? xc : rv[j] * scale - fi * pr[j];
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // row mypos(r) of the inverse is row r of A with column c moved to column perm_l[c]
  const auto Ai = gview_w(it.Ainv);
  for (int e = lane; e < kInvNB * kInvNB; e += 64) Ai[e] = 0.0;
  __syncthreads();
  if (mine) {
    for (int c = 0; c < m; ++c) {
      const double x = A[lane][c];
      if (!isfinite(x)) bad = true;
      Ai[mypos * kInvNB + perm_l[c]] = x;
    }
    const int J = j0 / kInvNB;
    it.blk[myrow] = J;
    it.slot[myrow] = lane;
    it.perm[j0 + lane] = myrow;
  }
  if (__ballot(bad) != 0ull && lane == 0) it.flag[0] = 1;
}

// T = A11^{-1} W[p, :] (T[:, J] = A11^{-1}; rows beyond nbe zero) and
// Lp = W[:, J] (columns beyond nbe zero); thread = one column of T and one row of Lp.
__global__ __launch_bounds__(256) void k_inv_rows(const InvItem *items, int j0) {
  __shared__ double Ai[kInvNB][kInvNB];
  __shared__ int pv[kInvNB];
  const InvItem it = items[blockIdx.y];
  const int n = it.n;
  if (j0 >= n || blockIdx.x * 256 >= n) return;
  const int nbe = min(kInvNB, n - j0);
  const int tid = threadIdx.x;
  for (int e = tid; e < kInvNB * kInvNB; e += 256) Ai[e / kInvNB][e % kInvNB] = it.Ainv[e];
  if (tid < kInvNB) pv[tid] = tid < nbe ? it.perm[j0 + tid] : 0;
  __syncthreads();
  const int c = blockIdx.x * 256 + tid;
  if (c >= n) return;
  const auto W = gview(it.W);
  const auto T = gview_w(it.T);
  const auto Lp = gview_w(it.Lp);
  double w[kInvNB];
#pragma unroll
  for (int k = 0; k < kInvNB; ++k) w[k] = k < nbe ? W[static_cast<size_t>(pv[k]) * it.ldw + c] : 0.0;
  const bool inJ = c >= j0 && c < j0 + nbe;
#pragma unroll 4
  for (int q = 0; q < kInvNB; ++q) {
    double s = 0.0;
    if (inJ) {
      s = Ai[q][c - j0];
    } else {
#pragma unroll
      for (int k = 0; k < kInvNB; ++k) s = fma(Ai[q][k], w[k], s);
    }
    T[static_cast<size_t>(q) * n + c] = s;   // zero rows beyond nbe: Ai is zero there
  }
#pragma unroll
  for (int q = 0; q < kInvNB; ++q)
    Lp[static_cast<size_t>(c) * kInvNB + q] = q < nbe ? W[static_cast<size_t>(c) * it.ldw + j0 + q] : 0.0;
}

// W <- (row a pivot of this step) ? T[slot] : base - Lp T, base = W outside J and
// 0 on J; 64x64 tiles of every item from one persistent grid, FP64 MFMA 16x16x4.
__global__ __launch_bounds__(256) void k_inv_update(const InvItem *items, int n_items, int j0) {
  extern __shared__ int pre[];   // [n_items + 1]
  __shared__ int scan[256];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) { carry = 0; pre[0] = 0; }
  __syncthreads();
  for (int base = 0; base < n_items; base += 256) {
    const int q = base + tid;
    int v = 0;
    if (q < n_items && items[q].n > j0) {
      const int nt = (items[q].n + 63) / 64;
      v = nt * nt;
    }
    scan[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int x = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += x;
      __syncthreads();
    }
    if (q < n_items) pre[q + 1] = carry + scan[tid];
    __syncthreads();
    if (tid == 0) carry += scan[255];
    __syncthreads();
  }
  const int total = pre[n_items];
  const int J = j0 / kInvNB;
  const int wr = wave >> 1, wc = wave & 1, lr = lane & 15, lk = lane >> 4;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n_items;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const InvItem &it = items[lo];
    const int n = it.n, nt = (n + 63) / 64, nbe = min(kInvNB, n - j0);
    const int local = t - pre[lo];
    const int r0 = (local / nt) * 64 + wr * 32, c0 = (local % nt) * 64 + wc * 32;
    const auto W = gview_w(it.W);
    const auto T = gview(it.T);
    const auto Lp = gview(it.Lp);
    const int ldw = it.ldw;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < kInvNB; k0 += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = r0 + i * 16 + lr;
        af[i] = r < n ? Lp[static_cast<size_t>(r) * kInvNB + k0 + lk] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cc = c0 + j * 16 + lr;
        bf[j] = cc < n ? T[static_cast<size_t>(k0 + lk) * n + cc] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + i * 16 + lk + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
        if (r >= n) continue;
        const bool pivrow = it.blk[r] == J;
        const int sl = pivrow ? it.slot[r] : 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int cc = c0 + j * 16 + lr;
          if (cc >= n) continue;
          const size_t o = static_cast<size_t>(r) * ldw + cc;
          double v;
          if (pivrow) {
            v = T[static_cast<size_t>(sl) * n + cc];
          } else {
            const bool inJ = cc >= j0 && cc < j0 + nbe;
            v = (inJ ? 0.0 : W[o]) - acc[i][j][q];
          }
          W[o] = v;
        }
      }
  }
}

// M^{-1}[i][j] = W[perm[i]][pos(j)] into a row-major FP64 destination.
__global__ __launch_bounds__(256) void k_inv_gather(const InvItem *items, double *out, int ldo) {
  const InvItem it = items[blockIdx.y];
  const int n = it.n;
  const int64_t total = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
    const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
    const int bj = it.blk[j];
    double v = NAN;
    if (!it.flag[0] && bj >= 0) v = it.W[static_cast<size_t>(it.perm[i]) * it.ldw + bj * kInvNB + it.slot[j]];
    out[static_cast<size_t>(i) * ldo + j] = v;
  }
}

int inv_update_lds(int n_items) { return static_cast<int>(sizeof(int) * (n_items + 1)); }

int setup_invert(int max_items) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_inv_update), hipFuncAttributeMaxDynamicSharedMemorySize,
                             inv_update_lds(max_items)) == hipSuccess ? 0 : -1;
}

// The elimination of every item (device array of n_items), n_max = largest n.
void launch_invert(hipStream_t s, const InvItem *items, int n_items, int n_max, int n_cu) {
  if (n_items <= 0 || n_max <= 0) return;
  const int nch = (n_max + 255) / 256;
  hipLaunchKernelGGL(k_inv_init, dim3(nch, n_items), dim3(256), 0, s, items);
  for (int j0 = 0; j0 < n_max; j0 += kInvNB) {
    hipLaunchKernelGGL(k_inv_tourn1, dim3(nch, n_items), dim3(256), 0, s, items, j0);
    if (nch > 1) hipLaunchKernelGGL(k_inv_tourn2, dim3(n_items), dim3(256), 0, s, items, j0);
    hipLaunchKernelGGL(k_inv_pivot, dim3(n_items), dim3(64), 0, s, items, j0);
    hipLaunchKernelGGL(k_inv_rows, dim3(nch, n_items), dim3(256), 0, s, items, j0);
    hipLaunchKernelGGL(k_inv_update, dim3(n_cu * 4), dim3(256), inv_update_lds(n_items), s, items, n_items, j0);
  }
}

void launch_inv_gather(hipStream_t s, const InvItem *items, double *out, int ldo, int n) {
  const int g = (static_cast<int64_t>(n) * n + 255) / 256 < 1024 ? static_cast<int>((static_cast<int64_t>(n) * n + 255) / 256) : 1024;
  hipLaunchKernelGGL(k_inv_gather, dim3(g > 0 ? g : 1, 1), dim3(256), 0, s, items, out, ldo);
}

}  // namespace ctaux
