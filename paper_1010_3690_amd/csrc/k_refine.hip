// FP64 refinement of N against its definition (Eq. Nmatrix):
//   M = e^V - G0 (e^V - 1) built from the tables (n^2 interpolations),
//   R = I - M N,  N <- N + N R   (one Newton-Schulz step, two FP64 MFMA GEMMs),
//   drift = ||N R||_F / ||N + N R||_F.
// The step squares the relative error of N, so it restores the FP64 inverse of
// the current configuration from an updated N whose error is small (FP64
// rounding drift, or the ~1e-7 error of FP32 storage), and the drift is the
// relative error N had before the step, to first order.
//
// All chains of a batch are refined together: the host packs chains into
// groups whose scratch (M and R per sector, plus an FP64 copy of N for FP32
// storage, n x n each, packed) fits the refinement pool, and each group costs
// five launches whatever its size.  The products run persistent over the
// 64x64 tiles of every chain and sector of the group.
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kRefBlocks = 64;   // workgroups per chain for the elementwise kernels

// Per-chain scratch of a group: [sector][M, R, Nd] blocks of n*n doubles.
__device__ __forceinline__ double *ref_slot(double *pool, const RefineItem &it, int sec, int which, int nslots) {
  const size_t nn = static_cast<size_t>(it.n) * it.n;
  return pool + it.off + (static_cast<size_t>(sec) * nslots + which) * nn;
}

// M (and, for FP32 storage, an FP64 copy of N) of both sectors.
template <typename T>
__global__ __launch_bounds__(256) void k_ref_build(const ChainDesc *descs, const ChainState *states,
                                                   const RefineItem *items, double *pool) {
  const RefineItem it = items[blockIdx.y];
  const ChainDesc &d = descs[it.chain];
  const ChainState &st = states[it.chain];
  const int n = it.n, par = st.parity;
  const int nslots = (sizeof(T) == sizeof(double)) ? 2 : 3;
  const double *tau = d.tau[par];
  const int32_t *site = d.site[par], *s0 = d.s0[par];
  const int64_t per = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < 2 * per; e += gridDim.x * 256ll) {
    const int sec = e >= per ? 1 : 0;
    const int64_t r = e - sec * per;
    const int i = static_cast<int>(r / n), j = static_cast<int>(r - static_cast<int64_t>(i) * n);
    const double evj = d.evd[sec][s0[j] + 2];
    double v = -g0_interp(d, sec, site[i], site[j], tau[i] - tau[j]) * (evj - 1.0);
    if (i == j) v += d.evd[sec][s0[i] + 2];
    ref_slot(pool, it, sec, 0, nslots)[r] = v;
    if (sizeof(T) != sizeof(double)) {
      const T *N = static_cast<const T *>(d.N[par][sec]);
      ref_slot(pool, it, sec, 2, nslots)[r] = static_cast<double>(N[static_cast<size_t>(i) * d.ld + j]);
    }
  }
}

// C = alpha A B + diag I on 64x64 tiles, FP64 MFMA 16x16x4, K staged through LDS
// in chunks of kGK with the next chunk's loads in flight during the current
// chunk's MFMAs.  mode 0: R = I - M N;  mode 1: T = N R (into M's slot).
constexpr int kGK = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_ref_gemm(const ChainDesc *descs, const ChainState *states,
                                                  const RefineItem *items, int n_items, double *pool, int mode) {
  extern __shared__ int pre[];   // [n_items + 1]
  __shared__ double As[2][64][kGK + 1];
  __shared__ double Bs[2][kGK][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nslots = (sizeof(T) == sizeof(double)) ? 2 : 3;
  block_prefix<256>(n_items, pre, [&](int q) {
    const int nt = (items[q].n + 63) / 64;
    return 2 * nt * nt;
  });
  const int total = pre[n_items];
  const int wr = wave >> 1, wc = wave & 1, lr = lane & 15, lk = lane >> 4;
  const ItemSpan span = xcd_items(1, 0);   // neighbouring tiles on one XCD
  for (int k = span.first;; k += span.stride) {
    const int t = span.item(k);
    if (t >= total) break;
    int lo = 0, hi = n_items;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const RefineItem it = items[lo];
    const ChainDesc &d = descs[it.chain];
    const ChainState &st = states[it.chain];
    const int n = it.n, nt = (n + 63) / 64;
    int local = t - pre[lo];
    const int sec = local / (nt * nt);
    local -= sec * nt * nt;
    const int r0 = (local / nt) * 64, c0 = (local % nt) * 64;
    double *Ms = ref_slot(pool, it, sec, 0, nslots);
    double *Rs = ref_slot(pool, it, sec, 1, nslots);
    // N as an FP64 operand: the storage itself (FP64) or its copy (FP32)
    const double *Nd;
    int ldn;
    if (sizeof(T) == sizeof(double)) {
      Nd = static_cast<const double *>(d.N[st.parity][sec]);
      ldn = d.ld;
    } else {
      Nd = ref_slot(pool, it, sec, 2, nslots);
      ldn = n;
    }
    const auto A = gview(mode == 0 ? Ms : Nd);
    const int lda = mode == 0 ? n : ldn;
    const auto B = gview(mode == 0 ? Nd : Rs);
    const int ldb = mode == 0 ? ldn : n;
    const auto C = gview_w(mode == 0 ? Rs : Ms);
    const double alpha = mode == 0 ? -1.0 : 1.0, diag = mode == 0 ? 1.0 : 0.0;
    // staging: thread tid loads row tid/4 of the A chunk (kGV consecutive k) and
    // row tid/(64/kGV) of the B chunk (kGV consecutive columns)
    constexpr int kGV = kGK / 4;
    const int ar = tid >> 2, ak = (tid & 3) * kGV;
    const int bk = tid / (64 / kGV), bc = (tid % (64 / kGV)) * kGV;
    double ra[kGV], rb[kGV];
    auto load = [&](int k0) {
#pragma unroll
      for (int i = 0; i < kGV; ++i) {
        const int r = r0 + ar, k = k0 + ak + i;
        ra[i] = (r < n && k < n) ? A[static_cast<size_t>(r) * lda + k] : 0.0;
        const int kb = k0 + bk, cc = c0 + bc + i;
        rb[i] = (kb < n && cc < n) ? B[static_cast<size_t>(kb) * ldb + cc] : 0.0;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int i = 0; i < kGV; ++i) {
        As[buf][ar][ak + i] = ra[i];
        Bs[buf][bk][bc + i] = rb[i];
      }
    };
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    load(0);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < n; k0 += kGK) {
      const bool more = k0 + kGK < n;
      if (more) load(k0 + kGK);   // in flight during this chunk's MFMAs
#pragma unroll
      for (int kk = 0; kk < kGK; kk += 4) {
        double af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = As[buf][wr * 32 + i * 16 + lr][kk + lk];
#pragma unroll
        for (int j = 0; j < 2; ++j) bf[j] = Bs[buf][kk + lk][wc * 32 + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = r0 + wr * 32 + i * 16 + lk + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
          const int cc = c0 + wc * 32 + j * 16 + lr;
          if (r < n && cc < n) C[static_cast<size_t>(r) * n + cc] = alpha * acc[i][j][q] + (r == cc ? diag : 0.0);
        }
  }
}

// N <- N + T (T = N R in M's slot), and per-workgroup partial sums of T^2 and N'^2.
template <typename T>
__global__ __launch_bounds__(256) void k_ref_apply(const ChainDesc *descs, const ChainState *states,
                                                   const RefineItem *items, double *pool, double *red) {
  const RefineItem it = items[blockIdx.y];
  const ChainDesc &d = descs[it.chain];
  const ChainState &st = states[it.chain];
  const int n = it.n, nslots = (sizeof(T) == sizeof(double)) ? 2 : 3;
  __shared__ double sh[2][4];
  for (int sec = 0; sec < 2; ++sec) {
    T *N = static_cast<T *>(d.N[st.parity][sec]);
    const double *t = ref_slot(pool, it, sec, 0, nslots);
    const double *nd = (sizeof(T) == sizeof(double)) ? nullptr : ref_slot(pool, it, sec, 2, nslots);
    const int64_t total = static_cast<int64_t>(n) * n;
    double s_t = 0.0, s_n = 0.0;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
      const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
      const size_t o = static_cast<size_t>(i) * d.ld + j;
      const double tv = t[e];
      const double nv = (nd ? nd[e] : static_cast<double>(N[o])) + tv;
      N[o] = static_cast<T>(nv);
      s_t += tv * tv;
      s_n += nv * nv;
    }
    s_t = wave_sum(s_t);
    s_n = wave_sum(s_n);
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = s_t; sh[1][threadIdx.x >> 6] = s_n; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double *r = red + ((static_cast<size_t>(blockIdx.y) * 2 + sec) * gridDim.x + blockIdx.x) * 2;
      r[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
      r[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
    __syncthreads();
  }
}

// Drift of every chain of the group, one wave per chain: lane l sums partials
// l, l + 64, ... and the lanes are summed on the DPP network (a fixed order).
// pass 0 records the drift the chain accumulated since its last refinement
// (last_drift, max_drift, the drift_tol check); every pass leaves its drift in
// pass_drift for the host's decision on one more step.
__global__ __launch_bounds__(64) void k_ref_reduce(const ChainDesc *descs, ChainState *states,
                                                   const RefineItem *items, int n_items, const double *red, int nb,
                                                   int pass, int scratch) {
  const int q = blockIdx.x, lane = threadIdx.x;
  if (q >= n_items) return;
  const int c = items[q].chain;
  ChainState &st = states[c];
  double drift = 0.0;
  for (int sec = 0; sec < 2; ++sec) {
    double a = 0.0, b = 0.0;
    const double *r = red + (static_cast<size_t>(q) * 2 + sec) * nb * 2;   // nb partials per sector
    for (int i = lane; i < nb; i += 64) {
      a += r[2 * i];
      b += r[2 * i + 1];
    }
    a = wave_sum_dpp(a);
    b = wave_sum_dpp(b);
    const double dr = (b > 0.0) ? sqrt(a / b) : 0.0;
    if (!isfinite(dr)) drift = INFINITY;
    else if (dr > drift) drift = dr;
  }
  if (lane != 0) return;
  st.pass_drift = drift;
  if (scratch) st.scratch_recomputes += 1;
  // A Newton step that left a non-finite N is repaired by a from-scratch
  // recompute (the host reads pass_drift); a from-scratch recompute that fails
  // (singular or non-finite M) stops the chain.  A failing chain is also
  // deactivated: the next block may already have been started (its start is
  // fused into the previous block's end), and its kernels then skip the chain.
  if (scratch && !isfinite(drift) && st.status == 0) {
    st.status = -4;
    st.err_index = -6;
    st.active = 0;
  }
  if (pass > 0) return;
  st.last_drift = drift;
  if (!(drift <= st.max_drift)) st.max_drift = drift;
  if (st.status == 0 && descs[c].drift_tol > 0.0 && drift > descs[c].drift_tol) {
    st.status = -4;   // N no longer represents the inverse of its definition
    st.err_index = -5;
    st.active = 0;
  }
}

int refine_slots(int precision) { return precision == kFP64 ? 2 : 3; }

size_t refine_need_doubles(int n, int precision) {
  return 2 * (static_cast<size_t>(refine_slots(precision)) * n * n + inv_scratch_doubles(n));
}

// Workgroups per chain of the elementwise kernels (the table build of M, the
// update N + T with its partial sums, the from-scratch store): kRefBlocks for
// batches of 8 chains or more; fewer chains take more, so that their n^2
// entries spread over the GPU.
static int elem_blocks(int n_chains) { return n_chains >= 8 ? kRefBlocks : (n_chains >= 2 ? 256 : 512); }

size_t refine_red_doubles(int n_chains) { return static_cast<size_t>(n_chains) * 2 * elem_blocks(n_chains) * 2; }

template <typename T>
static void launch_group_t(const Batch &b, hipStream_t s, const RefineItem *items, int n_items, int pass) {
  const int nb = elem_blocks(b.n_chains);
  hipLaunchKernelGGL(k_ref_build<T>, dim3(nb, n_items), dim3(256), 0, s, b.d_desc, b.d_state, items, b.r_pool);
  const size_t lds = sizeof(int) * (n_items + 1);
  for (int mode = 0; mode < 2; ++mode)
    hipLaunchKernelGGL(k_ref_gemm<T>, dim3(b.n_cu * 2), dim3(256), lds, s, b.d_desc, b.d_state, items, n_items,
                       b.r_pool, mode);
  hipLaunchKernelGGL(k_ref_apply<T>, dim3(nb, n_items), dim3(256), 0, s, b.d_desc, b.d_state, items, b.r_pool,
                     b.r_red);
  hipLaunchKernelGGL(k_ref_reduce, dim3(n_items), dim3(64), 0, s, b.d_desc, b.d_state, items, n_items, b.r_red, nb,
                     pass, 0);
}

// After the elimination: N <- M^{-1} in canonical order, N[i][j] = W[perm[i]][pos(j)]
// (k_invert.hip), with per-workgroup partial sums of |N_before - N_after|^2 and
// N_after^2 for the drift.  A singular M leaves NaN in the sums.
template <typename T>
__global__ __launch_bounds__(256) void k_ref_scratch_store(const ChainDesc *descs, const ChainState *states,
                                                           const RefineItem *items, const InvItem *inv, double *red) {
  const RefineItem it = items[blockIdx.y];
  const ChainDesc &d = descs[it.chain];
  const ChainState &st = states[it.chain];
  const int n = it.n;
  __shared__ double sh[2][4];
  for (int sec = 0; sec < 2; ++sec) {
    const InvItem &iv = inv[2 * blockIdx.y + sec];
    T *N = static_cast<T *>(d.N[st.parity][sec]);
    const bool bad = iv.flag[0] != 0;
    const int64_t total = static_cast<int64_t>(n) * n;
    double s_t = 0.0, s_n = 0.0;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += gridDim.x * 256ll) {
      const int i = static_cast<int>(e / n), j = static_cast<int>(e - static_cast<int64_t>(i) * n);
      const int bj = iv.blk[j];   // every row is a pivot once the elimination is complete
      const double nv = bj >= 0 ? iv.W[static_cast<size_t>(iv.perm[i]) * iv.ldw + bj * kInvNB + iv.slot[j]] : NAN;
      const size_t o = static_cast<size_t>(i) * d.ld + j;
      const double dv = static_cast<double>(N[o]) - nv;
      N[o] = static_cast<T>(nv);
      s_t += dv * dv;
      s_n += nv * nv;
    }
    if (bad) s_t = NAN;
    s_t = wave_sum(s_t);
    s_n = wave_sum(s_n);
    if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = s_t; sh[1][threadIdx.x >> 6] = s_n; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double *r = red + ((static_cast<size_t>(blockIdx.y) * 2 + sec) * gridDim.x + blockIdx.x) * 2;
      r[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
      r[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
    __syncthreads();
  }
}

template <typename T>
static void launch_scratch_t(const Batch &b, hipStream_t s, const RefineItem *items, const InvItem *inv, int n_items,
                             int n_max, int pass) {
  const int nb = elem_blocks(b.n_chains);
  hipLaunchKernelGGL(k_ref_build<T>, dim3(nb, n_items), dim3(256), 0, s, b.d_desc, b.d_state, items, b.r_pool);
  launch_invert(s, inv, 2 * n_items, n_max, b.n_cu);
  hipLaunchKernelGGL(k_ref_scratch_store<T>, dim3(nb, n_items), dim3(256), 0, s, b.d_desc, b.d_state, items, inv,
                     b.r_red);
  hipLaunchKernelGGL(k_ref_reduce, dim3(n_items), dim3(64), 0, s, b.d_desc, b.d_state, items, n_items, b.r_red, nb,
                     pass, 1);
}

void launch_scratch_group(const Batch &b, hipStream_t s, const RefineItem *items, const InvItem *inv, int n_items,
                          int n_max, int pass) {
  if (n_items <= 0) return;
  if (b.precision == kFP64) launch_scratch_t<double>(b, s, items, inv, n_items, n_max, pass);
  else launch_scratch_t<float>(b, s, items, inv, n_items, n_max, pass);
}

int setup_refine(const Batch &b) {
  const int lds = static_cast<int>(sizeof(int) * (b.n_chains + 1));
  if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_ref_gemm<double>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
      hipFuncSetAttribute(reinterpret_cast<const void *>(k_ref_gemm<float>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return -1;
  return setup_invert(2 * b.n_chains);
}

// One group of chains (items in device memory, scratch offsets within the pool).
void launch_refine_group(const Batch &b, hipStream_t s, const RefineItem *items, int n_items, int pass) {
  if (n_items <= 0) return;
  if (b.precision == kFP64) launch_group_t<double>(b, s, items, n_items, pass);
  else launch_group_t<float>(b, s, items, n_items, pass);
}

}  // namespace ctaux
