// Device helpers: counter-based random numbers, G0 interpolation, G entries.
#pragma once

#include "ctaux_internal.h"

namespace ctaux {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with Weyl-sequence key bumps.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * c[0], hi0 = __umulhi(m0, c[0]);
    uint32_t lo1 = m1 * c[2], hi1 = __umulhi(m1, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}

// 53-bit uniform in [0, 1) from two 32-bit words (high word first).
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
  uint64_t x = (static_cast<uint64_t>(hi) << 32) | lo;
  return static_cast<double>(x >> 11) * (1.0 / 9007199254740992.0);
}

// The five uniforms of proposal `index` of a chain: counter (index lo, index
// hi, chain, tag), key = seed; tag 0 -> (type, accept), 1 -> (tau, pick),
// 2 -> (spin, the second spin of a pair).
__device__ __forceinline__ void proposal_uniforms(const ChainDesc &d, uint64_t index, double u[5]) {
  uint32_t c[4];
  c[0] = static_cast<uint32_t>(index); c[1] = static_cast<uint32_t>(index >> 32);
  c[2] = d.chain_id; c[3] = 0;
  philox4x32_10(c, d.seed_lo, d.seed_hi);
  u[0] = u53(c[0], c[1]); u[1] = u53(c[2], c[3]);
  c[0] = static_cast<uint32_t>(index); c[1] = static_cast<uint32_t>(index >> 32);
  c[2] = d.chain_id; c[3] = 1;
  philox4x32_10(c, d.seed_lo, d.seed_hi);
  u[2] = u53(c[0], c[1]); u[3] = u53(c[2], c[3]);
  c[0] = static_cast<uint32_t>(index); c[1] = static_cast<uint32_t>(index >> 32);
  c[2] = d.chain_id; c[3] = 2;
  philox4x32_10(c, d.seed_lo, d.seed_hi);
  u[4] = u53(c[0], c[1]);
}

// The extra uniforms of a pair proposal: u_spin2 (the second word pair of tag
// 2), u_tau2 and u_pick2 (tag 3).
__device__ __forceinline__ void pair_uniforms(const ChainDesc &d, uint64_t index, double v[3]) {
  uint32_t c[4];
  c[0] = static_cast<uint32_t>(index); c[1] = static_cast<uint32_t>(index >> 32);
  c[2] = d.chain_id; c[3] = 2;
  philox4x32_10(c, d.seed_lo, d.seed_hi);
  v[0] = u53(c[2], c[3]);
  c[0] = static_cast<uint32_t>(index); c[1] = static_cast<uint32_t>(index >> 32);
  c[2] = d.chain_id; c[3] = 3;
  philox4x32_10(c, d.seed_lo, d.seed_hi);
  v[1] = u53(c[0], c[1]);
  v[2] = u53(c[2], c[3]);
}

// Pointers read from the chain descriptor are generic, and generic (flat)
// accesses are counted by both the vector-memory and the LDS wait counters, so
// any wait for an LDS result would also wait for every global load or store in
// flight.  Accesses through these global-address-space views are counted by
// the vector-memory counter only.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gview(const T *p) {
  return (const __attribute__((address_space(1))) T *)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gview_w(T *p) {
  return (__attribute__((address_space(1))) T *)(p);
}

// The candidate operands X and ZT (k_max candidates x ld vertices per sector)
// are stored in the order the skinny products' lanes read them: 16 x 16 blocks
// of (candidate, vertex), block (vertex group g, candidate tile t) at
// 256 (g RT + t), RT = ceil(k_max / 16), and inside a block entry (j, i) at
// 4 (16 ((i % 16) / 4) + j % 16) + i % 4.  A lane then reads four consecutive
// vertices of one candidate as 32 contiguous bytes, and the 64 lanes of a
// load (16 candidates x 16 vertices) one contiguous 2 KB block, where the
// row-major layout touched 16 cache lines per load for 32 bytes in each.
__device__ __forceinline__ size_t cand_offset(int j, int i, int rt) {
  return ((static_cast<size_t>(i >> 4) * rt + (j >> 4)) * 64 + (((i & 15) >> 2) << 4) + (j & 15)) * 4 + (i & 3);
}

// The rank-k operand Ac (n' rows x lda columns, lda a multiple of 8) in the
// order the update's MFMA lanes read it: blocks of 16 rows x 4 columns (one
// k-step), block (row tile t, step s) at 64 (t S + s), S = lda / 4, and inside
// a block entry (i, a) at 16 (a % 4) + i % 16.  A load of 64 lanes (16 rows,
// 4 consecutive k) then reads 512 contiguous bytes.
__device__ __forceinline__ size_t ac_offset(int i, int a, int steps) {
  return ((static_cast<size_t>(i >> 4) * steps + (a >> 2)) << 6) + ((a & 3) << 4) + (i & 15);
}

// Exclusive prefix sums pre[0..n] (pre[0] = 0) of count(i), i < n, as every
// workgroup (NT threads) of a persistent kernel builds them in LDS to find the
// owner of a work item.  Up to 64 entries one wave scans them with lane
// shuffles and one barrier publishes them; more, the workgroup scans NT at a
// time (Hillis-Steele).  pre is complete on return.
template <int NT, typename F>
__device__ __forceinline__ void block_prefix(int n, int *pre, F count) {
  __shared__ int scan[NT];
  __shared__ int carry;
  const int tid = threadIdx.x;
  if (n <= 64) {
    if (tid < 64) {
      int v = tid < n ? count(tid) : 0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(v, off, 64);
        if (tid >= off) v += x;
      }
      if (tid < n) pre[tid + 1] = v;
      if (tid == 0) pre[0] = 0;
    }
    __syncthreads();
    return;
  }
  if (tid == 0) { carry = 0; pre[0] = 0; }
  __syncthreads();
  for (int base = 0; base < n; base += NT) {
    const int i = base + tid;
    scan[tid] = i < n ? count(i) : 0;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const int x = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += x;
      __syncthreads();
    }
    if (i < n) pre[i + 1] = carry + scan[tid];
    __syncthreads();
    if (tid == 0) carry += scan[NT - 1];
    __syncthreads();
  }
}

// Chain and sub-block of a per-chain streaming kernel.  With xcd_g = G > 0 the
// grid is one-dimensional, 8 G ceil(C / 8) workgroups, and workgroup b serves
// chain (b % 8) + 8 (b / 8G) as sub-block (b / 8) % G: workgroups are handed to
// the eight XCDs round-robin, so all G workgroups of a chain run on one XCD and
// the chain's tables and operands stay in that XCD's L2.  With xcd_g = 0 the
// grid is (G, C).  The chain index may exceed the batch (the caller checks).
struct ChainBlock {
  int c, sub, g;
};
__device__ __forceinline__ ChainBlock chain_block(int xcd_g) {
  if (xcd_g == 0) return ChainBlock{static_cast<int>(blockIdx.y), static_cast<int>(blockIdx.x),
                                    static_cast<int>(gridDim.x)};
  const int b = blockIdx.x, slot = b >> 3;
  return ChainBlock{(b & 7) + 8 * (slot / xcd_g), slot % xcd_g, xcd_g};
}

// A worker's share of the items of a persistent grid (workers: the waves of a
// workgroup in wave mode, else the workgroup itself).  Workgroups are handed to
// the eight XCDs round-robin; with a grid of 8 G workgroups the items are dealt
// to the XCDs in chunks of kItemChunk consecutive items (chunk c to XCD c % 8),
// so that neighbouring items, which share a chain's operands and tables, meet
// in one L2 while chains of uneven cost still spread over all XCDs.  The
// worker's k-th item is item(k) for k = first, first + stride, ...; items grow
// with k, so a loop stops at the first item(k) >= total.  Another grid size,
// or chunked = false, takes items b * workers + w + k * G * workers.
constexpr int kItemChunk = 32;
struct ItemSpan {
  int first, stride, x;   // x < 0: no XCD mapping
  __device__ int item(int k) const {
    if (x < 0) return k;
    return ((k / kItemChunk) * 8 + x) * kItemChunk + (k % kItemChunk);
  }
};
__device__ __forceinline__ ItemSpan xcd_items(int workers, int w, bool chunked = true) {
  const int G = gridDim.x, b = blockIdx.x;
  if ((G & 7) || !chunked) return ItemSpan{b * workers + w, G * workers, -1};
  return ItemSpan{(b >> 3) * workers + w, (G >> 3) * workers, b & 7};
}

// Bare propagator G0_{xy}(dtau): linear interpolation on the uniform grid,
// dtau in (-beta, beta); dtau < 0 uses G0(dtau) = -G0(dtau + beta); dtau = 0
// reads the 0+ entry.
// The same on one table (n_tau points, spacing 1 / inv_h, period beta).
__device__ __forceinline__ double interp_table(const __attribute__((address_space(1))) double *tab, double beta,
                                               double inv_h, int n_tau, double dtau) {
  double sgn = 1.0;
  if (dtau < 0.0) { dtau += beta; sgn = -1.0; }
  double xx = dtau * inv_h;
  int m = static_cast<int>(floor(xx));
  m = m < 0 ? 0 : (m > n_tau - 2 ? n_tau - 2 : m);
  double w = xx - static_cast<double>(m);
  return sgn * ((1.0 - w) * tab[m] + w * tab[m + 1]);
}
__device__ __forceinline__ double g0_interp(const ChainDesc &d, int sec, int x, int y, double dtau) {
  const auto tab = gview(d.g0[sec] + static_cast<int64_t>(gview(d.site_disp)[x * d.nc + y]) * d.n_tau);
  return interp_table(tab, d.beta, d.inv_h, d.n_tau, dtau);
}


template <typename T>
__device__ __forceinline__ double ld_as_double(const T *p) { return static_cast<double>(*p); }

// Entry G_ij of the block-start Green's function matrix G = N_a G0 of the
// augmented configuration (old vertices 0..n-1, candidates n..n+k_ins-1).
//  old column j (V_j != 0):  G_ij = (N_a,ij e^{V_j} - delta_ij) / (e^{V_j} - 1)   (Eq. NfromG)
//     with N_a,ij = N_ij (old row) or Rt_{i-n, j} (candidate row);
//  candidate column j:       G_ij = (N Z)_{i, j-n} (old row) or (X Y + G0nn)_{i-n, j-n}.
template <typename T>
__device__ __forceinline__ double g_entry(const ChainDesc &d, const T *N, const int32_t *s0, int n,
                                          int sec, int i, int j) {
  if (j < n) {
    const double e = gview(d.evd[sec])[gview(s0)[j] + 2];
    const double nij = (i < n) ? static_cast<double>(gview(N)[static_cast<size_t>(i) * d.ld + j])
                               : gview(d.Rt[sec])[static_cast<size_t>(i - n) * d.ld + j];
    return (nij * e - (i == j ? 1.0 : 0.0)) / (e - 1.0);
  }
  const int jj = j - n;
  return (i < n) ? gview(d.YT[sec])[static_cast<size_t>(jj) * d.ld + i]
                 : gview(d.Gnn[sec])[static_cast<size_t>(i - n) * d.kmax + jj];
}

// Entry of the augmented block-start N_a = [[N, 0], [Rt, 1]].
template <typename T>
__device__ __forceinline__ double na_entry(const ChainDesc &d, const T *N, int n, int sec, int i, int j) {
  if (i < n) return (j < n) ? static_cast<double>(N[static_cast<size_t>(i) * d.ld + j]) : 0.0;
  if (j < n) return d.Rt[sec][static_cast<size_t>(i - n) * d.ld + j];
  return (i == j) ? 1.0 : 0.0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}


// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not
// wait for this wave's global stores to complete, so stores whose results are
// read only after a later full barrier stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave reductions on the DPP network (VALU lane moves, no LDS round trip).
// Prefix steps row_shr:1,2,4,8 inside each row of 16 lanes, then row_bcast:15
// and row_bcast:31 across rows; lane 63 ends with the reduction over all 64
// lanes (lanes shifted in from outside a row contribute the identity 0).
// The result is read from lane 63, so it is uniform across the wave.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
  return static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, dpp_u32<0x111, 0xf>(v));   // row_shr:1
  v = max(v, dpp_u32<0x112, 0xf>(v));   // row_shr:2
  v = max(v, dpp_u32<0x114, 0xf>(v));   // row_shr:4
  v = max(v, dpp_u32<0x118, 0xf>(v));   // row_shr:8
  v = max(v, dpp_u32<0x142, 0xa>(v));   // row_bcast:15 into rows 1 and 3
  v = max(v, dpp_u32<0x143, 0xc>(v));   // row_bcast:31 into rows 2 and 3
  return static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

// Sum over the wave in a fixed order (the same for every call).
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0x111, 0xf>(v);
  v += dpp_f64<0x112, 0xf>(v);
  v += dpp_f64<0x114, 0xf>(v);
  v += dpp_f64<0x118, 0xf>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), 63);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Value of v in lane `src` (src uniform across the wave).
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), src);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

}  // namespace ctaux
