// End of a block (Sec. IV C, "Recompute step"): the accepted changes P with
// Gamma^{-1} are applied to N in one rank-k update per sector,
//   N' = N_a - (G - I)_{:,P} Gamma^{-1} N_a{P,:}                 (Eq. Nshermanmorrison,
// equivalently D^{-1}(N - G_{:,P} Gamma^{-1} N_{P,:}) when every vertex changes once),
// and rows / columns of spin-0 vertices are deleted while storing.
//
// k_operands (with the skinny products) builds the compacted operands (and
// copies the times, sites and ids of the configuration after the block into
// compacted order), with Gamma~ = Gamma D^{-1} the column-scaled Gamma of the
// proposal loop (D_b = e^{V_b}/(e^{V_b} - 1) for an old vertex, 1 for a candidate)
//   Ac[i'][a] = ((G - I) D^{-1})_{map(i'), P_a}            (n' x k_a)
//   Bc[a][j'] = sum_b Gamma~^{-1}_{ab} N_a(P_b, map(j'))   (k_a x n')
// so that Ac Bc = (G - I)_{:,P} Gamma^{-1} N_a(P,:).
// and k_rankk computes N'[i'][j'] = N_a(map i', map j') - (Ac Bc)[i'][j'] on
// MFMA 16x16x4 tiles (FP64, or FP32 for FP32 storage), 64x64 or 32x32 outputs
// per workgroup, tiles of every chain scheduled from one persistent grid.
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

void launch_operands(const Batch &b, hipStream_t s);

// Ac and Bc of every chain in one launch (k_operands).
void launch_assemble(const Batch &b, hipStream_t s) { launch_operands(b, s); }

template <typename T>
struct Mfma;
// Accumulator layouts (checked on gfx950 with a probe of D = A B): lane l holds
// column l%16 of the 16x16 block; the FP64 instruction puts register q at row
// l/16 + 4q, the FP32 instruction at row 4(l/16) + q.
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  __device__ static int row(int lk, int q) { return lk + 4 * q; }
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  __device__ static int row(int lk, int q) { return 4 * lk + q; }
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Split-BF16x3 products: an FP32 value x is split into bf16 terms hi = rne(x) and
// lo = rne(x - hi); a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo lo term,
// ~2^-16 of the product, is dropped).  mfma_f32_16x16x16bf16_1k: lane l supplies
// A[l%16][4(l/16) + i] and B[4(l/16) + i][l%16], i < 4, and receives D in the
// layout of the FP32 16x16x4 instruction (row 4(l/16) + q).
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned bf16_rne_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;   // finite x
}

__device__ __forceinline__ void split_bf16(float x, short &hi, short &lo) {
  const unsigned h = bf16_rne_bits(x);
  hi = static_cast<short>(h);
  lo = static_cast<short>(bf16_rne_bits(x - __uint_as_float(h << 16)));
}

// Base value N_a(map i', map j') in the storage type.
template <typename T>
__device__ __forceinline__ T base_entry(const ChainDesc &d, const T *N, const double *Rt, int n, int mi, int mj) {
  if (mi < n) return (mj < n) ? gview(N)[static_cast<size_t>(mi) * d.ld + mj] : T(0);
  if (mj < n) return static_cast<T>(gview(Rt)[static_cast<size_t>(mi - n) * d.ld + mj]);
  return (mi == mj) ? T(1) : T(0);
}

// MFMA 16x16x4 operand layout (one 16x16 block): lane l supplies A[l%16][k0 + l/16]
// and B[k0 + l/16][l%16]; accumulator register q holds D[Mfma<T>::row(l/16, q)][l%16].
// Output tiles of TILE x TILE (64 or 32), each of the four waves owning a
// TILE/2 square of NB x NB MFMA blocks.  Persistent over the tiles of all
// chains: chain c owns tiles [prefix[c], prefix[c+1]), 2 sectors x
// ceil(n'/TILE)^2 each; every workgroup builds the prefix in LDS first.
template <typename T, int TILE, bool BF3 = false>
__global__ __launch_bounds__(256) void k_rankk(const ChainDesc *descs, const ChainState *states, int n_chains) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int SUB = TILE / 2, NB = SUB / 16;
  extern __shared__ int prefix[];   // [n_chains + 1]
  block_prefix<256>(n_chains, prefix, [&](int cc) {
    if (!states[cc].active) return 0;
    const int nt = (states[cc].n_new + TILE - 1) / TILE;
    return 2 * nt * nt;
  });
  const int total = prefix[n_chains];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const ItemSpan span = xcd_items(1, 0);   // neighbouring tiles on one XCD
  for (int k = span.first;; k += span.stride) {
    const int t = span.item(k);
    if (t >= total) break;
    // chain owning tile t (prefix is non-decreasing)
    int lo = 0, hi = n_chains;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const int c = lo;
    const ChainDesc &d = descs[c];
    const ChainState &st = states[c];
    const int n = st.n, np = st.n_new, ka = st.k_a;
    const int nt = (np + TILE - 1) / TILE;
    int local = t - prefix[c];
    const int sec = local / (nt * nt);
    local -= sec * nt * nt;
    const int ti = local / nt, tj = local - ti * nt;
    const int par = st.parity;
    const T *N = static_cast<const T *>(d.N[par][sec]);
    const auto Nout = gview_w(static_cast<T *>(d.N[par ^ 1][sec]));
    const auto Ac = gview(static_cast<const T *>(d.Ac[sec]));
    const auto Bc = gview(static_cast<const T *>(d.Bc[sec]));
    const double *Rt = d.Rt[sec];
    const auto map = gview(d.map);
    const int lda = d.lda, ldn = d.ld;
    const int row0 = ti * TILE + wr * SUB, col0 = tj * TILE + wc * SUB;
    // the N_a entries this lane updates, loaded before the k loop so that their
    // latency overlaps the products
    T base[NB][NB][4];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int cc = col0 + j * 16 + lr;
      const int mj = cc < np ? map[cc] : 0;
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = row0 + i * 16 + Mfma<T>::row(lk, q);
          base[i][j][q] = (r < np && cc < np) ? base_entry<T>(d, N, Rt, n, map[r], mj) : T(0);
        }
    }
    acc_t acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = Mfma<T>::zero();
    if constexpr (BF3) {
     if (ka > 0) {
      // split-BF16x3, k in steps of 16; entries beyond k_a are masked to zero
      for (int k0 = 0; k0 < ka; k0 += 16) {
        v4s ahi[NB], alo[NB], bhi[NB], blo[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int r = row0 + i * 16 + lr;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int k = k0 + 4 * lk + e;
            const float a = (r < np && k < ka) ? static_cast<float>(Ac[ac_offset(r, k, lda >> 2)]) : 0.f;
            short h, l;
            split_bf16(a, h, l);
            ahi[i][e] = h;
            alo[i][e] = l;
          }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int cc = col0 + j * 16 + lr;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int k = k0 + 4 * lk + e;
            const float b = (cc < np && k < ka) ? static_cast<float>(Bc[static_cast<size_t>(k) * ldn + cc]) : 0.f;
            short h, l;
            split_bf16(b, h, l);
            bhi[j][e] = h;
            blo[j][e] = l;
          }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            v4f c = acc[i][j];
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[i], bhi[j], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[i], blo[j], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[i], bhi[j], c, 0, 0, 0);
            acc[i][j] = c;
          }
      }
     }
    } else if (ka > 0) {
      // k in batches of KS k-steps; the next batch's operands are loaded before
      // the current batch's products (two batches in flight).  Ac and Bc are zero
      // between k_a and kpad; steps past kpad load nothing.
      constexpr int KS = TILE == 64 ? 2 : 4;   // bounded by the operand registers
      const int kpad = (ka + 7) & ~7;
      T a0[KS][NB], b0[KS][NB], a1[KS][NB], b1[KS][NB];
      auto load = [&](T (&av)[KS][NB], T (&bv)[KS][NB], int k0) {
#pragma unroll
        for (int u = 0; u < KS; ++u) {
          const bool kok = k0 + 4 * u < kpad;
          const int k = k0 + 4 * u + lk;
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            const int r = row0 + i * 16 + lr;
            av[u][i] = (kok && r < np) ? Ac[ac_offset(r, k, lda >> 2)] : T(0);
          }
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const int cc = col0 + j * 16 + lr;
            bv[u][j] = (kok && cc < np) ? Bc[static_cast<size_t>(k) * ldn + cc] : T(0);
          }
        }
      };
      auto mma = [&](const T (&av)[KS][NB], const T (&bv)[KS][NB], int k0) {
#pragma unroll
        for (int u = 0; u < KS; ++u) {
          if (k0 + 4 * u >= kpad) break;
#pragma unroll
          for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][j] = Mfma<T>::mma(av[u][i], bv[u][j], acc[i][j]);
        }
      };
      int k0 = 0;
      load(a0, b0, k0);
      while (true) {
        if (k0 + 4 * KS < kpad) load(a1, b1, k0 + 4 * KS);
        mma(a0, b0, k0);
        k0 += 4 * KS;
        if (k0 >= kpad) break;
        if (k0 + 4 * KS < kpad) load(a0, b0, k0 + 4 * KS);
        mma(a1, b1, k0);
        k0 += 4 * KS;
        if (k0 >= kpad) break;
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int cc = col0 + j * 16 + lr;
      if (cc >= np) continue;
#pragma unroll
      for (int i = 0; i < NB; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = row0 + i * 16 + Mfma<T>::row(lk, q);
          if (r < np) Nout[static_cast<size_t>(r) * ldn + cc] = base[i][j][q] - acc[i][j][q];
        }
      }
    }
  }
}

template <typename T>
static void launch_rankk_t(const Batch &b, hipStream_t s) {
  const int grid = b.n_cu * 8;
  const size_t lds = sizeof(int) * (b.n_chains + 1);
  if (b.rankk_tile == 32)
    hipLaunchKernelGGL((k_rankk<T, 32>), dim3(grid), dim3(256), lds, s, b.d_desc, b.d_state, b.n_chains);
  else
    hipLaunchKernelGGL((k_rankk<T, 64>), dim3(grid), dim3(256), lds, s, b.d_desc, b.d_state, b.n_chains);
}

void launch_rankk(const Batch &b, hipStream_t s) {
  if (b.precision == kFP64) {
    launch_rankk_t<double>(b, s);
  } else if (b.precision == kFP32) {
    launch_rankk_t<float>(b, s);
  } else {
    const int grid = b.n_cu * 8;
    const size_t lds = sizeof(int) * (b.n_chains + 1);
    if (b.rankk_tile == 32)
      hipLaunchKernelGGL((k_rankk<float, 32, true>), dim3(grid), dim3(256), lds, s, b.d_desc, b.d_state, b.n_chains);
    else
      hipLaunchKernelGGL((k_rankk<float, 64, true>), dim3(grid), dim3(256), lds, s, b.d_desc, b.d_state, b.n_chains);
  }
}

}  // namespace ctaux
