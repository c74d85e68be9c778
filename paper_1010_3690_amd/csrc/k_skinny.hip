// Skinny products with few rows on MFMA f64 16x16x4:
//   C[m][c] = sum_k A(m, k) * B(k, c),  m < M, k < K, c < Ncols,
// with A and B supplied by functors (array reads or gathers) and the result
// handed to an output functor.  They are
//   - the preparation products of a block (Sec. IV A): YT = ZT N^T, Rt = X N
//     (each reads N once) and Gnn = X YT^T + G0nn;
//   - the operand B_c = Gamma~^{-1} N_a(P, map) of the rank-k update (Sec. IV C),
//     with N_a gathered on the fly;
//   - the measurement (Sec. IV D): W = N gR, then G(x tau_j; y 0) = G0 + gL W
//     (gL read from its table for a few chains, interpolated inside the
//     product for many).
// A work item is a tile of 16*NRT rows and 16 columns (two tiles of 16 for
// some products in wave mode, skinny_cols) of one product of one chain (NRT
// covers the largest row count the product can have in the batch); items of
// all chains are enumerated from a per-chain prefix that every workgroup
// builds in LDS, and dealt to the XCDs in chunks (xcd_items).  Two execution
// modes:
//   - split-K: the 8 waves of a workgroup share one item, each taking one
//     contiguous eighth of K, and their partial tiles are summed in LDS in a
//     fixed order (few chains with long K: keeps the GPU busy);
//   - wave: every wave owns items on its own (many chains: no cross-wave
//     reduction, no barrier per item).
// Both sum in a fixed order, so results are deterministic.  The k loop keeps
// two batches of U k-steps in flight (operands of the next batch are loaded
// before the current batch's MFMAs), with U chosen so that NRT*U operand
// registers stay bounded.
#include "ctaux_device.h"

namespace ctaux {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kSkWaves = 8;
constexpr int kSkThreads = kSkWaves * 64;
constexpr int kMeasGRt = 1;               // row tiles per measurement G item
constexpr int kPrepRows = 32;             // rows (candidates) per preparation item

enum SkinnyKind : int { kSkPrep = 0, kSkGnn = 1, kSkMeasW = 2, kSkMeasG = 3, kSkAsmB = 4 };
enum SkinnyMode : int { kModeSplitK = 0, kModeWave = 1 };

// Column tiles of 16 per item.  In wave mode the preparation (and G_nn) and
// measurement products with up to two row tiles take two, so that each A operand
// loaded (candidate rows, gR, or the interpolated gL) serves two MFMA tiles; split-K
// items keep one (a few chains need the items for parallelism), and so do more
// row tiles (their operand registers would spill).
template <int MODE, int KIND, int NRT>
constexpr int skinny_cols() {
  return (MODE == kModeWave && NRT <= 2 &&
          (KIND == kSkPrep || KIND == kSkGnn || KIND == kSkMeasW || KIND == kSkMeasG))
             ? 2
             : 1;
}

// Work items of one chain for a kind (0 when the chain does not take part);
// cols: column tiles of 16 per item.
__device__ __forceinline__ int skinny_items(const ChainDesc &d, const ChainState &st, int kind, int cols = 1) {
  if (!st.active) return 0;
  const int n = st.n, w = 16 * cols;
  const int rg = (st.k_ins + kPrepRows - 1) / kPrepRows;   // row groups of the candidates
  if (kind == kSkPrep) return st.k_ins > 0 ? 4 * rg * ((n + w - 1) / w) : 0;
  if (kind == kSkGnn) return st.k_ins > 0 ? 2 * rg * ((st.k_ins + w - 1) / w) : 0;
  if (kind == kSkAsmB) return (st.k_a > 0 && st.n_new > 0) ? 2 * ((st.n_new + 15) >> 4) : 0;
  if (!st.meas_now) return 0;
  if (kind == kSkMeasW) return 2 * ((n + w - 1) / w);
  const int mtot = d.nc * (d.n_out + 1), rows = 16 * kMeasGRt;
  return 2 * ((mtot + rows - 1) / rows) * ((d.nc + w - 1) / w);
}

// acc[r] += A(16r + m, k) B(k, c) for k in [k_begin, k_end), this wave only.
// Lane l supplies A(16r + l%16, k0 + l/16) and B(k0 + l/16, c0 + l%16);
// bfn(k) returns B(k, c) for the lane's column (0 outside).
template <int NRT, int U, typename AF, typename BF>
__device__ __forceinline__ void wave_mma(AF afn, BF bfn, int M, int k_begin, int k_end, v4d (&acc)[NRT]) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  double b0[U], a0[U][NRT], b1[U], a1[U][NRT];
  auto load = [&](double (&bv)[U], double (&av)[U][NRT], int k0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 4 * u + lk;
      const bool kok = k < k_end;
      bv[u] = kok ? bfn(k) : 0.0;
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
        const int m = r * 16 + lr;
        av[u][r] = (kok && m < M) ? afn(m, k) : 0.0;
      }
    }
  };
  auto mma = [&](const double (&bv)[U], const double (&av)[U][NRT]) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int r = 0; r < NRT; ++r) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][r], bv[u], acc[r], 0, 0, 0);
  };
  constexpr int S = 4 * U;
  int k0 = k_begin;
  if (k0 >= k_end) return;
  load(b0, a0, k0);
  while (true) {
    load(b1, a1, k0 + S);
    mma(b0, a0);
    k0 += S;
    if (k0 >= k_end) break;
    load(b0, a0, k0 + S);
    mma(b1, a1);
    k0 += S;
    if (k0 >= k_end) break;
  }
}

// As wave_mma, with the k index permuted inside groups of 16: in step i of a
// group starting at k0, lane l supplies A(16r + l%16, k0 + 4(l/16) + i) and
// B(k0 + 4(l/16) + i, c).  The four steps of a group then read four
// consecutive k per lane, so operands stored along k (rows of N, of X, Zt,
// YT, gR, gL) load as whole 32-byte pieces, four lanes covering one 128-byte
// line.  The products are the same; only the order of the k terms changes.
// afn and bfn must accept any row below M and any k below k_end, and bfn any
// k for the lane's column (the caller clamps addresses and masks values).
template <int NRT, int U, typename AF, typename BF>
__device__ __forceinline__ void wave_mma_kv(AF afn, BF bfn, int M, int k_begin, int k_end, v4d (&acc)[NRT]) {
  static_assert(U % 4 == 0, "whole groups of four k-steps");
  constexpr int G = U / 4;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  double b0[G][4], a0[G][4][NRT], b1[G][4], a1[G][4][NRT];
  auto load = [&](double (&bv)[G][4], double (&av)[G][4][NRT], int k0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int kb = k0 + 16 * g + 4 * lk;
      if (kb + 3 < k_end) {
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[g][i] = bfn(kb + i);
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          const int m = r * 16 + lr;
          const bool mok = m < M;
          const int mc = mok ? m : 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double v = afn(mc, kb + i);
            av[g][i][r] = mok ? v : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = kb + i;
          const bool kok = k < k_end;
          bv[g][i] = kok ? bfn(k) : 0.0;
#pragma unroll
          for (int r = 0; r < NRT; ++r) {
            const int m = r * 16 + lr;
            av[g][i][r] = (kok && m < M) ? afn(m, k) : 0.0;
          }
        }
      }
    }
  };
  auto mma = [&](const double (&bv)[G][4], const double (&av)[G][4][NRT]) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < NRT; ++r)
          acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g][i][r], bv[g][i], acc[r], 0, 0, 0);
  };
  constexpr int S = 16 * G;
  int k0 = k_begin;
  if (k0 >= k_end) return;
  load(b0, a0, k0);
  while (true) {
    load(b1, a1, k0 + S);
    mma(b0, a0);
    k0 += S;
    if (k0 >= k_end) break;
    load(b0, a0, k0 + S);
    mma(b1, a1);
    k0 += S;
    if (k0 >= k_end) break;
  }
}

// As wave_mma_kv over k in [0, K) for NCT column tiles of 16 (the lane's column
// of tile t is c0 + 16 t + l % 16): each A operand loaded serves NCT MFMAs.
// bfn(k, t) returns B(k, c) for the lane's column of tile t (0 outside).
template <int NRT, int U, int NCT, typename AF, typename BF>
__device__ __forceinline__ void wave_mma_kv_cols(AF afn, BF bfn, int M, int K, v4d (&acc)[NRT][NCT]) {
  static_assert(U % 4 == 0, "whole groups of four k-steps");
  constexpr int G = U / 4;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  double b0[G][4][NCT], a0[G][4][NRT], b1[G][4][NCT], a1[G][4][NRT];
  auto load = [&](double (&bv)[G][4][NCT], double (&av)[G][4][NRT], int k0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int kb = k0 + 16 * g + 4 * lk;
      if (kb + 3 < K) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int t = 0; t < NCT; ++t) bv[g][i][t] = bfn(kb + i, t);
#pragma unroll
        for (int r = 0; r < NRT; ++r) {
          const int m = r * 16 + lr;
          const bool mok = m < M;
          const int mc = mok ? m : 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double v = afn(mc, kb + i);
            av[g][i][r] = mok ? v : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = kb + i;
          const bool kok = k < K;
#pragma unroll
          for (int t = 0; t < NCT; ++t) bv[g][i][t] = kok ? bfn(k, t) : 0.0;
#pragma unroll
          for (int r = 0; r < NRT; ++r) {
            const int m = r * 16 + lr;
            av[g][i][r] = (kok && m < M) ? afn(m, k) : 0.0;
          }
        }
      }
    }
  };
  auto mma = [&](const double (&bv)[G][4][NCT], const double (&av)[G][4][NRT]) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < NRT; ++r)
#pragma unroll
          for (int t = 0; t < NCT; ++t)
            acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g][i][r], bv[g][i][t], acc[r][t], 0, 0, 0);
  };
  constexpr int S = 16 * G;
  int k0 = 0;
  if (K <= 0) return;
  load(b0, a0, k0);
  while (true) {
    load(b1, a1, k0 + S);
    mma(b0, a0);
    k0 += S;
    if (k0 >= K) break;
    load(b0, a0, k0 + S);
    mma(b1, a1);
    k0 += S;
    if (k0 >= K) break;
  }
}

// One wave-mode item of NCT column tiles: C rows [0, M), columns [c0, c0 + 16 NCT),
// handed to out(m, c, value); operands stored along k (wave_mma_kv_cols).
template <int NRT, int NCT, typename AF, typename BF, typename OF>
__device__ __forceinline__ void skinny_item_cols(AF afn, BF bfn, OF out, int M, int K, int Ncols, int c0) {
  v4d acc[NRT][NCT];
#pragma unroll
  for (int r = 0; r < NRT; ++r)
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[r][t] = v4d{0.0, 0.0, 0.0, 0.0};
  wave_mma_kv_cols<NRT, 4, NCT>(afn, bfn, M, K, acc);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < NRT; ++r)
#pragma unroll
    for (int t = 0; t < NCT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = r * 16 + (lane >> 4) + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
        const int cc = c0 + 16 * t + (lane & 15);
        if (m < M && cc < Ncols) out(m, cc, acc[r][t][q]);
      }
}

// One item: C tile rows [0, M), columns [c0, c0 + 16), handed to out(m, c, value).
// UO overrides the k-steps per batch (0: the default for NRT).
// KV: operands stored along k, loaded four k at a time (wave_mma_kv; up to four
// row tiles).
template <int MODE, int NRT, int UO = 0, bool KV = false, typename AF, typename BF, typename OF>
__device__ __forceinline__ void skinny_item(AF afn, BF bfn, OF out, int M, int K, int Ncols, int c0, double *red) {
  constexpr bool kv = KV && NRT <= 4;
  constexpr int U = kv ? (NRT == 1 ? 8 : 4) : (UO ? UO : (NRT == 1 ? 8 : (NRT == 2 ? 4 : (NRT == 4 ? 2 : 1))));
  auto mma = [&](int kbeg, int kend, v4d (&acc)[NRT]) {
    if constexpr (kv) wave_mma_kv<NRT, U>(afn, bfn, M, kbeg, kend, acc);
    else wave_mma<NRT, U>(afn, bfn, M, kbeg, kend, acc);
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  v4d acc[NRT];
#pragma unroll
  for (int r = 0; r < NRT; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
  if (MODE == kModeWave) {
    mma(0, K, acc);
#pragma unroll
    for (int r = 0; r < NRT; ++r) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = r * 16 + (lane >> 4) + 4 * q;   // FP64 16x16x4 accumulator: row l/16 + 4q
        const int cc = c0 + (lane & 15);
        if (m < M && cc < Ncols) out(m, cc, acc[r][q]);
      }
    }
    return;
  }
  // contiguous eighths of K, rounded to whole groups of 16 k-steps
  const int chunk = (((K + kSkWaves - 1) / kSkWaves) + 15) & ~15;
  const int kb = wave * chunk;
  mma(kb, min(K, kb + chunk), acc);
  for (int w = 0; w < kSkWaves; ++w) {   // fixed-order reduction of the partial tiles
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < NRT; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double *p = red + (r * 64 + lane) * 4 + q;
          *p = (w == 0) ? acc[r][q] : *p + acc[r][q];
        }
      }
    }
    lds_barrier();
  }
  for (int e = tid; e < NRT * 256; e += kSkThreads) {
    const int r = e >> 8, l = (e >> 2) & 63, q = e & 3;
    const int m = r * 16 + (l >> 4) + 4 * q;
    const int cc = c0 + (l & 15);
    if (m < M && cc < Ncols) out(m, cc, red[e]);
  }
  lds_barrier();   // red is reused by the next item
}

// Inlined into each kernel: as a function of its own (kind 4 is called from two
// kernels) its lambdas and operand arrays would live in scratch memory.
template <typename T, int MODE, int NRT, int KIND>
__device__ __forceinline__ void skinny_dispatch(const ChainDesc &d, const ChainState &st, int local, double *red) {
  const int lane = threadIdx.x & 63, lr = lane & 15;
  const int n = st.n, par = st.parity;
  if constexpr (KIND == kSkPrep) {
    // per row group of candidates: items 0..2nt-1 YT[sec] = ZT N^T, 2nt..4nt-1 Rt[sec] = X N
    constexpr int NC = skinny_cols<MODE, KIND, NRT>();
    const int nt = (n + 16 * NC - 1) / (16 * NC);
    const int grp = local / (4 * nt), r0 = grp * kPrepRows;
    const int loc2 = local - grp * 4 * nt;
    const int job = loc2 / nt, c0 = (loc2 - job * nt) * 16 * NC, sec = job & 1, ld = d.ld;
    const auto A = gview((job < 2) ? d.ZT[sec] : d.X[sec]);
    const int rt = (d.kmax + 15) >> 4;
    const auto N = gview(static_cast<const T *>(d.N[par][sec]));
    const auto C = gview_w(((job < 2) ? d.YT[sec] : d.Rt[sec]) + static_cast<size_t>(r0) * ld);
    const int M = min(kPrepRows, st.k_ins - r0);
    const int c = c0 + lr;
    const bool cok = c < n;
    const int cc0 = cok ? c : 0;   // in-bounds address; the value is masked
    auto afn = [=](int m, int k) { return A[cand_offset(r0 + m, k, rt)]; };
    auto out = [=](int m, int cc, double v) { C[static_cast<size_t>(m) * ld + cc] = v; };
    if constexpr (NC > 1) {
      // column tile t: column c0 + 16 t + l % 16 (clamped in-bounds, masked)
      if (job < 2) {
        auto bfn = [=](int k, int t) {
          const int ct = c + 16 * t, cs = ct < n ? ct : 0;
          const double v = static_cast<double>(N[static_cast<size_t>(cs) * ld + k]);
          return ct < n ? v : 0.0;
        };
        skinny_item_cols<NRT, NC>(afn, bfn, out, M, n, n, c0);
      } else {
        auto bfn = [=](int k, int t) {
          const int ct = c + 16 * t, cs = ct < n ? ct : 0;
          const double v = static_cast<double>(N[static_cast<size_t>(k) * ld + cs]);
          return ct < n ? v : 0.0;
        };
        skinny_item_cols<NRT, NC>(afn, bfn, out, M, n, n, c0);
      }
    } else if (job < 2) {
      auto bfn = [=](int k) {
        const double v = static_cast<double>(N[static_cast<size_t>(cc0) * ld + k]);
        return cok ? v : 0.0;
      };
      skinny_item<MODE, NRT, 0, true>(afn, bfn, out, M, n, n, c0, red);
    } else {
      auto bfn = [=](int k) {
        const double v = static_cast<double>(N[static_cast<size_t>(k) * ld + cc0]);
        return cok ? v : 0.0;
      };
      skinny_item<MODE, NRT, 0, true>(afn, bfn, out, M, n, n, c0, red);
    }
  } else if constexpr (KIND == kSkGnn) {
    // Gnn[sec] = X YT^T + G0nn (K = 0 still writes Gnn = G0nn), per row group
    constexpr int NC = skinny_cols<MODE, KIND, NRT>();
    const int ki = st.k_ins, nt = (ki + 16 * NC - 1) / (16 * NC);
    const int grp = local / (2 * nt), r0 = grp * kPrepRows;
    const int loc2 = local - grp * 2 * nt;
    const int sec = loc2 / nt, c0 = (loc2 - sec * nt) * 16 * NC, ld = d.ld, km = d.kmax;
    const auto X = gview(d.X[sec]), YT = gview(d.YT[sec]);
    const int rt = (km + 15) >> 4;
    const auto G0nn = gview(d.G0nn[sec] + static_cast<size_t>(r0) * km);
    const auto Gnn = gview_w(d.Gnn[sec] + static_cast<size_t>(r0) * km);
    const int M = min(kPrepRows, ki - r0);
    const int c = c0 + lr;
    const bool cok = c < ki;
    const int cc0 = cok ? c : 0;
    auto afn = [=](int m, int k) { return X[cand_offset(r0 + m, k, rt)]; };
    auto bfn = [=](int k) {
      const double v = YT[static_cast<size_t>(cc0) * ld + k];
      return cok ? v : 0.0;
    };
    auto out = [=](int m, int cc, double v) {
      Gnn[static_cast<size_t>(m) * km + cc] = v + G0nn[static_cast<size_t>(m) * km + cc];
    };
    if constexpr (NC > 1) {
      auto bfn2 = [=](int k, int t) {
        const int ct = c + 16 * t, cs = ct < ki ? ct : 0;
        const double v = YT[static_cast<size_t>(cs) * ld + k];
        return ct < ki ? v : 0.0;
      };
      skinny_item_cols<NRT, NC>(afn, bfn2, out, M, n, ki, c0);
    } else {
      skinny_item<MODE, NRT, 0, true>(afn, bfn, out, M, n, ki, c0, red);
    }
  } else if constexpr (KIND == kSkAsmB) {
    // Bc[sec] = Gamma~^{-1} N_a(P, map): rows a < kpad (zero beyond k_a), K = k_a
    const int np = st.n_new, ka = st.k_a, kpad = (ka + 7) & ~7, nt = (np + 15) >> 4;
    const int sec = local / nt, c0 = (local - sec * nt) * 16, ld = d.ld, kcap = d.kcap;
    const auto Gi = gview(d.Ginv[sec]), Rt = gview(d.Rt[sec]);
    const auto N = gview(static_cast<const T *>(d.N[par][sec]));
    const auto Bc = gview_w(static_cast<T *>(d.Bc[sec]));
    const int c = c0 + lr;
    const int mj = c < np ? gview(d.map)[c] : -1;
    // P (k_a <= 64 entries) is copied once per item into this wave's part of
    // red (which wave mode leaves unused), so the gathers of N_a need no
    // dependent global load; batches of k-steps are as long as registers allow
    int *Ps = reinterpret_cast<int *>(red) + (threadIdx.x >> 6) * 64;
    Ps[lane] = lane < ka ? gview(d.P)[lane] : 0;
    __builtin_amdgcn_wave_barrier();
    auto afn = [=](int m, int k) { return m < ka ? Gi[m * kcap + k] : 0.0; };
    auto bfn = [=](int k) {
      if (mj < 0) return 0.0;
      const int pb = Ps[k];
      if (pb < n) return (mj < n) ? static_cast<double>(N[static_cast<size_t>(pb) * ld + mj]) : 0.0;
      if (mj < n) return Rt[static_cast<size_t>(pb - n) * ld + mj];
      return pb == mj ? 1.0 : 0.0;
    };
    auto out = [=](int m, int cc, double v) { Bc[static_cast<size_t>(m) * ld + cc] = static_cast<T>(v); };
    constexpr int UB = NRT <= 2 ? 8 : (NRT == 4 ? 4 : 1);   // bounded by the operand registers
    skinny_item<MODE, NRT, UB>(afn, bfn, out, kpad, ka, np, c0, red);
  } else if constexpr (KIND == kSkMeasW) {
    // W[sec] = N gR as (gRT N^T)^T: C[l][y]
    constexpr int NC = skinny_cols<MODE, KIND, NRT>();
    const int nt = (n + 16 * NC - 1) / (16 * NC);
    const int sec = local / nt, c0 = (local - sec * nt) * 16 * NC, ld = d.ld, nc = d.nc;
    const auto gR = gview(d.gR[sec]);
    const auto N = gview(static_cast<const T *>(d.N[par][sec]));
    const auto W = gview_w(d.W[sec]);
    const int c = c0 + lr;
    const bool cok = c < n;
    const int cc0 = cok ? c : 0;
    const int rt = (nc + 15) >> 4;
    auto afn = [=](int m, int k) { return gR[cand_offset(m, k, rt)]; };
    auto bfn = [=](int k) {
      const double v = static_cast<double>(N[static_cast<size_t>(cc0) * ld + k]);
      return cok ? v : 0.0;
    };
    if constexpr (MODE == kModeWave) {
      // many chains: row l of W at the time-ordered position of vertex l
      const auto pos = gview(d.mpos);
      auto out = [=](int m, int cc, double v) { W[static_cast<size_t>(pos[cc]) * nc + m] = v; };
      if constexpr (NC > 1) {
        auto bfn2 = [=](int k, int t) {
          const int ct = c + 16 * t, cs = ct < n ? ct : 0;
          const double v = static_cast<double>(N[static_cast<size_t>(cs) * ld + k]);
          return ct < n ? v : 0.0;
        };
        skinny_item_cols<NRT, NC>(afn, bfn2, out, nc, n, n, c0);
      } else {
        skinny_item<MODE, NRT, 0, true>(afn, bfn, out, nc, n, n, c0, red);
      }
    } else {
      auto out = [=](int m, int cc, double v) { W[static_cast<size_t>(cc) * nc + m] = v; };
      skinny_item<MODE, NRT, 0, true>(afn, bfn, out, nc, n, n, c0, red);
    }
  } else {
    // Gxy: rows m = j*nc + x (j = 0: tau = 0+, j >= 1: tau_{j-1}); item = 16*kMeasGRt rows x 16 columns y
    constexpr int NC = skinny_cols<MODE, KIND, NRT>();
    const int nc = d.nc, Mtot = nc * (d.n_out + 1), rows = 16 * kMeasGRt;
    const int ngroups = (Mtot + rows - 1) / rows, ntiles = (nc + 16 * NC - 1) / (16 * NC);
    const int sec = local / (ngroups * ntiles), rem = local - sec * ngroups * ntiles;
    const int g = rem / ntiles, c0 = (rem - g * ntiles) * 16 * NC;
    const int m0 = g * rows, M = min(rows, Mtot - m0);
    const auto W = gview(d.W[sec]);
    const double dt = d.beta / d.n_out;
    const auto Gxy = gview_w(d.Gxy[sec]);
    const int c = c0 + lr;
    const bool cok = c < nc;
    const int cc0 = cok ? c : 0;
    auto bfn = [=](int l) {
      const double v = W[static_cast<size_t>(l) * nc + cc0];
      return cok ? v : 0.0;
    };
    auto out = [&](int m, int cc, double v) {
      const int mm = m0 + m, j = mm / nc, x = mm - j * nc;
      const double tj = j == 0 ? 0.0 : (static_cast<double>(j - 1) + 0.5) * dt;
      Gxy[static_cast<size_t>(j) * nc * nc + x * nc + cc] = g0_interp(d, sec, x, cc, tj) + v;
    };
    if constexpr (MODE == kModeSplitK) {
      // few chains: gL from its table (k_meas_gL)
      const int ld = d.ld;
      const auto gL = gview(d.gL[sec] + static_cast<size_t>(m0) * ld);
      auto afn = [=](int m, int l) { return gL[static_cast<size_t>(m) * ld + l]; };
      skinny_item<MODE, NRT, 0, true>(afn, bfn, out, M, n, nc, c0, red);
    } else {
      // many chains: gL_{(j, x), l} = G0_{x x_l}(tau_j - tau_l) (e^{V_l} - 1)
      // interpolated where the product needs it (no table of (n_out + 1) nc n
      // entries per sector written and read back)
      // the sum over vertices runs in time order (k_meas_tsort; W is stored in it)
      const auto mtau = gview(d.mtau), mfac = gview(d.mfac + sec * d.n_cap);
      const auto msite = gview(d.msite);
      // one row tile: lane l supplies row l % 16 for every k (wave_mma_kv), so its
      // output time and site are fixed for the item and computed once here (a
      // masked row beyond M takes any in-range values)
      static_assert(NRT == 1, "one row tile per G item");
      const int mm = m0 + (lr < M ? lr : 0), jr = mm / nc, xr = mm - jr * nc;
      const double tjr = jr == 0 ? 0.0 : (static_cast<double>(jr - 1) + 0.5) * dt;
      // the functor captures the table parameters, not the chain descriptor (a
      // copy of which would sit in scratch memory)
      const auto g0s = gview(d.g0[sec]);
      const auto sdrow = gview(d.site_disp) + xr * nc;
      const int ntau = d.n_tau;
      const double beta = d.beta, inv_h = d.inv_h;
      auto afn = [=](int, int k) {
        const auto tab = g0s + static_cast<int64_t>(sdrow[msite[k]]) * ntau;
        return interp_table(tab, beta, inv_h, ntau, tjr - mtau[k]) * mfac[k];
      };
      auto bfn2 = [=](int l, int t) {
        const int ct = c + 16 * t, cs = ct < nc ? ct : 0;
        const double v = W[static_cast<size_t>(l) * nc + cs];
        return ct < nc ? v : 0.0;
      };
      skinny_item_cols<NRT, NC>(afn, bfn2, out, M, n, nc, c0);
    }
  }
}

// Persistent over the work items of all chains; one instantiation per product
// kind, so that each gets the registers of its own operands.
template <typename T, int MODE, int NRT, int KIND>
__global__ __launch_bounds__(kSkThreads) void k_skinny(const ChainDesc *descs, const ChainState *states,
                                                        int n_chains) {
  extern __shared__ int pre[];   // [n_chains + 1]
  __shared__ double red[NRT * 256];
  const int wave = threadIdx.x >> 6;
  block_prefix<kSkThreads>(n_chains, pre,
                           [&](int cc) { return skinny_items(descs[cc], states[cc], KIND, skinny_cols<MODE, KIND, NRT>()); });
  const int total = pre[n_chains];
  // the preparation products' items are dealt one by one (chunks cost them more
  // in balance than they save in L2 hits)
  constexpr bool chunked = KIND != kSkPrep;
  const ItemSpan span = (MODE == kModeWave) ? xcd_items(kSkWaves, wave, chunked) : xcd_items(1, 0, chunked);
  for (int k = span.first;; k += span.stride) {
    const int item = span.item(k);
    if (item >= total) break;
    int lo = 0, hi = n_chains;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= item) lo = mid; else hi = mid;
    }
    skinny_dispatch<T, MODE, NRT, KIND>(descs[lo], states[lo], item - pre[lo], red);
  }
}

// The operands of the rank-k update on the chain grid (a chain's workgroups on
// one XCD when many chains run):
//   Ac[i'][a] = ((G - I) D^{-1})_{map(i'), P_a} (the column scaling of the proposal
//   kernel's Gamma~, so that Ac Gamma~^{-1} = (G - I)_{:,P} Gamma^{-1}), element by element from the chain's
//   first workgroups up, after the configuration's times, sites and ids are
//   copied into compacted order;
//   with NRT > 0 also Bc = Gamma~^{-1} N_a(P, map), one wave per 16-column item
//   from the chain's last workgroups down.
// Both read only what the proposal kernel left.  One launch for both saves a
// kernel on the critical path of a few long chains; with many chains the MFMA
// registers of Bc would cut the occupancy the Ac gathers need, so Bc then runs
// as a persistent skinny product of its own (NRT = 0 here).
template <typename T, int NRT>
__global__ __launch_bounds__(256) void k_operands(const ChainDesc *descs, const ChainState *states, int n_chains,
                                                  int xcd_g) {
  __shared__ double red[4 * 32];   // P, 64 entries per wave, for the Bc items
  const ChainBlock cb = chain_block(xcd_g);
  const int c = cb.c;
  if (c >= n_chains) return;
  const ChainDesc &d = descs[c];
  const ChainState &st = states[c];
  if (!st.active) return;
  if constexpr (NRT > 0) {
    const int items = skinny_items(d, st, kSkAsmB);
    for (int item = (cb.g - 1 - cb.sub) * 4 + (threadIdx.x >> 6); item < items; item += cb.g * 4)
      skinny_dispatch<T, kModeWave, NRT, kSkAsmB>(d, st, item, red);
  }
  const int n = st.n, np = st.n_new, ka = st.k_a;
  const int par = st.parity;
  {
    // the configuration after the block (times, sites, ids) in compacted order;
    // the spins and the map itself were written by the proposal kernel
    const auto map = gview(d.map);
    const auto tau_o = gview(d.tau[par]), ctau = gview(d.ctau);
    const auto site_o = gview(d.site[par]), csite = gview(d.csite);
    const auto id_o = gview(d.id[par]), cid = gview(d.cid);
    const auto tau_n = gview_w(d.tau[par ^ 1]);
    const auto site_n = gview_w(d.site[par ^ 1]);
    const auto id_n = gview_w(d.id[par ^ 1]);
    for (int pos = cb.sub * 256 + threadIdx.x; pos < np; pos += cb.g * 256) {
      const int i = map[pos];
      if (i < n) {
        tau_n[pos] = tau_o[i];
        site_n[pos] = site_o[i];
        id_n[pos] = id_o[i];
      } else {
        tau_n[pos] = ctau[i - n];
        site_n[pos] = csite[i - n];
        id_n[pos] = cid[i - n];
      }
    }
  }
  if (ka == 0 || np == 0) return;
  const int kpad = (ka + 7) & ~7;
  const int32_t *s0 = d.s0[par];
  // Ac in ac_offset order: consecutive threads write consecutive entries of a
  // block (16 rows x one k-step); rows of the last row tile beyond n' are skipped
  const int steps = d.lda >> 2, sk = kpad >> 2, nrt = (np + 15) >> 4;
  const int64_t per_sec = static_cast<int64_t>(nrt) * sk * 64;   // Ac entries per sector
  const int64_t total = 2 * per_sec;
  const int *map = d.map, *P = d.P;
  for (int64_t e = cb.sub * 256ll + threadIdx.x; e < total; e += cb.g * 256ll) {
    const int sec = static_cast<int>(e / per_sec);
    const int r = static_cast<int>(e - sec * per_sec);
    const int rt = r / (sk * 64), rem = r - rt * sk * 64, s = rem >> 6, l = rem & 63;
    const int i = rt * 16 + (l & 15), a = 4 * s + (l >> 4);
    if (i >= np) continue;
    const T *N = static_cast<const T *>(d.N[par][sec]);
    double v = 0.0;
    if (a < ka) {
      // (G - I)_{map, P} D^{-1}: (N_a - I) for an old column, (G - I) for a candidate
      const int mi = gview(map)[i], pa = gview(P)[a];
      v = (pa < n ? na_entry<T>(d, N, n, sec, mi, pa) : g_entry<T>(d, N, s0, n, sec, mi, pa)) - (mi == pa ? 1.0 : 0.0);
    }
    gview_w(static_cast<T *>(d.Ac[sec]))[ac_offset(i, a, steps)] = static_cast<T>(v);
  }
}

template <typename T, int NRT>
static void launch_ops(const Batch &b, hipStream_t s) {
  hipLaunchKernelGGL((k_operands<T, NRT>), chain_grid(b), dim3(256), 0, s, b.d_desc, b.d_state, b.n_chains,
                     chain_grid_arg(b));
}

template <typename T, int MODE, int NRT, int KIND>
static void launch_kk(const Batch &b, hipStream_t s) {
  const size_t lds = sizeof(int) * (b.n_chains + 1);
  // the measurement products read the state the last block left (d_mstate)
  const ChainState *states = (KIND == kSkMeasW || KIND == kSkMeasG) ? b.d_mstate : b.d_state;
  hipLaunchKernelGGL((k_skinny<T, MODE, NRT, KIND>), dim3(b.n_cu * 2), dim3(kSkThreads), lds, s, b.d_desc, states,
                     b.n_chains);
}

// Only the (kind, row tiles, mode) combinations launch_skinny can choose are
// instantiated: preparation and G_nn take at most 2 row tiles (32 candidates),
// G one, B_c at most 4 (k_cap <= 64) and always one wave per item.
template <typename T, int MODE, int NRT>
static void launch_k(const Batch &b, hipStream_t s, int kind) {
  switch (kind) {
    case kSkPrep:
      if constexpr (NRT <= 2) launch_kk<T, MODE, NRT, kSkPrep>(b, s);
      break;
    case kSkGnn:
      if constexpr (NRT <= 2) launch_kk<T, MODE, NRT, kSkGnn>(b, s);
      break;
    case kSkMeasW:
      launch_kk<T, MODE, NRT, kSkMeasW>(b, s);
      break;
    case kSkMeasG:
      if constexpr (NRT == kMeasGRt) launch_kk<T, MODE, NRT, kSkMeasG>(b, s);
      break;
    default:
      if constexpr (MODE == kModeWave && NRT <= 4) launch_kk<T, MODE, NRT, kSkAsmB>(b, s);
      break;
  }
}

template <typename T, int MODE>
static void launch_m(const Batch &b, hipStream_t s, int kind, int nrt) {
  switch (nrt) {
    case 1: launch_k<T, MODE, 1>(b, s, kind); break;
    case 2: launch_k<T, MODE, 2>(b, s, kind); break;
    case 4: launch_k<T, MODE, 4>(b, s, kind); break;
    default: launch_k<T, MODE, 8>(b, s, kind); break;
  }
}

static int host_row_tiles(int M) {
  const int t = (M + 15) / 16;
  return t <= 1 ? 1 : (t <= 2 ? 2 : (t <= 4 ? 4 : 8));
}

void launch_skinny(const Batch &b, hipStream_t s, int kind) {
  // Row tiles per item cover the largest M the kind can have in this batch:
  // up to 32 candidates per row group (preparation), nc (W), k_a <= k_cap (B_c),
  // one tile (G).
  const int M = kind == kSkPrep || kind == kSkGnn ? (b.kmax < kPrepRows ? b.kmax : kPrepRows)
              : kind == kSkMeasW ? b.nc_max
              : kind == kSkAsmB ? ((b.kcap + 7) & ~7) : 16 * kMeasGRt;
  const int nrt = host_row_tiles(M);
  // Products with K = k_a (B_c) are short: one wave per item.  Otherwise split K
  // across the waves of a workgroup when few chains run (long K, few items).
  const bool wave = (kind == kSkAsmB || b.n_chains >= 8);
  if (b.precision != kFP64) {
    if (wave) launch_m<float, kModeWave>(b, s, kind, nrt);
    else launch_m<float, kModeSplitK>(b, s, kind, nrt);
  } else {
    if (wave) launch_m<double, kModeWave>(b, s, kind, nrt);
    else launch_m<double, kModeSplitK>(b, s, kind, nrt);
  }
}

void launch_operands(const Batch &b, hipStream_t s) {
  if (b.n_chains >= 8) {   // Ac here, Bc as a persistent skinny product
    if (b.precision != kFP64) launch_ops<float, 0>(b, s);
    else launch_ops<double, 0>(b, s);
    launch_skinny(b, s, kSkAsmB);
    return;
  }
  // row tiles of Bc cover k_cap (<= 64) rounded up to 8
  const int nrt = host_row_tiles((b.kcap + 7) & ~7);
  if (b.precision != kFP64) {
    if (nrt == 1) launch_ops<float, 1>(b, s);
    else if (nrt == 2) launch_ops<float, 2>(b, s);
    else launch_ops<float, 4>(b, s);
  } else {
    if (nrt == 1) launch_ops<double, 1>(b, s);
    else if (nrt == 2) launch_ops<double, 2>(b, s);
    else launch_ops<double, 4>(b, s);
  }
}

}  // namespace ctaux
