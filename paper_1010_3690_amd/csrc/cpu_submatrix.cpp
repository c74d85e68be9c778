// The CT-AUX submatrix update on the host CPU (C ABI in include/ctaux_cpu.h):
// one chain, FP64, single-threaded; the O(n^2 k) work of a block runs as
// cache-blocked matrix-matrix loops instead of the memory-bound rank-1 updates
// (Gull et al., Sec. IV).  Written for the host: row-major arrays, the rows of
// N streamed once per product with the block's small operands held in L1/L2.
//
// Algebra of a block (the same as the GPU library's):
//  * candidates j (the block's insertion proposals, in order) are pre-inserted
//    with spin 0; the augmented N_a = [[N, 0], [Rt, 1]] with Rt = X N,
//    X_ji = G0(tau_j - tau_i)(e^{V_i} - 1), and G of the candidate columns,
//    Y = N Z with Z_ij = G0(tau_i - tau_j), Gnn = X Y + G0nn (Sec. IV A);
//  * Gamma is kept column-scaled, Gamma~ = Gamma D^{-1} with D_b = e^{V_b}/(e^{V_b} - 1)
//    for an old vertex and 1 for a candidate, so its entries are those of
//    (N_a - I) (old columns) or (G - I) (candidate columns) minus 1/(gh_b D_b) on
//    the diagonal, gh_b = e^{V(s_b) - V(s0_b)} - 1 the net change of vertex b;
//  * a new change grows X = Gamma~^{-1} by partitioning (Sec. III B 2):
//    beta~ = d - w^T X s, sector ratio -gh D_p beta~ (Eq. ratS); or (growth
//    mode 1) an LU factorisation Gamma~ = L U grows by the solutions of
//    L y = s and U^T x = w, with beta~ = d - x^T y (Sec. III B 1, Eqs. lineq1,
//    lineq2, detrat): L gains the row [x^T 1], U the column [y; beta~], and a
//    repeated change takes X_aa from two triangular solves and factorises
//    Gamma~ again once accepted (in place of Bennett's rank-1 update);
//  * a further change of a vertex already in P replaces its gh (ratio by the
//    matrix determinant lemma, X by Sherman-Morrison), and a change back to the
//    block-start spin removes its slot (ratio X_aa / (-gh D_p), X by the Schur
//    complement): the modification the paper asks for repeated changes;
//  * N' = N_a - [(G - I)_{:,P} D^{-1}] Gamma~^{-1} N_a(P, :) on the vertices that
//    stay (Eq. Nshermanmorrison, spin-0 rows and columns deleted, Sec. IV C).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <immintrin.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ctaux_cpu.h"

namespace {

// ---- C += alpha A B on row-major FP64 arrays, read in place ----
// A kMr x kNr tile of C accumulates in twelve AVX2 registers (named
// variables, so that they are not kept in memory): per k step, kMr broadcasts
// of A and two loads of a row of B feed twelve FMAs.  The caller chooses
// leading dimensions that are not multiples of 512 doubles (N's is 64 m + 8),
// so that the rows of a tile fall in different cache sets.
constexpr int kMr = 6, kNr = 8, kKc = 256;

// full-width tile; rows of A beyond mr repeat row 0 and are not stored
void tile(int mr, int k, const double *a, int lda, const double *b, int ldb, double *c, int ldc, double alpha) {
  const double *a0 = a, *a1 = mr > 1 ? a + lda : a, *a2 = mr > 2 ? a + 2 * static_cast<size_t>(lda) : a;
  const double *a3 = mr > 3 ? a + 3 * static_cast<size_t>(lda) : a, *a4 = mr > 4 ? a + 4 * static_cast<size_t>(lda) : a;
  const double *a5 = mr > 5 ? a + 5 * static_cast<size_t>(lda) : a;
  __m256d c00 = _mm256_setzero_pd(), c01 = c00, c10 = c00, c11 = c00, c20 = c00, c21 = c00;
  __m256d c30 = c00, c31 = c00, c40 = c00, c41 = c00, c50 = c00, c51 = c00;
  for (int p = 0; p < k; ++p) {
    const double *bp = b + static_cast<size_t>(p) * ldb;
    const __m256d b0 = _mm256_loadu_pd(bp), b1 = _mm256_loadu_pd(bp + 4);
    __m256d ar = _mm256_broadcast_sd(a0 + p);
    c00 = _mm256_fmadd_pd(ar, b0, c00); c01 = _mm256_fmadd_pd(ar, b1, c01);
    ar = _mm256_broadcast_sd(a1 + p);
    c10 = _mm256_fmadd_pd(ar, b0, c10); c11 = _mm256_fmadd_pd(ar, b1, c11);
    ar = _mm256_broadcast_sd(a2 + p);
    c20 = _mm256_fmadd_pd(ar, b0, c20); c21 = _mm256_fmadd_pd(ar, b1, c21);
    ar = _mm256_broadcast_sd(a3 + p);
    c30 = _mm256_fmadd_pd(ar, b0, c30); c31 = _mm256_fmadd_pd(ar, b1, c31);
    ar = _mm256_broadcast_sd(a4 + p);
    c40 = _mm256_fmadd_pd(ar, b0, c40); c41 = _mm256_fmadd_pd(ar, b1, c41);
    ar = _mm256_broadcast_sd(a5 + p);
    c50 = _mm256_fmadd_pd(ar, b0, c50); c51 = _mm256_fmadd_pd(ar, b1, c51);
  }
  const __m256d al = _mm256_set1_pd(alpha);
  auto put = [&](int r, __m256d v0, __m256d v1) {
    double *cr = c + static_cast<size_t>(r) * ldc;
    _mm256_storeu_pd(cr, _mm256_fmadd_pd(al, v0, _mm256_loadu_pd(cr)));
    _mm256_storeu_pd(cr + 4, _mm256_fmadd_pd(al, v1, _mm256_loadu_pd(cr + 4)));
  };
  put(0, c00, c01);
  if (mr > 1) put(1, c10, c11);
  if (mr > 2) put(2, c20, c21);
  if (mr > 3) put(3, c30, c31);
  if (mr > 4) put(4, c40, c41);
  if (mr > 5) put(5, c50, c51);
}

// tile narrower than kNr (the last columns of C)
void tile_edge(int mr, int nr, int k, const double *a, int lda, const double *b, int ldb, double *c, int ldc,
               double alpha) {
  double acc[kMr][kNr] = {};
  for (int p = 0; p < k; ++p)
    for (int r = 0; r < mr; ++r) {
      const double ar = a[static_cast<size_t>(r) * lda + p];
      for (int q = 0; q < nr; ++q) acc[r][q] += ar * b[static_cast<size_t>(p) * ldb + q];
    }
  for (int r = 0; r < mr; ++r)
    for (int q = 0; q < nr; ++q) c[static_cast<size_t>(r) * ldc + q] += alpha * acc[r][q];
}

// C (m x n) += alpha A (m x k) B (k x n), alpha = +-1.  For each panel of kNr
// columns of B (kKc rows, held in L1) every strip of kMr rows of A passes.
void gemm(int m, int n, int k, const double *A, int lda, const double *B, int ldb, double *C, int ldc,
          double alpha) {
  for (int pc = 0; pc < k; pc += kKc) {
    const int kb = std::min(kKc, k - pc);
    for (int j0 = 0; j0 < n; j0 += kNr) {
      const int nr = std::min(kNr, n - j0);
      const double *b = B + static_cast<size_t>(pc) * ldb + j0;
      for (int i0 = 0; i0 < m; i0 += kMr) {
        const int mr = std::min(kMr, m - i0);
        const double *a = A + static_cast<size_t>(i0) * lda + pc;
        double *c = C + static_cast<size_t>(i0) * ldc + j0;
        if (nr == kNr)
          tile(mr, kb, a, lda, b, ldb, c, ldc, alpha);
        else
          tile_edge(mr, nr, kb, a, lda, b, ldb, c, ldc, alpha);
      }
    }
  }
}

// Y += N Z and Rt += X N in one pass over N (n0 x n0, leading dimension ldn):
// each block of kBr rows x kBw columns of N serves both products while it is
// in L1/L2 (Z, Y: n0 x kp; X, Rt: ki x n0)
void prep_products(int n0, int ki, int kp, const double *Nm, int ldn, const double *X, const double *Z, double *Y,
                   double *Rt) {
  constexpr int kBr = 24, kBw = 256;
  for (int c0 = 0; c0 < n0; c0 += kBw) {
    const int w = std::min(kBw, n0 - c0);
    for (int i0 = 0; i0 < n0; i0 += kBr) {
      const int r = std::min(kBr, n0 - i0);
      const double *blk = Nm + static_cast<size_t>(i0) * ldn + c0;
      gemm(r, kp, w, blk, ldn, Z + static_cast<size_t>(c0) * kp, kp, Y + static_cast<size_t>(i0) * kp, kp, 1.0);
      gemm(ki, w, r, X + i0, n0, blk, ldn, Rt + c0, n0, 1.0);
    }
  }
}

// leading dimension of an array of rows of length n: 64 m + 8 doubles
int pad_ld(int n) { return (n + 63) / 64 * 64 + 8; }

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ----
void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c[3] ^ k1;
    c[1] = static_cast<uint32_t>(p1);
    c[3] = static_cast<uint32_t>(p0);
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

double unit53(uint32_t hi, uint32_t lo) {
  return static_cast<double>(((static_cast<uint64_t>(hi) << 32) | lo) >> 11) * (1.0 / 9007199254740992.0);
}

// The five uniforms of proposal `index`: counter (index lo, index hi, chain, tag),
// key = seed; tag 0: type, accept; tag 1: tau, pick; tag 2: spin.
void uniforms(uint64_t seed, uint32_t chain, uint64_t index, double u[5]) {
  for (uint32_t tag = 0; tag < 3; ++tag) {
    uint32_t c[4] = {static_cast<uint32_t>(index), static_cast<uint32_t>(index >> 32), chain, tag};
    philox(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    if (tag == 0) { u[0] = unit53(c[0], c[1]); u[1] = unit53(c[2], c[3]); }
    else if (tag == 1) { u[2] = unit53(c[0], c[1]); u[3] = unit53(c[2], c[3]); }
    else u[4] = unit53(c[0], c[1]);
  }
}

// In-place inverse of the n x n row-major matrix a (leading dimension lda) by
// Gauss-Jordan elimination with partial pivoting; false if singular.
bool invert_gj(double *a, int n, int lda) {
  std::vector<int> piv(n);
  std::vector<double> prow(n);
  for (int col = 0; col < n; ++col) {
    int p = col;
    double best = fabs(a[static_cast<size_t>(col) * lda + col]);
    for (int r = col + 1; r < n; ++r) {
      const double v = fabs(a[static_cast<size_t>(r) * lda + col]);
      if (v > best) { best = v; p = r; }
    }
    if (!(best > 0.0) || !isfinite(best)) return false;
    piv[col] = p;
    if (p != col)
      for (int j = 0; j < n; ++j) std::swap(a[static_cast<size_t>(p) * lda + j], a[static_cast<size_t>(col) * lda + j]);
    double *rc = a + static_cast<size_t>(col) * lda;
    const double ip = 1.0 / rc[col];
    rc[col] = 1.0;
    for (int j = 0; j < n; ++j) rc[j] *= ip;
    for (int j = 0; j < n; ++j) prow[j] = rc[j];
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double *rr = a + static_cast<size_t>(r) * lda;
      const double f = rr[col];
      if (f == 0.0) continue;
      rr[col] = 0.0;
      for (int j = 0; j < n; ++j) rr[j] -= f * prow[j];
    }
  }
  for (int col = n - 1; col >= 0; --col)
    if (piv[col] != col)
      for (int r = 0; r < n; ++r)
        std::swap(a[static_cast<size_t>(r) * lda + piv[col]], a[static_cast<size_t>(r) * lda + col]);
  return true;
}

// Doolittle LU of the k x k matrix A (leading dimension ld) without pivoting,
// the factorisation the growth builds row by row; false on a zero pivot.
bool lu_nopiv(const double *A, int k, int ld, double *L, double *U) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      L[static_cast<size_t>(i) * ld + j] = (i == j) ? 1.0 : 0.0;
      U[static_cast<size_t>(i) * ld + j] = 0.0;
    }
  for (int i = 0; i < k; ++i) {
    for (int j = i; j < k; ++j) {   // row i of U
      double s = A[static_cast<size_t>(i) * ld + j];
      for (int q = 0; q < i; ++q) s -= L[static_cast<size_t>(i) * ld + q] * U[static_cast<size_t>(q) * ld + j];
      U[static_cast<size_t>(i) * ld + j] = s;
    }
    const double piv = U[static_cast<size_t>(i) * ld + i];
    if (!(piv != 0.0) || !std::isfinite(piv)) return false;
    for (int r = i + 1; r < k; ++r) {   // column i of L
      double s = A[static_cast<size_t>(r) * ld + i];
      for (int q = 0; q < i; ++q) s -= L[static_cast<size_t>(r) * ld + q] * U[static_cast<size_t>(q) * ld + i];
      L[static_cast<size_t>(r) * ld + i] = s / piv;
    }
  }
  return true;
}

}  // namespace

struct ctaux_cpu_chain {
  // model
  double beta, U, K, gamma, inv_h, p_flip;
  int nc, n_tau, n_disp;
  std::vector<int32_t> site_disp;
  std::vector<double> g0[2];
  double ev[2][5];   // exp(gamma sigma d), d = -2..2
  // options
  int kmax, meas_every, n_out, n_cap, ldn;   // ldn: leading dimension of N
  int64_t n_therm, log_cap;
  uint64_t seed;
  uint32_t chain_id;
  // state
  int n = 0, par = 0;
  int64_t done = 0, target = 0, next_id = 0, accepted = 0, blocks = 0;
  double sign = 1.0;
  std::vector<int64_t> id;
  std::vector<double> tau;
  std::vector<int32_t> site, spin;
  std::vector<double> N[2][2];   // [parity][sector], n_cap rows of ldn
  // block buffers
  std::vector<double> X[2], Z[2], Rt[2], Y[2], Gnn[2];   // X, Rt: ki x n0; Z, Y: n0 x kp; Gnn: ki x kp
  std::vector<double> Xi[2];     // Gamma~^{-1} (kmax x kmax, leading dimension kmax)
  // LU growth (Sec. III B 1): Gamma~ = L U, L unit lower, U upper (kmax x kmax)
  int growth = 0;                // 0: inversion by partitioning, 1: LU growth
  std::vector<double> Lm[2], Um[2];
  std::vector<double> obs;
  std::vector<uint8_t> log_acc;
  std::vector<double> log_R;
  std::string err;

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }

  // G0 of the pair (x, y) at time difference dt in (-beta, beta): linear
  // interpolation on the uniform grid, antiperiodic continuation, 0+ at dt = 0.
  double g0v(int sec, int x, int y, double dt) const {
    const double *t = g0[sec].data() + static_cast<size_t>(site_disp[x * nc + y]) * n_tau;
    double sg = 1.0;
    if (dt < 0.0) { dt += beta; sg = -1.0; }
    const double xx = dt * inv_h;
    int m = static_cast<int>(floor(xx));
    m = m < 0 ? 0 : (m > n_tau - 2 ? n_tau - 2 : m);
    const double w = xx - m;
    return sg * ((1.0 - w) * t[m] + w * t[m + 1]);
  }
  double e(int sec, int d) const { return ev[sec][d + 2]; }
  double *Nrow(int p, int sec, int i) { return N[p][sec].data() + static_cast<size_t>(i) * ldn; }

  int block(int64_t L);
  void measure();
};

int ctaux_cpu_chain::block(int64_t L) {
  const int n0 = n;
  // ---- proposals of the block and its insertion candidates (Sec. IV A) ----
  std::vector<int> type(L), pspin(L);
  std::vector<double> uacc(L), upick(L), ctau;
  std::vector<int> csite;
  for (int64_t t = 0; t < L; ++t) {
    double u[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    uniforms(seed, chain_id, static_cast<uint64_t>(done + t), u);
    const double pins = 0.5 * (1.0 - p_flip);
    type[t] = u[0] < pins ? 0 : (u[0] < 2.0 * pins ? 1 : 2);
    uacc[t] = u[1];
    upick[t] = u[3];
    pspin[t] = u[4] < 0.5 ? -1 : 1;
    if (type[t] == 0) {
      ctau.push_back(beta * u[2]);
      int x = static_cast<int>(floor(nc * u[3]));
      csite.push_back(x > nc - 1 ? nc - 1 : x);
    }
  }
  const int ki = static_cast<int>(ctau.size()), na = n0 + ki;
  const int kp = (ki + kNr - 1) / kNr * kNr;   // candidate columns padded to whole register tiles
  // ---- preparation products, per sector ----
  for (int sec = 0; sec < 2; ++sec) {
    X[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    Z[sec].assign(static_cast<size_t>(n0) * kp, 0.0);
    Rt[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    Y[sec].assign(static_cast<size_t>(n0) * kp, 0.0);
    Gnn[sec].assign(static_cast<size_t>(ki) * kp, 0.0);
    for (int i = 0; i < n0; ++i) {
      const double f = e(sec, spin[i]) - 1.0;
      for (int j = 0; j < ki; ++j) {
        X[sec][static_cast<size_t>(j) * n0 + i] = g0v(sec, csite[j], site[i], ctau[j] - tau[i]) * f;
        Z[sec][static_cast<size_t>(i) * kp + j] = g0v(sec, site[i], csite[j], tau[i] - ctau[j]);
      }
    }
    if (n0 > 0 && ki > 0) {
      prep_products(n0, ki, kp, Nrow(par, sec, 0), ldn, X[sec].data(), Z[sec].data(), Y[sec].data(), Rt[sec].data());
      gemm(ki, kp, n0, X[sec].data(), n0, Y[sec].data(), kp, Gnn[sec].data(), kp, 1.0);   // X Y
    }
    for (int j = 0; j < ki; ++j)
      for (int jj = 0; jj < ki; ++jj)
        Gnn[sec][static_cast<size_t>(j) * kp + jj] += g0v(sec, csite[j], csite[jj], ctau[j] - ctau[jj]);
  }
  // entries of the augmented N_a and of G for candidate columns
  auto na_at = [&](int sec, int i, int j) -> double {   // j < n0
    return i < n0 ? N[par][sec][static_cast<size_t>(i) * ldn + j] : Rt[sec][static_cast<size_t>(i - n0) * n0 + j];
  };
  auto g_cand = [&](int sec, int i, int j) -> double {   // j >= n0
    return i < n0 ? Y[sec][static_cast<size_t>(i) * kp + (j - n0)] : Gnn[sec][static_cast<size_t>(i - n0) * kp + (j - n0)];
  };
  // (Gamma~ entry before the diagonal term): (N_a - I) for an old column, (G - I) for a candidate
  auto gt = [&](int sec, int i, int j) -> double {
    return (j < n0 ? na_at(sec, i, j) : g_cand(sec, i, j)) - (i == j ? 1.0 : 0.0);
  };
  auto dscale = [&](int sec, int s0) -> double { return s0 == 0 ? 1.0 : e(sec, s0) / (e(sec, s0) - 1.0); };
  // ---- the proposal loop (Sec. IV B) ----
  std::vector<int> scur(na, 0), s0(na, 0), slot(na, -1), P;
  for (int i = 0; i < n0; ++i) scur[i] = s0[i] = spin[i];
  std::vector<double> gh[2];
  const bool lu = growth == 1;
  for (int sec = 0; sec < 2; ++sec) {
    Xi[sec].assign(static_cast<size_t>(kmax) * kmax, 0.0);
    if (lu) {
      Lm[sec].assign(static_cast<size_t>(kmax) * kmax, 0.0);
      Um[sec].assign(static_cast<size_t>(kmax) * kmax, 0.0);
    }
  }
  std::vector<double> sv(kmax), wv(kmax), v(kmax), u(kmax), ly[2], ux[2];
  ly[0].assign(kmax, 0.0); ly[1].assign(kmax, 0.0); ux[0].assign(kmax, 0.0); ux[1].assign(kmax, 0.0);
  // (Gamma~^{-1})_aa from the factors: L c = e_a, U z = c
  auto lu_inv_diag = [&](int sec, int a, int k) {
    const double *Lp = Lm[sec].data(), *Up = Um[sec].data();
    std::vector<double> cz(k, 0.0);
    for (int i = a; i < k; ++i) {
      double c = (i == a) ? 1.0 : 0.0;
      for (int j = a; j < i; ++j) c -= Lp[static_cast<size_t>(i) * kmax + j] * cz[j];
      cz[i] = c;
    }
    for (int i = k - 1; i >= a; --i) {
      double z = cz[i];
      for (int j = i + 1; j < k; ++j) z -= Up[static_cast<size_t>(i) * kmax + j] * cz[j];
      cz[i] = z / Up[static_cast<size_t>(i) * kmax + i];
    }
    return cz[a];
  };
  int ncur = n0, next_cand = 0, ka = 0;
  std::vector<int64_t> cid(ki, -1);
  int64_t L_eff = L;
  int rc = CTAUX_OK;
  const bool gz = gamma == 0.0;
  for (int64_t t = 0; t < L; ++t) {
    int p = -1, s_old = 0, s_new = 0;
    bool skip = false;
    if (type[t] == 0) {
      if (ncur + 1 > n_cap) {
        L_eff = t;
        rc = fail(CTAUX_ECAPACITY, "an insertion at proposal %lld would exceed n_cap=%d", (long long)(done + t), n_cap);
        break;
      }
      p = n0 + next_cand;
      s_new = pspin[t];
    } else if (ncur == 0) {
      skip = true;
    } else {
      int r = static_cast<int>(floor(ncur * upick[t]));
      if (r > ncur - 1) r = ncur - 1;
      for (int i = 0; i < n0 + next_cand; ++i)   // rank among interacting vertices, canonical order
        if (scur[i] != 0 && r-- == 0) { p = i; break; }
      s_old = scur[p];
      s_new = type[t] == 1 ? 0 : -s_old;
    }
    const double fpre = type[t] == 0 ? K / (ncur + 1.0) : (type[t] == 1 ? ncur / K : 1.0);
    double R = 0.0, rs[2] = {1.0, 1.0}, bt[2] = {0.0, 0.0}, ghn[2] = {0.0, 0.0}, dp[2] = {1.0, 1.0};
    const int a = skip || gz ? -1 : slot[p];
    if (!skip && !gz) {
      for (int sec = 0; sec < 2; ++sec) {
        ghn[sec] = e(sec, s_new - s0[p]) - e(sec, s_old - s0[p]);
        dp[sec] = dscale(sec, s0[p]);
        const double *xi = Xi[sec].data();
        if (a >= 0) {   // repeated change of slot a: net change from the block start
          const double go = gh[sec][a], gn = e(sec, s_new - s0[p]) - 1.0;
          const double xaa = lu ? lu_inv_diag(sec, a, ka) : xi[a * kmax + a];
          ghn[sec] = gn;
          rs[sec] = s_new == s0[p] ? xaa / (-go * dp[sec]) : (gn / go) * (1.0 + (1.0 / go - 1.0 / gn) / dp[sec] * xaa);
        } else {
          for (int b = 0; b < ka; ++b) {
            sv[b] = gt(sec, P[b], p);
            wv[b] = gt(sec, p, P[b]);
          }
          double dd = gt(sec, p, p) - 1.0 / (ghn[sec] * dp[sec]);
          if (lu) {   // L y = s, U^T x = w (Eqs. lineq1, lineq2), beta~ = d - x^T y (Eq. detrat)
            const double *Lp = Lm[sec].data(), *Up = Um[sec].data();
            double *y = ly[sec].data(), *x = ux[sec].data();
            for (int i = 0; i < ka; ++i) {
              double ys = sv[i], xs = wv[i];
              for (int j = 0; j < i; ++j) {
                ys -= Lp[static_cast<size_t>(i) * kmax + j] * y[j];
                xs -= Up[static_cast<size_t>(j) * kmax + i] * x[j];
              }
              y[i] = ys;
              x[i] = xs / Up[static_cast<size_t>(i) * kmax + i];
            }
            for (int i = 0; i < ka; ++i) dd -= x[i] * y[i];
          } else {
            for (int i = 0; i < ka; ++i) {
              double s = 0.0, s2 = 0.0;
              for (int j = 0; j < ka; ++j) {
                s += xi[i * kmax + j] * sv[j];
                s2 += wv[j] * xi[j * kmax + i];
              }
              v[i] = s;   // X s
              u[i] = s2;  // w^T X
            }
            for (int i = 0; i < ka; ++i) dd -= wv[i] * v[i];
          }
          bt[sec] = dd;
          rs[sec] = -ghn[sec] * dp[sec] * dd;   // the growth on acceptance recomputes X s and w^T X
        }
      }
    }
    if (!skip) R = fpre * rs[0] * rs[1];
    if (!isfinite(R)) {
      L_eff = t;
      rc = fail(CTAUX_ENUMERIC, "non-finite ratio at proposal %lld", (long long)(done + t));
      break;
    }
    const int acc = (!skip && uacc[t] < fabs(R)) ? 1 : 0;
    if (done + t < log_cap) {
      log_acc[done + t] = static_cast<uint8_t>(acc);
      log_R[done + t] = R;
    }
    if (acc) {
      accepted += 1;
      if (R < 0.0) sign = -sign;
      if (!gz && lu) {
        for (int sec = 0; sec < 2; ++sec) {
          if (a >= 0) {   // the net change of slot a, or its removal (re-factorised below)
            if (s_new != s0[p]) {
              gh[sec][a] = ghn[sec];
            } else {
              gh[sec][a] = gh[sec][ka - 1];
              gh[sec].pop_back();
            }
          } else {   // Gamma~ grows: L gains the row [x^T 1], U the column [y; beta~]
            double *Lp = Lm[sec].data(), *Up = Um[sec].data();
            const int k = ka;
            for (int j = 0; j < k; ++j) {
              Lp[static_cast<size_t>(k) * kmax + j] = ux[sec][j];
              Up[static_cast<size_t>(j) * kmax + k] = ly[sec][j];
            }
            Lp[static_cast<size_t>(k) * kmax + k] = 1.0;
            Up[static_cast<size_t>(k) * kmax + k] = bt[sec];
            gh[sec].push_back(ghn[sec]);
          }
        }
      }
      if (!gz && !lu) {
        for (int sec = 0; sec < 2; ++sec) {
          double *xi = Xi[sec].data();
          if (a >= 0) {
            const double xaa = xi[a * kmax + a], go = gh[sec][a];
            if (s_new != s0[p]) {   // Sherman-Morrison on the diagonal change
              const double del = (1.0 / go - 1.0 / ghn[sec]) / dp[sec], coef = del / (1.0 + del * xaa);
              for (int i = 0; i < ka; ++i) { v[i] = xi[i * kmax + a]; u[i] = xi[a * kmax + i]; }
              for (int i = 0; i < ka; ++i)
                for (int j = 0; j < ka; ++j) xi[i * kmax + j] -= coef * v[i] * u[j];
              gh[sec][a] = ghn[sec];
            } else {   // slot a leaves: Schur complement, the last slot moves into a
              const int last = ka - 1;
              for (int i = 0; i < ka; ++i) { v[i] = xi[i * kmax + a]; u[i] = xi[a * kmax + i]; }
              for (int i = 0; i < ka; ++i)
                for (int j = 0; j < ka; ++j) xi[i * kmax + j] -= v[i] * u[j] / xaa;
              for (int j = 0; j < ka; ++j) xi[a * kmax + j] = xi[last * kmax + j];
              for (int i = 0; i < ka; ++i) xi[i * kmax + a] = xi[i * kmax + last];
              for (int j = 0; j < ka; ++j) { xi[last * kmax + j] = 0.0; xi[j * kmax + last] = 0.0; }
              gh[sec][a] = gh[sec][last];
              gh[sec].pop_back();
            }
          } else {   // growth by partitioning with this sector's v = X s, u = w^T X
            const int k = ka;
            for (int b = 0; b < k; ++b) {
              sv[b] = gt(sec, P[b], p);
              wv[b] = gt(sec, p, P[b]);
            }
            for (int i = 0; i < k; ++i) {
              double s = 0.0, s2 = 0.0;
              for (int j = 0; j < k; ++j) {
                s += xi[i * kmax + j] * sv[j];
                s2 += wv[j] * xi[j * kmax + i];
              }
              v[i] = s;
              u[i] = s2;
            }
            const double ib = 1.0 / bt[sec];
            for (int i = 0; i < k; ++i)
              for (int j = 0; j < k; ++j) xi[i * kmax + j] += v[i] * u[j] * ib;
            for (int i = 0; i < k; ++i) {
              xi[i * kmax + k] = -v[i] * ib;
              xi[k * kmax + i] = -u[i] * ib;
            }
            xi[k * kmax + k] = ib;
            gh[sec].push_back(ghn[sec]);
          }
        }
      }
      if (!gz) {
        if (a >= 0) {
          if (s_new == s0[p]) {
            const int last = ka - 1;
            if (a != last) { P[a] = P[last]; slot[P[a]] = a; }
            P.pop_back();
            slot[p] = -1;
            ka -= 1;
          }
          if (lu) {   // a changed diagonal entry or a removed slot: factorise Gamma~ again
            std::vector<double> G(static_cast<size_t>(kmax) * kmax, 0.0);
            for (int sec = 0; sec < 2 && rc == CTAUX_OK; ++sec) {
              for (int i = 0; i < ka; ++i)
                for (int j = 0; j < ka; ++j)
                  G[static_cast<size_t>(i) * kmax + j] =
                      gt(sec, P[i], P[j]) - (i == j ? 1.0 / (gh[sec][j] * dscale(sec, s0[P[j]])) : 0.0);
              if (!lu_nopiv(G.data(), ka, kmax, Lm[sec].data(), Um[sec].data()))
                rc = fail(CTAUX_ENUMERIC, "zero pivot re-factorising Gamma at proposal %lld", (long long)(done + t));
            }
            if (rc != CTAUX_OK) {
              L_eff = t;
              break;
            }
          }
        } else {
          P.push_back(p);
          slot[p] = ka;
          ka += 1;
        }
      }
      scur[p] = s_new;
      if (type[t] == 0) {
        cid[next_cand] = next_id++;
        ncur += 1;
      } else if (type[t] == 1) {
        ncur -= 1;
      }
    }
    if (type[t] == 0) next_cand += 1;
  }
  // ---- the update of N with compaction (Sec. IV C) ----
  std::vector<int> map;
  for (int i = 0; i < na; ++i)
    if (scur[i] != 0) map.push_back(i);
  const int np = static_cast<int>(map.size());
  for (int sec = 0; sec < 2; ++sec) {
    // Gamma~^{-1} for the update from the final Gamma~ by pivoted elimination
    std::vector<double> Gi(static_cast<size_t>(ka) * (ka > 0 ? ka : 1));
    for (int i = 0; i < ka; ++i)
      for (int j = 0; j < ka; ++j)
        Gi[static_cast<size_t>(i) * ka + j] =
            gt(sec, P[i], P[j]) - (i == j ? 1.0 / (gh[sec][j] * dscale(sec, s0[P[j]])) : 0.0);
    if (ka > 0 && !invert_gj(Gi.data(), ka, ka)) {
      rc = fail(CTAUX_ENUMERIC, "singular Gamma at the end of a block");
      break;
    }
    // Bc = Gamma~^{-1} N_a(P, map), Ac = ((G - I) D^{-1})(map, P)
    const int ldbc = pad_ld(np);
    std::vector<double> Bc(static_cast<size_t>(ka) * ldbc, 0.0), Ac(static_cast<size_t>(np) * (ka > 0 ? ka : 1));
    for (int b = 0; b < ka; ++b) {
      const int pb = P[b];
      std::vector<double> row(np);
      for (int j = 0; j < np; ++j) {
        const int mj = map[j];
        row[j] = mj < n0 ? na_at(sec, pb, mj) : (pb == mj ? 1.0 : 0.0);
      }
      for (int a2 = 0; a2 < ka; ++a2) {
        const double g = Gi[static_cast<size_t>(a2) * ka + b];
        double *bc = Bc.data() + static_cast<size_t>(a2) * ldbc;
        for (int j = 0; j < np; ++j) bc[j] += g * row[j];
      }
    }
    for (int i = 0; i < np; ++i)
      for (int b = 0; b < ka; ++b) Ac[static_cast<size_t>(i) * ka + b] = gt(sec, map[i], P[b]);
    // N' = N_a(map, map) - Ac Bc, a strip of rows at a time: the rows are
    // gathered and then updated while they are still in cache (Bc in L2)
    constexpr int kStrip = 12 * kMr;
    for (int i0 = 0; i0 < np; i0 += kStrip) {
      const int ie = std::min(np, i0 + kStrip);
      for (int i = i0; i < ie; ++i) {
        const int mi = map[i];
        double *out = Nrow(par ^ 1, sec, i);
        if (mi < n0) {   // old row: runs of consecutive surviving columns, zeros under candidates
          const double *src = Nrow(par, sec, mi);
          int j = 0;
          while (j < np && map[j] < n0) {
            int e2 = j + 1;
            while (e2 < np && map[e2] == map[e2 - 1] + 1 && map[e2] < n0) ++e2;
            memcpy(out + j, src + map[j], sizeof(double) * (e2 - j));
            j = e2;
          }
          for (; j < np; ++j) out[j] = 0.0;
        } else {
          const double *src = Rt[sec].data() + static_cast<size_t>(mi - n0) * n0;
          for (int j = 0; j < np; ++j) {
            const int mj = map[j];
            out[j] = mj < n0 ? src[mj] : (mi == mj ? 1.0 : 0.0);
          }
        }
      }
      if (ka > 0)
        gemm(ie - i0, np, ka, Ac.data() + static_cast<size_t>(i0) * ka, ka, Bc.data(), ldbc, Nrow(par ^ 1, sec, i0), ldn,
             -1.0);
    }
  }

  if (rc == CTAUX_OK || rc == CTAUX_ECAPACITY) {
    std::vector<int64_t> nid(np);
    std::vector<double> ntau(np);
    std::vector<int32_t> nsite(np), nspin(np);
    for (int i = 0; i < np; ++i) {
      const int mi = map[i];
      nid[i] = mi < n0 ? id[mi] : cid[mi - n0];
      ntau[i] = mi < n0 ? tau[mi] : ctau[mi - n0];
      nsite[i] = mi < n0 ? site[mi] : csite[mi - n0];
      nspin[i] = scur[mi];
    }
    std::copy(nid.begin(), nid.end(), id.begin());
    std::copy(ntau.begin(), ntau.end(), tau.begin());
    std::copy(nsite.begin(), nsite.end(), site.begin());
    std::copy(nspin.begin(), nspin.end(), spin.begin());
    n = np;
    par ^= 1;
    done += L_eff;
    blocks += 1;
  }
  return rc;
}

// Measurement at the end of a block (Sec. IV D): with T = (e^V - 1) N,
// G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k).
void ctaux_cpu_chain::measure() {
  double *o = obs.data();
  const double w = sign;
  o[0] += 1.0;
  o[1] += w;
  o[2] += w * n;
  o[3] += w * static_cast<double>(n) * n;
  o[4] += n == 0 ? w : 0.0;
  std::vector<double> Wm(static_cast<size_t>(n) * nc), gr(static_cast<size_t>(n) * nc), dens(2 * nc);
  std::vector<int> cnt(n_disp, 0);
  for (int x = 0; x < nc; ++x)
    for (int y = 0; y < nc; ++y) cnt[site_disp[x * nc + y]] += 1;
  for (int sec = 0; sec < 2; ++sec) {
    for (int k = 0; k < n; ++k)
      for (int y = 0; y < nc; ++y) gr[static_cast<size_t>(k) * nc + y] = g0v(sec, site[k], y, tau[k]);
    std::fill(Wm.begin(), Wm.end(), 0.0);
    if (n > 0) gemm(n, nc, n, Nrow(par, sec, 0), ldn, gr.data(), nc, Wm.data(), nc, 1.0);   // N g
    for (int l = 0; l < n; ++l) {
      const double f = e(sec, spin[l]) - 1.0;
      for (int y = 0; y < nc; ++y) Wm[static_cast<size_t>(l) * nc + y] *= f;
    }
    // G(x t_j; y) = G0_xy(t_j) + sum_l gl_{(j,x) l} W_ly with gl tabulated once
    // per output time and site (t_0 = 0+, t_j = (j - 1/2) beta / n_out)
    std::vector<double> gl(n), gxy(nc);
    double *gs = o + 8 + static_cast<size_t>(sec) * n_disp * n_out;
    double dsum = 0.0;
    for (int j = 0; j <= n_out; ++j) {
      const double tj = j == 0 ? 0.0 : (j - 0.5) * beta / n_out;
      for (int x = 0; x < nc; ++x) {
        for (int l = 0; l < n; ++l) gl[l] = g0v(sec, x, site[l], tj - tau[l]);
        for (int y = 0; y < nc; ++y) gxy[y] = g0v(sec, x, y, tj);
        for (int l = 0; l < n; ++l) {
          const double *wl = Wm.data() + static_cast<size_t>(l) * nc;
          for (int y = 0; y < nc; ++y) gxy[y] += gl[l] * wl[y];
        }
        if (j == 0) {
          dens[sec * nc + x] = 1.0 - gxy[x];
          dsum += dens[sec * nc + x];
        } else {
          for (int y = 0; y < nc; ++y) {
            const int dd = site_disp[x * nc + y];
            gs[static_cast<size_t>(dd) * n_out + (j - 1)] += w * gxy[y] / cnt[dd];
          }
        }
      }
    }
    o[6 + sec] += w * dsum / nc;
  }
  double D = 0.0;
  for (int x = 0; x < nc; ++x) D += dens[x] * dens[nc + x];
  o[5] += w * D / nc;
}

extern "C" {

int ctaux_cpu_create(const ctaux_model *m, const ctaux_opts *o, int32_t chain_id, ctaux_cpu_chain **out) {
  if (!m || !o || !out) return CTAUX_EINVAL;
  *out = nullptr;
  if (!(m->beta > 0) || !(m->U >= 0) || !(m->K > 0) || m->n_sites < 1 || m->n_tau < 2 || m->n_disp < 1 ||
      !m->site_disp || !m->g0_up || !m->g0_dn || o->k_max < 1 || o->k_max > 128 || o->meas_every < 1 ||
      o->n_tau_out < 0 || o->n_cap < 1 || o->log_cap < 0 || !(o->p_flip >= 0.0 && o->p_flip <= 1.0) ||
      o->p_pair != 0.0)
    return CTAUX_EINVAL;
  for (int i = 0; i < m->n_sites * m->n_sites; ++i)
    if (m->site_disp[i] < 0 || m->site_disp[i] >= m->n_disp) return CTAUX_EINVAL;
  ctaux_cpu_chain *c = new ctaux_cpu_chain();
  c->beta = m->beta; c->U = m->U; c->K = m->K;
  c->nc = m->n_sites; c->n_tau = m->n_tau; c->n_disp = m->n_disp;
  c->gamma = acosh(1.0 + m->beta * m->U * m->n_sites / (2.0 * m->K));
  c->inv_h = (m->n_tau - 1) / m->beta;
  c->p_flip = o->p_flip;
  c->site_disp.assign(m->site_disp, m->site_disp + m->n_sites * m->n_sites);
  c->g0[0].assign(m->g0_up, m->g0_up + static_cast<size_t>(m->n_disp) * m->n_tau);
  c->g0[1].assign(m->g0_dn, m->g0_dn + static_cast<size_t>(m->n_disp) * m->n_tau);
  for (int sec = 0; sec < 2; ++sec)
    for (int d = -2; d <= 2; ++d) c->ev[sec][d + 2] = exp(c->gamma * (sec == 0 ? 1.0 : -1.0) * d);
  c->kmax = o->k_max; c->meas_every = o->meas_every; c->n_out = o->n_tau_out; c->n_cap = o->n_cap;
  c->ldn = pad_ld(o->n_cap);
  c->n_therm = o->n_therm; c->log_cap = o->log_cap; c->seed = o->seed; c->chain_id = static_cast<uint32_t>(chain_id);
  c->id.resize(o->n_cap); c->tau.resize(o->n_cap); c->site.resize(o->n_cap); c->spin.resize(o->n_cap);
  for (int p = 0; p < 2; ++p)
    for (int s = 0; s < 2; ++s) c->N[p][s].assign(static_cast<size_t>(o->n_cap) * c->ldn, 0.0);
  c->obs.assign(8 + 2 * static_cast<size_t>(m->n_disp) * o->n_tau_out, 0.0);
  c->log_acc.assign(static_cast<size_t>(o->log_cap), 0);
  c->log_R.assign(static_cast<size_t>(o->log_cap), 0.0);
  *out = c;
  return CTAUX_OK;
}

int ctaux_cpu_run(ctaux_cpu_chain *c, int64_t n_proposals) {
  if (!c || n_proposals < 0) return CTAUX_EINVAL;
  c->target = c->done + n_proposals;
  while (c->done < c->target) {
    // the block ends at the next measurement point past n_therm
    int64_t L = c->target - c->done < c->kmax ? c->target - c->done : c->kmax;
    int64_t mpt = (c->done / c->meas_every + 1) * c->meas_every;
    if (mpt <= c->n_therm) mpt = (c->n_therm / c->meas_every + 1) * c->meas_every;
    if (mpt - c->done < L) L = mpt - c->done;
    const int rc = c->block(L);
    if (rc) return rc;
    if (c->done % c->meas_every == 0 && c->done > c->n_therm) c->measure();
  }
  return CTAUX_OK;
}

int ctaux_cpu_get_state(const ctaux_cpu_chain *c, int64_t *proposals, int64_t *accepted, int64_t *blocks,
                        int32_t *order, double *sign) {
  if (!c) return CTAUX_EINVAL;
  if (proposals) *proposals = c->done;
  if (accepted) *accepted = c->accepted;
  if (blocks) *blocks = c->blocks;
  if (order) *order = c->n;
  if (sign) *sign = c->sign;
  return CTAUX_OK;
}

int ctaux_cpu_get_config(const ctaux_cpu_chain *c, int32_t cap, ctaux_vertex *out, int32_t *n_out) {
  if (!c || cap < 0 || (cap > 0 && !out)) return CTAUX_EINVAL;
  if (n_out) *n_out = c->n;
  for (int i = 0; i < c->n && i < cap; ++i) out[i] = ctaux_vertex{c->id[i], c->tau[i], c->site[i], c->spin[i]};
  return CTAUX_OK;
}

int ctaux_cpu_get_N(const ctaux_cpu_chain *c, int32_t sector, double *out, int32_t ld) {
  if (!c || sector < 0 || sector > 1 || !out || ld < c->n) return CTAUX_EINVAL;
  for (int i = 0; i < c->n; ++i)
    memcpy(out + static_cast<size_t>(i) * ld, c->N[c->par][sector].data() + static_cast<size_t>(i) * c->ldn,
           sizeof(double) * c->n);
  return CTAUX_OK;
}

int ctaux_cpu_get_decisions(const ctaux_cpu_chain *c, int64_t first, int64_t count, uint8_t *acc, double *R) {
  if (!c || first < 0 || count < 0 || first + count > c->log_cap || (count > 0 && (!acc || !R))) return CTAUX_EINVAL;
  memcpy(acc, c->log_acc.data() + first, static_cast<size_t>(count));
  memcpy(R, c->log_R.data() + first, sizeof(double) * count);
  return CTAUX_OK;
}

int ctaux_cpu_get_obs(const ctaux_cpu_chain *c, double *out, int32_t len) {
  if (!c || !out || len < static_cast<int32_t>(c->obs.size())) return CTAUX_EINVAL;
  memcpy(out, c->obs.data(), sizeof(double) * c->obs.size());
  return CTAUX_OK;
}

int ctaux_cpu_set_config(ctaux_cpu_chain *c, int32_t n, const ctaux_vertex *v, int64_t proposals_done,
                         int64_t next_id, double sign) {
  if (!c || n < 0 || n > c->n_cap || (n > 0 && !v) || proposals_done < 0 || (sign != 1.0 && sign != -1.0))
    return CTAUX_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(v[i].tau >= 0.0 && v[i].tau < c->beta) || v[i].site < 0 || v[i].site >= c->nc ||
        (v[i].s != 1 && v[i].s != -1) || (i > 0 && v[i].id <= v[i - 1].id))
      return c->fail(CTAUX_EINVAL, "invalid vertex %d", i);
  for (int i = 0; i < n; ++i) {
    c->id[i] = v[i].id; c->tau[i] = v[i].tau; c->site[i] = v[i].site; c->spin[i] = v[i].s;
  }
  c->n = n;
  c->par = 0;
  for (int sec = 0; sec < 2; ++sec) {
    double *a = c->N[0][sec].data();
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)   // N^{-1} of Eq. (Nmatrix)
        a[static_cast<size_t>(i) * c->ldn + j] =
            (i == j ? c->e(sec, c->spin[i]) : 0.0) -
            c->g0v(sec, c->site[i], c->site[j], c->tau[i] - c->tau[j]) * (c->e(sec, c->spin[j]) - 1.0);
    if (n > 0 && !invert_gj(a, n, c->ldn)) return c->fail(CTAUX_ENUMERIC, "singular configuration");
  }
  c->done = proposals_done;
  c->next_id = next_id;
  c->sign = sign;
  return CTAUX_OK;
}

const char *ctaux_cpu_last_error(const ctaux_cpu_chain *c) { return c ? c->err.c_str() : "null chain"; }

int ctaux_cpu_set_growth(ctaux_cpu_chain *c, int32_t mode) {
  if (!c || (mode != 0 && mode != 1)) return CTAUX_EINVAL;
  c->growth = mode;
  return CTAUX_OK;
}

void ctaux_cpu_destroy(ctaux_cpu_chain *c) { delete c; }

}  // extern "C"
