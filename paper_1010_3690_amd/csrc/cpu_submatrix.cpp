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
//    YT = (N Z)^T with Z_ij = G0(tau_i - tau_j), Gnn = X Y + G0nn (Sec. IV A);
//  * Gamma is kept column-scaled, Gamma~ = Gamma D^{-1} with D_b = e^{V_b}/(e^{V_b} - 1)
//    for an old vertex and 1 for a candidate, so its entries are those of
//    (N_a - I) (old columns) or (G - I) (candidate columns) minus 1/(gh_b D_b) on
//    the diagonal, gh_b = e^{V(s_b) - V(s0_b)} - 1 the net change of vertex b;
//  * a new change grows X = Gamma~^{-1} by partitioning (Sec. III B 2):
//    beta~ = d - w^T X s, sector ratio -gh D_p beta~ (Eq. ratS);
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

#include <string>
#include <vector>

#include "../../include/ctaux_cpu.h"

namespace {

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

}  // namespace

struct ctaux_cpu_chain {
  // model
  double beta, U, K, gamma, inv_h, p_flip;
  int nc, n_tau, n_disp;
  std::vector<int32_t> site_disp;
  std::vector<double> g0[2];
  double ev[2][5];   // exp(gamma sigma d), d = -2..2
  // options
  int kmax, meas_every, n_out, n_cap;
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
  std::vector<double> N[2][2];   // [parity][sector], n_cap x n_cap
  // block buffers
  std::vector<double> X[2], ZT[2], Rt[2], YT[2], Gnn[2];
  std::vector<double> Xi[2];     // Gamma~^{-1} (kmax x kmax, leading dimension kmax)
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
  double *Nrow(int p, int sec, int i) { return N[p][sec].data() + static_cast<size_t>(i) * n_cap; }

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
  // ---- preparation products, per sector ----
  for (int sec = 0; sec < 2; ++sec) {
    X[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    ZT[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    Rt[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    YT[sec].assign(static_cast<size_t>(ki) * n0, 0.0);
    Gnn[sec].assign(static_cast<size_t>(ki) * ki, 0.0);
    for (int j = 0; j < ki; ++j)
      for (int i = 0; i < n0; ++i) {
        X[sec][static_cast<size_t>(j) * n0 + i] = g0v(sec, csite[j], site[i], ctau[j] - tau[i]) * (e(sec, spin[i]) - 1.0);
        ZT[sec][static_cast<size_t>(j) * n0 + i] = g0v(sec, site[i], csite[j], tau[i] - ctau[j]);
      }
    // Rt = X N: four rows of N at a time are read once and used by every
    // candidate (four FMAs per load and store of a row of Rt)
    {
      int i = 0;
      for (; i + 4 <= n0; i += 4) {
        const double *n0r = Nrow(par, sec, i), *n1r = Nrow(par, sec, i + 1);
        const double *n2r = Nrow(par, sec, i + 2), *n3r = Nrow(par, sec, i + 3);
        for (int j = 0; j < ki; ++j) {
          const double *xj = X[sec].data() + static_cast<size_t>(j) * n0 + i;
          const double x0 = xj[0], x1 = xj[1], x2 = xj[2], x3 = xj[3];
          double *rt = Rt[sec].data() + static_cast<size_t>(j) * n0;
          for (int c = 0; c < n0; ++c) rt[c] += x0 * n0r[c] + x1 * n1r[c] + x2 * n2r[c] + x3 * n3r[c];
        }
      }
      for (; i < n0; ++i) {
        const double *nr = Nrow(par, sec, i);
        for (int j = 0; j < ki; ++j) {
          const double xji = X[sec][static_cast<size_t>(j) * n0 + i];
          double *rt = Rt[sec].data() + static_cast<size_t>(j) * n0;
          for (int c = 0; c < n0; ++c) rt[c] += xji * nr[c];
        }
      }
    }
    // YT = (N Z)^T: dot products of four rows of N with each candidate's Z column
    {
      int r = 0;
      for (; r + 4 <= n0; r += 4) {
        const double *n0r = Nrow(par, sec, r), *n1r = Nrow(par, sec, r + 1);
        const double *n2r = Nrow(par, sec, r + 2), *n3r = Nrow(par, sec, r + 3);
        for (int j = 0; j < ki; ++j) {
          const double *z = ZT[sec].data() + static_cast<size_t>(j) * n0;
          double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
          for (int c = 0; c < n0; ++c) {
            s0 += n0r[c] * z[c];
            s1 += n1r[c] * z[c];
            s2 += n2r[c] * z[c];
            s3 += n3r[c] * z[c];
          }
          double *yt = YT[sec].data() + static_cast<size_t>(j) * n0 + r;
          yt[0] = s0; yt[1] = s1; yt[2] = s2; yt[3] = s3;
        }
      }
      for (; r < n0; ++r) {
        const double *nr = Nrow(par, sec, r);
        for (int j = 0; j < ki; ++j) {
          const double *z = ZT[sec].data() + static_cast<size_t>(j) * n0;
          double s = 0.0;
          for (int c = 0; c < n0; ++c) s += nr[c] * z[c];
          YT[sec][static_cast<size_t>(j) * n0 + r] = s;
        }
      }
    }
    for (int j = 0; j < ki; ++j)
      for (int jj = 0; jj < ki; ++jj) {
        const double *x = X[sec].data() + static_cast<size_t>(j) * n0;
        const double *y = YT[sec].data() + static_cast<size_t>(jj) * n0;
        double s = 0.0;
        for (int i = 0; i < n0; ++i) s += x[i] * y[i];
        Gnn[sec][static_cast<size_t>(j) * ki + jj] = s + g0v(sec, csite[j], csite[jj], ctau[j] - ctau[jj]);
      }
  }
  // entries of the augmented N_a and of G for candidate columns
  auto na_at = [&](int sec, int i, int j) -> double {   // j < n0
    return i < n0 ? N[par][sec][static_cast<size_t>(i) * n_cap + j] : Rt[sec][static_cast<size_t>(i - n0) * n0 + j];
  };
  auto g_cand = [&](int sec, int i, int j) -> double {   // j >= n0
    return i < n0 ? YT[sec][static_cast<size_t>(j - n0) * n0 + i] : Gnn[sec][static_cast<size_t>(i - n0) * ki + (j - n0)];
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
  for (int sec = 0; sec < 2; ++sec) Xi[sec].assign(static_cast<size_t>(kmax) * kmax, 0.0);
  std::vector<double> sv(kmax), wv(kmax), v(kmax), u(kmax);
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
          const double go = gh[sec][a], gn = e(sec, s_new - s0[p]) - 1.0, xaa = xi[a * kmax + a];
          ghn[sec] = gn;
          rs[sec] = s_new == s0[p] ? xaa / (-go * dp[sec]) : (gn / go) * (1.0 + (1.0 / go - 1.0 / gn) / dp[sec] * xaa);
        } else {
          for (int b = 0; b < ka; ++b) {
            sv[b] = gt(sec, P[b], p);
            wv[b] = gt(sec, p, P[b]);
          }
          double dd = gt(sec, p, p) - 1.0 / (ghn[sec] * dp[sec]);
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
      if (!gz) {
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
        if (a >= 0) {
          if (s_new == s0[p]) {
            const int last = ka - 1;
            if (a != last) { P[a] = P[last]; slot[P[a]] = a; }
            P.pop_back();
            slot[p] = -1;
            ka -= 1;
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
    std::vector<double> Bc(static_cast<size_t>(ka) * np, 0.0), Ac(static_cast<size_t>(np) * (ka > 0 ? ka : 1));
    for (int b = 0; b < ka; ++b) {
      const int pb = P[b];
      std::vector<double> row(np);
      for (int j = 0; j < np; ++j) {
        const int mj = map[j];
        row[j] = mj < n0 ? na_at(sec, pb, mj) : (pb == mj ? 1.0 : 0.0);
      }
      for (int a2 = 0; a2 < ka; ++a2) {
        const double g = Gi[static_cast<size_t>(a2) * ka + b];
        double *bc = Bc.data() + static_cast<size_t>(a2) * np;
        for (int j = 0; j < np; ++j) bc[j] += g * row[j];
      }
    }
    for (int i = 0; i < np; ++i)
      for (int b = 0; b < ka; ++b) Ac[static_cast<size_t>(i) * ka + b] = gt(sec, map[i], P[b]);
    // N'[i][:] = N_a(map i, map) - Ac[i][:] Bc, row by row (Bc stays in cache)
    for (int i = 0; i < np; ++i) {
      const int mi = map[i];
      double *out = Nrow(par ^ 1, sec, i);
      for (int j = 0; j < np; ++j) {
        const int mj = map[j];
        out[j] = mj < n0 ? (mi < n0 ? N[par][sec][static_cast<size_t>(mi) * n_cap + mj] : Rt[sec][static_cast<size_t>(mi - n0) * n0 + mj])
                         : (mi == mj ? 1.0 : 0.0);
      }
      const double *ai = Ac.data() + static_cast<size_t>(i) * ka;
      int b = 0;
      for (; b + 4 <= ka; b += 4) {   // four rows of Bc per pass over the output row
        const double a0 = ai[b], a1 = ai[b + 1], a2 = ai[b + 2], a3 = ai[b + 3];
        const double *b0 = Bc.data() + static_cast<size_t>(b) * np, *b1 = b0 + np, *b2 = b1 + np, *b3 = b2 + np;
        for (int j = 0; j < np; ++j) out[j] -= a0 * b0[j] + a1 * b1[j] + a2 * b2[j] + a3 * b3[j];
      }
      for (; b < ka; ++b) {
        const double ac = ai[b];
        const double *bc = Bc.data() + static_cast<size_t>(b) * np;
        for (int j = 0; j < np; ++j) out[j] -= ac * bc[j];
      }
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
    for (int l = 0; l < n; ++l) {
      const double *nr = Nrow(par, sec, l);
      const double f = e(sec, spin[l]) - 1.0;
      for (int y = 0; y < nc; ++y) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += nr[k] * gr[static_cast<size_t>(k) * nc + y];
        Wm[static_cast<size_t>(l) * nc + y] = f * s;
      }
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
      o->n_tau_out < 0 || o->n_cap < 1 || o->log_cap < 0 || !(o->p_flip >= 0.0 && o->p_flip <= 1.0))
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
  c->n_therm = o->n_therm; c->log_cap = o->log_cap; c->seed = o->seed; c->chain_id = static_cast<uint32_t>(chain_id);
  c->id.resize(o->n_cap); c->tau.resize(o->n_cap); c->site.resize(o->n_cap); c->spin.resize(o->n_cap);
  for (int p = 0; p < 2; ++p)
    for (int s = 0; s < 2; ++s) c->N[p][s].assign(static_cast<size_t>(o->n_cap) * o->n_cap, 0.0);
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
    memcpy(out + static_cast<size_t>(i) * ld, c->N[c->par][sector].data() + static_cast<size_t>(i) * c->n_cap,
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
        a[static_cast<size_t>(i) * c->n_cap + j] =
            (i == j ? c->e(sec, c->spin[i]) : 0.0) -
            c->g0v(sec, c->site[i], c->site[j], c->tau[i] - c->tau[j]) * (c->e(sec, c->spin[j]) - 1.0);
    if (n > 0 && !invert_gj(a, n, c->n_cap)) return c->fail(CTAUX_ENUMERIC, "singular configuration");
  }
  c->done = proposals_done;
  c->next_id = next_id;
  c->sign = sign;
  return CTAUX_OK;
}

const char *ctaux_cpu_last_error(const ctaux_cpu_chain *c) { return c ? c->err.c_str() : "null chain"; }

void ctaux_cpu_destroy(ctaux_cpu_chain *c) { delete c; }

}  // extern "C"
