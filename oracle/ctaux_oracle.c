/*
 * CT-AUX oracle (TEST INFRASTRUCTURE ONLY): plain FP64 CPU walk with rank-1
 * updates.  Each function names the passage of Gull et al. (arXiv:1010.3690)
 * it follows.  Nothing here is blocked, fused or reordered beyond what those
 * definitions state; the code is meant to be checked against the paper by eye.
 */
#include "ctaux_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct oc_chain {
    /* model (Sec. II A) */
    double beta, U, K, gamma;
    int32_t nc, n_tau, n_disp;
    int32_t *site_disp;      /* [nc*nc] */
    double *g0[2];           /* [n_disp*n_tau] per sector */
    double inv_h;            /* (n_tau-1)/beta */
    double ev[2][3];         /* exp(gamma*sigma*s), sector x (s+1) */
    /* walk parameters */
    uint64_t seed;
    uint32_t chain_id;
    double p_flip, p_pair;
    int32_t meas_every, n_out, n_cap;
    int64_t n_therm;
    /* state */
    int32_t n;               /* current order */
    int64_t done;            /* proposals processed */
    int64_t next_id;
    double sign;
    int64_t *id;
    double *tau;
    int32_t *site, *s;
    double *N[2];            /* row-major, ld = n_cap */
    double *v1, *v2, *v3;    /* work vectors [n_cap+1] */
    /* decision log */
    int64_t log_cap;
    uint8_t *log_acc;
    double *log_R;
    /* last proposal */
    int32_t last_type, last_p, last_site, last_s, last_acc;
    double last_tau, last_R;
    int32_t last_p2, last_site2, last_s2;   /* second vertex of a pair proposal */
    double last_tau2;
    /* observables */
    double *obs;
    int32_t obs_len;
    /* momentum / Matsubara measurement */
    int32_t n_k, n_mats;
    double *kvecs, *site_pos;   /* [n_k*3], [nc*3] */
    double *obs_kw;             /* [2][n_k][n_mats][2] */
    char err[256];
};

static int fail(oc_chain *c, int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof c->err, fmt, ap);
    va_end(ap);
    return code;
}

const char *oc_error(const oc_chain *c) { return c ? c->err : "null chain"; }

/* ---------------- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) -------- */
void oc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u53(uint32_t hi, uint32_t lo) {
    uint64_t x = ((uint64_t)hi << 32) | lo;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

void oc_draws(uint64_t seed, uint32_t chain_id, uint64_t index, double out[5]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    for (uint32_t tag = 0; tag < 3; ++tag) {
        uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), chain_id, tag};
        oc_philox4x32_10(ctr, key, x);
        if (tag == 0) { out[0] = u53(x[0], x[1]); out[1] = u53(x[2], x[3]); }
        if (tag == 1) { out[2] = u53(x[0], x[1]); out[3] = u53(x[2], x[3]); }
        if (tag == 2) { out[4] = u53(x[0], x[1]); }
    }
}

/* Extra uniforms of a pair proposal: the second word pair of tag 2 (spin of
 * the second vertex) and tag 3 (its time and its pick). */
void oc_pair_draws(uint64_t seed, uint32_t chain_id, uint64_t index, double out[3]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    uint32_t c2[4] = {(uint32_t)index, (uint32_t)(index >> 32), chain_id, 2};
    oc_philox4x32_10(c2, key, x);
    out[0] = u53(x[2], x[3]);
    uint32_t c3[4] = {(uint32_t)index, (uint32_t)(index >> 32), chain_id, 3};
    oc_philox4x32_10(c3, key, x);
    out[1] = u53(x[0], x[1]);
    out[2] = u53(x[2], x[3]);
}

/* Eq. (gamma) with the cluster factor: cosh(gamma) = 1 + beta*U*Nc/(2K). */
double oc_gamma_of(double beta, double U, double K, int32_t n_sites) {
    return acosh(1.0 + beta * U * (double)n_sites / (2.0 * K));
}

/* ---------------- G0 lookup: linear interpolation, antiperiodic ----------- */
/* Table entry m holds G0(m*beta/(n_tau-1)); entry 0 is the 0+ limit.  For
 * dtau < 0 the value is -G0(dtau + beta) (fermionic antiperiodicity). */
double oc_g0_lookup(const oc_chain *c, int32_t sector, int32_t x, int32_t y, double dtau) {
    const double *tab = c->g0[sector] + (int64_t)c->site_disp[x * c->nc + y] * c->n_tau;
    double sgn = 1.0;
    if (dtau < 0.0) { dtau += c->beta; sgn = -1.0; }
    double xx = dtau * c->inv_h;
    int32_t m = (int32_t)floor(xx);
    if (m > c->n_tau - 2) m = c->n_tau - 2;
    if (m < 0) m = 0;
    double w = xx - (double)m;
    return sgn * ((1.0 - w) * tab[m] + w * tab[m + 1]);
}

static double g0v(const oc_chain *c, int sector, int i, int j) {
    /* (G0)_ij = G0_{x_i x_j}(tau_i - tau_j) of Eq. (Nmatrix); i == j gives 0+. */
    return oc_g0_lookup(c, sector, c->site[i], c->site[j], c->tau[i] - c->tau[j]);
}

static double expV(const oc_chain *c, int sector, int32_t s) { return c->ev[sector][s + 1]; }

/* ---------------- construction -------------------------------------------- */
oc_chain *oc_create(double beta, double U, double K, int32_t n_sites, int32_t n_tau,
                    int32_t n_disp, const int32_t *site_disp, const double *g0_up,
                    const double *g0_dn, uint64_t seed, uint32_t chain_id, double p_flip,
                    int32_t meas_every, int64_t n_therm, int32_t n_tau_out, int32_t n_cap) {
    if (!(beta > 0) || !(U >= 0) || !(K > 0) || n_sites < 1 || n_tau < 2 || n_disp < 1 ||
        !site_disp || !g0_up || !g0_dn || !(p_flip >= 0 && p_flip <= 1) || meas_every < 1 ||
        n_tau_out < 1 || n_cap < 1)
        return NULL;
    for (int i = 0; i < n_sites * n_sites; ++i)
        if (site_disp[i] < 0 || site_disp[i] >= n_disp) return NULL;
    for (int64_t i = 0; i < (int64_t)n_disp * n_tau; ++i)
        if (!isfinite(g0_up[i]) || !isfinite(g0_dn[i])) return NULL;
    oc_chain *c = (oc_chain *)calloc(1, sizeof *c);
    if (!c) return NULL;
    c->beta = beta; c->U = U; c->K = K;
    c->nc = n_sites; c->n_tau = n_tau; c->n_disp = n_disp;
    c->gamma = oc_gamma_of(beta, U, K, n_sites);
    c->inv_h = (double)(n_tau - 1) / beta;
    for (int sec = 0; sec < 2; ++sec) {
        double sigma = sec == 0 ? 1.0 : -1.0;
        for (int s = -1; s <= 1; ++s) c->ev[sec][s + 1] = exp(c->gamma * sigma * (double)s);
    }
    c->seed = seed; c->chain_id = chain_id; c->p_flip = p_flip;
    c->meas_every = meas_every; c->n_therm = n_therm; c->n_out = n_tau_out; c->n_cap = n_cap;
    c->sign = 1.0;
    size_t nn = (size_t)n_cap * n_cap;
    c->site_disp = (int32_t *)malloc(sizeof(int32_t) * n_sites * n_sites);
    c->g0[0] = (double *)malloc(sizeof(double) * n_disp * n_tau);
    c->g0[1] = (double *)malloc(sizeof(double) * n_disp * n_tau);
    c->id = (int64_t *)malloc(sizeof(int64_t) * (n_cap + 1));
    c->tau = (double *)malloc(sizeof(double) * (n_cap + 1));
    c->site = (int32_t *)malloc(sizeof(int32_t) * (n_cap + 1));
    c->s = (int32_t *)malloc(sizeof(int32_t) * (n_cap + 1));
    c->N[0] = (double *)malloc(sizeof(double) * nn);
    c->N[1] = (double *)malloc(sizeof(double) * nn);
    c->v1 = (double *)malloc(sizeof(double) * (n_cap + 1));
    c->v2 = (double *)malloc(sizeof(double) * (n_cap + 1));
    c->v3 = (double *)malloc(sizeof(double) * (n_cap + 1));
    c->obs_len = OC_OBS_HEADER + 2 * n_disp * n_tau_out;
    c->obs = (double *)calloc((size_t)c->obs_len, sizeof(double));
    if (!c->site_disp || !c->g0[0] || !c->g0[1] || !c->id || !c->tau || !c->site || !c->s ||
        !c->N[0] || !c->N[1] || !c->v1 || !c->v2 || !c->v3 || !c->obs) {
        oc_destroy(c);
        return NULL;
    }
    memcpy(c->site_disp, site_disp, sizeof(int32_t) * n_sites * n_sites);
    memcpy(c->g0[0], g0_up, sizeof(double) * n_disp * n_tau);
    memcpy(c->g0[1], g0_dn, sizeof(double) * n_disp * n_tau);
    c->last_type = -1;
    return c;
}

void oc_destroy(oc_chain *c) {
    if (!c) return;
    free(c->site_disp); free(c->g0[0]); free(c->g0[1]);
    free(c->id); free(c->tau); free(c->site); free(c->s);
    free(c->N[0]); free(c->N[1]);
    free(c->v1); free(c->v2); free(c->v3);
    free(c->log_acc); free(c->log_R); free(c->obs);
    free(c->kvecs); free(c->site_pos); free(c->obs_kw);
    free(c);
}

#define NE(c, sec, i, j) ((c)->N[sec][(size_t)(i) * (c)->n_cap + (j)])

/* ---------------- rank-1 kernels ------------------------------------------ */
/* Insertion of vertex (tau, x, s) at position n by bordering.  The new row and
 * column of N^{-1} follow from Eq. (Nmatrix):
 *   column: c_i = -G0(tau_i - tau)(e^{V(s)} - 1),   row: r_j = -G0(tau - tau_j)(e^{V_j} - 1),
 *   corner: m = e^{V(s)} - G0(0+)(e^{V(s)} - 1).
 * The determinant ratio det N'^{-1}/det N^{-1} is the Schur complement
 * S = m - r N c (needed in Eq. insprob). */
static double insert_ratio(oc_chain *c, int sec, double tau, int32_t x, int32_t s) {
    int n = c->n;
    double evs = expV(c, sec, s);
    double *cc = c->v1, *nc_ = c->v2;
    for (int i = 0; i < n; ++i)
        cc[i] = -oc_g0_lookup(c, sec, c->site[i], x, c->tau[i] - tau) * (evs - 1.0);
    double m = evs - oc_g0_lookup(c, sec, x, x, 0.0) * (evs - 1.0);
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += NE(c, sec, i, k) * cc[k];
        nc_[i] = acc;                                   /* N c */
    }
    double rnc = 0.0;
    for (int j = 0; j < n; ++j) {
        double r = -oc_g0_lookup(c, sec, x, c->site[j], tau - c->tau[j]) *
                   (expV(c, sec, c->s[j]) - 1.0);
        rnc += r * nc_[j];
    }
    return m - rnc;
}

static void insert_commit(oc_chain *c, int sec, double tau, int32_t x, double S) {
    /* N' = [[N + (Nc)(rN)/S, -Nc/S], [-rN/S, 1/S]]; the caller has already
     * appended the vertex at position n (so c->n is the old order here). */
    int n = c->n;
    double *nc_ = c->v2, *rn = c->v3;
    /* recompute N c (v2 was overwritten by the other sector's ratio) */
    double evs_new = expV(c, sec, c->s[n]);
    for (int i = 0; i < n; ++i)
        c->v1[i] = -oc_g0_lookup(c, sec, c->site[i], x, c->tau[i] - tau) * (evs_new - 1.0);
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += NE(c, sec, i, k) * c->v1[k];
        nc_[i] = acc;
    }
    for (int j = 0; j < n; ++j) rn[j] = 0.0;
    for (int k = 0; k < n; ++k) {
        double r = -oc_g0_lookup(c, sec, x, c->site[k], tau - c->tau[k]) *
                   (expV(c, sec, c->s[k]) - 1.0);
        for (int j = 0; j < n; ++j) rn[j] += r * NE(c, sec, k, j);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) NE(c, sec, i, j) += nc_[i] * rn[j] / S;
    for (int i = 0; i < n; ++i) NE(c, sec, i, n) = -nc_[i] / S;
    for (int j = 0; j < n; ++j) NE(c, sec, n, j) = -rn[j] / S;
    NE(c, sec, n, n) = 1.0 / S;
}

/* Removal of vertex p: det N'^{-1}/det N^{-1} = N_pp (cofactor of the minor),
 * N' = N_{-p,-p} - N_{-p,p} N_{p,-p} / N_pp, keeping the canonical order. */
static void remove_commit(oc_chain *c, int sec, int p) {
    int n = c->n;
    double npp = NE(c, sec, p, p);
    double *col = c->v1, *row = c->v2;
    for (int i = 0; i < n; ++i) { col[i] = NE(c, sec, i, p); row[i] = NE(c, sec, p, i); }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) NE(c, sec, i, j) -= col[i] * row[j] / npp;
    /* delete row and column p, shifting later entries down by one */
    for (int i = 0; i < n; ++i) {
        double *r = &NE(c, sec, i, 0);
        memmove(r + p, r + p + 1, sizeof(double) * (size_t)(n - p - 1));
    }
    for (int i = p; i < n - 1; ++i)
        memcpy(&NE(c, sec, i, 0), &NE(c, sec, i + 1, 0), sizeof(double) * (size_t)(n - 1));
}

/* Spin flip of vertex p, s -> s' (Eq. DysonG): with lambda = e^{V'_p - V_p} - 1,
 * G_{ip} = (N_ip e^{V_p} - delta_ip)/(e^{V_p} - 1) (Eq. NfromG) and
 * ratio r = 1 + (1 - G_pp) lambda, the update is
 * N' = N + (G_{:,p} - e_p) (lambda / r) N_{p,:}  (the printed relation carries
 * the 1/r normalisation implicitly). */
static double flip_ratio(const oc_chain *c, int sec, int p, int32_t s_new) {
    double evp = expV(c, sec, c->s[p]);
    double lambda = expV(c, sec, s_new) / evp - 1.0;
    if (lambda == 0.0) return 1.0;                   /* U = 0: weights do not depend on s */
    double gpp = (NE(c, sec, p, p) * evp - 1.0) / (evp - 1.0);
    return 1.0 + (1.0 - gpp) * lambda;
}

static void flip_commit(oc_chain *c, int sec, int p, int32_t s_new, double r) {
    int n = c->n;
    double evp = expV(c, sec, c->s[p]);
    double lambda = expV(c, sec, s_new) / evp - 1.0;
    if (lambda == 0.0) return;
    double *u = c->v1, *row = c->v2;
    for (int i = 0; i < n; ++i) {
        double gip = (NE(c, sec, i, p) * evp - (i == p ? 1.0 : 0.0)) / (evp - 1.0);
        u[i] = (gip - (i == p ? 1.0 : 0.0)) * (lambda / r);
        row[i] = NE(c, sec, p, i);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) NE(c, sec, i, j) += u[i] * row[j];
}

/* ---------------- pair updates (Sec. II B, Sec. IV B) ---------------------- */
/* Two vertices v_0, v_1 inserted together enlarge N^{-1} by two rows and two
 * columns.  By the block determinant formula the ratio det N''^{-1}/det N^{-1}
 * is the determinant of the 2x2 Schur complement
 *   S_ab = (N''^{-1})_{v_a v_b} - r_a N c_b,
 * with c_b, r_a the new column of v_b and the new row of v_a (as in
 * insert_ratio) and, from Eq. (Nmatrix),
 *   (N''^{-1})_{v_a v_b} = delta_ab e^{V(s_a)} - G0(tau_a - tau_b)(e^{V(s_b)} - 1)
 * (the diagonal reads G0 at 0+). */
static double pair_insert_ratio(oc_chain *c, int sec, const double tau[2], const int32_t x[2],
                                const int32_t s[2]) {
    int n = c->n;
    double *buf = (double *)malloc(sizeof(double) * 4 * (size_t)(n > 0 ? n : 1));
    double *col[2] = {buf, buf + n}, *ncol[2] = {buf + 2 * n, buf + 3 * n};
    for (int b = 0; b < 2; ++b) {
        double evb = expV(c, sec, s[b]);
        for (int i = 0; i < n; ++i)
            col[b][i] = -oc_g0_lookup(c, sec, c->site[i], x[b], c->tau[i] - tau[b]) * (evb - 1.0);
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += NE(c, sec, i, k) * col[b][k];
            ncol[b][i] = acc;
        }
    }
    double S[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double e = (a == b ? expV(c, sec, s[a]) : 0.0) -
                       oc_g0_lookup(c, sec, x[a], x[b], a == b ? 0.0 : tau[a] - tau[b]) *
                           (expV(c, sec, s[b]) - 1.0);
            double rnc = 0.0;
            for (int j = 0; j < n; ++j) {
                double r = -oc_g0_lookup(c, sec, x[a], c->site[j], tau[a] - c->tau[j]) *
                           (expV(c, sec, c->s[j]) - 1.0);
                rnc += r * ncol[b][j];
            }
            S[a][b] = e - rnc;
        }
    free(buf);
    return S[0][0] * S[1][1] - S[0][1] * S[1][0];
}

/* Appends vertex (tau, x, s) with the next id: bordering of both sectors. */
static int append_vertex(oc_chain *c, double tau, int32_t x, int32_t s) {
    int n = c->n;
    double S0 = insert_ratio(c, 0, tau, x, s), S1 = insert_ratio(c, 1, tau, x, s);
    if (!(S0 != 0.0) || !(S1 != 0.0) || !isfinite(S0) || !isfinite(S1))
        return fail(c, OC_ENUMERIC, "singular bordering in a pair insertion");
    c->tau[n] = tau; c->site[n] = x; c->s[n] = s; c->id[n] = c->next_id++;
    insert_commit(c, 0, tau, x, S0);
    insert_commit(c, 1, tau, x, S1);
    c->n = n + 1;
    return OC_OK;
}

/* Removes the vertex at position p from both sectors, keeping the canonical order. */
static void remove_vertex(oc_chain *c, int p) {
    int n = c->n;
    remove_commit(c, 0, p);
    remove_commit(c, 1, p);
    for (int i = p; i < n - 1; ++i) {
        c->tau[i] = c->tau[i + 1]; c->site[i] = c->site[i + 1];
        c->s[i] = c->s[i + 1]; c->id[i] = c->id[i + 1];
    }
    c->n = n - 1;
}

/* Removal of the vertices at positions a and b: by Jacobi's identity the
 * ratio det N''^{-1}/det N^{-1} (rows and columns a, b deleted from N^{-1}) is
 * the complementary minor det N[{a,b},{a,b}]. */
static double pair_remove_ratio(const oc_chain *c, int sec, int a, int b) {
    return NE(c, sec, a, a) * NE(c, sec, b, b) - NE(c, sec, a, b) * NE(c, sec, b, a);
}

static int32_t site_of(const oc_chain *c, double u_pick) {
    int32_t x = (int32_t)floor((double)c->nc * u_pick);
    return x > c->nc - 1 ? c->nc - 1 : x;
}

/* ---------------- measurement (Sec. IV D) ---------------------------------- */
/* With T = (e^V - 1) N, the estimator is
 *   G(x tau; y 0) = G0_xy(tau) + sum_{l,k} G0_{x x_l}(tau - tau_l) T_lk G0_{x_k y}(tau_k).
 * W[l][y] = sum_k T_lk G0_{x_k y}(tau_k) is formed first (n*n*Nc work). */
static void build_W(const oc_chain *c, int sec, double *W) {
    int n = c->n, nc = c->nc;
    double *gr = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nc);
    for (int k = 0; k < n; ++k)
        for (int y = 0; y < nc; ++y) gr[(size_t)k * nc + y] = oc_g0_lookup(c, sec, c->site[k], y, c->tau[k]);
    for (int l = 0; l < n; ++l) {
        double fl = expV(c, sec, c->s[l]) - 1.0;
        for (int y = 0; y < nc; ++y) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += NE(c, sec, l, k) * gr[(size_t)k * nc + y];
            W[(size_t)l * nc + y] = fl * acc;
        }
    }
    free(gr);
}

static double estimate_from_W(const oc_chain *c, int sec, const double *W, int x, int y, double tau) {
    double g = oc_g0_lookup(c, sec, x, y, tau);
    for (int l = 0; l < c->n; ++l)
        g += oc_g0_lookup(c, sec, x, c->site[l], tau - c->tau[l]) * W[(size_t)l * c->nc + y];
    return g;
}

int oc_estimate_G(const oc_chain *c, int32_t sector, int32_t x, int32_t y, double tau, double *out) {
    if (sector < 0 || sector > 1 || x < 0 || y < 0 || x >= c->nc || y >= c->nc || !(tau >= 0) ||
        !(tau < c->beta))
        return OC_EINVAL;
    double *W = (double *)malloc(sizeof(double) * (size_t)(c->n > 0 ? c->n : 1) * c->nc);
    build_W(c, sector, W);
    *out = estimate_from_W(c, sector, W, x, y, tau);
    free(W);
    return OC_OK;
}

/* Sec. IV D in cluster momenta and Matsubara frequencies: the estimator
 * G(x tau; y tau') = G0_xy(tau - tau') + sum_lk G0_{x x_l}(tau - tau_l) M_lk G0_{x_k y}(tau_k - tau')
 * transformed in both arguments,
 *   G(K, iw) = (1 / (beta Nc)) sum_xy int int exp(iw(tau - tau') - iK.(r_x - r_y)) G(x tau; y tau'),
 * gives G0(K, iw) + G0(K, iw)^2 S(K, w) / (beta Nc) with S as declared in the
 * header (fermionic antiperiodicity makes each factor a full-period transform).
 * S is summed here directly over all vertex pairs. */
static void measure_kw(oc_chain *c, double w) {
    int n = c->n;
    const double pi = 3.14159265358979323846;
    for (int sec = 0; sec < 2; ++sec)
        for (int q = 0; q < c->n_k; ++q) {
            const double *K = c->kvecs + 3 * q;
            for (int m = 0; m < c->n_mats; ++m) {
                double om = (2.0 * m + 1.0) * pi / c->beta;
                double sre = 0.0, sim = 0.0;
                for (int l = 0; l < n; ++l) {
                    const double *rl = c->site_pos + 3 * c->site[l];
                    double fl = expV(c, sec, c->s[l]) - 1.0;
                    double al = om * c->tau[l] - (K[0] * rl[0] + K[1] * rl[1] + K[2] * rl[2]);
                    for (int k = 0; k < n; ++k) {
                        const double *rk = c->site_pos + 3 * c->site[k];
                        double ak = -om * c->tau[k] + (K[0] * rk[0] + K[1] * rk[1] + K[2] * rk[2]);
                        double mlk = fl * NE(c, sec, l, k);
                        sre += mlk * cos(al + ak);
                        sim += mlk * sin(al + ak);
                    }
                }
                double *o = c->obs_kw + (((size_t)sec * c->n_k + q) * c->n_mats + m) * 2;
                o[0] += w * sre;
                o[1] += w * sim;
            }
        }
}

int oc_set_momentum(oc_chain *c, int32_t n_k, const double *kvecs, const double *site_pos,
                    int32_t n_matsubara) {
    if (n_k < 1 || n_matsubara < 1 || !kvecs || !site_pos) return fail(c, OC_EINVAL, "bad momentum set-up");
    free(c->kvecs); free(c->site_pos); free(c->obs_kw);
    c->kvecs = (double *)malloc(sizeof(double) * 3 * n_k);
    c->site_pos = (double *)malloc(sizeof(double) * 3 * c->nc);
    c->obs_kw = (double *)calloc((size_t)2 * n_k * n_matsubara * 2, sizeof(double));
    if (!c->kvecs || !c->site_pos || !c->obs_kw) return fail(c, OC_ENOMEM, "allocation failed");
    memcpy(c->kvecs, kvecs, sizeof(double) * 3 * n_k);
    memcpy(c->site_pos, site_pos, sizeof(double) * 3 * c->nc);
    c->n_k = n_k;
    c->n_mats = n_matsubara;
    return OC_OK;
}

int oc_get_obs_kw(const oc_chain *c, double *out) {
    if (!c->obs_kw) return OC_EINVAL;
    memcpy(out, c->obs_kw, sizeof(double) * 2 * (size_t)c->n_k * c->n_mats * 2);
    return OC_OK;
}

/* int_0^beta exp(i w s) g(s) ds for the linear interpolant g of a table: on
 * each segment [s0, s0 + h], with E = exp(i w s),
 *   int E (f0 + (f1 - f0)(s - s0)/h) ds = f0 (E1 - E0)/(i w) + (f1 - f0)/h (h E1/(i w) + (E1 - E0)/w^2). */
static void table_matsubara(const oc_chain *c, const double *tab, double om, double *re, double *im) {
    double h = c->beta / (double)(c->n_tau - 1);
    double sr = 0.0, si = 0.0;
    for (int m = 0; m + 1 < c->n_tau; ++m) {
        double s0 = m * h, s1 = (m + 1) * h;
        double e0r = cos(om * s0), e0i = sin(om * s0), e1r = cos(om * s1), e1i = sin(om * s1);
        double dr = e1r - e0r, di = e1i - e0i;
        double f0 = tab[m], sl = (tab[m + 1] - tab[m]) / h;
        /* (E1 - E0)/(i w) = (di - i dr)/w ;  h E1/(i w) = h (e1i - i e1r)/w ;  (E1 - E0)/w^2 */
        double ar = di / om, ai = -dr / om;
        double br = h * e1i / om + dr / (om * om), bi = -h * e1r / om + di / (om * om);
        sr += f0 * ar + sl * br;
        si += f0 * ai + sl * bi;
    }
    *re = sr;
    *im = si;
}

int oc_g0_matsubara(const oc_chain *c, int32_t sector, int32_t k, int32_t n, double *out) {
    if (!c->kvecs || sector < 0 || sector > 1 || k < 0 || k >= c->n_k || n < 0) return OC_EINVAL;
    const double pi = 3.14159265358979323846;
    double om = (2.0 * n + 1.0) * pi / c->beta;
    const double *K = c->kvecs + 3 * k;
    double gr = 0.0, gi = 0.0;
    for (int x = 0; x < c->nc; ++x)
        for (int y = 0; y < c->nc; ++y) {
            const double *rx = c->site_pos + 3 * x, *ry = c->site_pos + 3 * y;
            double ph = -(K[0] * (rx[0] - ry[0]) + K[1] * (rx[1] - ry[1]) + K[2] * (rx[2] - ry[2]));
            double tr, ti;
            table_matsubara(c, c->g0[sector] + (int64_t)c->site_disp[x * c->nc + y] * c->n_tau, om, &tr, &ti);
            gr += cos(ph) * tr - sin(ph) * ti;
            gi += cos(ph) * ti + sin(ph) * tr;
        }
    out[0] = gr / c->nc;
    out[1] = gi / c->nc;
    return OC_OK;
}

static void measure(oc_chain *c) {
    int n = c->n, nc = c->nc, no = c->n_out, nd = c->n_disp;
    double w = c->sign;
    double *o = c->obs;
    o[0] += 1.0;
    o[1] += w;
    o[2] += w * n;
    o[3] += w * (double)n * (double)n;
    o[4] += (n == 0) ? w : 0.0;
    double *W = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nc);
    double *dens = (double *)malloc(sizeof(double) * 2 * nc);
    int *cnt = (int *)calloc((size_t)nd, sizeof(int));
    for (int x = 0; x < nc; ++x)
        for (int y = 0; y < nc; ++y) cnt[c->site_disp[x * nc + y]]++;
    for (int sec = 0; sec < 2; ++sec) {
        build_W(c, sec, W);
        double dsum = 0.0;
        for (int x = 0; x < nc; ++x) {
            /* equal time: n_sigma(x) = 1 - G(x 0+; x 0) */
            dens[sec * nc + x] = 1.0 - estimate_from_W(c, sec, W, x, x, 0.0);
            dsum += dens[sec * nc + x];
        }
        o[6 + sec] += w * dsum / nc;
        double *gsum = o + OC_OBS_HEADER + (size_t)sec * nd * no;
        for (int j = 0; j < no; ++j) {
            double tj = ((double)j + 0.5) * c->beta / (double)no;
            for (int x = 0; x < nc; ++x)
                for (int y = 0; y < nc; ++y) {
                    int d = c->site_disp[x * nc + y];
                    gsum[(size_t)d * no + j] += w * estimate_from_W(c, sec, W, x, y, tj) / cnt[d];
                }
        }
    }
    double D = 0.0;
    for (int x = 0; x < nc; ++x) D += dens[x] * dens[nc + x];
    o[5] += w * D / nc;
    free(W); free(dens); free(cnt);
    if (c->obs_kw) measure_kw(c, w);
}

/* ---------------- the walk (Sec. II B) ------------------------------------- */
/* Proposal mix: insertion and removal with probability (1 - p_flip - p_pair)/2
 * each, insertion and removal of a pair of vertices (Sec. IV B) with p_pair/2
 * each, a spin flip with p_flip.  Acceptance ratios (Eq. insprob and its
 * detailed-balance partners), n the order before the move:
 *   insert K/(n+1), remove n/K, pair insert K^2/((n+1)(n+2)),
 *   pair remove n(n-1)/K^2, flip 1,
 * each times prod_sigma det N'^{-1}_sigma / det N^{-1}_sigma.  A pair is
 * proposed with density 2 (1/(2 beta Nc))^2 for the unordered pair and removed
 * with probability 1/C(n+2, 2), which gives the pair factors. */
static int step(oc_chain *c) {
    double u[5];
    int64_t idx = c->done;
    oc_draws(c->seed, c->chain_id, (uint64_t)idx, u);
    double u_type = u[0], u_acc = u[1], u_tau = u[2], u_pick = u[3], u_spin = u[4];
    double p_one = 0.5 * (1.0 - c->p_flip - c->p_pair);
    int type;
    if (u_type < p_one) type = 0;
    else if (u_type < 2.0 * p_one) type = 1;
    else if (u_type < 2.0 * p_one + 0.5 * c->p_pair) type = 3;
    else if (u_type < 2.0 * p_one + c->p_pair) type = 4;
    else type = 2;
    int n = c->n;
    double R = 0.0;
    int acc = 0;
    c->last_type = type; c->last_p = -1; c->last_tau = 0; c->last_site = -1; c->last_s = 0;
    c->last_p2 = -1; c->last_tau2 = 0; c->last_site2 = -1; c->last_s2 = 0;
    if (type == 0) {
        /* insertion: random time, site and auxiliary spin; R = K/(n+1) prod_sigma ratio */
        double tau = c->beta * u_tau;
        int32_t x = site_of(c, u_pick);
        int32_t s = u_spin < 0.5 ? -1 : 1;
        c->last_p = n; c->last_tau = tau; c->last_site = x; c->last_s = s;
        if (n + 1 > c->n_cap)
            return fail(c, OC_ECAPACITY, "order would exceed n_cap=%d", c->n_cap);
        double S0 = insert_ratio(c, 0, tau, x, s);
        double S1 = insert_ratio(c, 1, tau, x, s);
        R = c->K / (double)(n + 1) * S0 * S1;
        if (!isfinite(R)) return fail(c, OC_ENUMERIC, "non-finite insertion ratio at proposal %lld", (long long)idx);
        if (u_acc < fabs(R)) {
            acc = 1;
            c->tau[n] = tau; c->site[n] = x; c->s[n] = s; c->id[n] = c->next_id++;
            insert_commit(c, 0, tau, x, S0);
            insert_commit(c, 1, tau, x, S1);
            c->n = n + 1;
        }
    } else if (type == 3) {
        /* pair insertion: two independent (time, site, spin) draws */
        double v[3];
        oc_pair_draws(c->seed, c->chain_id, (uint64_t)idx, v);
        double tau[2] = {c->beta * u_tau, c->beta * v[1]};
        int32_t x[2] = {site_of(c, u_pick), site_of(c, v[2])};
        int32_t s[2] = {u_spin < 0.5 ? -1 : 1, v[0] < 0.5 ? -1 : 1};
        c->last_p = n; c->last_tau = tau[0]; c->last_site = x[0]; c->last_s = s[0];
        c->last_p2 = n + 1; c->last_tau2 = tau[1]; c->last_site2 = x[1]; c->last_s2 = s[1];
        if (n + 2 > c->n_cap)
            return fail(c, OC_ECAPACITY, "order would exceed n_cap=%d", c->n_cap);
        double S0 = pair_insert_ratio(c, 0, tau, x, s);
        double S1 = pair_insert_ratio(c, 1, tau, x, s);
        R = c->K * c->K / ((double)(n + 1) * (double)(n + 2)) * S0 * S1;
        if (!isfinite(R)) return fail(c, OC_ENUMERIC, "non-finite pair insertion ratio at proposal %lld", (long long)idx);
        if (u_acc < fabs(R)) {
            acc = 1;
            int rc = append_vertex(c, tau[0], x[0], s[0]);
            if (rc) return rc;
            rc = append_vertex(c, tau[1], x[1], s[1]);
            if (rc) return rc;
        }
    } else if (type == 4) {
        /* pair removal: an unordered pair of distinct vertices, picked by rank */
        if (n >= 2) {
            double v[3];
            oc_pair_draws(c->seed, c->chain_id, (uint64_t)idx, v);
            int32_t p1 = (int32_t)floor((double)n * u_pick);
            if (p1 > n - 1) p1 = n - 1;
            int32_t r2 = (int32_t)floor((double)(n - 1) * v[2]);
            if (r2 > n - 2) r2 = n - 2;
            int32_t p2 = r2 + (r2 >= p1 ? 1 : 0);
            c->last_p = p1; c->last_tau = c->tau[p1]; c->last_site = c->site[p1];
            c->last_p2 = p2; c->last_tau2 = c->tau[p2]; c->last_site2 = c->site[p2];
            R = (double)n * (double)(n - 1) / (c->K * c->K) * pair_remove_ratio(c, 0, p1, p2) *
                pair_remove_ratio(c, 1, p1, p2);
            if (!isfinite(R)) return fail(c, OC_ENUMERIC, "non-finite pair removal ratio at proposal %lld", (long long)idx);
            if (u_acc < fabs(R)) {
                acc = 1;
                remove_vertex(c, p1 > p2 ? p1 : p2);
                remove_vertex(c, p1 > p2 ? p2 : p1);
            }
        }
    } else if (n > 0) {
        int32_t p = (int32_t)floor((double)n * u_pick);
        if (p > n - 1) p = n - 1;
        c->last_p = p; c->last_tau = c->tau[p]; c->last_site = c->site[p];
        if (type == 1) {
            /* removal: ratio N_pp per sector, R = (n/K) prod_sigma N_pp */
            c->last_s = 0;
            R = (double)n / c->K * NE(c, 0, p, p) * NE(c, 1, p, p);
            if (!isfinite(R)) return fail(c, OC_ENUMERIC, "non-finite removal ratio at proposal %lld", (long long)idx);
            if (u_acc < fabs(R)) {
                acc = 1;
                remove_vertex(c, p);
            }
        } else {
            /* spin flip: R = prod_sigma (1 + (1 - G_pp) lambda_sigma) */
            int32_t s_new = -c->s[p];
            c->last_s = s_new;
            double r0 = flip_ratio(c, 0, p, s_new);
            double r1 = flip_ratio(c, 1, p, s_new);
            R = r0 * r1;
            if (!isfinite(R)) return fail(c, OC_ENUMERIC, "non-finite flip ratio at proposal %lld", (long long)idx);
            if (u_acc < fabs(R)) {
                acc = 1;
                flip_commit(c, 0, p, s_new, r0);
                flip_commit(c, 1, p, s_new, r1);
                c->s[p] = s_new;
            }
        }
    } else {
        R = 0.0;   /* remove or flip at order 0: rejected, still counted */
    }
    if (acc && R < 0.0) c->sign = -c->sign;
    c->last_R = R; c->last_acc = acc;
    if (idx < c->log_cap) { c->log_acc[idx] = (uint8_t)acc; c->log_R[idx] = R; }
    c->done = idx + 1;
    if (c->done % c->meas_every == 0 && c->done > c->n_therm) measure(c);
    return OC_OK;
}

int oc_run(oc_chain *c, int64_t n_proposals) {
    if (!c || n_proposals < 0) return OC_EINVAL;
    for (int64_t i = 0; i < n_proposals; ++i) {
        int rc = step(c);
        if (rc) return rc;
    }
    return OC_OK;
}

/* ---------------- accessors ----------------------------------------------- */
int oc_set_log(oc_chain *c, int64_t cap) {
    free(c->log_acc); free(c->log_R);
    c->log_acc = NULL; c->log_R = NULL; c->log_cap = 0;
    if (cap <= 0) return OC_OK;
    c->log_acc = (uint8_t *)calloc((size_t)cap, 1);
    c->log_R = (double *)calloc((size_t)cap, sizeof(double));
    if (!c->log_acc || !c->log_R) return fail(c, OC_ENOMEM, "log allocation failed");
    c->log_cap = cap;
    return OC_OK;
}

int oc_get_log(const oc_chain *c, int64_t first, int64_t count, uint8_t *acc, double *R) {
    if (first < 0 || count < 0 || first + count > c->log_cap || first + count > c->done) return OC_EINVAL;
    memcpy(acc, c->log_acc + first, (size_t)count);
    memcpy(R, c->log_R + first, sizeof(double) * (size_t)count);
    return OC_OK;
}

int32_t oc_order(const oc_chain *c) { return c->n; }
int64_t oc_proposals_done(const oc_chain *c) { return c->done; }
double oc_sign(const oc_chain *c) { return c->sign; }
double oc_gamma_value(const oc_chain *c) { return c->gamma; }

int oc_get_config(const oc_chain *c, int64_t *id, double *tau, int32_t *site, int32_t *s) {
    for (int i = 0; i < c->n; ++i) {
        if (id) id[i] = c->id[i];
        if (tau) tau[i] = c->tau[i];
        if (site) site[i] = c->site[i];
        if (s) s[i] = c->s[i];
    }
    return OC_OK;
}

int oc_get_N(const oc_chain *c, int32_t sector, double *out) {
    if (sector < 0 || sector > 1) return OC_EINVAL;
    for (int i = 0; i < c->n; ++i)
        for (int j = 0; j < c->n; ++j) out[(size_t)i * c->n + j] = NE(c, sector, i, j);
    return OC_OK;
}

/* Eq. (Nmatrix): (N^{-1})_ij = delta_ij e^{V_i} - G0(tau_i - tau_j)(e^{V_j} - 1). */
int oc_build_Minv(const oc_chain *c, int32_t sector, double *out) {
    if (sector < 0 || sector > 1) return OC_EINVAL;
    int n = c->n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            out[(size_t)i * n + j] = (i == j ? expV(c, sector, c->s[i]) : 0.0) -
                                     g0v(c, sector, i, j) * (expV(c, sector, c->s[j]) - 1.0);
    return OC_OK;
}

int oc_build_M_of(const oc_chain *c, int32_t sector, int32_t n, const double *tau,
                  const int32_t *site, const int32_t *s, double *out) {
    if (sector < 0 || sector > 1 || n < 0) return OC_EINVAL;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            out[(size_t)i * n + j] =
                (i == j ? expV(c, sector, s[i]) : 0.0) -
                oc_g0_lookup(c, sector, site[i], site[j], tau[i] - tau[j]) * (expV(c, sector, s[j]) - 1.0);
    return OC_OK;
}

int oc_set_config(oc_chain *c, int32_t n, const int64_t *id, const double *tau,
                  const int32_t *site, const int32_t *s, double *logabsdet, double *sgn) {
    if (n < 0 || n > c->n_cap) return fail(c, OC_ECAPACITY, "order %d exceeds n_cap", n);
    for (int i = 0; i < n; ++i) {
        if (!(tau[i] >= 0 && tau[i] < c->beta) || site[i] < 0 || site[i] >= c->nc ||
            (s[i] != 1 && s[i] != -1))
            return fail(c, OC_EINVAL, "invalid vertex %d", i);
        if (i > 0 && id[i] <= id[i - 1]) return fail(c, OC_EINVAL, "ids must ascend");
    }
    double lad[2] = {0, 0}, sg[2] = {1, 1};
    c->n = 0;
    for (int i = 0; i < n; ++i) {
        double S[2];
        for (int sec = 0; sec < 2; ++sec) S[sec] = insert_ratio(c, sec, tau[i], site[i], s[i]);
        c->tau[i] = tau[i]; c->site[i] = site[i]; c->s[i] = s[i]; c->id[i] = id[i];
        for (int sec = 0; sec < 2; ++sec) {
            if (!(S[sec] != 0.0) || !isfinite(S[sec]))
                return fail(c, OC_ENUMERIC, "singular configuration at vertex %d", i);
            insert_commit(c, sec, tau[i], site[i], S[sec]);
            lad[sec] += log(fabs(S[sec]));
            if (S[sec] < 0) sg[sec] = -sg[sec];
        }
        c->n = i + 1;
    }
    c->next_id = n > 0 ? id[n - 1] + 1 : 0;
    for (int sec = 0; sec < 2; ++sec) {
        if (logabsdet) logabsdet[sec] = lad[sec];
        if (sgn) sgn[sec] = sg[sec];
    }
    return OC_OK;
}

int oc_get_state(const oc_chain *c, int64_t *proposals_done, int64_t *next_id, double *sign) {
    *proposals_done = c->done; *next_id = c->next_id; *sign = c->sign;
    return OC_OK;
}

int oc_set_state(oc_chain *c, int64_t proposals_done, int64_t next_id, double sign) {
    if (proposals_done < 0 || (sign != 1.0 && sign != -1.0)) return OC_EINVAL;
    c->done = proposals_done; c->next_id = next_id; c->sign = sign;
    return OC_OK;
}

int oc_set_pair(oc_chain *c, double p_pair) {
    if (!(p_pair >= 0.0 && c->p_flip + p_pair <= 1.0))
        return fail(c, OC_EINVAL, "p_pair must be in [0, 1 - p_flip]");
    c->p_pair = p_pair;
    return OC_OK;
}

int oc_last_pair(const oc_chain *c, int32_t *p2, double *tau2, int32_t *site2, int32_t *s2) {
    *p2 = c->last_p2; *tau2 = c->last_tau2; *site2 = c->last_site2; *s2 = c->last_s2;
    return OC_OK;
}

int oc_last_proposal(const oc_chain *c, int32_t *type, int32_t *p, double *tau,
                     int32_t *site, int32_t *s_new, double *R, int32_t *acc) {
    *type = c->last_type; *p = c->last_p; *tau = c->last_tau; *site = c->last_site;
    *s_new = c->last_s; *R = c->last_R; *acc = c->last_acc;
    return OC_OK;
}

int32_t oc_obs_len(const oc_chain *c) { return c->obs_len; }

int oc_get_obs(const oc_chain *c, double *out) {
    memcpy(out, c->obs, sizeof(double) * (size_t)c->obs_len);
    return OC_OK;
}

int oc_reset_obs(oc_chain *c) {
    memset(c->obs, 0, sizeof(double) * (size_t)c->obs_len);
    if (c->obs_kw) memset(c->obs_kw, 0, sizeof(double) * 2 * (size_t)c->n_k * c->n_mats * 2);
    return OC_OK;
}
