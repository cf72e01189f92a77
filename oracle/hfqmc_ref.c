/*
 * hfqmc_ref.c -- plain, slow, obviously-correct CPU Hirsch-Fye QMC.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the HIP
 * path is judged.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the product library, and the product library never calls it.
 *
 * What it computes (Bluemer & Gorelik, arXiv:1006.2716):
 *   - the trapped Hubbard model, Eq. (1), is mapped by the local self-energy
 *     assumption (text after Eq. (2)) onto one Anderson impurity problem per
 *     inequivalent lattice site, each defined by its Weiss function G0_sigma(tau);
 *   - each impurity problem is solved by Hirsch-Fye QMC (the solver the paper
 *     names in its "Model and Methods" paragraph), on L = beta/dtau imaginary
 *     time slices.
 * The paper only names the solver; the formulas below are the standard
 * discrete-time construction of that solver:
 *   lambda   : cosh(lambda) = exp(dtau*U/2)                         (HS coupling)
 *   V_sigma  : diag(sigma*lambda*s_l), sigma = +1 (up), -1 (down)
 *   M_sigma  : 1 + (1 - G0_sigma)(exp(V_sigma) - 1)
 *   G_sigma  : M_sigma^{-1} G0_sigma                           (Dyson equation)
 *   flip l   : delta_sigma = exp(-2 sigma lambda s_l) - 1,
 *              R_sigma = 1 + (1 - G_sigma[l][l]) delta_sigma,   R = R_up R_dn
 *   accept   : Metropolis, u < R
 *   update   : G'[i][j] = G[i][j] + (delta/R)(G[i][l] - [i==l]) G[l][j]
 *              (Sherman-Morrison rank-one update)
 * Conventions (documented readings; the paper is silent on them):
 *   g(tau) = <T c(tau) c^dag(0)> > 0, so G[l][l] = g(0+) = 1 - n.
 *   The L input samples are g(tau_k), tau_k = k*dtau, k = 0..L-1, k = 0 is 0+.
 *   G0 matrix: G0[i][j] = g(tau_{i-j}) for i >= j, -g(tau_{i-j+L}) for i < j.
 *   Sweep: slices l = 0..L-1 in order.  Random numbers: Philox4x64-10
 *   (Salmon, Moraes, Dror, Shaw, SC'11) keyed by (seed, site); slice l of
 *   sweep w uses word (l >> 6) of the block at counter (l & 63, w + offset, 2, c);
 *   initial field s_l uses the top bit of word (l >> 6) of the block at counter
 *   (l & 63, 0, 1, c): 0 -> +1, 1 -> -1.  u = (x >> 11) * 2^-53.  c is the
 *   chain index: independent chains of one impurity share its key and differ
 *   in this counter word (c = 0 for a single chain).
 *   A from-scratch Dyson recompute replaces G after every `recompute_every`
 *   completed sweeps; then, once past the warm-up, every sweep is measured:
 *     n_sigma = 1 - (1/L) sum_l G_sigma[l][l]
 *     d       = (1/L) sum_l (1 - G_up[l][l]) (1 - G_dn[l][l])
 *     g_sigma(tau_k) = (1/L) sum_l eps_{lk} G_sigma[(l+k) mod L][l],
 *                      eps = -1 where l + k >= L;  g_sigma(tau_L) = n_sigma.
 *   Measured sweep m (0-based) falls in bin floor(m * n_bins / n_measure).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t L;
    double beta;
    double U;
    const double *weiss_up; /* L samples g(tau_k) */
    const double *weiss_dn;
    int64_t n_warmup;
    int64_t n_measure;
    int32_t recompute_every;
    int32_t n_bins;
    uint64_t seed;
    uint64_t site;
    int64_t sweep_offset;     /* added to the sweep index in the RNG counter */
    const int8_t *init_fields; /* NULL: draw from the generator */
    uint64_t chain;            /* chain index: counter word 3 of every draw */
} ref_problem;

typedef struct {
    double *bins;          /* n_bins x (2(L+1)+3): g_up[0..L], g_dn[0..L], n_up, n_dn, d */
    int8_t *final_fields;  /* L entries or NULL */
    double *final_green;   /* 2 x L x L (up then down, row-major) or NULL */
    int64_t proposals;
    int64_t accepts;
    int64_t nonpositive;   /* proposals with R <= 0 (rejected) */
    double max_drift;      /* max |G_updated - G_recomputed| over recomputes */
    int32_t status;        /* 0 ok, -1 invalid, -2 singular Dyson matrix */
    int64_t *hist;         /* NULL, or 2^L visit counts of the field at each
                              measured sweep (bit l set <=> s_l = -1); L <= 20 */
} ref_result;

/* ---------------- Philox4x64-10 (Salmon et al., SC'11) ---------------- */
void ref_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint64_t word_for(uint64_t seed, uint64_t site, int l, uint64_t c1, uint64_t purpose, uint64_t chain)
{
    uint64_t ctr[4] = {(uint64_t)(l & 63), c1, purpose, chain};
    uint64_t key[2] = {seed, site};
    uint64_t out[4];
    ref_philox4x64(ctr, key, out);
    return out[l >> 6];
}

/* ---------------- coupling: cosh(lambda) = exp(dtau U / 2) ---------------- */
int ref_lambda(double dtau, double U, double *lam)
{
    if (!(dtau > 0) || !(U >= 0) || !lam) return -1;
    /* acosh(1+m) = log1p(m + sqrt(m(m+2))), m = exp(dtau U/2) - 1 >= 0 */
    double m = expm1(0.5 * dtau * U);
    *lam = log1p(m + sqrt(m * (m + 2.0)));
    return 0;
}

/* ---------------- G0 matrix from its L samples (antiperiodic) ---------------- */
int ref_weiss_matrix(int L, const double *g, double *out)
{
    if (L < 1 || !g || !out) return -1;
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
            out[i * L + j] = (i >= j) ? g[i - j] : -g[i - j + L];
    return 0;
}

/* Solve A X = B (n x n, nrhs columns, row-major, in place) by LU with partial
 * pivoting.  A and B are overwritten.  Returns -2 on an exactly zero pivot. */
static int lu_solve(int n, double *A, double *B, int nrhs)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return -2;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
            for (int j = 0; j < nrhs; ++j) { double t = B[k * nrhs + j]; B[k * nrhs + j] = B[p * nrhs + j]; B[p * nrhs + j] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            A[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < nrhs; ++j) B[i * nrhs + j] -= f * B[k * nrhs + j];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < nrhs; ++j) {
            double v = B[k * nrhs + j];
            for (int m = k + 1; m < n; ++m) v -= A[k * n + m] * B[m * nrhs + j];
            B[k * nrhs + j] = v / A[k * n + k];
        }
    }
    return 0;
}

/* Dyson equation from scratch: G = [1 + (1 - G0)(exp(V) - 1)]^{-1} G0 with
 * V = diag(sigma lambda s_l).  G is L x L row-major. */
int ref_dyson(int L, const double *g, double lam, int sigma, const int8_t *s, double *G)
{
    if (L < 1 || !g || !s || !G || (sigma != 1 && sigma != -1)) return -1;
    double *G0 = (double *)malloc(sizeof(double) * L * L);
    double *M = (double *)malloc(sizeof(double) * L * L);
    if (!G0 || !M) { free(G0); free(M); return -1; }
    ref_weiss_matrix(L, g, G0);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
            double ev1 = exp(sigma * lam * s[j]) - 1.0;  /* (exp(V) - 1)_jj */
            double one_minus = (i == j ? 1.0 : 0.0) - G0[i * L + j];
            M[i * L + j] = (i == j ? 1.0 : 0.0) + one_minus * ev1;
        }
    memcpy(G, G0, sizeof(double) * L * L);
    int rc = lu_solve(L, M, G, L);
    free(G0); free(M);
    return rc;
}

static double flip_delta(double lam, int sigma, int s_l)
{
    return exp(-2.0 * sigma * lam * s_l) - 1.0;
}

/* Sherman-Morrison rank-one update of G for a flip of slice l with factor
 * delta and ratio R (both for this spin). */
static void sm_update(int L, double *G, int l, double delta, double R, double *col, double *row)
{
    for (int i = 0; i < L; ++i) col[i] = G[i * L + l] - (i == l ? 1.0 : 0.0);
    for (int j = 0; j < L; ++j) row[j] = G[l * L + j];
    double f = delta / R;
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
            G[i * L + j] += f * col[i] * row[j];
}

/* Start from the Dyson solution for fields s, then flip the listed slices in
 * order, each accepted unconditionally and applied by Sherman-Morrison.  The
 * fields are updated in place; ratios[k] (if non-NULL) receives R_up*R_dn of
 * flip k. */
int ref_force_flips(int L, const double *g_up, const double *g_dn, double lam, int8_t *s,
                    const int32_t *slices, int n, double *G_up, double *G_dn, double *ratios)
{
    if (L < 1 || !s || !G_up || !G_dn || (n > 0 && !slices)) return -1;
    int rc = ref_dyson(L, g_up, lam, +1, s, G_up);
    if (rc) return rc;
    rc = ref_dyson(L, g_dn, lam, -1, s, G_dn);
    if (rc) return rc;
    double *col = (double *)malloc(sizeof(double) * L);
    double *row = (double *)malloc(sizeof(double) * L);
    for (int k = 0; k < n; ++k) {
        int l = slices[k];
        if (l < 0 || l >= L) { free(col); free(row); return -1; }
        double du = flip_delta(lam, +1, s[l]), dd = flip_delta(lam, -1, s[l]);
        double Ru = 1.0 + (1.0 - G_up[l * L + l]) * du;
        double Rd = 1.0 + (1.0 - G_dn[l * L + l]) * dd;
        if (ratios) ratios[k] = Ru * Rd;
        sm_update(L, G_up, l, du, Ru, col, row);
        sm_update(L, G_dn, l, dd, Rd, col, row);
        s[l] = (int8_t)(-s[l]);
    }
    free(col); free(row);
    return 0;
}

/* ---------------- one full Markov chain ---------------- */
static int run_one(const ref_problem *p, ref_result *r)
{
    const int L = p->L;
    r->proposals = r->accepts = r->nonpositive = 0;
    r->max_drift = 0.0;
    if (L < 1 || !(p->beta > 0) || !(p->U >= 0) || !p->weiss_up || !p->weiss_dn ||
        p->n_bins < 1 || p->n_measure < p->n_bins || p->n_warmup < 0 || p->recompute_every < 1 ||
        !r->bins)
        return (r->status = -1);
    double dtau = p->beta / L, lam;
    ref_lambda(dtau, p->U, &lam);

    int8_t *s = (int8_t *)malloc(L);
    double *G[2], *Gf[2];
    const double *gw[2] = {p->weiss_up, p->weiss_dn};
    for (int a = 0; a < 2; ++a) {
        G[a] = (double *)malloc(sizeof(double) * L * L);
        Gf[a] = (double *)malloc(sizeof(double) * L * L);
    }
    double *col = (double *)malloc(sizeof(double) * L);
    double *row = (double *)malloc(sizeof(double) * L);
    const int NV = 2 * (L + 1) + 3;
    double *acc = (double *)calloc((size_t)p->n_bins * NV, sizeof(double));
    int64_t *cnt = (int64_t *)calloc(p->n_bins, sizeof(int64_t));
    double *meas = (double *)malloc(sizeof(double) * NV);

    for (int l = 0; l < L; ++l) {
        if (p->init_fields) s[l] = p->init_fields[l] >= 0 ? 1 : -1;
        else s[l] = (word_for(p->seed, p->site, l, 0, 1, p->chain) >> 63) ? -1 : 1;
    }
    int rc = 0;
    for (int a = 0; a < 2 && !rc; ++a) rc = ref_dyson(L, gw[a], lam, a == 0 ? 1 : -1, s, G[a]);

    const int64_t total = p->n_warmup + p->n_measure;
    for (int64_t w = 0; w < total && !rc; ++w) {
        for (int l = 0; l < L; ++l) {
            double du = flip_delta(lam, +1, s[l]), dd = flip_delta(lam, -1, s[l]);
            double Ru = 1.0 + (1.0 - G[0][l * L + l]) * du;
            double Rd = 1.0 + (1.0 - G[1][l * L + l]) * dd;
            double R = Ru * Rd;
            uint64_t x = word_for(p->seed, p->site, l, (uint64_t)(w + p->sweep_offset), 2, p->chain);
            double u = (double)(x >> 11) * 0x1.0p-53;
            r->proposals++;
            if (!(R > 0)) { r->nonpositive++; continue; }
            if (u < R) {
                sm_update(L, G[0], l, du, Ru, col, row);
                sm_update(L, G[1], l, dd, Rd, col, row);
                s[l] = (int8_t)(-s[l]);
                r->accepts++;
            }
        }
        if ((w + 1) % p->recompute_every == 0) {
            for (int a = 0; a < 2 && !rc; ++a) {
                rc = ref_dyson(L, gw[a], lam, a == 0 ? 1 : -1, s, Gf[a]);
                for (int i = 0; i < L * L && !rc; ++i) {
                    double dv = fabs(G[a][i] - Gf[a][i]);
                    if (dv > r->max_drift) r->max_drift = dv;
                }
                double *t = G[a]; G[a] = Gf[a]; Gf[a] = t;
            }
        }
        if (w >= p->n_warmup && !rc) {
            int64_t m = w - p->n_warmup;
            int b = (int)((m * p->n_bins) / p->n_measure);
            double nsum[2] = {0, 0}, dsum = 0;
            for (int l = 0; l < L; ++l) {
                nsum[0] += 1.0 - G[0][l * L + l];
                nsum[1] += 1.0 - G[1][l * L + l];
                dsum += (1.0 - G[0][l * L + l]) * (1.0 - G[1][l * L + l]);
            }
            for (int a = 0; a < 2; ++a) {
                for (int k = 0; k < L; ++k) {
                    double sum = 0;
                    for (int l = 0; l < L; ++l) {
                        int i = l + k;
                        if (i >= L) sum -= G[a][(i - L) * L + l];
                        else sum += G[a][i * L + l];
                    }
                    meas[a * (L + 1) + k] = sum / L;
                }
                meas[a * (L + 1) + L] = nsum[a] / L;
            }
            meas[2 * (L + 1) + 0] = nsum[0] / L;
            meas[2 * (L + 1) + 1] = nsum[1] / L;
            meas[2 * (L + 1) + 2] = dsum / L;
            for (int v = 0; v < NV; ++v) acc[(size_t)b * NV + v] += meas[v];
            cnt[b]++;
            if (r->hist && L <= 20) {
                uint32_t code = 0;
                for (int l = 0; l < L; ++l) if (s[l] < 0) code |= 1u << l;
                r->hist[code]++;
            }
        }
    }
    if (!rc) {
        for (int b = 0; b < p->n_bins; ++b)
            for (int v = 0; v < NV; ++v)
                r->bins[(size_t)b * NV + v] = acc[(size_t)b * NV + v] / (double)cnt[b];
        if (r->final_fields) memcpy(r->final_fields, s, L);
        if (r->final_green) {
            memcpy(r->final_green, G[0], sizeof(double) * L * L);
            memcpy(r->final_green + (size_t)L * L, G[1], sizeof(double) * L * L);
        }
    }
    free(s); free(col); free(row); free(acc); free(cnt); free(meas);
    for (int a = 0; a < 2; ++a) { free(G[a]); free(Gf[a]); }
    return (r->status = rc);
}

/* ---------------- many chains on a pool of host threads ---------------- */
typedef struct {
    const ref_problem *p;
    ref_result *r;
    int n;
    int next;
    pthread_mutex_t mu;
} pool_t;

static void *worker(void *arg)
{
    pool_t *pool = (pool_t *)arg;
    for (;;) {
        pthread_mutex_lock(&pool->mu);
        int i = pool->next++;
        pthread_mutex_unlock(&pool->mu);
        if (i >= pool->n) break;
        run_one(&pool->p[i], &pool->r[i]);
    }
    return NULL;
}

int ref_run(const ref_problem *problems, int n, ref_result *results, int n_threads)
{
    if (n < 0 || (n > 0 && (!problems || !results))) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n) n_threads = n > 0 ? n : 1;
    pool_t pool;
    pool.p = problems; pool.r = results; pool.n = n; pool.next = 0;
    pthread_mutex_init(&pool.mu, NULL);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * n_threads);
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, &pool);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&pool.mu);
    int rc = 0;
    for (int i = 0; i < n; ++i) if (results[i].status) rc = results[i].status;
    return rc;
}
