/*
 * gld_oracle.c -- plain FP64 CPU oracle for one time step of generalized
 * Langevin dynamics (GLD), Jung, Hanke & Schmid, "Generalized Langevin
 * dynamics: construction and numerical integration of non-Markovian
 * particle-based models" (arXiv:1808.00270).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this library.  It
 * shares no code, header, table or helper with the HIP path in the package;
 * the two are compared against each other on identical seeded inputs.
 *
 * Everything is written for clarity, in double precision, with literal
 * loops over particles, neighbours and memory lags:
 *
 *   - geometry      : minimum-image pairs within r_c, brute force O(N^2) or
 *                     a plain cell list (the latter checked against the former)
 *   - conservative  : WCA pair force (stand-in for the paper's tabulated
 *                     potential, Sec. IV / App. B use IBI; configs use WCA)
 *   - integrator    : eq. (GLD_integrator) with a, b of eq. (aa-bb), position
 *                     update with b as derived in App. A, eq. (rrstep)
 *   - dissipation   : eq. (dissipative_force2), literally: m = 0 pair term with
 *                     the current velocities, lags m = 1..m_max-1 acting on the
 *                     displacement history, kernels at the current distances
 *   - colored noise : Sec. II.C, eqs. (correlation_matrix)-(FT) and
 *                     Algorithm 1 (Lanczos per frequency, matrix-free
 *                     neighbour mat-vec, square root of the tridiagonal
 *                     projection by eigendecomposition)
 *   - dense noise   : for tiny N, the same vector from an explicit
 *                     eigendecomposition of every 3N x 3N spectral matrix
 *                     (frequency domain) and from the time-domain filter
 *                     matrices A_s of eq. (noise_production)
 *
 * Readings taken where the paper is silent or inconsistent (each one is a
 * documented design decision of the project):
 *   - discrete kernels K_m are inputs (the continuous -> discrete map is the
 *     caller's business);
 *   - position update uses b (App. A, eq. rrstep) rather than a (main text);
 *   - Algorithm 1's last step is normalised by 1/(2 m_max - 1), the period of
 *     the DFT of eq. (FT), and sums F_0 + 2 sum_{w>=1} F_w;
 *   - Lanczos acts on the real part of W_hat (the imaginary part cancels in
 *     the real inverse transform), stops on a relative tolerance and reports
 *     non-convergence after a fixed iteration cap;
 *   - history before step 0 is zero; white noise W_t exists for every integer
 *     t (also negative), so the colored noise is stationary from step 0;
 *   - white noise is Philox4x32-10 (Salmon et al., SC'11) with Box-Muller;
 *     key = seed, counter = (particle id, step lo, step hi, 0);
 *   - the distance dependent self memory Delta K^s of eq. (GLD_basic2) has
 *     the pair memory's tensor form (1 or e e^T) and enters F^D' and the
 *     noise correlation as eqs. (dissipative_force2), (stochastic_force2)
 *     write it; a and b use the isotropic K^s_0 alone.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_NOT_PD (-2)
#define ORC_ERR_NO_CONV (-3)
#define ORC_ERR_OOM (-5)

typedef struct {
    int64_t n;               /* number of particles                         */
    double box[3];           /* periodic box edge lengths                   */
    double dt, mass, kT;     /* time step, particle mass M, k_B T           */
    int32_t m_max;           /* memory length (number of lags incl. m = 0)  */
    int32_t n_r;             /* number of distance grid points              */
    const double *k_self;    /* [m_max]      K^s_m                          */
    const double *k_pair;    /* [n_r*m_max]  K^p_m(r_b), r_b = r0 + b dr    */
    double r0, dr;           /* distance grid                               */
    double r_cut, r_cut_min; /* pair cutoff; kernels frozen below r_cut_min */
    int32_t parallel;        /* 0: K^p * identity, 1: K^p * e e^T           */
    int32_t lanczos_max_iter;
    double wca_sigma, wca_eps;
    uint64_t seed;
    double lanczos_tol;      /* relative stopping tolerance of Algorithm 1  */
    const double *dk_self;   /* [n_r*m_max] Delta K^s_m(r_b), or NULL: none */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11) */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof(x));
}

/* Three standard normal numbers W_{p,c,t}, c = 0,1,2, for particle id p at
 * integer step t (t may be negative), from one Philox call + Box-Muller. */
void orc_gauss3(uint64_t seed, uint32_t pid, int64_t t, double z[3])
{
    const uint64_t tu = (uint64_t)t;
    const uint32_t ctr[4] = {pid, (uint32_t)tu, (uint32_t)(tu >> 32), 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two_pi = 6.283185307179586476925286766559;
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)x[k] + 0.5) * (1.0 / 4294967296.0);
    const double ra = sqrt(-2.0 * log(u[0]));
    const double rb = sqrt(-2.0 * log(u[2]));
    z[0] = ra * cos(two_pi * u[1]);
    z[1] = ra * sin(two_pi * u[1]);
    z[2] = rb * cos(two_pi * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

static void min_image(const orc_params *p, const double *ri, const double *rj, double d[3])
{
    for (int c = 0; c < 3; ++c) {
        double x = ri[c] - rj[c];
        x -= p->box[c] * nearbyint(x / p->box[c]);
        d[c] = x;
    }
}

typedef struct {
    int64_t i, j;  /* ordered pair, i != j                */
    double d[3];   /* R_i - R_j (minimum image)           */
    double r;      /* |d|                                 */
} orc_pair;

typedef struct {
    int64_t n, cap;
    orc_pair *v;
} pair_list;

static int push_pair(pair_list *L, int64_t i, int64_t j, const double d[3], double r)
{
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 1024;
        orc_pair *nv = (orc_pair *)realloc(L->v, (size_t)nc * sizeof(orc_pair));
        if (!nv) return ORC_ERR_OOM;
        L->v = nv;
        L->cap = nc;
    }
    orc_pair *q = &L->v[L->n++];
    q->i = i;
    q->j = j;
    memcpy(q->d, d, sizeof(q->d));
    q->r = r;
    return ORC_OK;
}

/* All ordered pairs (i, j), i != j, |R_ij| < r_cut, by testing every pair. */
static int pairs_brute(const orc_params *p, const double *R, pair_list *L)
{
    for (int64_t i = 0; i < p->n; ++i)
        for (int64_t j = 0; j < p->n; ++j) {
            if (i == j) continue;
            double d[3];
            min_image(p, R + 3 * i, R + 3 * j, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r < p->r_cut && push_pair(L, i, j, d, r)) return ORC_ERR_OOM;
        }
    return ORC_OK;
}

/* The same pair set from a plain cell list: cells of edge >= r_cut, neighbour
 * cell offsets {-1,0,1} reduced to distinct values per axis for small grids. */
static int pairs_cells(const orc_params *p, const double *R, pair_list *L)
{
    int nc[3];
    for (int c = 0; c < 3; ++c) {
        nc[c] = (int)floor(p->box[c] / p->r_cut);
        if (nc[c] < 1) nc[c] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)p->n * sizeof(int64_t));
    int *cell_of = (int *)malloc((size_t)p->n * 3 * sizeof(int));
    if (!head || !next || !cell_of) {
        free(head); free(next); free(cell_of);
        return ORC_ERR_OOM;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    /* insert in decreasing index order so that each chain lists ascending ids */
    for (int64_t i = p->n - 1; i >= 0; --i) {
        int ci[3];
        for (int c = 0; c < 3; ++c) {
            double x = R[3 * i + c] - p->box[c] * floor(R[3 * i + c] / p->box[c]);
            int k = (int)floor(x / p->box[c] * nc[c]);
            if (k >= nc[c]) k = nc[c] - 1;
            if (k < 0) k = 0;
            ci[c] = k;
            cell_of[3 * i + c] = k;
        }
        const int64_t cid = ((int64_t)ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
        next[i] = head[cid];
        head[cid] = i;
    }
    int offs[3][3], noff[3];
    for (int c = 0; c < 3; ++c) {
        if (nc[c] == 1) { noff[c] = 1; offs[c][0] = 0; }
        else if (nc[c] == 2) { noff[c] = 2; offs[c][0] = 0; offs[c][1] = 1; }
        else { noff[c] = 3; offs[c][0] = -1; offs[c][1] = 0; offs[c][2] = 1; }
    }
    int rc = ORC_OK;
    for (int64_t i = 0; i < p->n && rc == ORC_OK; ++i) {
        const int *ci = cell_of + 3 * i;
        for (int a = 0; a < noff[2]; ++a)
            for (int b = 0; b < noff[1]; ++b)
                for (int e = 0; e < noff[0]; ++e) {
                    const int cz = (ci[2] + offs[2][a] + nc[2]) % nc[2];
                    const int cy = (ci[1] + offs[1][b] + nc[1]) % nc[1];
                    const int cx = (ci[0] + offs[0][e] + nc[0]) % nc[0];
                    const int64_t cid = ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
                    for (int64_t j = head[cid]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double d[3];
                        min_image(p, R + 3 * i, R + 3 * j, d);
                        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                        if (r < p->r_cut && push_pair(L, i, j, d, r)) { rc = ORC_ERR_OOM; }
                    }
                }
    }
    free(head); free(next); free(cell_of);
    return rc;
}

static int find_pairs(const orc_params *p, const double *R, pair_list *L)
{
    L->n = 0;
    if (p->n <= 2048) return pairs_brute(p, R, L);
    return pairs_cells(p, R, L);
}

/* Exposed for the test-suite: ordered pairs (i, j) with their distance. */
int orc_pairs(const orc_params *p, const double *R, int use_cells, int64_t cap,
              int64_t *ij, double *r, int64_t *count)
{
    pair_list L = {0, 0, NULL};
    int rc = use_cells ? pairs_cells(p, R, &L) : pairs_brute(p, R, &L);
    if (rc) { free(L.v); return rc; }
    *count = L.n;
    if (L.n > cap) { free(L.v); return ORC_ERR_INVALID; }
    for (int64_t k = 0; k < L.n; ++k) {
        ij[2 * k] = L.v[k].i;
        ij[2 * k + 1] = L.v[k].j;
        r[k] = L.v[k].r;
    }
    free(L.v);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Tabulated pair kernel: linear interpolation on the distance grid,        */
/* frozen below r_cut_min (the paper uses the kernel at r_c,min there).      */
/* ------------------------------------------------------------------------ */

static void grid_locate(const orc_params *p, double r, int *b, double *f)
{
    if (r < p->r_cut_min) r = p->r_cut_min;
    double t = (r - p->r0) / p->dr;
    if (t < 0.0) t = 0.0;
    int k = (int)floor(t);
    if (k > p->n_r - 2) k = p->n_r - 2;
    if (k < 0) k = 0;
    *b = k;
    *f = t - (double)k;
}

/* K^p_m(r) for one lag m */
static double kpair_at(const orc_params *p, double r, int m)
{
    int b;
    double f;
    grid_locate(p, r, &b, &f);
    const double *t0 = p->k_pair + (size_t)b * p->m_max;
    const double *t1 = t0 + p->m_max;
    return t0[m] * (1.0 - f) + t1[m] * f;
}

/* Delta K^s_m(r) for one lag m (0 without a table) */
static double dks_at(const orc_params *p, double r, int m)
{
    if (!p->dk_self) return 0.0;
    int b;
    double f;
    grid_locate(p, r, &b, &f);
    const double *t0 = p->dk_self + (size_t)b * p->m_max;
    const double *t1 = t0 + p->m_max;
    return t0[m] * (1.0 - f) + t1[m] * f;
}

/* y += k * T_ij x, with T = 1 or e e^T */
static void apply_tensor(const orc_params *p, const orc_pair *q, double k, const double *x, double *y)
{
    if (!p->parallel) {
        y[0] += k * x[0];
        y[1] += k * x[1];
        y[2] += k * x[2];
    } else {
        const double e0 = q->d[0] / q->r, e1 = q->d[1] / q->r, e2 = q->d[2] / q->r;
        const double s = k * (e0 * x[0] + e1 * x[1] + e2 * x[2]);
        y[0] += s * e0;
        y[1] += s * e1;
        y[2] += s * e2;
    }
}

/* ------------------------------------------------------------------------ */
/* Conservative force: WCA, U = 4 eps [(s/r)^12 - (s/r)^6] + eps, r < 2^(1/6) s */
/* ------------------------------------------------------------------------ */

static void wca_pair(const orc_params *p, double r, double *u, double *f_over_r)
{
    const double rc = pow(2.0, 1.0 / 6.0) * p->wca_sigma;
    if (p->wca_eps == 0.0 || r >= rc) { *u = 0.0; *f_over_r = 0.0; return; }
    const double s6 = pow(p->wca_sigma / r, 6.0);
    *u = 4.0 * p->wca_eps * (s6 * s6 - s6) + p->wca_eps;
    *f_over_r = 24.0 * p->wca_eps * (2.0 * s6 * s6 - s6) / (r * r);
}

static void wca_forces(const orc_params *p, const pair_list *L, double *F)
{
    memset(F, 0, (size_t)p->n * 3 * sizeof(double));
    for (int64_t k = 0; k < L->n; ++k) {
        const orc_pair *q = &L->v[k];
        double u, fr;
        wca_pair(p, q->r, &u, &fr);
        for (int c = 0; c < 3; ++c) F[3 * q->i + c] += fr * q->d[c];
    }
}

/* total WCA energy (for gradient checks) */
double orc_wca_energy(const orc_params *p, const double *R)
{
    double E = 0.0;
    for (int64_t i = 0; i < p->n; ++i)
        for (int64_t j = i + 1; j < p->n; ++j) {
            double d[3];
            min_image(p, R + 3 * i, R + 3 * j, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double u, fr;
            wca_pair(p, r, &u, &fr);
            E += u;
        }
    return E;
}

int orc_wca_forces(const orc_params *p, const double *R, double *F)
{
    pair_list L = {0, 0, NULL};
    int rc = find_pairs(p, R, &L);
    if (!rc) wca_forces(p, &L, F);
    free(L.v);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Integrator coefficients, eq. (aa-bb) with isotropic K^s_0                 */
/* ------------------------------------------------------------------------ */

void orc_ab(const orc_params *p, double *a, double *b)
{
    const double x = p->dt * p->k_self[0] / (2.0 * p->mass);
    *b = 1.0 / (1.0 + x);
    *a = (*b) * (1.0 - x);
}

/* ------------------------------------------------------------------------ */
/* Dissipative force, eq. (dissipative_force2):                             */
/*   F_i = - sum_{j!=i} [ K^p_0(R_ij) T V_j + Delta K^s_0(R_ij) T V_i ]      */
/*         - 1/dt sum_{m=1}^{m_max-1} [ sum_{j!=i} K^p_m(R_ij) T dR_{j,n-m}  */
/*              + (K^s_m + sum_{k!=i} Delta K^s_m(R_ik) T) dR_{i,n-m} ]      */
/* hist[(m-1)][i][c] = dR_{i,n-m}.                                           */
/* ------------------------------------------------------------------------ */

static void dissipative_row(const orc_params *p, int64_t i, const orc_pair *nb, int64_t nnb,
                            const double *V, const double *hist, double *out)
{
    const int64_t N = p->n;
    double acc[3] = {0.0, 0.0, 0.0};
    double hsum[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < nnb; ++k) {
        const orc_pair *q = &nb[k];
        apply_tensor(p, q, kpair_at(p, q->r, 0), V + 3 * q->j, acc);
        for (int m = 1; m < p->m_max; ++m)
            apply_tensor(p, q, kpair_at(p, q->r, m), hist + ((size_t)(m - 1) * N + q->j) * 3, hsum);
        if (p->dk_self) {
            /* the two-particle part of the self memory acts on particle i's own velocity and history */
            apply_tensor(p, q, dks_at(p, q->r, 0), V + 3 * i, acc);
            for (int m = 1; m < p->m_max; ++m)
                apply_tensor(p, q, dks_at(p, q->r, m), hist + ((size_t)(m - 1) * N + i) * 3, hsum);
        }
    }
    for (int m = 1; m < p->m_max; ++m)
        for (int c = 0; c < 3; ++c)
            hsum[c] += p->k_self[m] * hist[((size_t)(m - 1) * N + i) * 3 + c];
    for (int c = 0; c < 3; ++c) out[c] = -acc[c] - hsum[c] / p->dt;
}

static void dissipative(const orc_params *p, const pair_list *L, const double *V,
                        const double *hist, double *FD)
{
    /* pairs are produced grouped by i; locate each particle's block */
    int64_t *start = (int64_t *)calloc((size_t)p->n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < L->n; ++k) start[L->v[k].i + 1]++;
    for (int64_t i = 0; i < p->n; ++i) start[i + 1] += start[i];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < p->n; ++i)
        dissipative_row(p, i, L->v + start[i], start[i + 1] - start[i], V, hist, FD + 3 * i);
    free(start);
}

/* ------------------------------------------------------------------------ */
/* Spectra: correlation sequences c_m = kT a_m K_m / dt (eq. stochastic_force2,
 * a_0 = 2, a_m = 1) and their length-(2 m_max - 1) DFT (eq. FT), which is
 * real because c_{-m} = c_m.                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_params p;
    int M, P;
    double *cosw;     /* [M*M] cos(2 pi w m / P)                 */
    double *S_hat;    /* [M]   self spectrum                      */
    double *Kp_hat;   /* [n_r*M] pair spectrum per distance bin   */
    double *DKs_hat;  /* [n_r*M] spectrum of Delta K^s per bin, or NULL */
    int last_iters;   /* largest Lanczos iteration count, last call */
} orc_ctx;

static double corr_coef(const orc_params *p, double Km, int m)
{
    const double am = (m == 0) ? 2.0 : 1.0;
    return p->kT * am * Km / p->dt;
}

void orc_destroy(orc_ctx *c);

orc_ctx *orc_create(const orc_params *p)
{
    if (p->n < 1 || p->m_max < 1 || p->n_r < 2 || p->dt <= 0 || p->mass <= 0) return NULL;
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->p = *p;
    c->M = p->m_max;
    c->P = 2 * p->m_max - 1;
    const int M = c->M, P = c->P;
    c->cosw = (double *)malloc((size_t)M * M * sizeof(double));
    c->S_hat = (double *)malloc((size_t)M * sizeof(double));
    c->Kp_hat = (double *)malloc((size_t)p->n_r * M * sizeof(double));
    if (!c->cosw || !c->S_hat || !c->Kp_hat) {
        free(c->cosw); free(c->S_hat); free(c->Kp_hat); free(c);
        return NULL;
    }
    const double two_pi = 6.283185307179586476925286766559;
    for (int w = 0; w < M; ++w)
        for (int m = 0; m < M; ++m)
            c->cosw[(size_t)w * M + m] = cos(two_pi * (double)(((int64_t)w * m) % P) / (double)P);
    for (int w = 0; w < M; ++w) {
        double s = corr_coef(p, p->k_self[0], 0);
        for (int m = 1; m < M; ++m) s += 2.0 * corr_coef(p, p->k_self[m], m) * c->cosw[(size_t)w * M + m];
        c->S_hat[w] = s;
    }
    for (int b = 0; b < p->n_r; ++b) {
        const double *kb = p->k_pair + (size_t)b * M;
        for (int w = 0; w < M; ++w) {
            double s = corr_coef(p, kb[0], 0);
            for (int m = 1; m < M; ++m) s += 2.0 * corr_coef(p, kb[m], m) * c->cosw[(size_t)w * M + m];
            c->Kp_hat[(size_t)b * M + w] = s;
        }
    }
    if (p->dk_self) {
        c->DKs_hat = (double *)malloc((size_t)p->n_r * M * sizeof(double));
        if (!c->DKs_hat) { orc_destroy(c); return NULL; }
        for (int b = 0; b < p->n_r; ++b) {
            const double *kb = p->dk_self + (size_t)b * M;
            for (int w = 0; w < M; ++w) {
                double s = corr_coef(p, kb[0], 0);
                for (int m = 1; m < M; ++m) s += 2.0 * corr_coef(p, kb[m], m) * c->cosw[(size_t)w * M + m];
                c->DKs_hat[(size_t)b * M + w] = s;
            }
        }
    }
    return c;
}

void orc_destroy(orc_ctx *c)
{
    if (!c) return;
    free(c->cosw); free(c->S_hat); free(c->Kp_hat); free(c->DKs_hat); free(c);
}

int orc_last_iters(const orc_ctx *c) { return c->last_iters; }

void orc_spectra(const orc_ctx *c, double *S_hat, double *Kp_hat)
{
    memcpy(S_hat, c->S_hat, (size_t)c->M * sizeof(double));
    memcpy(Kp_hat, c->Kp_hat, (size_t)c->p.n_r * c->M * sizeof(double));
}

static double kp_hat_at(const orc_ctx *c, double r, int w)
{
    int b;
    double f;
    grid_locate(&c->p, r, &b, &f);
    return c->Kp_hat[(size_t)b * c->M + w] * (1.0 - f) + c->Kp_hat[(size_t)(b + 1) * c->M + w] * f;
}

static double dks_hat_at(const orc_ctx *c, double r, int w)
{
    if (!c->DKs_hat) return 0.0;
    int b;
    double f;
    grid_locate(&c->p, r, &b, &f);
    return c->DKs_hat[(size_t)b * c->M + w] * (1.0 - f) + c->DKs_hat[(size_t)(b + 1) * c->M + w] * f;
}

/* y = K_hat_w x, matrix free over the pair list (Sec. II.C: iterate over the
 * neighbours instead of storing the sparse matrix); khp[k], dkh[k]: the pair
 * and the self-memory spectra of pair k at this frequency (dkh NULL: none) */
static void khat_apply(const orc_ctx *c, int w, const pair_list *L, const double *khp, const double *dkh,
                       const double *x, double *y)
{
    const int64_t n3 = 3 * c->p.n;
    for (int64_t I = 0; I < n3; ++I) y[I] = c->S_hat[w] * x[I];
    for (int64_t k = 0; k < L->n; ++k) {
        const orc_pair *q = &L->v[k];
        apply_tensor(&c->p, q, khp[k], x + 3 * q->j, y + 3 * q->i);
        if (dkh) apply_tensor(&c->p, q, dkh[k], x + 3 * q->i, y + 3 * q->i);
    }
}

/* ------------------------------------------------------------------------ */
/* Symmetric tridiagonal eigen-decomposition: implicit QR sweeps with a      */
/* Wilkinson shift and Givens bulge chasing (Golub & Van Loan, Sec. 8.3).    */
/* d[n] diagonal, e[n-1] off-diagonal (destroyed); Q[n*n] row-major gets the  */
/* eigenvectors as columns. Returns 0, or -1 if it fails to converge.        */
/* ------------------------------------------------------------------------ */

static int tridiag_eig(int n, double *d, double *e, double *Q)
{
    for (int i = 0; i < n * n; ++i) Q[i] = 0.0;
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    int hi = n - 1, guard = 0;
    while (hi > 0) {
        if (++guard > 60 * n + 100) return -1;
        if (fabs(e[hi - 1]) <= 1e-16 * (fabs(d[hi - 1]) + fabs(d[hi])) || e[hi - 1] == 0.0) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !(fabs(e[lo - 1]) <= 1e-16 * (fabs(d[lo - 1]) + fabs(d[lo])))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        /* Wilkinson shift: eigenvalue of the trailing 2x2 block closer to d[hi] */
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * hypot(delta, eh);
        const double mu = d[hi] - eh * eh / den;
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            double r = hypot(x, z), cs = 1.0, sn = 0.0;
            if (r != 0.0) { cs = x / r; sn = z / r; }
            if (k > lo) e[k - 1] = r;
            /* rotate rows/cols k, k+1 of the 2x2 block */
            const double a = d[k], b = e[k], dd = d[k + 1];
            d[k] = cs * cs * a + 2.0 * cs * sn * b + sn * sn * dd;
            d[k + 1] = sn * sn * a - 2.0 * cs * sn * b + cs * cs * dd;
            e[k] = cs * sn * (dd - a) + (cs * cs - sn * sn) * b;
            if (k + 1 < hi) {
                z = sn * e[k + 1];   /* new bulge at (k, k+2) */
                e[k + 1] = cs * e[k + 1];
                x = e[k];
            }
            for (int i = 0; i < n; ++i) {
                const double qk = Q[i * n + k], qk1 = Q[i * n + k + 1];
                Q[i * n + k] = cs * qk + sn * qk1;
                Q[i * n + k + 1] = -sn * qk + cs * qk1;
            }
        }
    }
    return 0;
}

int orc_tridiag_eig(int n, double *d, double *e, double *Q) { return tridiag_eig(n, d, e, Q); }

/* ------------------------------------------------------------------------ */
/* Colored noise by Algorithm 1                                              */
/* ------------------------------------------------------------------------ */

/* Re W_hat_{I,w} = sum_{m=-(M-1)}^{M-1} W_{I,n+m} cos(2 pi w m / P) for the
 * frequencies w in [w0, w1), written to What[(w-w0)*3N + I]. */
static void window_dft(const orc_ctx *c, int64_t step, const uint32_t *ids, int w0, int w1, double *What)
{
    const int M = c->M;
    const int64_t N = c->p.n;
    const int nw = w1 - w0;
#pragma omp parallel
    {
        double *win = (double *)malloc((size_t)(2 * M - 1) * 3 * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const uint32_t pid = ids ? ids[i] : (uint32_t)i;
            for (int s = -(M - 1); s <= M - 1; ++s)
                orc_gauss3(c->p.seed, pid, step + s, win + 3 * (s + M - 1));
            for (int w = 0; w < nw; ++w) {
                const double *cw = c->cosw + (size_t)(w0 + w) * M;
                for (int comp = 0; comp < 3; ++comp) {
                    double acc = win[3 * (M - 1) + comp];
                    for (int m = 1; m < M; ++m)
                        acc += (win[3 * (M - 1 + m) + comp] + win[3 * (M - 1 - m) + comp]) * cw[m];
                    What[(size_t)w * 3 * N + 3 * i + comp] = acc;
                }
            }
        }
        free(win);
    }
}

static double dotv(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/* x = sqrt(K_hat_w) b by Lanczos (Algorithm 1, one frequency). */
static int lanczos_sqrt(const orc_ctx *c, int w, const pair_list *L, const double *khp, const double *dkh,
                        const double *bvec, double *x, int *iters)
{
    const int64_t n3 = 3 * c->p.n;
    const int kmax = c->p.lanczos_max_iter;
    const double tol = c->p.lanczos_tol;
    const double nb = sqrt(dotv(n3, bvec, bvec));
    memset(x, 0, (size_t)n3 * sizeof(double));
    *iters = 0;
    if (nb == 0.0) return ORC_OK;
    double *Vb = (double *)malloc((size_t)(kmax + 1) * n3 * sizeof(double));
    double *Kv = (double *)malloc((size_t)n3 * sizeof(double));
    double *r = (double *)malloc((size_t)n3 * sizeof(double));
    double *xo = (double *)malloc((size_t)n3 * sizeof(double));
    double *alpha = (double *)malloc((size_t)(kmax + 1) * sizeof(double));
    double *beta = (double *)malloc((size_t)(kmax + 1) * sizeof(double));
    double *dd = (double *)malloc((size_t)(kmax + 1) * sizeof(double));
    double *ee = (double *)malloc((size_t)(kmax + 1) * sizeof(double));
    double *Q = (double *)malloc((size_t)(kmax + 1) * (kmax + 1) * sizeof(double));
    double *y = (double *)malloc((size_t)(kmax + 1) * sizeof(double));
    int rc = ORC_OK;
    if (!Vb || !Kv || !r || !xo || !alpha || !beta || !dd || !ee || !Q || !y) { rc = ORC_ERR_OOM; goto done; }

    /* v^1 = b / |b|, alpha^1 = v^1 K v^1 */
    for (int64_t I = 0; I < n3; ++I) Vb[I] = bvec[I] / nb;
    khat_apply(c, w, L, khp, dkh, Vb, Kv);
    alpha[0] = dotv(n3, Vb, Kv);
    if (alpha[0] <= 0.0) { rc = ORC_ERR_NOT_PD; goto done; }
    {
        const double s = nb * sqrt(alpha[0]);
        for (int64_t I = 0; I < n3; ++I) x[I] = s * Vb[I];
    }
    int k = 1; /* dimension of the current Krylov basis */
    for (;;) {
        if (k >= kmax) { rc = ORC_ERR_NO_CONV; break; }
        const double *vk = Vb + (size_t)(k - 1) * n3;
        const double *vkm = (k >= 2) ? Vb + (size_t)(k - 2) * n3 : NULL;
        /* r^{k+1} = K v^k - alpha^k v^k - beta^{k-1} v^{k-1} */
        for (int64_t I = 0; I < n3; ++I) {
            double t = Kv[I] - alpha[k - 1] * vk[I];
            if (vkm) t -= beta[k - 2] * vkm[I];
            r[I] = t;
        }
        beta[k - 1] = sqrt(dotv(n3, r, r));
        if (beta[k - 1] <= 1e-14 * fabs(alpha[k - 1]) || beta[k - 1] <= 1e-300) {
            break; /* invariant subspace reached: x is exact */
        }
        double *vn = Vb + (size_t)k * n3;
        for (int64_t I = 0; I < n3; ++I) vn[I] = r[I] / beta[k - 1];
        khat_apply(c, w, L, khp, dkh, vn, Kv);
        alpha[k] = dotv(n3, vn, Kv);
        const int kk = k + 1;
        for (int q = 0; q < kk; ++q) dd[q] = alpha[q];
        for (int q = 0; q + 1 < kk; ++q) ee[q] = beta[q];
        if (tridiag_eig(kk, dd, ee, Q)) { rc = ORC_ERR_NO_CONV; break; }
        for (int q = 0; q < kk; ++q)
            if (!(dd[q] > 0.0)) { rc = ORC_ERR_NOT_PD; break; }
        if (rc) break;
        /* y = sqrt(H) e_1 = Q diag(sqrt(theta)) Q^T e_1 */
        for (int a = 0; a < kk; ++a) {
            double s = 0.0;
            for (int q = 0; q < kk; ++q) s += Q[a * kk + q] * sqrt(dd[q]) * Q[0 * kk + q];
            y[a] = s;
        }
        memcpy(xo, x, (size_t)n3 * sizeof(double));
        for (int64_t I = 0; I < n3; ++I) {
            double s = 0.0;
            for (int a = 0; a < kk; ++a) s += Vb[(size_t)a * n3 + I] * y[a];
            x[I] = nb * s;
        }
        double diff = 0.0, nx = 0.0;
        for (int64_t I = 0; I < n3; ++I) {
            diff += (x[I] - xo[I]) * (x[I] - xo[I]);
            nx += x[I] * x[I];
        }
        k = kk;
        if (sqrt(diff) <= tol * sqrt(nx)) break;
    }
    *iters = k;
done:
    free(Vb); free(Kv); free(r); free(xo); free(alpha); free(beta);
    free(dd); free(ee); free(Q); free(y);
    return rc;
}

/* F^R_n restricted to the frequencies [w0, w1) (the full vector for w0 = 0,
 * w1 = m_max).  ids: particle ids used as Philox counters (NULL -> 0..N-1). */
static int noise_on_pairs(orc_ctx *c, int64_t step, const pair_list *L, const uint32_t *ids,
                          int w0, int w1, double *FR)
{
    const orc_params *p = &c->p;
    const int64_t n3 = 3 * p->n;
    memset(FR, 0, (size_t)n3 * sizeof(double));
    c->last_iters = 0;
    if (p->kT == 0.0) return ORC_OK;
    const int nw = w1 - w0;
    double *What = (double *)malloc((size_t)nw * n3 * sizeof(double));
    double *X = (double *)malloc((size_t)nw * n3 * sizeof(double));
    if (!What || !X) { free(What); free(X); return ORC_ERR_OOM; }
    window_dft(c, step, ids, w0, w1, What);
    int rc = ORC_OK, maxit = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < nw; ++w) {
        double *khp = (double *)malloc((size_t)(L->n ? L->n : 1) * sizeof(double));
        double *dkh = c->DKs_hat ? (double *)malloc((size_t)(L->n ? L->n : 1) * sizeof(double)) : NULL;
        for (int64_t k = 0; k < L->n; ++k) khp[k] = kp_hat_at(c, L->v[k].r, w0 + w);
        if (dkh)
            for (int64_t k = 0; k < L->n; ++k) dkh[k] = dks_hat_at(c, L->v[k].r, w0 + w);
        int it = 0;
        int r1 = lanczos_sqrt(c, w0 + w, L, khp, dkh, What + (size_t)w * n3, X + (size_t)w * n3, &it);
        free(khp);
        free(dkh);
#pragma omp critical
        {
            if (r1 && !rc) rc = r1;
            if (it > maxit) maxit = it;
        }
    }
    /* F_n = (1/P) (F_hat_0 + 2 sum_{w>=1} F_hat_w), summed in a fixed order */
    for (int w = 0; w < nw; ++w) {
        const double wt = ((w0 + w) == 0 ? 1.0 : 2.0) / (double)c->P;
        const double *xw = X + (size_t)w * n3;
        for (int64_t I = 0; I < n3; ++I) FR[I] += wt * xw[I];
    }
    c->last_iters = maxit;
    free(What); free(X);
    return rc;
}

int orc_noise(orc_ctx *c, int64_t step, const double *R, const uint32_t *ids, int w0, int w1, double *FR)
{
    if (w0 < 0 || w1 > c->M || w0 >= w1) return ORC_ERR_INVALID;
    pair_list L = {0, 0, NULL};
    int rc = find_pairs(&c->p, R, &L);
    if (!rc) rc = noise_on_pairs(c, step, &L, ids, w0, w1, FR);
    free(L.v);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Dense reference for tiny systems                                          */
/* ------------------------------------------------------------------------ */

/* cyclic Jacobi eigenvalue method for a symmetric n x n matrix A (destroyed):
 * eigenvalues in lam, eigenvectors as columns of Z. */
static void jacobi_eig(int n, double *A, double *lam, double *Z)
{
    for (int i = 0; i < n * n; ++i) Z[i] = 0.0;
    for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int pp = 0; pp < n - 1; ++pp)
            for (int q = pp + 1; q < n; ++q) {
                const double apq = A[pp * n + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * n + q] - A[pp * n + pp]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) { /* columns pp, q */
                    const double akp = A[k * n + pp], akq = A[k * n + q];
                    A[k * n + pp] = cs * akp - sn * akq;
                    A[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) { /* rows pp, q */
                    const double apk = A[pp * n + k], aqk = A[q * n + k];
                    A[pp * n + k] = cs * apk - sn * aqk;
                    A[q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double zkp = Z[k * n + pp], zkq = Z[k * n + q];
                    Z[k * n + pp] = cs * zkp - sn * zkq;
                    Z[k * n + q] = sn * zkp + cs * zkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

/* Dense 3N x 3N correlation matrix of lag m (eq. correlation_matrix):
 * K_m = c^s_m 1 on diagonal blocks and c^p_m(R_ij) T_ij off the diagonal. */
int orc_corr_matrix(const orc_ctx *c, const double *R, int m, double *K)
{
    const orc_params *p = &c->p;
    const int64_t n3 = 3 * p->n;
    if (m < 0 || m >= c->M) return ORC_ERR_INVALID;
    memset(K, 0, (size_t)n3 * n3 * sizeof(double));
    for (int64_t I = 0; I < n3; ++I) K[I * n3 + I] = corr_coef(p, p->k_self[m], m);
    pair_list L = {0, 0, NULL};
    int rc = pairs_brute(p, R, &L);
    if (rc) { free(L.v); return rc; }
    for (int64_t k = 0; k < L.n; ++k) {
        const orc_pair *q = &L.v[k];
        const double cp = corr_coef(p, kpair_at(p, q->r, m), m);
        const double cs = corr_coef(p, dks_at(p, q->r, m), m);
        for (int b = 0; b < 3; ++b) {
            double e[3] = {0, 0, 0}, col[3] = {0, 0, 0}, dcol[3] = {0, 0, 0};
            e[b] = 1.0;
            apply_tensor(p, q, cp, e, col);
            apply_tensor(p, q, cs, e, dcol);
            for (int a = 0; a < 3; ++a) {
                K[(3 * q->i + a) * n3 + 3 * q->j + b] = col[a];
                K[(3 * q->i + a) * n3 + 3 * q->i + b] += dcol[a];
            }
        }
    }
    free(L.v);
    return ORC_OK;
}

/* Dense spectral matrix K_hat_w (3N x 3N) from the pair list */
static int dense_khat(const orc_ctx *c, const pair_list *L, int w, double *K)
{
    const int64_t n3 = 3 * c->p.n;
    memset(K, 0, (size_t)n3 * n3 * sizeof(double));
    for (int64_t I = 0; I < n3; ++I) K[I * n3 + I] = c->S_hat[w];
    for (int64_t k = 0; k < L->n; ++k) {
        const orc_pair *q = &L->v[k];
        const double kp = kp_hat_at(c, q->r, w), ds = dks_hat_at(c, q->r, w);
        for (int b = 0; b < 3; ++b) {
            double e[3] = {0, 0, 0}, col[3] = {0, 0, 0}, dcol[3] = {0, 0, 0};
            e[b] = 1.0;
            apply_tensor(&c->p, q, kp, e, col);
            apply_tensor(&c->p, q, ds, e, dcol);
            for (int a = 0; a < 3; ++a) {
                K[(3 * q->i + a) * n3 + 3 * q->j + b] = col[a];
                K[(3 * q->i + a) * n3 + 3 * q->i + b] += dcol[a];
            }
        }
    }
    return ORC_OK;
}

/* sqrt(K_hat_w) for every w (dense, tiny N); returns NOT_PD on a
 * non-positive eigenvalue. Out: Ahat[w][3N][3N]. Also the smallest
 * eigenvalue over all w in *lam_min. */
int orc_dense_sqrt_spectra(const orc_ctx *c, const double *R, double *Ahat, double *lam_min)
{
    const int64_t n3 = 3 * c->p.n;
    pair_list L = {0, 0, NULL};
    int rc = pairs_brute(&c->p, R, &L);
    if (rc) { free(L.v); return rc; }
    double *K = (double *)malloc((size_t)n3 * n3 * sizeof(double));
    double *Z = (double *)malloc((size_t)n3 * n3 * sizeof(double));
    double *lam = (double *)malloc((size_t)n3 * sizeof(double));
    double lmin = INFINITY;
    for (int w = 0; w < c->M && rc == ORC_OK; ++w) {
        dense_khat(c, &L, w, K);
        jacobi_eig((int)n3, K, lam, Z);
        double *A = Ahat + (size_t)w * n3 * n3;
        for (int64_t I = 0; I < n3; ++I) {
            if (lam[I] < lmin) lmin = lam[I];
            if (!(lam[I] > 0.0)) rc = ORC_ERR_NOT_PD;
        }
        if (rc) break;
        for (int64_t I = 0; I < n3; ++I)
            for (int64_t J = 0; J < n3; ++J) {
                double s = 0.0;
                for (int64_t q = 0; q < n3; ++q) s += Z[I * n3 + q] * sqrt(lam[q]) * Z[J * n3 + q];
                A[I * n3 + J] = s;
            }
    }
    *lam_min = lmin;
    free(K); free(Z); free(lam); free(L.v);
    return rc;
}

/* Dense colored noise in the frequency domain:
 * F_n = (1/P) (sqrt(K_0) W_hat_0 + 2 sum_{w>=1} sqrt(K_w) Re W_hat_w). */
int orc_noise_dense_freq(orc_ctx *c, int64_t step, const double *R, double *FR)
{
    const int64_t n3 = 3 * c->p.n;
    const int M = c->M;
    double *Ahat = (double *)malloc((size_t)M * n3 * n3 * sizeof(double));
    double *What = (double *)malloc((size_t)M * n3 * sizeof(double));
    double lmin;
    int rc = orc_dense_sqrt_spectra(c, R, Ahat, &lmin);
    if (!rc) {
        window_dft(c, step, NULL, 0, M, What);
        memset(FR, 0, (size_t)n3 * sizeof(double));
        for (int w = 0; w < M; ++w) {
            const double wt = (w == 0 ? 1.0 : 2.0) / (double)c->P;
            const double *A = Ahat + (size_t)w * n3 * n3;
            for (int64_t I = 0; I < n3; ++I) {
                double s = 0.0;
                for (int64_t J = 0; J < n3; ++J) s += A[I * n3 + J] * What[(size_t)w * n3 + J];
                FR[I] += wt * s;
            }
        }
    }
    free(Ahat); free(What);
    return rc;
}

/* Time-domain filter matrices of eq. (noise_ansatz)/(noise_production):
 * A_s = (1/P) sum_{w=-(M-1)}^{M-1} sqrt(K_hat_|w|) cos(2 pi w s / P),
 * s = -(M-1)..M-1, stored at As[(s + M - 1)][3N][3N]. */
int orc_dense_filters(orc_ctx *c, const double *R, double *As)
{
    const int64_t n3 = 3 * c->p.n;
    const int M = c->M, P = c->P;
    double *Ahat = (double *)malloc((size_t)M * n3 * n3 * sizeof(double));
    double lmin;
    int rc = orc_dense_sqrt_spectra(c, R, Ahat, &lmin);
    if (!rc) {
        const double two_pi = 6.283185307179586476925286766559;
        for (int s = -(M - 1); s <= M - 1; ++s) {
            double *A = As + (size_t)(s + M - 1) * n3 * n3;
            memset(A, 0, (size_t)n3 * n3 * sizeof(double));
            for (int w = -(M - 1); w <= M - 1; ++w) {
                const int64_t ph = (((int64_t)w * s) % P + P) % P;
                const double cw = cos(two_pi * (double)ph / (double)P) / (double)P;
                const double *Aw = Ahat + (size_t)abs(w) * n3 * n3;
                for (int64_t k = 0; k < n3 * n3; ++k) A[k] += cw * Aw[k];
            }
        }
    }
    free(Ahat);
    return rc;
}

/* Colored noise from the literal time-domain sum of eq. (noise_production):
 * F_n = sum_s A_s W_{n+s}. */
int orc_noise_dense_time(orc_ctx *c, int64_t step, const double *R, double *FR)
{
    const int64_t N = c->p.n, n3 = 3 * N;
    const int M = c->M;
    double *As = (double *)malloc((size_t)(2 * M - 1) * n3 * n3 * sizeof(double));
    int rc = orc_dense_filters(c, R, As);
    if (!rc) {
        memset(FR, 0, (size_t)n3 * sizeof(double));
        double *Wv = (double *)malloc((size_t)n3 * sizeof(double));
        for (int s = -(M - 1); s <= M - 1; ++s) {
            for (int64_t i = 0; i < N; ++i) orc_gauss3(c->p.seed, (uint32_t)i, step + s, Wv + 3 * i);
            const double *A = As + (size_t)(s + M - 1) * n3 * n3;
            for (int64_t I = 0; I < n3; ++I) {
                double acc = 0.0;
                for (int64_t J = 0; J < n3; ++J) acc += A[I * n3 + J] * Wv[J];
                FR[I] += acc;
            }
        }
        free(Wv);
    }
    free(As);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Forces for a subset of rows, by brute-force neighbour search (used to     */
/* check very large systems on sampled particles).                           */
/* ------------------------------------------------------------------------ */

int orc_forces_rows(const orc_ctx *c, const double *R, const double *V, const double *hist,
                    const int64_t *rows, int64_t nrows, double *FC, double *FD)
{
    const orc_params *p = &c->p;
    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t i = rows[k];
        pair_list L = {0, 0, NULL};
        for (int64_t j = 0; j < p->n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, R + 3 * i, R + 3 * j, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r < p->r_cut) push_pair(&L, i, j, d, r);
        }
        double fc[3] = {0, 0, 0};
        for (int64_t q = 0; q < L.n; ++q) {
            double u, fr;
            wca_pair(p, L.v[q].r, &u, &fr);
            for (int cc = 0; cc < 3; ++cc) fc[cc] += fr * L.v[q].d[cc];
        }
        memcpy(FC + 3 * k, fc, sizeof(fc));
        if (FD) dissipative_row(p, i, L.v, L.n, V, hist, FD + 3 * k);
        free(L.v);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* One integrator step, eq. (GLD_integrator)                                 */
/* ------------------------------------------------------------------------ */

/* In:  R (unwrapped), V, hist = dR_{n-1..n-m_max+1} at step n.
 * Out: R, V, hist advanced to step n+1; FC, FD, FR = forces of step n.
 * Optional timings (seconds) of the dissipative force and the noise. */
int orc_step(orc_ctx *c, int64_t step, double *R, double *V, double *hist,
             double *FC, double *FD, double *FR, double *t_fd, double *t_fr)
{
    const orc_params *p = &c->p;
    const int64_t N = p->n, n3 = 3 * N;
    const int M = c->M;
    pair_list L = {0, 0, NULL};
    int rc = find_pairs(p, R, &L);
    if (rc) { free(L.v); return rc; }
    wca_forces(p, &L, FC);
#ifdef _OPENMP
    double t0 = omp_get_wtime();
#endif
    dissipative(p, &L, V, hist, FD);
#ifdef _OPENMP
    double t1 = omp_get_wtime();
    if (t_fd) *t_fd = t1 - t0;
#endif
    rc = noise_on_pairs(c, step, &L, NULL, 0, M, FR);
#ifdef _OPENMP
    if (t_fr) *t_fr = omp_get_wtime() - t1;
#endif
    free(L.v);
    if (rc) return rc;

    double a, b;
    orc_ab(p, &a, &b);
    const double dt = p->dt, Ms = p->mass;
    double *Rn = (double *)malloc((size_t)n3 * sizeof(double));
    double *FCn = (double *)malloc((size_t)n3 * sizeof(double));
    for (int64_t I = 0; I < n3; ++I)
        Rn[I] = R[I] + dt * b * V[I] + dt * dt / (2.0 * Ms) * b * (FC[I] + FD[I] + FR[I]);
    /* history: lag m+1 <- lag m, newest displacement at lag 1 */
    if (M > 2) memmove(hist + n3, hist, (size_t)(M - 2) * n3 * sizeof(double));
    if (M > 1)
        for (int64_t I = 0; I < n3; ++I) hist[I] = Rn[I] - R[I];
    pair_list L2 = {0, 0, NULL};
    rc = find_pairs(p, Rn, &L2);
    if (!rc) {
        wca_forces(p, &L2, FCn);
        for (int64_t I = 0; I < n3; ++I)
            V[I] = a * V[I] + dt / (2.0 * Ms) * (a * FC[I] + FCn[I]) + dt / Ms * b * (FD[I] + FR[I]);
        memcpy(R, Rn, (size_t)n3 * sizeof(double));
    }
    free(L2.v); free(Rn); free(FCn);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the OpenMP loops (timing on one core); n <= 0 leaves them */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
