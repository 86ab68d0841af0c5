/*
 * mdpd_oracle.c -- plain FP64 CPU reference of one many-body DPD (mDPD)
 * timestep, used ONLY as test infrastructure: the parity tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it.  The GPU library
 * never links, includes or calls anything in this directory, and this file
 * shares no code, header, table or constant with the GPU library.
 *
 * Everything here is written for clarity, not speed: O(N^2) brute-force pair
 * search (the definition), plus an independently written naive linked-cell
 * search that must return exactly the same neighbour lists (so exactly the
 * same sums), used for large systems.  Neighbours of particle i are always
 * visited in increasing index order, so every per-particle sum has one fixed
 * order regardless of search mode or thread count.
 *
 * What it computes follows the paper (Xia et al., "A GPU-accelerated package
 * for simulation of flow in nanoporous source rocks with many-body
 * dissipative particle dynamics"):
 *   - pair forces F = F^C + F^D + F^R, dissipative and random parts with the
 *     fluctuation-dissipation relation sigma^2 = 2 gamma kT, w^D = (w^R)^2,
 *     w^R = w^C = 1 - r/r_c                                  (Sec. 2.1)
 *   - mDPD conservative force A w^C rhat + B (rho_i + rho_j) w_d rhat with
 *     w_d = 1 - r/r_d, r_d < r_c                              (Sec. 2.1, Eq. 1)
 *   - many-body density rho_i = sum_{j != i} w_rho(r_ij),
 *     w_rho = 15/(2 pi r_d^3) (1 - r/r_d)^2, normalised so that the integral
 *     of 4 pi r^2 w_rho over r is one                        (Sec. 2.1)
 *   - velocity-Verlet in the order x(t+dt), phi, rho, f(t+dt), v(t+dt)
 *                                                             (Sec. 3.2, Alg. 1)
 *   - wall treatment: boundary volume fraction phi of a fluid particle from
 *     local frozen (wall) particles and a predictor-corrector that rejects
 *     a predicted position that penetrates the wall          (Sec. 2.2, 3.2)
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   R1  xi_ij = theta_ij / sqrt(dt), theta uniform on [-sqrt3, sqrt3] (zero
 *       mean, unit variance), drawn from Threefry-2x32-20 (Salmon et al.,
 *       SC'11) with key (seed, step) and counter (min(i,j), max(i,j)).
 *   R2  The dissipative force uses the half-step velocity of the standard
 *       velocity-Verlet loop; frozen particles have v = 0.
 *   R3  Cutoffs are strict (r < r_c, r < r_d); a coincident pair (r = 0)
 *       contributes w_rho(0) to the density and no pair force.
 *   R4  phi_i = sum_{frozen j, r<r_c} w_c^2 / sum_{j != i, r<r_c} w_c^2;
 *       if phi_i(x*) > phi_c the predicted step is rejected: x* <- x(t),
 *       v_half <- -v_half (bounce-back, no-slip) when wall_slip = 0; for
 *       wall_slip > 0 v_half is reflected about the unit wall normal
 *       n = unit(sum_{frozen j, r<r_c} w_c^2 (x_i - x_j)/r) at x*: normal
 *       part negated, tangential part times (2 wall_slip - 1); a zero normal
 *       sum, and a particle that was also sent back in the step before, fall
 *       back to bounce-back (it leaves the wall the way it came).
 *   R5  Mass m; body force acts on fluid as m*g.
 *   R6  Control of the effective fluid-solid dissipation (Sec. 2.2), on when
 *       diss_ctrl = eta > 0: for fluid i, the dissipative weight it gets from
 *       the solid, E_i = sum_{frozen j, r<r_c} w^D(r_ij), is measured and
 *       brought to the target T_i = eta rho_f W_D phi_i, the weight that
 *       fluid of number density rho_f (diss_rho) would give from the share
 *       phi_i (R4) of i's interaction sphere that the solid fills, with
 *       W_D = integral of w^D over the sphere = 2 pi r_c^3 / 15.  Each
 *       fluid-solid pair of i then dissipates with gamma s_i and fluctuates
 *       with sigma sqrt(s_i), s_i = T_i / E_i (sigma^2 = 2 gamma kT holds
 *       per pair); fluid-fluid pairs keep gamma.  eta = 1 makes the solid as
 *       dissipative as fluid at rest in its place (no slip); a smaller eta
 *       lets the fluid slip.  diss_ctrl = 0: s_i = 1.
 * parity pinned: every function here is checked by tests/test_oracle_pins.py,
 * tests/test_oracle_pins_phi_profile.py (boundary volume fraction and bin
 * profiles) and tests/test_oracle_tangent.py against known-answer vectors,
 * closed forms, conservation laws and the equations of state the paper
 * prints.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXT 8

typedef struct {
    double L[3];
    double rc, rd, kT, dt, mass;
    double g[3];
    double phi_c;
    double wall_slip;   /* corrector reflection: 0 bounce-back .. 1 specular */
    double A[ORC_MAXT * ORC_MAXT];
    double B[ORC_MAXT * ORC_MAXT];
    double gamma[ORC_MAXT * ORC_MAXT];
    uint32_t seed;
    int32_t ntypes;
    int32_t wall_model; /* 0: no wall treatment, 1: phi + predictor-corrector */
    int32_t search;     /* 0: brute force O(N^2), 1: naive linked cells   */
    double diss_ctrl;   /* reading R6: eta (0: no dissipation control)    */
    double diss_rho;    /* reading R6: the fluid number density rho_f     */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Threefry-2x32 with 20 rounds (Salmon, Moraes, Dror, Shaw, SC'11).         */
/* Key schedule: ks2 = 0x1BD11BDA ^ k0 ^ k1; key injection after every four  */
/* rounds adds ks[s%3], ks[(s+1)%3] and the injection counter s.             */
/* ------------------------------------------------------------------------ */
static uint32_t orc_rotl32(uint32_t x, unsigned r) { return (x << r) | (x >> (32u - r)); }

void orc_threefry2x32_20(const uint32_t ctr[2], const uint32_t key[2], uint32_t out[2])
{
    static const unsigned rot[8] = {13, 15, 26, 6, 17, 29, 16, 24};
    uint32_t ks[3];
    ks[0] = key[0];
    ks[1] = key[1];
    ks[2] = 0x1BD11BDAu ^ key[0] ^ key[1];
    uint32_t x0 = ctr[0] + ks[0];
    uint32_t x1 = ctr[1] + ks[1];
    for (int r = 0; r < 20; ++r) {
        x0 += x1;
        x1 = orc_rotl32(x1, rot[r % 8]);
        x1 ^= x0;
        if (r % 4 == 3) {
            uint32_t s = (uint32_t)(r / 4 + 1);
            x0 += ks[s % 3];
            x1 += ks[(s + 1) % 3] + s;
        }
    }
    out[0] = x0;
    out[1] = x1;
}

/* theta_ij: the first output word of Threefry with key (seed, step) and
 * counter (min id, max id); its top 24 bits k give the odd-centred uniform
 * t = (2k + 1 - 2^24) / 2^24 in (-1, 1), exact in binary, and
 * theta = sqrt(3) * t has zero mean and unit variance (reading R1). */
double orc_theta(uint32_t seed, uint32_t step, uint32_t i, uint32_t j)
{
    uint32_t ctr[2], key[2], out[2];
    ctr[0] = i < j ? i : j;
    ctr[1] = i < j ? j : i;
    key[0] = seed;
    key[1] = step;
    orc_threefry2x32_20(ctr, key, out);
    double k = (double)(out[0] >> 8);
    double t = (2.0 * k + 1.0 - 16777216.0) / 16777216.0;
    return sqrt(3.0) * t;
}

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA'14) used as the
 * element mixer of an order-independent neighbour-set hash. */
uint64_t orc_mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Geometry: minimum image by branch, squared distance without contraction. */
/* ------------------------------------------------------------------------ */
static double orc_min_image(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

static void orc_delta(const double *x, int64_t i, int64_t j, const double L[3], double d[3])
{
    for (int a = 0; a < 3; ++a) d[a] = orc_min_image(x[3 * i + a] - x[3 * j + a], L[a]);
}

static double orc_r2(const double d[3])
{
    double s = d[0] * d[0];
    s = s + d[1] * d[1];
    s = s + d[2] * d[2];
    return s;
}

/* Wrap one coordinate that lies in [-L, 2L) into [0, L). */
double orc_wrap(double x, double L)
{
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

/* Normalised many-body density weight (Sec. 2.1): 15/(2 pi r_d^3)(1-r/r_d)^2
 * for r < r_d, zero beyond. */
double orc_w_rho(double r, double rd)
{
    if (r >= rd) return 0.0;
    double u = 1.0 - r / rd;
    return 15.0 / (2.0 * M_PI * rd * rd * rd) * u * u;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists: for every i, all j != i with r_ij^2 < cutoff^2, in     */
/* increasing j.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int32_t *cnt;
    int32_t **idx;
} orc_nlist;

static void orc_nlist_free(orc_nlist *nl)
{
    if (!nl->idx) return;
    for (int64_t i = 0; i < nl->n; ++i) free(nl->idx[i]);
    free(nl->idx);
    free(nl->cnt);
    nl->idx = NULL;
    nl->cnt = NULL;
}

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void orc_push(int32_t **buf, int32_t *cap, int32_t *len, int32_t v)
{
    if (*len == *cap) {
        *cap = *cap ? 2 * *cap : 64;
        *buf = (int32_t *)realloc(*buf, (size_t)*cap * sizeof(int32_t));
    }
    (*buf)[(*len)++] = v;
}

static void orc_build_bruteforce(const double *x, int64_t n, const double L[3], double cut2,
                                 orc_nlist *nl)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int32_t *buf = NULL, cap = 0, len = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            orc_delta(x, i, j, L, d);
            if (orc_r2(d) < cut2) orc_push(&buf, &cap, &len, (int32_t)j);
        }
        nl->cnt[i] = len;
        nl->idx[i] = buf;
    }
}

/* Naive linked cells: cells no smaller than the cutoff (with a relative
 * margin far above rounding), 27-cell stencil, hits sorted by index so the
 * lists equal the brute-force ones. */
static int orc_build_cells(const double *x, int64_t n, const double L[3], double cutoff,
                           double cut2, orc_nlist *nl)
{
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int)floor(L[a] / (cutoff * (1.0 + 1e-10)));
        if (nc[a] < 3) return 0;
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    int64_t *next = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    int32_t *cell = (int32_t *)malloc((size_t)(n ? n : 1) * 3 * sizeof(int32_t));
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        int c3[3];
        for (int a = 0; a < 3; ++a) {
            int c = (int)floor(x[3 * i + a] / (L[a] / nc[a]));
            if (c < 0) c = 0;
            if (c >= nc[a]) c = nc[a] - 1;
            c3[a] = c;
            cell[3 * i + a] = c;
        }
        int64_t lin = c3[0] + (int64_t)nc[0] * (c3[1] + (int64_t)nc[1] * c3[2]);
        next[i] = head[lin];
        head[lin] = i;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int32_t *buf = NULL, cap = 0, len = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int cx = (cell[3 * i] + dx + nc[0]) % nc[0];
                    int cy = (cell[3 * i + 1] + dy + nc[1]) % nc[1];
                    int cz = (cell[3 * i + 2] + dz + nc[2]) % nc[2];
                    int64_t lin = cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
                    for (int64_t j = head[lin]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double d[3];
                        orc_delta(x, i, j, L, d);
                        if (orc_r2(d) < cut2) orc_push(&buf, &cap, &len, (int32_t)j);
                    }
                }
        if (len > 1) qsort(buf, (size_t)len, sizeof(int32_t), orc_cmp_i32);
        nl->cnt[i] = len;
        nl->idx[i] = buf;
    }
    free(head);
    free(next);
    free(cell);
    return 1;
}

static void orc_build(const double *x, int64_t n, const double L[3], double cutoff, int search,
                      orc_nlist *nl)
{
    nl->n = n;
    nl->cnt = (int32_t *)calloc((size_t)(n ? n : 1), sizeof(int32_t));
    nl->idx = (int32_t **)calloc((size_t)(n ? n : 1), sizeof(int32_t *));
    double cut2 = cutoff * cutoff;
    if (search == 1 && orc_build_cells(x, n, L, cutoff, cut2, nl)) return;
    orc_build_bruteforce(x, n, L, cut2, nl);
}

/* Per-particle neighbour count and order-independent set hash
 * (sum over j of mix64(j), modulo 2^64). */
void orc_neighbors(const orc_params *p, int64_t n, const double *x, double cutoff,
                   int64_t *count, uint64_t *hash)
{
    orc_nlist nl;
    orc_build(x, n, p->L, cutoff, p->search, &nl);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t h = 0;
        for (int32_t k = 0; k < nl.cnt[i]; ++k) h += orc_mix64((uint64_t)nl.idx[i][k]);
        count[i] = nl.cnt[i];
        hash[i] = h;
    }
    orc_nlist_free(&nl);
}

/* ------------------------------------------------------------------------ */
/* Many-body density (Sec. 2.1) for every particle, fluid and frozen alike */
/* (Alg. 1 computes rho for all local particles).                          */
/* ------------------------------------------------------------------------ */
static void orc_density_nl(const orc_params *p, int64_t n, const double *x, const orc_nlist *nl,
                           double *rho)
{
    double rd2 = p->rd * p->rd;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < nl->cnt[i]; ++k) {
            int64_t j = nl->idx[i][k];
            double d[3];
            orc_delta(x, i, j, p->L, d);
            double r2 = orc_r2(d);
            if (r2 < rd2) s += orc_w_rho(sqrt(r2), p->rd);
        }
        rho[i] = s;
    }
}

void orc_density(const orc_params *p, int64_t n, const double *x, double *rho)
{
    orc_nlist nl;
    orc_build(x, n, p->L, p->rc, p->search, &nl);
    orc_density_nl(p, n, x, &nl, rho);
    orc_nlist_free(&nl);
}

/* Boundary volume fraction of fluid particles (reading R4); frozen: 0. */
static void orc_phi_nl(const orc_params *p, int64_t n, const double *x, const uint8_t *frozen,
                       const orc_nlist *nl, double *phi)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (frozen[i]) {
            phi[i] = 0.0;
            continue;
        }
        double num = 0.0, den = 0.0;
        for (int32_t k = 0; k < nl->cnt[i]; ++k) {
            int64_t j = nl->idx[i][k];
            double d[3];
            orc_delta(x, i, j, p->L, d);
            double w = 1.0 - sqrt(orc_r2(d)) / p->rc;
            den += w * w;
            if (frozen[j]) num += w * w;
        }
        phi[i] = den > 0.0 ? num / den : 0.0;
    }
}

/* Wall normal of fluid particle i at positions x (Sec. 2.2, reading R4):
 * the w_c^2-weighted sum of the unit vectors from its frozen neighbours
 * within r_c to it, normalised; returns 0 when that sum is zero. */
static int orc_wall_normal(const orc_params *p, const double *x, const uint8_t *frozen,
                           const orc_nlist *nl, int64_t i, double nrm[3])
{
    double s[3] = {0.0, 0.0, 0.0};
    for (int32_t k = 0; k < nl->cnt[i]; ++k) {
        int64_t j = nl->idx[i][k];
        if (!frozen[j]) continue;
        double d[3];
        orc_delta(x, i, j, p->L, d);
        double r = sqrt(orc_r2(d));
        if (r == 0.0) continue;
        double w = 1.0 - r / p->rc;
        for (int a = 0; a < 3; ++a) s[a] += w * w * d[a] / r;
    }
    double len = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (!(len > 0.0)) return 0;
    for (int a = 0; a < 3; ++a) nrm[a] = s[a] / len;
    return 1;
}

void orc_phi(const orc_params *p, int64_t n, const double *x, const uint8_t *frozen, double *phi)
{
    orc_nlist nl;
    orc_build(x, n, p->L, p->rc, p->search, &nl);
    orc_phi_nl(p, n, x, frozen, &nl, phi);
    orc_nlist_free(&nl);
}

/* Dissipation control (reading R6): the factor s_i of the fluid-solid pairs
 * of every fluid particle i; 1 for frozen particles, for fluid without a
 * frozen neighbour and when the control is off.  phi: scratch of n. */
static void orc_diss_scale_nl(const orc_params *p, int64_t n, const double *x, const uint8_t *frozen,
                              const orc_nlist *nl, double *phi, double *s)
{
    const double WD = 2.0 * M_PI * p->rc * p->rc * p->rc / 15.0;
    orc_phi_nl(p, n, x, frozen, nl, phi);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        s[i] = 1.0;
        if (frozen[i] || !(p->diss_ctrl > 0.0)) continue;
        double E = 0.0;
        for (int32_t k = 0; k < nl->cnt[i]; ++k) {
            int64_t j = nl->idx[i][k];
            if (!frozen[j]) continue;
            double d[3];
            orc_delta(x, i, j, p->L, d);
            double w = 1.0 - sqrt(orc_r2(d)) / p->rc;
            E += w * w;
        }
        if (E > 0.0) s[i] = p->diss_ctrl * p->diss_rho * WD * phi[i] / E;
    }
}

void orc_diss_scale(const orc_params *p, int64_t n, const double *x, const uint8_t *frozen, double *s)
{
    orc_nlist nl;
    orc_build(x, n, p->L, p->rc, p->search, &nl);
    double *phi = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
    orc_diss_scale_nl(p, n, x, frozen, &nl, phi, s);
    free(phi);
    orc_nlist_free(&nl);
}

/* ------------------------------------------------------------------------ */
/* Pair forces (Sec. 2.1, Eq. 1) on every fluid particle; frozen: 0.        */
/* virial = sum over fluid i, j in N_c(i) of c_ij r_ij F^C_ij, c_ij = 1/2   */
/* if j is fluid (pair seen from both sides) and 1 if j is frozen; epair is */
/* the same weighted sum of the A-term pair potential (A r_c / 2) w_c^2.    */
/* dsc: the dissipation-control factors s_i of reading R6 (NULL: none).     */
/* ------------------------------------------------------------------------ */
static void orc_forces_nl(const orc_params *p, int64_t n, const double *x, const double *vh,
                          const int32_t *type, const uint8_t *frozen, const double *rho,
                          uint32_t step, const orc_nlist *nl, const double *dsc, double *F,
                          double *virial, double *epair)
{
    const int T = p->ntypes;
    const double rc = p->rc, rd = p->rd, rd2 = rd * rd;
    const double m = p->mass;
    double vir = 0.0, ep = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : vir, ep)
    for (int64_t i = 0; i < n; ++i) {
        if (frozen[i]) {
            F[3 * i] = F[3 * i + 1] = F[3 * i + 2] = 0.0;
            continue;
        }
        double f[3] = {0.0, 0.0, 0.0};
        double vir_i = 0.0, ep_i = 0.0;
        for (int32_t k = 0; k < nl->cnt[i]; ++k) {
            int64_t j = nl->idx[i][k];
            double d[3];
            orc_delta(x, i, j, p->L, d);
            double r2 = orc_r2(d);
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double e[3] = {d[0] / r, d[1] / r, d[2] / r};
            int tt = type[i] * T + type[j];
            double wc = 1.0 - r / rc;
            /* conservative, Eq. 1 */
            double fc = p->A[tt] * wc;
            if (r2 < rd2) fc += p->B[tt] * (rho[i] + rho[j]) * (1.0 - r / rd);
            /* dissipative: -gamma w^D (rhat . v_ij), w^D = wc^2 */
            double vj[3] = {0.0, 0.0, 0.0};
            if (!frozen[j])
                for (int a = 0; a < 3; ++a) vj[a] = vh[3 * j + a];
            double ev = e[0] * (vh[3 * i] - vj[0]) + e[1] * (vh[3 * i + 1] - vj[1]) +
                        e[2] * (vh[3 * i + 2] - vj[2]);
            double fd = -p->gamma[tt] * wc * wc * ev;
            /* random: sigma w^R xi, sigma^2 = 2 gamma kT, xi = theta / sqrt(dt) */
            double sigma = sqrt(2.0 * p->gamma[tt] * p->kT);
            double fr = sigma * wc * orc_theta(p->seed, step, (uint32_t)i, (uint32_t)j) / sqrt(p->dt);
            if (dsc && frozen[j]) {
                /* reading R6: gamma s_i and sigma sqrt(s_i) for a fluid-solid pair */
                fd *= dsc[i];
                fr *= sqrt(dsc[i]);
            }
            double fs = fc + fd + fr;
            for (int a = 0; a < 3; ++a) f[a] += fs * e[a];
            double c = frozen[j] ? 1.0 : 0.5;
            vir_i += c * r * fc;
            ep_i += c * 0.5 * p->A[tt] * rc * wc * wc;
        }
        for (int a = 0; a < 3; ++a) F[3 * i + a] = f[a] + m * p->g[a];
        vir += vir_i;
        ep += ep_i;
    }
    if (virial) *virial = vir;
    if (epair) *epair = ep;
}

void orc_forces(const orc_params *p, int64_t n, const double *x, const double *vh,
                const int32_t *type, const uint8_t *frozen, const double *rho, uint32_t step,
                double *F, double *virial, double *epair)
{
    orc_nlist nl;
    orc_build(x, n, p->L, p->rc, p->search, &nl);
    double *dsc = NULL, *phi = NULL;
    if (p->diss_ctrl > 0.0) {
        dsc = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
        phi = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
        orc_diss_scale_nl(p, n, x, frozen, &nl, phi, dsc);
    }
    orc_forces_nl(p, n, x, vh, type, frozen, rho, step, &nl, dsc, F, virial, epair);
    free(dsc);
    free(phi);
    orc_nlist_free(&nl);
}

/* ------------------------------------------------------------------------ */
/* A whole system advanced by velocity-Verlet in the order of Alg. 1.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_params p;
    int64_t n, nfluid;
    double *x, *v, *vh, *F, *rho, *phi, *xprev, *dsc, *phi2;
    int32_t *type;
    uint8_t *frozen;
    uint8_t *rej;  /* reading R4 with wall_slip > 0: sent back in the last step */
    uint32_t step;
    int64_t ncorr_last, ncorr_total;
    double virial, epair;
} orc_system;

static void orc_eval(orc_system *s)
{
    /* rho for all particles, then forces at the current step's noise */
    orc_nlist nl;
    orc_build(s->x, s->n, s->p.L, s->p.rc, s->p.search, &nl);
    orc_density_nl(&s->p, s->n, s->x, &nl, s->rho);
    const double *dsc = NULL;
    if (s->p.diss_ctrl > 0.0) {
        orc_diss_scale_nl(&s->p, s->n, s->x, s->frozen, &nl, s->phi2, s->dsc);
        dsc = s->dsc;
    }
    orc_forces_nl(&s->p, s->n, s->x, s->vh, s->type, s->frozen, s->rho, s->step, &nl, dsc, s->F,
                  &s->virial, &s->epair);
    orc_nlist_free(&nl);
}

void orc_destroy(orc_system *s)
{
    if (!s) return;
    free(s->x);
    free(s->v);
    free(s->vh);
    free(s->F);
    free(s->rho);
    free(s->phi);
    free(s->phi2);
    free(s->dsc);
    free(s->xprev);
    free(s->type);
    free(s->frozen);
    free(s->rej);
    free(s);
}

/* Positions must lie in [-L, 2L) per axis; they are wrapped into [0, L).
 * Forces at creation use the given velocities and noise step 0. */
orc_system *orc_create(const orc_params *p, int64_t n, const double *x, const double *v,
                       const int32_t *type, const uint8_t *frozen)
{
    orc_system *s = (orc_system *)calloc(1, sizeof(orc_system));
    size_t nn = (size_t)(n ? n : 1);
    s->p = *p;
    s->n = n;
    s->x = (double *)malloc(nn * 3 * sizeof(double));
    s->v = (double *)malloc(nn * 3 * sizeof(double));
    s->vh = (double *)malloc(nn * 3 * sizeof(double));
    s->F = (double *)malloc(nn * 3 * sizeof(double));
    s->xprev = (double *)malloc(nn * 3 * sizeof(double));
    s->rho = (double *)malloc(nn * sizeof(double));
    s->phi = (double *)calloc(nn, sizeof(double));
    s->phi2 = (double *)calloc(nn, sizeof(double));
    s->dsc = (double *)calloc(nn, sizeof(double));
    s->type = (int32_t *)malloc(nn * sizeof(int32_t));
    s->frozen = (uint8_t *)malloc(nn);
    s->rej = (uint8_t *)calloc(nn, 1);
    for (int64_t i = 0; i < n; ++i) {
        s->type[i] = type[i];
        s->frozen[i] = frozen[i] ? 1 : 0;
        if (!s->frozen[i]) s->nfluid++;
        for (int a = 0; a < 3; ++a) {
            s->x[3 * i + a] = orc_wrap(x[3 * i + a], p->L[a]);
            double va = s->frozen[i] ? 0.0 : v[3 * i + a];
            s->v[3 * i + a] = va;
            s->vh[3 * i + a] = va;
        }
    }
    s->step = 0;
    orc_eval(s);
    return s;
}

/* The corrector (reading R4) for the fluid particles with phi > phi_c:
 * back to x(t), half-step velocity negated or reflected. */
static int64_t orc_correct(orc_system *s)
{
    orc_nlist nl;
    orc_build(s->x, s->n, s->p.L, s->p.rc, s->p.search, &nl);
    orc_phi_nl(&s->p, s->n, s->x, s->frozen, &nl, s->phi);
    int64_t cnt = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        const int hit = !s->frozen[i] && s->phi[i] > s->p.phi_c;
        const int again = s->rej[i];
        s->rej[i] = (uint8_t)hit;
        if (!hit) continue;
        double nrm[3];
        double *v = &s->vh[3 * i];
        if (s->p.wall_slip > 0.0 && !again && orc_wall_normal(&s->p, s->x, s->frozen, &nl, i, nrm)) {
            double vn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
            double ft = 2.0 * s->p.wall_slip - 1.0;
            for (int a = 0; a < 3; ++a) v[a] = ft * (v[a] - vn * nrm[a]) - vn * nrm[a];
        } else {
            for (int a = 0; a < 3; ++a) v[a] = -v[a];
        }
        for (int a = 0; a < 3; ++a) s->x[3 * i + a] = s->xprev[3 * i + a];
        cnt++;
    }
    orc_nlist_free(&nl);
    return cnt;
}

void orc_step(orc_system *s, int64_t nsteps)
{
    const int64_t n = s->n;
    const double hdtm = 0.5 * s->p.dt / s->p.mass;
    for (int64_t it = 0; it < nsteps; ++it) {
        /* v(t+dt/2) and predicted x(t+dt) for fluid; frozen stay put */
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) s->xprev[3 * i + a] = s->x[3 * i + a];
            if (s->frozen[i]) continue;
            for (int a = 0; a < 3; ++a) {
                s->vh[3 * i + a] = s->v[3 * i + a] + hdtm * s->F[3 * i + a];
                s->x[3 * i + a] = orc_wrap(s->x[3 * i + a] + s->p.dt * s->vh[3 * i + a], s->p.L[a]);
            }
        }
        /* phi for fluid at the predicted positions, then the corrector */
        s->ncorr_last = 0;
        if (s->p.wall_model) {
            s->ncorr_last = orc_correct(s);
            s->ncorr_total += s->ncorr_last;
        }
        /* rho, f(t+dt), v(t+dt) */
        s->step += 1;
        orc_eval(s);
        for (int64_t i = 0; i < n; ++i) {
            if (s->frozen[i]) continue;
            for (int a = 0; a < 3; ++a) s->v[3 * i + a] = s->vh[3 * i + a] + hdtm * s->F[3 * i + a];
        }
    }
}

void orc_get(const orc_system *s, double *x, double *v, double *F, double *rho, double *vh)
{
    size_t n = (size_t)s->n;
    if (x) memcpy(x, s->x, n * 3 * sizeof(double));
    if (v) memcpy(v, s->v, n * 3 * sizeof(double));
    if (F) memcpy(F, s->F, n * 3 * sizeof(double));
    if (rho) memcpy(rho, s->rho, n * sizeof(double));
    if (vh) memcpy(vh, s->vh, n * 3 * sizeof(double));
}

/* Observables at the current step:
 * out[0] step, [1] KE = m/2 sum_f |v|^2, [2] kT = 2 KE / (3 dof) with dof =
 * N_f - 1 for a periodic fluid without walls or body force (momentum is then
 * conserved) and N_f otherwise, [3] P = (sum_f m|v|^2 + virial) / (3V),
 * [4..6] momentum, [7] Epot = epair + sum_i (pi r_d^4 B_ii / 30) rho_i^2,
 * [8] mean rho over fluid, [9] corrections in the last step, [10] total
 * corrections, [11] virial. */
void orc_observables(const orc_system *s, double *out)
{
    const int64_t n = s->n;
    double ke2 = 0.0, mom[3] = {0.0, 0.0, 0.0}, rho_sum = 0.0, emb = 0.0;
    int driven = (s->p.g[0] != 0.0 || s->p.g[1] != 0.0 || s->p.g[2] != 0.0);
    for (int64_t i = 0; i < n; ++i) {
        int t = s->type[i];
        double B = s->p.B[t * s->p.ntypes + t];
        emb += M_PI * pow(s->p.rd, 4) * B / 30.0 * s->rho[i] * s->rho[i];
        if (s->frozen[i]) continue;
        for (int a = 0; a < 3; ++a) {
            ke2 += s->p.mass * s->v[3 * i + a] * s->v[3 * i + a];
            mom[a] += s->p.mass * s->v[3 * i + a];
        }
        rho_sum += s->rho[i];
    }
    double dof = (double)s->nfluid;
    if (s->nfluid == n && !driven) dof -= 1.0;
    double V = s->p.L[0] * s->p.L[1] * s->p.L[2];
    out[0] = (double)s->step;
    out[1] = 0.5 * ke2;
    out[2] = dof > 0 ? ke2 / (3.0 * dof) : 0.0;
    out[3] = (ke2 + s->virial) / (3.0 * V);
    out[4] = mom[0];
    out[5] = mom[1];
    out[6] = mom[2];
    out[7] = s->epair + emb;
    out[8] = s->nfluid ? rho_sum / (double)s->nfluid : 0.0;
    out[9] = (double)s->ncorr_last;
    out[10] = (double)s->ncorr_total;
    out[11] = s->virial;
}

/* Bin profiles of fluid particles along one axis (bins of L/nbins).
 * quantity 0: number density; 1..3: mean velocity component x, y, z;
 * 4: kinetic temperature from velocities relative to the bin mean;
 * 5: mean many-body density.  Empty bins give 0. */
void orc_profile(const orc_system *s, int axis, int nbins, int quantity, double *out)
{
    double *cnt = (double *)calloc((size_t)nbins, sizeof(double));
    double *sv = (double *)calloc((size_t)nbins * 3, sizeof(double));
    double *acc = (double *)calloc((size_t)nbins, sizeof(double));
    double La = s->p.L[axis];
    for (int64_t i = 0; i < s->n; ++i) {
        if (s->frozen[i]) continue;
        int b = (int)floor(s->x[3 * i + axis] / La * nbins);
        if (b < 0) b = 0;
        if (b >= nbins) b = nbins - 1;
        cnt[b] += 1.0;
        for (int a = 0; a < 3; ++a) sv[3 * b + a] += s->v[3 * i + a];
        acc[b] += s->rho[i];
    }
    double vol = s->p.L[0] * s->p.L[1] * s->p.L[2] / nbins;
    if (quantity == 4) {
        double *ss = (double *)calloc((size_t)nbins, sizeof(double));
        for (int64_t i = 0; i < s->n; ++i) {
            if (s->frozen[i]) continue;
            int b = (int)floor(s->x[3 * i + axis] / La * nbins);
            if (b < 0) b = 0;
            if (b >= nbins) b = nbins - 1;
            for (int a = 0; a < 3; ++a) {
                double u = s->v[3 * i + a] - sv[3 * b + a] / cnt[b];
                ss[b] += s->p.mass * u * u;
            }
        }
        for (int b = 0; b < nbins; ++b) out[b] = cnt[b] > 0 ? ss[b] / (3.0 * cnt[b]) : 0.0;
        free(ss);
    } else {
        for (int b = 0; b < nbins; ++b) {
            if (quantity == 0)
                out[b] = cnt[b] / vol;
            else if (quantity >= 1 && quantity <= 3)
                out[b] = cnt[b] > 0 ? sv[3 * b + quantity - 1] / cnt[b] : 0.0;
            else
                out[b] = cnt[b] > 0 ? acc[b] / cnt[b] : 0.0;
        }
    }
    free(cnt);
    free(sv);
    free(acc);
}

uint32_t orc_current_step(const orc_system *s) { return s->step; }

/* theta for many (i, j) pairs at once (statistics checks). */
void orc_theta_many(uint32_t seed, uint32_t step, int64_t m, const uint32_t *i, const uint32_t *j,
                    double *out)
{
    for (int64_t k = 0; k < m; ++k) out[k] = orc_theta(seed, step, i[k], j[k]);
}

/* Number of threads the OpenMP loops above use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the OpenMP loops (ignored without OpenMP). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Forward-mode derivative (tangent) of a scalar loss of the trajectory.    */
/*                                                                          */
/* The state is advanced exactly as orc_step does (with walls, the         */
/* bounce-back corrector's decisions are taken on the state and held fixed: */
/* a corrected particle's position tangent goes back with it and its        */
/* half-step velocity tangent changes sign; wall_slip must be 0; with the   */
/* dissipation control of reading R6 the factor s_i carries its tangent     */
/* through phi_i and E_i), and next to every quantity q                     */
/* its tangent dq, the derivative along one direction in the inputs: the    */
/* initial positions and velocities (dx0, dv0, n x 3) and the pair tables   */
/* (dA, dB, dgamma, ntypes^2; dsigma = kT dgamma / sigma).  Any of them may */
/* be NULL (zero tangent).  The noise theta_ij depends only on (seed, step, */
/* ids), so it has no tangent; the wrap into [0, L) has derivative one.     */
/*                                                                          */
/* Loss of one state: l = w[0] mean_fluid(rho) + w[1] P + w[2] mean_fluid(  */
/* v_x), with P the virial pressure of orc_observables.  avg = 0: L is l of */
/* the state after nsteps; avg = 1: L is the mean of l over the states      */
/* after steps 1..nsteps (nsteps >= 1).  out[0] = L, out[1] = dL.           */
/* parity pinned against central finite differences of orc_step and        */
/* exact invariances (uniform translation, Galilean boost).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_params *p;
    int64_t n;
    const int32_t *type;
    const uint8_t *frozen;
    const double *dA, *dB, *dg;
} orc_tan_ctx;

/* rho and its tangent at positions x with tangent dx. */
static void orc_tan_density(const orc_tan_ctx *c, const double *x, const double *dx, const orc_nlist *nl,
                            double *rho, double *drho)
{
    const orc_params *p = c->p;
    const double rd = p->rd, rd2 = rd * rd, norm = 15.0 / (2.0 * M_PI * rd * rd * rd);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < c->n; ++i) {
        double s = 0.0, ds = 0.0;
        for (int32_t k = 0; k < nl->cnt[i]; ++k) {
            int64_t j = nl->idx[i][k];
            double d[3];
            orc_delta(x, i, j, p->L, d);
            double r2 = orc_r2(d);
            if (!(r2 < rd2)) continue;
            double r = sqrt(r2);
            double q = 1.0 - r / rd;
            s += norm * q * q;
            if (r2 == 0.0) continue;
            double dr = 0.0;
            for (int a = 0; a < 3; ++a) dr += d[a] / r * (dx[3 * i + a] - dx[3 * j + a]);
            ds += norm * 2.0 * q * (-dr / rd);
        }
        rho[i] = s;
        drho[i] = ds;
    }
}

/* The dissipation-control factor s_i of reading R6 and its tangent ds_i for
 * fluid particle i, from its phi_i and E_i as orc_diss_scale_nl takes them:
 * s = eta rho_f W_D phi / E with phi = E / S (S: all neighbours, E: frozen
 * ones, weights w_c^2); s = 1, ds = 0 without frozen neighbours. */
static void orc_tan_diss_scale(const orc_tan_ctx *c, const double *x, const double *dx, const orc_nlist *nl,
                               int64_t i, double *s, double *ds)
{
    const orc_params *p = c->p;
    const double K = p->diss_ctrl * p->diss_rho * 2.0 * M_PI * p->rc * p->rc * p->rc / 15.0;
    double S = 0.0, dS = 0.0, E = 0.0, dE = 0.0;
    for (int32_t k = 0; k < nl->cnt[i]; ++k) {
        int64_t j = nl->idx[i][k];
        double d[3];
        orc_delta(x, i, j, p->L, d);
        double r = sqrt(orc_r2(d));
        double w = 1.0 - r / p->rc, dw = 0.0;
        if (r > 0.0) {
            double dr = 0.0;
            for (int a = 0; a < 3; ++a) dr += d[a] / r * (dx[3 * i + a] - dx[3 * j + a]);
            dw = -dr / p->rc;
        }
        S += w * w;
        dS += 2.0 * w * dw;
        if (c->frozen[j]) {
            E += w * w;
            dE += 2.0 * w * dw;
        }
    }
    *s = 1.0;
    *ds = 0.0;
    if (!(E > 0.0)) return;
    double phi = E / S, dphi = (dE * S - E * dS) / (S * S);
    *s = K * phi / E;
    *ds = K * (dphi * E - phi * dE) / (E * E);
}

/* Forces and their tangent (fluid particles; frozen get 0), the virial and
 * its tangent. */
static void orc_tan_forces(const orc_tan_ctx *c, const double *x, const double *dx, const double *vh,
                           const double *dvh, const double *rho, const double *drho, uint32_t step,
                           const orc_nlist *nl, double *F, double *dF, double *vir_out, double *dvir_out)
{
    const orc_params *p = c->p;
    const int T = p->ntypes;
    const double rc = p->rc, rd = p->rd, rd2 = rd * rd, sdt = sqrt(p->dt);
    double vir = 0.0, dvir = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : vir, dvir)
    for (int64_t i = 0; i < c->n; ++i) {
        double f[3] = {0, 0, 0}, df[3] = {0, 0, 0};
        double si = 1.0, dsi = 0.0;
        if (!c->frozen[i] && p->diss_ctrl > 0.0) orc_tan_diss_scale(c, x, dx, nl, i, &si, &dsi);
        if (!c->frozen[i]) {
            for (int32_t k = 0; k < nl->cnt[i]; ++k) {
                int64_t j = nl->idx[i][k];
                double d[3], dd[3];
                orc_delta(x, i, j, p->L, d);
                double r2 = orc_r2(d);
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double e[3], de[3], dr = 0.0;
                for (int a = 0; a < 3; ++a) {
                    dd[a] = dx[3 * i + a] - dx[3 * j + a];
                    e[a] = d[a] / r;
                    dr += e[a] * dd[a];
                }
                for (int a = 0; a < 3; ++a) de[a] = (dd[a] - e[a] * dr) / r;
                int tt = c->type[i] * T + c->type[j];
                double A = p->A[tt], B = p->B[tt], gam = p->gamma[tt];
                double dA = c->dA ? c->dA[tt] : 0.0, dB = c->dB ? c->dB[tt] : 0.0;
                double dgam = c->dg ? c->dg[tt] : 0.0;
                double wc = 1.0 - r / rc, dwc = -dr / rc;
                /* conservative */
                double fc = A * wc, dfc = dA * wc + A * dwc;
                if (r2 < rd2) {
                    double wd = 1.0 - r / rd, dwd = -dr / rd;
                    double rs = rho[i] + rho[j], drs = drho[i] + drho[j];
                    fc += B * rs * wd;
                    dfc += dB * rs * wd + B * drs * wd + B * rs * dwd;
                }
                /* dissipative with the half-step velocities (frozen: v = 0) */
                double vij[3], dvij[3], ev = 0.0, dev = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double vj = c->frozen[j] ? 0.0 : vh[3 * j + a];
                    double dvj = c->frozen[j] ? 0.0 : dvh[3 * j + a];
                    vij[a] = vh[3 * i + a] - vj;
                    dvij[a] = dvh[3 * i + a] - dvj;
                    ev += e[a] * vij[a];
                    dev += de[a] * vij[a] + e[a] * dvij[a];
                }
                double fd = -gam * wc * wc * ev;
                double dfd = -dgam * wc * wc * ev - gam * 2.0 * wc * dwc * ev - gam * wc * wc * dev;
                /* random */
                double sigma = sqrt(2.0 * gam * p->kT);
                double dsigma = sigma > 0.0 ? p->kT * dgam / sigma : 0.0;
                double th = orc_theta(p->seed, step, (uint32_t)i, (uint32_t)j) / sdt;
                double fr = sigma * wc * th, dfr = (dsigma * wc + sigma * dwc) * th;
                if (p->diss_ctrl > 0.0 && c->frozen[j]) {
                    /* reading R6: gamma s_i, sigma sqrt(s_i) on a fluid-solid pair */
                    double rs = sqrt(si);
                    dfd = dsi * fd + si * dfd;
                    fd = si * fd;
                    dfr = dsi / (2.0 * rs) * fr + rs * dfr;
                    fr = rs * fr;
                }
                double fs = fc + fd + fr, dfs = dfc + dfd + dfr;
                for (int a = 0; a < 3; ++a) {
                    f[a] += fs * e[a];
                    df[a] += dfs * e[a] + fs * de[a];
                }
                double cw = c->frozen[j] ? 1.0 : 0.5;
                vir += cw * r * fc;
                dvir += cw * (dr * fc + r * dfc);
            }
            for (int a = 0; a < 3; ++a) f[a] += p->mass * p->g[a];
        }
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] = f[a];
            dF[3 * i + a] = df[a];
        }
    }
    *vir_out = vir;
    *dvir_out = dvir;
}

/* l and dl of one state (see above). */
static void orc_tan_loss(const orc_tan_ctx *c, const double *v, const double *dv, const double *rho,
                         const double *drho, double vir, double dvir, const double w[3], double *l,
                         double *dl)
{
    const orc_params *p = c->p;
    double nf = 0.0, sr = 0.0, dsr = 0.0, k2 = 0.0, dk2 = 0.0, svx = 0.0, dsvx = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
        if (c->frozen[i]) continue;
        nf += 1.0;
        sr += rho[i];
        dsr += drho[i];
        for (int a = 0; a < 3; ++a) {
            k2 += p->mass * v[3 * i + a] * v[3 * i + a];
            dk2 += 2.0 * p->mass * v[3 * i + a] * dv[3 * i + a];
        }
        svx += v[3 * i];
        dsvx += dv[3 * i];
    }
    const double V3 = 3.0 * p->L[0] * p->L[1] * p->L[2];
    const double inf = nf > 0.0 ? 1.0 / nf : 0.0;
    *l = w[0] * sr * inf + w[1] * (k2 + vir) / V3 + w[2] * svx * inf;
    *dl = w[0] * dsr * inf + w[1] * (dk2 + dvir) / V3 + w[2] * dsvx * inf;
}

int orc_tangent(const orc_params *p, int64_t n, const double *x0, const double *v0, const int32_t *type,
                const uint8_t *frozen, const double *dx0, const double *dv0, const double *dA,
                const double *dB, const double *dgamma, int64_t nsteps, const double w[3], int avg,
                double out[2])
{
    if ((p->wall_model != 0 && p->wall_slip != 0.0) || nsteps < 0 || (avg && nsteps < 1)) return -1;
    orc_tan_ctx c = {p, n, type, frozen, dA, dB, dgamma};
    size_t nn = (size_t)(n ? n : 1);
    double *x = (double *)malloc(nn * 3 * sizeof(double)), *dx = (double *)malloc(nn * 3 * sizeof(double));
    double *v = (double *)malloc(nn * 3 * sizeof(double)), *dv = (double *)malloc(nn * 3 * sizeof(double));
    double *vh = (double *)malloc(nn * 3 * sizeof(double)), *dvh = (double *)malloc(nn * 3 * sizeof(double));
    double *F = (double *)malloc(nn * 3 * sizeof(double)), *dF = (double *)malloc(nn * 3 * sizeof(double));
    double *rho = (double *)malloc(nn * sizeof(double)), *drho = (double *)malloc(nn * sizeof(double));
    double *xp = (double *)malloc(nn * 3 * sizeof(double)), *dxp = (double *)malloc(nn * 3 * sizeof(double));
    double *phi = (double *)malloc(nn * sizeof(double));
    const double hdtm = 0.5 * p->dt / p->mass;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            int k = 3 * (int)i + a;
            x[k] = orc_wrap(x0[k], p->L[a]);
            dx[k] = dx0 ? dx0[k] : 0.0;
            v[k] = frozen[i] ? 0.0 : v0[k];
            dv[k] = (frozen[i] || !dv0) ? 0.0 : dv0[k];
            vh[k] = v[k];
            dvh[k] = dv[k];
        }
    double vir = 0.0, dvir = 0.0, L = 0.0, dL = 0.0, l, dl;
    orc_nlist nl;
    orc_build(x, n, p->L, p->rc, p->search, &nl);
    orc_tan_density(&c, x, dx, &nl, rho, drho);
    orc_tan_forces(&c, x, dx, vh, dvh, rho, drho, 0, &nl, F, dF, &vir, &dvir);
    orc_nlist_free(&nl);
    for (int64_t s = 1; s <= nsteps; ++s) {
        memcpy(xp, x, nn * 3 * sizeof(double));
        memcpy(dxp, dx, nn * 3 * sizeof(double));
        for (int64_t i = 0; i < n; ++i) {
            if (frozen[i]) continue;
            for (int a = 0; a < 3; ++a) {
                int k = 3 * (int)i + a;
                vh[k] = v[k] + hdtm * F[k];
                dvh[k] = dv[k] + hdtm * dF[k];
                x[k] = orc_wrap(x[k] + p->dt * vh[k], p->L[a]);
                dx[k] = dx[k] + p->dt * dvh[k];
            }
        }
        if (p->wall_model) {
            /* the corrector (reading R4, bounce-back) with its decisions
             * taken on the primal state: x and its tangent go back, v_half
             * and its tangent change sign */
            orc_build(x, n, p->L, p->rc, p->search, &nl);
            orc_phi_nl(p, n, x, frozen, &nl, phi);
            orc_nlist_free(&nl);
            for (int64_t i = 0; i < n; ++i) {
                if (frozen[i] || !(phi[i] > p->phi_c)) continue;
                for (int a = 0; a < 3; ++a) {
                    int k = 3 * (int)i + a;
                    x[k] = xp[k];
                    dx[k] = dxp[k];
                    vh[k] = -vh[k];
                    dvh[k] = -dvh[k];
                }
            }
        }
        orc_build(x, n, p->L, p->rc, p->search, &nl);
        orc_tan_density(&c, x, dx, &nl, rho, drho);
        orc_tan_forces(&c, x, dx, vh, dvh, rho, drho, (uint32_t)s, &nl, F, dF, &vir, &dvir);
        orc_nlist_free(&nl);
        for (int64_t i = 0; i < n; ++i) {
            if (frozen[i]) continue;
            for (int a = 0; a < 3; ++a) {
                int k = 3 * (int)i + a;
                v[k] = vh[k] + hdtm * F[k];
                dv[k] = dvh[k] + hdtm * dF[k];
            }
        }
        if (avg) {
            orc_tan_loss(&c, v, dv, rho, drho, vir, dvir, w, &l, &dl);
            L += l / (double)nsteps;
            dL += dl / (double)nsteps;
        }
    }
    if (!avg) orc_tan_loss(&c, v, dv, rho, drho, vir, dvir, w, &L, &dL);
    out[0] = L;
    out[1] = dL;
    free(xp);
    free(dxp);
    free(phi);
    free(x);
    free(dx);
    free(v);
    free(dv);
    free(vh);
    free(dvh);
    free(F);
    free(dF);
    free(rho);
    free(drho);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pressure tensor of the current state (the tensor form of the virial     */
/* pressure of orc_observables, used for the stress across an interface):  */
/*   P_ab = [ sum_fluid m v_a v_b + sum_{fluid i, j in N_c(i)} c_ij         */
/*            d_a d_b / r F^C(r) ] / V,                                     */
/* d = x_i - x_j (minimum image), F^C = A w_c + B (rho_i + rho_j) w_d the    */
/* conservative pair force magnitude (Eq. 1), c_ij = 1/2 for fluid j and 1   */
/* for frozen j.  out[6] = xx, yy, zz, xy, xz, yz; its trace / 3 is the     */
/* pressure.  Brute-force pair search over all j (the definition).          */
/* ------------------------------------------------------------------------ */
void orc_stress(const orc_system *s, double out[6])
{
    const orc_params *p = &s->p;
    const int T = p->ntypes;
    const int64_t n = s->n;
    const double rc2 = p->rc * p->rc, rd2 = p->rd * p->rd;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        if (s->frozen[i]) continue;
        const double *v = s->v + 3 * i;
        acc[0] += p->mass * v[0] * v[0];
        acc[1] += p->mass * v[1] * v[1];
        acc[2] += p->mass * v[2] * v[2];
        acc[3] += p->mass * v[0] * v[1];
        acc[4] += p->mass * v[0] * v[2];
        acc[5] += p->mass * v[1] * v[2];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            orc_delta(s->x, i, j, p->L, d);
            double r2 = orc_r2(d);
            if (!(r2 < rc2) || r2 == 0.0) continue;
            double r = sqrt(r2);
            int tt = s->type[i] * T + s->type[j];
            double fc = p->A[tt] * (1.0 - r / p->rc);
            if (r2 < rd2) fc += p->B[tt] * (s->rho[i] + s->rho[j]) * (1.0 - r / p->rd);
            double c = s->frozen[j] ? 1.0 : 0.5;
            double k = c * fc / r;
            acc[0] += k * d[0] * d[0];
            acc[1] += k * d[1] * d[1];
            acc[2] += k * d[2] * d[2];
            acc[3] += k * d[0] * d[1];
            acc[4] += k * d[0] * d[2];
            acc[5] += k * d[1] * d[2];
        }
    }
    const double V = p->L[0] * p->L[1] * p->L[2];
    for (int a = 0; a < 6; ++a) out[a] = acc[a] / V;
}
