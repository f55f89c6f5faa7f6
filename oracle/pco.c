/*
 * pco.c -- plain FP64 CPU oracle of the 1D PIC-MCC positive-column step.
 *
 * TEST INFRASTRUCTURE ONLY (see pco.h).  Written for clarity, not speed:
 * one serial loop per species per step, the Thomas algorithm for Poisson's
 * equation, and the random draws taken from a counter-based Philox keyed by
 * (seed; particle id, step, block, stream) so that each draw is a function of
 * the particle and the step alone.
 *
 * Paper passages followed (Boeuf, "Ionization waves (striations) in a
 * low-current plasma column revisited with kinetic and fluid models"):
 *  - section II: particles on a grid, density by interpolation of positions,
 *    field from Poisson's equation each step, Monte Carlo collisions whose
 *    probability, type and scattering follow from the cross sections;
 *    periodic reinjection with unchanged velocity; Poisson solved with the
 *    Thomas algorithm; imposed mean field E = -E0 + E_sp;
 *  - section II: electron-atom elastic, excitation (one lumped level) and
 *    ionization collisions; ion-atom charge exchange (backward scattering);
 *  - section II, eq. (2): radial ambipolar losses, here as a per-particle
 *    removal frequency;
 *  - section V: the bounded variant (electrodes at both ends).
 * Where the paper is silent (op order, weighting, energy sharing, null
 * collision variant, fixed-point format, step order) the readings are the
 * ones listed in the design notes; each is marked "reading" below.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, so every product and sum is a separately rounded IEEE op).
 * The same file built with -fopenmp is the all-core timing build: the
 * particle loops run in parallel, every shared update is an atomic integer
 * add or bit-or, the ionizations are sorted by parent id before use and the
 * charge is an integer sum, so it computes bit for bit what the serial build
 * computes (without -fopenmp the pragmas are ignored).
 */
#include "pco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 */
#define QE   1.602176634e-19
#define ME   9.1093837015e-31
#define AMU  1.66053906660e-27
#define KB   1.380649e-23
#define EPS0 8.8541878128e-12
#define TORR (101325.0 / 760.0)
#define FIX  33554432.0            /* 2^25: fractional bits of the charge unit */
#define FIXI ((int64_t)1 << 25)

enum { ERR_RANGE = 16 };
enum { ST_E_STEP = 0, ST_I_STEP = 1, ST_E_INIT = 2, ST_I_INIT = 3, ST_VICTIM_E = 4, ST_VICTIM_I = 5,
       ST_EMIT = 6 };

typedef struct {
    int64_t n, cap;
    double *x, *vx, *vy, *vz;
    uint32_t* id;
    uint8_t* ev;
    int64_t evcap;
} species_t;

typedef struct {
    uint32_t pid;
    double x;
    double ve[3];  /* ejected electron */
    double vi[3];  /* new ion */
} birth_t;

struct pco_column {
    pco_config cfg;
    int nc, nn, periodic;
    double L, dx, inv_dx, dt, dti;
    double Ng, M, c_eps, qmdt_e, qmdt_i, W, fpc, E0, Vb;
    double sig_a, sig_e0, sig_i0;
    double nu_max, P_null, T_we, T_wi, P_cx;
    double mr2, sx4, si4;
    species_t sp[2];
    int64_t next_id[2];
    int64_t step;
    double* E;      /* nn + 1 entries: periodic ghost E[nc] = E[0] */
    int64_t *rho_e, *rho_i, *iz;
    uint32_t err;
    birth_t* births;
    int64_t nb, bcap;
    /* balanced sink: ionizations of the previous step and since the last ion step */
    int64_t births_last, births_since_ion;
    /* pair sink: the ids removed in the last step, per species */
    uint32_t* victims[2];
    int64_t n_victims;
    /* section V: cathode emission and the external circuit */
    double emit_n, emit_sig, circ_a, circ_jf, Jc, carry;
    int64_t vs_e, vs_ia, vs_i;   /* sums of v_x in 2^-20 m/s units */
};

/* ------------------------------------------------------------------ Philox */
/* Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw (SC'11):
 * ten rounds of two 32x32->64 multiplies, each round feeding the high halves
 * XORed with the other counter words and the round key; the key is bumped by
 * the two Weyl constants between rounds. */
void pco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0,1) from 52 bits of a word pair; exact in double */
static double u52(uint32_t lo, uint32_t hi)
{
    uint64_t r = ((uint64_t)hi << 32) | lo;
    return ((double)(r >> 12) + 0.5) * 0x1p-52;
}
/* uniform in (0,1) from one 32-bit word */
static double u32(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* sequential word stream from blocks 1, 2, ... of one (id, step, stream) */
typedef struct {
    uint32_t ctr[4], key[2], buf[4];
    int pos;
} kstream_t;

static void ks_init(kstream_t* s, const uint32_t key[2], uint32_t id, uint32_t step, uint32_t stream)
{
    s->key[0] = key[0]; s->key[1] = key[1];
    s->ctr[0] = id; s->ctr[1] = step; s->ctr[2] = 0; s->ctr[3] = stream;
    s->pos = 4;
}
static uint32_t ks_next(kstream_t* s)
{
    if (s->pos == 4) {
        s->ctr[2] += 1;
        pco_philox4x32_10(s->ctr, s->key, s->buf);
        s->pos = 0;
    }
    return s->buf[s->pos++];
}

/* isotropic unit vector by Marsaglia's (1972) disk rejection; reading: at most
 * 64 attempts, then the pole (never reached in practice: p = 0.2146^64). */
static void iso_dir(kstream_t* s, double n[3])
{
    for (int k = 0; k < 64; ++k) {
        double a = 2.0 * u32(ks_next(s)) - 1.0;
        double b = 2.0 * u32(ks_next(s)) - 1.0;
        double q = a * a + b * b;
        if (q < 1.0) {
            double r = 2.0 * sqrt(1.0 - q);
            n[0] = a * r; n[1] = b * r; n[2] = 1.0 - 2.0 * q;
            return;
        }
    }
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
}

/* standard normal pair by the polar method (Marsaglia and Bray 1964) */
static void gauss2(kstream_t* s, double g[2])
{
    for (int k = 0; k < 64; ++k) {
        double a = 2.0 * u32(ks_next(s)) - 1.0;
        double b = 2.0 * u32(ks_next(s)) - 1.0;
        double q = a * a + b * b;
        if (q < 1.0 && q > 0.0) {
            double f = sqrt(-2.0 * log(q) / q);
            g[0] = a * f; g[1] = b * f;
            return;
        }
    }
    g[0] = 0.0; g[1] = 0.0;
}

/* three independent normals: first pair, then the first of a second pair */
static void gauss3(kstream_t* s, double g[3])
{
    double p[2], q[2];
    gauss2(s, p);
    gauss2(s, q);
    g[0] = p[0]; g[1] = p[1]; g[2] = q[0];
}

/* ------------------------------------------------------- cross sections */
/* synthetic analytic forms (one lumped excitation level as for argon in the
 * paper, section II; shapes and numbers are the project's own) */
static double sig_el(const pco_column* c, double eps)
{
    if (c->cfg.el_p > 0.0) return c->cfg.el_A + c->cfg.el_B * sqrt(eps);
    if (eps > 0.0) return c->cfg.el_A + c->cfg.el_B / sqrt(eps);
    return c->cfg.el_A;
}
static double sig_thomson(double eps, double U, double s4)
{
    if (eps > U) {
        double t = U / eps;
        return s4 * t * (1.0 - t);
    }
    return 0.0;
}

/* -------------------------------------------------------------- helpers */
static void cell_of(const pco_column* c, double x, int* j, double* f)
{
    double s = x * c->inv_dx;
    int jj = (int)s;
    if (jj > c->nc - 1) jj = c->nc - 1;
    *j = jj;
    *f = s - (double)jj;
}

static int grow(species_t* s, int64_t need)
{
    if (need <= s->cap) return 0;
    int64_t cap = s->cap ? s->cap : 1024;
    while (cap < need) cap *= 2;
    double* a[4] = {s->x, s->vx, s->vy, s->vz};
    for (int k = 0; k < 4; ++k) {
        double* p = (double*)realloc(a[k], (size_t)cap * sizeof(double));
        if (!p) return -1;
        a[k] = p;
    }
    s->x = a[0]; s->vx = a[1]; s->vy = a[2]; s->vz = a[3];
    uint32_t* q = (uint32_t*)realloc(s->id, (size_t)cap * sizeof(uint32_t));
    if (!q) return -1;
    s->id = q;
    s->cap = cap;
    return 0;
}

static int grow_events(species_t* s, int64_t need)
{
    if (need <= s->evcap) return 0;
    int64_t cap = s->evcap ? s->evcap : 1024;
    while (cap < need) cap *= 2;
    uint8_t* p = (uint8_t*)realloc(s->ev, (size_t)cap);
    if (!p) return -1;
    memset(p + s->evcap, 0, (size_t)(cap - s->evcap));
    s->ev = p;
    s->evcap = cap;
    return 0;
}

/* -------------------------------------------------------------- create */
pco_column* pco_create(const pco_config* cfg)
{
    if (!cfg || cfg->n_cells < 2 || !(cfg->L > 0.0) || !(cfg->dt > 0.0) || cfg->ppc < 0 ||
        cfg->ion_subcycle < 1 || (cfg->el_p != 0.5 && cfg->el_p != -0.5) ||
        (cfg->bc != PCO_BOUNDED && cfg->bc != PCO_PERIODIC) || !(cfg->eps_cap > 0.0) ||
        !(cfg->g_cap > 0.0))
        return NULL;
    pco_column* c = (pco_column*)calloc(1, sizeof(pco_column));
    if (!c) return NULL;
    c->cfg = *cfg;
    c->nc = cfg->n_cells;
    c->periodic = cfg->bc == PCO_PERIODIC;
    c->nn = c->periodic ? c->nc : c->nc + 1;
    c->L = cfg->L;
    c->dx = cfg->L / (double)c->nc;
    c->inv_dx = (double)c->nc / cfg->L;
    c->dt = cfg->dt;
    c->dti = (double)cfg->ion_subcycle * cfg->dt;
    c->Ng = cfg->p_torr * TORR / (KB * cfg->Tg);
    c->M = cfg->M_amu * AMU;
    c->c_eps = 0.5 * ME / QE;
    c->qmdt_e = (-QE * cfg->dt) / ME;
    c->qmdt_i = (QE * c->dti) / c->M;
    /* macroparticle weight (real particles per m^2 of column cross-section) */
    c->W = cfg->ppc > 0 ? cfg->n0 * c->dx / (double)cfg->ppc : 0.0;
    /* field jump per fixed-point charge unit: e W 2^-25 / eps0  [V/m] */
    c->fpc = QE * c->W / FIX / EPS0;
    c->E0 = cfg->V / cfg->L;
    c->Vb = cfg->V;
    /* section V: emitted electrons per step J dt / (e W), their thermal speed,
     * the gap's R eps0 / (L dt) and the current density of one unit of the
     * v_x sums, e W / L 2^-20 */
    c->emit_n = cfg->emit_J * cfg->dt / (QE * c->W);
    c->emit_sig = sqrt(QE * cfg->emit_T / ME);
    c->circ_a = cfg->circuit_R * EPS0 / (cfg->L * cfg->dt);
    c->circ_jf = QE * c->W / cfg->L / 1048576.0;
    c->sig_a = sqrt(KB * cfg->Tg / c->M);
    c->sig_e0 = sqrt(cfg->Te0_eV * QE / ME);
    c->sig_i0 = sqrt(KB * cfg->Ti0_K / c->M);
    c->mr2 = 2.0 * ME / c->M;
    c->sx4 = 4.0 * cfg->ex_smax;
    c->si4 = 4.0 * cfg->iz_smax;

    /* null-collision bound: max of Ng*sigma_tot(eps)*v(eps) on a fine grid of
     * [0, eps_cap] with a 1e-3 margin (reading) */
    {
        const int G = 65536;
        double mx = 0.0;
        for (int k = 0; k <= G; ++k) {
            double eps = cfg->eps_cap * (double)k / (double)G;
            double v = sqrt(eps / c->c_eps);
            double s = sig_el(c, eps) + sig_thomson(eps, cfg->ex_U, c->sx4) +
                       sig_thomson(eps, cfg->iz_U, c->si4);
            double nu = s * v * c->Ng;
            if (nu > mx) mx = nu;
        }
        c->nu_max = mx * 1.001;
    }
    c->P_null = 1.0 - exp(-c->nu_max * c->dt);
    if (cfg->wall_mode == PCO_WALL_FIXED) {
        c->T_we = exp(-cfg->nu_w * c->dt);
        c->T_wi = exp(-cfg->nu_w * c->dti);
    } else {
        c->T_we = 2.0;
        c->T_wi = 2.0;
    }
    c->P_cx = 1.0 - exp(-c->Ng * cfg->cx_sigma * cfg->g_cap * c->dti);

    c->E = (double*)calloc((size_t)c->nn + 1, sizeof(double));
    c->rho_e = (int64_t*)calloc((size_t)c->nn, sizeof(int64_t));
    c->rho_i = (int64_t*)calloc((size_t)c->nn, sizeof(int64_t));
    c->iz = (int64_t*)calloc((size_t)c->nc, sizeof(int64_t));
    if (!c->E || !c->rho_e || !c->rho_i || !c->iz) { pco_destroy(c); return NULL; }
    return c;
}

void pco_destroy(pco_column* c)
{
    if (!c) return;
    for (int s = 0; s < 2; ++s) {
        free(c->sp[s].x); free(c->sp[s].vx); free(c->sp[s].vy); free(c->sp[s].vz);
        free(c->sp[s].id); free(c->sp[s].ev);
    }
    free(c->E); free(c->rho_e); free(c->rho_i); free(c->iz); free(c->births);
    free(c->victims[0]); free(c->victims[1]);
    free(c);
}

/* ---------------------------------------------------------------- deposit */
/* linear (cloud-in-cell) weighting into 64-bit fixed point with 25 fractional
 * bits: node j receives 2^25 - a and node j+1 receives a, a = trunc(f 2^25)
 * (reading of the "interpolation of the particle positions", section II). */
static void deposit_one(const pco_column* c, double x, int64_t* rho)
{
    int j; double f;
    cell_of(c, x, &j, &f);
    int64_t a = (int64_t)(f * FIX);
    if (a > FIXI) a = FIXI;
    int j1 = j + 1;
    if (c->periodic && j1 == c->nc) j1 = 0;
    rho[j] += FIXI - a;
    rho[j1] += a;
}

int pco_deposit(const pco_column* c, const double* x, int64_t n, int64_t* rho)
{
    if (!c || (n > 0 && (!x || !rho))) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (!(x[i] >= 0.0 && x[i] < c->L)) return -2;
    memset(rho, 0, (size_t)c->nn * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) deposit_one(c, x[i], rho);
    return 0;
}

/* ------------------------------------------------------------ field solve */
/* Thomas algorithm for -phi[j-1] + 2 phi[j] - phi[j+1] = b[j], j = 1..m,
 * with the boundary values already folded into b (section II).  The sweeps
 * run in x87 extended precision: in double their rounding error grows
 * roughly with the square of the node count (about 1e-11 of max|E| at 8000
 * nodes), too coarse for a reference. */
static void thomas(int m, const long double* b, long double* phi /* 1..m */)
{
    long double* cp = (long double*)malloc((size_t)(m + 1) * sizeof(long double));
    long double* bp = (long double*)malloc((size_t)(m + 1) * sizeof(long double));
    cp[1] = -1.0L / 2.0L;
    bp[1] = b[1] / 2.0L;
    for (int j = 2; j <= m; ++j) {
        long double den = 2.0L + cp[j - 1];          /* 2 - (-1) * cp[j-1] */
        cp[j] = -1.0L / den;
        bp[j] = (b[j] + bp[j - 1]) / den;            /* (b - (-1) bp[j-1]) / den */
    }
    phi[m] = bp[m];
    for (int j = m - 1; j >= 1; --j) phi[j] = bp[j] - cp[j] * phi[j + 1];
    free(cp);
    free(bp);
}

int pco_solve_field(const pco_column* c, const int64_t* rho_e, const int64_t* rho_i,
                    double* phi_out, double* E)
{
    if (!c || !rho_e || !rho_i || !E) return -1;
    const int nc = c->nc, nn = c->nn;
    long double* phi = (long double*)calloc((size_t)nn + 2, sizeof(long double));
    long double* b = (long double*)calloc((size_t)nn + 2, sizeof(long double));
    if (!phi || !b) { free(phi); free(b); return -3; }
    /* right-hand side dx^2 rho / eps0 with rho = e W Q 2^-25 / dx: dx fpc Q */
    const long double k = (long double)c->fpc * (long double)c->dx;
    const long double dx = c->dx, fpc = c->fpc;
    if (!c->periodic) {
        /* bounded: phi_0 = 0, phi_nc = V (section V, electrodes at both ends) */
        for (int j = 1; j < nc; ++j) b[j] = k * (long double)(rho_i[j] - rho_e[j]);
        b[nc - 1] += c->Vb;
        thomas(nc - 1, b, phi);
        phi[0] = 0.0L;
        phi[nc] = c->Vb;
        /* E at nodes: centred difference inside; half-cell Gauss's law at the
         * two electrodes (reading) */
        for (int j = 1; j < nc; ++j) E[j] = (double)((phi[j - 1] - phi[j + 1]) / (2.0L * dx));
        long double eh0 = (phi[0] - phi[1]) / dx;
        long double ehN = (phi[nc - 1] - phi[nc]) / dx;
        E[0] = (double)(eh0 - fpc * (long double)(rho_i[0] - rho_e[0]));
        E[nc] = (double)(ehN + fpc * (long double)(rho_i[nc] - rho_e[nc]));
    } else {
        /* periodic: neutralise the mean charge, gauge phi_0 = 0 (reading of the
         * periodic solve), then E = -E0 + E_sp (section II) */
        int64_t qt = 0;
        for (int j = 0; j < nc; ++j) qt += rho_i[j] - rho_e[j];
        const long double qs = (long double)qt / (long double)nc;
        for (int j = 1; j < nc; ++j) b[j] = k * ((long double)(rho_i[j] - rho_e[j]) - qs);
        thomas(nc - 1, b, phi);
        phi[0] = 0.0L;
        phi[nc] = 0.0L;
        for (int j = 0; j < nc; ++j) {
            long double pm = j == 0 ? phi[nc - 1] : phi[j - 1];
            long double pp = phi[j + 1];
            E[j] = (double)(-(long double)c->E0 + (pm - pp) / (2.0L * dx));
        }
    }
    if (phi_out)
        for (int j = 0; j < nn; ++j) phi_out[j] = (double)phi[j];
    free(phi);
    free(b);
    return 0;
}

static void field_update(pco_column* c)
{
    species_t* e = &c->sp[PCO_ELECTRON];
    species_t* i = &c->sp[PCO_ION];
    int64_t* re = c->rho_e;
    int64_t* ri = c->rho_i;
    const int nn = c->nn;
    memset(re, 0, (size_t)nn * sizeof(int64_t));
    memset(ri, 0, (size_t)nn * sizeof(int64_t));
    /* integer sums: any order of the additions gives the same charge */
    #pragma omp parallel for schedule(static) reduction(+ : re[:nn])
    for (int64_t k = 0; k < e->n; ++k) deposit_one(c, e->x[k], re);
    #pragma omp parallel for schedule(static) reduction(+ : ri[:nn])
    for (int64_t k = 0; k < i->n; ++k) deposit_one(c, i->x[k], ri);
    if (c->cfg.poisson) {
        pco_solve_field(c, c->rho_e, c->rho_i, NULL, c->E);
    } else {
        double e0 = c->periodic ? -c->E0 : -c->Vb / c->L;
        for (int j = 0; j < c->nn; ++j) c->E[j] = e0;
    }
    if (c->periodic) c->E[c->nc] = c->E[0];
}

static double gather(const pco_column* c, double x)
{
    int j; double f;
    cell_of(c, x, &j, &f);
    return c->E[j] + f * (c->E[j + 1] - c->E[j]);
}

/* ------------------------------------------------------------------ init */
int pco_init_column(pco_column* c)
{
    if (!c) return -1;
    const int64_t n0 = (int64_t)c->cfg.ppc * c->nc;
    const uint32_t key[2] = {(uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32)};
    for (int s = 0; s < 2; ++s) {
        species_t* p = &c->sp[s];
        if (grow(p, n0) || grow_events(p, n0)) return -3;
        const double sig = s == PCO_ELECTRON ? c->sig_e0 : c->sig_i0;
        const uint32_t stream = s == PCO_ELECTRON ? ST_E_INIT : ST_I_INIT;
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < n0; ++k) {
            uint32_t ctr[4] = {(uint32_t)k, 0u, 0u, stream}, w[4];
            pco_philox4x32_10(ctr, key, w);
            /* uniform load (section II: uniform and equal initial densities) */
            double x = u52(w[0], w[1]) * c->L;
            if (x >= c->L) x = 0.0;
            kstream_t ks;
            ks_init(&ks, key, (uint32_t)k, 0u, stream);
            double g[3];
            gauss3(&ks, g);
            p->x[k] = x;
            p->vx[k] = sig * g[0];
            p->vy[k] = sig * g[1];
            p->vz[k] = sig * g[2];
            p->id[k] = (uint32_t)k;
        }
        p->n = n0;
        c->next_id[s] = n0;
    }
    c->step = 0;
    field_update(c);
    /* leapfrog start: v^{-1/2} = v^0 - (q/m) E^0 dt/2 (ions with their own dt) */
    for (int s = 0; s < 2; ++s) {
        species_t* p = &c->sp[s];
        const double hq = 0.5 * (s == PCO_ELECTRON ? c->qmdt_e : c->qmdt_i);
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < p->n; ++k) p->vx[k] = p->vx[k] - hq * gather(c, p->x[k]);
    }
    return 0;
}

/* --------------------------------------------------------------- the step */
static int push_birth(pco_column* c, const birth_t* b)
{
    if (c->nb == c->bcap) {
        int64_t cap = c->bcap ? 2 * c->bcap : 256;
        birth_t* p = (birth_t*)realloc(c->births, (size_t)cap * sizeof(birth_t));
        if (!p) return -1;
        c->births = p;
        c->bcap = cap;
    }
    c->births[c->nb++] = *b;
    return 0;
}

static int cmp_birth(const void* a, const void* b)
{
    uint32_t x = ((const birth_t*)a)->pid, y = ((const birth_t*)b)->pid;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* move x by one step and apply the boundary; returns 1 if the particle left */
static int boundary(pco_column* c, double* xp, uint8_t* ev)
{
    double x = *xp;
    if (c->periodic) {
        /* reinjection at the opposite end with the same velocity (section II) */
        if (x >= c->L) x -= c->L;
        else if (x < 0.0) { x += c->L; if (x >= c->L) x = 0.0; }
        if (!(x >= 0.0 && x < c->L)) {
            #pragma omp atomic
            c->err |= ERR_RANGE;
            x = 0.0;
        }
        *xp = x;
        return 0;
    }
    if (x >= 0.0 && x < c->L) return 0;
    if (!(x < 0.0 || x >= c->L)) {   /* NaN */
        #pragma omp atomic
        c->err |= ERR_RANGE;
    }
    *ev = PCO_EV_ABSORB;
    return 1;
}

static int electron_pass(pco_column* c, uint8_t* dead, const uint32_t key[2])
{
    species_t* p = &c->sp[PCO_ELECTRON];
    const uint32_t step = (uint32_t)c->step;
    int failed = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < p->n; ++k) {
        uint8_t ev = PCO_EV_NONE;
        double x = p->x[k], vx = p->vx[k];
        const uint32_t id = p->id[k];
        /* gather and leapfrog push; the field acts on v_x only (1d3v) */
        double Ex = gather(c, x);
        vx = vx + c->qmdt_e * Ex;
        x = x + vx * c->dt;
        const double vpush = vx;   /* for the circuit's conduction current */
        int lost = boundary(c, &x, &ev);
        if (!lost) {
            uint32_t ctr[4] = {id, step, 0u, ST_E_STEP}, w[4];
            pco_philox4x32_10(ctr, key, w);
            double u0 = u52(w[0], w[1]), u1 = u52(w[2], w[3]);
            if (u0 >= c->T_we) {
                ev = PCO_EV_WALL;   /* radial loss to the tube wall, eq. (2) */
                lost = 1;
            } else if (u0 < c->P_null) {
                /* null-collision candidate: choose the process with u1 nu_max
                 * against the cumulative collision frequencies */
                double vy = p->vy[k], vz = p->vz[k];
                double v2 = (vx * vx + vy * vy) + vz * vz;
                double eps = c->c_eps * v2;
                double v = sqrt(v2);
                if (eps > c->cfg.eps_cap) {
                    #pragma omp atomic
                    c->err |= PCO_ERR_ECAP;
                }
                double s_el = sig_el(c, eps);
                double s_ex = sig_thomson(eps, c->cfg.ex_U, c->sx4);
                double s_iz = sig_thomson(eps, c->cfg.iz_U, c->si4);
                double nu1 = s_el * v * c->Ng;
                double nu2 = nu1 + s_ex * v * c->Ng;
                double nu3 = nu2 + s_iz * v * c->Ng;
                if (nu3 > c->nu_max) {
                    #pragma omp atomic
                    c->err |= PCO_ERR_NUMAX;
                }
                double R = u1 * c->nu_max;
                kstream_t ks;
                ks_init(&ks, key, id, step, ST_E_STEP);
                double n[3];
                if (R < nu1) {
                    /* elastic, isotropic in the lab frame, energy loss
                     * (2m/M)(1 - cos chi) on a cold gas */
                    ev = PCO_EV_ELASTIC;
                    iso_dir(&ks, n);
                    double cosx = ((vx * n[0] + vy * n[1]) + vz * n[2]) / v;
                    double fac = 1.0 - c->mr2 * (1.0 - cosx);
                    double vn = v * sqrt(fac);
                    vx = vn * n[0]; vy = vn * n[1]; vz = vn * n[2];
                } else if (R < nu2) {
                    /* lumped excitation: lose the threshold, isotropic */
                    ev = PCO_EV_EXCITE;
                    iso_dir(&ks, n);
                    double vn = sqrt((eps - c->cfg.ex_U) / c->c_eps);
                    vx = vn * n[0]; vy = vn * n[1]; vz = vn * n[2];
                } else if (R < nu3) {
                    /* ionization: share eps - U_iz between scattered and ejected
                     * electron, create an ion at the atom temperature */
                    ev = PCO_EV_IONIZE;
                    double us = u32(ks_next(&ks));
                    double er = eps - c->cfg.iz_U;
                    double ej;
                    if (c->cfg.energy_sharing == PCO_SHARE_EQUAL) ej = 0.5 * er;
                    else ej = c->cfg.opb_w * tan(us * atan(er / (2.0 * c->cfg.opb_w)));
                    double sc = er - ej;
                    double n2[3], g[3];
                    iso_dir(&ks, n);
                    iso_dir(&ks, n2);
                    gauss3(&ks, g);
                    double vs = sqrt(sc / c->c_eps);
                    double ve = sqrt(ej / c->c_eps);
                    vx = vs * n[0]; vy = vs * n[1]; vz = vs * n[2];
                    birth_t b;
                    b.pid = id;
                    b.x = x;
                    b.ve[0] = ve * n2[0]; b.ve[1] = ve * n2[1]; b.ve[2] = ve * n2[2];
                    b.vi[0] = c->sig_a * g[0]; b.vi[1] = c->sig_a * g[1]; b.vi[2] = c->sig_a * g[2];
                    /* list order is immaterial: the step sorts them by parent id */
                    #pragma omp critical(pco_births)
                    {
                        if (push_birth(c, &b)) failed = 1;
                    }
                    int j; double f;
                    cell_of(c, x, &j, &f);
                    #pragma omp atomic
                    c->iz[j] += 1;
                } else {
                    ev = PCO_EV_NULL;
                }
                p->vy[k] = vy;
                p->vz[k] = vz;
            }
        }
        p->x[k] = x;
        p->vx[k] = vx;
        dead[k] = (uint8_t)lost;
        if (!lost && c->cfg.circuit_R > 0.0) {
            const int64_t dv = (int64_t)(vpush * 1048576.0);
            #pragma omp atomic
            c->vs_e += dv;
        }
        p->ev[id] = ev;
    }
    return failed ? -3 : 0;
}

static void ion_pass(pco_column* c, uint8_t* dead, const uint32_t key[2])
{
    species_t* p = &c->sp[PCO_ION];
    const uint32_t step = (uint32_t)c->step;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < p->n; ++k) {
        uint8_t ev = PCO_EV_NONE;
        double x = p->x[k], vx = p->vx[k];
        const uint32_t id = p->id[k];
        double Ex = gather(c, x);
        vx = vx + c->qmdt_i * Ex;
        x = x + vx * c->dti;
        const double vpush = vx;   /* before charge exchange */
        int lost = boundary(c, &x, &ev);
        if (!lost) {
            uint32_t ctr[4] = {id, step, 0u, ST_I_STEP}, w[4];
            pco_philox4x32_10(ctr, key, w);
            double u0 = u52(w[0], w[1]), u1 = u52(w[2], w[3]);
            if (u0 >= c->T_wi) {
                ev = PCO_EV_WALL;
                lost = 1;
            } else if (u0 < c->P_cx) {
                /* charge exchange with a Maxwellian atom: null-collision bound
                 * Ng sigma g_cap, accept with g / g_cap; the ion takes the
                 * atom's velocity (backward scattering, section II) */
                double vy = p->vy[k], vz = p->vz[k];
                kstream_t ks;
                ks_init(&ks, key, id, step, ST_I_STEP);
                double g[3];
                gauss3(&ks, g);
                double ax = c->sig_a * g[0], ay = c->sig_a * g[1], az = c->sig_a * g[2];
                double dx = vx - ax, dy = vy - ay, dz = vz - az;
                double gr = sqrt((dx * dx + dy * dy) + dz * dz);
                if (gr > c->cfg.g_cap) {
                    #pragma omp atomic
                    c->err |= PCO_ERR_GCAP;
                }
                if (u1 * c->cfg.g_cap < gr) {
                    ev = PCO_EV_CX;
                    vx = ax; vy = ay; vz = az;
                } else {
                    ev = PCO_EV_NULL;
                }
                p->vy[k] = vy;
                p->vz[k] = vz;
            }
        }
        p->x[k] = x;
        p->vx[k] = vx;
        dead[k] = (uint8_t)lost;
        if (!lost && c->cfg.circuit_R > 0.0) {
            const int64_t dv = (int64_t)(vpush * 1048576.0);
            #pragma omp atomic
            c->vs_ia += dv;
        }
        p->ev[id] = ev;
    }
}

static void remove_dead(species_t* p, const uint8_t* dead)
{
    int64_t w = 0;
    for (int64_t k = 0; k < p->n; ++k) {
        if (dead[k]) continue;
        p->x[w] = p->x[k]; p->vx[w] = p->vx[k]; p->vy[w] = p->vy[k]; p->vz[w] = p->vz[k];
        p->id[w] = p->id[k];
        ++w;
    }
    p->n = w;
}

/* Balanced radial sink (the paper keeps the particle number constant by
 * removing an electron-ion pair for every ionization, section II): each
 * particle of a species is removed with probability (ionizations since its
 * previous step) / (its current count), so that as many are removed on
 * average as were created. */
static double survival(int64_t births, int64_t n)
{
    if (n <= 0) return 1.0;
    return 1.0 - (double)births / (double)n;
}

/* Pair sink, the paper's own loss model (section II): for every ionization
 * one electron and one ion, picked at random over the whole column, are
 * removed, so that the particle numbers stay constant.  Reading (the paper
 * does not say how the random choice is made): the ids of a species are
 * 0..N-1 (the products of an ionization take over the ids of its victims);
 * the victim of ionization r (the step's ionizations ranked by parent id) is
 * drawn uniformly among the particles present after the advance, without
 * replacement: attempt t gives the id floor(w N / 2^32), w being word
 * (t mod 4) of the Philox block with counter (r, step, t / 4, victim
 * stream), and the first attempt that no lower rank has taken is the victim.
 * Victims leave before the charge deposit and the field solve. */
#define VICTIM_TRIES 65536
static int pair_victims(pco_column* c, int s, int64_t nb, const uint32_t key[2], uint32_t* vid)
{
    species_t* p = &c->sp[s];
    const uint64_t n = (uint64_t)p->n;
    const uint32_t step = (uint32_t)c->step;
    for (int64_t r = 0; r < nb; ++r) {
        int found = 0;
        for (uint32_t t = 0; t < VICTIM_TRIES && !found; ++t) {
            uint32_t ctr[4] = {(uint32_t)r, step, t / 4u, s == PCO_ELECTRON ? ST_VICTIM_E : ST_VICTIM_I}, w[4];
            pco_philox4x32_10(ctr, key, w);
            const uint32_t id = (uint32_t)(((uint64_t)w[t % 4u] * n) >> 32);
            int taken = 0;
            for (int64_t q = 0; q < r; ++q) taken |= vid[q] == id;
            if (!taken) { vid[r] = id; found = 1; }
        }
        if (!found) { c->err |= PCO_ERR_BIRTHS; return 0; }
    }
    /* remove the victims: find each id's index */
    int64_t* index = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    uint8_t* dead = (uint8_t*)calloc((size_t)n + 1, 1);
    if (!index || !dead) { free(index); free(dead); return -3; }
    for (int64_t k = 0; k < p->n; ++k) index[p->id[k]] = k;
    for (int64_t r = 0; r < nb; ++r) dead[index[vid[r]]] = 1;
    remove_dead(p, dead);
    free(index);
    free(dead);
    return 0;
}

static int one_step(pco_column* c)
{
    const uint32_t key[2] = {(uint32_t)c->cfg.seed, (uint32_t)(c->cfg.seed >> 32)};
    species_t* e = &c->sp[PCO_ELECTRON];
    species_t* i = &c->sp[PCO_ION];
    const int ion_step = c->step % c->cfg.ion_subcycle == 0;
    if (c->cfg.wall_mode == PCO_WALL_BALANCED) {
        c->T_we = survival(c->births_last, e->n);
        if (ion_step) c->T_wi = survival(c->births_since_ion, i->n);
    }
    if (e->evcap) memset(e->ev, 0, (size_t)e->evcap);
    if (i->evcap) memset(i->ev, 0, (size_t)i->evcap);
    c->nb = 0;
    int64_t nmax = e->n > i->n ? e->n : i->n;
    uint8_t* dead = (uint8_t*)calloc((size_t)nmax + 1, 1);
    if (!dead) return -3;
    int rc = electron_pass(c, dead, key);
    if (rc) { free(dead); return rc; }
    remove_dead(e, dead);
    if (ion_step) {
        ion_pass(c, dead, key);
        remove_dead(i, dead);
        c->births_since_ion = 0;
    }
    free(dead);
    const int pair = c->cfg.wall_mode == PCO_WALL_PAIR;
    uint32_t* vid[2] = {NULL, NULL};
    c->n_victims = 0;
    if (pair && c->nb > 0) {
        /* ids must be 0..N-1, and there must be a victim for every ionization */
        if (e->n != c->next_id[0] || i->n != c->next_id[1]) c->err |= PCO_ERR_IDS;
        if (c->nb > PCO_PAIR_MAX_BIRTHS || c->nb > e->n || c->nb > i->n) {
            c->err |= PCO_ERR_BIRTHS;
            c->nb = 0;
        }
    }
    /* ionization products: ids by rank of the parent id within the step
     * (pair sink: the ids of the victims of the same rank) */
    if (c->nb > 0) {
        qsort(c->births, (size_t)c->nb, sizeof(birth_t), cmp_birth);
        if (pair) {
            vid[0] = (uint32_t*)malloc((size_t)c->nb * sizeof(uint32_t));
            vid[1] = (uint32_t*)malloc((size_t)c->nb * sizeof(uint32_t));
            if (!vid[0] || !vid[1]) { free(vid[0]); free(vid[1]); return -3; }
            int rc2 = pair_victims(c, PCO_ELECTRON, c->nb, key, vid[0]);
            if (!rc2) rc2 = pair_victims(c, PCO_ION, c->nb, key, vid[1]);
            if (rc2) { free(vid[0]); free(vid[1]); return rc2; }
        }
        if (grow(e, e->n + c->nb) || grow(i, i->n + c->nb)) return -3;
        for (int64_t r = 0; r < c->nb; ++r) {
            const birth_t* b = &c->births[r];
            int64_t ne = e->n++, ni = i->n++;
            e->x[ne] = b->x; e->vx[ne] = b->ve[0]; e->vy[ne] = b->ve[1]; e->vz[ne] = b->ve[2];
            e->id[ne] = pair ? vid[0][r] : (uint32_t)(c->next_id[PCO_ELECTRON] + r);
            i->x[ni] = b->x; i->vx[ni] = b->vi[0]; i->vy[ni] = b->vi[1]; i->vz[ni] = b->vi[2];
            i->id[ni] = pair ? vid[1][r] : (uint32_t)(c->next_id[PCO_ION] + r);
        }
        if (pair) {   /* kept for pco_get_victims */
            free(c->victims[0]);
            free(c->victims[1]);
            c->victims[0] = vid[0];
            c->victims[1] = vid[1];
            c->n_victims = c->nb;
        }
        if (!pair) {
            c->next_id[PCO_ELECTRON] += c->nb;
            c->next_id[PCO_ION] += c->nb;
        }
        if (c->next_id[0] > 0xFFFFFFFFll || c->next_id[1] > 0xFFFFFFFFll) c->err |= PCO_ERR_IDS;
        if (grow_events(e, c->next_id[0]) || grow_events(i, c->next_id[1])) return -3;
    }
    c->births_last = c->nb;
    c->births_since_ion += c->nb;
    /* external circuit (section V): the anode potential of this field solve
     * from the conduction current of the step -- v_x after the push of the
     * particles still present, ions from their last subcycle step -- and the
     * gap's displacement current, backward Euler in time:
     * V' (1 + a) = V_source + R J + a V with a = R eps0 / (L dt) */
    if (c->cfg.circuit_R > 0.0) {
        const int64_t vi = ion_step ? c->vs_ia : c->vs_i;
        const double J = c->circ_jf * (double)(vi - c->vs_e);
        c->Vb = (c->cfg.V + c->cfg.circuit_R * J + c->circ_a * c->Vb) / (1.0 + c->circ_a);
        c->Jc = J;
        c->vs_e = 0;
        if (ion_step) {
            c->vs_i = c->vs_ia;
            c->vs_ia = 0;
        }
    }
    field_update(c);
    /* cathode emission (section V): J dt / (e W) electrons per step with the
     * fraction carried over, after the field solve; each has a flux-weighted
     * half-Maxwellian velocity at emit_T (v_x from a Rayleigh draw, v_y, v_z
     * normal) and has flown a uniform fraction of a step from x = 0; ids follow
     * the products' and the draws come from the new id's own stream */
    if (c->cfg.emit_J > 0.0) {
        const double ce = c->carry + c->emit_n;
        const int64_t n_emit = (int64_t)floor(ce);
        c->carry = ce - (double)n_emit;
        if (grow(e, e->n + n_emit)) return -3;
        for (int64_t r = 0; r < n_emit; ++r) {
            const uint32_t id = (uint32_t)(c->next_id[PCO_ELECTRON] + r);
            uint32_t ctr[4] = {id, (uint32_t)c->step, 0u, ST_EMIT}, w[4];
            pco_philox4x32_10(ctr, key, w);
            const double vx = c->emit_sig * sqrt(-2.0 * log(u52(w[0], w[1])));
            double x = vx * c->dt * u52(w[2], w[3]);
            if (!(x < c->L)) x = 0.0;
            kstream_t ks;
            ks_init(&ks, key, id, (uint32_t)c->step, ST_EMIT);
            double g[2];
            gauss2(&ks, g);
            const int64_t m = e->n++;
            e->x[m] = x; e->vx[m] = vx; e->vy[m] = c->emit_sig * g[0]; e->vz[m] = c->emit_sig * g[1];
            e->id[m] = id;
        }
        c->next_id[PCO_ELECTRON] += n_emit;
        if (c->next_id[0] > 0xFFFFFFFFll) c->err |= PCO_ERR_IDS;
        if (grow_events(e, c->next_id[0])) return -3;
    }
    c->step += 1;
    return 0;
}

int pco_set_circuit(pco_column* c, double V_anode, int64_t vsum_ion, double emit_carry)
{
    if (!c || !(emit_carry >= 0.0 && emit_carry < 1.0)) return -1;
    c->Vb = V_anode;
    c->vs_i = vsum_ion;
    c->carry = emit_carry;
    return 0;
}

int pco_get_circuit(const pco_column* c, double out[3], int64_t* vsum_ion)
{
    if (!c || !vsum_ion) return -1;
    out[0] = c->Vb;
    out[1] = c->Jc;
    out[2] = c->carry;
    *vsum_ion = c->vs_i;
    return 0;
}

int pco_step(pco_column* c, int64_t n)
{
    if (!c || n < 0) return -1;
    for (int64_t k = 0; k < n; ++k) {
        int rc = one_step(c);
        if (rc) return rc;
    }
    return 0;
}

/* -------------------------------------------------------------- accessors */
int pco_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int32_t pco_n_nodes(const pco_column* c) { return c ? c->nn : -1; }
int64_t pco_count(const pco_column* c, int s) { return (c && (s == 0 || s == 1)) ? c->sp[s].n : -1; }
int64_t pco_step_index(const pco_column* c) { return c ? c->step : -1; }
int64_t pco_next_id(const pco_column* c, int s) { return (c && (s == 0 || s == 1)) ? c->next_id[s] : -1; }
uint32_t pco_errors(const pco_column* c) { return c ? c->err : 0u; }

double pco_constant(const pco_column* c, int which)
{
    if (!c) return NAN;
    switch (which) {
    case 0: return c->dx;
    case 1: return c->nu_max;
    case 2: return c->P_null;
    case 3: return c->W;
    case 4: return c->Ng;
    case 5: return c->P_cx;
    default: return NAN;
    }
}

int pco_get_state(const pco_column* c, int s, double* x, double* vx, double* vy, double* vz,
                  uint32_t* id)
{
    if (!c || (s != 0 && s != 1)) return -1;
    const species_t* p = &c->sp[s];
    if (p->n == 0) return 0;   /* nothing to copy (an empty species has no arrays) */
    size_t nb = (size_t)p->n * sizeof(double);
    if (x) memcpy(x, p->x, nb);
    if (vx) memcpy(vx, p->vx, nb);
    if (vy) memcpy(vy, p->vy, nb);
    if (vz) memcpy(vz, p->vz, nb);
    if (id) memcpy(id, p->id, (size_t)p->n * sizeof(uint32_t));
    return 0;
}

int pco_set_state(pco_column* c, int s, int64_t n, const double* x, const double* vx,
                  const double* vy, const double* vz, const uint32_t* id)
{
    if (!c || (s != 0 && s != 1) || n < 0) return -1;
    species_t* p = &c->sp[s];
    if (grow(p, n)) return -3;
    int64_t maxid = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!(x[k] >= 0.0 && x[k] < c->L)) return -2;
        if ((int64_t)id[k] + 1 > maxid) maxid = (int64_t)id[k] + 1;
    }
    if (n > 0) {
        size_t nb = (size_t)n * sizeof(double);
        memcpy(p->x, x, nb); memcpy(p->vx, vx, nb); memcpy(p->vy, vy, nb); memcpy(p->vz, vz, nb);
        memcpy(p->id, id, (size_t)n * sizeof(uint32_t));
    }
    p->n = n;
    if (maxid > c->next_id[s]) c->next_id[s] = maxid;
    if (grow_events(p, c->next_id[s])) return -3;
    return 0;
}

int pco_set_balance(pco_column* c, int64_t births_last, int64_t births_since_ion)
{
    if (!c || births_last < 0 || births_since_ion < 0) return -1;
    c->births_last = births_last;
    c->births_since_ion = births_since_ion;
    return 0;
}

int64_t pco_get_victims(const pco_column* c, int s, uint32_t* out, int64_t cap)
{
    if (!c || (s != 0 && s != 1) || cap < 0) return -1;
    int64_t m = c->n_victims < cap ? c->n_victims : cap;
    for (int64_t r = 0; r < m; ++r) out[r] = c->victims[s][r];
    return c->n_victims;
}

int pco_get_balance(const pco_column* c, int64_t out[2])
{
    if (!c || !out) return -1;
    out[0] = c->births_last;
    out[1] = c->births_since_ion;
    return 0;
}

int pco_set_counters(pco_column* c, int64_t step, int64_t next_e, int64_t next_i)
{
    if (!c || step < 0) return -1;
    c->step = step;
    c->next_id[0] = next_e;
    c->next_id[1] = next_i;
    if (grow_events(&c->sp[0], next_e) || grow_events(&c->sp[1], next_i)) return -3;
    return 0;
}

int pco_get_field(const pco_column* c, double* E, int64_t* rho_e, int64_t* rho_i)
{
    if (!c) return -1;
    if (E) memcpy(E, c->E, (size_t)c->nn * sizeof(double));
    if (rho_e) memcpy(rho_e, c->rho_e, (size_t)c->nn * sizeof(int64_t));
    if (rho_i) memcpy(rho_i, c->rho_i, (size_t)c->nn * sizeof(int64_t));
    return 0;
}

int pco_set_field(pco_column* c, const double* E)
{
    if (!c || !E) return -1;
    memcpy(c->E, E, (size_t)c->nn * sizeof(double));
    if (c->periodic) c->E[c->nc] = c->E[0];
    return 0;
}

int pco_get_events(const pco_column* c, int s, uint8_t* ev, int64_t len)
{
    if (!c || (s != 0 && s != 1) || !ev) return -1;
    int64_t n = c->next_id[s] < len ? c->next_id[s] : len;
    if (n > c->sp[s].evcap) n = c->sp[s].evcap;
    if (n > 0) memcpy(ev, c->sp[s].ev, (size_t)n);
    return 0;
}

/* ----------------------------------------------------------------- moments */
/* cell moments behind the diagnostics of section III: densities, mean energy
 * (T_e = 2/3 of it), flux, energy flux, ionization counts and the EEPF
 * histogram (normalised on the host as F = f / sqrt(eps)). */
int pco_moments(pco_column* c, int32_t cpg, int32_t reset_iz, int64_t* out)
{
    if (!c || !out || cpg < 1) return -1;
    const int nc = c->nc;
    const int ng = (nc + cpg - 1) / cpg;
    memset(out, 0, (size_t)(7 * nc + ng * 240) * sizeof(int64_t));
    const species_t* e = &c->sp[PCO_ELECTRON];
    const int64_t len = 7 * (int64_t)nc + (int64_t)ng * 240;
    (void)len;   /* the reduction's extent (OpenMP build) */
    #pragma omp parallel for schedule(static) reduction(+ : out[:len])
    for (int64_t k = 0; k < e->n; ++k) {
        int j; double f;
        cell_of(c, e->x[k], &j, &f);
        double vx = e->vx[k], vy = e->vy[k], vz = e->vz[k];
        double eps = c->c_eps * ((vx * vx + vy * vy) + vz * vz);
        out[j] += 1;
        out[nc + j] += (int64_t)(eps * 1048576.0);
        out[2 * nc + j] += (int64_t)(vx * 1024.0);
        out[3 * nc + j] += (int64_t)(eps * vx * 16.0);
        int b = (int)(eps * 4.0);
        if (b < 240) out[7 * nc + (j / cpg) * 240 + b] += 1;
    }
    const species_t* i = &c->sp[PCO_ION];
    #pragma omp parallel for schedule(static) reduction(+ : out[:len])
    for (int64_t k = 0; k < i->n; ++k) {
        int j; double f;
        cell_of(c, i->x[k], &j, &f);
        out[4 * nc + j] += 1;
        out[5 * nc + j] += (int64_t)(i->vx[k] * 1024.0);
    }
    for (int j = 0; j < nc; ++j) out[6 * nc + j] = c->iz[j];
    if (reset_iz) memset(c->iz, 0, (size_t)nc * sizeof(int64_t));
    return 0;
}
