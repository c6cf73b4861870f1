/*
 * sph_oracle.c -- plain FP64 CPU reference of one time step of the weakly
 * compressible SPH method with the dummy-particle wall treatment of
 * Rezavand, Zhang & Hu, "Generalised and efficient wall boundary condition
 * treatment in GPU-accelerated SPH" (arXiv 2110.02621).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The HIP product
 * path neither links nor calls it, and it shares no code with it.
 *
 * Style: every quantity is double, every sum runs in a fixed order, there is
 * no blocking, fusion or reordering beyond what the paper's equations state.
 * The library is built with -O2 -ffp-contract=off (no fused multiply-add).
 * Work is parallel over particles only (OpenMP); each particle's own sum is
 * sequential, so results do not depend on the thread count.
 *
 * Notation follows the paper: r_ij = r_i - r_j, e_ij = -r_ij/|r_ij|,
 * grad_i W_ij = W'(|r_ij|) r_ij/|r_ij|, m = particle mass, c = sound speed.
 *
 * Readings of points the paper leaves open (each listed with its reason in
 * the design notes of the repository):
 *   kernel      quintic Wendland C2 with kappa = 2 (Sec. 2.3, Fig. 1 caption;
 *               Sec. 4 opening paragraph): W = a_d (1-q/2)^4 (1+2q), q = r/h.
 *   Eq. (12)    the hydrostatic term carries the fluid density (Adami form):
 *               p_w = [sum p_f W + (g - a_w) . sum rho_f r_wf W] / sum W,
 *               and p_w = 0 when no fluid particle is within the support.
 *   wall rho    rho_w from the EOS, Eq. (3), with p_w; wall mass rho0 dx^d.
 *   sigma^0     one scalar per phase: the full-support lattice sum.
 *   reinit      Eq. (17) at the start of every step with rho* = rho^n.
 *   viscosity   the paper is inviscid; the viscous term here is the
 *               Morris-Fox-Zhu (1997) form with eta^2 = 0.01 h^2, walls
 *               no-slip (v_j = the wall velocity).
 *   penalty     Eqs. (13)-(15) with the unsigned normal distance
 *               delta = 2 |(r_i - r_w) . n_w| / dx (the magnitude of the
 *               projection, as in the penalty parameter itself) and the
 *               dimensionally consistent magnitude
 *               F_p = -2 gamma_p sum_w m_w/(rho_i rho_w) (1-delta)^2
 *                     |p_i e_iw . n_w| W'(r_iw) n_w   for delta < 1.
 *   normals     Eq. (16) over wall particles only, V_j = dx^d; n_w = 0 when
 *               |Psi| h <= 1e-4 (cancellation inside the wall: such sums
 *               are ~1e-14 in FP64 while real normals have |Psi| h > 5e-3).
 *   schedule    per step: Eq. (17) reinit at r^n, Eq. (19) half kick,
 *               Eq. (20) drift, cell rebuild, Eq. (12) wall pressure,
 *               Eq. (9)+(21) density update, Eq. (10)+(22) second kick.
 *   two phases  (two_phase = 1) fluid particles with index >= n_heavy are
 *               the light phase (reference density rho0_light, the same
 *               sound speed, Sec. 2.6): every particle carries its own
 *               reference density and mass rho0_k dx^d; the light phase is
 *               reinitialised by Eq. (18) and takes its density from the
 *               number density after the drift instead of Eq. (9) (Secs.
 *               2.1, 2.5, 2.6); Eq. (12) is divided by rho_f term by term
 *               (Sec. 2.3); a wall dummy takes the reference density and
 *               mass of the fluid particle it interacts with; the penalty
 *               of Eq. (13) acts on light-phase particles (and on all when
 *               penalty_on).  The Riemann solution of Eqs. (7)-(8) is used
 *               as printed for pairs of either phase: its density weighting
 *               carries the density ratio.
 *   moving walls a prescribed rigid translation of every wall dummy (the
 *               tank), X(t) = A0 sin(2 pi f0 t) (Sec. 4, sloshing tank),
 *               solved as it is stated, in the fixed frame: the walls sit at
 *               x_w(0) + X(t_n); in the pair terms of a step (evaluated at
 *               r^{n+1} with v^{n+1/2}) they move with the velocity of that
 *               step's displacement, (X(t_{n+1}) - X(t_n))/dt, which enters
 *               the Riemann states of Eq. (7), v* of Eq. (9) and the
 *               no-slip viscous term; a_w of Eq. (12) is X''(t_{n+1}).  At
 *               the initial state (t = 0) the walls move with X'(0).
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ALLOC 1
#define ORC_ERR_NBR_CAP 2
#define ORC_ERR_ARG 3

/* Neighbour buffer size per query point.  A compressed 3-D lattice has about
 * 81 neighbours inside 2h; 4096 leaves room for any physical state. */
#define ORC_NBR_CAP 4096

typedef struct {
    int32_t dim;        /* 2 or 3; the last axis is vertical */
    int32_t penalty_on; /* 1: Eq. (13) acts on every fluid-wall pair */
    double dx;          /* initial particle spacing */
    double h;           /* smoothing length */
    double rho0;        /* reference density */
    double c;           /* artificial sound speed, Eq. (3) */
    double mu;          /* dynamic viscosity (0 = inviscid, as the paper) */
    double gamma_p;     /* penalty strength, Eq. (13) */
    double dt;          /* time step */
    double g[3];        /* body force */
    double a_wall[3];   /* wall acceleration in Eq. (12) */
    double sigma0;      /* reference number density of Eq. (17) */
    int32_t two_phase;  /* 1: particles with index >= n_heavy are the light phase */
    int32_t cross_phase; /* two phases, momentum of a light particle i with a heavy
                            neighbour j: 0 = the printed Riemann p* of Eq. (8) with each
                            side's own state; 1 = the light phase sees the heavy particle
                            as a moving wall dummy: p* of Eq. (11) with p_w = p_j, the
                            light phase's EOS density rho0_light + p_w/c^2 and mass
                            rho0_light dx^d (Secs. 2.1, 2.5); 2 = the same with p_w the
                            pressure extrapolated to j from its light neighbours by the
                            two-phase form of Eq. (12), a_w = the tank's acceleration */
    int64_t n_heavy;    /* number of heavy-phase fluid particles (indices first) */
    double rho0_light;  /* reference density of the light phase */
    double wall_v[3];   /* velocity of the wall dummies in the pair terms (orc_step sets
                           it from the tank motion) */
    double motion_amp[3]; /* prescribed rigid translation of all walls (the tank):  */
    double motion_freq;   /* X(t) = motion_amp sin(2 pi motion_freq t), t = step dt  */
} orc_params;

/* ------------------------------------------------------------------ */
/* Kernel: quintic Wendland C2, support 2h (Sec. 2.3, Sec. 4).         */
/* ------------------------------------------------------------------ */

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static double wendland_alpha(int dim, double h)
{
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    return 21.0 / (16.0 * M_PI * h * h * h);
}

double orc_W(int dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return wendland_alpha(dim, h) * t * t * t * t * (1.0 + 2.0 * q);
}

/* dW/dr */
double orc_dW(int dim, double h, double r)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double t = 1.0 - 0.5 * q;
    return -5.0 * wendland_alpha(dim, h) * q * t * t * t / h;
}

/* ------------------------------------------------------------------ */
/* Neighbour search with a cell list (Sec. 3; Table 1 counts the sort   */
/* as part of the neighbour search).  A counting sort by cell key is    */
/* stable: particles of one cell keep their input order.                */
/* ------------------------------------------------------------------ */

/* Stable counting sort of n keys in [0, nkey): start[nkey+1] holds the
 * first slot of each key, order[n] the input indices in sorted order. */
int orc_counting_sort(int64_t n, const int32_t *key, int32_t nkey,
                      int32_t *start, int32_t *order)
{
    int64_t *fill = (int64_t *)calloc((size_t)nkey + 1, sizeof(int64_t));
    if (!fill) return ORC_ERR_ALLOC;
    for (int32_t k = 0; k <= nkey; ++k) start[k] = 0;
    for (int64_t i = 0; i < n; ++i) start[key[i] + 1] += 1;
    for (int32_t k = 0; k < nkey; ++k) start[k + 1] += start[k];
    for (int32_t k = 0; k < nkey; ++k) fill[k] = start[k];
    for (int64_t i = 0; i < n; ++i) order[fill[key[i]]++] = (int32_t)i;
    free(fill);
    return ORC_OK;
}

typedef struct {
    int dim;
    int64_t n;
    const double *x; /* n * dim, row-major */
    double lo[3];
    double L;
    int64_t nc[3];
    int32_t *start;
    int32_t *order;
} cellset;

static void cs_free(cellset *s)
{
    free(s->start);
    free(s->order);
    s->start = NULL;
    s->order = NULL;
}

static int cs_build(cellset *s, int dim, int64_t n, const double *x, double L)
{
    s->dim = dim;
    s->n = n;
    s->x = x;
    s->L = L;
    s->start = NULL;
    s->order = NULL;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        lo[k] = n ? x[k] : 0.0;
        hi[k] = lo[k];
    }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < dim; ++k) {
            double v = x[i * dim + k];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < dim) {
            s->lo[k] = lo[k] - L;
            s->nc[k] = (int64_t)floor((hi[k] - s->lo[k]) / L) + 2;
        } else {
            s->lo[k] = 0.0;
            s->nc[k] = 1;
        }
        ncell *= s->nc[k];
    }
    if (ncell > INT32_MAX - 1) return ORC_ERR_ARG;
    int32_t *key = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    s->start = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    s->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!key || !s->start || !s->order) {
        free(key);
        cs_free(s);
        return ORC_ERR_ALLOC;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) c[k] = (int64_t)floor((x[i * dim + k] - s->lo[k]) / L);
        key[i] = (int32_t)(c[0] + s->nc[0] * (c[1] + s->nc[1] * c[2]));
    }
    int rc = orc_counting_sort(n, key, (int32_t)ncell, s->start, s->order);
    free(key);
    return rc;
}

/* All j of the set with |xi - x_j|^2 < rc2, visiting cells in ascending
 * (z, y, x) order and particles of a cell in sorted order.  Returns the
 * count, or -1 when more than cap were found. */
static int cs_query(const cellset *s, const double *xi, double rc2, int32_t *out, int cap)
{
    if (s->n == 0) return 0;
    int dim = s->dim;
    int64_t c[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        double f = floor((xi[k] - s->lo[k]) / s->L);
        if (f < -2.0) return 0;
        if (f > (double)s->nc[k] + 1.0) return 0;
        c[k] = (int64_t)f;
    }
    int64_t zlo = dim == 3 ? c[2] - 1 : 0, zhi = dim == 3 ? c[2] + 1 : 0;
    int cnt = 0;
    for (int64_t cz = zlo; cz <= zhi; ++cz) {
        if (cz < 0 || cz >= s->nc[2]) continue;
        for (int64_t cy = c[1] - 1; cy <= c[1] + 1; ++cy) {
            if (cy < 0 || cy >= s->nc[1]) continue;
            for (int64_t cx = c[0] - 1; cx <= c[0] + 1; ++cx) {
                if (cx < 0 || cx >= s->nc[0]) continue;
                int64_t key = cx + s->nc[0] * (cy + s->nc[1] * cz);
                for (int32_t a = s->start[key]; a < s->start[key + 1]; ++a) {
                    int32_t j = s->order[a];
                    double r2 = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        double d = xi[k] - s->x[(int64_t)j * dim + k];
                        r2 += d * d;
                    }
                    if (r2 < rc2) {
                        if (cnt >= cap) return -1;
                        out[cnt++] = j;
                    }
                }
            }
        }
    }
    return cnt;
}

/* Neighbour counts and lists of every point of set A against set B, found
 * through B's cell list (pairs with |r_ab| < 2h, the point itself included
 * when A and B are the same set).  Pass list = NULL to count only. */
int orc_neighbours(int dim, double h, int64_t na, const double *xa, int64_t nb,
                   const double *xb, int32_t *count, const int64_t *offset, int32_t *list)
{
    cellset s;
    int rc = cs_build(&s, dim, nb, xb, 2.0 * h);
    if (rc) return rc;
    double rc2 = 4.0 * h * h;
    int err = 0;
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < na; ++i) {
            int cnt = cs_query(&s, xa + i * dim, rc2, nbr, ORC_NBR_CAP);
            if (cnt < 0) {
                err = ORC_ERR_NBR_CAP;
                cnt = 0;
            }
            count[i] = cnt;
            if (list)
                for (int a = 0; a < cnt; ++a) list[offset[i] + a] = nbr[a];
        }
        free(nbr);
    }
    cs_free(&s);
    return err;
}

/* Brute-force O(NA*NB) pair test in the precision the kernel decides in.
 * Points are given as integer cell coordinates plus an in-cell offset; the
 * relative vector is d_k = (o_ak - o_bk) - (c_bk - c_ak) L, rounded after
 * each operation, and r^2 = (d_0 d_0 + d_1 d_1) + d_2 d_2 without fused
 * multiply-add.  single = 1 evaluates all of it in IEEE binary32 (offsets,
 * L and rc2 must then hold binary32 values).  Cells must differ by at most
 * one per axis for a pair (larger differences are never pairs since L >= 2h).
 * Writes 1 into hit[a*nb + b] for every pair. */
int orc_pairs_bruteforce(int dim, int single, int64_t na, const int32_t *ca, const double *oa,
                         int64_t nb, const int32_t *cb, const double *ob, double L, double rc2,
                         uint8_t *hit)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < na; ++a) {
        for (int64_t b = 0; b < nb; ++b) {
            int far = 0;
            int s[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                s[k] = cb[b * dim + k] - ca[a * dim + k];
                if (s[k] < -1 || s[k] > 1) far = 1;
            }
            uint8_t is_pair = 0;
            if (!far) {
                if (single) {
                    float d[3] = {0.f, 0.f, 0.f};
                    for (int k = 0; k < dim; ++k) {
                        float t = (float)oa[a * dim + k] - (float)ob[b * dim + k];
                        d[k] = t - (float)s[k] * (float)L;
                    }
                    float r2 = d[0] * d[0] + d[1] * d[1];
                    if (dim == 3) r2 = r2 + d[2] * d[2];
                    is_pair = r2 < (float)rc2;
                } else {
                    double d[3] = {0.0, 0.0, 0.0};
                    for (int k = 0; k < dim; ++k) {
                        double t = oa[a * dim + k] - ob[b * dim + k];
                        d[k] = t - (double)s[k] * L;
                    }
                    double r2 = d[0] * d[0] + d[1] * d[1];
                    if (dim == 3) r2 = r2 + d[2] * d[2];
                    is_pair = r2 < rc2;
                }
            }
            hit[a * nb + b] = is_pair;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Riemann solver between two particle states, Eqs. (7)-(8).           */
/* ------------------------------------------------------------------ */

typedef struct {
    double Ubar, Ustar, Pbar, pstar, beta;
} riemann_out;

static riemann_out riemann(double rhoL, double UL, double pL, double rhoR, double UR, double pR,
                           double c)
{
    riemann_out o;
    double rhobar = 0.5 * (rhoL + rhoR);
    o.Ubar = (rhoL * UL + rhoR * UR) / (rhoL + rhoR);
    o.Pbar = (rhoL * pR + rhoR * pL) / (rhoL + rhoR);
    o.Ustar = o.Ubar + 0.5 * (pL - pR) / (c * rhobar);
    double jump = UL - UR;
    o.beta = fmin(3.0 * fmax(jump, 0.0), c);
    o.pstar = o.Pbar + rhoL * rhoR * o.beta * jump / (rhoL + rhoR);
    return o;
}

/* Exposed for the worked-example tests: writes U*, p*, U_bar, P_bar, beta. */
void orc_riemann(double rhoL, double UL, double pL, double rhoR, double UR, double pR, double c,
                 double *out5)
{
    riemann_out o = riemann(rhoL, UL, pL, rhoR, UR, pR, c);
    out5[0] = o.Ustar;
    out5[1] = o.pstar;
    out5[2] = o.Ubar;
    out5[3] = o.Pbar;
    out5[4] = o.beta;
}

/* Phase of fluid particle i and its reference density rho0_k. */
static int is_light(const orc_params *P, int64_t i) { return P->two_phase && i >= P->n_heavy; }
static double ref_rho(const orc_params *P, int64_t i) { return is_light(P, i) ? P->rho0_light : P->rho0; }
/* Equation of state, Eq. (3), for fluid particle i. */
static double eos_p(const orc_params *P, int64_t i, double rho) { return P->c * P->c * (rho - ref_rho(P, i)); }
/* Its inverse, for a wall dummy interacting with fluid particle i. */
static double eos_rho(const orc_params *P, int64_t i, double p) { return ref_rho(P, i) + p / (P->c * P->c); }
/* Particle mass rho0_k dx^d of fluid particle i (and of a wall dummy seen by i). */
static double mass_of(const orc_params *P, int64_t i)
{
    double v = P->dim == 2 ? P->dx * P->dx : P->dx * P->dx * P->dx;
    return ref_rho(P, i) * v;
}

static double dot(int dim, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < dim; ++k) s += a[k] * b[k];
    return s;
}

/* ------------------------------------------------------------------ */
/* Number density sigma_i = sum_j W_ij over fluid and wall particles,  */
/* j = i included (Eq. (4) without the mass; Eq. (17) definition).     */
/* ------------------------------------------------------------------ */
int orc_sigma(const orc_params *P, int64_t nf, const double *fx, int64_t nw, const double *wx,
              int64_t nq, const int64_t *qidx, double *sigma)
{
    int dim = P->dim;
    double h = P->h, rc2 = 4.0 * h * h;
    cellset sf, sw;
    int rc = cs_build(&sf, dim, nf, fx, 2.0 * h);
    if (rc) return rc;
    rc = cs_build(&sw, dim, nw, wx, 2.0 * h);
    if (rc) {
        cs_free(&sf);
        return rc;
    }
    int err = 0;
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t a_q = 0; a_q < nq; ++a_q) {
            int64_t i = qidx ? qidx[a_q] : a_q;
            const double *xi = fx + i * dim;
            double s = 0.0;
            for (int set = 0; set < 2; ++set) {
                const cellset *cs = set == 0 ? &sf : &sw;
                int cnt = cs_query(cs, xi, rc2, nbr, ORC_NBR_CAP);
                if (cnt < 0) {
                    err = ORC_ERR_NBR_CAP;
                    cnt = 0;
                }
                for (int a = 0; a < cnt; ++a) {
                    const double *xj = cs->x + (int64_t)nbr[a] * dim;
                    double r2 = 0.0;
                    for (int k = 0; k < dim; ++k) r2 += (xi[k] - xj[k]) * (xi[k] - xj[k]);
                    s += orc_W(dim, h, sqrt(r2));
                }
            }
            sigma[a_q] = s;
        }
        free(nbr);
    }
    cs_free(&sf);
    cs_free(&sw);
    return err;
}

/* Density reinitialisation for free-surface flow, Eq. (17):
 * rho = rho0 sigma/sigma0 + max(0, rho* - rho0 sigma/sigma0) rho0/rho*;
 * for the light phase of a two-phase run the internal-flow form, Eq. (18):
 * rho = rho0 sigma/sigma0. */
void orc_reinit(const orc_params *P, int64_t n, const double *sigma, const double *rho_star,
                double *rho)
{
    for (int64_t i = 0; i < n; ++i) {
        double r0 = ref_rho(P, i);
        double rs = r0 * sigma[i] / P->sigma0;
        if (is_light(P, i))
            rho[i] = rs;
        else
            rho[i] = rs + fmax(0.0, rho_star[i] - rs) * r0 / rho_star[i];
    }
}

/* Reference number density: the full-support lattice sum around one site
 * of a square (2-D) or cubic (3-D) lattice of spacing dx. */
double orc_sigma0(int dim, double dx, double h)
{
    int R = (int)ceil(2.0 * h / dx) + 1;
    double s = 0.0;
    int zr = dim == 3 ? R : 0;
    for (int kz = -zr; kz <= zr; ++kz)
        for (int ky = -R; ky <= R; ++ky)
            for (int kx = -R; kx <= R; ++kx) {
                double r = dx * sqrt((double)(kx * kx + ky * ky + kz * kz));
                s += orc_W(dim, h, r);
            }
    return s;
}

/* ------------------------------------------------------------------ */
/* Wall dummy pressure by force balance, Eq. (12) (Adami form, see the */
/* file header), one value per wall particle.                          */
/* ------------------------------------------------------------------ */
int orc_wall_pressure(const orc_params *P, int64_t nw, const double *wx, int64_t nf,
                      const double *fx, const double *frho, int64_t nq, const int64_t *qidx,
                      double *pw)
{
    int dim = P->dim;
    double h = P->h, rc2 = 4.0 * h * h;
    double gw[3];
    for (int k = 0; k < 3; ++k) gw[k] = P->g[k] - P->a_wall[k];
    cellset sf;
    int rc = cs_build(&sf, dim, nf, fx, 2.0 * h);
    if (rc) return rc;
    int err = 0;
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t a_q = 0; a_q < nq; ++a_q) {
            int64_t w = qidx ? qidx[a_q] : a_q;
            const double *xw = wx + w * dim;
            int cnt = cs_query(&sf, xw, rc2, nbr, ORC_NBR_CAP);
            if (cnt < 0) {
                err = ORC_ERR_NBR_CAP;
                cnt = 0;
            }
            double sumW = 0.0, sumPW = 0.0, sumRW[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < cnt; ++a) {
                int64_t f = nbr[a];
                double rwf[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
                for (int k = 0; k < dim; ++k) {
                    rwf[k] = xw[k] - fx[f * dim + k];
                    r2 += rwf[k] * rwf[k];
                }
                double W = orc_W(dim, h, sqrt(r2));
                double p_f = eos_p(P, f, frho[f]);
                if (P->two_phase) {
                    /* Eq. (12) divided by rho_f term by term (Sec. 2.3) */
                    sumW += W / frho[f];
                    sumPW += p_f / frho[f] * W;
                    for (int k = 0; k < dim; ++k) sumRW[k] += rwf[k] * W;
                } else {
                    sumW += W;
                    sumPW += p_f * W;
                    for (int k = 0; k < dim; ++k) sumRW[k] += frho[f] * rwf[k] * W;
                }
            }
            pw[a_q] = sumW > 0.0 ? (sumPW + dot(dim, gw, sumRW)) / sumW : 0.0;
        }
        free(nbr);
    }
    cs_free(&sf);
    return err;
}

/* ------------------------------------------------------------------ */
/* Wall normal estimate, Eq. (16): Psi_w = -sum_{j in wall} V_j grad_w  */
/* W_wj, V_j = dx^d, n_w = Psi/|Psi| (0 when Psi cancels).              */
/* ------------------------------------------------------------------ */
int orc_normals(const orc_params *P, int64_t nw, const double *wx, double *nrm, double *psi)
{
    int dim = P->dim;
    double h = P->h, rc2 = 4.0 * h * h;
    double V = dim == 2 ? P->dx * P->dx : P->dx * P->dx * P->dx;
    cellset sw;
    int rc = cs_build(&sw, dim, nw, wx, 2.0 * h);
    if (rc) return rc;
    int err = 0;
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t w = 0; w < nw; ++w) {
            const double *xw = wx + w * dim;
            int cnt = cs_query(&sw, xw, rc2, nbr, ORC_NBR_CAP);
            if (cnt < 0) {
                err = ORC_ERR_NBR_CAP;
                cnt = 0;
            }
            double Psi[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < cnt; ++a) {
                const double *xj = wx + (int64_t)nbr[a] * dim;
                double d[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
                for (int k = 0; k < dim; ++k) {
                    d[k] = xw[k] - xj[k];
                    r2 += d[k] * d[k];
                }
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double dW = orc_dW(dim, h, r);
                for (int k = 0; k < dim; ++k) Psi[k] -= V * dW * d[k] / r;
            }
            double norm = sqrt(dot(dim, Psi, Psi));
            for (int k = 0; k < dim; ++k) {
                if (psi) psi[w * dim + k] = Psi[k];
                nrm[w * dim + k] = norm * h > 1e-4 ? Psi[k] / norm : 0.0;
            }
        }
        free(nbr);
    }
    cs_free(&sw);
    return err;
}

/* ------------------------------------------------------------------ */
/* Mass conservation with the Riemann solution, Eq. (9):               */
/* drho_i/dt = 2 rho_i sum_j (m_j/rho_j) (v_i - v*) . grad_i W_ij,     */
/* v* = U* e_ij + (rho_i v_i + rho_j v_j)/(rho_i + rho_j) - Ubar e_ij. */
/* Wall dummies enter as particles with v = 0, p = p_w and the EOS      */
/* density (Sec. 2.3).                                                  */
/* ------------------------------------------------------------------ */
int orc_continuity(const orc_params *P, int64_t nf, const double *fx, const double *fv,
                   const double *frho, int64_t nw, const double *wx, const double *pw,
                   int64_t nq, const int64_t *qidx, double *drhodt)
{
    int dim = P->dim;
    double h = P->h, rc2 = 4.0 * h * h;
    cellset sf, sw;
    int rc = cs_build(&sf, dim, nf, fx, 2.0 * h);
    if (rc) return rc;
    rc = cs_build(&sw, dim, nw, wx, 2.0 * h);
    if (rc) {
        cs_free(&sf);
        return rc;
    }
    int err = 0;
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t a_q = 0; a_q < nq; ++a_q) {
            int64_t i = qidx ? qidx[a_q] : a_q;
            const double *xi = fx + i * dim, *vi = fv + i * dim;
            double rho_i = frho[i], p_i = eos_p(P, i, rho_i);
            double sum = 0.0;
            for (int set = 0; set < 2; ++set) {
                const cellset *cs = set == 0 ? &sf : &sw;
                int cnt = cs_query(cs, xi, rc2, nbr, ORC_NBR_CAP);
                if (cnt < 0) {
                    err = ORC_ERR_NBR_CAP;
                    cnt = 0;
                }
                for (int a = 0; a < cnt; ++a) {
                    int64_t j = nbr[a];
                    const double *xj = cs->x + j * dim;
                    double rij[3] = {0, 0, 0}, r2 = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        rij[k] = xi[k] - xj[k];
                        r2 += rij[k] * rij[k];
                    }
                    if (r2 == 0.0) continue; /* j = i or coincident: no gradient */
                    double r = sqrt(r2);
                    double e[3] = {0, 0, 0}, gradW[3] = {0, 0, 0}, vj[3] = {0, 0, 0};
                    double dW = orc_dW(dim, h, r);
                    for (int k = 0; k < dim; ++k) {
                        e[k] = -rij[k] / r;
                        gradW[k] = dW * rij[k] / r;
                    }
                    double rho_j, p_j, m_j;
                    if (set == 0) {
                        for (int k = 0; k < dim; ++k) vj[k] = fv[j * dim + k];
                        rho_j = frho[j];
                        p_j = eos_p(P, j, rho_j);
                        m_j = mass_of(P, j);
                    } else {
                        for (int k = 0; k < dim; ++k) vj[k] = P->wall_v[k];
                        p_j = pw[j];
                        rho_j = eos_rho(P, i, p_j);
                        m_j = mass_of(P, i);
                    }
                    /* Eq. (7): left state from i, right state from j. */
                    double UL = dot(dim, vi, e), UR = dot(dim, vj, e);
                    riemann_out rs = riemann(rho_i, UL, p_i, rho_j, UR, p_j, P->c);
                    double vstar[3] = {0, 0, 0}, diff[3] = {0, 0, 0};
                    for (int k = 0; k < dim; ++k) {
                        vstar[k] = rs.Ustar * e[k] + (rho_i * vi[k] + rho_j * vj[k]) / (rho_i + rho_j) -
                                   rs.Ubar * e[k];
                        diff[k] = vi[k] - vstar[k];
                    }
                    sum += m_j / rho_j * dot(dim, diff, gradW);
                }
            }
            drhodt[a_q] = 2.0 * rho_i * sum;
        }
        free(nbr);
    }
    cs_free(&sf);
    cs_free(&sw);
    return err;
}

/* ------------------------------------------------------------------ */
/* Momentum with the Riemann solution, Eq. (10), fluid-wall p* of      */
/* Eq. (11), penalty force Eqs. (13)-(15), viscous term and gravity.   */
/* ------------------------------------------------------------------ */
int orc_momentum(const orc_params *P, int64_t nf, const double *fx, const double *fv,
                 const double *frho, int64_t nw, const double *wx, const double *pw,
                 const double *wn, int64_t nq, const int64_t *qidx, double *acc)
{
    int dim = P->dim;
    double h = P->h, rc2 = 4.0 * h * h;
    double eta2 = 0.01 * h * h;
    cellset sf, sw;
    int rc = cs_build(&sf, dim, nf, fx, 2.0 * h);
    if (rc) return rc;
    rc = cs_build(&sw, dim, nw, wx, 2.0 * h);
    if (rc) {
        cs_free(&sf);
        return rc;
    }
    int err = 0;
    /* cross_phase = 2: the pressure each heavy particle carries as a moving
     * wall dummy of the light phase, from its light neighbours by the
     * two-phase form of Eq. (12) (each term divided by rho_f), with the
     * tank's acceleration as the dummy's; 0 without light neighbours. */
    double *pd = NULL;
    if (P->two_phase && P->cross_phase == 2) {
        pd = (double *)calloc((size_t)(nf ? nf : 1), sizeof(double));
        if (!pd) err = ORC_ERR_ALLOC;
    }
    if (pd) {
#pragma omp parallel
        {
            int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
            for (int64_t j = 0; j < nf; ++j) {
                if (is_light(P, j)) continue;
                const double *xj = fx + j * dim;
                int cnt = cs_query(&sf, xj, rc2, nbr, ORC_NBR_CAP);
                if (cnt < 0) {
                    err = ORC_ERR_NBR_CAP;
                    cnt = 0;
                }
                double sW = 0.0, sP = 0.0, sR[3] = {0, 0, 0};
                for (int a = 0; a < cnt; ++a) {
                    int64_t l = nbr[a];
                    if (!is_light(P, l)) continue;
                    double r2 = 0.0, rjl[3] = {0, 0, 0};
                    for (int k = 0; k < dim; ++k) {
                        rjl[k] = xj[k] - fx[l * dim + k];
                        r2 += rjl[k] * rjl[k];
                    }
                    double W = orc_W(dim, h, sqrt(r2));
                    double rl = frho[l];
                    sW += W / rl;
                    sP += eos_p(P, l, rl) / rl * W;
                    for (int k = 0; k < dim; ++k) sR[k] += rjl[k] * W;
                }
                double gR = 0.0;
                for (int k = 0; k < dim; ++k) gR += (P->g[k] - P->a_wall[k]) * sR[k];
                pd[j] = sW > 0.0 ? (sP + gR) / sW : 0.0;
            }
            free(nbr);
        }
    }
#pragma omp parallel
    {
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * ORC_NBR_CAP);
#pragma omp for schedule(static)
        for (int64_t a_q = 0; a_q < nq; ++a_q) {
            int64_t i = qidx ? qidx[a_q] : a_q;
            const double *xi = fx + i * dim, *vi = fv + i * dim;
            double rho_i = frho[i], p_i = eos_p(P, i, rho_i);
            int penalised = P->penalty_on || is_light(P, i);
            double A[3] = {0, 0, 0};     /* pressure part, Eq. (10)/(11) */
            double Vis[3] = {0, 0, 0};   /* viscous part */
            double Fp[3] = {0, 0, 0};    /* penalty part, Eq. (13) */
            for (int set = 0; set < 2; ++set) {
                const cellset *cs = set == 0 ? &sf : &sw;
                int cnt = cs_query(cs, xi, rc2, nbr, ORC_NBR_CAP);
                if (cnt < 0) {
                    err = ORC_ERR_NBR_CAP;
                    cnt = 0;
                }
                for (int a = 0; a < cnt; ++a) {
                    int64_t j = nbr[a];
                    const double *xj = cs->x + j * dim;
                    double rij[3] = {0, 0, 0}, r2 = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        rij[k] = xi[k] - xj[k];
                        r2 += rij[k] * rij[k];
                    }
                    if (r2 == 0.0) continue;
                    double r = sqrt(r2);
                    double e[3] = {0, 0, 0}, gradW[3] = {0, 0, 0}, vj[3] = {0, 0, 0};
                    double dW = orc_dW(dim, h, r);
                    for (int k = 0; k < dim; ++k) {
                        e[k] = -rij[k] / r;
                        gradW[k] = dW * rij[k] / r;
                    }
                    double rho_j, pstar, m;
                    if (set == 0) {
                        for (int k = 0; k < dim; ++k) vj[k] = fv[j * dim + k];
                        double p_j = eos_p(P, j, frho[j]);
                        if (P->cross_phase && is_light(P, i) && !is_light(P, j)) {
                            /* the heavy particle as a moving dummy of the light phase,
                             * carrying its own pressure (1) or the one extrapolated
                             * from its light neighbours (2) */
                            if (pd) p_j = pd[j];
                            rho_j = eos_rho(P, i, p_j);
                            pstar = (rho_i * p_j + rho_j * p_i) / (rho_i + rho_j); /* Eq. (11) */
                            m = mass_of(P, i);
                        } else {
                            rho_j = frho[j];
                            riemann_out rs =
                                riemann(rho_i, dot(dim, vi, e), p_i, rho_j, dot(dim, vj, e), p_j, P->c);
                            pstar = rs.pstar;
                            m = mass_of(P, j);
                        }
                    } else {
                        for (int k = 0; k < dim; ++k) vj[k] = P->wall_v[k];
                        double p_w = pw[j];
                        rho_j = eos_rho(P, i, p_w);
                        pstar = (rho_i * p_w + rho_j * p_i) / (rho_i + rho_j); /* Eq. (11) */
                        m = mass_of(P, i);
                    }
                    for (int k = 0; k < dim; ++k) A[k] += -2.0 * m * pstar / (rho_i * rho_j) * gradW[k];
                    /* viscous: 2 mu m_j/(rho_i rho_j) (r_ij . grad W)/(r^2 + eta^2) v_ij */
                    double visc = 2.0 * P->mu * m / (rho_i * rho_j) * dot(dim, rij, gradW) / (r2 + eta2);
                    for (int k = 0; k < dim; ++k) Vis[k] += visc * (vi[k] - vj[k]);
                    if (set == 1 && penalised) {
                        const double *n_w = wn + j * dim;
                        /* Eq. (15) with the magnitude of the normal projection */
                        double delta = 2.0 * fabs(dot(dim, rij, n_w)) / P->dx;
                        if (delta < 1.0) {
                            double lambda = (1.0 - delta) * (1.0 - delta); /* Eq. (14) */
                            double pen = P->gamma_p * lambda * fabs(p_i * dot(dim, e, n_w));
                            for (int k = 0; k < dim; ++k)
                                Fp[k] += -2.0 * m / (rho_i * rho_j) * pen * dW * n_w[k];
                        }
                    }
                }
            }
            for (int k = 0; k < dim; ++k) acc[a_q * dim + k] = A[k] + Vis[k] + Fp[k] + P->g[k];
        }
        free(nbr);
    }
    free(pd);
    cs_free(&sf);
    cs_free(&sw);
    return err;
}

/* ------------------------------------------------------------------ */
/* Global diagnostics: mass, momentum, kinetic and potential energy,   */
/* max |v|.  out[0]=M, out[1..3]=P, out[4]=Ek, out[5]=Ep, out[6]=vmax. */
/* Ep is -sum m g . r (zero at the coordinate origin).                 */
/* ------------------------------------------------------------------ */
void orc_diag(const orc_params *P, int64_t nf, const double *fx, const double *fv, double *out)
{
    int dim = P->dim;
    double M = 0, Pm[3] = {0, 0, 0}, Ek = 0, Ep = 0, vmax = 0;
    for (int64_t i = 0; i < nf; ++i) {
        const double *v = fv + i * dim, *x = fx + i * dim;
        double m = mass_of(P, i);
        M += m;
        for (int k = 0; k < dim; ++k) Pm[k] += m * v[k];
        double v2 = dot(dim, v, v);
        Ek += 0.5 * m * v2;
        Ep -= m * dot(dim, P->g, x);
        if (sqrt(v2) > vmax) vmax = sqrt(v2);
    }
    out[0] = M;
    for (int k = 0; k < 3; ++k) out[1 + k] = Pm[k];
    out[4] = Ek;
    out[5] = Ep;
    out[6] = vmax;
}

/* ------------------------------------------------------------------ */
/* Prescribed tank motion: X(t) = A0 sin(2 pi f0 t) with its velocity  */
/* and acceleration at t = step dt (all zero when f0 = 0).             */
/* ------------------------------------------------------------------ */
void orc_tank_motion(const orc_params *P, int64_t step, double *X, double *V, double *A)
{
    double w = 2.0 * M_PI * P->motion_freq, t = (double)step * P->dt;
    for (int k = 0; k < 3; ++k) {
        X[k] = P->motion_amp[k] * sin(w * t);
        V[k] = P->motion_amp[k] * w * cos(w * t);
        A[k] = -P->motion_amp[k] * w * w * sin(w * t);
    }
}

/* ------------------------------------------------------------------ */
/* Time stepping, Sec. 2.6: kick-drift-kick with the reinitialisation  */
/* at the start of each step.  State arrays are updated in place.      */
/*   fx, fv, frho, facc : fluid position, velocity, density, dv/dt     */
/*   wx0                : wall dummies at t = 0                        */
/*   wx                 : wall dummies at the end (x_w(0) + X(t))      */
/*   wn                 : wall normals (a translation keeps them)      */
/*   pw                 : wall pressure of the last step (output)      */
/*   step0              : index n of the state passed in (t = n dt)    */
/*   probe, nprobe, J   : optional; J += dt * mean_{w in probe} p_w    */
/*   damp               : v *= (1 - damp) after every step (relaxation  */
/*                        of a scene to rest; 0 for plain time steps)  */
/* The wall velocity and acceleration of each step come from the tank  */
/* motion (P->wall_v is not read).                                     */
/* ------------------------------------------------------------------ */
int orc_step(const orc_params *P, int64_t nf, double *fx, double *fv, double *frho,
             double *facc, int64_t nw, const double *wx0, double *wx, const double *wn,
             double *pw, int64_t step0, int nsteps, const int32_t *probe, int nprobe, double *J,
             double damp)
{
    int dim = P->dim;
    double dt = P->dt;
    size_t nd = (size_t)(nf ? nf : 1) * dim;
    double *sigma = (double *)malloc(sizeof(double) * (size_t)(nf ? nf : 1));
    double *rho_t = (double *)malloc(sizeof(double) * (size_t)(nf ? nf : 1));
    double *vhalf = (double *)malloc(sizeof(double) * nd);
    double *D = (double *)malloc(sizeof(double) * (size_t)(nf ? nf : 1));
    int rc = ORC_OK;
    if (!sigma || !rho_t || !vhalf || !D) rc = ORC_ERR_ALLOC;
    for (int n = 0; n < nsteps && rc == ORC_OK; ++n) {
        double X0[3], V0[3], A0[3], X1[3], V1[3], A1[3];
        orc_tank_motion(P, step0 + n, X0, V0, A0);
        orc_tank_motion(P, step0 + n + 1, X1, V1, A1);
        for (int64_t w = 0; w < nw; ++w)
            for (int k = 0; k < dim; ++k) wx[w * dim + k] = wx0[w * dim + k] + X0[k];
        /* Eq. (17): reinitialise the density at r^n with rho* = rho^n. */
        rc = orc_sigma(P, nf, fx, nw, wx, nf, NULL, sigma);
        if (rc) break;
        orc_reinit(P, nf, sigma, frho, rho_t);
        /* Eqs. (19)-(20): half kick and drift; the walls move to X(t_{n+1}). */
        for (int64_t i = 0; i < nf; ++i)
            for (int k = 0; k < dim; ++k) {
                vhalf[i * dim + k] = fv[i * dim + k] + 0.5 * dt * facc[i * dim + k];
                fx[i * dim + k] = fx[i * dim + k] + dt * vhalf[i * dim + k];
            }
        for (int64_t w = 0; w < nw; ++w)
            for (int k = 0; k < dim; ++k) wx[w * dim + k] = wx0[w * dim + k] + X1[k];
        orc_params Q = *P;
        for (int k = 0; k < 3; ++k) {
            Q.wall_v[k] = (X1[k] - X0[k]) / dt;
            Q.a_wall[k] = P->a_wall[k] + A1[k];
        }
        /* Eq. (12) at r^{n+1} from the reinitialised density. */
        rc = orc_wall_pressure(&Q, nw, wx, nf, fx, rho_t, nw, NULL, pw);
        if (rc) break;
        if (J && nprobe > 0) {
            double s = 0.0;
            for (int a = 0; a < nprobe; ++a) s += pw[probe[a]];
            *J += dt * s / nprobe;
        }
        /* Eqs. (9), (21): density update; in a two-phase run the light
         * phase takes rho0_light sigma/sigma0 at r^{n+1} instead. */
        rc = orc_continuity(&Q, nf, fx, vhalf, rho_t, nw, wx, pw, nf, NULL, D);
        if (rc) break;
        for (int64_t i = 0; i < nf; ++i) frho[i] = rho_t[i] + dt * D[i];
        if (P->two_phase && P->n_heavy < nf) {
            rc = orc_sigma(P, nf, fx, nw, wx, nf, NULL, sigma);
            if (rc) break;
            for (int64_t i = P->n_heavy; i < nf; ++i) frho[i] = P->rho0_light * sigma[i] / P->sigma0;
        }
        /* Eqs. (10), (22): acceleration at n+1 and second half kick. */
        rc = orc_momentum(&Q, nf, fx, vhalf, frho, nw, wx, pw, wn, nf, NULL, facc);
        if (rc) break;
        for (int64_t i = 0; i < nf; ++i)
            for (int k = 0; k < dim; ++k)
                fv[i * dim + k] = (1.0 - damp) * (vhalf[i * dim + k] + 0.5 * dt * facc[i * dim + k]);
    }
    free(sigma);
    free(rho_t);
    free(vhalf);
    free(D);
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
