/*
 * md_oracle.c -- plain, slow, FP64 CPU oracle for the NEMD channel micro-solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (Stephenson, Kermode & Lockerby, "Accelerating a hybrid
 * continuum-atomistic fluidic model with on-the-fly machine learning"):
 *   - Appendix A (MD parameters): a Lennard-Jones fluid, shifted LJ pair
 *     potential (Eq. LJ), frozen wall atoms, velocity-Verlet integration,
 *     a Berendsen thermostat acting on one velocity component, periodic
 *     boundaries in the streamwise (x) and spanwise (z) directions.
 *   - Sec. 2.1 (Hybrid method), Eq. momentumEq: every fluid atom carries the
 *     body force F = F_ext - (m/rho) dp/ds; here g = F/m along +x.
 *   - Sec. 2.1 / Sec. 2.4: the output is the time-averaged mass flow rate of
 *     a quasi-steady subdomain run, averaged after a start-up phase, started
 *     from a lattice with zero mean velocity.
 *   - Sec. 2.3 (Hyperparameters): the noise level of a run is estimated from
 *     the time-instantaneous data; here by the standard error of contiguous
 *     block means.
 *
 * Readings where the paper is silent are listed in the design notes; the ones
 * this file relies on are restated next to the code that implements them.
 *
 * Reduced LJ units: eps_ff = sigma_ff = m = k_B = 1.
 * Compile with -ffp-contract=off (no fused multiply-add contraction), no
 * fast-math, so every expression rounds as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the  */
/* published round function: two 32x32->64 multiplies per round, a Weyl key */
/* schedule, ten rounds.                                                     */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_seed(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

/* A 32-bit draw mapped to the open interval (0, 1). */
static double u01_open(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------ */
/* Parameters and state                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho;         /* fluid number density used to size N_f */
    double T0;          /* thermostat target temperature */
    double rc;          /* cut-off radius (fluid-fluid and wall-fluid) */
    double eps_wf, sigma_wf;
    double rho_wall;    /* wall FCC number density */
    int wall_layers;    /* FCC (100) layers per wall; 0 = no walls */
    int thermo_axis;    /* velocity component the thermostat acts on */
    double dt, tau_T;
    double Lx_nom, Lz_nom;  /* nominal periodic extents, snapped to the wall lattice */
    double bin_dy;      /* width of the wall-normal profile bins */
    int64_t n_equil;    /* steps before sampling starts */
    int n_blocks;       /* 0: standard error left to the caller (correlated-series
                           estimator over the series); >= 2: that many blocks */
    int64_t n_fluid;    /* 0: round(rho*Lx*Lz*h) */
    double delta;       /* gap between wall plane and the first lattice plane */
    double cell_w;      /* minimum cell width; 0 means rc */
    int periodic_y;     /* 1: bulk box, periodic in y with period h (needs wall_layers = 0) */
    double g_sin;       /* amplitude of a body force g_sin sin(2 pi y / h) along x, added to g */
} ora_params;

typedef struct {
    ora_params P;
    double h, g;
    uint64_t seed;
    double a_w, Lx, Lz;
    int64_t nf, nw;
    double *x, *v, *f;      /* fluid: N_f x 3, row-major */
    double *xw;             /* wall: N_w x 3 */
    double pe;              /* potential energy of the last force evaluation */
    /* cell grid (fluid cells; wall cells live in y-slabs -1 and ny) */
    int ncx, ncy, ncz;
    double inv_wx, inv_wy, inv_wz;   /* n_a / L_a */
    int *cell_of;           /* per fluid atom */
    int *fstart, *fcount, *forder;   /* fluid cells: start/count and atom ids */
    int *wstart, *wcount, *worder;   /* wall columns: 2 slabs x ncx*ncz */
    /* sampling */
    int64_t step;           /* steps taken so far */
    int64_t nsamp;          /* samples taken */
    double *series;         /* instantaneous q' per sampled step (grown) */
    int64_t series_cap;
    int nbins;
    double *bin_mvx, *bin_cnt;
    double Tsum[3];
    double lambda_last;
    int status;
    /* pair-force diagnostics of the last force evaluation: sums over fluid
     * atoms of the wall forces (lower wall: sites at y <= 0; upper: y > 0)
     * and of all pair forces, the fluid-fluid virial sum_{i<j} r_ij . f_ij
     * and its yy part */
    double fw_lo[3], fw_hi[3], ftot[3], vir, vir_yy;
    /* flow diagnostics over the sampled steps */
    double *disp;           /* per atom: unwrapped x displacement */
    int64_t wraps;          /* net crossings of the periodic plane x = 0 (+ along +x) */
    double p_start;         /* sum v_x when sampling began */
    double kick1, kick2;    /* sums of the x kick forces (pair + body) of the first
                               and second half-kicks of sampled steps */
    double fwx_sum, ftx_sum, fwy_lo_sum, fwy_hi_sum, vir_sum, viryy_sum;
    double *fwx_series;     /* per sampled step: wall force on the fluid along x */
    double *pw_series;      /* per sampled step: normal pressure on the walls,
                               (F_lo,y - F_hi,y) / (2 Lx Lz) */
} ora_sys;

/* Stated defaults (readings of the paper, see the design notes). */
void ora_default_params(ora_params *P)
{
    P->rho = 0.8; P->T0 = 1.0; P->rc = 2.5;
    P->eps_wf = 1.0; P->sigma_wf = 1.0; P->rho_wall = 1.0;
    P->wall_layers = 4; P->thermo_axis = 1;
    P->dt = 0.005; P->tau_T = 0.1;
    P->Lx_nom = 12.0; P->Lz_nom = 12.0;
    P->bin_dy = 0.25;
    P->n_equil = 0; P->n_blocks = 0; P->n_fluid = 0;
    P->delta = 1.0;
    P->cell_w = 0.0;
    P->periodic_y = 0;
    P->g_sin = 0.0;
}

/* ------------------------------------------------------------------------ */
/* Geometry (Appendix A: frozen wall atoms; walls bound the channel height)  */
/* Wall: FCC with cubic cell a_w = (4/rho_w)^(1/3), (100) faces normal to y. */
/* Layer k of the lower wall sits at y = -k a_w/2, of the upper at           */
/* y = h + k a_w/2; layer-k sites are (p a_w/2, y_k, q a_w/2) with p+q+k     */
/* even.  h is the distance between the innermost wall planes.              */
/* ------------------------------------------------------------------------ */
static void build_walls(ora_sys *S)
{
    const ora_params *P = &S->P;
    int nwx = (int)lround(P->Lx_nom / S->a_w);
    int nwz = (int)lround(P->Lz_nom / S->a_w);
    if (nwx < 1) nwx = 1;
    if (nwz < 1) nwz = 1;
    S->Lx = (double)nwx * S->a_w;
    S->Lz = (double)nwz * S->a_w;
    int64_t per_layer = 2 * (int64_t)nwx * nwz;
    S->nw = 2 * per_layer * P->wall_layers;
    S->xw = (double *)malloc(sizeof(double) * 3 * (S->nw > 0 ? S->nw : 1));
    double half = 0.5 * S->a_w;
    int64_t n = 0;
    for (int side = 0; side < 2; ++side) {
        for (int k = 0; k < P->wall_layers; ++k) {
            double y = (side == 0) ? -(double)k * half : S->h + (double)k * half;
            for (int q = 0; q < 2 * nwz; ++q)
                for (int p = 0; p < 2 * nwx; ++p) {
                    if (((p + q + k) & 1) != 0) continue;
                    S->xw[3 * n + 0] = (double)p * half;
                    S->xw[3 * n + 1] = y;
                    S->xw[3 * n + 2] = (double)q * half;
                    ++n;
                }
        }
    }
}

/* Fluid start (Sec. 2.4: new runs without a stored state begin from a
 * lattice whose mean velocity is zero).  The lattice
 * is a stack of square planes, successive planes shifted by half a spacing
 * in x and z, filling y in [delta, h - delta].  The plane count and in-plane
 * counts are the ones, among candidates with enough sites, that maximise the
 * closest site-site distance.  N_f of the sites are chosen by a Fisher-Yates
 * shuffle keyed by the seed, and kept in ascending site order. */
typedef struct { int nl, mx, mz; double s, ax, az; } lattice_t;

static lattice_t choose_lattice(int64_t nf, double Lx, double Lz, double D)
{
    lattice_t best = {1, 1, 1, 0.0, Lx, Lz};
    double best_d = -1.0;
    int nlmax = (int)floor(D / 0.5) + 1;
    if (nlmax < 1) nlmax = 1;
    for (int nl = 1; nl <= nlmax; ++nl) {
        double s = (nl > 1) ? D / (double)(nl - 1) : 0.0;
        int64_t per = (nf + nl - 1) / nl;
        int mx = (int)ceil(sqrt((double)per * Lx / Lz));
        if (mx < 1) mx = 1;
        int mz = (int)((per + mx - 1) / mx);
        if (mz < 1) mz = 1;
        double ax = Lx / (double)mx, az = Lz / (double)mz;
        double d = ax < az ? ax : az;
        if (nl > 1) {
            double inter = sqrt(0.25 * ax * ax + 0.25 * az * az + s * s);
            if (inter < d) d = inter;
        }
        if (nl > 2) {
            double two = 2.0 * s;
            if (two < d) d = two;
        }
        if (d > best_d) {
            best_d = d;
            best.nl = nl; best.mx = mx; best.mz = mz; best.s = s; best.ax = ax; best.az = az;
        }
    }
    return best;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Bulk box (periodic in y): nl planes evenly over the period, spacing h/nl,
 * the plane count chosen like the channel's (largest closest distance,
 * counting the spacing across the periodic boundary). */
static lattice_t choose_lattice_periodic(int64_t nf, double Lx, double Lz, double h)
{
    lattice_t best = {1, 1, 1, h, Lx, Lz};
    double best_d = -1.0;
    int nlmax = (int)floor(h / 0.5);
    if (nlmax < 2) nlmax = 2;
    for (int nl = 2; nl <= nlmax; nl += 2) {  /* even: the half-spacing shift alternates across the boundary */
        double s = h / (double)nl;
        int64_t per = (nf + nl - 1) / nl;
        int mx = (int)ceil(sqrt((double)per * Lx / Lz));
        if (mx < 1) mx = 1;
        int mz = (int)((per + mx - 1) / mx);
        if (mz < 1) mz = 1;
        double ax = Lx / (double)mx, az = Lz / (double)mz;
        double d = ax < az ? ax : az;
        double inter = sqrt(0.25 * ax * ax + 0.25 * az * az + s * s);
        if (inter < d) d = inter;
        if (2.0 * s < d) d = 2.0 * s;
        if (d > best_d) {
            best_d = d;
            best.nl = nl; best.mx = mx; best.mz = mz; best.s = s; best.ax = ax; best.az = az;
        }
    }
    return best;
}

static void init_fluid(ora_sys *S)
{
    const ora_params *P = &S->P;
    double D = S->h - 2.0 * P->delta;
    lattice_t L = P->periodic_y ? choose_lattice_periodic(S->nf, S->Lx, S->Lz, S->h)
                                : choose_lattice(S->nf, S->Lx, S->Lz, D);
    int64_t nsites = (int64_t)L.nl * L.mx * L.mz;
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * nsites);
    for (int64_t i = 0; i < nsites; ++i) perm[i] = i;
    uint32_t key[2];
    philox_seed(S->seed, key);
    for (int64_t i = nsites - 1; i >= 1; --i) {
        uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, 0u}, r[4];
        ora_philox4x32_10(ctr, key, r);
        int64_t j = (int64_t)(((uint64_t)r[0] * (uint64_t)(i + 1)) >> 32);
        int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    qsort(perm, (size_t)S->nf, sizeof(int64_t), cmp_i64);
    for (int64_t n = 0; n < S->nf; ++n) {
        int64_t site = perm[n];
        int i = (int)(site % L.mx);
        int k = (int)((site / L.mx) % L.mz);
        int l = (int)(site / ((int64_t)L.mx * L.mz));
        double off = (l & 1) ? 0.5 : 0.0;
        S->x[3 * n + 0] = ((double)i + off) * L.ax;
        if (P->periodic_y) S->x[3 * n + 1] = ((double)l + 0.5) * L.s;
        else S->x[3 * n + 1] = (L.nl > 1) ? P->delta + (double)l * L.s : 0.5 * S->h;
        S->x[3 * n + 2] = ((double)k + off) * L.az;
    }
    free(perm);

    /* Maxwell velocities: Box-Muller on Philox draws, counter (n, 1, 0, 0). */
    const double two_pi = 6.283185307179586;
    double sT = sqrt(P->T0);
    for (int64_t n = 0; n < S->nf; ++n) {
        uint32_t ctr[4] = {(uint32_t)n, 1u, 0u, 0u}, r[4];
        ora_philox4x32_10(ctr, key, r);
        double u0 = u01_open(r[0]), u1 = u01_open(r[1]);
        double u2 = u01_open(r[2]), u3 = u01_open(r[3]);
        double rad1 = sqrt(-2.0 * log(u0)), th1 = two_pi * u1;
        double rad2 = sqrt(-2.0 * log(u2)), th2 = two_pi * u3;
        S->v[3 * n + 0] = sT * (rad1 * cos(th1));
        S->v[3 * n + 1] = sT * (rad1 * sin(th1));
        S->v[3 * n + 2] = sT * (rad2 * cos(th2));
    }
    /* zero mean, then rescale to T0 over 3 N_f degrees of freedom */
    double m[3] = {0.0, 0.0, 0.0};
    for (int64_t n = 0; n < S->nf; ++n)
        for (int a = 0; a < 3; ++a) m[a] += S->v[3 * n + a];
    for (int a = 0; a < 3; ++a) m[a] = m[a] / (double)S->nf;
    double ss = 0.0;
    for (int64_t n = 0; n < S->nf; ++n) {
        for (int a = 0; a < 3; ++a) S->v[3 * n + a] = S->v[3 * n + a] - m[a];
        double vx = S->v[3 * n + 0], vy = S->v[3 * n + 1], vz = S->v[3 * n + 2];
        ss += vx * vx + vy * vy + vz * vz;
    }
    double T = ss / (3.0 * (double)S->nf);
    double scale = sqrt(P->T0 / T);
    for (int64_t n = 0; n < 3 * S->nf; ++n) S->v[n] = S->v[n] * scale;
}

/* ------------------------------------------------------------------------ */
/* Cell grid (a reading: cells of width >= r_c in x, y, z over the fluid     */
/* region [0,Lx) x [0,h) x [0,Lz); wall atoms are binned by (x, z) column    */
/* into a lower slab (y-index -1) and an upper slab (y-index ny)).  Cell     */
/* index rule: c_a = min(n_a - 1, floor(x_a * (n_a / L_a))), clamped at 0.   */
/* ------------------------------------------------------------------------ */
static int cell_axis(double x, double inv, int n)
{
    double t = floor(x * inv);
    int c;
    if (!(t >= 0.0)) c = 0;              /* also catches NaN */
    else if (t >= (double)(n - 1)) c = n - 1;
    else c = (int)t;
    return c;
}

static void setup_cells(ora_sys *S)
{
    const ora_params *P = &S->P;
    double wmin = P->cell_w > P->rc ? P->cell_w : P->rc;
    S->ncx = (int)floor(S->Lx / wmin);
    S->ncz = (int)floor(S->Lz / wmin);
    S->ncy = (int)floor(S->h / wmin);
    if (S->ncy < 1) S->ncy = 1;
    S->inv_wx = (double)S->ncx / S->Lx;
    S->inv_wy = (double)S->ncy / S->h;
    S->inv_wz = (double)S->ncz / S->Lz;
    int64_t nc = (int64_t)S->ncx * S->ncy * S->ncz;
    S->cell_of = (int *)malloc(sizeof(int) * (S->nf > 0 ? S->nf : 1));
    S->fstart = (int *)malloc(sizeof(int) * nc);
    S->fcount = (int *)malloc(sizeof(int) * nc);
    S->forder = (int *)malloc(sizeof(int) * (S->nf > 0 ? S->nf : 1));
    int64_t ncol = (int64_t)S->ncx * S->ncz;
    S->wstart = (int *)malloc(sizeof(int) * 2 * ncol);
    S->wcount = (int *)malloc(sizeof(int) * 2 * ncol);
    S->worder = (int *)malloc(sizeof(int) * (S->nw > 0 ? S->nw : 1));
    /* wall columns are static: counting sort once */
    memset(S->wcount, 0, sizeof(int) * 2 * ncol);
    int *wkey = (int *)malloc(sizeof(int) * (S->nw > 0 ? S->nw : 1));
    for (int64_t w = 0; w < S->nw; ++w) {
        int cx = cell_axis(S->xw[3 * w + 0], S->inv_wx, S->ncx);
        int cz = cell_axis(S->xw[3 * w + 2], S->inv_wz, S->ncz);
        int slab = (S->xw[3 * w + 1] <= 0.0) ? 0 : 1;
        wkey[w] = (int)(slab * ncol + (int64_t)cz * S->ncx + cx);
        S->wcount[wkey[w]]++;
    }
    int acc = 0;
    for (int64_t c = 0; c < 2 * ncol; ++c) { S->wstart[c] = acc; acc += S->wcount[c]; }
    int *cur = (int *)calloc((size_t)(2 * ncol), sizeof(int));
    for (int64_t w = 0; w < S->nw; ++w) {
        int c = wkey[w];
        S->worder[S->wstart[c] + cur[c]++] = (int)w;
    }
    free(cur);
    free(wkey);
}

/* Stable counting sort of fluid atoms (ascending atom id inside a cell). */
static void build_fluid_cells(ora_sys *S)
{
    int64_t nc = (int64_t)S->ncx * S->ncy * S->ncz;
    memset(S->fcount, 0, sizeof(int) * nc);
    for (int64_t i = 0; i < S->nf; ++i) {
        int cx = cell_axis(S->x[3 * i + 0], S->inv_wx, S->ncx);
        int cy = cell_axis(S->x[3 * i + 1], S->inv_wy, S->ncy);
        int cz = cell_axis(S->x[3 * i + 2], S->inv_wz, S->ncz);
        int c = (cz * S->ncy + cy) * S->ncx + cx;
        S->cell_of[i] = c;
        S->fcount[c]++;
    }
    int acc = 0;
    for (int64_t c = 0; c < nc; ++c) { S->fstart[c] = acc; acc += S->fcount[c]; }
    int *cur = (int *)calloc((size_t)nc, sizeof(int));
    for (int64_t i = 0; i < S->nf; ++i) {
        int c = S->cell_of[i];
        S->forder[S->fstart[c] + cur[c]++] = (int)i;
    }
    free(cur);
}

/* ------------------------------------------------------------------------ */
/* Pair interaction (Eq. LJ, shifted: energy shifted to zero at r_c, force   */
/* truncated; pairs interact when r^2 < r_c^2).                              */
/*   U(r) = 4 eps [(s/r)^12 - (s/r)^6],  f_ij = 24 eps [2 (s/r)^12 - (s/r)^6] */
/*   r_ij / r^2, with r_ij = r_i - r_j.                                       */
/* ------------------------------------------------------------------------ */
static double lj_u(double r2, double eps, double sig)
{
    double s2 = sig * sig / r2;
    double s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

static double lj_f_over_r(double r2, double eps, double sig)
{
    double s2 = sig * sig / r2;
    double s6 = s2 * s2 * s2;
    return 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
}

double ora_lj_energy(double r, double eps, double sig) { return lj_u(r * r, eps, sig); }
double ora_lj_force(double r, double eps, double sig) { return lj_f_over_r(r * r, eps, sig) * r; }

static double min_image(double d, double L)
{
    if (d > 0.5 * L) d = d - L;
    else if (d < -0.5 * L) d = d + L;
    return d;
}

/* O(N^2) reference: every fluid-fluid pair and every wall-fluid pair. */
double ora_forces_brute(ora_sys *S, double *f)
{
    const ora_params *P = &S->P;
    double rc2 = P->rc * P->rc;
    double ush_ff = lj_u(rc2, 1.0, 1.0);
    double ush_wf = lj_u(rc2, P->eps_wf, P->sigma_wf);
    double pe = 0.0;
    for (int64_t i = 0; i < S->nf; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, pei = 0.0;
        for (int64_t j = 0; j < S->nf; ++j) {
            if (j == i) continue;
            double dx = min_image(S->x[3 * i] - S->x[3 * j], S->Lx);
            double dy = S->x[3 * i + 1] - S->x[3 * j + 1];
            if (P->periodic_y) dy = min_image(dy, S->h);
            double dz = min_image(S->x[3 * i + 2] - S->x[3 * j + 2], S->Lz);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                double fr = lj_f_over_r(r2, 1.0, 1.0);
                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                pei += 0.5 * (lj_u(r2, 1.0, 1.0) - ush_ff);
            }
        }
        for (int64_t w = 0; w < S->nw; ++w) {
            double dx = min_image(S->x[3 * i] - S->xw[3 * w], S->Lx);
            double dy = S->x[3 * i + 1] - S->xw[3 * w + 1];
            double dz = min_image(S->x[3 * i + 2] - S->xw[3 * w + 2], S->Lz);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
                double fr = lj_f_over_r(r2, P->eps_wf, P->sigma_wf);
                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                pei += lj_u(r2, P->eps_wf, P->sigma_wf) - ush_wf;
            }
        }
        f[3 * i] = fx; f[3 * i + 1] = fy; f[3 * i + 2] = fz;
        pe += pei;
    }
    return pe;
}

/* Cell-list evaluation of exactly the same sum (27 neighbouring cells).
 * Also records the wall forces on the fluid, the total pair force and the
 * fluid-fluid virial (diagnostics, per atom then summed in atom order). */
double ora_forces_cells(ora_sys *S, double *f)
{
    const ora_params *P = &S->P;
    build_fluid_cells(S);
    double rc2 = P->rc * P->rc;
    double ush_ff = lj_u(rc2, 1.0, 1.0);
    double ush_wf = lj_u(rc2, P->eps_wf, P->sigma_wf);
    int nx = S->ncx, ny = S->ncy, nz = S->ncz;
    int64_t ncol = (int64_t)nx * nz;
    int64_t na = S->nf > 0 ? S->nf : 1;
    double *pe_atom = (double *)malloc(sizeof(double) * na);
    double *diag = (double *)malloc(sizeof(double) * 8 * na);  /* lo xyz, hi xyz, vir, vir_yy */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < S->nf; ++i) {
        int c = S->cell_of[i];
        int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
        double xi = S->x[3 * i], yi = S->x[3 * i + 1], zi = S->x[3 * i + 2];
        double fx = 0.0, fy = 0.0, fz = 0.0, pei = 0.0;
        double wl[3] = {0.0, 0.0, 0.0}, wh[3] = {0.0, 0.0, 0.0}, vir = 0.0, viryy = 0.0;
        for (int oz = -1; oz <= 1; ++oz) {
            int jz = (cz + oz + nz) % nz;
            for (int oy = -1; oy <= 1; ++oy) {
                int jy = cy + oy;
                if (P->periodic_y) jy = (jy + ny) % ny;
                for (int ox = -1; ox <= 1; ++ox) {
                    int jx = (cx + ox + nx) % nx;
                    if (jy >= 0 && jy < ny) {
                        int cc = (jz * ny + jy) * nx + jx;
                        for (int k = 0; k < S->fcount[cc]; ++k) {
                            int j = S->forder[S->fstart[cc] + k];
                            if (j == i) continue;
                            double dx = min_image(xi - S->x[3 * j], S->Lx);
                            double dy = yi - S->x[3 * j + 1];
                            if (P->periodic_y) dy = min_image(dy, S->h);
                            double dz = min_image(zi - S->x[3 * j + 2], S->Lz);
                            double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 < rc2) {
                                double fr = lj_f_over_r(r2, 1.0, 1.0);
                                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                                pei += 0.5 * (lj_u(r2, 1.0, 1.0) - ush_ff);
                                vir += 0.5 * fr * r2;
                                viryy += 0.5 * fr * dy * dy;
                            }
                        }
                    } else {
                        int slab = (jy < 0) ? 0 : 1;
                        int64_t wc = slab * ncol + (int64_t)jz * nx + jx;
                        for (int k = 0; k < S->wcount[wc]; ++k) {
                            int w = S->worder[S->wstart[wc] + k];
                            double dx = min_image(xi - S->xw[3 * w], S->Lx);
                            double dy = yi - S->xw[3 * w + 1];
                            double dz = min_image(zi - S->xw[3 * w + 2], S->Lz);
                            double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 < rc2) {
                                double fr = lj_f_over_r(r2, P->eps_wf, P->sigma_wf);
                                fx += fr * dx; fy += fr * dy; fz += fr * dz;
                                pei += lj_u(r2, P->eps_wf, P->sigma_wf) - ush_wf;
                                double *acc = (S->xw[3 * w + 1] <= 0.0) ? wl : wh;
                                acc[0] += fr * dx; acc[1] += fr * dy; acc[2] += fr * dz;
                            }
                        }
                    }
                }
            }
        }
        f[3 * i] = fx; f[3 * i + 1] = fy; f[3 * i + 2] = fz;
        pe_atom[i] = pei;
        double *dg = diag + 8 * i;
        dg[0] = wl[0]; dg[1] = wl[1]; dg[2] = wl[2];
        dg[3] = wh[0]; dg[4] = wh[1]; dg[5] = wh[2];
        dg[6] = vir; dg[7] = viryy;
    }
    double pe = 0.0;
    for (int a = 0; a < 3; ++a) { S->fw_lo[a] = 0.0; S->fw_hi[a] = 0.0; S->ftot[a] = 0.0; }
    S->vir = 0.0;
    S->vir_yy = 0.0;
    for (int64_t i = 0; i < S->nf; ++i) {
        pe += pe_atom[i];
        const double *dg = diag + 8 * i;
        for (int a = 0; a < 3; ++a) {
            S->fw_lo[a] += dg[a];
            S->fw_hi[a] += dg[3 + a];
            S->ftot[a] += f[3 * i + a];
        }
        S->vir += dg[6];
        S->vir_yy += dg[7];
    }
    free(pe_atom);
    free(diag);
    return pe;
}

/* ------------------------------------------------------------------------ */
/* Creation                                                                  */
/* ------------------------------------------------------------------------ */
ora_sys *ora_create(const ora_params *P, double h, double g, uint64_t seed)
{
    if (!(h > 2.0 * P->delta) || !(P->rc > 0.0) || P->n_blocks < 0 || P->n_blocks == 1) return NULL;
    if (P->periodic_y && (P->wall_layers != 0 || h < 3.0 * (P->cell_w > P->rc ? P->cell_w : P->rc))) return NULL;
    ora_sys *S = (ora_sys *)calloc(1, sizeof(ora_sys));
    S->P = *P;
    S->h = h; S->g = g; S->seed = seed;
    S->a_w = cbrt(4.0 / P->rho_wall);
    build_walls(S);
    if (S->Lx < 3.0 * P->rc || S->Lz < 3.0 * P->rc) { free(S->xw); free(S); return NULL; }
    S->nf = (P->n_fluid > 0) ? P->n_fluid : (int64_t)llround(P->rho * S->Lx * S->Lz * h);
    S->x = (double *)malloc(sizeof(double) * 3 * S->nf);
    S->v = (double *)malloc(sizeof(double) * 3 * S->nf);
    S->f = (double *)malloc(sizeof(double) * 3 * S->nf);
    init_fluid(S);
    setup_cells(S);
    S->nbins = (int)ceil(h / P->bin_dy);
    S->bin_mvx = (double *)calloc((size_t)S->nbins, sizeof(double));
    S->bin_cnt = (double *)calloc((size_t)S->nbins, sizeof(double));
    S->series_cap = 1024;
    S->series = (double *)malloc(sizeof(double) * S->series_cap);
    S->fwx_series = (double *)malloc(sizeof(double) * S->series_cap);
    S->pw_series = (double *)malloc(sizeof(double) * S->series_cap);
    S->disp = (double *)calloc((size_t)(S->nf > 0 ? S->nf : 1), sizeof(double));
    S->pe = ora_forces_cells(S, S->f);
    S->lambda_last = 1.0;
    return S;
}

void ora_free(ora_sys *S)
{
    if (!S) return;
    free(S->x); free(S->v); free(S->f); free(S->xw);
    free(S->cell_of); free(S->fstart); free(S->fcount); free(S->forder);
    free(S->wstart); free(S->wcount); free(S->worder);
    free(S->series); free(S->bin_mvx); free(S->bin_cnt);
    free(S->fwx_series); free(S->pw_series); free(S->disp);
    free(S);
}

void ora_info(const ora_sys *S, int64_t *nf, int64_t *nw, double box[3], int ncell[3])
{
    if (nf) *nf = S->nf;
    if (nw) *nw = S->nw;
    if (box) { box[0] = S->Lx; box[1] = S->h; box[2] = S->Lz; }
    if (ncell) { ncell[0] = S->ncx; ncell[1] = S->ncy; ncell[2] = S->ncz; }
}

void ora_get_state(const ora_sys *S, double *x, double *v)
{
    if (x) memcpy(x, S->x, sizeof(double) * 3 * S->nf);
    if (v) memcpy(v, S->v, sizeof(double) * 3 * S->nf);
}

void ora_set_state(ora_sys *S, const double *x, const double *v)
{
    if (x) memcpy(S->x, x, sizeof(double) * 3 * S->nf);
    if (v) memcpy(S->v, v, sizeof(double) * 3 * S->nf);
    S->pe = ora_forces_cells(S, S->f);
}

void ora_get_wall(const ora_sys *S, double *xw) { memcpy(xw, S->xw, sizeof(double) * 3 * S->nw); }

void ora_get_forces(const ora_sys *S, double *f, double *pe)
{
    if (f) memcpy(f, S->f, sizeof(double) * 3 * S->nf);
    if (pe) *pe = S->pe;
}

/* cell_of: per fluid atom; counts: per fluid cell; order: atom ids, cell-major,
 * ascending id inside a cell. */
void ora_cells(ora_sys *S, int *cell_of, int *counts, int *order)
{
    build_fluid_cells(S);
    int64_t nc = (int64_t)S->ncx * S->ncy * S->ncz;
    if (cell_of) memcpy(cell_of, S->cell_of, sizeof(int) * S->nf);
    if (counts) memcpy(counts, S->fcount, sizeof(int) * nc);
    if (order) memcpy(order, S->forder, sizeof(int) * S->nf);
}

/* ------------------------------------------------------------------------ */
/* Time stepping (Appendix A: velocity Verlet; Berendsen on one component).  */
/* One step, in order:                                                       */
/*   1. v += dt/2 (F + g x^)                                                 */
/*   2. x += dt v; wrap x and z into [0, L)                                  */
/*   3. F = F(x)                                                             */
/*   4. v += dt/2 (F + g x^)                                                 */
/*   5. T_c = sum v_c^2 / N_f;  lambda = sqrt(1 + dt/tau (T0/T_c - 1));       */
/*      v_c *= lambda   (c = thermostat axis)                                */
/*   6. if past n_equil: sample q' = sum v_x / (Lx Lz) and the y-profile.    */
/* ------------------------------------------------------------------------ */
static double wrap(double x, double L)
{
    double y = x;
    if (y >= L) y = y - L;
    else if (y < 0.0) y = y + L;
    if (y >= L) y = 0.0;
    return y;
}

static void sample(ora_sys *S)
{
    double sx = 0.0, t[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < S->nf; ++i) {
        double vx = S->v[3 * i], vy = S->v[3 * i + 1], vz = S->v[3 * i + 2];
        sx += vx;
        t[0] += vx * vx; t[1] += vy * vy; t[2] += vz * vz;
        int b = (int)floor(S->x[3 * i + 1] / S->P.bin_dy);
        if (b < 0) b = 0;
        if (b >= S->nbins) b = S->nbins - 1;
        S->bin_mvx[b] += vx;
        S->bin_cnt[b] += 1.0;
    }
    if (S->nsamp == S->series_cap) {
        S->series_cap *= 2;
        S->series = (double *)realloc(S->series, sizeof(double) * S->series_cap);
        S->fwx_series = (double *)realloc(S->fwx_series, sizeof(double) * S->series_cap);
        S->pw_series = (double *)realloc(S->pw_series, sizeof(double) * S->series_cap);
    }
    S->fwx_series[S->nsamp] = S->fw_lo[0] + S->fw_hi[0];
    S->pw_series[S->nsamp] = 0.5 * (S->fw_lo[1] - S->fw_hi[1]) / (S->Lx * S->Lz);
    S->series[S->nsamp++] = sx / (S->Lx * S->Lz);
    for (int a = 0; a < 3; ++a) S->Tsum[a] += t[a] / (double)S->nf;
    S->fwx_sum += S->fw_lo[0] + S->fw_hi[0];
    S->ftx_sum += S->ftot[0];
    S->fwy_lo_sum += S->fw_lo[1];
    S->fwy_hi_sum += S->fw_hi[1];
    S->vir_sum += S->vir;
    S->viryy_sum += S->vir_yy;
}

/* x body force on an atom at height y: g + g_sin sin(2 pi y / h) */
static double body_force(const ora_sys *S, double y)
{
    if (S->P.g_sin == 0.0) return S->g;
    return S->g + S->P.g_sin * sin(6.283185307179586 * y / S->h);
}

/* energy_trace (nullable): total energy per fluid atom after each step. */
void ora_run(ora_sys *S, int64_t steps, int thermostat_on, double *energy_trace)
{
    const ora_params *P = &S->P;
    double hdt = 0.5 * P->dt;
    int ax = P->thermo_axis;
    for (int64_t s = 0; s < steps; ++s) {
        int sampled = S->step + 1 > P->n_equil;
        if (sampled && S->nsamp == 0) {
            double px = 0.0;
            for (int64_t i = 0; i < S->nf; ++i) px += S->v[3 * i];
            S->p_start = px;
        }
        double k1 = 0.0;
        for (int64_t i = 0; i < S->nf; ++i) {
            double gx = body_force(S, S->x[3 * i + 1]);
            k1 += S->f[3 * i + 0] + gx;
            S->v[3 * i + 0] += hdt * (S->f[3 * i + 0] + gx);
            S->v[3 * i + 1] += hdt * S->f[3 * i + 1];
            S->v[3 * i + 2] += hdt * S->f[3 * i + 2];
            double xr = S->x[3 * i + 0] + P->dt * S->v[3 * i + 0];
            if (sampled) {
                S->disp[i] += P->dt * S->v[3 * i + 0];
                if (xr >= S->Lx) S->wraps += 1;
                else if (xr < 0.0) S->wraps -= 1;
            }
            S->x[3 * i + 0] = wrap(xr, S->Lx);
            S->x[3 * i + 1] = S->x[3 * i + 1] + P->dt * S->v[3 * i + 1];
            if (P->periodic_y) S->x[3 * i + 1] = wrap(S->x[3 * i + 1], S->h);
            S->x[3 * i + 2] = wrap(S->x[3 * i + 2] + P->dt * S->v[3 * i + 2], S->Lz);
        }
        S->pe = ora_forces_cells(S, S->f);
        double ss = 0.0, k2 = 0.0;
        for (int64_t i = 0; i < S->nf; ++i) {
            double gx = body_force(S, S->x[3 * i + 1]);
            k2 += S->f[3 * i + 0] + gx;
            S->v[3 * i + 0] += hdt * (S->f[3 * i + 0] + gx);
            S->v[3 * i + 1] += hdt * S->f[3 * i + 1];
            S->v[3 * i + 2] += hdt * S->f[3 * i + 2];
            double vc = S->v[3 * i + ax];
            ss += vc * vc;
        }
        if (sampled) { S->kick1 += k1; S->kick2 += k2; }
        if (thermostat_on) {
            double Tc = ss / (double)S->nf;
            double lam = sqrt(1.0 + (P->dt / P->tau_T) * (P->T0 / Tc - 1.0));
            for (int64_t i = 0; i < S->nf; ++i) S->v[3 * i + ax] = S->v[3 * i + ax] * lam;
            S->lambda_last = lam;
        }
        S->step += 1;
        if (S->step > P->n_equil) sample(S);
        if (energy_trace) {
            double ke = 0.0;
            for (int64_t i = 0; i < 3 * S->nf; ++i) ke += 0.5 * S->v[i] * S->v[i];
            energy_trace[s] = (ke + S->pe) / (double)S->nf;
        }
        for (int64_t i = 0; i < S->nf; ++i) {
            /* unstable: non-finite state, an atom outside the wall gap (the
             * period in a bulk box), or a periodic coordinate that one wrap
             * could not bring back (a move longer than the box in one step) */
            double X = S->x[3 * i], y = S->x[3 * i + 1], Z = S->x[3 * i + 2];
            int y_ok = P->periodic_y ? (y >= 0.0 && y < S->h) : (y > 0.0 && y < S->h);
            if (!y_ok || !(X >= 0.0 && X < S->Lx) || !(Z >= 0.0 && Z < S->Lz) ||
                !isfinite(S->v[3 * i]) || !isfinite(S->v[3 * i + 1]) || !isfinite(S->v[3 * i + 2]))
                S->status = -4;
        }
    }
}

/* Flow and force diagnostics over the sampled steps (see ora_sys):
 * out[0] sum of x displacements, [1] net crossings of x = 0, [2] sum v_x at
 * sampling start, [3] sum v_x now, [4] [5] first / second half-kick force
 * sums, [6] sum of the x wall force, [7] sum of the x total pair force,
 * [8] [9] sums of the y force of the lower / upper wall, [10] [11] sums of
 * the virial and its yy part, [12] samples. */
void ora_flow_diag(const ora_sys *S, double out[13])
{
    double d = 0.0, px = 0.0;
    for (int64_t i = 0; i < S->nf; ++i) { d += S->disp[i]; px += S->v[3 * i]; }
    out[0] = d; out[1] = (double)S->wraps; out[2] = S->p_start; out[3] = px;
    out[4] = S->kick1; out[5] = S->kick2; out[6] = S->fwx_sum; out[7] = S->ftx_sum;
    out[8] = S->fwy_lo_sum; out[9] = S->fwy_hi_sum; out[10] = S->vir_sum; out[11] = S->viryy_sum;
    out[12] = (double)S->nsamp;
}

void ora_wall_force_series(const ora_sys *S, double *out)
{
    memcpy(out, S->fwx_series, sizeof(double) * S->nsamp);
}

/* Per sampled step: the normal pressure the fluid exerts on the walls, the
   mean of the two walls' normal forces per unit area (by the yy momentum
   balance, the cross-section average of P_yy). */
void ora_pressure_series(const ora_sys *S, double *out)
{
    memcpy(out, S->pw_series, sizeof(double) * S->nsamp);
}

/* Per-atom x displacements over the sampled steps. */
void ora_displacements(const ora_sys *S, double *out) { memcpy(out, S->disp, sizeof(double) * S->nf); }

/* Pair-force diagnostics of the current positions: out[0..2] lower-wall
 * force on the fluid, [3..5] upper-wall force, [6..8] total pair force,
 * [9] fluid-fluid virial, [10] its yy part. */
void ora_force_diag(const ora_sys *S, double out[11])
{
    for (int a = 0; a < 3; ++a) { out[a] = S->fw_lo[a]; out[3 + a] = S->fw_hi[a]; out[6 + a] = S->ftot[a]; }
    out[9] = S->vir;
    out[10] = S->vir_yy;
}

/* ------------------------------------------------------------------------ */
/* Result: mean flux over the used samples, standard error of n_blocks       */
/* contiguous block means (a remainder is dropped from the front), flux      */
/* density J = q'/h, sampled temperatures, last potential energy per atom,   */
/* status (0 ok, -4 unstable, -5 not converged).                            */
/* ------------------------------------------------------------------------ */
int64_t ora_nsamples(const ora_sys *S) { return S->nsamp; }

void ora_series(const ora_sys *S, double *out) { memcpy(out, S->series, sizeof(double) * S->nsamp); }

void ora_profile(const ora_sys *S, double *mvx, double *cnt, int *nbins)
{
    if (nbins) *nbins = S->nbins;
    if (mvx) memcpy(mvx, S->bin_mvx, sizeof(double) * S->nbins);
    if (cnt) memcpy(cnt, S->bin_cnt, sizeof(double) * S->nbins);
}

/* Mean and standard error of a series from nb contiguous equal blocks; a
 * remainder of n mod nb samples is dropped from the front.  Also returns the
 * first-half and second-half means of the block means (for the convergence
 * test).  Returns the block length (0 when n < nb). */
int64_t ora_block_stats(const double *series, int64_t n, int nb, double out[4])
{
    int64_t B = (nb > 0) ? n / nb : 0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (B < 1 || nb < 2) return 0;
    int64_t r = n - (int64_t)nb * B;
    double *bm = (double *)malloc(sizeof(double) * nb);
    double mean = 0.0;
    for (int b = 0; b < nb; ++b) {
        double s = 0.0;
        for (int64_t k = 0; k < B; ++k) s += series[r + (int64_t)b * B + k];
        bm[b] = s / (double)B;
        mean += bm[b];
    }
    mean = mean / (double)nb;
    double var = 0.0;
    for (int b = 0; b < nb; ++b) var += (bm[b] - mean) * (bm[b] - mean);
    var = var / (double)(nb - 1);
    int h1 = nb / 2;
    double m1 = 0.0, m2 = 0.0;
    for (int b = 0; b < h1; ++b) m1 += bm[b];
    for (int b = h1; b < nb; ++b) m2 += bm[b];
    out[0] = mean;
    out[1] = sqrt(var / (double)nb);
    out[2] = m1 / (double)h1;
    out[3] = m2 / (double)(nb - h1);
    free(bm);
    return B;
}

void ora_result(const ora_sys *S, double out[8], int *status)
{
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    int st = S->status;
    if (S->nsamp >= 1)
        for (int a = 0; a < 3; ++a) out[3 + a] = S->Tsum[a] / (double)S->nsamp;
    if (S->P.n_blocks >= 2) {
        double bs[4];
        int64_t B = ora_block_stats(S->series, S->nsamp, S->P.n_blocks, bs);
        if (B >= 1) {
            out[0] = bs[0];
            out[1] = bs[1];
            out[2] = bs[0] / S->h;
            /* non-convergence (reading of the critical-shear remark, Sec. 3.2):
             * first-half and second-half block means differ by more than 8 SE,
             * or the spanwise temperature, which no thermostat touches, runs
             * away (> 1.5 T0). */
            if (st == 0 && (fabs(bs[3] - bs[2]) > 8.0 * bs[1] || out[5] > 1.5 * S->P.T0)) st = -5;
        } else if (st == 0) {
            st = -1;
        }
    } else if (st == 0 && S->nsamp < 2) {
        st = -1;
    }
    out[6] = S->pe / (double)S->nf;
    out[7] = S->lambda_last;
    if (status) *status = st;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Neighbour sets for a pair-list cut-off rl (brute force): for fluid atom i
 * (id order) the fluid atoms j != i and wall atoms w (reported as N_f + w)
 * with squared minimum-image distance below rl^2, in ascending index order.
 * counts[i] receives the set sizes; idx (nullable, capacity cap) the
 * concatenated sets.  Returns the total number of entries. */
int64_t ora_neighbors(const ora_sys *S, double rl, int *counts, int *idx, int64_t cap)
{
    double rl2 = rl * rl;
    int64_t tot = 0;
    for (int64_t i = 0; i < S->nf; ++i) {
        int c = 0;
        for (int64_t j = 0; j < S->nf + S->nw; ++j) {
            if (j == i) continue;
            const double *pj = j < S->nf ? &S->x[3 * j] : &S->xw[3 * (j - S->nf)];
            double dx = min_image(S->x[3 * i] - pj[0], S->Lx);
            double dy = S->x[3 * i + 1] - pj[1];
            double dz = min_image(S->x[3 * i + 2] - pj[2], S->Lz);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rl2) {
                if (idx && tot < cap) idx[tot] = (int)j;
                ++tot;
                ++c;
            }
        }
        counts[i] = c;
    }
    return tot;
}
