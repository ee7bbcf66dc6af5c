/*
 * FP64 CPU oracle for the coupled electrokinetic lattice step of Rivas, Frijters,
 * Pagonabarraga and Harting, "Mesoscopic electrohydrodynamic simulations of binary
 * colloidal suspensions" (arXiv:1712.08494).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP
 * library is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the HIP library: it has its own lattice tables, its own parameter
 * struct and its own solver.
 *
 * Everything is double precision, plain loops in the order the paper states the
 * method, with OpenMP only across independent z-planes (each thread writes its own
 * sites; every sum is taken per plane and then serially, so results do not depend
 * on the thread count).
 *
 * One step, all stages reading time-t fields (the paper gives no order; this is the
 * explicit reading):
 *   1. moments and Shan-Chen pseudopotentials            (Sec. II A; Sec. II C, eq. shanChenForce)
 *      virtual densities on solid sites next to fluid     (Sec. II E, Jansen et al.)
 *   2. charge and permittivity                            (Sec. II B eq. electric_potential,
 *                                                          eq. dielectric_constant; Sec. II E)
 *   3. variable-permittivity Poisson solve                (Sec. II D, eq. electric_potential;
 *                                                          option: the polarisation source, a
 *                                                          reading for Sec. III B, poisson_source)
 *   4. electric field E = -grad(phi) + E_ext              (Sec. II B)
 *   5. link fluxes and Nernst-Planck update               (Sec. II B eq. nernst-planck-disc,
 *                                                          upwind advection; Sec. II E
 *                                                          eq. ionic-fluxes-disc-2)
 *   6. forces on the fluids                               (Sec. II C: Shan-Chen, friction
 *                                                          eq. frictionforce, Kelvin eq. kelvin,
 *                                                          discrete total LB force)
 *   7. BGK collision with the velocity-shift forcing       (Sec. II A eq. BoltzmannBGKLattice,
 *                                                          second-order equilibrium)
 *   8. streaming with halfway bounce-back, momentum exchange (Sec. II E)
 *   9. rigid-particle update                              (Sec. II E, Newton, Hertz, lubrication)
 *
 * Readings of passages that are silent, garbled or inconsistent are stated where they
 * are used, tagged "Reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------ */
/* D3Q19 velocity set and weights (Sec. II A, the weights equation).                */
/* Order: rest, the 6 axis links, then the 12 face diagonals, each followed by its  */
/* opposite.                                                                        */
/* ------------------------------------------------------------------------------ */
#define OQ 19
static const int OC[OQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static double OW[OQ];
static int OOPP[OQ];
static const double CS2 = 1.0 / 3.0; /* speed of sound squared, Sec. II C */

static void lattice_setup(void) {
    for (int d = 0; d < OQ; ++d) {
        int c2 = OC[d][0] * OC[d][0] + OC[d][1] * OC[d][1] + OC[d][2] * OC[d][2];
        OW[d] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        for (int e = 0; e < OQ; ++e)
            if (OC[e][0] == -OC[d][0] && OC[e][1] == -OC[d][1] && OC[e][2] == -OC[d][2]) OOPP[d] = e;
    }
}

/* ------------------------------------------------------------------------------ */
/* Parameters (the oracle's own struct).                                           */
/* ------------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_z;          /* 1: solid layers at z = 0 and z = nz-1 */
    int32_t poisson_maxit;
    int32_t subsample;        /* sub-cells per axis for the solid fraction */
    int32_t move_particles;   /* 1: integrate particle motion every step */
    int32_t n_threads;        /* 0: OpenMP default */
    double tau, G, rho0;
    double D, beta;
    double dmu_plus, dmu_minus, drho_a, solvation_sign;
    double eps_a, eps_b, eps_p;
    double E_ext[3];
    double body_accel[3];
    double sigma_wall[2];     /* surface charge on the z = 0 wall and on the z = nz-1 wall */
    double poisson_tol;
    double particle_rho, k_hertz, eta;
    int32_t poisson_lagged;   /* 1: each step takes the lagged Fourier scheme of Sec. II D (periodic) */
    int32_t polarization;     /* 1: the external field also polarises the dielectric (see poisson_source) */
    int32_t reproject;        /* 1: moving particles are projected anew after every step (see reproject) */
} or_params;

typedef struct {
    or_params p;
    int64_t N;
    double *f[2], *fs[2];     /* populations (fs is the streaming target) */
    double *n[2], *nnew[2];   /* ion densities n+ and n- */
    double *phi;              /* potential phi_I (internal part) */
    double *rho[2], *u;       /* moments: rho^a, rho^b, barycentric velocity before forcing (3N) */
    double *uphys;            /* physical fluid velocity (3N), last step */
    double *psi[2];           /* Shan-Chen pseudopotentials of the fluids */
    double *q, *eps, *epsf;   /* charge, permittivity, fluid permittivity */
    double *E;                /* field (3N) */
    double *psis, *psif, *qc; /* solid fraction, fluid fraction, colloid charge */
    uint8_t *solid;           /* LB solid sites */
    int32_t *owner;           /* particle that covers (or partly covers) a site, -1 none */
    double *J[2], *A[2];      /* link fluxes per canonical link (3N each): diffusive+migration+solvation, advective */
    double *Phi[2];           /* force on each fluid component (3N each), last step */
    /* particles */
    int np;
    double *px, *pv, *pr, *pQ, *pF, *px0;
    /* Poisson bookkeeping */
    int last_iters;
    double last_rel, last_qmean;
    int64_t steps;
} or_state;

static inline int64_t IDX(const or_params* p, int x, int y, int z) {
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}
static inline int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

static void set_threads(const or_params* p) {
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#else
    (void)p;
#endif
}

/* ------------------------------------------------------------------------------ */
/* Second-order equilibrium (Sec. II A):                                            */
/*   f~_d = w_d rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]                 */
/* ------------------------------------------------------------------------------ */
static void equilibrium(double rho, const double u[3], double feq[OQ]) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int d = 0; d < OQ; ++d) {
        double cu = OC[d][0] * u[0] + OC[d][1] * u[1] + OC[d][2] * u[2];
        feq[d] = OW[d] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* ------------------------------------------------------------------------------ */
/* Exported small helpers for the pins.                                             */
/* ------------------------------------------------------------------------------ */
int or_lattice(int32_t* c, double* w) {
    lattice_setup();
    for (int d = 0; d < OQ; ++d) {
        for (int k = 0; k < 3; ++k) c[3 * d + k] = OC[d][k];
        w[d] = OW[d];
    }
    return OQ;
}

void or_equilibrium(double rho, const double* u, double* feq) {
    lattice_setup();
    equilibrium(rho, u, feq);
}

/* ------------------------------------------------------------------------------ */
/* Geometry: solid marking and solid fraction (Sec. II E).                           */
/* Reading: a site is LB-solid when its centre lies strictly inside a sphere; the   */
/* solid fraction counts sub-cell centres ((k+1/2)/h - 1/2 per axis, h = subsample) */
/* inside the sphere (minimum image); walls (if any) are solid with fraction 1.     */
/* The colloid charge is spread in proportion to the solid fraction and normalised  */
/* so that it sums to Q exactly (the printed normalising volume is a typo).        */
/* ------------------------------------------------------------------------------ */
static double min_image(double d, int n) {
    /* whole periods taken off at once: the same result as stepping by L for finite d,
       NaN (not an endless loop) for a non-finite one */
    double L = (double)n;
    if (d > 0.5 * L) d -= L * ceil((d - 0.5 * L) / L);
    if (d < -0.5 * L) d += L * ceil((-0.5 * L - d) / L);
    return d;
}

static void build_geometry(or_state* s) {
    const or_params* p = &s->p;
    int64_t N = s->N;
    for (int64_t i = 0; i < N; ++i) {
        s->solid[i] = 0; s->owner[i] = -1; s->psis[i] = 0.0; s->qc[i] = 0.0;
    }
    if (p->walls_z) {
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t a = IDX(p, x, y, 0), b = IDX(p, x, y, p->nz - 1);
                s->solid[a] = s->solid[b] = 1;
                s->psis[a] = s->psis[b] = 1.0;
            }
    }
    int h = p->subsample > 0 ? p->subsample : 8;
    for (int j = 0; j < s->np; ++j) {
        double X = s->px[3 * j], Y = s->px[3 * j + 1], Z = s->px[3 * j + 2], R = s->pr[j];
        int x0 = (int)floor(X - R) - 1, x1 = (int)ceil(X + R) + 1;
        int y0 = (int)floor(Y - R) - 1, y1 = (int)ceil(Y + R) + 1;
        int z0 = (int)floor(Z - R) - 1, z1 = (int)ceil(Z + R) + 1;
        for (int zz = z0; zz <= z1; ++zz)
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx) {
                    int x = wrap(xx, p->nx), y = wrap(yy, p->ny), z = wrap(zz, p->nz);
                    int64_t i = IDX(p, x, y, z);
                    double dx = min_image((double)x - X, p->nx);
                    double dy = min_image((double)y - Y, p->ny);
                    double dz = min_image((double)z - Z, p->nz);
                    /* count sub-cell centres inside the sphere */
                    int cnt = 0;
                    for (int a = 0; a < h; ++a)
                        for (int b = 0; b < h; ++b)
                            for (int c = 0; c < h; ++c) {
                                double sx = dx + ((a + 0.5) / h - 0.5);
                                double sy = dy + ((b + 0.5) / h - 0.5);
                                double sz = dz + ((c + 0.5) / h - 0.5);
                                if (sx * sx + sy * sy + sz * sz <= R * R) ++cnt;
                            }
                    if (cnt > 0 && s->owner[i] < 0 && !(p->walls_z && (z == 0 || z == p->nz - 1))) {
                        s->owner[i] = j;
                        s->psis[i] = (double)cnt / ((double)h * h * h);
                    }
                    if (dx * dx + dy * dy + dz * dz < R * R) s->solid[i] = 1;
                }
    }
    /* charge per site: Q_j psi_s / sum of psi_s over the sites of particle j */
    if (s->np > 0) {
        double* tot = (double*)calloc((size_t)s->np, sizeof(double));
        for (int64_t i = 0; i < N; ++i)
            if (s->owner[i] >= 0) tot[s->owner[i]] += s->psis[i];
        for (int64_t i = 0; i < N; ++i)
            if (s->owner[i] >= 0 && tot[s->owner[i]] > 0) s->qc[i] = s->pQ[s->owner[i]] * s->psis[i] / tot[s->owner[i]];
        free(tot);
    }
    for (int64_t i = 0; i < N; ++i) s->psif[i] = 1.0 - s->psis[i];
}

/* ------------------------------------------------------------------------------ */
/* Step 1: moments, virtual densities, pseudopotentials.                            */
/* ------------------------------------------------------------------------------ */
static void compute_moments(or_state* s) {
    const or_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (s->solid[i]) {
                    s->rho[0][i] = s->rho[1][i] = 0.0;
                    s->u[3 * i] = s->u[3 * i + 1] = s->u[3 * i + 2] = 0.0;
                    continue;
                }
                double r[2], m[3] = {0, 0, 0};
                for (int c = 0; c < 2; ++c) {
                    double acc = 0.0;
                    for (int d = 0; d < OQ; ++d) {
                        double fv = s->f[c][(int64_t)d * s->N + i];
                        acc += fv;
                        m[0] += fv * OC[d][0];
                        m[1] += fv * OC[d][1];
                        m[2] += fv * OC[d][2];
                    }
                    r[c] = acc;
                }
                s->rho[0][i] = r[0];
                s->rho[1][i] = r[1];
                double rt = r[0] + r[1];
                for (int k = 0; k < 3; ++k) s->u[3 * i + k] = m[k] / rt;
            }
    /* Virtual fluid densities (Jansen et al.): a solid site with at least one fluid
       D3Q19 neighbour carries the mean density of its fluid neighbours. */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (!s->solid[i]) continue;
                double acc[2] = {0, 0};
                int cnt = 0;
                for (int d = 1; d < OQ; ++d) {
                    int xx = x + OC[d][0], yy = y + OC[d][1], zz = z + OC[d][2];
                    if (p->walls_z && (zz < 0 || zz >= p->nz)) continue;
                    int64_t j = IDX(p, wrap(xx, p->nx), wrap(yy, p->ny), wrap(zz, p->nz));
                    if (s->solid[j]) continue;
                    acc[0] += s->rho[0][j];
                    acc[1] += s->rho[1][j];
                    ++cnt;
                }
                if (cnt > 0) {
                    /* written to the solid site only; fluid values read above are unchanged */
                    s->rho[0][i] = acc[0] / cnt;
                    s->rho[1][i] = acc[1] / cnt;
                }
            }
    /* psi = rho0 (1 - exp(-rho/rho0)) (Sec. II C) */
    for (int64_t i = 0; i < s->N; ++i)
        for (int c = 0; c < 2; ++c) s->psi[c][i] = p->rho0 * (1.0 - exp(-s->rho[c][i] / p->rho0));
}

/* ------------------------------------------------------------------------------ */
/* Step 2: charge density and permittivity.                                          */
/*   q = e(n+ - n-) + q_c                            (eq. electric_potential)         */
/*   eps_f = 1/2 [eps_a (1-c) + eps_b (1+c)], c = (rho_b - rho_a)/(rho_a + rho_b)     */
/*                                                   (eq. dielectric_constant)       */
/*   eps = eps_p psi_s + eps_f (1 - psi_s)           (particle permittivity mixing)  */
/* Reading: a solid site with no fluid neighbour has no fluid, c is taken as 0.     */
/* ------------------------------------------------------------------------------ */
static void compute_charge_perm(or_state* s) {
    const or_params* p = &s->p;
    for (int64_t i = 0; i < s->N; ++i) {
        s->q[i] = s->n[0][i] - s->n[1][i] + s->qc[i];
        double rt = s->rho[0][i] + s->rho[1][i];
        double c = rt > 0.0 ? (s->rho[1][i] - s->rho[0][i]) / rt : 0.0;
        double ef = 0.5 * (p->eps_a * (1.0 - c) + p->eps_b * (1.0 + c));
        s->epsf[i] = ef;
        s->eps[i] = p->eps_p * s->psis[i] + ef * (1.0 - s->psis[i]);
    }
}

/* ------------------------------------------------------------------------------ */
/* Step 3: Poisson, div(eps grad phi) = -q (eq. electric_potential).                */
/* Reading: 7-point finite-volume operator with face permittivity the mean of the    */
/* two sites, (A phi)_i = sum_{Q6} eps_{i,d} (phi_{i+d} - phi_i).  Walls: the wall    */
/* layers are outside the domain (zero flux across the wall face) and the wall      */
/* surface charge is a source in the adjacent layer.  The source is projected to    */
/* zero mean (compatibility of the periodic / Neumann problem); the removed mean is */
/* recorded.  The gauge is mean(phi) = 0 over the domain.  The paper uses an FFT    */
/* with the eps-gradient term lagged in time; this oracle solves the full variable- */
/* coefficient equation with plain conjugate gradients.                            */
/* ------------------------------------------------------------------------------ */
static inline int in_domain(const or_params* p, int z) {
    return !p->walls_z || (z >= 1 && z <= p->nz - 2);
}

static void apply_A(const or_state* s, const double* v, double* out) {
    const or_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (!in_domain(p, z)) { out[i] = 0.0; continue; }
                double acc = 0.0;
                for (int d = 1; d <= 6; ++d) {
                    int zz = z + OC[d][2];
                    if (p->walls_z && !in_domain(p, zz)) continue;
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(zz, p->nz));
                    double ef = 0.5 * (s->eps[i] + s->eps[j]);
                    acc += ef * (v[j] - v[i]);
                }
                out[i] = acc;
            }
}

static double dom_dot(const or_state* s, const double* a, const double* b) {
    const or_params* p = &s->p;
    double* part = (double*)calloc((size_t)p->nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z) {
        if (!in_domain(p, z)) continue;
        double acc = 0.0;
        for (int64_t i = IDX(p, 0, 0, z); i < IDX(p, 0, 0, z) + (int64_t)p->nx * p->ny; ++i) acc += a[i] * b[i];
        part[z] = acc;
    }
    double t = 0.0;
    for (int z = 0; z < p->nz; ++z) t += part[z];
    free(part);
    return t;
}

static double dom_sum(const or_state* s, const double* a, int64_t* count) {
    const or_params* p = &s->p;
    double t = 0.0;
    int64_t c = 0;
    for (int z = 0; z < p->nz; ++z) {
        if (!in_domain(p, z)) continue;
        double acc = 0.0;
        for (int64_t i = IDX(p, 0, 0, z); i < IDX(p, 0, 0, z) + (int64_t)p->nx * p->ny; ++i) acc += a[i];
        t += acc;
        c += (int64_t)p->nx * p->ny;
    }
    if (count) *count = c;
    return t;
}

static void dom_shift(or_state* s, double* a, double by) {
    const or_params* p = &s->p;
    for (int z = 0; z < p->nz; ++z) {
        if (!in_domain(p, z)) continue;
        for (int64_t i = IDX(p, 0, 0, z); i < IDX(p, 0, 0, z) + (int64_t)p->nx * p->ny; ++i) a[i] -= by;
    }
}

/* Source b with M phi = b, M = -A: b = q + wall charge in the adjacent layers, mean removed.
   Reading (option `polarization`, off by default): as printed, the potential is sourced by
   the charge alone and the field is E = -grad(phi) + E_ext, so an ion-free dielectric in a
   uniform external field stays unpolarised and feels no Kelvin force.  The droplet
   experiment of Sec. III B needs the field of the polarised medium.  With the option, Gauss's
   law holds for the total displacement eps (-grad phi + E_ext) through every face:
     sum_faces eps_f (phi_j - phi_i) = -(q_i - sum_faces eps_f (E_ext . c_d)),
   i.e. the source gains -sum over the six faces of eps_f (E_ext . c_d) (zero where eps is
   uniform; its sum over the domain vanishes). */
static void poisson_source(or_state* s, double* b) {
    const or_params* p = &s->p;
    for (int64_t i = 0; i < s->N; ++i) b[i] = 0.0;
    for (int z = 0; z < p->nz; ++z) {
        if (!in_domain(p, z)) continue;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                double v = s->q[i];
                if (p->walls_z && z == 1) v += p->sigma_wall[0];
                if (p->walls_z && z == p->nz - 2) v += p->sigma_wall[1];
                if (p->polarization)
                    for (int d = 1; d <= 6; ++d) {
                        int zz = z + OC[d][2];
                        if (p->walls_z && !in_domain(p, zz)) continue;
                        int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(zz, p->nz));
                        double ef = 0.5 * (s->eps[i] + s->eps[j]);
                        v -= ef * (p->E_ext[0] * OC[d][0] + p->E_ext[1] * OC[d][1] + p->E_ext[2] * OC[d][2]);
                    }
                b[i] = v;
            }
    }
    int64_t cnt = 0;
    double mean = dom_sum(s, b, &cnt) / (double)cnt;
    s->last_qmean = mean;
    dom_shift(s, b, mean);
}

/* Conjugate gradients for M phi = b (M = -A with the permittivity in s->eps), from the
   current phi, to ||b + A phi|| <= tol ||b||; gauge mean(phi) = 0.  Returns 0 or -4. */
static int cg_solve(or_state* s, const double* b, double tol, int maxit, int* iters_out, double* rel_out) {
    int64_t N = s->N;
    double* r = (double*)malloc(N * sizeof(double));
    double* pp = (double*)malloc(N * sizeof(double));
    double* Mp = (double*)malloc(N * sizeof(double));
    double bnorm = sqrt(dom_dot(s, b, b));
    int it = 0, status = 0;
    double relres = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < N; ++i) s->phi[i] = 0.0;
    } else {
        /* r = b - M phi = b + A phi */
        apply_A(s, s->phi, r);
        for (int64_t i = 0; i < N; ++i) r[i] = b[i] + r[i];
        int64_t cnt;
        dom_shift(s, r, dom_sum(s, r, &cnt) / (double)cnt);
        for (int64_t i = 0; i < N; ++i) pp[i] = r[i];
        double rr = dom_dot(s, r, r);
        while (sqrt(rr) > tol * bnorm && it < maxit) {
            apply_A(s, pp, Mp);
            for (int64_t i = 0; i < N; ++i) Mp[i] = -Mp[i];
            double alpha = rr / dom_dot(s, pp, Mp);
            for (int64_t i = 0; i < N; ++i) {
                s->phi[i] += alpha * pp[i];
                r[i] -= alpha * Mp[i];
            }
            dom_shift(s, r, dom_sum(s, r, &cnt) / (double)cnt);
            double rr_new = dom_dot(s, r, r);
            double beta = rr_new / rr;
            rr = rr_new;
            for (int64_t i = 0; i < N; ++i) pp[i] = r[i] + beta * pp[i];
            ++it;
        }
        /* gauge: mean(phi) = 0 over the domain */
        dom_shift(s, s->phi, dom_sum(s, s->phi, &cnt) / (double)cnt);
        /* true residual */
        apply_A(s, s->phi, r);
        for (int64_t i = 0; i < N; ++i) r[i] = b[i] + r[i];
        relres = sqrt(dom_dot(s, r, r)) / bnorm;
        if (relres > tol) status = -4;
    }
    *iters_out = it;
    *rel_out = relres;
    free(r); free(pp); free(Mp);
    return status;
}

static int poisson_solve(or_state* s, double tol, int maxit, int* iters, double* rel) {
    int64_t N = s->N;
    double* b = (double*)malloc(N * sizeof(double));
    poisson_source(s, b);
    int it = 0;
    double relres = 0.0;
    int status = cg_solve(s, b, tol, maxit, &it, &relres);
    /* Wall layers: the potential just outside the domain follows from Gauss's law at
       the charged wall face, phi_wall = phi_adjacent + sigma / eps_adjacent. */
    const or_params* p = &s->p;
    if (p->walls_z) {
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t a1 = IDX(p, x, y, 1), a0 = IDX(p, x, y, 0);
                int64_t b1 = IDX(p, x, y, p->nz - 2), b0 = IDX(p, x, y, p->nz - 1);
                s->phi[a0] = s->phi[a1] + p->sigma_wall[0] / s->eps[a1];
                s->phi[b0] = s->phi[b1] + p->sigma_wall[1] / s->eps[b1];
            }
    }
    s->last_iters = it;
    s->last_rel = relres;
    if (iters) *iters = it;
    if (rel) *rel = relres;
    free(b);
    return status;
}

/* The paper's lagged scheme for the variable-permittivity Poisson equation (Sec. II D):
   the term with the permittivity gradient is taken at the previous potential, which
   leaves a constant-coefficient Poisson equation for the new one, solved there by a
   Fourier method.  Discretely (periodic lattices): with eps_f = eps_i + (eps_j - eps_i)/2
   the finite-volume equation sum_f eps_f (phi_j - phi_i) = -s_i splits into
     eps_i L phi_i + sum_f (eps_j - eps_i)(phi_j - phi_i) / 2 = -s_i,
   L phi_i = sum_f (phi_j - phi_i) the 7-point Laplacian, so the new potential solves
     L phi = r,  r_i = [ -s_i - sum_f (eps_j - eps_i)(phi_old_j - phi_old_i) / 2 ] / eps_i,
   with the mean of r removed (the zero wavenumber) and mean(phi) = 0.  Readings: the
   printed equation omits the 1/eps on the gradient term, which the discrete split (and
   the units) require; the Fourier inversion is of the same 7-point Laplacian, so a
   potential that satisfies the finite-volume equation is a fixed point of the scheme.
   The oracle solves L phi = r by its definition, conjugate gradients with unit
   coefficients to 1e-13, not by Fourier transforms. */
static int poisson_lagged_solve(or_state* s, int* iters, double* rel) {
    const or_params* p = &s->p;
    int64_t N = s->N;
    double* b = (double*)malloc(N * sizeof(double));
    double* rhs = (double*)malloc(N * sizeof(double));
    double* ones = (double*)malloc(N * sizeof(double));
    poisson_source(s, b);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                double lag = 0.0;
                for (int d = 1; d <= 6; ++d) {
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    lag += 0.5 * (s->eps[j] - s->eps[i]) * (s->phi[j] - s->phi[i]);
                }
                rhs[i] = (-b[i] - lag) / s->eps[i];
            }
    int64_t cnt = 0;
    dom_shift(s, rhs, dom_sum(s, rhs, &cnt) / (double)cnt);
    /* M phi = -rhs with unit coefficients */
    for (int64_t i = 0; i < N; ++i) {
        rhs[i] = -rhs[i];
        ones[i] = 1.0;
    }
    /* a direct solve needs no starting guess: start from zero */
    for (int64_t i = 0; i < N; ++i) s->phi[i] = 0.0;
    double* eps = s->eps;
    s->eps = ones;
    int it = 0;
    double relres = 0.0;
    int status = cg_solve(s, rhs, 1e-13, 100000, &it, &relres);
    s->eps = eps;
    /* the accuracy of the step: relative residual of the finite-volume equation */
    double* r = rhs;
    apply_A(s, s->phi, r);
    for (int64_t i = 0; i < N; ++i) r[i] = b[i] + r[i];
    double bnorm = sqrt(dom_dot(s, b, b));
    s->last_iters = it;
    s->last_rel = bnorm > 0.0 ? sqrt(dom_dot(s, r, r)) / bnorm : 0.0;
    if (iters) *iters = it;
    if (rel) *rel = s->last_rel;
    free(b); free(rhs); free(ones);
    return status;
}

/* ------------------------------------------------------------------------------ */
/* Step 4: field E = -grad(phi_I) + E_ext by central differences (Sec. II B).        */
/* Reading: on the wall layers the normal component is one-sided.                   */
/* ------------------------------------------------------------------------------ */
static void compute_field(or_state* s) {
    const or_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                double ex = -0.5 * (s->phi[IDX(p, wrap(x + 1, p->nx), y, z)] - s->phi[IDX(p, wrap(x - 1, p->nx), y, z)]);
                double ey = -0.5 * (s->phi[IDX(p, x, wrap(y + 1, p->ny), z)] - s->phi[IDX(p, x, wrap(y - 1, p->ny), z)]);
                double ez;
                if (p->walls_z && z == 0)
                    ez = -(s->phi[IDX(p, x, y, 1)] - s->phi[i]);
                else if (p->walls_z && z == p->nz - 1)
                    ez = -(s->phi[i] - s->phi[IDX(p, x, y, p->nz - 2)]);
                else
                    ez = -0.5 * (s->phi[IDX(p, x, y, wrap(z + 1, p->nz))] - s->phi[IDX(p, x, y, wrap(z - 1, p->nz))]);
                s->E[3 * i] = ex + p->E_ext[0];
                s->E[3 * i + 1] = ey + p->E_ext[1];
                s->E[3 * i + 2] = ez + p->E_ext[2];
            }
}

/* ------------------------------------------------------------------------------ */
/* Step 5: link fluxes on the D3Q7 links and the Nernst-Planck update.               */
/* For the canonical link (i, i+e_k), with n~ = n/psi_f (0 where psi_f = 0) and      */
/* q~ = z e n~ (eq. ionic-fluxes-disc-2):                                            */
/*   J = -D psi_f(i) psi_f(i+k) [ (n~_{i+k} - n~_i)                                  */
/*                               - (beta/4)(q~_i + q~_{i+k})(E_i + E_{i+k}).e_k      */
/*                               + s (beta dmu/(2 drho_a))(n~_i + n~_{i+k})           */
/*                                   (rho^a_{i+k} - rho^a_i) ]                       */
/* J is the physical flux from i to i+k.  Reading: the "E'" of the printed formula   */
/* is the field at the neighbour.  s is the solvation sign (+1: the printed flux).  */
/* Advection, first-order upwind (Sec. II B): each LB-fluid site sends              */
/* n_i max(u_i.e_k, 0) to i+k, so A = n_i max(u_i.e_k,0) - n_{i+k} max(-u_{i+k}.e_k,0).*/
/* Readings: the printed upwind sum uses only the site's own outflow, which is not  */
/* conservative; the donor-cell form above is its conservative counterpart, and it  */
/* acts only between LB-fluid sites.  u is the physical fluid velocity of the       */
/* forced scheme, u = (sum_s sum_d f^s_d c_d + (1/2) sum_s Phi^s) / rho: the         */
/* pre-force barycentric velocity is far from zero at a resting interface, where    */
/* the Shan-Chen force is large, and would advect ions spuriously.  The advection   */
/* does not enter the friction force, so this is not circular.                      */
/* Update: n_i(t+1) = n_i - sum over the 6 links of the outgoing flux J + A.        */
/* ------------------------------------------------------------------------------ */
static void compute_link_fluxes(or_state* s) {
    const or_params* p = &s->p;
    double kap[2];
    for (int sp = 0; sp < 2; ++sp) {
        double dmu = sp == 0 ? p->dmu_plus : p->dmu_minus;
        kap[sp] = (dmu == 0.0) ? 0.0 : p->solvation_sign * p->beta * dmu / (2.0 * p->drho_a);
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                for (int k = 0; k < 3; ++k) {
                    int d = 1 + 2 * k; /* the +e_k link */
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    for (int sp = 0; sp < 2; ++sp) {
                        double zv = sp == 0 ? 1.0 : -1.0;
                        double pfi = s->psif[i], pfj = s->psif[j];
                        double J = 0.0;
                        if (pfi > 0.0 && pfj > 0.0) {
                            double ni = s->n[sp][i] / pfi, nj = s->n[sp][j] / pfj;
                            double Esum = s->E[3 * i + k] + s->E[3 * j + k];
                            double br = (nj - ni) - 0.25 * p->beta * zv * (ni + nj) * Esum +
                                        kap[sp] * (ni + nj) * (s->rho[0][j] - s->rho[0][i]);
                            J = -p->D * br * pfi * pfj;
                        }
                        s->J[sp][3 * i + k] = J;
                    }
                }
            }
}

static void advect_and_update_ions(or_state* s) {
    const or_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                for (int k = 0; k < 3; ++k) {
                    int d = 1 + 2 * k;
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    for (int sp = 0; sp < 2; ++sp) {
                        double A = 0.0;
                        if (!s->solid[i] && !s->solid[j]) {
                            double ui = s->uphys[3 * i + k], uj = s->uphys[3 * j + k];
                            A = s->n[sp][i] * (ui > 0.0 ? ui : 0.0) - s->n[sp][j] * (-uj > 0.0 ? -uj : 0.0);
                        }
                        s->A[sp][3 * i + k] = A;
                    }
                }
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                for (int sp = 0; sp < 2; ++sp) {
                    double out = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        int d = 2 + 2 * k; /* the -e_k link: the canonical link of the neighbour below */
                        int64_t m = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                        out += (s->J[sp][3 * i + k] + s->A[sp][3 * i + k]) - (s->J[sp][3 * m + k] + s->A[sp][3 * m + k]);
                    }
                    s->nnew[sp][i] = s->n[sp][i] - out;
                }
            }
}

/* ------------------------------------------------------------------------------ */
/* Step 6: forces on the fluid components.                                          */
/* Shan-Chen (eq. shanChenForce) with G_ab = G, G_a+- = dmu+-/(drho_a cs2),           */
/* G_b+- = 0, ion pseudopotentials psi+- = n+- (dilute limit):                       */
/*   Phi^a_SC = -psi^a sum_{d} w_d [G psi^b + G_a+ psi^+ + G_a- psi^-](i+d) c_d        */
/*   Phi^b_SC = -psi^b sum_{d} w_d  G psi^a(i+d) c_d                                  */
/* Reading: fluid neighbours inside solids carry the virtual densities; ion          */
/* pseudopotentials count only on LB-fluid neighbours.                              */
/* Friction (eq. frictionforce) from the discrete fluxes, half the sum over the six  */
/* links of the site: F_fr = (1/(beta D)) (1/2) sum_{Q6} sum_+- J c_d.                */
/* Kelvin (Sec. II C), central form: F_K = +((eps_f - eps_bar)/4) sum_{Q6} E^2(i+d) c_d.   */
/* Reading: eq. kelvin prints -(eps - eps_bar)/2 grad E^2, but the Landau form it is     */
/* derived from, -E^2 grad(eps)/2 + grad(E^2 phi d eps/d phi)/2 with the permittivity law */
/* (phi d eps/d phi = eps - eps_bar), gives +(eps - eps_bar)/2 grad E^2, and the discrete */
/* total force of Sec. II E carries the plus sign.  The plus sign is taken: with it the  */
/* dielectric drop of Sec. III B elongates along the field, as reported there.           */
/* Reading: the non-Shan-Chen forces (and the body force rho g) are split between    */
/* the components by mass fraction rho^s / rho.                                     */
/* ------------------------------------------------------------------------------ */
static void compute_forces(or_state* s) {
    const or_params* p = &s->p;
    double Gpm[2];
    Gpm[0] = (p->dmu_plus == 0.0) ? 0.0 : p->solvation_sign * p->dmu_plus / (p->drho_a * CS2);
    Gpm[1] = (p->dmu_minus == 0.0) ? 0.0 : p->solvation_sign * p->dmu_minus / (p->drho_a * CS2);
    double ebar = 0.5 * (p->eps_a + p->eps_b);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                for (int k = 0; k < 3; ++k) s->Phi[0][3 * i + k] = s->Phi[1][3 * i + k] = s->uphys[3 * i + k] = 0.0;
                if (s->solid[i]) continue;
                double sa[3] = {0, 0, 0}, sb[3] = {0, 0, 0};
                for (int d = 1; d < OQ; ++d) {
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    double ion = s->solid[j] ? 0.0 : (Gpm[0] * s->n[0][j] + Gpm[1] * s->n[1][j]);
                    double ta = OW[d] * (p->G * s->psi[1][j] + ion);
                    double tb = OW[d] * (p->G * s->psi[0][j]);
                    for (int k = 0; k < 3; ++k) {
                        sa[k] += ta * OC[d][k];
                        sb[k] += tb * OC[d][k];
                    }
                }
                double Ffr[3] = {0, 0, 0}, FK[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) {
                    int64_t m = IDX(p, wrap(x - (k == 0), p->nx), wrap(y - (k == 1), p->ny), wrap(z - (k == 2), p->nz));
                    double jsum = 0.0;
                    for (int sp = 0; sp < 2; ++sp) jsum += s->J[sp][3 * i + k] + s->J[sp][3 * m + k];
                    Ffr[k] = 0.5 * jsum / (p->beta * p->D);
                    int64_t up = IDX(p, wrap(x + (k == 0), p->nx), wrap(y + (k == 1), p->ny), wrap(z + (k == 2), p->nz));
                    double E2u = s->E[3 * up] * s->E[3 * up] + s->E[3 * up + 1] * s->E[3 * up + 1] + s->E[3 * up + 2] * s->E[3 * up + 2];
                    double E2m = s->E[3 * m] * s->E[3 * m] + s->E[3 * m + 1] * s->E[3 * m + 1] + s->E[3 * m + 2] * s->E[3 * m + 2];
                    FK[k] = 0.25 * (s->epsf[i] - ebar) * (E2u - E2m);
                }
                double ra = s->rho[0][i], rb = s->rho[1][i], rt = ra + rb;
                for (int k = 0; k < 3; ++k) {
                    double Frest = Ffr[k] + FK[k] + rt * p->body_accel[k];
                    s->Phi[0][3 * i + k] = -s->psi[0][i] * sa[k] + (ra / rt) * Frest;
                    s->Phi[1][3 * i + k] = -s->psi[1][i] * sb[k] + (rb / rt) * Frest;
                    /* physical velocity: mean of the pre- and post-collision momentum */
                    s->uphys[3 * i + k] = s->u[3 * i + k] + 0.5 * (s->Phi[0][3 * i + k] + s->Phi[1][3 * i + k]) / rt;
                }
            }
}

/* ------------------------------------------------------------------------------ */
/* Steps 7-8: collision and streaming.                                              */
/*   u_e^s = u + tau Phi^s / rho^s   (velocity shift, Sec. II A)                       */
/*   f*  = f - (f - f~(rho^s, u_e^s)) / tau                                          */
/* Push streaming to r + c_d.  A population headed into a solid site is reflected   */
/* half-way (Sec. II E).  Reading (the printed coefficient and time arguments are   */
/* garbled): the standard moving-wall rule                                         */
/*   f_{d*}(r, t+1) = f*_d(r) - 6 w_d rho^s(r) (c_d . v),                              */
/* with v the velocity of the particle that owns the solid site (0 for walls), and  */
/* the momentum handed to that particle per link is (2 f*_d - 6 w_d rho^s (c_d.v)) c_d.*/
/* ------------------------------------------------------------------------------ */
static void collide(or_state* s) {
    const or_params* p = &s->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (s->solid[i]) continue;
                for (int c = 0; c < 2; ++c) {
                    double ue[3];
                    for (int k = 0; k < 3; ++k) ue[k] = s->u[3 * i + k] + p->tau * s->Phi[c][3 * i + k] / s->rho[c][i];
                    double feq[OQ];
                    equilibrium(s->rho[c][i], ue, feq);
                    for (int d = 0; d < OQ; ++d) {
                        double* fv = &s->f[c][(int64_t)d * s->N + i];
                        *fv = *fv - (*fv - feq[d]) / p->tau;
                    }
                }
            }
}

static void stream(or_state* s) {
    const or_params* p = &s->p;
    int64_t N = s->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (s->solid[i]) continue;
                for (int d = 0; d < OQ; ++d) {
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    for (int c = 0; c < 2; ++c) {
                        double fstar = s->f[c][(int64_t)d * N + i];
                        if (s->solid[j]) {
                            double cv = 0.0;
                            int o = s->owner[j];
                            if (o >= 0)
                                cv = OC[d][0] * s->pv[3 * o] + OC[d][1] * s->pv[3 * o + 1] + OC[d][2] * s->pv[3 * o + 2];
                            s->fs[c][(int64_t)OOPP[d] * N + i] = fstar - 6.0 * OW[d] * s->rho[c][i] * cv;
                        } else {
                            s->fs[c][(int64_t)d * N + j] = fstar;
                        }
                    }
                }
            }
}

/* momentum handed to the particles by the links of this step (serial, plain) */
static void momentum_exchange(or_state* s) {
    const or_params* p = &s->p;
    int64_t N = s->N;
    for (int j = 0; j < s->np; ++j) s->pF[3 * j] = s->pF[3 * j + 1] = s->pF[3 * j + 2] = 0.0;
    if (s->np == 0) return;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (s->solid[i]) continue;
                for (int d = 1; d < OQ; ++d) {
                    int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(z + OC[d][2], p->nz));
                    if (!s->solid[j] || s->owner[j] < 0) continue;
                    int o = s->owner[j];
                    double cv = OC[d][0] * s->pv[3 * o] + OC[d][1] * s->pv[3 * o + 1] + OC[d][2] * s->pv[3 * o + 2];
                    for (int c = 0; c < 2; ++c) {
                        double fstar = s->f[c][(int64_t)d * N + i];
                        double dp = 2.0 * fstar - 6.0 * OW[d] * s->rho[c][i] * cv;
                        for (int k = 0; k < 3; ++k) s->pF[3 * o + k] += dp * OC[d][k];
                    }
                }
            }
}

/* ------------------------------------------------------------------------------ */
/* Step 9: particles (Sec. II E).  Force = momentum exchange + sum of q_c E over the */
/* particle's sites + Hertz contact + lubrication; symplectic Euler (v then x).      */
/* Readings: the Hertz force on i is +k_H delta^{3/2} n_ij (repulsive); lubrication as */
/* printed with eta the fluid dynamic viscosity parameter; translation only.        */
/* ------------------------------------------------------------------------------ */
static void particle_update(or_state* s) {
    const or_params* p = &s->p;
    if (s->np == 0) return;
    /* electric force on the distributed particle charge */
    for (int64_t i = 0; i < s->N; ++i) {
        int o = s->owner[i];
        if (o < 0) continue;
        for (int k = 0; k < 3; ++k) s->pF[3 * o + k] += s->qc[i] * s->E[3 * i + k];
    }
    int L[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < s->np; ++a)
        for (int b = 0; b < s->np; ++b) {
            if (a == b) continue;
            double dv[3], dist2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                dv[k] = min_image(s->px[3 * a + k] - s->px[3 * b + k], L[k]);
                dist2 += dv[k] * dv[k];
            }
            double dist = sqrt(dist2);
            if (dist == 0.0) continue;
            double nh[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
            double delta = s->pr[a] + s->pr[b] - dist;
            if (delta > 0.0) {
                double fh = p->k_hertz * pow(delta, 1.5);
                for (int k = 0; k < 3; ++k) s->pF[3 * a + k] += fh * nh[k];
            }
            double gap = dist - s->pr[a] - s->pr[b];
            if (gap < 2.0 / 3.0 && gap > 0.0) {
                double rp = 0.5 * (s->pr[a] + s->pr[b]);
                double nv = 0.0;
                for (int k = 0; k < 3; ++k) nv += nh[k] * (s->pv[3 * a + k] - s->pv[3 * b + k]);
                double fl = -1.5 * M_PI * p->eta * rp * rp * nv * (1.0 / gap - 1.0);
                for (int k = 0; k < 3; ++k) s->pF[3 * a + k] += fl * nh[k];
            }
        }
    if (!p->move_particles) return;
    for (int a = 0; a < s->np; ++a) {
        double m = p->particle_rho * (4.0 / 3.0) * M_PI * s->pr[a] * s->pr[a] * s->pr[a];
        for (int k = 0; k < 3; ++k) {
            s->pv[3 * a + k] += s->pF[3 * a + k] / m;
            s->px[3 * a + k] += s->pv[3 * a + k];
        }
    }
}

/* ------------------------------------------------------------------------------ */
/* Moving particles (Sec. II E): once the particles have moved, the projection is    */
/* redone (solid mask, solid fraction, owner and charge per site, build_geometry)    */
/* and the sites the move converts are handled:                                       */
/*  - fluid -> solid (covered): the site's fluid momentum sum_s sum_d f^s_d c_d goes  */
/*    to the covering particle and its populations are removed.  Reading: the        */
/*    printed F_c carries a minus sign; conservation of momentum, which the text      */
/*    states as the purpose, makes the particle's gain the fluid's loss.             */
/*  - solid -> fluid (uncovered): populations f~(rho_bar^s, v) with v the velocity of */
/*    the particle that covered the site and rho_bar^s the mean density of its D3Q19  */
/*    neighbours that are fluid before and after the move (Reading: printed as a sum; */
/*    the mean, as for the virtual densities).  The particle gives up the momentum of */
/*    the new fluid, sum_s rho_bar^s v (Reading: the sign as for F_c).               */
/* Ions live where the fluid fraction is positive (the partial-volume fluxes carry    */
/* them into sites whose centre lies inside a particle).  Reading: the ion events are */
/* therefore those of the fluid fraction: a site whose fraction drops to zero has its */
/* ions shared equally among its axis (D3Q7) neighbours that keep a positive fraction */
/* (the displacement is isotropic, the ions move on the axis links and equal shares   */
/* keep them exactly); a site whose fraction rises from zero starts without ions,     */
/* which it already holds.                                                            */
/* The momentum transfers change the particle velocities at once (the same as adding */
/* them to the next step's force in the symplectic update).                          */
/* ------------------------------------------------------------------------------ */
static void reproject(or_state* s) {
    const or_params* p = &s->p;
    int64_t N = s->N;
    uint8_t* was_solid = (uint8_t*)malloc((size_t)N);
    int32_t* was_owner = (int32_t*)malloc((size_t)N * sizeof(int32_t));
    double* was_psif = (double*)malloc((size_t)N * sizeof(double));
    memcpy(was_solid, s->solid, (size_t)N);
    memcpy(was_owner, s->owner, (size_t)N * sizeof(int32_t));
    memcpy(was_psif, s->psif, (size_t)N * sizeof(double));
    build_geometry(s);
    double* dP = (double*)calloc((size_t)(3 * (s->np > 0 ? s->np : 1)), sizeof(double));
    double feq[OQ];
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (!was_solid[i] && s->solid[i]) {
                    int o = s->owner[i];
                    for (int c = 0; c < 2; ++c)
                        for (int d = 0; d < OQ; ++d) {
                            double* fv = &s->f[c][(int64_t)d * N + i];
                            if (o >= 0)
                                for (int k = 0; k < 3; ++k) dP[3 * o + k] += *fv * OC[d][k];
                            *fv = 0.0;
                        }
                }
                if (was_psif[i] > 0.0 && s->psif[i] == 0.0) {
                    int cnt = 0;
                    for (int d = 1; d <= 6; ++d) {
                        int zz = z + OC[d][2];
                        if (p->walls_z && (zz < 0 || zz >= p->nz)) continue;
                        int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(zz, p->nz));
                        if (s->psif[j] > 0.0) ++cnt;
                    }
                    for (int sp = 0; sp < 2 && cnt > 0; ++sp) {
                        double share = s->n[sp][i] / cnt;
                        for (int d = 1; d <= 6; ++d) {
                            int zz = z + OC[d][2];
                            if (p->walls_z && (zz < 0 || zz >= p->nz)) continue;
                            int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(zz, p->nz));
                            if (s->psif[j] > 0.0) s->n[sp][j] += share;
                        }
                        s->n[sp][i] = 0.0;
                    }
                }
            }
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t i = IDX(p, x, y, z);
                if (!(was_solid[i] && !s->solid[i])) continue;
                int o = was_owner[i];
                double v[3] = {0, 0, 0};
                if (o >= 0)
                    for (int k = 0; k < 3; ++k) v[k] = s->pv[3 * o + k];
                for (int c = 0; c < 2; ++c) {
                    double acc = 0.0;
                    int cnt = 0;
                    for (int d = 1; d < OQ; ++d) {
                        int zz = z + OC[d][2];
                        if (p->walls_z && (zz < 0 || zz >= p->nz)) continue;
                        int64_t j = IDX(p, wrap(x + OC[d][0], p->nx), wrap(y + OC[d][1], p->ny), wrap(zz, p->nz));
                        if (was_solid[j] || s->solid[j]) continue;
                        double r = 0.0;
                        for (int e = 0; e < OQ; ++e) r += s->f[c][(int64_t)e * N + j];
                        acc += r;
                        ++cnt;
                    }
                    double rb = cnt > 0 ? acc / cnt : 0.0;
                    or_equilibrium(rb, v, feq);
                    for (int d = 0; d < OQ; ++d) s->f[c][(int64_t)d * N + i] = feq[d];
                    if (o >= 0)
                        for (int k = 0; k < 3; ++k) dP[3 * o + k] -= rb * v[k];
                }
            }
    for (int j = 0; j < s->np; ++j) {
        double m = p->particle_rho * (4.0 / 3.0) * M_PI * s->pr[j] * s->pr[j] * s->pr[j];
        for (int k = 0; k < 3; ++k) s->pv[3 * j + k] += dP[3 * j + k] / m;
    }
    free(dP);
    free(was_solid);
    free(was_owner);
    free(was_psif);
}

/* ------------------------------------------------------------------------------ */
/* Public API                                                                       */
/* ------------------------------------------------------------------------------ */
static double* dalloc(int64_t n) { return (double*)calloc((size_t)n, sizeof(double)); }

void or_destroy(or_state* s);

/* particles: n x 8 doubles (x, y, z, vx, vy, vz, radius, charge) */
or_state* or_create(const or_params* prm, const double* rho_a, const double* rho_b, const double* n_plus,
                    const double* n_minus, const double* particles, int32_t n_particles) {
    lattice_setup();
    if (prm->poisson_lagged && prm->walls_z) return NULL; /* the lagged Fourier scheme is periodic */
    if (prm->poisson_lagged && prm->polarization) return NULL; /* its right-hand side has no polarisation term */
    /* with walls the wall faces carry no displacement, so a polarising field normal to them is undefined */
    if (prm->polarization && prm->walls_z && prm->E_ext[2] != 0.0) return NULL;
    if (prm->reproject && !prm->move_particles) return NULL; /* only moving particles are projected anew */
    or_state* s = (or_state*)calloc(1, sizeof(or_state));
    s->p = *prm;
    set_threads(&s->p);
    int64_t N = (int64_t)prm->nx * prm->ny * prm->nz;
    s->N = N;
    for (int c = 0; c < 2; ++c) {
        s->f[c] = dalloc(OQ * N); s->fs[c] = dalloc(OQ * N);
        s->n[c] = dalloc(N); s->nnew[c] = dalloc(N);
        s->rho[c] = dalloc(N); s->psi[c] = dalloc(N);
        s->J[c] = dalloc(3 * N); s->A[c] = dalloc(3 * N); s->Phi[c] = dalloc(3 * N);
    }
    s->phi = dalloc(N); s->u = dalloc(3 * N); s->uphys = dalloc(3 * N); s->q = dalloc(N); s->eps = dalloc(N); s->epsf = dalloc(N);
    s->E = dalloc(3 * N); s->psis = dalloc(N); s->psif = dalloc(N); s->qc = dalloc(N);
    s->solid = (uint8_t*)calloc((size_t)N, 1);
    s->owner = (int32_t*)calloc((size_t)N, sizeof(int32_t));
    s->np = n_particles;
    int np = n_particles > 0 ? n_particles : 1;
    s->px = dalloc(3 * np); s->pv = dalloc(3 * np); s->pr = dalloc(np); s->pQ = dalloc(np);
    s->pF = dalloc(3 * np); s->px0 = dalloc(3 * np);
    for (int j = 0; j < n_particles; ++j) {
        for (int k = 0; k < 3; ++k) {
            s->px[3 * j + k] = particles[8 * j + k];
            s->px0[3 * j + k] = particles[8 * j + k];
            s->pv[3 * j + k] = particles[8 * j + 3 + k];
        }
        s->pr[j] = particles[8 * j + 6];
        s->pQ[j] = particles[8 * j + 7];
    }
    build_geometry(s);
    /* initial populations f = f~(rho^s, 0) on fluid sites (Reading: fluid at rest) */
    double zero[3] = {0, 0, 0}, feq[OQ];
    /* Reading: the given ion densities are per unit fluid volume; a site holds them in
       proportion to its fluid fraction (Sec. II E: at equilibrium the amount of ions at
       a site is proportional to psi_f), so fully solid sites start empty. */
    for (int64_t i = 0; i < N; ++i) {
        s->n[0][i] = n_plus[i] * s->psif[i];
        s->n[1][i] = n_minus[i] * s->psif[i];
        if (s->solid[i]) continue;
        const double* rr[2] = {rho_a, rho_b};
        for (int c = 0; c < 2; ++c) {
            equilibrium(rr[c][i], zero, feq);
            for (int d = 0; d < OQ; ++d) s->f[c][(int64_t)d * N + i] = feq[d];
        }
    }
    compute_moments(s);
    compute_charge_perm(s);
    poisson_solve(s, s->p.poisson_tol, s->p.poisson_maxit, NULL, NULL);
    compute_field(s);
    return s;
}

void or_destroy(or_state* s) {
    if (!s) return;
    for (int c = 0; c < 2; ++c) {
        free(s->f[c]); free(s->fs[c]); free(s->n[c]); free(s->nnew[c]); free(s->rho[c]); free(s->psi[c]);
        free(s->J[c]); free(s->A[c]); free(s->Phi[c]);
    }
    free(s->phi); free(s->u); free(s->uphys); free(s->q); free(s->eps); free(s->epsf); free(s->E); free(s->psis);
    free(s->psif); free(s->qc); free(s->solid); free(s->owner);
    free(s->px); free(s->pv); free(s->pr); free(s->pQ); free(s->pF); free(s->px0);
    free(s);
}

/* One full step from the current state.  Returns 0, or -4 if the Poisson solve did
   not reach its tolerance. */
static int step_once(or_state* s) {
    compute_moments(s);
    compute_charge_perm(s);
    int st = s->p.poisson_lagged ? poisson_lagged_solve(s, NULL, NULL)
                                 : poisson_solve(s, s->p.poisson_tol, s->p.poisson_maxit, NULL, NULL);
    compute_field(s);
    compute_link_fluxes(s);
    compute_forces(s);
    advect_and_update_ions(s);
    collide(s);
    stream(s);
    momentum_exchange(s);
    particle_update(s);
    for (int c = 0; c < 2; ++c) {
        double* t = s->f[c]; s->f[c] = s->fs[c]; s->fs[c] = t;
        t = s->n[c]; s->n[c] = s->nnew[c]; s->nnew[c] = t;
    }
    if (s->p.reproject && s->np > 0) reproject(s);
    s->steps++;
    return st;
}

int or_step(or_state* s, int32_t nsteps) {
    set_threads(&s->p);
    int worst = 0;
    for (int t = 0; t < nsteps; ++t) {
        int st = step_once(s);
        if (st != 0) worst = st;
    }
    /* refresh the diagnostic fields for the state now held */
    compute_moments(s);
    compute_charge_perm(s);
    return worst;
}

/* One lagged Fourier solve (see poisson_lagged_solve) for the current state, from the
   potential it holds. */
int or_poisson_lagged(or_state* s, int32_t* iters, double* rel) {
    set_threads(&s->p);
    compute_moments(s);
    compute_charge_perm(s);
    int it = 0;
    int st = poisson_lagged_solve(s, &it, rel);
    compute_field(s);
    if (iters) *iters = it;
    return st;
}

int or_poisson(or_state* s, double tol, int32_t maxit, int32_t* iters, double* rel) {
    set_threads(&s->p);
    compute_moments(s);
    compute_charge_perm(s);
    int it = 0;
    int st = poisson_solve(s, tol, maxit, &it, rel);
    compute_field(s);
    if (iters) *iters = it;
    return st;
}

/* Field ids: 0 rho_a, 1 rho_b, 2 n+, 3 n-, 4 phi, 5-7 u (x,y,z), 8 q, 9 eps,
   10 psi_s, 11 solid, 12-14 E, 15 owner, 16 q_c, 17-19 Phi^a, 20-22 Phi^b,
   23-25 J+ (x,y,z links), 26-28 J-, 29-31 A+, 32-34 A-, 35-37 physical velocity */
int or_get_field(const or_state* s, int32_t which, double* out) {
    int64_t N = s->N;
    for (int64_t i = 0; i < N; ++i) {
        double v;
        switch (which) {
            case 0: v = s->rho[0][i]; break;
            case 1: v = s->rho[1][i]; break;
            case 2: v = s->n[0][i]; break;
            case 3: v = s->n[1][i]; break;
            case 4: v = s->phi[i]; break;
            case 5: case 6: case 7: v = s->u[3 * i + (which - 5)]; break;
            case 8: v = s->q[i]; break;
            case 9: v = s->eps[i]; break;
            case 10: v = s->psis[i]; break;
            case 11: v = s->solid[i]; break;
            case 12: case 13: case 14: v = s->E[3 * i + (which - 12)]; break;
            case 15: v = s->owner[i]; break;
            case 16: v = s->qc[i]; break;
            case 17: case 18: case 19: v = s->Phi[0][3 * i + (which - 17)]; break;
            case 20: case 21: case 22: v = s->Phi[1][3 * i + (which - 20)]; break;
            case 23: case 24: case 25: v = s->J[0][3 * i + (which - 23)]; break;
            case 26: case 27: case 28: v = s->J[1][3 * i + (which - 26)]; break;
            case 29: case 30: case 31: v = s->A[0][3 * i + (which - 29)]; break;
            case 32: case 33: case 34: v = s->A[1][3 * i + (which - 32)]; break;
            case 35: case 36: case 37: v = s->uphys[3 * i + (which - 35)]; break;
            default: return -1;
        }
        out[i] = v;
    }
    return 0;
}

/* populations of component c (0 = a, 1 = b), 19 x N in the oracle's velocity order */
void or_get_populations(const or_state* s, int32_t c, double* out) {
    memcpy(out, s->f[c], sizeof(double) * OQ * s->N);
}

/* Replace the dynamic state (populations, ions, potential warm start, particle
   velocities and positions) so that a single step can be checked from any state. */
void or_set_state(or_state* s, const double* fa, const double* fb, const double* np_, const double* nm,
                  const double* phi, const double* particles) {
    int64_t N = s->N;
    memcpy(s->f[0], fa, sizeof(double) * OQ * N);
    memcpy(s->f[1], fb, sizeof(double) * OQ * N);
    memcpy(s->n[0], np_, sizeof(double) * N);
    memcpy(s->n[1], nm, sizeof(double) * N);
    memcpy(s->phi, phi, sizeof(double) * N);
    if (particles)
        for (int j = 0; j < s->np; ++j)
            for (int k = 0; k < 3; ++k) {
                s->px[3 * j + k] = particles[8 * j + k];
                s->pv[3 * j + k] = particles[8 * j + 3 + k];
            }
    compute_moments(s);
    compute_charge_perm(s);
}

/* Change the external field between steps (the drop experiments of Sec. III B relax the
   fluid before a field is applied).  Returns -1 where the field is undefined. */
int or_set_field(or_state* s, const double* E_ext) {
    if (s->p.polarization && s->p.walls_z && E_ext[2] != 0.0) return -1;
    for (int k = 0; k < 3; ++k) s->p.E_ext[k] = E_ext[k];
    return 0;
}

/* particles out: n x 9 doubles (x, y, z, vx, vy, vz, Fx, Fy, Fz of the last step) */
void or_get_particles(const or_state* s, double* out) {
    for (int j = 0; j < s->np; ++j) {
        for (int k = 0; k < 3; ++k) {
            out[9 * j + k] = s->px[3 * j + k];
            out[9 * j + 3 + k] = s->pv[3 * j + k];
            out[9 * j + 6 + k] = s->pF[3 * j + k];
        }
    }
}

/* Observables (FP64): [0] sum rho_a (fluid), [1] sum rho_b, [2] sum n+, [3] sum n-,
   [4] sum q, [5-7] fluid momentum, [8] max |u|, [9] Poisson iterations, [10] Poisson
   relative residual, [11] removed source mean, [12-14] mean particle displacement,
   [15-17] particle momentum. */
void or_observables(const or_state* s, double* out) {
    double t[18];
    memset(t, 0, sizeof(t));
    int64_t N = s->N;
    for (int64_t i = 0; i < N; ++i) {
        t[2] += s->n[0][i];
        t[3] += s->n[1][i];
        t[4] += s->q[i];
        if (s->solid[i]) continue;
        t[0] += s->rho[0][i];
        t[1] += s->rho[1][i];
        double rt = s->rho[0][i] + s->rho[1][i];
        double um = 0.0;
        for (int k = 0; k < 3; ++k) {
            t[5 + k] += rt * s->u[3 * i + k];
            um += s->u[3 * i + k] * s->u[3 * i + k];
        }
        um = sqrt(um);
        if (um > t[8]) t[8] = um;
    }
    t[9] = s->last_iters;
    t[10] = s->last_rel;
    t[11] = s->last_qmean;
    for (int j = 0; j < s->np; ++j) {
        double m = s->p.particle_rho * (4.0 / 3.0) * M_PI * s->pr[j] * s->pr[j] * s->pr[j];
        for (int k = 0; k < 3; ++k) {
            t[12 + k] += (s->px[3 * j + k] - s->px0[3 * j + k]) / s->np;
            t[15 + k] += m * s->pv[3 * j + k];
        }
    }
    memcpy(out, t, sizeof(t));
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
