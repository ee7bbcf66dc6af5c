/*
 * ek.h — C ABI of the MI355X (gfx950) coupled electrokinetic lattice library.
 *
 * The library advances the coupled lattice method of Rivas, Frijters, Pagonabarraga
 * and Harting, "Mesoscopic electrohydrodynamic simulations of binary colloidal
 * suspensions" (arXiv:1712.08494), Sec. II:
 *   - two fluid components a, b on a D3Q19 lattice with BGK collision and the
 *     Shan-Chen velocity-shift forcing (Sec. II A, eq. BoltzmannBGKLattice);
 *   - two monovalent ion species by the link-flux Nernst-Planck scheme on the six
 *     D3Q7 links (Sec. II B, eq. nernst-planck-disc; Sec. II E, eq. ionic-fluxes-disc-2);
 *   - Shan-Chen fluid/fluid and solvation couplings, ion friction and the Kelvin
 *     force (Sec. II C, eqs. shanChenForce, frictionforce, kelvin);
 *   - the variable-permittivity Poisson equation (Sec. II D, eq. electric_potential);
 *   - resolved rigid spheres: halfway bounce-back, momentum exchange, solid fraction,
 *     distributed charge and permittivity (Sec. II E).
 *
 * Conventions for every call:
 *   - Lattice sites are indexed x fastest: i = x + nx * (y + ny * z).
 *   - Host arrays are double precision; they are borrowed for the duration of the
 *     call only and never retained.
 *   - Device memory of a context is allocated by ek_init and released by ek_destroy, or
 *     carved from a workspace the caller owns (ek_workspace_bytes, ek_init_ws).
 *   - All work of a context is enqueued on the HIP stream given to ek_init (which may
 *     be a stream owned by the caller, e.g. PyTorch's current stream).
 *   - Calls return an ek_status; no exception or signal crosses the ABI.  On error,
 *     ek_last_error(ctx) holds a message.  A context is not thread safe; one context
 *     must not be used from two threads at once.
 */
#ifndef EK_H
#define EK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ek_status;
#define EK_OK 0
#define EK_EINVAL (-1)     /* invalid argument or parameter */
#define EK_ENOMEM (-2)     /* device or host allocation failed */
#define EK_EHIP (-3)       /* a HIP runtime call failed */
#define EK_ENOCONV (-4)    /* Poisson solve stopped at maxit above the tolerance */
#define EK_ENONFINITE (-5) /* a NaN or Inf was found by ek_observables */
#define EK_ESTATE (-6)     /* call not valid in the context's current state */

#define EK_POISSON_AUTO 0 /* multigrid when every axis divides by 4, else SOR */
#define EK_POISSON_SOR 1  /* red-black successive over-relaxation */
#define EK_POISSON_MG 2   /* geometric multigrid V-cycles (EINVAL if the lattice cannot be coarsened) */
#define EK_POISSON_FFT 3  /* the lagged Fourier scheme of Sec. II D, periodic lattices only: each step solves
                             L phi = r once by FFT, L the 7-point Laplacian and
                             r = [-s - sum_f (eps_j - eps_i)(phi_old_j - phi_old_i)/2] / eps with the
                             gradient term at the previous potential (mean(r) and mean(phi) = 0); a
                             converged finite-volume potential is its fixed point.  The initial potential
                             and ek_poisson use the converged solver (multigrid or SOR) */

#define EK_FP64 0 /* populations, ions, charge and permittivity in double */
#define EK_FP32 1 /* populations as float deviations from w_d rho_ref, ions in float; phi stays double */

typedef struct ek_params {
    int32_t nx, ny, nz;         /* lattice size; nx must be even (red-black ordering) */
    int32_t walls_z;            /* 0: periodic in z; 1: solid charged walls at z = 0 and z = nz-1 */
    int32_t precision;          /* EK_FP64 or EK_FP32 */
    int32_t poisson_maxit;      /* maximum Poisson iterations per solve (SOR sweeps or V-cycles) */
    int32_t poisson_solver;     /* EK_POISSON_AUTO, EK_POISSON_SOR, EK_POISSON_MG or EK_POISSON_FFT */
    int32_t subsample;          /* sub-cells per axis for the particle solid fraction (e.g. 8) */
    int32_t move_particles;     /* 1: integrate particle motion every step */
    double tau;                 /* BGK relaxation time of both fluids (> 1/2) */
    double G;                   /* fluid/fluid Shan-Chen coupling G_ab */
    double rho0;                /* pseudopotential reference density: psi = rho0 (1 - exp(-rho/rho0)) */
    double rho_ref[2];          /* FP32 deviation reference densities of a, b; <= 0: the harmonic mean
                                   2 lo hi / (lo + hi) of the initial fluid range [lo, hi] */
    double D;                   /* ion diffusivity (both species) */
    double beta;                /* 1 / k_B T */
    double dmu[2];              /* Gibbs transfer energies of the cation and the anion */
    double drho_a;              /* bulk difference of rho^a between the phases (solvation scale) */
    double solvation_sign;      /* +1: the printed discrete solvation flux; -1 flips flux and coupling together */
    double eps_a, eps_b, eps_p; /* permittivities of fluid a, fluid b and the particles */
    double E_ext[3];            /* uniform external field */
    double body_accel[3];       /* uniform body acceleration g (force density rho g) */
    double sigma_wall[2];       /* surface charge density of the z = 0 and z = nz-1 walls */
    double poisson_tol;         /* relative residual ||r||_2 <= tol ||s||_2 of the Poisson solve */
    double sor_omega;           /* over-relaxation factor; <= 0: chosen from the lattice size */
    double particle_rho;        /* particle mass density (mass = rho_p 4/3 pi r^3) */
    double k_hertz;             /* Hertz contact stiffness */
    double eta;                 /* dynamic viscosity used by the lubrication force */
    int32_t phi_history;        /* warm start of each Poisson solve from the potentials of the last steps:
                                   1 the previous one, 2 linear and 3 quadratic extrapolation in time;
                                   0 adaptive: the order (2 or 3) whose last measured start residual was
                                   smaller, the other re-probed every 64 steps (deterministic) */
    int32_t moment_state;       /* 1: store, per site and component, the density and the equilibrium
                                   velocity u_e = u' + Phi / rho of the last collision instead of the 19
                                   populations.  At tau = 1 the post-collision populations are the
                                   equilibria of exactly these values (Sec. II A, BGK at tau = 1), so the
                                   step is the same computation with populations gathered from the
                                   neighbours by the moments pass (halfway bounce-back at the walls): 8
                                   values per site instead of 38 cross HBM.  Requires tau = 1 and no
                                   particles; not with ek_forward_ckpt / ek_adjoint or batches.
                                   ek_get_populations reconstructs the populations.  0: stored populations */
    int32_t sweep_band;         /* workgroup order of the lattice stencil sweeps (force and fused passes): each
                                   of the 8 XCDs sweeps its eighth of the z-planes in bands of sweep_band
                                   consecutive workgroups (256 sites each) of a plane, through every plane of
                                   its slab before the next band, so that the stencil's neighbour planes stay
                                   in the XCD's L2.  0 or -1: whole planes in turn (measured fastest since the
                                   particle sites run in a kernel of their own).  Used when nx*ny is a multiple
                                   of 256, nz of 8 and the band divides a plane; otherwise whole planes.
                                   Results do not depend on it (bit for bit) */
    int32_t poisson_cycles;     /* 0: each step's Poisson solve runs multigrid V-cycles until the relative
                                   residual meets poisson_tol, which reads residuals back to the host (one or
                                   two synchronisations per step).  1..64: each step runs exactly that many
                                   V-cycles and reads nothing back, so ek_step only enqueues work; the start
                                   and end residuals stay on the device and ek_observables reports them
                                   (poisson_rel, poisson_rel0, and poisson_rel_max, the largest since its last
                                   call).  The warm start is then linear in time unless phi_history is set.
                                   Multigrid contexts only (EK_EINVAL otherwise).  ek_poisson and the solve of
                                   ek_init always run to the tolerance */
    int32_t fp32_plain_collision; /* FP32 populations: 0 (default) makes the collision conserve each site's
                                   mass exactly: the moments pass sums the populations in FP64, and the rest
                                   population takes the remainder of the other 18, stored as two floats (8 B
                                   more per site and component).  At a steady state the FP32 roundings of a
                                   plain collision repeat identically every step, and the mass then drifts
                                   linearly (about 5e-9 per step on the walls/interface column).  1: the plain
                                   FP32 collision.  FP64 and the tau = 1 moment state ignore it */
    int32_t polarization;       /* 1: the external field also polarises the dielectric.  As printed (Sec. II D,
                                   eq. electric_potential) the potential is sourced by the charge alone and
                                   E = -grad phi + E_ext, so an ion-free dielectric feels no Kelvin force in a
                                   uniform field.  With 1 the solve imposes Gauss's law on the total
                                   displacement eps (-grad phi + E_ext) through every face: the source gains
                                   -sum over the six faces of eps_face (E_ext . c_d).  Needed for the dielectric
                                   droplet of Sec. III B.  Not with EK_POISSON_FFT, reverse mode, or walls with
                                   E_ext[2] != 0 (the wall faces carry no displacement) (EK_EINVAL).
                                   0 (default): the printed model */
    int32_t reproject;          /* 1: moving particles are projected anew after every step (Sec. II E): solid
                                   mask, solid fraction, owner and charge per site follow the particles; a
                                   fluid site they cover hands its momentum to the particle, a site they
                                   uncover gets the equilibrium at the mean density of its neighbours that
                                   stay fluid, moving with the particle (which gives up that momentum), and
                                   the ions of a site whose fluid fraction drops to zero are shared equally
                                   among its axis neighbours that keep fluid.  Needs move_particles = 1,
                                   every axis at least 2 ceil(max radius) + 9 sites long and a move below
                                   one site per step; subsample at most 31; not with ek_autotune_multigrid.
                                   The projection walks a box of (2 ceil(r) + 9)^3 sites per particle,
                                   checking the particles whose boxes meet it (0.6 ms per step for 200
                                   spheres of radius 4 at 256^3), and rebuilds the list of particle-path
                                   sites on the device.  Device memory: np^2 ints besides the boxes.
                                   0 (default): the mask set up by ek_init stays (the particles may still
                                   move) */
} ek_params;

typedef struct ek_particle {
    double x[3];   /* centre (lattice units, site centres at integers) */
    double v[3];   /* velocity */
    double radius; /* sphere radius */
    double charge; /* total charge Q, spread over the covered sites by solid fraction */
} ek_particle;

typedef struct ek_obs {
    double sum_rho[2];     /* total mass of a and b over fluid sites */
    double sum_n[2];       /* total cations, anions over all sites */
    double sum_q;          /* total charge (ions + particles) */
    double momentum[3];    /* total fluid momentum sum_d f_d c_d (pre-collision) */
    double max_u;          /* max |u| of the pre-force barycentric velocity */
    double source_mean;    /* mean removed from the Poisson source by the last solve */
    double poisson_rel;    /* relative residual reached by the last solve (-1 after a lagged Fourier step:
                              not measured) */
    int64_t poisson_iters; /* iterations (SOR sweeps or V-cycles) of the last solve */
    int64_t poisson_total; /* iterations summed over all solves since ek_init */
    int32_t poisson_mg_levels; /* multigrid levels in use (0: SOR) */
    int64_t steps;         /* steps taken since ek_init */
    double drift[3];       /* mean particle displacement since ek_init */
    double pmomentum[3];   /* total particle momentum */
    int32_t nonfinite;     /* 1 if a NaN or Inf was found in the populations or ions */
    int32_t negative_ions; /* number of sites with a negative ion density */
    double poisson_rel0;   /* relative residual of the starting guess of the last solve */
    double poisson_rel_max;/* largest relative residual reached by the step solves since the previous
                              ek_observables call (the tolerance is met when it is <= poisson_tol) */
} ek_obs;

/* Kernel classes timed when timing is on (ek_set_timing). */
#define EK_T_MOMENTS 0   /* moments, pseudopotentials, charge, permittivity, virtual densities */
#define EK_T_POISSON 1   /* all Poisson sweeps, residuals and reductions of a solve */
#define EK_T_FORCE 2     /* total force and physical velocity pass */
#define EK_T_FUSED 3     /* fused ion update + force + collide + stream pass */
#define EK_T_PARTICLE 4  /* particle force sums and integration */
#define EK_T_ITER 5      /* Poisson iterations: SOR sweep chunks (count = sweeps) or V-cycles (count = cycles) */
#define EK_T_SMOOTH 6    /* red-black colour passes on the lattice itself (SOR or multigrid smoothing): one event
                            pair per group of back-to-back passes, count = passes */
#define EK_T_COUNT 7

/* Single kernels timed at timing level 3 (ek_kernel_name gives each one's name). */
#define EK_K_MOMENTS 0
#define EK_K_VIRTUAL 1
#define EK_K_SOURCE_MEAN 2
#define EK_K_EXTRAPOLATE 3
#define EK_K_RESIDUAL 4
#define EK_K_REDUCE 5
#define EK_K_COARSEN 6           /* coarse-grid face coefficients, every level */
#define EK_K_SOR 7               /* red-black colour pass on the lattice */
#define EK_K_SOR_BLACK_FROM 8    /* black pass after the fused interpolation + red pass */
#define EK_K_RESTRICT_FINE 9
#define EK_K_RESTRICT 10
#define EK_K_SMOOTH 11           /* colour pass on a launched coarse grid */
#define EK_K_TAIL 12             /* single-workgroup solve of the two smallest grids */
#define EK_K_PROLONG_RED_FINE 13
#define EK_K_PROLONG_FINE 14
#define EK_K_PROLONG 15
#define EK_K_FINALIZE 16
#define EK_K_FORCE 17
#define EK_K_FUSED 18
#define EK_K_PARTICLE 19         /* particle forces and integration */
#define EK_K_LAGGED 20           /* a whole lagged Fourier solve (right-hand side, transforms, division) */
#define EK_K_REPROJECT 21        /* projection of moving particles after their step (reproject) */
#define EK_K_SOR_RB 22           /* one whole red-black lattice sweep in one pass (colour-split solves) */
#define EK_K_COUNT 23

typedef struct ek_timing {
    double ms[EK_T_COUNT];    /* summed device time per class (HIP events) */
    int64_t count[EK_T_COUNT];/* launches (or solves for EK_T_POISSON) per class */
    double kernel_ms[EK_K_COUNT];      /* timing level 3: summed device time per kernel */
    int64_t kernel_count[EK_K_COUNT];  /* timing level 3: launches per kernel */
} ek_timing;

/* Name of kernel id k (EK_K_*), "" for other k.  Host-only. */
const char* ek_kernel_name(int32_t k);

/* Field ids for ek_get_field (one double per site, x fastest). */
#define EK_F_RHO_A 0
#define EK_F_RHO_B 1
#define EK_F_N_PLUS 2
#define EK_F_N_MINUS 3
#define EK_F_PHI 4
#define EK_F_UX 5     /* pre-force barycentric velocity */
#define EK_F_UY 6
#define EK_F_UZ 7
#define EK_F_Q 8      /* charge density of the current state */
#define EK_F_EPS 9    /* permittivity of the current state */
#define EK_F_PSI_S 10 /* solid fraction */
#define EK_F_SOLID 11 /* 1 on LB-solid sites */
#define EK_F_EX 12    /* field E = -grad phi + E_ext of the current potential */
#define EK_F_EY 13
#define EK_F_EZ 14

/* Minimum-image separation along a periodic axis of n sites (the particle geometry's
   helper): d minus the whole periods n that bring it into [-n/2, n/2], taken off at once,
   so that a non-finite d gives NaN.  Host-only, needs no GPU; NaN for n <= 0. */
double ek_min_image(double d, int32_t n);

/* D3Q19 velocity set used by ek_get_populations: c[19][3] and weights w[19]
   (Sec. II A, weights 1/3, 1/18, 1/36).  Returns 19. */
int32_t ek_lattice(int32_t* c, double* w);

/* Create a context and set up the initial state (Sec. II A-E):
   - marks LB-solid sites (site centre strictly inside a sphere) and wall layers,
     counts the solid fraction psi_s by sub-cell centres, spreads each particle's
     charge in proportion to psi_s so that it sums to Q exactly, and builds the
     bounce-back link lists;
   - populations f = f~(rho^s, u = 0) on fluid sites;
   - ion densities n+- = n_plus, n_minus scaled by the fluid fraction 1 - psi_s;
   - the initial potential by a Poisson solve from zero.
   rho_a, rho_b, n_plus, n_minus: host arrays of nx*ny*nz doubles (required).
   parts: host array of n_parts particles (may be NULL when n_parts == 0).
   stream: a hipStream_t (NULL for the null stream).
   Errors: EK_EINVAL (bad sizes, tau <= 1/2, odd nx, non-positive fluid density,
   overlapping particles), EK_ENOMEM, EK_EHIP, EK_ENOCONV (initial solve).  On failure
   *out still holds a context for ek_last_error; release it with ek_destroy. */
ek_status ek_init(const ek_params* p, const double* rho_a, const double* rho_b, const double* n_plus,
                  const double* n_minus, const ek_particle* parts, int32_t n_parts, void* stream,
                  struct ek_ctx** out);

/* Device memory that ek_init_ws needs for these parameters and particles (a pure host
   computation: the particle geometry is built on the host to count boundary links; no
   device call).  The layout is that of ek_init: populations, ions, moments, potentials,
   multigrid levels, geometry and reduction scratch.  Errors: those of ek_init's argument
   checks; EK_EINVAL for EK_POISSON_FFT (hipFFT plans hold a work area of their own). */
ek_status ek_workspace_bytes(const ek_params* p, const ek_particle* parts, int32_t n_parts, size_t* bytes);

/* As ek_init, but every device buffer of the context is carved from `workspace`, a device
   allocation of ws_bytes >= ek_workspace_bytes(...) bytes owned by the caller (e.g. a torch
   uint8 tensor), which must outlive the context; the library allocates no device memory for
   it.  Buffers created by later calls (ek_forward_ckpt / ek_adjoint checkpoints, the
   autotuner's state copy, a moment-state population export) still come from hipMalloc.
   Errors: as ek_init; EK_ENOMEM if the workspace is too small; EK_EINVAL for a null
   workspace or EK_POISSON_FFT. */
ek_status ek_init_ws(const ek_params* p, const double* rho_a, const double* rho_b, const double* n_plus,
                     const double* n_minus, const ek_particle* parts, int32_t n_parts, void* workspace,
                     size_t ws_bytes, void* stream, struct ek_ctx** out);

/* Advance nsteps full steps of the coupled method, every stage reading the state at time t
   (Sec. II; the paper gives no order within a step): moments, pseudopotentials and virtual
   densities (Sec. II A, II C, II E), charge and permittivity (eq. electric_potential, eq.
   dielectric_constant), the Poisson solve (Sec. II D), the link fluxes and the ion update
   (eq. nernst-planck-disc, eq. ionic-fluxes-disc-2), the Shan-Chen, solvation, friction and
   Kelvin forces (eqs. shanChenForce, frictionforce, kelvin), the BGK collision with the
   velocity shift (eq. BoltzmannBGKLattice), streaming with halfway bounce-back and momentum
   exchange, and the particle update (Sec. II E).  Each solve starts from the potential
   extrapolated in time as ek_params.phi_history says (default: adaptive, the order 2 or 3
   whose last start residual was smaller).  Work is enqueued on the context's stream.  With
   poisson_cycles = 0 the Poisson convergence test reads residuals back to the host; with
   poisson_cycles > 0 nothing is read back and the call returns without waiting.  Returns
   EK_ENOCONV if a solve stopped at maxit (the step is still taken with the last iterate). */
ek_status ek_step(struct ek_ctx* ctx, int32_t nsteps);

/* Solve the Poisson equation for the charge and permittivity of the current state
   (Sec. II D): sum over the six links of eps_face (phi_j - phi_i) = -(q_i + wall
   charge), eps_face the mean of the two sites, source projected to zero mean, gauge
   mean(phi) = 0, starting from the current potential with the context's solver
   (multigrid V-cycles or red-black SOR; a lattice with an odd periodic y or z axis has no
   red-black colouring, and its SOR sweeps take three colours).  iters, rel_res may be
   NULL.  Returns EK_ENOCONV if the tolerance was not met (phi keeps the last iterate).
   Multigrid solves of a context's own potential work on colour-split copies of the
   potential and charge; with EK_POISSON_SITE_ORDER=1 in the environment at ek_init the
   context keeps them in site order instead (a diagnostic: the results are bit-identical). */
ek_status ek_poisson(struct ek_ctx* ctx, double tol, int32_t maxit, int32_t* iters, double* rel_res);

/* Change the external field E_ext (3 doubles, lattice units) of a running context; it takes
   effect from the next step.  The paper's drop experiments relax the fluid without a field
   and then apply one, and let a deformed drop relax back after switching it off (Sec. III B);
   restarting a context from its densities instead would reset the populations to
   equilibrium.  The next Poisson solve starts from the potentials of the old field.  Reverse-
   mode checkpoints taken before the change are dropped.  Errors: EK_ESTATE (no context, or
   a replica of a batch), EK_EINVAL (null or non-finite field; a polarising field normal to
   walls). */
ek_status ek_set_field(struct ek_ctx* ctx, const double* E_ext);

/* Shape of the multigrid V-cycle (contexts whose lattice the multigrid coarsens): red-black
   Gauss-Seidel sweeps before and after the coarse-grid correction on the lattice itself
   (fine_pre, fine_post), on the coarse grids smoothed by separate launches (coarse_pre,
   coarse_post) and on the upper grid of the last two, which one workgroup handles in LDS
   (tail_pre, tail_post); red-black SOR sweeps on the coarsest grid; omega relaxes the
   smoothing sweeps (1 is Gauss-Seidel).  Defaults 1, 2, 1, 2, 3, 3, 10, 1.2.  Counts in
   0..64, omega in (0, 2); the lattice needs at least one sweep per cycle.  The solve still
   runs to the Poisson tolerance; the shape only trades work per cycle against cycles.
   Errors: EK_EINVAL, EK_ESTATE. */
ek_status ek_set_multigrid(struct ek_ctx* ctx, int32_t fine_pre, int32_t fine_post, int32_t coarse_pre,
                           int32_t coarse_post, int32_t tail_pre, int32_t tail_post, int32_t coarsest_sweeps,
                           double omega);

/* Candidate V-cycle shapes of ek_autotune_multigrid, the default first: writes, if not
   NULL, 7 counts per candidate to shapes (the first seven arguments of ek_set_multigrid
   after the context, in order) and its omega to omegas.  Returns the number of candidates
   (at most 16).  Needs no context or GPU. */
int32_t ek_autotune_candidates(int32_t* shapes, double* omegas);

/* Pick the V-cycle shape that steps this context fastest.  From the current state every
   candidate runs one untimed step (which captures its cycle graph and estimates its
   convergence rate), then trial_steps timed steps (HIP events on the context's stream),
   each time from the same saved copy of the state, in two rounds over the candidates
   (each candidate's faster round counts).  The state (populations, ions, potential and
   its two predecessors, particles, step counters, warm-start bookkeeping) is restored
   afterwards and the fastest shape set as by ek_set_multigrid; a candidate earlier in
   the list (the default first) within 1 % of the fastest is preferred to it.  A step runs a
   whole number of V-cycles, so a window of a few steps can favour a shape that happens
   to save a cycle on those steps; about 100 trial steps follow the long-run rate.  best (host, may be NULL) receives its index in the
   ek_autotune_candidates order, ms_per_step (host, may be NULL, room for every candidate)
   each candidate's mean milliseconds per step.  Device memory: a copy of the state
   (about (2 x 19 + 2) N element sizes + 24 N bytes), held only during the call.  The Poisson
   tolerance of the context applies; a solve that stops at maxit counts with its time.
   Synchronises.  Errors: EK_EINVAL (trial_steps outside 1..1000, a context solved by SOR),
   EK_ESTATE (replica of a batch), EK_ENOMEM, EK_EHIP; on an error the shape in place
   before the call is kept. */
ek_status ek_autotune_multigrid(struct ek_ctx* ctx, int32_t trial_steps, int32_t* best, double* ms_per_step);

/* FP64 totals and diagnostics of the current state (synchronises the stream): the
   conserved sums of the method (fluid masses, ion numbers, charge, with the colloid charge
   of Sec. II E; momentum), the largest velocity, the Poisson diagnostics of the last solves
   and the mean particle drift.  The totals are sums in a fixed order, so they are
   deterministic.  field_mask selects fields (bit k = field id k of ek_get_field, k <=
   EK_F_EZ) that are also copied to host_fields, n_fields x nx*ny*nz doubles in increasing id
   order; host_fields may be NULL when field_mask is 0.  Returns EK_ENONFINITE if populations
   or ion densities hold a NaN or Inf (out and the fields are still written), EK_EINVAL for
   mask bits beyond EK_F_EZ or a null host_fields. */
ek_status ek_observables(struct ek_ctx* ctx, ek_obs* out, uint32_t field_mask, double* host_fields);

/* For callers that cannot allocate device memory or wait for the device (work captured in
   a HIP graph, serving loops): the totals of ek_observables written to device memory,
   enqueued on the context's stream without any host synchronisation or allocation.  d_out:
   device pointer to 11 doubles: sum rho_a, sum rho_b (fluid sites), sum n+, sum n-, sum q,
   momentum x, y, z, max |u|, count of non-finite values, count of negative ion densities.
   The per-workgroup partial sums go to a file-scope device array of the library (128 KiB on
   each GPU, held until the process ends; a fixed grid of at most 1024 workgroups strides over
   any lattice size, so the partials use at most 88 KiB of it) instead of the context's
   buffers.  The summation order differs from ek_observables' (the same values to FP64
   rounding).  All calls on one GPU share that array: calls that may overlap (several
   streams or threads) race and must be serialised by the caller.  Errors: EK_ESTATE,
   EK_EINVAL (null d_out), EK_EHIP. */
ek_status ek_observables_device(struct ek_ctx* ctx, double* d_out);

/* Copy one field of the current state to host memory (nx*ny*nz doubles): the fluid and ion
   densities, potential, pre-force velocity (Sec. II A-D), charge and permittivity (eqs.
   electric_potential, dielectric_constant), solid fraction and mask (Sec. II E) or the field
   E = -grad phi + E_ext.  Synchronises. */
ek_status ek_get_field(struct ek_ctx* ctx, int32_t field, double* host_out);

/* (Sec. II A) Copy the populations of component comp (0 = a, 1 = b) to host memory as
   19 * nx*ny*nz doubles, velocity-major in the order of ek_lattice.  FP32 contexts
   return f = deviation + w_d rho_ref. */
ek_status ek_get_populations(struct ek_ctx* ctx, int32_t comp, double* host_out);

/* Copy the particles to host memory as n_parts x 9 doubles: x(3), v(3) and the
   force F(3) of the last step (Sec. II E: momentum exchange, q_c E, Hertz, lubrication). */
ek_status ek_get_particles(struct ek_ctx* ctx, double* host_out);

/* Device bytes held by the context. */
ek_status ek_device_bytes(const struct ek_ctx* ctx, size_t* bytes);

/* Per-kernel HIP event timing: 0 off, 1 kernel classes (a few events per step),
   2 classes plus the lattice-level red-black passes (EK_T_SMOOTH, one event pair per
   group of back-to-back passes; it adds events between small kernels and launches
   the multigrid cycle without its graph, so use it for per-launch figures, not for
   step rates), 3 an event pair around every kernel launch of a step (EK_K_*, in
   kernel_ms / kernel_count; classes are not timed then; the cycle runs without its graph).
   Any call clears the accumulated times. */
ek_status ek_set_timing(struct ek_ctx* ctx, int32_t enable);

/* Accumulated times since timing was turned on (synchronises the stream). */
ek_status ek_get_timing(struct ek_ctx* ctx, ek_timing* out);

/* Release the context and its device memory (synchronises the stream). */
ek_status ek_destroy(struct ek_ctx* ctx);

const char* ek_status_str(ek_status s);
const char* ek_last_error(const struct ek_ctx* ctx);

/* ---------------------------------------------------------------------------------
 * Reverse mode: gradients of a scalar objective L of the state after T steps, with
 * respect to the state before them and to the external field, the two fluid
 * permittivities and the Shan-Chen coupling (Sec. II A-D).  The adjoint is the exact
 * transpose of the discrete step (streaming, collision with the velocity shift, the
 * Shan-Chen, ion-solvation, friction and Kelvin forces, the link fluxes with donor-cell
 * advection, the central-difference field and the Poisson equation, whose potential is
 * the implicit solution: its adjoint is one more solve with the same symmetric operator).
 * Periodic lattices without particles only (EK_EINVAL otherwise).  The transposed
 * passes are FP64.  An FP32 context runs its own forward steps; its checkpoints are its
 * states widened to FP64 in an FP64 twin context (built from the same parameters and
 * fields at each ek_forward_ckpt, same stream), which recomputes every segment in FP64
 * and reverses it: the gradient of the FP64 step linearised along segments restarted
 * from the FP32 trajectory.  The twin is held until the next ek_forward_ckpt or
 * ek_destroy and adds an FP64 context's memory.
 * --------------------------------------------------------------------------------- */

/* Advance nsteps steps (as ek_step) keeping a device checkpoint of the state every
   `every` steps and at the end, for a later ek_adjoint; replaces the checkpoints of any
   earlier call.  Device memory: (nsteps / every + 2) x 43 N doubles.
   Errors: EK_EINVAL (bad counts, unsupported context), EK_ENOMEM, EK_ENOCONV as ek_step. */
ek_status ek_forward_ckpt(struct ek_ctx* ctx, int32_t nsteps, int32_t every);

/* Reverse the last ek_forward_ckpt run.  Inputs (device pointers, FP64, read only):
     adj_f  2 x 19 x N: dL/df of components a then b at the end of the run, each
            velocity-major in the ek_lattice order, x fastest
     adj_n  2 x N: dL/dn+ then dL/dn- at the end of the run
   Outputs: grad (host, 6 doubles) = dL/d[E_ext x, E_ext y, E_ext z, eps_a, eps_b, G];
   adj_f0, adj_n0 (device, optional, NULL to skip): the same sensitivities for the
   state at the start of the run.  Each segment of `every` steps is recomputed from its
   checkpoint (device memory `every` x 41 N doubles) and reversed step by step; every
   reverse step solves the adjoint Poisson equation to the context's Poisson tolerance
   (same solver and V-cycle shape, started from the adjoint potentials of the previous
   reverse steps extrapolated in time).
   On return the context holds the state at the end of the run again (an FP32 context
   never leaves it: its FP64 twin does the recomputing).  Synchronises.
   Errors: EK_ESTATE (no checkpointed run), EK_EINVAL, EK_ENOMEM, EK_ENOCONV (an
   adjoint solve stopped at maxit; the gradient is still returned). */
ek_status ek_adjoint(struct ek_ctx* ctx, const double* adj_f, const double* adj_n, double* grad, double* adj_f0,
                     double* adj_n0);

/* ---------------------------------------------------------------------------------
 * Batched replicas: many independent lattices (a parameter sweep) advanced together,
 * one graph launch per step for all of them.  Every replica is a full context of the
 * method above (Sec. II), periodic, without particles, with a lattice the multigrid
 * can coarsen (every axis divisible by 4); all share one precision.  Each stage of a
 * step (moments, Poisson V-cycles per grid level, force pass, fused sweep) is a single
 * launch over the work of all replicas; the whole step is captured once into a HIP
 * graph (one per buffer parity), so a step is one host call and no host
 * synchronisation.  Each step runs exactly `cycles` multigrid V-cycles from the
 * extrapolated potential; the relative residual each replica reaches is recorded on
 * the device (ek_batch_residuals) instead of steering the step.
 * The batch owns a HIP stream of its own (default priority); calls that return data
 * synchronise it.
 * --------------------------------------------------------------------------------- */
struct ek_batch;

/* params, rho_a, rho_b, n_plus, n_minus: arrays of n_rep entries (host, borrowed for the
   call; field arrays as in ek_init).  cycles: V-cycles per step (1..64).
   Errors: EK_EINVAL (walls, mixed precision, lattice not coarsenable, bad cycles), or
   any ek_init error of a replica (message names the replica).  On failure *out still
   holds a batch for ek_batch_last_error; release it with ek_batch_destroy. */
ek_status ek_batch_init(const ek_params* params, int32_t n_rep, const double* const* rho_a,
                        const double* const* rho_b, const double* const* n_plus, const double* const* n_minus,
                        int32_t cycles, struct ek_batch** out);

/* Enqueue nsteps steps of every replica (one graph launch each); returns without waiting. */
ek_status ek_batch_step(struct ek_batch* b, int32_t nsteps);

/* Wait for the batch's stream. */
ek_status ek_batch_sync(struct ek_batch* b);

/* Relative Poisson residual of every replica after the last step (last) and the largest
   over the steps since the previous call (worst; the running maximum restarts with each
   call); either may be NULL.  Synchronises. */
ek_status ek_batch_residuals(struct ek_batch* b, double* last, double* worst);

/* Borrow replica r's context for the export calls (ek_get_field, ek_get_populations,
   ek_observables).  It stays owned by the batch: ek_step, ek_poisson and ek_destroy
   return EK_ESTATE on it. */
ek_status ek_batch_replica(struct ek_batch* b, int32_t r, struct ek_ctx** ctx);

/* Set the batch's V-cycle shape (shape: the seven counts of ek_set_multigrid; omega its
   relaxation) and V-cycles per step (1..64), and capture its step graphs again.  The state
   is kept.  Errors: EK_EINVAL, EK_ESTATE, EK_EHIP. */
ek_status ek_batch_set_cycle(struct ek_batch* b, const int32_t* shape, double omega, int32_t cycles);

/* Autotuner of the batched launch (a project-written tuner, no paper counterpart): for
   every candidate shape of ek_autotune_candidates, the fewest V-cycles per step (up to 8)
   whose worst relative Poisson residual over trial_steps steps (1..1000) stays within
   max_residual, each timed with HIP events on the batch stream from the same saved state
   of every replica.  The fastest is applied (an earlier candidate within 1 % is preferred)
   and the state put back, so stepping continues from where it was.  best (optional): 8
   int32, the shape's seven counts and the cycles; omega, ms_per_step (optional): its
   relaxation and time per step of the whole batch.  Needs device memory for one copy of
   every replica's state while it runs.  Errors: EK_EINVAL, EK_ESTATE, EK_ENOMEM, EK_EHIP,
   EK_ENOCONV (no candidate met the bound; the previous shape and cycles stay). */
ek_status ek_batch_autotune(struct ek_batch* b, int32_t trial_steps, double max_residual, int32_t* best,
                            double* omega, double* ms_per_step);

/* Release the batch, its replicas and its stream. */
ek_status ek_batch_destroy(struct ek_batch* b);
const char* ek_batch_last_error(const struct ek_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* EK_H */
