// Internal declarations shared by the kernels (ek_kernels.hip) and the host runtime
// (ek_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ek {

constexpr int kBlock = 256;   // threads per site-kernel workgroup (4 wave64)
constexpr int kRedSlots = 12; // doubles per workgroup in reduction scratch
constexpr int kResSites = 4;   // sites per thread of the residual kernel

// Scalar parameters of a context, passed by value to every kernel.
struct Scalars {
    int nx, ny, nz;
    int nxy;
    unsigned N;
    int walls;        // solid layers at z = 0 and z = nz-1
    int colloids;     // per-site geometry arrays present
    int kelvin;       // eps_a != eps_b: Kelvin force active
    int ion_sc;       // solvation Shan-Chen coupling active
    int polar;        // the external field polarises the dielectric (Poisson source term)
    int z0, z1;       // Poisson domain in z (inclusive)
    unsigned ndomain; // sites in the Poisson domain
    int ncolor;       // colours of a lattice Gauss-Seidel sweep: 2, or 3 with an odd periodic y or z axis
    double inv_nx, inv_ny, inv_nxy, inv_hx;  // 1/nx, 1/ny, 1/(nx ny), 1/(nx/2): exact index division
    // Banded workgroup order of the stencil sweeps (site_banded): workgroups of one z-plane
    // (plane_blocks of them) are grouped in bands of `band`, and each XCD walks its slab of
    // slab_planes planes band by band; band = 0 keeps the plain slab order.
    int band, plane_blocks, slab_planes;
    // Moving particles projected anew every step (ek_params.reproject): sub-cells per axis
    // of the solid fraction, and the half-width and side of the box of sites around a
    // particle that a step's projection can change (rp_box = 2 rp_half + 1)
    int reproject, subs, rp_half, rp_box;
    double tau, inv_tau, G, rho0, D, beta;
    double kap_p, kap_m;   // s beta dmu+- / (2 drho_a)
    double G_p, G_m;       // s dmu+- / (drho_a c_s^2)
    double eps_a, eps_b, eps_p, eps_bar;
    double E_ext[3];
    double g_body[3];
    double sigma0, sigma1;
    double rref[2];        // deviation reference densities
};

// Device pointers of a context for one precision.
template <typename T>
struct Fields {
    const T* f[2];      // populations of a, b at time t (19 N each, velocity-major)
    T* fn[2];           // populations at t+1
    const T* n[2];      // ions at time t: [0] mean density (n+ + n-)/2, [1] ionic charge n+ - n-
    T* nn[2];           // the same at t+1
    T* mom;             // 8 N: rho_a - rho_ref_a, rho_b - rho_ref_b, psi_a, psi_b, chi_a, ux, uy, uz
    T* uph;             // 3 N: physical velocity
    T* q;               // charge density
    T* eps;             // permittivity
    double* phi;        // potential (double)
    const uint8_t* flags;    // bit0 solid, bit1 fluid next to a solid, bit2 solid next to fluid,
                             // bit3 the site or an axis neighbour partly covered
    const T* psif;           // fluid fraction
    const T* qc;             // particle charge per site
    const int32_t* owner;    // particle owning a site, -1 none
    const int32_t* linkbase; // first particle link of a fluid site
    double* linkdp;          // 6 doubles per particle link: (component, xyz) momentum handed over
    const int32_t* vlist;    // solid sites next to fluid (virtual densities)
    int nv;
    const int32_t* plist;    // sites that take the particle path (flag bits 0, 1 or 3), ascending; with
                             // moving particles rebuilt on the device after every projection, unordered
    int npl;                 // its length, or with npl_dev its capacity
    const int32_t* npl_dev;  // device-held length (moving particles), or null
    const double* pv;        // particle velocities (3 per particle)
    double* red;             // reduction scratch
    double* scal;            // device scalars: [0] source mean, [1..3] rr, ss, sum phi
    // tau = 1 moment state (null with population storage), site-major: site j's values at
    // ms + 8 j, component c at + 4 c: rho_c - rho_ref_c, then the equilibrium velocity u_e
    // (x, y, z) of the collision of step t - 1; msn receives those of step t
    const T* ms;
    T* msn;
    const double* rho0;      // initial densities (2 N, FP64): the populations w_d rho0 before the first step
    int ms_first;            // 1 until the first step has written a moment state
    // FP32 population contexts with the exact-mass collision (null otherwise): the low FP32
    // part of each site's rest population (2 N, a then b; the stored rest value is the high
    // part), and the part of each site's summed mass that the FP32 mass slot does not hold
    // (2 N), from the moments pass to the collision
    T* rlo;
    T* mlo;
};

// One coarse level of the Poisson multigrid: cell-centred, periodic in all axes, with
// the operator held as face coefficients (a zero face decouples two cells, which is how
// the wall layers enter the coarse levels).
struct MGLevel {
    int nx, ny, nz;
    unsigned n;
    double* phi;  // correction on this level
    double* s;    // restricted residual (right-hand side)
    double* ax;   // coefficient of the face to the +x neighbour
    double* ay;
    double* az;
    double inv_nx, inv_ny, inv_hx;  // 1/nx, 1/ny, 1/(nx/2) for div_exact
};

unsigned site_blocks(unsigned n);
unsigned residual_blocks(unsigned n);  // workgroups of the residual kernel for n sites

// Reverse-mode (adjoint) fields of a periodic FP64 context for one reverse step: the
// sensitivities of a scalar objective L to the step's inputs and intermediates.  All
// arrays are N-major doubles.
struct AdjFields {
    const double* lf[2];  // dL/df at t+1 of components a, b (19 N each, velocity-major)
    double* lfo[2];       // dL/df at t
    const double* ln[2];  // dL/dn+, dL/dn- at t+1
    double* lno[2];       // the same at t
    double* aS;           // 6 N: dL/d(sum_d w_d chi_a(i+d) c_d), dL/d(sum_d w_d psi_a(i+d) c_d)
    double* aF;           // 3 N: dL/d(non-Shan-Chen force: friction + Kelvin + body)
    double* aE;           // 3 N: dL/dE
    double* arho;         // 2 N: dL/drho^a, dL/drho^b (partial sums)
    double* au;           // 3 N: dL/du' (pre-force velocity)
    double* an;           // 2 N: dL/dn+, dL/dn- at t (partial sums)
    double* aeps;         // N: dL/deps (partial sum)
    double* rhs;          // N: dL/dphi, the right-hand side of the adjoint Poisson equation
    const double* mu;     // N: adjoint potential, M mu = dL/dphi projected to zero mean
    double* gred;         // kRedSlots doubles per workgroup: parameter-gradient partials
};

// Slots of AdjFields::gred: dL/dE_ext (x, y, z), dL/deps_a and dL/deps_b through the site
// permittivity, dL/d(eps_bar) of the Kelvin force, dL/dG.
constexpr int kAdjEx = 0, kAdjEa = 3, kAdjEb = 4, kAdjEbar = 5, kAdjG = 6, kAdjSlots = 7;

// Batched replicas: per-replica descriptors in device memory and block tables mapping
// each workgroup of a batched launch to (replica, workgroup within the replica).
constexpr int kMaxLevels = 8;

template <typename T>
struct RepDesc {
    Scalars S;
    Fields<T> F;
    double* phi_prev;
    MGLevel mg[kMaxLevels];  // grid g >= 1 is mg[g - 1]
    int nl;                  // number of coarse grids
    int tail_mid;            // the tail kernel also handles grid nl - 1 (mg[nl - 2])
    int coarse_iters;
    double coarse_omega;
    int mid_pre, mid_post;  // sweeps of the tail kernel's upper grid
    double smooth_omega;    // relaxation of the smoothing sweeps
};

struct BlockRef {
    int rep;
    int blk;
};

enum BatchOp {
    kB_MOMENTS, kB_EXTRAPOLATE, kB_RESIDUAL, kB_FINALIZE, kB_FORCE, kB_FUSED, kB_PROLONG_FINE,  // site tables
    kB_SOR,                                                                                    // colour table
    kB_COARSEN_FINE, kB_COARSEN, kB_RESTRICT_FINE, kB_RESTRICT, kB_SMOOTH, kB_PROLONG            // level tables
};

template <typename T>
void launch_batch(BatchOp op, const RepDesc<T>* D, const BlockRef* tab, unsigned nblocks, int grid, int color,
                  hipStream_t st);
template <typename T> void launch_batch_source_mean(const RepDesc<T>* D, int n_rep, hipStream_t st);
template <typename T> void launch_batch_reduce(const RepDesc<T>* D, int n_rep, hipStream_t st);
template <typename T> void launch_batch_tail(const RepDesc<T>* D, int n_rep, hipStream_t st);

template <typename T> void launch_mg_coarsen_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, hipStream_t st);
void launch_mg_coarsen(const MGLevel& f, const MGLevel& c, hipStream_t st);
void launch_mg_smooth(const MGLevel& L, int color, double omega, hipStream_t st);
template <typename T>
void launch_mg_restrict_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, bool split, double red_omega,
                             hipStream_t st);
// red_omega > 0: the restriction also takes the first red pass of the coarse pre-smoothing
void launch_mg_restrict(const MGLevel& f, const MGLevel& c, double red_omega, hipStream_t st);
template <typename T>
void launch_mg_prolong_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, bool split, hipStream_t st);
// Colour-split fields: interpolation onto the lattice with the first red pass of the
// post-smoothing; the interpolated black values go to blk (N/2 doubles), which the black
// pass launch_sor_black_from reads as the black sites' current values.
template <typename T>
void launch_mg_prolong_red_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, double omega, double* blk,
                                hipStream_t st);
template <typename T>
void launch_sor_black_from(const Scalars& S, const Fields<T>& F, double omega, const double* blk, hipStream_t st);
// One whole red-black sweep in one pass, colour-split fields from pin to pout (F.phi is not
// read); only where sor_rb_fits(S).
bool sor_rb_fits(const Scalars& S);
template <typename T>
void launch_sor_rb(const Scalars& S, const Fields<T>& F, const double* pin, double* pout, double omega,
                   hipStream_t st);
void launch_mg_prolong(const MGLevel& c, const MGLevel& f, hipStream_t st);
void launch_mg_tail(const MGLevel& mid, const MGLevel& coarse, int has_mid, int iters, double omega, int mid_pre,
                    int mid_post, double mid_omega, hipStream_t st);

template <typename T> void launch_moments(const Scalars& S, const Fields<T>& F, unsigned nblk, hipStream_t st);
template <typename T> void launch_virtual(const Scalars& S, const Fields<T>& F, hipStream_t st);
void launch_source_mean(const Scalars& S, double* red, unsigned nblk, double* scal, hipStream_t st);
// split: F.phi and F.q hold the colour-split potential and charge (multigrid contexts)
template <typename T>
void launch_sor(const Scalars& S, const Fields<T>& F, int color, double omega, bool split, hipStream_t st);
// From site-order fields (split false) with phis, qs non-null: also writes their colour-split copies
template <typename T>
void launch_residual(const Scalars& S, const Fields<T>& F, unsigned nblk, bool split, double* phis, T* qs,
                     hipStream_t st);
void launch_reduce(const double* red, unsigned nblk, int nvals, const int* is_max, double* out, hipStream_t st);
// gauge mean(phi) = 0 (phi = 0 when zero != 0) and the wall layers of the potential
// split_src: the colour-split solved potential, or null to gauge F.phi in place
template <typename T>
void launch_phi_finalize(const Scalars& S, const Fields<T>& F, int zero, const double* split_src, hipStream_t st);
void launch_phi_extrapolate(const Scalars& S, double* phi, double* prev, double* prev2, int history,
                            hipStream_t st);
template <typename T> void launch_force(const Scalars& S, const Fields<T>& F, hipStream_t st);
template <typename T> void launch_fused(const Scalars& S, const Fields<T>& F, hipStream_t st);
// lagged Fourier Poisson scheme (ek_fft.hip): right-hand side r from the potential held,
// and the spectral division of the forward transform (nz, ny, nx/2+1 complex doubles)
template <typename T> void launch_lag_rhs(const Scalars& S, const Fields<T>& F, double* rhs, hipStream_t st);
void launch_lag_table(double* tab, int nx, int ny, int nz, hipStream_t st);  // nx/2+1+ny+nz doubles
void launch_lag_scale(double* spec, const double* tab, int nx, int ny, int nz, hipStream_t st);
// populations of component c at time t of a moment-state context (FP64, 19 N, f not g)
template <typename T> void launch_export_pop(const Scalars& S, const Fields<T>& F, int c, double* out, hipStream_t st);
// one workgroup per particle: link momenta, q_c E over its sites, Hertz and lubrication
// against every other particle, then symplectic Euler into xn, vn (pF receives the force)
template <typename T>
void launch_particle_step(const Scalars& S, const Fields<T>& F, int np, const int32_t* link_off,
                          const int32_t* link_idx, const int32_t* site_off, const int32_t* site_idx, const double* x,
                          const double* v, const double* r, double* pF, double* xn, double* vn, double rho_p,
                          double k_h, double eta, int move, hipStream_t st);
template <typename T> void launch_observe(const Scalars& S, const Fields<T>& F, unsigned nblk, hipStream_t st);

// Projection of moving particles after their step (ek_params.reproject).  Work arrays: the
// geometry of the step's start (flags, owner, fluid fraction), per particle and box site
// the sub-cell count and centre test of the new position and the site's conversion, per
// site the ion shares of a site whose fluid fraction drops to zero, per particle the box
// origin and the summed solid fraction.
template <typename T>
struct Reproj {
    int np;
    const double* x;     // positions after the step (3 np)
    double* v;           // velocities after the step (3 np); the conversions' impulses are added
    const double* rad;   // radii
    const double* Q;     // charges
    double rho_p;        // particle mass density
    uint8_t* flags;      // the context's geometry, updated in place
    int32_t* owner;
    T* psif;
    T* qc;
    const uint8_t* flags_old;  // copies taken before the projection
    const int32_t* owner_old;
    const T* psif_old;
    int32_t* origin;     // 3 np: lowest lattice corner of each particle's box (not wrapped)
    int16_t* cnt;        // np x box^3: sub-cells of the site inside the particle
    uint8_t* inside;     // np x box^3: the site's centre strictly inside the particle
    uint8_t* event;      // np x box^3: 1 covered, 2 uncovered (for the particle handling it)
    double* evm;         // 3 x np x box^3: the particle's momentum change from that site
    T* share;            // 2 N: ion shares (mean density, charge) of a site losing its fluid
    double* ptot;        // np: summed solid fraction of each particle's sites
    int32_t* nb;         // np x np: per particle, the particles whose boxes meet its box, ascending (itself included)
    int32_t* nnb;        // np: how many
    int32_t* plist;      // the context's particle-path list, rebuilt from the boxes
    int32_t* npl;        // its length (device)
};
template <typename T>
void launch_reproject(const Scalars& S, const Fields<T>& F, const Reproj<T>& P, hipStream_t st);
// the observables from a fixed grid of nblk workgroups (grid-stride), partial sums in red
template <typename T>
void launch_observe_strided(const Scalars& S, const Fields<T>& F, unsigned nblk, double* red, hipStream_t st);
// device-side relative residuals of a solve without host read-back (scal[28..30])
void launch_track_residual(double* scal, hipStream_t st);
template <typename T>
void launch_init_pop_flags(const Scalars& S, T* f, const double* rho, double rref, const uint8_t* flags, hipStream_t st);
template <typename T>
void launch_init_ions(const Scalars& S, const Fields<T>& F, T* ion_s, T* ion_c, const double* np_, const double* nm_,
                      hipStream_t st);
template <typename T>
void launch_ion_species(const T* ion_s, const T* ion_c, double* dst, unsigned n, double sign, hipStream_t st);
template <typename T> void launch_to_double(const T* src, double* dst, unsigned n, double add, hipStream_t st);
template <typename T> void launch_add_lo(const T* lo, double* dst, unsigned n, hipStream_t st);
template <typename T> void launch_field_e(const Scalars& S, const Fields<T>& F, int k, double* dst, hipStream_t st);
template <typename T> void launch_upload(T* dst, const double* src, unsigned n, hipStream_t st);

void launch_adj_force(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st);
void launch_adj_links(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st);
void launch_adj_rhs(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st);
void launch_adj_final(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st);

}  // namespace ek
