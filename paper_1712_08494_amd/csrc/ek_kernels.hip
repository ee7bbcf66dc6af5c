// HIP kernels (gfx950 / CDNA4) of the coupled electrokinetic lattice step.
//
// One step (Rivas et al., arXiv:1712.08494, Sec. II), all stages reading time-t fields:
//   k_moments  : rho^s, pre-force velocity, Shan-Chen pseudopotentials, charge and
//                permittivity; FP64 partial sums of the charge          (Sec. II A-C, II E)
//   k_virtual  : virtual fluid densities on solid sites next to fluid    (Sec. II E)
//   k_sor      : red-black over-relaxed sweeps of the variable-eps Poisson equation
//   k_residual : FP64 residual / source / potential sums                 (Sec. II D)
//   k_force    : total force and physical velocity u = u' + sum Phi / 2 rho
//   k_fused    : link-flux Nernst-Planck update of both ion species, Shan-Chen +
//                friction + Kelvin forces, BGK collide with velocity shift, push
//                streaming with halfway bounce-back and momentum exchange
//                                                                      (Sec. II A-C, II E)
//   k_particle_*: particle force sums and integration                    (Sec. II E)
//
// Everything here is HBM-bandwidth bound stencil work: no MFMA.  Site kernels map one
// thread to one site (x fastest, coalesced SoA access) and remap workgroups so that each
// of the eight XCDs sweeps a contiguous slab of the lattice (its z-neighbour planes stay
// in that XCD's L2).  Reductions are wave64 shuffles + LDS + a fixed-order final pass,
// so results are deterministic run to run.
#include "ek_device.h"

namespace ek {

// ------------------------------------------------------------------------------------
// Indexing helpers
// ------------------------------------------------------------------------------------
unsigned site_blocks(unsigned n) {
    unsigned b = (n + kBlock - 1) / kBlock;
    return (b + 7u) & ~7u;  // a multiple of the 8 XCDs, see xcd_linear()
}

// Geometry modes, a template parameter of the site kernels so that unused cases cost
// nothing: kPeriodic (no solid site), kWalls (wall layers only, decided by z),
// kColloids (per-site flags and fluid fractions; wall layers are marked there too).
constexpr int kPeriodic = 0, kWalls = 1, kColloids = 2;

template <typename T, int G>
__device__ __forceinline__ bool is_solid(unsigned j, int zj, const Scalars& S, const Fields<T>& F) {
    if (G == kPeriodic) return false;
    if (G == kWalls) return zj == 0 || zj == S.nz - 1;
    return (F.flags[j] & 1u) != 0;
}

template <typename T, int G>
__device__ __forceinline__ T fluid_fraction(unsigned j, int zj, const Scalars& S, const Fields<T>& F) {
    if (G == kPeriodic) return T(1);
    if (G == kWalls) return (zj == 0 || zj == S.nz - 1) ? T(0) : T(1);
    return F.psif[j];
}

// run-time dispatch helpers (used outside the hot kernels)
template <typename T>
__device__ __forceinline__ bool solid_at(unsigned j, int zj, const Scalars& S, const Fields<T>& F) {
    return S.colloids ? (F.flags[j] & 1u) != 0 : wall_layer(zj, S);
}

template <typename T>
__device__ __forceinline__ T psif_at(unsigned j, int zj, const Scalars& S, const Fields<T>& F) {
    return S.colloids ? F.psif[j] : (wall_layer(zj, S) ? T(0) : T(1));
}

template <typename T> __device__ __forceinline__ T expm1T(T v);
template <> __device__ __forceinline__ float expm1T<float>(float v) { return expm1f(v); }
template <> __device__ __forceinline__ double expm1T<double>(double v) { return expm1(v); }

template <typename T> __device__ __forceinline__ T pseudo(T rho, const Scalars& S) {
    // psi = rho0 (1 - exp(-rho / rho0)), Sec. II C, written as -rho0 expm1(-rho / rho0): in
    // the minority phase (rho ~ 0.01) the difference 1 - exp(...) would lose about two of
    // FP32's seven digits.
    const T r0 = T(S.rho0);
    return -r0 * expm1T<T>(-rho / r0);
}

// Fluid permittivity (eq. dielectric_constant) mixed with the particle permittivity
// by the solid fraction (Sec. II E).
template <typename T> __device__ __forceinline__ T eps_fluid(T ra, T rb, const Scalars& S) {
    const T rt = ra + rb;
    const T c = rt > T(0) ? (rb - ra) / rt : T(0);
    return T(0.5) * (T(S.eps_a) * (T(1) - c) + T(S.eps_b) * (T(1) + c));
}

// Sums (or maxima) of nvals values over nblk partial records, fixed order: deterministic.
constexpr int kRedThreads = 1024;

// Each thread accumulates whole records (value k of record b at red[k * nblk + b]; a few
// records are in flight at once) in increasing record order; wave64 shuffles and a sum
// over the waves in order finish the job.  Fixed order throughout: deterministic.  NV is
// the number of values read (at least nvals).
template <int NV, int kFly>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ red, unsigned nblk, int nvals,
                                                        const int* is_max_d, double* __restrict__ out) {
    __shared__ double sm[NV][kRedThreads / 64];
    bool mx[NV];
    double a[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        mx[k] = k < nvals && is_max_d ? is_max_d[k] != 0 : false;
        a[k] = mx[k] ? -1e300 : 0.0;
    }
    for (unsigned b0 = threadIdx.x; b0 < nblk; b0 += kFly * kRedThreads) {
        double v[kFly][NV];
#pragma unroll
        for (int j = 0; j < kFly; ++j) {
            const unsigned b = b0 + j * kRedThreads;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                v[j][k] = (k < nvals && b < nblk) ? red[(size_t)k * nblk + b] : (mx[k] ? -1e300 : 0.0);
        }
#pragma unroll
        for (int j = 0; j < kFly; ++j)
#pragma unroll
            for (int k = 0; k < NV; ++k) a[k] = mx[k] ? fmax(a[k], v[j][k]) : a[k] + v[j][k];
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double v = a[k];
#pragma unroll
        for (int s2 = 32; s2 > 0; s2 >>= 1) {
            const double o = __shfl_down(v, s2, 64);
            v = mx[k] ? fmax(v, o) : v + o;
        }
        if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nvals) {
        const int k = threadIdx.x;
        double v = sm[k][0];
        const bool m = is_max_d ? is_max_d[k] != 0 : false;
        for (int w = 1; w < kRedThreads / 64; ++w) v = m ? fmax(v, sm[k][w]) : v + sm[k][w];
        out[k] = v;
    }
}

void launch_reduce(const double* red, unsigned nblk, int nvals, const int* is_max, double* out, hipStream_t st) {
    if (nvals <= 3)
        hipLaunchKernelGGL((k_reduce<3, 4>), dim3(1), dim3(kRedThreads), 0, st, red, nblk, nvals, is_max, out);
    else
        hipLaunchKernelGGL((k_reduce<kRedSlots, 2>), dim3(1), dim3(kRedThreads), 0, st, red, nblk, nvals, is_max,
                           out);
}

// ------------------------------------------------------------------------------------
// Step 1: moments, pseudopotentials, charge and permittivity.
// Populations are stored as deviations g_d = f_d - w_d rho_ref (both precisions), so
//   rho = rho_ref + sum_d g_d,  rho u = sum_d g_d c_d   (sum_d w_d c_d = 0).
// Moment slots (N values each): 0 rho_a - rho_ref_a, 1 rho_b - rho_ref_b, 2 psi_a,
// 3 psi_b, 4 chi_a = G psi_b + G_a+ n+ + G_a- n- (the Shan-Chen source felt by fluid a;
// ions count on LB-fluid sites only), 5..7 pre-force velocity.  Solid sites hold
// rho = 0 (or the virtual density, written by k_virtual).
// ------------------------------------------------------------------------------------
constexpr int kMomSlots = 8;

// Occupancy requested for the fused kernel (waves per SIMD): four keeps FP32 at 128 VGPRs
// without spills; FP64 needs the registers of two.  The force kernel spills at four in
// FP32 and runs faster at three (170 VGPRs).
template <typename T> constexpr int kHotOcc = sizeof(T) == 4 ? 4 : 2;
template <typename T> constexpr int kForceOcc = sizeof(T) == 4 ? 3 : 2;

// Equilibrium of direction d (Sec. II A) in deviation form, f~_d - w_d rho_ref, for the
// deviation dr = rho - rho_ref, density rs, velocity u and usq = u.u.  The collision
// (fused sweep) and the moment-state gather evaluate it with this one expression, without
// multiply-add contraction, so that both round it the same way whatever surrounds it.
template <typename T>
__device__ __forceinline__ T usq_of(T u0, T u1, T u2) {
#pragma clang fp contract(off)
    return u0 * u0 + u1 * u1 + u2 * u2;
}

template <typename T>
__device__ __forceinline__ T geq_dev(int d, T dr, T rs, T u0, T u1, T u2, T usq) {
#pragma clang fp contract(off)
    const T cu = T(vx(d)) * u0 + T(vy(d)) * u1 + T(vz(d)) * u2;
    return T(storage_weight<T>(d)) * (dr + rs * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq));
}

// tau = 1 moment state.  At tau = 1 the post-collision populations of a site are the
// equilibria of its density and shifted velocity u_e = u' + Phi / rho (Sec. II A-C), so a
// site's 4 values per component stand for its 19 post-collision populations.  Streaming
// then makes the population arriving at site i in direction d (deviation form) the
// equilibrium of the source site i - c_d or, where that source is a wall layer, the
// halfway bounce-back of i's own population in the opposite direction (resting walls).
// Populations are never stored: the moments pass gathers them.
template <typename T>
struct MsSite {
    T dr, rs, u0, u1, u2, usq;
};

// The moment state is site-major: the 8 values of site j at ms[8 j .. 8 j + 7] (component
// c at 4 c: deviation, u_e x, y, z), one aligned 16-byte (FP32) or 32-byte (FP64) vector
// per component.
template <typename T> struct Vec4;
template <> struct Vec4<float> {
    using type = float4;
    using native = float __attribute__((ext_vector_type(4)));
};
template <> struct Vec4<double> {
    using type = double4;
    using native = double __attribute__((ext_vector_type(4)));
};

template <typename T>
__device__ __forceinline__ MsSite<T> ms_site(const Scalars& S, const Fields<T>& F, int c, unsigned j) {
    const typename Vec4<T>::type v = reinterpret_cast<const typename Vec4<T>::type*>(F.ms)[(size_t)2 * j + c];
    MsSite<T> a;
    a.dr = v.x;
    a.u0 = v.y;
    a.u1 = v.z;
    a.u2 = v.w;
    a.rs = T(S.rref[c]) + a.dr;
    a.usq = usq_of<T>(a.u0, a.u1, a.u2);
    return a;
}

// Population (deviation form) arriving at fluid site i, direction d, component c.  PM 1:
// gathered from the moment state; PM 2: the initial populations w_d (rho0 - rho_ref).
template <typename T, int PM>
__device__ __forceinline__ T arriving(const Scalars& S, const Fields<T>& F, int c, int d, unsigned i, int z,
                                      const Nbr& o, const MsSite<T>& own) {
    if (PM == 2) return (T)(storage_weight<T>(d) * (F.rho0[(size_t)c * S.N + i] - S.rref[c]));
    if (d != kRest) {
        const int od = opposite(d);
        const int zs = z - vz(d);
        if (!(S.walls && (zs == 0 || zs == S.nz - 1))) {
            const MsSite<T> a = ms_site<T>(S, F, c, i + offset_of(o, od));
            return geq_dev<T>(d, a.dr, a.rs, a.u0, a.u1, a.u2, a.usq);
        }
        return geq_dev<T>(od, own.dr, own.rs, own.u0, own.u1, own.u2, own.usq);
    }
    return geq_dev<T>(d, own.dr, own.rs, own.u0, own.u1, own.u2, own.usq);
}

// returns this site's contribution to the FP64 charge sum of the Poisson domain.  PM 0:
// populations read from storage; 1, 2: see arriving().
template <typename T, int G, int PM = 0>
__device__ __forceinline__ double moments_body(const Scalars& S, const Fields<T>& F, unsigned i) {
    // No multiply-add contraction here: a gathered population must enter the sums rounded
    // exactly as a stored one does, so both population sources give the same moments.
#pragma clang fp contract(off)
    double qsum = 0.0;
    if (i < S.N) {
        const int z = site_z(i, S);
        const bool solid = is_solid<T, G>(i, z, S, F);
        T da = T(-S.rref[0]), db = T(-S.rref[1]), ux = 0, uy = 0, uz = 0, pa = 0, pb = 0;
        if (!solid) {
            T sa = 0, sb = 0, mx = 0, my = 0, mz = 0;
            // FP32 populations with the exact-mass rest population (F.rlo set): the mass is
            // summed in FP64, where the 19 stored values and the rest population's low part
            // add up exactly, and the part the FP32 mass slot cannot hold goes to F.mlo
            const bool xm = sizeof(T) == 4 && PM == 0 && F.rlo != nullptr;
            double sad = 0.0, sbd = 0.0;
            Nbr o{};
            MsSite<T> own0{}, own1{};
            if (PM == 1) {
                int x, y, zz;
                site_xyz(i, S, x, y, zz);
                o = make_nbr(x, y, zz, S);
                own0 = ms_site<T>(S, F, 0, i);
                own1 = ms_site<T>(S, F, 1, i);
            }
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                const T a = PM == 0 ? __builtin_nontemporal_load(F.f[0] + (size_t)d * S.N + i)
                                    : arriving<T, PM>(S, F, 0, d, i, z, o, own0);
                const T b = PM == 0 ? __builtin_nontemporal_load(F.f[1] + (size_t)d * S.N + i)
                                    : arriving<T, PM>(S, F, 1, d, i, z, o, own1);
                sa += a;
                sb += b;
                if (xm) {
                    sad += (double)a;
                    sbd += (double)b;
                }
                const T s = a + b;
                if (vx(d) > 0) mx += s;
                if (vx(d) < 0) mx -= s;
                if (vy(d) > 0) my += s;
                if (vy(d) < 0) my -= s;
                if (vz(d) > 0) mz += s;
                if (vz(d) < 0) mz -= s;
            }
            if (xm) {
                sad += (double)F.rlo[i];
                sbd += (double)F.rlo[(size_t)S.N + i];
                sa = (T)sad;
                sb = (T)sbd;
                F.mlo[i] = (T)(sad - (double)sa);
                F.mlo[(size_t)S.N + i] = (T)(sbd - (double)sb);
            }
            da = sa;
            db = sb;
            const T ra = T(S.rref[0]) + sa, rb = T(S.rref[1]) + sb;
            const T rt = ra + rb;
            ux = mx / rt;
            uy = my / rt;
            uz = mz / rt;
            pa = pseudo<T>(ra, S);
            pb = pseudo<T>(rb, S);
        }
        const T ion_s = F.n[0][i], ion_c = F.n[1][i];
        const T npl = ion_s + T(0.5) * ion_c, nmi = ion_s - T(0.5) * ion_c;
        const T chi = T(S.G) * pb + (solid ? T(0) : T(S.G_p) * npl + T(S.G_m) * nmi);
        const size_t N = S.N;
        F.mom[i] = da;
        F.mom[N + i] = db;
        F.mom[2 * N + i] = pa;
        F.mom[3 * N + i] = pb;
        F.mom[4 * N + i] = chi;
        F.mom[5 * N + i] = ux;
        F.mom[6 * N + i] = uy;
        F.mom[7 * N + i] = uz;
        const T qc = G == kColloids ? F.qc[i] : T(0);
        const T q = ion_c + qc;
        const T psis = T(1) - fluid_fraction<T, G>(i, z, S, F);
        const T ra = T(S.rref[0]) + da, rb = T(S.rref[1]) + db;
        F.q[i] = q;
        F.eps[i] = T(S.eps_p) * psis + eps_fluid<T>(ra, rb, S) * (T(1) - psis);
        if (z >= S.z0 && z <= S.z1) qsum = (double)q;
    }
    return qsum;
}

template <typename T, int G, int PM>
__global__ __launch_bounds__(kBlock) void k_moments(Scalars S, Fields<T> F) {
    double v[1] = {moments_body<T, G, PM>(S, F, xcd_linear())};
    const bool mx[1] = {false};
    block_reduce_store<1>(v, mx, F.red, blockIdx.x, gridDim.x);
}

// population source of a context: 0 stored populations, 1 moment state, 2 initial densities
template <typename T> __host__ __device__ inline int pop_mode(const Fields<T>& F) {
    return F.ms == nullptr ? 0 : (F.ms_first ? 2 : 1);
}

template <typename T> void launch_moments(const Scalars& S, const Fields<T>& F, unsigned nblk, hipStream_t st) {
    const int pm = pop_mode(F);
    if (S.colloids)
        hipLaunchKernelGGL((k_moments<T, kColloids, 0>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (S.walls && pm == 0)
        hipLaunchKernelGGL((k_moments<T, kWalls, 0>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (S.walls && pm == 1)
        hipLaunchKernelGGL((k_moments<T, kWalls, 1>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (S.walls)
        hipLaunchKernelGGL((k_moments<T, kWalls, 2>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (pm == 0)
        hipLaunchKernelGGL((k_moments<T, kPeriodic, 0>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (pm == 1)
        hipLaunchKernelGGL((k_moments<T, kPeriodic, 1>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else
        hipLaunchKernelGGL((k_moments<T, kPeriodic, 2>), dim3(nblk), dim3(kBlock), 0, st, S, F);
}

// Virtual densities (Sec. II E, after Jansen et al.): a solid site with a fluid D3Q19
// neighbour carries the mean density of its fluid neighbours, used only by the
// Shan-Chen sums (and the permittivity of partly covered sites).
// ALL: every solid site next to fluid (flag bit 2) instead of the list built at set-up
// (moving particles change the mask).
template <typename T, bool ALL>
__global__ __launch_bounds__(kBlock) void k_virtual(Scalars S, Fields<T> F) {
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    if (ALL ? t >= S.N || !(F.flags[t] & 4u) : (int)t >= F.nv) return;
    const unsigned i = ALL ? t : (unsigned)F.vlist[t];
    int x, y, z;
    site_xyz(i, S, x, y, z);
    const Nbr o = make_nbr(x, y, z, S);
    T sa = 0, sb = 0;
    int cnt = 0;
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        if (d == kRest) continue;
        const unsigned j = i + offset_of(o, d);
        const int zj = wrapc(z + vz(d), S.nz);
        if (solid_at(j, zj, S, F)) continue;
        sa += F.mom[j];
        sb += F.mom[(size_t)S.N + j];
        ++cnt;
    }
    if (cnt == 0) return;
    const size_t N = S.N;
    const T da = sa / T(cnt), db = sb / T(cnt);
    const T ra = T(S.rref[0]) + da, rb = T(S.rref[1]) + db;
    const T pb = pseudo<T>(rb, S);
    F.mom[i] = da;
    F.mom[N + i] = db;
    F.mom[2 * N + i] = pseudo<T>(ra, S);
    F.mom[3 * N + i] = pb;
    F.mom[4 * N + i] = T(S.G) * pb;
    const T psis = T(1) - psif_at(i, z, S, F);
    F.eps[i] = T(S.eps_p) * psis + eps_fluid<T>(ra, rb, S) * (T(1) - psis);
}

template <typename T> void launch_virtual(const Scalars& S, const Fields<T>& F, hipStream_t st) {
    if (S.reproject) {
        hipLaunchKernelGGL((k_virtual<T, true>), dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F);
        return;
    }
    if (F.nv <= 0) return;
    hipLaunchKernelGGL((k_virtual<T, false>), dim3((F.nv + kBlock - 1) / kBlock), dim3(kBlock), 0, st, S, F);
}

// Mean of the Poisson source over the domain: (sum q + wall charges) / sites.
__device__ void source_mean_body(const Scalars& S, const double* __restrict__ red, unsigned nblk, double* scal) {
    __shared__ double sm[kRedThreads / 64];
    double a = 0.0;
    for (unsigned b0 = threadIdx.x; b0 < nblk; b0 += 4 * kRedThreads) {
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned b = b0 + j * kRedThreads;
            v[j] = b < nblk ? red[b] : 0.0;
        }
        a += v[0];
        a += v[1];
        a += v[2];
        a += v[3];
    }
#pragma unroll
    for (int s2 = 32; s2 > 0; s2 >>= 1) a += __shfl_down(a, s2, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = sm[0];
        for (int w = 1; w < kRedThreads / 64; ++w) tot += sm[w];
        if (S.walls) tot += (S.sigma0 + S.sigma1) * (double)S.nxy;
        scal[0] = tot / (double)S.ndomain;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_source_mean(Scalars S, const double* __restrict__ red, unsigned nblk,
                                                             double* scal) {
    source_mean_body(S, red, nblk, scal);
}

void launch_source_mean(const Scalars& S, double* red, unsigned nblk, double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_source_mean, dim3(1), dim3(kRedThreads), 0, st, S, red, nblk, scal);
}

// ------------------------------------------------------------------------------------
// Poisson (Sec. II D): sum_{Q6} eps_f (phi_j - phi_i) = -s_i, eps_f = (eps_i + eps_j)/2,
// s = q + wall charge in the layer next to a wall - mean.  Links leaving the domain (the
// wall faces) carry no flux; links of an axis of length 1 join a site to itself and
// contribute nothing, so they are skipped.
// ------------------------------------------------------------------------------------
//
// Inside a multigrid solve the lattice potential and charge can be held colour-split (SP):
// the sites of colour (x + y + z) % 2 = 1 follow those of colour 0, each colour in site
// order, so a colour pass reads and writes whole cache lines of its own colour.  Axes are
// even there, site i of colour c sits at c N/2 + i/2, and every neighbour has the other
// colour.  The permittivity stays in site order.
template <bool SP>
__device__ __forceinline__ unsigned cidx(const Scalars& S, unsigned i, int color) {
    return SP ? (color ? (S.N >> 1) : 0u) + (i >> 1) : i;
}

// The row with the neighbour potentials supplied by pv(j, colour, ox, oy, oz) for the
// neighbour j at offset (ox, oy, oz); poisson_row reads them from F.phi.  Evaluated
// without multiply-add contraction, so that callers supplying the neighbour values
// differently (loaded, or interpolated on the fly) round the row identically.  Every
// operand is fetched before the arithmetic: the faces that an axis of length 1 or a wall
// leaves out are fetched too (their indices are lattice sites: the site itself, or a wall
// layer) and then not used, so the loads carry no branches and issue together.
// The permittivities come from ev(j, ox, oy, oz) the same way and the charge from qv()
// (poisson_row_v: from F.eps and F.q).
template <typename T, bool SP, typename PV, typename EV, typename QV>
__device__ __forceinline__ void poisson_row_ve(unsigned i, int x, int y, int z, const Scalars& S, const Fields<T>& F,
                                               PV&& pv, EV&& ev, QV&& qv, double& diag, double& offsum, double& src) {
#pragma clang fp contract(off)
    const int own = SP ? ((x + y + z) & 1) : 0, nb = own ^ 1;
    const unsigned xa = i + (x == 0 ? S.nx - 1 : -1), xb = i + (x == S.nx - 1 ? -(S.nx - 1) : 1);
    const unsigned ya = i + (y == 0 ? (S.ny - 1) * S.nx : -S.nx), yb = i + (y == S.ny - 1 ? -(S.ny - 1) * S.nx : S.nx);
    const unsigned za = i + (z == 0 ? (S.nz - 1) * S.nxy : -S.nxy), zb = i + (z == S.nz - 1 ? -(S.nz - 1) * S.nxy : S.nxy);
    const double ei = ev(i, 0, 0, 0);
    const double exa = ev(xa, -1, 0, 0), exb = ev(xb, 1, 0, 0), eya = ev(ya, 0, -1, 0), eyb = ev(yb, 0, 1, 0),
                 eza = ev(za, 0, 0, -1), ezb = ev(zb, 0, 0, 1);
    const double pxa = pv(xa, nb, -1, 0, 0), pxb = pv(xb, nb, 1, 0, 0), pya = pv(ya, nb, 0, -1, 0),
                 pyb = pv(yb, nb, 0, 1, 0), pza = pv(za, nb, 0, 0, -1), pzb = pv(zb, nb, 0, 0, 1);
    double s = qv();
    diag = 0.0;
    offsum = 0.0;
    double pol = 0.0;  // sum over the faces of eps_f (E_ext . c_d): the polarisation source
    // A face that is left out (an axis of length 1, a wall) is taken with a zero
    // coefficient: adding +0 leaves every sum as it is, and the row has no branches, so the
    // loads of consecutive rows can overlap.
    {
        const bool on = S.nx > 1;
        const double ea = on ? 0.5 * (ei + exa) : 0.0, eb = on ? 0.5 * (ei + exb) : 0.0;
        diag += ea + eb;
        offsum += ea * pxa + eb * pxb;
        pol += S.E_ext[0] * (eb - ea);
    }
    {
        const bool on = S.ny > 1;
        const double ea = on ? 0.5 * (ei + eya) : 0.0, eb = on ? 0.5 * (ei + eyb) : 0.0;
        diag += ea + eb;
        offsum += ea * pya + eb * pyb;
        pol += S.E_ext[1] * (eb - ea);
    }
    {
        const bool lo = S.nz > 1 && !(S.walls && z == S.z0), hi = S.nz > 1 && !(S.walls && z == S.z1);
        const double ea = lo ? 0.5 * (ei + eza) : 0.0, eb = hi ? 0.5 * (ei + ezb) : 0.0;
        diag += ea;
        offsum += ea * pza;
        pol -= S.E_ext[2] * ea;
        diag += eb;
        offsum += eb * pzb;
        pol += S.E_ext[2] * eb;
    }
    if (S.walls && z == S.z0) s += S.sigma0;
    if (S.walls && z == S.z1) s += S.sigma1;
    if (S.polar) s -= pol;
    src = s - F.scal[0];
}

template <typename T, bool SP, typename PV>
__device__ __forceinline__ void poisson_row_v(unsigned i, int x, int y, int z, const Scalars& S, const Fields<T>& F,
                                              PV&& pv, double& diag, double& offsum, double& src) {
    poisson_row_ve<T, SP>(
        i, x, y, z, S, F, pv, [&](unsigned j, int, int, int) { return (double)F.eps[j]; },
        [&]() { return (double)F.q[cidx<SP>(S, i, SP ? ((x + y + z) & 1) : 0)]; }, diag, offsum, src);
}

template <typename T, bool SP = false>
__device__ __forceinline__ void poisson_row(unsigned i, int x, int y, int z, const Scalars& S, const Fields<T>& F,
                                            double& diag, double& offsum, double& src) {
    poisson_row_v<T, SP>(
        i, x, y, z, S, F, [&](unsigned j, int c, int, int, int) { return F.phi[cidx<SP>(S, j, c)]; }, diag, offsum,
        src);
}

// Over-relaxed Gauss-Seidel update, without multiply-add contraction so that every kernel
// that applies it (separate or fused with the interpolation) rounds it the same way.
__device__ __forceinline__ double sor_update(double p, double gs, double omega) {
#pragma clang fp contract(off)
    return p + omega * (gs - p);
}

// Colour of a site when a periodic y or z axis has odd length L >= 3.  On such an axis the
// link from L - 1 back to 0 joins two sites of equal parity, so (x + y + z) % 2 is no
// colouring.  Per axis the colour is the parity, except 2 for the last index of an odd
// periodic axis (a proper colouring of an odd cycle with three values); the sum of the
// three axis colours mod 3 differs between any two neighbours, so the sites of one colour
// are independent and each pass is well defined.
__device__ __forceinline__ int color3(const Scalars& S, int x, int y, int z) {
    const int cy = ((S.ny & 1) && S.ny >= 3 && y == S.ny - 1) ? 2 : (y & 1);
    const int cz = ((S.nz & 1) && S.nz >= 3 && !S.walls && z == S.nz - 1) ? 2 : (z & 1);
    return ((x & 1) + cy + cz) % 3;
}

// One colour of a Gauss-Seidel sweep.  Two colours (the usual red-black ordering): thread
// -> site of that colour ((x + y + z) % 2 == color).  Three colours: thread -> domain site,
// threads of other colours return.  sor_site computes the new value and where it goes;
// with OWN the site's current value is read from own[i / 2] (the black values left by the
// fused interpolation and red pass) instead of F.phi.
template <typename T, bool SP = false, bool OWN = false>
__device__ __forceinline__ bool sor_site(const Scalars& S, const Fields<T>& F, unsigned t, int color, double omega,
                                         unsigned& o, double& v, const double* own = nullptr) {
    unsigned i;
    int x, y, z;
    if (S.ncolor == 3) {
        if (t >= S.ndomain) return false;
        i = t + (unsigned)S.z0 * (unsigned)S.nxy;
        site_xyz(i, S, x, y, z);
        if (color3(S, x, y, z) != color) return false;
    } else {
        const unsigned half = (unsigned)(S.nx >> 1);
        const unsigned rows = (unsigned)S.ny * (unsigned)(S.z1 - S.z0 + 1);
        if (t >= half * rows) return false;
        const unsigned row = div_exact(t, S.inv_hx), m = t - row * half;
        const unsigned zr = div_exact(row, S.inv_ny);
        y = (int)(row - zr * (unsigned)S.ny);
        z = S.z0 + (int)zr;
        x = 2 * m + ((color + y + z) & 1);
        i = x + S.nx * (y + S.ny * z);
    }
    o = cidx<SP>(S, i, color);
    const double p = OWN ? own[i >> 1] : F.phi[o];
    double diag, offsum, src;
    poisson_row<T, SP>(i, x, y, z, S, F, diag, offsum, src);
    if (diag <= 0.0) {  // an isolated site keeps its value (with OWN: the one in own)
        if (!OWN) return false;
        v = p;
        return true;
    }
    const double gs = (offsum + src) / diag;
    v = sor_update(p, gs, omega);
    return true;
}

template <typename T, bool SP = false>
__device__ __forceinline__ void sor_body(const Scalars& S, const Fields<T>& F, unsigned t, int color, double omega) {
    unsigned o;
    double v;
    if (sor_site<T, SP>(S, F, t, color, omega, o, v)) F.phi[o] = v;
}

template <typename T, bool SP>
__global__ __launch_bounds__(kBlock) void k_sor(Scalars S, Fields<T> F, int color, double omega) {
    sor_body<T, SP>(S, F, xcd_linear(), color, omega);
}

// The black pass after k_mg_prolong_red_fine: own values from blk.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sor_black_from(Scalars S, Fields<T> F, double omega,
                                                           const double* __restrict__ blk) {
    unsigned o;
    double v;
    if (sor_site<T, true, true>(S, F, xcd_linear(), 1, omega, o, v, blk)) F.phi[o] = v;
}

template <typename T>
void launch_sor_black_from(const Scalars& S, const Fields<T>& F, double omega, const double* blk, hipStream_t st) {
    const unsigned n = (unsigned)(S.nx / 2) * S.ny * (S.z1 - S.z0 + 1);
    hipLaunchKernelGGL(k_sor_black_from<T>, dim3(site_blocks(n)), dim3(kBlock), 0, st, S, F, omega, blk);
}

// One whole red-black sweep in one pass over colour-split fields, from pin to pout.  A
// workgroup owns a tile of kRbTX x kRbTY sites over a range of planes and marches up
// through them, holding three planes of the old potential, four of the permittivity and
// three of new red values in LDS.  At plane k it computes the red update of plane k on the
// tile and a one-site ring around it, then the black update of plane k - 1 on the tile.
// The red update reads only old black values, the black update only new red ones, both
// from LDS, so the result is the one the two colour passes give, bit for bit: the same
// rows, in the same operand order.  The ring's red values are computed again by the
// neighbouring tiles, which need them too; the second buffer keeps the old values that
// other workgroups still read.  Two colour passes move 2 x 18 B/site in FP32 (each
// re-reads the charge and permittivity of both colours); this pass 24 B/site.  With walls
// the wall layers are copied, so that every value a row of the next pass reads is set.
constexpr int kRbTX = 64, kRbTY = 4, kRbLX = kRbTX + 4, kRbLY = kRbTY + 4, kRbP = kRbLX * kRbLY;
constexpr int kRbRed = (kRbTX + 2) / 2 * (kRbTY + 2);  // red sites of the tile and its ring, per plane

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sor_rb(Scalars S, Fields<T> F, const double* __restrict__ pin,
                                                  double* __restrict__ pout, double omega, int zc, unsigned nwork) {
    static_assert(kRbTX * kRbTY == kBlock && kRbRed <= kBlock, "one tile site and one ring red site per thread");
    constexpr int kLoads = (kRbP + kBlock - 1) / kBlock;  // LDS positions per thread and plane
    constexpr int kHalfRow = kRbTX / 2, kRingRow = (kRbTX + 2) / 2;
    __shared__ double sphi[3][kRbP];  // old potential, planes k - 1, k, k + 1
    __shared__ T seps[4][kRbP];       // permittivity, planes k - 2 .. k + 1
    __shared__ double sred[3][kRbP];  // new red values, planes k - 2, k - 1, k (tile and ring)
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned w = (b & 7u) * (nb >> 3) + (b >> 3);  // XCD-contiguous ranges of tiles
    if (w >= nwork) return;
    const unsigned ntx = (unsigned)S.nx / kRbTX, nty = (unsigned)S.ny / kRbTY;
    const unsigned tx = w % ntx, rest = w / ntx, ty = rest % nty, chunk = rest / nty;
    const int x0 = (int)tx * kRbTX, y0 = (int)ty * kRbTY;
    const int zs = S.z0 + (int)chunk * zc, ze = min(zs + zc, S.z1 + 1);  // planes [zs, ze)
    const int t = threadIdx.x;
    const unsigned nx = (unsigned)S.nx, nxy = (unsigned)S.nxy, half = (unsigned)S.N >> 1;
    // a plane index k in [zs - 2, ze + 1] that is a lattice plane (with walls: 0 .. nz - 1)
    auto inside = [&](int k) { return !S.walls || (k >= 0 && k < S.nz); };
    auto zplane = [&](int k) { return S.walls ? min(max(k, 0), S.nz - 1) : wrapc(k, S.nz); };
    auto s3 = [&](int k) { return (k - zs + 3) % 3; };  // k >= zs - 2
    auto s4 = [&](int k) { return (k - zs + 4) % 4; };
    // colour-split index of the site at in-plane offset xy (x + nx y, colour parity c of
    // x + y) in plane z
    auto split = [&](unsigned xy, int c, int z) {
        const unsigned i = xy + nxy * (unsigned)z;
        return (((c + z) & 1) ? half : 0u) + (i >> 1);
    };
    // The thread's LDS positions of a plane (in-plane offsets and parities are the same in
    // every plane).  The next plane's potential and permittivity go to registers one step
    // ahead and into LDS at the next step, so their loads overlap a step's arithmetic.
    unsigned f_xy[kLoads];
    int f_c[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
        const int p = min(t + j * kBlock, kRbP - 1);
        const int ly = p / kRbLX, lx = p - ly * kRbLX;
        const int x = wrapc(x0 - 2 + lx, S.nx), y = wrapc(y0 - 2 + ly, S.ny);
        f_xy[j] = (unsigned)x + nx * (unsigned)y;
        f_c[j] = (x + y) & 1;
    }
    double rphi[kLoads];
    T reps[kLoads];
    auto fetch = [&](int k) {
        const int zz = zplane(k);
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            rphi[j] = pin[split(f_xy[j], f_c[j], zz)];
            reps[j] = F.eps[f_xy[j] + nxy * (unsigned)zz];
        }
    };
    auto commit = [&](int k) {
        if (!inside(k)) return;  // not a plane: never read
        double* dp = sphi[s3(k)];
        T* de = seps[s4(k)];
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int p = t + j * kBlock;
            if (p < kRbP) {
                dp[p] = rphi[j];
                de[p] = reps[j];
            }
        }
    };
    // The thread's red site of the tile and ring (t < kRbRed), and its tile site: the black
    // sites of the tile for t < kBlock / 2, the red ones for the others.  Both depend on the
    // parity of the plane: [0] even planes, [1] odd.
    int r_x[2], r_p[2], r_y = 0;
    unsigned r_xy[2];
    int b_x[2], b_p[2], b_y;
    unsigned b_xy[2];
    {
        const int ly = 1 + t / kRingRow, m = t - (ly - 1) * kRingRow;
        r_y = wrapc(y0 - 2 + ly, S.ny);
        const int u = t & (kBlock / 2 - 1), r = u / kHalfRow, mb = u - r * kHalfRow;
        b_y = y0 + r;
        const int want = t < kBlock / 2 ? 1 : 0;  // colour of the tile site
#pragma unroll
        for (int pz = 0; pz < 2; ++pz) {
            const int lx = 1 + ((r_y + pz + 1) & 1) + 2 * m;  // x + y + z even (x0 is even)
            r_x[pz] = wrapc(x0 - 2 + lx, S.nx);
            r_p[pz] = ly * kRbLX + lx;
            r_xy[pz] = (unsigned)r_x[pz] + nx * (unsigned)r_y;
            const int bx = 2 * mb + ((b_y + pz + want) & 1);  // x + y + z has the wanted parity
            b_x[pz] = x0 + bx;
            b_p[pz] = (2 + r) * kRbLX + 2 + bx;
            b_xy[pz] = (unsigned)b_x[pz] + nx * (unsigned)b_y;
        }
    }
    const bool black = t < kBlock / 2;
    // charges, one step ahead: of the red site of plane k and of the black tile site of plane k - 1
    auto q_red = [&](int k) {
        const int zz = zplane(k), pz = zz & 1;
        return t < kRbRed ? F.q[(r_xy[pz] + nxy * (unsigned)zz) >> 1] : T(0);  // red: the first half
    };
    auto q_black = [&](int k) {
        const int zz = zplane(k), pz = zz & 1;
        return black ? F.q[half + ((b_xy[pz] + nxy * (unsigned)zz) >> 1)] : T(0);
    };
    // the row at LDS position p of plane k with neighbour potentials from plane ring v
    auto update = [&](const double (*v)[kRbP], int p, int k, int x, int y, int zz, T q) {
        double diag, offsum, src;
        poisson_row_ve<T, true>(
            0u, x, y, zz, S, F, [&](unsigned, int, int ox, int oy, int oz) { return v[s3(k + oz)][p + ox + oy * kRbLX]; },
            [&](unsigned, int ox, int oy, int oz) { return (double)seps[s4(k + oz)][p + ox + oy * kRbLX]; },
            [&]() { return (double)q; }, diag, offsum, src);
        const double old = sphi[s3(k)][p];
        return diag > 0.0 ? sor_update(old, (offsum + src) / diag, omega) : old;  // an isolated site keeps its value
    };
    fetch(zs - 2);
    commit(zs - 2);
    fetch(zs - 1);
    commit(zs - 1);
    fetch(zs);
    commit(zs);
    fetch(zs + 1);
    T qr = q_red(zs - 1), qb = T(0);
    for (int k = zs - 1; k <= ze; ++k) {
        if (k >= zs) {
            commit(k + 1);
            if (k + 2 <= ze + 1) fetch(k + 2);
        }
        const T qr_next = q_red(min(k + 1, ze)), qb_next = q_black(k);
        __syncthreads();
        const int zz = zplane(k), pz = zz & 1;
        if (t < kRbRed) {  // red site of plane k in the tile or its ring
            const bool wall = S.walls && (k < S.z0 || k > S.z1);
            const int p = r_p[pz];
            sred[s3(k)][p] = wall ? sphi[s3(k)][p] : update(sphi, p, k, r_x[pz], r_y, zz, qr);
        }
        __syncthreads();
        const int kb = k - 1;
        if (kb >= zs) {  // plane kb: black update, and the red values of the tile
            const int zb = zplane(kb), pb = zb & 1, p = b_p[pb];
            const unsigned o = (black ? half : 0u) + ((b_xy[pb] + nxy * (unsigned)zb) >> 1);
            pout[o] = black ? update(sred, p, kb, b_x[pb], b_y, zb, qb) : sred[s3(kb)][p];
        }
        if (S.walls && ((k == zs - 1 && zs == S.z0) || (k == ze && ze == S.z1 + 1))) {  // a wall layer
            const int p = b_p[pz];
            pout[(black ? half : 0u) + ((b_xy[pz] + nxy * (unsigned)zz) >> 1)] = sphi[s3(k)][p];
        }
        __syncthreads();
        qr = qr_next;
        qb = qb_next;
    }
}

// Whether k_sor_rb covers the lattice: two colours, whole tiles in x and y, and enough
// planes for its LDS window.
bool sor_rb_fits(const Scalars& S) {
    return S.ncolor == 2 && S.nx % kRbTX == 0 && S.ny % kRbTY == 0 && S.nz >= 8 && S.z1 - S.z0 + 1 >= 4;
}

template <typename T>
void launch_sor_rb(const Scalars& S, const Fields<T>& F, const double* pin, double* pout, double omega,
                   hipStream_t st) {
    const int nzd = S.z1 - S.z0 + 1;
    const unsigned tiles = (unsigned)(S.nx / kRbTX) * (unsigned)(S.ny / kRbTY);
    // planes per workgroup: about 2048 workgroups, at least 8 planes each (the window's
    // two extra planes cost little against them)
    const int zc = std::max(8, (int)((tiles * (unsigned)nzd + 2047) / 2048));
    const unsigned chunks = (unsigned)((nzd + zc - 1) / zc), nwork = tiles * chunks;
    const unsigned nblk = (nwork + 7) / 8 * 8;  // whole XCD rounds; the extra workgroups return
    hipLaunchKernelGGL(k_sor_rb<T>, dim3(nblk), dim3(kBlock), 0, st, S, F, pin, pout, omega, zc, nwork);
}

template <typename T>
void launch_sor(const Scalars& S, const Fields<T>& F, int color, double omega, bool split, hipStream_t st) {
    const unsigned n = S.ncolor == 3 ? S.ndomain : (unsigned)(S.nx / 2) * S.ny * (S.z1 - S.z0 + 1);
    if (split)
        hipLaunchKernelGGL((k_sor<T, true>), dim3(site_blocks(n)), dim3(kBlock), 0, st, S, F, color, omega);
    else
        hipLaunchKernelGGL((k_sor<T, false>), dim3(site_blocks(n)), dim3(kBlock), 0, st, S, F, color, omega);
}

// Residual r = s + A phi: FP64 partial sums of r.r, s.s and phi over the domain.
// The operands are fetched for a lattice site whether or not i lies in the domain (outside
// it: a wall layer, or the last site past the end) and the sums take zeros there, so the
// loads of the sites a thread handles carry no branches and can overlap.
template <typename T, bool SP = false>
__device__ __forceinline__ void residual_body(const Scalars& S, const Fields<T>& F, unsigned i, double (&v)[3]) {
    const unsigned k = i < S.N ? i : S.N - 1;
    int x, y, z;
    site_xyz(k, S, x, y, z);
    const bool in = i < S.N && z >= S.z0 && z <= S.z1;
    const double p = F.phi[cidx<SP>(S, k, (x + y + z) & 1)];
    double diag, offsum, src;
    poisson_row<T, SP>(k, x, y, z, S, F, diag, offsum, src);
    const double res = src + offsum - diag * p;
    v[0] = in ? res * res : 0.0;
    v[1] = in ? src * src : 0.0;
    v[2] = in ? p : 0.0;
}

// Each thread takes kResSites sites, kBlock apart (a workgroup covers kResSites x kBlock
// consecutive sites), and sums them in order before the block reduction: fewer records
// for the reducer to read.  From site-order fields (SP false) the kernel can also write
// the colour-split copies of the potential and charge (phis, qs non-null) for the
// multigrid solve that follows.
template <typename T, bool SP>
__global__ __launch_bounds__(kBlock) void k_residual(Scalars S, Fields<T> F, double* __restrict__ phis,
                                                     T* __restrict__ qs) {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned lb = (b & 7u) * (nb >> 3) + (b >> 3);  // XCD-contiguous ranges, as xcd_linear
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kResSites; ++j) {
        const unsigned i = (lb * kResSites + j) * kBlock + threadIdx.x;
        if (!SP && phis && i < S.N) {
            int x, y, z;
            site_xyz(i, S, x, y, z);
            const unsigned o = cidx<true>(S, i, (x + y + z) & 1);
            phis[o] = F.phi[i];
            qs[o] = F.q[i];
        }
        double v[3];
        residual_body<T, SP>(S, F, i, v);
        acc[0] += v[0];
        acc[1] += v[1];
        acc[2] += v[2];
    }
    const bool mx[3] = {false, false, false};
    block_reduce_store<3>(acc, mx, F.red, blockIdx.x, gridDim.x);
}

unsigned residual_blocks(unsigned n) { return site_blocks((n + kResSites - 1) / kResSites); }

template <typename T>
void launch_residual(const Scalars& S, const Fields<T>& F, unsigned nblk, bool split, double* phis, T* qs,
                     hipStream_t st) {
    if (split)
        hipLaunchKernelGGL((k_residual<T, true>), dim3(nblk), dim3(kBlock), 0, st, S, F, (double*)nullptr,
                           (T*)nullptr);
    else
        hipLaunchKernelGGL((k_residual<T, false>), dim3(nblk), dim3(kBlock), 0, st, S, F, phis, qs);
}

// Gauge mean(phi) = 0 over the domain (scal[3] = sum of phi), or phi = 0 when zero != 0.
__device__ __forceinline__ void finalize_body(const Scalars& S, double* phi, const double* scal, int zero, unsigned i) {
    if (i >= S.N) return;
    const int z = site_z(i, S);
    if (z < S.z0 || z > S.z1) return;
    phi[i] = zero ? 0.0 : phi[i] - scal[3] / (double)S.ndomain;
}

// The gauge, and with walls the wall layers from the gauged potential next to them (Gauss's
// law at the charged wall face): phi_wall = phi_adjacent + sigma / eps_adjacent.  The
// solved potential is read from src, colour-split when SP (it is F.phi otherwise).
template <typename T, bool SP>
__global__ __launch_bounds__(kBlock) void k_phi_finalize(Scalars S, Fields<T> F, int zero, const double* src) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    if (z < S.z0 || z > S.z1) return;
    const double p = zero ? 0.0 : src[cidx<SP>(S, i, (x + y + z) & 1)] - F.scal[3] / (double)S.ndomain;
    F.phi[i] = p;
    if (S.walls && z == S.z0) F.phi[i - S.nxy] = p + S.sigma0 / (double)F.eps[i];
    if (S.walls && z == S.z1) F.phi[i + S.nxy] = p + S.sigma1 / (double)F.eps[i];
}

template <typename T>
void launch_phi_finalize(const Scalars& S, const Fields<T>& F, int zero, const double* split_src, hipStream_t st) {
    if (split_src)
        hipLaunchKernelGGL((k_phi_finalize<T, true>), dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, zero,
                           split_src);
    else
        hipLaunchKernelGGL((k_phi_finalize<T, false>), dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, zero,
                           (const double*)F.phi);
}

// Warm start of the next solve by linear extrapolation in time,
// phi <- 2 phi(t-1) - phi(t-2), keeping phi(t-1) for the following step.
__device__ __forceinline__ void extrapolate_body(const Scalars& S, double* phi, double* phi_prev, unsigned i) {
    if (i >= S.N) return;
    const int z = site_z(i, S);
    if (z < S.z0 || z > S.z1) return;
    const double p = phi[i];
    phi[i] = 2.0 * p - phi_prev[i];
    phi_prev[i] = p;
}

// Start of the next solve from the last potentials phi(t-1), phi(t-2), phi(t-3) (held in
// phi, prev, prev2): the previous one, or the linear or quadratic extrapolation in time;
// the history shifts by one step.
__global__ __launch_bounds__(kBlock) void k_phi_extrapolate(Scalars S, double* phi, double* prev, double* prev2,
                                                            int history) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    const int z = site_z(i, S);
    if (z < S.z0 || z > S.z1) return;
    const double p1 = phi[i], p2 = prev[i];
    double v = p1;
    if (history == 2) v = 2.0 * p1 - p2;
    if (history >= 3) v = 3.0 * (p1 - p2) + prev2[i];
    phi[i] = v;
    prev2[i] = p2;
    prev[i] = p1;
}

void launch_phi_extrapolate(const Scalars& S, double* phi, double* prev, double* prev2, int history,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_phi_extrapolate, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, phi, prev, prev2,
                       history);
}

// ------------------------------------------------------------------------------------
// Geometric multigrid for the same Poisson operator.  Cell-centred coarsening by 2 per
// axis; a coarse face coefficient is half the sum of the four fine faces it covers (the
// finite-volume flux of a cell twice as wide); the residual is restricted by summing the
// eight children; the correction is interpolated trilinearly (weights 3/4, 1/4 per axis),
// falling back to the parent across a zero face.  Smoothing is red-black Gauss-Seidel.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned lid(const MGLevel& L, int x, int y, int z) {
    return (unsigned)x + (unsigned)L.nx * ((unsigned)y + (unsigned)L.ny * (unsigned)z);
}

// Fine-level face coefficient between (x, y, z) and its +k neighbour: zero unless both
// cells are in the Poisson domain.
template <typename T>
__device__ __forceinline__ double fine_face(int k, int x, int y, int z, const Scalars& S, const Fields<T>& F) {
    if (z < S.z0 || z > S.z1) return 0.0;
    int xn = x, yn = y, zn = z;
    if (k == 0) xn = wrapc(x + 1, S.nx);
    if (k == 1) yn = wrapc(y + 1, S.ny);
    if (k == 2) {
        zn = wrapc(z + 1, S.nz);
        if (zn < S.z0 || zn > S.z1) return 0.0;
    }
    const unsigned i = x + S.nx * (y + S.ny * z), j = xn + S.nx * (yn + S.ny * zn);
    return 0.5 * ((double)F.eps[i] + (double)F.eps[j]);
}

template <typename T>
__device__ __forceinline__ void coarsen_fine_body(const Scalars& S, const Fields<T>& F, const MGLevel& C, unsigned t) {
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    double ax = 0, ay = 0, az = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            ax += fine_face<T>(0, 2 * I + 1, 2 * J + a, 2 * K + b, S, F);
            ay += fine_face<T>(1, 2 * I + a, 2 * J + 1, 2 * K + b, S, F);
            az += fine_face<T>(2, 2 * I + a, 2 * J + b, 2 * K + 1, S, F);
        }
    C.ax[t] = 0.5 * ax;
    C.ay[t] = 0.5 * ay;
    C.az[t] = 0.5 * az;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_coarsen_fine(Scalars S, Fields<T> F, MGLevel C) {
    coarsen_fine_body<T>(S, F, C, xcd_linear());
}

template <typename T> void launch_mg_coarsen_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_coarsen_fine<T>, dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c);
}

__device__ __forceinline__ void coarsen_body(const MGLevel& Fl, const MGLevel& C, unsigned t) {
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    double ax = 0, ay = 0, az = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            ax += Fl.ax[lid(Fl, 2 * I + 1, 2 * J + a, 2 * K + b)];
            ay += Fl.ay[lid(Fl, 2 * I + a, 2 * J + 1, 2 * K + b)];
            az += Fl.az[lid(Fl, 2 * I + a, 2 * J + b, 2 * K + 1)];
        }
    C.ax[t] = 0.5 * ax;
    C.ay[t] = 0.5 * ay;
    C.az[t] = 0.5 * az;
}

__global__ __launch_bounds__(kBlock) void k_mg_coarsen(MGLevel Fl, MGLevel C) {
    coarsen_body(Fl, C, xcd_linear());
}

void launch_mg_coarsen(const MGLevel& f, const MGLevel& c, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_coarsen, dim3(site_blocks(c.n)), dim3(kBlock), 0, st, f, c);
}

// Row of a coarse level: diagonal, off-diagonal sum, at cell (x, y, z).
__device__ __forceinline__ void mg_row(const MGLevel& L, int x, int y, int z, double& diag, double& off) {
    const int xm = wrapc(x - 1, L.nx), xp = wrapc(x + 1, L.nx);
    const int ym = wrapc(y - 1, L.ny), yp = wrapc(y + 1, L.ny);
    const int zm = wrapc(z - 1, L.nz), zp = wrapc(z + 1, L.nz);
    const unsigned i = lid(L, x, y, z);
    const double a0 = L.ax[i], a1 = L.ax[lid(L, xm, y, z)];
    const double b0 = L.ay[i], b1 = L.ay[lid(L, x, ym, z)];
    const double c0 = L.az[i], c1 = L.az[lid(L, x, y, zm)];
    diag = a0 + a1 + b0 + b1 + c0 + c1;
    off = a0 * L.phi[lid(L, xp, y, z)] + a1 * L.phi[lid(L, xm, y, z)] + b0 * L.phi[lid(L, x, yp, z)] +
          b1 * L.phi[lid(L, x, ym, z)] + c0 * L.phi[lid(L, x, y, zp)] + c1 * L.phi[lid(L, x, y, zm)];
}

__device__ __forceinline__ void smooth_body(const MGLevel& L, int color, double omega, unsigned t) {
    const unsigned half = (unsigned)(L.nx >> 1);
    if (t >= half * (unsigned)L.ny * (unsigned)L.nz) return;
    const unsigned row = div_exact(t, L.inv_hx), m = t - row * half;
    const int z = (int)div_exact(row, L.inv_ny), y = (int)row - z * L.ny;
    const int x = 2 * m + ((color + y + z) & 1);
    double diag, off;
    mg_row(L, x, y, z, diag, off);
    if (diag <= 0.0) return;
    const unsigned i = lid(L, x, y, z);
    L.phi[i] = L.phi[i] + omega * ((off + L.s[i]) / diag - L.phi[i]);
}

__global__ __launch_bounds__(kBlock) void k_mg_smooth(MGLevel L, int color, double omega) {
    smooth_body(L, color, omega, xcd_linear());
}

void launch_mg_smooth(const MGLevel& L, int color, double omega, hipStream_t st) {
    const unsigned n = L.n / 2;
    hipLaunchKernelGGL(k_mg_smooth, dim3(site_blocks(n)), dim3(kBlock), 0, st, L, color, omega);
}

// Start of a coarse grid's correction: zero, except that with red_omega > 0 the red cells
// ((I + J + K) even) take the first red pass of the pre-smoothing here.  From a zero
// correction every neighbour term of that pass vanishes and it reduces to
// omega s / diag, written as the sweep writes it (same operand order), so the grid's
// first separate pass can be skipped.
__device__ __forceinline__ void coarse_start(const MGLevel& C, int I, int J, int K, unsigned t, double s,
                                             double red_omega) {
    double v = 0.0;
    if (red_omega > 0.0 && ((I + J + K) & 1) == 0) {
        const int xm = wrapc(I - 1, C.nx), ym = wrapc(J - 1, C.ny), zm = wrapc(K - 1, C.nz);
        const double diag = C.ax[t] + C.ax[lid(C, xm, J, K)] + C.ay[t] + C.ay[lid(C, I, ym, K)] + C.az[t] +
                            C.az[lid(C, I, J, zm)];
        if (diag > 0.0) {
            const double p = 0.0, off = 0.0;
            v = p + red_omega * ((off + s) / diag - p);
        }
    }
    C.phi[t] = v;
}

// Residuals of the eight lattice cells under coarse cell t, summed.  The eight rows
// share their stencil points: the 2x2x2 block and the four neighbours across each of its
// six faces (32 sites), loaded once each.  Rows as in poisson_row, same operand order.
template <typename T, bool SP = false>
__device__ __forceinline__ void restrict_fine_body(const Scalars& S, const Fields<T>& F, const MGLevel& C, unsigned t,
                                                   double red_omega = 0.0) {
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    int xs[4], ys[4], zs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        xs[k] = wrapc(2 * I - 1 + k, S.nx);
        ys[k] = wrapc(2 * J - 1 + k, S.ny);
        zs[k] = wrapc(2 * K - 1 + k, S.nz);
    }
    auto at = [&](int a, int b, int c) {
        return (unsigned)xs[a] + (unsigned)S.nx * ((unsigned)ys[b] + (unsigned)S.ny * (unsigned)zs[c]);
    };
    auto col = [&](int a, int b, int c) { return (xs[a] + ys[b] + zs[c]) & 1; };
    double P[4][4][4];
    T E[4][4][4];  // permittivity in its storage precision (exactly widened where used)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int outer = (a == 0 || a == 3) + (b == 0 || b == 3) + (c == 0 || c == 3);
                if (outer <= 1) {
                    const unsigned g = at(a, b, c);
                    P[c][b][a] = F.phi[cidx<SP>(S, g, col(a, b, c))];
                    E[c][b][a] = F.eps[g];
                }
            }
    const double mean = F.scal[0];
    double sum = 0.0;
#pragma unroll
    for (int c = 1; c < 3; ++c)
#pragma unroll
        for (int b = 1; b < 3; ++b)
#pragma unroll
            for (int a = 1; a < 3; ++a) {
                const int z = zs[c];
                if (z < S.z0 || z > S.z1) continue;
                const double ei = (double)E[c][b][a];
                double diag = 0.0, off = 0.0, pol = 0.0;
                {
                    const double ea = 0.5 * (ei + (double)E[c][b][a - 1]), eb = 0.5 * (ei + (double)E[c][b][a + 1]);
                    diag += ea + eb;
                    off += ea * P[c][b][a - 1] + eb * P[c][b][a + 1];
                    pol += S.E_ext[0] * (eb - ea);
                }
                {
                    const double ea = 0.5 * (ei + (double)E[c][b - 1][a]), eb = 0.5 * (ei + (double)E[c][b + 1][a]);
                    diag += ea + eb;
                    off += ea * P[c][b - 1][a] + eb * P[c][b + 1][a];
                    pol += S.E_ext[1] * (eb - ea);
                }
                if (!(S.walls && z == S.z0)) {
                    const double ea = 0.5 * (ei + (double)E[c - 1][b][a]);
                    diag += ea;
                    off += ea * P[c - 1][b][a];
                    pol -= S.E_ext[2] * ea;
                }
                if (!(S.walls && z == S.z1)) {
                    const double eb = 0.5 * (ei + (double)E[c + 1][b][a]);
                    diag += eb;
                    off += eb * P[c + 1][b][a];
                    pol += S.E_ext[2] * eb;
                }
                double src = (double)F.q[cidx<SP>(S, at(a, b, c), col(a, b, c))];
                if (S.walls && z == S.z0) src += S.sigma0;
                if (S.walls && z == S.z1) src += S.sigma1;
                if (S.polar) src -= pol;
                src -= mean;
                sum += src + off - diag * P[c][b][a];
            }
    C.s[t] = sum;
    coarse_start(C, I, J, K, t, sum, red_omega);
}

template <typename T, bool SP>
__global__ __launch_bounds__(kBlock) void k_mg_restrict_fine(Scalars S, Fields<T> F, MGLevel C, double red_omega) {
    restrict_fine_body<T, SP>(S, F, C, xcd_linear(), red_omega);
}

template <typename T>
void launch_mg_restrict_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, bool split, double red_omega,
                             hipStream_t st) {
    if (split)
        hipLaunchKernelGGL((k_mg_restrict_fine<T, true>), dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c,
                           red_omega);
    else
        hipLaunchKernelGGL((k_mg_restrict_fine<T, false>), dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c,
                           red_omega);
}

__device__ __forceinline__ void restrict_body(const MGLevel& Fl, const MGLevel& C, unsigned t, double red_omega = 0.0) {
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    double sum = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const int x = 2 * I + a, y = 2 * J + b, z = 2 * K + c;
                double diag, off;
                mg_row(Fl, x, y, z, diag, off);
                const unsigned i = lid(Fl, x, y, z);
                sum += Fl.s[i] + off - diag * Fl.phi[i];
            }
    C.s[t] = sum;
    coarse_start(C, I, J, K, t, sum, red_omega);
}

// The same with one thread per cell of Fl: eight consecutive lanes hold the children of
// one coarse cell (child a + 2b + 4c), and the sum runs over them in the order of
// restrict_body.  The launched coarse grids are small (32 k and 4 k coarse cells at 128^3),
// and eight times the threads hide the loads of the rows far better.
__global__ __launch_bounds__(kBlock) void k_mg_restrict(MGLevel Fl, MGLevel C, double red_omega) {
    const unsigned t = xcd_linear();
    if (t >= 8u * C.n) return;  // groups of eight lanes leave together (blockDim is a multiple of 8)
    const unsigned pc = t >> 3, ch = t & 7u;
    int I, J, K;
    level_xyz(pc, C, I, J, K);
    const int x = 2 * I + (int)(ch & 1u), y = 2 * J + (int)((ch >> 1) & 1u), z = 2 * K + (int)(ch >> 2);
    double diag, off;
    mg_row(Fl, x, y, z, diag, off);
    const unsigned i = lid(Fl, x, y, z);
    const double r = Fl.s[i] + off - diag * Fl.phi[i];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) sum += __shfl(r, k, 8);
    if (ch == 0) {
        C.s[pc] = sum;
        coarse_start(C, I, J, K, pc, sum, red_omega);
    }
}

void launch_mg_restrict(const MGLevel& f, const MGLevel& c, double red_omega, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_restrict, dim3(site_blocks(8u * c.n)), dim3(kBlock), 0, st, f, c, red_omega);
}

// Trilinear interpolation of the coarse correction at the fine cell (x, y, z).
__device__ __forceinline__ double mg_interp(const MGLevel& C, int x, int y, int z) {
    const int I = x >> 1, J = y >> 1, K = z >> 1;
    const int dx = (x & 1) ? 1 : -1, dy = (y & 1) ? 1 : -1, dz = (z & 1) ? 1 : -1;
    const int In = wrapc(I + dx, C.nx), Jn = wrapc(J + dy, C.ny), Kn = wrapc(K + dz, C.nz);
    const double fx = C.ax[lid(C, dx > 0 ? I : In, J, K)];
    const double fy = C.ay[lid(C, I, dy > 0 ? J : Jn, K)];
    const double fz = C.az[lid(C, I, J, dz > 0 ? K : Kn)];
    const double wx = fx > 0.0 ? 0.25 : 0.0, wy = fy > 0.0 ? 0.25 : 0.0, wz = fz > 0.0 ? 0.25 : 0.0;
    const int xs[2] = {I, In}, ys[2] = {J, Jn}, zs[2] = {K, Kn};
    const double wxs[2] = {1.0 - wx, wx}, wys[2] = {1.0 - wy, wy}, wzs[2] = {1.0 - wz, wz};
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) v += wxs[a] * wys[b] * wzs[c] * C.phi[lid(C, xs[a], ys[b], zs[c])];
    return v;
}

// The same interpolation onto the lattice.  Coarse faces of the first coarse grid are
// zero only where it wraps across the wall layers in z (every other face averages
// positive permittivities), so the weights follow from the indices and no coefficient
// is read.
template <typename T>
__device__ __forceinline__ void prolong_fine_body(const Scalars& S, const Fields<T>& F, const MGLevel& C, unsigned i) {
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    if (z < S.z0 || z > S.z1) return;
    const int I = x >> 1, J = y >> 1, K = z >> 1;
    const int dx = (x & 1) ? 1 : -1, dy = (y & 1) ? 1 : -1, dz = (z & 1) ? 1 : -1;
    const int In = wrapc(I + dx, C.nx), Jn = wrapc(J + dy, C.ny), Kn = wrapc(K + dz, C.nz);
    const bool zwrap = S.walls && (K + dz < 0 || K + dz >= C.nz);
    const double wx = 0.25, wy = 0.25, wz = zwrap ? 0.0 : 0.25;
    const int xs[2] = {I, In}, ys[2] = {J, Jn}, zs[2] = {K, Kn};
    const double wxs[2] = {1.0 - wx, wx}, wys[2] = {1.0 - wy, wy}, wzs[2] = {1.0 - wz, wz};
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) v += wxs[a] * wys[b] * wzs[c] * C.phi[lid(C, xs[a], ys[b], zs[c])];
    F.phi[i] += v;
}

// Trilinear correction of one lattice site from the coarse potentials P of the cells
// (I - 1 .. I + 1) x (J - 1 .. J + 1) x (K - 1 .. K + 1): xo, yo, zo index the site's own
// coarse cell and its neighbour towards the site, weighted 3/4 and 1/4 (wzs carries the
// fall-back to the parent across a wall).  The terms and their order are those of
// prolong_fine_body.
__device__ __forceinline__ double prolong_corr(const double (&P)[3][3][3], const int (&xo)[2], const int (&yo)[2],
                                               const int (&zo)[2], const double (&wzs)[2]) {
#pragma clang fp contract(off)
    const double wxs[2] = {0.75, 0.25}, wys[2] = {0.75, 0.25};
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) v += wxs[a] * wys[b] * wzs[c] * P[zo[c]][yo[b]][xo[a]];
    return v;
}

__device__ __forceinline__ void load_coarse27(const MGLevel& C, int I, int J, int K, double (&P)[3][3][3]) {
#pragma unroll
    for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int ox = 0; ox < 3; ++ox)
                P[oz][oy][ox] = C.phi[lid(C, wrapc(I + ox - 1, C.nx), wrapc(J + oy - 1, C.ny), wrapc(K + oz - 1, C.nz))];
}

// The same, one thread per coarse cell for its eight lattice children: the 3x3x3 coarse
// neighbourhood is loaded once into registers and each child is interpolated with exactly
// the expression and order of prolong_fine_body (bit-identical); the two x-children of a
// row are read and written as one 16-byte pair (colour-split, SP: one value in each
// colour half).
template <typename T, bool SP>
__global__ __launch_bounds__(kBlock) void k_mg_prolong_fine(Scalars S, Fields<T> F, MGLevel C) {
    const unsigned t = xcd_linear();
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    double P[3][3][3];  // coarse potential at (I + ox - 1, J + oy - 1, K + oz - 1), periodic
    load_coarse27(C, I, J, K, P);
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const int z = 2 * K + cz;
        if (z < S.z0 || z > S.z1) continue;
        const int dz = cz ? 1 : -1;
        const bool zwrap = S.walls && (K + dz < 0 || K + dz >= C.nz);
        const double wz = zwrap ? 0.0 : 0.25;
        const double wzs[2] = {1.0 - wz, wz};
        const int zo[2] = {1, 1 + dz};
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int y = 2 * J + cy;
            const int dy = cy ? 1 : -1;
            const int yo[2] = {1, 1 + dy};
            const unsigned i0 = (unsigned)(2 * I) + (unsigned)S.nx * ((unsigned)y + (unsigned)S.ny * (unsigned)z);
            double2 f;
            double2* row = nullptr;
            unsigned o0 = 0, o1 = 0;
            if (SP) {
                o0 = cidx<SP>(S, i0, (y + z) & 1);
                o1 = cidx<SP>(S, i0 + 1, (y + z + 1) & 1);
                f.x = F.phi[o0];
                f.y = F.phi[o1];
            } else {
                row = reinterpret_cast<double2*>(F.phi + i0);
                f = *row;
            }
            double vv[2];
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int dx = cx ? 1 : -1;
                const int xo[2] = {1, 1 + dx};
                vv[cx] = prolong_corr(P, xo, yo, zo, wzs);
            }
            f.x += vv[0];
            f.y += vv[1];
            if (SP) {
                F.phi[o0] = f.x;
                F.phi[o1] = f.y;
            } else {
                *row = f;
            }
        }
    }
}

template <typename T>
void launch_mg_prolong_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, bool split, hipStream_t st) {
    if (split)
        hipLaunchKernelGGL((k_mg_prolong_fine<T, true>), dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c);
    else
        hipLaunchKernelGGL((k_mg_prolong_fine<T, false>), dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c);
}

// The interpolation onto the lattice fused with the first red pass of the post-smoothing
// (colour-split fields).  One thread per coarse cell.  Its four red children take the
// interpolated correction and then their Gauss-Seidel update; their six black neighbours
// (three in the block, three around it) are interpolated on the fly from the same 3x3x3
// coarse registers.  Its four black children's interpolated values go to blk (indexed
// like the black half), and the black pass that follows reads them from there: written in
// place they could reach a neighbouring thread that still needs the old values.  Every
// value is the one the separate interpolation and red pass compute: the same expressions
// in the same order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_prolong_red_fine(Scalars S, Fields<T> F, MGLevel C, double omega,
                                                                double* __restrict__ blk) {
    const unsigned t = xcd_linear();
    if (t >= C.n) return;
    int I, J, K;
    level_xyz(t, C, I, J, K);
    double P[3][3][3];
    load_coarse27(C, I, J, K, P);
    // correction at the lattice site (2I + rx, 2J + ry, 2K + rz), rx, ry, rz in -1..2 (its
    // coarse cell and the neighbour towards it lie in P); the offsets are compile-time
    // constants once the loops below unroll, so P stays in registers
    auto corr_at = [&](int rx, int ry, int rz) {
        const int dx = (rx & 1) ? 1 : -1, dy = (ry & 1) ? 1 : -1, dz = (rz & 1) ? 1 : -1;
        const int xo[2] = {1 + (rx >> 1), 1 + (rx >> 1) + dx}, yo[2] = {1 + (ry >> 1), 1 + (ry >> 1) + dy},
                  zo[2] = {1 + (rz >> 1), 1 + (rz >> 1) + dz};  // >> 1: floor, also for -1
        const int Kw = wrapc(K + (rz >> 1), C.nz);
        const bool zwrap = S.walls && (Kw + dz < 0 || Kw + dz >= C.nz);
        const double wz = zwrap ? 0.0 : 0.25;
        const double wzs[2] = {1.0 - wz, wz};
        return prolong_corr(P, xo, yo, zo, wzs);
    };
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int x = 2 * I + cx, y = 2 * J + cy, z = 2 * K + cz;
                if (z < S.z0 || z > S.z1) continue;
                const unsigned i = (unsigned)x + (unsigned)S.nx * ((unsigned)y + (unsigned)S.ny * (unsigned)z);
                const int col = (cx + cy + cz) & 1;
                const double p = F.phi[cidx<true>(S, i, col)] + corr_at(cx, cy, cz);
                if (col) {
                    blk[i >> 1] = p;
                    continue;
                }
                double diag, offsum, src;
                poisson_row_v<T, true>(
                    i, x, y, z, S, F,
                    [&](unsigned j, int c, int ox, int oy, int oz) {
                        return F.phi[cidx<true>(S, j, c)] + corr_at(cx + ox, cy + oy, cz + oz);
                    },
                    diag, offsum, src);
                double v = p;
                if (diag > 0.0) v = sor_update(p, (offsum + src) / diag, omega);
                F.phi[cidx<true>(S, i, 0)] = v;
            }
}

template <typename T>
void launch_mg_prolong_red_fine(const Scalars& S, const Fields<T>& F, const MGLevel& c, double omega, double* blk,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_mg_prolong_red_fine<T>, dim3(site_blocks(c.n)), dim3(kBlock), 0, st, S, F, c, omega, blk);
}


__device__ __forceinline__ void prolong_body(const MGLevel& C, const MGLevel& Fl, unsigned i) {
    if (i >= Fl.n) return;
    int x, y, z;
    level_xyz(i, Fl, x, y, z);
    Fl.phi[i] += mg_interp(C, x, y, z);
}

__global__ __launch_bounds__(kBlock) void k_mg_prolong(MGLevel C, MGLevel Fl) {
    prolong_body(C, Fl, xcd_linear());
}

void launch_mg_prolong(const MGLevel& c, const MGLevel& f, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_prolong, dim3(site_blocks(f.n)), dim3(kBlock), 0, st, c, f);
}

// The last two levels in one workgroup: on the upper of them ("mid", at most kTailMid
// cells) red-black Gauss-Seidel sweeps, restriction to the coarsest level (at most
// kTailCoarse cells), red-black SOR sweeps there, interpolation back and more sweeps on
// the mid grid.  The mid grid's face coefficients are float (this grid only carries a
// coarse-grid correction; the lattice-level residual stays FP64).  When has_mid is 0 only
// the coarsest solve runs, and the coarsest grid may use the whole LDS allocation.
constexpr int kTailThreads = 512;
constexpr unsigned kTailMid = 4096, kTailCoarse = 512;
constexpr unsigned kTailCoarseOnly = kTailMid + kTailCoarse;

template <typename C>
struct TailGrid {
    int nx, ny, nz;
    unsigned n;
    double* phi;
    const double* rhs;
    const C* ax;
    const C* ay;
    const C* az;
    C* idiag;  // 1 / diagonal (0 for a decoupled cell)
};

template <typename C>
__device__ __forceinline__ unsigned tid3(const TailGrid<C>& L, int x, int y, int z) {
    return (unsigned)x + (unsigned)L.nx * ((unsigned)y + (unsigned)L.ny * (unsigned)z);
}

template <typename C>
__device__ __forceinline__ void tail_row(const TailGrid<C>& L, int x, int y, int z, double& diag, double& off) {
    const int xm = wrapc(x - 1, L.nx), xp = wrapc(x + 1, L.nx);
    const int ym = wrapc(y - 1, L.ny), yp = wrapc(y + 1, L.ny);
    const int zm = wrapc(z - 1, L.nz), zp = wrapc(z + 1, L.nz);
    const unsigned i = tid3(L, x, y, z);
    const double a0 = L.ax[i], a1 = L.ax[tid3(L, xm, y, z)];
    const double b0 = L.ay[i], b1 = L.ay[tid3(L, x, ym, z)];
    const double c0 = L.az[i], c1 = L.az[tid3(L, x, y, zm)];
    diag = a0 + a1 + b0 + b1 + c0 + c1;
    off = a0 * L.phi[tid3(L, xp, y, z)] + a1 * L.phi[tid3(L, xm, y, z)] + b0 * L.phi[tid3(L, x, yp, z)] +
          b1 * L.phi[tid3(L, x, ym, z)] + c0 * L.phi[tid3(L, x, y, zp)] + c1 * L.phi[tid3(L, x, y, zm)];
}

template <typename C>
__device__ void tail_inverse_diagonal(const TailGrid<C>& L) {
    for (unsigned t = threadIdx.x; t < L.n; t += blockDim.x) {
        const int x = t % L.nx, r = t / L.nx, y = r % L.ny, z = r / L.ny;
        double diag, off;
        tail_row(L, x, y, z, diag, off);
        L.idiag[t] = diag > 0.0 ? (C)(1.0 / diag) : (C)0;
    }
}

template <typename C>
__device__ void tail_sweeps(const TailGrid<C>& L, int sweeps, double omega) {
    const unsigned half = L.n / 2, hx = (unsigned)(L.nx >> 1);
    for (int it = 0; it < sweeps; ++it)
        for (int color = 0; color < 2; ++color) {
            for (unsigned t = threadIdx.x; t < half; t += blockDim.x) {
                const unsigned row = t / hx, m = t % hx;
                const int y = row % L.ny, z = row / L.ny;
                const int x = 2 * m + ((color + y + z) & 1);
                double diag, off;
                tail_row(L, x, y, z, diag, off);
                const unsigned i = tid3(L, x, y, z);
                L.phi[i] = L.phi[i] + omega * ((off + L.rhs[i]) * (double)L.idiag[i] - L.phi[i]);
            }
            __syncthreads();
        }
}

template <typename C>
__device__ void tail_load_coeffs(const MGLevel& G, C* ax, C* ay, C* az) {
    for (unsigned t = threadIdx.x; t < G.n; t += blockDim.x) {
        ax[t] = (C)G.ax[t];
        ay[t] = (C)G.ay[t];
        az[t] = (C)G.az[t];
    }
}

// Cell h of colour c of a red-black grid (h < n/2, even nx): coordinates.
__device__ __forceinline__ void rb_cell(unsigned h, int c, unsigned hx, double inv_hx, int ny, double inv_ny, int& x,
                                        int& y, int& z) {
    const unsigned row = div_exact(h, inv_hx), m = h - row * hx;
    z = (int)div_exact(row, inv_ny);
    y = (int)row - z * ny;
    x = 2 * (int)m + ((c + y + z) & 1);
}

// Periodic neighbour indices of cell i = (x, y, z), packed (+1 side | -1 side << 16).
struct PackedNbr {
    unsigned x, y, z;
};

__device__ __forceinline__ PackedNbr packed_nbr(unsigned i, int x, int y, int z, int nx, int ny, int nz) {
    const unsigned nxu = (unsigned)nx, nxy = (unsigned)(nx * ny), n = nxy * (unsigned)nz;
    const unsigned xm = x == 0 ? i + nxu - 1 : i - 1, xp = x == nx - 1 ? i + 1 - nxu : i + 1;
    const unsigned ym = y == 0 ? i + nxy - nxu : i - nxu, yp = y == ny - 1 ? i + nxu - nxy : i + nxu;
    const unsigned zm = z == 0 ? i + n - nxy : i - nxy, zp = z == nz - 1 ? i + nxy - n : i + nxy;
    return PackedNbr{xp | (xm << 16), yp | (ym << 16), zp | (zm << 16)};
}

// An owned cell of the mid grid with its row in registers.
struct MidRow {
    unsigned i;  // cell index (n when the slot is empty)
    PackedNbr nb;
    float a0, a1, b0, b1, c0, c1;  // faces to +x, -x, +y, -y, +z, -z
    float idiag;                   // 1 / diagonal (0 for a decoupled cell)
    double rhs, phi;
};

// The tail with a mid grid.  Every cell is owned by one thread (cell h of each colour by
// thread h % NT), which keeps its row (neighbour indices, coefficients, inverse diagonal,
// right-hand side) and its potential in registers for the whole call; LDS holds the
// potentials the neighbours read, and the residuals for the restriction.  Loads are
// coalesced through LDS.  The arithmetic and its order are those of the row-by-row form
// (tail_row, tail_sweeps), so the result does not depend on the thread count.
template <int NT>
__device__ __forceinline__ void tail_mid_body(const MGLevel M, const MGLevel Cg, int coarse_iters, double coarse_omega, int mid_pre,
                              int mid_post, double mid_omega) {
    extern __shared__ double lds[];
    constexpr int kSlots = kTailMid / 2 / NT;
    double* phim = lds;
    double* res = phim + kTailMid;  // right-hand side while loading, then the residuals
    double* phic = res + kTailMid;
    double* sc = phic + kTailCoarse;
    double* cax = sc + kTailCoarse;
    double* cay = cax + kTailCoarse;
    double* caz = cay + kTailCoarse;
    float* fax = (float*)(caz + kTailCoarse);
    float* fay = fax + kTailMid;
    float* faz = fay + kTailMid;
    for (unsigned t = threadIdx.x; t < M.n; t += NT) {
        fax[t] = (float)M.ax[t];
        fay[t] = (float)M.ay[t];
        faz[t] = (float)M.az[t];
        res[t] = M.s[t];
    }
    for (unsigned t = threadIdx.x; t < Cg.n; t += NT) {
        cax[t] = Cg.ax[t];
        cay[t] = Cg.ay[t];
        caz[t] = Cg.az[t];
    }
    __syncthreads();
    const unsigned halfm = M.n / 2, hxm = (unsigned)(M.nx >> 1);
    const double inv_hxm = 1.0 / hxm, inv_nym = 1.0 / M.ny;
    MidRow R[2][kSlots];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            MidRow& r = R[c][k];
            const unsigned h = threadIdx.x + k * NT;
            r.i = M.n;
            if (h < halfm) {
                int x, y, z;
                rb_cell(h, c, hxm, inv_hxm, M.ny, inv_nym, x, y, z);
                const unsigned i = (unsigned)x + (unsigned)M.nx * ((unsigned)y + (unsigned)M.ny * (unsigned)z);
                r.i = i;
                r.nb = packed_nbr(i, x, y, z, M.nx, M.ny, M.nz);
                r.a0 = fax[i];
                r.a1 = fax[r.nb.x >> 16];
                r.b0 = fay[i];
                r.b1 = fay[r.nb.y >> 16];
                r.c0 = faz[i];
                r.c1 = faz[r.nb.z >> 16];
                const double a0 = r.a0, a1 = r.a1, b0 = r.b0, b1 = r.b1, c0 = r.c0, c1 = r.c1;
                const double diag = a0 + a1 + b0 + b1 + c0 + c1;
                r.idiag = diag > 0.0 ? (float)(1.0 / diag) : 0.0f;
                r.rhs = res[i];
                r.phi = 0.0;
                phim[i] = 0.0;
            }
        }
    __syncthreads();
    // (both lambdas must inline: the row array has to stay in registers)
    auto off_of = [&](const MidRow& r) __attribute__((always_inline)) {
        const double a0 = r.a0, a1 = r.a1, b0 = r.b0, b1 = r.b1, c0 = r.c0, c1 = r.c1;
        return a0 * phim[r.nb.x & 0xffffu] + a1 * phim[r.nb.x >> 16] + b0 * phim[r.nb.y & 0xffffu] +
               b1 * phim[r.nb.y >> 16] + c0 * phim[r.nb.z & 0xffffu] + c1 * phim[r.nb.z >> 16];
    };
    auto mid_sweeps = [&](int sweeps) __attribute__((always_inline)) {
        for (int it = 0; it < sweeps; ++it)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    MidRow& r = R[c][k];
                    if (r.i < M.n) {
                        const double off = off_of(r);
                        r.phi = r.phi + mid_omega * ((off + r.rhs) * (double)r.idiag - r.phi);
                        phim[r.i] = r.phi;
                    }
                }
                __syncthreads();
            }
    };
    mid_sweeps(mid_pre);
    // residuals of the owned cells (the right-hand side in res is no longer needed: every
    // owner holds its own), then the coarse right-hand side: the sum over eight children
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const MidRow& r = R[c][k];
            if (r.i < M.n) {
                const double a0 = r.a0, a1 = r.a1, b0 = r.b0, b1 = r.b1, c0 = r.c0, c1 = r.c1;
                const double diag = a0 + a1 + b0 + b1 + c0 + c1;
                const double off = off_of(r);
                res[r.i] = r.rhs + off - diag * r.phi;
            }
        }
    __syncthreads();
    const unsigned mnx = (unsigned)M.nx, mnxy = (unsigned)(M.nx * M.ny);
    const unsigned cnx = (unsigned)Cg.nx, cnxy = (unsigned)(Cg.nx * Cg.ny);
    const double inv_cnx = 1.0 / cnx, inv_cny = 1.0 / Cg.ny;
    for (unsigned t = threadIdx.x; t < Cg.n; t += NT) {
        const unsigned r = div_exact(t, inv_cnx), I = t - r * cnx;
        const unsigned K = div_exact(r, inv_cny), J = r - K * (unsigned)Cg.ny;
        const unsigned b = 2 * I + mnx * 2 * J + mnxy * 2 * K;
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int a = 0; a < 2; ++a) sum += res[b + a + mnx * bb + mnxy * c];
        sc[t] = sum;
        phic[t] = 0.0;
    }
    __syncthreads();
    // coarsest grid: thread h < n/2 owns cell h of each colour
    const unsigned halfc = Cg.n / 2, hxc = cnx >> 1;
    const double inv_hxc = 1.0 / hxc;
    unsigned ci[2];
    PackedNbr cn[2];
    double cidg[2], crhs[2], cphi[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        ci[c] = Cg.n;
        const unsigned h = threadIdx.x;
        if (h < halfc) {
            int x, y, z;
            rb_cell(h, c, hxc, inv_hxc, Cg.ny, inv_cny, x, y, z);
            const unsigned i = (unsigned)x + cnx * (unsigned)y + cnxy * (unsigned)z;
            ci[c] = i;
            cn[c] = packed_nbr(i, x, y, z, Cg.nx, Cg.ny, Cg.nz);
            const double a0 = cax[i], a1 = cax[cn[c].x >> 16], b0 = cay[i], b1 = cay[cn[c].y >> 16];
            const double c0 = caz[i], c1 = caz[cn[c].z >> 16];
            const double diag = a0 + a1 + b0 + b1 + c0 + c1;
            cidg[c] = diag > 0.0 ? 1.0 / diag : 0.0;
            crhs[c] = sc[i];
            cphi[c] = 0.0;
        }
    }
    for (int it = 0; it < coarse_iters; ++it)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (ci[c] < Cg.n) {
                const unsigned i = ci[c];
                const PackedNbr& q = cn[c];
                const double a0 = cax[i], a1 = cax[q.x >> 16], b0 = cay[i], b1 = cay[q.y >> 16];
                const double c0 = caz[i], c1 = caz[q.z >> 16];
                const double off = a0 * phic[q.x & 0xffffu] + a1 * phic[q.x >> 16] + b0 * phic[q.y & 0xffffu] +
                                   b1 * phic[q.y >> 16] + c0 * phic[q.z & 0xffffu] + c1 * phic[q.z >> 16];
                cphi[c] = cphi[c] + coarse_omega * ((off + crhs[c]) * cidg[c] - cphi[c]);
                phic[i] = cphi[c];
            }
            __syncthreads();
        }
    // trilinear interpolation of the coarse correction onto the owned cells (parent only
    // across a zero face)
    const double inv_mnx = 1.0 / mnx, inv_mny = 1.0 / M.ny;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            MidRow& r = R[c][k];
            if (r.i < M.n) {
                const unsigned row = div_exact(r.i, inv_mnx);
                const int x = (int)(r.i - row * mnx);
                const int z = (int)div_exact(row, inv_mny), y = (int)row - z * M.ny;
                const int I = x >> 1, J = y >> 1, K = z >> 1;
                const int dx = (x & 1) ? 1 : -1, dy = (y & 1) ? 1 : -1, dz = (z & 1) ? 1 : -1;
                const unsigned In = wrapc(I + dx, Cg.nx), Jn = cnx * wrapc(J + dy, Cg.ny), Kn = cnxy * wrapc(K + dz, Cg.nz);
                const unsigned I0 = I, J0 = cnx * J, K0 = cnxy * K;
                const double fx = cax[(dx > 0 ? I0 : In) + J0 + K0];
                const double fy = cay[I0 + (dy > 0 ? J0 : Jn) + K0];
                const double fz = caz[I0 + J0 + (dz > 0 ? K0 : Kn)];
                const double wx = fx > 0.0 ? 0.25 : 0.0, wy = fy > 0.0 ? 0.25 : 0.0, wz = fz > 0.0 ? 0.25 : 0.0;
                const unsigned xs[2] = {I0, In}, ys[2] = {J0, Jn}, zs[2] = {K0, Kn};
                const double wxs[2] = {1.0 - wx, wx}, wys[2] = {1.0 - wy, wy}, wzs[2] = {1.0 - wz, wz};
                double v = 0.0;
#pragma unroll
                for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int a = 0; a < 2; ++a) v += wxs[a] * wys[b] * wzs[cc] * phic[xs[a] + ys[b] + zs[cc]];
                r.phi += v;
                phim[r.i] = r.phi;
            }
        }
    __syncthreads();
    mid_sweeps(mid_post);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < kSlots; ++k)
            if (R[c][k].i < M.n) M.phi[R[c][k].i] = R[c][k].phi;
}

__device__ __forceinline__ void tail_body(const MGLevel& M, const MGLevel& Cg, int has_mid, int coarse_iters, double coarse_omega,
                          int mid_pre = 2, int mid_post = 2, double mid_omega = 1.0) {
    extern __shared__ double lds[];
    if (has_mid) {
        tail_mid_body<kTailThreads>(M, Cg, coarse_iters, coarse_omega, mid_pre, mid_post, mid_omega);
    } else {
        double* phic = lds;
        double* sc = phic + kTailCoarseOnly;
        float* cax = (float*)(sc + kTailCoarseOnly);
        float* cay = cax + kTailCoarseOnly;
        float* caz = cay + kTailCoarseOnly;
        float* cid = caz + kTailCoarseOnly;
        tail_load_coeffs(Cg, cax, cay, caz);
        for (unsigned t = threadIdx.x; t < Cg.n; t += blockDim.x) {
            sc[t] = Cg.s[t];
            phic[t] = 0.0;
        }
        __syncthreads();
        const TailGrid<float> Lc{Cg.nx, Cg.ny, Cg.nz, Cg.n, phic, sc, cax, cay, caz, cid};
        tail_inverse_diagonal(Lc);
        __syncthreads();
        tail_sweeps(Lc, coarse_iters, coarse_omega);
        for (unsigned t = threadIdx.x; t < Cg.n; t += blockDim.x) Cg.phi[t] = phic[t];
    }
}

__global__ __launch_bounds__(kTailThreads) void k_mg_tail(MGLevel M, MGLevel Cg, int has_mid, int coarse_iters,
                                                         double coarse_omega, int mid_pre, int mid_post,
                                                         double mid_omega) {
    tail_body(M, Cg, has_mid, coarse_iters, coarse_omega, mid_pre, mid_post, mid_omega);
}

size_t mg_tail_lds_bytes() {
    const size_t with_mid = 2 * kTailMid * 8 + 5 * kTailCoarse * 8 + 3 * kTailMid * 4;
    const size_t coarse_only = 2 * kTailCoarseOnly * 8 + 4 * kTailCoarseOnly * 4;
    return with_mid > coarse_only ? with_mid : coarse_only;
}

void launch_mg_tail(const MGLevel& mid, const MGLevel& coarse, int has_mid, int iters, double omega, int mid_pre,
                    int mid_post, double mid_omega, hipStream_t st) {
    hipLaunchKernelGGL(k_mg_tail, dim3(1), dim3(kTailThreads), mg_tail_lds_bytes(), st, mid, coarse, has_mid, iters,
                       omega, mid_pre, mid_post, mid_omega);
}

// ------------------------------------------------------------------------------------
// Link fluxes (Sec. II B, II E eq. ionic-fluxes-disc-2), for the link lo -> hi along axis k:
//   J = -D psi_f(lo) psi_f(hi) [ (n~_hi - n~_lo) - (beta/4)(q~_lo + q~_hi)(E_lo + E_hi)_k
//                              + s (beta dmu / 2 drho_a)(n~_lo + n~_hi)(rho^a_hi - rho^a_lo) ]
// n~ = n / psi_f, q~ = z e n~.  Both end sites evaluate a link with identical operands in
// identical order, so the two see bit-identical fluxes and the update conserves ions.
// ------------------------------------------------------------------------------------
// The same flux written for the stored variables s = (n+ + n-)/2 and c = n+ - n-
// (an exact linear recombination of the two species' fluxes):
//   J_s = (J+ + J-)/2 = w [ (s~_hi - s~_lo) - (beta/4)(c~_lo + c~_hi)/2 Es
//                           + ((k+ + k-) S + (k+ - k-) C/2) dra / 2 ]
//   J_c =  J+ - J-    = w [ (c~_hi - c~_lo) - (beta/4) 2 (s~_lo + s~_hi) Es
//                           + ((k+ - k-) S + (k+ + k-) C/2) dra ]
// with S = s~_lo + s~_hi, C = c~_lo + c~_hi, Es = (E_lo + E_hi)_k, dra the rho^a
// difference, w = -D psi_f(lo) psi_f(hi), k+- = s beta dmu+- / (2 drho_a).  The charge
// flux is rounded relative to its own terms, not to the salt concentration.
template <typename T>
__device__ __forceinline__ void link_flux(T sl, T cl, T sh, T ch, T w, T Elo, T Ehi, T ralo, T rahi,
                                          const Scalars& S, T& Js, T& Jc) {
#pragma clang fp contract(off)
    const T es = Elo + Ehi;
    const T dra = rahi - ralo;
    const T qb = T(0.25) * T(S.beta);
    const T ss = sl + sh, cs = cl + ch;
    const T ksum = T(S.kap_p) + T(S.kap_m), kdif = T(S.kap_p) - T(S.kap_m);
    const T bs = (sh - sl) - qb * (T(0.5) * cs) * es + T(0.5) * (ksum * ss + kdif * (T(0.5) * cs)) * dra;
    const T bc = (ch - cl) - qb * (T(2) * ss) * es + (kdif * ss + ksum * (T(0.5) * cs)) * dra;
    Js = w * bs;
    Jc = w * bc;
}

// Donor-cell advection across lo -> hi (only between LB-fluid sites).
template <typename T>
__device__ __forceinline__ T advect(T nlo, T nhi, T ulo, T uhi) {
#pragma clang fp contract(off)
    return nlo * (ulo > T(0) ? ulo : T(0)) - nhi * (uhi < T(0) ? -uhi : T(0));
}

// Potential values around a site shared by the field evaluations of one site: the six
// axis neighbours (a[k][0] at -e_k, a[k][1] at +e_k) and the six second neighbours.
struct PhiStar {
    double c;
    double a[3][2];
    double b[3][2];
};

__device__ __forceinline__ PhiStar load_phi_star(unsigned i, int x, int y, int z, const Nbr& o, const Scalars& S,
                                                 const double* phi) {
    PhiStar P;
    P.c = phi[i];
    P.a[0][0] = phi[i + o.xm];
    P.a[0][1] = phi[i + o.xp];
    P.a[1][0] = phi[i + o.ym];
    P.a[1][1] = phi[i + o.yp];
    P.a[2][0] = phi[i + o.zm];
    P.a[2][1] = phi[i + o.zp];
    const int row = S.nx * (y + S.ny * z);
    P.b[0][0] = phi[wrapc(x - 2, S.nx) + row];
    P.b[0][1] = phi[wrapc(x + 2, S.nx) + row];
    const int zr = S.nx * S.ny * z;
    P.b[1][0] = phi[x + S.nx * wrapc(y - 2, S.ny) + zr];
    P.b[1][1] = phi[x + S.nx * wrapc(y + 2, S.ny) + zr];
    const int xy = x + S.nx * y;
    P.b[2][0] = phi[xy + S.nxy * wrapc(z - 2, S.nz)];
    P.b[2][1] = phi[xy + S.nxy * wrapc(z + 2, S.nz)];
    return P;
}

// Field component k at the site (E0), at its -e_k neighbour (El) and at its +e_k
// neighbour (Eh); the normal component on a wall layer is one-sided.
__device__ __forceinline__ void field_line(int k, int z, const PhiStar& P, const Scalars& S, double& El, double& E0,
                                           double& Eh) {
    E0 = -0.5 * (P.a[k][1] - P.a[k][0]) + S.E_ext[k];
    if (k == 2 && S.walls && z - 1 == 0)
        El = -(P.c - P.a[2][0]) + S.E_ext[2];
    else
        El = -0.5 * (P.c - P.b[k][0]) + S.E_ext[k];
    if (k == 2 && S.walls && z + 1 == S.nz - 1)
        Eh = -(P.a[2][1] - P.c) + S.E_ext[2];
    else
        Eh = -0.5 * (P.b[k][1] - P.c) + S.E_ext[k];
}

// The six links of (non-wall) site i: friction sums (sum over species of J on the +k and
// -k link, per axis), and when kUpdate the new ion densities.  El/Eh of every axis are
// returned for the Kelvin force.
template <typename T, int G, bool kUpdate>
__device__ __forceinline__ void site_links(unsigned i, int z, const Nbr& o, bool solid_i, const PhiStar& P,
                                           const Scalars& S, const Fields<T>& F, T (&jsum)[3], double (&El)[3],
                                           double (&Eh)[3], T& np_new, T& nm_new) {
    const T s_i = F.n[0][i], c_i = F.n[1][i];
    const T ra_i = F.mom[i];
    const T pf_i = fluid_fraction<T, G>(i, z, S, F);
    const T inv_i = G == kColloids ? (pf_i > T(0) ? T(1) / pf_i : T(0)) : T(1);
    const T ts_i = s_i * inv_i, tc_i = c_i * inv_i;
    T out_s = T(0), out_c = T(0);
    T u_i[3];
    if (kUpdate && !solid_i) {
        u_i[0] = F.uph[i];
        u_i[1] = F.uph[(size_t)S.N + i];
        u_i[2] = F.uph[2 * (size_t)S.N + i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int offm = k == 0 ? o.xm : (k == 1 ? o.ym : o.zm);
        const int offp = k == 0 ? o.xp : (k == 1 ? o.yp : o.zp);
        const unsigned lo = i + offm, hi = i + offp;
        const int zlo = k == 2 ? wrapc(z - 1, S.nz) : z, zhi = k == 2 ? wrapc(z + 1, S.nz) : z;
        double E0;
        field_line(k, z, P, S, El[k], E0, Eh[k]);
        const T Ei = (T)E0, Elo = (T)El[k], Ehi = (T)Eh[k];
        const T s_lo = F.n[0][lo], c_lo = F.n[1][lo], s_hi = F.n[0][hi], c_hi = F.n[1][hi];
        const T ra_lo = F.mom[lo], ra_hi = F.mom[hi];
        const T pf_lo = fluid_fraction<T, G>(lo, zlo, S, F), pf_hi = fluid_fraction<T, G>(hi, zhi, S, F);
        T inv_lo = T(1), inv_hi = T(1);
        if (G == kColloids) {
            inv_lo = pf_lo > T(0) ? T(1) / pf_lo : T(0);
            inv_hi = pf_hi > T(0) ? T(1) / pf_hi : T(0);
        }
        const T wlo = (pf_lo > T(0) && pf_i > T(0)) ? -T(S.D) * pf_lo * pf_i : T(0);
        const T whi = (pf_i > T(0) && pf_hi > T(0)) ? -T(S.D) * pf_i * pf_hi : T(0);
        T Js_lo, Jc_lo, Js_hi, Jc_hi;
        link_flux<T>(s_lo * inv_lo, c_lo * inv_lo, ts_i, tc_i, wlo, Elo, Ei, ra_lo, ra_i, S, Js_lo, Jc_lo);
        link_flux<T>(ts_i, tc_i, s_hi * inv_hi, c_hi * inv_hi, whi, Ei, Ehi, ra_i, ra_hi, S, Js_hi, Jc_hi);
        jsum[k] = T(2) * (Js_hi + Js_lo);  // sum over both species of J on the two links
        if (kUpdate) {
            T As_lo = 0, Ac_lo = 0, As_hi = 0, Ac_hi = 0;
            if (!solid_i) {
                if (!is_solid<T, G>(lo, zlo, S, F)) {
                    const T u_lo = F.uph[(size_t)k * S.N + lo];
                    As_lo = advect<T>(s_lo, s_i, u_lo, u_i[k]);
                    Ac_lo = advect<T>(c_lo, c_i, u_lo, u_i[k]);
                }
                if (!is_solid<T, G>(hi, zhi, S, F)) {
                    const T u_hi = F.uph[(size_t)k * S.N + hi];
                    As_hi = advect<T>(s_i, s_hi, u_i[k], u_hi);
                    Ac_hi = advect<T>(c_i, c_hi, u_i[k], u_hi);
                }
            }
            out_s += (Js_hi + As_hi) - (Js_lo + As_lo);
            out_c += (Jc_hi + Ac_hi) - (Jc_lo + Ac_lo);
        }
    }
    if (kUpdate) {
        np_new = s_i - out_s;  // mean ion density
        nm_new = c_i - out_c;  // ionic charge
    }
}

// Forces on both fluid components at fluid site i (Sec. II C):
//   Phi^a = -psi^a sum_d w_d chi_a(i+d) c_d + (rho^a/rho) F,   chi_a = G psi^b + G_a+ n+ + G_a- n-
//   Phi^b = -psi^b sum_d w_d G psi^a(i+d) c_d + (rho^b/rho) F
//   F = (1/(2 beta D)) sum_{Q6} sum_+- J c_d  +  ((eps_f - eps_bar)/4) sum_{Q6} E^2(i+d) c_d  +  rho g
// The Kelvin term takes the sign of the discrete total force of Sec. II E and of the Landau
// form that eq. kelvin is derived from (+(eps - eps_bar)/2 grad E^2); eq. kelvin itself
// prints a minus sign.
template <typename T>
__device__ __forceinline__ void site_forces(unsigned i, const Nbr& o, T ra, T rb, const T (&jsum)[3],
                                            const double (&El)[3], const double (&Eh)[3], const Scalars& S,
                                            const Fields<T>& F, const double* phi, T (&Pa)[3], T (&Pb)[3]) {
    const size_t N = S.N;
    const T psa = F.mom[2 * N + i], psb = F.mom[3 * N + i];
    T sa[3] = {0, 0, 0}, sb[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        if (d == kRest) continue;
        const unsigned j = i + offset_of(o, d);
        const T w = T(weight(d));
        const T ta = w * F.mom[4 * N + j];
        const T tb = w * F.mom[2 * N + j];
        if (vx(d) > 0) { sa[0] += ta; sb[0] += tb; }
        if (vx(d) < 0) { sa[0] -= ta; sb[0] -= tb; }
        if (vy(d) > 0) { sa[1] += ta; sb[1] += tb; }
        if (vy(d) < 0) { sa[1] -= ta; sb[1] -= tb; }
        if (vz(d) > 0) { sa[2] += ta; sb[2] += tb; }
        if (vz(d) < 0) { sa[2] -= ta; sb[2] -= tb; }
    }
    const T G = T(S.G);
    T FK[3] = {0, 0, 0};
    if (S.kelvin) {
        // full field vectors at the six neighbours: the component along the link comes
        // from the axis line, the two others from the twelve face-diagonal potentials
        const double ex = S.E_ext[0], ey = S.E_ext[1], ez = S.E_ext[2];
        auto dg = [&](int sx, int sy, int sz) {
            int off = (sx < 0 ? o.xm : (sx > 0 ? o.xp : 0)) + (sy < 0 ? o.ym : (sy > 0 ? o.yp : 0)) +
                      (sz < 0 ? o.zm : (sz > 0 ? o.zp : 0));
            return phi[i + off];
        };
        const double pxpy = dg(1, 1, 0), pxmy = dg(1, -1, 0), mxpy = dg(-1, 1, 0), mxmy = dg(-1, -1, 0);
        const double pxpz = dg(1, 0, 1), pxmz = dg(1, 0, -1), mxpz = dg(-1, 0, 1), mxmz = dg(-1, 0, -1);
        const double pypz = dg(0, 1, 1), pymz = dg(0, 1, -1), mypz = dg(0, -1, 1), mymz = dg(0, -1, -1);
        auto sq = [](double a, double b, double c) { return a * a + b * b + c * c; };
        const double e2_px = sq(Eh[0], -0.5 * (pxpy - pxmy) + ey, -0.5 * (pxpz - pxmz) + ez);
        const double e2_mx = sq(El[0], -0.5 * (mxpy - mxmy) + ey, -0.5 * (mxpz - mxmz) + ez);
        const double e2_py = sq(-0.5 * (pxpy - mxpy) + ex, Eh[1], -0.5 * (pypz - pymz) + ez);
        const double e2_my = sq(-0.5 * (pxmy - mxmy) + ex, El[1], -0.5 * (mypz - mymz) + ez);
        const double e2_pz = sq(-0.5 * (pxpz - mxpz) + ex, -0.5 * (pypz - mypz) + ey, Eh[2]);
        const double e2_mz = sq(-0.5 * (pxmz - mxmz) + ex, -0.5 * (pymz - mymz) + ey, El[2]);
        const T fac = T(0.25) * (eps_fluid<T>(ra, rb, S) - T(S.eps_bar));
        FK[0] = fac * (T)(e2_px - e2_mx);
        FK[1] = fac * (T)(e2_py - e2_my);
        FK[2] = fac * (T)(e2_pz - e2_mz);
    }
    const T rt = ra + rb;
    const T ifr = T(0.5) / (T(S.beta) * T(S.D));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T Frest = jsum[k] * ifr + FK[k] + rt * T(S.g_body[k]);
        Pa[k] = -psa * sa[k] + (ra / rt) * Frest;
        Pb[k] = -psb * (G * sb[k]) + (rb / rt) * Frest;
    }
}

// ------------------------------------------------------------------------------------
// Total force and physical velocity u = u' + (Phi^a + Phi^b) / (2 rho) of every fluid
// site (needed by the donor-cell ion advection of the neighbours).
// ------------------------------------------------------------------------------------
// With particles most sites have no solid D3Q19 neighbour and fluid fraction 1 on their
// axis stencil (flag bits 0, 1 and 3 clear); there the particle path computes exactly what
// the periodic path does (unit fractions, no bounce-back).  Those sites run in the periodic
// kernel, which skips the others; the others (about 1 % of the lattice at the 256^3
// workload's sphere density) run in a second kernel over the list of their indices, so
// the plain sites keep the periodic kernel's registers and occupancy.
constexpr uint8_t kParticlePath = 1u | 2u | 8u;

template <typename T, int G>
__device__ __forceinline__ void force_body(const Scalars& S, const Fields<T>& F, unsigned i) {
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    const size_t N = S.N;
    if (is_solid<T, G>(i, z, S, F)) {
        F.uph[i] = T(0);
        F.uph[N + i] = T(0);
        F.uph[2 * N + i] = T(0);
        return;
    }
    const Nbr o = make_nbr(x, y, z, S);
    const PhiStar P = load_phi_star(i, x, y, z, o, S, F.phi);
    T jsum[3], dp, dm;
    double El[3], Eh[3];
    site_links<T, G, false>(i, z, o, false, P, S, F, jsum, El, Eh, dp, dm);
    const T ra = T(S.rref[0]) + F.mom[i], rb = T(S.rref[1]) + F.mom[N + i];
    T Pa[3], Pb[3];
    site_forces<T>(i, o, ra, rb, jsum, El, Eh, S, F, F.phi, Pa, Pb);
    const T rt2 = T(2) * (ra + rb);
#pragma unroll
    for (int k = 0; k < 3; ++k) F.uph[(size_t)k * N + i] = F.mom[(size_t)(5 + k) * N + i] + (Pa[k] + Pb[k]) / rt2;
}

// G = kColloids: the plain sites of a context with particles (the periodic path).
template <typename T, int G>
__global__ __launch_bounds__(kBlock, kForceOcc<T>) void k_force(Scalars S, Fields<T> F) {
    const unsigned i = site_banded(S);
    if (G == kColloids) {
        if (i >= S.N || (F.flags[i] & kParticlePath) != 0) return;
        force_body<T, kPeriodic>(S, F, i);
    } else {
        force_body<T, G>(S, F, i);
    }
}

// The particle-path sites, from their list.
template <typename T>
__global__ __launch_bounds__(kBlock, kForceOcc<T>) void k_force_part(Scalars S, Fields<T> F) {
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    const unsigned n = F.npl_dev ? (unsigned)*F.npl_dev : (unsigned)F.npl;
    if (t < n) force_body<T, kColloids>(S, F, (unsigned)F.plist[t]);
}

template <typename T> void launch_force(const Scalars& S, const Fields<T>& F, hipStream_t st) {
    const dim3 g(site_blocks(S.N)), b(kBlock);
    if (S.colloids) {  // with moving particles the list is sized by its capacity and read on the device
        hipLaunchKernelGGL((k_force<T, kColloids>), g, b, 0, st, S, F);
        if (F.npl > 0)
            hipLaunchKernelGGL((k_force_part<T>), dim3(site_blocks((unsigned)F.npl)), b, 0, st, S, F);
    } else if (S.walls)
        hipLaunchKernelGGL((k_force<T, kWalls>), g, b, 0, st, S, F);
    else
        hipLaunchKernelGGL((k_force<T, kPeriodic>), g, b, 0, st, S, F);
}

// ------------------------------------------------------------------------------------
// Fused sweep: ion update (all sites), then for fluid sites forces, BGK collision with
// the velocity shift u_e^s = u' + tau Phi^s / rho^s (Sec. II A) and push streaming.
// A population headed into a solid site returns half-way (Sec. II E):
//   g_{d*}(i, t+1) = g*_d(i) - 6 w_d rho^s(i) (c_d . v)      (w_d = w_{d*})
// and, for a particle site, the momentum (2 f*_d - 6 w_d rho^s (c_d . v)) c_d is written
// to the link's record (deterministic per-particle sum later).  The collision reads each
// population only when tau != 1: at tau = 1 the post-collision state is the equilibrium
// of the moments (already in the moment slots), and populations are streamed as written.
// ------------------------------------------------------------------------------------
template <typename T, int G, bool MS = false>
__device__ __forceinline__ void fused_body(const Scalars& S, const Fields<T>& F, unsigned i) {
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    if (G == kWalls && (z == 0 || z == S.nz - 1)) return;  // wall layers hold no ions and no fluid
    const size_t N = S.N;
    const Nbr o = make_nbr(x, y, z, S);
    const bool solid_i = is_solid<T, G>(i, z, S, F);
    const PhiStar P = load_phi_star(i, x, y, z, o, S, F.phi);
    T jsum[3], np_new, nm_new;
    double El[3], Eh[3];
    site_links<T, G, true>(i, z, o, solid_i, P, S, F, jsum, El, Eh, np_new, nm_new);
    F.nn[0][i] = np_new;  // mean ion density
    F.nn[1][i] = nm_new;  // ionic charge
    if (solid_i) return;

    const T da = F.mom[i], db = F.mom[N + i];
    const T ra = T(S.rref[0]) + da, rb = T(S.rref[1]) + db;
    const T u0 = F.mom[5 * N + i], u1 = F.mom[6 * N + i], u2 = F.mom[7 * N + i];
    T Pa[3], Pb[3];
    site_forces<T>(i, o, ra, rb, jsum, El, Eh, S, F, F.phi, Pa, Pb);

    const bool near = G == kColloids ? (F.flags[i] & 2u) != 0 : (G == kWalls && (z == 1 || z == S.nz - 2));
    const int link = (G == kColloids && near && F.linkdp) ? F.linkbase[i] : 0;
    const bool tau1 = S.tau == 1.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T rs = c == 0 ? ra : rb;
        const T dr = c == 0 ? da : db;
        const T P0 = c == 0 ? Pa[0] : Pb[0], P1 = c == 0 ? Pa[1] : Pb[1], P2 = c == 0 ? Pa[2] : Pb[2];
        const T tau = T(S.tau);
        const T ue0 = u0 + tau * P0 / rs, ue1 = u1 + tau * P1 / rs, ue2 = u2 + tau * P2 / rs;
        if (MS) {  // tau = 1 moment state: the density and u_e stand for the post-collision populations
            const typename Vec4<T>::native v = {dr, ue0, ue1, ue2};
            __builtin_nontemporal_store(v, reinterpret_cast<typename Vec4<T>::native*>(F.msn) + (size_t)2 * i + c);
            continue;
        }
        const T usq = usq_of<T>(ue0, ue1, ue2);
        const T* fc = F.f[c];
        T* fo = F.fn[c];
        int lk = link;
        // FP32 exact-mass collision: the post-collision populations must hold exactly the mass
        // the moments pass summed (the FP32 slot plus F.mlo); the rest population takes the
        // remainder of the other 18, kept as an FP32 pair (stored value + F.rlo).  Without it
        // the FP32 rounding of a steady state repeats identically every step and the mass
        // drifts linearly in time.
        const bool xm = sizeof(T) == 4 && F.rlo != nullptr;
        double other = 0.0;
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            const T w = T(weight(d));
            const T geq = geq_dev<T>(d, dr, rs, ue0, ue1, ue2, usq);
            T gs = geq;
            if (!tau1) {
                const T g = __builtin_nontemporal_load(fc + (size_t)d * N + i);
                gs = g - (g - geq) * T(S.inv_tau);
            }
            if (xm) {
                if (d == kRest) continue;
                other += (double)gs;
            }
            const unsigned j = i + offset_of(o, d);
            bool bounce = false;
            if (G != kPeriodic && d != kRest && near) bounce = is_solid<T, G>(j, wrapc(z + vz(d), S.nz), S, F);
            if (bounce) {
                T cv = T(0);
                int own = -1;
                if (G == kColloids) {
                    own = F.owner[j];
                    if (own >= 0)
                        cv = T(vx(d)) * T(F.pv[3 * own]) + T(vy(d)) * T(F.pv[3 * own + 1]) +
                             T(vz(d)) * T(F.pv[3 * own + 2]);
                }
                const T corr = T(6) * w * rs * cv;
                __builtin_nontemporal_store(gs - corr, fo + (size_t)opposite(d) * N + i);
                if (own >= 0 && F.linkdp) {
                    const double dp = 2.0 * ((double)gs + weight(d) * S.rref[c]) - (double)corr;
                    double* rec = F.linkdp + (size_t)lk * 6 + 3 * c;
                    rec[0] = dp * vx(d);
                    rec[1] = dp * vy(d);
                    rec[2] = dp * vz(d);
                    ++lk;
                }
            } else {
                __builtin_nontemporal_store(gs, fo + (size_t)d * N + j);
            }
        }
        if (xm) {
            const double g0 = ((double)dr + (double)F.mlo[(size_t)c * N + i]) - other;
            const T hi = (T)g0;
            __builtin_nontemporal_store(hi, fo + (size_t)kRest * N + i);
            F.rlo[(size_t)c * N + i] = (T)(g0 - (double)hi);
        }
    }
}

// G = kColloids: the plain sites of a context with particles (the periodic path).
template <typename T, int G, bool MS>
__global__ __launch_bounds__(kBlock, kHotOcc<T>) void k_fused(Scalars S, Fields<T> F) {
    const unsigned i = site_banded(S);
    if (G == kColloids) {
        if (i >= S.N || (F.flags[i] & kParticlePath) != 0) return;
        fused_body<T, kPeriodic, MS>(S, F, i);
    } else {
        fused_body<T, G, MS>(S, F, i);
    }
}

// The particle-path sites, from their list: in FP32 three waves per SIMD, where the
// exact-mass collision needs no scratch.
template <typename T> constexpr int kPartOcc = sizeof(T) == 4 ? 3 : kHotOcc<T>;

template <typename T>
__global__ __launch_bounds__(kBlock, kPartOcc<T>) void k_fused_part(Scalars S, Fields<T> F) {
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    const unsigned n = F.npl_dev ? (unsigned)*F.npl_dev : (unsigned)F.npl;
    if (t < n) fused_body<T, kColloids, false>(S, F, (unsigned)F.plist[t]);
}

template <typename T> void launch_fused(const Scalars& S, const Fields<T>& F, hipStream_t st) {
    const dim3 g(site_blocks(S.N)), b(kBlock);
    const bool ms = F.ms != nullptr;  // a moment-state context writes it from the first step on
    if (S.colloids) {  // with moving particles the list is sized by its capacity and read on the device
        hipLaunchKernelGGL((k_fused<T, kColloids, false>), g, b, 0, st, S, F);
        if (F.npl > 0)
            hipLaunchKernelGGL((k_fused_part<T>), dim3(site_blocks((unsigned)F.npl)), b, 0, st, S, F);
    } else if (S.walls && ms)
        hipLaunchKernelGGL((k_fused<T, kWalls, true>), g, b, 0, st, S, F);
    else if (S.walls)
        hipLaunchKernelGGL((k_fused<T, kWalls, false>), g, b, 0, st, S, F);
    else if (ms)
        hipLaunchKernelGGL((k_fused<T, kPeriodic, true>), g, b, 0, st, S, F);
    else
        hipLaunchKernelGGL((k_fused<T, kPeriodic, false>), g, b, 0, st, S, F);
}

// ------------------------------------------------------------------------------------
// Particles (Sec. II E), one workgroup per particle: the momentum handed over by the
// particle's links, q_c E over its sites, the Hertz contact (+k_H delta^{3/2} n, repulsive)
// and lubrication with every other particle, summed per thread and then in a fixed tree
// order; then symplectic Euler (v, then x).  All read the positions and velocities of the
// step's start and write the next buffers, so the particles are independent.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_particle_step(Scalars S, Fields<T> F, int np, const int32_t* link_off,
                                                          const int32_t* link_idx, const int32_t* site_off,
                                                          const int32_t* site_idx, const double* __restrict__ x,
                                                          const double* __restrict__ v, const double* __restrict__ rad,
                                                          double* __restrict__ pF, double* __restrict__ xn,
                                                          double* __restrict__ vn, double rho_p, double k_h, double eta,
                                                          int move) {
    const int a = blockIdx.x;
    double f[3] = {0.0, 0.0, 0.0};
    if (S.reproject) {
        // No link or site lists (the mask moves): the particle's box around its position at
        // the step's start.  Each link from a fluid site i to a site of this particle
        // returned f*_d - corr into i's opposite direction, so f*_d is recovered from it.
        const int B = S.rp_box, B3 = B * B * B;
        const int ox = (int)floor(x[3 * a]) - S.rp_half, oy = (int)floor(x[3 * a + 1]) - S.rp_half,
                  oz = (int)floor(x[3 * a + 2]) - S.rp_half;
        const size_t N = S.N;
        for (int t = threadIdx.x; t < B3; t += blockDim.x) {
            const int sx = wrapc(ox + t % B, S.nx), sy = wrapc(oy + (t / B) % B, S.ny), sz = wrapc(oz + t / (B * B), S.nz);
            const unsigned i = (unsigned)sx + (unsigned)S.nx * ((unsigned)sy + (unsigned)S.ny * (unsigned)sz);
            if (F.owner[i] == a) {
                const double qv = (double)F.qc[i];
                f[0] += qv * efield(0, sx, sy, sz, F.phi, S);
                f[1] += qv * efield(1, sx, sy, sz, F.phi, S);
                f[2] += qv * efield(2, sx, sy, sz, F.phi, S);
            }
            if (F.flags[i] & 1u) continue;
            const Nbr o = make_nbr(sx, sy, sz, S);
            for (int d = 0; d < kQ; ++d) {
                if (d == kRest) continue;
                const unsigned j = i + offset_of(o, d);
                if (!(F.flags[j] & 1u) || F.owner[j] != a) continue;
                const T cv = T(vx(d)) * T(v[3 * a]) + T(vy(d)) * T(v[3 * a + 1]) + T(vz(d)) * T(v[3 * a + 2]);
                for (int c = 0; c < 2; ++c) {
                    const T rs = T(S.rref[c]) + F.mom[(size_t)c * N + i];
                    const T corr = T(6) * T(weight(d)) * rs * cv;
                    const double gs = (double)F.fn[c][(size_t)opposite(d) * N + i] + (double)corr;
                    const double dp = 2.0 * (gs + weight(d) * S.rref[c]) - (double)corr;
                    f[0] += dp * vx(d);
                    f[1] += dp * vy(d);
                    f[2] += dp * vz(d);
                }
            }
        }
    } else {
        for (int t = link_off[a] + threadIdx.x; t < link_off[a + 1]; t += blockDim.x) {
            const double* rec = F.linkdp + (size_t)link_idx[t] * 6;
            f[0] += rec[0] + rec[3];
            f[1] += rec[1] + rec[4];
            f[2] += rec[2] + rec[5];
        }
        for (int t = site_off[a] + threadIdx.x; t < site_off[a + 1]; t += blockDim.x) {
            const unsigned i = (unsigned)site_idx[t];
            int sx, sy, sz;
            site_xyz(i, S, sx, sy, sz);
            const double qv = (double)F.qc[i];
            f[0] += qv * efield(0, sx, sy, sz, F.phi, S);
            f[1] += qv * efield(1, sx, sy, sz, F.phi, S);
            f[2] += qv * efield(2, sx, sy, sz, F.phi, S);
        }
    }
    const int L[3] = {S.nx, S.ny, S.nz};
    for (int b = threadIdx.x; b < np; b += blockDim.x) {
        if (b == a) continue;
        double dv[3], d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            dv[k] = min_image(x[3 * a + k] - x[3 * b + k], L[k]);
            d2 += dv[k] * dv[k];
        }
        const double dist = sqrt(d2);
        if (!(dist > 0.0)) continue;
        const double nh[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
        const double delta = rad[a] + rad[b] - dist;
        if (delta > 0.0) {
            const double fh = k_h * pow(delta, 1.5);
            for (int k = 0; k < 3; ++k) f[k] += fh * nh[k];
        }
        const double gap = dist - rad[a] - rad[b];
        if (gap < 2.0 / 3.0 && gap > 0.0) {
            const double rp = 0.5 * (rad[a] + rad[b]);
            double nv = 0.0;
            for (int k = 0; k < 3; ++k) nv += nh[k] * (v[3 * a + k] - v[3 * b + k]);
            const double fl = -1.5 * M_PI * eta * rp * rp * nv * (1.0 / gap - 1.0);
            for (int k = 0; k < 3; ++k) f[k] += fl * nh[k];
        }
    }
    __shared__ double sm[3][kBlock];
    for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] = f[k];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = rho_p * (4.0 / 3.0) * M_PI * rad[a] * rad[a] * rad[a];
        for (int k = 0; k < 3; ++k) {
            const double Fk = sm[k][0];
            pF[3 * a + k] = Fk;
            const double vv = move ? v[3 * a + k] + Fk / m : v[3 * a + k];
            vn[3 * a + k] = vv;
            xn[3 * a + k] = move ? x[3 * a + k] + vv : x[3 * a + k];
        }
    }
}

template <typename T>
void launch_particle_step(const Scalars& S, const Fields<T>& F, int np, const int32_t* link_off,
                          const int32_t* link_idx, const int32_t* site_off, const int32_t* site_idx, const double* x,
                          const double* v, const double* r, double* pF, double* xn, double* vn, double rho_p,
                          double k_h, double eta, int move, hipStream_t st) {
    if (np <= 0) return;
    hipLaunchKernelGGL(k_particle_step<T>, dim3(np), dim3(kBlock), 0, st, S, F, np, link_off, link_idx, site_off,
                       site_idx, x, v, r, pF, xn, vn, rho_p, k_h, eta, move);
}

// ------------------------------------------------------------------------------------
// Observables: FP64 partial sums of mass, ions, charge, momentum; max |u|; counts of
// non-finite values and negative ion densities.
// ------------------------------------------------------------------------------------
// The observables of one site, added into v: [0, 1] rho^a, rho^b (fluid sites), [2, 3] n+, n-,
// [4] charge, [5..7] momentum, [8] |u| (the caller keeps the maximum), [9] non-finite
// values, [10] negative ion densities.
template <typename T, int PM>
__device__ __forceinline__ void observe_site(const Scalars& S, const Fields<T>& F, unsigned i, double (&v)[11]) {
#pragma clang fp contract(off)  // gathered populations rounded as stored ones (see moments_body)
    int x, y, z;
    site_xyz(i, S, x, y, z);
    const double is_ = (double)F.n[0][i], ic_ = (double)F.n[1][i];
    const double np_ = is_ + 0.5 * ic_, nm_ = is_ - 0.5 * ic_;
    v[2] += np_;
    v[3] += nm_;
    v[4] += np_ - nm_ + (S.colloids ? (double)F.qc[i] : 0.0);
    int bad = !isfinite(np_) || !isfinite(nm_);
    v[10] += (np_ < 0.0) + (nm_ < 0.0);
    if (!solid_at(i, z, S, F)) {
        double sa = 0, sb = 0, m[3] = {0, 0, 0};
        const Nbr o = make_nbr(x, y, z, S);
        MsSite<T> own0{}, own1{};
        if (PM == 1) {
            own0 = ms_site<T>(S, F, 0, i);
            own1 = ms_site<T>(S, F, 1, i);
        }
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            double a = PM == 0 ? (double)F.f[0][(size_t)d * S.N + i]
                               : (double)arriving<T, PM>(S, F, 0, d, i, z, o, own0);
            double b = PM == 0 ? (double)F.f[1][(size_t)d * S.N + i]
                               : (double)arriving<T, PM>(S, F, 1, d, i, z, o, own1);
            if (PM == 0 && d == kRest && F.rlo) {  // the rest population's low part
                a = a + (double)F.rlo[i];
                b = b + (double)F.rlo[(size_t)S.N + i];
            }
            bad |= !isfinite(a) || !isfinite(b);
            sa += a;
            sb += b;
            m[0] += (a + b) * vx(d);
            m[1] += (a + b) * vy(d);
            m[2] += (a + b) * vz(d);
        }
        const double ra = S.rref[0] + sa, rb = S.rref[1] + sb;
        v[0] += ra;
        v[1] += rb;
        v[5] += m[0];
        v[6] += m[1];
        v[7] += m[2];
        v[8] = fmax(v[8], sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / (ra + rb));
    }
    v[9] += bad;
}

template <typename T, int PM>
__global__ __launch_bounds__(kBlock) void k_observe(Scalars S, Fields<T> F) {
    const unsigned i = xcd_linear();
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < S.N) observe_site<T, PM>(S, F, i, v);
    const bool mx[11] = {false, false, false, false, false, false, false, false, true, false, false};
    block_reduce_store<11>(v, mx, F.red, blockIdx.x, gridDim.x);
}

// The same sums from a fixed grid of workgroups striding over the lattice, with the partial
// sums in `red` (11 x gridDim.x doubles): the scratch does not grow with the lattice.
template <typename T, int PM>
__global__ __launch_bounds__(kBlock) void k_observe_strided(Scalars S, Fields<T> F, double* red) {
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < S.N; i += gridDim.x * kBlock)
        observe_site<T, PM>(S, F, i, v);
    const bool mx[11] = {false, false, false, false, false, false, false, false, true, false, false};
    block_reduce_store<11>(v, mx, red, blockIdx.x, gridDim.x);
}

template <typename T> void launch_observe(const Scalars& S, const Fields<T>& F, unsigned nblk, hipStream_t st) {
    const int pm = pop_mode(F);
    if (pm == 0)
        hipLaunchKernelGGL((k_observe<T, 0>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else if (pm == 1)
        hipLaunchKernelGGL((k_observe<T, 1>), dim3(nblk), dim3(kBlock), 0, st, S, F);
    else
        hipLaunchKernelGGL((k_observe<T, 2>), dim3(nblk), dim3(kBlock), 0, st, S, F);
}

template <typename T>
void launch_observe_strided(const Scalars& S, const Fields<T>& F, unsigned nblk, double* red, hipStream_t st) {
    const int pm = pop_mode(F);
    if (pm == 0)
        hipLaunchKernelGGL((k_observe_strided<T, 0>), dim3(nblk), dim3(kBlock), 0, st, S, F, red);
    else if (pm == 1)
        hipLaunchKernelGGL((k_observe_strided<T, 1>), dim3(nblk), dim3(kBlock), 0, st, S, F, red);
    else
        hipLaunchKernelGGL((k_observe_strided<T, 2>), dim3(nblk), dim3(kBlock), 0, st, S, F, red);
}

// Relative residuals of a solve run without a host read-back, kept on the device: the start
// (scal[24], scal[25]) and end (scal[1], scal[2]) sums of squares give scal[30] and scal[29];
// scal[28] keeps the largest end value since it was last cleared.
__global__ void k_track_residual(double* scal) {
    if (threadIdx.x != 0) return;
    const double rel = scal[2] > 0.0 ? sqrt(scal[1] / scal[2]) : 0.0;
    const double rel0 = scal[25] > 0.0 ? sqrt(scal[24] / scal[25]) : 0.0;
    scal[29] = rel;
    scal[30] = rel0;
    scal[28] = fmax(scal[28], rel);
}

void launch_track_residual(double* scal, hipStream_t st) {
    hipLaunchKernelGGL(k_track_residual, dim3(1), dim3(64), 0, st, scal);
}

// Populations of component c at time t (FP64, f_d = g_d + w_d rho_ref, velocity-major) of a
// moment-state context, gathered as in the moments pass; solid sites hold w_d rho_ref.
template <typename T, int PM>
__global__ __launch_bounds__(kBlock) void k_export_pop(Scalars S, Fields<T> F, int c, double* out) {
#pragma clang fp contract(off)  // as the population export: the stored value plus w_d rho_ref
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    const bool solid = solid_at(i, z, S, F);
    const Nbr o = make_nbr(x, y, z, S);
    MsSite<T> own{};
    if (PM == 1 && !solid) own = ms_site<T>(S, F, c, i);
#pragma unroll
    for (int d = 0; d < kQ; ++d) {
        const double g = solid ? 0.0 : (double)arriving<T, PM>(S, F, c, d, i, z, o, own);
        out[(size_t)d * S.N + i] = g + weight(d) * S.rref[c];
    }
}

template <typename T> void launch_export_pop(const Scalars& S, const Fields<T>& F, int c, double* out, hipStream_t st) {
    if (pop_mode(F) == 1)
        hipLaunchKernelGGL((k_export_pop<T, 1>), dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, c, out);
    else
        hipLaunchKernelGGL((k_export_pop<T, 2>), dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, c, out);
}

// dst[i] += lo[i] (FP64): the low part of the FP32 rest population, added to its export.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_lo(const T* __restrict__ lo, double* __restrict__ dst, unsigned n) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = dst[i] + (double)lo[i];
}

template <typename T> void launch_add_lo(const T* lo, double* dst, unsigned n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_lo<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, lo, dst, n);
}

// ------------------------------------------------------------------------------------
// Initialisation and export
// ------------------------------------------------------------------------------------
// f = f~(rho, u = 0) = w_d rho on fluid sites, stored as g_d = w_d (rho - rho_ref).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_pop(Scalars S, T* f, const double* rho, double rref,
                                                      const uint8_t* flags) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    const int z = site_z(i, S);
    const bool solid = S.colloids ? (flags[i] & 1u) != 0 : wall_layer(z, S);
    const double dr = solid ? 0.0 : rho[i] - rref;
#pragma unroll
    for (int d = 0; d < kQ; ++d) f[(size_t)d * S.N + i] = (T)(storage_weight<T>(d) * dr);
}

// Ions are stored as the mean density s = (n+ + n-)/2 and the ionic charge c = n+ - n-
// (both scaled by the fluid fraction at set-up), so that the charge keeps its own
// relative precision in FP32 however large the salt concentration.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_ions(Scalars S, Fields<T> F, T* ion_s, T* ion_c, const double* np_,
                                                      const double* nm_) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    const int z = site_z(i, S);
    const double pf = (double)psif_at(i, z, S, F);
    ion_s[i] = (T)(0.5 * (np_[i] + nm_[i]) * pf);
    ion_c[i] = (T)((np_[i] - nm_[i]) * pf);
}

template <typename T>
void launch_init_ions(const Scalars& S, const Fields<T>& F, T* ion_s, T* ion_c, const double* np_, const double* nm_,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_init_ions<T>, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, ion_s, ion_c, np_, nm_);
}

// n+ (sign = +1) or n- (sign = -1) in double from the stored mean and charge
template <typename T>
__global__ void k_ion_species(const T* __restrict__ ion_s, const T* __restrict__ ion_c, double* __restrict__ dst,
                              unsigned n, double sign) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)ion_s[i] + sign * 0.5 * (double)ion_c[i];
}

template <typename T>
void launch_ion_species(const T* ion_s, const T* ion_c, double* dst, unsigned n, double sign, hipStream_t st) {
    hipLaunchKernelGGL(k_ion_species<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, ion_s, ion_c, dst, n,
                       sign);
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ src, double* __restrict__ dst, unsigned n, double add) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i] + add;
}

template <typename T> void launch_to_double(const T* src, double* dst, unsigned n, double add, hipStream_t st) {
    hipLaunchKernelGGL(k_to_double<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, src, dst, n, add);
}

template <typename T>
__global__ void k_upload(T* __restrict__ dst, const double* __restrict__ src, unsigned n) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (T)src[i];
}

template <typename T> void launch_upload(T* dst, const double* src, unsigned n, hipStream_t st) {
    hipLaunchKernelGGL(k_upload<T>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, dst, src, n);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_field_e(Scalars S, Fields<T> F, int k, double* dst) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    dst[i] = efield(k, x, y, z, F.phi, S);
}

template <typename T> void launch_field_e(const Scalars& S, const Fields<T>& F, int k, double* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_field_e<T>, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, k, dst);
}

// explicit instantiations
#define EK_INST(T)                                                                                              \
    template void launch_moments<T>(const Scalars&, const Fields<T>&, unsigned, hipStream_t);                  \
    template void launch_virtual<T>(const Scalars&, const Fields<T>&, hipStream_t);                            \
    template void launch_sor<T>(const Scalars&, const Fields<T>&, int, double, bool, hipStream_t);             \
    template void launch_residual<T>(const Scalars&, const Fields<T>&, unsigned, bool, double*, T*, hipStream_t); \
    template void launch_phi_finalize<T>(const Scalars&, const Fields<T>&, int, const double*, hipStream_t);   \
    template void launch_force<T>(const Scalars&, const Fields<T>&, hipStream_t);                              \
    template void launch_fused<T>(const Scalars&, const Fields<T>&, hipStream_t);                              \
    template void launch_export_pop<T>(const Scalars&, const Fields<T>&, int, double*, hipStream_t);           \
    template void launch_particle_step<T>(const Scalars&, const Fields<T>&, int, const int32_t*, const int32_t*,  \
                                          const int32_t*, const int32_t*, const double*, const double*, const double*, \
                                          double*, double*, double*, double, double, double, int, hipStream_t);                \
    template void launch_observe<T>(const Scalars&, const Fields<T>&, unsigned, hipStream_t);                  \
    template void launch_add_lo<T>(const T*, double*, unsigned, hipStream_t);                  \
    template void launch_observe_strided<T>(const Scalars&, const Fields<T>&, unsigned, double*, hipStream_t);                  \
    template void launch_init_ions<T>(const Scalars&, const Fields<T>&, T*, T*, const double*, const double*,  \
                                      hipStream_t);                                                             \
    template void launch_ion_species<T>(const T*, const T*, double*, unsigned, double, hipStream_t);           \
    template void launch_to_double<T>(const T*, double*, unsigned, double, hipStream_t);                       \
    template void launch_field_e<T>(const Scalars&, const Fields<T>&, int, double*, hipStream_t);              \
    template void launch_upload<T>(T*, const double*, unsigned, hipStream_t);                               \
    template void launch_mg_coarsen_fine<T>(const Scalars&, const Fields<T>&, const MGLevel&, hipStream_t);    \
    template void launch_mg_restrict_fine<T>(const Scalars&, const Fields<T>&, const MGLevel&, bool, double,      \
                                             hipStream_t);                                                       \
    template void launch_mg_prolong_fine<T>(const Scalars&, const Fields<T>&, const MGLevel&, bool, hipStream_t); \
    template void launch_mg_prolong_red_fine<T>(const Scalars&, const Fields<T>&, const MGLevel&, double, double*, \
                                                hipStream_t);                                                      \
    template void launch_sor_black_from<T>(const Scalars&, const Fields<T>&, double, const double*, hipStream_t); \
    template void launch_sor_rb<T>(const Scalars&, const Fields<T>&, const double*, double*, double, hipStream_t);

EK_INST(float)
EK_INST(double)


// ------------------------------------------------------------------------------------
// Batched replicas: the same bodies, one launch per stage for every replica.  Each
// workgroup finds its replica and its workgroup index inside that replica in a block
// table; the replica's parameters and pointers come from a descriptor in device memory
// (uniform per workgroup, so they are read through the scalar cache).  Batched
// replicas are periodic without particles.
// ------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void kb_moments(const RepDesc<T>* __restrict__ D, const BlockRef* __restrict__ tab) {
    const BlockRef e = tab[blockIdx.x];
    const RepDesc<T>& R = D[e.rep];
    double v[1] = {moments_body<T, kPeriodic>(R.S, R.F, (unsigned)e.blk * kBlock + threadIdx.x)};
    const bool mx[1] = {false};
    block_reduce_store<1>(v, mx, R.F.red, e.blk, (R.S.N + kBlock - 1) / kBlock);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_residual(const RepDesc<T>* __restrict__ D, const BlockRef* __restrict__ tab) {
    const BlockRef e = tab[blockIdx.x];
    const RepDesc<T>& R = D[e.rep];
    double v[3];
    residual_body<T>(R.S, R.F, (unsigned)e.blk * kBlock + threadIdx.x, v);
    const bool mx[3] = {false, false, false};
    block_reduce_store<3>(v, mx, R.F.red, e.blk, (R.S.N + kBlock - 1) / kBlock);
}

template <typename T>
__global__ __launch_bounds__(kBlock, kForceOcc<T>) void kb_force(const RepDesc<T>* __restrict__ D,
                                                               const BlockRef* __restrict__ tab) {
    const BlockRef e = tab[blockIdx.x];
    const RepDesc<T>& R = D[e.rep];
    force_body<T, kPeriodic>(R.S, R.F, (unsigned)e.blk * kBlock + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBlock, kHotOcc<T>) void kb_fused(const RepDesc<T>* __restrict__ D,
                                                               const BlockRef* __restrict__ tab) {
    const BlockRef e = tab[blockIdx.x];
    const RepDesc<T>& R = D[e.rep];
    fused_body<T, kPeriodic>(R.S, R.F, (unsigned)e.blk * kBlock + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_misc(const RepDesc<T>* __restrict__ D, const BlockRef* __restrict__ tab,
                                                  int op, int grid, int color) {
    const BlockRef e = tab[blockIdx.x];
    const RepDesc<T>& R = D[e.rep];
    const unsigned t = (unsigned)e.blk * kBlock + threadIdx.x;
    switch (op) {
        case kB_EXTRAPOLATE: extrapolate_body(R.S, R.F.phi, R.phi_prev, t); break;
        case kB_FINALIZE: finalize_body(R.S, R.F.phi, R.F.scal, 0, t); break;
        case kB_PROLONG_FINE: prolong_fine_body<T>(R.S, R.F, R.mg[0], t); break;
        case kB_SOR: sor_body<T>(R.S, R.F, t, color, R.smooth_omega); break;
        case kB_COARSEN_FINE:
            if (t < R.mg[0].n) coarsen_fine_body<T>(R.S, R.F, R.mg[0], t);
            break;
        case kB_COARSEN:
            if (t < R.mg[grid - 1].n) coarsen_body(R.mg[grid - 2], R.mg[grid - 1], t);
            break;
        case kB_RESTRICT_FINE:
            if (t < R.mg[0].n) restrict_fine_body<T>(R.S, R.F, R.mg[0], t);
            break;
        case kB_RESTRICT:
            if (t < R.mg[grid].n) restrict_body(R.mg[grid - 1], R.mg[grid], t);
            break;
        case kB_SMOOTH:
            if (t < R.mg[grid - 1].n / 2) smooth_body(R.mg[grid - 1], color, R.smooth_omega, t);
            break;
        case kB_PROLONG:
            if (t < R.mg[grid - 1].n) prolong_body(R.mg[grid], R.mg[grid - 1], t);
            break;
        default: break;
    }
}

template <typename T>
void launch_batch(BatchOp op, const RepDesc<T>* D, const BlockRef* tab, unsigned nblocks, int grid, int color,
                  hipStream_t st) {
    if (nblocks == 0) return;
    const dim3 g(nblocks), b(kBlock);
    switch (op) {
        case kB_MOMENTS: hipLaunchKernelGGL(kb_moments<T>, g, b, 0, st, D, tab); break;
        case kB_RESIDUAL: hipLaunchKernelGGL(kb_residual<T>, g, b, 0, st, D, tab); break;
        case kB_FORCE: hipLaunchKernelGGL(kb_force<T>, g, b, 0, st, D, tab); break;
        case kB_FUSED: hipLaunchKernelGGL(kb_fused<T>, g, b, 0, st, D, tab); break;
        default: hipLaunchKernelGGL(kb_misc<T>, g, b, 0, st, D, tab, (int)op, grid, color); break;
    }
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void kb_source_mean(const RepDesc<T>* __restrict__ D) {
    const RepDesc<T>& R = D[blockIdx.x];
    source_mean_body(R.S, R.F.red, (R.S.N + kBlock - 1) / kBlock, R.F.scal);
}

template <typename T> void launch_batch_source_mean(const RepDesc<T>* D, int n_rep, hipStream_t st) {
    hipLaunchKernelGGL(kb_source_mean<T>, dim3(n_rep), dim3(kRedThreads), 0, st, D);
}

// Per replica: residual sums -> scal[1..3], relative residual -> scal[4], its running
// maximum -> scal[5].
template <typename T>
__global__ __launch_bounds__(kRedThreads) void kb_reduce(const RepDesc<T>* __restrict__ D) {
    const RepDesc<T>& R = D[blockIdx.x];
    const unsigned nblk = (R.S.N + kBlock - 1) / kBlock;
    __shared__ double sm[kRedThreads];
    double tot[3];
    for (int k = 0; k < 3; ++k) {
        double a = 0.0;
        for (unsigned b = threadIdx.x; b < nblk; b += kRedThreads) a += R.F.red[(size_t)k * nblk + b];
        sm[threadIdx.x] = a;
        __syncthreads();
        for (int s2 = kRedThreads / 2; s2 > 0; s2 >>= 1) {
            if ((int)threadIdx.x < s2) sm[threadIdx.x] += sm[threadIdx.x + s2];
            __syncthreads();
        }
        tot[k] = sm[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* sc = R.F.scal;
        sc[1] = tot[0];
        sc[2] = tot[1];
        sc[3] = tot[2];
        const double rel = tot[1] > 0.0 ? sqrt(tot[0] / tot[1]) : 0.0;
        sc[4] = rel;
        sc[5] = fmax(sc[5], rel);
    }
}

template <typename T> void launch_batch_reduce(const RepDesc<T>* D, int n_rep, hipStream_t st) {
    hipLaunchKernelGGL(kb_reduce<T>, dim3(n_rep), dim3(kRedThreads), 0, st, D);
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void kb_tail(const RepDesc<T>* __restrict__ D) {
    const RepDesc<T>& R = D[blockIdx.x];
    const int nl = R.nl;
    tail_body(R.tail_mid ? R.mg[nl - 2] : R.mg[nl - 1], R.mg[nl - 1], R.tail_mid, R.coarse_iters, R.coarse_omega,
              R.mid_pre, R.mid_post, R.smooth_omega);
}

template <typename T> void launch_batch_tail(const RepDesc<T>* D, int n_rep, hipStream_t st) {
    hipLaunchKernelGGL(kb_tail<T>, dim3(n_rep), dim3(kTailThreads), mg_tail_lds_bytes(), st, D);
}

#define EK_BATCH_INST(T)                                                                                          \
    template void launch_batch<T>(BatchOp, const RepDesc<T>*, const BlockRef*, unsigned, int, int, hipStream_t); \
    template void launch_batch_source_mean<T>(const RepDesc<T>*, int, hipStream_t);                             \
    template void launch_batch_reduce<T>(const RepDesc<T>*, int, hipStream_t);                                  \
    template void launch_batch_tail<T>(const RepDesc<T>*, int, hipStream_t);

EK_BATCH_INST(float)
EK_BATCH_INST(double)

// population initialisation needs the flags pointer, exposed separately
template <typename T>
void launch_init_pop_flags(const Scalars& S, T* f, const double* rho, double rref, const uint8_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_init_pop<T>, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, f, rho, rref, flags);
}
template void launch_init_pop_flags<float>(const Scalars&, float*, const double*, double, const uint8_t*, hipStream_t);
template void launch_init_pop_flags<double>(const Scalars&, double*, const double*, double, const uint8_t*,
                                            hipStream_t);

}  // namespace ek
