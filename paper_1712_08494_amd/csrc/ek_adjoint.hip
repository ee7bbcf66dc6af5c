// Adjoint (reverse mode) of one coupled lattice step on a periodic FP64 lattice without
// particles: given dL/d(state at t+1), produce dL/d(state at t) and accumulate the
// gradient with respect to E_ext, eps_a, eps_b and G.
//
// The forward step (Sec. II A-D) at each site, with everything read at time t:
//   rho^s = sum_d f^s_d,  u' = sum_s sum_d f^s_d c_d / rho,  psi^s = rho0 (1 - e^{-rho^s/rho0})
//   q = n+ - n-,  eps = (eps_a (1 - c) + eps_b (1 + c)) / 2,  c = (rho^b - rho^a) / rho
//   M phi = q - mean(q) (M = -div eps grad, face eps the mean of two sites), mean(phi) = 0
//   E = -grad phi + E_ext (central differences)
//   J+- on the D3Q7 links (diffusion, migration, solvation), A+- donor-cell advection by
//   the physical velocity U = u' + (Phi^a + Phi^b) / (2 rho)
//   Phi^a = -psi^a S^a + (rho^a / rho) F,  Phi^b = -psi^b G S^b + (rho^b / rho) F,
//   S^a = sum_d w_d chi_a(i+d) c_d, S^b = sum_d w_d psi^a(i+d) c_d, chi_a = G psi^b + G+ n+ + G- n-,
//   F = (1 / (2 beta D)) sum_{Q6} sum_+- J c_d + ((eps - eps_bar)/4) sum_{Q6} |E(i+d)|^2 c_d + rho g
//   n(t+1) = n - sum_{Q6} (J + A),  f* = f - (f - f~(rho^s, u' + tau Phi^s / rho^s)) / tau,
//   f(i + c_d, t+1) = f*_d(i)
// The reverse step transposes these in the opposite order.  Gather form throughout (no
// atomics): a site's sensitivity collects the terms of every stencil that reads it, so
// stencil outputs (the Shan-Chen sums, the force F, the field E) are materialised first
// and gathered by the next pass:
//   k_adj_force : transposes of streaming, collision, ion update + advection, physical
//                 velocity and the force assembly at the site
//   k_adj_links : transposed Shan-Chen stencils, link fluxes (with the friction force) and
//                 the Kelvin force's field dependence
//   k_adj_rhs   : transposed central difference: dL/dphi, the adjoint Poisson source
//   (host)      : the adjoint Poisson equation M mu = dL/dphi (M is symmetric: the same
//                 multigrid solver); the potential is the implicit solution, so its
//                 derivative is -M^{-1} times the derivative of the residual
//   k_adj_final : permittivity and charge terms of the Poisson equation, the moments,
//                 and dL/df, dL/dn at time t
#include "ek_device.h"

namespace ek {

namespace {

constexpr double kZ[2] = {1.0, -1.0};  // valence of n+, n-

// n+ and n- at a site from the stored mean density and charge
__device__ __forceinline__ void species_at(const Fields<double>& F, unsigned j, double (&n)[2]) {
    const double s = F.n[0][j], c = F.n[1][j];
    n[0] = s + 0.5 * c;
    n[1] = s - 0.5 * c;
}

__device__ __forceinline__ double efield_at(int k, unsigned j, const double* phi, const Scalars& S) {
    int x, y, z;
    site_xyz(j, S, x, y, z);
    return efield(k, x, y, z, phi, S);
}

__device__ __forceinline__ double efield_sq_at(unsigned j, const double* phi, const Scalars& S) {
    int x, y, z;
    site_xyz(j, S, x, y, z);
    return efield_sq(x, y, z, phi, S);
}

__device__ __forceinline__ int axis_off(const Nbr& o, int k, int sgn) {
    return k == 0 ? (sgn < 0 ? o.xm : o.xp) : (k == 1 ? (sgn < 0 ? o.ym : o.yp) : (sgn < 0 ? o.zm : o.zp));
}

// Adds the workgroup sums of NV values to gred[blockIdx.x][base .. base + NV): each
// workgroup owns its record, so the accumulation over reverse steps is deterministic.
template <int NV>
__device__ __forceinline__ void block_sum_add(double (&v)[NV], double* gred, int base) {
    __shared__ double sm[NV][kBlock / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = v[k];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) a += __shfl_down(a, s, 64);
        if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = sm[k][0];
            for (int w = 1; w < kBlock / 64; ++w) a += sm[k][w];
            gred[(size_t)(base + k) * gridDim.x + blockIdx.x] += a;
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------------------
// Pass 1: streaming, collision, ion update, advection, physical velocity and force
// assembly, transposed at each site.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_force(Scalars S, Fields<double> F, AdjFields A) {
    const unsigned i = xcd_linear();
    double red[2] = {0.0, 0.0};  // eps_bar, G
    if (i < S.N) {
        const size_t N = S.N;
        int x, y, z;
        site_xyz(i, S, x, y, z);
        const Nbr o = make_nbr(x, y, z, S);
        const double ra = S.rref[0] + F.mom[i], rb = S.rref[1] + F.mom[N + i], rt = ra + rb;
        const double psa = F.mom[2 * N + i], psb = F.mom[3 * N + i];
        const double u[3] = {F.mom[5 * N + i], F.mom[6 * N + i], F.mom[7 * N + i]};
        const double U[3] = {F.uph[i], F.uph[N + i], F.uph[2 * N + i]};
        double ni[2];
        species_at(F, i, ni);
        const double kap[2] = {S.kap_p, S.kap_m};

        // forward force at the site
        double sa[3] = {0, 0, 0}, sb[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            if (d == kRest) continue;
            const unsigned j = i + offset_of(o, d);
            const double w = weight(d);
            const double ta = w * F.mom[4 * N + j], tb = w * F.mom[2 * N + j];
            sa[0] += vx(d) * ta; sa[1] += vy(d) * ta; sa[2] += vz(d) * ta;
            sb[0] += vx(d) * tb; sb[1] += vy(d) * tb; sb[2] += vz(d) * tb;
        }
        const double rai = F.mom[i];
        const double ef = 0.5 * (S.eps_a * (1.0 - (rb - ra) / rt) + S.eps_b * (1.0 + (rb - ra) / rt));
        double Fr[3], dK[3];
        for (int k = 0; k < 3; ++k) {
            const unsigned lo = i + axis_off(o, k, -1), hi = i + axis_off(o, k, 1);
            const double Ei = efield(k, x, y, z, F.phi, S);
            const double El = efield_at(k, lo, F.phi, S), Eh = efield_at(k, hi, F.phi, S);
            double nl[2], nh[2];
            species_at(F, lo, nl);
            species_at(F, hi, nh);
            const double ral = F.mom[lo], rah = F.mom[hi];
            double js = 0.0;
            for (int sp = 0; sp < 2; ++sp) {
                const double Jh = -S.D * ((nh[sp] - ni[sp]) - 0.25 * S.beta * kZ[sp] * (ni[sp] + nh[sp]) * (Ei + Eh) +
                                          kap[sp] * (ni[sp] + nh[sp]) * (rah - rai));
                const double Jl = -S.D * ((ni[sp] - nl[sp]) - 0.25 * S.beta * kZ[sp] * (nl[sp] + ni[sp]) * (El + Ei) +
                                          kap[sp] * (nl[sp] + ni[sp]) * (rai - ral));
                js += Jh + Jl;
            }
            dK[k] = efield_sq_at(hi, F.phi, S) - efield_sq_at(lo, F.phi, S);
            Fr[k] = js / (2.0 * S.beta * S.D) + 0.25 * (ef - S.eps_bar) * dK[k] + rt * S.g_body[k];
        }
        double P[2][3];
        for (int k = 0; k < 3; ++k) {
            P[0][k] = -psa * sa[k] + (ra / rt) * Fr[k];
            P[1][k] = -psb * (S.G * sb[k]) + (rb / rt) * Fr[k];
        }

        // collision and streaming: dL/df*_d(i) = dL/df_d(i + c_d, t+1)
        double lrho[2], lu[3] = {0, 0, 0}, lP[2][3];
        for (int c = 0; c < 2; ++c) {
            const double rs = c == 0 ? ra : rb;
            double ue[3];
            for (int k = 0; k < 3; ++k) ue[k] = u[k] + S.tau * P[c][k] / rs;
            const double usq = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
            double lr = 0.0, lue[3] = {0, 0, 0};
            const double* lfc = A.lf[c];
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                const double leq = S.inv_tau * lfc[(size_t)d * N + i + offset_of(o, d)];
                const double cu = vx(d) * ue[0] + vy(d) * ue[1] + vz(d) * ue[2];
                const double w = weight(d);
                lr += leq * w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                const double g = leq * w * rs;
                lue[0] += g * (3.0 * vx(d) + 9.0 * cu * vx(d) - 3.0 * ue[0]);
                lue[1] += g * (3.0 * vy(d) + 9.0 * cu * vy(d) - 3.0 * ue[1]);
                lue[2] += g * (3.0 * vz(d) + 9.0 * cu * vz(d) - 3.0 * ue[2]);
            }
            lrho[c] = lr - S.tau * (lue[0] * P[c][0] + lue[1] * P[c][1] + lue[2] * P[c][2]) / (rs * rs);
            for (int k = 0; k < 3; ++k) {
                lu[k] += lue[k];
                lP[c][k] = S.tau * lue[k] / rs;
            }
        }

        // ion update n(t+1) = n - sum (J + A) and the donor-cell advection
        double ln_i[2] = {A.ln[0][i], A.ln[1][i]};
        double an[2] = {ln_i[0], ln_i[1]};
        double lU[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) {
            const unsigned lo = i + axis_off(o, k, -1), hi = i + axis_off(o, k, 1);
            const double up = U[k] > 0.0 ? U[k] : 0.0, um = U[k] < 0.0 ? -U[k] : 0.0;
            for (int sp = 0; sp < 2; ++sp) {
                const double lFh = A.ln[sp][hi] - ln_i[sp];  // the link (i, i + e_k)
                const double lFl = ln_i[sp] - A.ln[sp][lo];  // the link (i - e_k, i)
                an[sp] += lFh * up - lFl * um;
                lU[k] += ni[sp] * ((U[k] > 0.0 ? lFh : 0.0) + (U[k] < 0.0 ? lFl : 0.0));
            }
        }
        // physical velocity U = u' + (Phi^a + Phi^b) / (2 rho)
        double lUP = 0.0;
        for (int k = 0; k < 3; ++k) {
            lu[k] += lU[k];
            lP[0][k] += lU[k] / (2.0 * rt);
            lP[1][k] += lU[k] / (2.0 * rt);
            lUP += lU[k] * (P[0][k] + P[1][k]);
        }
        lrho[0] -= lUP / (2.0 * rt * rt);
        lrho[1] -= lUP / (2.0 * rt * rt);

        // force assembly
        double lpsa = 0.0, lpsb = 0.0, leps = 0.0;
        for (int k = 0; k < 3; ++k) {
            lpsa -= lP[0][k] * sa[k];
            lpsb -= lP[1][k] * S.G * sb[k];
            A.aS[(size_t)k * N + i] = -psa * lP[0][k];
            A.aS[(size_t)(3 + k) * N + i] = -psb * S.G * lP[1][k];
            const double lF = (ra * lP[0][k] + rb * lP[1][k]) / rt;
            A.aF[(size_t)k * N + i] = lF;
            red[1] += lP[1][k] * (-psb * sb[k]);
            lrho[0] += Fr[k] * rb * (lP[0][k] - lP[1][k]) / (rt * rt) + lF * S.g_body[k];
            lrho[1] += Fr[k] * ra * (lP[1][k] - lP[0][k]) / (rt * rt) + lF * S.g_body[k];
            leps += 0.25 * lF * dK[k];
            red[0] -= 0.25 * lF * dK[k];
        }
        lrho[0] += lpsa * exp(-ra / S.rho0);
        lrho[1] += lpsb * exp(-rb / S.rho0);
        A.arho[i] = lrho[0];
        A.arho[N + i] = lrho[1];
        for (int k = 0; k < 3; ++k) A.au[(size_t)k * N + i] = lu[k];
        A.an[i] = an[0];
        A.an[N + i] = an[1];
        A.aeps[i] = leps;
    }
    block_sum_add<2>(red, A.gred, kAdjEbar);
}

// ------------------------------------------------------------------------------------
// Pass 2: transposed Shan-Chen stencils, link fluxes and the Kelvin force's dependence on
// the field at the neighbours.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_links(Scalars S, Fields<double> F, AdjFields A) {
    const unsigned i = xcd_linear();
    double red[4] = {0, 0, 0, 0};  // E_ext x, y, z, G
    if (i < S.N) {
        const size_t N = S.N;
        int x, y, z;
        site_xyz(i, S, x, y, z);
        const Nbr o = make_nbr(x, y, z, S);
        const double ra = S.rref[0] + F.mom[i], rb = S.rref[1] + F.mom[N + i];
        const double psb = F.mom[3 * N + i];
        const double kap[2] = {S.kap_p, S.kap_m};

        // S^a_m reads chi_a(i) and S^b_m reads psi^a(i) for m = i - c_d
        double lchi = 0.0, lpsa = 0.0;
#pragma unroll
        for (int d = 0; d < kQ; ++d) {
            if (d == kRest) continue;
            const unsigned m = i + offset_of(o, opposite(d));
            const double w = weight(d);
            lchi += w * (vx(d) * A.aS[m] + vy(d) * A.aS[N + m] + vz(d) * A.aS[2 * N + m]);
            lpsa += w * (vx(d) * A.aS[3 * N + m] + vy(d) * A.aS[4 * N + m] + vz(d) * A.aS[5 * N + m]);
        }
        double an[2] = {S.G_p * lchi, S.G_m * lchi};
        red[3] += lchi * psb;
        double lrho[2] = {lpsa * exp(-ra / S.rho0), S.G * lchi * exp(-rb / S.rho0)};

        // link fluxes of the six links of the site, with the friction force of both ends
        double ni[2];
        species_at(F, i, ni);
        const double rai = F.mom[i];
        const double ifr = 1.0 / (2.0 * S.beta * S.D);
        double lE[3] = {0, 0, 0}, kel = 0.0;
        for (int k = 0; k < 3; ++k) {
            const unsigned lo = i + axis_off(o, k, -1), hi = i + axis_off(o, k, 1);
            const double Ei = efield(k, x, y, z, F.phi, S);
            const double El = efield_at(k, lo, F.phi, S), Eh = efield_at(k, hi, F.phi, S);
            double nl[2], nh[2];
            species_at(F, lo, nl);
            species_at(F, hi, nh);
            const double ral = F.mom[lo], rah = F.mom[hi];
            const double aFi = A.aF[(size_t)k * N + i], aFl = A.aF[(size_t)k * N + lo], aFh = A.aF[(size_t)k * N + hi];
            for (int sp = 0; sp < 2; ++sp) {
                const double bz = 0.25 * S.beta * kZ[sp];
                const double lni = A.ln[sp][i];
                // the link (i, i + e_k): this site is its low end
                double lJ = (A.ln[sp][hi] - lni) + ifr * (aFi + aFh);
                double Ss = ni[sp] + nh[sp];
                an[sp] += lJ * (-S.D) * (-1.0 - bz * (Ei + Eh) + kap[sp] * (rah - rai));
                lE[k] += lJ * S.D * bz * Ss;
                lrho[0] += lJ * S.D * kap[sp] * Ss;
                // the link (i - e_k, i): this site is its high end
                lJ = (lni - A.ln[sp][lo]) + ifr * (aFl + aFi);
                Ss = nl[sp] + ni[sp];
                an[sp] += lJ * (-S.D) * (1.0 - bz * (El + Ei) + kap[sp] * (rai - ral));
                lE[k] += lJ * S.D * bz * Ss;
                lrho[0] -= lJ * S.D * kap[sp] * Ss;
            }
            // Kelvin force of the neighbours: F_K(i - e_k) reads +|E(i)|^2, F_K(i + e_k) reads -|E(i)|^2
            kel += 0.25 * (F.eps[lo] - S.eps_bar) * aFl - 0.25 * (F.eps[hi] - S.eps_bar) * aFh;
        }
        for (int k = 0; k < 3; ++k) {
            lE[k] += 2.0 * efield(k, x, y, z, F.phi, S) * kel;
            A.aE[(size_t)k * N + i] = lE[k];
            red[k] += lE[k];
        }
        A.arho[i] += lrho[0];
        A.arho[N + i] += lrho[1];
        A.an[i] += an[0];
        A.an[N + i] += an[1];
    }
    double gE[3] = {red[0], red[1], red[2]}, gG[1] = {red[3]};
    block_sum_add<3>(gE, A.gred, kAdjEx);
    block_sum_add<1>(gG, A.gred, kAdjG);
}

// ------------------------------------------------------------------------------------
// Pass 3: dL/dphi from the central-difference field, and its workgroup sums (slot 0 of
// F.red, the layout the source-mean kernel reads).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_rhs(Scalars S, Fields<double> F, AdjFields A) {
    const unsigned i = xcd_linear();
    double v[1] = {0.0};
    if (i < S.N) {
        const size_t N = S.N;
        int x, y, z;
        site_xyz(i, S, x, y, z);
        const Nbr o = make_nbr(x, y, z, S);
        double l = 0.0;
        for (int k = 0; k < 3; ++k)
            l += 0.5 * (A.aE[(size_t)k * N + i + axis_off(o, k, 1)] - A.aE[(size_t)k * N + i + axis_off(o, k, -1)]);
        A.rhs[i] = l;
        v[0] = l;
    }
    const bool mx[1] = {false};
    block_reduce_store<1>(v, mx, F.red, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------------------
// Pass 4: with the adjoint potential mu, the charge and permittivity terms of the Poisson
// equation, then the moments: dL/df and dL/dn at time t.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_adj_final(Scalars S, Fields<double> F, AdjFields A) {
    const unsigned i = xcd_linear();
    double red[2] = {0.0, 0.0};  // eps_a, eps_b
    if (i < S.N) {
        const size_t N = S.N;
        int x, y, z;
        site_xyz(i, S, x, y, z);
        const Nbr o = make_nbr(x, y, z, S);
        const double mui = A.mu[i], phii = F.phi[i];
        double leps = A.aeps[i];
        for (int k = 0; k < 3; ++k)
            for (int sg = -1; sg <= 1; sg += 2) {
                const unsigned j = i + axis_off(o, k, sg);
                leps += 0.5 * (F.phi[j] - phii) * (mui - A.mu[j]);
            }
        const double ra = S.rref[0] + F.mom[i], rb = S.rref[1] + F.mom[N + i], rt = ra + rb;
        const double cmp = (rb - ra) / rt;
        double lrho[2] = {A.arho[i], A.arho[N + i]};
        lrho[0] += leps * 0.5 * (S.eps_b - S.eps_a) * (-2.0 * rb / (rt * rt));
        lrho[1] += leps * 0.5 * (S.eps_b - S.eps_a) * (2.0 * ra / (rt * rt));
        red[0] += leps * 0.5 * (1.0 - cmp);
        red[1] += leps * 0.5 * (1.0 + cmp);
        // u' = (sum of momenta) / rho
        double lm[3], ud = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double lu = A.au[(size_t)k * N + i];
            lm[k] = lu / rt;
            ud += lu * F.mom[(size_t)(5 + k) * N + i];
        }
        lrho[0] -= ud / rt;
        lrho[1] -= ud / rt;
        const double keep = 1.0 - S.inv_tau;  // the part of f that survives the collision
        for (int c = 0; c < 2; ++c) {
            const double* lfc = A.lf[c];
            double* out = A.lfo[c];
#pragma unroll
            for (int d = 0; d < kQ; ++d) {
                double v = lrho[c] + vx(d) * lm[0] + vy(d) * lm[1] + vz(d) * lm[2];
                if (keep != 0.0) v += keep * lfc[(size_t)d * N + i + offset_of(o, d)];
                out[(size_t)d * N + i] = v;
            }
        }
        A.lno[0][i] = A.an[i] + mui;
        A.lno[1][i] = A.an[N + i] - mui;
    }
    block_sum_add<2>(red, A.gred, kAdjEa);
}

void launch_adj_force(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_force, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, A);
}
void launch_adj_links(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_links, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, A);
}
void launch_adj_rhs(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_rhs, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, A);
}
void launch_adj_final(const Scalars& S, const Fields<double>& F, const AdjFields& A, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_final, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, A);
}

}  // namespace ek
