// Moving particles projected anew after every step (Sec. II E).  Once k_particle_step has
// moved the particles, the solid mask, solid fraction, owner and charge of the sites near
// each particle are recomputed, and the sites the move converts are handled:
//  - a fluid site the move covers hands its fluid momentum to the covering particle (its
//    populations are no longer read: solid sites are skipped by every pass);
//  - a solid site the move uncovers gets the equilibrium of the mean density of its D3Q19
//    neighbours that are fluid before and after the move, with the velocity of the particle
//    that covered it, which gives up that momentum;
//  - the ions of a site whose fluid fraction drops to zero are shared equally among its
//    axis neighbours that keep fluid (ions live where the fluid fraction is positive).
// The momentum signs follow from momentum conservation (the printed forces F_c and F_d
// carry their own sign conventions); the neighbour density is the mean (printed as a sum),
// as for the virtual densities.
//
// Layout.  Every particle owns a box of rp_box^3 sites centred on its new position, wide
// enough to hold every site whose geometry the step can change (the move is below one site
// per step) and their neighbours.  A few workgroups per particle walk its box, one thread
// per box site; sites in several boxes are resolved from all boxes that meet (the owner is
// the lowest particle index with a covered sub-cell, a site is solid if its centre is
// inside any particle), so every thread writes the same values there.  Each conversion is
// handled by exactly one thread (of the new owner's box for a covered site, of the old
// owner's for an uncovered one), and per-site work that adds (ion shares, charge) by the
// lowest-indexed particle whose box holds the site.  Per-particle sums run in one
// workgroup per particle in a fixed tree order, so results are deterministic.
#include "ek_device.h"

namespace ek {

namespace {

constexpr double kHalfDiag = 0.8661;  // above sqrt(3)/2: no sub-cell centre is further from its site

struct BoxSite {
    int x, y, z;
    unsigned i;
};

__device__ __forceinline__ BoxSite box_site(const Scalars& S, const int32_t* origin, int a, int t) {
    const int B = S.rp_box;
    const int bx = t % B, by = (t / B) % B, bz = t / (B * B);
    BoxSite s;
    s.x = wrapc(origin[3 * a] + bx, S.nx);
    s.y = wrapc(origin[3 * a + 1] + by, S.ny);
    s.z = wrapc(origin[3 * a + 2] + bz, S.nz);
    s.i = (unsigned)s.x + (unsigned)S.nx * ((unsigned)s.y + (unsigned)S.ny * (unsigned)s.z);
    return s;
}

// Index of lattice site (x, y, z) in particle j's box, or -1 if the box does not hold it.
__device__ __forceinline__ int box_index(const Scalars& S, const int32_t* origin, int j, int x, int y, int z) {
    const int B = S.rp_box;
    const int ox = wrapc(x - origin[3 * j], S.nx), oy = wrapc(y - origin[3 * j + 1], S.ny),
              oz = wrapc(z - origin[3 * j + 2], S.nz);
    if (ox >= B || oy >= B || oz >= B) return -1;
    return ox + B * (oy + B * oz);
}

// Whether the boxes of particles a and j share a site: along every axis the circular
// distance between their lowest corners is below the box side.
__device__ __forceinline__ bool boxes_meet(const Scalars& S, const int32_t* origin, int a, int j) {
    const int n[3] = {S.nx, S.ny, S.nz};
    for (int k = 0; k < 3; ++k) {
        const int d = ((origin[3 * a + k] - origin[3 * j + k]) % n[k] + n[k]) % n[k];
        if (d >= S.rp_box && n[k] - d >= S.rp_box) return false;
    }
    return true;
}

// The lowest particle index whose box holds the site (x, y, z) of particle a's box: every
// such box meets a's box, so only those (ascending in P.nb) are scanned.
template <typename T>
__device__ __forceinline__ int first_box(const Scalars& S, const Reproj<T>& P, int a, int x, int y, int z) {
    const int32_t* nb = P.nb + (size_t)a * P.np;
    for (int m = 0; m < P.nnb[a]; ++m)
        if (box_index(S, P.origin, nb[m], x, y, z) >= 0) return nb[m];
    return P.np;
}

__device__ __forceinline__ bool wall_layer(const Scalars& S, int z) { return S.walls && (z == 0 || z == S.nz - 1); }

// Block-wide sum of n doubles per thread in a fixed tree order (result in s[k][0]).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*s)[kBlock]) {
    for (int k = 0; k < NV; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < NV; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
}

}  // namespace

// Pass 1: each particle's box origin, and for every box site the sub-cell count and the
// centre test at the new position (the same arithmetic as the set-up projection).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_mark(Scalars S, Reproj<T> P) {
#pragma clang fp contract(off)
    const int a = blockIdx.x;
    const double X = P.x[3 * a], Y = P.x[3 * a + 1], Z = P.x[3 * a + 2], R = P.rad[a];
    // every workgroup of the particle derives the box corner; the first one stores it
    const int32_t org[3] = {(int)floor(X) - S.rp_half, (int)floor(Y) - S.rp_half, (int)floor(Z) - S.rp_half};
    if (blockIdx.y == 0 && threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) P.origin[3 * a + k] = org[k];
    const int B3 = S.rp_box * S.rp_box * S.rp_box, h = S.subs;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, org, 0, t);
        const double dx = min_image((double)s.x - X, S.nx), dy = min_image((double)s.y - Y, S.ny),
                     dz = min_image((double)s.z - Z, S.nz);
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double d = sqrt(d2);
        int c = 0;
        if (d + kHalfDiag < R) {
            c = h * h * h;
        } else if (d - kHalfDiag <= R) {
            for (int ia = 0; ia < h; ++ia) {
                const double sx = dx + ((ia + 0.5) / h - 0.5);
                for (int ib = 0; ib < h; ++ib) {
                    const double sy = dy + ((ib + 0.5) / h - 0.5);
                    const double sxy = sx * sx + sy * sy;
                    for (int ie = 0; ie < h; ++ie) {
                        const double sz = dz + ((ie + 0.5) / h - 0.5);
                        if (sxy + sz * sz <= R * R) ++c;
                    }
                }
            }
        }
        const size_t k = (size_t)a * B3 + t;
        P.cnt[k] = (int16_t)c;
        P.inside[k] = d2 < R * R;
    }
}

// Pass 1b: for each particle, the particles whose boxes meet its own, in ascending order.
// Only they can hold a site of its box, so the later passes scan them instead of every box.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_pairs(Scalars S, Reproj<T> P) {
    const int a = blockIdx.x;
    if (threadIdx.x != 0) return;
    if (a == 0) *P.npl = 0;  // the particle-path list is rebuilt by k_rp_list
    int m = 0;
    for (int j = 0; j < P.np; ++j)
        if (boxes_meet(S, P.origin, a, j)) P.nb[(size_t)a * P.np + m++] = j;
    P.nnb[a] = m;
}

// Pass 2: the new solid mark, owner and fluid fraction of every box site, from all boxes.
// Wall layers keep theirs.  Bits 1-3 of the flags are recomputed in pass 5.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_resolve(Scalars S, Reproj<T> P) {
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    const double cells = (double)S.subs * S.subs * S.subs;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, P.origin, a, t);
        if (wall_layer(S, s.z)) continue;
        int own = -1, c = 0;
        uint8_t solid = 0;
        const int32_t* nb = P.nb + (size_t)a * P.np;
        for (int m = 0; m < P.nnb[a]; ++m) {  // ascending: the lowest covering index owns the site
            const int j = nb[m];
            const int tj = box_index(S, P.origin, j, s.x, s.y, s.z);
            if (tj < 0) continue;
            const size_t k = (size_t)j * B3 + tj;
            if (own < 0 && P.cnt[k] > 0) {
                own = j;
                c = P.cnt[k];
            }
            solid |= P.inside[k];
        }
        P.owner[s.i] = own;
        P.psif[s.i] = (T)(1.0 - (double)c / cells);
        P.flags[s.i] = solid;
    }
}

// Pass 3: the conversions (momentum records, fresh fluid) and the ion shares.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_convert(Scalars S, Fields<T> F, Reproj<T> P) {
#pragma clang fp contract(off)
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    const size_t N = S.N;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, P.origin, a, t);
        const size_t k = (size_t)a * B3 + t;
        P.event[k] = 0;
        P.evm[3 * k] = P.evm[3 * k + 1] = P.evm[3 * k + 2] = 0.0;
        if (wall_layer(S, s.z)) continue;
        const unsigned i = s.i;
        const bool was = P.flags_old[i] & 1, now = P.flags[i] & 1;
        const Nbr o = make_nbr(s.x, s.y, s.z, S);
        if (!was && now && P.owner[i] == a) {  // covered: its fluid momentum goes to the particle
            double m[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < kQ; ++d) {
                    if (d == kRest) continue;
                    const double g = (double)F.fn[c][(size_t)d * N + i];
                    m[0] += g * vx(d);
                    m[1] += g * vy(d);
                    m[2] += g * vz(d);
                }
            P.event[k] = 1;
            for (int q = 0; q < 3; ++q) P.evm[3 * k + q] = m[q];
        }
        if (was && !now && P.owner_old[i] == a) {  // uncovered: fresh fluid moving with the particle
            const double v0 = P.v[3 * a], v1 = P.v[3 * a + 1], v2 = P.v[3 * a + 2];
            const double usq = v0 * v0 + v1 * v1 + v2 * v2;
            double dm[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 2; ++c) {
                double acc = 0.0;
                int cnt = 0;
                for (int d = 0; d < kQ; ++d) {
                    if (d == kRest) continue;
                    const unsigned j = i + offset_of(o, d);
                    if ((P.flags_old[j] & 1) || (P.flags[j] & 1)) continue;
                    double r = S.rref[c];
                    for (int e = 0; e < kQ; ++e) r += (double)F.fn[c][(size_t)e * N + j];
                    if (F.rlo) r += (double)F.rlo[(size_t)c * N + j];
                    acc += r;
                    ++cnt;
                }
                const double rb = cnt > 0 ? acc / cnt : 0.0;
                for (int d = 0; d < kQ; ++d) {
                    const double cu = vx(d) * v0 + vy(d) * v1 + vz(d) * v2;
                    const double feq = weight(d) * rb * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                    const double g = feq - weight(d) * S.rref[c];
                    const T gt = (T)g;
                    F.fn[c][(size_t)d * N + i] = gt;
                    if (d == kRest && F.rlo) F.rlo[(size_t)c * N + i] = (T)(g - (double)gt);
                }
                dm[0] -= rb * v0;
                dm[1] -= rb * v1;
                dm[2] -= rb * v2;
            }
            P.event[k] = 2;
            for (int q = 0; q < 3; ++q) P.evm[3 * k + q] = dm[q];
        }
        if (P.psif_old[i] > T(0) && P.psif[i] == T(0) && P.owner[i] == a) {  // its ions move away
            int cnt = 0;
            for (int d = 0; d < kQ; ++d) {
                if (vsq(d) != 1) continue;  // the six axis links
                const int zz = s.z + vz(d);
                if (S.walls && (zz < 0 || zz >= S.nz)) continue;
                if (P.psif[i + offset_of(o, d)] > T(0)) ++cnt;
            }
            if (cnt > 0) {
                P.share[i] = F.nn[0][i] / T(cnt);
                P.share[N + i] = F.nn[1][i] / T(cnt);
            }
        }
    }
}

// Pass 4: the ion shares, gathered by each receiving site; the giving sites are emptied.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_ions(Scalars S, Fields<T> F, Reproj<T> P) {
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    const size_t N = S.N;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, P.origin, a, t);
        if (wall_layer(S, s.z) || first_box(S, P, a, s.x, s.y, s.z) != a) continue;
        const unsigned i = s.i;
        const Nbr o = make_nbr(s.x, s.y, s.z, S);
        auto gives = [&](unsigned j, int zj) {
            if (wall_layer(S, zj) || !(P.psif_old[j] > T(0) && P.psif[j] == T(0))) return false;
            // a site with no axis neighbour keeping fluid keeps its ions (no shares written)
            const int jx = (int)(j % (unsigned)S.nx), jy = (int)((j / (unsigned)S.nx) % (unsigned)S.ny);
            const Nbr oj = make_nbr(jx, jy, zj, S);
            for (int d = 0; d < kQ; ++d) {
                if (vsq(d) != 1) continue;  // the six axis links
                const int zz = zj + vz(d);
                if (S.walls && (zz < 0 || zz >= S.nz)) continue;
                if (P.psif[j + offset_of(oj, d)] > T(0)) return true;
            }
            return false;
        };
        if (P.psif[i] == T(0)) {
            if (gives(i, s.z)) {
                F.nn[0][i] = T(0);
                F.nn[1][i] = T(0);
            }
            continue;
        }
        T add0 = T(0), add1 = T(0);
        bool any = false;
        for (int d = 0; d < kQ; ++d) {
            if (vsq(d) != 1) continue;  // the six axis links
            const int zz = s.z + vz(d);
            if (S.walls && (zz < 0 || zz >= S.nz)) continue;
            const unsigned j = i + offset_of(o, d);
            if (gives(j, wrapc(zz, S.nz))) {
                add0 += P.share[j];
                add1 += P.share[N + j];
                any = true;
            }
        }
        if (any) {
            F.nn[0][i] += add0;
            F.nn[1][i] += add1;
        }
    }
}

// Pass 5: per particle, the impulse of its conversions and the summed solid fraction.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_sum(Scalars S, Reproj<T> P) {
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < B3; t += blockDim.x) {
        const size_t k = (size_t)a * B3 + t;
        if (P.event[k]) {
            acc[0] += P.evm[3 * k];
            acc[1] += P.evm[3 * k + 1];
            acc[2] += P.evm[3 * k + 2];
        }
        const BoxSite s = box_site(S, P.origin, a, t);
        if (P.owner[s.i] == a) acc[3] += 1.0 - (double)P.psif[s.i];
    }
    __shared__ double sm[4][kBlock];
    block_sum<4>(acc, sm);
    if (threadIdx.x == 0) {
        const double R = P.rad[a];
        const double m = P.rho_p * (4.0 / 3.0) * M_PI * R * R * R;
        for (int q = 0; q < 3; ++q) P.v[3 * a + q] += sm[q][0] / m;
        P.ptot[a] = sm[3][0];
    }
}

// Pass 6: charge per site and the neighbour flag bits of every box site.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_finish(Scalars S, Reproj<T> P) {
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, P.origin, a, t);
        if (first_box(S, P, a, s.x, s.y, s.z) != a) continue;
        const unsigned i = s.i;
        const int own = P.owner[i];
        const double psis = 1.0 - (double)P.psif[i];
        P.qc[i] = (own >= 0 && P.ptot[own] > 0.0) ? (T)(P.Q[own] * psis / P.ptot[own]) : T(0);
        const Nbr o = make_nbr(s.x, s.y, s.z, S);
        const uint8_t si = P.flags[i] & 1;
        bool other = false;
        for (int d = 0; d < kQ; ++d) {
            if (d == kRest) continue;
            if ((P.flags[i + offset_of(o, d)] & 1) != si) other = true;
        }
        bool part = psis > 0.0;
        for (int d = 0; d < kQ && !part; ++d) part = vsq(d) == 1 && P.psif[i + offset_of(o, d)] < T(1);
        // every box site is rewritten, so bits 1-3 are set from scratch
        P.flags[i] = (uint8_t)(si | (other ? (si ? 4 : 2) : 0) | (part ? 8 : 0));
    }
}

// Pass 7: the particle-path sites (flag bits 0, 1 or 3), gathered from the boxes (each
// site by the lowest-indexed box that holds it) into the context's list, in no particular
// order: every such site lies in a box (a box reaches four sites beyond its sphere), and
// the list kernels handle each listed site by itself.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rp_list(Scalars S, Reproj<T> P) {
    const int a = blockIdx.x;
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    for (int t = blockIdx.y * kBlock + threadIdx.x; t < B3; t += kBlock * gridDim.y) {
        const BoxSite s = box_site(S, P.origin, a, t);
        if ((P.flags[s.i] & (1u | 2u | 8u)) == 0 || first_box(S, P, a, s.x, s.y, s.z) != a) continue;
        P.plist[atomicAdd(P.npl, 1)] = (int32_t)s.i;
    }
}

template <typename T>
void launch_reproject(const Scalars& S, const Fields<T>& F, const Reproj<T>& P, hipStream_t st) {
    if (P.np <= 0) return;
    // the per-site passes split each box over a few workgroups (one per particle would
    // leave most of the chip idle with a few hundred particles); the per-particle sums keep one
    const int B3 = S.rp_box * S.rp_box * S.rp_box;
    const dim3 g(P.np), gs(P.np, std::min(8, (B3 + 4 * kBlock - 1) / (4 * kBlock))), b(kBlock);
    hipLaunchKernelGGL(k_rp_mark<T>, gs, b, 0, st, S, P);
    hipLaunchKernelGGL(k_rp_pairs<T>, g, dim3(64), 0, st, S, P);
    hipLaunchKernelGGL(k_rp_resolve<T>, gs, b, 0, st, S, P);
    hipLaunchKernelGGL(k_rp_convert<T>, gs, b, 0, st, S, F, P);
    hipLaunchKernelGGL(k_rp_ions<T>, gs, b, 0, st, S, F, P);
    hipLaunchKernelGGL(k_rp_sum<T>, g, b, 0, st, S, P);
    hipLaunchKernelGGL(k_rp_finish<T>, gs, b, 0, st, S, P);
    hipLaunchKernelGGL(k_rp_list<T>, gs, b, 0, st, S, P);
}

template void launch_reproject<float>(const Scalars&, const Fields<float>&, const Reproj<float>&, hipStream_t);
template void launch_reproject<double>(const Scalars&, const Fields<double>&, const Reproj<double>&, hipStream_t);

}  // namespace ek
