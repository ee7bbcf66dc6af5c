// Device helpers shared by the step kernels (ek_kernels.hip) and the adjoint kernels
// (ek_adjoint.hip): workgroup-to-site mapping, periodic neighbour offsets, the
// central-difference field and the deterministic FP64 block reduction.
#pragma once

#include "ek_internal.h"
#include "ek_lattice.h"

namespace ek {

// Workgroups are dispatched round-robin over the 8 XCDs (XCD = blockIdx % 8).  Give XCD k
// the contiguous block range [k * nb/8, (k+1) * nb/8) so its L2 holds a slab of planes.
// The kernels that use it run kBlock threads per workgroup; the constant saves the load of
// the workgroup size from the kernel's implicit arguments that blockDim.x costs.
__device__ __forceinline__ unsigned xcd_linear() {
    const unsigned nb = gridDim.x;  // multiple of 8 (site_blocks)
    const unsigned b = blockIdx.x;
    const unsigned lb = (b & 7u) * (nb >> 3) + (b >> 3);
    return lb * kBlock + threadIdx.x;
}

// The same XCD split for the stencil sweeps over the lattice, with the slab walked band by
// band when S.band > 0: a band is S.band consecutive workgroups of one z-plane (a few x-rows),
// taken in every plane of the slab before the next band starts.  The workgroups resident on
// an XCD at any time then cover a few rows of many consecutive planes, so the z-neighbour
// rows their stencils read were fetched by the workgroups just before them and still sit in
// the XCD's L2.  In the plain order the resident workgroups cover whole planes, and at
// 256 x 256 the neighbour planes of the stencil's arrays (256 KB per FP32 plane) exceed the
// 4 MB L2.  Requires nz % 8 == 0 and whole planes of workgroups (checked by the host).
__device__ __forceinline__ unsigned site_banded(const Scalars& S) {
    const unsigned b = blockIdx.x;
    const unsigned x8 = b & 7u, s = b >> 3;  // XCD and position in its sequence
    if (S.band <= 0) return (x8 * (gridDim.x >> 3) + s) * kBlock + threadIdx.x;
    const unsigned B = (unsigned)S.band, P = (unsigned)S.plane_blocks, nzs = (unsigned)S.slab_planes;
    const unsigned per_band = nzs * B;
    const unsigned band = s / per_band, rem = s - band * per_band;
    const unsigned zz = rem / B, j = rem - zz * B;
    const unsigned lb = (x8 * nzs + zz) * P + band * B + j;
    return lb * kBlock + threadIdx.x;
}

// Minimum image of a separation along a periodic axis of length n: the whole periods that
// stepping by n would remove are taken off at once, so the result equals the stepping loop
// for every finite d and is NaN (not an endless loop) for a non-finite one.
__host__ __device__ inline double min_image(double d, int n) {
    const double L = (double)n;
    if (d > 0.5 * L) d -= L * ceil((d - 0.5 * L) / L);
    if (d < -0.5 * L) d += L * ceil((-0.5 * L - d) / L);
    return d;
}

struct Nbr {
    int xm, xp, ym, yp, zm, zp;  // index offsets to the -1/+1 neighbour along each axis (periodic)
};

__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, const Scalars& S) {
    Nbr o;
    o.xm = x == 0 ? S.nx - 1 : -1;
    o.xp = x == S.nx - 1 ? -(S.nx - 1) : 1;
    o.ym = y == 0 ? (S.ny - 1) * S.nx : -S.nx;
    o.yp = y == S.ny - 1 ? -(S.ny - 1) * S.nx : S.nx;
    o.zm = z == 0 ? (S.nz - 1) * S.nxy : -S.nxy;
    o.zp = z == S.nz - 1 ? -(S.nz - 1) * S.nxy : S.nxy;
    return o;
}

__device__ __forceinline__ int offset_of(const Nbr& o, int d) {
    return (vx(d) < 0 ? o.xm : (vx(d) > 0 ? o.xp : 0)) + (vy(d) < 0 ? o.ym : (vy(d) > 0 ? o.yp : 0)) +
           (vz(d) < 0 ? o.zm : (vz(d) > 0 ? o.zp : 0));
}

// Exact floor(a / d) from a precomputed 1/d (FP64), for a, d < 2^32: (a + 1/2)/d lies at
// least 1/(2d) from an integer, far more than the rounding of the two FP64 operations.  A
// few FP64 instructions instead of an integer division's long sequence.
__device__ __forceinline__ unsigned div_exact(unsigned a, double inv_d) {
    return (unsigned)(((double)a + 0.5) * inv_d);
}

// Coordinates of lattice site i.
__device__ __forceinline__ void site_xyz(unsigned i, const Scalars& S, int& x, int& y, int& z) {
    const unsigned r = div_exact(i, S.inv_nx);
    x = (int)(i - r * (unsigned)S.nx);
    z = (int)div_exact(i, S.inv_nxy);
    y = (int)(r - (unsigned)z * (unsigned)S.ny);
}

__device__ __forceinline__ int site_z(unsigned i, const Scalars& S) { return (int)div_exact(i, S.inv_nxy); }

// Coordinates of cell t of a multigrid level.
__device__ __forceinline__ void level_xyz(unsigned t, const MGLevel& L, int& x, int& y, int& z) {
    const unsigned r = div_exact(t, L.inv_nx);
    x = (int)(t - r * (unsigned)L.nx);
    z = (int)div_exact(r, L.inv_ny);
    y = (int)(r - (unsigned)z * (unsigned)L.ny);
}

__device__ __forceinline__ int wrapc(int a, int n) {
    return n == 1 ? 0 : (a < 0 ? a + n : (a >= n ? a - n : a));
}

__device__ __forceinline__ double phi_at(const double* phi, int x, int y, int z, const Scalars& S) {
    return phi[wrapc(x, S.nx) + S.nx * (wrapc(y, S.ny) + S.ny * wrapc(z, S.nz))];
}

// Component k of E = -grad(phi) + E_ext at site (x, y, z): central differences, one-sided
// for the normal component on the wall layers.
__device__ __forceinline__ double efield(int k, int x, int y, int z, const double* phi, const Scalars& S) {
    double e;
    if (k == 0) {
        e = -0.5 * (phi_at(phi, x + 1, y, z, S) - phi_at(phi, x - 1, y, z, S));
    } else if (k == 1) {
        e = -0.5 * (phi_at(phi, x, y + 1, z, S) - phi_at(phi, x, y - 1, z, S));
    } else {
        if (S.walls && z == 0)
            e = -(phi_at(phi, x, y, 1, S) - phi_at(phi, x, y, 0, S));
        else if (S.walls && z == S.nz - 1)
            e = -(phi_at(phi, x, y, z, S) - phi_at(phi, x, y, z - 1, S));
        else
            e = -0.5 * (phi_at(phi, x, y, z + 1, S) - phi_at(phi, x, y, z - 1, S));
    }
    return e + S.E_ext[k];
}

__device__ __forceinline__ double efield_sq(int x, int y, int z, const double* phi, const Scalars& S) {
    double a = efield(0, x, y, z, phi, S), b = efield(1, x, y, z, phi, S), c = efield(2, x, y, z, phi, S);
    return a * a + b * b + c * c;
}

__device__ __forceinline__ bool wall_layer(int z, const Scalars& S) { return S.walls && (z == 0 || z == S.nz - 1); }

// ------------------------------------------------------------------------------------
// FP64 block reduction of NV values (sums, or maxima where is_max) into record `slot` of
// nrec records, stored value-major (value k of record b at red[k * nrec + b]) so that a
// reducer reads each value's records contiguously.
// ------------------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], const bool (&is_max)[NV], double* red,
                                                   unsigned slot, unsigned nrec) {
    __shared__ double sm[NV][kBlock / 64];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = v[k];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
            double b = __shfl_down(a, s, 64);
            a = is_max[k] ? fmax(a, b) : a + b;
        }
        v[k] = a;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sm[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = sm[k][0];
            for (int w = 1; w < kBlock / 64; ++w) a = is_max[k] ? fmax(a, sm[k][w]) : a + sm[k][w];
            red[(size_t)k * nrec + slot] = a;
        }
    }
}

}  // namespace ek
