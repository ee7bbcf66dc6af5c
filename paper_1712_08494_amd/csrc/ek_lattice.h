// D3Q19 lattice of the GPU path (Sec. II A: one rest velocity, six axis links and
// twelve face diagonals, weights 1/3, 1/18, 1/36, c_s^2 = 1/3).
//
// Velocities are numbered lexicographically in (c_z, c_y, c_x): the five with c_z = -1,
// the nine with c_z = 0 (rest at d = 9), the five with c_z = +1.  With that order the
// opposite of d is 18 - d, and the streaming targets of one site fall on three z-planes
// in contiguous runs of d.  All helpers are constexpr so that fully unrolled loops
// fold them to immediates.
#pragma once

namespace ek {

constexpr int kQ = 19;
constexpr int kRest = 9;

__host__ __device__ constexpr int vz(int d) { return d < 5 ? -1 : (d < 14 ? 0 : 1); }

__host__ __device__ constexpr int vx(int d) {
    return (d >= 5 && d < 14) ? ((d - 5) % 3) - 1 : ((d % 14) == 1 ? -1 : ((d % 14) == 3 ? 1 : 0));
}

__host__ __device__ constexpr int vy(int d) {
    return (d >= 5 && d < 14) ? ((d - 5) / 3) - 1 : ((d % 14) == 0 ? -1 : ((d % 14) == 4 ? 1 : 0));
}

__host__ __device__ constexpr int opposite(int d) { return 18 - d; }

__host__ __device__ constexpr int vsq(int d) { return vx(d) * vx(d) + vy(d) * vy(d) + vz(d) * vz(d); }

__host__ __device__ constexpr double weight(int d) {
    return vsq(d) == 0 ? 1.0 / 3.0 : (vsq(d) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

}  // namespace ek
