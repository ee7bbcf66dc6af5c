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

// Weights of the equilibrium in the storage precision.  The collision sets each population
// to w_d times the site's density deviation plus velocity terms, so the stored density
// deviation is multiplied by the sum of the weights at every step.  The FP32 roundings of
// 1/3, 1/18 and 1/36 sum to 1 + 1.5e-8, which would grow a deviation by 7.5e-5 over 5000
// steps; these FP32 values sum to 1 exactly: w2 = 1864135 / 2^26 (1/36 to 6e-8), w1 = 2 w2,
// w0 = 1 - 24 w2 = 2796203 / 2^23, each exact in FP32.  FP64 uses the exact fractions.
__host__ __device__ constexpr double weight_fp32(int d) {
    return vsq(d) == 0 ? 2796203.0 / 8388608.0 : (vsq(d) == 1 ? 1864135.0 / 33554432.0 : 1864135.0 / 67108864.0);
}

template <typename T>
__host__ __device__ constexpr double storage_weight(int d) {
    return sizeof(T) == 4 ? weight_fp32(d) : weight(d);
}

}  // namespace ek
