// The paper's lagged Fourier scheme for the variable-permittivity Poisson equation
// (Sec. II D), periodic lattices.  The permittivity-gradient term is taken at the previous
// potential; what remains is a constant-coefficient Poisson equation for the new one,
// inverted here with one forward and one inverse FFT (hipFFT, FP64).  Discretely: with
// eps_f = eps_i + (eps_j - eps_i)/2 the finite-volume equation
//   sum_f eps_f (phi_j - phi_i) = -s_i
// splits into eps_i L phi_i + sum_f (eps_j - eps_i)(phi_j - phi_i)/2 = -s_i, with
// L phi_i = sum_f (phi_j - phi_i), so
//   L phi = r,  r_i = [ -s_i - sum_f (eps_j - eps_i)(phi_old_j - phi_old_i)/2 ] / eps_i.
// The Fourier inversion is of this same 7-point Laplacian (eigenvalue
// sum_axes 2 cos(2 pi k / n) - 2), so a potential that solves the finite-volume equation is
// a fixed point.  The zero wavenumber is dropped: mean(r) removed, mean(phi) = 0.
#include "ek_device.h"

namespace ek {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_lag_rhs(Scalars S, Fields<T> F, double* __restrict__ rhs) {
    const unsigned i = xcd_linear();
    if (i >= S.N) return;
    int x, y, z;
    site_xyz(i, S, x, y, z);
    const Nbr o = make_nbr(x, y, z, S);
    const double ei = (double)F.eps[i], pi = F.phi[i];
    const int off[6] = {o.xp, o.xm, o.yp, o.ym, o.zp, o.zm};
    double lag = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const unsigned j = i + off[k];
        lag += 0.5 * ((double)F.eps[j] - ei) * (F.phi[j] - pi);
    }
    const double s = (double)F.q[i] - F.scal[0];  // source with its mean removed
    rhs[i] = (-s - lag) / ei;
}

// Per-axis parts of the 7-point Laplacian's eigenvalues, 2 cos(2 pi k / n) - 2, for the
// nx/2 + 1 wavenumbers along x, then ny along y, then nz along z (set up once per context).
__global__ void k_lag_table(double* __restrict__ tab, int nx, int ny, int nz) {
    const int hx1 = nx / 2 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= hx1 + ny + nz) return;
    const double twopi = 6.283185307179586476925286766559;
    const int n = t < hx1 ? nx : (t < hx1 + ny ? ny : nz);
    const int k = t < hx1 ? t : (t < hx1 + ny ? t - hx1 : t - hx1 - ny);
    tab[t] = 2.0 * cos(twopi * k / n) - 2.0;
}

// Spectrum of a real-to-complex transform of an (nz, ny, nx) array, x fastest: nx/2 + 1
// wavenumbers along x.  Divide by the Laplacian's eigenvalue and by N (the inverse
// transform is unnormalised); zero wavenumber dropped.
__global__ __launch_bounds__(kBlock) void k_lag_scale(double2* __restrict__ spec, const double* __restrict__ tab,
                                                      int nx, int ny, int nz, double inv_hx1, double inv_ny,
                                                      double inv_n) {
    const unsigned hx1 = (unsigned)(nx / 2 + 1);
    const unsigned total = hx1 * (unsigned)ny * (unsigned)nz;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const unsigned r = div_exact(t, inv_hx1), kx = t - r * hx1;
    const unsigned kz = div_exact(r, inv_ny), ky = r - kz * (unsigned)ny;
    if (t == 0) {
        spec[0] = make_double2(0.0, 0.0);
        return;
    }
    const double lam = tab[kx] + tab[hx1 + ky] + tab[hx1 + ny + kz];
    const double g = inv_n / lam;
    const double2 v = spec[t];
    spec[t] = make_double2(v.x * g, v.y * g);
}

template <typename T> void launch_lag_rhs(const Scalars& S, const Fields<T>& F, double* rhs, hipStream_t st) {
    hipLaunchKernelGGL(k_lag_rhs<T>, dim3(site_blocks(S.N)), dim3(kBlock), 0, st, S, F, rhs);
}

void launch_lag_table(double* tab, int nx, int ny, int nz, hipStream_t st) {
    const int n = nx / 2 + 1 + ny + nz;
    hipLaunchKernelGGL(k_lag_table, dim3((n + 63) / 64), dim3(64), 0, st, tab, nx, ny, nz);
}

void launch_lag_scale(double* spec, const double* tab, int nx, int ny, int nz, hipStream_t st) {
    const unsigned hx1 = (unsigned)(nx / 2 + 1);
    const unsigned total = hx1 * (unsigned)ny * (unsigned)nz;
    hipLaunchKernelGGL(k_lag_scale, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       reinterpret_cast<double2*>(spec), tab, nx, ny, nz, 1.0 / hx1, 1.0 / ny,
                       1.0 / ((double)nx * ny * nz));
}

template void launch_lag_rhs<float>(const Scalars&, const Fields<float>&, double*, hipStream_t);
template void launch_lag_rhs<double>(const Scalars&, const Fields<double>&, double*, hipStream_t);

}  // namespace ek
