// Thermally activated escape of a uniaxial spin in a transverse field
// (Sec. III.B): many independent single spins, E = -D s_z^2 - H s_x, each
// started at the bottom of the well (sin theta = h, phi = 0) and run through
// the pulse-noise schedule until s_z < 0.  One thread per run with its state
// in registers, stepped by the explicit Runge-Kutta tableau of the chosen
// integrator; the kick is the lattice kick with the run index as site index.
#include "lll_device.hpp"

namespace lll {

// Pulses k0 .. k1-1 for every run i < n_runs whose time is still negative
// (not escaped).  The state s[3][n_runs] carries over between launches
// (k0 == 0 starts from the well).  times[i] = number of completed steps x dt
// at the first step end or kick after which s_z < 0.  *active gains the
// number of runs still going at the end of the launch.
template <bool PREC>
__global__ void __launch_bounds__(256)
    escape_kernel(RepDev R, Tableau tb, int64_t n_runs, int64_t n, double dt, int64_t k0,
                  int64_t k1, double h, double* sx, double* sy, double* sz, double* times,
                  unsigned int* active) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool live = i < n_runs && times[i] < 0.0;
    double x = 0, y = 0, z = 0;
    if (live) {
        if (k0 == 0) {
            x = h;
            y = 0.0;
            z = sqrt(1.0 - h * h);
        } else {
            x = sx[i];
            y = sy[i];
            z = sz[i];
        }
    }
    const Coef<double> C = load_coef<double>(R);
    const int64_t n1 = n / 2;
    for (int64_t k = k0; k < k1 && live; ++k) {
        for (int64_t q = 0; q < n; ++q) {
            if (q == n1) {
                const uint4 w = philox_site(R.seed, (uint32_t)i, (uint32_t)k, R.rid, 0u);
                (void)kick_spin<double>(x, y, z, w, R.sigma);
                if (z < 0.0) {
                    times[i] = (double)(k * n + q) * dt;
                    live = false;
                    break;
                }
            }
            // loops unrolled to the largest tableau so that K stays in registers
            double K[6][3];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (j >= tb.stages) break;
                double yx = x, yy = y, yz = z;
#pragma unroll
                for (int l = 0; l < j; ++l) {
                    const double a = tb.a[j][l];
                    if (a == 0.0) continue;
                    yx += a * K[l][0];
                    yy += a * K[l][1];
                    yz += a * K[l][2];
                }
                // no exchange: zero neighbour sum; h = H x + 2 D s_z z
                stage_k<double, PREC, ANIS_Z>(yx, yy, yz, 0.0, 0.0, 0.0, C, 0.0, 0.0, 0.0, 0.0,
                                              K[j][0], K[j][1], K[j][2]);
            }
#pragma unroll
            for (int l = 0; l < 6; ++l) {
                if (l >= tb.stages) break;
                const double b = tb.b[l];
                if (b == 0.0) continue;
                x += b * K[l][0];
                y += b * K[l][1];
                z += b * K[l][2];
            }
            if (z < 0.0) {
                times[i] = (double)(k * n + q + 1) * dt;
                live = false;
                break;
            }
        }
    }
    if (i < n_runs && live) {
        sx[i] = x;
        sy[i] = y;
        sz[i] = z;
    }
    const unsigned long long b = __ballot(live);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(active, (unsigned int)__popcll(b));
}

hipError_t launch_escape(const RepDev& R, const Tableau& tb, int precession, int64_t n_runs,
                         int64_t n, double dt, int64_t k0, int64_t k1, double h, double* sx,
                         double* sy, double* sz, double* times, unsigned int* active,
                         hipStream_t st) {
    if (n_runs <= 0) return hipSuccess;
    if (tb.stages < 1 || tb.stages > 6) return hipErrorInvalidValue;
    const int64_t nb = (n_runs + 255) / 256;
    if (precession)
        hipLaunchKernelGGL(escape_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, R, tb, n_runs,
                           n, dt, k0, k1, h, sx, sy, sz, times, active);
    else
        hipLaunchKernelGGL(escape_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, R, tb,
                           n_runs, n, dt, k0, k1, h, sx, sy, sz, times, active);
    return hipGetLastError();
}

}  // namespace lll
