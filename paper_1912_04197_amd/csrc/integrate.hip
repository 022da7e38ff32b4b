// Kick-drift-kick leapfrog (Section "Numerical solvers" lists leapfrog among
// the symplectic steppers) and the energy / momentum diagnostics the paper
// monitors in its validation runs (Section "Validation scenarios").
// All state is FP64.
#include "bhx_impl.h"

namespace bhx {
namespace {

// k semi-implicit Euler substeps with the acceleration held: v += dt a, then
// x += dt v, each rounded as written.
__global__ __launch_bounds__(256) void k_euler_substeps(double *__restrict__ pos,
                                                        double *__restrict__ vel,
                                                        const double *__restrict__ acc,
                                                        int64_t n3, double dt, int k)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const double a = acc[i];
    double v = vel[i], x = pos[i];
    for (int j = 0; j < k; j++) {
        v = v + dt * a;
        x = x + dt * v;
    }
    vel[i] = v;
    pos[i] = x;
}

// v += dt/2 a ; x += dt v
__global__ __launch_bounds__(256) void k_kick_drift(double *__restrict__ pos,
                                                    double *__restrict__ vel,
                                                    const double *__restrict__ acc, int64_t n3,
                                                    double h, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const double v = vel[i] + h * acc[i];
    vel[i] = v;
    pos[i] = pos[i] + dt * v;
}

// v += dt/2 a
__global__ __launch_bounds__(256) void k_kick(double *__restrict__ vel,
                                              const double *__restrict__ acc, int64_t n3, double h)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    vel[i] = vel[i] + h * acc[i];
}

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-block partial sums of {E_kin, E_pot, P, L}; E_pot = 1/2 sum m phi.
__global__ __launch_bounds__(256) void k_diag_partial(const double *__restrict__ pos,
                                                      const double *__restrict__ vel,
                                                      const double *__restrict__ mass,
                                                      const double *__restrict__ phi, int64_t n,
                                                      double *__restrict__ part)
{
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        const double u = vel[3 * i], v = vel[3 * i + 1], w = vel[3 * i + 2];
        const double m = mass[i];
        q[0] += 0.5 * m * (u * u + v * v + w * w);
        q[1] += 0.5 * m * phi[i];
        q[2] += m * u;
        q[3] += m * v;
        q[4] += m * w;
        q[5] += m * (y * w - z * v);
        q[6] += m * (z * u - x * w);
        q[7] += m * (x * v - y * u);
    }
    __shared__ double red[4][8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 8; k++) {
        const double t = wave_sum(q[k]);
        if (lane == 0) red[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 8)
        part[blockIdx.x * 8 + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ __launch_bounds__(64) void k_diag_final(const double *__restrict__ part, int nblk,
                                                   double *__restrict__ out)
{
    for (int k = 0; k < 8; k++) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 64) t += part[b * 8 + k];
        t = wave_sum(t);
        if (threadIdx.x == 0) out[k] = t;
    }
}

inline unsigned blocks(int64_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

hipError_t launch_kick_drift(hipStream_t s, double *pos, double *vel, const double *acc, int64_t n,
                             double dt)
{
    if (n <= 0) return hipSuccess;
    k_kick_drift<<<blocks(3 * n), 256, 0, s>>>(pos, vel, acc, 3 * n, 0.5 * dt, dt);
    return hipGetLastError();
}

hipError_t launch_euler_substeps(hipStream_t s, double *pos, double *vel, const double *acc,
                                 int64_t n, double dt, int k)
{
    if (n <= 0 || k <= 0) return hipSuccess;
    k_euler_substeps<<<blocks(3 * n), 256, 0, s>>>(pos, vel, acc, 3 * n, dt, k);
    return hipGetLastError();
}

hipError_t launch_kick(hipStream_t s, double *vel, const double *acc, int64_t n, double dt)
{
    if (n <= 0) return hipSuccess;
    k_kick<<<blocks(3 * n), 256, 0, s>>>(vel, acc, 3 * n, 0.5 * dt);
    return hipGetLastError();
}

hipError_t launch_diag_reduce(hipStream_t s, const double *pos, const double *vel,
                              const double *mass, const double *phi, int64_t n, double *part,
                              double *out8_device)
{
    unsigned nb = blocks(n);
    if (nb > (unsigned)kRedBlocks) nb = kRedBlocks;
    if (nb < 1) nb = 1;
    k_diag_partial<<<nb, 256, 0, s>>>(pos, vel, mass, phi, n, part);
    k_diag_final<<<1, 64, 0, s>>>(part, (int)nb, out8_device);
    return hipGetLastError();
}

}  // namespace bhx
