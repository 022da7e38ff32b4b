// Kick-drift-kick leapfrog (Section "Numerical solvers" lists leapfrog among
// the symplectic steppers), the energy / momentum diagnostics the paper
// monitors in its validation runs (Section "Validation scenarios", by
// compensated sums) and the gravity time-step bound of eq. (dt_g).
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

// v += dt/2 a ; x += dt v, each one fused multiply-add (the multi-step
// path's kick and drift round them the same way)
__global__ __launch_bounds__(256) void k_kick_drift(double *__restrict__ pos,
                                                    double *__restrict__ vel,
                                                    const double *__restrict__ acc, int64_t n3,
                                                    double h, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const double v = fma(h, acc[i], vel[i]);
    vel[i] = v;
    pos[i] = fma(dt, v, pos[i]);
}

// v += dt/2 a
__global__ __launch_bounds__(256) void k_kick(double *__restrict__ vel,
                                              const double *__restrict__ acc, int64_t n3, double h)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    vel[i] = fma(h, acc[i], vel[i]);
}

// The sorted state of a multi-step call from the caller's arrays, in caller
// order (the first build sorts it); masses and softening lengths are checked
// here once, as each build checks them on the caller-order path.
__global__ __launch_bounds__(256) void k_state_pack(
    const double *__restrict__ pos, const double *__restrict__ vel,
    const double *__restrict__ acc, const double *__restrict__ mass,
    const double *__restrict__ eps, int64_t n, Body *__restrict__ body,
    double *__restrict__ tvel, double *__restrict__ tacc, double *__restrict__ beps2,
    uint32_t *__restrict__ idx, uint32_t *__restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const double m = mass[i];
        bad = !(isfinite(m) && m >= 0.0);
        body[i] = Body{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], m};
        for (int a = 0; a < 3; a++) {
            tvel[3 * i + a] = vel[3 * i + a];
            tacc[3 * i + a] = acc[3 * i + a];
        }
        if (eps) {
            const double e = eps[i];
            bad |= !(isfinite(e) && e >= 0.0);
            beps2[i] = e * e;
        }
        idx[i] = (uint32_t)i;
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, ST_NONFINITE);
}

// The end of a multi-step call: the state back to the caller's arrays.
__global__ __launch_bounds__(256) void k_state_unpack(const Body *__restrict__ body,
                                                      const double *__restrict__ tvel,
                                                      const double *__restrict__ tacc,
                                                      const uint32_t *__restrict__ idx, int64_t n,
                                                      double *__restrict__ pos,
                                                      double *__restrict__ vel,
                                                      double *__restrict__ acc)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int64_t o = idx[s];
    const Body b = body[s];
    pos[3 * o] = b.x;
    pos[3 * o + 1] = b.y;
    pos[3 * o + 2] = b.z;
    for (int a = 0; a < 3; a++) {
        vel[3 * o + a] = tvel[3 * s + a];
        acc[3 * o + a] = tacc[3 * s + a];
    }
}

// Compensated FP64 sums: a value is carried as s + c with c the rounding
// error of s, accumulated by error-free transformations (TwoSum: s' = s + t
// and the exact error of that addition), so a sum of many terms of mixed signs
// (momenta, whose total is small against its terms) keeps its low digits.
struct CSum {
    double s, c;
};
__device__ inline CSum csum_zero() { return CSum{0.0, 0.0}; }

__device__ inline void csum_add(CSum &a, double t)
{
#pragma clang fp contract(off)
    const double s = a.s + t;
    const double bp = s - a.s;
    const double e = (a.s - (s - bp)) + (t - bp);
    a.s = s;
    a.c += e;
}

__device__ inline void csum_merge(CSum &a, const CSum &b)
{
    csum_add(a, b.s);
    a.c += b.c;
}

__device__ inline CSum wave_csum(CSum v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const CSum w{__shfl_xor(v.s, o), __shfl_xor(v.c, o)};
        csum_merge(v, w);
    }
    return v;
}

// Per-block compensated partial sums of {E_kin, E_pot, P, L};
// E_pot = 1/2 sum m phi. part[blk][k] = {s, c}.
__global__ __launch_bounds__(256) void k_diag_partial(const double *__restrict__ pos,
                                                      const double *__restrict__ vel,
                                                      const double *__restrict__ mass,
                                                      const double *__restrict__ phi, int64_t n,
                                                      double *__restrict__ part)
{
#pragma clang fp contract(off)
    CSum q[8];
    for (int k = 0; k < 8; k++) q[k] = csum_zero();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        const double u = vel[3 * i], v = vel[3 * i + 1], w = vel[3 * i + 2];
        const double m = mass[i];
        csum_add(q[0], 0.5 * m * (u * u + v * v + w * w));
        csum_add(q[1], 0.5 * m * phi[i]);
        csum_add(q[2], m * u);
        csum_add(q[3], m * v);
        csum_add(q[4], m * w);
        csum_add(q[5], m * (y * w - z * v));
        csum_add(q[6], m * (z * u - x * w));
        csum_add(q[7], m * (x * v - y * u));
    }
    __shared__ CSum red[4][8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 8; k++) {
        const CSum t = wave_csum(q[k]);
        if (lane == 0) red[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        CSum t = red[0][threadIdx.x];
        for (int w = 1; w < 4; w++) csum_merge(t, red[w][threadIdx.x]);
        part[2 * (blockIdx.x * 8 + threadIdx.x)] = t.s;
        part[2 * (blockIdx.x * 8 + threadIdx.x) + 1] = t.c;
    }
}

// The blocks' partial sums added in a fixed order (compensated), out[k] = s + c.
__global__ __launch_bounds__(64) void k_diag_final(const double *__restrict__ part, int nblk,
                                                   double *__restrict__ out)
{
#pragma clang fp contract(off)
    for (int k = 0; k < 8; k++) {
        CSum t = csum_zero();
        for (int b = threadIdx.x; b < nblk; b += 64) {
            const CSum p{part[2 * (b * 8 + k)], part[2 * (b * 8 + k) + 1]};
            csum_merge(t, p);
        }
        t = wave_csum(t);
        if (threadIdx.x == 0) out[k] = t.s + t.c;
    }
}

// eq. (dt_g): the largest density m / ((4/3) pi r^3) of the massive bodies,
// by a signed 64-bit atomic maximum of its bit pattern (order-preserving for
// non-negative doubles, +inf included; the -1.0 it starts from orders below
// them), so the result does not depend on the order of the updates.
__global__ __launch_bounds__(64) void k_rho_init(long long *__restrict__ work)
{
    if (threadIdx.x == 0) work[0] = __double_as_longlong(-1.0);
}

__global__ __launch_bounds__(256) void k_rho_max(const double *__restrict__ mass,
                                                 const double *__restrict__ radius, int64_t n,
                                                 long long *__restrict__ work,
                                                 uint32_t *__restrict__ status)
{
#pragma clang fp contract(off)
    double best = -1.0;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const double m = mass[i], r = radius[i];
        bad |= !(isfinite(m) && isfinite(r) && m >= 0.0 && r >= 0.0);
        if (!(m > 0.0) || !(r >= 0.0) || !isfinite(r)) continue;
        const double vol = (4.0 / 3.0) * 3.141592653589793 * (r * r * r);
        const double rho = m / vol;  // +inf for a point mass
        best = rho > best ? rho : best;
    }
    for (int o = 32; o > 0; o >>= 1) best = fmax(best, __shfl_xor(best, o));
    if ((threadIdx.x & 63) == 0) {
        if (best >= 0.0) atomicMax(&work[0], __double_as_longlong(best));
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, ST_NONFINITE);
}

__global__ __launch_bounds__(64) void k_dt_from_rho(const long long *__restrict__ work, double G,
                                                    double *__restrict__ out)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0) return;
    const double rho = __longlong_as_double(work[0]);
    out[0] = rho < 0.0 ? __builtin_huge_val() : 0.5 / sqrt(G * rho);
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

hipError_t launch_state_pack(const Workspace &w, hipStream_t s, const double *pos,
                             const double *vel, const double *acc, const double *mass,
                             const double *eps, int64_t n, uint32_t *status)
{
    if (n <= 0) return hipSuccess;
    k_state_pack<<<blocks(n), 256, 0, s>>>(pos, vel, acc, mass, eps, n, w.body, w.tvel, w.tacc,
                                           w.beps2, w.idx[0], status);
    return hipGetLastError();
}

hipError_t launch_state_unpack(const Workspace &w, hipStream_t s, double *pos, double *vel,
                               double *acc, int64_t n)
{
    if (n <= 0) return hipSuccess;
    k_state_unpack<<<blocks(n), 256, 0, s>>>(w.body, w.tvel, w.tacc, w.idx[0], n, pos, vel, acc);
    return hipGetLastError();
}

hipError_t launch_kick(hipStream_t s, double *vel, const double *acc, int64_t n, double dt)
{
    if (n <= 0) return hipSuccess;
    k_kick<<<blocks(3 * n), 256, 0, s>>>(vel, acc, 3 * n, 0.5 * dt);
    return hipGetLastError();
}

hipError_t launch_dt_bound(hipStream_t s, const double *mass, const double *radius, int64_t n,
                           double G, long long *work, double *out, uint32_t *status)
{
    k_rho_init<<<1, 64, 0, s>>>(work);
    if (n > 0) {
        unsigned nb = blocks(n);
        if (nb > 4096u) nb = 4096u;
        k_rho_max<<<nb, 256, 0, s>>>(mass, radius, n, work, status);
    }
    k_dt_from_rho<<<1, 64, 0, s>>>(work, G, out);
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
