// Direct N^2 sum, eq. (Newton) with every term softened as in
// eq. (Force_rComp): a_i = G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps_ij^2)^(3/2).
//
// One thread per target, 256 targets per block; sources stream through LDS in
// tiles of 256 (positions in FP64 so that d_ij is formed in FP64 even in FP32C
// mode, where only the pair arithmetic after the difference is FP32 and FP32
// partial sums over at most 32 sources are added into FP64 accumulators).
// When the targets give too few blocks to fill the GPU, block row y sums only
// the y-th range of source tiles into a partial buffer, and a second kernel
// adds the rows in order (so the result does not depend on scheduling).
#include <cmath>
#include <mutex>
#include <type_traits>

#include "bhx_impl.h"

namespace bhx {
namespace {

constexpr int kTile = 256;

// One source as a tile holds it in LDS: one record per source, so a sweep
// reads it from a single address with immediate offsets.
struct alignas(16) SrcD {  // FP64: position, mass, half the squared softening
    double x, y, z, m, eh, pad;
};
struct alignas(16) SrcF {  // FP32C: FP64 position; FP32 mass and half squared softening
    double x, y, z;
    float m, eh;
};

template <int PREC, bool PEPS, bool PHI>
__global__ __launch_bounds__(kTile) void k_direct(const double *__restrict__ pos,
                                                  const double *__restrict__ mass,
                                                  const double *__restrict__ eps, int64_t n,
                                                  double eps0sq, double G,
                                                  double *__restrict__ acc,
                                                  double *__restrict__ phi, int64_t chunk,
                                                  double *__restrict__ part)
{
    using Src = typename std::conditional<PREC == BH_FP64, SrcD, SrcF>::type;
    __shared__ Src src[kTile];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kTile + tid;
    const bool valid = i < n;
    const double xi = valid ? pos[3 * i] : 0.0, yi = valid ? pos[3 * i + 1] : 0.0,
                 zi = valid ? pos[3 * i + 2] : 0.0;
    double ei2 = 0.0;
    if (PEPS && valid) {
        const double e = eps[i];
        ei2 = e * e;
    }
    const double ehi = 0.5 * ei2;  // (eps_i^2 + eps_j^2) / 2 = ehi + eps_j^2 / 2 exactly
    const float e2hB = (float)ehi;
    const float eps0f = (float)eps0sq;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;

    // this block row's sources: [s_lo, s_hi)
    const int64_t s_lo = (int64_t)blockIdx.y * chunk;
    const int64_t s_hi = s_lo + chunk < n ? s_lo + chunk : n;
    for (int64_t base = s_lo; base < s_hi; base += kTile) {
        const int64_t j = base + tid;
        if (j < s_hi) {
            double eh = 0.0;
            if (PEPS) {
                const double e = eps[j];
                eh = 0.5 * (e * e);
            }
            if constexpr (PREC == BH_FP64)
                src[tid] = SrcD{pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], mass[j], eh, 0.0};
            else  // the FP32 operands, rounded once per source
                src[tid] = SrcF{pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], (float)mass[j],
                                (float)eh};
        }
        __syncthreads();
        const int cnt = (int)((s_hi - base) < kTile ? (s_hi - base) : kTile);
        const int skip = (valid && i >= base && i < base + cnt) ? (int)(i - base) : -1;
        if constexpr (PREC == BH_FP64) {
#pragma unroll 4
            for (int jj = 0; jj < cnt; jj++) {
                const SrcD q = src[jj];
                const double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                const double e2 = PEPS ? ehi + q.eh : eps0sq;
                const double r2 = dx * dx + dy * dy + dz * dz + e2;
                if (jj != skip && positive_normal(r2)) {
                    const double rinv = rsqrt_f64(r2);
                    const double inv3 = rinv * rinv * rinv;
                    ax += q.m * dx * inv3;
                    ay += q.m * dy * inv3;
                    az += q.m * dz * inv3;
                    if (PHI) ph -= q.m * rinv;
                }
            }
        } else {
            for (int j0 = 0; j0 < cnt; j0 += 32) {
                const int jn = j0 + 32 < cnt ? j0 + 32 : cnt;
                float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
#pragma unroll 4
                for (int jj = j0; jj < jn; jj++) {
                    const SrcF q = src[jj];
                    const float dx = (float)(q.x - xi), dy = (float)(q.y - yi),
                                dz = (float)(q.z - zi);
                    const float e2 = PEPS ? q.eh + e2hB : eps0f;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, e2)));
                    const float rinv =
                        (jj != skip && positive_normal_f(r2)) ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    const float mr = q.m * rinv;
                    const float mr3 = mr * rinv * rinv;
                    fx = fmaf(mr3, dx, fx);
                    fy = fmaf(mr3, dy, fy);
                    fz = fmaf(mr3, dz, fz);
                    if (PHI) fp -= mr;
                }
                ax += (double)fx;
                ay += (double)fy;
                az += (double)fz;
                if (PHI) ph += (double)fp;
            }
        }
        __syncthreads();
    }
    if (valid && gridDim.y == 1) {
        acc[3 * i] = G * ax;
        acc[3 * i + 1] = G * ay;
        acc[3 * i + 2] = G * az;
        if (PHI) phi[i] = G * ph;
    } else if (valid) {
        double *q = part + 4 * ((int64_t)blockIdx.y * n + i);
        q[0] = ax;
        q[1] = ay;
        q[2] = az;
        q[3] = ph;
    }
}

// acc_i = G * sum over the block rows of their partial sums, in row order.
__global__ __launch_bounds__(256) void k_direct_reduce(const double *__restrict__ part,
                                                       int64_t n, int rows, double G,
                                                       double *__restrict__ acc,
                                                       double *__restrict__ phi)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    for (int r = 0; r < rows; r++) {
        const double *q = part + 4 * ((int64_t)r * n + i);
        ax += q[0];
        ay += q[1];
        az += q[2];
        ph += q[3];
    }
    acc[3 * i] = G * ax;
    acc[3 * i + 1] = G * ay;
    acc[3 * i + 2] = G * az;
    if (phi) phi[i] = G * ph;
}

template <int PREC, bool PEPS>
hipError_t launch_p(hipStream_t s, const double *pos, const double *mass, const double *eps,
                    int64_t n, double eps0sq, double G, double *acc, double *phi, double *part)
{
    // rows of source ranges (whole tiles) so that targets x rows reaches
    // kDirectBlocks; rows * n <= kDirectBlocks * kTile fits the partial buffer
    const int64_t tb = (n + kTile - 1) / kTile;
    int64_t rows = tb >= kDirectBlocks ? 1 : kDirectBlocks / tb;
    if (rows > kDirectSplits) rows = kDirectSplits;
    if (rows > tb) rows = tb;  // at least one source tile per row
    const int64_t tiles = (tb + rows - 1) / rows;
    const int64_t chunk = tiles * kTile;
    rows = (tb + tiles - 1) / tiles;
    if (!part) rows = 1;
    const dim3 grid((unsigned)tb, (unsigned)rows);
    const int64_t ch = rows == 1 ? n : chunk;
    if (phi)
        k_direct<PREC, PEPS, true>
            <<<grid, kTile, 0, s>>>(pos, mass, eps, n, eps0sq, G, acc, phi, ch, part);
    else
        k_direct<PREC, PEPS, false>
            <<<grid, kTile, 0, s>>>(pos, mass, eps, n, eps0sq, G, acc, phi, ch, part);
    if (rows > 1)
        k_direct_reduce<<<(unsigned)tb, 256, 0, s>>>(part, n, (int)rows, G, acc, phi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_direct(hipStream_t s, const double *pos, const double *mass, const double *eps,
                         int64_t n, double eps0sq, double G, int precision, double *acc,
                         double *phi, double *part)
{
    if (n <= 0) return hipSuccess;
    if (precision == BH_FP64)
        return eps ? launch_p<BH_FP64, true>(s, pos, mass, eps, n, eps0sq, G, acc, phi, part)
                   : launch_p<BH_FP64, false>(s, pos, mass, eps, n, eps0sq, G, acc, phi, part);
    return eps ? launch_p<BH_FP32C, true>(s, pos, mass, eps, n, eps0sq, G, acc, phi, part)
               : launch_p<BH_FP32C, false>(s, pos, mass, eps, n, eps0sq, G, acc, phi, part);
}

}  // namespace bhx

// ------------------------------------------------- no-allocation entry point

namespace {

// The split-row partial sums of bh_compute_accel_direct_noalloc: one array
// per device, held by the library until the process ends and shared by every
// call on that device (calls that overlap on one device race on it).
__device__ __align__(256) double scratch[bhx::kDirectPart];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// The device address of this device's scratch array (the array's name is
// only a host-side stand-in), looked up once per device with it current.
bh_status scratch_ptr(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BH_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BH_E_HIP;
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return BH_OK;
}

}  // namespace

extern "C" bh_status bh_compute_accel_direct_noalloc(void *hip_stream, int32_t precision,
                                                     double G, const double *pos,
                                                     const double *mass, double softening,
                                                     const double *eps, double *acc, double *phi,
                                                     int64_t n)
{
    if (n < 0 || n > BH_NOALLOC_MAX_N) return BH_E_CAPACITY;
    if (precision != BH_FP64 && precision != BH_FP32C) return BH_E_INVALID;
    if (!std::isfinite(G)) return BH_E_INVALID;
    if (!(std::isfinite(softening) && softening >= 0.0)) return BH_E_INVALID;
    if (n > 0 && (!pos || !mass || !acc)) return BH_E_INVALID;
    if (n == 0) return BH_OK;
    double *part = nullptr;
    const bh_status st = scratch_ptr(&part);
    if (st != BH_OK) return st;
    // every partial sum is written before it is read (no clearing needed):
    // row r of the split writes 4 doubles for each of the n targets
    const hipError_t e = bhx::launch_direct((hipStream_t)hip_stream, pos, mass, eps, n,
                                            softening * softening, G, precision, acc, phi, part);
    return e == hipSuccess ? BH_OK : BH_E_HIP;
}
