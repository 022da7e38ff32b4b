// Barnes-Hut walk (subsection "Force computation"), one wavefront per group
// of 64 Morton-consecutive target bodies.
//
// The paper gives each body its own thread and its own traversal. Here the 64
// lanes of a wave walk the tree together, but every stack entry carries a
// 64-bit lane mask: the lanes whose own traversal reaches that node. At an
// internal node each lane evaluates its own opening test in FP64
// (s^2 < theta^2 D^2, eq. accuracy); the lanes that accept it queue the node
// as one interaction (eq. Force_thetaTrue) and the others carry on into the
// children. A leaf queues its bodies for the lanes that reached it
// (eq. Force_leaf), excluding each lane's own body. So each body gets exactly
// the interaction set of its own depth-first walk, in the same order.
//
// Interactions are queued in LDS and evaluated 64 at a time: lane k fetches
// and converts queue item k once, then every lane sweeps the 64 staged items
// from LDS. In FP32C mode the staged coordinates are FP32 offsets from the
// group's first body (so near pairs keep their precision), pair terms are
// FP32, and each sweep's FP32 partial sums are added into FP64 accumulators.
#include "bhx_impl.h"

namespace bhx {
namespace {

constexpr int kStack = 256;  // >= 7 pending siblings x 22 levels + 8
constexpr int kQueue = 128;  // a flush happens at 64; a leaf chunk adds <= 64
constexpr int kBatch = 64;

struct alignas(16) ItemF {  // FP32C staged source
    float x, y, z, m;
    float e2h;     // half of the source's squared softening
    int32_t src;   // sorted body index, or ~node
    uint32_t mlo, mhi;
};
struct alignas(16) ItemD {  // FP64 staged source
    double x, y, z, m;
    double e2;  // source's squared softening (eps_j^2 or <eps^2>_N)
    int32_t src, pad;
    uint64_t mask;
};

__device__ inline uint64_t uniform64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The opening test, rounded exactly as written: accept iff s^2 < theta^2 D^2.
__device__ inline bool accept_node(double cx, double cy, double cz, double bx, double by,
                                   double bz, double s2, double th2)
{
#pragma clang fp contract(off)
    double dx = cx - bx, dy = cy - by, dz = cz - bz;
    double D2 = dx * dx + dy * dy + dz * dz;
    return s2 < th2 * D2;
}

template <int PREC, bool PEPS, bool PHI, bool CNT>
__global__ __launch_bounds__(64) void k_walk(
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const NodeInfo *__restrict__ ninfo, const NodeMom *__restrict__ nmom,
    const double *__restrict__ neps2, const uint32_t *__restrict__ idx,
    const TreeHeader *__restrict__ hdr, uint32_t *__restrict__ status, int64_t n, double th2,
    double eps0sq, double G, double *__restrict__ acc, double *__restrict__ phi,
    int32_t *__restrict__ counts)
{
    using Item = typename std::conditional<PREC == BH_FP64, ItemD, ItemF>::type;
    __shared__ int32_t st_node[kStack];
    __shared__ uint64_t st_mask[kStack];
    __shared__ int32_t q_src[kQueue];
    __shared__ uint64_t q_mask[kQueue];
    __shared__ Item items[kBatch];
    __shared__ double s2tab[kLevels];

    const int lane = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * 64;
    const int64_t s = g0 + lane;
    const bool valid = s < n;
    const int32_t self = (int32_t)s;
    const Body me = body[valid ? s : g0];
    const double eb2 = PEPS ? beps2[valid ? s : g0] : 0.0;
    const uint64_t active = __ballot(valid);
    if (lane < kLevels) s2tab[lane] = hdr->s2[lane];

    // FP32C: coordinates relative to the group's first body
    const Body org = body[g0];
    const float rx = (float)(me.x - org.x), ry = (float)(me.y - org.y), rz = (float)(me.z - org.z);
    const float e2hB = (float)(0.5 * eb2);
    const float eps0f = (float)eps0sq;
    const bool lane_hi = lane >= 32;
    const uint32_t lbit = 1u << (lane & 31);

    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    int32_t cnode = 0, cpair = 0;

    int sp = 1, qn = 0;
    if (lane == 0) {
        st_node[0] = 0;
        st_mask[0] = active;
    }
    __syncthreads();

    // Evaluates the first c queued items, then shifts the rest down.
    auto flush = [&](int c) {
        if (lane < c) {
            const int32_t src = q_src[lane];
            const uint64_t mk = q_mask[lane];
            double x, y, z, m, e2;
            if (src >= 0) {
                const Body b = body[src];
                x = b.x, y = b.y, z = b.z, m = b.m;
                e2 = PEPS ? beps2[src] : 0.0;
            } else {
                const NodeMom nm = nmom[~src];
                x = nm.x, y = nm.y, z = nm.z, m = nm.m;
                e2 = PEPS ? neps2[~src] : 0.0;
            }
            if constexpr (PREC == BH_FP64) {
                items[lane] = ItemD{x, y, z, m, e2, src, 0, mk};
            } else {
                items[lane] = ItemF{(float)(x - org.x), (float)(y - org.y), (float)(z - org.z),
                                    (float)m, (float)(0.5 * e2), src, (uint32_t)mk,
                                    (uint32_t)(mk >> 32)};
            }
        }
        __syncthreads();
        if constexpr (PREC == BH_FP64) {
            for (int j = 0; j < c; j++) {
                const ItemD it = items[j];
                const bool on = ((it.mask >> lane) & 1ull) && it.src != self;
                const double dx = it.x - me.x, dy = it.y - me.y, dz = it.z - me.z;
                const double e2 = PEPS ? 0.5 * (eb2 + it.e2) : eps0sq;
                const double r2 = dx * dx + dy * dy + dz * dz + e2;
                if (on && r2 > 0.0) {
                    const double r = sqrt(r2);
                    const double inv3 = 1.0 / (r2 * r);
                    ax += it.m * dx * inv3;
                    ay += it.m * dy * inv3;
                    az += it.m * dz * inv3;
                    if (PHI) ph -= it.m / r;
                }
                if (CNT && on) {
                    if (it.src < 0)
                        cnode++;
                    else
                        cpair++;
                }
            }
        } else {
            float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
            for (int j = 0; j < c; j++) {
                const ItemF it = items[j];
                const bool on = ((lane_hi ? it.mhi : it.mlo) & lbit) && it.src != self;
                const float dx = it.x - rx, dy = it.y - ry, dz = it.z - rz;
                const float e2 = PEPS ? it.e2h + e2hB : eps0f;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, e2)));
                const float rinv = (on && r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f;
                const float mr = it.m * rinv;
                const float mr3 = mr * rinv * rinv;
                fx = fmaf(mr3, dx, fx);
                fy = fmaf(mr3, dy, fy);
                fz = fmaf(mr3, dz, fz);
                if (PHI) fp -= mr;
                if (CNT && on) {
                    if (it.src < 0)
                        cnode++;
                    else
                        cpair++;
                }
            }
            ax += (double)fx;
            ay += (double)fy;
            az += (double)fz;
            if (PHI) ph += (double)fp;
        }
        const int rem = qn - c;
        int32_t t_src = 0;
        uint64_t t_mask = 0;
        if (lane < rem) {
            t_src = q_src[c + lane];
            t_mask = q_mask[c + lane];
        }
        __syncthreads();
        if (lane < rem) {
            q_src[lane] = t_src;
            q_mask[lane] = t_mask;
        }
        qn = rem;
        __syncthreads();
    };

    while (sp > 0) {
        sp--;
        const int32_t k = __builtin_amdgcn_readfirstlane(st_node[sp]);
        const uint64_t M = uniform64(st_mask[sp]);
        const NodeInfo info = ninfo[k];
        if (info.child0 < 0) {
            // leaf: every body for the lanes that reached it
            for (int off = 0; off < info.count; off += 64) {
                const int c = min(64, info.count - off);
                __syncthreads();
                if (lane < c) {
                    q_src[qn + lane] = info.first + off + lane;
                    q_mask[qn + lane] = M;
                }
                qn += c;
                __syncthreads();
                if (qn >= kBatch) flush(kBatch);
            }
        } else {
            const NodeMom nm = nmom[k];
            const bool ok = accept_node(nm.x, nm.y, nm.z, me.x, me.y, me.z,
                                        s2tab[node_level(info)], th2);
            const uint64_t A = __ballot(ok) & M;
            const uint64_t O = M & ~A;
            __syncthreads();
            if (A) {
                if (lane == 0) {
                    q_src[qn] = ~k;
                    q_mask[qn] = A;
                }
                qn++;
            }
            if (O) {
                const int nch = node_nchild(info);
                if (sp + nch > kStack) {
                    if (lane == 0) atomicOr(status, ST_STACK);
                    break;
                }
                if (lane < nch) {
                    st_node[sp + nch - 1 - lane] = info.child0 + lane;
                    st_mask[sp + nch - 1 - lane] = O;
                }
                sp += nch;
            }
            __syncthreads();
            if (qn >= kBatch) flush(kBatch);
        }
    }
    while (qn > 0) flush(min(qn, kBatch));

    if (valid) {
        const int64_t o = idx[s];
        acc[3 * o] = G * ax;
        acc[3 * o + 1] = G * ay;
        acc[3 * o + 2] = G * az;
        if (PHI) phi[o] = G * ph;
        if (CNT) {
            counts[2 * o] = cnode;
            counts[2 * o + 1] = cpair;
        }
    }
}

template <int PREC, bool PEPS, bool PHI, bool CNT>
hipError_t launch_t(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    const unsigned grid = (unsigned)((p.n + 63) / 64);
    k_walk<PREC, PEPS, PHI, CNT><<<grid, 64, 0, s>>>(
        w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.idx[0], w.hdr, &w.hdr->status, p.n, p.th2,
        p.eps0sq, p.G, p.acc, p.phi, p.counts);
    return hipGetLastError();
}

template <int PREC, bool PEPS>
hipError_t launch_p(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    const bool phi = p.phi != nullptr, cnt = p.counts != nullptr;
    if (phi && cnt) return launch_t<PREC, PEPS, true, true>(w, s, p);
    if (phi) return launch_t<PREC, PEPS, true, false>(w, s, p);
    if (cnt) return launch_t<PREC, PEPS, false, true>(w, s, p);
    return launch_t<PREC, PEPS, false, false>(w, s, p);
}

}  // namespace

hipError_t launch_walk(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    if (p.n <= 0) return hipSuccess;
    if (p.precision == BH_FP64)
        return p.per_body_eps ? launch_p<BH_FP64, true>(w, s, p)
                              : launch_p<BH_FP64, false>(w, s, p);
    return p.per_body_eps ? launch_p<BH_FP32C, true>(w, s, p) : launch_p<BH_FP32C, false>(w, s, p);
}

}  // namespace bhx
