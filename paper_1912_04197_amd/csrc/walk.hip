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
// (eq. Force_leaf), each lane's own body excluded from its mask. So each body
// gets exactly the interaction set of its own walk; only the summation order
// differs from a depth-first walk.
//
// Traversal: a stack entry is the child range of one opened node with the
// mask of the lanes that opened it. Each round pops up to 8 ranges (up to 64
// nodes), the lanes load those nodes in parallel into LDS (one memory latency
// per round instead of one per node), and the wave then decides them one after
// another from LDS. A round pops only as many ranges as can be expanded while
// leaving room for a depth-first descent, so the stack cannot overflow.
//
// Evaluation: interactions are queued in LDS and evaluated 64 at a time: lane
// k fetches queue item k and stages it, then every lane sweeps the staged
// items. In FP32C mode each pair offset x_j - x_B is formed in FP64 and
// rounded once to FP32 (close pairs keep full FP32 precision whatever the
// group's extent), the rest of the pair term is FP32, and FP32 partial sums
// over at most 16 items are added into FP64 accumulators.
#include <type_traits>

#include "bhx_impl.h"

namespace bhx {
namespace {

constexpr int kStack = 320;    // LDS traversal stack of child ranges
constexpr int kReserve = 150;  // a depth-first descent adds <= 7 ranges per level
constexpr int kRanges = 8;     // ranges popped per round (<= 8 nodes each)
constexpr int kPop = 8 * kRanges;
constexpr int kQueue = 128;  // a flush happens at 64; a leaf chunk adds <= 64
constexpr int kBatch = 64;
constexpr int kFlush = 16;   // FP32 partial sums span at most this many items

struct alignas(16) ItemF {  // FP32C staged source
    double x, y, z;
    float m;
    float e2h;  // half of the source's squared softening
    uint32_t mlo, mhi;
    int32_t src;  // sorted body index, or ~node
    int32_t pad;
};
struct alignas(16) ItemD {  // FP64 staged source
    double x, y, z, m;
    double e2;  // source's squared softening (eps_j^2 or <eps^2>_N)
    uint64_t mask;
    int32_t src, pad0;
    int64_t pad1;
};
struct alignas(16) PopNode {  // a popped stack entry with its node loaded
    double x, y, z, s2;
    uint64_t mask;
    int32_t first, count, child0, nch;  // child0 < 0: leaf
    int32_t node, pad0;
    int64_t pad1;
};

__device__ inline uint64_t uniform64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline int32_t uniform32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

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
    const TreeHeader *__restrict__ hdr, int64_t n, int ngroups,
    int per_xcd, double th2, double eps0sq, double G, double *__restrict__ acc,
    double *__restrict__ phi, int32_t *__restrict__ counts)
{
    using Item = typename std::conditional<PREC == BH_FP64, ItemD, ItemF>::type;
    __shared__ int32_t st_c0[kStack];
    __shared__ int32_t st_n[kStack];
    __shared__ uint64_t st_mask[kStack];
    __shared__ PopNode pn[kPop];
    __shared__ int32_t q_src[kQueue];
    __shared__ uint64_t q_mask[kQueue];
    __shared__ Item items[kBatch];
    __shared__ double s2tab[kLevels];

    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // (so spatially compact) range of groups to share its L2.
    const int grp = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
    if (grp >= ngroups) return;

    const int lane = threadIdx.x;
    const int64_t g0 = (int64_t)grp * 64;
    const int64_t s = g0 + lane;
    const bool valid = s < n;
    const Body me = body[valid ? s : g0];
    const double eb2 = PEPS ? beps2[valid ? s : g0] : 0.0;
    const uint64_t active = __ballot(valid);
    if (lane < kLevels) s2tab[lane] = hdr->s2[lane];

    const float e2hB = (float)(0.5 * eb2);
    const float eps0f = (float)eps0sq;
    const bool lane_hi = lane >= 32;
    const uint32_t lbit = 1u << (lane & 31);

    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    int32_t cnode = 0, cpair = 0;

    int sp = 1, qn = 0;
    if (lane == 0) {
        st_c0[0] = 0;  // the root, as a range of one
        st_n[0] = 1;
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
                items[lane] = ItemD{x, y, z, m, e2, mk, src, 0, 0};
            } else {
                items[lane] = ItemF{x,   y, z, (float)m, (float)(0.5 * e2), (uint32_t)mk,
                                    (uint32_t)(mk >> 32), src, 0};
            }
        }
        __syncthreads();
        if constexpr (PREC == BH_FP64) {
#pragma unroll 1
            for (int j = 0; j < c; j++) {
                const ItemD it = items[j];
                const bool on = (it.mask >> lane) & 1ull;
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
#pragma unroll 1
            for (int j0 = 0; j0 < c; j0 += kFlush) {
                const int jn = min(c, j0 + kFlush);
                float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
#pragma unroll 2
                for (int j = j0; j < jn; j++) {
                    const ItemF it = items[j];
                    const bool on = (lane_hi ? it.mhi : it.mlo) & lbit;
                    const float dx = (float)(it.x - me.x), dy = (float)(it.y - me.y),
                                dz = (float)(it.z - me.z);
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
        // Pop cr ranges: after expanding them (each popped range may push up
        // to 8 ranges) at least kReserve entries stay free for a depth-first
        // descent, which adds at most 7 ranges per level below.
        int cr = min(kRanges, sp);
        const int room = (kStack - kReserve - sp) / 7;
        if (cr > room) cr = room > 1 ? room : 1;
        const int base = sp - cr;
        {
            const int r = lane >> 3, o = lane & 7;
            int32_t k = -1;
            uint64_t mk = 0;
            if (r < cr) {
                const int e = base + r;
                if (o < st_n[e]) {
                    k = st_c0[e] + o;
                    mk = st_mask[e];
                }
            }
            PopNode p;
            p.node = k;
            if (k >= 0) {
                const NodeInfo info = ninfo[k];
                const NodeMom nm = nmom[k];
                p.x = nm.x, p.y = nm.y, p.z = nm.z;
                p.s2 = s2tab[node_level(info)];
                p.mask = mk;
                p.first = info.first, p.count = info.count, p.child0 = info.child0;
                p.nch = node_nchild(info);
            }
            pn[lane] = p;
        }
        sp = base;
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < kPop; j++) {
            if (uniform32(pn[j].node) < 0) continue;
            const uint64_t M = uniform64(pn[j].mask);
            const int32_t child0 = uniform32(pn[j].child0);
            if (child0 < 0) {
                // leaf: its bodies, for the lanes that reached it
                const int32_t first = uniform32(pn[j].first);
                const int32_t count = uniform32(pn[j].count);
                for (int off = 0; off < count; off += 64) {
                    const int cc = min(64, count - off);
                    if (lane < cc) {
                        const int32_t src = first + off + lane;
                        const int64_t rel = (int64_t)src - g0;
                        uint64_t mk = M;
                        if (rel >= 0 && rel < 64) mk &= ~(1ull << rel);  // not itself
                        q_src[qn + lane] = src;
                        q_mask[qn + lane] = mk;
                    }
                    qn += cc;
                    __syncthreads();
                    if (qn >= kBatch) flush(kBatch);
                }
            } else {
                const bool ok = accept_node(pn[j].x, pn[j].y, pn[j].z, me.x, me.y, me.z,
                                            pn[j].s2, th2);
                const uint64_t A = __ballot(ok) & M;
                const uint64_t O = M & ~A;
                if (A) {
                    // accepted by the lanes in A: one monopole interaction
                    if (lane == 0) {
                        q_src[qn] = ~pn[j].node;
                        q_mask[qn] = A;
                    }
                    qn++;
                }
                if (O) {
                    // opened by the lanes in O: visit all of its children
                    if (lane == 0) {
                        st_c0[sp] = child0;
                        st_n[sp] = pn[j].nch;
                        st_mask[sp] = O;
                    }
                    sp++;
                }
                __syncthreads();
                if (qn >= kBatch) flush(kBatch);
            }
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
    const int ngroups = (int)((p.n + 63) / 64);
    const int per_xcd = (ngroups + 7) / 8;
    k_walk<PREC, PEPS, PHI, CNT><<<8 * per_xcd, 64, 0, s>>>(
        w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.idx[0], w.hdr, p.n, ngroups,
        per_xcd, p.th2, p.eps0sq, p.G, p.acc, p.phi, p.counts);
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
