// Barnes-Hut walk (subsection "Force computation"): one wavefront serves a
// group of GB Morton-consecutive target bodies (GB = 64, 32 or 16), with
// 64 / GB lanes per body.
//
// The paper gives each body its own thread and its own traversal. Here the
// lanes of a wave walk the tree together, but every stack entry carries a
// GB-bit body mask: the bodies whose own traversal reaches that node. At an
// internal node each body evaluates its own opening test in FP64
// (s^2 < theta^2 D^2, eq. accuracy); the bodies that accept it take the node
// as one interaction (eq. Force_thetaTrue) and the others carry on into the
// children. A leaf contributes its bodies one by one (eq. Force_leaf) to the
// bodies that reached it, each body's own index cleared from its mask. So each
// body gets exactly the interaction set of its own walk; only the summation
// order differs from a depth-first walk.
//
// Traversal rounds: a stack entry is the child range of one opened node with
// its body mask. A round pops up to 8 ranges (up to 64 nodes); the lanes load
// those nodes in parallel (one memory latency per round), test them against
// the group (64 / GB nodes per instruction), and then do the bookkeeping for
// all popped nodes at once: lane p handles popped node p, and prefix sums over
// the lanes place the pushed child ranges and the queued interactions. A round
// pops only as many ranges as can be expanded while keeping room for a
// depth-first descent, so the stack cannot overflow.
//
// Evaluation: the interaction queue holds descriptors (a leaf's body range or
// one accepted node, with a body mask). Whenever 64 items are queued, lane k
// expands item k (binary search over the descriptors' item offsets), loads it
// and stages it in LDS; then the lanes of each body sweep the staged items,
// each taking every (64 / GB)-th one. In FP32C mode each pair offset
// x_j - x_B is formed in FP64 and rounded once to FP32 (close pairs keep full
// FP32 precision whatever the group's extent), the rest of the pair term is
// FP32, and FP32 partial sums over at most 16 items per lane are added into
// FP64 accumulators. The per-lane FP64 sums of a body are added at the end in
// a fixed order, so results are deterministic.
#include <cstddef>
#include <type_traits>

#include "bhx_impl.h"

namespace bhx {
namespace {

constexpr int kStack = 320;    // LDS traversal stack of child ranges
constexpr int kReserve = 150;  // a depth-first descent adds <= 7 ranges per level
constexpr int kRanges = 8;     // ranges popped per round (<= 8 nodes each)
constexpr int kPop = 8 * kRanges;
constexpr int kRing = 128;     // interaction descriptors: <= 64 left over + 64 new
constexpr int kBatch = 64;     // items staged per evaluation batch
constexpr int kFlush = 16;     // FP32 partial sums span at most this many items per lane

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
struct alignas(16) PopCom {  // popped node as the opening test needs it
    double x, y, z, s2;      // s2 = +inf for a leaf (never accepted)
};
struct alignas(16) PopData {  // popped node as the bookkeeping needs it
    uint64_t mask;
    int32_t node, first, count, child0;  // child0 < 0: leaf
    int32_t nch, pad;
};

__device__ inline int32_t uniform32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint32_t lanes_below(uint64_t m)  // set bits of m below this lane
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes (exact, integer).
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
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

template <int PREC, bool PEPS, bool PHI, bool CNT, int GB>
__global__ __launch_bounds__(64) void k_walk(
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const NodeInfo *__restrict__ ninfo, const NodeMom *__restrict__ nmom,
    const double *__restrict__ neps2, const uint32_t *__restrict__ idx,
    const SceneBox *__restrict__ box, const int32_t *__restrict__ groups, int64_t n,
    int ngroups, int per_xcd, double th2, double eps0sq, double G, double *__restrict__ acc,
    double *__restrict__ phi, int32_t *__restrict__ counts)
{
    static_assert(GB == 64 || GB == 32 || GB == 16, "group size");
    constexpr int LPB = 64 / GB;  // lanes per body
    constexpr uint64_t kBodyMask = GB == 64 ? ~0ull : ((1ull << GB) - 1ull);
    using Item = typename std::conditional<PREC == BH_FP64, ItemD, ItemF>::type;

    __shared__ int32_t st_c0[kStack];
    __shared__ int32_t st_n[kStack];
    __shared__ uint64_t st_mask[kStack];
    __shared__ int32_t dq_a[kRing];      // leaf: first body; node: ~node
    __shared__ int32_t dq_n[kRing];      // items in the descriptor
    __shared__ uint32_t dq_at[kRing];    // running item number of its first item
    __shared__ uint64_t dq_mask[kRing];
    __shared__ double s2tab[kLevels];
    // The popped nodes are read only before a round's evaluations and the
    // staged items only during them, so the two share one LDS region.
    union Shared {
        struct {
            PopCom pc[kPop];
            PopData pd[kPop];
        } pop;
        Item items[kBatch];
    };
    __shared__ Shared sh;
    PopCom *const pc = sh.pop.pc;
    PopData *const pd = sh.pop.pd;
    Item *const items = sh.items;

    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous
    // (so spatially compact) range of groups to share its L2.
    const int grp = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
    if (grp >= ngroups) return;

    const int lane = threadIdx.x;
    const int bq = GB == 64 ? lane : lane % GB;  // body of this lane within the group
    const int sub = GB == 64 ? 0 : lane / GB;    // which share of the items it sweeps
    // the group: up to GB consecutive sorted bodies of one scene
    int64_t g0 = (int64_t)grp * GB;
    int gcount = (int)min((int64_t)GB, n - g0);
    int scene = 0;
    if (groups) {
        g0 = groups[3 * grp];
        gcount = groups[3 * grp + 1];
        scene = groups[3 * grp + 2];
    }
    const int64_t s = g0 + bq;
    const bool valid = bq < gcount;
    const Body me = body[valid ? s : g0];
    const double eb2 = PEPS ? beps2[valid ? s : g0] : 0.0;
    const uint64_t active = __ballot(valid) & kBodyMask;
    if (lane < kLevels) s2tab[lane] = box[scene].s2[lane];

    const float e2hB = (float)(0.5 * eb2);
    const float eps0f = (float)eps0sq;
    const int woff = (int)offsetof(ItemF, mlo) + (bq >= 32 ? 4 : 0);

    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    int32_t cnode = 0, cpair = 0;

    int sp = 1;              // stack entries
    int dq_head = 0, dq_tail = 0;
    uint32_t queued = 0;     // items ever queued
    uint32_t consumed = 0;   // items ever evaluated
    if (lane == 0) {
        st_c0[0] = scene;  // the scene's root (node `scene`), as a range of one
        st_n[0] = 1;
        st_mask[0] = active;
    }
    __syncthreads();

    // Stages the next c queued items and sweeps them.
    auto evaluate = [&](int c) {
        if (lane < c) {
            const uint32_t q = consumed + (uint32_t)lane;
            int lo = 0, hi = dq_tail - dq_head - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (dq_at[(dq_head + mid) % kRing] <= q)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int d = (dq_head + lo) % kRing;
            const int32_t a = dq_a[d];
            uint64_t mk = dq_mask[d];
            int32_t src;
            double x, y, z, m, e2;
            if (a >= 0) {
                src = a + (int32_t)(q - dq_at[d]);
                const int64_t rel = (int64_t)src - g0;
                if (rel >= 0 && rel < GB) mk &= ~(1ull << rel);  // not itself
                const Body b = body[src];
                x = b.x, y = b.y, z = b.z, m = b.m;
                e2 = PEPS ? beps2[src] : 0.0;
            } else {
                src = a;
                const NodeMom nm = nmom[~a];
                x = nm.x, y = nm.y, z = nm.z, m = nm.m;
                e2 = PEPS ? neps2[~a] : 0.0;
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
            for (int jj = 0; jj < c; jj += LPB) {
                const int j = jj + sub;
                const ItemD it = items[j < c ? j : jj];
                const bool on = j < c && ((it.mask >> bq) & 1ull);
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
            for (int j0 = 0; j0 < c; j0 += kFlush * LPB) {
                const int jn = min(c, j0 + kFlush * LPB);
                float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
                // jj is the same on every lane; lane share `sub` takes item jj + sub
#pragma unroll 2
                for (int jj = j0; jj < jn; jj += LPB) {
                    const int j = jj + sub;
                    const ItemF it = items[j < jn ? j : jj];
                    bool on;
                    if constexpr (GB == 64) {
                        // lanes 32..63 read the high word of the body mask
                        const uint32_t w = *(const uint32_t *)((const char *)&items[jj] + woff);
                        on = (w >> (bq & 31)) & 1u;
                    } else {
                        on = j < jn && ((it.mlo >> bq) & 1u);
                    }
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
        consumed += (uint32_t)c;
        // retire fully evaluated descriptors
        while (dq_head < dq_tail) {
            const int d = dq_head % kRing;
            const uint32_t end = (uint32_t)uniform32((int32_t)(dq_at[d] + (uint32_t)dq_n[d]));
            if (end > consumed) break;
            dq_head++;
        }
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
        int32_t k = -1;
        uint64_t mk = 0;
        {
            const int r = lane >> 3, o = lane & 7;
            if (r < cr) {
                const int e = base + r;
                if (o < st_n[e]) {
                    k = st_c0[e] + o;
                    mk = st_mask[e];
                }
            }
        }
        // compact the popped nodes into slots 0..nv-1
        const uint64_t vb = __ballot(k >= 0);
        const int nv = __popcll(vb);
        if (k >= 0) {
            const int slot = (int)lanes_below(vb);
            const NodeInfo info = ninfo[k];
            const NodeMom nm = nmom[k];
            const bool leaf = info.child0 < 0;
            pc[slot] = PopCom{nm.x, nm.y, nm.z,
                              leaf ? __builtin_huge_val() : s2tab[node_level(info)]};
            pd[slot] = PopData{mk, k, info.first, info.count, info.child0, node_nchild(info), 0};
        }
        sp = base;
        __syncthreads();

        // Opening tests: 64 / GB popped nodes per step, one per share of
        // lanes. The group's GB-bit result for popped node p goes to lane p.
        uint64_t accepted = 0;
#pragma unroll 1
        for (int p0 = 0; p0 < nv; p0 += LPB) {
            const int p = p0 + sub;
            const PopCom q = pc[p < nv ? p : 0];
            const bool ok = p < nv && accept_node(q.x, q.y, q.z, me.x, me.y, me.z, q.s2, th2);
            const uint64_t bal = __ballot(ok);
#pragma unroll
            for (int t = 0; t < LPB; t++) {
                const uint64_t field = (bal >> (t * GB)) & kBodyMask;
                if (lane == p0 + t) accepted = field;
            }
        }

        // Bookkeeping for popped node `lane`, all lanes at once.
        const bool mine = lane < nv;
        PopData my = PopData{0ull, 0, 0, 0, 0, 0, 0};
        if (mine) my = pd[lane];
        const bool leaf = mine && my.child0 < 0;
        const uint64_t M = my.mask;
        const uint64_t A = (mine && !leaf) ? (accepted & M) : 0ull;
        const uint64_t O = (mine && !leaf) ? (M & ~accepted) : 0ull;
        // opened by the bodies in O: push the child range
        const uint64_t pushb = __ballot(O != 0);
        if (O != 0) {
            const int e = sp + (int)lanes_below(pushb);
            st_c0[e] = my.child0;
            st_n[e] = my.nch;
            st_mask[e] = O;
        }
        sp += __popcll(pushb);
        // a leaf, or accepted by the bodies in A: queue a descriptor
        const bool hasq = leaf || A != 0;
        const uint64_t qb = __ballot(hasq);
        const uint32_t nitems = leaf ? (uint32_t)my.count : (A != 0 ? 1u : 0u);
        const uint32_t incl = wave_incl_scan(nitems);
        if (hasq) {
            const int d = (dq_tail + (int)lanes_below(qb)) % kRing;
            dq_a[d] = leaf ? my.first : ~my.node;
            dq_n[d] = (int32_t)nitems;
            dq_at[d] = queued + incl - nitems;
            dq_mask[d] = leaf ? M : A;
        }
        dq_tail += __popcll(qb);
        queued += (uint32_t)__shfl(incl, 63);
        __syncthreads();
        while (queued - consumed >= (uint32_t)kBatch) evaluate(kBatch);
    }
    while (queued != consumed) evaluate((int)min(queued - consumed, (uint32_t)kBatch));

    // add the lanes' partial sums of each body in a fixed order
#pragma unroll
    for (int o = GB; o < 64; o <<= 1) {
        ax += __shfl_xor(ax, o);
        ay += __shfl_xor(ay, o);
        az += __shfl_xor(az, o);
        if (PHI) ph += __shfl_xor(ph, o);
        if (CNT) {
            cnode += __shfl_xor(cnode, o);
            cpair += __shfl_xor(cpair, o);
        }
    }
    if (valid && sub == 0) {
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

template <int PREC, bool PEPS, bool PHI, bool CNT, int GB>
hipError_t launch_t(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    const int ngroups = p.groups ? p.n_groups : (int)((p.n + GB - 1) / GB);
    const int per_xcd = (ngroups + 7) / 8;
    if (ngroups == 0) return hipSuccess;
    k_walk<PREC, PEPS, PHI, CNT, GB><<<8 * per_xcd, 64, 0, s>>>(
        w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.idx[0], w.box, p.groups, p.n, ngroups,
        per_xcd, p.th2, p.eps0sq, p.G, p.acc, p.phi, p.counts);
    return hipGetLastError();
}

template <int PREC, bool PEPS, bool PHI, bool CNT>
hipError_t launch_g(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    switch (p.group) {
        case 64: return launch_t<PREC, PEPS, PHI, CNT, 64>(w, s, p);
        case 32: return launch_t<PREC, PEPS, PHI, CNT, 32>(w, s, p);
        default: return launch_t<PREC, PEPS, PHI, CNT, 16>(w, s, p);
    }
}

template <int PREC, bool PEPS>
hipError_t launch_p(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    const bool phi = p.phi != nullptr, cnt = p.counts != nullptr;
    if (phi && cnt) return launch_g<PREC, PEPS, true, true>(w, s, p);
    if (phi) return launch_g<PREC, PEPS, true, false>(w, s, p);
    if (cnt) return launch_g<PREC, PEPS, false, true>(w, s, p);
    return launch_g<PREC, PEPS, false, false>(w, s, p);
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
