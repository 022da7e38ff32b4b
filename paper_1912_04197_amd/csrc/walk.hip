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
// those nodes in parallel (one memory latency per round). Lane p bounds the
// distance from popped node p to the group's bounding box; where the opening
// test comes out the same for the whole box (by a margin far above rounding)
// that is every body's decision, and only the remaining "mixed" nodes are
// tested body by body (64 / GB nodes per instruction). Then the bookkeeping
// for all popped nodes runs at once: lane p handles popped node p, and prefix
// sums over the lanes place the pushed child ranges and the queued
// interactions. A round pops only as many ranges as can be expanded while
// keeping room for a depth-first descent, so the stack cannot overflow.
//
// Evaluation: the interaction queue holds descriptors (a leaf's body range or
// one accepted node, with a body mask). Whenever 64 items are queued, lane k
// expands item k (each descriptor starting inside the batch flags its first
// item; a ballot of the flags gives every item its descriptor) and loads it.
// An item that reaches more than GB / 6 bodies of the group is dense: the
// dense items are staged in LDS and the lanes of each body sweep them, each
// taking every (64 / GB)-th one. A sparse item becomes (item, body) pairs, one
// pair per lane, whose terms are added into per-body FP64 sums in LDS; most
// leaf bodies near the group's edge reach only a few of its bodies, and a
// sweep would leave most lanes idle on them. In FP32C mode each pair offset
// x_j - x_B is formed in FP64 and rounded once to FP32 (close pairs keep full
// FP32 precision whatever the group's extent), the rest of the pair term is
// FP32, and in the sweep FP32 partial sums over at most 16 items per lane are
// added into FP64 accumulators. The per-lane FP64 sums of a body and its pair
// sums are added at the end in a fixed order; the pair sums are LDS atomics of
// a single wave, applied in a fixed order, so results are deterministic.
#include <cstddef>
#include <type_traits>

#include "bhx_impl.h"
#include "walk_traverse.h"

namespace bhx {
namespace {

using walkx::kPop;
using walkx::PopCom;
using walkx::PopData;
constexpr int kStack = 256;    // LDS traversal stack of child ranges
constexpr int kRing = 128;     // interaction descriptors: <= 64 left over + 64 new
constexpr int kBatch = 64;     // items staged per evaluation batch
constexpr int kFlush = 16;     // FP32 partial sums span at most this many items per lane
constexpr int kPairCap = 448;  // body pairs evaluated one per lane in one batch
// Items per unrolled step of the dense sweep, by group size.
template <int GB>
constexpr int kSweepUnroll = GB == 64 ? 4 : 1;

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
    double e2h;  // half the source's squared softening (eps_j^2 or <eps^2>_N)
    uint64_t mask;
    int32_t src, pad0;
    int64_t pad1;
};
// Quadrupole term of an accepted node with traceless Q (xx, yy, zz, xy, xz,
// yz), d = COM - x_B, inv5 = 1/r^5 and ri2 = 1/r^2 of the softened distance:
// a += -Q d / r^5 + 5/2 (d.Q d) d / r^7 and phi += -(d.Q d) / (2 r^5), before
// the factor G.
template <typename T>
__device__ inline void quad_term(const T *Q, T dx, T dy, T dz, T inv5, T ri2, T &ax, T &ay, T &az,
                                 T &ph)
{
    const T qx = Q[0] * dx + Q[3] * dy + Q[4] * dz;
    const T qy = Q[3] * dx + Q[1] * dy + Q[5] * dz;
    const T qz = Q[4] * dx + Q[5] * dy + Q[2] * dz;
    const T dqd = dx * qx + dy * qy + dz * qz;
    const T c = T(2.5) * dqd * inv5 * ri2;
    ax += c * dx - qx * inv5;
    ay += c * dy - qy * inv5;
    az += c * dz - qz * inv5;
    ph -= T(0.5) * dqd * inv5;
}

template <int PREC, bool PEPS, bool PHI, bool CNT, int GB, bool QUAD>
__global__ __launch_bounds__(64) void k_walk(
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const NodeInfo *__restrict__ ninfo, const NodeMom *__restrict__ nmom,
    const double *__restrict__ neps2, const double *__restrict__ nquad,
    const uint32_t *__restrict__ idx,
    const SceneBox *__restrict__ box, const int32_t *__restrict__ groups, int64_t n,
    int ngroups, int per_xcd, double th2, double eps0sq, double G, double *__restrict__ acc,
    double *__restrict__ phi, int32_t *__restrict__ counts, bool acc_sorted)
{
    static_assert(GB == 64 || GB == 32 || GB == 16, "group size");
    constexpr int LPB = 64 / GB;  // lanes per body
    constexpr uint64_t kBodyMask = GB == 64 ? ~0ull : ((1ull << GB) - 1ull);
    using Item = typename std::conditional<PREC == BH_FP64, ItemD, ItemF>::type;
    using QT = typename std::conditional<PREC == BH_FP64, double, float>::type;

    // Items that reach at most kSparse bodies of the group are evaluated as
    // (item, body) pairs, one pair per lane, into per-body FP64 sums in LDS.
    constexpr int kSparse = GB / 6;

    __shared__ walkx::Lds<kStack, kRing> L;
    int32_t *const dq_a = L.dq_a;
    int32_t *const dq_n = L.dq_n;
    uint32_t *const dq_at = L.dq_at;
    uint64_t *const dq_mask = L.dq_mask;
    // The popped nodes are read only before a round's evaluations and the
    // staged items only during them, so the two share one LDS region.
    union Shared {
        struct {
            PopCom pc[kPop];
            PopData pd[kPop];
        } pop;
        struct {
            Item items[kBatch];      // dense items first, then the sparse ones
            uint16_t rec[kPairCap];  // pair: item slot << 6 | body
            QT quad[QUAD ? 6 * kBatch : 1];  // node items' quadrupoles, by slot
        } ev;
    };
    __shared__ Shared sh;
    __shared__ double pacc[3 * GB];  // pair sums per body: x, y, z
    __shared__ double pphi[PHI ? GB : 1];
    __shared__ int32_t pcnt[CNT ? 2 * GB : 1];
    PopCom *const pc = sh.pop.pc;
    PopData *const pd = sh.pop.pd;
    Item *const items = sh.ev.items;
    uint16_t *const rec = sh.ev.rec;
    QT *const qbuf = sh.ev.quad;

    // Blocks are dealt to the 8 XCDs round-robin. One scene: give each XCD a
    // contiguous (so spatially compact) range of groups to share its L2. A
    // group table (several scenes) is already in dealing order, costliest
    // first (per_xcd = 0): block b takes group b.
    const int grp = per_xcd ? (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3)
                            : (int)blockIdx.x;
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
    const double ebh = 0.5 * eb2;  // (eps_B^2 + e_j^2) / 2 = ebh + e_j^2 / 2 exactly
    const uint64_t active = __ballot(valid) & kBodyMask;
    // the group's bounding box (exact: min and max of its bodies' coordinates)
    double glo[3], ghi[3];  // the group's bounding box
    walkx::group_box<GB>(valid, me.x, me.y, me.z, glo, ghi);
    if (lane < kLevels) L.s2tab[lane] = box[scene].s2[lane];

    const float e2hB = (float)(0.5 * eb2);
    const float eps0f = (float)eps0sq;
    // every body of the wave has a positive FP32 softening (the sweep's r^2 > 0 test is moot)
    const bool soft_all =
        __ballot(!valid || positive_normal_f(PEPS ? e2hB : eps0f)) == ~0ull;
    const int woff = (int)offsetof(ItemF, mlo) + (bq >= 32 ? 4 : 0);

    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    int32_t cnode = 0, cpair = 0;

    int sp = 1;              // stack entries
    int dq_head = 0, dq_tail = 0;
    uint32_t queued = 0;     // items ever queued
    uint32_t consumed = 0;   // items ever evaluated
    if (lane == 0) {
        L.st_c0[0] = scene;  // the scene's root (node `scene`), as a range of one
        L.st_n[0] = 1;
        L.st_mask[0] = active;
    }
    for (int i = lane; i < 3 * GB; i += 64) pacc[i] = 0.0;
    if (PHI && lane < GB) pphi[lane] = 0.0;
    if (CNT)
        for (int i = lane; i < 2 * GB; i += 64) pcnt[i] = 0;
    __syncthreads();

    // Stages the next c queued items and evaluates them: the dense ones by
    // a sweep of the lanes of each body, the sparse ones as pairs.
    auto evaluate = [&](int c) {
        // Load item `lane` and its body mask; the split below decides where
        // in LDS it goes.
        uint64_t mk = 0;
        int32_t src = 0;
        double x = 0.0, y = 0.0, z = 0.0, m = 0.0, e2 = 0.0;
        double qn[QUAD ? 6 : 1] = {};
        // The descriptor of item consumed + lane: each descriptor that starts
        // inside the batch flags its first item (only the head descriptor can
        // start at item 0, and it may also start before the batch), so item
        // L belongs to the head plus as many descriptors as start in 1..L.
        // The flags use the pair list's space, free until the items are split.
        uint16_t *const flag = rec;
        flag[lane] = 0;
#pragma unroll
        for (int h = 0; h < kRing; h += 64) {
            if (h + lane < dq_tail - dq_head) {
                const uint32_t rel = dq_at[(dq_head + h + lane) & (kRing - 1)] - consumed;
                if (rel < (uint32_t)c) flag[rel] = 1;
            }
        }
        __syncthreads();
        const uint64_t starts = __ballot(flag[lane] != 0) & ~1ull;
        const int dsel = (int)lanes_below(starts) + (int)((starts >> lane) & 1ull);
        if (lane < c) {
            const uint32_t q = consumed + (uint32_t)lane;
            const int d = (dq_head + dsel) & (kRing - 1);
            const int32_t a = dq_a[d];
            mk = dq_mask[d];
            if (a >= 0) {
                src = a + (int32_t)(q - dq_at[d]);
                if (!check_ok(src < n, CK_INDEX)) src = 0;
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
                if constexpr (QUAD)
                    for (int t = 0; t < 6; t++) qn[t] = nquad[6 * (int64_t)(~a) + t];
            }
        }
        // Split the batch: an item reaching at most kSparse bodies becomes
        // that many (item, body) pairs while they fit in the pair list; the
        // others are dense and go to slots 0..nd-1, the sparse ones after.
        const int pk = __popcll(mk);
        const bool sparse = lane < c && pk <= kSparse;
        const uint32_t pv = sparse ? (uint32_t)pk : 0u;
        const uint32_t pend = wave_incl_scan(pv);
        const bool fits = sparse && pend <= (uint32_t)kPairCap;
        const bool dense = lane < c && !fits;
        const uint64_t db = __ballot(dense);
        const uint64_t fb = __ballot(fits && pk > 0);
        const int nd = __popcll(db);
        const int np = fb ? __builtin_amdgcn_readlane((int)pend, 63 - __builtin_clzll(fb)) : 0;
        BHX_CHECK(np <= kPairCap, CK_PAIRS);
        if (dense || (fits && pk > 0)) {
            const int slot = dense ? (int)lanes_below(db) : nd + (int)lanes_below(fb);
            if constexpr (PREC == BH_FP64) {
                items[slot] = ItemD{x, y, z, m, 0.5 * e2, mk, src, 0, 0};
            } else {
                items[slot] = ItemF{x,   y, z, (float)m, (float)(0.5 * e2), (uint32_t)mk,
                                    (uint32_t)(mk >> 32), src, 0};
            }
            if constexpr (QUAD)
                if (src < 0)
                    for (int t = 0; t < 6; t++) qbuf[6 * slot + t] = (QT)qn[t];
            if (fits) {
                uint64_t bits = mk;
                uint32_t at = pend - pv;
                while (bits) {
                    rec[at++] = (uint16_t)(slot << 6 | __builtin_ctzll(bits));
                    bits &= bits - 1;
                }
            }
        }
        __syncthreads();
        if constexpr (PREC == BH_FP64) {
#pragma unroll 1
            for (int jj = 0; jj < nd; jj += LPB) {
                const int j = jj + sub < nd ? jj + sub : jj;
                const ItemD it = items[j];
                const bool on = jj + sub < nd && ((it.mask >> bq) & 1ull);
                const double dx = it.x - me.x, dy = it.y - me.y, dz = it.z - me.z;
                const double e2 = PEPS ? ebh + it.e2h : eps0sq;
                const double r2 = dx * dx + dy * dy + dz * dz + e2;
                if (on && positive_normal(r2)) {
                    const double rinv = rsqrt_f64(r2), inv2 = rinv * rinv;
                    const double inv3 = inv2 * rinv;
                    ax += it.m * dx * inv3;
                    ay += it.m * dy * inv3;
                    az += it.m * dz * inv3;
                    if (PHI) ph -= it.m * rinv;
                    if constexpr (QUAD)
                        if (it.src < 0)
                            quad_term(qbuf + 6 * j, dx, dy, dz, inv3 * inv2, inv2, ax, ay, az, ph);
                }
                if (CNT && on) {
                    if (it.src < 0)
                        cnode++;
                    else
                        cpair++;
                }
            }
        } else {
          // With every body of the wave softened (its FP32 half eps^2 a normal
          // number), r^2 >= that softening for every pair, so r^2 is a
          // positive normal number and the test is dropped.
          auto sweep = [&](auto all_soft) {
#pragma unroll 1
            for (int j0 = 0; j0 < nd; j0 += kFlush * LPB) {
                const int jn = min(nd, j0 + kFlush * LPB);
                float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
                // jj is the same on every lane; lane share `sub` takes item jj + sub
#pragma unroll kSweepUnroll<GB>
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
                    const bool live =
                        decltype(all_soft)::value ? on : (on && positive_normal_f(r2));
                    const float rinv = live ? __builtin_amdgcn_rsqf(r2) : 0.f;
                    const float mr = it.m * rinv;
                    const float mr3 = mr * rinv * rinv;
                    fx = fmaf(mr3, dx, fx);
                    fy = fmaf(mr3, dy, fy);
                    fz = fmaf(mr3, dz, fz);
                    if (PHI) fp -= mr;
                    if constexpr (QUAD)
                        if (it.src < 0) {
                            const float ri2 = rinv * rinv;
                            quad_term(qbuf + 6 * (j < jn ? j : jj), dx, dy, dz, ri2 * ri2 * rinv, ri2,
                                      fx, fy, fz, fp);
                        }
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
          };
          if (soft_all)
              sweep(std::true_type{});
          else
              sweep(std::false_type{});
        }
        // Pairs: lane i takes pair i of the list; its body's coordinates come
        // from that body's lane. Each pair term goes into the body's FP64 sums.
#pragma unroll 1
        for (int i0 = 0; i0 < np; i0 += 64) {
            const int i = i0 + lane;
            const bool on = i < np;
            const uint32_t r = rec[on ? i : i0];
            const int k = (int)(r >> 6), b = (int)(r & 63u);
            const double tx = __shfl(me.x, b), ty = __shfl(me.y, b), tz = __shfl(me.z, b);
            double fx = 0.0, fy = 0.0, fz = 0.0, fp = 0.0;
            bool src_node;
            if constexpr (PREC == BH_FP64) {
                const double te = __shfl(ebh, b);
                const ItemD it = items[k];
                src_node = it.src < 0;
                const double dx = it.x - tx, dy = it.y - ty, dz = it.z - tz;
                const double e2 = PEPS ? te + it.e2h : eps0sq;
                const double r2 = dx * dx + dy * dy + dz * dz + e2;
                if (on && positive_normal(r2)) {
                    const double rinv = rsqrt_f64(r2), inv2 = rinv * rinv;
                    const double inv3 = inv2 * rinv;
                    fx = it.m * dx * inv3;
                    fy = it.m * dy * inv3;
                    fz = it.m * dz * inv3;
                    if (PHI) fp = -it.m * rinv;
                    if constexpr (QUAD)
                        if (src_node)
                            quad_term(qbuf + 6 * k, dx, dy, dz, inv3 * inv2, inv2, fx, fy, fz, fp);
                }
            } else {
                const float te = __shfl(e2hB, b);
                const ItemF it = items[k];
                src_node = it.src < 0;
                const float dx = (float)(it.x - tx), dy = (float)(it.y - ty), dz = (float)(it.z - tz);
                const float e2 = PEPS ? it.e2h + te : eps0f;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, e2)));
                const float rinv = (on && positive_normal_f(r2)) ? __builtin_amdgcn_rsqf(r2) : 0.f;
                const float mr = it.m * rinv;
                const float mr3 = mr * rinv * rinv;
                float gxf = mr3 * dx, gyf = mr3 * dy, gzf = mr3 * dz, gpf = -mr;
                if constexpr (QUAD)
                    if (src_node) {
                        const float ri2 = rinv * rinv;
                        quad_term(qbuf + 6 * k, dx, dy, dz, ri2 * ri2 * rinv, ri2, gxf, gyf, gzf, gpf);
                    }
                fx = (double)gxf;
                fy = (double)gyf;
                fz = (double)gzf;
                if (PHI) fp = (double)gpf;
            }
            if (on) {
                __hip_atomic_fetch_add(&pacc[3 * b], fx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(&pacc[3 * b + 1], fy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(&pacc[3 * b + 2], fz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (PHI)
                    __hip_atomic_fetch_add(&pphi[b], fp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (CNT)
                    __hip_atomic_fetch_add(&pcnt[2 * b + (src_node ? 0 : 1)], 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        consumed += (uint32_t)c;
        // retire the fully evaluated descriptors: they form a prefix of the
        // queue, and one batch completes at most 64 of them
        {
            const int da = dq_head + lane;
            bool done = false;
            if (da < dq_tail) {
                const int d = da & (kRing - 1);
                done = dq_at[d] + (uint32_t)dq_n[d] <= consumed;
            }
            dq_head += __popcll(__ballot(done));
        }
        __syncthreads();
    };

    while (sp > 0) {
        walkx::traverse_round<GB>(L, pc, pd, sp, dq_tail, queued, ninfo, nmom, glo, ghi, me.x, me.y,
                                  me.z, th2);
        BHX_CHECK(dq_tail - dq_head <= kRing, CK_RING);
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
    // then the pair sums, which were complete at the last barrier
    if (sub == 0) {
        ax += pacc[3 * bq];
        ay += pacc[3 * bq + 1];
        az += pacc[3 * bq + 2];
        if (PHI) ph += pphi[bq];
        if (CNT) {
            cnode += pcnt[2 * bq];
            cpair += pcnt[2 * bq + 1];
        }
    }
    if (valid && sub == 0) {
        const int64_t o = idx[s];
        const int64_t oa = acc_sorted ? s : o;  // where acc and phi go
        acc[3 * oa] = G * ax;
        acc[3 * oa + 1] = G * ay;
        acc[3 * oa + 2] = G * az;
        if (PHI) phi[oa] = G * ph;
        if (CNT) {
            counts[2 * o] = cnode;
            counts[2 * o + 1] = cpair;
        }
    }
}

template <int PREC, bool PEPS, bool PHI, bool CNT, int GB, bool QUAD>
hipError_t launch_t(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    const int ngroups = p.groups ? p.n_groups : (int)((p.n + GB - 1) / GB);
    const int per_xcd = p.groups ? 0 : (ngroups + 7) / 8;
    if (ngroups == 0) return hipSuccess;
    k_walk<PREC, PEPS, PHI, CNT, GB, QUAD><<<p.groups ? ngroups : 8 * per_xcd, 64, 0, s>>>(
        w.body, w.beps2, w.ninfo, w.nmom, w.neps2, p.nquad, w.idx[0], w.box, p.groups, p.n, ngroups,
        per_xcd, p.th2, p.eps0sq, p.G, p.acc, p.phi, p.counts, p.acc_sorted);
    return hipGetLastError();
}

template <int PREC, bool PEPS, bool PHI, bool CNT>
hipError_t launch_g(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    switch (p.group) {
        case 64:
            return p.nquad ? launch_t<PREC, PEPS, PHI, CNT, 64, true>(w, s, p)
                           : launch_t<PREC, PEPS, PHI, CNT, 64, false>(w, s, p);
        case 32:
            return p.nquad ? launch_t<PREC, PEPS, PHI, CNT, 32, true>(w, s, p)
                           : launch_t<PREC, PEPS, PHI, CNT, 32, false>(w, s, p);
        default:
            return p.nquad ? launch_t<PREC, PEPS, PHI, CNT, 16, true>(w, s, p)
                           : launch_t<PREC, PEPS, PHI, CNT, 16, false>(w, s, p);
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

BHX_DEFINE_TAKE_CHECKS(walk_take_checks)

hipError_t launch_walk(const Workspace &w, hipStream_t s, const WalkParams &p)
{
    if (p.n <= 0) return hipSuccess;
    if (p.precision == BH_FP64)
        return p.per_body_eps ? launch_p<BH_FP64, true>(w, s, p)
                              : launch_p<BH_FP64, false>(w, s, p);
    return p.per_body_eps ? launch_p<BH_FP32C, true>(w, s, p) : launch_p<BH_FP32C, false>(w, s, p);
}

}  // namespace bhx
