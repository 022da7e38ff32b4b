// The traversal shared by the forward walk (walk.hip) and the VJP walk
// (adjoint.hip): one wavefront walks the tree for a group of target bodies,
// every stack entry carrying the mask of the bodies whose own walk reaches it,
// and each body taking its own opening decisions (eq. accuracy), so both
// kernels see exactly the interaction lists of the per-body walk.
#pragma once

#include "bhx_impl.h"

namespace bhx {
namespace walkx {

// Relative margin of the group-box opening test. The per-body test's D^2
// and theta^2 D^2 carry a relative rounding error below 1e-15, so a box
// bound that clears the threshold by this margin decides every body alike.
constexpr double kMacMargin = 1e-12;
constexpr int kRanges = 8;      // ranges popped per round (<= 8 nodes each)
constexpr int kPop = 8 * kRanges;
constexpr int kReserve = 150;   // a depth-first descent adds <= 7 ranges per level

struct alignas(16) PopCom {  // popped node as the opening test needs it
    double x, y, z, s2;      // s2 = +inf for a leaf (never accepted)
};
struct alignas(16) PopData {  // popped node as the bookkeeping needs it
    uint64_t mask;
    int32_t node, first, count, child0;  // child0 < 0: leaf
    int32_t nch, pad;
};

// The opening test, rounded exactly as written: accept iff s^2 < theta^2 D^2.
__device__ inline bool accept_node(double cx, double cy, double cz, double bx, double by,
                                   double bz, double s2, double th2)
{
#pragma clang fp contract(off)
    double dx = cx - bx, dy = cy - by, dz = cz - bz;
    double D2 = dx * dx + dy * dy + dz * dz;
    return s2 < th2 * D2;
}

// The LDS a traversal works in: the stack of child ranges, the queue of
// interaction descriptors (a leaf's body range or one accepted node, with
// the mask of the bodies that take it) and the popped nodes of a round.
template <int kStack, int kRing>
struct Lds {
    static_assert((kRing & (kRing - 1)) == 0, "ring indices wrap by masking");
    int32_t st_c0[kStack];
    uint8_t st_n[kStack];
    uint64_t st_mask[kStack];
    int32_t dq_a[kRing];    // leaf: first body; node: ~node
    int32_t dq_n[kRing];    // items in the descriptor
    uint32_t dq_at[kRing];  // running item number of its first item
    uint64_t dq_mask[kRing];
    double s2tab[kLevels];  // squared cell side per level
};

// The group's bounding box: exact min and max of its bodies' coordinates
// (lanes of invalid bodies do not count).
template <int GB>
__device__ inline void group_box(bool valid, double x, double y, double z, double lo[3],
                                 double hi[3])
{
    lo[0] = valid ? x : __builtin_huge_val(), hi[0] = valid ? x : -__builtin_huge_val();
    lo[1] = valid ? y : __builtin_huge_val(), hi[1] = valid ? y : -__builtin_huge_val();
    lo[2] = valid ? z : __builtin_huge_val(), hi[2] = valid ? z : -__builtin_huge_val();
#pragma unroll
    for (int o = 1; o < GB; o <<= 1)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
        }
}

// One traversal round. Pops up to kRanges child ranges (at most 64 nodes,
// lane 8 r + o taking child o of range r) so that after expanding them at
// least kReserve stack entries stay free for a depth-first descent; loads
// the nodes and compacts them into slots 0..nv-1 of pc/pd. Opening tests:
// lane p first bounds popped node p's distance to the group's bounding box;
// when the test comes out the same for every point of the box, with a
// margin far above the rounding of the per-body test, that is every body's
// decision. The other ("mixed") internal nodes are tested by every body,
// 64 / GB nodes per step (one per share of lanes), and the group's GB-bit
// result for popped node p goes to lane p. Then the bookkeeping for popped
// node `lane`, all lanes at once: a node opened by the bodies in O pushes
// its child range with mask O; a leaf, or a node accepted by the bodies in
// A, queues a descriptor (mask: the bodies that reached the leaf, or A).
// Counters: sp (stack entries), dq_tail (descriptors queued), queued (items
// queued). Ends with the queue's new entries visible to the whole wave.
template <int GB, int kStack, int kRing>
__device__ inline void traverse_round(Lds<kStack, kRing> &L, PopCom *pc, PopData *pd, int &sp,
                                      int &dq_tail, uint32_t &queued,
                                      const NodeInfo *__restrict__ ninfo,
                                      const NodeMom *__restrict__ nmom, const double glo[3],
                                      const double ghi[3], double bx, double by, double bz,
                                      double th2)
{
    constexpr int LPB = 64 / GB;  // lanes per body
    constexpr uint64_t kBodyMask = GB == 64 ? ~0ull : ((1ull << GB) - 1ull);
    const int lane = threadIdx.x;
    const int sub = GB == 64 ? 0 : lane / GB;

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
            if (o < L.st_n[e]) {
                k = L.st_c0[e] + o;
                mk = L.st_mask[e];
            }
        }
    }
    const uint64_t vb = __ballot(k >= 0);
    const int nv = __popcll(vb);
    if (k >= 0) {
        const int slot = (int)lanes_below(vb);
        const NodeInfo info = ninfo[k];
        const NodeMom nm = nmom[k];
        const bool leaf = info.child0 < 0;
        pc[slot] = PopCom{nm.x, nm.y, nm.z, leaf ? __builtin_huge_val() : L.s2tab[node_level(info)]};
        pd[slot] = PopData{mk, k, info.first, info.count, info.child0, node_nchild(info), 0};
    }
    sp = base;
    __syncthreads();

    uint64_t accepted = 0;
    bool mixed = false;
    if (lane < nv) {
        const PopCom q = pc[lane];
        if (q.s2 < __builtin_huge_val()) {
            const double ex = fmax(0.0, fmax(glo[0] - q.x, q.x - ghi[0]));
            const double ey = fmax(0.0, fmax(glo[1] - q.y, q.y - ghi[1]));
            const double ez = fmax(0.0, fmax(glo[2] - q.z, q.z - ghi[2]));
            const double fx = fmax(fabs(q.x - glo[0]), fabs(q.x - ghi[0]));
            const double fy = fmax(fabs(q.y - glo[1]), fabs(q.y - ghi[1]));
            const double fz = fmax(fabs(q.z - glo[2]), fabs(q.z - ghi[2]));
            const double dmin2 = ex * ex + ey * ey + ez * ez;
            const double dmax2 = fx * fx + fy * fy + fz * fz;
            if (q.s2 < th2 * dmin2 * (1.0 - kMacMargin))
                accepted = kBodyMask;
            else if (!(q.s2 > th2 * dmax2 * (1.0 + kMacMargin)))
                mixed = true;
        }
    }
    uint64_t mb = __ballot(mixed);
#pragma unroll 1
    while (mb) {
        int ps[LPB];
#pragma unroll
        for (int t = 0; t < LPB; t++) {
            ps[t] = mb ? __builtin_ctzll(mb) : -1;
            mb &= mb - 1;
        }
        int p = ps[0];
#pragma unroll
        for (int t = 1; t < LPB; t++)
            if (sub == t) p = ps[t];
        const PopCom q = pc[p < 0 ? 0 : p];
        const bool ok = p >= 0 && accept_node(q.x, q.y, q.z, bx, by, bz, q.s2, th2);
        const uint64_t bal = __ballot(ok);
#pragma unroll
        for (int t = 0; t < LPB; t++) {
            const uint64_t field = (bal >> (t * GB)) & kBodyMask;
            if (lane == ps[t]) accepted = field;
        }
    }

    const bool mine = lane < nv;
    PopData my = PopData{0ull, 0, 0, 0, 0, 0, 0};
    if (mine) my = pd[lane];
    const bool leaf = mine && my.child0 < 0;
    const uint64_t M = my.mask;
    const uint64_t A = (mine && !leaf) ? (accepted & M) : 0ull;
    const uint64_t O = (mine && !leaf) ? (M & ~accepted) : 0ull;
    const uint64_t pushb = __ballot(O != 0);
    if (O != 0) {
        const int e = sp + (int)lanes_below(pushb);
        if (check_ok(e < kStack, CK_STACK)) {
            L.st_c0[e] = my.child0;
            L.st_n[e] = (uint8_t)my.nch;
            L.st_mask[e] = O;
        }
    }
    sp += __popcll(pushb);
    const bool hasq = leaf || A != 0;
    const uint64_t qb = __ballot(hasq);
    const uint32_t nitems = leaf ? (uint32_t)my.count : (A != 0 ? 1u : 0u);
    const uint32_t incl = wave_incl_scan(nitems);
    if (hasq) {
        const int d = (dq_tail + (int)lanes_below(qb)) & (kRing - 1);
        L.dq_a[d] = leaf ? my.first : ~my.node;
        L.dq_n[d] = (int32_t)nitems;
        L.dq_at[d] = queued + incl - nitems;
        L.dq_mask[d] = leaf ? M : A;
    }
    dq_tail += __popcll(qb);
    queued += (uint32_t)__shfl(incl, 63);
    __syncthreads();
}

}  // namespace walkx
}  // namespace bhx
