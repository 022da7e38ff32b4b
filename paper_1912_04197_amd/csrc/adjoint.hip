// Vector-Jacobian products of the force map (the gradient of
// sum_i lambda_i . a_i with respect to positions and masses), with the tree
// and every opening decision held fixed, and the elementwise parts of the
// kick-drift-kick adjoint.
//
// For one softened term t = G m_s d / r^3 (d = X_s - x_i, r^2 = |d|^2 + e2)
// and the target's upstream lambda:
//   dt/dd = G m_s K, K = I / r^3 - 3 d d^T / r^5   (x_i gets -K lambda, X_s +K lambda)
//   dt/dm_s = G d / r^3,   dt/de2 = -3/2 G m_s d / r^5.
// A node source passes its adjoints to its members through its centre of mass
// X_N = sum m_j x_j / m_N, its mass m_N = sum m_j and its mass-weighted
// softening <eps^2>_N = sum m_j eps_j^2 / m_N.
//
// Tree VJP, on the GPU:
//   1. the same build as the forward evaluation (deterministic, so the same
//      tree and decisions);
//   2. a walk with the forward walk's traversal and decisions (one wave per
//      64 Morton-consecutive targets, per-lane masks, batched rounds, staged
//      items split into dense items and pairs); each target's terms are
//      summed in registers and LDS, each source's terms are summed over the
//      group and added with FP64 atomics into the body or node adjoints;
//   3. node adjoints become per-node coefficients (A = gX / m_N,
//      E = ge2 / m_N, C = gm - X.A - <eps^2> E), summed from the root down
//      over each leaf's ancestors (found through a parent table);
//   4. per body: g_x += m_j sum A, g_m += sum C + x_j . sum A + eps_j^2 sum E,
//      plus its own target and source terms, added into the caller's arrays.
// Source-side atomics make the last bits of the gradients order-dependent.
#include <type_traits>

#include "bhx_impl.h"
#include "walk_traverse.h"

namespace bhx {
namespace {

using walkx::kPop;
using walkx::PopCom;
using walkx::PopData;
constexpr int kStack = 320;
constexpr int kRing = 128;
constexpr int kBatch = 64;

struct alignas(16) ItemV {  // staged source
    double x, y, z, m;
    double e2;      // source's squared softening (eps_j^2 or <eps^2>_N)
    uint64_t mask;
    int32_t src;    // sorted body index, or ~node
    float gm;       // G m rounded to FP32 (FP32C terms)
    float e2h;      // half the squared softening rounded to FP32 (FP32C terms)
    int32_t pad;
};
// Lane exchanges inside a row of 16 lanes (DPP): quad_perm [1,0,3,2] is
// lane ^ 1, quad_perm [2,3,0,1] is lane ^ 2, row_ror:4 and row_ror:8 rotate
// the row by 4 and 8 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRor4 = 0x124, kDppRor8 = 0x128;
template <int CTRL>
__device__ inline double dpp(double v)
{
    const uint64_t u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
template <int CTRL>
__device__ inline float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

constexpr int kPairCap = 448;  // pairs per batch

// badj: per sorted body {gX x, y, z, gm}; nadj: per node {gX x, y, z, gm, ge2}.
//
// The traversal and the opening decisions are those of the forward walk. A
// staged batch is split like the forward walk's: a dense item (reaching
// more than kSparse of the group's bodies) is swept by the lanes of its
// bodies, eight items at a time; each lane takes the eight in an order set by
// its lane bits so that three halving exchanges (lane ^ 1, ^ 2, ^ 32) leave
// lane L with one item's source-side terms summed over eight lanes, and three
// more (rotations by 4 and 8 inside a row, lane ^ 16) complete the sum over
// the group; then eight lanes add the eight sums to the item's adjoints with
// FP64 atomics. A sparse item becomes (item, body) pairs, one per lane, whose
// target-side terms go to per-body and whose source-side terms go to per-item
// FP64 sums in LDS, flushed to the adjoints once per batch.
template <bool PEPS, int GB, bool F32>
__global__ __launch_bounds__(64) void k_vjp_walk(
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const NodeInfo *__restrict__ ninfo, const NodeMom *__restrict__ nmom,
    const double *__restrict__ neps2, const uint32_t *__restrict__ idx,
    const SceneBox *__restrict__ box, int64_t n, int ngroups, int per_xcd, double th2,
    double eps0sq, double G, const double *__restrict__ lambda, double *__restrict__ gt,
    double *__restrict__ badj, double *__restrict__ nadj)
{
    static_assert(GB == 64 || GB == 32 || GB == 16, "group size");
    constexpr int NC = PEPS ? 5 : 4;  // source-side components: gX (3), gm, g<eps^2>
    constexpr int LPB = 64 / GB;      // lanes per body
    constexpr uint64_t kBodyMask = GB == 64 ? ~0ull : ((1ull << GB) - 1ull);
    constexpr int kSparse = GB / 4;   // items reaching at most this many bodies go to pair mode
    // FP32C: every term in FP32 from the FP64 offset rounded once, the terms
    // of a step summed in FP32 and added into FP64 sums and adjoints
    using VT = typename std::conditional<F32, float, double>::type;
    __shared__ walkx::Lds<kStack, kRing> L;
    int32_t *const dq_a = L.dq_a;
    int32_t *const dq_n = L.dq_n;
    uint32_t *const dq_at = L.dq_at;
    uint64_t *const dq_mask = L.dq_mask;
    union Shared {
        struct {
            PopCom pc[kPop];
            PopData pd[kPop];
        } pop;
        struct {
            ItemV items[kBatch];     // dense items first, then the sparse ones
            uint16_t rec[kPairCap];  // pair: item slot << 6 | body
        } ev;
    };
    __shared__ Shared sh;
    __shared__ double tacc[3 * GB];      // pair target-side sums per body
    __shared__ double sacc[5 * kBatch];  // pair source-side sums per staged item
    PopCom *const pc = sh.pop.pc;
    PopData *const pd = sh.pop.pd;
    ItemV *const items = sh.ev.items;
    uint16_t *const rec = sh.ev.rec;

    const int grp = (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3);
    if (grp >= ngroups) return;
    const int lane = threadIdx.x;
    const int bq = GB == 64 ? lane : lane % GB;  // body of this lane within the group
    const int sub = GB == 64 ? 0 : lane / GB;    // which share of the items it takes
    const int64_t g0 = (int64_t)grp * GB;
    const int64_t s = g0 + bq;
    const bool valid = s < n;
    const Body me = body[valid ? s : g0];
    const double eb2 = PEPS ? beps2[valid ? s : g0] : 0.0;
    const float ebhf = (float)(0.5 * eb2);  // FP32C: half the target's squared softening
    double lx = 0.0, ly = 0.0, lz = 0.0;
    if (valid) {
        const int64_t o = idx[s];
        lx = lambda[3 * o];
        ly = lambda[3 * o + 1];
        lz = lambda[3 * o + 2];
    }
    const uint64_t active = __ballot(valid) & kBodyMask;
    if (lane < kLevels) L.s2tab[lane] = box[0].s2[lane];
    double glo[3], ghi[3];  // the group's bounding box
    walkx::group_box<GB>(valid, me.x, me.y, me.z, glo, ghi);
    // This lane's order of its share's eight items of a dense step: slot bits
    // 2 and 1 follow lane bits 0 and 1, slot bit 0 lane bit 5 (GB = 64) or 3.
    const int perm = ((lane & 1) << 2) | (lane & 2) | (GB == 64 ? lane >> 5 : (lane >> 3) & 1);

    double gx = 0.0, gy = 0.0, gz = 0.0;  // target-side gradient of this lane's body
    const VT lxv = (VT)lx, lyv = (VT)ly, lzv = (VT)lz;
    int sp = 1, dq_head = 0, dq_tail = 0;
    uint32_t queued = 0, consumed = 0;
    if (lane == 0) {
        L.st_c0[0] = 0;
        L.st_n[0] = 1;
        L.st_mask[0] = active;
    }
    for (int i = lane; i < 3 * GB; i += 64) tacc[i] = 0.0;
    __syncthreads();

    // One softened term of source (x, y, z, m, e2) on a target at (bx, by, bz)
    // with softening eb and upstream (ux, uy, uz): the target-side gradient is
    // minus the first three source-side components. In FP32C the offset is the
    // FP64 difference rounded once and the rest of the term is FP32; the term
    // counts when its r^2 is a positive normal number of the precision used.
    // In FP32C the pair softening is the sum of the two halves rounded to
    // FP32 (ebh: the target's), as in the forward FP32C walk.
    auto term = [&](const ItemV &it, double bx, double by, double bz, double eb, float ebh, VT ux,
                    VT uy, VT uz, bool on, VT out[5]) {
        out[0] = out[1] = out[2] = out[3] = out[4] = VT(0);
        if constexpr (F32) {
            const float dx = (float)(it.x - bx), dy = (float)(it.y - by), dz = (float)(it.z - bz);
            const float e2 = PEPS ? it.e2h + ebh : (float)eps0sq;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, e2)));
            if (on && positive_normal_f(r2)) {
                const float rinv = __builtin_amdgcn_rsqf(r2), inv2 = rinv * rinv;
                const float inv3 = inv2 * rinv;
                const float inv5 = inv3 * inv2;
                const float ld = ux * dx + uy * dy + uz * dz;
                const float gms = it.gm;
                const float c = 3.0f * ld * inv5;
                out[0] = gms * (ux * inv3 - dx * c);
                out[1] = gms * (uy * inv3 - dy * c);
                out[2] = gms * (uz * inv3 - dz * c);
                out[3] = (float)G * ld * inv3;
                out[4] = -1.5f * gms * ld * inv5;
            }
        } else {
            const double dx = it.x - bx, dy = it.y - by, dz = it.z - bz;
            const double e2 = PEPS ? 0.5 * (eb + it.e2) : eps0sq;
            const double r2 = dx * dx + dy * dy + dz * dz + e2;
            if (on && positive_normal(r2)) {
                const double rinv = rsqrt_f64(r2), inv2 = rinv * rinv;
                const double inv3 = inv2 * rinv;
                const double inv5 = inv3 * inv2;
                const double ld = ux * dx + uy * dy + uz * dz;
                const double gms = G * it.m;
                out[0] = gms * (ux * inv3 - 3.0 * dx * ld * inv5);
                out[1] = gms * (uy * inv3 - 3.0 * dy * ld * inv5);
                out[2] = gms * (uz * inv3 - 3.0 * dz * ld * inv5);
                out[3] = G * ld * inv3;
                out[4] = -1.5 * gms * ld * inv5;
            }
        }
    };
    // adds a source-side sum to the item's adjoints (e2 = (eps_B^2 + <eps^2>_N) / 2)
    auto flush = [&](int32_t src, const double v[5]) {
        if (src >= 0) {
            double *b = badj + 4 * (int64_t)src;
            unsafeAtomicAdd(b, v[0]);
            unsafeAtomicAdd(b + 1, v[1]);
            unsafeAtomicAdd(b + 2, v[2]);
            unsafeAtomicAdd(b + 3, v[3]);
        } else {
            double *b = nadj + 5 * (int64_t)(~src);
            unsafeAtomicAdd(b, v[0]);
            unsafeAtomicAdd(b + 1, v[1]);
            unsafeAtomicAdd(b + 2, v[2]);
            unsafeAtomicAdd(b + 3, v[3]);
            if (PEPS) unsafeAtomicAdd(b + 4, 0.5 * v[4]);
        }
    };

    auto evaluate = [&](int c) {
        uint64_t mk = 0;
        ItemV ld_it{0.0, 0.0, 0.0, 0.0, 0.0, 0ull, 0, 0.f, 0.f, 0};
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
                int32_t src = a + (int32_t)(q - dq_at[d]);
                if (!check_ok(src < n, CK_INDEX)) src = 0;
                const int64_t rel = (int64_t)src - g0;
                if (rel >= 0 && rel < GB) mk &= ~(1ull << rel);
                const Body b = body[src];
                const double e2 = PEPS ? beps2[src] : 0.0;
                ld_it = ItemV{b.x,  b.y, b.z, b.m, e2, mk, src, (float)(G * b.m),
                              (float)(0.5 * e2), 0};
            } else {
                const NodeMom nm = nmom[~a];
                const double e2 = PEPS ? neps2[~a] : 0.0;
                ld_it = ItemV{nm.x, nm.y, nm.z, nm.m, e2, mk, a, (float)(G * nm.m),
                              (float)(0.5 * e2), 0};
            }
        }
        const int pk = __popcll(mk);
        const bool sparse = lane < c && pk <= kSparse;
        const uint32_t pv = sparse ? (uint32_t)pk : 0u;
        const uint32_t pend = wave_incl_scan(pv);
        const bool fits = sparse && pend <= (uint32_t)kPairCap;
        const bool dense = lane < c && !fits;
        const uint64_t db = __ballot(dense);
        const uint64_t fb = __ballot(fits && pk > 0);
        const int nd = __popcll(db);
        const int ns = __popcll(fb);
        const int np = fb ? __builtin_amdgcn_readlane((int)pend, 63 - __builtin_clzll(fb)) : 0;
        BHX_CHECK(np <= kPairCap, CK_PAIRS);
        if (dense || (fits && pk > 0)) {
            const int slot = dense ? (int)lanes_below(db) : nd + (int)lanes_below(fb);
            items[slot] = ld_it;
            if (fits) {
#pragma unroll
                for (int q = 0; q < 5; q++) sacc[5 * slot + q] = 0.0;
                uint64_t bits = mk;
                uint32_t at = pend - pv;
                while (bits) {
                    rec[at++] = (uint16_t)(slot << 6 | __builtin_ctzll(bits));
                    bits &= bits - 1;
                }
            }
        }
        __syncthreads();

        // dense items, eight per share of lanes per step
#pragma unroll 1
        for (int j0 = 0; j0 < nd; j0 += 8 * LPB) {
            VT v[8][NC];
            VT sx = VT(0), sy = VT(0), sz = VT(0);  // FP32C: this step's target-side terms
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const int j = j0 + 8 * sub + (t ^ perm);
                const ItemV it = items[j < nd ? j : j0];
                const bool on = j < nd && ((it.mask >> bq) & 1ull);
                VT o[5];
                term(it, me.x, me.y, me.z, eb2, ebhf, lxv, lyv, lzv, on, o);
                if constexpr (F32) {
                    sx -= o[0];
                    sy -= o[1];
                    sz -= o[2];
                } else {
                    gx -= o[0];
                    gy -= o[1];
                    gz -= o[2];
                }
#pragma unroll
                for (int q = 0; q < NC; q++) v[t][q] = o[q];
            }
            if constexpr (F32) {
                gx += (double)sx;
                gy += (double)sy;
                gz += (double)sz;
            }
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int q = 0; q < NC; q++) v[t][q] += dpp<kDppXor1>(v[t + 4][q]);
#pragma unroll
            for (int t = 0; t < 2; t++)
#pragma unroll
                for (int q = 0; q < NC; q++) v[t][q] += dpp<kDppXor2>(v[t + 2][q]);
#pragma unroll
            for (int q = 0; q < NC; q++) {
                VT w;
                if constexpr (GB == 64) {
                    w = v[0][q] + __shfl_xor(v[1][q], 32);
                    w += dpp<kDppRor4>(w);
                    w += dpp<kDppRor8>(w);
                    w += __shfl_xor(w, 16);
                } else {
                    w = v[0][q] + dpp<kDppRor8>(v[1][q]);  // lane ^ 8 inside the row
                    w += __shfl_xor(w, 4);
                    if (GB == 32) w += __shfl_xor(w, 16);
                }
                v[0][q] = w;
            }
            // each share's sums of items j0 + 8 sub + perm sit in its lanes with
            // lane bits 2 and 3, 4 (GB = 64) or 2 (and 4 for GB = 32) clear
            const int j = j0 + 8 * sub + perm;
            const bool lead = GB == 64 ? (lane & 28) == 0 : GB == 32 ? (lane & 20) == 0 : (lane & 4) == 0;
            if (lead && j < nd) {
                double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < NC; q++) o[q] = (double)v[0][q];
                flush(items[j].src, o);
            }
        }

        // sparse items as pairs
#pragma unroll 1
        for (int i0 = 0; i0 < np; i0 += 64) {
            const int i = i0 + lane;
            const bool on = i < np;
            const uint32_t r = rec[on ? i : i0];
            const int k = (int)(r >> 6), b = (int)(r & 63u);
            const double bx = __shfl(me.x, b), by = __shfl(me.y, b), bz = __shfl(me.z, b);
            const double eb = PEPS && !F32 ? __shfl(eb2, b) : 0.0;
            const float ebh = PEPS && F32 ? __shfl(ebhf, b) : 0.f;
            const VT ux = __shfl(lxv, b), uy = __shfl(lyv, b), uz = __shfl(lzv, b);
            const ItemV it = items[k];
            VT o[5];
            term(it, bx, by, bz, eb, ebh, ux, uy, uz, on, o);
            if (on) {
#pragma unroll
                for (int q = 0; q < 3; q++)
                    __hip_atomic_fetch_add(&tacc[3 * b + q], -(double)o[q], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
                for (int q = 0; q < NC; q++)
                    __hip_atomic_fetch_add(&sacc[5 * k + q], (double)o[q], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        if (lane < ns) {
            const int k = nd + lane;
            double o[5];
#pragma unroll
            for (int q = 0; q < 5; q++) o[q] = sacc[5 * k + q];
            flush(items[k].src, o);
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

    // the lanes' shares of each body, in a fixed order, then its pair sums
#pragma unroll
    for (int o = GB; o < 64; o <<= 1) {
        gx += __shfl_xor(gx, o);
        gy += __shfl_xor(gy, o);
        gz += __shfl_xor(gz, o);
    }
    if (valid && sub == 0) {
        gt[3 * s] = gx + tacc[3 * bq];
        gt[3 * s + 1] = gy + tacc[3 * bq + 1];
        gt[3 * s + 2] = gz + tacc[3 * bq + 2];
    }
}

// Zeroes body adjoints (4 per body) and node adjoints (5 per node that
// exists), and writes each node's parent (-1 for the root).
__global__ __launch_bounds__(256) void k_vjp_clear(double *__restrict__ badj, int64_t n,
                                                   double *__restrict__ nadj,
                                                   int32_t *__restrict__ nparent,
                                                   const NodeInfo *__restrict__ ninfo,
                                                   const TreeHeader *__restrict__ hdr,
                                                   int64_t node_cap)
{
    int64_t nn = 0;
    for (int l = 0; l < kLevels; l++) nn += hdr->level_count[l];
    if (nn > node_cap) nn = node_cap;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int64_t i = t; i < 4 * n; i += stride) badj[i] = 0.0;
    for (int64_t i = t; i < 5 * nn; i += stride) nadj[i] = 0.0;
    if (t == 0 && nn > 0) nparent[0] = -1;
    for (int64_t k = t; k < nn; k += stride) {
        const NodeInfo info = ninfo[k];
        if (info.child0 < 0) continue;
        const int nch = node_nchild(info);
        for (int o = 0; o < nch; o++)
            if (check_ok((int64_t)info.child0 + o < nn, CK_INDEX)) nparent[info.child0 + o] = (int32_t)k;
    }
}

// Per-node coefficients of the member update, from the node's adjoints.
__device__ inline void node_coeffs(const double *__restrict__ nadj, const NodeMom &nm, double e2,
                                   int64_t k, double out[5])
{
    const double *a = nadj + 5 * k;
    if (nm.m > 0.0) {
        const double inv = 1.0 / nm.m;
        out[0] = a[0] * inv;
        out[1] = a[1] * inv;
        out[2] = a[2] * inv;
        out[4] = a[4] * inv;
        out[3] = a[3] - (nm.x * out[0] + nm.y * out[1] + nm.z * out[2]) - e2 * out[4];
    } else {
        out[0] = out[1] = out[2] = out[4] = 0.0;
        out[3] = a[3];
    }
}

// Every leaf hands the ancestor sums of the node coefficients to its
// members and adds the members' own terms into the caller's gradient arrays
// (caller order, +=). A leaf collects its chain of ancestors through the
// parent table (at most kLevels nodes) and sums their coefficients from the
// root down.
__global__ __launch_bounds__(256) void k_vjp_finish(
    const TreeHeader *__restrict__ hdr, const NodeInfo *__restrict__ ninfo,
    const NodeMom *__restrict__ nmom, const double *__restrict__ neps2,
    const int32_t *__restrict__ nparent, const double *__restrict__ nadj,
    const Body *__restrict__ body, const double *__restrict__ beps2, int use_eps,
    const uint32_t *__restrict__ idx, const double *__restrict__ gt,
    const double *__restrict__ badj, double *__restrict__ g_pos, double *__restrict__ g_mass,
    int64_t node_cap)
{
    int64_t nn = 0;
    for (int l = 0; l < kLevels; l++) nn += hdr->level_count[l];
    if (nn > node_cap) nn = node_cap;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nn;
         k += (int64_t)gridDim.x * 256) {
        const NodeInfo info = ninfo[k];
        if (info.child0 >= 0) continue;
        int32_t chain[kLevels];  // chain[d]: the leaf's ancestor d levels up, or -1
        int32_t cur = (int32_t)k;
#pragma unroll
        for (int d = 0; d < kLevels; d++) {
            chain[d] = cur;
            cur = cur >= 0 ? nparent[cur] : -1;
        }
        double p[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int d = kLevels - 1; d >= 0; d--) {
            const int32_t c = chain[d];
            if (c < 0) continue;
            double cf[5];
            node_coeffs(nadj, nmom[c], use_eps ? neps2[c] : 0.0, c, cf);
            for (int q = 0; q < 5; q++) p[q] = p[q] + cf[q];
        }
        for (int32_t s = info.first; s < info.first + info.count; s++) {
            const Body b = body[s];
            const double e2 = use_eps ? beps2[s] : 0.0;
            const int64_t o = idx[s];
            const double *ba = badj + 4 * (int64_t)s;
            g_pos[3 * o] += gt[3 * s] + ba[0] + b.m * p[0];
            g_pos[3 * o + 1] += gt[3 * s + 1] + ba[1] + b.m * p[1];
            g_pos[3 * o + 2] += gt[3 * s + 2] + ba[2] + b.m * p[2];
            g_mass[o] += ba[3] + p[3] + b.x * p[0] + b.y * p[1] + b.z * p[2] + e2 * p[4];
        }
    }
}

// Direct-sum VJP, gathered per body p (no atomics):
//   g_x_p += G sum_{q != p} K(d_pq) (m_p lambda_q - m_q lambda_p)
//   g_m_p += G sum_{q != p} lambda_q . (x_p - x_q) / r^3
template <bool PEPS>
__global__ __launch_bounds__(256) void k_direct_vjp(const double *__restrict__ pos,
                                                    const double *__restrict__ mass,
                                                    const double *__restrict__ eps, int64_t n,
                                                    double eps0sq, double G,
                                                    const double *__restrict__ lambda,
                                                    double *__restrict__ g_pos,
                                                    double *__restrict__ g_mass, int64_t chunk,
                                                    double *__restrict__ part)
{
    constexpr int T = 256;
    __shared__ double sx[T], sy[T], sz[T], sm[T], se[T], slx[T], sly[T], slz[T];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * T + tid;
    const bool valid = p < n;
    const double xp = valid ? pos[3 * p] : 0.0, yp = valid ? pos[3 * p + 1] : 0.0,
                 zp = valid ? pos[3 * p + 2] : 0.0, mp = valid ? mass[p] : 0.0;
    const double lpx = valid ? lambda[3 * p] : 0.0, lpy = valid ? lambda[3 * p + 1] : 0.0,
                 lpz = valid ? lambda[3 * p + 2] : 0.0;
    double ep2 = 0.0;
    if (PEPS && valid) ep2 = eps[p] * eps[p];
    double gx = 0.0, gy = 0.0, gz = 0.0, gm = 0.0;
    // this block row's sources: [s_lo, s_hi) (one row unless the targets
    // alone give too few blocks; the rows' partial sums are then added in
    // row order by k_direct_vjp_reduce)
    const int64_t s_lo = (int64_t)blockIdx.y * chunk;
    const int64_t s_hi = s_lo + chunk < n ? s_lo + chunk : n;
    for (int64_t base = s_lo; base < s_hi; base += T) {
        const int64_t q = base + tid;
        if (q < s_hi) {
            sx[tid] = pos[3 * q];
            sy[tid] = pos[3 * q + 1];
            sz[tid] = pos[3 * q + 2];
            sm[tid] = mass[q];
            slx[tid] = lambda[3 * q];
            sly[tid] = lambda[3 * q + 1];
            slz[tid] = lambda[3 * q + 2];
            if (PEPS) se[tid] = eps[q] * eps[q];
        }
        __syncthreads();
        const int cnt = (int)((s_hi - base) < T ? (s_hi - base) : T);
        for (int j = 0; j < cnt; j++) {
            if (base + j == p) continue;
            const double dx = sx[j] - xp, dy = sy[j] - yp, dz = sz[j] - zp;
            const double e2 = PEPS ? 0.5 * (ep2 + se[j]) : eps0sq;
            const double r2 = dx * dx + dy * dy + dz * dz + e2;
            if (!positive_normal(r2)) continue;
            const double rinv = rsqrt_f64(r2), inv2 = rinv * rinv;
            const double inv3 = inv2 * rinv;
            const double inv5 = inv3 * inv2;
            // w = m_p lambda_q - m_q lambda_p ; K w = w / r^3 - 3 d (d.w) / r^5
            const double wx = mp * slx[j] - sm[j] * lpx, wy = mp * sly[j] - sm[j] * lpy,
                         wz = mp * slz[j] - sm[j] * lpz;
            const double dw = dx * wx + dy * wy + dz * wz;
            gx += wx * inv3 - 3.0 * dx * dw * inv5;
            gy += wy * inv3 - 3.0 * dy * dw * inv5;
            gz += wz * inv3 - 3.0 * dz * dw * inv5;
            gm -= (slx[j] * dx + sly[j] * dy + slz[j] * dz) * inv3;
        }
        __syncthreads();
    }
    if (valid && gridDim.y == 1) {
        g_pos[3 * p] += G * gx;
        g_pos[3 * p + 1] += G * gy;
        g_pos[3 * p + 2] += G * gz;
        g_mass[p] += G * gm;
    } else if (valid) {
        double *o = part + 4 * ((int64_t)blockIdx.y * n + p);
        o[0] = gx;
        o[1] = gy;
        o[2] = gz;
        o[3] = gm;
    }
}

// Adds G times the rows' partial sums, in row order, into the gradients.
__global__ __launch_bounds__(256) void k_direct_vjp_reduce(const double *__restrict__ part,
                                                           int64_t n, int rows, double G,
                                                           double *__restrict__ g_pos,
                                                           double *__restrict__ g_mass)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    double gx = 0.0, gy = 0.0, gz = 0.0, gm = 0.0;
    for (int r = 0; r < rows; r++) {
        const double *o = part + 4 * ((int64_t)r * n + p);
        gx += o[0];
        gy += o[1];
        gz += o[2];
        gm += o[3];
    }
    g_pos[3 * p] += G * gx;
    g_pos[3 * p + 1] += G * gy;
    g_pos[3 * p + 2] += G * gz;
    g_mass[p] += G * gm;
}

// Adjoint of the second kick: abar += dt/2 vbar.
__global__ __launch_bounds__(256) void k_adj_kick(double *__restrict__ abar,
                                                  const double *__restrict__ vbar, int64_t n3,
                                                  double h)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n3) abar[i] += h * vbar[i];
}

// Adjoint of the drift and the first kick: vbar += dt xbar; abar = dt/2 vbar.
__global__ __launch_bounds__(256) void k_adj_drift_kick(double *__restrict__ vbar,
                                                        double *__restrict__ abar,
                                                        const double *__restrict__ xbar,
                                                        int64_t n3, double dt, double h)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const double v = vbar[i] + dt * xbar[i];
    vbar[i] = v;
    abar[i] = h * v;
}

// x_out = x_in + dt (v + dt/2 a); v += dt/2 a (kick and drift into a new buffer)
__global__ __launch_bounds__(256) void k_kick_drift_to(const double *__restrict__ x_in,
                                                       double *__restrict__ v,
                                                       const double *__restrict__ a,
                                                       double *__restrict__ x_out, int64_t n3,
                                                       double h, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const double u = v[i] + h * a[i];
    v[i] = u;
    x_out[i] = x_in[i] + dt * u;
}

__global__ __launch_bounds__(256) void k_copy(double *__restrict__ dst,
                                              const double *__restrict__ src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

inline unsigned blocks(int64_t items, unsigned cap = 1u << 30)
{
    int64_t b = (items + 255) / 256;
    if (b < 1) b = 1;
    return (unsigned)(b < (int64_t)cap ? b : cap);
}

}  // namespace

BHX_DEFINE_TAKE_CHECKS(adjoint_take_checks)

hipError_t launch_tree_vjp(const Workspace &w, const AdjointWork &aw, hipStream_t s,
                           const WalkParams &p, const double *lambda, double *g_pos,
                           double *g_mass)
{
    if (p.n <= 0) return hipSuccess;
    k_vjp_clear<<<1024, 256, 0, s>>>(aw.badj, p.n, aw.nadj, aw.nparent, w.ninfo, w.hdr,
                                     w.node_cap);
    const int gb = p.group == 16 || p.group == 32 ? p.group : 64;
    const int ngroups = (int)((p.n + gb - 1) / gb);
    const int per_xcd = (ngroups + 7) / 8;
    auto walk = [&](auto peps, auto gbc) {
        if (p.precision == BH_FP32C)
            k_vjp_walk<decltype(peps)::value, decltype(gbc)::value, true>
                <<<8 * per_xcd, 64, 0, s>>>(w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.idx[0],
                                            w.box, p.n, ngroups, per_xcd, p.th2, p.eps0sq, p.G,
                                            lambda, aw.gt, aw.badj, aw.nadj);
        else
            k_vjp_walk<decltype(peps)::value, decltype(gbc)::value, false>
                <<<8 * per_xcd, 64, 0, s>>>(w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.idx[0],
                                            w.box, p.n, ngroups, per_xcd, p.th2, p.eps0sq, p.G,
                                            lambda, aw.gt, aw.badj, aw.nadj);
    };
    using T = std::true_type;
    using F = std::false_type;
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    if (p.per_body_eps) {
        if (gb == 16) walk(T{}, I16{});
        else if (gb == 32) walk(T{}, I32{});
        else walk(T{}, I64{});
    } else {
        if (gb == 16) walk(F{}, I16{});
        else if (gb == 32) walk(F{}, I32{});
        else walk(F{}, I64{});
    }
    const int use_eps = p.per_body_eps ? 1 : 0;
    k_vjp_finish<<<blocks(p.n, 4096), 256, 0, s>>>(w.hdr, w.ninfo, w.nmom, w.neps2, aw.nparent,
                                                   aw.nadj, w.body, w.beps2, use_eps, w.idx[0],
                                                   aw.gt, aw.badj, g_pos, g_mass, w.node_cap);
    return hipGetLastError();
}

hipError_t launch_direct_vjp(hipStream_t s, const double *pos, const double *mass,
                             const double *eps, int64_t n, double eps0sq, double G,
                             const double *lambda, double *g_pos, double *g_mass, double *part)
{
    if (n <= 0) return hipSuccess;
    // rows of source tiles as in the direct sum: targets x rows reaches
    // kDirectBlocks, and rows * n <= kDirectBlocks * 256 fits the buffer
    const int64_t tb = (n + 255) / 256;
    int64_t rows = tb >= kDirectBlocks ? 1 : kDirectBlocks / tb;
    if (rows > kDirectSplits) rows = kDirectSplits;
    if (rows > tb) rows = tb;
    const int64_t tiles = (tb + rows - 1) / rows;
    rows = (tb + tiles - 1) / tiles;
    if (!part) rows = 1;
    const int64_t chunk = rows == 1 ? n : tiles * 256;
    const dim3 grid((unsigned)tb, (unsigned)rows);
    if (eps)
        k_direct_vjp<true><<<grid, 256, 0, s>>>(pos, mass, eps, n, eps0sq, G, lambda, g_pos,
                                                g_mass, chunk, part);
    else
        k_direct_vjp<false><<<grid, 256, 0, s>>>(pos, mass, eps, n, eps0sq, G, lambda, g_pos,
                                                 g_mass, chunk, part);
    if (rows > 1)
        k_direct_vjp_reduce<<<(unsigned)tb, 256, 0, s>>>(part, n, (int)rows, G, g_pos, g_mass);
    return hipGetLastError();
}

hipError_t launch_adj_kick(hipStream_t s, double *abar, const double *vbar, int64_t n, double dt)
{
    if (n <= 0) return hipSuccess;
    k_adj_kick<<<blocks(3 * n), 256, 0, s>>>(abar, vbar, 3 * n, 0.5 * dt);
    return hipGetLastError();
}

hipError_t launch_adj_drift_kick(hipStream_t s, double *vbar, double *abar, const double *xbar,
                                 int64_t n, double dt)
{
    if (n <= 0) return hipSuccess;
    k_adj_drift_kick<<<blocks(3 * n), 256, 0, s>>>(vbar, abar, xbar, 3 * n, dt, 0.5 * dt);
    return hipGetLastError();
}

hipError_t launch_kick_drift_to(hipStream_t s, const double *x_in, double *v, const double *a,
                                double *x_out, int64_t n, double dt)
{
    if (n <= 0) return hipSuccess;
    k_kick_drift_to<<<blocks(3 * n), 256, 0, s>>>(x_in, v, a, x_out, 3 * n, 0.5 * dt, dt);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, double *dst, const double *src, int64_t count)
{
    if (count <= 0) return hipSuccess;
    k_copy<<<blocks(count), 256, 0, s>>>(dst, src, count);
    return hipGetLastError();
}

}  // namespace bhx
