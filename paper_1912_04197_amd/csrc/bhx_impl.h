// Internal declarations shared by the HIP translation units of libbhx.
// Device data layout, the tree header, and the kernel launchers each unit
// provides. Nothing here is part of the C ABI (include/bhx.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bhx.h"
#include "checks.h"

namespace bhx {

constexpr int kMaxLevel = 21;           // cells on a 2^21 grid per axis
constexpr int kLevels = kMaxLevel + 1;  // levels 0..21
constexpr uint32_t kQMax = 2097151u;    // 2^21 - 1

// Device status bits, latched until bh_sync().
enum : uint32_t { ST_NONFINITE = 1u, ST_CAPACITY = 2u, ST_STACK = 4u };

// One body in Morton order: position and mass (32 B, one aligned load pair).
struct alignas(32) Body {
    double x, y, z, m;
};

// One node's moments: centre of mass and mass.
struct alignas(32) NodeMom {
    double x, y, z, m;
};

// One node's structure: sorted body range, first child (-1 for a leaf),
// level in bits 0..7, number of children in bits 8..15 and the scene the
// node belongs to in bits 16..31.
struct alignas(16) NodeInfo {
    int32_t first, count, child0, lvl_nch;
};

__host__ __device__ inline int node_level(const NodeInfo &i) { return i.lvl_nch & 0xff; }
__host__ __device__ inline int node_nchild(const NodeInfo &i) { return (i.lvl_nch >> 8) & 0xff; }
__host__ __device__ inline int node_scene(const NodeInfo &i)
{
    return (int)((uint32_t)i.lvl_nch >> 16);
}
constexpr int kMaxScenes = 65535;

// Root cube of one scene. lo_enc / hi_enc hold the per-axis minimum and
// maximum as order-preserving integers while the box is being reduced.
struct SceneBox {
    unsigned long long lo_enc[3], hi_enc[3];
    double lo[3], hi[3];  // per-axis bounding box
    double L, S;          // root cube side and quantisation scale 2^21 / L
    double x0[3];         // root cube corner
    double s2[kLevels];   // squared cell side per level
};

// Tree header, written on the device by the build and read by later kernels,
// so a whole force evaluation runs without host round trips.
struct TreeHeader {
    int32_t level_count[kLevels + 1];  // nodes created per level (all scenes)
    uint32_t status;                   // ST_* bits
    int32_t cell_max;                  // most bodies in one node of level kHintLevel
};
// The level whose largest node the build reports for the choice of sort.
constexpr int kHintLevel = 5;
constexpr int kHintWords = 2 + kLevels;  // pinned launch-hint words of a workspace
// The levels 1..kPrefixLevels of a single scene's tree are read off the
// sorted keys: a level-kPrefixLevels cell is the key's top 3 kPrefixLevels
// bits, and the first body of each such cell gives every cell range above it.
constexpr int kPrefixLevels = 5;
constexpr int kPrefixCells = 1 << (3 * kPrefixLevels);  // 32768
constexpr int kPrefixShift = 63 - 3 * kPrefixLevels;

// Body layout of one call: n bodies in n_scenes contiguous scenes. For one
// scene every table is implicit (nullptr); otherwise scene_of gives each
// body's scene, chunks the bbox work items {scene, first, end} (none crosses
// a scene) and groups the walk groups {first, count, scene} (at most 64
// bodies, none crosses a scene), all in device memory.
struct Layout {
    int64_t n = 0;
    int n_scenes = 1;
    const int64_t *offsets = nullptr;  // device, n_scenes + 1
    const uint16_t *scene_of = nullptr;
    const int32_t *chunks = nullptr;   // [n_chunks][3]
    int n_chunks = 0;
    const int32_t *groups = nullptr;   // [n_groups][3]
    int n_groups = 0;
};
constexpr int kBoxChunk = 4096;  // bodies per bbox work item
constexpr int64_t kSmallBuild = 4096;  // a single scene this small is built by one block

// Morton interleave of 21-bit cell coordinates (x in the highest bit of
// each triplet) and its inverse.
// Spreads the low 21 bits of v so that bit i lands on bit 3i.
__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Inverse of spread3.
__device__ inline uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

// Number of set bits of m below this lane.
__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave (exact, integer), by DPP
// lane moves: four shifts within each row of 16 lanes, then the last lane of
// row 0 is added to row 1 and of row 2 to row 3, and the last lane of row 1
// to rows 2 and 3. Every lane of the wave must be active.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast31, 0xc, 0xf, false);
    return (uint32_t)x;
}

// 1 / sqrt(r2) in FP64 for a positive normal r2: the hardware estimate
// (relative error about 2^-24) refined by two Newton-Raphson steps on
// f(y) = y^-2 - r2, y <- y + y (1 - r2 y^2) / 2, each step squaring the
// relative error; on the whole normal range the result is within one ulp of
// the exact value. Cheaper than a correctly rounded sqrt followed by
// divisions, and well inside the FP64 parity bars.
__device__ inline double rsqrt_f64(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    double e = fma(-(r2 * y), y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-(r2 * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// A pair term counts only when its squared softened distance is a positive
// normal number in the precision it is computed in: r^2 = 0 (coincident
// unsoftened bodies) and subnormal r^2 (the same coincidence below the
// number range, where 1 / r^3 overflows) contribute nothing.
// r2 is a positive normal number (not 0, subnormal, infinite or NaN).
__device__ inline bool positive_normal(double r2) { return __builtin_amdgcn_class(r2, 0x100); }
// The FP32 pair terms' form of the same test (finite r2 at or above FLT_MIN).
constexpr float kFltMin = __FLT_MIN__;
__device__ inline bool positive_normal_f(float r2) { return r2 >= kFltMin; }

// Workspace owned by a context; sized once for n_max bodies.
struct Workspace {
    int64_t n_cap = 0, node_cap = 0;
    int sort_blocks_cap = 0, max_scenes = 1;
    uint64_t *keys[2] = {nullptr, nullptr};
    uint32_t *idx[2] = {nullptr, nullptr};
    uint32_t *sort_counts = nullptr;  // [256][sort blocks], scanned per digit row
    uint32_t *sort_totals = nullptr;  // [256]
    Body *body = nullptr;             // sorted bodies
    double *beps2 = nullptr;          // sorted eps^2
    // The state of a multi-step call, kept in the Morton order of the last
    // build (body, beps2 and idx[0], the caller index of each sorted body,
    // belong to it): velocities and accelerations in sorted order, and the
    // drifted state before the next sort (same order as the sorted state).
    double *tvel = nullptr;           // [n_cap][3]
    double *tacc = nullptr;           // [n_cap][3]
    Body *sbody = nullptr;            // [n_cap]
    double *svel = nullptr;           // [n_cap][3]
    double *seps2 = nullptr;          // [n_cap]
    uint32_t *scidx = nullptr;        // [n_cap]
    NodeInfo *ninfo = nullptr;
    NodeMom *nmom = nullptr;
    double *neps2 = nullptr;
    double *nquad = nullptr;      // [node_cap][6] quadrupoles, only with BH_FLAG_QUAD
    SceneBox *box = nullptr;      // [max_scenes]
    TreeHeader *hdr = nullptr;
    int32_t *counts = nullptr;    // [n_cap][2] per-body walk counts, caller order
    double *scratch = nullptr;    // [n_cap] potential for diagnostics
    double *red_part = nullptr;   // [reduction blocks][8][2] compensated partial sums
    double *dpart = nullptr;      // [kDirectPart] partial direct sums of split source ranges
    // Launch hints of the last build, written by the device into pinned host
    // memory (-1 before the first build): [0] its deepest non-empty level (the
    // next build launches the levels down to one below it one by one and the
    // rest in one block), [1] the most bodies in one node of level kHintLevel
    // (which picks the next build's sort), [2 + l] its node count on level l
    // (which picks how level l is split), kHintWords words in all.
    int32_t *depth_host = nullptr;
    int32_t *depth_dev = nullptr;  // the same memory as the device sees it
    // [kPrefixCells] first sorted body of each level-kPrefixLevels cell, or
    // INT32_MAX ("none"): set at creation, written by one build and restored
    // to "none" by the same build once read.
    int32_t *prefix_mark = nullptr;
};

// The direct sum splits its sources over up to kDirectSplits block rows when
// the targets alone give fewer than kDirectBlocks blocks; each row's partial
// sums (4 doubles per target) go to a workspace buffer of kDirectPart doubles
// and are added in row order.
constexpr int kDirectBlocks = 1024;
constexpr int kDirectSplits = 64;
constexpr int64_t kDirectPart = (int64_t)kDirectBlocks * 256 * 4;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRedBlocks = 512;

// Upper bound on the node count of the trees of n bodies in up to `scenes`
// scenes with the given bucket size: one root per scene, and every level
// below holds at most min(n, 8 n / (leaf + 1)) nodes, because its nodes are
// disjoint non-empty children of cells holding more than `leaf` bodies.
inline int64_t node_capacity(int64_t n, int leaf, int scenes = 1)
{
    if (n <= 0) return scenes > 1 ? scenes : 1;
    int64_t internal = n / (leaf + 1);
    int64_t per_level = 8 * internal < n ? 8 * internal : n;
    return (int64_t)(scenes > 1 ? scenes : 1) + (int64_t)kMaxLevel * per_level;
}

// Launchers (tree.hip). All enqueue on `s` and never synchronise; `bucket`
// (if given) receives the sort the build enqueued (bucket_sort_hint). The build
// launches one kernel per tree level down to one below the depth the
// previous build reported (a host read of pinned memory, frozen in a
// captured graph) and handles deeper levels in one block: any depth is
// built correctly, a deeper one more slowly.
hipError_t launch_build(const Workspace &w, hipStream_t s, const Layout &lay, const double *pos,
                        const double *mass, const double *eps, int leaf, bool *bucket = nullptr);
// The same build for one step on the sorted state (multi-step calls, more
// than kSmallBuild bodies or several scenes): the step's first kick and its
// drift (v = v + dt/2 a, x = x + dt v) run in the bounding-box pass over the
// sorted state of the previous build, and the gather carries velocities,
// softening and caller indices into the new order.
hipError_t launch_build_state(const Workspace &w, hipStream_t s, const Layout &lay, bool use_eps,
                              int leaf, double dt, bool *bucket = nullptr);
// Whether the next build of `lay` sorts by buckets of the top key bits (one
// scene above kSmallBuild bodies whose last build's level-kHintLevel nodes
// all fit a block's range) rather than by eight key passes; a host read of
// the pinned hints, frozen in a captured graph. Either sort gives the same
// order; the choice only affects speed.
bool bucket_sort_hint(const Workspace &w, const Layout &lay);
// scene_of[i] = scene of body i, from device offsets of n_scenes scenes
hipError_t launch_scene_of(hipStream_t s, const int64_t *offsets, int n_scenes,
                           uint16_t *scene_of);

struct WalkParams {
    int64_t n;
    const int32_t *groups = nullptr;  // walk groups of a multi-scene layout
    int n_groups = 0;
    double th2;     // theta^2
    double eps0sq;  // uniform softening squared (per-body eps not given)
    double G;
    double *acc;    // caller order, n x 3 (sorted order with acc_sorted)
    double *phi;    // caller order or nullptr (sorted order with acc_sorted)
    bool acc_sorted = false;
    int32_t *counts;  // caller order n x 2 or nullptr
    bool per_body_eps;
    int precision;
    int group;  // target bodies per wavefront: 64, 32 or 16
    const double *nquad = nullptr;  // node quadrupoles: add their terms (or nullptr)
};
constexpr int kDefaultWalkGroup = 64;
constexpr int64_t kSmallWalk = 131072;  // below this many bodies the default group is 16
// walk.hip
hipError_t launch_walk(const Workspace &w, hipStream_t s, const WalkParams &p);

// direct.hip
hipError_t launch_direct(hipStream_t s, const double *pos, const double *mass, const double *eps,
                         int64_t n, double eps0sq, double G, int precision, double *acc,
                         double *phi, double *part);

// adjoint.hip: workspace of the VJPs (BH_FLAG_ADJOINT)
// The trees a checkpointed segment's recomputation builds, one per step, kept
// for the VJPs at the same positions: slot k holds sorted bodies, eps^2,
// caller indices and keys (n each), the node tables (node_cap each), the
// scene box and the tree header of step k.
struct TreeSlots {
    int count = 0;
    int64_t n = 0, node_cap = 0;
    Body *body = nullptr;
    double *beps2 = nullptr;
    uint32_t *idx = nullptr;
    uint64_t *keys = nullptr;
    NodeInfo *ninfo = nullptr;
    NodeMom *nmom = nullptr;
    double *neps2 = nullptr;
    SceneBox *box = nullptr;
    TreeHeader *hdr = nullptr;
};
// A workspace whose tree arrays are slot k's (scratch arrays shared with w).
Workspace slot_view(const Workspace &w, const TreeSlots &t, int k);
// ORs the slots' status words into *status and clears them.
hipError_t launch_merge_status(hipStream_t s, TreeHeader *slot_hdr, int count, uint32_t *status);

struct AdjointWork {
    TreeSlots trees;         // allocated by the first segment VJP that fits in memory
    double *gt = nullptr;    // [n_cap][3] target-side gradients, sorted order
    double *badj = nullptr;  // [n_cap][4] source-side body adjoints, sorted order
    double *nadj = nullptr;  // [node_cap][5] node adjoints: gX, gm, g<eps^2>
    int32_t *nparent = nullptr;  // [node_cap] parent of each node (-1: the root)
    double *vwork = nullptr; // [n_cap][3] velocity while a segment is recomputed
    double *awork = nullptr; // [n_cap][3] acceleration while a segment is recomputed
};
hipError_t launch_tree_vjp(const Workspace &w, const AdjointWork &aw, hipStream_t s,
                           const WalkParams &p, const double *lambda, double *g_pos,
                           double *g_mass);
hipError_t launch_direct_vjp(hipStream_t s, const double *pos, const double *mass,
                             const double *eps, int64_t n, double eps0sq, double G,
                             const double *lambda, double *g_pos, double *g_mass, double *part);
hipError_t launch_adj_kick(hipStream_t s, double *abar, const double *vbar, int64_t n, double dt);
hipError_t launch_adj_drift_kick(hipStream_t s, double *vbar, double *abar, const double *xbar,
                                 int64_t n, double dt);
hipError_t launch_kick_drift_to(hipStream_t s, const double *x_in, double *v, const double *a,
                                double *x_out, int64_t n, double dt);
hipError_t launch_copy(hipStream_t s, double *dst, const double *src, int64_t count);

// integrate.hip
hipError_t launch_kick_drift(hipStream_t s, double *pos, double *vel, const double *acc, int64_t n,
                             double dt);
// contacts.hip: contact components of the bodies of the last build (label
// in caller order, size: n int32 scratch, counters: 3 device words).
hipError_t launch_contacts(const Workspace &w, hipStream_t s, const double *radius, int64_t n,
                           double skin, int32_t *label, int32_t *size,
                           unsigned long long *counters);
hipError_t launch_euler_substeps(hipStream_t s, double *pos, double *vel, const double *acc,
                                 int64_t n, double dt, int k);
hipError_t launch_kick(hipStream_t s, double *vel, const double *acc, int64_t n, double dt);
// The sorted state of a multi-step call from the caller's arrays (identity
// order; checks masses and softening lengths, flagging ST_NONFINITE), and
// back to them at its end.
hipError_t launch_state_pack(const Workspace &w, hipStream_t s, const double *pos,
                             const double *vel, const double *acc, const double *mass,
                             const double *eps, int64_t n, uint32_t *status);
hipError_t launch_state_unpack(const Workspace &w, hipStream_t s, double *pos, double *vel,
                               double *acc, int64_t n);
// Largest body density m / ((4/3) pi r^3) over the massive bodies and the
// gravity time-step bound 1 / (2 sqrt(G rho)) of eq. (dt_g) into out[0]
// (+inf with no massive body); work[0] is scratch; bad input sets ST_NONFINITE.
hipError_t launch_dt_bound(hipStream_t s, const double *mass, const double *radius, int64_t n,
                           double G, long long *work, double *out, uint32_t *status);
hipError_t launch_diag_reduce(hipStream_t s, const double *pos, const double *vel,
                              const double *mass, const double *phi, int64_t n, double *part,
                              double *out8_device);

}  // namespace bhx
