// C ABI of libbhx (declared in include/bhx.h): context and workspace
// ownership, host-side argument checks, launch sequencing on the caller's
// stream, the device status latch, multi-scene layouts and graph capture of
// integration steps.
#include <algorithm>
#include <dlfcn.h>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bhx_impl.h"

using bhx::Workspace;

struct bh_ctx {
    bh_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    Workspace w;
    std::string err;
    int64_t tree_n = -1;   // n of the last build, -1 before any
    bool bucket = false;   // the last build sorted by buckets of the top key bits
    bool tree_eps = false; // the last build had per-body eps
    int64_t walk_n = -1;   // n of the last walk that wrote counts
    double *diag_out = nullptr;
    bhx::AdjointWork aw;
    // BH_FLAG_TIMING: event triples (build start, walk start, walk end) not
    // yet folded into the totals
    std::vector<hipEvent_t> ev_pool;
    int ev_used = 0;
    int64_t timed_evals = 0;
    double build_ms = 0.0, walk_ms = 0.0;
    // several scenes: device tables of the current layout and their host copies
    int64_t *d_offsets = nullptr;
    uint16_t *d_scene_of = nullptr;
    int32_t *d_chunks = nullptr, *d_groups = nullptr;
    int64_t max_chunks = 0, max_groups = 0;
    std::vector<int64_t> h_offsets;
    std::vector<int32_t> h_chunks, h_groups;
    int layout_group = 0;
    uint64_t layout_gen = 0;  // bumped whenever the layout tables are re-uploaded
    bhx::Layout batch;
    // BH_FLAG_GRAPH: one captured step, replayed on a stream of the context
    hipStream_t cstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<double> gkey;
    bool capturing = false;
    int gdepth = -1;  // depth hint the captured step's build was launched with
    int gbucket = -1; // sort the captured step's build was launched with (bucket_sort_hint)
};

namespace {

// roctx ranges for BH_FLAG_MARKERS, resolved from the ROCm tracing library at
// run time so that the library does not depend on it.
struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};
const Roctx &roctx()
{
    static const Roctx r = [] {
        Roctx x;
        for (const char *lib : {"librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"}) {
            void *h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            x.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
            x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
            if (x.push && x.pop) break;
            x = Roctx{};
        }
        return x;
    }();
    return r;
}

}  // namespace

namespace {

bh_status fail(bh_ctx *c, bh_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

bh_status hip_fail(bh_ctx *c, hipError_t e, const char *what)
{
    return fail(c, BH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHX_HIP(c, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, int64_t count)
{
    if (count < 1) count = 1;
    return hipMalloc((void **)p, (size_t)count * sizeof(T));
}

void free_slots(bhx::TreeSlots &t)
{
    void *ptrs[] = {t.body, t.beps2, t.idx, t.keys, t.ninfo, t.nmom, t.neps2, t.box, t.hdr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    t = bhx::TreeSlots{};
}

void free_aw(bhx::AdjointWork &a)
{
    free_slots(a.trees);
    void *ptrs[] = {a.gt, a.badj, a.nadj, a.nparent, a.vwork, a.awork};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    a = bhx::AdjointWork{};
}

void free_ws(Workspace &w)
{
    void *ptrs[] = {w.keys[0], w.keys[1], w.idx[0],  w.idx[1],      w.sort_counts,
                    w.sort_totals, w.body, w.beps2, w.ninfo, w.nmom, w.neps2, w.box,
                    w.hdr, w.counts, w.scratch, w.red_part, w.nquad, w.dpart,
                    w.tvel, w.tacc, w.sbody, w.svel, w.seps2, w.scidx, w.prefix_mark};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (w.depth_host) (void)hipHostFree(w.depth_host);
    w = Workspace{};
}

void free_extras(bh_ctx *c)
{
    void *ptrs[] = {c->d_offsets, c->d_scene_of, c->d_chunks, c->d_groups, c->diag_out};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto ev : c->gev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->cstream) (void)hipStreamDestroy(c->cstream);
    for (auto ev : c->ev_pool)
        if (ev) (void)hipEventDestroy(ev);
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

bh_status check_bodies(bh_ctx *c, const double *pos, const double *mass, int64_t n)
{
    if (!c) return BH_E_INVALID;
    if (n < 0) return fail(c, BH_E_INVALID, "n < 0");
    if (n > c->w.n_cap) return fail(c, BH_E_CAPACITY, "n exceeds the context's n_max");
    if (n > 0 && (!pos || !mass)) return fail(c, BH_E_INVALID, "NULL pos or mass with n > 0");
    return BH_OK;
}

constexpr int kEvTriples = 256;

// Adds the elapsed times of the recorded event triples to the totals.
bh_status fold_timing(bh_ctx *c)
{
    if (c->ev_used == 0) return BH_OK;
    BHX_HIP(c, hipEventSynchronize(c->ev_pool[3 * c->ev_used - 1]));
    for (int t = 0; t < c->ev_used; t++) {
        float b = 0.f, w = 0.f;
        BHX_HIP(c, hipEventElapsedTime(&b, c->ev_pool[3 * t], c->ev_pool[3 * t + 1]));
        BHX_HIP(c, hipEventElapsedTime(&w, c->ev_pool[3 * t + 1], c->ev_pool[3 * t + 2]));
        c->build_ms += b;
        c->walk_ms += w;
        c->timed_evals++;
    }
    c->ev_used = 0;
    return BH_OK;
}

// A roctx range over one phase's enqueueing (BH_FLAG_MARKERS), popped when
// the scope ends.
struct Marker {
    bool on;
    Marker(const bh_ctx *c, const char *name)
        : on((c->cfg.flags & BH_FLAG_MARKERS) && roctx().push != nullptr)
    {
        if (on) roctx().push(name);
    }
    Marker(const Marker &) = delete;
    Marker &operator=(const Marker &) = delete;
    ~Marker()
    {
        if (on) roctx().pop();
    }
};

bh_status record(bh_ctx *c, int which)
{
    if (!(c->cfg.flags & BH_FLAG_TIMING) || c->capturing) return BH_OK;
    if (which == 0 && c->ev_used == kEvTriples) {
        bh_status s = fold_timing(c);
        if (s) return s;
    }
    BHX_HIP(c, hipEventRecord(c->ev_pool[3 * c->ev_used + which], c->stream));
    if (which == 2) c->ev_used++;
    return BH_OK;
}

// Bodies per walk wavefront for a call on n bodies: the configured size, or
// by default 64 for large calls and 16 below 2^17 bodies, where 64-body groups
// leave too few wavefronts to fill the chip.
int walk_group(const bh_ctx *c, int64_t n)
{
    if (c->cfg.walk_group) return c->cfg.walk_group;
    return n < bhx::kSmallWalk ? 16 : bhx::kDefaultWalkGroup;
}

// The same for the adjoint walk, whose per-item work is heavier: measured
// best at 16 below 2^15 bodies, 32 up to 2^19, 64 above.
int vjp_group(const bh_ctx *c, int64_t n)
{
    if (c->cfg.walk_group) return c->cfg.walk_group;
    return n < (1 << 15) ? 16 : n < (1 << 19) ? 32 : 64;
}

bhx::Layout single(int64_t n)
{
    bhx::Layout L;
    L.n = n;
    return L;
}

// The walk of the tree just built, for the bodies of `lay`.
bh_status walk(bh_ctx *c, const Workspace &w, const bhx::Layout &lay, double softening,
               bool use_eps, double theta, double *acc, double *phi, bool acc_sorted)
{
    const int64_t n = lay.n;
    c->tree_n = n;
    c->tree_eps = use_eps;
    bhx::WalkParams p;
    p.n = n;
    p.th2 = theta * theta;
    p.eps0sq = softening * softening;
    p.G = c->cfg.G;
    p.acc = acc;
    p.phi = phi;
    p.acc_sorted = acc_sorted;
    p.counts = (c->cfg.flags & BH_FLAG_COUNTS) ? w.counts : nullptr;
    p.per_body_eps = use_eps;
    p.precision = c->cfg.precision;
    p.group = walk_group(c, n);
    p.nquad = w.nquad;
    p.groups = lay.groups;
    p.n_groups = lay.n_groups;
    {
        Marker m(c, "bhx walk");
        BHX_HIP(c, bhx::launch_walk(w, c->stream, p));
    }
    if (p.counts) c->walk_n = n;
    return BH_OK;
}

// Build and walk on the context's tree arrays, or on those of `w` (a tree
// slot of the adjoint).
bh_status force_tree(bh_ctx *c, const bhx::Layout &lay, const double *pos, const double *mass,
                     double softening, const double *eps, double theta, double *acc, double *phi,
                     const Workspace *w = nullptr)
{
    const Workspace &ws = w ? *w : c->w;
    bh_status st = record(c, 0);
    if (st) return st;
    {
        Marker m(c, "bhx build");
        BHX_HIP(c, bhx::launch_build(ws, c->stream, lay, pos, mass, eps, c->cfg.leaf_size,
                                     &c->bucket));
    }
    st = record(c, 1);
    if (st) return st;
    st = walk(c, ws, lay, softening, eps != nullptr, theta, acc, phi, false);
    if (st) return st;
    return record(c, 2);
}

bh_status force_direct(bh_ctx *c, const double *pos, const double *mass, double softening,
                       const double *eps, double *acc, double *phi, int64_t n, int precision)
{
    Marker m(c, "bhx direct");
    BHX_HIP(c, bhx::launch_direct(c->stream, pos, mass, eps, n, softening * softening, c->cfg.G,
                                  precision, acc, phi, c->w.dpart));
    return BH_OK;
}

// VJP of the force map at pos (tree when theta >= 0, else direct), added
// into g_pos and g_mass.
bh_status vjp(bh_ctx *c, const double *pos, const double *mass, double softening,
              const double *eps, double theta, const double *lambda, double *g_pos,
              double *g_mass, int64_t n, const Workspace *tree = nullptr)
{
    if (n == 0) return BH_OK;
    Marker m(c, "bhx vjp");
    if (theta >= 0.0) {
        // `tree`: the tree of these positions, built by the segment's
        // recomputation and kept in a slot; else build it here
        if (!tree) {
            BHX_HIP(c, bhx::launch_build(c->w, c->stream, single(n), pos, mass, eps,
                                         c->cfg.leaf_size, &c->bucket));
            c->tree_n = n;
            c->tree_eps = eps != nullptr;
        }
        bhx::WalkParams p;
        p.n = n;
        p.th2 = theta * theta;
        p.eps0sq = softening * softening;
        p.G = c->cfg.G;
        p.acc = nullptr;
        p.phi = nullptr;
        p.counts = nullptr;
        p.per_body_eps = eps != nullptr;
        p.precision = c->cfg.precision;  // FP32C terms in an FP32C context
        p.group = vjp_group(c, n);
        BHX_HIP(c, bhx::launch_tree_vjp(tree ? *tree : c->w, c->aw, c->stream, p, lambda, g_pos,
                                        g_mass));
    } else {
        BHX_HIP(c, bhx::launch_direct_vjp(c->stream, pos, mass, eps, n, softening * softening,
                                          c->cfg.G, lambda, g_pos, g_mass, c->w.dpart));
    }
    return BH_OK;
}

// Uploads the tables of a layout of n_scenes contiguous scenes (host
// offsets), unless the context already holds the same layout.
bh_status set_layout(bh_ctx *c, int32_t n_scenes, const int64_t *offsets)
{
    if (n_scenes < 1 || n_scenes > c->w.max_scenes || !offsets)
        return fail(c, BH_E_INVALID, "n_scenes outside 1..max_scenes, or NULL offsets");
    if (offsets[0] != 0) return fail(c, BH_E_INVALID, "offsets[0] must be 0");
    for (int32_t k = 0; k < n_scenes; k++)
        if (offsets[k + 1] <= offsets[k])
            return fail(c, BH_E_INVALID, "every scene needs at least one body");
    const int64_t n = offsets[n_scenes];
    if (n > c->w.n_cap) return fail(c, BH_E_CAPACITY, "total bodies exceed n_max");
    const int gb = walk_group(c, n);
    if (c->layout_group == gb && (int64_t)c->h_offsets.size() == n_scenes + 1 &&
        std::equal(c->h_offsets.begin(), c->h_offsets.end(), offsets))
        return BH_OK;
    // The tables are rewritten in place: wait until no queued or replayed step
    // still reads them, and drop a graph captured with the old layout.
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    if (c->cstream) BHX_HIP(c, hipStreamSynchronize(c->cstream));
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    c->layout_gen++;
    c->h_offsets.assign(offsets, offsets + n_scenes + 1);
    c->h_chunks.clear();
    c->h_groups.clear();
    for (int32_t k = 0; k < n_scenes; k++) {
        for (int64_t f = offsets[k]; f < offsets[k + 1]; f += bhx::kBoxChunk) {
            const int64_t e = std::min(offsets[k + 1], f + bhx::kBoxChunk);
            c->h_chunks.insert(c->h_chunks.end(), {k, (int32_t)f, (int32_t)e});
        }
    }
    // Walk groups in the order the blocks are dealt, costliest first (the
    // scenes by decreasing size: a body of a larger scene walks a deeper tree
    // and interacts more), each scene's groups in Morton order, so that the
    // cheap groups of small scenes fill the end of the launch.
    std::vector<int32_t> by_size((size_t)n_scenes);
    for (int32_t k = 0; k < n_scenes; k++) by_size[(size_t)k] = k;
    std::stable_sort(by_size.begin(), by_size.end(), [&](int32_t a, int32_t b) {
        return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
    });
    for (int32_t k : by_size) {
        for (int64_t f = offsets[k]; f < offsets[k + 1]; f += gb) {
            const int64_t e = std::min(offsets[k + 1], f + gb);
            c->h_groups.insert(c->h_groups.end(), {(int32_t)f, (int32_t)(e - f), k});
        }
    }
    const int64_t nchunks = (int64_t)c->h_chunks.size() / 3, ngroups = (int64_t)c->h_groups.size() / 3;
    if (nchunks > c->max_chunks || ngroups > c->max_groups)
        return fail(c, BH_E_CAPACITY, "layout tables exceed the context's capacity");
    // pageable sources: the copies complete before the calls return
    BHX_HIP(c, hipMemcpy(c->d_offsets, offsets, (size_t)(n_scenes + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice));
    BHX_HIP(c, hipMemcpy(c->d_chunks, c->h_chunks.data(), c->h_chunks.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    BHX_HIP(c, hipMemcpy(c->d_groups, c->h_groups.data(), c->h_groups.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    BHX_HIP(c, bhx::launch_scene_of(c->stream, c->d_offsets, n_scenes, c->d_scene_of));
    c->layout_group = gb;
    bhx::Layout &L = c->batch;
    L.n = n;
    L.n_scenes = n_scenes;
    L.offsets = c->d_offsets;
    L.scene_of = c->d_scene_of;
    L.chunks = c->d_chunks;
    L.n_chunks = (int)nchunks;
    L.groups = c->d_groups;
    L.n_groups = (int)ngroups;
    return BH_OK;
}

// One kick-drift-kick step of the bodies of `lay` on the context's stream.
bh_status kdk_step(bh_ctx *c, const bhx::Layout &lay, double *pos, double *vel,
                   const double *mass, double softening, const double *eps, double theta,
                   double dt, double *acc)
{
    Marker m(c, "bhx step");
    BHX_HIP(c, bhx::launch_kick_drift(c->stream, pos, vel, acc, lay.n, dt));
    bh_status s = theta >= 0.0
                      ? force_tree(c, lay, pos, mass, softening, eps, theta, acc, nullptr)
                      : force_direct(c, pos, mass, softening, eps, acc, nullptr, lay.n,
                                     c->cfg.precision);
    if (s) return s;
    BHX_HIP(c, bhx::launch_kick(c->stream, vel, acc, lay.n, dt));
    return BH_OK;
}

// Multi-step calls on a tree (more than kSmallBuild bodies, or several
// scenes) keep the state in the Morton order of the last build between
// steps: packed from the caller's arrays at the start of the call and
// written back at its end.
bool sorted_state(const bhx::Layout &lay, double theta, int32_t nsteps, bool graph)
{
    return theta >= 0.0 && (nsteps > 1 || graph) &&
           (lay.n_scenes > 1 || lay.n > bhx::kSmallBuild);
}

// One kick-drift-kick step on the sorted state: the first kick and the drift
// run in the build's bounding-box pass, the walk writes the accelerations in
// sorted order and the second kick uses them there.
bh_status kdk_step_state(bh_ctx *c, const bhx::Layout &lay, double softening, bool use_eps,
                         double theta, double dt)
{
    Marker m(c, "bhx step");
    Workspace &w = c->w;
    bh_status st = record(c, 0);
    if (st) return st;
    {
        Marker mb(c, "bhx build");
        BHX_HIP(c, bhx::launch_build_state(w, c->stream, lay, use_eps, c->cfg.leaf_size, dt,
                                           &c->bucket));
    }
    st = record(c, 1);
    if (st) return st;
    st = walk(c, w, lay, softening, use_eps, theta, w.tacc, nullptr, true);
    if (st) return st;
    st = record(c, 2);
    if (st) return st;
    BHX_HIP(c, bhx::launch_kick(c->stream, w.tvel, w.tacc, lay.n, dt));
    return BH_OK;
}

// One step of either kind.
bh_status any_step(bh_ctx *c, bool state, const bhx::Layout &lay, double *pos, double *vel,
                   const double *mass, double softening, const double *eps, double theta,
                   double dt, double *acc)
{
    return state ? kdk_step_state(c, lay, softening, eps != nullptr, theta, dt)
                 : kdk_step(c, lay, pos, vel, mass, softening, eps, theta, dt, acc);
}

// nsteps steps. With BH_FLAG_GRAPH one step is captured once per argument set
// on the context's own stream and replayed; that stream is ordered after the
// caller's stream and the caller's stream after it, with events.
bh_status run_steps(bh_ctx *c, const bhx::Layout &lay, double *pos, double *vel,
                    const double *mass, double softening, const double *eps, double theta,
                    double dt, int32_t nsteps, double *acc)
{
    if (nsteps <= 0 || lay.n == 0) return BH_OK;
    const bool graph = (c->cfg.flags & BH_FLAG_GRAPH) != 0;
    const bool state = sorted_state(lay, theta, nsteps, graph);
    if (state)
        BHX_HIP(c, bhx::launch_state_pack(c->w, c->stream, pos, vel, acc, mass, eps, lay.n,
                                          &c->w.hdr->status));
    if (!graph) {
        for (int32_t k = 0; k < nsteps; k++) {
            bh_status s = any_step(c, state, lay, pos, vel, mass, softening, eps, theta, dt, acc);
            if (s) return s;
        }
        if (state) BHX_HIP(c, bhx::launch_state_unpack(c->w, c->stream, pos, vel, acc, lay.n));
        return BH_OK;
    }
    // everything a captured step bakes in: pointers, sizes, the layout tables'
    // generation (their contents and the grid sizes derived from them) and the
    // physical parameters
    std::vector<double> key = {(double)(uintptr_t)pos, (double)(uintptr_t)vel,
                               (double)(uintptr_t)mass, (double)(uintptr_t)eps,
                               (double)(uintptr_t)acc, (double)lay.n, (double)(uintptr_t)lay.groups,
                               (double)lay.n_scenes, (double)lay.n_groups, (double)lay.n_chunks,
                               (double)(lay.groups ? c->layout_gen : 0), softening, theta, dt};
    hipStream_t caller = c->stream;
    // The build launches one kernel per tree level down to one below the
    // depth its previous run reported (pinned memory the device writes), and
    // handles any deeper level in one block: a captured step keeps the hint
    // it was captured with (levels 0..gdepth split by their own launches, so
    // trees of depth up to gdepth + 1 at full width), so it is captured again
    // once a replayed build reports a deeper tree than that, or when the first
    // capture had no hint yet (it launched every level).
    const int depth_now = c->w.depth_host ? *(const volatile int32_t *)c->w.depth_host : -1;
    const bool deeper = depth_now >= 0 && (c->gdepth < 0 || depth_now > c->gdepth + 1);
    // likewise when the hints now pick the other sort (same order, other speed)
    const int bucket_now = bhx::bucket_sort_hint(c->w, lay) ? 1 : 0;
    if (!c->gexec || key != c->gkey || deeper || bucket_now != c->gbucket) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        if (c->graph) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
        }
        BHX_HIP(c, hipStreamBeginCapture(c->cstream, hipStreamCaptureModeThreadLocal));
        c->stream = c->cstream;
        c->capturing = true;
        c->gdepth = depth_now;
        c->gbucket = bucket_now;
        bh_status s = any_step(c, state, lay, pos, vel, mass, softening, eps, theta, dt, acc);
        c->capturing = false;
        c->stream = caller;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cstream, &g);
        if (s) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        c->graph = g;
        BHX_HIP(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
        c->gkey = key;
    }
    BHX_HIP(c, hipEventRecord(c->gev[0], caller));
    BHX_HIP(c, hipStreamWaitEvent(c->cstream, c->gev[0], 0));
    for (int32_t k = 0; k < nsteps; k++) {
        Marker m(c, "bhx step (graph)");
        BHX_HIP(c, hipGraphLaunch(c->gexec, c->cstream));
    }
    BHX_HIP(c, hipEventRecord(c->gev[1], c->cstream));
    BHX_HIP(c, hipStreamWaitEvent(caller, c->gev[1], 0));
    if (state) BHX_HIP(c, bhx::launch_state_unpack(c->w, caller, pos, vel, acc, lay.n));
    return BH_OK;
}

// The argument checks the two leapfrog VJPs share.
bh_status check_vjp_args(bh_ctx *c, double softening, double theta, double dt, int32_t nsteps)
{
    if (!(c->cfg.flags & BH_FLAG_ADJOINT))
        return fail(c, BH_E_STATE, "the context was created without BH_FLAG_ADJOINT");
    if ((c->cfg.flags & BH_FLAG_QUAD) && theta >= 0.0)
        return fail(c, BH_E_STATE, "no VJP of the quadrupole walk (BH_FLAG_QUAD)");
    if (std::isnan(theta) || std::isinf(theta)) return fail(c, BH_E_INVALID, "theta not finite");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (!std::isfinite(dt)) return fail(c, BH_E_INVALID, "dt not finite");
    if (nsteps < 0) return fail(c, BH_E_INVALID, "nsteps < 0");
    return BH_OK;
}

// The reverse sweep over nsteps steps whose end positions are traj[0..):
// per step, last first, the second kick's adjoint, the force VJP at the
// step's end positions, then the drift's and the first kick's.
bh_status reverse_sweep(bh_ctx *c, const double *traj, const double *mass, double softening,
                        const double *eps, double theta, double dt, int32_t nsteps, double *xbar,
                        double *vbar, double *abar, double *g_mass, int64_t n,
                        bool kept_trees = false)
{
    const int64_t n3 = 3 * n;
    for (int32_t k = nsteps - 1; k >= 0; k--) {
        BHX_HIP(c, bhx::launch_adj_kick(c->stream, abar, vbar, n, dt));
        const Workspace slot = kept_trees ? bhx::slot_view(c->w, c->aw.trees, k) : c->w;
        bh_status s = vjp(c, traj + (int64_t)k * n3, mass, softening, eps, theta, abar, xbar,
                          g_mass, n, kept_trees ? &slot : nullptr);
        if (s) return s;
        BHX_HIP(c, bhx::launch_adj_drift_kick(c->stream, vbar, abar, xbar, n, dt));
    }
    return BH_OK;
}

// Tree slots for the nsteps steps of a segment of n bodies: kept from an
// earlier call when large enough, else allocated once the device has twice
// their size free; false (the VJPs then rebuild their trees) otherwise.
bool ensure_tree_slots(bh_ctx *c, int32_t nsteps, int64_t n)
{
    bhx::TreeSlots &t = c->aw.trees;
    if (t.count >= nsteps && t.n >= n) return true;
    free_slots(t);
    const int64_t node_cap = bhx::node_capacity(n, c->cfg.leaf_size, 1);
    const size_t per = (size_t)n * (sizeof(bhx::Body) + sizeof(double) + sizeof(uint32_t) +
                                    sizeof(uint64_t)) +
                       (size_t)node_cap * (sizeof(bhx::NodeInfo) + sizeof(bhx::NodeMom) +
                                           sizeof(double)) +
                       sizeof(bhx::SceneBox) + sizeof(bhx::TreeHeader);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || per * (size_t)nsteps * 2 > free_b)
        return false;
    t.n = n;
    t.node_cap = node_cap;
    const int64_t k = nsteps;
    hipError_t r = hipSuccess;
    auto A = [&](hipError_t x) {
        if (r == hipSuccess) r = x;
    };
    A(dalloc(&t.body, k * n));
    A(dalloc(&t.beps2, k * n));
    A(dalloc(&t.idx, k * n));
    A(dalloc(&t.keys, k * n));
    A(dalloc(&t.ninfo, k * node_cap));
    A(dalloc(&t.nmom, k * node_cap));
    A(dalloc(&t.neps2, k * node_cap));
    A(dalloc(&t.box, k));
    A(dalloc(&t.hdr, k));
    if (r == hipSuccess) r = hipMemset(t.hdr, 0, (size_t)k * sizeof(bhx::TreeHeader));
    if (r != hipSuccess) {
        (void)hipGetLastError();
        free_slots(t);
        return false;
    }
    t.count = nsteps;
    return true;
}

}  // namespace

extern "C" {

bh_status bh_create(const bh_config *cfg, void *hip_stream, bh_ctx **out)
{
    if (!cfg || !out) return BH_E_INVALID;
    *out = nullptr;
    if (cfg->n_max < 0 || cfg->n_max > ((int64_t)1 << 30)) return BH_E_INVALID;
    if (cfg->leaf_size < 1 || cfg->leaf_size > 64) return BH_E_INVALID;
    if (cfg->precision != BH_FP64 && cfg->precision != BH_FP32C) return BH_E_INVALID;
    if (!std::isfinite(cfg->G)) return BH_E_INVALID;
    if (cfg->flags &
        ~(uint32_t)(BH_FLAG_COUNTS | BH_FLAG_TIMING | BH_FLAG_ADJOINT | BH_FLAG_GRAPH |
                    BH_FLAG_QUAD | BH_FLAG_MARKERS))
        return BH_E_INVALID;
    if (cfg->max_scenes < 0 || cfg->max_scenes > bhx::kMaxScenes) return BH_E_INVALID;
    if (cfg->walk_group != 0 && cfg->walk_group != 16 && cfg->walk_group != 32 &&
        cfg->walk_group != 64)
        return BH_E_INVALID;

    if (cfg->flags & BH_FLAG_MARKERS) (void)roctx();  // resolve the library once, here
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_E_OOM;
    c->cfg = *cfg;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return BH_E_HIP;
    }
    Workspace &w = c->w;
    const int64_t n = cfg->n_max > 0 ? cfg->n_max : 1;
    w.n_cap = cfg->n_max;
    const int max_scenes = cfg->max_scenes > 0 ? cfg->max_scenes : 1;
    int64_t node_cap = bhx::node_capacity(n, cfg->leaf_size, max_scenes);
    if (node_cap > INT32_MAX - 16) node_cap = INT32_MAX - 16;
    w.node_cap = node_cap;
    w.sort_blocks_cap = (int)((n + bhx::kSortTile - 1) / bhx::kSortTile);
    w.max_scenes = max_scenes;
    hipError_t r = hipSuccess;
    auto A = [&](hipError_t x) {
        if (r == hipSuccess) r = x;
    };
    A(dalloc(&w.keys[0], n));
    A(dalloc(&w.keys[1], n));
    A(dalloc(&w.idx[0], n));
    A(dalloc(&w.idx[1], n));
    A(dalloc(&w.sort_counts, (int64_t)256 * w.sort_blocks_cap));
    A(dalloc(&w.sort_totals, 256));
    A(dalloc(&w.body, n));
    A(dalloc(&w.beps2, n));
    A(dalloc(&w.tvel, 3 * n));
    A(dalloc(&w.tacc, 3 * n));
    A(dalloc(&w.sbody, n));
    A(dalloc(&w.svel, 3 * n));
    A(dalloc(&w.seps2, n));
    A(dalloc(&w.scidx, n));
    A(dalloc(&w.ninfo, node_cap));
    A(dalloc(&w.prefix_mark, bhx::kPrefixCells));
    if (r == hipSuccess)
        r = hipMemsetD32((hipDeviceptr_t)w.prefix_mark, INT32_MAX, bhx::kPrefixCells);
    A(dalloc(&w.nmom, node_cap));
    A(dalloc(&w.neps2, node_cap));
    A(dalloc(&w.box, max_scenes));
    if (max_scenes > 1) {
        c->max_chunks = n / bhx::kBoxChunk + max_scenes;
        c->max_groups = n / 16 + max_scenes;
        A(dalloc(&c->d_offsets, max_scenes + 1));
        A(dalloc(&c->d_scene_of, n));
        A(dalloc(&c->d_chunks, 3 * c->max_chunks));
        A(dalloc(&c->d_groups, 3 * c->max_groups));
    }
    if (cfg->flags & BH_FLAG_GRAPH) {
        A(hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking));
        A(hipEventCreateWithFlags(&c->gev[0], hipEventDisableTiming));
        A(hipEventCreateWithFlags(&c->gev[1], hipEventDisableTiming));
    }
    A(dalloc(&w.hdr, 1));
    if (cfg->flags & BH_FLAG_COUNTS) A(dalloc(&w.counts, 2 * n));
    if (cfg->flags & BH_FLAG_QUAD) A(dalloc(&w.nquad, 6 * node_cap));
    A(dalloc(&w.scratch, 4 * n));
    A(dalloc(&w.red_part, (int64_t)bhx::kRedBlocks * 16));
    A(dalloc(&w.dpart, bhx::kDirectPart));
    A(dalloc(&c->diag_out, 8));
    A(hipHostMalloc((void **)&w.depth_host, bhx::kHintWords * sizeof(int32_t),
                    hipHostMallocMapped));
    if (r == hipSuccess) {
        for (int i = 0; i < bhx::kHintWords; i++) w.depth_host[i] = -1;
        r = hipHostGetDevicePointer((void **)&w.depth_dev, w.depth_host, 0);
    }
    if (cfg->flags & BH_FLAG_ADJOINT) {
        A(dalloc(&c->aw.gt, 3 * n));
        A(dalloc(&c->aw.badj, 4 * n));
        A(dalloc(&c->aw.nadj, 5 * node_cap));
        A(dalloc(&c->aw.nparent, node_cap));
        A(dalloc(&c->aw.vwork, 3 * n));
        A(dalloc(&c->aw.awork, 3 * n));
    }
    if (cfg->flags & BH_FLAG_TIMING) {
        c->ev_pool.resize(3 * kEvTriples, nullptr);
        for (auto &ev : c->ev_pool)
            if (r == hipSuccess) r = hipEventCreate(&ev);
    }
    if (r == hipSuccess) r = hipMemset(w.hdr, 0, sizeof(bhx::TreeHeader));
    if (r == hipSuccess) r = hipDeviceSynchronize();
    if (r != hipSuccess) {
        bh_status st = (r == hipErrorOutOfMemory) ? BH_E_OOM : BH_E_HIP;
        free_ws(w);
        free_aw(c->aw);
        free_extras(c);
        delete c;
        return st;
    }
    *out = c;
    return BH_OK;
}

void bh_destroy(bh_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->cstream) (void)hipStreamSynchronize(c->cstream);
    free_ws(c->w);
    free_aw(c->aw);
    free_extras(c);
    delete c;
}

bh_status bh_set_stream(bh_ctx *c, void *hip_stream)
{
    if (!c) return BH_E_INVALID;
    c->stream = (hipStream_t)hip_stream;
    return BH_OK;
}

const char *bh_last_error(const bh_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

bh_status bh_sync(bh_ctx *c)
{
    if (!c) return BH_E_INVALID;
    uint32_t st = 0;
    BHX_HIP(c, hipMemcpyAsync(&st, &c->w.hdr->status, sizeof(st), hipMemcpyDeviceToHost,
                              c->stream));
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    uint32_t ck = 0;  // device checks (checked build only)
    BHX_HIP(c, bhx::walk_take_checks(&ck));
    BHX_HIP(c, bhx::adjoint_take_checks(&ck));
    BHX_HIP(c, bhx::tree_take_checks(&ck));
    if (ck) {
        static const char *names[] = {"traversal stack", "interaction ring", "pair list",
                                      "index bounds", "key order", "child partition",
                                      "bucket range"};
        std::string msg = "device check failed:";
        for (int b = 0; b < 7; b++)
            if (ck & (1u << b)) msg += std::string(" ") + names[b];
        return fail(c, BH_E_CHECK, msg);
    }
    if (st == 0) return BH_OK;
    const uint32_t zero = 0;
    BHX_HIP(c, hipMemcpyAsync(&c->w.hdr->status, &zero, sizeof(zero), hipMemcpyHostToDevice,
                              c->stream));
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    if (st & bhx::ST_NONFINITE)
        return fail(c, BH_E_NONFINITE, "non-finite position, mass or softening, or negative mass");
    if (st & bhx::ST_CAPACITY) return fail(c, BH_E_CAPACITY, "node table overflow");
    return fail(c, BH_E_STACK, "unknown device status");
}

bh_status bh_build_tree(bh_ctx *c, const double *pos, const double *mass, const double *eps,
                        int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    BHX_HIP(c, bhx::launch_build(c->w, c->stream, single(n), pos, mass, eps, c->cfg.leaf_size,
                                 &c->bucket));
    c->tree_n = n;
    c->tree_eps = eps != nullptr;
    return BH_OK;
}

bh_status bh_compute_accel(bh_ctx *c, const double *pos, const double *mass, double softening,
                           const double *eps, double theta, double *acc, double *phi, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!finite_nonneg(theta)) return fail(c, BH_E_INVALID, "theta must be finite and >= 0");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (n > 0 && !acc) return fail(c, BH_E_INVALID, "NULL acc");
    return force_tree(c, single(n), pos, mass, softening, eps, theta, acc, phi);
}

bh_status bh_compute_accel_direct(bh_ctx *c, const double *pos, const double *mass,
                                  double softening, const double *eps, double *acc, double *phi,
                                  int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (n > 0 && !acc) return fail(c, BH_E_INVALID, "NULL acc");
    return force_direct(c, pos, mass, softening, eps, acc, phi, n, c->cfg.precision);
}

bh_status bh_step_leapfrog(bh_ctx *c, double *pos, double *vel, const double *mass,
                           double softening, const double *eps, double theta, double dt,
                           int32_t nsteps, double *acc, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (std::isnan(theta) || std::isinf(theta)) return fail(c, BH_E_INVALID, "theta not finite");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (!std::isfinite(dt)) return fail(c, BH_E_INVALID, "dt not finite");
    if (nsteps < 0) return fail(c, BH_E_INVALID, "nsteps < 0");
    if (n > 0 && (!vel || !acc)) return fail(c, BH_E_INVALID, "NULL vel or acc");
    return run_steps(c, single(n), pos, vel, mass, softening, eps, theta, dt, nsteps, acc);
}

bh_status bh_step_euler(bh_ctx *c, double *pos, double *vel, const double *mass,
                        double softening, const double *eps, double theta, double dt,
                        int32_t nsteps, int32_t every, double *acc, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (std::isnan(theta) || std::isinf(theta)) return fail(c, BH_E_INVALID, "theta not finite");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (!std::isfinite(dt)) return fail(c, BH_E_INVALID, "dt not finite");
    if (nsteps < 0) return fail(c, BH_E_INVALID, "nsteps < 0");
    if (every < 1) return fail(c, BH_E_INVALID, "every < 1");
    if (n > 0 && (!vel || !acc)) return fail(c, BH_E_INVALID, "NULL vel or acc");
    if (n == 0) return BH_OK;
    // substeps in runs of `every` (one fused launch each), gravity after each
    // full run
    for (int32_t done = 0; done < nsteps;) {
        const int32_t k = nsteps - done < every ? nsteps - done : every;
        BHX_HIP(c, bhx::launch_euler_substeps(c->stream, pos, vel, acc, n, dt, k));
        done += k;
        if (k == every) {
            s = theta >= 0.0 ? force_tree(c, single(n), pos, mass, softening, eps, theta, acc, nullptr)
                             : force_direct(c, pos, mass, softening, eps, acc, nullptr, n,
                                            c->cfg.precision);
            if (s) return s;
        }
    }
    return BH_OK;
}

bh_status bh_contact_components(bh_ctx *c, const double *pos, const double *mass,
                                const double *radius, double skin, int32_t *label,
                                int64_t *n_contacts, int64_t *n_aggregates, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!finite_nonneg(skin)) return fail(c, BH_E_INVALID, "skin must be finite and >= 0");
    if (!n_contacts || !n_aggregates) return fail(c, BH_E_INVALID, "NULL count outputs");
    if (n > 0 && (!radius || !label)) return fail(c, BH_E_INVALID, "NULL radius or label");
    if (n > INT32_MAX) return fail(c, BH_E_CAPACITY, "labels are int32");
    *n_contacts = 0;
    *n_aggregates = 0;
    if (n == 0) return BH_OK;
    BHX_HIP(c, bhx::launch_build(c->w, c->stream, single(n), pos, mass, radius, c->cfg.leaf_size,
                                 &c->bucket));
    c->tree_n = n;
    c->tree_eps = true;
    auto *counters = (unsigned long long *)c->diag_out;
    BHX_HIP(c, bhx::launch_contacts(c->w, c->stream, radius, n, skin, label,
                                    (int32_t *)c->w.scratch, counters));
    unsigned long long h[2];
    BHX_HIP(c, hipMemcpyAsync(h, counters, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    *n_contacts = (int64_t)h[0];
    *n_aggregates = (int64_t)h[1];
    return bh_sync(c);
}

bh_status bh_batched_accel(bh_ctx *c, int32_t n_scenes, const int64_t *offsets, const double *pos,
                           const double *mass, double softening, const double *eps, double theta,
                           double *acc, double *phi)
{
    if (!c) return BH_E_INVALID;
    bh_status s = set_layout(c, n_scenes, offsets);
    if (s) return s;
    const int64_t n = c->batch.n;
    s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!finite_nonneg(theta)) return fail(c, BH_E_INVALID, "theta must be finite and >= 0");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (!acc) return fail(c, BH_E_INVALID, "NULL acc");
    return force_tree(c, c->batch, pos, mass, softening, eps, theta, acc, phi);
}

bh_status bh_batched_step(bh_ctx *c, int32_t n_scenes, const int64_t *offsets, double *pos,
                          double *vel, const double *mass, double softening, const double *eps,
                          double theta, double dt, int32_t nsteps, double *acc)
{
    if (!c) return BH_E_INVALID;
    bh_status s = set_layout(c, n_scenes, offsets);
    if (s) return s;
    const int64_t n = c->batch.n;
    s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!finite_nonneg(theta)) return fail(c, BH_E_INVALID, "theta must be finite and >= 0");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (!std::isfinite(dt)) return fail(c, BH_E_INVALID, "dt not finite");
    if (nsteps < 0) return fail(c, BH_E_INVALID, "nsteps < 0");
    if (!vel || !acc) return fail(c, BH_E_INVALID, "NULL vel or acc");
    return run_steps(c, c->batch, pos, vel, mass, softening, eps, theta, dt, nsteps, acc);
}

bh_status bh_accel_vjp(bh_ctx *c, const double *pos, const double *mass, double softening,
                       const double *eps, double theta, const double *lambda, double *g_pos,
                       double *g_mass, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!(c->cfg.flags & BH_FLAG_ADJOINT))
        return fail(c, BH_E_STATE, "the context was created without BH_FLAG_ADJOINT");
    if ((c->cfg.flags & BH_FLAG_QUAD) && theta >= 0.0)
        return fail(c, BH_E_STATE, "no VJP of the quadrupole walk (BH_FLAG_QUAD)");
    if (std::isnan(theta) || std::isinf(theta)) return fail(c, BH_E_INVALID, "theta not finite");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (n > 0 && (!lambda || !g_pos || !g_mass))
        return fail(c, BH_E_INVALID, "NULL lambda, g_pos or g_mass");
    return vjp(c, pos, mass, softening, eps, theta, lambda, g_pos, g_mass, n);
}

bh_status bh_leapfrog_vjp(bh_ctx *c, const double *pos, const double *vel, const double *acc,
                          const double *mass, double softening, const double *eps, double theta,
                          double dt, int32_t nsteps, double *traj, double *xbar, double *vbar,
                          double *abar, double *g_mass, int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    s = check_vjp_args(c, softening, theta, dt, nsteps);
    if (s) return s;
    if (n > 0 && (!vel || !acc || !xbar || !vbar || !abar || !g_mass || (nsteps > 0 && !traj)))
        return fail(c, BH_E_INVALID, "NULL vel, acc, traj, xbar, vbar, abar or g_mass");
    if (n == 0 || nsteps == 0) return BH_OK;
    const int64_t n3 = 3 * n;
    bhx::AdjointWork &aw = c->aw;
    // the tree of each recomputed step is kept for the VJP at the same
    // positions when there is room (same build, so the same tree)
    const bool keep = theta >= 0.0 && ensure_tree_slots(c, nsteps, n);
    // recompute the segment's positions exactly as bh_step_leapfrog does
    BHX_HIP(c, bhx::launch_copy(c->stream, aw.vwork, vel, n3));
    BHX_HIP(c, bhx::launch_copy(c->stream, aw.awork, acc, n3));
    for (int32_t k = 0; k < nsteps; k++) {
        const double *x_in = k == 0 ? pos : traj + (int64_t)(k - 1) * n3;
        double *x_out = traj + (int64_t)k * n3;
        BHX_HIP(c, bhx::launch_kick_drift_to(c->stream, x_in, aw.vwork, aw.awork, x_out, n, dt));
        const Workspace slot = keep ? bhx::slot_view(c->w, aw.trees, k) : c->w;
        s = theta >= 0.0 ? force_tree(c, single(n), x_out, mass, softening, eps, theta, aw.awork,
                                      nullptr, keep ? &slot : nullptr)
                         : force_direct(c, x_out, mass, softening, eps, aw.awork, nullptr, n,
                                        c->cfg.precision);
        if (s) return s;
        BHX_HIP(c, bhx::launch_kick(c->stream, aw.vwork, aw.awork, n, dt));
    }
    s = reverse_sweep(c, traj, mass, softening, eps, theta, dt, nsteps, xbar, vbar, abar, g_mass,
                      n, keep);
    if (s) return s;
    // bad input found by the slot builds is reported like the context's own
    if (keep)
        BHX_HIP(c, bhx::launch_merge_status(c->stream, aw.trees.hdr, nsteps, &c->w.hdr->status));
    return BH_OK;
}

bh_status bh_leapfrog_vjp_stored(bh_ctx *c, const double *traj, const double *mass,
                                 double softening, const double *eps, double theta, double dt,
                                 int32_t nsteps, double *xbar, double *vbar, double *abar,
                                 double *g_mass, int64_t n)
{
    bh_status s = check_bodies(c, traj, mass, n);
    if (s) return s;
    s = check_vjp_args(c, softening, theta, dt, nsteps);
    if (s) return s;
    if (n > 0 && (!xbar || !vbar || !abar || !g_mass))
        return fail(c, BH_E_INVALID, "NULL xbar, vbar, abar or g_mass");
    if (n == 0 || nsteps == 0) return BH_OK;
    return reverse_sweep(c, traj, mass, softening, eps, theta, dt, nsteps, xbar, vbar, abar,
                         g_mass, n);
}

bh_status bh_walk_counts(bh_ctx *c, int32_t *counts, int64_t n)
{
    if (!c) return BH_E_INVALID;
    if (!(c->cfg.flags & BH_FLAG_COUNTS) || c->walk_n < 0)
        return fail(c, BH_E_STATE, "no walk counts (BH_FLAG_COUNTS unset or no tree walk yet)");
    if (n != c->walk_n) return fail(c, BH_E_INVALID, "n differs from the last walk");
    if (n > 0 && !counts) return fail(c, BH_E_INVALID, "NULL counts");
    if (n > 0)
        BHX_HIP(c, hipMemcpyAsync(counts, c->w.counts, (size_t)n * 2 * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, c->stream));
    return BH_OK;
}

bh_status bh_tree_export(bh_ctx *c, bh_tree_view *out)
{
    if (!c || !out) return BH_E_INVALID;
    if (c->tree_n < 0) return fail(c, BH_E_STATE, "no tree has been built");
    bhx::TreeHeader h;
    bhx::SceneBox b;
    BHX_HIP(c, hipMemcpyAsync(&h, c->w.hdr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    BHX_HIP(c, hipMemcpyAsync(&b, c->w.box, sizeof(b), hipMemcpyDeviceToHost, c->stream));
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    int64_t nn = 0;
    int depth = 0;
    for (int l = 0; l < bhx::kLevels; l++) {
        int64_t cnt = h.level_count[l];
        if (cnt > c->w.node_cap - nn) cnt = c->w.node_cap - nn;
        nn += cnt;
        if (cnt > 0) depth = l;
    }
    std::memset(out, 0, sizeof(*out));
    out->n = c->tree_n;
    out->nnodes = nn;
    out->depth = depth;
    out->info = (const int32_t *)c->w.ninfo;
    out->mom = (const double *)c->w.nmom;
    out->eps2 = c->tree_eps ? c->w.neps2 : nullptr;
    out->quad = c->w.nquad;
    out->order = c->w.idx[0];
    out->keys = c->w.keys[0];
    for (int a = 0; a < 3; a++) {
        out->box[a] = b.lo[a];
        out->box[3 + a] = b.x0[a];
    }
    out->box[6] = b.L;
    out->box[7] = b.S;
    return BH_OK;
}

bh_status bh_stats(bh_ctx *c, bh_stats_t *out)
{
    if (!c || !out) return BH_E_INVALID;
    bh_tree_view v;
    bh_status s = bh_tree_export(c, &v);
    if (s) return s;
    std::memset(out, 0, sizeof(*out));
    out->nnodes = v.nnodes;
    out->depth = v.depth;
    out->bucket_sort = c->bucket ? 1 : 0;
    if (c->walk_n > 0) {
        std::vector<int32_t> h((size_t)c->walk_n * 2);
        BHX_HIP(c, hipMemcpyAsync(h.data(), c->w.counts, h.size() * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, c->stream));
        BHX_HIP(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < h.size(); i += 2) {
            out->total_nodes_accepted += h[i];
            out->total_leaf_pairs += h[i + 1];
        }
    }
    s = fold_timing(c);
    if (s) return s;
    out->timed_evals = c->timed_evals;
    out->build_ms = c->build_ms;
    out->walk_ms = c->walk_ms;
    return BH_OK;
}

bh_status bh_timing_reset(bh_ctx *c)
{
    if (!c) return BH_E_INVALID;
    bh_status s = fold_timing(c);
    if (s) return s;
    c->timed_evals = 0;
    c->build_ms = c->walk_ms = 0.0;
    return BH_OK;
}

bh_status bh_gravity_dt_bound(bh_ctx *c, const double *mass, const double *radius, int64_t n,
                              double *dt_out)
{
    if (!c) return BH_E_INVALID;
    if (!dt_out) return fail(c, BH_E_INVALID, "NULL dt_out");
    if (n < 0) return fail(c, BH_E_INVALID, "n < 0");
    if (n > 0 && (!mass || !radius)) return fail(c, BH_E_INVALID, "NULL mass or radius with n > 0");
    if (!(c->cfg.G > 0.0)) return fail(c, BH_E_INVALID, "the context's G must be positive");
    auto *work = (long long *)c->diag_out;
    double *out = c->diag_out + 1;
    BHX_HIP(c, bhx::launch_dt_bound(c->stream, mass, radius, n, c->cfg.G, work, out,
                                    &c->w.hdr->status));
    double dt = 0.0;
    BHX_HIP(c, hipMemcpyAsync(&dt, out, sizeof(dt), hipMemcpyDeviceToHost, c->stream));
    bh_status st = bh_sync(c);
    if (st) return st;
    *dt_out = dt;
    return BH_OK;
}

bh_status bh_diagnostics(bh_ctx *c, const double *pos, const double *vel, const double *mass,
                         double softening, const double *eps, double out[8], int64_t n)
{
    bh_status s = check_bodies(c, pos, mass, n);
    if (s) return s;
    if (!out) return fail(c, BH_E_INVALID, "NULL out");
    if (!finite_nonneg(softening)) return fail(c, BH_E_INVALID, "softening must be finite and >= 0");
    if (n > 0 && !vel) return fail(c, BH_E_INVALID, "NULL vel");
    for (int k = 0; k < 8; k++) out[k] = 0.0;
    if (n == 0) return BH_OK;
    double *acc_tmp = c->w.scratch, *phi = c->w.scratch + 3 * n;
    s = force_direct(c, pos, mass, softening, eps, acc_tmp, phi, n, BH_FP64);
    if (s) return s;
    BHX_HIP(c, bhx::launch_diag_reduce(c->stream, pos, vel, mass, phi, n, c->w.red_part,
                                       c->diag_out));
    BHX_HIP(c, hipMemcpyAsync(out, c->diag_out, 8 * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    BHX_HIP(c, hipStreamSynchronize(c->stream));
    return BH_OK;
}

}  // extern "C"
