/*
 * bhx.h -- C ABI of the MI355X Barnes-Hut / direct-sum self-gravity library.
 *
 * What is computed follows Ferrari, Lavagna & Blazquez, "A parallel-GPU code
 * for asteroid aggregation problems with angular particles" (MNRAS 2020),
 * Section "Gravitational dynamics":
 *   - the direct N^2 sum of eq. (Newton), every term softened as in
 *     eq. (Force_rComp): a_i = G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps_ij^2)^(3/2),
 *     d_ij = x_j - x_i;
 *   - an octree rebuilt on every call (subsection "Hierarchical treecode
 *     algorithm"): a root cube around the bounding box, split homogeneously
 *     into octants until a cell holds at most `leaf_size` bodies (or is 21
 *     levels deep), with node mass and centre of mass from eq. (COMinternal);
 *   - a per-body walk from the root (subsection "Force computation"): a leaf
 *     adds its bodies one by one (eq. Force_leaf), an internal node of side s
 *     at distance D = |COM - x_B| is accepted as one mass at its centre of mass
 *     when s^2 < theta^2 D^2 (eqs. accuracy, Force_thetaTrue), otherwise all of
 *     its children are visited;
 *   - a kick-drift-kick leapfrog (Section "Numerical solvers" lists leapfrog
 *     among the symplectic steppers).
 * Outputs are accelerations (force / m_B). With per-body softening lengths
 * eps_i the pair softening is eps_ij^2 = (eps_i^2 + eps_j^2) / 2 and a node
 * term uses (eps_B^2 + <eps^2>_N) / 2, <eps^2>_N mass-weighted over the node.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller.
 *   pos, vel, acc : n x 3 row-major float64 (x0 y0 z0 x1 y1 z1 ...)
 *   mass          : n float64, >= 0
 *   eps           : n float64 per-body softening lengths, or NULL to use the
 *                   scalar `softening` for every term
 *   phi           : n float64 potential (-G sum m_j / r), or NULL
 * Outputs are written in the caller's body order.
 *
 * Execution: all compute calls are asynchronous on the context's HIP stream
 * and return after enqueueing. Host-detectable argument errors return at once
 * with nothing enqueued. Errors found on the device (non-finite input,
 * negative mass, node table overflow) are latched in the
 * context and returned by the next bh_sync(); outputs of a failed call are
 * undefined. A context is not thread-safe; use one per stream.
 */
#ifndef BHX_H
#define BHX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bh_ctx bh_ctx;

typedef enum {
    BH_OK = 0,
    BH_E_INVALID = 1,   /* bad argument, found on the host; nothing enqueued */
    BH_E_NONFINITE = 2, /* device found a NaN/Inf position, mass or softening, or a negative mass */
    BH_E_CAPACITY = 3,  /* n > n_max, or the node table overflowed */
    BH_E_OOM = 4,       /* device allocation failed */
    BH_E_HIP = 5,       /* a HIP runtime call failed; see bh_last_error() */
    BH_E_STACK = 6,     /* reserved: an unknown device status; the walk's traversal stack is
                           sized so that trees of at most 21 levels cannot overflow it */
    BH_E_STATE = 7,     /* call out of order, e.g. bh_tree_export() before any build */
    BH_E_CHECK = 8      /* only from libbhx_checked.so (the same library with device-side
                           invariant checks): a check failed (bh_last_error names it) */
} bh_status;

/* precision of the pairwise terms */
enum { BH_FP64 = 0, BH_FP32C = 1 };

/* bh_config.flags */
enum {
    BH_FLAG_COUNTS = 1u, /* keep per-body walk counts for bh_walk_counts() */
    BH_FLAG_TIMING = 2u, /* record HIP events around every tree build and walk
                            on the context's stream; totals in bh_stats() */
    BH_FLAG_ADJOINT = 4u, /* allocate the workspace of bh_accel_vjp and
                             bh_leapfrog_vjp at creation */
    BH_FLAG_GRAPH = 8u,   /* bh_step_leapfrog and bh_batched_step capture one
                             step in a HIP graph (once per set of arguments)
                             and replay it nsteps times on a stream of the
                             context, ordered after and before the caller's
                             stream by events */
    BH_FLAG_QUAD = 16u,   /* beyond the paper's monopole nodes: keep each node's
                             traceless quadrupole Q = sum m (3 d d^T - |d|^2 I)
                             about its centre of mass, and add to every accepted
                             node's term G (-Q d / r^5 + 5/2 (d.Q d) d / r^7),
                             d = COM - x_B, r^2 = |d|^2 + eps^2 (potential
                             -G (d.Q d) / (2 r^5)). Leaf pairs and opening
                             decisions are unchanged. The force VJPs do not
                             support it (BH_E_STATE). */
    BH_FLAG_MARKERS = 32u /* push roctx ranges ("bhx build", "bhx walk", "bhx
                             direct", "bhx vjp", "bhx step", "bhx step
                             (graph)") around the host-side enqueueing of each
                             phase, for profiler timelines (rocprofv3
                             --marker-trace); the roctx library is loaded at
                             bh_create and the flag does nothing when it is
                             absent */
};

typedef struct {
    int64_t n_max;     /* largest n any call will pass; workspace is sized for it */
    int32_t leaf_size; /* bucket size: a cell with more bodies is split; 1..64 */
    int32_t precision; /* BH_FP64: all FP64. BH_FP32C: each pair offset is
                          formed in FP64 and rounded once to FP32, the rest of
                          the pair term is FP32, and FP32 partial sums are
                          flushed to FP64 accumulators; FP64 positions, opening
                          test, moments and outputs */
    double G;          /* gravitational constant */
    uint32_t flags;    /* BH_FLAG_* */
    int32_t walk_group; /* target bodies served by one wavefront in the tree
                           walk: 64, 32 or 16 (64/walk_group lanes per body);
                           0 = the library's default (forces: 16 for calls
                           on fewer than 2^17 bodies, else 64; force VJPs: 16
                           below 2^15, 32 below 2^19, else 64). Results do not
                           depend on it beyond rounding. */
    int32_t max_scenes; /* largest n_scenes of bh_batched_*; 0 means 1 */
} bh_config;

/* Creates a context on the current HIP device, bound to `hip_stream`
 * (a hipStream_t; NULL = the null stream). Allocates the whole workspace for
 * cfg->n_max bodies, including the worst-case node table, so later calls never
 * allocate. Errors: BH_E_INVALID (NULL pointers, n_max < 0, leaf_size outside
 * 1..64, precision unknown, G not finite, unknown flags, walk_group not in
 * {0, 16, 32, 64}), BH_E_OOM, BH_E_HIP. */
bh_status bh_create(const bh_config *cfg, void *hip_stream, bh_ctx **out);

/* Frees the context and its workspace after waiting for its stream. NULL is a no-op. */
void bh_destroy(bh_ctx *ctx);

/* Rebinds the context to another HIP stream (later calls enqueue there). */
bh_status bh_set_stream(bh_ctx *ctx, void *hip_stream);

/* Waits for the context's stream, then returns and clears the latched device
 * status (BH_OK if every call since the last bh_sync succeeded). */
bh_status bh_sync(bh_ctx *ctx);

/* Text of the last error on this context (never NULL; "" when none). */
const char *bh_last_error(const bh_ctx *ctx);

/* Builds the octree of n bodies (bounding cube, Morton keys, stable radix
 * sort, level-by-level octree, bottom-up moments by eq. COMinternal) and keeps
 * it in the context until the next build. eps may be NULL (uniform softening:
 * node softening moments are not formed). Errors: BH_E_INVALID (n < 0, NULL
 * pointers with n > 0), BH_E_CAPACITY (n > n_max); device: BH_E_NONFINITE. */
bh_status bh_build_tree(bh_ctx *ctx, const double *pos, const double *mass, const double *eps,
                        int64_t n);

/* Barnes-Hut accelerations: builds the tree as bh_build_tree() does, then walks
 * it once per body with opening parameter theta (>= 0; 0 opens every node and
 * gives the direct sum's pair set). softening >= 0 is used when eps == NULL.
 * acc (n x 3) is overwritten; phi may be NULL. Errors: as bh_build_tree, plus
 * BH_E_INVALID for theta or softening negative or not finite, acc == NULL. */
bh_status bh_compute_accel(bh_ctx *ctx, const double *pos, const double *mass, double softening,
                           const double *eps, double theta, double *acc, double *phi, int64_t n);

/* Direct N^2 accelerations (eq. Newton with softening), all pairs j != i.
 * Same arguments and errors as bh_compute_accel without theta. */
bh_status bh_compute_accel_direct(bh_ctx *ctx, const double *pos, const double *mass,
                                  double softening, const double *eps, double *acc, double *phi,
                                  int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the direct
 * sum of bh_compute_accel_direct without a context, computed by the same
 * kernels in `precision` (BH_FP64 or BH_FP32C) with gravitational constant G,
 * on hip_stream (NULL = the default stream), asynchronously. It allocates
 * nothing: when the targets alone give too few blocks to fill the GPU
 * (n < 262144), the split-row partial sums go to a library-owned device array
 * of 2^20 doubles (8 MiB) on each device, reserved with the library's code
 * and held until the process ends. Every call on a device shares that array
 * and keeps the last call's contents, so calls that overlap on one device
 * (different streams, or host threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe. Every partial sum
 * a call reads it has written first, so the array needs no clearing.
 * Arguments and layout as bh_compute_accel_direct (device pointers, outputs
 * in caller order); there is no device-side check of the inputs.
 * Errors (no side effects): BH_E_CAPACITY for n < 0 or n > BH_NOALLOC_MAX_N;
 * BH_E_INVALID for another precision, G not finite, softening negative or not
 * finite, NULL pos, mass or acc with n > 0; BH_E_HIP when the array's device
 * address cannot be obtained or the launch fails. n = 0 is a no-op. */
#define BH_NOALLOC_MAX_N ((int64_t)1 << 30)
bh_status bh_compute_accel_direct_noalloc(void *hip_stream, int32_t precision, double G,
                                          const double *pos, const double *mass, double softening,
                                          const double *eps, double *acc, double *phi, int64_t n);

/* nsteps kick-drift-kick leapfrog steps of dt, in place on pos and vel:
 * v += dt/2 a; x += dt v; a = A(x); v += dt/2 a. `acc` must hold the
 * acceleration at the input positions (e.g. from bh_compute_accel) and is
 * updated, so consecutive calls do one force evaluation per step. theta >= 0
 * selects the tree, theta < 0 the direct sum. With the tree, more than 4096
 * bodies (or several scenes) and nsteps > 1 (or BH_FLAG_GRAPH), the state is
 * kept inside the context between the steps of the call, in the Morton
 * order of each step's sort: pos, vel and acc are read at the start of the
 * call and written at its end. The results equal those of nsteps one-step calls bit
 * for bit unless two bodies share a cell of the finest (2^21) grid, whose
 * order within their leaf may then differ. Errors: as bh_compute_accel, plus
 * BH_E_INVALID for nsteps < 0, dt not finite, vel == NULL. */
bh_status bh_step_leapfrog(bh_ctx *ctx, double *pos, double *vel, const double *mass,
                           double softening, const double *eps, double theta, double dt,
                           int32_t nsteps, double *acc, int64_t n);

/* nsteps semi-implicit (symplectic) Euler substeps of dt, in place, with the
 * two-rate gravity scheme of Section "The asteroid aggregation problem" (the
 * paper prefers this stepper, Section "Numerical solvers"): each substep
 * kicks v += dt a and then drifts x += dt v with the new velocity, and gravity
 * is evaluated (a = A(x), tree for theta >= 0, direct sum otherwise) only after
 * every `every`-th substep of the call, the acceleration being held in
 * between. every = 1 is plain semi-implicit Euler. `acc` holds the
 * acceleration of the last evaluation on entry and on return. Runs eagerly
 * (BH_FLAG_GRAPH does not apply). Errors: as bh_step_leapfrog, plus
 * BH_E_INVALID for every < 1. */
bh_status bh_step_euler(bh_ctx *ctx, double *pos, double *vel, const double *mass,
                        double softening, const double *eps, double theta, double dt,
                        int32_t nsteps, int32_t every, double *acc, int64_t n);

/* Per-body walk counts of the last bh_compute_accel / bh_step_leapfrog force
 * evaluation (tree mode), in caller order: counts[2i] = accepted internal
 * nodes, counts[2i+1] = leaf body pairs. counts is a device pointer to n x 2
 * int32. Needs BH_FLAG_COUNTS at creation (else BH_E_STATE); n must equal the
 * last walk's n (else BH_E_INVALID). */
bh_status bh_walk_counts(bh_ctx *ctx, int32_t *counts, int64_t n);

/* Many independent scenes in one call: n_scenes clouds stored back to back,
 * scene k being bodies offsets[k] .. offsets[k+1]-1 (offsets: HOST array of
 * n_scenes + 1 int64, offsets[0] = 0, every scene non-empty, total <= n_max,
 * n_scenes <= max_scenes). Each scene gets its own root cube and tree and its
 * bodies feel only the bodies of their own scene; one launch of each build and
 * walk kernel serves all scenes. The tables of a layout are uploaded once and
 * reused while the offsets stay the same. bh_batched_accel is
 * bh_compute_accel per scene; bh_batched_step is bh_step_leapfrog per scene
 * (graph-captured with BH_FLAG_GRAPH). Errors: as bh_compute_accel /
 * bh_step_leapfrog, plus BH_E_INVALID for a bad layout. */
bh_status bh_batched_accel(bh_ctx *ctx, int32_t n_scenes, const int64_t *offsets,
                           const double *pos, const double *mass, double softening,
                           const double *eps, double theta, double *acc, double *phi);
bh_status bh_batched_step(bh_ctx *ctx, int32_t n_scenes, const int64_t *offsets, double *pos,
                          double *vel, const double *mass, double softening, const double *eps,
                          double theta, double dt, int32_t nsteps, double *acc);

/* Aggregate identification (Section "Post-processing: aggregate
 * identification"): the graph whose vertices are the bodies and whose edges
 * are their contacts, and its connected components. A contact is two spheres
 * (radius: n float64, >= 0, device) whose centres are within
 * r_i + r_j + skin: |x_i - x_j|^2 <= (r_i + r_j + skin)^2 in FP64 as written.
 * label (n int32, device, caller order) receives for every body the smallest
 * index of its component; *n_contacts the number of contact pairs and
 * *n_aggregates the number of components with more than one body (host
 * outputs). Builds the tree of pos/mass (the build's checks apply to radius as
 * a softening array) and synchronises. Errors: as bh_build_tree, plus
 * BH_E_INVALID for a NULL radius, label or count output, skin negative or not
 * finite; BH_E_CAPACITY for n >= 2^31. */
bh_status bh_contact_components(bh_ctx *ctx, const double *pos, const double *mass,
                                const double *radius, double skin, int32_t *label,
                                int64_t *n_contacts, int64_t *n_aggregates, int64_t n);

/* Autotuner for bh_batched_step: times every bucket size in {4, 8, 16, 32}
 * and walk group size in {16, 32, 64} (other settings from *base) on scratch
 * copies of the given state (the caller's arrays are not modified): one
 * graph-captured warm-up step, then `steps` steps timed with HIP events. Each
 * candidate gets a context of its own, so this call allocates and frees
 * device memory; it synchronises hip_stream first and returns when done.
 * With the BHX_AUTOTUNE_CACHE environment variable naming a file, results
 * are read from and appended to it (JSON lines keyed by the layout, the
 * precision and the physical parameters). out receives the fastest choice
 * and its time per step. Errors: BH_E_INVALID for bad arguments, BH_E_OOM if
 * no candidate fits, or any error of the calls it makes. */
typedef struct {
    int32_t leaf_size, walk_group;
    double ms_per_step;
} bh_tune_result;
bh_status bh_autotune(const bh_config *base, void *hip_stream, int32_t n_scenes,
                      const int64_t *offsets, const double *pos, const double *vel,
                      const double *mass, double softening, const double *eps, double theta,
                      double dt, int32_t steps, bh_tune_result *out);

/* Vector-Jacobian product of the force map: ADDS to g_pos (n x 3) and g_mass
 * (n) the gradient of sum_i lambda_i . a_i with respect to the positions and
 * masses, lambda being n x 3 in caller order. theta >= 0 differentiates the
 * Barnes-Hut map of bh_compute_accel with its tree and every opening decision
 * held fixed (both are piecewise constant in the inputs): a node term passes
 * its adjoint to the node's members through the centre of mass, the node
 * mass and the mass-weighted softening (eq. COMinternal). theta < 0
 * differentiates the direct sum. The tree form is computed in the context's
 * precision: in BH_FP32C each term's offset is the FP64 difference rounded
 * once and the rest of the term is FP32, with FP32 partial sums over at most
 * 8 items added into FP64 sums and adjoints (the error is bounded by a small
 * multiple of 2^-24 times the sum of the terms' absolute values); the direct
 * form is FP64 in either precision. The tree form adds source-side terms with
 * atomics, so its last bits depend on scheduling. Needs BH_FLAG_ADJOINT (else BH_E_STATE). Errors: as
 * bh_compute_accel, plus BH_E_INVALID for NULL lambda, g_pos or g_mass. */
bh_status bh_accel_vjp(bh_ctx *ctx, const double *pos, const double *mass, double softening,
                       const double *eps, double theta, const double *lambda, double *g_pos,
                       double *g_mass, int64_t n);

/* Backward pass over one segment of kick-drift-kick steps, for a gradient
 * through bh_step_leapfrog with checkpointing. The segment starts from pos,
 * vel and acc = A(pos) (the checkpoint, unchanged) and takes nsteps steps of
 * dt; the positions after each step are recomputed into traj (caller-owned,
 * nsteps x n x 3 float64) with the context's precision, exactly as
 * bh_step_leapfrog computes them. On entry xbar, vbar (n x 3) hold the
 * gradient with respect to the segment's final positions and velocities and
 * abar (n x 3) the gradient with respect to its final acceleration; on return
 * they hold the gradient with respect to pos, vel and acc. One
 * bh_accel_vjp-equivalent product is taken per step (at the positions after
 * it) and its mass gradient ADDED to g_mass. The dependence of acc on pos is
 * left to the caller (a bh_accel_vjp at the rollout's first positions with
 * the final abar). With the tree, the context keeps the tree of each
 * recomputed step for the product at the same positions instead of building
 * it again: the first call allocates nsteps slots of about 52 B per body and
 * 56 B per node of the node-table bound when the device has twice that free
 * (else the products rebuild), held until bh_destroy. Needs BH_FLAG_ADJOINT.
 * Errors: as bh_step_leapfrog, plus BH_E_INVALID for NULL traj, xbar, vbar,
 * abar or g_mass. */
bh_status bh_leapfrog_vjp(bh_ctx *ctx, const double *pos, const double *vel, const double *acc,
                          const double *mass, double softening, const double *eps, double theta,
                          double dt, int32_t nsteps, double *traj, double *xbar, double *vbar,
                          double *abar, double *g_mass, int64_t n);

/* The same backward pass over steps whose positions the caller kept, with no
 * recomputation: traj (nsteps x n x 3 float64, caller-owned, unchanged) holds
 * the positions after each of the nsteps steps, in order, as
 * bh_step_leapfrog computed them; xbar, vbar, abar and g_mass as for
 * bh_leapfrog_vjp. A rollout whose positions all fit in device memory (24 B
 * per body and step) then costs one force VJP per step and no force
 * evaluation in its backward pass. Needs BH_FLAG_ADJOINT. Errors: as
 * bh_leapfrog_vjp. */
bh_status bh_leapfrog_vjp_stored(bh_ctx *ctx, const double *traj, const double *mass,
                                 double softening, const double *eps, double theta, double dt,
                                 int32_t nsteps, double *xbar, double *vbar, double *abar,
                                 double *g_mass, int64_t n);

/* Borrowed device view of the tree of the last build, valid until the next
 * build or bh_destroy. Bodies are held in Morton order: order[s] is the caller
 * index of the s-th sorted body and keys[s] its 63-bit Morton key (the three
 * 21-bit integer cell coordinates interleaved, x bit most significant in each
 * triplet). Node k, packed:
 *   info[4k..4k+3] = {first, count, child0, level | (nchild << 8)}: the cell's
 *     bodies are sorted positions first .. first+count-1; child0 is the index
 *     of its first child (children are contiguous, in octant order) or -1 for
 *     a leaf; level is 0..21 and nchild 0..8;
 *   mom[4k..4k+3] = {centre of mass x, y, z, mass};
 *   eps2[k] = <eps^2>_N, or eps2 == NULL when the build had no per-body eps.
 * Node 0 is the root. box = {lo_x, lo_y, lo_z, x0_x, x0_y, x0_z, L, S}: the
 * per-axis minimum, root cube corner, side, and quantisation scale 2^21 / L.
 * nnodes and depth are read back from the device, so this call synchronises
 * the stream. Errors: BH_E_STATE if no tree was built. */
typedef struct {
    int64_t n, nnodes;
    int32_t depth, pad;
    const int32_t *info;
    const double *mom;
    const double *eps2;
    const uint32_t *order;
    const uint64_t *keys;
    double box[8];
    const double *quad; /* quad[6k..6k+5] = node k's (xx, yy, zz, xy, xz, yz)
                           quadrupole, or NULL without BH_FLAG_QUAD */
} bh_tree_view;
bh_status bh_tree_export(bh_ctx *ctx, bh_tree_view *out);

/* Summary (synchronises): node count and depth of the last build, and which
 * sort it used (bucket_sort = 1: two passes on the top 16 key bits, one more
 * on the scene index for a batch, and one block per range of whole buckets,
 * chosen for one scene, or a batch of at most 256 scenes, of more than 4096
 * bodies when the previous build's level-5 nodes held at most 1024 bodies
 * each; 0: eight 8-bit passes, or the one-block build); totals of accepted
 * nodes and leaf pairs over all bodies of the last walk (0 unless
 * BH_FLAG_COUNTS); with BH_FLAG_TIMING, the number of tree force evaluations
 * and the summed device time (ms, HIP events on the context's stream) of their
 * build and walk phases since creation or the last bh_timing_reset(). Both
 * sorts give the same order. */
typedef struct {
    int64_t nnodes;
    int32_t depth;
    int32_t bucket_sort;
    int64_t total_nodes_accepted, total_leaf_pairs;
    int64_t timed_evals;
    double build_ms, walk_ms;
} bh_stats_t;
bh_status bh_stats(bh_ctx *ctx, bh_stats_t *out);

/* Zeroes the BH_FLAG_TIMING totals (synchronises). */
bh_status bh_timing_reset(bh_ctx *ctx);

/* Largest gravity time step allowed by eq. (dt_g) (Section "The asteroid
 * aggregation problem", "Gravitational dynamics"): Delta t_g < T_g / 2 =
 * 1 / (2 sqrt(G rho)), rho the material density of the bodies and G the
 * context's. Bodies of different densities are bounded by the densest one,
 * rho_i = mass_i / ((4/3) pi radius_i^3) (mass, radius: n float64 device
 * arrays, radius >= 0; massless bodies are skipped). *dt_out (host) receives
 * the bound: +inf when no body is massive, 0 when a massive body has radius 0.
 * Synchronises. Errors: BH_E_INVALID (NULL dt_out, n < 0, NULL arrays with
 * n > 0, G <= 0); device: BH_E_NONFINITE (a non-finite or negative mass or
 * radius). */
bh_status bh_gravity_dt_bound(bh_ctx *ctx, const double *mass, const double *radius, int64_t n,
                              double *dt_out);

/* Energy and momenta of a state, by compensated FP64 reductions on the device:
 * out (host, 8 doubles) = {E_kin, E_pot, Px, Py, Pz, Lx, Ly, Lz}, with
 * E_pot = 1/2 sum m_i phi_i from the direct sum and L about the origin.
 * Synchronises. Errors: as bh_compute_accel_direct. */
bh_status bh_diagnostics(bh_ctx *ctx, const double *pos, const double *vel, const double *mass,
                         double softening, const double *eps, double out[8], int64_t n);

/* Measured vector FMA rate of the current device: the achievable ceiling
 * reported beside the datasheet peak for the walk and the direct sum, which
 * are bound by plain VALU arithmetic. One launch of 8 wavefronts per SIMD on
 * every compute unit; each lane runs 8 independent fused multiply-add chains
 * of `iters` steps, in FP32 (precision BH_FP32C; non-packed instructions, as
 * the library's kernels use) or FP64 (BH_FP64). *tflops (host) receives
 * 2 x FMAs / device time of that launch (HIP events on hip_stream, NULL = the
 * default stream), timed after one shorter untimed launch. Allocates and frees
 * its own output (4 or 8 bytes per thread); synchronises. Errors: BH_E_INVALID
 * for a NULL tflops, iters outside [1, 2^24] (a launch of at most about 2 s)
 * or another precision; BH_E_OOM;
 * BH_E_HIP. */
bh_status bh_probe_fma(void *hip_stream, int32_t precision, int64_t iters, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* BHX_H */
