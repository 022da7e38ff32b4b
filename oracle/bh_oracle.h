/*
 * bh_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU oracle for the gravity hot path of
 * Ferrari, Lavagna & Blazquez, "A parallel-GPU code for asteroid aggregation
 * problems with angular particles" (MNRAS 2020), Section "Gravitational
 * dynamics". Only tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the GPU library never does, and the two share no code.
 *
 * Conventions (all arrays are host memory owned by the caller):
 *   pos, vel, acc : n x 3 row-major float64
 *   mass          : n float64, must be >= 0
 *   eps           : n float64 per-body softening lengths, or NULL for the
 *                   uniform softening length eps0
 *   targets       : optional list of nt body indices to evaluate (NULL = all n,
 *                   then nt must equal n); outputs are indexed 0..nt-1
 * Return codes: 0 ok, 1 invalid argument, 2 non-finite input, 3 negative
 * mass, 4 out of memory.
 */
#ifndef BH_ORACLE_H
#define BH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVEL 21

typedef struct orc_tree orc_tree;

/* Direct N^2 sum, eq. (Newton) with Plummer softening, eq. (Force_rComp). */
int orc_direct(int64_t n, const double *pos, const double *mass, const double *eps,
               double eps0, double G, const int64_t *targets, int64_t nt,
               double *acc, double *phi, double *absacc);

/* Octree over all n bodies: root cube, recursive octant subdivision down to
 * buckets of at most `leaf` bodies (or level 21), moments bottom-up by
 * eq. (COMinternal). Returns NULL and sets *err on failure. */
orc_tree *orc_tree_build(int64_t n, const double *pos, const double *mass,
                         const double *eps, int32_t leaf, int *err);
void orc_tree_free(orc_tree *t);
int64_t orc_tree_nnodes(const orc_tree *t);
/* box[0..2] = per-axis minimum, box[3..5] = cube corner x0, box[6] = side L,
 * box[7] = quantisation scale S = 2^21 / L */
void orc_tree_box(const orc_tree *t, double box[8]);
/* Copies the node table (any pointer may be NULL to skip it). com is nn x 3.
 * order[k] is the body at segment position k; q is n x 3 integer coords. */
void orc_tree_export(const orc_tree *t, int32_t *level, int64_t *first, int64_t *count,
                     int64_t *child0, int32_t *nchild, double *nmass, double *com,
                     double *eps2, int64_t *order, uint32_t *q);

/* Barnes-Hut accelerations by a per-body depth-first walk of the tree, using
 * the opening rule of eq. (accuracy) and the terms of eqs. (Force_leaf),
 * (Force_thetaTrue), (Force_rComp). counts (nt x 2, may be NULL) receives the
 * number of accepted internal nodes and of leaf body pairs per target. */
int orc_tree_accel(const orc_tree *t, const double *pos, const double *mass,
                   const double *eps, double eps0, double G, double theta,
                   const int64_t *targets, int64_t nt, double *acc, double *phi,
                   double *absacc, int64_t *counts);

/* Traceless quadrupole moments of every node, Q = sum m (3 d d^T - |d|^2 I)
 * about the node's centre of mass (an optional refinement beyond the paper's
 * monopole nodes), computed from the definition over each node's bodies. */
int orc_tree_quadrupoles(orc_tree *t, const double *pos, const double *mass);

/* Copies the quadrupoles (nnodes x 6) in node order; needs orc_tree_quadrupoles. */
int orc_tree_quad_export(const orc_tree *t, double *out);

/* orc_tree_accel with, when quad != 0, each accepted node's quadrupole term
 * added (orc_tree_quadrupoles must have run). Leaf pairs are unchanged. */
int orc_tree_accel_q(const orc_tree *t, const double *pos, const double *mass,
                     const double *eps, double eps0, double G, double theta,
                     const int64_t *targets, int64_t nt, double *acc, double *phi,
                     double *absacc, int64_t *counts, int quad);

/* Kick-drift-kick leapfrog, nsteps steps of dt. acc holds the acceleration at
 * the input positions and is updated in place. theta < 0 selects the direct
 * sum, otherwise a Barnes-Hut tree with the given leaf size is rebuilt every
 * step. */
int orc_leapfrog(int64_t n, double *pos, double *vel, const double *mass,
                 const double *eps, double eps0, double G, double theta, int32_t leaf,
                 double dt, int32_t nsteps, double *acc);

/* Semi-implicit (symplectic) Euler, the paper's preferred stepper (Section
 * "Numerical solvers"), with the two-rate scheme of Section "The asteroid
 * aggregation problem": every substep of dt kicks v += dt a then drifts
 * x += dt v; gravity is evaluated (a = A(x)) only after every `every`-th
 * substep and held constant in between. acc holds the acceleration of the
 * last evaluation and is updated in place; theta < 0 selects the direct sum. */
int orc_euler(int64_t n, double *pos, double *vel, const double *mass, const double *eps,
              double eps0, double G, double theta, int32_t leaf, double dt, int32_t nsteps,
              int32_t every, double *acc);

/* Aggregate identification (Section "Post-processing: aggregate
 * identification"): bodies are the vertices of a graph whose edges are the
 * contacts; aggregates are its connected components with more than one body.
 * A contact here is two spheres of radii r_i, r_j closer than
 * r_i + r_j + skin: |x_i - x_j|^2 <= (r_i + r_j + skin)^2 in FP64 as written.
 * label[i] = smallest body index of i's component; *n_contacts = number of
 * contact pairs; *n_aggregates = components with more than one body. All
 * pairs are tested. */
int orc_contact_components(int64_t n, const double *pos, const double *radius, double skin,
                           int32_t *label, int64_t *n_contacts, int64_t *n_aggregates);

/* Largest gravity time step of eq. (dt_g), 1 / (2 sqrt(G rho_max)), with
 * rho_max the largest density m_i / ((4/3) pi r_i^3) over the massive bodies
 * (+inf when none is massive, 0 when a massive body has radius 0). */
int orc_gravity_dt_bound(int64_t n, const double *mass, const double *radius, double G,
                         double *dt);

/* out[0] kinetic energy, out[1] potential energy 1/2 sum m phi (direct sum),
 * out[2..4] linear momentum, out[5..7] angular momentum about the origin. */
int orc_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass,
                    const double *eps, double eps0, double G, double out[8]);

/* Vector-Jacobian products of the force map, with the tree and every opening
 * decision held fixed (they are piecewise constant in the inputs). For an
 * upstream lambda (nt x 3, one row per body), ADDS to g_pos (n x 3) and
 * g_mass (n) the gradient of sum_i lambda_i . a_i. The direct form sums all
 * pairs; the tree form walks the same interaction lists as orc_tree_accel and
 * carries node adjoints to the node's members through the centre of mass,
 * the node mass and the mass-weighted softening. Single-threaded. */
int orc_direct_vjp(int64_t n, const double *pos, const double *mass, const double *eps,
                   double eps0, double G, const double *lambda, double *g_pos, double *g_mass);
int orc_tree_vjp(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                 double eps0, double G, double theta, const double *lambda, double *g_pos,
                 double *g_mass);

/* Error scale of orc_tree_vjp: the same walk and node hand-down, with every
 * contribution replaced by the magnitudes of its parts (G m_s (|l_a| / r^3 +
 * 3 |d_a| sum_b |l_b||d_b| / r^5) for positions, G sum_b |l_b||d_b| / r^3 and
 * 3/2 G m_s sum_b |l_b||d_b| / r^5 for mass and softening, and the absolute
 * values of the hand-down factors) and all of them added. Each output bounds
 * the absolute value of orc_tree_vjp's and is what the rounding of a
 * different evaluation order or precision is relative to. ADDS like
 * orc_tree_vjp. */
int orc_tree_vjp_abs(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                     double eps0, double G, double theta, const double *lambda, double *g_pos,
                     double *g_mass);

/* Gradient of a scalar loss through nsteps kick-drift-kick steps that start
 * from (pos0, vel0) with a0 = A(pos0): given xbar, vbar = dL/dx_T, dL/dv_T,
 * writes gx0 = dL/dx0, gv0 = dL/dv0 and gm = dL/dm (all decisions of every
 * tree fixed). Reverse mode over the stored trajectory. */
int orc_rollout_grad(int64_t n, const double *pos0, const double *vel0, const double *mass,
                     const double *eps, double eps0, double G, double theta, int32_t leaf,
                     double dt, int32_t nsteps, const double *xbar, const double *vbar,
                     double *gx0, double *gv0, double *gm);

/* Number of OpenMP threads the oracle uses. */
int orc_num_threads(void);
/* Sets the number of OpenMP threads for the oracle's later calls (k >= 1). */
void orc_set_num_threads(int k);

#ifdef __cplusplus
}
#endif
#endif
