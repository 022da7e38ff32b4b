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

/* Kick-drift-kick leapfrog, nsteps steps of dt. acc holds the acceleration at
 * the input positions and is updated in place. theta < 0 selects the direct
 * sum, otherwise a Barnes-Hut tree with the given leaf size is rebuilt every
 * step. */
int orc_leapfrog(int64_t n, double *pos, double *vel, const double *mass,
                 const double *eps, double eps0, double G, double theta, int32_t leaf,
                 double dt, int32_t nsteps, double *acc);

/* out[0] kinetic energy, out[1] potential energy 1/2 sum m phi (direct sum),
 * out[2..4] linear momentum, out[5..7] angular momentum about the origin. */
int orc_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass,
                    const double *eps, double eps0, double G, double out[8]);

/* Number of OpenMP threads the oracle uses. */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
