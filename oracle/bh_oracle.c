/*
 * bh_oracle.c -- TEST INFRASTRUCTURE ONLY (see bh_oracle.h).
 *
 * Plain FP64 C, compiled with -ffp-contract=off so every product and sum is
 * rounded as written. Nothing here is blocked, fused or reordered beyond what
 * the definitions below state; OpenMP only splits the independent targets.
 *
 * What is computed, and where it comes from in Ferrari, Lavagna & Blazquez
 * (MNRAS 2020), Section "Gravitational dynamics":
 *   - direct sum: eq. (Newton), with every term softened as in
 *     eq. (Force_rComp) (r^2 = |d|^2 + eps^2);
 *   - octree: cubes split homogeneously along the three axes, recursively,
 *     until a node holds few enough bodies (subsection "Hierarchical treecode
 *     algorithm"); node mass and centre of mass bottom-up by eq. (COMinternal);
 *   - walk: for each body from the root down, a leaf contributes body-to-body
 *     terms (eq. Force_leaf); an internal node whose ratio size/distance is
 *     below theta contributes its monopole (eqs. accuracy, Force_thetaTrue);
 *     otherwise all children are visited (subsection "Force computation").
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - the root is the cube of side L = largest bounding-box extent, centred
 *     on the box (L = 0 -> 1);
 *   - cells are defined on a 2^21 integer grid: q = clamp(floor((x - x0) * S),
 *     0, 2^21 - 1) with S = 2^21 / L; the cell of a body at level l is the top
 *     l bits of its three integer coordinates; level 21 cells are leaves;
 *   - a cell is split while it holds more than `leaf` bodies (the paper's
 *     leaves hold one body, i.e. leaf = 1); empty octants are not created;
 *   - "Radius of N" is the cell side s = L / 2^l and the distance is the
 *     unsoftened |COM_N - x_B|; a node is accepted iff s^2 < theta^2 D^2
 *     (a tie opens it);
 *   - a leaf is always summed body by body, skipping the body itself;
 *   - per-body softening: eps_ij^2 = (eps_i^2 + eps_j^2) / 2 for body pairs,
 *     (eps_B^2 + <eps^2>_N) / 2 for node terms, <eps^2>_N mass-weighted;
 *   - a term with r^2 = 0 contributes nothing;
 *   - a node with zero mass has its centre of mass at the cell centre;
 *   - the result is the acceleration F / m_B.
 */
#include "bh_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 2097151u /* 2^21 - 1 */

struct orc_tree {
    int64_t n;
    int32_t leaf;
    int has_eps;
    double lo[3], hi[3], L, x0[3], S;
    uint32_t *q;    /* n x 3 */
    int64_t *order; /* segment position -> body */
    int64_t nn, cap;
    int32_t *level;
    int64_t *first, *count, *child0;
    int32_t *nchild;
    double *m, *com, *eps2;
    double *quad; /* nn x 6 traceless quadrupoles, after orc_tree_quadrupoles */
};

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

static int check_bodies(int64_t n, const double *pos, const double *mass, const double *eps,
                        double eps0)
{
    if (n < 0) return 1;
    if (n > 0 && (!pos || !mass)) return 1;
    if (!eps && !(eps0 >= 0.0 && isfinite(eps0))) return 1;
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(pos[3 * i]) || !isfinite(pos[3 * i + 1]) || !isfinite(pos[3 * i + 2]))
            return 2;
        if (!isfinite(mass[i])) return 2;
        if (mass[i] < 0.0) return 3;
        if (eps && !(eps[i] >= 0.0 && isfinite(eps[i]))) return 1;
    }
    return 0;
}

/* A term contributes only when its squared softened distance is a positive
 * normal double. r^2 = 0 is two coincident unsoftened bodies (eq. Force_rComp
 * exists to keep such forces finite); a subnormal r^2 (|d| below 1.5e-154 with
 * no softening) is the same coincidence below the double range, where
 * 1 / r^3 is not representable; both are read as contributing nothing. */
static int term_counts(double r2) { return r2 >= DBL_MIN; }

/* One softened term from a source of mass gm/G at offset d from the target.
 * Adds G m d / r^3 to acc, -G m / r to *phi and G m |d| / r^3 to *aabs. */
static void add_term(double dx, double dy, double dz, double e2, double gm, double *acc,
                     double *phi, double *aabs)
{
    double d2 = dx * dx + dy * dy + dz * dz;
    double r2 = d2 + e2;
    if (!term_counts(r2)) return;
    double r = sqrt(r2);
    double inv3 = 1.0 / (r2 * r);
    acc[0] += gm * dx * inv3;
    acc[1] += gm * dy * inv3;
    acc[2] += gm * dz * inv3;
    *phi -= gm / r;
    *aabs += gm * sqrt(d2) * inv3;
}

/* ------------------------------------------------------------------ direct */

int orc_direct(int64_t n, const double *pos, const double *mass, const double *eps,
               double eps0, double G, const int64_t *targets, int64_t nt, double *acc,
               double *phi, double *absacc)
{
    int rc = check_bodies(n, pos, mass, eps, eps0);
    if (rc) return rc;
    if (!targets && nt != n) return 1;
    if (nt < 0 || (nt > 0 && !acc)) return 1;
    if (targets)
        for (int64_t t = 0; t < nt; t++)
            if (targets[t] < 0 || targets[t] >= n) return 1;
    double e02 = eps0 * eps0;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = targets ? targets[t] : t;
        double a[3] = {0.0, 0.0, 0.0}, p = 0.0, aa = 0.0;
        double ei2 = eps ? eps[i] * eps[i] : 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue; /* j != i in eq. (Newton) */
            double e2 = eps ? 0.5 * (ei2 + eps[j] * eps[j]) : e02;
            add_term(pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                     pos[3 * j + 2] - pos[3 * i + 2], e2, G * mass[j], a, &p, &aa);
        }
        acc[3 * t] = a[0];
        acc[3 * t + 1] = a[1];
        acc[3 * t + 2] = a[2];
        if (phi) phi[t] = p;
        if (absacc) absacc[t] = aa;
    }
    return 0;
}

/* -------------------------------------------------------------------- tree */

static int grow(orc_tree *t, int64_t need)
{
    if (need <= t->cap) return 0;
    int64_t cap = t->cap ? t->cap : 64;
    while (cap < need) cap *= 2;
#define GROW(p, T)                                        \
    do {                                                  \
        void *np_ = realloc(t->p, (size_t)cap * sizeof(T)); \
        if (!np_) return 4;                               \
        t->p = (T *)np_;                                  \
    } while (0)
    GROW(level, int32_t);
    GROW(first, int64_t);
    GROW(count, int64_t);
    GROW(child0, int64_t);
    GROW(nchild, int32_t);
    GROW(m, double);
    GROW(eps2, double);
#undef GROW
    void *c = realloc(t->com, (size_t)cap * 3 * sizeof(double));
    if (!c) return 4;
    t->com = (double *)c;
    t->cap = cap;
    return 0;
}

static int octant_of(const uint32_t *q, int shift)
{
    return (int)((((q[0] >> shift) & 1u) << 2) | (((q[1] >> shift) & 1u) << 1) |
                 ((q[2] >> shift) & 1u));
}

/* Moments of one node (eq. COMinternal). A leaf sums its own bodies; an
 * internal node combines its children's mass and centre of mass. */
static void node_moments(orc_tree *t, int64_t k, const double *pos, const double *mass,
                         const double *eps)
{
    double ms = 0.0, mx = 0.0, my = 0.0, mz = 0.0, me = 0.0;
    if (t->nchild[k] == 0) {
        for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; s++) {
            int64_t b = t->order[s];
            ms += mass[b];
            mx += pos[3 * b] * mass[b];
            my += pos[3 * b + 1] * mass[b];
            mz += pos[3 * b + 2] * mass[b];
            if (eps) me += eps[b] * eps[b] * mass[b];
        }
    } else {
        for (int64_t c = t->child0[k]; c < t->child0[k] + t->nchild[k]; c++) {
            ms += t->m[c];
            mx += t->com[3 * c] * t->m[c];
            my += t->com[3 * c + 1] * t->m[c];
            mz += t->com[3 * c + 2] * t->m[c];
            me += t->eps2[c] * t->m[c];
        }
    }
    t->m[k] = ms;
    if (ms > 0.0) {
        t->com[3 * k] = mx / ms;
        t->com[3 * k + 1] = my / ms;
        t->com[3 * k + 2] = mz / ms;
        t->eps2[k] = eps ? me / ms : 0.0;
    } else {
        /* massless node: centre of its cell */
        const uint32_t *qb = t->q + 3 * t->order[t->first[k]];
        int sh = ORC_MAX_LEVEL - t->level[k];
        double s = ldexp(t->L, -t->level[k]);
        for (int a = 0; a < 3; a++)
            t->com[3 * k + a] = t->x0[a] + ((double)(qb[a] >> sh) + 0.5) * s;
        t->eps2[k] = 0.0;
    }
}

static int build_node(orc_tree *t, int64_t k, int32_t level, int64_t first, int64_t count,
                      int64_t *tmp, const double *pos, const double *mass, const double *eps)
{
    t->level[k] = level;
    t->first[k] = first;
    t->count[k] = count;
    t->child0[k] = -1;
    t->nchild[k] = 0;
    if (count > t->leaf && level < ORC_MAX_LEVEL) {
        /* homogeneous split into 8 octants; the child at level+1 is chosen
         * by bit (20 - level) of each integer coordinate */
        int shift = ORC_MAX_LEVEL - 1 - level;
        int64_t cnt[8] = {0}, start[8], fill[8];
        for (int64_t s = first; s < first + count; s++)
            cnt[octant_of(t->q + 3 * t->order[s], shift)]++;
        int64_t acc = 0;
        int nch = 0;
        for (int o = 0; o < 8; o++) {
            start[o] = acc;
            fill[o] = acc;
            acc += cnt[o];
            nch += cnt[o] > 0;
        }
        for (int64_t s = first; s < first + count; s++) {
            int64_t b = t->order[s];
            tmp[fill[octant_of(t->q + 3 * b, shift)]++] = b;
        }
        memcpy(t->order + first, tmp, (size_t)count * sizeof(int64_t));
        int64_t c0 = t->nn;
        int rc = grow(t, t->nn + nch);
        if (rc) return rc;
        t->nn += nch;
        t->child0[k] = c0;
        t->nchild[k] = nch;
        int64_t c = c0;
        for (int o = 0; o < 8; o++) {
            if (!cnt[o]) continue;
            rc = build_node(t, c, level + 1, first + start[o], cnt[o], tmp, pos, mass, eps);
            if (rc) return rc;
            c++;
        }
    }
    node_moments(t, k, pos, mass, eps);
    return 0;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->q);
    free(t->order);
    free(t->level);
    free(t->first);
    free(t->count);
    free(t->child0);
    free(t->nchild);
    free(t->m);
    free(t->com);
    free(t->eps2);
    free(t->quad);
    free(t);
}

orc_tree *orc_tree_build(int64_t n, const double *pos, const double *mass, const double *eps,
                         int32_t leaf, int *err)
{
    int rc = check_bodies(n, pos, mass, eps, 0.0);
    if (!rc && leaf < 1) rc = 1;
    if (rc) {
        if (err) *err = rc;
        return NULL;
    }
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) goto oom;
    t->n = n;
    t->leaf = leaf;
    t->has_eps = eps != NULL;
    t->q = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(uint32_t));
    t->order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!t->q || !t->order) goto oom;

    /* root cube around the bounding box */
    for (int a = 0; a < 3; a++) {
        t->lo[a] = n > 0 ? pos[a] : 0.0;
        t->hi[a] = t->lo[a];
    }
    for (int64_t i = 1; i < n; i++)
        for (int a = 0; a < 3; a++) {
            double x = pos[3 * i + a];
            if (x < t->lo[a]) t->lo[a] = x;
            if (x > t->hi[a]) t->hi[a] = x;
        }
    double L = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = t->hi[a] - t->lo[a];
        if (e > L) L = e;
    }
    if (L == 0.0) L = 1.0;
    t->L = L;
    for (int a = 0; a < 3; a++) t->x0[a] = (t->lo[a] + t->hi[a]) * 0.5 - L * 0.5;
    t->S = 2097152.0 / L;

    /* integer grid coordinates */
    for (int64_t i = 0; i < n; i++) {
        t->order[i] = i;
        for (int a = 0; a < 3; a++) {
            double f = floor((pos[3 * i + a] - t->x0[a]) * t->S);
            uint32_t v;
            if (!(f >= 0.0))
                v = 0u;
            else if (f > (double)QMAX)
                v = QMAX;
            else
                v = (uint32_t)f;
            t->q[3 * i + a] = v;
        }
    }
    if (n == 0) return t; /* empty tree: no nodes */

    if (grow(t, 1)) goto oom;
    t->nn = 1;
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp) goto oom;
    rc = build_node(t, 0, 0, 0, n, tmp, pos, mass, eps);
    free(tmp);
    if (rc) goto oom;
    return t;
oom:
    orc_tree_free(t);
    if (err) *err = 4;
    return NULL;
}

int64_t orc_tree_nnodes(const orc_tree *t) { return t ? t->nn : 0; }

void orc_tree_box(const orc_tree *t, double box[8])
{
    for (int a = 0; a < 3; a++) {
        box[a] = t->lo[a];
        box[3 + a] = t->x0[a];
    }
    box[6] = t->L;
    box[7] = t->S;
}

void orc_tree_export(const orc_tree *t, int32_t *level, int64_t *first, int64_t *count,
                     int64_t *child0, int32_t *nchild, double *nmass, double *com, double *eps2,
                     int64_t *order, uint32_t *q)
{
    size_t nn = (size_t)t->nn, n = (size_t)t->n;
    if (level) memcpy(level, t->level, nn * sizeof(int32_t));
    if (first) memcpy(first, t->first, nn * sizeof(int64_t));
    if (count) memcpy(count, t->count, nn * sizeof(int64_t));
    if (child0) memcpy(child0, t->child0, nn * sizeof(int64_t));
    if (nchild) memcpy(nchild, t->nchild, nn * sizeof(int32_t));
    if (nmass) memcpy(nmass, t->m, nn * sizeof(double));
    if (com) memcpy(com, t->com, nn * 3 * sizeof(double));
    if (eps2) memcpy(eps2, t->eps2, nn * sizeof(double));
    if (order) memcpy(order, t->order, n * sizeof(int64_t));
    if (q) memcpy(q, t->q, n * 3 * sizeof(uint32_t));
}

/* Traceless quadrupole of every node about its centre of mass, from its
 * definition over the node's bodies: Q = sum_j m_j (3 d_j d_j^T - |d_j|^2 I),
 * d_j = x_j - COM_N, stored as (xx, yy, zz, xy, xz, yz). */
int orc_tree_quadrupoles(orc_tree *t, const double *pos, const double *mass)
{
    if (!t || (t->n > 0 && (!pos || !mass))) return 1;
    free(t->quad);
    t->quad = (double *)calloc((size_t)(t->nn > 0 ? t->nn : 1) * 6, sizeof(double));
    if (!t->quad) return 4;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < t->nn; k++) {
        double q[6] = {0, 0, 0, 0, 0, 0};
        const double *c = t->com + 3 * k;
        for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; s++) {
            int64_t b = t->order[s];
            double d[3] = {pos[3 * b] - c[0], pos[3 * b + 1] - c[1], pos[3 * b + 2] - c[2]};
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double m = mass[b];
            q[0] += m * (3.0 * d[0] * d[0] - d2);
            q[1] += m * (3.0 * d[1] * d[1] - d2);
            q[2] += m * (3.0 * d[2] * d[2] - d2);
            q[3] += m * 3.0 * d[0] * d[1];
            q[4] += m * 3.0 * d[0] * d[2];
            q[5] += m * 3.0 * d[1] * d[2];
        }
        for (int a = 0; a < 6; a++) t->quad[6 * k + a] = q[a];
    }
    return 0;
}

int orc_tree_quad_export(const orc_tree *t, double *out)
{
    if (!t || !t->quad || (t->nn > 0 && !out)) return 1;
    memcpy(out, t->quad, (size_t)t->nn * 6 * sizeof(double));
    return 0;
}

/* Quadrupole correction of an accepted node, d = COM_N - x_B, softened
 * r^2 = |d|^2 + e2: from the potential -G (d^T Q d) / (2 r^5) the
 * acceleration is G (-Q d / r^5 + 5/2 (d^T Q d) d / r^7). */
static void add_quad_term(double dx, double dy, double dz, double e2, double G, const double *Q,
                          double *acc, double *phi)
{
    double r2 = dx * dx + dy * dy + dz * dz + e2;
    if (!term_counts(r2)) return;
    double qd[3] = {Q[0] * dx + Q[3] * dy + Q[4] * dz, Q[3] * dx + Q[1] * dy + Q[5] * dz,
                    Q[4] * dx + Q[5] * dy + Q[2] * dz};
    double dqd = dx * qd[0] + dy * qd[1] + dz * qd[2];
    double r = sqrt(r2);
    double inv5 = 1.0 / (r2 * r2 * r);
    double inv7 = inv5 / r2;
    acc[0] += G * (-qd[0] * inv5 + 2.5 * dqd * dx * inv7);
    acc[1] += G * (-qd[1] * inv5 + 2.5 * dqd * dy * inv7);
    acc[2] += G * (-qd[2] * inv5 + 2.5 * dqd * dz * inv7);
    *phi -= 0.5 * G * dqd * inv5;
}

typedef struct {
    const orc_tree *t;
    const double *pos, *mass, *eps;
    double e02, G, theta2;
    int quad; /* add the quadrupole term of accepted nodes */
} walk_ctx;

typedef struct {
    int64_t b;
    double x[3], eb2; /* target position, eps_B^2 */
    double a[3], phi, aabs;
    int64_t nacc, npair;
} walk_state;

static void walk_node(const walk_ctx *w, walk_state *st, int64_t k)
{
    const orc_tree *t = w->t;
    if (t->nchild[k] == 0) {
        /* leaf: classical body-to-body terms (eq. Force_leaf) */
        for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; s++) {
            int64_t j = t->order[s];
            if (j == st->b) continue;
            double e2 = w->eps ? 0.5 * (st->eb2 + w->eps[j] * w->eps[j]) : w->e02;
            add_term(w->pos[3 * j] - st->x[0], w->pos[3 * j + 1] - st->x[1],
                     w->pos[3 * j + 2] - st->x[2], e2, w->G * w->mass[j], st->a, &st->phi,
                     &st->aabs);
            st->npair++;
        }
        return;
    }
    /* internal node: opening test of eq. (accuracy) */
    double dx = t->com[3 * k] - st->x[0];
    double dy = t->com[3 * k + 1] - st->x[1];
    double dz = t->com[3 * k + 2] - st->x[2];
    double D2 = dx * dx + dy * dy + dz * dz;
    double s = ldexp(t->L, -t->level[k]);
    if (s * s < w->theta2 * D2) {
        /* accepted: monopole at the centre of mass (eq. Force_thetaTrue) */
        double e2 = w->eps ? 0.5 * (st->eb2 + t->eps2[k]) : w->e02;
        add_term(dx, dy, dz, e2, w->G * t->m[k], st->a, &st->phi, &st->aabs);
        if (w->quad) add_quad_term(dx, dy, dz, e2, w->G, t->quad + 6 * k, st->a, &st->phi);
        st->nacc++;
        return;
    }
    for (int64_t c = t->child0[k]; c < t->child0[k] + t->nchild[k]; c++) walk_node(w, st, c);
}

int orc_tree_accel(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                   double eps0, double G, double theta, const int64_t *targets, int64_t nt,
                   double *acc, double *phi, double *absacc, int64_t *counts)
{
    return orc_tree_accel_q(t, pos, mass, eps, eps0, G, theta, targets, nt, acc, phi, absacc,
                            counts, 0);
}

int orc_tree_accel_q(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                     double eps0, double G, double theta, const int64_t *targets, int64_t nt,
                     double *acc, double *phi, double *absacc, int64_t *counts, int quad)
{
    if (!t) return 1;
    if (quad && !t->quad) return 1;
    int64_t n = t->n;
    if (!(theta >= 0.0) || !isfinite(theta)) return 1;
    if (!eps && !(eps0 >= 0.0 && isfinite(eps0))) return 1;
    if ((eps != NULL) != (t->has_eps != 0)) return 1;
    if (!targets && nt != n) return 1;
    if (nt < 0 || (nt > 0 && !acc)) return 1;
    if (targets)
        for (int64_t i = 0; i < nt; i++)
            if (targets[i] < 0 || targets[i] >= n) return 1;
    walk_ctx w = {t, pos, mass, eps, eps0 * eps0, G, theta * theta, quad};

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; i++) {
        walk_state st;
        memset(&st, 0, sizeof(st));
        st.b = targets ? targets[i] : i;
        for (int a = 0; a < 3; a++) st.x[a] = pos[3 * st.b + a];
        st.eb2 = eps ? eps[st.b] * eps[st.b] : 0.0;
        walk_node(&w, &st, 0);
        for (int a = 0; a < 3; a++) acc[3 * i + a] = st.a[a];
        if (phi) phi[i] = st.phi;
        if (absacc) absacc[i] = st.aabs;
        if (counts) {
            counts[2 * i] = st.nacc;
            counts[2 * i + 1] = st.npair;
        }
    }
    return 0;
}

/* --------------------------------------------------------------- leapfrog */

static int accel_all(int64_t n, const double *pos, const double *mass, const double *eps,
                     double eps0, double G, double theta, int32_t leaf, double *acc)
{
    if (theta < 0.0) return orc_direct(n, pos, mass, eps, eps0, G, NULL, n, acc, NULL, NULL);
    int err = 0;
    orc_tree *t = orc_tree_build(n, pos, mass, eps, leaf, &err);
    if (!t) return err;
    int rc = orc_tree_accel(t, pos, mass, eps, eps0, G, theta, NULL, n, acc, NULL, NULL, NULL);
    orc_tree_free(t);
    return rc;
}

int orc_leapfrog(int64_t n, double *pos, double *vel, const double *mass, const double *eps,
                 double eps0, double G, double theta, int32_t leaf, double dt, int32_t nsteps,
                 double *acc)
{
    if (n < 0 || nsteps < 0 || !isfinite(dt)) return 1;
    if (n > 0 && (!vel || !acc)) return 1;
    double h = 0.5 * dt;
    for (int32_t s = 0; s < nsteps; s++) {
        for (int64_t i = 0; i < 3 * n; i++) vel[i] += h * acc[i]; /* kick */
        for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * vel[i]; /* drift */
        int rc = accel_all(n, pos, mass, eps, eps0, G, theta, leaf, acc);
        if (rc) return rc;
        for (int64_t i = 0; i < 3 * n; i++) vel[i] += h * acc[i]; /* kick */
    }
    return 0;
}

int orc_euler(int64_t n, double *pos, double *vel, const double *mass, const double *eps,
              double eps0, double G, double theta, int32_t leaf, double dt, int32_t nsteps,
              int32_t every, double *acc)
{
    if (n < 0 || nsteps < 0 || every < 1 || !isfinite(dt)) return 1;
    if (n > 0 && (!vel || !acc)) return 1;
    for (int32_t s = 1; s <= nsteps; s++) {
        for (int64_t i = 0; i < 3 * n; i++) vel[i] += dt * acc[i]; /* kick, held gravity */
        for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * vel[i]; /* drift, new velocity */
        if (s % every == 0) {
            int rc = accel_all(n, pos, mass, eps, eps0, G, theta, leaf, acc);
            if (rc) return rc;
        }
    }
    return 0;
}

/* ------------------------------------------------------------- aggregates */

static int64_t uf_find(int32_t *parent, int64_t x)
{
    while (parent[x] != x) x = parent[x];
    return x;
}

int orc_contact_components(int64_t n, const double *pos, const double *radius, double skin,
                           int32_t *label, int64_t *n_contacts, int64_t *n_aggregates)
{
    if (n < 0 || n > 2147483647 || !(skin >= 0.0) || !isfinite(skin)) return 1;
    if (n > 0 && (!pos || !radius || !label || !n_contacts || !n_aggregates)) return 1;
    for (int64_t i = 0; i < n; i++) label[i] = (int32_t)i;
    int64_t contacts = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = i + 1; j < n; j++) {
            double dx = pos[3 * j] - pos[3 * i];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            double dist2 = dx * dx + dy * dy + dz * dz;
            double R = radius[i] + radius[j] + skin;
            if (dist2 <= R * R) {
                contacts++;
                /* union: the larger root is attached to the smaller */
                int64_t a = uf_find(label, i), b = uf_find(label, j);
                if (a != b) {
                    if (a < b)
                        label[b] = (int32_t)a;
                    else
                        label[a] = (int32_t)b;
                }
            }
        }
    }
    int64_t *size = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!size) return 4;
    for (int64_t i = 0; i < n; i++) label[i] = (int32_t)uf_find(label, i);
    for (int64_t i = 0; i < n; i++) size[label[i]]++;
    int64_t agg = 0;
    for (int64_t i = 0; i < n; i++) agg += size[i] > 1;
    free(size);
    *n_contacts = contacts;
    *n_aggregates = agg;
    return 0;
}

int orc_diagnostics(int64_t n, const double *pos, const double *vel, const double *mass,
                    const double *eps, double eps0, double G, double out[8])
{
    int rc = check_bodies(n, pos, mass, eps, eps0);
    if (rc) return rc;
    if (n > 0 && !vel) return 1;
    double *phi = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *acc = (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    if (!phi || !acc) {
        free(phi);
        free(acc);
        return 4;
    }
    rc = orc_direct(n, pos, mass, eps, eps0, G, NULL, n, acc, phi, NULL);
    for (int a = 0; a < 8; a++) out[a] = 0.0;
    for (int64_t i = 0; !rc && i < n; i++) {
        const double *x = pos + 3 * i, *v = vel + 3 * i;
        double m = mass[i];
        out[0] += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        out[1] += 0.5 * m * phi[i];
        out[2] += m * v[0];
        out[3] += m * v[1];
        out[4] += m * v[2];
        out[5] += m * (x[1] * v[2] - x[2] * v[1]);
        out[6] += m * (x[2] * v[0] - x[0] * v[2]);
        out[7] += m * (x[0] * v[1] - x[1] * v[0]);
    }
    free(phi);
    free(acc);
    return rc;
}

/* eq. (dt_g): the gravity time step must satisfy Delta t_g < T_g / 2 =
 * 1 / (2 sqrt(G rho)), rho the material density of the bodies. For a set of
 * bodies the bound is the one of the densest body, rho_i = m_i / V_i with
 * V_i = (4/3) pi r_i^3 (the shortest characteristic time). Massless bodies are
 * skipped; with none left the bound is +inf, and a massive body of radius 0
 * (infinite density) gives 0. */
int orc_gravity_dt_bound(int64_t n, const double *mass, const double *radius, double G,
                         double *dt)
{
    if (n < 0 || !dt || (n > 0 && (!mass || !radius)) || !(G > 0.0) || !isfinite(G)) return 1;
    double rho_max = -1.0;
    for (int64_t i = 0; i < n; i++) {
        double m = mass[i], r = radius[i];
        if (!isfinite(m) || !isfinite(r)) return 2;
        if (m < 0.0) return 3;
        if (r < 0.0) return 1;
        if (m == 0.0) continue;
        double vol = (4.0 / 3.0) * 3.141592653589793 * (r * r * r);
        double rho = m / vol; /* +inf for r = 0 */
        if (rho > rho_max) rho_max = rho;
    }
    *dt = rho_max < 0.0 ? INFINITY : 0.5 / sqrt(G * rho_max);
    return 0;
}

/* ------------------------------------------------------------------- VJPs */

/* Adjoint of one softened term t = G m_s d / r^3, d = X_s - x_i,
 * r^2 = |d|^2 + e2, for upstream l (the target's lambda):
 *   dt/dd = G m_s K, K = I / r^3 - 3 d d^T / r^5;  dt/dm_s = G d / r^3;
 *   dt/de2 = -3/2 G m_s d / r^5.
 * Writes gd = G m_s K l (so g_x_i -= gd, g_X_s += gd), gm = G l.d / r^3
 * and ge2 = -3/2 G m_s (l.d) / r^5. A term whose r^2 is not a positive normal
 * double contributes 0 (as in add_term). */
static void term_vjp(const double d[3], double e2, double G, double ms, const double l[3],
                     double gd[3], double *gm, double *ge2)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2;
    gd[0] = gd[1] = gd[2] = 0.0;
    *gm = 0.0;
    *ge2 = 0.0;
    if (!term_counts(r2)) return;
    double r = sqrt(r2);
    double inv3 = 1.0 / (r2 * r);
    double inv5 = inv3 / r2;
    double ld = l[0] * d[0] + l[1] * d[1] + l[2] * d[2];
    for (int a = 0; a < 3; a++) gd[a] = G * ms * (l[a] * inv3 - 3.0 * d[a] * ld * inv5);
    *gm = G * ld * inv3;
    *ge2 = -1.5 * G * ms * ld * inv5;
}

/* Magnitudes of the parts of one term of term_vjp, for error bounds: with
 * |l|.|d| = sum_a |l_a| |d_a|, gd_a = G m_s (|l_a| / r^3 + 3 |d_a| |l|.|d| / r^5),
 * gm = G |l|.|d| / r^3 and ge2 = 3/2 G m_s |l|.|d| / r^5: each bounds the
 * absolute value of the corresponding part of term_vjp (triangle inequality)
 * and is what a rounding of every operation in it is relative to. */
static void term_vjp_abs(const double d[3], double e2, double G, double ms, const double l[3],
                         double gd[3], double *gm, double *ge2)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2;
    gd[0] = gd[1] = gd[2] = 0.0;
    *gm = 0.0;
    *ge2 = 0.0;
    if (!term_counts(r2)) return;
    double r = sqrt(r2);
    double inv3 = 1.0 / (r2 * r);
    double inv5 = inv3 / r2;
    double ld = fabs(l[0]) * fabs(d[0]) + fabs(l[1]) * fabs(d[1]) + fabs(l[2]) * fabs(d[2]);
    for (int a = 0; a < 3; a++) gd[a] = G * ms * (fabs(l[a]) * inv3 + 3.0 * fabs(d[a]) * ld * inv5);
    *gm = G * ld * inv3;
    *ge2 = 1.5 * G * ms * ld * inv5;
}

int orc_direct_vjp(int64_t n, const double *pos, const double *mass, const double *eps,
                   double eps0, double G, const double *lambda, double *g_pos, double *g_mass)
{
    int rc = check_bodies(n, pos, mass, eps, eps0);
    if (rc) return rc;
    if (n > 0 && (!lambda || !g_pos || !g_mass)) return 1;
    double e02 = eps0 * eps0;
    for (int64_t i = 0; i < n; i++) {
        const double *l = lambda + 3 * i;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double d[3] = {pos[3 * j] - pos[3 * i], pos[3 * j + 1] - pos[3 * i + 1],
                           pos[3 * j + 2] - pos[3 * i + 2]};
            double e2 = eps ? 0.5 * (eps[i] * eps[i] + eps[j] * eps[j]) : e02;
            double gd[3], gm, ge2;
            term_vjp(d, e2, G, mass[j], l, gd, &gm, &ge2);
            for (int a = 0; a < 3; a++) {
                g_pos[3 * i + a] -= gd[a];
                g_pos[3 * j + a] += gd[a];
            }
            g_mass[j] += gm;
        }
    }
    return 0;
}

typedef struct {
    const orc_tree *t;
    const double *pos, *mass, *eps, *lambda;
    double e02, G, theta2;
    double *g_pos, *g_mass;     /* body adjoints */
    double *nX, *nm, *ne2;      /* node adjoints: centre of mass, mass, <eps^2> */
    int absmode;                /* accumulate the magnitudes of every contribution */
} vjp_ctx;

static void vjp_node(vjp_ctx *w, int64_t b, const double xb[3], double eb2, const double l[3],
                     int64_t k)
{
    const orc_tree *t = w->t;
    double gd[3], gm, ge2;
    if (t->nchild[k] == 0) {
        for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; s++) {
            int64_t j = t->order[s];
            if (j == b) continue;
            double d[3] = {w->pos[3 * j] - xb[0], w->pos[3 * j + 1] - xb[1],
                           w->pos[3 * j + 2] - xb[2]};
            double e2 = w->eps ? 0.5 * (eb2 + w->eps[j] * w->eps[j]) : w->e02;
            if (w->absmode) term_vjp_abs(d, e2, w->G, w->mass[j], l, gd, &gm, &ge2);
            else term_vjp(d, e2, w->G, w->mass[j], l, gd, &gm, &ge2);
            for (int a = 0; a < 3; a++) {
                w->g_pos[3 * b + a] += w->absmode ? gd[a] : -gd[a];
                w->g_pos[3 * j + a] += gd[a];
            }
            w->g_mass[j] += gm;
        }
        return;
    }
    double d[3] = {t->com[3 * k] - xb[0], t->com[3 * k + 1] - xb[1], t->com[3 * k + 2] - xb[2]};
    double D2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double sd = ldexp(t->L, -t->level[k]);
    if (sd * sd < w->theta2 * D2) {
        double e2 = w->eps ? 0.5 * (eb2 + t->eps2[k]) : w->e02;
        if (w->absmode) term_vjp_abs(d, e2, w->G, t->m[k], l, gd, &gm, &ge2);
        else term_vjp(d, e2, w->G, t->m[k], l, gd, &gm, &ge2);
        for (int a = 0; a < 3; a++) {
            w->g_pos[3 * b + a] += w->absmode ? gd[a] : -gd[a];
            w->nX[3 * k + a] += gd[a];
        }
        w->nm[k] += gm;
        if (w->eps) w->ne2[k] += 0.5 * ge2; /* e2 = (eps_B^2 + <eps^2>_N) / 2 */
        return;
    }
    for (int64_t c = t->child0[k]; c < t->child0[k] + t->nchild[k]; c++) vjp_node(w, b, xb, eb2, l, c);
}

static int tree_vjp(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                    double eps0, double G, double theta, const double *lambda, double *g_pos,
                    double *g_mass, int absmode)
{
    if (!t) return 1;
    int64_t n = t->n;
    if (!(theta >= 0.0) || !isfinite(theta)) return 1;
    if (!eps && !(eps0 >= 0.0 && isfinite(eps0))) return 1;
    if ((eps != NULL) != (t->has_eps != 0)) return 1;
    if (n > 0 && (!lambda || !g_pos || !g_mass)) return 1;
    if (n == 0) return 0;
    int64_t nn = t->nn;
    double *nX = (double *)calloc((size_t)nn * 3, sizeof(double));
    double *nm = (double *)calloc((size_t)nn, sizeof(double));
    double *ne2 = (double *)calloc((size_t)nn, sizeof(double));
    if (!nX || !nm || !ne2) {
        free(nX);
        free(nm);
        free(ne2);
        return 4;
    }
    vjp_ctx w = {t, pos, mass, eps, lambda, eps0 * eps0, G, theta * theta, g_pos, g_mass,
                 nX, nm, ne2, absmode};
    for (int64_t b = 0; b < n; b++) {
        double eb2 = eps ? eps[b] * eps[b] : 0.0;
        vjp_node(&w, b, pos + 3 * b, eb2, lambda + 3 * b, 0);
    }
    /* A node's centre of mass X_N = sum m_j x_j / m_N, its mass m_N = sum m_j
     * and softening <eps^2>_N = sum m_j eps_j^2 / m_N depend on every member:
     *   dX_N/dx_j = m_j / m_N,  dX_N/dm_j = (x_j - X_N) / m_N,  dm_N/dm_j = 1,
     *   d<eps^2>_N/dm_j = (eps_j^2 - <eps^2>_N) / m_N. */
    for (int64_t k = 0; k < nn; k++) {
        double mN = t->m[k];
        for (int64_t s = t->first[k]; s < t->first[k] + t->count[k]; s++) {
            int64_t j = t->order[s];
            g_mass[j] += nm[k];
            if (!(mN > 0.0)) continue;
            double dot = 0.0;
            for (int a = 0; a < 3; a++) {
                g_pos[3 * j + a] += mass[j] / mN * nX[3 * k + a];
                double dx = pos[3 * j + a] - t->com[3 * k + a];
                dot += (absmode ? fabs(dx) : dx) * nX[3 * k + a];
            }
            g_mass[j] += dot / mN;
            if (eps) {
                double de = eps[j] * eps[j] - t->eps2[k];
                g_mass[j] += ne2[k] * (absmode ? fabs(de) : de) / mN;
            }
        }
    }
    free(nX);
    free(nm);
    free(ne2);
    return 0;
}

int orc_tree_vjp(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                 double eps0, double G, double theta, const double *lambda, double *g_pos,
                 double *g_mass)
{
    return tree_vjp(t, pos, mass, eps, eps0, G, theta, lambda, g_pos, g_mass, 0);
}

int orc_tree_vjp_abs(const orc_tree *t, const double *pos, const double *mass, const double *eps,
                     double eps0, double G, double theta, const double *lambda, double *g_pos,
                     double *g_mass)
{
    return tree_vjp(t, pos, mass, eps, eps0, G, theta, lambda, g_pos, g_mass, 1);
}

/* VJP of A at pos for upstream lam: adds into gx and gm. */
static int accel_vjp(int64_t n, const double *pos, const double *mass, const double *eps,
                     double eps0, double G, double theta, int32_t leaf, const double *lam,
                     double *gx, double *gm)
{
    if (theta < 0.0) return orc_direct_vjp(n, pos, mass, eps, eps0, G, lam, gx, gm);
    int err = 0;
    orc_tree *t = orc_tree_build(n, pos, mass, eps, leaf, &err);
    if (!t) return err;
    int rc = orc_tree_vjp(t, pos, mass, eps, eps0, G, theta, lam, gx, gm);
    orc_tree_free(t);
    return rc;
}

int orc_rollout_grad(int64_t n, const double *pos0, const double *vel0, const double *mass,
                     const double *eps, double eps0, double G, double theta, int32_t leaf,
                     double dt, int32_t nsteps, const double *xbar, const double *vbar,
                     double *gx0, double *gv0, double *gm)
{
    if (n < 0 || nsteps < 0 || !isfinite(dt)) return 1;
    if (n == 0) return 0;
    size_t n3 = (size_t)n * 3;
    /* forward: positions x_0..x_T (each step's acceleration is A(x_k)) */
    double *X = (double *)malloc((size_t)(nsteps + 1) * n3 * sizeof(double));
    double *v = (double *)malloc(n3 * sizeof(double));
    double *a = (double *)malloc(n3 * sizeof(double));
    double *xb = (double *)malloc(n3 * sizeof(double));
    double *vb = (double *)malloc(n3 * sizeof(double));
    double *ab = (double *)malloc(n3 * sizeof(double));
    int rc = 0;
    if (!X || !v || !a || !xb || !vb || !ab) {
        rc = 4;
        goto done;
    }
    memcpy(X, pos0, n3 * sizeof(double));
    memcpy(v, vel0, n3 * sizeof(double));
    rc = accel_all(n, X, mass, eps, eps0, G, theta, leaf, a);
    if (rc) goto done;
    double h = 0.5 * dt;
    for (int32_t s = 0; s < nsteps; s++) {
        double *x = X + (size_t)s * n3, *xn = X + (size_t)(s + 1) * n3;
        for (size_t i = 0; i < n3; i++) v[i] += h * a[i];
        for (size_t i = 0; i < n3; i++) xn[i] = x[i] + dt * v[i];
        rc = accel_all(n, xn, mass, eps, eps0, G, theta, leaf, a);
        if (rc) goto done;
        for (size_t i = 0; i < n3; i++) v[i] += h * a[i];
    }
    /* Reverse mode. Step s maps (x_s, v_s, a_s) to (x_{s+1}, v_{s+1}, a_{s+1}):
     *   u = v_s + h a_s;  x_{s+1} = x_s + dt u;  a_{s+1} = A(x_{s+1});
     *   v_{s+1} = u + h a_{s+1}.
     * a_{s+1} feeds this step's second kick and step s+1's first kick, so its
     * adjoint is complete after this step's second kick has been added, and
     * one VJP per step is applied at x_{s+1}; a_0 = A(x_0) takes one more. */
    memcpy(xb, xbar, n3 * sizeof(double));
    memcpy(vb, vbar, n3 * sizeof(double));
    for (size_t i = 0; i < n3; i++) ab[i] = 0.0;
    for (size_t i = 0; i < (size_t)n; i++) gm[i] = 0.0;
    for (int32_t s = nsteps - 1; s >= 0; s--) {
        const double *xn = X + (size_t)(s + 1) * n3;
        for (size_t i = 0; i < n3; i++) ab[i] += h * vb[i];          /* second kick */
        rc = accel_vjp(n, xn, mass, eps, eps0, G, theta, leaf, ab, xb, gm);
        if (rc) goto done;
        for (size_t i = 0; i < n3; i++) vb[i] += dt * xb[i];         /* drift: u-bar */
        for (size_t i = 0; i < n3; i++) ab[i] = h * vb[i];           /* first kick */
    }
    rc = accel_vjp(n, X, mass, eps, eps0, G, theta, leaf, ab, xb, gm);
    if (rc) goto done;
    memcpy(gx0, xb, n3 * sizeof(double));
    memcpy(gv0, vb, n3 * sizeof(double));
done:
    free(X);
    free(v);
    free(a);
    free(xb);
    free(vb);
    free(ab);
    return rc;
}
