"""Every planted mistake in the oracle must make at least one pin fail.

Each mutant is a copy of the oracle's C source with one plausible mistake
(a dropped term, a wrong sign or index, a swapped operand, a wrong constant),
compiled to a temporary library; the pins run against it and at least one of
them must raise. This checks that the pins fix the oracle, not only that the
oracle agrees with itself.
"""
import os

import pytest

import _pins
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "bh_oracle.c")

MUTANTS = {
    "subnormal_r2_counts": ("static int term_counts(double r2) { return r2 >= DBL_MIN; }",
                            "static int term_counts(double r2) { return r2 > 0.0; }"),
    "dt_g_no_half": ("*dt = rho_max < 0.0 ? INFINITY : 0.5 / sqrt(G * rho_max);",
                     "*dt = rho_max < 0.0 ? INFINITY : 1.0 / sqrt(G * rho_max);"),
    "dt_g_least_dense": ("if (rho > rho_max) rho_max = rho;",
                         "if (rho_max < 0.0 || rho < rho_max) rho_max = rho;"),
    "dt_g_radius_squared": ("double vol = (4.0 / 3.0) * 3.141592653589793 * (r * r * r);",
                            "double vol = (4.0 / 3.0) * 3.141592653589793 * (r * r);"),
    "contact_strict": ("if (dist2 <= R * R) {", "if (dist2 < R * R) {"),
    "contact_union_larger": ("label[b] = (int32_t)a;\n                    else\n                        label[a] = (int32_t)b;",
                             "label[a] = (int32_t)b;\n                    else\n                        label[b] = (int32_t)a;"),
    "contact_aggregate_singles": ("agg += size[i] > 1;", "agg += size[i] > 0;"),
    "quad_sign": ("acc[0] += G * (-qd[0] * inv5 + 2.5 * dqd * dx * inv7);",
                  "acc[0] += G * (qd[0] * inv5 + 2.5 * dqd * dx * inv7);"),
    "quad_trace_kept": ("q[0] += m * (3.0 * d[0] * d[0] - d2);", "q[0] += m * (3.0 * d[0] * d[0]);"),
    "quad_offdiag_factor": ("q[3] += m * 3.0 * d[0] * d[1];", "q[3] += m * d[0] * d[1];"),
    "quad_r7": ("double inv7 = inv5 / r2;", "double inv7 = inv5 / r;"),
    "euler_drift_first": ("for (int64_t i = 0; i < 3 * n; i++) vel[i] += dt * acc[i]; /* kick, held gravity */\n        for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * vel[i]; /* drift, new velocity */",
                          "for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * vel[i]; /* drift, new velocity */\n        for (int64_t i = 0; i < 3 * n; i++) vel[i] += dt * acc[i]; /* kick, held gravity */"),
    "euler_every_ignored": ("if (s % every == 0) {", "if (1) {"),
    "pair_sign": ("acc[0] += gm * dx * inv3;", "acc[0] -= gm * dx * inv3;"),
    "pair_drop_z": ("double d2 = dx * dx + dy * dy + dz * dz;", "double d2 = dx * dx + dy * dy;"),
    "r3_to_r2": ("double inv3 = 1.0 / (r2 * r);\n    acc[0]", "double inv3 = 1.0 / r2;\n    acc[0]"),
    "direct_swap_ij": ("add_term(pos[3 * j] - pos[3 * i],", "add_term(pos[3 * i] - pos[3 * j],"),
    "direct_self": ("if (j == i) continue; /* j != i in eq. (Newton) */", ""),
    "soft_receiver_only": ("double e2 = eps ? 0.5 * (ei2 + eps[j] * eps[j]) : e02;",
                           "double e2 = eps ? ei2 : e02;"),
    "soft_no_half": ("0.5 * (st->eb2 + w->eps[j] * w->eps[j])", "(st->eb2 + w->eps[j] * w->eps[j])"),
    "node_soft": ("0.5 * (st->eb2 + t->eps2[k])", "0.5 * (st->eb2 + st->eb2)"),
    "mac_inverted": ("if (s * s < w->theta2 * D2) {", "if (s * s > w->theta2 * D2) {"),
    "mac_drop_z": ("double D2 = dx * dx + dy * dy + dz * dz;\n    double s = ldexp",
                   "double D2 = dx * dx + dy * dy;\n    double s = ldexp"),
    "mac_half_side": ("double s = ldexp(t->L, -t->level[k]);\n    if",
                      "double s = ldexp(t->L, -t->level[k] - 1);\n    if"),
    "walk_self": ("if (j == st->b) continue;", ""),
    "com_unweighted": ("mx += t->com[3 * c] * t->m[c];", "mx += t->com[3 * c];"),
    "leaf_com_y_from_x": ("my += pos[3 * b + 1] * mass[b];", "my += pos[3 * b] * mass[b];"),
    "octant_bit": ("int shift = ORC_MAX_LEVEL - 1 - level;", "int shift = ORC_MAX_LEVEL - level;"),
    "octant_order": ("return (int)((((q[0] >> shift) & 1u) << 2) | (((q[1] >> shift) & 1u) << 1) |",
                     "return (int)((((q[1] >> shift) & 1u) << 2) | (((q[0] >> shift) & 1u) << 1) |"),
    "leaf_rule": ("if (count > t->leaf && level < ORC_MAX_LEVEL) {",
                  "if (count >= t->leaf && level < ORC_MAX_LEVEL) {"),
    "root_half_box": ("t->x0[a] = (t->lo[a] + t->hi[a]) * 0.5 - L * 0.5;",
                      "t->x0[a] = t->lo[a] + L * 0.25;"),
    "kick_full": ("vel[i] += h * acc[i]; /* kick */\n        for (int64_t i = 0; i < 3 * n; i++) pos[i]",
                  "vel[i] += dt * acc[i]; /* kick */\n        for (int64_t i = 0; i < 3 * n; i++) pos[i]"),
    "drift_old_acc": ("for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * vel[i]; /* drift */",
                      "for (int64_t i = 0; i < 3 * n; i++) pos[i] += dt * (vel[i] - 0.5 * dt * acc[i]);"),
    "ekin_no_half": ("out[0] += 0.5 * m * (v[0] * v[0]", "out[0] += m * (v[0] * v[0]"),
    "angmom_sign": ("out[7] += m * (x[0] * v[1] - x[1] * v[0]);", "out[7] += m * (x[1] * v[0] - x[0] * v[1]);"),
    "vjp_abs_outer_factor": ("gd[a] = G * ms * (fabs(l[a]) * inv3 + 3.0 * fabs(d[a]) * ld * inv5);",
                             "gd[a] = G * ms * (fabs(l[a]) * inv3 + fabs(d[a]) * ld * inv5);"),
    "vjp_abs_target_sign": ("w->g_pos[3 * b + a] += w->absmode ? gd[a] : -gd[a];\n                w->g_pos[3 * j + a]",
                            "w->g_pos[3 * b + a] += -gd[a];\n                w->g_pos[3 * j + a]"),
    "vjp_abs_signed_handdown": ("dot += (absmode ? fabs(dx) : dx) * nX[3 * k + a];",
                                "dot += dx * nX[3 * k + a];"),
    "vjp_drop_outer": ("gd[a] = G * ms * (l[a] * inv3 - 3.0 * d[a] * ld * inv5);",
                       "gd[a] = G * ms * (l[a] * inv3);"),
    "vjp_outer_factor": ("gd[a] = G * ms * (l[a] * inv3 - 3.0 * d[a] * ld * inv5);",
                         "gd[a] = G * ms * (l[a] * inv3 - 2.0 * d[a] * ld * inv5);"),
    "vjp_source_sign": ("                g_pos[3 * j + a] += gd[a];\n            }\n            g_mass[j] += gm;\n        }\n    }\n    return 0;",
                        "                g_pos[3 * j + a] -= gd[a];\n            }\n            g_mass[j] += gm;\n        }\n    }\n    return 0;"),
    "vjp_mass_term": ("3.0 * d[a] * ld * inv5);\n    *gm = G * ld * inv3;",
                      "3.0 * d[a] * ld * inv5);\n    *gm = G * ld * inv5;"),
    "vjp_node_com_mass": ("g_mass[j] += dot / mN;", "g_mass[j] += dot;"),
    "vjp_node_pos_weight": ("g_pos[3 * j + a] += mass[j] / mN * nX[3 * k + a];",
                            "g_pos[3 * j + a] += nX[3 * k + a];"),
    "vjp_node_eps": ("g_mass[j] += ne2[k] * (absmode ? fabs(de) : de) / mN;", "(void)de;"),
    "rollout_no_a0": ("    rc = accel_vjp(n, X, mass, eps, eps0, G, theta, leaf, ab, xb, gm);\n    if (rc) goto done;\n    memcpy(gx0",
                      "    memcpy(gx0"),
    "rollout_kick": ("for (size_t i = 0; i < n3; i++) ab[i] += h * vb[i];", "for (size_t i = 0; i < n3; i++) ab[i] += dt * vb[i];"),
    "rollout_drift": ("for (size_t i = 0; i < n3; i++) vb[i] += dt * xb[i];", "for (size_t i = 0; i < n3; i++) vb[i] += h * xb[i];"),
}


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutated = tmp_path / "bh_oracle.c"
    mutated.write_text(source.replace(old, new))
    lib = oracle.compile_source(str(mutated), str(tmp_path / "liboracle_mutant.so"))
    failed = []
    try:
        oracle.use_library(lib)
        for pin in _pins.ALL_PINS:
            try:
                pin()
            except Exception as e:  # an exception of any kind is a caught mutant
                failed.append((pin.__name__, type(e).__name__))
    finally:
        oracle.use_library(None)
    assert failed, f"mutant {name} passed every pin"
