"""Mutation check of the oracle's pins.  Each mutant plants one plausible
mistake in a copy of the oracle's C source -- a dropped factor, a flipped
sign, a wrong index or divisor, a missing bound, a strict comparison, a
wrong round count -- builds it with the oracle's own flags, and runs the
oracle's pins (CPU) against that build in a child process.  Every mutant
must make at least one pin fail: a pin set that let one through would not
pin the oracle."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "thetis_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_multipliers_cpu.py", "tests/test_rounding_general_cpu.py",
        "tests/test_map_cpu.py"]

MUTANTS = [
    ("gradient_drops_beta",
     "double g = s->ctil[j] + s->beta * dot + s->rho * (s->y[j] - s->ybar[j]);",
     "double g = s->ctil[j] + dot + s->rho * (s->y[j] - s->ybar[j]);"),
    ("prox_term_sign",
     "double g = s->ctil[j] + s->beta * dot + s->rho * (s->y[j] - s->ybar[j]);",
     "double g = s->ctil[j] + s->beta * dot - s->rho * (s->y[j] - s->ybar[j]);"),
    ("upper_bound_not_clipped",
     "        if (yn > p->ub[j]) yn = p->ub[j];\n        double d = yn - s->y[j];",
     "        double d = yn - s->y[j];"),
    ("residual_update_drops_value",
     "s->r[p->ridx[e]] += d * p->cval[e];\n        return;",
     "s->r[p->ridx[e]] += d;\n        return;"),
    ("slack_sign_swapped",
     "p->sense[i] > 0 ? -1.0 : (p->sense[i] < 0 ? 1.0 : 0.0)",
     "p->sense[i] > 0 ? 1.0 : (p->sense[i] < 0 ? -1.0 : 0.0)"),
    ("curvature_drops_beta",
     "        return s->beta * a2 + s->rho;",
     "        return a2 + s->rho;"),
    ("penalty_drops_half",
     "f += -s->ubar[i] * w + 0.5 * s->beta * w * w;",
     "f += -s->ubar[i] * w + s->beta * w * w;"),
    ("dual_clip_wrong_side",
     "if (s->rho == 0.0) {\n            if (p->sense[i] > 0 && ui < 0.0) ui = 0.0;",
     "if (s->rho == 0.0) {\n            if (p->sense[i] > 0 && ui > 0.0) ui = 0.0;"),
    ("dual_quadratic_term",
     "double phi = bu - uu / (2.0 * s->beta);",
     "double phi = bu - uu / s->beta;"),
    ("simplex_projection_divisor",
     "double t = (csum - 1.0) / (double)(j + 1);",
     "double t = (csum - 1.0) / (double)(j + 2);"),
    ("multiplier_step_sign",
     "s->ubar[i] = s->ubar[i] - s->beta * w;",
     "s->ubar[i] = s->ubar[i] + s->beta * w;"),
    ("vc_threshold_unscaled",
     "            if (s2 < T) T = s2;\n        }\n        double cst = 0.0;\n"
     "        for (int64_t j = 0; j < n; ++j) { sol[j] = x[j] >= T ? 1 : 0;",
     "        }\n        double cst = 0.0;\n"
     "        for (int64_t j = 0; j < n; ++j) { sol[j] = x[j] >= T ? 1 : 0;"),
    ("philox_nine_rounds", "for (int round = 0; round < 10; ++round)", "for (int round = 0; round < 9; ++round)"),
    ("cover_rounds_too_few",
     "(int32_t)ceil(log(2.0 * (double)m))",
     "(int32_t)ceil(log((double)m))"),
    ("packing_alteration_strict",
     "if (w2 >= w) tot += w2;",
     "if (w2 > w) tot += w2;"),
    ("block_curvature_drops_beta",
     "    return s->beta * best + s->rho;",
     "    return best + s->rho;"),
    ("block_curvature_sums_columns",
     "        if (a2 > best) best = a2;",
     "        best += a2;"),
    ("blocks_sharing_a_row_accepted",
     "if (last_row[t] == i) { shared = 1; break; }",
     "if (last_row[t] == i) { break; }"),
    ("class_order_descending",
     "if (x->key != y->key) return x->key < y->key ? -1 : 1;",
     "if (x->key != y->key) return x->key < y->key ? 1 : -1;"),
    ("mis_threshold_not_strict",
     "sol[j] = x[j] > T ? 1 : 0;",
     "sol[j] = x[j] >= T ? 1 : 0;"),
    ("region_growing_last_label_first",
     "                lab[t] = (int32_t)ks[k - 1].idx;",
     "                lab[t] = (int32_t)ks[0].idx;"),
    ("step_scale_dropped",
     "            yn = s->y[j] - s->gamma * g / L;",
     "            yn = s->y[j] - g / L;"),
    ("map_sampling_shifted_draw",
     "                        if (l < 0 && u < cum) l = a;",
     "                        if (l < 0 && u < cum - mu[a] * 0.5) l = a;"),
    ("equality_violation_signed",
     "(p->sense[i] < 0 ? ax - p->b[i] : fabs(ax - p->b[i]));",
     "(p->sense[i] < 0 ? ax - p->b[i] : ax - p->b[i]);"),
    ("prox_box_minimiser_sign",
     "        double y = yb - red / rho;",
     "        double y = yb + red / rho;"),
    ("cover_threshold_divisor",
     "            if (sm / (double)f < T) T = sm / (double)f;",
     "            if (sm < T) T = sm;"),
    ("subset_sum_skips_largest",
     "            for (int64_t t = B - 1; t >= a; --t) if (reach[t - a]) reach[t] = 1;",
     "            for (int64_t t = B - 2; t >= a; --t) if (reach[t - a]) reach[t] = 1;"),
    ("block_gradient_drops_beta",
     "        s->g[i] = s->ctil[j] + s->beta * dot + s->rho * (s->y[j] - s->ybar[j]);",
     "        s->g[i] = s->ctil[j] + dot + s->rho * (s->y[j] - s->ybar[j]);"),
    ("cover_completion_smallest_x",
     "if (xt[j] > bx) { bx = xt[j]; pickc = j; ba = p->val[e]; }",
     "if (bx < 0.0 || xt[j] < bx) { bx = xt[j]; pickc = j; ba = p->val[e]; }"),
    ("mis_alteration_keeps_one_end",
     "if (pick[a] && pick[b]) { drop[a] = 1; drop[b] = 1; }",
     "if (pick[a] && pick[b]) { drop[a] = 1; }"),
    ("cut_cost_not_halved",
     "            cst *= 0.5;     /* each (edge,label) pair owns two rows */",
     ""),
    ("penalty_prox_term_doubled",
     "            double d = s->y[j] - s->ybar[j];\n            f += 0.5 * s->rho * d * d;",
     "            double d = s->y[j] - s->ybar[j];\n            f += s->rho * d * d;"),
    ("uniform_schedule_never_draws_the_last_unit",
     "(uint64_t)t, 0)) * (double)U);",
     "(uint64_t)t, 0)) * (double)(U - 1));"),
    ("perm_schedule_keeps_the_identity",
     "            ks[t].key = ph_word(s->seed, ST_PERM, (uint64_t)s->epoch, (uint64_t)t, 0);",
     "            ks[t].key = (uint64_t)t;"),
    ("lp_dual_block_ignores_fixed_label",
     "            if (p->fixed[t] >= 0 && i != p->fixed[t]) continue;\n            int64_t j = p->bfirst[t] + i;\n            double red = p->c[j];\n            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red -= p->cval[e] * u[p->ridx[e]];\n            if (red < best) best = red;",
     "            int64_t j = p->bfirst[t] + i;\n            double red = p->c[j];\n            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red -= p->cval[e] * u[p->ridx[e]];\n            if (red < best) best = red;"),
    ("lp_dual_unclipped_multiplier",
     "        double ui = s->ubar[i];\n        if (p->sense[i] > 0 && ui < 0.0) ui = 0.0;",
     "        double ui = s->ubar[i];\n        if (0 && p->sense[i] > 0 && ui < 0.0) ui = 0.0;"),
    ("map_energy_pair_transposed",
     "(int64_t)lab[p->pw_ends[2 * e]] * p->k + lab[p->pw_ends[2 * e + 1]]",
     "(int64_t)lab[p->pw_ends[2 * e + 1]] * p->k + lab[p->pw_ends[2 * e]]"),
    ("recomputed_residual_slack_sign",
     "        if (p->sense[i] > 0) acc -= s->y[p->n + i];\n        else if (p->sense[i] < 0) acc += s->y[p->n + i];\n        s->r[i] = acc - p->b[i];",
     "        if (p->sense[i] > 0) acc += s->y[p->n + i];\n        else if (p->sense[i] < 0) acc -= s->y[p->n + i];\n        s->r[i] = acc - p->b[i];"),
    ("mis_keep_draw_other_counter",
     "                pick[j] = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)j, 0)) < xt ? 1 : 0;\n                drop[j] = 0;\n            }\n            for (int64_t i = 0; i < m; ++i) {\n                int32_t a",
     "                pick[j] = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)j, 5)) < xt ? 1 : 0;\n                drop[j] = 0;\n            }\n            for (int64_t i = 0; i < m; ++i) {\n                int32_t a"),
    ("region_growing_radius_other_counter",
     "double rad = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, 0, 1));",
     "double rad = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, 1, 1));"),
    ("packing_alpha_not_relative",
     "            double v = (ax - p->b[i]) / p->b[i];\n            if (v > alpha) alpha = v;",
     "            double v = ax - p->b[i];\n            if (v > alpha) alpha = v;"),
    ("packing_alteration_capacity_two",
     "                    if (tot > 1.0) drop[j] = 1;",
     "                    if (tot > 2.0) drop[j] = 1;"),
    ("covering_alpha_ignores_q",
     "double alpha = isinf(q) ? 0.0 : eps / q;",
     "double alpha = isinf(q) ? 0.0 : eps;"),
    ("global_lmax_not_the_maximum",
     "        if (s->L[t] > s->Lmax) s->Lmax = s->L[t];\n    }\n    return s;",
     "        if (t == 0) s->Lmax = s->L[t];\n    }\n    return s;"),
    ("colouring_ignores_earlier_conflicts",
     "                    if (o >= 0 && o < t) stamp[p->ucolour[o]] = t;",
     "                    if (o >= 0 && o < t - 1) stamp[p->ucolour[o]] = t;"),
    ("map_argmax_ties_to_higher_label",
     "for (int32_t a = 1; a < k; ++a) if (mu[a] > mu[l]) l = a;",
     "for (int32_t a = 1; a < k; ++a) if (mu[a] >= mu[l]) l = a;"),
]


def run_mutant(tmp_path, name, old, new):
    """Builds one mutant and runs the pins against it in a child process;
    returns None when a pin failed, else a description of the survival."""
    src = open(SRC).read()
    if src.count(old) != 1:
        return f"{name}: mutation site not unique"
    d = tmp_path / name
    d.mkdir()
    mutated = d / "thetis_oracle_mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = d / "liborc_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-o",
                           str(lib), str(mutated), "-lm"])
    env = dict(os.environ, THETIS_ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                          *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # 0: every pin passed (the mistake survived); 2-5: the run itself broke
    if res.returncode in (0, 2, 3, 4, 5):
        return f"{name}: rc {res.returncode}\n{res.stdout[-1500:]}"
    return None


def test_pins_catch_every_planted_mistake(tmp_path):
    """The mutants run side by side (one child process each)."""
    import concurrent.futures as cf
    workers = max(1, min(8, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as pool:
        out = list(pool.map(lambda m: run_mutant(tmp_path, *m), MUTANTS))
    survivors = [o for o in out if o is not None]
    assert not survivors, "\n\n".join(survivors)
