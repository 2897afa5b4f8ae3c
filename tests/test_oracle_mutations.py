"""Each plausible mistake planted in a copy of the oracle's C source must make
at least one pin fail.  The mistakes are planted on the CPU, in a temporary
copy; the committed oracle is never modified."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
import tests.test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fsp_oracle.c")

# (name, original text, mistaken text)
MUTATIONS = [
    ("head_drops_machine0_term", "r[k] = F[k] > e ? F[k] : e;", "r[k] = F[k];"),
    ("head_includes_machine_k", "for (int h = 0; h < k; ++h) before", "for (int h = 0; h <= k; ++h) before"),
    ("tail_dropped", "int64_t v = tl + q[l];", "int64_t v = tl;"),
    ("tail_includes_machine_l", "for (int h = l + 1; h < m; ++h) after", "for (int h = l; h < m; ++h) after"),
    ("lag_dropped", "int64_t arrive = tk + lag_of(p, m, j, k, l);", "int64_t arrive = tk;"),
    ("lag_after_machine_l", "tl = (tl > arrive ? tl : arrive) + p[j * m + l];",
     "tl = (tl > tk ? tl : tk) + p[j * m + l] + (arrive - tk);"),
    ("johnson_second_group_ascending", "return u->b > v->b ? -1 : 1;", "return u->b < v->b ? -1 : 1;"),
    ("johnson_first_group_descending", "return u->a < v->a ? -1 : 1;", "return u->a > v->a ? -1 : 1;"),
    ("johnson_unshifted_times", "rec[i].a = p[j * m + k] + L;", "rec[i].a = p[j * m + k];"),
    ("front_drops_max", "int64_t s = c[k] > c[k - 1] ? c[k] : c[k - 1];", "int64_t s = c[k - 1];"),
    ("adjacent_pairs_only", "for (int l = k + 1; l < m; ++l, ++pi) {",
     "for (int l = k + 1; l < m && l <= k + 1; ++l, ++pi) {"),
    ("tk_starts_at_front", "int64_t tk = r[k], tl = r[l];", "int64_t tk = F[k], tl = r[l];"),
    ("tl_starts_at_head_k", "int64_t tk = r[k], tl = r[l];", "int64_t tk = r[k], tl = r[k];"),
    ("complete_node_wrong_machine", "return F[m - 1];\n  }\n\n  /* Step 3", "return F[m > 1 ? m - 2 : 0];\n  }\n\n  /* Step 3"),
    ("prune_rule_inverted", "return rule == 1 ? (lb <= ub) : (lb < ub);", "return rule == 1 ? (lb < ub) : (lb <= ub);"),
    ("leaf_accepts_ties", "if (clb < ub) {\n          ub = clb;", "if (clb <= ub) {\n          ub = clb;"),
    ("duplicate_ids_accepted", "if (j >= n || used[j]) return ORC_INVALID;", "if (j >= n) return ORC_INVALID;"),
    ("one_machine_tail_dropped", "const int64_t v = head + work + min_after;",
     "const int64_t v = head + work;"),
    ("one_machine_head_ignores_front", "if (front[h] > head) head = front[h];", ""),
    ("one_machine_head_includes_machine_h", "if (g < h) before += p[job * m + g];",
     "if (g <= h) before += p[job * m + g];"),
    ("neh_total_ascending", "while (b >= 0 && (tot[idx[b]] < tot[x] ||",
     "while (b >= 0 && (tot[idx[b]] > tot[x] ||"),
    ("neh_tie_larger_id_first", "(tot[idx[b]] == tot[x] && idx[b] > x))) {",
     "(tot[idx[b]] == tot[x] && idx[b] < x))) {"),
    ("neh_latest_position_on_ties", "if (best < 0 || c < best) {\n        best = c;\n        best_pos = pos;",
     "if (best < 0 || c <= best) {\n        best = c;\n        best_pos = pos;"),
    ("bnb_leaves_not_counted", "st->leaves++;", ""),
    ("bnb_leaf_not_counted_pruned", "memcpy(perm_out, child + 1, (size_t)n);\n          st->found = 1;\n        } else {\n          st->nodes_pruned++;",
     "memcpy(perm_out, child + 1, (size_t)n);\n          st->found = 1;\n        } else {\n          (void)0;"),
    ("bnb_root_not_counted_branched", "st->nodes_branched++;", "if (d > 0) st->nodes_branched++;"),
    ("bnb_pruned_root_not_counted", "  } else {\n    st->nodes_pruned++;\n  }\n  uint8_t child",
     "  } else {\n    (void)0;\n  }\n  uint8_t child"),
    ("bnb_unkept_child_not_counted", "        ++nk;\n      } else {\n        st->nodes_pruned++;",
     "        ++nk;\n      } else {\n        (void)0;"),
    ("one_machine_largest_tail", "if (min_after < 0 || after < min_after) min_after = after;",
     "if (min_after < 0 || after > min_after) min_after = after;"),
    # the per-depth choice of bound
    ("choice_bounds_swapped", "    return orc_lower_bound_one_machine(p, n, m, node);\n  return orc_lower_bound(p, n, m, node);",
     "    return orc_lower_bound(p, n, m, node);\n  return orc_lower_bound_one_machine(p, n, m, node);"),
    ("choice_depth_off_by_one", "((lb1_mask[d >> 5] >> (d & 31)) & 1u)",
     "((lb1_mask[(d + 1) >> 5] >> ((d + 1) & 31)) & 1u)"),
    ("choice_mask_ignored", "  if (lb1_mask && d > 0 && d < n &&", "  if (0 && lb1_mask && d > 0 && d < n &&"),
]

PINS = [
    pins.test_makespan_equals_heaviest_lattice_path,
    pins.test_johnson_order_is_a_johnson_sequence,
    pins.test_two_machines_root_bound_is_optimum,
    pins.test_two_machines_every_node_bound_is_best_completion,
    pins.test_bound_never_exceeds_any_completion,
    pins.test_exact_with_zero_or_one_job_left,
    pins.test_identical_jobs_closed_form,
    pins.test_bound_is_monotone_along_branches,
    pins.test_pair_values_equal_relaxation_optimum,
    pins.test_malformed_nodes_bound_to_minus_one,
    pins.test_bnb_tiny_config_nine_jobs_five_machines,
    pins.test_one_machine_bound_never_exceeds_the_pair_bound,
    pins.test_one_machine_bound_never_exceeds_any_completion,
    pins.test_one_machine_bound_exact_with_zero_or_one_job_left,
    pins.test_one_machine_bound_identical_jobs_closed_form,
    pins.test_identical_jobs_search_counters_closed_form,
]


def _run_pins():
    failed = []
    for f in PINS:
        try:
            f(O)
        except AssertionError:
            failed.append(f.__name__)
    for case in pins._bound_cases():
        try:
            pins.test_hand_worked_examples(O, case)
        except AssertionError:
            failed.append("hand:" + case["name"])
    for case in pins._neh_cases():
        try:
            pins.test_hand_worked_neh(O, case)
        except AssertionError:
            failed.append("neh:" + case["name"])
    for rule in (0, 1):
        try:
            pins.test_critical_tree_is_order_independent(O, rule)
        except AssertionError:
            failed.append("critical_tree_%d" % rule)
        try:
            pins.test_critical_tree_with_the_bound_chosen_per_depth(O, rule)
        except AssertionError:
            failed.append("critical_tree_choice_%d" % rule)
    return failed


@pytest.mark.parametrize("name,orig,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor not found: " + name
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "mut.c")
        so = os.path.join(td, "libmut.so")
        open(c, "w").write(src.replace(orig, bad))
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread",
                               "-o", so, c])
        O.use_library(so)
        try:
            failed = _run_pins()
        finally:
            O.use_library(None)
    assert failed, "no pin caught the planted mistake " + name
