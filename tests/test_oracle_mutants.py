"""Mutation check of the oracle pins.

Each case plants one plausible mistake (a dropped term, a wrong index or
comparison, a swapped operand) in a private copy of oracle/oracle.c, builds
it with gcc on the CPU, and requires that the pin battery of
tests/test_oracle_pins.py rejects the mutant.  The real oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

import oracle
import test_oracle_pins as pins
import test_oracle_pins_next as nxt

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = [
    ("csr keeps duplicates", "if (i > 0 && pairs[i] == pairs[i - 1]) continue;", "(void)0;"),
    ("csr keeps self-loops", "    if (u == v) continue;\n    pairs[np++]", "    pairs[np++]"),
    ("bfs depth off by one", "depth[v] = du + 1;", "depth[v] = du + 2;"),
    ("bfs parent is self", "parent[v] = u;\n        queue[tail++] = v;",
     "parent[v] = v;\n        queue[tail++] = v;"),
    ("bfs m_comp extra term", "mc += off[u + 1] - off[u];", "mc += off[u + 1] - off[u] + 1;"),
    ("do: P excludes Q", "lhs_common *= (uint64_t)p;", "lhs_common *= (uint64_t)(p - q);"),
    ("do: non-strict switch", "if (!switched && lhs_common * a_den > rhs_common * a_num)",
     "if (!switched && lhs_common * a_den >= rhs_common * a_num)"),
    ("do: switch allowed twice", "switched = 1;\n        }\n      } else {\n        if (lhs_common",
     "switched = 0;\n        }\n      } else {\n        if (lhs_common"),
    ("do: num/den swapped", "lhs_common * a_den > rhs_common * a_num",
     "lhs_common * a_num > rhs_common * a_den"),
    ("do: pull tie switches", "if (lhs_common * b_den < rhs_common * b_num) cur = 0;",
     "if (lhs_common * b_den <= rhs_common * b_num) cur = 0;"),
    ("edges read: exit position", "cnt += j + 1;", "cnt += j;"),
    ("edges read: candidate set", "if (depth[v] != -1 && depth[v] <= k) continue;",
     "if (depth[v] != -1 && depth[v] < k) continue;"),
    ("dijkstra ignores weight", "uint64_t nd = d[u] + (uint64_t)w[e];", "uint64_t nd = d[u] + 1;"),
    ("dijkstra largest tight parent", "(parent[v] == -1 || u < parent[v])",
     "(parent[v] == -1 || u > parent[v])"),
    ("floyd-warshall skips last pivot", "for (int32_t k = 0; k < n; ++k)\n    for (int32_t i = 0; i < n; ++i) {",
     "for (int32_t k = 0; k < n - 1; ++k)\n    for (int32_t i = 0; i < n; ++i) {"),
    ("bfs checker loose", "(a - b > 1 || b - a > 1)", "(a - b > 2 || b - a > 2)"),
    ("sssp checker loose", "if ((uint64_t)dist[v] > nd)", "if ((uint64_t)dist[v] > nd + 1)"),
    ("package local test", "if (v < n_local) {", "if (v <= n_local) {"),
    ("package sends local id", "ids_out[slot] = conv[v];", "ids_out[slot] = v;"),
    ("share conv is local id", "lconv[g2l[v]] = rank[v];", "lconv[g2l[v]] = g2l[v];"),
    ("partitioned combine drops new", "if (S->label[v] == -1 || rlab[q][i] < S->label[v])",
     "if (rlab[q][i] < S->label[v])"),
    ("dupall backward tests level k-1", "if (L[col[e]] == k) {", "if (L[col[e]] == k - 1) {"),
    ("dupall backward keeps scanning", "              nl[p][nlen[p]++] = v;\n              break;",
     "              nl[p][nlen[p]++] = v;"),
    ("dupall forward skips hosted rows", "if (owner[u] != p) continue;",
     "if (owner[u] == p) continue;"),
    ("dupall no broadcast", "if (label[p][v] == -1) label[p][v] = k + 1;", "(void)0;"),
    ("dupall per-partition edge count", "unsigned __int128 lhs = (unsigned __int128)(uint64_t)qlen * (uint64_t)m;",
     "unsigned __int128 lhs = (unsigned __int128)(uint64_t)qlen * (uint64_t)(m / nparts);"),
    ("dupall pull twice", "          cur = 1;\n          switched = 1;\n        }\n      } else if (lhs * b_den",
     "          cur = 1;\n        }\n      } else if (lhs * b_den"),
    ("cc labels with the last vertex", "label[v] = s;\n          queue[tail++] = v;",
     "label[v] = v > s ? v : s;\n          queue[tail++] = v;"),
    ("cc scans descending", "for (int32_t s = 0; s < n; ++s) {\n    if (label[s] != -1) continue;",
     "for (int32_t s = n - 1; s >= 0; --s) {\n    if (label[s] != -1) continue;"),
    ("pagerank divides by receiver degree", "double share = rank[u] / (double)deg;",
     "double share = rank[u] / (double)(off[u + 2 < n + 1 ? u + 2 : n] - off[u + 1] + 1);"),
    ("pagerank teleport not divided by n", "double nr = (1.0 - d) / (double)n + d * acc[v];",
     "double nr = (1.0 - d) + d * acc[v];"),
    ("pagerank undamped accumulation", "double nr = (1.0 - d) / (double)n + d * acc[v];",
     "double nr = (1.0 - d) / (double)n + acc[v];"),
    ("pagerank threshold on new rank", "if (diff > tol * rank[v]) converged = 0;",
     "if (diff > tol) converged = 0;"),
]


def battery(orc):
    pins.test_csr_golden(orc)
    pins.test_csr_matches_scipy_and_synth(orc, 8)
    pins.test_bfs_path_closed_form(orc)
    pins.test_bfs_grid_manhattan(orc, (7, 5))
    pins.test_bfs_star_complete_isolated_disconnected(orc)
    pins.test_bfs_vs_floyd_warshall_and_matrix_powers(orc, 0)
    pins.test_do_schedule_golden(orc)
    pins.test_do_schedule_extremes(orc)
    pins.test_edges_inspected_golden(orc)
    pins.test_sssp_golden_diamond(orc)
    pins.test_sssp_path_prefix_sums_and_grid(orc)
    pins.test_sssp_vs_floyd_warshall_and_scipy(orc, 0)
    pins.test_checkers_reject_planted_errors(orc)
    pins.test_share_build_golden(orc)
    pins.test_package_golden(orc)
    pins.test_partitioned_bfs_equals_bfs(orc, 4)
    nxt.test_dupall_golden(orc)
    nxt.test_dupall_equals_bfs_and_schedule(orc, 1)
    nxt.test_dupall_equals_bfs_and_schedule(orc, 3)
    nxt.test_dupall_closed_forms(orc)
    nxt.test_cc_golden_and_isolated(orc)
    nxt.test_cc_matches_scipy_and_reachability(orc, 1)
    nxt.test_cc_rmat_and_grid(orc)
    nxt.test_pagerank_regular_graphs_stay_uniform(orc)
    nxt.test_pagerank_star_closed_form(orc)
    nxt.test_pagerank_matches_dense_iteration_and_solve(orc, 0)
    nxt.test_pagerank_threshold_stops_when_all_updates_small(orc)


def test_battery_passes_on_real_oracle(orc):
    battery(orc)


_CHILD = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, test_oracle_mutants as t
t.battery(oracle.Oracle(oracle.load({so!r})))
"""


def run_battery_in_child(so):
    # A mutant may also crash (e.g. read past a row); a crash counts as a
    # rejection, so the battery runs in its own process.
    here = os.path.dirname(os.path.abspath(__file__))
    code = _CHILD.format(root=os.path.dirname(here), tests=here, so=str(so))
    return subprocess.run([sys.executable, "-c", code], capture_output=True,
                          text=True, timeout=300)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_rejected(name, old, new, tmp_path):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not unique: {old!r}"
    src = tmp_path / "oracle_mut.c"
    src.write_text(text.replace(old, new))
    so = tmp_path / "liborc_mut.so"
    subprocess.check_call(oracle.build_cmd(str(src), str(so)))
    r = run_battery_in_child(so)
    assert r.returncode != 0, f"mutant '{name}' survived the pins"
