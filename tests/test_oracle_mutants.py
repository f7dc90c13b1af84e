"""Planted mistakes: each copy of the oracle's C source with one plausible
mistake (a wrong increment, a transposed operand, a dropped term, a wrong
comparison, a dropped push, a forbidden set taken over the wrong neighbours)
must fail at least one of the named pins in tests/test_oracle_pins.py --
pins that come from brute force, closed forms, library routines or
hand-worked fixtures, not from the C file.  Each mutant is compiled into a
temporary library and the pins run in a child pytest process against it
(ATOS_ORACLE_LIB), under a time limit: a mutant that no longer terminates
also counts as caught."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "atos_oracle.c")

# (name, text in the source, replacement, pins expected to catch it)
MUTANTS = [
    ("bfs_increment", "depth[w] = depth[u] + 1;", "depth[w] = depth[u] + 2;",
     "bfs_brute_force_all_graphs or bfs_closed_forms"),
    ("jacobi_transposed", "acc += x[cols[e]] * inv_deg[cols[e]];", "acc += x[cols[e]] * inv_deg[v];",
     "pagerank_vs_linear_solve_tiny or pagerank_star_closed_form"),
    ("jacobi_no_teleport", "double nv = (1.0 - lambda) * teleport + lambda * acc;",
     "double nv = lambda * acc;",
     "pagerank_isolated_vertices or pagerank_star_closed_form or golden_fixtures"),
    ("greedy_skips_colour", "while (mark[c] == v + 1) ++c;", "while (mark[c] == v + 1) c += 2;",
     "greedy_matches_networkx or greedy_closed_forms"),
    ("push_bsp_counts_pops_as_pushes", "pushes += d;", "pushes += 1;",
     "push_bsp_first_round_counts or push_bsp_star_hand_worked"),
    ("push_bsp_non_strict_filter", "if (residue[v] > epsilon) frontier[fsize++] = (int32_t)v;",
     "if (residue[v] >= epsilon) frontier[fsize++] = (int32_t)v;",
     "push_bsp_star_hand_worked"),
    ("push_bsp_share_by_receiver", "for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) residue[cols[e]] += share;",
     "for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) residue[cols[e]] += share * (double)d / (double)(offsets[cols[e] + 1] - offsets[cols[e]]);",
     "push_bsp_star_hand_worked or push_bsp_single_edge"),
    ("push_bsp_init_scatter_by_receiver",
     "residue[cols[e]] += (1.0 - lambda) * lambda / (double)d;",
     "residue[cols[e]] += (1.0 - lambda) * lambda / (double)(offsets[cols[e] + 1] - offsets[cols[e]]);",
     "push_bsp_star_hand_worked"),
    ("fifo_forbids_every_neighbour", "if (w == v || color[w] < 0 || !outranks(key, w, v)) continue;",
     "if (w == v || color[w] < 0) continue;", "color_fifo_hand_traced"),
    ("fifo_drops_loser_push", "                    } else if (!queued[w]) {\n                        queued[w] = 1;\n                        PUSH(2 * w);\n                    }",
     "                    }", "color_fifo_hand_traced"),
    ("fifo_winner_recolours", "                    if (outranks(key, w, v)) {\n                        lost = 1;",
     "                    if (!outranks(key, w, v)) {\n                        lost = 1;",
     "color_fifo_hand_traced or color_fifo_complete_graph"),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, pins):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"{name}: the mutated text must occur exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle.build(str(src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ATOS_ORACLE_LIB=lib)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins]
    try:
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=20)
    except subprocess.TimeoutExpired:
        return  # the mutant no longer terminates: caught
    assert "no tests ran" not in r.stdout, r.stdout[-2000:]
    assert r.returncode != 0, f"{name} was not caught by [{pins}]:\n{r.stdout[-2000:]}"


def test_unmutated_source_passes_the_same_pins(tmp_path):
    lib = oracle.build(SRC, str(tmp_path / "libsame.so"))
    env = dict(os.environ, ATOS_ORACLE_LIB=lib)
    pins = " or ".join(sorted({p for m in MUTANTS for p in m[3].split(" or ")}))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:]
