"""Plant plausible mistakes in copies of the oracle and check that the pins
catch every one of them (CPU only; each mutant runs in its own process so a
mutant that crashes counts as caught without taking pytest down)."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# name -> list of (original snippet, planted replacement); every original must
# occur in flo.c, so a rewrite of the oracle makes this test fail loudly.
MUTANTS = {
    "tie_makes_edge": [("if (g->f[w] < g->f[u]) {", "if (g->f[w] <= g->f[u]) {"),
                       ("if (g->f[w] < g->f[u])\n", "if (g->f[w] <= g->f[u])\n")],
    "adjacent_is_hamming": [("g->neighbourhood == FLO_ADJACENT && llabs(a - x[i]) != 1", "0")],
    "adjacent_wraps": [("g->neighbourhood == FLO_ADJACENT && llabs(a - x[i]) != 1",
                        "g->neighbourhood == FLO_ADJACENT && llabs(a - x[i]) != 1 "
                        "&& llabs(a - x[i]) != g->radix[i] - 1")],
    "edge_reversed": [("if (g->f[w] < g->f[u]) {", "if (g->f[w] > g->f[u]) {"),
                      ("if (g->f[w] < g->f[u])\n", "if (g->f[w] > g->f[u])\n")],
    "param0_least_significant": [
        ("g->stride[i] = (i == n - 1) ? 1 : g->stride[i + 1] * g->radix[i + 1];",
         "g->stride[n - 1 - i] = (i == n - 1) ? 1 : g->stride[n - 1 - (i + 1)] * g->radix[n - 1 - (i + 1)];")],
    "no_teleport": [("(1.0 - d) * total", "0.0 * total")],
    "no_sink_spreading": [("(d * sink_mass + (1.0 - d) * total)", "((1.0 - d) * total)")],
    "sink_self_loop": [("(d * sink_mass + (1.0 - d) * total)", "((1.0 - d) * total)"),
                       ("next[w] = d * acc + spread;",
                        "next[w] = d * acc + spread + (g->out_deg[w] == 0 ? d * r[w] : 0.0);")],
    "divide_by_in_degree": [("acc += r[u] / (double)g->out_deg[u];",
                             "acc += r[u] / (double)(g->in_ptr[w + 1] - g->in_ptr[w]);")],
    "no_damping": [("next[w] = d * acc + spread;", "next[w] = acc + spread;")],
    "strict_threshold": [("(double)g->f[v] <= threshold", "(double)g->f[v] < threshold")],
    "threshold_without_one": [("(1.0 + p) * g->f_opt", "p * g->f_opt")],
    "minima_are_sources": [("g->M += (g->out_deg[v] == 0);",
                            "g->M += (g->in_ptr[v + 1] == g->in_ptr[v]);"),
                           ("if (g->out_deg[v] != 0)\n            continue;\n        g->minima[m++] = v;",
                            "if (g->in_ptr[v + 1] != g->in_ptr[v])\n            continue;\n        g->minima[m++] = v;")],
    "rows_by_raw_position_of_target": [("g->in_src[fill[w]++] = u;", "g->in_src[fill[w]++] = w;")],
    "f_opt_is_first_node": [("if ((double)g->f[v] < g->f_opt)", "if (v == 0)")],
    "zero_fitness_accepted": [("if (!isnan(v) && !(v > 0.0f))", "if (!isnan(v) && v < 0.0f)")],
    "dag_ascending_order": [("if (fa > fb) return -1;\n    if (fa < fb) return 1;",
                             "if (fa < fb) return -1;\n    if (fa > fb) return 1;")],
    "dag_without_one": [("r[w] = 1.0 + d * sum_get(&acc);", "r[w] = (w == 0) + d * sum_get(&acc);")],
    "dag_divide_by_in_degree": [("sum_add(&acc, r[u] / (double)g->out_deg[u]);",
                                 "sum_add(&acc, r[u] / (double)(g->in_ptr[w + 1] - g->in_ptr[w]));")],
    "plateau_over_all_nodes": [("for (int64_t j = 0; j < g->M; ++j)\n"
                                "        g->plateau_minima += has_equal_neighbour(g, g->minima[j], nb);",
                                "for (int64_t j = 0; j < g->N; ++j)\n"
                                "        g->plateau_minima += has_equal_neighbour(g, j, nb);")],
    "plateau_any_neighbour": [("if (g->f[g->node_of[nb[j]]] == g->f[v])\n            return 1;",
                               "if (g->f[g->node_of[nb[j]]] >= g->f[v])\n            return 1;")],
    "plateau_first_neighbour_only": [("for (int64_t j = 0; j < k; ++j)\n        if (g->f[g->node_of[nb[j]]] == g->f[v])",
                                      "for (int64_t j = 0; j < k && j < 1; ++j)\n        if (g->f[g->node_of[nb[j]]] == g->f[v])")],
    "naive_inverted": [("double q = g->f_opt / (double)g->f[g->minima[j]];",
                        "double q = (double)g->f[g->minima[j]] / g->f_opt;")],
    "naive_bins_rounded": [("int64_t b = (int64_t)floor(q * (double)n_bins);",
                            "int64_t b = (int64_t)floor(q * (double)n_bins + 0.5);")],
    "naive_over_first_nodes": [("double q = g->f_opt / (double)g->f[g->minima[j]];",
                                "double q = g->f_opt / (double)g->f[j];")],
}


def _mutant_source(tmp_path, name, edits):
    src = open(oracle.SRC).read()
    for old, new in edits:
        assert src.count(old) >= 1, f"{name}: snippet not in flo.c: {old!r}"
        src = src.replace(old, new)
    path = tmp_path / f"flo_{name}.c"
    path.write_text(src)
    return str(path)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    src = _mutant_source(tmp_path, name, MUTANTS[name])
    lib = str(tmp_path / f"lib_{name}.so")
    oracle.build(src=src, out=lib)
    code = (
        "import sys; sys.path[:0] = [%r, %r]\n"
        "import pins\n"
        "failed = pins.run_quick(%r)\n"
        "print('FAILED_CHECKS', failed)\n"
        "sys.exit(3 if failed else 0)\n" % (ROOT, HERE, lib))
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    # exit 3: some pin failed; any other non-zero exit: the mutant crashed
    assert res.returncode != 0, f"mutant {name} passed every pin:\n{res.stdout}{res.stderr}"


def test_unmutated_oracle_passes_quick_pins():
    import pins
    assert pins.run_quick(oracle.LIB) == []
