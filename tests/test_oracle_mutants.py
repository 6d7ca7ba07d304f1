"""Plants plausible mistakes in a copy of the oracle's C source and checks
that the pin tests catch every one of them.

Each mutant is compiled with gcc into a temporary library and the pin tests
run against it in a child process (``MPLP_ORACLE_LIB`` points the oracle's
loader at the mutant).  A mutant that passes all pins means the pins have a
hole; the test then fails and names the mutant.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mplp_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("mplp half dropped on u", "hu[s] = 0.5 * mn;\n    }", "hu[s] = mn;\n    }"),
    ("mplp half dropped on v", "hv[t] = 0.5 * mn;\n    }\n}", "hv[t] = mn;\n    }\n}"),
    ("row min instead of column min", "for (int s = 0; s < L; ++s) mn = fmin(mn, g[(size_t)s * L + t]);\n        hv[t] = 0.5",
     "for (int s = 0; s < L; ++s) mn = fmin(mn, g[(size_t)t * L + s]);\n        hv[t] = 0.5"),
    ("v correction drops its base", "                hv[t] = hv[t] + mn;", "                hv[t] = mn;"),
    ("u correction drops its base", "                hu[s] = hu[s] + mn;", "                hu[s] = mn;"),
    ("u corrected before v", "/* (H), second line", "/* (H), second line */ for (int s = 0; s < L; ++s) { double mn = INFINITY; for (int t = 0; t < L; ++t) mn = fmin(mn, g[(size_t)s * L + t] - hv[t] - hu[s]); hu[s] = hu[s] + mn; } /*"),
    ("wrong sign in write back", "- hu[s] - hv[t];", "- hu[s] + hv[t];"),
    ("wrong index in aggregate", "+ Tu_u[s] + Tu_v[t];", "+ Tu_u[s] + Tu_v[s];"),
    ("transposed table in aggregate", "g[(size_t)s * L + t] = Te[(size_t)s * L + t] + Tu_u[s]",
     "g[(size_t)s * L + t] = Te[(size_t)t * L + s] + Tu_u[s]"),
    ("uniform half dropped", "for (int t = 0; t < L; ++t) hv[t] = 0.5 * mn;", "for (int t = 0; t < L; ++t) hv[t] = mn;"),
    ("dual drops edge terms", "for (size_t i = 0; i < (size_t)L * L; ++i) mn = fmin(mn, T[i]);\n        d += mn;",
     "for (size_t i = 0; i < (size_t)L * L; ++i) mn = fmin(mn, T[i]);\n        d += 0.0 * mn;"),
    ("dual uses max", "for (int s = 0; s < L; ++s) mn = fmin(mn, Tu[(size_t)u * L + s]);",
     "for (int s = 0; s < L; ++s) mn = fmax(mn == INFINITY ? -INFINITY : mn, Tu[(size_t)u * L + s]);"),
    ("decode transposed table", "cost[x] += row[x];", "cost[x] += Te[(size_t)e * L * L + (size_t)x * L + labels[v]];"),
    ("decode ties to highest label", "if (cost[x] < cost[best]) best = x;", "if (cost[x] <= cost[best]) best = x;"),
    ("decode ignores neighbours", "if (edges[2 * e + 1] != u) continue;", "continue;"),
    ("energy transposed lookup", "(size_t)labels[u] * L + labels[v]];", "(size_t)labels[v] * L + labels[u]];"),
    ("energy drops unaries", "for (int u = 0; u < n; ++u) en += unaries", "for (int u = 0; u < 0; ++u) en += unaries"),
    ("circle method wrong partner", "b = ((r - k) % (N - 1)", "b = ((r - k + 1) % (N - 1)"),
    ("greedy ignores the second node", "if (!busy[u] && !busy[v]) {", "if (!busy[u]) {"),
    ("reversed input not transposed", "double x = (a < b) ? src[(size_t)s * L + t] : src[(size_t)t * L + s];",
     "double x = src[(size_t)s * L + t];"),
    ("duplicates accepted", "if (keys[e] == keys[e - 1]) { free(keys); return ORC_EINVAL; }", ""),
    ("brute force skips labellings", "while (i < n && ++y[i] == L) y[i++] = 0;", "while (i < n && (y[i] += 2) >= L) y[i++] = 0;"),
    ("colouring: d free on the fan's first node", "int d = smallest_free(k, fan[len - 1]);", "int d = smallest_free(k, fan[0]);"),
    ("colouring: no path swap", "for (int i = 0; i + 1 < np; ++i) paint(k, path[i], path[i + 1], was[i] == c ? d : c);",
     "for (int i = 0; i + 1 < np; ++i) paint(k, path[i], path[i + 1], was[i]);"),
    ("colouring: fan not rotated", "        paint(k, u, fan[i], cn);\n", "        paint(k, u, fan[i + 1], cn);\n"),
    ("tangent: MPLP half of u not halved", "dhu[s] = 0.5 * dg[(size_t)s * L + at];", "dhu[s] = dg[(size_t)s * L + at];"),
    ("tangent: second line drops u's half", "- dhv[t] - dhu[at]);", "- dhv[t]);"),
    ("tangent: third line reads v at the wrong label", "dg[(size_t)s * L + at] - dhv[at] - dhu[s]",
     "dg[(size_t)s * L + at] - dhv[s] - dhu[s]"),
    ("tangent: aggregate misses v", "aggregate(L, dTe, dTu_u, dTu_v, dg);", "aggregate(L, dTe, dTu_u, dTu_u, dg);"),
    ("tangent: tables not carried", "    write_back(L, dTe, dTu_u, dTu_v, dg, dhu, dhv);\n",
     "    for (int s = 0; s < L; ++s) { dTu_u[s] = dhu[s]; dTu_v[s] = dhv[s]; }\n"),
    ("tangent: node term at label 0", "d += dTu[(size_t)u * L + at];", "d += dTu[(size_t)u * L];"),
    ("colouring: largest colour first", "for (int c = 0; c < k->C && !grown; ++c) {", "for (int c = k->C - 1; c >= 0 && !grown; --c) {"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique/present: {name}"
    mut = src.replace(old, new)
    c = tmp_path / "mut.c"
    c.write_text(mut)
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(so),
                    str(c), "-lm"], check=True)
    env = dict(os.environ, MPLP_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_schedule.py",
                        "tests/test_oracle_derivative.py", "tests/test_oracle_plateau.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant '{name}' survived every pin:\n{r.stdout[-2000:]}"


# The mutants of the update, the dual, the energy, brute force and the
# schedule's matching property that the randomized property tests
# (test_oracle_properties.py) catch on their own, with hypothesis's search
# fixed by its seed; the others (orientation, rounding details, the exact
# schedule rule, the derivative) are pinned by the tests above only.
PROPERTY_CATCHES = [
    "mplp half dropped on u", "mplp half dropped on v", "row min instead of column min",
    "v correction drops its base", "u correction drops its base", "wrong sign in write back",
    "wrong index in aggregate", "transposed table in aggregate", "dual drops edge terms", "dual uses max",
    "energy transposed lookup", "energy drops unaries", "greedy ignores the second node", "duplicates accepted",
    "brute force skips labellings", "colouring: d free on the fan's first node", "colouring: no path swap",
    "colouring: fan not rotated",
]


@pytest.mark.slow
@pytest.mark.parametrize("name", PROPERTY_CATCHES)
def test_properties_catch_mutant(tmp_path, name):
    old, new = next((o, n) for m, o, n in MUTANTS if m == name)
    src = open(SRC).read()
    c = tmp_path / "mut.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-o", str(so),
                    str(c), "-lm"], check=True)
    env = dict(os.environ, MPLP_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--hypothesis-seed=0",
                        "tests/test_oracle_properties.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant '{name}' survived the property tests:\n{r.stdout[-2000:]}"
