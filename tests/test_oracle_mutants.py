"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle (its C source or its
Python compositions), rebuilds the copy and runs the pins of that part of
the oracle against it; the pins must fail.  The mistakes are the kind a
reader could make when writing the definitions out: a dropped neighbour, a
wrong index, a flipped clamp, a border off by one, a wrong step count,
other tie rules, a wrong gradient route or scale, and in the compositions
a wrong h, reversed differences, a wrong border marker, the wrong
reconstruction direction, wrapping u8 arithmetic, wrong QDT updates and
wrong granulometry sums.  Runs on the CPU, several copies at a time."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

PINS = "tests/test_oracle_pins.py"
OPS = "tests/test_oracle_operators.py"
QDT = "tests/test_oracle_qdt.py"
GRAN = "tests/test_oracle_granulometry.py"

# (name, file in oracle/, text, replacement, occurrence (1-based), pin file)
MUTANTS = [
    ("dropped_neighbour", "oracle.c", "for (int64_t dx = -1; dx <= 1; ++dx) {\n            int64_t xx = x + dx;\n"
     "            if (xx < 0 || xx >= X) continue;\n            double v = f[yy * X + xx];\n            if (better",
     "for (int64_t dx = -1; dx <= 0; ++dx) {\n            int64_t xx = x + dx;\n"
     "            if (xx < 0 || xx >= X) continue;\n            double v = f[yy * X + xx];\n            if (better", 1, PINS),
    ("mirrored_column_index", "oracle.c", "double v = f[yy * X + xx];\n            if (better(op, v, best)) best = v;",
     "double v = f[yy * X + (X - 1 - xx)];\n            if (better(op, v, best)) best = v;", 1, PINS),
    ("clamp_sign", "oracle.c", "if (op == ORACLE_DILATE) return m[i] < v ? m[i] : v;",
     "if (op == ORACLE_DILATE) return m[i] > v ? m[i] : v;", 1, PINS),
    ("border_off_by_one", "oracle.c", "if (xx < 0 || xx >= X) continue;\n            double v = f[yy * X + xx];\n"
     "            if (better", "if (xx < 0 || xx >= X - 1) continue;\n            double v = f[yy * X + xx];\n"
     "            if (better", 1, PINS),
    ("chain_one_step_short", "oracle.c", "for (int64_t t = 0; t < n; ++t) {\n        oracle_step",
     "for (int64_t t = 0; t + 1 < n; ++t) {\n        oracle_step", 1, PINS),
    ("reconstruction_counts_last_step", "oracle.c", "if (changed == 0) { status = 0; break; }",
     "if (changed == 0) { status = 0; ++count; break; }", 1, PINS),
    ("last_extremum_wins_ties", "oracle.c", "if (!found || better(op, v, best)) {",
     "if (!found || !better(op, best, v)) {", 1, PINS),
    ("neighbourhood_wins_mask_ties", "oracle.c", "(m[i] <= best) : (m[i] >= best)",
     "(m[i] < best) : (m[i] > best)", 1, PINS),
    ("gradient_not_routed", "oracle.c", "gp[(y + dy) * X + (x + dx)] += g[i];", "gp[y * X + x] += g[i]; (void)dy; (void)dx;",
     1, PINS),
    ("mask_gradient_scale", "oracle.c", "if (g_mask) g_mask[i] += g[i];", "if (g_mask) g_mask[i] += 2 * g[i];", 1, PINS),
    ("hmax_wrong_h", "__init__.py", "_sub_in_dtype(f, _h_in_dtype(f.dtype, h))",
     "_sub_in_dtype(f, _h_in_dtype(f.dtype, h + 1))", 1, OPS),
    ("dome_reversed_difference", "__init__.py", "return _sub_in_dtype(f, r), steps, conv", "return _sub_in_dtype(r, f), steps, conv",
     1, OPS),
    ("hfill_border_fill_swapped", "__init__.py", "_border_marker(f, f.max())", "_border_marker(f, f.min())", 1, OPS),
    ("border_marker_missing_column", "__init__.py", "    m[:, -1] = f[:, -1]\n", "", 1, OPS),
    ("raobj_wrong_direction", "__init__.py", "reconstruct(DILATE, _border_marker(f, f.min()), f, max_steps)",
     "reconstruct(ERODE, _border_marker(f, f.min()), f, max_steps)", 1, OPS),
    ("open_rec_dilated_marker", "__init__.py", "return reconstruct(DILATE, chain(ERODE, f, int(s)), f, max_steps)",
     "return reconstruct(DILATE, chain(DILATE, f, int(s)), f, max_steps)", 1, OPS),
    ("open_rec_one_erosion_too_many", "__init__.py", "return reconstruct(DILATE, chain(ERODE, f, int(s)), f, max_steps)",
     "return reconstruct(DILATE, chain(ERODE, f, int(s) + 1), f, max_steps)", 1, OPS),
    ("u8_subtraction_wraps", "__init__.py", "return np.maximum(d, 0).astype(np.uint8)", "return d.astype(np.uint8)", 1, OPS),
    ("qdt_ties_take_later_step", "__init__.py", "upd = res > r", "upd = res >= r", 1, QDT),
    ("qdt_distance_off_by_one", "__init__.py", "d[upd] = j\n", "d[upd] = j - 1\n", 1, QDT),
    ("qdt_eta_plus_two", "__init__.py", "np.where(g - e > 1, e + 1, g)", "np.where(g - e > 1, e + 2, g)", 1, QDT),
    ("qdt_no_eta", "__init__.py", "np.where(g - e > 1, e + 1, g)", "g", 1, QDT),
    ("qdt_residual_against_input", "__init__.py", "res = _sub_in_dtype(cur, nxt)", "res = _sub_in_dtype(f, nxt)", 1, QDT),
    ("qdt_dilation_for_erosion", "__init__.py", "nxt = step(ERODE, cur)", "nxt = step(DILATE, cur)", 1, QDT),
    ("granulometry_closing_for_opening", "__init__.py", "math.fsum(opening(f, s)", "math.fsum(closing(f, s)", 1, GRAN),
    ("pattern_spectrum_sign", "__init__.py", "return G, G[:-1] - G[1:]", "return G, G[1:] - G[:-1]", 1, GRAN),
    ("opening_extra_dilation", "__init__.py", "return chain(DILATE, chain(ERODE, f, int(s)), int(s))",
     "return chain(DILATE, chain(ERODE, f, int(s)), int(s) + 1)", 1, GRAN),
    ("asf_closing_first", "__init__.py", "g = closing(opening(g, s), s)", "g = opening(closing(g, s), s)", 1, GRAN),
    ("granulometry_skips_g0", "__init__.py", "for s in range(int(s_max) + 1)])", "for s in range(1, int(s_max) + 2)])",
     1, GRAN),
]


def plant(workdir, fname, old, new, occurrence):
    pkg = os.path.join(workdir, "oracle")
    shutil.copytree(ORACLE, pkg, ignore=shutil.ignore_patterns("__pycache__", "*.tmp"))
    path = os.path.join(pkg, fname)
    text = open(path).read()
    assert text.count(old) >= occurrence, f"{fname}: text to replace not found"
    idx = -1
    for _ in range(occurrence):
        idx = text.index(old, idx + 1)
    open(path, "w").write(text[:idx] + new + text[idx + len(old):])
    if fname.endswith(".c"):
        subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-w", "-o",
                        os.path.join(pkg, "liboracle.so"), path], check=True, timeout=120)
    return pkg


def run_pins(workdir, pin_file):
    env = dict(os.environ, ORACLE_PACKAGE_DIR=workdir, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        pin_file], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_planted_mistakes_fail_the_pins(tmp_path):
    if not os.path.exists(os.path.join(ORACLE, "liboracle.so")):
        from oracle import build
        build.build()

    def one(m):
        name, fname, old, new, occ, pin_file = m
        work = str(tmp_path / name)
        os.makedirs(work)
        plant(work, fname, old, new, occ)
        rc, out = run_pins(work, pin_file)
        return name, rc, out

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(one, MUTANTS))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    broken = [(n, rc, out) for n, rc, out in results if rc not in (0, 1)]
    assert not broken, f"mutant runs that did not run their pins: {broken}"
    assert not survivors, f"planted mistakes that every pin accepted: {[n for n, _ in survivors]}"


def test_unmodified_copy_passes_the_pins(tmp_path):
    """The copy mechanism itself: an unmodified copy passes every pin file."""
    work = str(tmp_path / "identity")
    os.makedirs(work)
    plant(work, "oracle.c", "enum { ORACLE_DILATE", "enum { ORACLE_DILATE", 1)
    for pin_file in (PINS, OPS, QDT, GRAN):
        rc, out = run_pins(work, pin_file)
        assert rc == 0, out


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_text_is_present(mutant):
    """Every planted mistake still applies to the current oracle source."""
    _, fname, old, _, occ, _ = mutant
    assert open(os.path.join(ORACLE, fname)).read().count(old) >= occ
