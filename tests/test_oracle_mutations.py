"""The oracle's pins catch plausible mistakes.

Each case plants one mistake -- a dropped term, a wrong sign, power, factor
or index, an operand of the wrong body -- in a copy of the oracle (on the
CPU, in a temporary directory; the oracle in the tree is never touched),
then runs tests/test_oracle_pins.py against that copy: at least one pin must
fail.  A mutant that every pin accepted would mark a gap in the pins.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what the mistake is, file under oracle/, text, replacement, occurrence)
MUTANTS = [
    ("softening dropped from r^2", "nbody_oracle.c",
     "double s = dx * dx + dy * dy + dz * dz + eps2;",
     "double s = dx * dx + dy * dy + dz * dz;", 1),
    ("s^-1 instead of s^-3/2", "nbody_oracle.c",
     "double inv_s32 = 1.0 / (s * sqrt(s));", "double inv_s32 = 1.0 / s;", 1),
    ("G left out", "nbody_oracle.c", "out[0] = G * ax;", "out[0] = ax;", 1),
    ("pair difference reversed", "nbody_oracle.c",
     "double dx = px[j] - xi[0];", "double dx = xi[0] - px[j];", 1),
    ("full kick instead of half", "nbody_oracle.c",
     "      v[q] = v[q] + half * acc[q];\n      x[q]",
     "      v[q] = v[q] + dt * acc[q];\n      x[q]", 1),
    ("closing half-kick dropped", "nbody_oracle.c",
     "for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q] + half * acc[q];",
     "for (int64_t q = 0; q < 3 * n; ++q) v[q] = v[q];", 1),
    ("VJP: h with the wrong sign", "nbody_oracle.c",
     "double hx = mk * gx[j] - m[j] * gxk;", "double hx = mk * gx[j] + m[j] * gxk;", 1),
    ("VJP: factor 3 of s^-5/2 wrong", "nbody_oracle.c",
     "sx += s32 * hx - 3.0 * s52 * eh * ex;", "sx += s32 * hx - 2.0 * s52 * eh * ex;", 1),
    ("VJP: dL/dm sign", "nbody_oracle.c", "*gm_out = -G * sm;", "*gm_out = G * sm;", 1),
    ("VJP: target's gradient used for the source's", "nbody_oracle.c",
     "double ge = gx[j] * ex + gy[j] * ey + gz[j] * ez;",
     "double ge = gxk * ex + gyk * ey + gzk * ez;", 1),
    ("adjoint: dt/2 instead of dt in vbar", "nbody_oracle.c",
     "gv[q] = gv[q] + dt * gx[q];", "gv[q] = gv[q] + half * gx[q];", 1),
    ("adjoint: VJP at x_t instead of x_t+1", "nbody_oracle.c",
     "oracle_accel_vjp(n, traj + (size_t)(t + 1) * q3,",
     "oracle_accel_vjp(n, traj + (size_t)t * q3,", 1),
    ("potential: s^-1 instead of s^-1/2", "nbody_oracle.c",
     "row += m[j] / sqrt(s);", "row += m[j] / s;", 1),
    ("kinetic energy without 1/2", "nbody_oracle.c",
     "kin += 0.5 * m[i] *", "kin += m[i] *", 1),
    ("Morton code: y and z bits swapped", "__init__.py",
     "for axis, shift in ((0, 2), (1, 1), (2, 0)):",
     "for axis, shift in ((0, 2), (1, 0), (2, 1)):", 1),
]


def _copy_tree(dst):
    for d in ("oracle", "tests", "paper_2203_08263_amd"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__",
                                                      "csrc", "valu_microbench"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)


@pytest.mark.slow
@pytest.mark.parametrize("what,fname,old,new,count", MUTANTS,
                         ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, what, fname, old, new, count):
    _copy_tree(str(tmp_path))
    path = tmp_path / "oracle" / fname
    src = path.read_text()
    assert src.count(old) >= count, "mutation target not found: %s" % what
    path.write_text(src.replace(old, new, count))
    if fname.endswith(".c"):   # the mutant must still compile
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", str(tmp_path / "probe.so"), str(path), "-lm"])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x",
                        "-p", "no:cacheprovider", "tests/test_oracle_pins.py"],
                       cwd=str(tmp_path), capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 1, "pins did not catch: %s\n%s" % (what, r.stdout[-2000:])
