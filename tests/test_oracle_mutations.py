"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU, in a temporary
directory), rebuilds it and runs the pin suite ``test_oracle.py`` against the copy. A mutant
that passes every pin would mean a gap in the pins; one no-op edit checks the harness itself.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "drift sign (d=2)": ("ell[1] = -q[0]; ell[2] = -q[1];", "ell[1] = q[0]; ell[2] = q[1];"),
    "drift sign (d=1)": ("ell[0] = tau; ell[1] = -q[0]; ell[2] = 2.0 * G[0];",
                         "ell[0] = tau; ell[1] = q[0]; ell[2] = 2.0 * G[0];"),
    "centre value not replaced": ("s->w[0] -= tau;", "s->w[0] -= 0.0 * tau;"),
    "tau factor": ("tau = (pr->variant == 0) ? 2.0 * (G[0] + G[3]) / (h * h) : 0.0;",
                   "tau = (pr->variant == 0) ? 1.0 * (G[0] + G[3]) / (h * h) : 0.0;"),
    "inverse metric off-diagonal sign": ("G12 = -g12 / det", "G12 = g12 / det"),
    "mixed derivative factor": ("ell[4] = 2.0 * G[1];", "ell[4] = 1.0 * G[1];"),
    "Hessian off-diagonal": ("H12 = ac[4]", "H12 = 2.0 * ac[4]"),
    "trace(G H) cross term": ("G11 * H11 + 2.0 * G12 * H12 + G22 * H22",
                              "G11 * H11 + G12 * H12 + G22 * H22"),
    "metric cross term dropped": ("g12 += ac[1] * ac[2];", "g12 += 0.0;"),
    "transposed operand in G grad z": ("double Gz1 = G11 * ac[1] + G12 * ac[2];",
                                       "double Gz1 = G11 * ac[1] + G12 * ac[1];"),
    "q without G": ("q1 += trGH * Gz1;", "q1 += trGH * ac[1];"),
    "h uses max": ("if (h2 < h)\n            h = h2;", "if (h2 > h)\n            h = h2;"),
    "h factor": ("double h = 0.25 * (umax[0] - umin[0]);", "double h = 0.3 * (umax[0] - umin[0]);"),
    "barycentre divisor": ("cbar[a] /= (double)K;", "cbar[a] /= (double)(K + 1);"),
    "h scaling of first derivatives": ("scale[1] = scale[2] = 1.0 / h;",
                                       "scale[1] = scale[2] = 1.0 / (h * h);"),
    "knn tie-break": ("return ka < kb || (ka == kb && ia < ib);",
                      "return ka < kb || (ka == kb && ia > ib);"),
    "eigenvalues ascending": ("if (A[order[b]][order[b]] > A[order[a]][order[a]]) {",
                              "if (A[order[b]][order[b]] < A[order[a]][order[a]]) {"),
    "monomial index": ("row[4] = xi * eta;", "row[4] = xi * xi;"),
    "weighted row not rescaled": ("s->w[r] *= sw;", "s->w[r] *= 1.0;"),
    "weighted data not rescaled": ("z[k * 3 + c] * sw : z[k * 3 + c]", "z[k * 3 + c] : z[k * 3 + c]"),
    "weight on the centre row": ("if (r > 0 && pr->w_nbr != 1.0)", "if (pr->w_nbr != 1.0)"),
    "weight not square-rooted": ("const double sw = sqrt(pr->w_nbr);", "const double sw = pr->w_nbr;"),
    "divergence flux at +-h": ("dp = a1 + 2.0 * a2 * (0.5 * h)", "dp = a1 + 2.0 * a2 * h"),
    "divergence without s(0)": ("ap = 1.0 / (h * h * s0 * sp)", "ap = 1.0 / (h * h * sp)"),
    "divergence drift sign": ("ell[1] = (ap - am) * h;", "ell[1] = (am - ap) * h;"),
}
NOOP = ("xi = u[(r - 1) * 2] * ih;", "xi = u[(r - 1) * 2] * ih + 0.0;")


def _run(tmp, name, edit):
    src = open(os.path.join(ROOT, "oracle", "mvgd_oracle.c")).read()
    assert edit[0] in src, name
    d = os.path.join(tmp, "m%d" % abs(hash(name)))
    for sub in ("oracle", "tests", "paper_1603_04100_amd"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    with open(os.path.join(d, "oracle", "mvgd_oracle.c"), "w") as f:
        f.write(src.replace(edit[0], edit[1]))
    env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=d)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join("tests", "test_oracle.py")], cwd=d, env=env,
                       capture_output=True, text=True, timeout=900)
    return r.returncode


def test_planted_mistakes_are_caught(tmp_path):
    cases = dict(MUTANTS)
    cases["(no-op control)"] = NOOP
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        rcs = dict(zip(cases, ex.map(lambda kv: _run(str(tmp_path), *kv), cases.items())))
    survived = [k for k, rc in rcs.items() if rc == 0 and k != "(no-op control)"]
    assert not survived, f"pins missed: {survived}"
    assert rcs["(no-op control)"] == 0, "harness broken: the unmodified oracle fails its pins"
