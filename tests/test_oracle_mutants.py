"""Planted mistakes: every plausible slip in the oracle must fail a pin.

Each case edits one expression of ``oracle/hier.c`` (a dropped or swapped
term, a wrong sign or index, a transposed operand), compiles the mutant with
gcc into a temporary directory, and runs the pin battery in a child process
(a mutant may misbehave).  The unmodified source must pass the battery; every
mutant must fail it.
"""
import os
import subprocess
import sys
import tempfile

import pytest

from oracle import hier as oracle_hier

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("tt weights swapped", "t[k + d] = p->sy * Mx[d] - p->sx * My[d];",
     "t[k + d] = p->sx * Mx[d] - p->sy * My[d];"),
    ("tt sign", "t[k + d] = p->sy * Mx[d] - p->sx * My[d];",
     "t[k + d] = p->sy * Mx[d] + p->sx * My[d];"),
    ("info translation weights swapped", "M[d] = p->sx * Mx[d] + p->sy * My[d];",
     "M[d] = p->sy * Mx[d] + p->sx * My[d];"),
    ("G transposed in the upward pass", "s += p->G[i][j] * t[j];", "s += p->G[j][i] * t[j];"),
    ("G not transposed in the downward pass", "acc += p->G[j][i] * in[j];", "acc += p->G[i][j] * in[j];"),
    ("down y sign", "Ly[d] = p->sy * L[d] - p->sx * s[q + d];", "Ly[d] = p->sy * L[d] + p->sx * s[q + d];"),
    ("down x weights", "Lx[d] = p->sx * L[d] + p->sy * s[q + d];", "Lx[d] = p->sy * L[d] + p->sx * s[q + d];"),
    ("shift taken from the wrong child", "dxp[d] = cx[d] - p->c[d];", "dxp[d] = cy[d] - p->c[d];"),
    ("shift scale inverted", "sqrt((double)nx * n / (double)ny)", "sqrt((double)ny * n / (double)nx)"),
    ("cross-product sign", "A[0][0] = 0.0;   A[0][1] = -u[2];", "A[0][0] = 0.0;   A[0][1] = u[2];"),
    ("centroid weight", "((double)nx * cx[d] + (double)ny * cy[d]) / n",
     "((double)nx * cx[d] + (double)nx * cy[d]) / n"),
    ("Householder sign convention", "xnorm * xnorm);\n        double beta = (alpha >= 0.0) ? -nrm : nrm;",
     "xnorm * xnorm);\n        double beta = (alpha >= 0.0) ? nrm : -nrm;"),
    ("T22 not transposed", "p->T22[i][j] = (j <= i) ? A[j][i] : 0.0;", "p->T22[i][j] = (j <= i) ? A[i][j] : 0.0;"),
    ("G = Q instead of Q^T", "p->G[i][j] = Q[j][i];", "p->G[i][j] = Q[i][j];"),
    ("x is the upper half", "int64_t x = build_rec(B, lo, s);\n    int64_t y = build_rec(B, s + 1, hi);",
     "int64_t y = build_rec(B, lo, s);\n    int64_t x = build_rec(B, s + 1, hi);"),
    ("split order y before z", "code = (code << 1) | ((qz >> l) & 1u);\n        code = (code << 1) | ((qy >> l) & 1u);",
     "code = (code << 1) | ((qy >> l) & 1u);\n        code = (code << 1) | ((qz >> l) & 1u);"),
    ("20-bit quantisation", "double t = ((x - lo) / h) * 2097152.0;", "double t = ((x - lo) / h) * 1048576.0;"),
    ("rows of y before x", "if (p->x >= 0) off = offsets_rec(B, p->x, off);\n    if (p->y >= 0) off = offsets_rec(B, p->y, off);",
     "if (p->y >= 0) off = offsets_rec(B, p->y, off);\n    if (p->x >= 0) off = offsets_rec(B, p->x, off);"),
    ("leaf read in sorted order", "else { int64_t u = B->perm[-(p->x + 1)]; for (int d = 0; d < 3; ++d) Mx[d] = v[3 * u + d]; }",
     "else { int64_t u = -(p->x + 1); for (int d = 0; d < 3; ++d) Mx[d] = v[3 * u + d]; }"),
    ("Case I rank-2 fix dropped", "if (k == 3) p->T22[2][2] = 0.0;", ""),
    ("root Velocity-set ignored", "if (root) for (int d = 0; d < 6; ++d) L[d] = root[d * nrhs + r];", ""),
    ("root Info-set halves swapped", "if (root) for (int d = 0; d < 6; ++d) root[d * nrhs + r] = M[d];",
     "if (root) for (int d = 0; d < 6; ++d) root[d * nrhs + r] = M[(d + 3) % 6];"),
    ("explicit last block sign", "J[(q + d) * ncol + 3 * (nx + b) + d] = -p->sx / sqrt((double)ny);",
     "J[(q + d) * ncol + 3 * (nx + b) + d] = p->sx / sqrt((double)ny);"),
    # leaf boxes of up to s beads
    ("bucket translation sign not flipped (up)", "for (int d = 0; d < 3; ++d) { M[d] = -t[d]; M[3 + d] = t[3 + d]; }",
     "for (int d = 0; d < 3; ++d) { M[d] = t[d]; M[3 + d] = t[3 + d]; }"),
    ("bucket translation sign not flipped (down)", "for (int d = 0; d < 3; ++d) { t[d] = -L[d]; t[3 + d] = L[3 + d]; }",
     "for (int d = 0; d < 3; ++d) { t[d] = L[d]; t[3 + d] = L[3 + d]; }"),
    ("bucket rotation rows transposed", "for (int e = 0; e < 3; ++e) X[(3 + e) * m + 3 * b + d] = A[e][d];",
     "for (int e = 0; e < 3; ++e) X[(3 + e) * m + 3 * b + d] = A[d][e];"),
    ("bucket centroid weight", "for (int d = 0; d < 3; ++d) p->c[d] /= (double)n;",
     "for (int d = 0; d < 3; ++d) p->c[d] /= (double)(n + 1);"),
    ("bucket T22 not transposed", "p->T22[i][j] = (j <= i) ? X[(3 + i) * m + 3 + j] : 0.0;",
     "p->T22[i][j] = (j <= i) ? X[(3 + j) * m + 3 + i] : 0.0;"),
    ("bucket reflectors applied in reverse upward", "    for (int j = 0; j < 6; ++j) {\n        if (p->htau[j] == 0.0) continue;",
     "    for (int j = 5; j >= 0; --j) {\n        if (p->htau[j] == 0.0) continue;"),
    ("bucket Householder sign convention", "const double beta = (alpha >= 0.0) ? -nrm : nrm;",
     "const double beta = (alpha >= 0.0) ? nrm : -nrm;"),
    ("bucket residue rows shifted", "for (int64_t i = 0; i < p->dim; ++i) out[p->off + i] = t[6 + i];",
     "for (int64_t i = 0; i < p->dim; ++i) out[p->off + i] = t[5 + i];"),
]

BATTERY = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
from oracle import hier
from tests import pins
import workloads as W
lib = hier.load({lib!r})
B = lambda pos: hier.Body(pos, lib=lib)
fails = []
def check(name, ok):
    if not ok: fails.append(name)
rng = np.random.default_rng(3)
cube = rng.uniform(-2, 7, (60, 3))
check('tree', pins.oracle_tree(B(cube)) == pins.bisection_tree(cube))
# bead pairs split only at the 21st bit level
base = rng.uniform(0, 1, (12, 3))
near = base + (3.0 / 2**21) * np.array([1.0, 0, 0])
pair = np.concatenate([base, near, [[0, 0, 0], [1, 1, 1]]])
check('tree-near', pins.oracle_tree(B(pair)) == pins.bisection_tree(pair))
ell = W.ellipsoid_body(rng, 90, (12, 7, 4), jitter=0.2, center=(3, -1, 2))
b = B(ell)
check('infoset', pins.infoset_identity_error(b, rng) < 1e-12)
check('lapack', pins.lapack_convention_error(b) < 1e-10)
check('factor', pins.factor_error(b) < 1e-12)
check('projector', pins.projector_error(b, rng) < 1e-12)
check('roundtrip', pins.roundtrip_error(b, rng) < 1e-12)
check('norm', pins.norm_error(b, rng) < 1e-12)
check('explicit', pins.explicit_error(b, rng) < 1e-12)
check('blocks', pins.block_structure_error(b) < 1e-13)
check('case1', pins.case1_error(hier.Body, 0.3, 0.7, 1.1, lib=lib) < 1e-12)
check('fullq', pins.full_q_inverse_error(b, rng) < 1e-12)
check('rootrows', pins.root_rows_error(B(cube[:30])) < 1e-12)
# translation invariance (rank-2 pivots must not flip reflector signs)
pos = np.random.default_rng(30).uniform(-2, 7, (150, 3))
tr = W.ellipsoid_body(np.random.default_rng(30), 150, (20, 12, 8), jitter=0.3)
q0 = B(tr).explicit(); q1 = B(tr + np.array([0.25, -0.5, 2.0])).explicit()
check('translation', np.abs(q0 - q1).max() < 1e-12)
# leaf boxes of up to s beads
for sb in (3, 8):
    bb = hier.Body(ell, lib=lib, s=sb)
    check(f'bucket-infoset-{{sb}}', pins.infoset_identity_error(bb, rng) < 1e-12)
    check(f'bucket-lapack-{{sb}}', pins.bucket_lapack_error(bb) < 1e-11)
    check(f'bucket-projector-{{sb}}', pins.projector_error(bb, rng) < 1e-12)
    check(f'bucket-fullq-{{sb}}', pins.full_q_inverse_error(bb, rng) < 1e-12)
    check(f'bucket-explicit-{{sb}}', pins.explicit_error(bb, rng) < 1e-12)
print('FAILS', fails)
sys.exit(1 if fails else 0)
"""


def _run_battery(lib_path):
    code = BATTERY.format(root=ROOT, lib=lib_path)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    return p.returncode, p.stdout + p.stderr


def _compile(src_text, d):
    src = os.path.join(d, "hier.c")
    lib = os.path.join(d, "liboracle_hier.so")
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib, src, "-lm"])
    return lib


def test_unmodified_oracle_passes_battery():
    with open(oracle_hier.SRC) as f:
        text = f.read()
    with tempfile.TemporaryDirectory() as d:
        rc, out = _run_battery(_compile(text, d))
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    with open(oracle_hier.SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site not unique: {name}"
    with tempfile.TemporaryDirectory() as d:
        rc, out = _run_battery(_compile(text.replace(old, new), d))
    assert rc != 0, f"mutant '{name}' passed every pin:\n{out}"
