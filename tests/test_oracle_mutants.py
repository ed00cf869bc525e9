"""Mutation test of the oracle's pins: plant one plausible mistake at a time
in a copy of the oracle (on the CPU), rebuild it, and require that at least
one pin fails.  A mistake no pin catches would mean the pins are too weak."""
from __future__ import annotations

import os
import shutil

import pytest

import oracle
from tests import oracle_pins

MUTANTS = [
    ("diagonal distance is dx", "dist[k] = ddiag;", "dist[k] = dx;"),
    ("ties go to the last neighbour", "if (s > smax) {", "if (s >= smax) {"),
    ("transposed neighbour offset",
     "(int64_t)(y + LEMO_DY[k]) * nx + (x + LEMO_DX[k])",
     "(int64_t)(y + LEMO_DX[k]) * nx + (x + LEMO_DY[k])"),
    ("dx and dy swapped", "dist[k] = dy;\n    else\n      dist[k] = dx;",
     "dist[k] = dx;\n    else\n      dist[k] = dy;"),
    ("donors of the perimeter ignored", "dnum[c] = 0;\n      for (int k = 0; k < 8; ++k) {",
     "dnum[c] = 0;\n      if (lemo_is_perimeter(ny, nx, y, x)) continue;\n      for (int k = 0; k < 8; ++k) {"),
    ("stack visits donors in reverse", "for (int k = (int)dnum[c] - 1; k >= 0; --k) {",
     "for (int k = 0; k < (int)dnum[c]; ++k) {"),
    ("first level offset is 1", "levels[ls++] = 0;", "levels[ls++] = 1;"),
    ("cell does not count itself", "uint32_t a = 1u;", "uint32_t a = 0u;"),
    ("perimeter is uplifted", "for (int32_t y = 1; y < ny - 1; ++y) {\n    for (int32_t x = 1; x < nx - 1; ++x) {\n      const int64_t c = (int64_t)y * nx + x;\n      h[c] = h[c] + (Ufield",
     "for (int32_t y = 0; y < ny; ++y) {\n    for (int32_t x = 0; x < nx; ++x) {\n      const int64_t c = (int64_t)y * nx + x;\n      h[c] = h[c] + (Ufield"),
    ("F without dt", "const double f = ((kc * dt) * am) / d;", "const double f = (kc * am) / d;"),
    ("area without cell size", "const double area = (double)count[c] * dxdy;\n    const double am",
     "const double area = (double)count[c];\n    const double am"),
    ("wrong sign in the update", "h[c] = (h[c] + f * h[r]) / (1.0 + f);",
     "h[c] = (h[c] - f * h[r]) / (1.0 + f);"),
    ("old receiver height (reverse order)",
     "for (int64_t i = 0; i < n; ++i) {\n    const int32_t c = order[i];\n    const int32_t r = rec[c];\n    if (r == c) continue;\n    const int32_t cy = c / nx, cx = c % nx, ry = r / nx, rx = r % nx;\n    const double d = (cy != ry && cx != rx) ? ddiag : (cy != ry ? dy : dx);\n    const double area = (double)count[c] * dxdy;\n    const double am",
     "for (int64_t i = n - 1; i >= 0; --i) {\n    const int32_t c = order[i];\n    const int32_t r = rec[c];\n    if (r == c) continue;\n    const int32_t cy = c / nx, cx = c % nx, ry = r / nx, rx = r % nx;\n    const double d = (cy != ry && cx != rx) ? ddiag : (cy != ry ? dy : dx);\n    const double area = (double)count[c] * dxdy;\n    const double am"),
    ("pits are not uplifted", "h[c] = h[c] + (Ufield ? Ufield[c] * dt : udt);",
     "if (h[c] > 0.5) h[c] = h[c] + (Ufield ? Ufield[c] * dt : udt);"),
    ("K field ignored", "const double kc = Kfield ? Kfield[c] : K;\n    const double f = ((kc",
     "const double kc = K;\n    const double f = ((kc"),
    ("Newton divides by d, not d^n", "pow(area, m)) / pow(d, nexp);", "pow(area, m)) / d;"),
    ("Newton residual with the wrong sign", "(hnew - h0 + f * pow(g, nexp))",
     "(hnew - h0 - f * pow(g, nexp))"),
    ("Newton stops after one iteration", "fabs(delta) > eps && it < max_iter",
     "fabs(delta) > eps && it < 1"),
    ("Newton iteration cap ignored", "fabs(delta) > eps && it < max_iter",
     "fabs(delta) > eps && it < 1000"),
    ("Newton iterate below the receiver kept",
     "if (!(next - hn > 0.0)) next = 0.5 * (hnew + hn);", "(void)0;"),
    ("Newton stops at the first iterate not above the receiver",
     "if (!(next - hn > 0.0)) next = 0.5 * (hnew + hn);",
     "if (!(next - hn > 0.0)) { hnew = next; break; }"),
    ("Newton guard admits a zero gap",
     "if (!(next - hn > 0.0)) next = 0.5 * (hnew + hn);",
     "if (!(next - hn >= 0.0)) next = 0.5 * (hnew + hn);"),
    ("Newton overshoot replaced by the midpoint towards h0",
     "if (!(next - hn > 0.0)) next = 0.5 * (hnew + hn);",
     "if (!(next - hn > 0.0)) next = 0.5 * (hnew + h0);"),
    ("Newton erodes a cell not above its receiver", "if (h0 - hn > 0.0) {", "if (1) {"),
    ("MFD shares not normalised", "pexp) / wsum[d];", "pexp);"),
    ("MFD erosion with the old receiver height", "sumfh += f * h[r];", "sumfh += f * h0[r];"),
    ("projection multiplies by F", "if (f > 0.0) h[c] = h[r] + uc / f;",
     "if (f > 0.0) h[c] = h[r] + uc * f;"),
    ("projection with the exponent n, not 1/n", "h[r] + pow(uc / f, 1.0 / nexp)",
     "h[r] + pow(uc / f, nexp)"),
    ("projection ignores the U field", "const double uc = Ufield ? Ufield[c] * dt : udt;",
     "const double uc = udt;"),
    ("projection without uplift of sinks",
     "lemo_uplift(p->ny, p->nx, p->dt, p->U, U, h);\n    lemo_project_heights",
     "lemo_project_heights"),
    ("projection measures the slope to the old receiver height",
     "if (f > 0.0) h[c] = h[r] + uc / f;", "if (f > 0.0) h[c] = h[c] + uc / f;"),
    ("MFD levels by the shallowest receiver", "if (h0[c] - h0[r] > 0.0 && level[r] + 1 > l) l = level[r] + 1;",
     "if (h0[c] - h0[r] > 0.0 && (l == 0 || level[r] + 1 < l)) l = level[r] + 1;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = open(oracle.SOURCE).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    mutated = src.replace(old, new, 1)
    d = tmp_path / "m"
    d.mkdir()
    (d / "lem_oracle.c").write_text(mutated)
    shutil.copy(os.path.join(os.path.dirname(oracle.SOURCE), "lem_oracle.h"), d / "lem_oracle.h")
    path = oracle.build(str(d / "lem_oracle.c"), str(d / "libmut.so"))
    lib = oracle.load(path)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"no pin catches the mutant '{name}'"
