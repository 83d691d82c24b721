"""The oracle's pins have teeth: plant one plausible mistake at a time in a
copy of the oracle source (CPU only), build it, and check that the pin suites
fail against it.  Each mutation changes what the oracle computes (a dropped or
wrong term, a wrong index, a transposed operand, a wrong sign in a rule)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mls_oracle.c")

MUTATIONS = [
    ("cross term replaced", "b[4] = ux * uy;", "b[4] = ux * ux;"),
    ("values read from column 0", "R[r * D + d] += wb * (double)vals[i * D + d];",
     "R[r * D + d] += wb * (double)vals[i * D];"),
    ("moment uses b[r] twice", "M[r * m + c] += wb * b[c];", "M[r * m + c] += wb * b[r];"),
    ("forward solve transposed", "v -= L[r][q] * z[q];", "v -= L[q][r] * z[q];"),
    ("back solve transposed", "v -= L[q][r] * y[q];", "v -= L[r][q] * y[q];"),
    ("equilibration not undone", "out[(int64_t)d * out_stride] = s[0] * y[0];",
     "out[(int64_t)d * out_stride] = y[0];"),
    ("gaussian scaled by h not h^2", "return exp(-(rho2 / (h * h)));",
     "return exp(-(rho2 / h));"),
    ("wendland factor", "(4.0 * s + 1.0)", "(4.0 * s + 2.0)"),
    ("lower triangle not mirrored", "for (int c = 0; c < r; ++c) M[r * m + c] = M[c * m + r];",
     ";"),
    ("grid row uses dx", "py = y0 + (double)r * dy;", "py = y0 + (double)r * dx;"),
    ("ladder accepts everything", "if (!(piv >= tau)) { ok = 0; break; }",
     "if (!(piv > 0.0)) { ok = 0; break; }"),
    ("weight floor ignored", "if (!(M[0] >= floor_w)) {", "if (0) {"),
    ("invpow exponent sign", "return pow(rho2 / (h * h), -alpha);",
     "return pow(rho2 / (h * h), alpha);"),
    ("case bit order", "(v1 >= lv ? 2 : 0) | (v2 >= lv ? 4 : 0)",
     "(v1 >= lv ? 4 : 0) | (v2 >= lv ? 2 : 0)"),
    ("tie counts below", "cs = (v0 >= lv ? 1 : 0)", "cs = (v0 > lv ? 1 : 0)"),
    ("saddle rule inverted", "joined = (c >= lv);", "joined = (c < lv);"),
    ("crossing from the wrong end", "case 2: va = v3; vb = v2; break;",
     "case 2: va = v2; vb = v3; break;"),
    ("segment reversed", "{0, 3}, {1, 0}, {1, 3}", "{3, 0}, {1, 0}, {1, 3}"),
    ("right edge x off by one", "*x = x0 + (double)(j + 1) * dx;", "*x = x0 + (double)j * dx;"),
    ("gradient equilibration factor", "mk >= 3 ? s[1] * y[1] / h : 0.0",
     "mk >= 3 ? s[0] * y[1] / h : 0.0"),
    ("gradient without 1/h", "mk >= 3 ? s[2] * y[2] / h : 0.0", "mk >= 3 ? s[2] * y[2] : 0.0"),
    ("gradient axes swapped", "mk >= 3 ? s[1] * y[1] / h : 0.0",
     "mk >= 3 ? s[2] * y[2] / h : 0.0"),
    ("rigid perpendicular turned the other way", "out[0] = -v[1];\n  out[1] = v[0];",
     "out[0] = v[1];\n  out[1] = -v[0];"),
    ("rigid length not restored", "out[0] = nv * fr[0] / nf + qs[0];",
     "out[0] = fr[0] / nf + qs[0];"),
    ("rigid centroid dropped", "out[out_stride] = nv * fr[1] / nf + qs[1];",
     "out[out_stride] = nv * fr[1] / nf;"),
    ("layout clamps only the corner's own line", "for (int i = 0; i < 3; ++i) {",
     "for (int i = 0; i < 1; ++i) {"),
    ("layout spring pushes instead of pulling", "    fx -= s * ax;\n    fy -= s * ay;",
     "    fx += s * ax;\n    fy += s * ay;"),
    ("layout temperature ignored", "  if (fl > t) {", "  if (fl > 1e300) {"),
    ("layout node-edge force reversed", "const double s = -C / (rx * rx + ry * ry + eta);",
     "const double s = C / (rx * rx + ry * ry + eta);"),
    ("sampled layout step offsets the wrong node", "pos_out[2 * i] = pos_in[2 * v] + mv[0];",
     "pos_out[2 * i] = pos_in[2 * i] + mv[0];"),
    ("band tie counts below", "if (v >= iso[(int64_t)d * n_iso + k]) ++b;",
     "if (v > iso[(int64_t)d * n_iso + k]) ++b;"),
    ("adaptive level 0 fades too", "        if (j > 0) {\n          a = (s - fade_lo)",
     "        if (j >= 0) {\n          a = (s - fade_lo)"),
    ("adaptive levels coarsen", "double step = spacing / ldexp(1.0, j);",
     "double step = spacing * ldexp(1.0, j);"),
    ("adaptive pixel size of the wrong axis", "double px = gx * dx, py = gy * dy;",
     "double px = gx * dy, py = gy * dy;"),
    ("adaptive distance in steps, not pixels", "double e = fabs(t - round(t)) * s;",
     "double e = fabs(t - round(t));"),
]

PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_contour_pins.py",
             "tests/test_oracle_grad_pins.py", "tests/test_oracle_rigid_pins.py",
             "tests/test_oracle_layout_pins.py", "tests/test_oracle_map_pins.py"]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old}"
    mut = tmp_path / "mls_oracle.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp",
                           "-fPIC", "-shared", "-o", str(lib), str(mut), "-lm"])
    env = dict(os.environ, MLS_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p",
                        "no:cacheprovider", *PIN_FILES], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
