"""Planted mistakes: each must make the oracle's pins fail.

Every case below copies one oracle source, changes one expression into a plausible
mistake (a dropped factor, a flipped sign, a swapped operand, the wrong image or
branch), builds the copy in a temporary directory and runs the pin files against it in
a subprocess (the bindings load a copy named by DILBM_ORACLE_LIB / DILBM_ORACLE3_LIB).
The pins must fail for every mutant and pass for an unchanged copy built the same way.
The oracle itself is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORA = os.path.join(ROOT, "oracle")
SRC2 = os.path.join(ORA, "dilbm_oracle.c")
SRC3 = os.path.join(ORA, "dilbm3d_oracle.c")

PINS2 = ["tests/test_oracle_pointwise.py", "tests/test_oracle_solver.py",
         "tests/test_oracle_bodies.py", "tests/test_oracle_boundaries.py"]
BODIES = ["tests/test_oracle_bodies.py"]
PINS3 = ["tests/test_oracle3d.py", "tests/test_oracle3d_q27.py", "tests/test_oracle3d_open.py"]

# (name, source, text, replacement, pin files that must catch it)
MUTANTS = [
    # body update of the 2-D step: Eqs. (22)-(24), (28), (29), caught by the body pins alone
    ("disc inertia m R^2", SRC2, "const double I = 0.5 * m * R * R;",
     "const double I = m * R * R;", BODIES),
    ("disc mass in the update", SRC2,
     "const double m = s->brho[b] * M_PI * R * R; /* disc of unit depth */",
     "const double m = s->brho[b] * M_PI * R * R * R; /* disc of unit depth */", BODIES),
    ("attractive pair wiring", SRC2,
     "ora_pp_force(min_image(s->bx[b] - s->bx[c], p->nx), min_image(s->by[b] - s->by[c], p->ny),",
     "ora_pp_force(min_image(s->bx[c] - s->bx[b], p->nx), min_image(s->by[c] - s->by[b], p->ny),",
     BODIES),
    ("pair distance without the minimum image", SRC2,
     "ora_pp_force(min_image(s->bx[b] - s->bx[c], p->nx),",
     "ora_pp_force((s->bx[b] - s->bx[c]),", BODIES),
    ("pair uses the body's own radius for the partner", SRC2, "R, s->br[c], p->xi",
     "R, R, p->xi", BODIES),
    ("overlap branch with the soft-zone stiffness", SRC2, "k = (ri + rj - d) / eps_p1;",
     "k = (ri + rj - d) / eps_p;", BODIES),
    ("wall image on the wrong side", SRC2,
     "? 2.0 * (Y - h) : -2.0 * ((N - h) - Y);", "? -2.0 * (Y - h) : 2.0 * ((N - h) - Y);",
     BODIES),
    ("image across the farther surface", SRC2, "(Y - h <= (N - h) - Y)",
     "(Y - h > (N - h) - Y)", BODIES),
    ("x wall measured on y", SRC2, "const double X = s->bx[b], h = p->wall_h, N = p->nx;",
     "const double X = s->by[b], h = p->wall_h, N = p->nx;", BODIES),
    ("wall soft zone with the overlap stiffness", SRC2,
     "k = (2.0 * r + xi - d) * (2.0 * r + xi - d) / eps_w;",
     "k = (2.0 * r + xi - d) * (2.0 * r + xi - d) / eps_w1;", BODIES),
    ("buoyancy factor inverted", SRC2,
     "(p->rho0 / s->brho[b] - 1.0) * m * p->g[1]", "(s->brho[b] / p->rho0 - 1.0) * m * p->g[1]",
     BODIES),
    ("forward-Euler position", SRC2, "*x += 0.5 * (*ux + ux_new);", "*x += ux_new;", BODIES),
    ("spin against the torque", SRC2, "const double om_new = *om + T / I;",
     "const double om_new = *om - T / I;", BODIES),
    ("torque sign in the reduction", SRC2, "s->bT[b] += s->e_rx[e] * fy - s->e_ry[e] * fx;",
     "s->bT[b] += s->e_ry[e] * fx - s->e_rx[e] * fy;", BODIES),
    # the node operator and the step
    ("u* without half the body force", SRC2, "const double usx_star = (jx + 0.5 * Gx) / rho;",
     "const double usx_star = (jx + Gx) / rho;", PINS2),
    ("Eq. (17) without the factor 1/2", SRC2, "ux += 0.5 * wb * (usx[b] - usx_star);",
     "ux += wb * (usx[b] - usx_star);", PINS2),
    ("Eq. (14) with l of the wrong sign", SRC2, "return 0.5 * (1.0 + tanh(2.0 * l / eps));",
     "return 0.5 * (1.0 + tanh(-2.0 * l / eps));", PINS2),
    ("Eq. (15) without (1 - 1/2tau)", SRC2,
     "F[i] = (1.0 - 1.0 / (2.0 * tau)) * WT[i] * rho * (lin + quad / (2.0 * CS2 * CS2));",
     "F[i] = WT[i] * rho * (lin + quad / (2.0 * CS2 * CS2));", PINS2),
    ("several bodies not normalised", SRC2, "const double scale = S > 1.0 ? 1.0 / S : 1.0;",
     "const double scale = 1.0;", PINS2),
    ("Guo forcing without (1 - 1/2tau)", SRC2,
     "Gi[i] = (1.0 - 1.0 / (2.0 * tau)) * WT[i] * (ax * Gx + ay * Gy);",
     "Gi[i] = WT[i] * (ax * Gx + ay * Gy);", PINS2),
    # open ends (non-equilibrium extrapolation)
    ("extrapolation without the relaxation factor", SRC2,
     "(1.0 - 1.0 / tau) * (f[i] - feq_nb[i])", "(f[i] - feq_nb[i])", PINS2),
    ("neighbour velocity without half the body force", SRC2,
     "const double ux = (jx + 0.5 * Gx) / rho, uy = (jy + 0.5 * Gy) / rho;",
     "const double ux = jx / rho, uy = jy / rho;", PINS2),
    # the three-dimensional oracle
    ("3-D sphere inertia 2/3", SRC3, "const double I = 0.4 * m * R * R;",
     "const double I = (2.0 / 3.0) * m * R * R;", PINS3),
    ("3-D sphere mass of a disc", SRC3, "return rho_s * 4.0 / 3.0 * M_PI * R * R * R;",
     "return rho_s * M_PI * R * R;", PINS3),
    ("3-D omega x r sign", SRC3, "U[0] + W[1] * r[2] - W[2] * r[1]",
     "U[0] - W[1] * r[2] + W[2] * r[1]", PINS3),
    ("3-D u* without half the body force", SRC3,
     "ust[a] = (j[a] + 0.5 * G[a]) / rho;", "ust[a] = j[a] / rho;", PINS3),
    ("3-D interface width doubled", SRC3, "return 0.5 * (1.0 + tanh(2.0 * l / p->eps));",
     "return 0.5 * (1.0 + tanh(l / p->eps));", PINS3),
    ("D3Q27 corner weight 1/108", SRC3, "(n == 2 ? 1.0 / 54.0 : 1.0 / 216.0)",
     "(n == 2 ? 1.0 / 54.0 : 1.0 / 108.0)", PINS3),
    ("D3Q27 edge and corner weights swapped", SRC3, "(n == 2 ? 1.0 / 54.0 : 1.0 / 216.0)",
     "(n == 2 ? 1.0 / 216.0 : 1.0 / 54.0)", PINS3),
    ("3-D extrapolation without the relaxation factor", SRC3,
     "(1.0 - 1.0 / tau) * (f[i] - feq_nb[i]) - weight(q, i) * rho0;",
     "(f[i] - feq_nb[i]) - weight(q, i) * rho0;", PINS3),
    ("3-D neighbour velocity without half the body force", SRC3,
     "u_nb[a] = (j[a] + 0.5 * G[a]) / rho;", "u_nb[a] = j[a] / rho;", PINS3),
    ("3-D outlet extrapolated from itself", SRC3, "(in ? 1 : nx - 2)", "(in ? 1 : nx - 1)",
     PINS3),
    ("3-D duct profile without the z factor", SRC3, "if (p->inlet_profile == 2)",
     "if (p->inlet_profile == 3)", PINS3),
    ("3-D inlet takes the neighbour's velocity", SRC3, "u_nb = p->inlet_kind == 1;",
     "u_nb = 1;", PINS3),
    ("D3Q27 corner direction flipped in z", SRC3,
     "                                 1, -1, -1, 1, 1, -1, 1, -1};",
     "                                 -1, -1, -1, 1, 1, -1, 1, -1};", PINS3),
]


def _build_copy(src, text, repl, tmp, tag):
    from oracle.binding import compile_c

    body = open(src).read()
    if text is not None:
        assert body.count(text) == 1, f"mutation site of {tag!r} not found exactly once"
        body = body.replace(text, repl)
    csrc = os.path.join(tmp, os.path.basename(src))
    with open(csrc, "w") as f:
        f.write(body)
    # the header next to the source
    for h in ("dilbm_oracle.h", "dilbm3d_oracle.h"):
        with open(os.path.join(ORA, h)) as fi, open(os.path.join(tmp, h), "w") as fo:
            fo.write(fi.read())
    lib = os.path.join(tmp, "lib" + os.path.splitext(os.path.basename(src))[0] + ".so")
    compile_c(csrc, lib, force=True)
    return lib


def _run_pins(lib, src, files):
    env = dict(os.environ)
    env["DILBM_ORACLE3_LIB" if src == SRC3 else "DILBM_ORACLE_LIB"] = lib
    env["OMP_NUM_THREADS"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *files], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _case(args):
    name, src, text, repl, files = args
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_copy(src, text, repl, tmp, name)
        return name, _run_pins(lib, src, files)


@pytest.fixture(scope="module")
def outcomes(oracle_lib):
    cases = list(MUTANTS)
    cases.append(("unchanged 2-D copy", SRC2, None, None, PINS2))
    cases.append(("unchanged 3-D copy", SRC3, None, None, PINS3))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(_case, cases))


def test_unchanged_copies_pass(outcomes):
    for name in ("unchanged 2-D copy", "unchanged 3-D copy"):
        rc, out = outcomes[name]
        assert rc == 0, f"{name}: pins fail on an unchanged copy\n{out}"


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(outcomes, name):
    rc, out = outcomes[name]
    # exit status 1: tests ran and at least one failed (not a collection or usage error)
    assert rc == 1, f"mutant {name!r} was not caught (exit {rc})\n{out}"
