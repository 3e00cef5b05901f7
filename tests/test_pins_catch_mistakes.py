"""The oracle's pins are strong enough: each plausible mistake planted in a
copy of the oracle (a wrong weight, sign, factor, index or mapping) makes at
least one of the CPU pin tests fail.  The copy is compiled with the oracle's
own flags and loaded in a separate pytest run; nothing here touches the GPU
library, whose code the pins must not depend on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
# fast pins first: the run stops at the first failure
PIN_TESTS = ["tests/test_oracle_lattice.py", "tests/test_oracle_mrt.py", "tests/test_oracle_spalding.py",
             "tests/test_oracle_wfb.py", "tests/test_oracle_paper_numbers.py", "tests/test_oracle_initial_state.py",
             "tests/test_oracle_cells.py", "tests/test_oracle_wall_nodes.py", "tests/test_oracle_flows.py",
             "tests/test_oracle_mrt_flows.py"]

# name: (text in lbm_oracle.c, planted replacement)
MISTAKES = {
    "diagonal weight 1/18": ("(n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0", "(n2 == 1) ? 1.0 / 18.0 : 1.0 / 18.0"),
    "equilibrium (e.u)^2 coefficient": ("4.5 * eu * eu", "4.0 * eu * eu"),
    "equilibrium u.u sign": ("- 1.5 * uu", "+ 1.5 * uu"),
    "full force in the velocity": ("j[0] += 0.5 * fx;", "j[0] += 1.0 * fx;"),
    "Guo prefactor dropped": ("+ (1.0 - 1.0 / (2.0 * taue)) * force[a];", "+ force[a];"),
    "Guo second-order term": ("9.0 * eu * ef", "3.0 * eu * ef"),
    "Smagorinsky constant 18 -> 9": ("18.0 * cs * cs", "9.0 * cs * cs"),
    "Smagorinsky Q without the 2": ("sqrt(2.0 * pp)", "sqrt(pp)"),
    "wall stress sign": ("taux = -(vx / U) * tauw;", "taux = (vx / U) * tauw;"),
    "wall stress without rho": ("double tauw = rho * utau * utau;", "double tauw = utau * utau;"),
    "full stress on the diagonals": ("f[a7] += 0.5 * taux;", "f[a7] += 1.0 * taux;"),
    "top wall not mirrored": ("if (wall == 1) { a7 = MIR[7]; a14 = MIR[14]; a11 = MIR[11]; a17 = MIR[17]; }", ""),
    "Spalding cubic term dropped": ("- k * k / 2.0 - k * k * k / 6.0);\n}", "- k * k / 2.0);\n}"),
    "Newton derivative term": ("double dh = sp + p * dsp;", "double dh = sp;"),
    "bounce-back onto itself": ("f[a] = src_get(s, OPP[a], x, y, z);", "f[a] = src_get(s, a, x, y, z);"),
    "mirror source not mirrored": ("f[a] = src_get(s, MIR[a], sx, y, sz);", "f[a] = src_get(s, OPP[a], sx, y, sz);"),
    "streaming from the wrong side": ("int sx = wrap(x - E[a][0], p->nx);", "int sx = wrap(x + E[a][0], p->nx);"),
    "bounce-back set of the free-slip wall": ("(E[a][0] == 0 && E[a][2] == 0)", "(E[a][0] == 0)"),
    "statistics u_x u_z for u_x u_y": ("r[6] += mom[1] * mom[2];", "r[6] += mom[1] * mom[3];"),
    "initial profile distance without y1": ("double d = (double)dy + p->y1;\n        prof[y]", "double d = (double)dy;\n        prof[y]"),
    "MRT energy row": ("case 1: return 19.0 * e2 - 30.0;", "case 1: return 19.0 * e2 - 31.0;"),
    "MRT heat flux relaxed at the m rate": ("case 4: case 6: case 8: return p->s_q;", "case 4: case 6: case 8: return p->s_m;"),
    "MRT stress relaxed at the pi rate": ("case 10: case 12: return p->s_pi;", "case 9: case 10: case 12: return p->s_pi;"),
    "MRT force without the half rate": ("(1.0 - 0.5 * sk) * mf", "(1.0 - sk) * mf"),
    "MRT inverse without the row norm": ("v += mrow(k, a) * mstar[k] / n2;", "v += mrow(k, a) * mstar[k] / 19.0;"),
    "van Driest exponent without A+": ("exp(-(d * ut / nu0) / p->vd_aplus)", "exp(-(d * ut / nu0))"),
    "van Driest damping inverted": ("return p->cs * (1.0 - exp(", "return p->cs * (exp("),
    "one noise draw for all components": ("3u * c + (uint64_t)i", "3u * c"),
    "relaxation multiplied by tau": ("out[a] = f[a] - (f[a] - fe[a]) / taue +", "out[a] = f[a] - (f[a] - fe[a]) * taue +"),
    "nu0 without the 1/3": ("double nu0 = (p->tau0 - 0.5) / 3.0;\n        utau", "double nu0 = (p->tau0 - 0.5);\n        utau"),
    "wall velocity without the half force": ("    jx += 0.5 * p->fx;\n    double vx", "    double vx"),
    "statistics sample count": ("o->stats[8 * y + 7] += (double)p->nx * p->nz;", "o->stats[8 * y + 7] += (double)p->nx;"),
    "spanwise streaming from the wrong side": ("int sz = wrap(z - E[a][2], p->nz);", "int sz = wrap(z + E[a][2], p->nz);"),
    "analytic initial state: wrong direction": ("    return feq(a, 1.0, u);\n}", "    return feq(OPP[a], 1.0, u);\n}"),
    "wall node gather without the in-plane shift": ("f[a] = s->fw[(((int64_t)w * 5 + in_index(w, a)) * p->nz + sz) * p->nx + sx];", "f[a] = s->fw[(((int64_t)w * 5 + in_index(w, a)) * p->nz + z) * p->nx + x];"),
    "wall node arrivals without the in-plane shift": ("int sx = wrap(x - E[b][0], p->nx), sz = wrap(z - E[b][2], p->nz);\n                        f[b] = o->fpost", "int sx = x, sz = z;\n                        f[b] = o->fpost"),
    "wall node 14a sign": ("o[7] = g[13] + 0.5 * tx;", "o[7] = g[13] - 0.5 * tx;"),
    "wall node 14c copy of the uncorrected value": ("o[8] = o[7];", "o[8] = g[13];"),
    "bounce-back node mirrored": ("for (int a = 0; a < Q; ++a) o[a] = g[OPP[a]];", "for (int a = 0; a < Q; ++a) o[a] = g[MIR[a]];"),
    "wall node velocity u_y for u_z": ("u[0] = mom[0]; u[1] = mom[1]; u[2] = mom[3];", "u[0] = mom[0]; u[1] = mom[1]; u[2] = mom[2];"),
    "wall node start without the plain moments": ("u[0] = r; u[1] = jx / r; u[2] = jz / r;", "u[0] = r; u[1] = jx; u[2] = jz / r;"),
    "same-step wall node stress from the previous record": (
        "if (p->wall_nodes == 2 && wall_node_update(o, o->urec_new, o->fw_new, &maxit)",
        "if (p->wall_nodes == 2 && wall_node_update(o, o->urec, o->fw_new, &maxit)"),
    "opposite of a direction": ("E[b][1] == -E[a][1] && E[b][2] == -E[a][2]) OPP[a] = b;",
                                "E[b][1] == -E[a][1] && E[b][2] == E[a][2]) OPP[a] = b;"),
}


def _build(tmp, text):
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    with open(c, "w") as fh:
        fh.write(text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-w", "-o", so, c, "-lm"], check=True)
    return so


def _pins(so):
    # four threads, or the share of the cores a pytest-xdist worker was given
    env = dict(os.environ, ORC_LIB_PATH=so, OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "4"))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
                          + PIN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_pins_pass_on_the_oracle_itself(tmp_path):
    with open(SRC) as fh:
        r = _pins(_build(str(tmp_path), fh.read()))
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MISTAKES[name]
    with open(SRC) as fh:
        text = fh.read()
    assert text.count(old) == 1, "the planted mistake no longer matches the oracle source"
    r = _pins(_build(str(tmp_path), text.replace(old, new)))
    assert r.returncode != 0, "%s survived every pin:\n%s" % (name, r.stdout[-2000:])
