"""The oracle's pins catch plausible mistakes.  Each case plants one mistake in a copy of
``oracle/lbm_ref.c`` (a dropped term, a wrong sign or index, a swapped operand), builds it, and
runs the CPU pin suite against the broken build in a subprocess; the suite must fail.  The
mistakes are planted in the oracle, on the CPU, never in the HIP path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_ref.c")
PIN_FILES = ["tests/test_oracle_identities.py", "tests/test_oracle_adjoint.py",
             "tests/test_oracle_physics.py"]

# (name, text in lbm_ref.c, replacement)
MUTANTS = [
    ("M row entry", "{0, -2, 0, 2, 0, 1, -1, -1, 1},", "{0, -2, 0, 2, 0, 1, 1, -1, 1},"),
    ("N row entry", "{-4, 1, 1, 1, 1},", "{-4, 1, 1, 1, 2},"),
    ("D2Q9 velocity", "static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};",
     "static const int EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, -1};"),
    ("D2Q9 weight", "1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};", "1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 35};"),
    ("buoyancy sign", "d->gbeta * (T - d->T0);", "d->gbeta * (d->T0 - T);"),
    ("l0 half step", "0.5 * (1.0 + phi * 0.5 * d->nu / K)", "0.5 * (1.0 + phi * d->nu / K)"),
    ("Forchheimer drag dropped", "- phi * Fphi / sqrt(K) * umag * ux", "- 0.0 * umag * ux"),
    ("pressure factor", "d->cs2 / (1.0 - W9[0]) * (sum18", "d->cs2 / W9[0] * (sum18"),
    ("meq porosity", "out[7] = rho0 * (ux * ux - uy * uy) / phi;",
     "out[7] = rho0 * (ux * ux - uy * uy);"),
    ("forcing sign", "out[4] = -rho0 * Fx;", "out[4] = rho0 * Fx;"),
    ("forcing factor (I - Lambda/2)", "(1.0 - 0.5 * d->s[k]) * S[k]", "S[k]"),
    ("thermal equilibrium", "out[1] = ux * T / sigma;", "out[1] = uy * T / sigma;"),
    ("D2Q5 weight", "const double wt = (i == 0) ? (1.0 - varpi) / 5.0 : (4.0 + varpi) / 20.0;",
     "const double wt = (i == 0) ? (1.0 + varpi) / 5.0 : (4.0 + varpi) / 20.0;"),
    ("heat source Psi3", "p->varpi * d->Q / p->sigma, 0.0};", "0.0, 0.0};"),
    ("Eq. (36) half step", "T += 0.5 * d->Q / p->sigma;", "T += d->Q / p->sigma;"),
    ("adiabatic wall T", "else Tb = mf->T;", "else Tb = 0.5;"),
    ("wall pressure", "mb->phip = mf->phip;           /* phi_b p_b = phi_f p_f */",
     "mb->phip = mf->phip / mf->phi * phib;"),
    ("five-point stencil", "48.0 * c->mac[r + 1].T", "47.0 * c->mac[r + 1].T"),
    ("trapezoid weight", "(y == 0 || y == ny - 1) ? 0.5 : 1.0;", "(y == 0) ? 0.5 : 1.0;"),
    ("tau_T from nu", "0.5 + d->nu / (p->sigma * d->csT2 * p->Pr)",
     "0.5 + d->nu / (d->csT2 * p->Pr)"),
    ("g beta from Ma", "p->Ma * p->Ma * d->cs2 / (d->dT * d->L)", "p->Ma * d->cs2 / (d->dT * d->L)"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mutant = tmp_path / "lbm_ref_mutant.c"
    mutant.write_text(src.replace(old, new))
    so = tmp_path / "liblbmref_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
                           "-fopenmp", "-fPIC", "-shared", "-o", str(so), str(mutant), "-lm"])
    env = dict(os.environ, LBM_REF_LIB=str(so), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + PIN_FILES, cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode != 0, f"pins did not catch: {name}\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "error" in r.stdout.lower()
