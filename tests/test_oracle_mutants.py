"""Plants plausible mistakes in a copy of the oracle source (on the CPU) and checks that the
oracle pins catch every one: a dropped or doubled term, a wrong sign, a wrong tensor index,
a wrong ghost source, a missing direction, the O(v/c) terms, the cubic heat capacity.  Each mutant is compiled with gcc into a temporary
directory and the pin module is run against it in a child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = [
    ("0.5 * C * (ER - EL);", "0.5 * C * (EL - ER);"),
    ("0.5 * C * (ER - EL);", "1.0 * C * (ER - EL);"),
    ("phi[0] = 0.5 * (x[1 + d][L] + x[1 + d][R])", "phi[0] = 0.5 * (x[1 + (d + 1) % 3][L] + x[1 + d][R])"),
    ("(fdj[L] * EL + fdj[R] * ER)", "(fdj[L] * EL + fdj[L] * ER)"),
    ("0.5 * c2 * (fdj[L]", "0.5 * g->c * (fdj[L]"),
    ("- 0.5 * C * (x[1 + j][R] - x[1 + j][L]);", "- 0.5 * C * (x[1 + d][R] - x[1 + d][L]);"),
    ("if (a == 0 && b == 2) return 4;", "if (a == 0 && b == 2) return 5;"),
    ("return q * q / (2.0 * fdd);", "return q * q / fdd;"),
    ("double fc = fL > fR ? fL : fR;", "double fc = fL < fR ? fL : fR;"),
    ("double tau = 0.5 * (cell_tau(g, sigL, fL) + cell_tau(g, sigR, fR));", "double tau = cell_tau(g, sigL, fL);"),
    ("corr = sqrt(-expm1(-tau) / tau);", "corr = -expm1(-tau) / tau;"),
    ("double diag = (q == 0) ? dE[c] : 1.0 + sR;", "double diag = (q == 0) ? dE[c] : 1.0;"),
    ("R[0][c] += -En[c] - sP * g->aR * T4;", "R[0][c] += -En[c] + sP * g->aR * T4;"),
    ("+ sP * (g->aR * T4 - E[c]);", "+ sP * (g->aR * T4 - 0.5 * E[c]);"),
    ("- 3.0 * (1.0 - eta) * sP * g->aR * Ts4;", "- 2.0 * (1.0 - eta) * sP * g->aR * Ts4;"),
    ("o.dE[c] = 1.0 + sP * (1.0 - eta);", "o.dE[c] = 1.0 + sP;"),
    ("double gv = alpha * (T - Tn) + sP * (aR * T3 * T - E);", "double gv = alpha * (T - Tn) + sP * (aR * T3 - E);"),
    ("src[d] = side ? 0 : n[d] - 1;", "src[d] = side ? 1 : n[d] - 1;"),
    ("src[d] = side ? n[d] - 1 : 0;", "src[d] = side ? n[d] - 2 : 0;"),
    ("return g->c * g->dt * sigma_R(cf, i); }", "return g->dt * sigma_R(cf, i); }"),
    ("return cf->rho[i] * g->cv; }", "return g->cv; }"),
    ("double q = 10.0 * g->h * sigR;", "double q = 10.0 * sigR;"),
    ("for (int d = 0; d < 3; ++d) div +=", "for (int d = 0; d < 2; ++d) div +="),
    ("const double chi = (3.0 + 4.0 * g * g)", "const double chi = (3.0 + 2.0 * g * g)"),
    ("beam = 0.5 * (3.0 * chi - 1.0);", "beam = 0.5 * (3.0 * chi + 1.0);"),
    ("if (g > 1.0) g = 1.0;", "if (g > 2.0) g = 2.0;"),
    ("g = Fm / (c * E[i]);", "g = Fm / E[i];"),
    ("fxy = beam * nx * ny;", "fxy = beam * nx * nz;"),
    ("double fxx = 1.0 / 3.0, fyy = 1.0 / 3.0,", "double fxx = 1.0 / 3.0, fyy = 0.3,"),
]

# caught by the O(v/c) pins
VEL_MUTANTS = [
    ("y[1 + q][c] -= sR * g->c * x[0][c] * (b[q] + fb[q]);", "y[1 + q][c] -= sR * g->c * x[0][c] * fb[q];"),
    ("y[1 + q][c] -= sR * g->c * x[0][c] * (b[q] + fb[q]);", "y[1 + q][c] += sR * g->c * x[0][c] * (b[q] + fb[q]);"),
    ("return (sR - 2.0 * sP) * bF / g->c", "return (sR - sP) * bF / g->c"),
    ("(sP - sR) * (bb + bfb) * E;", "(sP - sR) * bb * E;"),
    ("R[4][c] -= vel_energy(g, cf, c, E[c], Fc);", "R[4][c] += vel_energy(g, cf, c, E[c], Fc);"),
    ("if (o.vscale) o.vscale[c] = 1.0 - eta;", "if (o.vscale) o.vscale[c] = 1.0;"),
    ("Tb += X / a;", "Tb -= X / a;"),
    ("fb[a] += cf->f[tens(a, k)][i] * b[k];", "fb[a] += cf->f[tens(a, a)][i] * b[k];"),
]

# caught by the cubic heat-capacity pins
GAS_MUTANTS = [
    ("return g->cv_cubic ? 0.25 * alpha * T * T * T * T : alpha * T;", "return g->cv_cubic ? alpha * T * T * T * T : alpha * T;"),
    ("return g->cv_cubic ? alpha * T * T * T : alpha; }", "return alpha; }"),
    ("double den = 0.25 * alpha + sP * aR;", "double den = alpha + sP * aR;"),
    ("eta * (gas_e(g, a, Tn[c]) - gas_e(g, a, Ts));", "eta * (gas_e(g, a, Tn[c]));"),
]


# caught by the scaled-residual pins (the convergence measure and full-size checker)
RESIDUAL_MUTANTS = [
    ("double half = 0.5 * g->dt / g->h * sumC;", "double half = g->dt / g->h * sumC;"),
    ("double dFn = sqrt(nF) + g->c * sqrt(nE);", "double dFn = sqrt(nF) + 10.0 * g->c * sqrt(nE);"),
    ("*WT = gas_C(g, alpha_of(g, cf, c), T[c]) + 4.0 * sP", "*WT = gas_C(g, alpha_of(g, cf, c), T[c]) + 3.0 * sP"),
    ("double RT = (T[c] == 0.0 && R[4][c] > 0.0) ? 0.0 : R[4][c];", "double RT = R[4][c];"),
    ("*WF = 1.0 + s_R(g, cf, c) + half;", "*WF = 1.0 + sP + half;"),
    ("sumC += C[d][c] + C[d][c + step(g, d)];", "sumC += 2.0 * C[d][c];"),
    ("for (int q = 1; q < 4; ++q) rF +=", "for (int q = 0; q < 4; ++q) rF +="),
    ("if (out[1] > out[3]) out[3] = out[1];", ";"),
]


# caught by the energy-correction pins (Sec. 2.3.4)
ENERGY_MUTANTS = [
    ("double dEc = sP * g->aR * TN4 - (sP * eta * E[c] + bE[c] - En[c]);",
     "double dEc = sP * g->aR * TN4 - (bE[c] - En[c]);"),
    ("T[c] = gas_T_of_e(g, a, gas_e(g, a, T[c]) + dE[c]);", "T[c] = gas_T_of_e(g, a, gas_e(g, a, T[c]) - dE[c]);"),
    ("scale += En[c] + gas_e(g, a, Tn[c]);", "scale += En[c];"),
    ("return g->cv_cubic ? sqrt(sqrt(4.0 * e / alpha)) : e / alpha;", "return g->cv_cubic ? sqrt(sqrt(e / alpha)) : e / alpha;"),
]


# caught by the boundary pins (open, Marshak, reflecting faces)
BOUNDARY_MUTANTS = [
    ("double in_now = 0.5 * (x[0][c] + sin_ * x[1 + d][c] / a);", "double in_now = 0.5 * (x[0][c] - sin_ * x[1 + d][c] / a);"),
    ("x[1 + j][gi] += delta * sin_ * g->c * g->c * cf->f[tens(d, j)][c] / a;",
     "x[1 + j][gi] += delta * sin_ * g->c * cf->f[tens(d, j)][c] / a;"),
    ("x[0][gi] = (linear ? 0.0 : 8.0 * g->finc[face] / g->c) - 4.0 * sin_", "x[0][gi] = (linear ? 0.0 : 4.0 * g->finc[face] / g->c) - 4.0 * sin_"),
    ("- 4.0 * sin_ * x[1 + d][c] / g->c - x[0][c];", "+ 4.0 * sin_ * x[1 + d][c] / g->c - x[0][c];"),
    ("x[1 + d][gi] = -x[1 + d][c];", "x[1 + d][gi] = x[1 + d][c];"),
    ("if (j != d) f[tens(d, j)][gi] = -f[tens(d, j)][gi];", "if (j != d) f[tens(d, j)][gi] = f[tens(d, j)][gi];"),
]


CASES = ([(m, "test_oracle_pins.py") for m in MUTANTS] + [(m, "test_oracle_velocity_pins.py") for m in VEL_MUTANTS] +
         [(m, "test_oracle_gas_pins.py") for m in GAS_MUTANTS] +
         [(m, "test_oracle_residual_pins.py") for m in RESIDUAL_MUTANTS] +
         [(m, "test_oracle_energy_pins.py") for m in ENERGY_MUTANTS] +
         [(m, "test_oracle_boundary_pins.py") for m in BOUNDARY_MUTANTS])


@pytest.mark.slow
@pytest.mark.parametrize("k", range(len(CASES)))
def test_pins_catch_planted_mistake(k, tmp_path):
    (before, after), pins = CASES[k]
    src = open(SRC).read()
    assert before in src, before
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(before, after, 1))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-I", os.path.join(ROOT, "oracle"),
                    "-o", str(so), str(path), "-lm"], check=True)
    env = dict(os.environ, VETTAM_ORACLE_SO=str(so), OMP_NUM_THREADS="2")
    # a mutant that stalls the solver is caught by the per-test time limit (the pins take ~5 s)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", pins),
                        "-x", "-q", "-p", "no:cacheprovider", "--timeout", "20"], env=env, capture_output=True,
                       text=True, cwd=ROOT, timeout=600)
    # caught = the pins ran and at least one of them failed (exit code 1 with failures in the
    # summary); a collection or usage error (exit codes 2-5) is no catch
    assert r.returncode == 1 and " failed" in r.stdout, (
        f"mutant not caught (rc {r.returncode}): {after}\n{r.stdout[-2000:]}\n{r.stderr[-2000:]}")
