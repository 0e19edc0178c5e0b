"""The oracle's pins must catch plausible misreadings of Sec. 2.2.

Each case below plants one mistake in a private copy of oracle.c (in a
temporary directory; the repository's oracle is untouched), rebuilds it and
runs tests/test_oracle_pins.py against the copy: at least one pin must fail.
The mistakes are the ones a reader could make in the density sum (which h
in W), the force sum (h_ij, which mass), the viscosity (the means rho_ij and
c_ij, eta), the energy equation (its 1/2), the predictor-corrector update
(Eqs. e-predictor, e-corrector, r-new) and the time step of Eq.
(dt-stability).  CPU only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "density_hi": ("s += m[j] * or_W(r, 0.5 * (h[i] + h[j]));", "s += m[j] * or_W(r, h[i]);"),
    "density_hmax": ("s += m[j] * or_W(r, 0.5 * (h[i] + h[j]));",
                     "s += m[j] * or_W(r, fmax(h[i], h[j]));"),
    "density_no_self": ("double s = m[i] * or_W(0.0, h[i]);", "double s = 0.0;"),
    "force_hij_max": ("double hij = 0.5 * (h[i] + h[j]);\n            double dvx",
                      "double hij = fmax(h[i], h[j]);\n            double dvx"),
    "force_mass_i": ("sx -= m[j] * Pi * gx;", "sx -= m[i] * Pi * gx;"),
    "visc_cij_max": ("double cij = 0.5 * (c[i] + c[j]);\n            double nu",
                     "double cij = fmax(c[i], c[j]);\n            double nu"),
    "visc_rhoij_rhoi": ("double rhoij = 0.5 * (rho[i] + rho[j]);", "double rhoij = rho[i];"),
    "visc_no_eta": ("mu = hij * rv / (r2 + eta * hij * hij);", "mu = hij * rv / (r2 + hij * hij);"),
    "dedt_no_half": ("se += 0.5 * m[j] * Pi", "se += m[j] * Pi"),
    "dedt_mass_i": ("se += 0.5 * m[j] * Pi", "se += 0.5 * m[i] * Pi"),
    "e_corrector_euler": ("e[i] = 0.5 * (e[i] + et[i]) + 0.5 * dt * E[i];",
                          "e[i] = e[i] + dt * E[i];"),
    "e_predictor_half_dt": ("et[i] = e[i] + dt * E[i];", "et[i] = e[i] + 0.5 * dt * E[i];"),
    "drift_vt_only": ("x[i] = x[i] + 0.5 * dt * (vtx[i] + vx[i]);", "x[i] = x[i] + dt * vtx[i];"),
    "cfl_no_s_in_root": ("sqrt(smin * (q + fabs(E[i])))", "sqrt(q + fabs(E[i]))"),
    "cfl_0.6_beta": ("1.2 * beta * mumax", "0.6 * beta * mumax"),
    "cfl_signed_E": ("sqrt(smin * (q + fabs(E[i])))", "sqrt(smin * (q + E[i]))"),
    "cfl_ci_not_cij": ("double cij = 0.5 * (c[i] + c[j]);\n            if (cij > cmax)",
                       "double cij = c[i];\n            if (cij > cmax)"),
}


@pytest.fixture(scope="module")
def oracle_src():
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        return f.read()


def _tree(dst):
    ign = shutil.ignore_patterns("*.so", "*.so.tmp*", "__pycache__")
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"), ignore=ign)
    os.makedirs(os.path.join(dst, "tests"))
    for f in ("conftest.py", "test_oracle_pins.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))
    pkg = os.path.join(dst, "paper_1807_08116_amd")
    os.makedirs(pkg)
    for f in ("__init__.py", "ic.py"):          # seeded input generators only
        shutil.copy(os.path.join(ROOT, "paper_1807_08116_amd", f), os.path.join(pkg, f))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)


def _run_pins(tmp_path, src):
    _tree(str(tmp_path))
    with open(tmp_path / "oracle" / "oracle.c", "w") as f:
        f.write(src)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "tests/test_oracle_pins.py"],
                       cwd=str(tmp_path), capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, "\n".join(r.stdout.strip().splitlines()[-3:])


@pytest.mark.slow
def test_unmutated_copy_passes(tmp_path, oracle_src):
    # control: the copied tree itself is sound, so a failure below is the mutant's
    rc, tail = _run_pins(tmp_path, oracle_src)
    assert rc == 0, tail


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, oracle_src, name):
    old, new = MUTANTS[name]
    assert oracle_src.count(old) == 1, "mutation site not unique: " + name
    rc, tail = _run_pins(tmp_path, oracle_src.replace(old, new))
    assert rc == 1, "mutant %s passed every pin:\n%s" % (name, tail)
    assert "failed" in tail, tail
