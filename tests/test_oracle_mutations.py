"""The pins must be able to fail: plant plausible mistakes in a copy of the
oracle source (CPU only), build each mutant, and check that every mutant fails
at least one pin of test_oracle_pins.py."""
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle as om
import tests.test_oracle_pins as pins

MUTANTS = {
    "r_ij sign (x only)": ("const double dx = x[i] - x[j];", "const double dx = x[j] - x[i];"),
    "inverse square law -> 1/r": ("const double inv3 = inv * inv * inv;", "const double inv3 = inv * inv;"),
    "self term kept": ("if (j == i) continue;", ""),
    "softening dropped in field": ("const double s2 = d2 + eps2;", "const double s2 = d2 + (phi ? eps2 : 0.0);"),
    "transposed component": ("neumaier_add(&sy, &cy, qj * dy * inv3);", "neumaier_add(&sy, &cy, qj * dx * inv3);"),
    "weight not applied": ("const double qj = w * q[j];", "const double qj = q[j];"),
    "drift without 1/2 (Eq. G)": ("x[i] = x[i] + vx[i] * dt + ax[i] * dt * dt / 2.0;",
                                   "x[i] = x[i] + vx[i] * dt + ax[i] * dt * dt;"),
    "kick uses new a only (Eq. H)": ("vx[i] = vx[i] + (ax[i] + bx[i]) * dt / 2.0;", "vx[i] = vx[i] + bx[i] * dt;"),
    "q/m inverted": ("const double qm = q[i] / m[i];", "const double qm = m[i] / q[i];"),
    "emittance sign (Eq. I)": ("const double e2 = xx * vv - xv * xv;", "const double e2 = xx * vv + xv * xv;"),
    "potential energy double counted": ("t[i] = 0.5 * w * q[i] * phi[i];", "t[i] = w * q[i] * phi[i];"),
    "kinetic energy without weight": ("0.5 * w * m[i] * (vx[i] * vx[i]", "0.5 * m[i] * (vx[i] * vx[i]"),
    "momentum without weight": ("t[i] = w * m[i] * v[a][i];", "t[i] = m[i] * v[a][i];"),
    "field magnitude sum drops |r_ij|": ("fabs(qj) * sqrt(d2) * inv3", "fabs(qj) * inv3"),
    "field magnitude sum drops |q|": ("fabs(qj) * sqrt(d2) * inv3", "qj * sqrt(d2) * inv3"),
    "potential magnitude sum drops |q|": ("fabs(qj) * inv);", "qj * inv);"),
    "potential magnitude sum drops softening": ("fabs(qj) * inv);", "fabs(qj) / sqrt(d2));"),
}

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

PIN_FUNCS = [
    pins.test_electron_field_at_one_micron,
    pins.test_two_charges_term_magnitudes_closed_form,
    lambda o: [pins.test_symmetric_polyhedra_closed_forms(o, s) for s in ("tetrahedron", "octahedron", "cube")],
    lambda o: [pins.test_brute_force_50_digits(o, e) for e in (0.0, 2e-7)],
    pins.test_force_is_minus_gradient_of_potential,
    pins.test_invariants,
    pins.test_two_body_trajectory_closed_form,
    pins.test_energy_error_second_order,
    pins.test_momentum_conserved,
    pins.test_emittance_closed_forms,
    pins.test_energy_momentum_com_closed_forms,
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(workdir, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(om.__file__), "pp_oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    tag = "".join(c if c.isalnum() else "_" for c in name)
    path = os.path.join(workdir, f"m_{tag}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = om.build(path, os.path.join(workdir, f"lib_{tag}.so"))
    mutant = om.Oracle(lib)
    failures = 0
    for fn in PIN_FUNCS:
        try:
            fn(mutant)
        except (AssertionError, ValueError, FloatingPointError, ZeroDivisionError):
            failures += 1
    assert failures > 0, f"no pin catches the planted mistake: {name}"

