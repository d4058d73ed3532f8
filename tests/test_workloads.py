"""Input generators: the paper's printed setup arithmetic, seeding and the
centre-of-mass frame."""
import json
import math
import os

import numpy as np
import pytest

from paper_2502_10640_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_setup.json")))


def test_paper_cube_weight_16():
    g = GOLD["cube_16"]
    b = wl.paper_cube(g["n_side"], g["side_m"], g["density_m3"], g["dt_s"])
    assert b.n == g["n_p"]
    assert round(b.weight, 1) == g["weight_approx"]
    assert b.dt == g["dt_s"]
    assert np.all(b.vx == 0) and np.all(b.vy == 0) and np.all(b.vz == 0)
    assert np.all(np.abs(b.x) < g["side_m"] / 2)


def test_paper_cube_weight_32():
    b = wl.paper_cube(GOLD["cube_32"]["n_side"])
    assert round(b.weight, 2) == GOLD["cube_32"]["weight_approx"]


def test_paper_cube_spacing_8():
    x, y, z = wl.cube_lattice(GOLD["cube_8_spacing"]["n_side"], 1e-4)
    assert z[1] - z[0] == pytest.approx(GOLD["cube_8_spacing"]["spacing_m"], rel=1e-12, abs=0)
    assert wl.paper_cube(8).meta["spacing"] == pytest.approx(12.5e-6, rel=1e-12, abs=0)


def test_named_workload_constants():
    """Derived constants of the named workloads (plasma frequency from the
    electron density, spacing from the volume, eps and dt from them)."""
    b = wl.workload("cold_sphere_2048")[0]
    assert b.n == 2048
    assert b.meta["omega_p"] == pytest.approx(2.7564e11, rel=1e-4, abs=0)
    assert b.dt == pytest.approx(3.6279e-14, rel=1e-4, abs=0)
    assert b.softening == pytest.approx(1.2694e-8, rel=1e-4, abs=0)
    assert b.weight == pytest.approx(1e8 / 2048, rel=1e-15, abs=0)
    g = wl.workload("gaussian_65536", n_override=4096)[0]
    assert g.meta["omega_p"] == pytest.approx(1.2715e12, rel=1e-4, abs=0)
    # paper's run: dt = 1e-13 s at n0 = 5e16 m^-3 gives omega_p dt ~ 1.26e-3
    assert wl.plasma_frequency(5e16) * 1e-13 == pytest.approx(1.2614e-3, rel=1e-3, abs=0)


def test_seeded_and_centred():
    a = wl.workload("gaussian_65536", n_override=5000)[0]
    b = wl.workload("gaussian_65536", n_override=5000)[0]
    for u, v in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(u, v)
    for arr, scale in ((a.x, 50e-6), (a.vz, 4.2e5)):
        assert abs(arr.mean()) < 1e-15 * scale
    assert np.std(a.x) == pytest.approx(50e-6, rel=0.05, abs=0)
    sv = math.sqrt(wl.EV / wl.M_ELECTRON)
    assert np.std(a.vx) == pytest.approx(sv, rel=0.05, abs=0)
    s = wl.workload("cold_sphere_2048")[0]
    r = np.sqrt(s.x ** 2 + s.y ** 2 + s.z ** 2)
    assert r.max() < 100e-6 * 1.02  # recentring moves the origin by ~R/sqrt(N)
    # uniform in volume: median radius = R / 2^(1/3)
    assert np.median(r) == pytest.approx(100e-6 / 2 ** (1 / 3), rel=0.03, abs=0)


def test_sweep_sizes():
    sizes = wl.sweep_sizes()
    assert len(sizes) == 64
    assert min(sizes) >= 4096 and max(sizes) <= 131072
    assert sizes == wl.sweep_sizes()
    bunches = wl.workload("sweep_64", n_override=4)
    assert [b.n for b in bunches] == sizes[:4]
    assert [round(b.meta["dt_omega"], 4) for b in bunches] == list(wl.SWEEP_DT)
    arrays, offsets = wl.concat(bunches)
    assert offsets[1] == (sizes[0], sizes[1])
    assert arrays[0].shape[0] == sum(sizes[:4])
