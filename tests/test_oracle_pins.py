"""Pins of the CPU FP64 oracle against facts fixed by the paper and by
mathematics, not by the oracle itself (arXiv 2502.10640 Sec. 2.1-2.2).

Each test names the plausible oracle mistake it would catch.
"""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle.oracle import OracleState, default
from paper_2502_10640_amd import workloads as wl

def approx(expected, rel=None, abs=0.0):
    """pytest.approx without its default 1e-12 absolute slack (SI values here
    are often far below 1e-12)."""
    return pytest.approx(expected, rel=rel, abs=abs)


GOLD = os.path.join(os.path.dirname(__file__), "golden")
CF = json.load(open(os.path.join(GOLD, "closed_forms.json")))

E = wl.E_CHARGE
ME = wl.M_ELECTRON


@pytest.fixture(scope="module")
def orc():
    return default()


def _field(orc, pos, q, w=1.0, eps=0.0, **kw):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.broadcast_to(np.asarray(q, dtype=np.float64), (pos.shape[0],)).copy()
    return orc.field(pos[:, 0], pos[:, 1], pos[:, 2], q, w, eps, **kw)


def _vec(f):
    return np.stack([f["ex"], f["ey"], f["ez"]], axis=1)


# ---------------------------------------------------------------------------
# Coulomb's law, Eq. (A)/(B)
# ---------------------------------------------------------------------------

def test_coulomb_constant_codata(orc):
    # wrong eps0 or a missing 4 pi
    assert orc.k == approx(8.9875517923e9, rel=1e-10)


def test_electron_field_at_one_micron(orc):
    """Field of one electron 1 um away equals e/(4 pi eps0)/d^2 = 1439.96 V/m,
    pointing towards the electron (negative source); the force on a second
    electron is repulsive (Sec. 2.1: the bunch expands under repulsion).
    Catches: wrong sign of r_ij, wrong power of the distance, wrong constant."""
    f = _field(orc, [[0, 0, 0], [1e-6, 0, 0]], -E, want_phi=True)
    v = _vec(f)
    assert v[0, 0] == approx(CF["electron_field_at_1um"]["value_V_per_m"], rel=1e-9)
    assert v[1, 0] == approx(-CF["electron_field_at_1um"]["value_V_per_m"], rel=1e-9)
    assert np.all(v[:, 1:] == 0)
    force0 = -E * v[0, 0]          # electron at the origin, partner at +x
    assert force0 < 0              # pushed away from the partner
    # potential of the partner at each electron: -e/(4 pi eps0)/d
    assert f["phi"][0] == approx(-1.4399645478e-3, rel=1e-9)


def test_two_charges_term_magnitudes_closed_form(orc):
    """One pair of unlike charges with softening: at each particle the sum of
    the field terms' magnitudes is A = k |w q_j| d / (d^2 + eps^2)^(3/2) and that
    of the potential terms P = k |w q_j| / (d^2 + eps^2)^(1/2) (Sec. 2.1,
    Eq. (A) for one term).  Catches a magnitude sum that drops |r_ij|, drops the
    absolute value of the charge or drops the softening; the potential itself
    must keep the sign of the source charge."""
    k = 1.0 / (4.0 * math.pi * wl.EPS0)
    d, eps, w = 3e-6, 1.25e-6, 2.5
    qs = np.array([-E, 3.0 * E])
    f = _field(orc, [[0, 0, 0], [0, d, 0]], qs, w=w, eps=eps, want_phi=True, want_amag=True, want_pmag=True)
    s2 = d * d + eps * eps
    for i, j in ((0, 1), (1, 0)):
        assert f["amag"][i] == approx(k * abs(w * qs[j]) * d / s2 ** 1.5, rel=1e-14)
        assert f["pmag"][i] == approx(k * abs(w * qs[j]) / math.sqrt(s2), rel=1e-14)
        assert f["phi"][i] == approx(k * w * qs[j] / math.sqrt(s2), rel=1e-14)
    assert f["phi"][1] < 0 < f["pmag"][1]
    # |E| equals A for a single term
    mag = np.linalg.norm(_vec(f), axis=1)
    np.testing.assert_allclose(mag, f["amag"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("shape", ["tetrahedron", "octahedron", "cube"])
def test_symmetric_polyhedra_closed_forms(orc, shape):
    """Equidistant vertex sets with centroid at the origin: radial field
    |E| = C k Q / a^2 with C derived by hand.  Catches dropped terms, wrong
    index exclusion and wrong geometry factors."""
    a = 3e-6
    if shape == "tetrahedron":
        s = a / (2 * math.sqrt(2))
        pos = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) * s
        C = CF["tetrahedron_side_a"]["C"]
    elif shape == "octahedron":
        pos = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float) * a
        C = CF["octahedron_vertex_s"]["C"]
    else:
        pos = np.array([[i, j, k] for i in (-.5, .5) for j in (-.5, .5) for k in (-.5, .5)]) * a
        C = CF["cube_side_a"]["C"]
    key = {"tetrahedron": "tetrahedron_side_a", "octahedron": "octahedron_vertex_s", "cube": "cube_side_a"}[shape]
    CA, CP = CF[key]["CA"], CF[key]["CP"]
    Q = 2 * E
    f = _field(orc, pos, 2 * E, w=1.0, want_phi=True, want_amag=True, want_pmag=True)
    v = _vec(f)
    k = orc.k
    mag = np.linalg.norm(v, axis=1)
    np.testing.assert_allclose(mag, C * k * Q / a ** 2, rtol=1e-13)
    rhat = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    np.testing.assert_allclose(v / mag[:, None], rhat, atol=1e-13)  # outward for Q > 0
    # sums of the terms' magnitudes, and the potential (all terms of one sign)
    np.testing.assert_allclose(f["amag"], CA * k * Q / a ** 2, rtol=1e-13, atol=0)
    np.testing.assert_allclose(f["pmag"], CP * k * Q / a, rtol=1e-13, atol=0)
    np.testing.assert_allclose(f["phi"], CP * k * Q / a, rtol=1e-13, atol=0)


def _decimal_field(pos, q, w, eps, prec=50):
    getcontext().prec = prec
    k = Decimal(1) / (Decimal(4) * Decimal("3.14159265358979323846264338327950288419716939937510")
                      * Decimal("8.8541878128e-12"))
    P = [[Decimal(float(c)) for c in p] for p in pos]
    Qd = [Decimal(float(x)) * Decimal(float(w)) for x in q]
    e2 = Decimal(float(eps)) ** 2
    out, amag, pmag, phi = [], [], [], []
    for i in range(len(P)):
        acc = [Decimal(0)] * 3
        am, pm, ph = Decimal(0), Decimal(0), Decimal(0)
        for j in range(len(P)):
            if i == j:
                continue
            d = [P[i][c] - P[j][c] for c in range(3)]
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
            s = (r2 + e2).sqrt()
            f = Qd[j] / (s * s * s)
            acc = [acc[c] + f * d[c] for c in range(3)]
            am += abs(Qd[j]) * r2.sqrt() / (s * s * s)
            pm += abs(Qd[j]) / s
            ph += Qd[j] / s
        out.append([float(k * a) for a in acc])
        amag.append(float(k * am))
        pmag.append(float(k * pm))
        phi.append(float(k * ph))
    return np.array(out), np.array(amag), np.array(pmag), np.array(phi)


@pytest.mark.parametrize("eps", [0.0, 2e-7])
def test_brute_force_50_digits(orc, eps):
    """Tiny random bunch with mixed charges: agreement with a 50-digit decimal
    evaluation to within FP64 rounding of the result."""
    rng = np.random.default_rng(7)
    n = 13
    pos = rng.normal(size=(n, 3)) * 1e-6
    q = rng.choice([-1.0, 1.0, 2.0], size=n) * E
    f = _field(orc, pos, q, w=3.5, eps=eps, want_phi=True, want_amag=True, want_pmag=True)
    ref, ref_amag, ref_pmag, ref_phi = _decimal_field(pos, q, 3.5, eps)
    # the magnitude sums themselves, then each output relative to its own scale
    np.testing.assert_allclose(f["amag"], ref_amag, rtol=1e-15, atol=0)
    np.testing.assert_allclose(f["pmag"], ref_pmag, rtol=1e-15, atol=0)
    err = np.abs(_vec(f) - ref).max(axis=1) / ref_amag
    assert err.max() < 4e-16
    assert (np.abs(f["phi"] - ref_phi) / ref_pmag).max() < 4e-16


def test_force_is_minus_gradient_of_potential(orc):
    """E_i = -grad_i phi_i (the softened force derives from the softened
    potential): central differences of the oracle's own phi reproduce its E.
    Catches a wrong softening exponent or sign in either."""
    rng = np.random.default_rng(3)
    n = 40
    pos = rng.normal(size=(n, 3)) * 1e-5
    q = np.full(n, -E)
    eps = 3e-6
    f = _field(orc, pos, q, w=10.0, eps=eps)
    E0 = _vec(f)
    h = 1e-9
    for i in (0, 7, 21):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fp = _field(orc, pp, q, w=10.0, eps=eps, recv=[i], want_phi=True)["phi"][0]
            fm = _field(orc, pm, q, w=10.0, eps=eps, recv=[i], want_phi=True)["phi"][0]
            grad = (fp - fm) / (2 * h)
            assert -grad == approx(E0[i, c], rel=1e-6, abs=1e-6 * np.abs(E0[i]).max())


def test_invariants(orc):
    """Newton's third law, charge reversal, exact power-of-two scaling,
    permutation equivariance, receiver subsets."""
    rng = np.random.default_rng(11)
    n = 300
    pos = rng.normal(size=(n, 3)) * 2e-5
    q = rng.choice([-1.0, 1.0], size=n) * E
    w, eps = 7.0, 1e-7
    f = _field(orc, pos, q, w=w, eps=eps, want_amag=True)
    v = _vec(f)
    Qi = (w * q)[:, None]
    # sum_i Q_i E_i = 0 (antisymmetry of Eq. (A))
    tot = (Qi * v).sum(axis=0)
    assert np.abs(tot).max() <= 1e-13 * (np.abs(Qi[:, 0]) * f["amag"]).sum()
    # q -> -q flips E bit for bit
    np.testing.assert_array_equal(_vec(_field(orc, pos, -q, w=w, eps=eps)), -v)
    # r -> 2r and eps -> 2 eps give E / 4 exactly (power of two)
    np.testing.assert_array_equal(_vec(_field(orc, 2 * pos, q, w=w, eps=2 * eps)), v / 4)
    # permutation equivariance (summation order changes: rounding only)
    perm = rng.permutation(n)
    vp = _vec(_field(orc, pos[perm], q[perm], w=w, eps=eps))
    assert (np.abs(vp - v[perm]).max(axis=1) / f["amag"][perm]).max() < 1e-15
    # receiver subset = same values (i's own loop is unchanged)
    sub = np.array([5, 0, 299, 17])
    vs = _vec(_field(orc, pos, q, w=w, eps=eps, recv=sub))
    np.testing.assert_array_equal(vs, v[sub])


def test_paper_cube_symmetry(orc):
    """The paper's cell-centred cubic lattice (Sec. 2.1 setup) is symmetric under
    x -> -x and under x <-> y; the field must follow."""
    x, y, z = wl.cube_lattice(6, 1e-4)
    n = x.shape[0]
    q = np.full(n, -E)
    f = orc.field(x, y, z, q, 12.2, 0.0, want_amag=True)
    idx = {(round(a * 1e9), round(b * 1e9), round(c * 1e9)): i for i, (a, b, c) in enumerate(zip(x, y, z))}
    mx = np.array([idx[(round(-a * 1e9), round(b * 1e9), round(c * 1e9))] for a, b, c in zip(x, y, z)])
    sw = np.array([idx[(round(b * 1e9), round(a * 1e9), round(c * 1e9))] for a, b, c in zip(x, y, z)])
    tol = 1e-14 * f["amag"]
    assert np.all(np.abs(f["ex"][mx] + f["ex"]) <= tol)
    assert np.all(np.abs(f["ey"][mx] - f["ey"]) <= tol)
    assert np.all(np.abs(f["ey"][sw] - f["ex"]) <= tol)


def test_gauss_law_uniform_sphere(orc):
    """Inside a uniformly charged sphere the radial field is k Q_tot r / R^3
    (Gauss's law); the discrete sum reproduces it on average.  Catches a wrong
    power of the distance or a wrong total charge scaling."""
    b = wl.cold_sphere(6000, 100e-6, 1e8, 1e-3, 0.01, 0, seed=5)
    f = orc.field(b.x, b.y, b.z, b.q, b.weight, b.softening)
    r = np.sqrt(b.x ** 2 + b.y ** 2 + b.z ** 2)
    er = (f["ex"] * b.x + f["ey"] * b.y + f["ez"] * b.z) / r
    Qtot = b.weight * b.q.sum()
    inner = (r > 0.2e-4) & (r < 0.8e-4)
    ratio = er[inner] / (orc.k * Qtot * r[inner] / (100e-6) ** 3)
    assert np.median(ratio) == approx(1.0, abs=0.02)


# ---------------------------------------------------------------------------
# Velocity Verlet, Eqs. (G)/(H), and a = (q/m)E, Eq. (D)/(F)
# ---------------------------------------------------------------------------

def _two_body_time(xi, d0, C):
    return math.sqrt(d0 ** 3 / (2 * C)) * (math.sqrt(xi * (xi - 1)) + math.log(math.sqrt(xi) + math.sqrt(xi - 1)))


def _two_electrons(d0, w, dt):
    z = np.zeros(2)
    q, m = wl.electron_arrays(2)
    return OracleState(np.array([-d0 / 2, d0 / 2]), z, z, z, z, z, q, m, w, 0.0, dt)


def test_two_body_trajectory_closed_form(orc):
    """Two electrons released from rest: separation d(t) follows the closed
    form t(xi) of the 1/d^2 repulsion (energy conservation of the relative
    coordinate).  Error must shrink 4x when dt halves (second order).
    Catches a wrong q/m, a missing 1/2 in Eq. (G) or (H), a wrong sign."""
    d0, w = 1e-6, 5.0
    C = 2 * (1 / (4 * math.pi * wl.EPS0)) * w * E ** 2 / ME  # d'' = C / d^2
    T = 3 * math.sqrt(d0 ** 3 / (2 * C))
    xi_ref = brentq(lambda xi: _two_body_time(xi, d0, C) - T, 1 + 1e-12, 100, xtol=1e-15)
    errs = []
    for nsteps in (400, 800):
        s = _two_electrons(d0, w, T / nsteps)
        orc.vv(s, nsteps)
        xi = (s.x[1] - s.x[0]) / d0
        errs.append(abs(xi - xi_ref) / xi_ref)
        assert s.vx[1] > 0 > s.vx[0]
    assert errs[1] < 1e-5
    assert 3.5 < errs[0] / errs[1] < 4.5


def _small_sphere(n=64, seed=2, dt_omega=0.02):
    return wl.cold_sphere(n, 20e-6, 1e6, 0.05, dt_omega, 0, seed)


def _state(b):
    return OracleState(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.q, b.m, b.weight, b.softening, b.dt)


def test_energy_error_second_order(orc):
    """Softened energy is conserved up to O(dt^2): max |dE| over a fixed time
    span drops ~4x when dt halves."""
    b = _small_sphere()
    errs = []
    for k in (1, 2):
        s = _state(b)
        s.dt = b.dt / k
        e0 = orc.diag_state(s)["total"]
        worst = 0.0
        for _ in range(40):
            orc.vv(s, 5 * k)
            worst = max(worst, abs(orc.diag_state(s)["total"] - e0) / abs(e0))
        errs.append(worst)
    assert errs[0] < 1e-3
    assert 3.3 < errs[0] / errs[1] < 4.7


def test_momentum_conserved(orc):
    b = wl.gaussian_bunch(200, 5e-6, 1.0, 1e5, 0.01, 0.02, 0, seed=4)
    s = _state(b)
    p0 = np.array(orc.diag_state(s)["momentum"])
    scale = (b.weight * b.m * np.sqrt(b.vx ** 2 + b.vy ** 2 + b.vz ** 2)).sum()
    orc.vv(s, 60)
    p1 = np.array(orc.diag_state(s)["momentum"])
    assert np.abs(p1 - p0).max() < 1e-13 * scale


def test_time_reversible(orc):
    """Velocity Verlet is time-symmetric: n steps, reverse v, n steps returns
    to the start up to rounding."""
    b = _small_sphere(48, seed=9)
    s = _state(b)
    orc.vv(s, 30)
    s.vx, s.vy, s.vz = -s.vx, -s.vy, -s.vz
    s.a_valid = False
    orc.vv(s, 30)
    scale = np.abs(b.x).max()
    assert np.abs(s.x - b.x).max() < 1e-11 * scale
    assert np.abs(s.z - b.z).max() < 1e-11 * scale


def test_split_run_bitwise(orc):
    """50 + 50 steps equal 100 steps bit for bit (a(t) is carried over)."""
    b = _small_sphere(40, seed=13)
    s1, s2 = _state(b), _state(b)
    orc.vv(s1, 100)
    orc.vv(s2, 50)
    orc.vv(s2, 50)
    for f in ("x", "y", "z", "vx", "vy", "vz", "ax"):
        np.testing.assert_array_equal(getattr(s1, f), getattr(s2, f))


def _sphere_xi(omega_t):
    return brentq(lambda xi: math.sqrt(1.5) * (math.sqrt(xi * (xi - 1)) +
                  math.log(math.sqrt(xi) + math.sqrt(xi - 1))) - omega_t, 1 + 1e-14, 10, xtol=1e-15)


def test_uniform_sphere_self_similar_expansion(orc):
    """Cold uniform sphere (the 2 048-particle workload, 100 steps of
    0.01/omega_p): radii scale by xi(omega_p t) of the shell model; at
    omega_p t = 1, xi = 1.15838726."""
    assert _sphere_xi(1.0) == approx(CF["uniform_sphere_xi_at_omega_t_1"]["value"], abs=1e-8)
    b = wl.workload("cold_sphere_2048")[0]
    s = _state(b)
    r0 = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
    checks = {25: 0.25, 100: 1.0}
    done = 0
    for step, wt in checks.items():
        orc.vv(s, step - done)
        done = step
        r = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
        assert r / r0 == approx(_sphere_xi(wt), rel=5e-3)


# ---------------------------------------------------------------------------
# Diagnostics, Eq. (I) and the Sec. 3.2 observables
# ---------------------------------------------------------------------------

def test_emittance_closed_forms(orc):
    """Eq. (I) on hand-made phase-space sets: a correlated line has zero
    emittance; an uncorrelated cross has <x^2><v^2> = 1/4 -> 1/2."""
    q, m = wl.electron_arrays(4)
    z = np.zeros(4)
    d = orc.diag(np.array([1., -1, 2, -2]), z, z, np.array([3., -3, 6, -6]), z, z, q, m, 1.0, 1e-6)
    assert d["emittance"][0] == approx(0.0, abs=1e-12)
    d = orc.diag(np.array([1., -1, 0, 0]), z, z, np.array([0., 0, 1, -1]), z, z, q, m, 1.0, 1e-6)
    assert d["emittance"][0] == approx(0.5, rel=1e-15)
    assert d["x_rms"][0] == approx(math.sqrt(0.5), rel=1e-15)
    assert d["v_rms"][0] == approx(math.sqrt(0.5), rel=1e-15)
    assert d["x_max"][0] == 1.0 and d["v_max"][0] == 1.0
    # raw (as printed) vs centred moments after a shift of x
    d = orc.diag(np.array([6., 4, 5, 5]), z, z, np.array([0., 0, 1, -1]), z, z, q, m, 1.0, 1e-6)
    assert d["emittance_centered"][0] == approx(0.5, rel=1e-14)
    # raw: <x^2> = 25.5, <v^2> = 0.5, <xv> = 0 -> sqrt(12.75)
    assert d["emittance"][0] == approx(math.sqrt(12.75), rel=1e-14)


def test_energy_momentum_com_closed_forms(orc):
    q, m = wl.electron_arrays(2)
    w = 3.0
    x = np.array([0.0, 2e-6])
    z = np.zeros(2)
    vx = np.array([1e5, -3e5])
    d = orc.diag(x, z, z, vx, z, z, q, m, w, 0.0)
    assert d["kinetic"] == approx(0.5 * w * ME * (1e10 + 9e10), rel=1e-15)
    # PE of two macro-electrons: k (w e)^2 / d
    assert d["potential"] == approx((1 / (4 * math.pi * wl.EPS0)) * (w * E) ** 2 / 2e-6, rel=1e-12)
    assert d["momentum"][0] == approx(w * ME * (1e5 - 3e5), rel=1e-15)
    assert d["com"][0] == approx(1e-6, rel=1e-15)
    assert d["com_velocity"][0] == approx(-1e5, rel=1e-15)
    assert d["nonfinite"] == 0
    x2 = x.copy()
    x2[1] = np.nan
    assert orc.diag(x2, z, z, vx, z, z, q, m, w, 0.0)["nonfinite"] == 1


def test_thread_count_independent(orc):
    """Each receiver's sum runs in j order, so thread count cannot change bits."""
    import subprocess
    import sys
    code = ("import numpy as np, sys; sys.path.insert(0, %r);"
            "from oracle.oracle import default;"
            "rng=np.random.default_rng(1); p=rng.normal(size=(3,500));"
            "f=default().field(p[0],p[1],p[2],np.ones(500),1.0,0.1);"
            "sys.stdout.write(f['ex'].tobytes().hex()[:4000])") % os.path.dirname(GOLD.rstrip('/')).rsplit('/tests', 1)[0]
    outs = []
    for nt in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   text=True, check=True).stdout)
    assert outs[0] == outs[1] and len(outs[0]) > 100


def test_set_num_threads_keeps_bits(orc):
    """The in-process thread setter (used for the serial CPU rate) changes the
    thread count, not the results."""
    before = orc.num_threads()
    rng = np.random.default_rng(2)
    p = rng.normal(size=(3, 700))
    q = rng.choice([-1.0, 1.0], size=700)
    try:
        outs = []
        for nt in (1, 5):
            orc.set_num_threads(nt)
            assert orc.num_threads() == nt
            f = orc.field(p[0], p[1], p[2], q, 1.0, 0.05, want_phi=True)
            outs.append(b"".join(f[k].tobytes() for k in ("ex", "ey", "ez", "phi")))
        assert outs[0] == outs[1]
        with pytest.raises(ValueError):
            orc.set_num_threads(0)
    finally:
        orc.set_num_threads(before)
