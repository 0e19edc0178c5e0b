"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is a closed form, a
conservation law, a continuum limit, a library routine computing the same
definition another way, or brute force.  CPU only.
"""
import math

import numpy as np
import pytest
from scipy import integrate

PI = math.pi


# ---------------------------------------------------------------- kernels --

@pytest.mark.parametrize("h", [0.3, 1.0, 2.5])
def test_cubic_spline_normalised(orc, h):
    # Sec. 2.2: the kernel integrates to one over space.
    val, _ = integrate.quad(lambda r: 4 * PI * r * r * orc.W(r, h), 0, 2 * h, points=[h],
                            epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10
    assert orc.W(2 * h, h) == 0.0 and orc.W(2.5 * h, h) == 0.0   # compact support


@pytest.mark.parametrize("h", [0.7, 1.3])
def test_cubic_spline_smooth(orc, h):
    # Continuity of W, W' and W'' at xi = 1 and of W, W' at xi = 2, and
    # dW/dxi -> 0 as xi -> 0 (Sec. 2.2).  Together with the normalisation
    # these fix the piecewise cubic uniquely.
    f = lambda xi: orc.W(xi * h, h)
    d = 1e-5
    for xi0 in (1.0, 2.0):
        assert abs(f(xi0 - 1e-9) - f(xi0 + 1e-9)) < 1e-7 / h ** 3
        left = (f(xi0) - f(xi0 - d)) / d
        right = (f(xi0 + d) - f(xi0)) / d
        assert abs(left - right) < 1e-3 / h ** 3
    l2 = (f(1 - 2 * d) - 2 * f(1 - d) + f(1)) / d ** 2
    r2 = (f(1) - 2 * f(1 + d) + f(1 + 2 * d)) / d ** 2
    assert abs(l2 - r2) < 1e-2 / h ** 3
    assert abs((f(1e-6) - f(0)) / 1e-6) < 1e-4 / h ** 3
    assert f(0.0) > f(0.5) > f(1.0) > f(1.5) > f(2.0) == 0.0


@pytest.mark.parametrize("h", [0.4, 1.0, 3.0])
def test_spiky_kernel_normalised_and_derivative(orc, h):
    val, _ = integrate.quad(lambda r: 4 * PI * r * r * orc.Wp(r, h), 0, 2 * h,
                            epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) < 1e-10
    # dW_p/dxi must be the derivative of W_p with respect to xi = r/h.
    for xi in (0.0, 0.3, 1.0, 1.7, 1.99):
        d = 1e-6
        num = (orc.Wp((xi + d) * h, h) - orc.Wp(max(xi - d, 0.0) * h, h)) / (xi + d - max(xi - d, 0.0))
        assert abs(num - orc.dWp_dxi(xi * h, h)) < 1e-5 * abs(orc.dWp_dxi(0.0, h))
    # non-zero slope at the origin: the reason the paper uses W_p for forces
    assert orc.dWp_dxi(0.0, h) < 0.0
    assert orc.dWp_dxi(2.0 * h, h) == 0.0


# -------------------------------------------------------------- predicate --

def test_predicate_ties_and_symmetry(orc):
    # cut = h_i + h_j exactly representable: a pair at exactly that distance
    # is not a neighbour (xi < 2 is strict), one ulp closer is.
    p0 = (0.0, 0.0, 0.0)
    assert not orc.pred(p0, 0.5, (1.0, 0.0, 0.0), 0.5)
    assert orc.pred(p0, 0.5, (np.nextafter(np.float32(1.0), np.float32(0)).item(), 0.0, 0.0), 0.5)
    assert not orc.pred(p0, 0.25, (0.0, 0.0, 0.5), 0.25)
    assert not orc.pred(p0, 0.5, (0.0, 0.0, 0.0 + 1.0), 0.5)
    rng = np.random.default_rng(1)
    for _ in range(2000):
        a = rng.normal(size=3) * 3
        b = a + rng.normal(size=3) * 0.3
        ha, hb = rng.uniform(0.01, 0.3, 2)
        assert orc.pred(a, ha, b, hb) == orc.pred(b, hb, a, ha)


def test_predicate_matches_geometry_away_from_boundary(orc):
    # Away from |r| = h_i + h_j the FP32 test equals the exact FP64 geometry.
    rng = np.random.default_rng(2)
    n_checked = 0
    for _ in range(5000):
        a = rng.uniform(-10, 10, 3)
        b = a + rng.normal(size=3) * 0.2
        ha, hb = rng.uniform(0.01, 0.2, 2)
        r = np.linalg.norm(a - b)
        if abs(r - (ha + hb)) < 1e-5 * (ha + hb):
            continue
        n_checked += 1
        assert orc.pred(a, ha, b, hb) == (r < ha + hb)
    assert n_checked > 4900


# ------------------------------------------------------- grid, sort, rows --

def _clustered(rng, n):
    """Dense core + sparse envelope + exact duplicates: variable h over ~20x."""
    r = rng.pareto(2.5, n) * 0.3
    u = rng.normal(size=(n, 3))
    pos = u / np.linalg.norm(u, axis=1)[:, None] * r[:, None]
    pos[n // 10: n // 10 + 20] = pos[0]          # coincident particles
    h = 0.02 + 0.08 * r + rng.uniform(0, 0.01, n)
    return pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), h


@pytest.mark.parametrize("scale", [0, -1, 1])
def test_grid_rule_properties(orc, scale):
    rng = np.random.default_rng(3)
    x, y, z, h = _clustered(rng, 3000)
    g = orc.grid(x, y, z, h, scale)
    gd = orc.grid_dict(g)
    key, lev = orc.keys(x, y, z, h, g)
    t = h * (2.0 + 2.0 ** -9)
    L0 = gd["L0"]
    assert math.frexp(L0)[0] == 0.5                          # power of two
    assert L0 >= t.min() and L0 / 2 < t.min()
    L = L0 * 2.0 ** lev
    assert np.all(L >= t)
    assert np.all((lev == 0) | (L / 2 < t))                   # first level that fits
    # the cell side of level l is L0 2^(l + scale); levels do not depend on it
    np.testing.assert_array_equal(gd["L"], L0 * 2.0 ** (np.arange(gd["nlev"]) + scale))
    np.testing.assert_array_equal(lev, orc.keys(x, y, z, h, orc.grid(x, y, z, h))[1])
    # every particle lies inside its cell
    for l in range(gd["nlev"]):
        sel = lev == l
        if not sel.any():
            assert gd["ncell"][l] == 0
            continue
        Ll, o, dim, base = gd["L"][l], gd["org"][l], gd["dim"][l], gd["base"][l]
        loc = key[sel].astype(np.int64) - base
        cx = loc % dim[0]
        cy = (loc // dim[0]) % dim[1]
        cz = loc // (dim[0] * dim[1])
        for c, p, d in ((cx, x[sel], 0), (cy, y[sel], 1), (cz, z[sel], 2)):
            assert np.all(o[d] + c * Ll <= p) and np.all(p < o[d] + (c + 1) * Ll)
            assert np.all((c >= 0) & (c < dim[d]))
        assert np.all(loc < gd["ncell"][l])
    assert gd["M"] == gd["ncell"].sum()


def test_counting_sort_matches_library(orc):
    rng = np.random.default_rng(4)
    x, y, z, h = _clustered(rng, 5000)
    s = orc.sort_gas(x, y, z, h)
    M = s["grid"].M
    np.testing.assert_array_equal(s["count"], np.bincount(s["key"], minlength=M))
    np.testing.assert_array_equal(s["off"], np.concatenate([[0], np.cumsum(s["count"])]))
    np.testing.assert_array_equal(s["perm"], np.argsort(s["key"], kind="stable"))
    hm = np.zeros(M)
    np.maximum.at(hm, s["key"], h)
    np.testing.assert_array_equal(s["hmax"], hm)


def test_neighbour_rows_two_methods_agree(orc):
    rng = np.random.default_rng(5)
    for n in (1, 2, 50, 3000):
        x, y, z, h = _clustered(rng, max(n, 30))
        x, y, z, h = x[:n], y[:n], z[:n], h[:n]
        a = orc.nbrs_brute(x, y, z, h)
        b = orc.nbrs_kdtree(x, y, z, h)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        off, idx = a
        rows = [set(idx[off[i]:off[i + 1]].tolist()) for i in range(n)]
        for i in range(n):
            r = idx[off[i]:off[i + 1]]
            assert i not in rows[i]
            assert np.all(np.diff(r) > 0)
            for j in r:
                assert i in rows[j]                                  # symmetric


def test_slot_rows(orc):
    rng = np.random.default_rng(6)
    x, y, z, h = _clustered(rng, 1500)
    s = orc.sort_gas(x, y, z, h)
    off, idx = orc.nbrs_brute(x, y, z, h)
    soff, sidx = orc.rows_to_slots(s["perm"], off, idx)
    perm = s["perm"]
    for sl in range(0, 1500, 7):
        got = perm[sidx[soff[sl]:soff[sl + 1]]]
        exp = idx[off[perm[sl]]:off[perm[sl] + 1]]
        np.testing.assert_array_equal(np.sort(got), exp)
        assert np.all(np.diff(sidx[soff[sl]:soff[sl + 1]]) > 0)


# ------------------------------------------------------------------ SPH ----

def _lattice(n, d):
    g = np.arange(n) * d
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


@pytest.mark.parametrize("hd,tol", [(1.2, 2e-3), (1.5, 3e-3), (2.0, 3e-4)])
def test_lattice_density_normalisation(orc, hd, tol):
    # Uniform lattice of spacing d and particle mass m: the SPH density of an
    # interior particle (Eq. SPH-mass-density, self term included) tends to
    # m/d^3 as h/d grows, by the kernel's normalisation.  Dropping the self
    # term, using h_i + h_j instead of the mean, or a wrong kernel constant
    # each moves it by > 5%.
    n, d = 13, 0.1
    x, y, z = _lattice(n, d)
    N = len(x)
    m = np.full(N, 2.0 * d ** 3)
    h = np.full(N, hd * d)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)
    c = (n // 2) * n * n + (n // 2) * n + n // 2
    assert abs(rho[c] / 2.0 - 1.0) < tol


@pytest.mark.parametrize("hd,tol", [(1.5, 0.025), (2.0, 0.006)])
def test_lattice_pressure_gradient_limit(orc, hd, tol):
    # Eq. (dv_dt): a = -grad p / rho.  Uniform density, e linear in x, so
    # p = (gamma-1) rho e has gradient (gamma-1) rho k along x: the SPH sum of
    # Eq. (dv_dt-SPH) must approach -(gamma-1) k at an interior particle.
    # Pins the sign, the W_p normalisation, the 1/h_ij of grad W_p.
    n, d, gam, k = 14, 0.1, 5.0 / 3.0, 0.3
    x, y, z = _lattice(n, d)
    N = len(x)
    m = np.full(N, d ** 3)
    h = np.full(N, hd * d)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)
    zero = np.zeros(N)
    ax, ay, az, de = orc.sph_force(x, y, z, zero, zero, zero, m, h, rho, 1.0 + k * x,
                                   gam, 1.0, 2.0, 0.1, off, idx)
    c = (n // 2) * n * n + (n // 2) * n + n // 2
    expect = -(gam - 1) * k
    assert abs(ax[c] / expect - 1) < tol
    assert abs(ay[c]) < 1e-12 and abs(az[c]) < 1e-12


@pytest.mark.parametrize("hd,tol", [(1.5, 0.025), (2.0, 0.006)])
def test_lattice_divergence_limit(orc, hd, tol):
    # Eq. (de_dt): de/dt = -(p/rho) div v.  Uniform expansion v = c r has
    # div v = 3c and r.v > 0 for every pair, so the viscosity is off and
    # Eq. (de_dt-SPH) must approach -3 c p / rho.  Pins the 1/2 and the sign.
    n, d, gam, cdiv = 14, 0.1, 5.0 / 3.0, 0.2
    x, y, z = _lattice(n, d)
    N = len(x)
    m = np.full(N, d ** 3)
    h = np.full(N, hd * d)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)
    e = np.ones(N)
    ax, ay, az, de = orc.sph_force(x, y, z, cdiv * x, cdiv * y, cdiv * z, m, h, rho, e,
                                   gam, 1.0, 2.0, 0.1, off, idx)
    c = (n // 2) * n * n + (n // 2) * n + n // 2
    p = (gam - 1) * rho[c] * e[c]
    assert abs(de[c] / (-3 * cdiv * p / rho[c]) - 1) < tol
    # compression heats, and viscosity adds to the heating
    ax2, _, _, de2 = orc.sph_force(x, y, z, -cdiv * x, -cdiv * y, -cdiv * z, m, h, rho, e,
                                   gam, 0.0, 0.0, 0.1, off, idx)
    ax3, _, _, de3 = orc.sph_force(x, y, z, -cdiv * x, -cdiv * y, -cdiv * z, m, h, rho, e,
                                   gam, 1.0, 2.0, 0.1, off, idx)
    assert abs(de2[c] / (3 * cdiv * p / rho[c]) - 1) < tol
    assert de3[c] > de2[c] > 0


def _gas_blob(rng, n):
    x, y, z, h = _clustered(rng, n)
    m = rng.uniform(0.5, 1.5, n) / n
    v = rng.normal(size=(n, 3)) * 0.3
    e = rng.uniform(0.02, 0.1, n)
    return x, y, z, v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy(), m, h, e


def test_sph_conservation_laws(orc):
    # Pi_ij symmetric and grad W_p antisymmetric: total momentum and angular
    # momentum are conserved exactly, and sum m (v.a + de/dt) = 0 pins the
    # 1/2 of Eq. (de_dt-SPH) against the momentum equation.
    rng = np.random.default_rng(7)
    x, y, z, vx, vy, vz, m, h, e = _gas_blob(rng, 2000)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)
    ax, ay, az, de = orc.sph_force(x, y, z, vx, vy, vz, m, h, rho, e, 5 / 3, 1.0, 2.0, 0.1, off, idx)
    scale = np.sum(m * np.sqrt(ax ** 2 + ay ** 2 + az ** 2))
    for comp in (ax, ay, az):
        assert abs(np.sum(m * comp)) < 1e-12 * scale
    r = np.stack([x, y, z], 1)
    a = np.stack([ax, ay, az], 1)
    Lz = np.sum(m[:, None] * np.cross(r, a), axis=0)
    assert np.all(np.abs(Lz) < 1e-12 * np.sum(m * np.linalg.norm(r, axis=1) * np.linalg.norm(a, axis=1)))
    work = m * (vx * ax + vy * ay + vz * az)
    heat = m * de
    assert abs(np.sum(work + heat)) < 1e-11 * (np.sum(np.abs(work)) + np.sum(np.abs(heat)))
    # Galilean invariance
    ax2, ay2, az2, de2 = orc.sph_force(x, y, z, vx + 3.0, vy - 1.0, vz, m, h, rho, e,
                                       5 / 3, 1.0, 2.0, 0.1, off, idx)
    np.testing.assert_allclose(ax2, ax, rtol=1e-9, atol=1e-12 * np.abs(ax).max())
    np.testing.assert_allclose(de2, de, rtol=1e-9, atol=1e-12 * np.abs(de).max())


def test_two_particle_sph_closed_form(orc):
    # Two gas particles on the x axis at -1/2 and +1/2 with h = m = e = 1,
    # gamma = 5/3, alpha = 1, beta = 2, eta = 0.1, worked by hand from the
    # density sum (self term included), the ideal-gas law, the viscosity
    # (mu with r^2 + eta h^2 in the denominator, as printed), the momentum
    # and energy equations (Sec. 2.2), with xi = 1:
    #   W(0) = 1/pi, W(1) = 1/(4 pi)  ->  rho = 5/(4 pi), p = 5/(6 pi),
    #   p/rho^2 = 8 pi/15, c = sqrt(gamma (gamma - 1) e) = sqrt(10)/3,
    #   grad_i W_p = -(45/(64 pi)) r_ij/|r_ij| = +45/(64 pi) x  (r_ij = -x).
    # Receding (v_i = -1/4, v_j = +1/4): no viscosity, Pi = 16 pi/15, so
    #   a_i = -Pi 45/(64 pi) = -3/4 and de_i/dt = Pi (v_ij . grad W)/2 = -3/16.
    # Approaching (v_i = +1/4, v_j = -1/4): mu = -0.5/1.1 = -5/11 and
    #   nu = mu (beta mu - alpha c)/rho = (4 pi/11)(10/11 + sqrt(10)/3).
    x = np.array([-0.5, 0.5]); y = np.zeros(2); z = np.zeros(2)
    m = np.ones(2); h = np.ones(2); e = np.ones(2)
    off = np.array([0, 1, 2], dtype=np.int64); idx = np.array([1, 0], dtype=np.int32)
    rho = orc.density(x, y, z, m, h, off, idx)
    np.testing.assert_allclose(rho, 5 / (4 * PI), rtol=1e-15)
    p, c = orc.eos(rho, e, 5 / 3)
    np.testing.assert_allclose(p / rho ** 2, 8 * PI / 15, rtol=1e-14)
    np.testing.assert_allclose(c, math.sqrt(10) / 3, rtol=1e-14)
    zero = np.zeros(2)

    def force(v):
        return orc.sph_force(x, y, z, np.array([v, -v]), zero, zero, m, h, rho, e,
                             5 / 3, 1.0, 2.0, 0.1, off, idx)
    ax, ay, az, de = force(-0.25)
    np.testing.assert_allclose(ax, [-0.75, 0.75], rtol=1e-14)
    np.testing.assert_allclose(de, [-3 / 16, -3 / 16], rtol=1e-14)
    assert np.all(ay == 0) and np.all(az == 0)
    ax, ay, az, de = force(0.25)
    Pi = 16 * PI / 15 + (4 * PI / 11) * (10 / 11 + math.sqrt(10) / 3)
    g = 45 / (64 * PI)
    np.testing.assert_allclose(ax, [-g * Pi, g * Pi], rtol=1e-14)
    np.testing.assert_allclose(de, [0.25 * g * Pi, 0.25 * g * Pi], rtol=1e-14)


def test_viscosity_scaling(orc):
    # nu = mu (beta mu - alpha c)/rho_ij: the alpha part of the heating is
    # linear in alpha and the beta part scales as |v|^3 (mu ~ v, mu^2 dv ~ v^3).
    rng = np.random.default_rng(8)
    x, y, z, vx, vy, vz, m, h, e = _gas_blob(rng, 800)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)

    def heat(a, b, s):
        return orc.sph_force(x, y, z, s * vx, s * vy, s * vz, m, h, rho, e, 5 / 3, a, b, 0.1,
                             off, idx)[3]
    base1 = heat(0, 0, 1.0)
    da1 = heat(1, 0, 1.0) - base1
    da2 = heat(2, 0, 1.0) - base1
    np.testing.assert_allclose(da2, 2 * da1, rtol=1e-9, atol=1e-14)
    db1 = heat(0, 1, 1.0) - base1
    base2 = heat(0, 0, 2.0)
    db2 = heat(0, 1, 2.0) - base2
    np.testing.assert_allclose(db2, 8 * db1, rtol=1e-9, atol=1e-14)
    assert np.sum(m * da1) > 0 and np.sum(m * db1) > 0          # dissipative


# -------------------------------------------------------------- gravity ----

def test_gravity_two_body_closed_form(orc):
    G, eps = 1.7, 0.05
    x = np.array([0.0, 0.6]); y = np.zeros(2); z = np.zeros(2)
    m = np.array([2.0, 3.0])
    ax, ay, az, pot = orc.gravity(x, y, z, m, G, eps)
    d2 = 0.36 + eps * eps
    assert abs(ax[0] - G * 3.0 * 0.6 / d2 ** 1.5) < 1e-14
    assert abs(ax[1] + G * 2.0 * 0.6 / d2 ** 1.5) < 1e-14
    assert abs(pot[0] + G * 3.0 / math.sqrt(d2)) < 1e-14
    assert ay[0] == 0 and az[1] == 0


def test_gravity_newton_third_law(orc):
    rng = np.random.default_rng(9)
    n = 3000
    x, y, z = rng.normal(size=(3, n))
    m = rng.uniform(0.1, 1.0, n)
    ax, ay, az, pot = orc.gravity(x, y, z, m, 1.0, 0.01)
    for comp in (ax, ay, az):
        assert abs(np.sum(m * comp)) < 1e-13 * np.sum(m * np.abs(comp))
    r = np.stack([x, y, z], 1)
    a = np.stack([ax, ay, az], 1)
    L = np.sum(m[:, None] * np.cross(r, a), axis=0)
    assert np.all(np.abs(L) < 1e-13 * np.sum(m * np.linalg.norm(r, 1) * np.linalg.norm(a, 1)))
    # subset evaluation agrees with the full one
    t = np.array([5, 17, 2999, 0])
    bx, by, bz, bp = orc.gravity(x, y, z, m, 1.0, 0.01, targets=t)
    np.testing.assert_array_equal(bx, ax[t])
    np.testing.assert_array_equal(bp, pot[t])


def _plummer_menc(r, a, rt):
    X = lambda s: s ** 3 / (s * s + a * a) ** 1.5
    return np.minimum(X(r), X(rt)) / X(rt)


def test_gravity_plummer_profile(orc):
    # Radial field of a sampled (truncated) Plummer sphere against
    # -G M(<r)/r^2 in radial shells: statistical, softening O(eps^2).
    from paper_1807_08116_amd import ic
    rng = np.random.default_rng(10)
    pos, m = ic.plummer(12000, 1.0, 1.0, rng)
    x, y, z = pos.T.copy()
    ax, ay, az, pot = orc.gravity(x, y, z, m, 1.0, 0.01)
    r = np.linalg.norm(pos, axis=1)
    ar = (ax * x + ay * y + az * z) / r
    for lo, hi in ((0.3, 0.6), (0.6, 1.0), (1.0, 1.6), (1.6, 3.0)):
        sel = (r > lo) & (r < hi)
        ratio = np.mean(-ar[sel] * r[sel] ** 2 / _plummer_menc(r[sel], 1.0, 5.0))
        assert abs(ratio - 1) < 0.03, (lo, hi, ratio)
    # potential energy of the truncated sphere: -G int M(r) dM(r) / r
    rt = 5.0
    Xt = rt ** 3 / (rt * rt + 1.0) ** 1.5          # Plummer mass fraction inside rt
    dens = lambda s: 3.0 / (4 * PI) * (1 + s * s) ** -2.5 / Xt
    Wint, _ = integrate.quad(lambda s: -_plummer_menc(s, 1.0, rt) * 4 * PI * s * dens(s), 0, rt)
    Wsim = 0.5 * np.sum(m * pot)
    assert abs(Wsim / Wint - 1) < 0.02


# ----------------------------------------------------------- integrator ----

def test_predictor_corrector_second_order_kepler(orc):
    # Halo-only eccentric two-body orbit: the scheme is second order in dt
    # (Sec. 2.2), so the position error at a fixed time falls ~4x when dt
    # halves (reference: the same scheme at a 32x smaller step).
    prm = dict(G=1.0, eps=1e-4, gamma=5 / 3, alpha=1, beta=2, eta=0.1)

    def run(dt, t_end=1.2):
        v = 0.35                       # below the circular speed 0.5: eccentric
        st = {"ng": 0, "x": np.array([-0.5, 0.5]), "y": np.zeros(2), "z": np.zeros(2),
              "vx": np.zeros(2), "vy": np.array([-v, v]), "vz": np.zeros(2),
              "m": np.array([0.5, 0.5]), "e": np.zeros(0), "h": np.zeros(0)}
        cache = None
        for _ in range(int(round(t_end / dt))):
            st, cache = orc.pc_step(st, prm, dt, cache)
        return np.array([st["x"][1], st["y"][1]])
    ref = run(0.02 / 32)
    e_a = np.linalg.norm(run(0.02) - ref)
    e_b = np.linalg.norm(run(0.01) - ref)
    assert 3.3 < e_a / e_b < 4.7, e_a / e_b


def test_diagnostics_closed_form(orc):
    x = np.array([1.0, -1.0]); y = np.zeros(2); z = np.zeros(2)
    vx = np.zeros(2); vy = np.array([1.0, -1.0]); vz = np.zeros(2)
    m = np.array([1.0, 1.0]); e = np.array([0.25])
    pot = np.array([-0.5, -0.5])
    d = orc.diagnostics(x, y, z, vx, vy, vz, m, e, pot, 1)
    np.testing.assert_allclose(d, [1.0, 0.25, -0.5, 0.75, 0, 0, 0, 0, 0, 2.0], atol=1e-15)


# --------------------------------------------------------- step control ----

def test_cfl_lattice_at_rest_closed_form(orc):
    # Eq. (dt-stability) on a lattice at rest with no forces: s_i = d, all
    # c_ij = c, mu = 0, Q = E = 0, so dt = C d / (c (1 + 1.2 alpha)).
    n, d = 6, 0.1
    x, y, z = _lattice(n, d)
    N = len(x)
    h = np.full(N, 0.75 * d)
    off, idx = orc.nbrs_brute(x, y, z, h)
    c = np.full(N, 0.3)
    zero = np.zeros(N)
    for C, alpha in ((0.5, 1.0), (0.8, 0.5)):
        dt = orc.cfl_dt(x, y, z, zero, zero, zero, h, c, zero, zero, zero, zero, C, alpha, 2.0,
                        0.1, off, idx)
        assert abs(dt - C * d / (0.3 * (1 + 1.2 * alpha))) < 1e-15
    # an acceleration and a compressive pair can only shorten the step
    q = np.zeros(N)
    q[5] = 4.0
    v = np.zeros(N)
    v[7] = 1.0
    dt0 = orc.cfl_dt(x, y, z, zero, zero, zero, h, c, zero, zero, zero, zero, 0.5, 1, 2, 0.1, off, idx)
    dt1 = orc.cfl_dt(x, y, z, zero, zero, zero, h, c, q, zero, zero, zero, 0.5, 1, 2, 0.1, off, idx)
    dt2 = orc.cfl_dt(x, y, z, v, zero, zero, h, c, zero, zero, zero, zero, 0.5, 1, 2, 0.1, off, idx)
    assert dt1 < dt0 and dt2 < dt0
    # no neighbours at all: no constraint
    far = np.arange(3) * 10.0
    o1, i1 = orc.nbrs_brute(far, far * 0, far * 0, np.full(3, 0.1))
    assert orc.cfl_dt(far, far * 0, far * 0, *([np.zeros(3)] * 3), np.full(3, 0.1), np.ones(3),
                      *([np.zeros(3)] * 4), 0.5, 1, 2, 0.1, o1, i1) == float("inf")


def test_h_update_lattice(orc):
    # h = sigma (m/rho)^(1/3): on a lattice rho -> m/d^3, so h -> sigma d.
    n, d = 13, 0.1
    x, y, z = _lattice(n, d)
    N = len(x)
    m = np.full(N, d ** 3)
    h = np.full(N, 1.5 * d)
    off, idx = orc.nbrs_brute(x, y, z, h)
    rho = orc.density(x, y, z, m, h, off, idx)
    hn = orc.update_h(m, rho, 1.25)
    c = (n // 2) * n * n + (n // 2) * n + n // 2
    assert abs(hn[c] / (1.25 * d) - 1) < 1e-3
    assert np.all(orc.update_h(m, rho, 2.5) == 2 * hn)          # linear in sigma


@pytest.mark.parametrize("h", [0.5, 2.0])
def test_kernel_values_golden(orc, h):
    # Hand-evaluated values of the printed kernels (tests/golden/kernel_values.txt).
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "kernel_values.txt")
    rows = np.loadtxt(path, comments="#")
    scale = PI * h ** 3
    for xi, w, wp, dwp in rows:
        assert abs(orc.W(xi * h, h) * scale - w) < 1e-14
        assert abs(orc.Wp(xi * h, h) * scale - wp) < 1e-14
        assert abs(orc.dWp_dxi(xi * h, h) * scale - dwp) < 1e-14


# ------------------------------ unequal smoothing lengths, masses, energies --
# Hand-derived closed forms for a pair with h_1 != h_2, m_1 != m_2 and
# e_1 != e_2 (derivation in tests/golden/two_particle_unequal.md, Sec. 2.2):
# they fix h_ij = (h_i + h_j)/2 in the density and in grad W_p, the means
# rho_ij and c_ij of the viscosity, and which mass enters each sum.

def _unequal_pair(v1):
    x = np.array([-0.75, 0.75]); y = np.zeros(2); z = np.zeros(2)
    m = np.array([1.0, 2.0]); h = np.array([1.0, 3.0]); e = np.array([1.0, 2.0])
    vx = np.array([v1, -v1])
    off = np.array([0, 1, 2], dtype=np.int64); idx = np.array([1, 0], dtype=np.int32)
    return x, y, z, vx, m, h, e, off, idx


UNEQ_RHO = np.array([1145.0 / (1024.0 * PI), 7363.0 / (55296.0 * PI)])
UNEQ_P = 2048.0 * PI / 3435.0 + 73728.0 * PI / 7363.0       # P_1 + P_2
UNEQ_G = 1125.0 / (16384.0 * PI)                             # |grad W_p|


def test_two_particle_unequal_density(orc):
    x, y, z, vx, m, h, e, off, idx = _unequal_pair(0.0)
    assert orc.pred((x[0], 0, 0), h[0], (x[1], 0, 0), h[1])     # |r| < h_1 + h_2
    rho = orc.density(x, y, z, m, h, off, idx)
    np.testing.assert_allclose(rho, UNEQ_RHO, rtol=1e-15)
    p, c = orc.eos(rho, e, 5 / 3)
    np.testing.assert_allclose(p / rho ** 2, [2048 * PI / 3435, 73728 * PI / 7363], rtol=1e-14)
    np.testing.assert_allclose(c, [math.sqrt(10) / 3, math.sqrt(20) / 3], rtol=1e-15)


@pytest.mark.parametrize("approaching", [False, True])
def test_two_particle_unequal_forces(orc, approaching):
    x, y, z, vx, m, h, e, off, idx = _unequal_pair(0.25 if approaching else -0.25)
    zero = np.zeros(2)
    ax, ay, az, de = orc.sph_force(x, y, z, vx, zero, zero, m, h, UNEQ_RHO, e,
                                   5 / 3, 1.0, 2.0, 0.1, off, idx)
    Pi = UNEQ_P
    if approaching:
        mu = -30.0 / 53.0
        c12 = (math.sqrt(10) + math.sqrt(20)) / 6
        rho12 = 0.5 * (UNEQ_RHO[0] + UNEQ_RHO[1])
        Pi += mu * (2.0 * mu - 1.0 * c12) / rho12
    g = UNEQ_G
    np.testing.assert_allclose(ax, [-2 * Pi * g, Pi * g], rtol=1e-14)
    sgn = 1.0 if approaching else -1.0
    np.testing.assert_allclose(de, [sgn * Pi * g / 2, sgn * Pi * g / 4], rtol=1e-14)
    assert np.all(ay == 0) and np.all(az == 0)
    # the energy identity holds for the unequal pair as well
    assert abs(np.sum(m * (vx * ax + de))) < 1e-14 * np.sum(m * np.abs(de))


def test_cfl_unequal_pair_closed_form(orc):
    # Eq. (dt-stability) with every term non-zero (derivation in
    # tests/golden/two_particle_unequal.md): s = 1/2, c_max = 0.4,
    # |mu|_max = 10/7, and particle 2's sqrt(s (|Q| + |E|)) = 2 binds.
    x = np.array([-0.25, 0.25]); y = np.zeros(2); z = np.zeros(2)
    vx = np.array([0.5, -0.5]); zero = np.zeros(2)
    h = np.ones(2); c = np.array([0.3, 0.5])
    qx = np.array([3.0, 0.0]); qy = np.array([4.0, 0.0]); E = np.array([1.0, -8.0])
    off = np.array([0, 1, 2], dtype=np.int64); idx = np.array([1, 0], dtype=np.int32)
    dt = orc.cfl_dt(x, y, z, vx, zero, zero, h, c, qx, qy, zero, E, 0.6, 1.0, 2.0, 0.1,
                    off, idx)
    expect = 0.3 / (0.88 + 24.0 / 7.0 + 2.0)
    assert abs(dt / expect - 1) < 1e-15, (dt, expect)
    # with particle 2 at rest in Q and E, particle 1's root term sqrt(1/2 * 6)
    # binds: |Q_1| is the vector norm 5 (not |3| + |4|)
    dt1 = orc.cfl_dt(x, y, z, vx, zero, zero, h, c, qx, qy, zero, np.array([1.0, 0.0]),
                     0.6, 1.0, 2.0, 0.1, off, idx)
    expect1 = 0.3 / (0.88 + 24.0 / 7.0 + math.sqrt(3.0))
    assert abs(dt1 / expect1 - 1) < 1e-15, (dt1, expect1)


def _pair_state(v1):
    x, y, z, vx, m, h, e, off, idx = _unequal_pair(v1)
    return {"ng": 2, "x": x, "y": y, "z": z, "vx": vx, "vy": np.zeros(2), "vz": np.zeros(2),
            "m": m, "h": h, "e": e}


@pytest.mark.parametrize("approaching,t_end", [(False, 0.4), (True, 0.1)])
def test_gas_predictor_corrector_second_order(orc, approaching, t_end):
    # Eqs. (v-predictor)..(e-corrector) on a gas-only system (G = 0: the
    # pair above, receding, or approaching with the viscosity switched on
    # for the whole interval).  The scheme is second order, so its error at
    # t_end against a tight DOP853 solution of the same equations of motion
    # (dr/dt = v, dv/dt = Q, de/dt = E, with Q and E the oracle's sums at
    # the current state, density refreshed at the current positions) falls
    # ~4x per halving of dt, in the positions, velocities and energies.
    from scipy.integrate import solve_ivp
    prm = dict(G=0.0, eps=0.01, gamma=5 / 3, alpha=1.0, beta=2.0, eta=0.1)
    st0 = _pair_state(0.25 if approaching else -0.25)

    def rhs(t, yv):
        st = dict(st0)
        st["x"], st["vx"], st["e"] = yv[0:2].copy(), yv[2:4].copy(), yv[4:6].copy()
        f = orc.forces(st, prm)
        ax, _, _ = orc.total_accel(st, f)
        return np.concatenate([yv[2:4], ax, f["dedt"]])

    y0 = np.concatenate([st0["x"], st0["vx"], st0["e"]])
    sol = solve_ivp(rhs, (0.0, t_end), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    ref = sol.y[:, -1]
    if approaching:
        assert np.all(sol.y[2, :] - sol.y[3, :] > 0)          # r.v < 0 throughout

    def run(dt):
        st, cache = st0, None
        for _ in range(int(round(t_end / dt))):
            st, cache = orc.pc_step(st, prm, dt, cache)
        return np.concatenate([st["x"], st["vx"], st["e"]])

    errs = []
    for dt in (t_end / 20, t_end / 40, t_end / 80):
        d = run(dt) - ref
        errs.append([np.max(np.abs(d[0:2])), np.max(np.abs(d[2:4])), np.max(np.abs(d[4:6]))])
    errs = np.array(errs)
    for k, name in enumerate(("x", "v", "e")):
        for a, b in ((0, 1), (1, 2)):
            ratio = errs[a, k] / errs[b, k]
            assert 3.3 < ratio < 4.7, (name, errs[:, k])
