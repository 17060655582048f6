"""Pins of the oracle's pore model (Secs. 4-5 of the paper): the boundary
trace against closed-form ballistic paths, the all-pairs forces against the
pinned 3D all-pairs function, the dimer closed form and minus the energy
gradient, and the integrator and thermostat against invariants and closed
forms.  CPU only."""
import math

import numpy as np
import pytest

import oracle


def fold(u, lo, hi):
    """Position after specular reflections between walls at lo and hi of a
    point whose unfolded coordinate is u."""
    w = hi - lo
    q = np.mod(u - lo, 2.0 * w)
    return lo + np.where(q <= w, q, 2.0 * w - q)


def free_run(model, x0, v0, steps):
    """A single atom (no partner, so no force) stepped by the oracle,
    recording its position after every step."""
    xs, vs = [], []
    x, v = np.array([x0], dtype=float), np.array([v0], dtype=float)
    for _ in range(steps):
        x, v, _ = oracle.pm_run(model, x, v, 1, every=0)
        xs.append(x[0].copy())
        vs.append(v[0].copy())
    return np.array(xs), np.array(vs)


def test_reflection_between_pore_walls_closed_form():
    """An atom moving along y inside the pore bounces between y = 0 and
    y = ly: y(t) is the folded straight line and v_y flips at each wall."""
    m = oracle.pm_model(2, lx=8.0, ly=4.0, k=1.0, dt=0.125)
    xs, vs = free_run(m, [2.0, 1.0], [0.0, -3.0], 200)
    t = 0.125 * np.arange(1, 201)
    assert np.abs(xs[:, 0] - 2.0).max() == 0.0
    assert np.abs(xs[:, 1] - fold(1.0 - 3.0 * t, 0.0, 4.0)).max() <= 1e-12
    # the sign of v_y is the direction of the folded line at the step's end
    u = np.mod(1.0 - 3.0 * t, 8.0)
    expected = np.where(u < 4.0, -3.0, 3.0)
    mid = np.abs(xs[:, 1] - np.round(xs[:, 1] / 4.0) * 4.0) > 1e-9  # not exactly on a wall
    assert np.array_equal(vs[mid, 1], expected[mid])


def test_corner_reflection_closed_form():
    """Diagonal motion into the corner (0, 0) of the pore: each axis folds on
    its own."""
    m = oracle.pm_model(2, lx=8.0, ly=8.0, k=1.0, dt=0.0625)
    xs, _ = free_run(m, [1.5, 0.75], [-2.0, -2.0], 40)
    t = 0.0625 * np.arange(1, 41)
    assert np.abs(xs[:, 0] - fold(1.5 - 2.0 * t, 0.0, 8.0)).max() <= 1e-12
    assert np.abs(xs[:, 1] - fold(0.75 - 2.0 * t, 0.0, 8.0)).max() <= 1e-12


def test_outer_space_periodic_in_y_and_x():
    """In the outer space, y is periodic with period (2k+1) ly from -k ly, and
    x (outside the mouth) is periodic with period k lx from lx."""
    k, lx, ly = 2.0, 6.0, 4.0
    m = oracle.pm_model(2, lx=lx, ly=ly, k=k, dt=0.25)
    xs, vs = free_run(m, [10.0, 3.0], [0.0, 5.0], 100)
    t = 0.25 * np.arange(1, 101)
    assert np.abs(xs[:, 1] - (-k * ly + np.mod(3.0 + k * ly + 5.0 * t, (2 * k + 1) * ly))).max() <= 1e-11
    assert np.all(vs[:, 1] == 5.0)
    # leftwards below the mouth (y = -2): wraps from x = lx to x = (k+1) lx
    xs, vs = free_run(m, [9.0, -2.0], [-1.5, 0.0], 100)
    assert np.abs(xs[:, 0] - (lx + np.mod(9.0 - lx - 1.5 * t, k * lx))).max() <= 1e-11
    assert np.all(vs[:, 0] == -1.5)


def test_round_trip_through_the_mouth():
    """An atom heading left inside the mouth enters the pore, reflects at
    x = 0, leaves through the mouth and then circulates rightwards in the
    outer space (re-entering at x = lx it is moving away from the pore)."""
    k, lx, ly = 1.0, 6.0, 4.0
    m = oracle.pm_model(2, lx=lx, ly=ly, k=k, dt=0.25)
    x0, v = lx + 1.0, 1.0
    xs, vs = free_run(m, [x0, 2.0], [-v, 0.0], 120)
    t = 0.25 * np.arange(1, 121)
    t_in, t_wall = (x0 - lx) / v, x0 / v  # entering the pore, hitting x = 0
    exp = np.where(t <= t_wall, x0 - v * t, v * (t - t_wall))
    out = v * (t - t_wall) >= lx
    exp = np.where(out, lx + np.mod(v * (t - t_wall) - lx, k * lx), exp)
    assert np.abs(xs[:, 0] - exp).max() <= 1e-11
    assert np.all(vs[t < t_wall, 0] == -v) and np.all(vs[t > t_wall, 0] == v)
    # the pore count of the records follows the same times
    x, vv, rec = oracle.pm_run(m, [[x0, 2.0]], [[-v, 0.0]], 120, every=1)
    inside = (t > t_in) & (t < t_wall + lx / v)
    assert np.array_equal(rec[1:, 3].astype(bool), inside)
    assert rec[-1, 4] == 1.0  # one wall reflection


def test_3d_mouth_is_bounded_in_z():
    """In 3D the mouth also needs 0 <= z < lz: an atom heading left at z
    above the mouth wraps instead of entering the pore."""
    m = oracle.pm_model(3, lx=6.0, ly=4.0, lz=4.0, k=1.0, dt=0.25)
    p, v, r = oracle.pm_trace(m, [6.5, 2.0, 5.0], [-1.0, 0.0, 0.0], [-4.0, 0.0, 0.0])
    assert np.allclose(p, [11.5, 2.0, 5.0], rtol=0, atol=1e-12) and r == 0
    p, v, r = oracle.pm_trace(m, [6.5, 2.0, 3.0], [-1.0, 0.0, 0.0], [-4.0, 0.0, 0.0])
    assert np.allclose(p, [5.5, 2.0, 3.0], rtol=0, atol=1e-12) and r == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_free_particles_stay_in_the_domain_with_their_speeds(dim):
    """Non-interacting atoms (epsilon = 0) from random states: after 3000
    steps every atom is inside the pore or the outer space, its speed is
    unchanged (reflections and wraps keep |v|), and walls were hit."""
    rng = np.random.default_rng(4)
    lx, ly, lz, k = 5.0, 3.0, 3.0, 1.0
    m = oracle.pm_model(dim, lx, ly, lz, k=k, epsilon=0.0, dt=0.01)
    n = 300
    x = np.empty((n, dim))
    x[:, 0] = rng.uniform(0.0, (k + 1) * lx, n)
    inside = x[:, 0] < lx
    for a, l in ((1, ly), (2, lz))[:dim - 1]:
        x[:, a] = np.where(inside, rng.uniform(0.0, l, n), rng.uniform(-k * l, (k + 1) * l, n))
    v = rng.normal(0.0, 3.0, (n, dim))
    x1, v1, rec = oracle.pm_run(m, x, v, 3000, every=3000)
    assert np.allclose(np.linalg.norm(v1, axis=1), np.linalg.norm(v, axis=1), rtol=1e-13)
    pore = x1[:, 0] < lx
    for a, l in ((1, ly), (2, lz))[:dim - 1]:
        assert np.all(x1[pore, a] >= 0) and np.all(x1[pore, a] <= l)
        assert np.all(x1[~pore, a] >= -k * l) and np.all(x1[~pore, a] < (k + 1) * l)
    assert np.all(x1[:, 0] >= 0) and np.all(x1[:, 0] < (k + 1) * lx)
    assert rec[-1, 3] == pore.sum() and rec[-1, 4] > 100


def test_3d_forces_equal_the_pinned_all_pairs_function():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 6.0, (40, 3))
    m = oracle.pm_model(3, 10.0, 10.0, 10.0, epsilon=1.3, sigma=0.9)
    f, u, e = oracle.pm_forces(m, x)
    fr, ur, er = oracle.allpairs(x, (0.0, 0.0, 0.0), 1.3, 0.9)
    assert np.array_equal(f, fr) and np.array_equal(u, ur) and e == er


def test_2d_dimer_closed_form():
    m = oracle.pm_model(2, 10.0, 10.0)
    c, s = math.cos(0.7), math.sin(0.7)
    for r, uexp, fexp in ((1.0, 0.0, 24.0), (2 ** (1 / 6), -1.0, 0.0), (1.5, -0.320336594278575, -1.15802883104616)):
        x = np.array([[3.0, 3.0], [3.0 + r * c, 3.0 + r * s]])
        f, u, e = oracle.pm_forces(m, x)
        assert e == pytest.approx(uexp, abs=1e-11)
        # force on atom 0 along the unit vector from 1 to 0 (positive: repulsive)
        assert np.dot(f[0], [-c, -s]) == pytest.approx(fexp, abs=1e-10)
        assert np.allclose(f[0], -f[1], rtol=0, atol=1e-13)


def test_2d_forces_are_minus_the_energy_gradient():
    rng = np.random.default_rng(2)
    g = np.stack(np.meshgrid(np.arange(6), np.arange(5), indexing="ij"), -1).reshape(-1, 2)
    x = 1.2 * g + rng.uniform(-0.15, 0.15, g.shape)
    m = oracle.pm_model(2, 20.0, 20.0)
    f, _, _ = oracle.pm_forces(m, x)
    h = 1e-6
    for i in (0, 7, 29):
        for a in (0, 1):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            de = (oracle.pm_forces(m, xp)[2] - oracle.pm_forces(m, xm)[2]) / (2 * h)
            assert -de == pytest.approx(f[i, a], rel=1e-6, abs=1e-7)
    assert np.abs(f.sum(axis=0)).max() <= 1e-11 * np.abs(f).sum()


def _lattice_gas(dim, n_side, a=1.15):
    g = np.stack(np.meshgrid(*[np.arange(n_side)] * dim, indexing="ij"), -1).reshape(-1, dim)
    return 0.6 + a * g


@pytest.mark.parametrize("dim", [2, 3])
def test_nve_energy_error_is_second_order(dim):
    """Interacting atoms in the middle of a large pore, never reaching a wall
    within the run: velocity Verlet with the all-pairs forces, whose largest
    energy deviation over a fixed time falls by about four when dt halves."""
    n_side = 6 if dim == 2 else 4
    x = _lattice_gas(dim, n_side) + 20.0
    rng = np.random.default_rng(8)
    v = rng.normal(0.0, 1.0, x.shape)
    devs = []
    for dt in (0.004, 0.002):
        m = oracle.pm_model(dim, 48.0, 48.0, 48.0, k=1.0, dt=dt)
        _, _, r = oracle.pm_run(m, x, v, int(round(1.0 / dt)), every=1)
        assert r[-1, 4] == 0 and r[-1, 3] == len(x)
        e = r[:, 1] + r[:, 2]
        devs.append(np.abs(e - e[0]).max() / abs(e[0]))
    assert devs[0] < 1e-3
    assert 3.5 < devs[0] / devs[1] < 4.5


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_with_wall_reflections(dim):
    """The same gas packed near the walls of a small pore: a reflection keeps
    the kinetic energy, but a half step's kick taken before the normal
    velocity flips leaves an O(dt) energy error per wall hit, so the error
    is first order in dt; it stays small and shrinks as dt does."""
    n_side = 6 if dim == 2 else 4
    x = _lattice_gas(dim, n_side)
    rng = np.random.default_rng(8)
    v = rng.normal(0.0, 1.0, x.shape)
    devs = []
    for dt in (0.004, 0.001):
        m = oracle.pm_model(dim, 8.0, 8.0, 8.0, k=1.0, dt=dt)
        _, _, r = oracle.pm_run(m, x, v, int(round(1.0 / dt)), every=1)
        assert r[-1, 4] > 0  # walls were hit
        e = r[:, 1] + r[:, 2]
        devs.append(np.abs(e - e[0]).max() / abs(e[0]))
    assert devs[0] < 1e-3 and devs[1] < devs[0] / 1.5


def test_berendsen_free_gas_closed_form():
    """Free atoms (epsilon = 0): F3 leaves v unchanged and reflections keep
    |v|, so the temperature the thermostat measures at step s follows
    T_s = t0 + (1 - dt/tau)^(s-1) (T_1 - t0)."""
    rng = np.random.default_rng(3)
    n, dim = 200, 3
    x = np.empty((n, dim))
    x[:, 0] = rng.uniform(0.0, 5.0, n)
    x[:, 1:] = rng.uniform(0.0, 5.0, (n, 2))
    v = rng.normal(0.0, 2.0, (n, dim))
    dt, tau, t0 = 0.01, 0.25, 1.5
    m = oracle.pm_model(dim, 5.0, 5.0, 5.0, k=1.0, epsilon=0.0, dt=dt, tau=tau, t0=t0)
    _, _, rec = oracle.pm_run(m, x, v, 60, every=1)
    T = 2.0 * rec[1:, 1] / (dim * n)
    T1 = float(np.sum(v * v)) / (dim * n)
    s = np.arange(1, 61)
    assert np.allclose(T, t0 + (1 - dt / tau) ** (s - 1) * (T1 - t0), rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_pore_pressure_ideal_gas_limit(dim):
    """epsilon = 0: no virial, so the pore pressure is 2 K_pore / (d V), i.e.
    rho T over the molecules in the pore (the ideal-gas law)."""
    rng = np.random.default_rng(6)
    lx, ly, lz = 7.0, 5.0, 4.0
    m = oracle.pm_model(dim, lx, ly, lz, k=1.0, epsilon=0.0, dt=0.01)
    n = 150
    x = np.empty((n, dim))
    x[:, 0] = rng.uniform(0.0, 2 * lx, n)
    inside = x[:, 0] < lx
    for a, l in ((1, ly), (2, lz))[:dim - 1]:
        x[:, a] = np.where(inside, rng.uniform(0.0, l, n), rng.uniform(-l, 2 * l, n))
    v = rng.normal(0.0, 1.3, (n, dim))
    x1, v1, rec = oracle.pm_run(m, x, v, 50, every=25)
    V = lx * ly * (lz if dim == 3 else 1.0)
    for xs, vs, r in ((x, v, rec[0]), (x1, v1, rec[-1])):
        p = xs[:, 0] < lx
        T_pore = np.sum(vs[p] ** 2) / (dim * p.sum())
        assert r[5] == pytest.approx(p.sum() * T_pore / V, rel=1e-13)


def test_pore_pressure_of_a_dimer_closed_form():
    """Two molecules at rest at distance r: inside the pore the pressure is
    r f(r) / (d V) with r f(r) = 24 eps (2 (s/r)^12 - (s/r)^6); with one of
    them outside (across the mouth) it is half of that."""
    lx, ly = 8.0, 6.0
    m = oracle.pm_model(2, lx, ly, k=1.0, dt=1e-9)
    for r in (1.0, 1.1, 1.5):
        rf = 24.0 * (2.0 * r ** -12 - r ** -6)
        _, _, rec = oracle.pm_run(m, [[3.0, 3.0], [3.0 + r, 3.0]], np.zeros((2, 2)), 0)
        assert rec[0, 5] == pytest.approx(rf / (2 * lx * ly), rel=1e-13)
        _, _, rec = oracle.pm_run(m, [[lx - 0.4, 3.0], [lx - 0.4 + r, 3.0]], np.zeros((2, 2)), 0)
        assert rec[0, 3] == 1
        assert rec[0, 5] == pytest.approx(0.5 * rf / (2 * lx * ly), rel=1e-13)


def test_pore_virial_is_minus_the_scaling_derivative_of_the_energy():
    """For molecules all in the pore, sum_{i<j} r_ij . f_ij = -dU(lambda x) /
    d lambda at lambda = 1 (the virial theorem's pair term), so
    (P - 2 K / (d V)) d V equals minus the derivative by central
    differences."""
    rng = np.random.default_rng(12)
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(3), indexing="ij"), -1)
    x = 1.0 + 1.1 * g.reshape(-1, 3) + rng.uniform(-0.1, 0.1, (48, 3))
    m = oracle.pm_model(3, 8.0, 8.0, 8.0, k=1.0, dt=1e-9)
    _, _, rec = oracle.pm_run(m, x, np.zeros_like(x), 0)
    W = rec[0, 5] * 3 * 8.0 ** 3
    h = 1e-6
    dU = (oracle.pm_forces(m, (1 + h) * x)[2] - oracle.pm_forces(m, (1 - h) * x)[2]) / (2 * h)
    assert W == pytest.approx(-dU, rel=1e-7)
