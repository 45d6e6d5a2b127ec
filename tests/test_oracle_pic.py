"""Pins of the oracle's particle coupling (CPU only): the relativistic Boris
push and the charge-conserving deposition against properties that hold
exactly, and Gauss's law of the coupled particle-field step (Appendix A:
with a charge-conserving current the scheme keeps D.(A_E E) - 4 pi rho
constant; with a filtered current the conserved density is the filtered one).
The divergences, the total current and the rotation angle are written out
here, independently of the oracle."""
import math

import numpy as np
import pytest

from oracle import ref

from oracle_helpers import gauss_E_lhs_2d


def _cfg(shape=(20, 24), d=(1.0, 1.0), dt=None, **kw):
    if dt is None:
        dt = 0.6 / math.sqrt(1.0 / d[0] ** 2 + 1.0 / d[1] ** 2)
    return ref.Config(ndim=2, shape=shape, dt=dt, d=d, **kw)


def _zeros(cfg, k=3):
    return [np.zeros(cfg.shape) for _ in range(k)]


def _particles(rng, cfg, n, umax=2.0):
    ny, nx = cfg.shape
    x = rng.uniform(0, nx * cfg.d[0], n)
    y = rng.uniform(0, ny * cfg.d[1], n)
    u = [rng.uniform(-umax, umax, n) for _ in range(3)]
    return x, y, u


def _div_J(cfg, J):
    """D.J at the nodes (i, j) for J placed like E, cells dx x dy."""
    dx, dy = cfg.d[0], cfg.d[1]
    return (J[0] - np.roll(J[0], 1, axis=1)) / dx + (J[1] - np.roll(J[1], 1, axis=0)) / dy


def _rho(cfg, q, w, x, y):
    r = np.zeros(cfg.shape)
    ref.pic_deposit_charge(cfg, q, w, x, y, r)
    return r


@pytest.mark.parametrize("d", [(1.0, 1.0), (0.7, 1.3)])
def test_deposition_satisfies_discrete_continuity(d):
    """(rho^{n+1} - rho^n)/dt + D.J^{n+1/2} = 0 at every node to rounding,
    for particles in every direction, across cell edges and the periodic
    boundary, on square and anisotropic cells (no fields: ballistic moves)."""
    rng = np.random.default_rng(11)
    cfg = _cfg(d=d)
    E, B, J = _zeros(cfg), _zeros(cfg), _zeros(cfg)
    x, y, u = _particles(rng, cfg, 400, umax=5.0)
    ny, nx = cfg.shape
    # a few on nodes, on cell edges and at the domain edge
    x[:4] = [0.0, d[0] * 3, d[0] * (nx - 1e-9), d[0] * 7.5]
    y[:4] = [d[1] * 2, 0.0, d[1] * (ny - 1e-9), d[1] * 4.0]
    q, m, w = -1.3, 0.7, 0.25
    rho0 = _rho(cfg, q, w, x, y)
    ref.pic_push_deposit(cfg, E, B, q, m, w, x, y, *u, J)
    rho1 = _rho(cfg, q, w, x, y)
    res = (rho1 - rho0) / cfg.dt + _div_J(cfg, J)
    scale = np.abs(rho1 - rho0).max() / cfg.dt
    assert scale > 0
    assert np.abs(res).max() <= 1e-13 * scale


def test_total_current_is_the_particle_current():
    """sum J dx dy = sum q w v^{n+1/2} per component (the first moment of the
    linear shape is the position; the out-of-plane weights sum to one)."""
    rng = np.random.default_rng(12)
    cfg = _cfg(d=(0.8, 1.1))
    E, B, J = _zeros(cfg), _zeros(cfg), _zeros(cfg)
    x, y, u = _particles(rng, cfg, 50)
    q, m, w = 2.0, 3.0, 0.5
    u0 = [a.copy() for a in u]
    ref.pic_push_deposit(cfg, E, B, q, m, w, x, y, *u, J)
    for a, b in zip(u0, u):   # no field: the momenta are unchanged
        assert np.array_equal(a, b)
    g = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    area = cfg.d[0] * cfg.d[1]
    for c in range(3):
        want = q * w * np.sum(u[c] / g)
        assert J[c].sum() * area == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_boris_rotation_in_a_uniform_magnetic_field():
    """B = B0 z: |u| and gamma are kept, and the in-plane momentum turns by
    -2 atan(q B0 dt / (2 m gamma)) per step (clockwise for q B0 > 0), so
    after n steps it is the start vector rotated by n times that angle."""
    cfg = _cfg(shape=(8, 8))
    E, B = _zeros(cfg), _zeros(cfg)
    B0, q, m = 0.8, 1.5, 1.2
    B[2][:] = B0
    x, y = np.array([3.3]), np.array([4.1])
    u = [np.array([0.9]), np.array([-0.4]), np.array([0.3])]
    gam = math.sqrt(1.0 + 0.9 ** 2 + 0.4 ** 2 + 0.3 ** 2)
    th = -2.0 * math.atan(q * B0 * cfg.dt / (2.0 * m * gam))
    nsteps = 40
    for _ in range(nsteps):
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
    c, s = math.cos(nsteps * th), math.sin(nsteps * th)
    want = (c * 0.9 - s * (-0.4), s * 0.9 + c * (-0.4), 0.3)
    for a, b in zip(u, want):
        assert a[0] == pytest.approx(b, abs=1e-13)


def test_boris_kick_in_a_uniform_electric_field():
    """B = 0, E uniform (so B^n = 0): each step adds (q dt / m) E exactly."""
    cfg = _cfg(shape=(8, 10))
    E, B = _zeros(cfg), _zeros(cfg)
    Ev = (0.3, -0.2, 0.05)
    for c in range(3):
        E[c][:] = Ev[c]
    q, m = -0.5, 2.0
    x, y = np.array([1.2, 5.5]), np.array([3.3, 0.4])
    u = [np.array([0.1, -0.2]), np.array([0.0, 0.3]), np.array([0.2, 0.0])]
    u0 = [a.copy() for a in u]
    for n in range(1, 6):
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
        for c in range(3):
            np.testing.assert_allclose(u[c], u0[c] + n * q * cfg.dt / m * Ev[c], rtol=0, atol=1e-14)


def test_exb_drift():
    """Crossed uniform E = E0 y and B = B0 z: a particle starting at rest
    drifts at E x B / B^2 = (E0 / B0) x on average over whole gyrations."""
    cfg = _cfg(shape=(8, 64), dt=0.05)
    E, B = _zeros(cfg), _zeros(cfg)
    E0, B0, q, m = 0.004, 1.0, 1.0, 1.0
    E[1][:] = E0
    B[2][:] = B0
    x, y = np.array([10.0]), np.array([4.0])
    u = [np.zeros(1), np.zeros(1), np.zeros(1)]
    period = 2.0 * math.pi * m / (q * B0)
    nsteps = int(round(10 * period / cfg.dt))
    x_un = 0.0
    for _ in range(nsteps):
        x_prev = x[0]
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
        dxs = x[0] - x_prev
        if dxs < -cfg.shape[1] / 2:
            dxs += cfg.shape[1] * cfg.d[0]
        x_un += dxs
    v_mean = x_un / (nsteps * cfg.dt)
    assert v_mean == pytest.approx(E0 / B0, rel=2e-3)


@pytest.mark.parametrize("p", [0, 2])
def test_coupled_step_keeps_gauss_law(p):
    """Two species of opposite charge coupled to the field step with a
    converged mass-matrix solve: D.(A_E E) - 4 pi F^p rho stays at its
    initial value over the steps (rho from the particles' positions, F the
    current's filter, so the filtered charge obeys continuity with the
    filtered current)."""
    rng = np.random.default_rng(20 + p)
    cfg = _cfg(shape=(20, 24), sweeps=400, tol=1e-14, filter_passes=p)
    E = [rng.normal(0, 0.05, cfg.shape) for _ in range(3)]
    B = [rng.normal(0, 0.05, cfg.shape) for _ in range(3)]
    species = []
    for q in (1.0, -1.0):
        x, y, u = _particles(rng, cfg, 300, umax=1.0)
        species.append([q, 1.0, 0.02, x, y, u])

    def g_of():
        rho = np.zeros(cfg.shape)
        for q, m, w, x, y, u in species:
            ref.pic_deposit_charge(cfg, q, w, x, y, rho)
        frho = rho if p == 0 else ref.filt(cfg, rho)
        return gauss_E_lhs_2d(E) - 4 * math.pi * frho

    g0 = g_of()
    scale = np.abs(g0).max()
    for _ in range(5):
        J = _zeros(cfg)
        for q, m, w, x, y, u in species:
            ref.pic_push_deposit(cfg, E, B, q, m, w, x, y, *u, J)
        st = ref.step(cfg, E, B, J, 1.0)
        assert not any(st.nonconverged)
    assert np.abs(g_of() - g0).max() <= 1e-11 * scale


def test_stencil_guard():
    """A particle that would cross a cell or more in one step is refused."""
    cfg = _cfg(shape=(8, 8), dt=0.7)
    E, B = _zeros(cfg), _zeros(cfg)
    E[0][:] = 50.0   # accelerates to nearly c: 0.7 cells per step is still fine
    x, y = np.array([2.0]), np.array([2.0])
    u = [np.array([1e6]), np.zeros(1), np.zeros(1)]
    ref.pic_push_deposit(cfg, E, B, 1.0, 1.0, 1.0, x, y, *u, _zeros(cfg))
    wide = _cfg(shape=(8, 8), d=(0.5, 0.5), dt=0.3)   # 0.3 c dt = 0.6 cell at c: fine
    ref.pic_push_deposit(wide, E, B, 1.0, 1.0, 1.0, x, y, *u, _zeros(wide))
    fast = ref.Config(ndim=2, shape=(8, 8), dt=1.2, d=(1.0, 1.0))   # above the CFL bound
    with pytest.raises(ValueError):
        ref.pic_push_deposit(fast, E, B, 1.0, 1.0, 1.0, x, y, *u, _zeros(fast))


def _coords(cfg, off):
    """physical (x, y) of a component sitting at (i + off_x, j + off_y)"""
    ny, nx = cfg.shape
    X = (np.arange(nx) + off[0]) * cfg.d[0]
    Y = (np.arange(ny) + off[1]) * cfg.d[1]
    return np.broadcast_to(X[None, :], cfg.shape), np.broadcast_to(Y[:, None], cfg.shape)


def test_gather_uses_staggered_positions():
    """Fields linear in the coordinate of their own staggered positions are
    interpolated exactly at the particle (linear shapes): E_x(x), E_y(y)
    (curl-free, so B^n = 0) give the kick (q dt / m) E(x_p); weak gradients
    of E along the other axes kick by the local value up to a rotation of
    second order; B components linear in x and y with E = 0 turn the
    momentum by the angle of the local field.  Particles stay clear of the
    periodic seam."""
    cfg = _cfg(shape=(16, 20), d=(0.9, 1.1))
    q, m = 1.0, 1.0
    h = q * cfg.dt / m
    rng = np.random.default_rng(31)
    n = 12
    xs = rng.uniform(3 * cfg.d[0], 15 * cfg.d[0], n)
    ys = rng.uniform(3 * cfg.d[1], 11 * cfg.d[1], n)
    offs_E = ((0.5, 0.0), (0.0, 0.5), (0.0, 0.0))
    offs_B = ((0.0, 0.5), (0.5, 0.0), (0.5, 0.5))
    # E_x linear in x, E_y linear in y
    for c, (a, b) in ((0, (0.3, 0.05)), (1, (-0.2, 0.07))):
        E, B = _zeros(cfg), _zeros(cfg)
        X, Y = _coords(cfg, offs_E[c])
        E[c][:] = a + b * (X if c == 0 else Y)
        x, y = xs.copy(), ys.copy()
        u = [np.zeros(n) for _ in range(3)]
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
        want = h * (a + b * (xs if c == 0 else ys))
        np.testing.assert_allclose(u[c], want, rtol=0, atol=1e-14)
    # weak gradients along the other axes (their curl adds a rotation of
    # second order): E_x(y), E_y(x), E_z(x, y)
    for c, (gx, gy) in ((0, (0.0, 1e-4)), (1, (1e-4, 0.0)), (2, (1e-4, -1e-4))):
        E, B = _zeros(cfg), _zeros(cfg)
        X, Y = _coords(cfg, offs_E[c])
        E[c][:] = 1.0 + gx * X + gy * Y
        x, y = xs.copy(), ys.copy()
        u = [np.zeros(n) for _ in range(3)]
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
        np.testing.assert_allclose(u[c], h * (1.0 + gx * xs + gy * ys), rtol=0, atol=1e-9)
    # B components linear in both coordinates: rotation by the local field
    for c, (b0, b1, b2) in ((2, (0.5, 0.04, -0.02)), (0, (0.4, -0.03, 0.025)), (1, (-0.6, 0.02, 0.03))):
        E, B = _zeros(cfg), _zeros(cfg)
        X, Y = _coords(cfg, offs_B[c])
        B[c][:] = b0 + b1 * X + b2 * Y
        x, y = xs.copy(), ys.copy()
        u = [np.zeros(n) for _ in range(3)]
        p1, p2 = (c + 1) % 3, (c + 2) % 3          # the plane the rotation turns
        u[p1][:] = 0.6
        ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
        gam = math.sqrt(1.0 + 0.36)
        th = -2.0 * np.arctan(h * (b0 + b1 * xs + b2 * ys) / (2.0 * gam))
        np.testing.assert_allclose(u[p1], 0.6 * np.cos(th), rtol=0, atol=1e-14)
        np.testing.assert_allclose(u[p2], 0.6 * np.sin(th), rtol=0, atol=1e-14)


def test_push_uses_B_at_the_integer_time_level():
    """The force uses B^n = B^{n-1/2} - (dt/2) curl E^n: with B^{n-1/2} = 0 and
    E_z = g (x - x_p) (zero at the particle, its curl a uniform
    B_y^n = (dt/2) g), a particle with momentum along z turns about y by
    -2 atan(q dt B_y^n / (2 m gamma))."""
    cfg = _cfg(shape=(12, 16))
    q, m, g = 1.0, 1.0, 0.3
    xp, yp = 7.25 * cfg.d[0], 5.5 * cfg.d[1]
    E, B = _zeros(cfg), _zeros(cfg)
    X, _ = _coords(cfg, (0.0, 0.0))
    E[2][:] = g * (X - xp)
    x, y = np.array([xp]), np.array([yp])
    u = [np.zeros(1), np.zeros(1), np.array([0.6])]
    ref.pic_push_deposit(cfg, E, B, q, m, 1.0, x, y, *u, _zeros(cfg))
    gam = math.sqrt(1.0 + 0.36)
    th = -2.0 * math.atan(q * cfg.dt * (0.5 * cfg.dt * g) / (2.0 * m * gam))
    assert u[2][0] == pytest.approx(0.6 * math.cos(th), abs=1e-14)
    assert u[0][0] == pytest.approx(0.6 * math.sin(th), abs=1e-14)
    assert abs(u[1][0]) < 1e-15
