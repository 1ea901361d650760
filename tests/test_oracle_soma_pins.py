"""Pins of the diffusion and soma clustering oracle (Eq 4.3, Algorithms 6-7,
Sec 4.5.2, Sec 4.7.1) against what the mathematics fixes: the exact discrete
eigenmodes of the scheme with zero concentration beyond the grid, the
analytic point-source solution of the diffusion equation (the convergence
test of Fig 4.9), closed forms of decay and secretion, exact central
differences of linear fields, mass balance, and the clustering the model
produces (Fig 4.18)."""
import math

import numpy as np
import pytest

from oracle import soma


def _mode(R, k):
    i = np.arange(R)
    s = [np.sin(math.pi * kk * (i + 1) / (R + 1)) for kk in k]
    return s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]


@pytest.mark.parametrize("k", [(1, 1, 1), (1, 2, 3), (5, 3, 7)])
def test_eigenmodes_of_the_scheme(k):
    """sin(pi k (i + 1) / (R + 1)) vanishes one point beyond both ends of the
    grid, and the second difference maps it to -4 sin^2(pi k / (2 (R + 1)))
    times itself: one step of Eq 4.3 multiplies the product mode by
    (1 - mu dt) - 4 c sum_a sin^2(pi k_a / (2 (R + 1))), c = nu dt / dx^2."""
    R, S, nu, mu, dt = 24, 48.0, 0.7, 0.013, 0.8
    p = soma.make_params(space=S, resolution=R, n_substances=1, diffusion=nu, decay=mu, dt=dt)
    u0 = _mode(R, k)
    u1 = soma.diffusion_step(u0, p)
    c = nu * dt / (S / R) ** 2
    lam = (1.0 - mu * dt) - 4.0 * c * sum(math.sin(math.pi * kk / (2 * (R + 1))) ** 2 for kk in k)
    assert np.abs(u1 - lam * u0).max() <= 1e-14 * np.abs(u0).max() * 8, np.abs(u1 - lam * u0).max()


def test_decay_alone_is_exact():
    p = soma.make_params(space=10.0, resolution=8, n_substances=1, diffusion=0.0, decay=0.05, dt=0.5)
    u = np.random.default_rng(2).random((8, 8, 8))
    assert np.array_equal(soma.diffusion_step(u, p), u * (1.0 - 0.05 * 0.5))


def test_mass_is_conserved_before_the_boundary_is_reached():
    """Without decay, the interior second differences telescope: the total
    mass is constant while the stencil's support (one point per step) stays
    inside the grid."""
    R = 61
    p = soma.make_params(lo=-61.0, space=122.0, resolution=R, n_substances=1, diffusion=1.0, decay=0.0, dt=0.5)
    u = np.zeros((R, R, R))
    u[30, 30, 30] = 1.0
    m0 = u.sum()
    for _ in range(20):
        u = soma.diffusion_step(u, p)
    assert abs(u.sum() - m0) <= 1e-13
    assert u[30, 30, 9] == 0.0 and u[30, 30, 10] > 0.0  # support radius 20


def test_point_source_converges_to_the_analytic_solution():
    """Fig 4.9's convergence test: an instantaneous point source of unit mass
    at the centre of [-100, 100]^3 (nu = 1, no decay) against
    exp(-r^2 / (4 nu t)) / (4 pi nu t)^(3/2) at r ~ sqrt(1000) um after
    t = 100.  The error falls as the resolution grows (31, 61, 121 points
    per axis) and is below 3 % at the finest."""
    nu, T, dt = 1.0, 100.0, 0.25
    errs = []
    for R in (31, 61, 121):
        S = 200.0
        dx = S / R
        p = soma.make_params(lo=-100.0, space=S, resolution=R, n_substances=1, diffusion=nu, decay=0.0, dt=dt)
        u = np.zeros((R, R, R))
        c = (R - 1) // 2
        u[c, c, c] = 1.0 / dx ** 3
        for _ in range(int(round(T / dt))):
            u = soma.diffusion_step(u, p)
        i = c + int(round(math.sqrt(1000.0) / dx))
        r = (i - c) * dx
        exact = math.exp(-r * r / (4 * nu * T)) / (4 * math.pi * nu * T) ** 1.5
        errs.append(abs(u[c, c, i] - exact) / exact)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.03, errs


def test_gradient_of_a_linear_field_is_exact():
    R, S = 12, 24.0
    p = soma.make_params(space=S, resolution=R, n_substances=1)
    k, j, i = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    u = 3.0 * i - 2.0 * j + 5.0 * k
    dx = S / R
    # interior voxel (5, 6, 7): exact central differences
    g = soma.gradient(u, ((5 + 0.5) * dx, (6 + 0.5) * dx, (7 + 0.5) * dx), p)
    assert np.array_equal(g, np.array([3.0, -2.0, 5.0]) / dx)
    # a voxel on the lower x face: the neighbour beyond the grid is zero
    g = soma.gradient(u, (0.1, (6 + 0.5) * dx, (7 + 0.5) * dx), p)
    assert g[0] == (u[7, 6, 1] - 0.0) / (2 * dx)
    assert soma.voxel((0.1, (6 + 0.5) * dx, (7 + 0.5) * dx), p) == 0 + R * (6 + R * 7)
    assert soma.voxel((S, S, S), p) == R ** 3 - 1  # the upper faces belong to the last voxel


def test_secretion_adds_the_cells_of_each_voxel():
    """No diffusion, decay or movement: one step adds, per substance and
    voxel, the number of cells of that type in it times the quantity
    (Algorithm 6), counted here independently with numpy."""
    rng = np.random.default_rng(4)
    R, S, n = 10, 20.0, 3000
    p = soma.make_params(space=S, resolution=R, n_substances=2, diffusion=0.0, decay=0.0, dt=1.0,
                         secretion=0.375, gradient_weight=0.0)
    pos = rng.uniform(0, S, size=(n, 3))
    pos[:50] = pos[50]  # 51 cells in one voxel
    t = rng.integers(0, 2, size=n).astype(np.int32)
    t[:51] = 1
    o = soma.OracleSoma(pos, t, p)
    o.step(1)
    v = np.clip(np.floor(pos / (S / R)).astype(np.int64), 0, R - 1)
    lin = v[:, 0] + R * (v[:, 1] + R * v[:, 2])
    expect = np.zeros((2, R ** 3))
    np.add.at(expect, (t, lin), 0.375)
    assert np.array_equal(o.u.reshape(2, -1), expect)
    assert o.u.reshape(2, -1)[1, lin[50]] >= 51 * 0.375
    assert np.array_equal(o.pos(), pos)


def test_chemotaxis_follows_the_normalised_gradient():
    """A cell in a field rising along +x moves by the gradient weight along
    +x (Algorithm 7); in the last voxel the zero beyond the grid turns the
    gradient inwards; a step that would leave the space ends on its face
    (closed space; it needs a negative field, since the zero beyond the grid
    makes every gradient of a non-negative field point inwards at the
    faces); in a flat field a cell does not move."""
    R, S = 10, 20.0
    p = soma.make_params(space=S, resolution=R, n_substances=2, diffusion=0.0, decay=0.0, secretion=0.0,
                         gradient_weight=0.75)
    k, j, i = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    u = np.stack([i + 1.0, -(i + 1.0)])
    pos = np.array([[5.0, 7.0, 9.0], [19.9, 7.0, 9.0], [19.9, 7.0, 9.0]])
    o = soma.OracleSoma(pos, np.array([0, 0, 1], np.int32), p, conc=u)
    o.step(1)
    assert np.array_equal(o.pos()[0], [5.75, 7.0, 9.0])
    assert np.array_equal(o.pos()[1], [19.9 - 0.75, 7.0, 9.0])
    assert np.array_equal(o.pos()[2], [20.0, 7.0, 9.0])
    o = soma.OracleSoma(pos[:1], np.zeros(1, np.int32), p, conc=np.ones((2, R, R, R)))
    o.step(1)
    assert np.array_equal(o.pos()[0], pos[0])


def _nearest(pa, pb, same):
    d = np.linalg.norm(pa[:, None, :] - pb[None, :, :], axis=2)
    if same:
        np.fill_diagonal(d, np.inf)
    return d.min(axis=1).mean()


def test_two_types_cluster():
    """Soma clustering (Sec 4.7.1, Fig 4.18): two randomly mixed cell types,
    each secreting its substance and climbing its gradient, end up closer to
    cells of their own type than to the other type."""
    rng = np.random.default_rng(6)
    R, S, n = 20, 100.0, 400
    p = soma.make_params(space=S, resolution=R, n_substances=2, diffusion=1.0, decay=0.01, dt=1.0)
    pos = rng.uniform(0, S, size=(n, 3))
    t = (np.arange(n) % 2).astype(np.int32)
    o = soma.OracleSoma(pos, t, p)

    def score(q):
        a, b = q[t == 0], q[t == 1]
        return _nearest(a, a, True) + _nearest(b, b, True), _nearest(a, b, False) + _nearest(b, a, False)

    same0, other0 = score(pos)
    o.step(300)
    same1, other1 = score(o.pos())
    assert same1 < 0.5 * same0, (same0, same1)
    assert same1 < 0.5 * other1, (same1, other1)
