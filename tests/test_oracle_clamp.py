"""Pins of the oracle's pointwise stage (Sec. 3, Strang splitting; inert case).

With no reaction the source stage of the Strang split reduces to keeping the
air volume fraction z1 inside [eps, 1 - eps] (the "alpha floor" of the
workloads, eps = 1e-6).  The clamp acts on z1 alone: the partial densities,
the momenta and the total energy are not touched by it.  These pins check
the oracle's full step against a no-clamp step assembled from the oracle's
line sweep (pinned elsewhere) followed by numpy's ``clip`` -- the clamp's
definition written independently of the oracle -- on states whose hydro
update leaves z1 outside the bounds.

The functions ``check_*`` raise AssertionError on a mismatch and are run
both by pytest and by ``test_oracle_mutations.py`` against oracle builds with
planted mistakes in the clamp.
"""
import numpy as np
import pytest

import oracle

RHO_AIR, RHO_WATER, P0 = 1.2, 1000.0, 1.0e5


def _pure_row(nx=64, u=0.0):
    """One row: pure water (z1 = 0 exactly) on the left, pure air (z1 = 1
    exactly) on the right, a sharp interface, uniform pressure and velocity.
    z1 = 0 and 1 lie outside [eps, 1 - eps], so the clamp must move every
    cell that the hydro update leaves at a pure value."""
    prim = np.empty((6, 1, nx))
    prim[0] = 0.0
    prim[0, 0, nx // 2:] = 1.0
    prim[1], prim[2], prim[3], prim[4], prim[5] = RHO_AIR, RHO_WATER, u, 0.0, P0
    return prim


def _no_clamp_step(P, U, dt):
    """x sweep of the row (the oracle's line sweep); with ny = 1 and v = 0 the
    y sweep is the identity (every y face sees the same state on both
    sides, so the flux differences vanish exactly)."""
    q = U[:, 0, :].copy()
    return oracle.unit_sweep_line(P, q, dt / P.dx)[:, None, :]


def check_row_clamp(eps, u):
    P = oracle.Problem(nx=64, ny=1, dx=1.0e-4, dy=1.0e-4, zeps=eps)
    o = oracle.Oracle(P)
    o.set_primitive(_pure_row(u=u))
    dt, _ = o.cfl_dt()
    ref = _no_clamp_step(P, o.U, dt)
    o.step_dt(dt)
    z_ref = ref[5]
    # the hydro update must leave z1 outside the bounds on both sides
    assert np.count_nonzero(z_ref < eps) > 10 and np.count_nonzero(z_ref > 1.0 - eps) > 10
    np.testing.assert_array_equal(o.U[5], np.clip(z_ref, eps, 1.0 - eps))
    # far from the interface the pure values become exactly eps and 1 - eps
    assert o.U[5, 0, 0] == eps and o.U[5, 0, -1] == 1.0 - eps
    # the clamp leaves the partial densities, momenta and energy untouched
    np.testing.assert_array_equal(o.U[:5], ref[:5])


def check_bubble_bounds(steps=12):
    """A 2D air bubble with pure phases (z1 = 0 or 1 outside the interface)
    hit by a shock: after every step z1 lies in [eps, 1 - eps], and the pure
    far field sits exactly on the bounds."""
    eps = 1.0e-6
    nx, ny = 48, 40
    P = oracle.Problem(nx=nx, ny=ny, dx=1.0e-5, dy=1.0e-5, zeps=eps)
    y, x = np.mgrid[0:ny, 0:nx] + 0.5
    r = np.hypot(x - 30.0, y - 20.0)
    prim = np.empty((6, ny, nx))
    prim[0] = np.where(r < 8.0, 1.0, 0.0)
    prim[1], prim[2], prim[3], prim[4] = RHO_AIR, RHO_WATER, 0.0, 0.0
    prim[5] = np.where(x < 12.0, 1.0e9, P0)
    o = oracle.Oracle(P)
    o.set_primitive(prim)
    for _ in range(steps):
        dt, _ = o.cfl_dt()
        o.step_dt(dt)
        z = o.U[5]
        assert z.min() >= eps and z.max() <= 1.0 - eps, (z.min(), z.max())
    assert o.U[5, 0, 0] == eps and o.U[5, 20, 30] == 1.0 - eps


def check_sampled_cells(eps, u):
    """The oracle's sampled-cell step (used at sizes where a full oracle step
    is too slow) applies the same clamp: on the pure-phase row every cell
    equals clip(no-clamp step) in z1 and the no-clamp step elsewhere."""
    P = oracle.Problem(nx=64, ny=1, dx=1.0e-4, dy=1.0e-4, zeps=eps)
    o = oracle.Oracle(P)
    o.set_primitive(_pure_row(u=u))
    dt, _ = o.cfl_dt()
    ref = _no_clamp_step(P, o.U, dt)
    cells = np.arange(64, dtype=np.int64)
    got = o.step_cells(o.U, 0, dt, cells)
    np.testing.assert_array_equal(got[5], np.clip(ref[5, 0], eps, 1.0 - eps))
    np.testing.assert_array_equal(got[:5], ref[:5, 0])


def run_all():
    check_row_clamp(1.0e-6, 0.0)
    check_row_clamp(1.0e-3, 150.0)
    check_bubble_bounds()
    check_sampled_cells(1.0e-6, 0.0)
    check_sampled_cells(1.0e-3, 150.0)


@pytest.mark.parametrize("eps,u", [(1.0e-6, 0.0), (1.0e-6, 150.0), (1.0e-3, -80.0)])
def test_row_clamp(eps, u):
    check_row_clamp(eps, u)


def test_bubble_bounds():
    check_bubble_bounds()


@pytest.mark.parametrize("eps,u", [(1.0e-6, 0.0), (1.0e-3, 150.0)])
def test_sampled_cells_clamp(eps, u):
    check_sampled_cells(eps, u)
