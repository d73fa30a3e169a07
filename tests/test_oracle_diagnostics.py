"""Pins of the oracle's diagnostics (Sec. 4.2 transverse averages, domain
integrals, Sec. 4.5 mass-weighted log-binned PDF) against plain numpy
definitions and closed forms."""
import numpy as np
import pytest

import oracle
from paper_1905_05727_amd import scenario as S


def bubble_oracle(nx=90, ny=40, steps=30):
    sc = S.single_bubble(nx=nx, ny=ny, radius=8.0, centre=(50.0, 20.0), shock_x=25.0)
    o = oracle.Oracle(oracle.Problem(nx, ny, sc.dx, sc.dy, cfl=0.4))
    o.set_primitive(sc.prim)
    o.run(steps)
    return o


def test_y_averages_match_definition():
    o = bubble_oracle()
    p, r, u = o.y_averages()
    pr = o.primitive()
    np.testing.assert_allclose(p, pr["p"].mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(r, pr["rho"].mean(axis=0), rtol=1e-13)
    np.testing.assert_allclose(u, (pr["rho"] * pr["u"]).sum(axis=0) / pr["rho"].sum(axis=0),
                               rtol=1e-12, atol=1e-9)


def test_y_averages_of_y_uniform_field_are_the_row():
    sc = S.shock_tube_1d(nx=120)
    o = oracle.Oracle(oracle.Problem(120, 5, sc.dx, sc.dx, cfl=0.5, limiter=oracle.MINMOD))
    o.set_primitive(np.repeat(sc.prim, 5, axis=1))
    o.run(40)
    p, r, u = o.y_averages()
    pr = o.primitive()
    np.testing.assert_allclose(p, pr["p"][0], rtol=1e-15)
    np.testing.assert_allclose(r, pr["rho"][0], rtol=1e-15)
    np.testing.assert_allclose(u, pr["u"][0], rtol=1e-13, atol=1e-12)


def test_integrals():
    o = bubble_oracle()
    got = o.integrals()
    area = o.prob.dx * o.prob.dy
    scale = np.abs(o.U).sum(axis=(1, 2)) * area
    scale[3] = scale[2]                       # rho v sums to ~0 by symmetry: momentum scale
    assert np.all(np.abs(got - o.U.sum(axis=(1, 2)) * area) <= 1e-13 * scale)
    prim = S.uniform_state(7, 5, dx=2e-3, z1=0.25, rho1=1.2, rho2=1000.0)
    u = oracle.Oracle(oracle.Problem(7, 5, 2e-3, 2e-3))
    u.set_primitive(prim)
    M = u.integrals()
    A = 7 * 5 * 4e-6
    assert M[0] == pytest.approx(0.25 * 1.2 * A, rel=1e-14)
    assert M[1] == pytest.approx(0.75 * 1000.0 * A, rel=1e-14)
    assert M[5] == pytest.approx(0.25 * A, rel=1e-14)


def test_log_histogram_against_numpy():
    o = bubble_oracle(steps=40)
    lo, dn, nb = 4.0, 0.02, 300       # 1e4 .. 1e10 Pa
    area = o.prob.dx * o.prob.dy
    m_ref = o.U[1].sum() * area
    f = o.log_histogram(9, lo, dn, nb, m_ref)
    edges = oracle.log_edges(lo, dn, nb)
    np.testing.assert_allclose(edges, 10.0 ** (lo + np.arange(nb + 1) * dn), rtol=1e-14)
    p = o.primitive()["p"].ravel()
    w = o.U[1].ravel() * area
    keep = (p >= edges[0]) & (p < edges[-1])
    h, _ = np.histogram(p[keep], bins=edges, weights=w[keep])
    np.testing.assert_allclose(f, h / (m_ref * dn), rtol=1e-12, atol=1e-300)
    assert (f.sum() * dn) == pytest.approx(w[keep].sum() / m_ref, rel=1e-12)
