"""The seeded workload generators: bubble counts, radii, spacing rules, the
shocked strip and reproducibility (no solver arithmetic is involved)."""
import numpy as np
import pytest

from paper_1905_05727_amd import scenario as S


def pair_stats(b):
    d = np.hypot(b[:, None, 0] - b[None, :, 0], b[:, None, 1] - b[None, :, 1])
    rs = b[:, None, 2] + b[None, :, 2]
    np.fill_diagonal(d, np.inf)
    return (d - rs).min(), (d / rs).min()       # min edge gap, min centre / mean diameter


@pytest.mark.parametrize("factor", [0.0, 2.5])
def test_place_bubbles_rules(factor):
    rng = np.random.default_rng(42)
    b = S.place_bubbles(rng, 120, 2048, 1024, 10.0, 30.0, 4.0, x_lo=16.0, centre_factor=factor)
    assert b.shape == (120, 3)
    assert np.all((b[:, 2] >= 10.0) & (b[:, 2] <= 30.0))
    gap, ratio = pair_stats(b)
    assert gap >= 4.0 - 1e-9
    assert ratio >= factor - 1e-12
    # inside the domain, clear of the shocked strip and of the walls by the gap
    assert np.all(b[:, 0] - b[:, 2] >= 16.0 + 4.0 - 1e-9)
    assert np.all(b[:, 0] + b[:, 2] <= 2048 - 4.0 + 1e-9)
    assert np.all(b[:, 1] - b[:, 2] >= 4.0 - 1e-9)
    assert np.all(b[:, 1] + b[:, 2] <= 1024 - 4.0 + 1e-9)


def test_place_bubbles_fails_loudly_when_impossible():
    with pytest.raises(RuntimeError):
        S.place_bubbles(np.random.default_rng(0), 50, 64, 64, 20.0, 20.0, 2.0, x_lo=2.0,
                        max_draws=2000)


def test_workload_fields_are_reproducible_and_spaced():
    a, b = S.random_field_4096_spaced(), S.random_field_4096_spaced()
    assert np.array_equal(a.meta["bubbles"], b.meta["bubbles"])
    assert a.meta["nbubbles"] == 200 and a.steps == 5000
    assert pair_stats(a.meta["bubbles"])[1] >= 2.5
    g = S.random_field_4096()
    assert g.meta["nbubbles"] == 200 and pair_stats(g.meta["bubbles"])[0] >= 4.0
    r = S.roofline_8192(n=8192)
    assert r.meta["nbubbles"] == 2000 and r.steps == 1000
    assert pair_stats(r.meta["bubbles"])[1] >= 2.5
    assert np.all((r.meta["bubbles"][:, 2] >= 16) & (r.meta["bubbles"][:, 2] <= 48))


def test_shocked_strip_and_ambient_state():
    sc = S.random_field_4096()
    rho1, u1, _ = S.stiffened_gas_shock(1.0e9)
    z, rho2, u, p = sc.prim[0], sc.prim[2], sc.prim[3], sc.prim[5]
    assert np.all(p[:, :16] == 1.0e9) and np.all(u[:, :16] == u1) and np.all(rho2[:, :16] == rho1)
    far = z[:, 16:] < 1e-5                      # liquid cells ahead of the shock
    assert np.all(p[:, 16:][far] == S.P_AMBIENT) and np.all(u[:, 16:][far] == 0.0)
    assert z.min() >= S.Z_EPS and z.max() <= 1 - S.Z_EPS + 1e-15   # eps + (1 - 2 eps) w, rounded


def test_serving_workload():
    reqs = S.serving_workload(24, steps=500)
    assert [r.nx for r in reqs] == [r.ny for r in reqs]
    assert set(r.nx for r in reqs) <= {128, 256, 512}
    for r in reqs:
        b = r.meta["bubbles"]
        assert 1 <= len(b) <= 8 and 0.5e9 <= r.meta["p_shock"] <= 2.0e9
        assert np.all((b[:, 2] >= 0.05 * r.nx - 1e-9) & (b[:, 2] <= 0.15 * r.nx + 1e-9))
        if len(b) > 1:
            gap, ratio = pair_stats(b)
            assert gap >= 2.0 - 1e-9 and ratio >= 2.0 - 1e-12
    again = S.serving_workload(24, steps=500)
    assert all(np.array_equal(x.prim, y.prim) for x, y in zip(reqs, again))
