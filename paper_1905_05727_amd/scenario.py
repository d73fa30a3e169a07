"""Seeded synthetic inputs: shock / air-bubble scenarios in water.

This module only builds primitive fields (volume fraction, phase densities,
velocity, pressure) on a cell-centred grid.  It holds none of the solver's
arithmetic: the conversion to conserved variables is done separately by the
solver library and by the test oracle.  Both take these fields as plain data.

Scenario shapes follow the problem statement of the paper (Sec. 2.4): a planar
shocked region at the left end feeding a right-running shock into a liquid
seeded with air-filled cavities, transverse periodic or transmissive walls.
The energetic liquid of the paper is replaced by inert water (stiffened gas,
gamma = 4.4, p_inf = 6e8 Pa); air is an ideal gas (gamma = 1.4, Table 2).

Interfaces are smeared with a tanh profile one cell wide; the air volume
fraction is z1 = eps + (1 - 2 eps) w with w in [0, 1] the smeared indicator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WATER_GAMMA = 4.4
WATER_PINF = 6.0e8
AIR_GAMMA = 1.4          # Table 2
AIR_PINF = 0.0
P_AMBIENT = 1.0e5        # Sec. 2.4: initial pressure of unshocked materials
RHO_AIR = 1.2            # Sec. 2.4: initial air density
RHO_WATER = 1000.0
Z_EPS = 1.0e-6

SEEDS = {"random_4096x2048": 1905, "roofline_8192": 5727, "serving": 2019}

# Liquid nitromethane, Cochran-Chan equation of state (Eqs. (2)-(4), Table 1):
# (Gamma_0, A [Pa], B [Pa], C, D, rho_0 [kg/m3]); c_v = 1714 J/(kg K).
NM_CC = (1.19, 0.819e9, 1.51e9, 4.53, 1.42, 1134.0)
NM_CV = 1714.0
RHO_NM = 1134.0           # Sec. 2.4
# Arrhenius kinetics of liquid nitromethane (Eq. (6), Table 3): pre-exponential
# factor C [1/s], activation temperature Ta [K], heat of reaction Q [J/kg];
# with c_v,2 [J/(kg K)] of Table 1 for the temperature of Eq. (5).
NM_RX = (2.6e9, 11350.0, 4.46e6, NM_CV)


@dataclass
class Scenario:
    """Primitive initial fields plus the grid / material description."""
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    prim: np.ndarray                      # (6, ny, nx): z1, rho1, rho2, u, v, p
    cfl: float = 0.4
    limiter: str = "vanleer"
    bc: tuple = ("transmissive",) * 4     # xlo, xhi, ylo, yhi
    gamma1: float = AIR_GAMMA
    pinf1: float = AIR_PINF
    gamma2: float = WATER_GAMMA
    pinf2: float = WATER_PINF
    zeps: float = Z_EPS
    steps: int = 0                        # step count of the workload
    t_end: float = 0.0                    # end time of the workload (0: none)
    eos2: int = 0                         # liquid EoS: 0 stiffened gas, 1 Cochran-Chan
    cc: tuple = NM_CC                     # Cochran-Chan parameters when eos2 == 1
    reactive: bool = False                # 7th plane: reaction progress lambda
    rx: tuple = NM_RX
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Rankine-Hugoniot state behind a planar shock in a stiffened gas
# (the shocked inflow region of Sec. 2.4, here for water instead of NM).
def stiffened_gas_shock(p1: float, rho0: float = RHO_WATER, p0: float = P_AMBIENT,
                        gamma: float = WATER_GAMMA, pinf: float = WATER_PINF):
    """State behind a right-running shock of pressure p1 into gas at rest.

    A stiffened gas behaves as an ideal gas in the shifted pressure p + p_inf,
    so the ideal-gas Hugoniot applies with p -> p + p_inf.
    Returns (rho1, u1, shock_speed).
    """
    P0 = p0 + pinf
    P1 = p1 + pinf
    mu = (gamma - 1.0) / (gamma + 1.0)
    ratio = P1 / P0
    rho1 = rho0 * (ratio + mu) / (mu * ratio + 1.0)
    c0 = math.sqrt(gamma * P0 / rho0)
    S = c0 * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ratio + (gamma - 1.0) / (2.0 * gamma))
    u1 = S * (1.0 - rho0 / rho1)
    return rho1, u1, S


def _cc_energy(rho: float, p: float, cc=NM_CC) -> float:
    """Specific internal energy of the Cochran-Chan liquid, Eq. (2) solved for e."""
    G, A, B, C, D, r0 = cc
    v = r0 / rho
    pref = A * v ** (-C) - B * v ** (-D)
    eref = (-A / (r0 * (1.0 - C)) * (v ** (1.0 - C) - 1.0)
            + B / (r0 * (1.0 - D)) * (v ** (1.0 - D) - 1.0))
    return eref + (p - pref) / (rho * G)


def cochran_chan_shock(p1: float, rho0: float = RHO_NM, p0: float = P_AMBIENT, cc=NM_CC):
    """State behind a right-running shock of pressure p1 into the Cochran-Chan
    liquid at rest (the Hugoniot initialisation of the shocked region of
    Sec. 2.4): the density solves the energy jump condition
    e1 - e0 = (p1 + p0)(1/rho0 - 1/rho1)/2.  Returns (rho1, u1, shock_speed)."""
    from scipy.optimize import brentq
    e0 = _cc_energy(rho0, p0, cc)

    def f(r1):
        return _cc_energy(r1, p1, cc) - e0 - 0.5 * (p1 + p0) * (1.0 / rho0 - 1.0 / r1)

    rho1 = brentq(f, rho0 * (1.0 + 1e-9), rho0 * 4.0, xtol=1e-12, rtol=1e-15, maxiter=500)
    u1 = math.sqrt((p1 - p0) * (1.0 / rho0 - 1.0 / rho1))
    S = u1 / (1.0 - rho0 / rho1)
    return rho1, u1, S


# --------------------------------------------------------------------------
# Cavity-field arithmetic printed in the paper (used by the paper-shaped
# scenario helpers and pinned against its worked numbers).
def regular_spacing(d_c: float, phi: float) -> float:
    """Eq. (6_1): spacing of a square cavity array of porosity phi."""
    return math.sqrt(math.pi * d_c * d_c / (4.0 * phi))


def cavity_count(phi: float, L: float, W: float, d_c: float) -> float:
    """Eq. (7): number of equal cavities of diameter d_c in an L x W domain."""
    return 4.0 * phi * L * W / (math.pi * d_c * d_c)


def number_density_3d(phi: float, d_c: float) -> float:
    """Sec. 5.5: equivalent 3-D number density 6 phi / (pi d_c^3)."""
    return 6.0 * phi / (math.pi * d_c ** 3)


# --------------------------------------------------------------------------
def _zfrac(w: np.ndarray, eps: float) -> np.ndarray:
    return eps + (1.0 - 2.0 * eps) * w


def _blank(nx: int, ny: int) -> np.ndarray:
    prim = np.empty((6, ny, nx), dtype=np.float64)
    prim[0] = 0.0            # w (air indicator), turned into z1 at the end
    prim[1] = RHO_AIR
    prim[2] = RHO_WATER
    prim[3] = 0.0
    prim[4] = 0.0
    prim[5] = P_AMBIENT
    return prim


def _paint_bubble(w: np.ndarray, xc: float, yc: float, R: float) -> None:
    """w = max(w, 0.5 (1 - tanh(r - R))) with r in cell units, cell centres at
    (i + 0.5, j + 0.5); evaluated on a window wide enough for the tail to
    fall below 1e-13."""
    ny, nx = w.shape
    h = R + 16.0
    # cells whose centre lies within h of the centre: a window symmetric about it
    i0 = max(0, int(math.ceil(xc - h - 0.5)))
    i1 = min(nx, int(math.floor(xc + h - 0.5)) + 1)
    j0 = max(0, int(math.ceil(yc - h - 0.5)))
    j1 = min(ny, int(math.floor(yc + h - 0.5)) + 1)
    if i0 >= i1 or j0 >= j1:
        return
    xs = (np.arange(i0, i1, dtype=np.float64) + 0.5) - xc
    ys = (np.arange(j0, j1, dtype=np.float64) + 0.5) - yc
    r = np.sqrt(ys[:, None] * ys[:, None] + xs[None, :] * xs[None, :])
    wb = 0.5 * (1.0 - np.tanh(r - R))
    np.maximum(w[j0:j1, i0:i1], wb, out=w[j0:j1, i0:i1])


def _finish(prim: np.ndarray, eps: float) -> np.ndarray:
    prim[0] = _zfrac(prim[0], eps)
    return prim


def make_reactive(sc: Scenario, strip: int) -> Scenario:
    """Add the reaction progress variable as a 7th primitive plane: lambda = 1
    (unreacted liquid) everywhere except the initially shocked region, where it
    is 0 so that the shocked liquid releases no energy (Sec. 2.4).  Requires
    the Cochran-Chan liquid."""
    assert sc.eos2 == 1, "the reactive model is defined for the Cochran-Chan liquid"
    lam = np.ones((1, sc.ny, sc.nx))
    lam[0, :, :strip] = 0.0
    sc.prim = np.concatenate([sc.prim, lam], axis=0)
    sc.reactive = True
    return sc


def place_bubbles(rng: np.random.Generator, n: int, nx: int, ny: int, rmin: float,
                  rmax: float, gap: float, x_lo: float, max_draws: int = 1_000_000,
                  centre_factor: float = 0.0):
    """Seeded rejection sampling of n non-overlapping circles (cell units).

    Radius uniform in [rmin, rmax]; centre uniform with the circle inside
    [x_lo + gap, nx - gap] x [gap, ny - gap]; edge-to-edge distance to every
    accepted circle at least `gap`, and, if centre_factor > 0, centre-to-centre
    distance at least centre_factor x the mean diameter of the pair (the
    minimum spacing of 2.5 cavity diameters of Sec. 3 is centre_factor = 2.5).
    Raises after max_draws rejected draws.
    """
    xs = np.empty(n)
    ys = np.empty(n)
    rs = np.empty(n)
    k = 0
    draws = 0
    while k < n:
        draws += 1
        if draws > max_draws:
            raise RuntimeError(f"bubble placement failed after {max_draws} draws ({k}/{n})")
        R = rng.uniform(rmin, rmax)
        xmin, xmax = x_lo + gap + R, nx - gap - R
        ymin, ymax = gap + R, ny - gap - R
        if xmax <= xmin or ymax <= ymin:
            continue
        x = rng.uniform(xmin, xmax)
        y = rng.uniform(ymin, ymax)
        if k:
            d2 = (xs[:k] - x) ** 2 + (ys[:k] - y) ** 2
            lim = rs[:k] + R + gap
            if centre_factor > 0.0:
                lim = np.maximum(lim, centre_factor * (rs[:k] + R))
            if np.any(d2 < lim * lim):
                continue
        xs[k], ys[k], rs[k] = x, y, R
        k += 1
    return np.stack([xs, ys, rs], axis=1)


# --------------------------------------------------------------------------
# Workloads
def shock_tube_1d(nx: int = 1000, ny: int = 1, x0: float = 0.7, length: float = 1.0,
                  p_left: float = 1.0e9, rho_left: float = 1000.0, p_right: float = 1.0e5,
                  rho_right: float = 1.0, t_end: float = 2.4e-4, eps: float = Z_EPS,
                  sharp: bool = False) -> Scenario:
    """Two-material shock tube: high-pressure water left of x0, air right of it;
    minmod, CFL 0.5.  The air volume fraction is smeared by tanh over the cell
    size (sharp=False) or a step at x0 (sharp=True).  The pressure is a step
    at x0 in both cases: blending it through the smeared zone would hand the
    air of the mixed cells an internal energy of the order of the water
    pressure and launch a spuriously fast air shock."""
    dx = length / nx
    prim = _blank(nx, ny)
    xc = (np.arange(nx, dtype=np.float64) + 0.5) * dx
    if sharp:
        w = (xc > x0).astype(np.float64)
    else:
        w = 0.5 * (1.0 + np.tanh((xc - x0) / dx))
    prim[0] = w[None, :]
    prim[1] = rho_right
    prim[2] = rho_left
    prim[5] = np.where(xc > x0, p_right, p_left)[None, :]
    return Scenario("shock_tube_1d", nx, ny, dx, dx, _finish(prim, eps), cfl=0.5,
                    limiter="minmod", t_end=t_end,
                    meta=dict(x0=x0, p_left=p_left, rho_left=rho_left, p_right=p_right,
                              rho_right=rho_right))


def single_bubble(nx: int = 1024, ny: int = 512, dx: float = 1.0e-5, radius: float = 64.0,
                  centre=(400.0, 256.0), shock_x: float = 320.0, p_shock: float = 1.0e9,
                  steps: int = 2000, eps: float = Z_EPS, liquid: str = "water",
                  reactive: bool = False) -> Scenario:
    """One air bubble in water hit by a planar 1 GPa shock; the shocked water
    occupies x < shock_x (cell units).  Mirror symmetric about y = ny/2 when
    the centre lies on it."""
    prim = _blank(nx, ny)
    (rho1, u1, S), kw = _liquid(prim, liquid, p_shock, int(shock_x))
    _paint_bubble(prim[0], centre[0], centre[1], radius)
    sc = Scenario("single_bubble", nx, ny, dx, dx, _finish(prim, eps), cfl=0.4,
                  steps=steps, meta=dict(p_shock=p_shock, shock_speed=S, rho1=rho1, u1=u1,
                                         radius=radius, centre=centre, shock_x=shock_x,
                                         liquid=liquid), **kw)
    return make_reactive(sc, int(shock_x)) if reactive else sc


def random_bubbles(nx: int, ny: int, nbubbles: int, rmin: float, rmax: float, gap: float,
                   seed: int, dx: float = 1.0e-5, p_shock: float = 1.0e9, strip: int = 16,
                   steps: int = 0, name: str = "random_bubbles", eps: float = Z_EPS,
                   bubbles: np.ndarray | None = None, centre_factor: float = 0.0) -> Scenario:
    """Random air-bubble field in water; a planar shock enters from x = 0 out of
    a shocked strip of `strip` cells.  Bubbles are placed by seeded rejection
    sampling (numpy PCG64 stream of `seed`)."""
    if bubbles is None:
        rng = np.random.default_rng(seed)
        bubbles = place_bubbles(rng, nbubbles, nx, ny, rmin, rmax, gap, x_lo=float(strip),
                                centre_factor=centre_factor)
    prim = _blank(nx, ny)
    rho1, u1, S = stiffened_gas_shock(p_shock)
    prim[2, :, :strip] = rho1
    prim[3, :, :strip] = u1
    prim[5, :, :strip] = p_shock
    for x, y, R in bubbles:
        _paint_bubble(prim[0], x, y, R)
    porosity = float(np.pi * np.sum(bubbles[:, 2] ** 2) / (nx * ny))
    return Scenario(name, nx, ny, dx, dx, _finish(prim, eps), cfl=0.4, steps=steps,
                    meta=dict(seed=seed, p_shock=p_shock, shock_speed=S, porosity=porosity,
                              nbubbles=len(bubbles), bubbles=bubbles))


def random_field_4096(seed: int = SEEDS["random_4096x2048"]) -> Scenario:
    """4096 x 2048, 200 bubbles, radius U[20, 40] cells, edge gap >= 4, 5000 steps."""
    return random_bubbles(4096, 2048, 200, 20.0, 40.0, 4.0, seed, steps=5000,
                          name="random_4096x2048")


def random_field_4096_spaced(seed: int = SEEDS["random_4096x2048"]) -> Scenario:
    """The 4096 x 2048 field (200 bubbles, radius U[20, 40] cells, 5000 steps)
    placed with the minimum centre spacing of Sec. 3: 2.5 mean diameters of
    each pair.  With an edge gap of only 4 cells the scheme of Sec. 3 (no
    positivity treatment) drives the thin water gaps between close bubbles to
    a non-physical state once the shock arrives; the spacing rule is what the
    paper uses to avoid that."""
    return random_bubbles(4096, 2048, 200, 20.0, 40.0, 4.0, seed, steps=5000,
                          name="random_4096x2048_spaced", centre_factor=2.5)


def ligament_crop(x_hi: int = 256, y_lo: int = 480, y_hi: int = 760) -> Scenario:
    """Window [0, x_hi) x [y_lo, y_hi) of the 4096 x 2048 field (edge gap 4
    cells) with the shocked strip and the bubbles lying wholly inside it: the
    pair at (77.4, 585.5) r 31.8 and (125.8, 640.8) r 37.3, whose water gap is
    4.4 cells wide."""
    full = random_field_4096()
    b = np.asarray(full.meta["bubbles"])
    inside = ((b[:, 0] + b[:, 2] < x_hi - 8) & (b[:, 1] - b[:, 2] > y_lo + 4)
              & (b[:, 1] + b[:, 2] < y_hi - 4))
    bb = b[inside].copy()
    bb[:, 1] -= y_lo
    return random_bubbles(x_hi, y_hi - y_lo, len(bb), 0.0, 0.0, 4.0, 0, bubbles=bb,
                          name="ligament_crop")


def roofline_8192(seed: int = SEEDS["roofline_8192"], n: int = 8192) -> Scenario:
    """8192 x 8192, 2000 bubbles, radius U[16, 48] cells, 1000 steps; placed
    with the minimum centre spacing of Sec. 3 (2.5 mean diameters of each
    pair, edge gaps of 50 cells and more), so that the state stays physical
    over the step count (thin water gaps between bubbles do not, see
    random_field_4096_spaced)."""
    return random_bubbles(n, n, 2000, 16.0, 48.0, 4.0, seed, steps=1000, name="roofline_8192",
                          centre_factor=2.5)


def serving_request(rng: np.random.Generator, sizes=(128, 256, 512), steps: int = 500,
                    eps: float = Z_EPS, centre_factor: float = 2.0) -> Scenario:
    """One independent shock-bubble solve of the serving workload: square grid
    drawn from `sizes`, 1-8 bubbles of radius U[0.05, 0.15] x width with edge
    gap >= 2 cells and centre spacing >= centre_factor mean diameters of each
    pair (2: edge gaps of at least the sum of the radii, so no thin water gap
    fails under the shock), shock pressure U[0.5, 2] GPa; placement retried."""
    n = int(rng.choice(sizes))
    nb = int(rng.integers(1, 9))
    p_shock = float(rng.uniform(0.5e9, 2.0e9))
    sub_seed = int(rng.integers(0, 2 ** 62))
    for attempt in range(64):
        try:
            sub = np.random.default_rng(sub_seed + attempt)
            b = place_bubbles(sub, nb, n, n, 0.05 * n, 0.15 * n, 2.0, x_lo=16.0,
                              max_draws=20000, centre_factor=centre_factor)
            break
        except RuntimeError:
            continue
    else:
        raise RuntimeError("serving request: bubble placement failed")
    sc = random_bubbles(n, n, nb, 0.0, 0.0, 2.0, 0, p_shock=p_shock, steps=steps,
                        name=f"serving_{n}", eps=eps, bubbles=b)
    sc.meta["p_shock"] = p_shock
    return sc


def serving_workload(nreq: int = 256, seed: int = SEEDS["serving"], sizes=(128, 256, 512),
                     steps: int = 500, centre_factor: float = 2.0):
    """The list of serving requests, reproducible from `seed`."""
    rng = np.random.default_rng(seed)
    return [serving_request(rng, sizes=sizes, steps=steps, centre_factor=centre_factor)
            for _ in range(nreq)]


def poisson_arrivals(n: int, rate: float, seed: int = SEEDS["serving"]) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# --------------------------------------------------------------------------
# Paper-shaped cavity fields (Sec. 2.4, Sec. 3, App. A), water/air instead of
# nitromethane/air.  Lengths in cells: the paper resolves a cavity diameter by
# 100 cells (dx = 1 um for d_c = 100 um).
def _paint_bubble_periodic_y(w: np.ndarray, xc: float, yc: float, R: float) -> None:
    ny = w.shape[0]
    for shift in (-ny, 0, ny):
        if yc + shift + R + 16.0 >= 0.0 and yc + shift - R - 16.0 <= ny:
            _paint_bubble(w, xc, yc + shift, R)


def _liquid(prim: np.ndarray, liquid: str, p_shock: float, strip: int):
    """Fill the liquid density and the shocked strip; returns (post-shock state,
    Scenario EoS keyword arguments)."""
    if liquid == "nm":
        prim[2] = RHO_NM
        rho1, u1, S = cochran_chan_shock(p_shock)
        kw = dict(eos2=1, cc=NM_CC)
    else:
        rho1, u1, S = stiffened_gas_shock(p_shock)
        kw = {}
    prim[2, :, :strip] = rho1
    prim[3, :, :strip] = u1
    prim[5, :, :strip] = p_shock
    return (rho1, u1, S), kw


def regular_array(d_c: int = 100, phi: float = 0.08, length: int = 24000, strip: int = 500,
                  p_shock: float = 1.0e9, dx: float = 1.0e-6, eps: float = Z_EPS,
                  steps: int = 0, liquid: str = "water", reactive: bool = False) -> Scenario:
    """Square array of equal cavities (Sec. 2.4, Fig. 1(b)): spacing from
    Eq. (6_1), domain width = one spacing with periodic top/bottom walls, a
    shocked strip of `strip` cells at the transmissive left wall."""
    delta = regular_spacing(float(d_c), phi)
    ny = int(round(delta))
    nx = int(length)
    prim = _blank(nx, ny)
    (rho1, u1, S), kw = _liquid(prim, liquid, p_shock, strip)
    R = 0.5 * d_c
    x = strip + 0.5 * delta
    centres = []
    while x + R + 2.0 <= nx:
        _paint_bubble_periodic_y(prim[0], x, 0.5 * ny, R)
        centres.append((x, 0.5 * ny, R))
        x += delta
    sc = Scenario("regular_array", nx, ny, dx, dx, _finish(prim, eps), cfl=0.4,
                  bc=("transmissive", "transmissive", "periodic", "periodic"), steps=steps,
                  meta=dict(spacing=delta, ncavities=len(centres), p_shock=p_shock,
                            shock_speed=S, bubbles=np.array(centres), liquid=liquid), **kw)
    return make_reactive(sc, strip) if reactive else sc


def random_cavities(d_c: int = 100, phi: float = 0.08, length: int = 24000, width: int = 2000,
                    strip: int = 500, min_spacing: float = 2.5, p_shock: float = 1.0e9,
                    dx: float = 1.0e-6, seed: int = 1905, eps: float = Z_EPS,
                    steps: int = 0, max_draws: int = 2_000_000,
                    liquid: str = "water", reactive: bool = False) -> Scenario:
    """Random field of equal cavities (Sec. 2.4, Fig. 1(c)): the count from
    Eq. (7) over the region ahead of the shocked strip, centres uniform with a
    minimum centre-to-centre distance of `min_spacing` diameters (Sec. 3),
    measured periodically across the top/bottom walls."""
    nx, ny = int(length), int(width)
    region = nx - strip
    ncav = int(round(cavity_count(phi, float(region), float(ny), float(d_c))))
    R = 0.5 * d_c
    dmin = min_spacing * d_c
    rng = np.random.default_rng(seed)
    xs = np.empty(ncav)
    ys = np.empty(ncav)
    k = draws = 0
    while k < ncav:
        draws += 1
        if draws > max_draws:
            raise RuntimeError(f"cavity placement failed ({k}/{ncav})")
        x = rng.uniform(strip + R + 2.0, nx - R - 2.0)
        y = rng.uniform(0.0, ny)
        if k:
            ddy = np.abs(ys[:k] - y)
            ddy = np.minimum(ddy, ny - ddy)
            if np.any((xs[:k] - x) ** 2 + ddy ** 2 < dmin * dmin):
                continue
        xs[k], ys[k] = x, y
        k += 1
    prim = _blank(nx, ny)
    (rho1, u1, S), kw = _liquid(prim, liquid, p_shock, strip)
    for x, y in zip(xs, ys):
        _paint_bubble_periodic_y(prim[0], x, y, R)
    cen = np.stack([xs, ys, np.full(ncav, R)], axis=1)
    sc = Scenario("random_cavities", nx, ny, dx, dx, _finish(prim, eps), cfl=0.4,
                  bc=("transmissive", "transmissive", "periodic", "periodic"), steps=steps,
                  meta=dict(seed=seed, ncavities=ncav, porosity_target=phi, p_shock=p_shock,
                            shock_speed=S, bubbles=cen, nbubbles=ncav, liquid=liquid), **kw)
    return make_reactive(sc, strip) if reactive else sc


def uniform_state(nx: int, ny: int, dx: float = 1.0e-3, z1: float = Z_EPS,
                  rho1: float = RHO_AIR, rho2: float = RHO_WATER, u: float = 0.0,
                  v: float = 0.0, p: float = P_AMBIENT) -> np.ndarray:
    prim = np.empty((6, ny, nx), dtype=np.float64)
    prim[0], prim[1], prim[2], prim[3], prim[4], prim[5] = z1, rho1, rho2, u, v, p
    return prim
