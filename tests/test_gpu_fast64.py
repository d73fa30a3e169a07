"""Fast FP64 mode (MF_FP64_FAST) through the C ABI against the FP64 oracle.

The mode keeps FP64 storage and arithmetic but takes divisions and square
roots from the hardware seeds refined by a second-order series and fuses
multiply-adds, so it is not bit-compatible with the oracle's correctly rounded
operation sequence.  Its gate is the one stated for the FP64 path: relative L1
<= 1e-12 per field after the fixed step count.  Momentum planes whose L1 norm
is at round-off level (a y-uniform run, where rho v is zero to within its own
rounding) are checked on the momentum scale instead.
"""
import numpy as np
import pytest

import oracle
from paper_1905_05727_amd import scenario as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1905_05727_amd import meso  # noqa: E402

LIM = {"vanleer": oracle.VANLEER, "minmod": oracle.MINMOD}
BCO = {"transmissive": oracle.TRANSMISSIVE, "periodic": oracle.PERIODIC}
GATE = 1e-12


def say(*a):
    print(*a, flush=True)


def oracle_of(sc):
    bc = [BCO[b] for b in sc.bc]
    P = oracle.Problem(sc.nx, sc.ny, sc.dx, sc.dy, gamma1=sc.gamma1, pinf1=sc.pinf1,
                       gamma2=sc.gamma2, pinf2=sc.pinf2, cfl=sc.cfl, zeps=sc.zeps,
                       limiter=LIM[sc.limiter], bc_xlo=bc[0], bc_xhi=bc[1], bc_ylo=bc[2],
                       bc_yhi=bc[3], eos2=sc.eos2, cc=sc.cc, reactive=int(sc.reactive),
                       rx=sc.rx)
    o = oracle.Oracle(P)
    o.set_primitive(sc.prim)
    return o


def plane_errors(U, V):
    """Relative L1 per conserved plane; the two momentum planes share the
    larger of their two L1 norms as denominator."""
    nc = V.shape[0]
    d = np.abs(U - V).reshape(nc, -1).sum(axis=1)
    n = np.abs(V).reshape(nc, -1).sum(axis=1)
    n[2] = n[3] = max(n[2], n[3])
    return d / np.maximum(n, 1e-300)


def check(U, V, what, gate=GATE):
    e = plane_errors(U, V)
    exact = float(np.mean(U == V))
    say(f"{what}: rel L1 per plane {np.array2string(e, precision=2)}, "
        f"exactly equal {exact:.3f}")
    assert np.all(e <= gate), (what, e)


def bubble(nx, ny, limiter="vanleer", periodic=False):
    sc = S.single_bubble(nx=nx, ny=ny, radius=min(nx, ny) / 5, centre=(nx * 0.55, ny / 2),
                         shock_x=nx * 0.3)
    sc.limiter = limiter
    if periodic:
        sc.bc = ("periodic",) * 4
    return sc


def test_fast64_shock_tube():
    sc = S.shock_tube_1d()
    say(f"case: fp64_fast shock tube 1000x1 to t={sc.t_end}")
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        taken = s.run_to_time(sc.t_end)
        U = s.read_conserved()
        t, n, _ = s.time()
    o = oracle_of(sc)
    no = o.run(10 ** 6, t_end=sc.t_end)
    assert t == o.t == sc.t_end and abs(taken - no) <= 1 and n == taken
    check(U, o.U, "shock tube")


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("limiter", ["vanleer", "minmod"])
@pytest.mark.parametrize("shape", [(300, 200), (253, 37), (5, 300)])
def test_fast64_bubble(shape, limiter, fused):
    nx, ny = shape
    sc = bubble(nx, ny, limiter=limiter)
    say(f"case: fp64_fast bubble {nx}x{ny} {limiter} fused={fused}")
    o = oracle_of(sc)
    with meso.Solver.from_scenario(sc, precision="fp64_fast", fused=fused) as s:
        s.run_steps(60)
        U = s.read_conserved()
        t, n, _ = s.time()
    o.run(60)
    assert n == 60 and abs(t - o.t) <= 1e-12 * o.t
    check(U, o.U, f"{nx}x{ny} {limiter}")


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (4, 4), (9, 1)])
def test_fast64_degenerate_periodic(shape):
    nx, ny = shape
    rng = np.random.default_rng(nx * 17 + ny)
    prim = S.uniform_state(nx, ny, dx=1e-3)
    prim[0] = rng.uniform(0.2, 0.8, (ny, nx))
    prim[3] = rng.uniform(-20.0, 20.0, (ny, nx))
    prim[4] = rng.uniform(-20.0, 20.0, (ny, nx))
    prim[5] = 1e5 * rng.uniform(0.9, 1.1, (ny, nx))
    sc = S.Scenario("degenerate", nx, ny, 1e-3, 1e-3, prim, bc=("periodic",) * 4)
    say(f"case: fp64_fast degenerate periodic {nx}x{ny}")
    o = oracle_of(sc)
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        s.run_steps(7)
        U = s.read_conserved()
    o.run(7)
    check(U, o.U, f"{nx}x{ny}")


def test_fast64_single_bubble_2000_steps():
    """The 1024 x 512 single bubble at its fixed 2000 steps."""
    sc = S.single_bubble()
    say("case: fp64_fast single bubble 1024x512, 2000 steps")
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        s.run_steps(2000)
        U = s.read_conserved()
        rho, p = s.read_field("rho"), s.read_field("p")
        t, n, _ = s.time()
    o = oracle_of(sc)
    o.run(2000)
    say(f"t {t!r} oracle {o.t!r}")
    assert n == 2000 and abs(t - o.t) <= 1e-12 * o.t
    check(U, o.U, "1024x512 after 2000 steps")
    pr = o.primitive()
    for name, a, b in (("rho", rho, pr["rho"]), ("p", p, pr["p"])):
        e = float(np.abs(a - b).sum() / np.abs(b).sum())
        say(f"{name}: rel L1 {e:.3e}")
        assert e <= GATE


@pytest.mark.parametrize("start", [3, 4])
def test_fast64_roofline_8192_sampled(start):
    """The 8192^2 roofline workload in the benchmark's launch configuration:
    one fast-FP64 step from the state the mode reached after `start` steps,
    checked on sampled cells against the oracle's step from the same state
    with the same dt (each value within 1e-13 of its plane's magnitude), and
    the step's dt against the oracle's full-grid CFL bound."""
    sc = S.roofline_8192()
    n = sc.nx
    say(f"case: fp64_fast roofline 8192x8192 sampled, start={start}")
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        info = s.launch_info()
        s.run_steps(start)
        U0 = s.read_conserved()
        t0, n0, _ = s.time()
        s.run_steps(1)
        U1 = s.read_conserved()
        _, _, dt = s.time()
    o = oracle_of(sc)
    o.U[...] = U0
    o.t, o.step = t0, n0
    dto, _ = o.cfl_dt()
    say(f"dt {dt!r} oracle {dto!r}")
    assert abs(dt - dto) <= 1e-14 * dto
    rng = np.random.default_rng(100 + start)
    ii = list(rng.integers(0, n, 3000))
    jj = list(rng.integers(0, n, 3000))
    tw, th = info["tile_w"], info["tile_h"]
    for a in (0, 1, 2, n - 3, n - 2, n - 1, tw - 1, tw, tw + 1):
        for b in (0, 1, 2, n - 3, n - 2, n - 1, th - 1, th, th + 1):
            ii.append(a)
            jj.append(b)
    cells = np.array(jj, dtype=np.int64) * n + np.array(ii, dtype=np.int64)
    exp = o.step_cells(U0, n0, dt, cells)
    got = U1.reshape(6, -1)[:, cells]
    scale = np.abs(U0.reshape(6, -1)).max(axis=1)[:, None]
    scale[2:4] = max(scale[2, 0], scale[3, 0])
    err = (np.abs(got - exp) / scale).max()
    say(f"sampled one-step max scaled error {err:.3e}")
    assert err <= 1e-13


def test_fast64_nitromethane_bubble():
    """Cochran-Chan liquid (Eqs. (2)-(4), Table 1), 200 steps."""
    sc = S.single_bubble(nx=240, ny=120, dx=1e-6, radius=24, centre=(132, 60), shock_x=72,
                         liquid="nm", p_shock=7.81e9)
    say("case: fp64_fast nitromethane bubble 240x120, 200 steps")
    o = oracle_of(sc)
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        s.run_steps(200)
        U = s.read_conserved()
    o.run(200)
    check(U, o.U, "nitromethane 240x120")


def test_fast64_reactive_bubble():
    """Reacting nitromethane (seventh plane, Arrhenius stage of Eq. (6)),
    200 steps."""
    sc = S.single_bubble(nx=240, ny=120, dx=1e-6, radius=24, centre=(132, 60), shock_x=72,
                         liquid="nm", p_shock=7.81e9)
    sc = S.make_reactive(sc, 72)
    say("case: fp64_fast reacting nitromethane bubble 240x120, 200 steps")
    o = oracle_of(sc)
    with meso.Solver.from_scenario(sc, precision="fp64_fast") as s:
        s.run_steps(200)
        U = s.read_conserved()
    o.run(200)
    check(U, o.U, "reacting nitromethane 240x120")
