"""Continuous-batching server: every solve's result is identical alone and in
the mix, admission stays inside the HBM budget, failures stay isolated."""
import numpy as np
import pytest

from paper_1905_05727_amd import scenario as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1905_05727_amd import meso, serve  # noqa: E402

import oracle  # noqa: E402


def say(*a):
    print(*a, flush=True)


def small_requests(n, seed=7, sizes=(48, 64, 100, 130, 260)):
    rng = np.random.default_rng(seed)
    return [S.serving_request(rng, sizes=sizes, steps=0) for _ in range(n)]


@pytest.mark.parametrize("prec", ["fp64", "fp32_fp64acc", "fp32"])
def test_alone_equals_in_mix(prec):
    reqs = small_requests(9)
    nsteps = 37
    say(f"case: 9 requests {[r.nx for r in reqs]}, {nsteps} steps, {prec}")
    got = {}
    with serve.Server(1 << 30, max_slots=5, precision=prec, max_inflight=3) as srv:
        tickets = []
        for k, sc in enumerate(reqs):
            tickets.append(srv.submit(sc, nsteps))
            for _ in range(k % 4):           # staggered arrivals: solves overlap at offsets
                srv.tick()
        srv.drain()
        for k, tk in enumerate(tickets):
            assert srv.poll(tk) == serve.REQ_DONE
            got[k] = srv.result(tk)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["active"] == 0 and st["queued"] == 0
    for k, sc in enumerate(reqs):
        U, t, n = serve.solve_alone(sc, nsteps, precision=prec)
        Ub, tb, nb = got[k]
        assert n == nb == nsteps and t == tb
        assert np.array_equal(U, Ub), f"request {k} ({sc.nx}^2) differs in the mix"
    if prec == "fp64":
        sc = reqs[0]
        o = oracle.Oracle(oracle.Problem(sc.nx, sc.ny, sc.dx, sc.dy, cfl=sc.cfl))
        o.set_primitive(sc.prim)
        o.run(nsteps)
        assert np.array_equal(o.U, got[0][0])


@pytest.mark.parametrize("prec", ["fp64", "fp32_fp64acc", "fp32"])
def test_loaded_server_tail_equals_alone(prec, monkeypatch):
    """Sixteen 512^2 solves admitted together: the load gives 16-row segments
    (the segment model over 16 grids of 3 strips), so each solve's last 16
    rows go into 4-row segments dispatched after all the others.  Every
    result equals its lone solve bit for bit."""
    monkeypatch.delenv("MESO_SERVE_SEG_H", raising=False)
    monkeypatch.delenv("MESO_SERVE_TAPER", raising=False)
    reqs = small_requests(16, seed=5, sizes=(512,))
    nsteps = 12
    say(f"case: 16 requests of 512^2, {nsteps} steps, {prec}")
    with serve.Server(2 << 30, max_slots=16, precision=prec, max_inflight=3) as srv:
        tickets = [srv.submit(sc, nsteps) for sc in reqs]
        srv.drain()
        got = [srv.result(tk) for tk in tickets]
    for k, sc in enumerate(reqs):
        U, t, n = serve.solve_alone(sc, nsteps, precision=prec)
        Ub, tb, nb = got[k]
        assert n == nb == nsteps and t == tb
        assert np.array_equal(U, Ub), f"request {k} differs under load"


def test_mixed_liquids_alone_equals_in_mix():
    """Water and nitromethane requests in one server: each tick runs one
    batched launch per liquid; every result equals its lone solve."""
    water = small_requests(3, seed=17, sizes=(64, 100))
    nm = [S.single_bubble(nx=n, ny=m, dx=1e-6, radius=m / 5, centre=(n * 0.55, m / 2),
                          shock_x=n * 0.3, liquid="nm", p_shock=7.81e9)
          for n, m in ((64, 48), (120, 60), (260, 40))]
    reqs = [water[0], nm[0], water[1], nm[1], nm[2], water[2]]
    say("case: mixed liquids, 6 requests, 23 steps, fp64")
    with serve.Server(1 << 29, max_slots=4, precision="fp64") as srv:
        tks = [srv.submit(sc, 23) for sc in reqs]
        srv.drain()
        got = [srv.result(tk) for tk in tks]
    for sc, (Ub, tb, nb) in zip(reqs, got):
        U, t, n = serve.solve_alone(sc, 23, precision="fp64")
        assert nb == n == 23 and tb == t
        assert np.array_equal(U, Ub)


def test_finished_reports_each_ticket_once():
    reqs = small_requests(5, seed=13, sizes=(64, 100))
    say("case: finished tickets, 5 requests")
    with serve.Server(1 << 28, max_slots=3, precision="fp32_fp64acc") as srv:
        tks = [srv.submit(sc, 9) for sc in reqs]
        seen = []
        while len(seen) < len(tks):
            srv.tick()
            seen += srv.finished()
        assert sorted(seen) == sorted(tks) and len(set(seen)) == len(tks)
        assert srv.finished() == []
        for tk in tks:
            assert srv.poll(tk) == serve.REQ_DONE
            srv.result(tk)


def test_admission_stays_within_budget():
    reqs = small_requests(6, seed=11, sizes=(200,))
    per = serve.Server.request_bytes(200, 200, "fp32_fp64acc")
    budget = int(2.5 * per)
    say(f"case: budget {budget} B = 2.5 requests")
    with serve.Server(budget, max_slots=8, precision="fp32_fp64acc") as srv:
        tks = [srv.submit(sc, 15) for sc in reqs]
        peak_active = 0
        while True:
            a, q = srv.tick()
            peak_active = max(peak_active, a)
            if a == 0 and q == 0:
                break
        srv.drain()
        st = srv.stats()
        assert st["peak_bytes"] <= budget and peak_active == 2
        for tk in tks:
            assert srv.poll(tk) == serve.REQ_DONE
            srv.result(tk)


def test_failed_request_is_isolated():
    reqs = small_requests(3, seed=3, sizes=(64,))
    bad = reqs[1]
    bad.prim = bad.prim.copy()
    bad.prim[5, 5, 5] = np.nan
    say("case: one NaN request among three")
    with serve.Server(1 << 28, max_slots=4, precision="fp64") as srv:
        tks = [srv.submit(sc, 12) for sc in reqs]
        srv.drain()
        assert srv.poll(tks[1]) == serve.REQ_FAILED
        with pytest.raises(meso.MesoError) as ei:
            srv.result(tks[1])
        assert ei.value.status == -3
        for k in (0, 2):
            U, _, _ = srv.result(tks[k])
            assert np.array_equal(U, serve.solve_alone(reqs[k], 12, "fp64")[0])


def test_server_validation():
    sc = small_requests(1)[0]
    with serve.Server(1 << 20, max_slots=2, precision="fp32_fp64acc") as srv:
        big = S.single_bubble(nx=1024, ny=512)
        with pytest.raises(meso.MesoError) as ei:
            srv.submit(big, 5)                     # can never fit in 1 MiB
        assert ei.value.status == -2
        srv.precision = "fp64"                     # options must match the server's
        with pytest.raises(meso.MesoError) as ei:
            srv.submit(sc, 5)
        assert ei.value.status == -1


def test_serve_poisson_replay():
    reqs = small_requests(16, seed=5, sizes=(64, 128))
    arr = S.poisson_arrivals(len(reqs), rate=400.0, seed=1)
    say("case: 16 requests, Poisson 400/s, 60 steps")
    with serve.Server(1 << 30, max_slots=8, precision="fp32_fp64acc") as srv:
        res = serve.serve(srv, reqs, arr, 60)
    assert np.all(res["latencies"] > 0) and res["p99_s"] >= res["p50_s"]
    assert res["stats"]["completed"] == 16


def test_serving_workload_sizes_alone_equals_in_mix():
    """Requests of the serving workload itself (128^2, 256^2, 512^2 grids,
    0.5-2 GPa shocks), FP32-bulk mode, batched vs alone."""
    reqs = S.serving_workload(6, steps=0)
    nsteps = 80
    say(f"case: serving sizes {[r.nx for r in reqs]}, {nsteps} steps")
    with serve.Server(4 << 30, max_slots=4, precision="fp32_fp64acc") as srv:
        tks = [srv.submit(sc, nsteps) for sc in reqs]
        srv.drain()
        got = [srv.result(tk) for tk in tks]
    for sc, (Ub, tb, nb) in zip(reqs, got):
        U, t, n = serve.solve_alone(sc, nsteps)
        assert nb == n == nsteps and tb == t and np.array_equal(U, Ub)


SEG_SERVE = [(None, None), ("1", None), ("4", None), ("64", None), ("16", "4,16"),
             ("64", "2,8"), ("12", "0,0")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_segment_height_changes_no_value(prec, monkeypatch):
    """The server picks the rows per workgroup segment from the load; fixing
    it at 1, 4 or 64 rows (MESO_SERVE_SEG_H), or giving each solve a tail of
    shorter segments dispatched last (MESO_SERVE_TAPER), gives the same bits
    as the automatic choice."""
    reqs = small_requests(6, seed=11)
    nsteps = 23
    res = {}
    for seg, taper in SEG_SERVE:
        for var, val in (("MESO_SERVE_SEG_H", seg), ("MESO_SERVE_TAPER", taper)):
            if val is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, val)
        say(f"case: 6 requests {[r.nx for r in reqs]}, {nsteps} steps, {prec}, segment {seg}, "
            f"tail {taper}")
        with serve.Server(1 << 30, max_slots=4, precision=prec, max_inflight=3) as srv:
            tickets = [srv.submit(sc, nsteps) for sc in reqs]
            srv.drain()
            res[(seg, taper)] = [srv.result(tk) for tk in tickets]
    monkeypatch.delenv("MESO_SERVE_SEG_H", raising=False)
    monkeypatch.delenv("MESO_SERVE_TAPER", raising=False)
    for key in SEG_SERVE[1:]:
        for (a, ta, na), (b, tb, nb) in zip(res[(None, None)], res[key]):
            assert na == nb == nsteps and ta == tb
            assert np.array_equal(a, b)
