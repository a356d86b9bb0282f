"""GPU tests of the continuous-batching server: every result equals the
plain solve of the same request (bitwise: each grid's arithmetic does not
depend on what runs beside it), requests admitted while others run,
admission bounded by the memory budget, warm-started sessions, cancel."""
import time

import numpy as np
import pytest

from paper_2111_09859_amd import grids as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_09859_amd import api
    s = api.Solver(0)
    yield s
    s.close()


def say(*a):
    print(*a, flush=True)


def method(**kw):
    from paper_2111_09859_amd import api
    base = dict(equation="HJ", gamma="LAD", eps=0.2, precision="fp32", tol=1e-6,
                stall_window=200, max_iter=3000)
    base.update(kw)
    return api.make_method(**base)


def mix():
    return [(G.channel(65, 33), dict(scheme="E6")),
            (G.cylinder(48, 40, rout=6.0, dr1=1e-2, ratio=1.12), dict(scheme="C6", curvature=True)),
            (G.ellipse(40, 33, axis_ratio=2.0, ratio=1.15, rout=5.0, dr1=1e-2),
             dict(scheme="C6", curvature=True)),
            (G.duct(17, nx=12), dict(scheme="C6")),
            (G.channel(129, 65), dict(scheme="C6")),
            (G.star_grain(64), dict(scheme="E6", eps=0.15)),
            (G.channel(37, 29), dict(equation="POISSON", scheme="E4", tol=1e-7)),
            (G.box2d(33), dict(equation="EIKONAL", scheme="E4", max_iter=400))]


def test_server_results_equal_solo(solver):
    from paper_2111_09859_amd import api
    cases = mix()
    solo = []
    for spec, kw in cases:
        p = solver.prepare(spec, kw["scheme"], "fp32")
        out = solver.solve(p, method(**kw), check=False)
        solo.append((out["phi"].cpu().numpy(), out["iters"], out["status"]))
    srv = api.Server(solver, budget_bytes=256 << 20, max_slots=16)
    try:
        ids = []
        for spec, kw in cases:
            p = solver.prepare(spec, kw["scheme"], "fp32")
            ids.append(srv.submit(p, method(**kw), hist_cap=4000))
        for i, rid in enumerate(ids):
            st = srv.wait(rid, 120.0)
            info = srv.poll(rid)
            a, it, s0 = solo[i]
            b = srv.result(rid).cpu().numpy()
            say(f"[server] req {i} {cases[i][0].name} status={st} iters={info['iters']} "
                f"solo_iters={it} max|diff|={np.abs(a - b).max():.3e}")
            assert st == s0 and info["iters"] == it
            assert np.array_equal(a, b, equal_nan=True)
            h = srv.history(rid, 4000)
            assert len(h) == it
        stats = srv.stats()
        say(f"[server] stats {stats}")
        assert stats["done"] == len(cases) and stats["peak_active"] >= 2
    finally:
        srv.close()


def test_server_admits_while_running_and_respects_budget(solver):
    from paper_2111_09859_amd import _lib as L, api
    spec = G.channel(129, 65)
    p = solver.prepare(spec, "C6", "fp32")
    m = method(scheme="C6")
    one = L.wd_workspace_bytes(solver.ctx, [p.desc], [m])
    budget = int(2.5 * one)       # at most two of these grids at once
    srv = api.Server(solver, budget_bytes=budget, max_slots=8)
    try:
        first = srv.submit(p, m)
        time.sleep(0.05)
        later = [srv.submit(p, m) for _ in range(4)]
        big = srv.submit(solver.prepare(G.channel(1025, 513), "C6", "fp32"), m)
        assert srv.wait(big, 60.0) == L.WD_ERR_NO_MEMORY
        for rid in [first] + later:
            assert srv.wait(rid, 120.0) in (0, 2)
        infos = [srv.poll(r) for r in [first] + later]
        # some request was admitted while an earlier one was still running
        assert any(b["t_admit"] < a["t_done"] for a, b in zip(infos, infos[1:]))
        st = srv.stats()
        say(f"[server budget] one={one} budget={budget} stats={st}")
        assert st["peak_bytes"] <= budget
        ref = srv.result(first).cpu().numpy()
        for r in later:
            assert np.array_equal(srv.result(r).cpu().numpy(), ref)
    finally:
        srv.close()


def test_server_warm_started_session(solver):
    """Receding star-shaped port: each step warm-starts from the previous
    field (kept on the device) and matches the plain warm-started solve."""
    import torch
    from paper_2111_09859_amd import api
    srv = api.Server(solver, budget_bytes=256 << 20, max_slots=8)
    try:
        phi_srv = None
        phi_ref = None
        iters = []
        for k in range(3):
            spec = G.star_grain(96, step=4 * k)
            p = solver.prepare(spec, "E6", "fp32")
            m = method(scheme="E6", eps=0.15, warm_start=k > 0)
            if phi_srv is None:
                phi_srv = torch.zeros(spec.shape, dtype=torch.float32, device=solver.device)
                phi_ref = torch.zeros_like(phi_srv)
            rid = srv.submit(p, m, phi=phi_srv, session=7)
            st = srv.wait(rid, 120.0)
            ref = solver.solve(p, m, phi=phi_ref, check=False)
            info = srv.poll(rid)
            iters.append(info["iters"])
            say(f"[session] step {k} status={st} iters={info['iters']}")
            assert st == ref["status"] and info["iters"] == ref["iters"]
            assert torch.equal(phi_srv, phi_ref)
        assert iters[1] < iters[0] and iters[2] < iters[0]
    finally:
        srv.close()


def test_server_cancel_queued(solver):
    from paper_2111_09859_amd import _lib as L, api
    spec = G.channel(129, 65)
    p = solver.prepare(spec, "C6", "fp32")
    srv = api.Server(solver, budget_bytes=64 << 20, max_slots=1)
    try:
        a = srv.submit(p, method(scheme="C6"))
        b = srv.submit(p, method(scheme="C6"))
        srv.cancel(b)
        assert srv.wait(b, 60.0) == L.WD_ERR_CANCELLED
        assert srv.wait(a, 120.0) in (0, 2)
    finally:
        srv.close()
