"""Serving: requests queued on a Server run setup, plane waves and solve on
the library's worker threads (one stream each) and must give the results of
the same requests solved directly; at most max_slots run at once."""
import numpy as np
import pytest

from cases import CASES, QUAD

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KHAT = (0.0, 0.0, 1.0)
E0 = (1.0, 0.0, 0.0)


def _problem(name, ctx=None):
    from paper_2003_11679_amd import Problem
    build, eps_r, sigma, freq, n, R = CASES[name]
    xyz, tri = build()
    p = Problem(freq, ctx=ctx)
    p.add_object(xyz, tri, eps_r=eps_r, sigma=sigma)
    p.set_grid(-1, n=n, near_radius=R)
    p.set_quadrature(**QUAD)
    return p


def _far(p):
    th = np.linspace(0.0, np.pi, 13)
    return p.far_field(np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1))


def test_served_requests_match_direct_solves():
    from paper_2003_11679_amd import Server, FP32
    names = ["sphere2", "sphere2_lossy", "bar_small", "sphere2", "bar_small", "sphere2_lossy"]
    srv = Server(max_slots=3)
    tickets = []
    for nm in names:
        p = _problem(nm, ctx=srv.ctx)
        tickets.append((nm, srv.submit(p, KHAT, E0, FP32, tol=1e-6, restart=200)))
    print(f"[serving] submitted {len(tickets)}", flush=True)
    results = {}
    for nm, t in tickets:
        p = srv.take(t)
        results.setdefault(nm, []).append((p.currents(), _far(p)))
    srv.close()
    for nm in set(names):
        d = _problem(nm)
        d.setup()
        d.set_planewaves(KHAT, E0)
        rep = d.solve(FP32, tol=1e-6, restart=200)
        assert rep["converged"], rep
        (u, v), F = d.currents(), _far(d)
        for (us, vs), Fs in results[nm]:
            ef = np.abs(Fs - F).max() / np.abs(F).max()
            eu = np.linalg.norm(us - u) / np.linalg.norm(u)
            print(f"  {nm}: currents {eu:.2e} far field {ef:.2e}", flush=True)
            assert ef < 1e-5, (nm, ef)
            assert eu < (1e-5 if nm.startswith("sphere") else 1e-3), (nm, eu)


def test_slots_bound_concurrency_and_every_request_finishes():
    from paper_2003_11679_amd import Server, FP32
    srv = Server(max_slots=2)
    ts = [srv.submit(_problem("sphere2", ctx=srv.ctx), KHAT, E0, FP32, tol=1e-6) for _ in range(5)]
    import time
    infos = []
    for t in ts:
        while True:
            i = srv.poll(t)
            if i["done"]:
                break
            time.sleep(0.01)
        infos.append(i)
    for t in ts:
        srv.take(t)
    srv.close()
    assert all(i["status"] == 0 for i in infos), infos
    # at no instant do more than 2 requests run
    ev = sorted([(i["t_start_s"], 1) for i in infos] + [(i["t_end_s"], -1) for i in infos])
    live = peak = 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    assert peak <= 2, peak
    assert all(i["footprint"] > 0 for i in infos)


def test_server_errors():
    from paper_2003_11679_amd import Server, SieError
    srv = Server(max_slots=1)
    with pytest.raises(SieError):
        srv.poll(12345)
    srv.close()


def test_binding_memory_budget_serialises_and_is_never_exceeded():
    """A budget that holds one request's footprint estimate (plus a margin
    below a second one) admits one request at a time although four slots
    are free; the admitted footprints never sum above the budget."""
    from paper_2003_11679_amd import Server, FP32
    probe = _problem("sphere2")
    fp = probe.footprint()
    budget = int(1.5 * fp)
    srv = Server(hbm_budget_bytes=budget, max_slots=4)
    ts = [srv.submit(_problem(nm, ctx=srv.ctx), KHAT, E0, FP32, tol=1e-6)
          for nm in ("sphere2",) * 4]
    import time
    done = []
    for t in ts:
        while True:
            i = srv.poll(t)
            if i["done"]:
                break
            time.sleep(0.01)
        done.append(i)
        srv.take(t)
    srv.close()
    assert all(i["status"] == 0 for i in done), done
    ev = sorted([(i["t_start_s"], i["footprint"]) for i in done] + [(i["t_end_s"], -i["footprint"]) for i in done])
    use = peak = 0
    live = peak_live = 0
    for _, f in ev:
        use += f
        live += 1 if f > 0 else -1
        peak = max(peak, use)
        peak_live = max(peak_live, live)
    assert all(i["footprint"] <= budget for i in done)
    assert peak <= budget, (peak, budget)
    assert peak_live == 1, peak_live
