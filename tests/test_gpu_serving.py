"""Continuous-batching solve server (``amgdg_server_*``) through the C-ABI.

Every request's status, iteration count, residual and solution must equal, bit
for bit, what ``amgdg_solve`` gives for that right-hand side alone: whatever
shares its batch, whichever column it lands in, whenever it joins, and when an
HBM budget forces it to queue or forces batches of another key out.
"""
import numpy as np
import pytest

import paper_2504_13373_amd as am
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_H = {}


def handle(name):
    if name not in _H:
        print(f"[gpu-serving] building case {name}", flush=True)
        w = {"sipg3": lambda: configs.poisson2d_delaunay(side=33, p=3, n_levels=4, r=3),
             "c1": lambda: configs.poisson2d_split(),
             "ldg2": lambda: configs.convdiff2d_delaunay(side=17, p=2, peclet=100.0, n_levels=3, r=4)}[name]()
        h, _ = am.setup_from_workload(w, mixed=True)
        _H[name] = (w, h)
    return _H[name]


def rhs(n, seed):
    return torch.as_tensor(np.random.default_rng(seed).standard_normal(n)).to(DEV).contiguous()


def alone(h, b, method, prec, rtol, max_it, x0=None, restart=30):
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    rc, st = am.amgdg_solve(h, b, x, method, prec, rtol, max_it, restart=restart,
                            flags=am.AMGDG_X0 if x0 is not None else 0)
    torch.cuda.synchronize()
    return rc, st.iterations[0], st.rel_residual[0], x


def run_server(srv, waves, steps_between=3):
    """Submits the waves of requests with a few server steps in between, so
    later waves join batches that are mid-flight; returns tag -> outcome."""
    out = {}
    for i, wave in enumerate(waves):
        for submit in wave:
            submit()
        if i + 1 < len(waves):
            for _ in range(steps_between):
                srv.step(wait=True)
                for o in srv.poll():
                    out[o[0]] = o
    while srv.step(wait=True) > 0:
        for o in srv.poll():
            out[o[0]] = o
    for o in srv.poll():
        out[o[0]] = o
    return out


def check_equal(res, ref, x, tag):
    rc, its, relres, xa = ref
    tg, status, its_s, rel_s, lat = res
    assert tg == tag
    assert status == (am.AMGDG_OK if rc == am.AMGDG_OK else am.AMGDG_ENOCONV), (tag, status, rc)
    assert its_s == its, (tag, its_s, its)
    assert rel_s == relres, (tag, rel_s, relres)
    assert torch.equal(x, xa), tag
    assert lat > 0


@pytest.mark.parametrize("method,prec", [(am.AMGDG_PCG, am.AMGDG_FP64), (am.AMGDG_FCG, am.AMGDG_MIXED)])
def test_server_equals_alone(method, prec):
    w, h = handle("sipg3")
    n = w.A.n
    B = [rhs(n, 100 + i) for i in range(7)]
    x0 = {3: rhs(n, 300), 5: rhs(n, 305)}          # two requests start from a guess
    refs = [alone(h, B[i], method, prec, 1e-8, 5000, x0.get(i)) for i in range(7)]
    X = [x0[i].clone() if i in x0 else torch.full_like(B[i], float("nan")) for i in range(7)]
    srv = am.Server(width=3, hbm_budget_bytes=1 << 40)

    def sub(i):
        return lambda: srv.submit(h, B[i], X[i], method, prec, 1e-8, 5000,
                                  flags=am.AMGDG_X0 if i in x0 else 0, tag=i)
    out = run_server(srv, [[sub(0), sub(1)], [sub(2), sub(3), sub(4)], [sub(5), sub(6)]])
    srv.close()
    assert sorted(out) == list(range(7))
    for i in range(7):
        check_equal(out[i], refs[i], X[i], i)


def test_server_budget_queues_and_evicts():
    """A budget of one batch: the two keys (PCG FP64 on one hierarchy, FCG
    mixed on another) take turns, each batch released when idle."""
    w1, h1 = handle("sipg3")
    w2, h2 = handle("c1")
    width = 2
    budget = max(am.amgdg_batch_bytes(h1, width), am.amgdg_batch_bytes(h2, width))
    jobs = []
    for i in range(6):
        w, h, meth, prec = ((w1, h1, am.AMGDG_PCG, am.AMGDG_FP64) if i % 2 == 0
                            else (w2, h2, am.AMGDG_FCG, am.AMGDG_MIXED))
        b = rhs(w.A.n, 500 + i)
        jobs.append((h, b, meth, prec, alone(h, b, meth, prec, 1e-9, 5000)))
    X = [torch.zeros_like(j[1]) for j in jobs]
    srv = am.Server(width=width, hbm_budget_bytes=budget)
    subs = [(lambda i=i: srv.submit(jobs[i][0], jobs[i][1], X[i], jobs[i][2], jobs[i][3], 1e-9, 5000, tag=i))
            for i in range(6)]
    out = run_server(srv, [subs[:4], subs[4:]], steps_between=2)
    srv.close()
    assert sorted(out) == list(range(6))
    for i in range(6):
        check_equal(out[i], jobs[i][4], X[i], i)


def test_server_failures_stay_in_their_column():
    """A NaN right-hand side, a zero one and an iteration limit end their own
    requests only; the others in the same batch still equal their solo runs."""
    w, h = handle("sipg3")
    n = w.A.n
    good = [rhs(n, 700 + i) for i in range(3)]
    refs = [alone(h, b, am.AMGDG_PCG, am.AMGDG_FP64, 1e-8, 5000) for b in good]
    capped = rhs(n, 710)
    ref_cap = alone(h, capped, am.AMGDG_PCG, am.AMGDG_FP64, 1e-8, 3)
    assert ref_cap[0] == am.AMGDG_ENOCONV and ref_cap[1] == 3
    bad = rhs(n, 720)
    bad[7] = float("nan")
    zero = torch.zeros(n, dtype=torch.float64, device=DEV)
    Xg = [torch.zeros_like(b) for b in good]
    Xc, Xb, Xz = torch.zeros_like(capped), torch.zeros_like(bad), torch.full_like(zero, 5.0)
    srv = am.Server(width=4, hbm_budget_bytes=1 << 40)
    subs = [lambda: srv.submit(h, good[0], Xg[0], tag=0), lambda: srv.submit(h, bad, Xb, tag=10),
            lambda: srv.submit(h, capped, Xc, max_it=3, tag=11), lambda: srv.submit(h, zero, Xz, tag=12),
            lambda: srv.submit(h, good[1], Xg[1], tag=1), lambda: srv.submit(h, good[2], Xg[2], tag=2)]
    out = run_server(srv, [subs[:4], subs[4:]])
    srv.close()
    for i in range(3):
        check_equal(out[i], refs[i], Xg[i], i)
    assert out[10][1] == am.AMGDG_ENAN
    check_equal(out[11], ref_cap, Xc, 11)
    assert out[12][1] == am.AMGDG_OK and out[12][2] == 0
    assert torch.count_nonzero(Xz).item() == 0


def test_server_mixes_fgmres_and_cg():
    """Non-symmetric requests (FGMRES, one batch each, FP64 and mixed, two
    restart lengths) overlap with CG batches on another hierarchy; every
    result equals its solo run bit for bit."""
    wl, hl = handle("ldg2")
    ws, hs = handle("sipg3")
    jobs = []
    for i in range(8):
        if i % 2 == 0:
            meth, prec, rst = am.AMGDG_FGMRES, (am.AMGDG_FP64 if i % 4 == 0 else am.AMGDG_MIXED), (30 if i < 4 else 7)
            w, h = wl, hl
        else:
            meth, prec, rst = am.AMGDG_PCG, am.AMGDG_FP64, 0
            w, h = ws, hs
        b = rhs(w.A.n, 900 + i)
        jobs.append((h, b, meth, prec, rst, alone(h, b, meth, prec, 1e-8, 3000, restart=max(rst, 1))))
    X = [torch.zeros_like(j[1]) for j in jobs]
    srv = am.Server(width=2, hbm_budget_bytes=1 << 40)
    subs = [(lambda i=i: srv.submit(jobs[i][0], jobs[i][1], X[i], jobs[i][2], jobs[i][3], 1e-8, 3000,
                                    restart=max(jobs[i][4], 1), tag=i)) for i in range(8)]
    out = run_server(srv, [subs[:3], subs[3:6], subs[6:]], steps_between=4)
    srv.close()
    assert sorted(out) == list(range(8))
    for i in range(8):
        check_equal(out[i], jobs[i][5], X[i], i)


def test_fgmres_nan_rhs():
    w, h = handle("ldg2")
    b = rhs(w.A.n, 950)
    b[3] = float("nan")
    x = torch.zeros_like(b)
    with pytest.raises(am.AmgdgError) as e:
        am.amgdg_solve(h, b, x, am.AMGDG_FGMRES, am.AMGDG_FP64, 1e-8, 100)
    assert e.value.code == am.AMGDG_ENAN
    good = rhs(w.A.n, 951)
    ref = alone(h, good, am.AMGDG_FGMRES, am.AMGDG_FP64, 1e-8, 3000)
    xg = torch.zeros_like(good)
    srv = am.Server(width=2, hbm_budget_bytes=1 << 40)
    out = run_server(srv, [[lambda: srv.submit(h, b, x, am.AMGDG_FGMRES, tag=0),
                            lambda: srv.submit(h, good, xg, am.AMGDG_FGMRES, max_it=3000, tag=1)]])
    srv.close()
    assert out[0][1] == am.AMGDG_ENAN
    check_equal(out[1], ref, xg, 1)


def test_server_rejects_bad_requests():
    w, h = handle("c1")
    b = rhs(w.A.n, 1)
    x = torch.zeros_like(b)
    srv = am.Server(width=2, hbm_budget_bytes=1 << 40)
    with pytest.raises(am.AmgdgError) as e:
        srv.submit(h, b, x, am.AMGDG_STATIONARY, tag=0)
    assert e.value.code == am.AMGDG_EUNSUPPORTED
    with pytest.raises(am.AmgdgError) as e:
        srv.submit(h, b, x, am.AMGDG_FGMRES, restart=0, tag=0)
    assert e.value.code == am.AMGDG_EUNSUPPORTED
    srv.close()
    small = am.Server(width=2, hbm_budget_bytes=am.amgdg_batch_bytes(h, 2) - 1)
    with pytest.raises(am.AmgdgError) as e:
        small.submit(h, b, x, tag=0)
    assert e.value.code == am.AMGDG_ENOMEM
    small.close()
    with pytest.raises(am.AmgdgError) as e:
        am.Server(width=65, hbm_budget_bytes=1 << 30)
    assert e.value.code == am.AMGDG_EUNSUPPORTED


def test_server_catalogue_mix():
    """Requests over a catalogue of operators of different sizes and orders
    (SIPG with flexible CG, LDG-upwind with FGMRES(30), FP32 V-cycle), all in
    flight together: each equals its solo solve bit for bit."""
    cat = configs.serving_catalogue(n_ops=6, t_min=300, t_max=3000, seed=5)
    hs = [am.setup_from_workload(w, mixed=True)[0] for w in cat]
    jobs = []
    for i in range(12):
        k = i % len(cat)
        w = cat[k]
        g = np.random.default_rng(2000 + i)
        b = torch.as_tensor(g.standard_normal(w.A.n) if w.krylov == "pcg" else g.uniform(-1, 1, w.A.n)).to(DEV)
        meth = am.AMGDG_FCG if w.krylov == "pcg" else am.AMGDG_FGMRES
        jobs.append((hs[k], b, meth, alone(hs[k], b, meth, am.AMGDG_MIXED, 1e-8, 4000)))
    assert {j[2] for j in jobs} == {am.AMGDG_FCG, am.AMGDG_FGMRES}
    X = [torch.zeros_like(j[1]) for j in jobs]
    srv = am.Server(width=3, hbm_budget_bytes=1 << 40)
    subs = [(lambda i=i: srv.submit(jobs[i][0], jobs[i][1], X[i], jobs[i][2], am.AMGDG_MIXED, 1e-8, 4000, tag=i))
            for i in range(12)]
    out = run_server(srv, [subs[:5], subs[5:9], subs[9:]], steps_between=3)
    srv.close()
    for i in range(12):
        check_equal(out[i], jobs[i][3], X[i], i)
    for h in hs:
        h.close()
