"""Parity at the benchmark sizes, in the launch configurations bench.py times.

* 2D Poisson SIPG p=3 on 256^2 jittered points (1,300,500 dofs) and 2D LDG +
  upwind p=2 on 363^2 points (1,572,528 dofs, Peclet 100): the FP64 oracle is
  set up at full size on the host, so setup, V-cycle and a prefix of the
  Krylov iterations are compared with it directly.
* 3D Poisson SIPG p=2 on 64^3 x 6 tetrahedra (15,728,640 dofs) with 16 columns:
  too large for the oracle's setup in seconds, so sampled element rows of the
  16-column MFMA products (A x, the sweep, and the sweep on D^{-1} A) are
  checked against the caller's own matrix on the host, and the 16-column
  V-cycle against the single-column one.
* The structured hex problem at M = 5 (262,144 dofs, LDG, 16 candidates):
  the oracle is set up at full size; the levels whose candidate blocks are
  well conditioned are compared directly, the solve for validity.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2504_13373_amd as am
from oracle import amg, krylov, rcb
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_C = {}


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype).contiguous()


def case(name):
    if name not in _C:
        print(f"[gpu-fullsize] building {name}", flush=True)
        if name == "poisson2d":
            w = configs.poisson2d_delaunay(side=256)
        else:
            w = configs.convdiff2d_delaunay(side=363, peclet=100.0)
        aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
        H = amg.setup(w.A.to_scipy(), w.A.nb, aggs, w.params, w.B1)
        h, _ = am.setup_from_workload(w, mixed=True)
        print(f"[gpu-fullsize] {name}: {w.A.n} dofs, {h.n_levels} levels", flush=True)
        _C[name] = (w, H, h)
    return _C[name]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["poisson2d", "convdiff"])
def test_fullsize_setup_and_vcycle(name):
    w, H, h = case(name)
    N = len(H.levels) - 1
    assert h.n_levels == N + 1
    for k in range(N):
        info = am.amgdg_level_info_get(h, k)
        L = H.levels[k]
        assert info.n == L.A.shape[0] and info.s == L.s
        assert abs(info.omega - L.omega) <= 1e-12 * L.omega, (k, info.omega, L.omega)
        assert list(info.sweeps)[: L.B.shape[1]] == list(L.sweeps), k
    A1 = sp.bsr_matrix((am.amgdg_export_level(h, 1, am.AMGDG_A_VALS), am.amgdg_export_level(h, 1, am.AMGDG_A_COLIDX),
                        am.amgdg_export_level(h, 1, am.AMGDG_A_ROWPTR)), shape=H.levels[1].A.shape).tocsr()
    assert sp.linalg.norm(A1 - H.levels[1].A) <= 1e-9 * sp.linalg.norm(H.levels[1].A)
    r = np.random.default_rng(61).standard_normal(w.A.n)
    zo = amg.vcycle(H, r)
    z = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    am.amgdg_vcycle(h, to_dev(r), z)
    z32 = torch.zeros(w.A.n, dtype=torch.float32, device=DEV)
    am.amgdg_vcycle(h, to_dev(r, torch.float32), z32, precision=am.AMGDG_MIXED)
    torch.cuda.synchronize()
    assert rel(z.cpu().numpy(), zo) <= 1e-10
    assert rel(z32.double().cpu().numpy(), zo) <= 1e-4


@pytest.mark.timeout(600)
def test_fullsize_restriction_through_M():
    """The level-0 restriction through M = R (D - omega A) at full size (the
    entry-wise block-CSR kernel, a wavefront per block row) against the
    oracle's R (D - omega A) x, and each of five columns bit-identical to the
    same column restricted alone."""
    w, H, h = case("poisson2d")
    info = am.amgdg_level_info_get(h, 0)
    assert info.restrict_resid == 1
    L = H.levels[0]
    A = L.A.tocoo()
    on = (A.row // L.nb) == (A.col // L.nb)
    D = sp.csr_matrix((A.data[on], (A.row[on], A.col[on])), shape=L.A.shape)
    perm = am.amgdg_export_level(h, 0, am.AMGDG_PERM)
    dofs = (perm[:, None] * L.nb + np.arange(L.nb)).ravel()  # internal dof -> caller dof
    n1 = info.n_agg * info.s
    X = np.random.default_rng(63).standard_normal((w.A.n, 5))
    Mo = (L.T.T @ (D - L.omega * L.A)).tocsr()
    want = Mo @ X
    Y5 = torch.zeros((n1, 5), dtype=torch.float64, device=DEV)
    am.amgdg_apply(h, 0, am.AMGDG_OP_RESTRICT_RESID, to_dev(X[dofs]), None, Y5, flags=am.AMGDG_INTERNAL_ORDER)
    torch.cuda.synchronize()
    assert rel(Y5.cpu().numpy(), want) <= 1e-12, rel(Y5.cpu().numpy(), want)
    for c in range(5):
        y1 = torch.zeros((n1, 1), dtype=torch.float64, device=DEV)
        am.amgdg_apply(h, 0, am.AMGDG_OP_RESTRICT_RESID, to_dev(X[dofs, c:c + 1]), None, y1,
                       flags=am.AMGDG_INTERNAL_ORDER)
        torch.cuda.synchronize()
        assert torch.equal(y1[:, 0].cpu(), Y5[:, c].contiguous().cpu()), c


@pytest.mark.timeout(600)
def test_fullsize_pcg_prefix_matches_oracle():
    """40 PCG iterations (capped) on the 1.3M-dof case: the iterate equals the
    oracle's after the same 40 iterations."""
    w, H, h = case("poisson2d")
    A = w.A.to_scipy()
    xo, ito, _ = krylov.pcg(A, w.b, lambda v: amg.vcycle(H, v), 1e-30, 40)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    rc, st = am.amgdg_solve(h, to_dev(w.b), x, am.AMGDG_PCG, am.AMGDG_FP64, 1e-30, 40)
    assert rc == am.AMGDG_ENOCONV and st.iterations[0] == 40 == ito
    assert rel(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.timeout(600)
def test_fullsize_fgmres_prefix_matches_oracle():
    """FGMRES(30) capped at 45 iterations (one restart) on the 1.57M-dof
    non-symmetric case, against the oracle's FGMRES."""
    w, H, h = case("convdiff")
    A = w.A.to_scipy()
    xo, ito, _ = krylov.fgmres(A, w.b, lambda v: amg.vcycle(H, v), 1e-30, 30, 45)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    rc, st = am.amgdg_solve(h, to_dev(w.b), x, am.AMGDG_FGMRES, am.AMGDG_FP64, 1e-30, 45, restart=30)
    assert rc == am.AMGDG_ENOCONV and st.iterations[0] == 45 == ito
    assert rel(x.cpu().numpy(), xo) <= 1e-8


def _block_rows_product(Ab, elems, X, absolute=False):
    """(A X), or (|A| |X|), restricted to the dofs of the element rows `elems`,
    from the caller's BSR."""
    nb = Ab.nb
    out = np.zeros((len(elems), nb, X.shape[1]))
    for t, e in enumerate(elems):
        for j in range(Ab.row_ptr[e], Ab.row_ptr[e + 1]):
            c = Ab.col_idx[j]
            blk, xb = Ab.vals[j], X[c * nb:(c + 1) * nb]
            out[t] += (np.abs(blk) @ np.abs(xb)) if absolute else (blk @ xb)
    return out


@pytest.mark.timeout(900)
def test_fullsize_3d_mfma_products_and_vcycle():
    print("[gpu-fullsize] building poisson3d 64^3 x 6, 16 columns", flush=True)
    w = configs.poisson3d_kuhn(n=64, n_rhs=16)
    h, _ = am.setup_from_workload(w, mixed=True)
    n, nb, m = w.A.n, w.A.nb, 16
    info = am.amgdg_level_info_get(h, 0)
    g = np.random.default_rng(71)
    X = g.standard_normal((n, m))
    B = g.standard_normal((n, m))
    elems = np.sort(g.choice(w.A.n_brow, 400, replace=False))
    dofs = (elems[:, None] * nb + np.arange(nb)).ravel()
    AX = _block_rows_product(w.A, elems, X).reshape(-1, m)
    absAX = _block_rows_product(w.A, elems, X, absolute=True).reshape(-1, m)
    Dinv = np.stack([np.linalg.inv(w.A.vals[w.A.row_ptr[e] + np.nonzero(
        w.A.col_idx[w.A.row_ptr[e]:w.A.row_ptr[e + 1]] == e)[0][0]]) for e in elems])
    for prec, dt, tol in ((am.AMGDG_FP64, torch.float64, 1e-12), (am.AMGDG_MIXED, torch.float32, 2e-5)):
        Y = torch.zeros((n, m), dtype=dt, device=DEV)
        am.amgdg_apply(h, 0, am.AMGDG_OP_SPMV, to_dev(X, dt), None, Y, precision=prec)
        torch.cuda.synchronize()
        err = np.abs(Y.double().cpu().numpy()[dofs] - AX).max() / np.abs(absAX).max()
        assert err <= tol, (prec, err)
        am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP, to_dev(X, dt), to_dev(B, dt), Y, precision=prec)
        torch.cuda.synchronize()
        R = (B[dofs] - AX).reshape(len(elems), nb, m)
        want = X[dofs] + info.omega * np.einsum("eij,ejc->eic", Dinv, R).reshape(-1, m)
        scale = np.abs(X[dofs]).max() + info.omega * np.abs(Dinv).max() * nb * (np.abs(B).max() + np.abs(absAX).max())
        err = np.abs(Y.double().cpu().numpy()[dofs] - want).max() / scale
        assert err <= tol, (prec, err)
        # the V-cycle's sweep on S = D^{-1} A, with B standing for D^{-1} b
        am.amgdg_apply(h, 0, am.AMGDG_OP_SWEEP_SCALED, to_dev(X, dt), to_dev(B, dt), Y, precision=prec)
        torch.cuda.synchronize()
        SX = np.einsum("eij,ejc->eic", Dinv, AX.reshape(len(elems), nb, m)).reshape(-1, m)
        absSX = np.einsum("eij,ejc->eic", np.abs(Dinv), absAX.reshape(len(elems), nb, m)).reshape(-1, m)
        want = X[dofs] + info.omega * (B[dofs] - SX)
        scale = np.abs(X[dofs]).max() + info.omega * (np.abs(B).max() + np.abs(absSX).max())
        err = np.abs(Y.double().cpu().numpy()[dofs] - want).max() / scale
        assert err <= tol, (prec, err)
        del Y
    # 16-column V-cycle (MFMA level 0) against single-column V-cycles
    Z = torch.zeros((n, m), dtype=torch.float64, device=DEV)
    Bd = to_dev(B)
    am.amgdg_vcycle(h, Bd, Z)
    for c in (0, 11):
        z = torch.zeros(n, dtype=torch.float64, device=DEV)
        am.amgdg_vcycle(h, Bd[:, c].contiguous(), z)
        torch.cuda.synchronize()
        assert rel(Z[:, c].cpu().numpy(), z.cpu().numpy()) <= 1e-12, c
    # a capped 16-column mixed solve: every column's true residual falls and stays finite
    Xs = torch.zeros((n, m), dtype=torch.float64, device=DEV)
    rc, st = am.amgdg_solve(h, to_dev(w.b), Xs, am.AMGDG_FCG, am.AMGDG_MIXED, 1e-30, 30)
    assert rc == am.AMGDG_ENOCONV and st.max_iterations == 30
    relres = np.array(list(st.rel_residual)[:m])
    assert np.all(np.isfinite(relres)) and np.all(relres < 1.0), relres
    h.close()


@pytest.mark.timeout(600)
def test_fullsize_hex_m5_ldg_r16():
    """The structured hex problem at the largest size bench.py --workload hex
    times: 32^3 Q1 hexahedra (262,144 dofs), LDG, 16 candidates, 5 levels.
    The oracle is set up at full size.  Levels 0 and 1 truncate well-conditioned
    candidate blocks (16 columns to 11 and 15; smallest relative gap at the cut
    5e-6), so their damping, relaxation sweeps, D^{-1} and the coarse operators
    A_1 and A_2 are held to the full bar, and so are level 2's damping and
    sweep counts (the split-row kernel's power-iteration and relaxation modes).  Every single step on every level is
    compared with the host product of the exported operators, in both
    precisions, one and three columns.  Level 2 keeps all 16 columns of
    nearly collapsed blocks (condition 1e10), so below it only the solve is
    checked for validity: pCG to the paper's 1e-7 in true residual, in the
    oracle's iteration count within one."""
    print("[gpu-fullsize] building hex M=5 ldg r=16", flush=True)
    w = configs.poisson3d_hex(5, flux="ldg", r=16)
    A = w.A.to_scipy()
    aggs, _ = rcb.rcb_hierarchy(w.centroids, w.params.n_levels, w.params.bisections)
    H = amg.setup(A, w.A.nb, aggs, w.params, w.B1)
    h, _ = am.setup_from_workload(w, mixed=True)
    try:
        assert h.n_levels == len(H.levels) == 5
        for k in (0, 1):
            info, L = am.amgdg_level_info_get(h, k), H.levels[k]
            assert info.n == L.A.shape[0] and info.s == L.s
            assert abs(info.omega - L.omega) <= 1e-12 * L.omega, (k, info.omega, L.omega)
            assert list(info.sweeps)[: L.B.shape[1]] == list(L.sweeps), k
            assert rel(am.amgdg_export_level(h, k, am.AMGDG_DINV), L.Dinv) <= 1e-12
            n1 = H.levels[k + 1].A.shape[0]
            rp = am.amgdg_export_level(h, k + 1, am.AMGDG_A_ROWPTR)
            ci = am.amgdg_export_level(h, k + 1, am.AMGDG_A_COLIDX)
            v = am.amgdg_export_level(h, k + 1, am.AMGDG_A_VALS)
            A1 = sp.bsr_matrix((v, ci, rp), shape=(n1, n1)).tocsr()
            ref = H.levels[k + 1].A
            assert sp.linalg.norm(A1 - ref) <= 1e-9 * sp.linalg.norm(ref), k
        # level 2 (A_2 held to 1e-9 above) runs its power iteration and candidate
        # relaxation through the split-row sweep kernel: its damping and sweep
        # counts are held to the same bar
        info, L = am.amgdg_level_info_get(h, 2), H.levels[2]
        assert abs(info.omega - L.omega) <= 1e-12 * L.omega, (info.omega, L.omega)
        assert list(info.sweeps)[: L.B.shape[1]] == list(L.sweeps), (list(info.sweeps), list(L.sweeps))
        # every single step on every level against the host product of the exported
        # operators (level 2's long rows take the split-row kernel), and a column
        # of a 3-column launch equal to the same column alone
        from test_gpu_parity import OPS, host_op
        g = np.random.default_rng(29)
        for prec, dt in ((am.AMGDG_FP64, torch.float64), (am.AMGDG_MIXED, torch.float32)):
            for k in range(h.n_levels - 1):
                info = am.amgdg_level_info_get(h, k)
                n, n1 = info.n, info.n_agg * info.s
                for op in OPS:
                    nx = n1 if op == "prolong" else n
                    ny = n1 if op.startswith("restrict") else n
                    xs = g.standard_normal((nx, 3))
                    bs = g.standard_normal((ny, 3))
                    if prec == am.AMGDG_MIXED:
                        xs, bs = (v.astype(np.float32).astype(np.float64) for v in (xs, bs))
                    code = getattr(am, "AMGDG_OP_" + op.upper())
                    y3 = torch.zeros((ny, 3), dtype=dt, device=DEV)
                    am.amgdg_apply(h, k, code, to_dev(xs, dt), to_dev(bs, dt), y3, precision=prec)
                    y1 = torch.zeros(ny, dtype=dt, device=DEV)
                    am.amgdg_apply(h, k, code, to_dev(xs[:, 0], dt), to_dev(bs[:, 0], dt), y1, precision=prec)
                    torch.cuda.synchronize()
                    assert torch.equal(y3[:, 0], y1), (prec, k, op)
                    want, scale = host_op(op, k, h, w, xs, bs, prec)
                    err = np.abs(y3.double().cpu().numpy() - want).max(axis=0) / np.abs(scale).max(axis=0)
                    tol = 1e-13 if prec == am.AMGDG_FP64 else 64 * 2.0 ** -24 * 4
                    assert np.all(err <= tol), (prec, k, op, err)
        _, ito = krylov.pcg(A, w.b, lambda r: amg.vcycle(H, r), 1e-7, 200)[:2]
        x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
        rc, st = am.amgdg_solve(h, to_dev(w.b), x, am.AMGDG_PCG, am.AMGDG_FP64, 1e-7, 200)
        assert rc == am.AMGDG_OK and abs(st.iterations[0] - ito) <= 1, (st.iterations[0], ito)
        assert np.linalg.norm(w.b - A @ x.cpu().numpy()) <= 1e-7 * np.linalg.norm(w.b)
        print(f"[gpu-fullsize] hex M=5: pCG {st.iterations[0]} iterations (oracle {ito})", flush=True)
    finally:
        h.close()


@pytest.mark.timeout(900)
def test_fullsize_oversampled_long_rows():
    """The headline mesh (Delaunay of 256^2 jittered points, SIPG p=3,
    1,300,500 dofs) with the paper's oversampled coarse spaces: r = 40, s_J
    per aggregate, 7 levels.  Levels 3 and 4 (26- and 35-dof units, rows across
    much of the level) are too long for one x staging in FP64 and run the
    chunked form.  The products with A_k, the sweeps with D^{-1} and on
    S = D^{-1} A_k, and the residual are checked on 300 sampled block rows
    against the exported operators, in both precisions, and a column of a
    3-column launch equals the same column alone."""
    print("[gpu-fullsize] building the oversampled 2D hierarchy", flush=True)
    w = configs.poisson2d_delaunay(side=256, p=3, n_levels=7, r=40)
    h, _ = am.setup_from_workload(w, mixed=True)
    try:
        g = np.random.default_rng(31)
        for k in (3, 4):
            info = am.amgdg_level_info_get(h, k)
            n, nb = info.n, info.nb
            rp = am.amgdg_export_level(h, k, am.AMGDG_A_ROWPTR)
            ci = am.amgdg_export_level(h, k, am.AMGDG_A_COLIDX)
            Av = am.amgdg_export_level(h, k, am.AMGDG_A_VALS)
            Dinv = am.amgdg_export_level(h, k, am.AMGDG_DINV)
            rows = np.sort(g.choice(info.n_units, size=min(300, info.n_units), replace=False))
            print(f"[gpu-fullsize] oversampled level {k}: {info.n_units} units of {nb}, "
                  f"{int(np.diff(rp).max())} blocks in the longest row", flush=True)
            for prec, dt in ((am.AMGDG_FP64, torch.float64), (am.AMGDG_MIXED, torch.float32)):
                x = g.standard_normal((n, 3))
                b = g.standard_normal((n, 3))
                if prec == am.AMGDG_MIXED:
                    x, b = x.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
                A32 = Av.astype(np.float32).astype(np.float64) if prec == am.AMGDG_MIXED else Av
                D32 = Dinv.astype(np.float32).astype(np.float64) if prec == am.AMGDG_MIXED else Dinv
                om = info.omega if prec == am.AMGDG_FP64 else float(np.float32(info.omega))
                X = x.reshape(info.n_units, nb, 3)
                B = b.reshape(info.n_units, nb, 3)
                want, scale = {}, {}
                ax = np.stack([np.einsum("kij,kjc->ic", A32[rp[e]:rp[e + 1]], X[ci[rp[e]:rp[e + 1]]]) for e in rows])
                aax = np.stack([np.einsum("kij,kjc->ic", np.abs(A32[rp[e]:rp[e + 1]]), np.abs(X[ci[rp[e]:rp[e + 1]]]))
                                for e in rows])
                # S = D^{-1} A formed in FP64 (then rounded for FP32), as the library forms it
                S = {e: np.einsum("ij,kjl->kil", Dinv[e], Av[rp[e]:rp[e + 1]]) for e in rows}
                if prec == am.AMGDG_MIXED:
                    S = {e: v.astype(np.float32).astype(np.float64) for e, v in S.items()}
                sx = np.stack([np.einsum("kij,kjc->ic", S[e], X[ci[rp[e]:rp[e + 1]]]) for e in rows])
                asx = np.stack([np.einsum("kij,kjc->ic", np.abs(np.einsum("ij,kjl->kil", Dinv[e], Av[rp[e]:rp[e + 1]])),
                                          np.abs(X[ci[rp[e]:rp[e + 1]]])) for e in rows])
                Dr, Br, Xr = D32[rows], B[rows], X[rows]
                want["spmv"], scale["spmv"] = ax, aax
                want["residual"], scale["residual"] = Br - ax, np.abs(Br) + aax
                want["sweep"] = Xr + om * np.einsum("uij,ujc->uic", Dr, Br - ax)
                scale["sweep"] = np.abs(Xr) + om * np.einsum("uij,ujc->uic", np.abs(Dr), np.abs(Br) + aax)
                want["sweep_scaled"] = Xr + om * (Br - sx)
                scale["sweep_scaled"] = np.abs(Xr) + om * (np.abs(Br) + asx)
                for op in ("spmv", "residual", "sweep", "sweep_scaled"):
                    code = getattr(am, "AMGDG_OP_" + op.upper())
                    y3 = torch.zeros((n, 3), dtype=dt, device=DEV)
                    am.amgdg_apply(h, k, code, to_dev(x, dt), to_dev(b, dt), y3, precision=prec)
                    y1 = torch.zeros(n, dtype=dt, device=DEV)
                    am.amgdg_apply(h, k, code, to_dev(x[:, 0], dt), to_dev(b[:, 0], dt), y1, precision=prec)
                    torch.cuda.synchronize()
                    assert torch.equal(y3[:, 0], y1), (prec, k, op)
                    got = y3.double().cpu().numpy().reshape(info.n_units, nb, 3)[rows]
                    err = np.abs(got - want[op]).max(axis=(0, 1)) / np.abs(scale[op]).max(axis=(0, 1))
                    tol = 1e-13 if prec == am.AMGDG_FP64 else 64 * 2.0 ** -24 * 4
                    assert np.all(err <= tol), (prec, k, op, err)
                    print(f"[gpu-fullsize]   level {k} {op} {'fp64' if prec == am.AMGDG_FP64 else 'fp32'} "
                          f"error {err.max():.2e}", flush=True)
    finally:
        h.close()
