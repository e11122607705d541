"""GPU parity of the paper's default coarse spaces against the FP64 oracle:
oversampled candidates with a coarse size per aggregate (eq:sik), the
h*-step (Algorithm 5's replicated level, eq:sik's second case) and elements
of 27 and 64 dofs (Q2 and Q3 on the structured hex mesh of Section 5.1).

Cases (all through amgdg_setup, the library's own partition):
* sipg3_os: 2D SIPG p=3 on the Delaunay of 30^2 jittered points (1,682
  triangles, 16,820 dofs), r = 40 (the median dofs of a level-1 aggregate),
  n_cut = 3: level-1 aggregates of 3 and 4 triangles keep 10 or 14 coarse
  dofs, level-2 ones 15 or 16, level-3 ones 20 or 21 (padded units);
* hex_r64: Q1 LDG on 8^3 hexahedra, r = 64 (s = 11, 15);
* hex_q2: Q2 LDG (nb = 27) on 8^3 hexahedra, r = 64 (s = 36, 48);
* hex_q2_hstar: the same with an h*-step first (s_e from 8 to 25 per element,
  then 19..32 and 33..34 per aggregate);
* hex_q3: Q3 LDG (nb = 64) on 4^3 hexahedra, r = 64 (s = 64).
The candidate relaxation is capped at 20 sweeps, which keeps the singular
values at every cut separated (smallest gap above 1e-6 of sigma_1).
Coarse levels whose units differ in size are stored padded to the largest;
the comparisons map the library's padded numbering (AMGDG_UNIT_DOFS) to the
oracle's compact one, and check that the padding holds zeros (and the unit
diagonal of A and D^{-1})."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2504_13373_amd as am
from oracle import amg, krylov, rcb
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CASES = ["sipg3_os", "hex_r64", "hex_q2", "hex_q2_hstar", "hex_q3"]


def _relax20(w):
    w.params.relax_max = 20
    return w


def _cases():
    return {
        "sipg3_os": lambda: _relax20(configs.poisson2d_delaunay(side=30, p=3, n_levels=4, r=40)),
        "hex_r64": lambda: configs.poisson3d_hex(3, flux="ldg", r=64, relax_max=20),
        "hex_q2": lambda: configs.poisson3d_hex(3, p=2, flux="ldg", r=64, relax_max=20),
        "hex_q2_hstar": lambda: configs.poisson3d_hex(3, p=2, flux="ldg", r=64, relax_max=20, hstar=True),
        "hex_q3": lambda: configs.poisson3d_hex(2, p=3, flux="ldg", r=64, relax_max=20),
    }


_CACHE = {}


def oracle_aggs(w):
    prm = w.params
    if prm.hstar_top:
        aggs, leaf = rcb.rcb_hierarchy(w.centroids, prm.n_levels - 1, prm.bisections)
        return rcb.replicate_top(aggs, leaf)
    return rcb.rcb_hierarchy(w.centroids, prm.n_levels, prm.bisections)[0]


def case(name):
    if name not in _CACHE:
        print(f"[gpu-oversampled] building case {name}", flush=True)
        w = _cases()[name]()
        aggs = oracle_aggs(w)
        H = amg.setup(w.A.to_scipy(), w.A.nb, aggs, w.params, w.B1)
        h, _ = am.setup_from_workload(w, mixed=True)
        _CACHE[name] = (w, aggs, H, h)
    return _CACHE[name]


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype).contiguous()


def real_index(h, k):
    """Padded row of every real dof of level k, in the oracle's order."""
    info = am.amgdg_level_info_get(h, k)
    sz = am.amgdg_export_level(h, k, am.AMGDG_UNIT_DOFS)
    idx = np.arange(info.n_units)[:, None] * info.nb + np.arange(info.nb)[None, :]
    return idx[np.arange(info.nb)[None, :] < sz[:, None]], sz


def bsr(h, k, which, shape):
    rp_, ci_, v_ = {"A": (am.AMGDG_A_ROWPTR, am.AMGDG_A_COLIDX, am.AMGDG_A_VALS),
                    "T": (am.AMGDG_T_ROWPTR, am.AMGDG_T_COLIDX, am.AMGDG_T_VALS),
                    "R": (am.AMGDG_R_ROWPTR, am.AMGDG_R_COLIDX, am.AMGDG_R_VALS)}[which]
    rp = am.amgdg_export_level(h, k, rp_)
    ci = am.amgdg_export_level(h, k, ci_)
    v = am.amgdg_export_level(h, k, v_)
    return sp.bsr_matrix((v, ci, rp), shape=shape).tocsr(), (rp, ci)


def padded_shape(h, k):
    info = am.amgdg_level_info_get(h, k)
    return info.n_units * info.nb


@pytest.mark.parametrize("name", CASES)
def test_setup_parity_unequal_units(name):
    w, aggs, H, h = case(name)
    N = len(H.levels) - 1
    assert h.n_levels == N + 1
    pats = amg.block_patterns(w.A.row_ptr, w.A.col_idx, aggs)
    for k in range(N):
        L, Ln = H.levels[k], H.levels[k + 1]
        info = am.amgdg_level_info_get(h, k)
        ik, sz = real_index(h, k)
        ik1, sz1 = real_index(h, k + 1)
        assert np.array_equal(sz, L.sizes) and np.array_equal(sz1, Ln.sizes), k
        assert info.n_dofs == L.A.shape[0] and info.s == L.s and info.nb == int(L.sizes.max())
        assert abs(info.omega - L.omega) <= 1e-12 * L.omega, (k, info.omega, L.omega)
        assert list(info.sweeps)[: L.B.shape[1]] == list(L.sweeps), (k, list(info.sweeps), list(L.sweeps))
        n, n1 = padded_shape(h, k), padded_shape(h, k + 1)
        # D^{-1}: real blocks, unit diagonal on the padding
        Dg = am.amgdg_export_level(h, k, am.AMGDG_DINV)
        Dcsr = sp.block_diag(list(Dg), format="csr")
        Do = L.Dinv_bd.to_csr()
        assert sp.linalg.norm(Dcsr[ik][:, ik] - Do) <= 1e-12 * sp.linalg.norm(Do), k
        pad = np.setdiff1d(np.arange(n), ik)
        if len(pad):
            assert np.array_equal(Dcsr[pad][:, pad].toarray(), np.eye(len(pad)))
        B_in = am.amgdg_export_level(h, k, am.AMGDG_B_INPUT)
        B = am.amgdg_export_level(h, k, am.AMGDG_B_RELAXED)
        assert rel(B_in[ik], L.B_in) <= 1e-10 and rel(B[ik], L.B) <= 1e-10, (k, rel(B[ik], L.B))
        assert np.all(B[pad] == 0.0)
        # P~: row i of the export holds its aggregate's s_J columns
        Pu = am.amgdg_export_level(h, k, am.AMGDG_PTILDE)
        coffs = np.concatenate([[0], np.cumsum(L.s_agg)])
        Pc = L.P.tocoo()
        J = np.searchsorted(coffs, Pc.col, side="right") - 1
        Po = np.zeros((L.P.shape[0], info.s))
        Po[Pc.row, Pc.col - coffs[J]] = Pc.data
        assert rel(Pu[ik], Po) <= 1e-9, (k, rel(Pu[ik], Po))
        assert np.all(Pu[pad] == 0.0)
        sv = am.amgdg_export_level(h, k, am.AMGDG_SVALS)
        assert rel(sv, np.stack(L.sv)) <= 1e-10, k
        # T, R = T^T, A_{k+1}: patterns bit for bit, values on the real dofs
        T, (trp, tci) = bsr(h, k, "T", (n, n1))
        assert np.array_equal(trp, pats[k]["T_ptr"]) and np.array_equal(tci, pats[k]["T_idx"])
        assert sp.linalg.norm(T[ik][:, ik1] - L.T) <= 1e-9 * sp.linalg.norm(L.T), k
        R, _ = bsr(h, k, "R", (n1, n))
        assert abs(R - T.T).max() == 0.0
        A1, (arp, aci) = bsr(h, k + 1, "A", (n1, n1))
        assert np.array_equal(arp, pats[k]["A_ptr"]) and np.array_equal(aci, pats[k]["A_idx"])
        assert sp.linalg.norm(A1[ik1][:, ik1] - Ln.A) <= 1e-9 * sp.linalg.norm(Ln.A), k
        pad1 = np.setdiff1d(np.arange(n1), ik1)
        if len(pad1):
            assert np.array_equal(A1[pad1][:, pad1].toarray(), np.eye(len(pad1)))
            assert abs(A1[pad1][:, ik1]).max() == 0.0 and abs(A1[ik1][:, pad1]).max() == 0.0


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", [am.AMGDG_FP64, am.AMGDG_MIXED])
@pytest.mark.parametrize("m", [1, 3, 16])
def test_single_kernels_unequal_units(name, prec, m):
    """Every single step on every level (padded coarse levels included) against
    the host product of the exported operators."""
    from test_gpu_parity import OPS, host_op
    w, aggs, H, h = case(name)
    N = h.n_levels - 1
    g = np.random.default_rng(23 + m)
    dt = torch.float64 if prec == am.AMGDG_FP64 else torch.float32
    for k in range(N):
        info = am.amgdg_level_info_get(h, k)
        n, n1 = info.n, info.n_agg * info.s
        for op in OPS:
            nx = n1 if op == "prolong" else n
            ny = n1 if op.startswith("restrict") else n
            x = g.standard_normal((nx, m))
            b = g.standard_normal((ny, m))
            if prec == am.AMGDG_MIXED:
                x, b = x.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
            y = torch.zeros((ny, m), dtype=dt, device=DEV)
            am.amgdg_apply(h, k, getattr(am, "AMGDG_OP_" + op.upper()), to_dev(x, dt), to_dev(b, dt), y, precision=prec)
            torch.cuda.synchronize()
            want, scale = host_op(op, k, h, w, x, b, prec)
            err = np.abs(y.double().cpu().numpy() - want).max(axis=0) / np.abs(scale).max(axis=0)
            tol = 1e-13 if prec == am.AMGDG_FP64 else 64 * 2.0 ** -24 * 4
            assert np.all(err <= tol), (name, k, op, m, err)


@pytest.mark.parametrize("name", CASES)
def test_vcycle_parity_unequal_units(name):
    w, aggs, H, h = case(name)
    g = np.random.default_rng(8)
    b1, b2 = g.standard_normal(w.A.n), g.standard_normal(w.A.n)
    out = []
    for b in (b1, b2):
        z = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
        am.amgdg_vcycle(h, to_dev(b), z)
        torch.cuda.synchronize()
        out.append(z.cpu().numpy())
    zo = amg.vcycle(H, b1)
    assert rel(out[0], zo) <= 1e-10, rel(out[0], zo)
    assert abs(out[0] @ b2 - b1 @ out[1]) <= 1e-11 * abs(out[0] @ b2)
    z = torch.zeros(w.A.n, dtype=torch.float32, device=DEV)
    am.amgdg_vcycle(h, to_dev(b1, torch.float32), z, precision=am.AMGDG_MIXED)
    torch.cuda.synchronize()
    assert rel(z.double().cpu().numpy(), zo) <= 1e-4


@pytest.mark.parametrize("name", CASES)
def test_pcg_and_mixed_parity_unequal_units(name):
    import scipy.sparse.linalg as spla
    w, aggs, H, h = case(name)
    A = w.A.to_scipy()
    xo, ito, _ = krylov.pcg(A, w.b, lambda r: amg.vcycle(H, r), 1e-8, 5000)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    rc, st = am.amgdg_solve(h, to_dev(w.b), x, am.AMGDG_PCG, am.AMGDG_FP64, 1e-8, 5000)
    assert rc == am.AMGDG_OK and st.iterations[0] == ito, (st.iterations[0], ito)
    assert rel(x.cpu().numpy(), xo) <= 1e-10
    xref = spla.spsolve(A.tocsc(), w.b)
    x.zero_()
    rc, st = am.amgdg_solve(h, to_dev(w.b), x, am.AMGDG_FCG, am.AMGDG_MIXED, 1e-11, 20000)
    assert rc == am.AMGDG_OK
    fwd = rel(x.cpu().numpy(), xref)
    assert fwd <= 1e-8, fwd
    print(f"[oversampled {name}] pCG {ito} iterations (GPU {st.iterations[0]} mixed to 1e-11), "
          f"mixed forward error {fwd:.2e}", flush=True)
