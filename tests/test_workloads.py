"""Checks of the synthetic input generators (DG assembly): manufactured-solution
convergence orders (SIPG and LDG: p+1 on these meshes; the paper's manufactured
solution of Section 5.1 in its 2D form, which vanishes on the unit square's
boundary), symmetry and definiteness, mesh statistics."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads import configs, dg, mesh as meshes

PI = np.pi


def u_exact(x):
    return np.exp(np.sin(PI * x[:, 0]) * np.sin(PI * x[:, 1])) - 1.0


def grad_u(x):
    e = np.exp(np.sin(PI * x[:, 0]) * np.sin(PI * x[:, 1]))
    return np.stack([e * PI * np.cos(PI * x[:, 0]) * np.sin(PI * x[:, 1]),
                     e * PI * np.sin(PI * x[:, 0]) * np.cos(PI * x[:, 1])], 1)


def lap_u(x):
    s = np.sin(PI * x[:, 0]) * np.sin(PI * x[:, 1])
    g2 = (grad_u(x) ** 2).sum(1) / np.exp(s) ** 2
    return np.exp(s) * (-2 * PI ** 2 * s + g2)


def rates(errs):
    e = np.array(errs)
    return np.log2(e[:-1] / e[1:])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_sipg_mms_order(p):
    errs = []
    for side in (9, 17, 33):
        m = meshes.jittered_delaunay(side)
        A = dg.assemble_sipg(m, p).to_scipy()
        b = dg.load_vector(m, p, lambda x: -lap_u(x))
        errs.append(dg.l2_error(m, p, spla.spsolve(A.tocsc(), b), u_exact))
    assert np.all(np.abs(rates(errs) - (p + 1)) < 0.3)


@pytest.mark.parametrize("eps", [1.0, 1e-2])
def test_ldg_upwind_mms_order(eps):
    beta = np.array([np.cos(0.3), np.sin(0.3)])
    p = 2
    errs = []
    for side in (9, 17, 33):
        m = meshes.jittered_delaunay(side)
        A = dg.assemble_ldg_upwind(m, p, beta, eps).to_scipy()
        b = dg.load_vector(m, p, lambda x: -eps * lap_u(x) + grad_u(x) @ beta)
        errs.append(dg.l2_error(m, p, spla.spsolve(A.tocsc(), b), u_exact))
    assert np.all(rates(errs) > p + 0.5)


def test_sipg_symmetric_spd_and_pattern():
    m = meshes.jittered_delaunay(9)
    Ab = dg.assemble_sipg(m, 2)
    A = Ab.to_scipy().toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)
    # pattern: diagonal + face neighbours
    assert Ab.nnzb == m.n_elem + 2 * len(m.int_faces)


def test_ldg_pure_convection_part_is_semidefinite():
    m = meshes.jittered_delaunay(9)
    A = dg.assemble_ldg_upwind(m, 1, np.array([np.cos(0.3), np.sin(0.3)]), 0.0).to_scipy().toarray()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > -1e-12


def test_mesh_statistics():
    m = meshes.jittered_delaunay(65)
    assert m.n_elem == 2 * 64 * 64
    assert np.all(m.volumes() > 0.1 * (1 / 64) ** 2 / 2)
    m3 = meshes.kuhn_cube(4)
    assert m3.n_elem == 6 * 64
    assert np.isclose(m3.volumes().sum(), 1.0)
    assert len(m3.bnd_faces) == 6 * 16 * 2


def test_config_c1_sizes():
    w = configs.poisson2d_split()
    assert w.A.n == 1536 and w.A.nnzb == 512 + 2 * 736


@pytest.mark.parametrize("n_elem", [513, 700, 1100, 2049, 3000, 4097, 5500])
@pytest.mark.parametrize("p", [1, 2, 4])
def test_catalogue_aggregation_keeps_uniform_coarse_size(n_elem, p):
    """The serving catalogue's rule (8-way aggregation for p = 1, 4-way
    otherwise; levels until the coarsest holds at most 2,048 dofs) gives every
    aggregate of every level at least r = 3 dofs, hence one coarse block size
    s = min(ceil(|A_J| / n_cut), |A_J|, r) = 3 per level (eq:sik)."""
    from oracle import rcb
    rng = np.random.default_rng(n_elem)
    cent = rng.random((n_elem, 2))
    nb = (p + 1) * (p + 2) // 2
    bis = 3 if p == 1 else 2
    L = configs.levels_for_coarsest(n_elem, bis)
    aggs, _ = rcb.rcb_hierarchy(cent, L, bis)
    dofs = np.full(n_elem, nb)
    for k, a in enumerate(aggs):
        per = np.bincount(a, weights=dofs).astype(int)
        s = {min(-(-int(d) // 3), int(d), 3) for d in per}
        assert s == {3}, (k, sorted(set(per.tolist()))[:5])
        dofs = np.full(len(per), 3)
    assert len(dofs) * 3 <= 2048 or L == 2
