"""amgdg_vcycle_static, the V-cycle entry point that allocates nothing (its
level vectors live in the library's static per-GPU workspace), against
amgdg_vcycle through the C-ABI.  Both launch the same kernels in the same
order, so the results are bit-identical.  Two calls in a row, the second on a
smaller input (a smaller hierarchy, fewer columns), each compared with the
allocating entry point; then an input too large for the workspace is
rejected before any work is queued."""
import numpy as np
import pytest

import paper_2504_13373_amd as am
from workloads import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _handle(w):
    print(f"[no-alloc] setting up {w.name} ({w.A.n} dofs)", flush=True)
    h, _ = am.setup_from_workload(w, mixed=True)
    return h


def _check(h, n, m, prec, flags, seed):
    dt = torch.float64 if prec == am.AMGDG_FP64 else torch.float32
    g = np.random.default_rng(seed)
    shape = (n, m) if m > 1 else (n,)
    r = torch.as_tensor(g.standard_normal(shape)).to(DEV, dtype=dt).contiguous()
    z_ref = torch.zeros_like(r)
    am.amgdg_vcycle(h, r, z_ref, precision=prec, flags=flags)
    z = torch.full_like(r, float("nan"))
    am.amgdg_vcycle_static(h, r, z, precision=prec, flags=flags)
    torch.cuda.synchronize()
    assert torch.isfinite(z).all()
    assert torch.equal(z, z_ref), (m, prec, flags)


def test_static_vcycle_matches_allocating_vcycle_twice_second_smaller():
    big = _handle(configs.poisson2d_delaunay(side=33, p=3, n_levels=4, r=3))      # 20,480 dofs
    small = _handle(configs.poisson2d_split())                                      # 1,536 dofs
    try:
        print("[no-alloc] call 1: 20,480 dofs, 3 columns, FP64, caller order", flush=True)
        _check(big, 20480, 3, am.AMGDG_FP64, 0, 1)
        print("[no-alloc] call 2: 1,536 dofs, 1 column, FP32 V-cycle, caller order", flush=True)
        _check(small, 1536, 1, am.AMGDG_MIXED, 0, 2)
        print("[no-alloc] internal order, both precisions", flush=True)
        _check(big, 20480, 1, am.AMGDG_MIXED, am.AMGDG_INTERNAL_ORDER, 3)
        _check(small, 1536, 5, am.AMGDG_FP64, am.AMGDG_INTERNAL_ORDER, 4)
    finally:
        big.close()
        small.close()


def test_static_vcycle_rejects_inputs_beyond_the_workspace():
    w = configs.poisson2d_delaunay(side=129, p=3, n_levels=4, r=3)                 # about 330k dofs
    h = _handle(w)
    try:
        r = torch.zeros((w.A.n, 64), dtype=torch.float64, device=DEV)
        z = torch.zeros_like(r)
        with pytest.raises(am.AmgdgError) as e:
            am.amgdg_vcycle_static(h, r, z)
        assert e.value.code == am.AMGDG_EUNSUPPORTED
        assert "static workspace" in str(e.value)
        # the same handle still serves inputs that fit
        _check(h, w.A.n, 1, am.AMGDG_FP64, 0, 5)
    finally:
        h.close()
