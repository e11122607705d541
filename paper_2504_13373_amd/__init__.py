"""Python binding of libamgdg (geometric alpha-SA multigrid for DG, HIP on gfx950).

Argument marshalling only: every step of the setup and of the solve runs in the
library's HIP kernels.  Functions carry the names of the C entry points
declared in include/amgdg.h.  Device arrays are torch tensors on a ROCm device
(their data pointers are passed through); host arrays are numpy arrays.  The
library must have been built (``python -m paper_2504_13373_amd.build``); if it
is missing, every call raises.
"""
import ctypes
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamgdg.so")

# status codes
AMGDG_OK, AMGDG_EINVAL, AMGDG_ESINGULAR, AMGDG_ENOMEM = 0, -1, -2, -3
AMGDG_EHIP, AMGDG_ENAN, AMGDG_EBREAKDOWN, AMGDG_EUNSUPPORTED, AMGDG_ENOCONV = -4, -5, -6, -7, 1
# export items
AMGDG_PERM, AMGDG_T_ROWPTR, AMGDG_T_COLIDX, AMGDG_A_ROWPTR, AMGDG_A_COLIDX = 1, 2, 3, 4, 5
AMGDG_R_ROWPTR, AMGDG_R_COLIDX = 6, 7
AMGDG_A_VALS, AMGDG_T_VALS, AMGDG_R_VALS, AMGDG_DINV = 10, 11, 12, 13
AMGDG_B_RELAXED, AMGDG_B_INPUT, AMGDG_PTILDE, AMGDG_SVALS, AMGDG_UNIT_DOFS = 14, 15, 16, 17, 18
AMGDG_M_ROWPTR, AMGDG_M_COLIDX, AMGDG_M_VALS = 19, 20, 21
# precision, methods, flags, ops
AMGDG_FP64, AMGDG_MIXED = 0, 1
AMGDG_STATIONARY, AMGDG_PCG, AMGDG_FCG, AMGDG_FGMRES = 0, 1, 2, 3
AMGDG_X0, AMGDG_INTERNAL_ORDER, AMGDG_EAGER = 1, 2, 4
AMGDG_TUNE_LANES = 1
(AMGDG_OP_SPMV, AMGDG_OP_SWEEP, AMGDG_OP_SWEEP0, AMGDG_OP_RESIDUAL, AMGDG_OP_RESTRICT,
 AMGDG_OP_PROLONG, AMGDG_OP_COARSE, AMGDG_OP_SWEEP_SCALED, AMGDG_OP_RESTRICT_SCALED,
 AMGDG_OP_RESTRICT_RESID, AMGDG_OP_SWEEP_SCALED_RESID) = range(11)


class amgdg_params(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("r", ctypes.c_int32), ("t_pre", ctypes.c_int32),
                ("t_post", ctypes.c_int32), ("q_power", ctypes.c_int32), ("relax_max", ctypes.c_int32),
                ("omega_fixed", ctypes.c_double), ("gamma", ctypes.c_double), ("n_cut", ctypes.c_double),
                ("b_update", ctypes.c_int32), ("mixed", ctypes.c_int32), ("pow_seed", ctypes.c_uint64),
                ("b1_seed", ctypes.c_uint64), ("delta", ctypes.c_double), ("hstar_smooth", ctypes.c_int32),
                ("matfree_levels", ctypes.c_int32), ("restrict_resid", ctypes.c_int32)]


class amgdg_level_info(ctypes.Structure):
    _fields_ = [("n_units", ctypes.c_int64), ("nb", ctypes.c_int32), ("s", ctypes.c_int32),
                ("n", ctypes.c_int64), ("nnzb", ctypes.c_int64), ("nnzb_T", ctypes.c_int64),
                ("n_agg", ctypes.c_int64), ("omega", ctypes.c_double), ("rho", ctypes.c_double),
                ("r", ctypes.c_int32), ("sweeps", ctypes.c_int32 * 64), ("bytes_A", ctypes.c_int64),
                ("bytes_Dinv", ctypes.c_int64), ("bytes_T", ctypes.c_int64), ("bytes_R", ctypes.c_int64),
                ("n_dofs", ctypes.c_int64), ("matfree", ctypes.c_int32), ("bytes_handle", ctypes.c_int64),
                ("nnzb_M", ctypes.c_int64), ("restrict_resid", ctypes.c_int32), ("bytes_M", ctypes.c_int64),
                ("nnzb_S", ctypes.c_int64)]


class amgdg_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 64), ("rel_residual", ctypes.c_double * 64),
                ("max_iterations", ctypes.c_int32), ("all_converged", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


class AmgdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"amgdg error {code}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

_SIGS = {
    "amgdg_default_params": (None, [ctypes.POINTER(amgdg_params)]),
    "amgdg_last_error": (ctypes.c_char_p, []),
    "amgdg_partition_rcb": (_I32, [_I64, _I32, _P, _I32, _I32, _P, _P]),
    "amgdg_plan_create": (_I32, [ctypes.POINTER(_P), _I64, _P, _P, _I64, _I32, _P]),
    "amgdg_plan_destroy": (None, [_P]),
    "amgdg_plan_size": (_I32, [_P, _I32, _I32, ctypes.POINTER(_I64)]),
    "amgdg_plan_export": (_I32, [_P, _I32, _I32, _P, _I64]),
    "amgdg_setup": (_I32, [ctypes.POINTER(_P), _I64, _I32, _P, _P, _P, _I64, _P, _P, _P,
                           ctypes.POINTER(amgdg_params), _P, _P]),
    "amgdg_destroy": (_I32, [_P]),
    "amgdg_num_levels": (_I32, [_P]),
    "amgdg_level_info_get": (_I32, [_P, _I32, ctypes.POINTER(amgdg_level_info)]),
    "amgdg_export_level": (_I32, [_P, _I32, _I32, _P, _I64, _P]),
    "amgdg_solve": (_I32, [_P, _I32, _P, _P, _I32, _I32, _D, _I32, _I32, _I32,
                           ctypes.POINTER(amgdg_solve_stats), _P]),
    "amgdg_vcycle": (_I32, [_P, _I32, _P, _P, _I32, _I32, _P]),
    "amgdg_vcycle_static": (_I32, [_P, _I32, _P, _P, _I32, _I32, _P]),
    "amgdg_apply": (_I32, [_P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _P]),
    "amgdg_batch_bytes": (_I32, [_P, _I32, _I32, ctypes.POINTER(_I64)]),
    "amgdg_server_create": (_I32, [ctypes.POINTER(_P), _I32, _I64]),
    "amgdg_server_submit": (_I32, [_P, _P, _P, _P, _I32, _I32, _D, _I32, _I32, _I32, _I64]),
    "amgdg_server_step": (_I32, [_P, _I32, ctypes.POINTER(_I64)]),
    "amgdg_server_poll": (_I32, [_P, _I32, _P, _P, _P, _P, _P, ctypes.POINTER(_I32)]),
    "amgdg_server_destroy": (_I32, [_P]),
    "amgdg_autotune": (_I32, [_P, _I32, _I32, _P]),
    "amgdg_tuning_get": (_I32, [_P, _I32, _I32, _P]),
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2504_13373_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def amgdg_last_error():
    return lib().amgdg_last_error().decode()


def _check(rc):
    if rc < 0:
        raise AmgdgError(rc, amgdg_last_error())
    return rc


def _ptr(a):
    """Host numpy array -> c_void_p (C-contiguous required)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    """Device tensor -> c_void_p."""
    if t is None:
        return None
    assert t.is_contiguous(), "tensor must be contiguous"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return None


# ------------------------------------------------------------------ host-only entry points

def amgdg_default_params(**overrides):
    p = amgdg_params()
    lib().amgdg_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def amgdg_partition_rcb(centroids, n_levels, bisections):
    """Returns (agg (n_levels-1, n_elem) int32, leaf_order (n_elem,) int64)."""
    c = np.ascontiguousarray(centroids, dtype=np.float64)
    n, dim = c.shape
    agg = np.zeros((max(n_levels - 1, 1), n), dtype=np.int32)
    leaf = np.zeros(n, dtype=np.int64)
    _check(lib().amgdg_partition_rcb(n, dim, _ptr(c), n_levels, bisections, _ptr(agg), _ptr(leaf)))
    return agg[: n_levels - 1], leaf


class Plan:
    """Symbolic plan (host only): amgdg_plan_create / _size / _export / _destroy."""

    h = None

    def __init__(self, n_elem, row_ptr, col_idx, n_levels, agg_of_elem):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        ag = np.ascontiguousarray(agg_of_elem, dtype=np.int32) if n_levels > 1 else None
        h = ctypes.c_void_p()
        _check(lib().amgdg_plan_create(ctypes.byref(h), n_elem, _ptr(rp), _ptr(ci), len(ci), n_levels, _ptr(ag)))
        self.h = h

    def export(self, k, what):
        cnt = ctypes.c_int64()
        _check(lib().amgdg_plan_size(self.h, k, what, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.int64 if what == AMGDG_PERM else np.int32)
        _check(lib().amgdg_plan_export(self.h, k, what, _ptr(out), out.nbytes))
        return out

    def close(self):
        if self.h:
            lib().amgdg_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module's globals may already be gone; the
        # process's memory is released with it
        if not _finalizing():
            self.close()


def amgdg_plan_create(n_elem, row_ptr, col_idx, n_levels, agg_of_elem):
    return Plan(n_elem, row_ptr, col_idx, n_levels, agg_of_elem)


# ------------------------------------------------------------------ GPU entry points

class Handle:
    """An amgdg_handle: the multigrid hierarchy resident on the GPU."""

    h = None

    def __init__(self, h):
        self.h = h

    def level_info(self, k):
        return amgdg_level_info_get(self, k)

    @property
    def n_levels(self):
        return lib().amgdg_num_levels(self.h)

    def close(self):
        if self.h:
            lib().amgdg_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if not _finalizing():
            self.close()


def amgdg_setup(n_elem, nb, row_ptr, col_idx, vals, agg_of_elem, params, B1=None, adj_ptr=None, adj_idx=None,
                stream=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    ag = np.ascontiguousarray(agg_of_elem, dtype=np.int32) if params.n_levels > 1 else None
    b1 = None if B1 is None else np.ascontiguousarray(B1, dtype=np.float64)
    ap = None if adj_ptr is None else np.ascontiguousarray(adj_ptr, dtype=np.int32)
    ai = None if adj_idx is None else np.ascontiguousarray(adj_idx, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().amgdg_setup(ctypes.byref(h), n_elem, nb, _ptr(rp), _ptr(ci), _ptr(v), len(ci), _ptr(ap), _ptr(ai),
                             _ptr(ag), ctypes.byref(params), _ptr(b1), _stream(stream)))
    return Handle(h)


def amgdg_destroy(handle):
    handle.close()


def amgdg_level_info_get(handle, k):
    info = amgdg_level_info()
    _check(lib().amgdg_level_info_get(handle.h, k, ctypes.byref(info)))
    return info


def _export_shape(info, what, n_elem):
    nb, s, r = info.nb, info.s, info.r
    return {
        AMGDG_PERM: (n_elem, np.int64),
        AMGDG_A_ROWPTR: (info.n_units + 1, np.int32), AMGDG_A_COLIDX: (info.nnzb, np.int32),
        AMGDG_A_VALS: ((info.nnzb, nb, nb), np.float64),
        AMGDG_T_ROWPTR: (info.n_units + 1, np.int32), AMGDG_T_COLIDX: (info.nnzb_T, np.int32),
        AMGDG_T_VALS: ((info.nnzb_T, nb, s), np.float64),
        AMGDG_R_ROWPTR: (info.n_agg + 1, np.int32), AMGDG_R_COLIDX: (info.nnzb_T, np.int32),
        AMGDG_R_VALS: ((info.nnzb_T, s, nb), np.float64),
        AMGDG_DINV: ((info.n_units, nb, nb), np.float64),
        AMGDG_B_RELAXED: ((info.n, r), np.float64), AMGDG_B_INPUT: ((info.n, r), np.float64),
        AMGDG_PTILDE: ((info.n, s), np.float64), AMGDG_SVALS: ((info.n_agg, r), np.float64),
        AMGDG_UNIT_DOFS: (info.n_units, np.int32),
        AMGDG_M_ROWPTR: (info.n_agg + 1, np.int32), AMGDG_M_COLIDX: (info.nnzb_M, np.int32),
        AMGDG_M_VALS: ((info.nnzb_M, s, nb), np.float64),
    }[what]


def amgdg_export_level(handle, k, what, stream=None):
    info = amgdg_level_info_get(handle, k)
    n_elem = amgdg_level_info_get(handle, 0).n_units
    shape, dt = _export_shape(info, what, n_elem)
    out = np.zeros(shape, dtype=dt)
    _check(lib().amgdg_export_level(handle.h, k, what, _ptr(out), out.nbytes, _stream(stream)))
    return out


def amgdg_solve(handle, b, x, method=AMGDG_PCG, precision=AMGDG_FP64, rtol=1e-8, max_it=10000, restart=30,
                flags=0, stream=None):
    """b, x: device float64 tensors of shape (n,) or (n, m).  Returns (status, stats)."""
    m = 1 if b.dim() == 1 else b.shape[1]
    st = amgdg_solve_stats()
    rc = _check(lib().amgdg_solve(handle.h, m, _dptr(b), _dptr(x), method, precision, rtol, max_it, restart,
                                  flags, ctypes.byref(st), _stream(stream)))
    return rc, st


def amgdg_vcycle(handle, r, z, precision=AMGDG_FP64, flags=0, stream=None):
    m = 1 if r.dim() == 1 else r.shape[1]
    _check(lib().amgdg_vcycle(handle.h, m, _dptr(r), _dptr(z), precision, flags, _stream(stream)))


def amgdg_vcycle_static(handle, r, z, precision=AMGDG_FP64, flags=0, stream=None):
    m = 1 if r.dim() == 1 else r.shape[1]
    _check(lib().amgdg_vcycle_static(handle.h, m, _dptr(r), _dptr(z), precision, flags, _stream(stream)))


def amgdg_apply(handle, k, op, x, b, y, precision=AMGDG_FP64, flags=0, stream=None):
    m = 1 if y.dim() == 1 else y.shape[1]
    _check(lib().amgdg_apply(handle.h, k, op, m, precision, _dptr(x), _dptr(b), _dptr(y), flags, _stream(stream)))


def amgdg_autotune(handle, m=1, flags=0, stream=None):
    _check(lib().amgdg_autotune(handle.h, m, flags, _stream(stream)))


def amgdg_tuning_get(handle, k, m=1):
    """dict of the launch shapes in use on level k for m columns."""
    import numpy as np
    out = np.zeros(16, np.int32)
    _check(lib().amgdg_tuning_get(handle.h, k, m, _ptr(out)))
    names = ("A", "T", "R")
    return {"lanes": dict(zip(names, out[0:3].tolist())), "cols64": dict(zip(names, out[3:6].tolist())),
            "cols32": dict(zip(names, out[6:9].tolist())), "mfma64": dict(zip(names, out[9:12].tolist())),
            "mfma32": dict(zip(names, out[12:15].tolist())), "lanes_tuned": bool(out[15])}


def amgdg_batch_bytes(handle, width, restart=0):
    out = _I64(0)
    _check(lib().amgdg_batch_bytes(handle.h, width, restart, ctypes.byref(out)))
    return out.value


class Server:
    """Continuous-batching solve server (``amgdg_server_*``).  Submitted tensors
    must stay alive until their tag is reported by :meth:`poll`."""

    def __init__(self, width, hbm_budget_bytes):
        h = _P()
        _check(lib().amgdg_server_create(ctypes.byref(h), width, int(hbm_budget_bytes)))
        self.h = h
        self._keep = {}

    def submit(self, handle, b, x, method=AMGDG_PCG, precision=AMGDG_FP64, rtol=1e-8, max_it=10000, restart=30,
               flags=0, tag=0):
        _check(lib().amgdg_server_submit(self.h, handle.h, _dptr(b), _dptr(x), method, precision, rtol, max_it,
                                         restart, flags, int(tag)))
        self._keep[int(tag)] = (b, x)

    def step(self, wait=True):
        n = _I64(0)
        _check(lib().amgdg_server_step(self.h, 1 if wait else 0, ctypes.byref(n)))
        return n.value

    def poll(self, capacity=64):
        """List of (tag, status, iterations, rel_residual, latency_s)."""
        import numpy as np
        tags = np.zeros(capacity, np.int64)
        stat = np.zeros(capacity, np.int32)
        its = np.zeros(capacity, np.int32)
        rel = np.zeros(capacity, np.float64)
        lat = np.zeros(capacity, np.float64)
        n = _I32(0)
        _check(lib().amgdg_server_poll(self.h, capacity, _ptr(tags), _ptr(stat), _ptr(its), _ptr(rel), _ptr(lat),
                                       ctypes.byref(n)))
        out = []
        for i in range(n.value):
            out.append((int(tags[i]), int(stat[i]), int(its[i]), float(rel[i]), float(lat[i])))
            self._keep.pop(int(tags[i]), None)
        return out

    def close(self):
        if self.h:
            _check(lib().amgdg_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hierarchy(centroids, n_levels, bisections, hstar_top=False):
    """Element -> level-k aggregate maps ((n_levels-1, n_elem) int32) from
    amgdg_partition_rcb.  With hstar_top the first coarse level replicates
    level 0 (Algorithm 5's h*-step at the top): its aggregates are the single
    elements, numbered in the partition's depth-first leaf order so that the
    children of every coarser aggregate stay consecutive; the geometric levels
    follow."""
    if not hstar_top:
        return amgdg_partition_rcb(centroids, n_levels, bisections)[0]
    agg, leaf = amgdg_partition_rcb(centroids, n_levels - 1, bisections)
    pos = np.empty(len(leaf), dtype=np.int32)
    pos[leaf] = np.arange(len(leaf), dtype=np.int32)
    return np.ascontiguousarray(np.vstack([pos[None, :], agg]) if n_levels > 2 else pos[None, :])


def setup_from_workload(w, mixed=False, stream=None, **overrides):
    """Convenience: set up a handle for a ``workloads.configs.Workload``."""
    prm = w.params
    p = amgdg_default_params(n_levels=prm.n_levels, r=prm.r, t_pre=prm.t_pre, t_post=prm.t_post,
                             q_power=prm.q_power, relax_max=prm.relax_max, omega_fixed=prm.omega_fixed,
                             gamma=prm.gamma, n_cut=prm.n_cut, mixed=int(mixed), pow_seed=prm.pow_seed,
                             delta=prm.delta, hstar_smooth=int(getattr(prm, "hstar_smooth", False)))
    for k, v in overrides.items():
        setattr(p, k, v)
    agg = hierarchy(w.centroids, prm.n_levels, prm.bisections, getattr(prm, "hstar_top", False))
    adj_ptr, adj_idx = w.adjacency
    return amgdg_setup(w.A.n_brow, w.A.nb, w.A.row_ptr, w.A.col_idx, w.A.vals, agg, p, B1=w.B1,
                       adj_ptr=adj_ptr, adj_idx=adj_idx, stream=stream), agg
