"""Python binding of libmfgmg.so (ctypes): argument marshalling only.

Every call forwards to the C ABI declared in include/mfgmg.h; all arithmetic
of the solver runs in the library's HIP kernels.  Device arrays are torch
tensors on the current HIP device (any object with ``data_ptr()``, ``dtype``
and ``numel()``); host arrays are numpy arrays.  The library must have been
built (``python -m paper_1907_06696_amd.build``); loading fails loudly
otherwise -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmfgmg.so")

FP32, FP64 = 0, 1
GUARD_NONE, GUARD_FP64, GUARD_FP32 = 0, 1, 2
MAX_LEVELS = 14

OK, ERR_INVALID, ERR_STATE, ERR_NOMEM, ERR_HIP, ERR_NOCONV, ERR_MESH = 0, -1, -2, -3, -4, -5, -6

# exported names, in the order of include/mfgmg.h
EXPORTS = [
    "mfgmg_create", "mfgmg_refine", "mfgmg_finalize_mesh", "mfgmg_info", "mfgmg_cells",
    "mfgmg_support_points", "mfgmg_node_types", "mfgmg_constraints", "mfgmg_transfer",
    "mfgmg_leaf_quadrature_points", "mfgmg_set_viscosity", "mfgmg_cell_viscosity",
    "mfgmg_smoother_lambda", "mfgmg_inverse_diagonal", "mfgmg_vmult", "mfgmg_vmult_add", "mfgmg_vcycle",
    "mfgmg_prolongate", "mfgmg_restrict", "mfgmg_smooth", "mfgmg_coarse_solve",
    "mfgmg_assemble_rhs", "mfgmg_apply_div", "mfgmg_apply_grad", "mfgmg_apply_pmass",
    "mfgmg_default_opts", "mfgmg_solve_stokes",
    "mfgmg_local_levels", "mfgmg_local_nodes", "mfgmg_local_transfer", "mfgmg_vcycle_local",
    "mfgmg_features", "mfgmg_fit_objective", "mfgmg_fit_targets", "mfgmg_set_scaling", "mfgmg_use_scaling",
    "mfgmg_vcycle_factor", "mfgmg_mlp_forward", "mfgmg_mlp_backward", "mfgmg_mlp_work_size", "mfgmg_mlp_adam",
    "mfgmg_mlp_train", "mfgmg_apply_mlp", "mfgmg_vmult_uniform_noalloc",
    "mfgmg_last_error", "mfgmg_destroy", "mfgmg_set_boundary", "mfgmg_set_element",
]
N_PARAMS = 6147
MLP_CACHE = 131


BC_DIRICHLET, BC_NOFLUX = 0, 1
BOUNDARY = {"dirichlet": BC_DIRICHLET, "noflux": BC_NOFLUX}


class Info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("unit_exponent", C.c_int32),
                ("n_cells", C.c_int64 * (MAX_LEVELS + 1)), ("n_nodes", C.c_int64 * (MAX_LEVELS + 1)),
                ("n_u", C.c_int64 * (MAX_LEVELS + 1)), ("n_free", C.c_int64 * (MAX_LEVELS + 1)),
                ("n_hanging", C.c_int64 * (MAX_LEVELS + 1)), ("uniform", C.c_int32 * (MAX_LEVELS + 1)),
                ("n_p", C.c_int64), ("n_p_hanging", C.c_int64), ("boundary", C.c_int32), ("element_k", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("vcycle_prec", C.c_int32), ("schur_rtol", C.c_double), ("schur_max_iter", C.c_int32),
                ("use_scaling", C.c_int32), ("verbose", C.c_int32), ("use_graph", C.c_int32),
                ("krylov", C.c_int32), ("idr_s", C.c_int32), ("block", C.c_int32), ("schur", C.c_int32),
                ("schur_degree", C.c_int32), ("hierarchy", C.c_int32), ("idr_fp64_from", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("vcycles", C.c_int32), ("inner_cg_iterations", C.c_int64),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("converged", C.c_int32),
                ("fp64_from", C.c_int32)]


_lib = None


def load():
    """Load libmfgmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1907_06696_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    sig = {
        "mfgmg_create": [i32, C.POINTER(vp)],
        "mfgmg_refine": [vp, vp, i64, i32],
        "mfgmg_finalize_mesh": [vp],
        "mfgmg_set_boundary": [vp, i32],
        "mfgmg_set_element": [vp, i32],
        "mfgmg_info": [vp, C.POINTER(Info)],
        "mfgmg_cells": [vp, i32, vp],
        "mfgmg_support_points": [vp, i32, i32, vp],
        "mfgmg_node_types": [vp, i32, i32, vp],
        "mfgmg_constraints": [vp, i32, i32, C.POINTER(i64), C.POINTER(i64), vp, vp, vp, vp],
        "mfgmg_transfer": [vp, i32, C.POINTER(i64), vp, vp, vp],
        "mfgmg_leaf_quadrature_points": [vp, vp],
        "mfgmg_set_viscosity": [vp, vp, vp],
        "mfgmg_cell_viscosity": [vp, i32, vp],
        "mfgmg_smoother_lambda": [vp, i32, C.POINTER(C.c_double)],
        "mfgmg_inverse_diagonal": [vp, i32, i32, vp, vp],
        "mfgmg_vmult": [vp, i32, i32, vp, vp, vp],
        "mfgmg_vmult_add": [vp, i32, i32, vp, vp, vp],
        "mfgmg_vcycle": [vp, i32, vp, vp, vp],
        "mfgmg_prolongate": [vp, i32, i32, vp, vp, vp],
        "mfgmg_restrict": [vp, i32, i32, vp, vp, vp],
        "mfgmg_smooth": [vp, i32, i32, vp, vp, i32, vp],
        "mfgmg_coarse_solve": [vp, i32, vp, vp, vp],
        "mfgmg_assemble_rhs": [vp, vp, vp, vp],
        "mfgmg_apply_div": [vp, vp, vp, vp],
        "mfgmg_apply_grad": [vp, vp, vp, vp],
        "mfgmg_apply_pmass": [vp, vp, vp, vp],
        "mfgmg_default_opts": [C.POINTER(SolveOpts)],
        "mfgmg_solve_stokes": [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp],
        "mfgmg_local_levels": [vp, C.POINTER(i32), vp, vp],
        "mfgmg_local_nodes": [vp, i32, vp, vp],
        "mfgmg_local_transfer": [vp, i32, C.POINTER(i64), vp, vp, vp],
        "mfgmg_vcycle_local": [vp, i32, vp, vp, vp],
        "mfgmg_features": [vp, i32, vp, vp],
        "mfgmg_fit_objective": [vp, i32, vp, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), vp, vp],
        "mfgmg_fit_targets": [vp, i32, i32, C.c_double, vp, vp, vp],
        "mfgmg_set_scaling": [vp, i32, vp, vp],
        "mfgmg_use_scaling": [vp, i32],
        "mfgmg_vcycle_factor": [vp, C.POINTER(C.c_double), vp],
        "mfgmg_mlp_forward": [vp, vp, i64, vp, vp, vp],
        "mfgmg_mlp_backward": [vp, vp, vp, vp, i64, vp, vp, vp],
        "mfgmg_mlp_work_size": [i64],
        "mfgmg_mlp_adam": [vp, vp, vp, vp, i64, C.c_double, vp],
        "mfgmg_mlp_train": [vp, vp, vp, i64, i32, i32, C.c_double, C.c_uint64, vp, vp],
        "mfgmg_apply_mlp": [vp, vp, i32, C.POINTER(i32), vp, vp],
        "mfgmg_vmult_uniform_noalloc": [i32, i32, vp, vp, vp, vp],
        "mfgmg_last_error": [vp],
        "mfgmg_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.mfgmg_last_error.restype = C.c_char_p
    lib.mfgmg_destroy.restype = None
    lib.mfgmg_mlp_work_size.restype = C.c_int64
    _lib = lib
    return lib


class MFGMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mfgmg error {code}: {msg}")
        self.code = code


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data)


_DTYPE_NAME = {FP32: "float32", FP64: "float64"}


def _current_device():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_device()
    except ImportError:
        pass
    return None


def _prec_of(t):
    name = str(t.dtype)
    if name.endswith("float64"):
        return FP64
    if name.endswith("float32"):
        return FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev_ptr(t, n, prec, what):
    """Device pointer of tensor `t` after checking everything the C ABI cannot
    check itself: a GPU tensor on the current device, contiguous, of the
    precision `prec` (FP32 / FP64), with exactly `n` entries.  Raises
    ValueError (TypeError for a foreign dtype) before any library call."""
    if t is None:
        raise ValueError(f"{what}: a tensor is required")
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: must be a GPU tensor (got device {getattr(t, 'device', '?')})")
    cur = _current_device()
    idx = getattr(getattr(t, "device", None), "index", None)
    if cur is not None and idx is not None and idx != cur:
        raise ValueError(f"{what}: tensor is on device {idx}, the current device is {cur}")
    if _prec_of(t) != prec:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {_DTYPE_NAME[prec]}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if int(t.numel()) != int(n):
        raise ValueError(f"{what}: {int(t.numel())} entries, expected {int(n)}")
    return C.c_void_p(int(t.data_ptr()))


def _host_f64(a, n, what):
    """Contiguous FP64 host copy of `a` with exactly `n` entries."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{what}: {a.size} values, expected {n}")
    return a


def current_stream():
    """hipStream_t of torch's current stream (0 if torch is unavailable)."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(0)


class Solver:
    """Owns one mfgmg context (mesh, level hierarchy, device data)."""

    def __init__(self, base_level):
        self.lib = load()
        h = C.c_void_p()
        self._check(self.lib.mfgmg_create(int(base_level), C.byref(h)), None)
        self.h = h
        self._info = None

    def _check(self, code, h="self"):
        if code != OK:
            hh = self.h if h == "self" else None
            msg = self.lib.mfgmg_last_error(hh)
            raise MFGMGError(code, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.mfgmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- mesh
    def set_boundary(self, bc):
        """Velocity boundary condition before finalize_mesh: "dirichlet"
        (u = 0, the default) or "noflux" (u . n = 0)."""
        if bc not in BOUNDARY:
            raise ValueError(f"unknown boundary condition {bc!r} (expected one of {sorted(BOUNDARY)})")
        self._check(self.lib.mfgmg_set_boundary(self.h, BOUNDARY[bc]))

    def set_element(self, k):
        """Taylor-Hood pair before finalize_mesh: k = 1 (Q2-Q1, the default)
        or k = 2 (Q3-Q2; uniform meshes with u = 0)."""
        self._check(self.lib.mfgmg_set_element(self.h, int(k)))

    def refine(self, cells, levels_up):
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 4)
        self._check(self.lib.mfgmg_refine(self.h, _np_ptr(cells), len(cells), int(levels_up)))

    def finalize_mesh(self):
        self._check(self.lib.mfgmg_finalize_mesh(self.h))
        self._info = None

    def info(self):
        if self._info is None:
            inf = Info()
            self._check(self.lib.mfgmg_info(self.h, C.byref(inf)))
            L = inf.n_levels
            self._info = {
                "L": L, "U": inf.unit_exponent,
                "n_cells": [int(inf.n_cells[l]) for l in range(L + 1)],
                "n_nodes": [int(inf.n_nodes[l]) for l in range(L + 1)],
                "n_u": [int(inf.n_u[l]) for l in range(L + 1)],
                "n_free": [int(inf.n_free[l]) for l in range(L + 1)],
                "n_hanging": [int(inf.n_hanging[l]) for l in range(L + 1)],
                "uniform": [bool(inf.uniform[l]) for l in range(L + 1)],
                "n_p": int(inf.n_p), "n_p_hanging": int(inf.n_p_hanging),
                "boundary": "noflux" if inf.boundary == BC_NOFLUX else "dirichlet",
                "element_k": int(inf.element_k),
            }
        return self._info

    def cells(self, level):
        L = self.info()["L"]
        n = self.info()["n_cells"][level] if 1 <= level <= L else 1   # the library rejects bad levels
        out = np.empty((n, 4), dtype=np.int32)
        self._check(self.lib.mfgmg_cells(self.h, level, _np_ptr(out)))
        return out

    def support_points(self, level, field=0):
        n = self.info()["n_nodes"][level] if field == 0 else self.info()["n_p"]
        out = np.empty(n, dtype=np.int64)
        self._check(self.lib.mfgmg_support_points(self.h, level, field, _np_ptr(out)))
        return out

    def node_types(self, level, field=0):
        """field 0: Q2 node kinds (0 free, 1 Dirichlet, 2 hanging); 1: leaf Q1
        node kinds; 2: per Q2 node, the constrained velocity components as
        bits (bit c: dof 3 node + c)."""
        n = self.info()["n_nodes"][level] if field in (0, 2) else self.info()["n_p"]
        out = np.empty(n, dtype=np.uint8)
        self._check(self.lib.mfgmg_node_types(self.h, level, field, _np_ptr(out)))
        return out

    def constraints(self, level, field=0):
        nh, nnz = C.c_int64(), C.c_int64()
        self._check(self.lib.mfgmg_constraints(self.h, level, field, C.byref(nh), C.byref(nnz),
                                               None, None, None, None))
        node = np.empty(nh.value, np.int64)
        ptr = np.empty(nh.value + 1, np.int64)
        master = np.empty(nnz.value, np.int64)
        w = np.empty(nnz.value, np.float64)
        self._check(self.lib.mfgmg_constraints(self.h, level, field, C.byref(nh), C.byref(nnz), _np_ptr(node),
                                               _np_ptr(ptr), _np_ptr(master), _np_ptr(w)))
        return node, ptr, master, w

    def transfer(self, level):
        nnz = C.c_int64()
        self._check(self.lib.mfgmg_transfer(self.h, level, C.byref(nnz), None, None, None))
        ptr = np.empty(self.info()["n_nodes"][level] + 1, np.int64)
        col = np.empty(nnz.value, np.int64)
        w = np.empty(nnz.value, np.float64)
        self._check(self.lib.mfgmg_transfer(self.h, level, C.byref(nnz), _np_ptr(ptr), _np_ptr(col), _np_ptr(w)))
        return ptr, col, w

    def quad_points_per_cell(self):
        """Gauss points per leaf cell: 27 for Q2-Q1, 64 for Q3-Q2."""
        return 64 if self.info()["element_k"] == 2 else 27

    def leaf_quadrature_points(self):
        L = self.info()["L"]
        out = np.empty((self.info()["n_cells"][L], self.quad_points_per_cell(), 3), dtype=np.float64)
        self._check(self.lib.mfgmg_leaf_quadrature_points(self.h, _np_ptr(out)))
        return out

    # ------------------------------------------------------------- device
    def set_viscosity(self, mu_qp, stream=None):
        mu_qp = np.ascontiguousarray(mu_qp, dtype=np.float64)
        L = self.info()["L"]
        nq = self.quad_points_per_cell()
        if mu_qp.size != nq * self.info()["n_cells"][L]:
            raise ValueError(f"mu_qp must have {nq} values per leaf cell")
        self._check(self.lib.mfgmg_set_viscosity(self.h, _np_ptr(mu_qp), stream or current_stream()))

    def cell_viscosity(self, level):
        out = np.empty(self.info()["n_cells"][level], np.float64)
        self._check(self.lib.mfgmg_cell_viscosity(self.h, level, _np_ptr(out)))
        return out

    def smoother_lambda(self, level):
        v = C.c_double()
        self._check(self.lib.mfgmg_smoother_lambda(self.h, level, C.byref(v)))
        return v.value

    def _level(self, level, lo=1):
        L = self.info()["L"]
        if not lo <= int(level) <= L:
            raise ValueError(f"level {level} outside {lo}..{L}")
        return int(level)

    def _nu(self, level):
        return self.info()["n_u"][level]

    def inverse_diagonal(self, level, dst, stream=None):
        level = self._level(level)
        p = _prec_of(dst)
        self._check(self.lib.mfgmg_inverse_diagonal(self.h, level, p, _dev_ptr(dst, self._nu(level), p, "dst"),
                                                    stream or current_stream()))

    def vmult(self, level, src, dst, stream=None):
        level = self._level(level)
        p, n = _prec_of(src), self._nu(level)
        self._check(self.lib.mfgmg_vmult(self.h, level, p, _dev_ptr(src, n, p, "vmult src"),
                                         _dev_ptr(dst, n, p, "vmult dst"), stream or current_stream()))

    def vmult_add(self, level, src, dst, stream=None):
        level = self._level(level)
        p, n = _prec_of(src), self._nu(level)
        self._check(self.lib.mfgmg_vmult_add(self.h, level, p, _dev_ptr(src, n, p, "vmult_add src"),
                                             _dev_ptr(dst, n, p, "vmult_add dst"), stream or current_stream()))

    def vcycle(self, rhs, x, stream=None):
        p, n = _prec_of(rhs), self._nu(self.info()["L"])
        self._check(self.lib.mfgmg_vcycle(self.h, p, _dev_ptr(rhs, n, p, "vcycle rhs"), _dev_ptr(x, n, p, "vcycle x"),
                                          stream or current_stream()))

    def prolongate(self, level, coarse, fine, stream=None):
        level = self._level(level, 2)
        p = _prec_of(coarse)
        self._check(self.lib.mfgmg_prolongate(self.h, level, p, _dev_ptr(coarse, self._nu(level - 1), p, "coarse"),
                                              _dev_ptr(fine, self._nu(level), p, "fine"), stream or current_stream()))

    def restrict(self, level, fine, coarse, stream=None):
        level = self._level(level, 2)
        p = _prec_of(fine)
        self._check(self.lib.mfgmg_restrict(self.h, level, p, _dev_ptr(fine, self._nu(level), p, "fine"),
                                            _dev_ptr(coarse, self._nu(level - 1), p, "coarse"),
                                            stream or current_stream()))

    def smooth(self, level, b, x, x_is_zero=False, stream=None):
        level = self._level(level)
        p, n = _prec_of(b), self._nu(level)
        self._check(self.lib.mfgmg_smooth(self.h, level, p, _dev_ptr(b, n, p, "smooth b"), _dev_ptr(x, n, p, "smooth x"),
                                          int(x_is_zero), stream or current_stream()))

    def coarse_solve(self, b, x, stream=None):
        p, n = _prec_of(b), self._nu(1)
        self._check(self.lib.mfgmg_coarse_solve(self.h, p, _dev_ptr(b, n, p, "coarse b"), _dev_ptr(x, n, p, "coarse x"),
                                                stream or current_stream()))

    def assemble_rhs(self, f_qp, rhs, stream=None):
        L = self.info()["L"]
        f_qp = _host_f64(f_qp, self.quad_points_per_cell() * 3 * self.info()["n_cells"][L], "f_qp")
        self._check(self.lib.mfgmg_assemble_rhs(self.h, _np_ptr(f_qp), _dev_ptr(rhs, self._nu(L), FP64, "rhs"),
                                                stream or current_stream()))

    def apply_div(self, u, p_out, stream=None):
        i = self.info()
        self._check(self.lib.mfgmg_apply_div(self.h, _dev_ptr(u, i["n_u"][i["L"]], FP64, "u"),
                                             _dev_ptr(p_out, i["n_p"], FP64, "p_out"), stream or current_stream()))

    def apply_grad(self, p, u_out, stream=None):
        i = self.info()
        self._check(self.lib.mfgmg_apply_grad(self.h, _dev_ptr(p, i["n_p"], FP64, "p"),
                                              _dev_ptr(u_out, i["n_u"][i["L"]], FP64, "u_out"),
                                              stream or current_stream()))

    def apply_pmass(self, p, p_out, stream=None):
        i = self.info()
        self._check(self.lib.mfgmg_apply_pmass(self.h, _dev_ptr(p, i["n_p"], FP64, "p"),
                                               _dev_ptr(p_out, i["n_p"], FP64, "p_out"), stream or current_stream()))

    def solve_stokes(self, rhs_u, u_out, p_out, rhs_p=None, stream=None, raise_on_noconv=True, **opts):
        o = SolveOpts()
        self.lib.mfgmg_default_opts(C.byref(o))
        names = {"krylov": {"fgmres": 0, "gmres": 1, "idr": 2}, "block": {"triangular": 0, "diagonal": 1},
                 "schur": {"cg": 0, "cheb": 1}, "hierarchy": {"global": 0, "local": 1}}
        fields = {f for f, _ in SolveOpts._fields_}
        for k, v in opts.items():
            if k not in fields:
                raise ValueError(f"unknown solver option {k!r}")
            if k == "vcycle_prec" and isinstance(v, str):
                v = FP32 if v.lower() == "fp32" else FP64
            elif k in names and isinstance(v, str):
                v = names[k][v.lower()]
            setattr(o, k, v)
        i = self.info()
        nu, npp = i["n_u"][i["L"]], i["n_p"]
        args = (_dev_ptr(rhs_u, nu, FP64, "rhs_u"),
                _dev_ptr(rhs_p, npp, FP64, "rhs_p") if rhs_p is not None else None,
                _dev_ptr(u_out, nu, FP64, "u_out"), _dev_ptr(p_out, npp, FP64, "p_out"))
        st = SolveStats()
        code = self.lib.mfgmg_solve_stokes(self.h, *args, C.byref(o), C.byref(st), stream or current_stream())
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_}
        if code != OK and not (code == ERR_NOCONV and not raise_on_noconv):
            self._check(code)
        return stats

    # ---------------------------------------------------- local smoothing
    def local_levels(self):
        """(base, n_cells[l], n_nodes[l]) of the local-smoothing hierarchy."""
        base = C.c_int32()
        nc = np.zeros(MAX_LEVELS + 1, np.int64)
        nn = np.zeros(MAX_LEVELS + 1, np.int64)
        self._check(self.lib.mfgmg_local_levels(self.h, C.byref(base), _np_ptr(nc), _np_ptr(nn)))
        return base.value, nc, nn

    def local_nodes(self, level):
        base, _, nn = self.local_levels()
        if not base < int(level) <= self.info()["L"]:
            raise ValueError(f"local level {level} outside {base + 1}..{self.info()['L']}")
        keys = np.empty(int(nn[level]), np.int64)
        kinds = np.empty(int(nn[level]), np.uint8)
        self._check(self.lib.mfgmg_local_nodes(self.h, int(level), _np_ptr(keys), _np_ptr(kinds)))
        return keys, kinds

    def local_transfer(self, level):
        base, _, nn = self.local_levels()
        if not base < int(level) <= self.info()["L"]:
            raise ValueError(f"local level {level} outside {base + 1}..{self.info()['L']}")
        nnz = C.c_int64()
        self._check(self.lib.mfgmg_local_transfer(self.h, int(level), C.byref(nnz), None, None, None))
        ptr = np.empty(int(nn[level]) + 1, np.int64)
        col = np.empty(nnz.value, np.int64)
        w = np.empty(nnz.value, np.float64)
        self._check(self.lib.mfgmg_local_transfer(self.h, int(level), C.byref(nnz), _np_ptr(ptr), _np_ptr(col),
                                                  _np_ptr(w)))
        return ptr, col, w

    def vcycle_local(self, rhs, x, stream=None):
        p, n = _prec_of(rhs), self._nu(self.info()["L"])
        self._check(self.lib.mfgmg_vcycle_local(self.h, p, _dev_ptr(rhs, n, p, "vcycle rhs"),
                                                _dev_ptr(x, n, p, "vcycle x"), stream or current_stream()))

    # ------------------------------------------------ learned smoother scaling
    def features(self, level, out=None, stream=None):
        import torch
        level = self._level(level)
        n = self.info()["n_cells"][level]
        out = torch.empty((n, 27), dtype=torch.float32, device="cuda") if out is None else out
        self._check(self.lib.mfgmg_features(self.h, level, _dev_ptr(out, 27 * n, FP32, "features out"),
                                            stream or current_stream()))
        return out

    def fit_objective(self, level, y, lam_fixed=0.0, grad=True, stream=None):
        import torch
        level = self._level(level, 2)
        n = 3 * self.info()["n_cells"][level]
        J, lam = C.c_double(), C.c_double()
        yp = _dev_ptr(y, n, FP32, "y")
        g = torch.empty_like(y) if grad else None
        self._check(self.lib.mfgmg_fit_objective(self.h, level, yp, float(lam_fixed), C.byref(J), C.byref(lam),
                                                 _dev_ptr(g, n, FP32, "grad") if grad else None,
                                                 stream or current_stream()))
        return J.value, lam.value, g

    def fit_targets(self, level, steps=30, lr=0.05, stream=None):
        import torch
        level = self._level(level, 2)
        if int(steps) < 0:
            raise ValueError("steps must be >= 0")
        n = self.info()["n_cells"][level]
        y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        hist = np.zeros(int(steps) + 1)
        self._check(self.lib.mfgmg_fit_targets(self.h, level, int(steps), float(lr), _dev_ptr(y, 3 * n, FP32, "y"),
                                               _np_ptr(hist), stream or current_stream()))
        return y, hist

    def set_scaling(self, level, y=None, stream=None):
        level = self._level(level, 2)
        yp = _dev_ptr(y, 3 * self.info()["n_cells"][level], FP32, "y") if y is not None else None
        self._check(self.lib.mfgmg_set_scaling(self.h, level, yp, stream or current_stream()))

    def use_scaling(self, on):
        self._check(self.lib.mfgmg_use_scaling(self.h, int(bool(on))))

    def vcycle_factor(self, stream=None):
        r = C.c_double()
        self._check(self.lib.mfgmg_vcycle_factor(self.h, C.byref(r), stream or current_stream()))
        return r.value

    def apply_mlp(self, w, guard="fp32", stream=None):
        """Install the network's scalings; guard None/False, "fp64" or "fp32"
        (the V-cycle precision of the solve they are for; True means "fp64")."""
        g = {None: GUARD_NONE, False: GUARD_NONE, True: GUARD_FP64, "fp64": GUARD_FP64, "fp32": GUARD_FP32}
        if guard not in g:
            raise ValueError(f"guard must be one of {list(g)}")
        used = C.c_int32()
        fac = np.zeros(2)
        self._check(self.lib.mfgmg_apply_mlp(self.h, _dev_ptr(w, N_PARAMS, FP32, "weights"), g[guard],
                                             C.byref(used), _np_ptr(fac), stream or current_stream()))
        return bool(used.value), fac


def _lib_check(code):
    if code != OK:
        raise MFGMGError(code, "")


def _rows(x, width, what):
    """Number of samples of an [n, width] FP32 tensor (checked by _dev_ptr)."""
    shape = tuple(getattr(x, "shape", ()))
    if len(shape) != 2 or shape[1] != width:
        raise ValueError(f"{what}: shape {shape}, expected [n, {width}]")
    return int(shape[0])


def mlp_forward(w, x, stream=None):
    """y [n,3], cache [n,131] for FP32 device tensors w [6147], x [n,27]."""
    import torch
    lib = load()
    n = _rows(x, 27, "x")
    args = (_dev_ptr(w, N_PARAMS, FP32, "weights"), _dev_ptr(x, 27 * n, FP32, "x"))
    y = torch.empty((n, 3), dtype=torch.float32, device=x.device)
    cache = torch.empty((n, MLP_CACHE), dtype=torch.float32, device=x.device)
    _lib_check(lib.mfgmg_mlp_forward(*args, n, _dev_ptr(y, 3 * n, FP32, "y"),
                                     _dev_ptr(cache, MLP_CACHE * n, FP32, "cache"), stream or current_stream()))
    return y, cache


def mlp_backward(w, x, cache, dy, stream=None):
    import torch
    lib = load()
    n = _rows(x, 27, "x")
    args = (_dev_ptr(w, N_PARAMS, FP32, "weights"), _dev_ptr(x, 27 * n, FP32, "x"),
            _dev_ptr(cache, MLP_CACHE * n, FP32, "cache"), _dev_ptr(dy, 3 * n, FP32, "dy"))
    dw = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
    nwork = int(lib.mfgmg_mlp_work_size(n))
    work = torch.empty(nwork, dtype=torch.float32, device=x.device)
    _lib_check(lib.mfgmg_mlp_backward(*args, n, _dev_ptr(dw, N_PARAMS, FP32, "dw"), _dev_ptr(work, nwork, FP32, "work"),
                                      stream or current_stream()))
    return dw


def mlp_adam(w, dw, m, v, step, lr, stream=None):
    if int(step) < 1:
        raise ValueError("Adam step counts from 1")
    _lib_check(load().mfgmg_mlp_adam(_dev_ptr(w, N_PARAMS, FP32, "weights"), _dev_ptr(dw, N_PARAMS, FP32, "dw"),
                                     _dev_ptr(m, N_PARAMS, FP32, "m"), _dev_ptr(v, N_PARAMS, FP32, "v"), int(step),
                                     float(lr), stream or current_stream()))


def mlp_train(w, feats, targets, epochs=20, batch=4096, lr=1e-3, seed=0, stream=None):
    """Train in place; returns the per-epoch mean squared error."""
    n = _rows(feats, 27, "feats")
    args = (_dev_ptr(w, N_PARAMS, FP32, "weights"), _dev_ptr(feats, 27 * n, FP32, "feats"),
            _dev_ptr(targets, 3 * n, FP32, "targets"))
    hist = np.zeros(max(int(epochs), 1))
    _lib_check(load().mfgmg_mlp_train(*args, n, int(epochs), int(batch), float(lr), int(seed), _np_ptr(hist),
                                      stream or current_stream()))
    return hist[:epochs]


def vmult_uniform_noalloc(n_edge, mu, src, dst, stream=None):
    """dst = A src on the uniform n_edge^3 mesh (32 or 64) with cell viscosity
    mu [n^3], without a context and without any allocation in the library
    (its static work array is shared by every call on a GPU)."""
    n = int(n_edge)
    if n not in (32, 64):
        raise ValueError("n_edge must be 32 or 64")
    p = _prec_of(src)
    nu = 3 * (2 * n + 1) ** 3
    args = (_dev_ptr(mu, n ** 3, p, "mu"), _dev_ptr(src, nu, p, "src"), _dev_ptr(dst, nu, p, "dst"))
    lib = load()
    code = lib.mfgmg_vmult_uniform_noalloc(n, p, *args, stream or current_stream())
    if code != OK:
        msg = lib.mfgmg_last_error(None)
        raise MFGMGError(code, msg.decode() if msg else "")
