"""ctypes binding of ``include/rav.h`` (argument marshalling only).

Every numerical step runs inside ``librav.so``; this module only converts
torch tensors to device pointers, passes the current HIP stream and turns
negative status codes into :class:`RavError`.  Importing it fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librav.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rav.h")

RAV_OK, RAV_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "RAV_OK", 1: "RAV_NOT_CONVERGED", -1: "RAV_EINVAL", -2: "RAV_ENOMEM",
                -3: "RAV_ESINGULAR", -4: "RAV_EDIVERGED", -5: "RAV_EDEVICE", -6: "RAV_EUNSUPPORTED"}
SMOOTHERS = {"rav": 0, "av": 1, "mv": 2}
KINDS = {"vertex": 0, "element": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
FORMATS = {"rows": 0, "factored": 1}
DISCRETIZATIONS = {"taylor-hood": 0, "q1q1": 1, "q1q1-adaptive": 2}


class RavError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class RavInclusion(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double), ("r", ctypes.c_double)]


class RavProblemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("bc_dirichlet_mask", ctypes.c_uint), ("eta_out", ctypes.c_double), ("eta_in", ctypes.c_double),
                ("n_incl", ctypes.c_int), ("incl", ctypes.POINTER(RavInclusion)), ("patch", ctypes.c_int),
                ("smoother", ctypes.c_int), ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("inv_precision", ctypes.c_int), ("coarse_galerkin", ctypes.c_int),
                ("inv_format", ctypes.c_int), ("discretization", ctypes.c_int), ("beta", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_L = ctypes.c_long
_D = ctypes.c_double
_S = ctypes.c_int   # rav_status
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

SIGNATURES = {
    "rav_create": (_S, [ctypes.POINTER(RavProblemDesc), _P, ctypes.POINTER(_P)]),
    "rav_factor_patches": (_S, [_P]),
    "rav_dofs": (_S, [_P, _I, ctypes.POINTER(_L), ctypes.POINTER(_L)]),
    "rav_n_levels": (_S, [_P, ctypes.POINTER(_I)]),
    "rav_n_patches": (_S, [_P, _I, ctypes.POINTER(_L)]),
    "rav_assemble_rhs": (_S, [_P, ctypes.POINTER(_D), _I, _P]),
    "rav_residual": (_S, [_P, _I, _P, _P, _P, ctypes.POINTER(_D)]),
    "rav_assemble_rhs_lid": (_S, [_P, _D, _P]),
    "rav_smooth": (_S, [_P, _I, _I, _P, _P]),
    "rav_restrict": (_S, [_P, _I, _P, _P]),
    "rav_prolong_add": (_S, [_P, _I, _P, _P]),
    "rav_coarse_solve": (_S, [_P, _P, _P]),
    "rav_vcycle": (_S, [_P, _P, _P]),
    "rav_solve": (_S, [_P, _P, _P, _D, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "rav_set_params": (_S, [_P, _D, _I, _I]),
    "rav_solve_gmres": (_S, [_P, _P, _P, _D, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "rav_solve_gmres_noalloc": (_S, [_P, _P, _P, _D, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)]),
    "rav_set_patch_omega": (_S, [_P, _I, _P]),
    "rav_get_patch_map": (_S, [_P, _I, _L, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "rav_get_owner": (_S, [_P, _I, _P]),
    "rav_map_patch": (_S, [ctypes.POINTER(RavProblemDesc), _I, _L, ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_I)]),
    "rav_map_owner": (_S, [ctypes.POINTER(RavProblemDesc), _I, ctypes.POINTER(_I)]),
    "rav_get_patch_inverse": (_S, [_P, _I, _L, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "rav_export_matrix": (_S, [_P, _I, ctypes.POINTER(_D)]),
    "rav_time_sweep": (_S, [_P, _I, _I, _P, _P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "rav_stream_copy": (_S, [_P, _P, _P, _L]),
    "rav_profile_begin": (_S, [_P, _I, _I]),
    "rav_profile_end": (_S, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(_I)]),
    "rav_destroy": (_S, [_P]),
    "rav_set_fallback": (_S, [_P, _D, ctypes.POINTER(_I)]),
    "rav_mlp_create": (_S, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_P)]),
    "rav_mlp_get": (_S, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_D)]),
    "rav_mlp_destroy": (_S, [_P]),
    "rav_learn_patch_omega": (_S, [_P, _P, _I, _P]),
    "rav_learn_set_omega": (_S, [_P, _P]),
    "rav_learn_twogrid": (_S, [_P, _P, _P, _I, ctypes.POINTER(_D), _P, ctypes.POINTER(_D)]),
    "rav_learn_step": (_S, [_P, _P, _P, _I, _D, ctypes.POINTER(_D)]),
    "rav_batch_create": (_S, [ctypes.POINTER(RavProblemDesc), _I, _P, ctypes.POINTER(_P)]),
    "rav_batch_factor": (_S, [_P]),
    "rav_batch_size": (_S, [_P, ctypes.POINTER(_I)]),
    "rav_batch_dofs": (_S, [_P, _I, ctypes.POINTER(_L), ctypes.POINTER(_L)]),
    "rav_batch_assemble_rhs": (_S, [_P, _I, ctypes.POINTER(_D), _I, _P]),
    "rav_batch_vcycle": (_S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "rav_batch_solve": (_S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _I, ctypes.POINTER(_I),
                             ctypes.POINTER(_D)]),
    "rav_batch_solve_gmres": (_S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _I, _I, ctypes.POINTER(_I),
                                   ctypes.POINTER(_D)]),
    "rav_create_batch": (_S, [ctypes.POINTER(RavProblemDesc), _I, _P, ctypes.POINTER(_P)]),
    "rav_solve_batch": (_S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, _I, ctypes.POINTER(_I),
                             ctypes.POINTER(_D)]),
    "rav_batch_destroy": (_S, [_P]),
    "rav_batch_last_error": (ctypes.c_char_p, [_P]),
    "rav_last_error": (ctypes.c_char_p, [_P]),
    "rav_set_device_allocator": (_S, [_ALLOC_FN, _RELEASE_FN, _P]),
    "rav_create_adaptive": (_S, [ctypes.POINTER(RavProblemDesc), ctypes.POINTER(_I), ctypes.POINTER(_L), _L, _L,
                                 _P, ctypes.POINTER(_P)]),
    "rav_assemble_rhs_dirichlet": (_S, [_P, _P, _P]),
    "rav_adaptive_level_info": (_S, [_P, _I, ctypes.POINTER(_L)]),
    "rav_adaptive_host_export": (_S, [ctypes.POINTER(RavProblemDesc), ctypes.POINTER(_I), ctypes.POINTER(_L), _L, _L,
                                      _I, _I, ctypes.POINTER(_D), ctypes.POINTER(_L), ctypes.POINTER(_L)]),
}


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/rav.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:rav_status|const char\*)\s+(rav_\w+)\s*\(", text, re.M)))


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    try:   # torch's HIP runtime first: the library then uses the runtime torch's streams belong to
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def _ptr(t) -> int:
    """Device pointer of a contiguous torch tensor (or a raw integer address)."""
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Hierarchy:
    """A RAV multigrid hierarchy (one ``rav_ctx``)."""

    def __init__(self, dim=2, n_cells=32, n_levels=3, dmask=0b1111, kind="vertex", smoother="rav",
                 omega=0.66, nu_pre=2, nu_post=2, precision="fp64", eta_out=1.0, eta_in=1.0,
                 inclusions=None, stream=None, galerkin=False, inv_format="rows", discretization="taylor-hood",
                 beta=0.1):
        self.lib = lib()
        incl = np.zeros((0, 4)) if inclusions is None else np.asarray(inclusions, dtype=np.float64)
        if incl.size and incl.shape[1] == dim + 1:   # (cx, cy[, cz], r) -> (cx, cy, cz, r)
            full = np.zeros((len(incl), 4))
            full[:, :dim] = incl[:, :dim]
            full[:, 3] = incl[:, dim]
            incl = full
        self._incl = (RavInclusion * max(len(incl), 1))()
        for i, row in enumerate(incl):
            self._incl[i] = RavInclusion(*row)
        self.desc = RavProblemDesc(dim, n_cells, n_levels, dmask, eta_out, eta_in, len(incl),
                                   ctypes.cast(self._incl, ctypes.POINTER(RavInclusion)), KINDS[kind],
                                   SMOOTHERS[smoother], omega, nu_pre, nu_post, PRECISIONS[precision],
                                   1 if galerkin else 0, FORMATS[inv_format], DISCRETIZATIONS[discretization],
                                   beta)
        self.stream = _stream() if stream is None else stream
        h = _P()
        st = self.lib.rav_create(ctypes.byref(self.desc), self.stream, ctypes.byref(h))
        if st < 0:
            raise RavError(st, self.lib.rav_last_error(None).decode())
        self.h = h
        self.dim, self.n_levels = dim, n_levels

    def _chk(self, st):
        if st < 0:
            raise RavError(st, self.lib.rav_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.rav_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self):
        return self._chk(self.lib.rav_factor_patches(self.h))

    def dofs(self, level):
        nt, nf = _L(), _L()
        self._chk(self.lib.rav_dofs(self.h, level, ctypes.byref(nt), ctypes.byref(nf)))
        return nt.value, nf.value

    def n_patches(self, level):
        n = _L()
        self._chk(self.lib.rav_n_patches(self.h, level, ctypes.byref(n)))
        return n.value

    def assemble_rhs(self, params, b):
        p = np.ascontiguousarray(params, dtype=np.float64)
        return self._chk(self.lib.rav_assemble_rhs(self.h, p.ctypes.data_as(ctypes.POINTER(_D)), len(p), _ptr(b)))

    def assemble_rhs_lid(self, b, lid_u=1.0):
        return self._chk(self.lib.rav_assemble_rhs_lid(self.h, lid_u, _ptr(b)))

    def residual(self, level, x, b, r, norm=False):
        nv = _D()
        self._chk(self.lib.rav_residual(self.h, level, _ptr(x), _ptr(b), _ptr(r),
                                        ctypes.byref(nv) if norm else None))
        return nv.value if norm else None

    def smooth(self, level, sweeps, x, b):
        return self._chk(self.lib.rav_smooth(self.h, level, sweeps, _ptr(x), _ptr(b)))

    def restrict(self, level, rf, bc):
        return self._chk(self.lib.rav_restrict(self.h, level, _ptr(rf), _ptr(bc)))

    def prolong_add(self, level, xc, xf):
        return self._chk(self.lib.rav_prolong_add(self.h, level, _ptr(xc), _ptr(xf)))

    def coarse_solve(self, b0, x0):
        return self._chk(self.lib.rav_coarse_solve(self.h, _ptr(b0), _ptr(x0)))

    def vcycle(self, x, b):
        return self._chk(self.lib.rav_vcycle(self.h, _ptr(x), _ptr(b)))

    def solve(self, x, b, rtol=1e-8, maxit=200):
        it, rel = _I(), _D()
        st = self.lib.rav_solve(self.h, _ptr(x), _ptr(b), rtol, maxit, ctypes.byref(it), ctypes.byref(rel))
        if st < 0 and st != -4:
            self._chk(st)
        return st, it.value, rel.value

    def solve_gmres(self, x, b, rtol=1e-8, maxit=300, restart=30):
        it, rel = _I(), _D()
        st = self.lib.rav_solve_gmres(self.h, _ptr(x), _ptr(b), rtol, maxit, restart, ctypes.byref(it),
                                      ctypes.byref(rel))
        if st < 0 and st != -4:
            self._chk(st)
        return st, it.value, rel.value

    def solve_gmres_noalloc(self, x, b, rtol=1e-8, maxit=300, restart=30):
        it, rel = _I(), _D()
        st = self.lib.rav_solve_gmres_noalloc(self.h, _ptr(x), _ptr(b), rtol, maxit, restart, ctypes.byref(it),
                                              ctypes.byref(rel))
        if st < 0 and st != -4:
            self._chk(st)
        return st, it.value, rel.value

    def set_params(self, omega, nu_pre, nu_post):
        return self._chk(self.lib.rav_set_params(self.h, omega, nu_pre, nu_post))

    def set_patch_omega(self, level, omega_dev):
        return self._chk(self.lib.rav_set_patch_omega(self.h, level, None if omega_dev is None else _ptr(omega_dev)))

    def patch_map(self, level, patch):
        dofs = (_I * 512)()
        own = (_I * 512)()
        n = _I()
        self._chk(self.lib.rav_get_patch_map(self.h, level, patch, dofs, ctypes.byref(n), own))
        return np.array(dofs[:n.value], dtype=np.int64), np.array(own[:n.value], dtype=bool)

    def owner(self, level):
        import torch
        nt, _ = self.dofs(level)
        out = torch.empty(nt, dtype=torch.int32, device="cuda")
        self._chk(self.lib.rav_get_owner(self.h, level, _ptr(out)))
        return out

    def patch_inverse(self, level, patch):
        buf = (_D * (128 * 128))()
        r, c = _I(), _I()
        self._chk(self.lib.rav_get_patch_inverse(self.h, level, patch, buf, ctypes.byref(r), ctypes.byref(c)))
        return np.ctypeslib.as_array(buf)[: r.value * c.value].reshape(r.value, c.value).copy()

    def export_matrix(self, level):
        nt, _ = self.dofs(level)
        out = np.zeros((nt, nt))
        self._chk(self.lib.rav_export_matrix(self.h, level, out.ctypes.data_as(ctypes.POINTER(_D))))
        return out

    def profile_begin(self, level, max_launches=4096):
        return self._chk(self.lib.rav_profile_begin(self.h, level, max_launches))

    def profile_end(self):
        a, c, n = ctypes.c_float(), ctypes.c_float(), _I()
        self._chk(self.lib.rav_profile_end(self.h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(n)))
        return a.value, c.value, n.value

    def set_fallback(self, rho_max):
        fb = _I()
        self._chk(self.lib.rav_set_fallback(self.h, rho_max, ctypes.byref(fb)))
        return fb.value

    def learn_patch_omega(self, mlp, level, omega_dev):
        return self._chk(self.lib.rav_learn_patch_omega(self.h, mlp.h, level, _ptr(omega_dev)))

    def learn_set_omega(self, mlp):
        return self._chk(self.lib.rav_learn_set_omega(self.h, None if mlp is None else mlp.h))

    def learn_twogrid(self, mlp, x0, nu=2, grad_omega=None, want_theta=True):
        loss = _D()
        gt = (_D * 5313)() if want_theta else None
        self._chk(self.lib.rav_learn_twogrid(self.h, mlp.h, _ptr(x0), nu, ctypes.byref(loss),
                                             None if grad_omega is None else _ptr(grad_omega), gt))
        return loss.value, (np.ctypeslib.as_array(gt).copy() if want_theta else None)

    def learn_step(self, mlp, x0, nu=2, lr=1e-3):
        loss = _D()
        self._chk(self.lib.rav_learn_step(self.h, mlp.h, _ptr(x0), nu, lr, ctypes.byref(loss)))
        return loss.value

    def time_sweep(self, level, reps, x, b):
        a, c = ctypes.c_float(), ctypes.c_float()
        self._chk(self.lib.rav_time_sweep(self.h, level, reps, _ptr(x), _ptr(b), ctypes.byref(a), ctypes.byref(c)))
        return a.value, c.value


def _adaptive_desc(n_grids, smoother, omega, nu_pre, nu_post, beta, eta, dmask=0b1111):
    return make_desc(dim=2, n_cells=0, n_levels=n_grids, dmask=dmask, smoother=smoother, omega=omega,
                     nu_pre=nu_pre, nu_post=nu_post, eta_out=eta, eta_in=eta, discretization="q1q1-adaptive",
                     beta=beta)


def _leaf_arrays(grids):
    leaves = np.ascontiguousarray(np.concatenate([np.asarray(g, dtype=np.int32).reshape(-1, 3) for g in grids]))
    counts = np.array([len(g) for g in grids], dtype=np.int64)
    return leaves, counts


class AdaptiveHierarchy(Hierarchy):
    """Stabilized Q1-Q1 on a hierarchy of adaptively refined quadtree grids
    (``rav_create_adaptive``): ``grids`` lists the leaf arrays (n, 3) of
    (x0, y0, s), coarsest first, in lattice units of the rectangle
    ``lattice`` x ``lattice_y`` (default: the square); ``dmask`` the sides
    with Dirichlet velocity (bit 0: x = 0, 1: x = max, 2: y = 0, 3: y = max)."""

    def __init__(self, grids, lattice, smoother="rav", omega=0.66, nu_pre=2, nu_post=2, beta=0.05, eta=1.0,
                 stream=None, lattice_y=None, dmask=0b1111):
        self.lib = lib()
        self.desc = _adaptive_desc(len(grids), smoother, omega, nu_pre, nu_post, beta, eta, dmask)
        leaves, counts = _leaf_arrays(grids)
        self.stream = _stream() if stream is None else stream
        h = _P()
        ly = lattice if lattice_y is None else lattice_y
        st = self.lib.rav_create_adaptive(ctypes.byref(self.desc), leaves.ctypes.data_as(ctypes.POINTER(_I)),
                                          counts.ctypes.data_as(ctypes.POINTER(_L)), int(lattice), int(ly),
                                          self.stream, ctypes.byref(h))
        if st < 0:
            raise RavError(st, self.lib.rav_last_error(None).decode())
        self.h = h
        self.dim, self.n_levels = 2, len(grids)

    def level_info(self, level):
        """dict: vertices, stored (padded) and true operator and patch entries,
        MV colours, distinct value tuples, patch configurations, entry format."""
        out = (_L * 9)()
        self._chk(self.lib.rav_adaptive_level_info(self.h, level, out))
        keys = ("vertices", "operator_entries_padded", "patch_entries_padded", "mv_colours", "operator_entries",
                "patch_entries", "value_tuples", "patch_configurations", "wide")
        return dict(zip(keys, (int(v) for v in out)))

    def assemble_rhs_dirichlet(self, ud, b):
        """b = -L_all[:, masked] u_D on the finest grid; ud: host float64
        array (2, n_vertices) or flat, u_x then u_y per regular vertex."""
        u = np.ascontiguousarray(np.asarray(ud, dtype=np.float64).reshape(-1))
        n_total, _ = self.dofs(self.n_levels - 1)
        if u.size != 2 * (n_total // 3):
            raise ValueError(f"ud holds {u.size} values; the finest grid needs 2 x {n_total // 3}")
        return self._chk(self.lib.rav_assemble_rhs_dirichlet(self.h, u.ctypes.data_as(_P), _ptr(b)))


def adaptive_host_export(grids, lattice, level, what, beta=0.05, eta=1.0, lattice_y=None, dmask=0b1111):
    """Host-only set-up of one adaptive grid (``rav_adaptive_host_export``):
    what = "operator" | "prolong" | "lid" | "colours" | "vertices"."""
    kinds = {"operator": 0, "prolong": 1, "lid": 2, "colours": 3, "vertices": 4}
    desc = _adaptive_desc(len(grids), "mv" if what == "colours" else "rav", 0.66, 2, 2, beta, eta, dmask)
    leaves, counts = _leaf_arrays(grids)
    rows, cols = _L(), _L()
    ly = lattice if lattice_y is None else lattice_y
    args = (ctypes.byref(desc), leaves.ctypes.data_as(ctypes.POINTER(_I)), counts.ctypes.data_as(ctypes.POINTER(_L)),
            int(lattice), int(ly), level, kinds[what])
    st = lib().rav_adaptive_host_export(*args, None, ctypes.byref(rows), ctypes.byref(cols))
    if st < 0:
        raise RavError(st, lib().rav_last_error(None).decode())
    out = np.zeros((rows.value, cols.value))
    st = lib().rav_adaptive_host_export(*args, out.ctypes.data_as(ctypes.POINTER(_D)), ctypes.byref(rows),
                                        ctypes.byref(cols))
    if st < 0:
        raise RavError(st, lib().rav_last_error(None).decode())
    return out if cols.value > 1 else out[:, 0]


class MLP:
    """Per-patch damping network (``rav_mlp``): 16 -> 64 -> 64 -> 1, FP32."""

    NPARAM = 5313

    def __init__(self, theta):
        self.lib = lib()
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.NPARAM:
            raise ValueError("the network has 5313 parameters")
        h = _P()
        st = self.lib.rav_mlp_create(th.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h))
        if st < 0:
            raise RavError(st, "rav_mlp_create")
        self.h = h

    def theta(self):
        out = np.zeros(self.NPARAM, dtype=np.float32)
        st = self.lib.rav_mlp_get(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), None)
        if st < 0:
            raise RavError(st, "rav_mlp_get")
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.rav_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent problems solved together (one ``rav_batch``).

    ``problems`` is a list of dicts with the keyword arguments of
    :class:`Hierarchy` (dim, n_cells, n_levels, dmask, omega, eta_out, eta_in,
    inclusions, precision, nu_pre, nu_post)."""

    def __init__(self, problems, stream=None):
        self.lib = lib()
        n = len(problems)
        self.descs = (RavProblemDesc * n)()
        self._keep = []
        for i, p in enumerate(problems):
            dim = p.get("dim", 2)
            incl = p.get("inclusions")
            incl = np.zeros((0, 4)) if incl is None else np.asarray(incl, dtype=np.float64)
            if incl.size and incl.shape[1] == dim + 1:
                full = np.zeros((len(incl), 4))
                full[:, :dim] = incl[:, :dim]
                full[:, 3] = incl[:, dim]
                incl = full
            arr = (RavInclusion * max(len(incl), 1))()
            for j, row in enumerate(incl):
                arr[j] = RavInclusion(*row)
            self._keep.append(arr)
            self.descs[i] = RavProblemDesc(dim, p["n_cells"], p["n_levels"], p.get("dmask", 0b1111),
                                           p.get("eta_out", 1.0), p.get("eta_in", 1.0), len(incl),
                                           ctypes.cast(arr, ctypes.POINTER(RavInclusion)),
                                           KINDS[p.get("kind", "vertex")], SMOOTHERS["rav"], p.get("omega", 0.66),
                                           p.get("nu_pre", 2), p.get("nu_post", 2),
                                           PRECISIONS[p.get("precision", "fp64")], 1 if p.get("galerkin") else 0,
                                           FORMATS[p.get("inv_format", "rows")])
        self.n = n
        self.stream = _stream() if stream is None else stream
        h = _P()
        st = self.lib.rav_batch_create(self.descs, n, self.stream, ctypes.byref(h))
        if st < 0:
            raise RavError(st, self.lib.rav_batch_last_error(None).decode())
        self.h = h

    def _chk(self, st):
        if st < 0:
            raise RavError(st, self.lib.rav_batch_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.rav_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self):
        return self._chk(self.lib.rav_batch_factor(self.h))

    def dofs(self, problem):
        nt, nf = _L(), _L()
        self._chk(self.lib.rav_batch_dofs(self.h, problem, ctypes.byref(nt), ctypes.byref(nf)))
        return nt.value, nf.value

    def assemble_rhs(self, problem, params, b):
        p = np.ascontiguousarray(params, dtype=np.float64)
        return self._chk(self.lib.rav_batch_assemble_rhs(self.h, problem, p.ctypes.data_as(ctypes.POINTER(_D)),
                                                         len(p), _ptr(b)))

    @staticmethod
    def _ptrs(ts):
        arr = (_P * len(ts))()
        for i, t in enumerate(ts):
            arr[i] = _ptr(t)
        return arr

    def vcycle(self, xs, bs):
        return self._chk(self.lib.rav_batch_vcycle(self.h, self._ptrs(xs), self._ptrs(bs)))

    def solve(self, xs, bs, rtol=1e-8, maxit=200):
        its = (_I * self.n)()
        rel = (_D * self.n)()
        st = self.lib.rav_batch_solve(self.h, self._ptrs(xs), self._ptrs(bs), rtol, maxit, its, rel)
        if st < 0 and st != -4:
            self._chk(st)
        return st, list(its), list(rel)

    def solve_gmres(self, xs, bs, rtol=1e-8, maxit=300, restart=30):
        its = (_I * self.n)()
        rel = (_D * self.n)()
        st = self.lib.rav_batch_solve_gmres(self.h, self._ptrs(xs), self._ptrs(bs), rtol, maxit, restart, its, rel)
        if st < 0 and st != -4:
            self._chk(st)
        return st, list(its), list(rel)


def make_desc(dim=2, n_cells=32, n_levels=3, dmask=0b1111, kind="vertex", smoother="rav", omega=0.66,
              nu_pre=2, nu_post=2, precision="fp64", eta_out=1.0, eta_in=1.0, galerkin=False, inv_format="rows",
              discretization="taylor-hood", beta=0.1):
    """Descriptor without inclusions (for the host-only map functions)."""
    return RavProblemDesc(dim, n_cells, n_levels, dmask, eta_out, eta_in, 0, None, KINDS[kind],
                          SMOOTHERS[smoother], omega, nu_pre, nu_post, PRECISIONS[precision], 1 if galerkin else 0,
                          FORMATS[inv_format], DISCRETIZATIONS[discretization], beta)


def map_patch(desc, level, patch):
    """Host-only patch map: (global DoFs in local order, owned flags)."""
    dofs = (_I * 512)()
    own = (_I * 512)()
    n = _I()
    st = lib().rav_map_patch(ctypes.byref(desc), level, patch, dofs, ctypes.byref(n), own)
    if st < 0:
        raise RavError(st, "rav_map_patch")
    return np.array(dofs[:n.value], dtype=np.int64), np.array(own[:n.value], dtype=bool)


def map_owner(desc, level, n_total):
    """Host-only owner map (int32, -1 for masked DoFs)."""
    out = np.zeros(n_total, dtype=np.int32)
    st = lib().rav_map_owner(ctypes.byref(desc), level, out.ctypes.data_as(ctypes.POINTER(_I)))
    if st < 0:
        raise RavError(st, "rav_map_owner")
    return out


_allocator = None   # the ctypes callbacks of the installed allocator (kept alive here)


def set_device_allocator(alloc=None, release=None):
    """Device memory of the library's buffers from Python callables:
    alloc(nbytes) -> device address (int), release(address).  No arguments
    restore hipMalloc/hipFree.  Only while no context, batch or network
    exists (``rav_set_device_allocator``)."""
    global _allocator
    fa = _ALLOC_FN() if alloc is None else _ALLOC_FN(lambda n, user: alloc(n) or None)   # None: NULL
    fr = _RELEASE_FN() if release is None else _RELEASE_FN(lambda ptr, user: release(ptr))
    st = lib().rav_set_device_allocator(fa, fr, None)
    if st < 0:
        raise RavError(st, lib().rav_last_error(None).decode())
    _allocator = None if alloc is None else (fa, fr)


def use_torch_allocator():
    """Serve the library's device buffers from PyTorch's caching allocator
    (current device and stream)."""
    import torch
    set_device_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                         lambda p: torch.cuda.caching_allocator_delete(p))


def stream_copy(dst, src, n=None, stream=None):
    st = lib().rav_stream_copy(_stream() if stream is None else stream, _ptr(dst), _ptr(src),
                               dst.numel() if n is None else n)
    if st < 0:
        raise RavError(st, "stream copy failed")
