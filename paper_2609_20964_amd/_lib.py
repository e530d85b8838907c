"""ctypes binding of libwgeo.so: struct layouts, signatures and error mapping.

Argument marshalling only; every step of the reconstruction runs in the HIP
library.  The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwgeo.so")

WG_OK, WG_PENDING = 0, 1
WG_EINVAL, WG_ENOMEM, WG_ENOTCONV, WG_ENUMERIC, WG_EDEVICE, WG_ESTATE = -1, -2, -3, -4, -5, -6
WG_BC_NEUMANN, WG_BC_DIRICHLET = 0, 1
WG_FP32_FP64REDUCE, WG_FP64 = 0, 1
WG_VERTEX_QUADRATURE, WG_EXACT_QUADRATURE = 0, 1
CODE_NAMES = {WG_EINVAL: "WG_EINVAL", WG_ENOMEM: "WG_ENOMEM", WG_ENOTCONV: "WG_ENOTCONV",
              WG_ENUMERIC: "WG_ENUMERIC", WG_EDEVICE: "WG_EDEVICE", WG_ESTATE: "WG_ESTATE"}


class WgGrid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("lo", C.c_double * 3), ("h", C.c_double)]


class WgSolveOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_iters", C.c_int), ("warm_start", C.c_int),
                ("precision", C.c_int), ("deterministic", C.c_int), ("quadrature", C.c_int)]


class WgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("refinements", C.c_int), ("rel_res", C.c_double),
                ("iso_c", C.c_double), ("chi_mean", C.c_double), ("n_tris", C.c_int64),
                ("status", C.c_int), ("ms", C.c_float * 8), ("bytes_resident", C.c_size_t)]

    def as_dict(self):
        return {"iters": self.iters, "refinements": self.refinements, "rel_res": self.rel_res,
                "iso_c": self.iso_c, "chi_mean": self.chi_mean, "n_tris": self.n_tris,
                "status": self.status, "ms": list(self.ms), "bytes_resident": self.bytes_resident}


class WgRequest(C.Structure):
    _fields_ = [("grid", WgGrid), ("d_xyz", C.c_void_p), ("d_nrm", C.c_void_p), ("n_points", C.c_int),
                ("d_q", C.c_void_p), ("n_q", C.c_int), ("d_gphi", C.c_void_p), ("opts", WgSolveOpts),
                ("d_phi", C.c_void_p), ("d_nrm_out", C.c_void_p), ("d_gxyz", C.c_void_p),
                ("d_gnrm_pts", C.c_void_p), ("d_gnrm", C.c_void_p), ("d_gq", C.c_void_p)]


class WgResult(C.Structure):
    _fields_ = [("status", C.c_int), ("stats", WgStats), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


class WgOrientOpts(C.Structure):
    _fields_ = [("gamma_r", C.c_double), ("n_tol", C.c_int), ("refine", C.c_int)]


class WgOrientInfo(C.Structure):
    _fields_ = [("spacing2", C.c_double), ("rd0", C.c_double), ("rd", C.c_double), ("ds", C.c_double),
                ("n_probes", C.c_int), ("n_flipped", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class WgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "wg_last_error": (C.c_char_p, []),
    "wg_recon_footprint": (C.c_size_t, [C.POINTER(WgGrid), C.c_int]),
    "wg_grid_from_bbox": (C.c_int, [C.POINTER(C.c_double * 3), C.POINTER(C.c_double * 3), C.c_double, C.c_int,
                                    C.POINTER(WgGrid)]),
    "wg_grid_from_cloud": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_int, C.POINTER(WgGrid), C.c_void_p]),
    "wg_recon_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(WgGrid), C.c_int, C.c_void_p]),
    "wg_recon_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(WgSolveOpts),
                                   C.POINTER(WgStats)]),
    "wg_sample_sdf_normals": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "wg_recon_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                C.c_void_p, C.POINTER(WgSolveOpts), C.POINTER(WgStats)]),
    "wg_recon_wait": (C.c_int, [C.c_void_p]),
    "wg_recon_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.POINTER(WgSolveOpts), C.POINTER(WgStats)]),
    "wg_poisson_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(WgSolveOpts),
                                   C.POINTER(WgStats)]),
    "wg_poisson_solve_noalloc": (C.c_int, [C.POINTER(WgGrid), C.c_void_p, C.c_void_p, C.c_int,
                                           C.POINTER(WgSolveOpts), C.POINTER(WgStats), C.c_void_p]),
    "wg_mg_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "wg_sdf_from_field": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.POINTER(WgStats)]),
    "wg_get_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "wg_get_mesh": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "wg_recon_destroy": (None, [C.c_void_p]),
    "wg_recon_stream": (C.c_void_p, [C.c_void_p]),
    "wg_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_size_t, C.c_int, C.c_int]),
    "wg_submit": (C.c_int, [C.c_void_p, C.POINTER(WgRequest), C.POINTER(C.c_uint64)]),
    "wg_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(WgResult)]),
    "wg_server_now": (C.c_double, [C.c_void_p]),
    "wg_server_destroy": (None, [C.c_void_p]),
    "wg_profile_enable": (None, [C.c_uint]),
    "wg_profile_read": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "wg_profile_reset": (None, []),
    "wg_profile_walk_counts": (C.c_int, [C.POINTER(C.c_uint64 * 4)]),
    "wg_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "wg_dpca_normals": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "wg_orient_normals": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(WgOrientOpts), C.c_void_p,
                                    C.POINTER(WgOrientInfo), C.c_void_p]),
}

PROF_KINDS = {"splat": 0, "sweep": 1, "smooth": 2, "resid64": 3, "transfer": 4, "cgupdate": 5, "mc": 6,
              "sdf": 7, "sample": 8}


def profile_enable(kinds):
    mask = 0
    for k in kinds:
        mask |= 1 << PROF_KINDS[k]
    lib().wg_profile_enable(mask)


def profile_read(kind):
    ms, n, u = C.c_double(), C.c_int64(), C.c_double()
    check(lib().wg_profile_read(PROF_KINDS[kind], C.byref(ms), C.byref(n), C.byref(u)))
    return {"ms": ms.value, "launches": n.value, "units": u.value}


def profile_walk_counts():
    """Distance-walk test counts since the last reset (wg_profile_walk_counts)."""
    out = (C.c_uint64 * 4)()
    check(lib().wg_profile_walk_counts(C.byref(out)))
    return {"tri_tests": out[0], "aabb_tests": out[1], "obb_tests": out[2], "nodes": out[3]}


def lib():
    """Load libwgeo.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime: load it first, so that libwgeo.so binds
        # to the runtime torch's tensors and streams belong to (loading the
        # library first brings in a second runtime that then sees no device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_20964_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    m = lib().wg_last_error()
    return m.decode() if m else ""


def check(rc, allow=(WG_OK,)):
    """Raise WgError for a negative code not in ``allow``; return rc."""
    if rc < 0 and rc not in allow:
        raise WgError(rc, last_error())
    return rc


def make_grid(n, lo=(0.0, 0.0, 0.0), h=None):
    if isinstance(n, int):
        n = (n, n, n)
    g = WgGrid()
    g.n[:] = [int(v) for v in n]
    g.lo[:] = [float(v) for v in lo]
    g.h = float(1.0 / max(n) if h is None else h)
    return g


def grid_from_bbox(lo, hi, density, pad=3):
    """(n, lo, h) of wg_grid_from_bbox (host arithmetic)."""
    g = WgGrid()
    check(lib().wg_grid_from_bbox(C.byref((C.c_double * 3)(*map(float, lo))), C.byref((C.c_double * 3)(*map(float, hi))),
                                  float(density), int(pad), C.byref(g)))
    return tuple(g.n), tuple(g.lo), g.h


def make_opts(rel_tol=1e-6, max_iters=500, warm_start=False, precision=WG_FP32_FP64REDUCE, deterministic=False,
              quadrature=WG_VERTEX_QUADRATURE):
    o = WgSolveOpts()
    o.rel_tol = float(rel_tol)
    o.max_iters = int(max_iters)
    o.warm_start = int(bool(warm_start))
    o.precision = int(precision)
    o.deterministic = int(bool(deterministic))
    o.quadrature = int(quadrature)
    return o


def profile_reset():
    lib().wg_profile_reset()
