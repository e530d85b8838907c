"""ctypes loader for the oracle's C module (Marching Cubes rule, mesh distance,
ray parity).  Builds ``liboracle_mcdist.so`` with gcc on first use if it is
missing.  Test infrastructure only."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "mcdist.c")
_LIB = os.path.join(_HERE, "liboracle_mcdist.so")
_lib = None


def build(force=False):
    """Compile the C module (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_mc.restype = ctypes.c_int64
        L.oracle_mc.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int64, P, P, P]
        L.oracle_mc_case.restype = ctypes.c_int
        L.oracle_mc_case.argtypes = [ctypes.c_int, P]
        L.oracle_mesh_distance.restype = None
        L.oracle_mesh_distance.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P, P, P, P]
        L.oracle_ray_parity.restype = None
        L.oracle_ray_parity.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def mc_case(case):
    out = np.zeros(48, dtype=np.int32)
    n = lib().oracle_mc_case(int(case), _p(out))
    return out[:3 * n].reshape(n, 3)


def marching_cubes(chi, c):
    """chi: float64 [nz, ny, nx].  Returns (tri_cube [T,3] (i,j,k), tri_edge [T,3],
    tri_xyz [T,3,3] grid units)."""
    chi = np.ascontiguousarray(chi, dtype=np.float64)
    nz, ny, nx = chi.shape
    L = lib()
    T = L.oracle_mc(_p(chi), nx, ny, nz, float(c), 0, None, None, None)
    cube = np.zeros((T, 3), np.int32)
    edge = np.zeros((T, 3), np.int32)
    xyz = np.zeros((T, 3, 3), np.float64)
    if T:
        L.oracle_mc(_p(chi), nx, ny, nz, float(c), T, _p(cube), _p(edge), _p(xyz))
    return cube, edge, xyz


def mesh_distance(pts, tri_xyz):
    """Brute-force distance (grid units) from pts [M,3] to triangles [T,3,3]."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri_xyz, dtype=np.float64).reshape(-1, 9)
    m = pts.shape[0]
    d = np.zeros(m)
    arg = np.zeros(m, np.int64)
    bary = np.zeros((m, 3))
    lib().oracle_mesh_distance(m, _p(pts), tri.shape[0], _p(tri), _p(d), _p(arg), _p(bary))
    return d, arg, bary


def ray_parity(pts, tri_xyz, direction=(0.5773502691896258, 0.5163977794943222, 0.6324555320336759)):
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri_xyz, dtype=np.float64).reshape(-1, 9)
    dvec = np.asarray(direction, np.float64)
    dvec = np.ascontiguousarray(dvec / np.linalg.norm(dvec))
    inside = np.zeros(pts.shape[0], np.int32)
    lib().oracle_ray_parity(pts.shape[0], _p(pts), tri.shape[0], _p(tri), _p(dvec), _p(inside))
    return inside.astype(bool)
