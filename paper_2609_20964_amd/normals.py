"""Normals for unoriented clouds (Warp-Geo Sec. 2.1-2.2): thin wrappers over
wg_dpca_normals and wg_orient_normals (argument marshalling only)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _points(xyz):
    if not (xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2 and xyz.shape[1] == 3):
        raise ValueError("xyz must be a float32 CUDA tensor [N, 3]")
    return xyz.contiguous()


def dpca_normals(xyz, radius=0.1, eps=0.0):
    """Unoriented unit normals [N, 3] by distance-weighted PCA (Eq. 1-6);
    radius R of Table 1, eps of Eq. 2 (<= 0: 1e-6 R)."""
    x = _points(xyz)
    out = torch.empty_like(x)
    s = torch.cuda.current_stream(x.device)
    L.check(L.lib().wg_dpca_normals(x.data_ptr(), x.shape[0], float(radius), float(eps), out.data_ptr(),
                                    s.cuda_stream))
    return out


def orient_normals(xyz, nrm, gamma_r=2.5, n_tol=2, refine=True, counts=False):
    """Outward orientation by ray casting (Eq. 7-14 and the refinement of
    Sec. 2.2).  Returns (oriented normals [N, 3], info dict, counts [N, 4] or
    None: N and N_one along +n, then along -n, of the input normals)."""
    x = _points(xyz)
    n = _points(nrm).clone()
    if n.shape != x.shape:
        raise ValueError("xyz and nrm differ in shape")
    o = L.WgOrientOpts(float(gamma_r), int(n_tol), int(bool(refine)))
    info = L.WgOrientInfo()
    cnt = torch.empty((x.shape[0], 4), dtype=torch.int32, device=x.device) if counts else None
    s = torch.cuda.current_stream(x.device)
    L.check(L.lib().wg_orient_normals(x.data_ptr(), x.shape[0], n.data_ptr(), C.byref(o),
                                      cnt.data_ptr() if cnt is not None else None, C.byref(info), s.cuda_stream))
    return n, info.as_dict(), cnt


def oriented_normals(xyz, radius=0.1, gamma_r=2.5, n_tol=2, refine=True):
    """D-PCA then orientation: the normals the Poisson path takes."""
    n, info, _ = orient_normals(xyz, dpca_normals(xyz, radius), gamma_r, n_tol, refine)
    return n, info
