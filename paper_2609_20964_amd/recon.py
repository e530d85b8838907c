"""Python face of the reconstruction handle and its autograd function.

``Recon`` wraps one ``wg_recon`` handle (resident device state for one grid);
``reconstruct`` is a ``torch.autograd.Function`` whose backward is the
library's hand-written reverse pass (one adjoint Poisson solve, Warp-Geo
Sec. 2.5).  Torch provides device memory and the stream; every computation runs
in libwgeo.so.
"""
from __future__ import annotations

import ctypes as C
import warnings

import torch

from . import _lib as L


def _dev(t, dtype, shape_last=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape [N, {shape_last}]")
    return C.c_void_p(t.data_ptr())


def _precision(p):
    codes = {"fp32": L.WG_FP32_FP64REDUCE, "fp64": L.WG_FP64}
    if p not in codes:
        raise ValueError(f"precision must be one of {sorted(codes)}")
    return codes[p]


def _quadrature(q):
    codes = {"vertex": L.WG_VERTEX_QUADRATURE, "exact": L.WG_EXACT_QUADRATURE}
    if q not in codes:
        raise ValueError(f"quadrature must be one of {sorted(codes)}")
    return codes[q]


def grid_from_cloud(xyz, density, pad=3):
    """(n, lo, h) of a grid over the bounding box of the device points xyz
    [N,3] with density cells per unit length (wg_grid_from_cloud)."""
    g = L.WgGrid()
    L.check(L.lib().wg_grid_from_cloud(_dev(xyz, torch.float32, 3, "xyz"), int(xyz.shape[0]), float(density),
                                       int(pad), C.byref(g), C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return tuple(g.n), tuple(g.lo), g.h


class Recon:
    """One reconstruction grid resident on the current CUDA device.

    Parameters: n (cells per axis, int or 3-tuple), max_points, lo (grid
    origin) and h (cell edge; default 1/max(n), i.e. the unit cube).  The
    handle runs on the torch stream current at creation.
    """

    def __init__(self, n, max_points, lo=(0.0, 0.0, 0.0), h=None, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.grid = L.make_grid(n, lo, h)
        self.n = tuple(self.grid.n)
        self.h = self.grid.h
        self.lo = tuple(self.grid.lo)
        self.max_points = int(max_points)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            handle = C.c_void_p()
            L.check(L.lib().wg_recon_create(C.byref(handle), C.byref(self.grid), self.max_points,
                                           C.c_void_p(self.stream.cuda_stream)))
        self._h = handle
        self.generation = 0
        self.n_points = 0
        self.last_stats = None
        self._pending = None

    @staticmethod
    def footprint(n, max_points, lo=(0.0, 0.0, 0.0), h=None):
        g = L.make_grid(n, lo, h)
        return int(L.lib().wg_recon_footprint(C.byref(g), int(max_points)))

    @property
    def cells(self):
        return self.n[0] * self.n[1] * self.n[2]

    def close(self):
        if getattr(self, "_h", None):
            L.lib().wg_recon_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _alive(self):
        if not self._h:
            raise RuntimeError("handle is closed")
        return self._h

    # -- forward ---------------------------------------------------------------
    def forward(self, xyz, nrm, rel_tol=1e-6, max_iters=500, warm_start=False, precision="fp32",
                deterministic=False, quadrature="vertex"):
        """Splat, solve, extract, distance (F1-F7).  Returns the stats dict.

        precision "fp32" (FP32 splat, FP32 sweeps, FP64 reductions and
        refinement) or "fp64" (the right-hand side in FP64, summed exactly);
        deterministic: the splat sums in 64-bit fixed point, so b, chi and phi
        do not depend on the order points and threads are taken in;
        quadrature "vertex" (the 7-point system) or "exact" (the Galerkin
        integrals of Eq. 21 and 26 taken exactly: 27-point stiffness and
        consistent right-hand side; fp32 and not deterministic)."""
        npts = int(xyz.shape[0])
        px = _dev(xyz, torch.float32, 3, "xyz")
        pn = _dev(nrm, torch.float32, 3, "nrm")
        if nrm.shape[0] != npts:
            raise ValueError("xyz and nrm differ in length")
        st = L.WgStats()
        o = L.make_opts(rel_tol, max_iters, warm_start, _precision(precision), deterministic, _quadrature(quadrature))
        rc = L.check(L.lib().wg_recon_forward(self._alive(), px, pn, npts, C.byref(o), C.byref(st)),
                     allow=(L.WG_OK, L.WG_ENOTCONV))
        if rc == L.WG_ENOTCONV:
            warnings.warn(f"Poisson solve stopped at rel. residual {st.rel_res:.3e}")
        self.generation += 1
        self.n_points = npts
        self.last_stats = st.as_dict()
        return self.last_stats

    def sdf_from_field(self, chi, c):
        """Surface {chi = c} and the signed distance to it on every node (F6-F7)
        for a given float64 field chi [N] (wg_sdf_from_field).  Returns stats."""
        if chi.numel() != self.cells:
            raise ValueError(f"chi must hold {self.cells} cells")
        st = L.WgStats()
        chi = chi.contiguous()
        L.check(L.lib().wg_sdf_from_field(self._alive(), _dev(chi, torch.float64, None, "chi"), float(c),
                                          C.byref(st)))
        self.generation += 1
        self.n_points = 0
        self.last_stats = st.as_dict()
        return self.last_stats

    def sample(self, q, normals=True):
        """SDF and unit normals at query points q [Q,3] (F8)."""
        nq = int(q.shape[0])
        pq = _dev(q, torch.float32, 3, "q")
        phi = torch.empty(nq, dtype=torch.float32, device=q.device)
        nrm = torch.empty((nq, 3), dtype=torch.float32, device=q.device) if normals else None
        L.check(L.lib().wg_sample_sdf_normals(self._alive(), pq, nq, C.c_void_p(phi.data_ptr()),
                                              C.c_void_p(nrm.data_ptr()) if nrm is not None else None))
        return phi, nrm

    def step(self, xyz, nrm, q, rel_tol=1e-6, max_iters=500, warm_start=True, normals=True, precision="fp32",
             deterministic=False, quadrature="vertex"):
        """Pipelined forward + sampling for moving-boundary loops (wg_recon_step):
        returns (stats, phi [Q], nrm [Q,3] or None) once the surface is extracted;
        the distance walk and the sampling finish on the handle's second stream
        while the next step splats and solves.  The outputs are complete after
        wait() (or a device synchronisation), or once the next step returns."""
        npts, nq = int(xyz.shape[0]), int(q.shape[0])
        if nrm.shape[0] != npts:
            raise ValueError("xyz and nrm differ in length")
        px, pn = _dev(xyz, torch.float32, 3, "xyz"), _dev(nrm, torch.float32, 3, "nrm")
        pq = _dev(q, torch.float32, 3, "q")
        phi = torch.empty(nq, dtype=torch.float32, device=q.device)
        nout = torch.empty((nq, 3), dtype=torch.float32, device=q.device) if normals else None
        st = L.WgStats()
        o = L.make_opts(rel_tol, max_iters, warm_start, _precision(precision), deterministic, _quadrature(quadrature))
        rc = L.check(L.lib().wg_recon_step(self._alive(), px, pn, npts, pq, nq, C.c_void_p(phi.data_ptr()),
                                           C.c_void_p(nout.data_ptr()) if nout is not None else None,
                                           C.byref(o), C.byref(st)), allow=(L.WG_OK, L.WG_ENOTCONV))
        if rc == L.WG_ENOTCONV:
            warnings.warn(f"Poisson solve stopped at rel. residual {st.rel_res:.3e}")
        # the library writes these on its second stream: keep them (and q) alive
        # until that work is ordered before any reuse of their memory
        self._pending = (q, phi, nout)
        self.generation += 1
        self.n_points = npts
        self.last_stats = st.as_dict()
        return self.last_stats, phi, nout

    def wait(self):
        """Order the handle's stream after the last step's distance walk and sampling."""
        L.check(L.lib().wg_recon_wait(self._alive()))
        self._pending = None

    # -- reverse ---------------------------------------------------------------
    def backward(self, q, gphi, gnrm=None, want_gq=False, rel_tol=1e-6, max_iters=500):
        """Reverse pass (B1-B6) of the last forward sampled at q.
        Returns (g_xyz [N,3], g_nrm [N,3], g_q [Q,3] or None)."""
        nq = int(q.shape[0])
        dev = q.device
        gx = torch.empty((self.n_points, 3), dtype=torch.float32, device=dev)
        gn = torch.empty((self.n_points, 3), dtype=torch.float32, device=dev)
        gq = torch.empty((nq, 3), dtype=torch.float32, device=dev) if want_gq else None
        st = L.WgStats()
        o = L.make_opts(rel_tol, max_iters, False)
        rc = L.check(L.lib().wg_recon_backward(
            self._alive(), _dev(q, torch.float32, 3, "q"), nq, _dev(gphi, torch.float32, None, "gphi"),
            _dev(gnrm, torch.float32, 3, "gnrm") if gnrm is not None else None,
            C.c_void_p(gx.data_ptr()), C.c_void_p(gn.data_ptr()),
            C.c_void_p(gq.data_ptr()) if gq is not None else None, C.byref(o), C.byref(st)),
            allow=(L.WG_OK, L.WG_ENOTCONV))
        if rc == L.WG_ENOTCONV:
            warnings.warn(f"adjoint solve stopped at rel. residual {st.rel_res:.3e}")
        self.last_backward_stats = st.as_dict()
        return gx, gn, gq

    # -- standalone solve and exports ---------------------------------------------
    def poisson(self, b, x=None, bc="neumann", rel_tol=1e-10, max_iters=1000, quadrature="vertex"):
        """Solve A x = b on this grid (float32 b [N], float64 x [N])."""
        if b.numel() != self.cells or (x is not None and x.numel() != self.cells):
            raise ValueError(f"b and x must hold {self.cells} cells")
        if x is None:
            x = torch.zeros(self.cells, dtype=torch.float64, device=b.device)
            warm = False
        else:
            warm = True
        st = L.WgStats()
        o = L.make_opts(rel_tol, max_iters, warm, quadrature=_quadrature(quadrature))
        bcode = {"neumann": L.WG_BC_NEUMANN, "dirichlet": L.WG_BC_DIRICHLET}[bc]
        rc = L.check(L.lib().wg_poisson_solve(self._alive(), _dev(b, torch.float32, None, "b"),
                                              _dev(x, torch.float64, None, "x"), bcode, C.byref(o),
                                              C.byref(st)), allow=(L.WG_OK, L.WG_ENOTCONV))
        return x, st.as_dict()

    def mg_apply(self, r, bc="neumann"):
        """z = M r: one V-cycle of the solver's multigrid preconditioner (float32 [N])."""
        if r.numel() != self.cells:
            raise ValueError(f"r must hold {self.cells} cells")
        z = torch.empty_like(r)
        bcode = {"neumann": L.WG_BC_NEUMANN, "dirichlet": L.WG_BC_DIRICHLET}[bc]
        L.check(L.lib().wg_mg_apply(self._alive(), _dev(r, torch.float32, None, "r"), C.c_void_p(z.data_ptr()),
                                    bcode))
        return z

    def fields(self):
        """Resident fields of the last forward: b, chi (zero mean), phi, keys."""
        N = self.cells
        dev = self.device
        b = torch.empty(N, dtype=torch.float32, device=dev)
        chi = torch.empty(N, dtype=torch.float64, device=dev)
        phi = torch.empty(N, dtype=torch.float32, device=dev)
        keys = torch.empty(max(self.n_points, 1), dtype=torch.int32, device=dev)
        L.check(L.lib().wg_get_fields(self._alive(), C.c_void_p(b.data_ptr()), C.c_void_p(chi.data_ptr()),
                                      C.c_void_p(phi.data_ptr()), C.c_void_p(keys.data_ptr())))
        shp = (self.n[2], self.n[1], self.n[0])
        return {"b": b.view(shp), "chi": chi.view(shp), "phi": phi.view(shp), "keys": keys[:self.n_points]}

    def mesh(self):
        """Triangles of the last forward: vertices [T,3,3] (grid units) and info [T,2]."""
        T = C.c_int64()
        L.check(L.lib().wg_get_mesh(self._alive(), None, None, 0, C.byref(T)))
        tris = torch.empty((max(T.value, 1), 3, 3), dtype=torch.float32, device=self.device)
        info = torch.empty((max(T.value, 1), 2), dtype=torch.int32, device=self.device)
        L.check(L.lib().wg_get_mesh(self._alive(), C.c_void_p(tris.data_ptr()), C.c_void_p(info.data_ptr()),
                                    T.value, C.byref(T)))
        return tris[:T.value], info[:T.value]


class _ReconFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, nrm, q, recon, rel_tol, max_iters, warm_start, precision, deterministic, quadrature):
        recon.forward(xyz.detach().contiguous(), nrm.detach().contiguous(), rel_tol, max_iters, warm_start, precision,
                      deterministic, quadrature)
        phi, n = recon.sample(q.detach().contiguous())
        ctx.recon = recon
        ctx.generation = recon.generation
        ctx.rel_tol, ctx.max_iters = rel_tol, max_iters
        ctx.save_for_backward(q)
        return phi, n

    @staticmethod
    def backward(ctx, gphi, gn):
        (q,) = ctx.saved_tensors
        r = ctx.recon
        if r.generation != ctx.generation:
            raise RuntimeError("the handle ran another forward before this backward")
        if gphi is None:
            gphi = torch.zeros(q.shape[0], dtype=torch.float32, device=q.device)
        gx, gnp, gq = r.backward(q.detach().contiguous(), gphi.contiguous(),
                                 gn.contiguous() if gn is not None else None,
                                 want_gq=ctx.needs_input_grad[2], rel_tol=ctx.rel_tol, max_iters=ctx.max_iters)
        return gx, gnp, gq, None, None, None, None, None, None, None


def reconstruct(xyz, nrm, q, recon: Recon, rel_tol=1e-6, max_iters=500, warm_start=False, precision="fp32",
                deterministic=False, quadrature="vertex"):
    """Differentiable SDF and normals at q from the oriented cloud (xyz, nrm).

    Gradients flow to xyz, nrm and q through the library's adjoint."""
    return _ReconFn.apply(xyz, nrm, q, recon, rel_tol, max_iters, warm_start, precision, deterministic, quadrature)
