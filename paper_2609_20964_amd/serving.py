"""Python client of the library's continuous-batching server (wg_server_*).

Requests carry device tensors; the server copies them at submit, runs up to
``max_inflight`` requests concurrently on resident handles admitted by HBM
footprint, and writes each request's outputs into the tensors given at submit.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


class Ticket:
    def __init__(self, tid, outputs, n_points):
        self.id = tid
        self.outputs = outputs        # keeps output tensors alive until polled
        self.n_points = n_points
        self.result = None


class Server:
    def __init__(self, hbm_budget_bytes, max_inflight=4, device=None):
        dev = torch.cuda.current_device() if device is None else device
        h = C.c_void_p()
        L.check(L.lib().wg_server_create(C.byref(h), int(hbm_budget_bytes), int(max_inflight), int(dev)))
        self._h = h
        self.device = torch.device("cuda", dev)

    def now(self):
        return L.lib().wg_server_now(self._h)

    def submit(self, n, xyz, nrm, q, gphi=None, rel_tol=1e-6, max_iters=500, normals=True, lo=(0, 0, 0), h=None,
               gnrm=None, want_gq=False, precision="fp32", deterministic=False, quadrature="vertex"):
        """Queue one reconstruction; returns a Ticket.  Inputs are copied before return.

        gphi (dL/dphi(q), [Q]) asks for the reverse pass: the outputs then hold
        g_xyz and g_nrm for the points, and g_q [Q,3] if want_gq; gnrm [Q,3]
        adds dL/dn(q)."""
        req = L.WgRequest()
        req.grid = L.make_grid(n, lo, h)
        npts, nq = int(xyz.shape[0]), int(q.shape[0])
        for t in (xyz, nrm, q):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        phi = torch.empty(nq, dtype=torch.float32, device=q.device)
        nout = torch.empty((nq, 3), dtype=torch.float32, device=q.device) if normals else None
        gx = gn = gq = None
        if gphi is None and (gnrm is not None or want_gq):
            raise ValueError("gnrm / want_gq need gphi")
        if gphi is not None:
            gphi = gphi.contiguous()     # held in a local until wg_submit has copied it
            gx = torch.empty((npts, 3), dtype=torch.float32, device=q.device)
            gn = torch.empty((npts, 3), dtype=torch.float32, device=q.device)
            if want_gq:
                gq = torch.empty((nq, 3), dtype=torch.float32, device=q.device)
        if gnrm is not None:
            assert gnrm.is_cuda and gnrm.dtype == torch.float32 and gnrm.shape == (nq, 3)
            gnrm = gnrm.contiguous()
        req.d_xyz, req.d_nrm, req.n_points = xyz.data_ptr(), nrm.data_ptr(), npts
        req.d_q, req.n_q = q.data_ptr(), nq
        req.d_gphi = gphi.data_ptr() if gphi is not None else None
        req.opts = L.make_opts(rel_tol, max_iters, False, {"fp32": L.WG_FP32_FP64REDUCE, "fp64": L.WG_FP64}[precision],
                               deterministic,
                               {"vertex": L.WG_VERTEX_QUADRATURE, "exact": L.WG_EXACT_QUADRATURE}[quadrature])
        req.d_phi = phi.data_ptr()
        req.d_nrm_out = nout.data_ptr() if nout is not None else None
        req.d_gxyz = gx.data_ptr() if gx is not None else None
        req.d_gnrm_pts = gn.data_ptr() if gn is not None else None
        req.d_gnrm = gnrm.data_ptr() if gnrm is not None else None
        req.d_gq = gq.data_ptr() if gq is not None else None
        torch.cuda.current_stream().synchronize()      # inputs must be complete before the copy
        tid = C.c_uint64()
        L.check(L.lib().wg_submit(self._h, C.byref(req), C.byref(tid)))
        return Ticket(tid.value, {"phi": phi, "nrm": nout, "g_xyz": gx, "g_nrm": gn, "g_q": gq}, npts)

    def poll(self, ticket):
        """None while pending; else (status, outputs dict, result dict)."""
        res = L.WgResult()
        rc = L.lib().wg_poll(self._h, C.c_uint64(ticket.id), C.byref(res))
        if rc == L.WG_PENDING:
            return None
        if rc == L.WG_ESTATE:
            raise L.WgError(rc, L.last_error())
        ticket.result = {"status": rc, "stats": res.stats.as_dict(), "t_submit": res.t_submit,
                         "t_start": res.t_start, "t_done": res.t_done}
        return rc, ticket.outputs, ticket.result

    def close(self):
        if getattr(self, "_h", None):
            L.lib().wg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
