"""Gradient-based shape optimisation (Warp-Geo Sec. 3.3).

A compact parameterisation of the geometry (here the 16 Fourier coefficients
of a star-shaped body) generates the oriented cloud; the library reconstructs
the SDF and its reverse pass returns the gradient with respect to the points
and normals, which torch chains to the coefficients through the
parameterisation.  The loss matches the reconstructed SDF to a target SDF
(Eq. 40), sampled at target points: L = mean_j (phi(q_j) - phi_target_j)^2, by
default with target points on the target surface (phi_target = 0).  Adam takes
the steps.  The reconstruction and its gradient run in the HIP library; the
parameterisation and the optimiser are the caller's torch code.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import synth
from .recon import Recon, reconstruct


@dataclass
class History:
    loss: list = field(default_factory=list)
    coeff_err: list = field(default_factory=list)    # max |c - c_target| when the target is known
    coeffs: list = field(default_factory=list)


def optimise_shape(shape: synth.StarShape, dirs, coeffs0, targets, phi_target=None, n=64, epochs=100, lr=2e-3,
                   rel_tol=1e-6, target_coeffs=None, device="cuda", callback=None):
    """Adam over the coefficients of ``shape`` (points along body-frame
    directions ``dirs``) so that the reconstructed SDF matches ``phi_target``
    (zeros by default) at ``targets`` [T,3] on an n^3 unit-cube grid.  Returns
    (coefficients, History)."""
    theta = torch.tensor(np.asarray(coeffs0, np.float64), requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    q = torch.as_tensor(np.asarray(targets, np.float32), device=device)
    tgt = (torch.zeros(q.shape[0], dtype=torch.float32, device=device) if phi_target is None
           else torch.as_tensor(np.asarray(phi_target, np.float32), device=device))
    r = Recon(n, len(dirs))
    hist = History()
    try:
        for epoch in range(epochs):
            pts, nrm = synth.star_points_torch(shape, dirs, theta)
            phi, _ = reconstruct(pts.float().to(device).contiguous(), nrm.float().to(device).contiguous(), q, r,
                                 rel_tol=rel_tol, warm_start=epoch > 0)
            loss = ((phi - tgt) ** 2).mean()
            opt.zero_grad()
            loss.backward()
            opt.step()
            hist.loss.append(float(loss.item()))
            c = theta.detach().numpy().copy()
            hist.coeffs.append(c)
            if target_coeffs is not None:
                hist.coeff_err.append(float(np.abs(c - np.asarray(target_coeffs)).max()))
            if callback is not None:
                callback(epoch, hist)
    finally:
        r.close()
    return theta.detach().numpy(), hist
