"""GPU reverse pass (through the C ABI) against the FP64 oracle's reverse pass.

Bar: 1e-3 relative (L2) on gradients, and per component within 1e-3 of the
largest reference component.  The forward is solved to rel. residual 1e-10 so
that the comparison measures the adjoint, not the solve tolerance.
"""
import numpy as np
import pytest

from oracle import discretize as D
from oracle import pipeline as P
from paper_2609_20964_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _close(got, want, tol=1e-3):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    comp = np.abs(got - want).max() / np.abs(want).max()
    print(f"rel {rel:.2e} comp {comp:.2e}", flush=True)
    return rel <= tol and comp <= 3 * tol


def test_reverse_pass_small_star_with_normals_and_queries():
    from paper_2609_20964_amd.recon import Recon
    g = D.Grid.unit(20)
    c0 = np.array([0.03, -0.02, 0.015, 0.01])
    shape = synth.StarShape(c0, semi_axes=(0.3, 0.2, 0.22))
    x, n = synth.star(c0, 1500, 12, semi_axes=(0.3, 0.2, 0.22))
    tdirs = synth.unit_sphere_dirs(np.random.default_rng(13), 300)
    q = (synth.X0 + synth.StarShape(c0 + 0.01, semi_axes=(0.3, 0.2, 0.22)).rho(tdirs)[:, None] * tdirs)
    q = q.astype(np.float32)
    wn = np.random.default_rng(14).standard_normal((300, 3)).astype(np.float32) / 300
    ref = P.Recon(g, x, n)
    phi_ref, _ = ref.sample(q)
    gphi = (2.0 * phi_ref / 300).astype(np.float32)
    gx_ref, gn_ref, gq_ref = ref.backward(q, gphi.astype(np.float64), wn.astype(np.float64))
    r = Recon(20, len(x))
    r.forward(_cuda(x), _cuda(n), rel_tol=1e-10, max_iters=5000)
    phi, _ = r.sample(_cuda(q))
    gx, gn, gq = r.backward(_cuda(q), _cuda(gphi), _cuda(wn), want_gq=True, rel_tol=1e-10, max_iters=5000)
    assert _close(gx.cpu().numpy(), gx_ref)
    assert _close(gn.cpu().numpy(), gn_ref)
    assert _close(gq.cpu().numpy(), gq_ref)
    r.close()


@pytest.mark.parametrize("n", [(20, 20, 20), (24, 20, 28)])
def test_reverse_pass_exact_quadrature(n):
    """The reverse pass of the exact-quadrature system: the adjoint solve on
    the 27-point stiffness and the transposed consistent right-hand side."""
    from paper_2609_20964_amd.recon import Recon
    g = D.Grid(n, (0.0, 0.0, 0.0), 1.0 / 20)
    c0 = np.array([0.03, -0.02, 0.015, 0.01])
    x, nr = synth.star(c0, 1500, 12, semi_axes=(0.3, 0.2, 0.22))
    tdirs = synth.unit_sphere_dirs(np.random.default_rng(13), 300)
    q = (synth.X0 + synth.StarShape(c0 + 0.01, semi_axes=(0.3, 0.2, 0.22)).rho(tdirs)[:, None] * tdirs)
    q = q.astype(np.float32)
    wn = np.random.default_rng(14).standard_normal((300, 3)).astype(np.float32) / 300
    ref = P.Recon(g, x, nr, exact=True)
    phi_ref, _ = ref.sample(q)
    gphi = (2.0 * phi_ref / 300).astype(np.float32)
    gx_ref, gn_ref, gq_ref = ref.backward(q, gphi.astype(np.float64), wn.astype(np.float64))
    r = Recon(n, len(x), h=1.0 / 20)
    r.forward(_cuda(x), _cuda(nr), rel_tol=1e-10, max_iters=5000, quadrature="exact")
    phi, _ = r.sample(_cuda(q))
    assert np.abs(phi.cpu().numpy() - phi_ref).max() <= 1e-4 * g.h
    # the reverse pass follows the forward's quadrature whatever its options say
    gx, gn, gq = r.backward(_cuda(q), _cuda(gphi), _cuda(wn), want_gq=True, rel_tol=1e-10, max_iters=5000)
    assert _close(gx.cpu().numpy(), gx_ref)
    assert _close(gn.cpu().numpy(), gn_ref)
    assert _close(gq.cpu().numpy(), gq_ref)
    r.close()


def test_autograd_function_matches_oracle_chain():
    from paper_2609_20964_amd.recon import Recon, reconstruct
    g = D.Grid.unit(24)
    x, n = synth.sphere(2500, radius=0.28, seed=21)
    q = synth.uniform_queries(800, 22)
    ref = P.Recon(g, x, n)
    phi_ref, n_ref = ref.sample(q)
    w = np.random.default_rng(23).standard_normal((800, 3))
    # L = mean phi^2 + mean (w . n(q))
    gx_ref, gn_ref, gq_ref = ref.backward(q, 2.0 * phi_ref / 800, w / 800)
    r = Recon(24, len(x))
    tx = _cuda(x).requires_grad_(True)
    tn = _cuda(n).requires_grad_(True)
    tq = _cuda(q).requires_grad_(True)
    phi, nq = reconstruct(tx, tn, tq, r, rel_tol=1e-10, max_iters=5000)
    loss = (phi ** 2).mean() + (nq * _cuda(w)).sum(1).mean()
    loss.backward()
    assert _close(tx.grad.cpu().numpy(), gx_ref)
    assert _close(tn.grad.cpu().numpy(), gn_ref)
    assert _close(tq.grad.cpu().numpy(), gq_ref)
    r.close()


def test_differentiable_case_16_coefficients_128():
    """The 16-coefficient superellipsoid at 128^3: dL/dc from the GPU adjoint
    against dL/dc from the oracle's adjoint, both chained through the same
    shape generator."""
    from paper_2609_20964_amd.recon import Recon
    case = synth.diff_case()
    g = D.Grid.unit(128)
    ct = torch.tensor(case.shape.coeffs, dtype=torch.float64, requires_grad=True)
    xt, nt = synth.star_points_torch(case.shape, case.dirs, ct)
    x = xt.detach().numpy().astype(np.float32)
    n = nt.detach().numpy().astype(np.float32)
    T = len(case.targets)
    r = Recon(128, len(x))
    r.forward(_cuda(x), _cuda(n), rel_tol=1e-10, max_iters=5000)
    phi, _ = r.sample(_cuda(case.targets))
    gphi = 2.0 * phi / T
    gx, gn, _ = r.backward(_cuda(case.targets), gphi.contiguous(), rel_tol=1e-10, max_iters=5000)
    (grad_gpu,) = torch.autograd.grad(
        (xt * gx.cpu().double()).sum() + (nt * gn.cpu().double()).sum(), ct, retain_graph=True)
    ref = P.Recon(g, x, n)
    phi_ref, _ = ref.sample(case.targets)
    assert np.abs(phi.cpu().numpy() - phi_ref).max() <= 1e-4 * g.h
    gx_ref, gn_ref, _ = ref.backward(case.targets, 2.0 * phi_ref / T)
    (grad_ref,) = torch.autograd.grad((xt * torch.tensor(gx_ref)).sum() + (nt * torch.tensor(gn_ref)).sum(), ct)
    print("dL/dc gpu", grad_gpu.numpy(), "\noracle", grad_ref.numpy(), flush=True)
    assert _close(grad_gpu.numpy(), grad_ref.numpy())
    r.close()


def test_adjoint_against_central_differences_on_the_gpu():
    """Directional derivatives of L = mean phi(q)^2 from the GPU adjoint
    against central finite differences of GPU forwards (no oracle): along
    random normal perturbations (b is linear in the normals), and along random
    position perturbations that keep every point in its central cell (the
    splat weights are smooth inside a cell)."""
    from paper_2609_20964_amd.recon import Recon
    n = 64
    g = D.Grid.unit(n)
    c = synth.draw_star_coeffs(81)
    x, nrm = synth.star(c, 20000, 82)
    q = synth.star(c + 0.01, 2000, 83)[0]
    rng = np.random.default_rng(84)
    r = Recon(n, len(x))

    def loss(xx, nn):
        r.forward(_cuda(xx), _cuda(nn), rel_tol=1e-11, max_iters=5000)
        phi, _ = r.sample(_cuda(q), normals=False)
        return float((phi.double() ** 2).mean())

    loss(x, nrm)
    phi, _ = r.sample(_cuda(q), normals=False)
    gx, gn, _ = r.backward(_cuda(q), (2.0 / len(q)) * phi, rel_tol=1e-11, max_iters=5000)
    gx, gn = gx.cpu().double().numpy(), gn.cpu().double().numpy()
    # normals
    dn = rng.standard_normal(nrm.shape)
    eps = 1e-3
    fd = (loss(x, nrm + eps * dn) - loss(x, nrm - eps * dn)) / (2 * eps)
    ad = float((gn * dn).sum())
    print(f"normals: adjoint {ad:.6e} fd {fd:.6e}", flush=True)
    assert abs(ad - fd) <= 1e-2 * abs(fd)
    # positions, restricted to points that stay in their cells at +-eps
    dx = rng.standard_normal(x.shape)
    eps = 2e-2 * g.h
    k0 = D.cell_keys(g, x)[0]
    stay = np.ones(len(x), bool)
    for s in (1, -1):
        xs = (x.astype(np.float64) + s * eps * dx).astype(np.float32)
        stay &= (D.cell_keys(g, xs)[0] == k0).all(1)
    dx[~stay] = 0.0
    xp = (x.astype(np.float64) + eps * dx).astype(np.float32)
    xm = (x.astype(np.float64) - eps * dx).astype(np.float32)
    step = (xp.astype(np.float64) - xm.astype(np.float64)) / 2   # the perturbation FP32 actually applies
    fd = (loss(xp, nrm) - loss(xm, nrm)) / 1.0
    ad = float((gx * (2 * step)).sum())
    print(f"positions ({stay.mean():.3f} of points moved): adjoint {ad:.6e} fd {fd:.6e}", flush=True)
    assert abs(ad - fd) <= 2e-2 * abs(fd)
    r.close()


def test_shape_optimisation_recovers_the_target_shape():
    """Sec. 3.3's inverse design on the library's gradients: Adam over the 16
    coefficients of a star-shaped body, started from the target's coefficients
    perturbed by up to 0.02 each.  The loss is Eq. (40): the squared mismatch
    of the reconstructed SDF with the target's SDF (reconstructed from the
    target shape's cloud by the same pipeline), at 8192 points in a band
    around the target surface, 64^3 grid; it is 0 at the target's coefficients.
    Within 60 epochs the loss falls by at least 10x and the largest coefficient
    error by at least 2x."""
    import torch

    from paper_2609_20964_amd.optimize import optimise_shape
    from paper_2609_20964_amd.recon import Recon
    c_t = synth.draw_star_coeffs(1101)
    start = c_t + np.random.default_rng(1102).uniform(-0.02, 0.02, c_t.shape)
    dirs = synth.unit_sphere_dirs(np.random.default_rng(1103), 20000)
    rng = np.random.default_rng(1104)
    tdirs = synth.unit_sphere_dirs(rng, 8192)
    q = (synth.X0 + (synth.StarShape(c_t).rho(tdirs) * rng.uniform(0.85, 1.15, 8192))[:, None] * tdirs)
    q = q.astype(np.float32)
    pts, nrm = synth.star_points_torch(synth.StarShape(c_t), dirs, torch.tensor(c_t, dtype=torch.float64))
    r = Recon(64, len(dirs))
    r.forward(pts.detach().float().cuda().contiguous(), nrm.detach().float().cuda().contiguous(), rel_tol=1e-6)
    phi_t, _ = r.sample(_cuda(q), normals=False)
    phi_t = phi_t.cpu().numpy()
    r.close()
    _, hist = optimise_shape(synth.StarShape(start), dirs, start, q, phi_target=phi_t, n=64, epochs=60, lr=2e-3,
                             target_coeffs=c_t)
    print("loss", [f"{v:.3e}" for v in hist.loss[::6]], "coeff err", [f"{v:.4f}" for v in hist.coeff_err[::6]],
          flush=True)
    assert min(hist.loss[-5:]) <= hist.loss[0] / 10
    assert hist.coeff_err[-1] <= hist.coeff_err[0] / 2
