"""Continuous-batching server: each result alone equals the same request in the
mix (SDF within 1e-4 h, gradients within 1e-3), HBM-footprint admission, and
rejection of a request larger than the budget."""
import time

import numpy as np
import pytest

from angles import angle
from paper_2609_20964_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _requests():
    out = []
    rng = np.random.default_rng(601)
    for i, (n, npts, grad) in enumerate([(32, 6000, False), (64, 30000, True), (32, 12000, True),
                                         (64, 9000, False), (48, 15000, False), (32, 4000, True)]):
        c = synth.draw_star_coeffs(700 + i)
        semi = rng.uniform(0.12, 0.28, 3)
        x, nn = synth.star(c, npts, [701, i], semi_axes=semi, p=rng.uniform(2, 5))
        q = synth.uniform_queries(4096, [702, i])
        out.append((n, x, nn, q, grad))
    return out


def _alone(n, x, nn, q, grad):
    from paper_2609_20964_amd.recon import Recon
    r = Recon(n, len(x))
    r.forward(_cuda(x), _cuda(nn), rel_tol=1e-10, max_iters=5000)
    phi, nq = r.sample(_cuda(q))
    res = {"phi": phi.cpu().numpy()}
    if grad:
        gphi = 2.0 * phi / len(q)
        gx, gn, _ = r.backward(_cuda(q), gphi.contiguous(), rel_tol=1e-10, max_iters=5000)
        res["gphi"] = gphi
        res["g_xyz"], res["g_nrm"] = gx.cpu().numpy(), gn.cpu().numpy()
    r.close()
    return res


def _wait(srv, tickets, timeout=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for i, t in enumerate(tickets):
            if i in done:
                continue
            out = srv.poll(t)
            if out is not None:
                done[i] = out
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return [done[i] for i in range(len(tickets))]


def test_alone_equals_in_the_mix():
    from paper_2609_20964_amd.serving import Server
    reqs = _requests()
    alone = [_alone(*r) for r in reqs]
    srv = Server(hbm_budget_bytes=8 << 30, max_inflight=4)
    tickets = []
    for (n, x, nn, q, grad), a in zip(reqs, alone):
        tickets.append(srv.submit(n, _cuda(x), _cuda(nn), _cuda(q), gphi=a.get("gphi"), rel_tol=1e-10,
                                  max_iters=5000))
    results = _wait(srv, tickets)
    for (n, x, nn, q, grad), a, (st, outs, info) in zip(reqs, alone, results):
        assert st == 0, info
        assert np.abs(outs["phi"].cpu().numpy() - a["phi"]).max() <= 1e-4 / n
        if grad:
            for k in ("g_xyz", "g_nrm"):
                got, want = outs[k].cpu().numpy(), a[k]
                assert np.linalg.norm(got - want) <= 1e-3 * np.linalg.norm(want)
        assert info["t_submit"] <= info["t_start"] <= info["t_done"]
    srv.close()


def test_deterministic_requests_alone_equal_mix_bit_for_bit():
    """deterministic=1: each request served in the mix (four slots, persistent
    and non-persistent walks) gives the SDF and normals of the same request run
    alone, bit for bit; the reverse pass (FP32 atomics) within 1e-3."""
    from paper_2609_20964_amd.recon import Recon
    from paper_2609_20964_amd.serving import Server
    reqs = _requests()
    alone = []
    for n, x, nn, q, grad in reqs:
        r = Recon(n, len(x))
        r.forward(_cuda(x), _cuda(nn), rel_tol=1e-10, max_iters=5000, deterministic=True)
        phi, nq = r.sample(_cuda(q))
        res = {"phi": phi.cpu().numpy(), "nrm": nq.cpu().numpy()}
        if grad:
            gphi = 2.0 * phi / len(q)
            gx, gn, _ = r.backward(_cuda(q), gphi.contiguous(), rel_tol=1e-10, max_iters=5000)
            res["gphi"], res["g_xyz"], res["g_nrm"] = gphi, gx.cpu().numpy(), gn.cpu().numpy()
        alone.append(res)
        r.close()
    srv = Server(hbm_budget_bytes=8 << 30, max_inflight=4)
    tickets = [srv.submit(n, _cuda(x), _cuda(nn), _cuda(q), gphi=a.get("gphi"), rel_tol=1e-10, max_iters=5000,
                          deterministic=True) for (n, x, nn, q, grad), a in zip(reqs, alone)]
    results = _wait(srv, tickets)
    srv.close()
    for (n, x, nn, q, grad), a, (st, outs, info) in zip(reqs, alone, results):
        assert st == 0, info
        assert np.array_equal(outs["phi"].cpu().numpy(), a["phi"])
        assert np.array_equal(outs["nrm"].cpu().numpy(), a["nrm"])
        if grad:
            for k in ("g_xyz", "g_nrm"):
                got, want = outs[k].cpu().numpy(), a[k]
                assert np.linalg.norm(got - want) <= 1e-3 * np.linalg.norm(want)


def test_admission_by_footprint_and_rejection():
    from paper_2609_20964_amd._lib import WG_ENOMEM, WgError
    from paper_2609_20964_amd.recon import Recon
    from paper_2609_20964_amd.serving import Server
    fp64 = Recon.footprint(64, 1 << 15)
    # room for one 64^3 handle only: concurrent requests of two sizes must take turns
    srv = Server(hbm_budget_bytes=int(fp64 * 1.3), max_inflight=3)
    reqs = _requests()
    tickets = [srv.submit(n, _cuda(x), _cuda(nn), _cuda(q), rel_tol=1e-8) for (n, x, nn, q, g) in reqs]
    results = _wait(srv, tickets)
    assert all(st == 0 for st, _, _ in results)
    with pytest.raises(WgError) as e:
        x, nn = synth.sphere(1000)
        srv.submit(256, _cuda(x), _cuda(nn), _cuda(synth.uniform_queries(16, 1)))
    assert e.value.code == WG_ENOMEM
    srv.close()


@pytest.mark.parametrize("n", [128, 256])
def test_device_filling_requests_take_turns(n):
    """Two 128^3 or two 256^3 requests (each one's walk fills the device alone)
    take turns in arrival order: the second starts only once the first has
    binned, splatted, solved and extracted its surface (its distance walk then
    runs beside the second's solve), smaller ones may run beside them, and the
    two give the same field."""
    from paper_2609_20964_amd.serving import Server
    srv = Server(hbm_budget_bytes=16 << 30, max_inflight=3)
    x, nn = synth.sphere(20000, seed=603)
    q = synth.uniform_queries(1024, 604)
    reqs = [(n, x, nn), (n, x, nn), (32, *synth.sphere(4000, seed=605)), (64, *synth.sphere(8000, seed=606))]
    tickets = [srv.submit(n, _cuda(a), _cuda(b), _cuda(q), rel_tol=1e-6) for n, a, b in reqs]
    results = _wait(srv, tickets)
    assert all(st == 0 for st, _, _ in results), [r[2] for r in results]
    (_, o0, i0), (_, o1, i1) = results[0], results[1]
    # the first's turn: splat, solve, iso-value and surface (GPU-timed, the
    # host waits for each of them before its turn ends)
    turn_s = sum(i0["stats"]["ms"][:4]) / 1e3
    print("first", i0["t_start"], i0["t_done"], "turn", turn_s, "second", i1["t_start"], i1["t_done"], flush=True)
    assert i1["t_start"] >= i0["t_start"] + 0.9 * turn_s, (i0, i1)
    assert np.abs(o0["phi"].cpu().numpy() - o1["phi"].cpu().numpy()).max() <= 1e-4 / n
    srv.close()


def test_device_filling_successor_runs_beside_the_walk():
    """A 256^3 request that starts with another one queued runs the pipelined
    forward: its turn ends once its distance walk is enqueued (its walk time is
    then reported as 0) and the next one may start beside the walk.  A request
    with a reverse pass keeps its turn to the end even with a successor queued
    (its adjoint solve would meet the successor's solve), so that successor
    starts only once it is done.  Fields, normals and gradients equal those of
    the same request reconstructed alone.  A first 256^3 request holds the turn
    while the others are submitted, so they are all queued behind it."""
    from paper_2609_20964_amd.recon import Recon
    from paper_2609_20964_amd.serving import Server
    c = synth.draw_star_coeffs(632)
    xa, na = (_cuda(a) for a in synth.star(c, 60000, 633))
    q = _cuda(synth.uniform_queries(4096, 634))
    gphi = _cuda(np.random.default_rng(635).standard_normal(4096) / 4096)
    srv = Server(hbm_budget_bytes=16 << 30, max_inflight=2)
    tickets = [srv.submit(256, xa, na, q, rel_tol=1e-6) for _ in range(2)]
    tickets.append(srv.submit(256, xa, na, q, gphi=gphi, rel_tol=1e-6))
    tickets.append(srv.submit(256, xa, na, q, rel_tol=1e-6))
    results = _wait(srv, tickets)
    srv.close()
    assert all(st == 0 for st, _, _ in results), [r[2] for r in results]
    (_, ob, ib), (_, oc, ic), (_, od, id_) = results[1:]
    turn_s = sum(ib["stats"]["ms"][:4]) / 1e3
    for name, i in (("second", ib), ("third (reverse pass)", ic), ("fourth", id_)):
        print(name, i["t_start"], i["t_done"], "walk ms", i["stats"]["ms"][4], flush=True)
    assert ib["stats"]["ms"][4] == 0.0 and ic["stats"]["ms"][4] > 0.0
    assert ic["t_start"] >= ib["t_start"] + 0.9 * turn_s
    assert id_["t_start"] >= ic["t_done"]
    r = Recon(256, 60000)
    r.forward(xa, na, rel_tol=1e-6)
    phi, nrm = r.sample(q)
    gx, gn, _ = r.backward(q, gphi, rel_tol=1e-6)
    r.close()
    h = 1.0 / 256
    ok = np.linalg.norm(nrm.cpu().numpy(), axis=1) > 0
    for _, o, _ in results:
        assert np.abs(o["phi"].cpu().numpy() - phi.cpu().numpy()).max() <= 1e-4 * h
        assert angle(o["nrm"].cpu().numpy()[ok], nrm.cpu().numpy()[ok]).max() <= 1e-3
    assert _close(oc["g_xyz"].cpu().numpy(), gx.cpu().numpy())
    assert _close(oc["g_nrm"].cpu().numpy(), gn.cpu().numpy())


def _close(got, want, tol=1e-3, comp_tol=1e-2):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    comp = np.abs(got - want).max() / np.abs(want).max()
    print(f"    rel {rel:.2e} comp {comp:.2e}", flush=True)
    return rel <= tol and comp <= comp_tol


def _band_queries(c, semi, p, n_q, seed):
    """Queries in a band around a star shape (radius scaled by 0.9-1.1), so
    that every query's nearest triangle is unambiguous."""
    rng = np.random.default_rng(seed)
    dirs = synth.unit_sphere_dirs(rng, n_q)
    rho = synth.StarShape(np.asarray(c, np.float64), tuple(semi), float(p)).rho(dirs)
    return (synth.X0 + (rho * rng.uniform(0.9, 1.1, n_q))[:, None] * dirs).astype(np.float32)


def test_served_results_match_the_oracle():
    """Every served result against the FP64 oracle at rel. res 1e-10: phi at the
    queries within 1e-4 h, normals within 1e-3 rad (99th percentile), and for
    the three gradient requests g_xyz and g_nrm (one also with a normal term
    and query gradients g_q) within 1e-3 relative in L2.  The mix holds a 128^3
    request and five requests on four slots: requests that start while others
    run take the non-persistent distance walk.

    Per component the point gradients are held to 1e-2 of the largest, not
    1e-3: the loss has kinks where a node's nearest triangle switches, and at
    128^3 nodes sit within 1e-7 cells of such a switch (two triangles of
    adjacent cubes whose distances differ by 5.6e-8 cells, closest points
    1.6e-3 cells apart, at node (67, 95, 66) of the 128^3 request).  The FP32
    splat moves the mesh by ~3e-7 cells against the oracle's FP64 one, enough
    to pick the other triangle there, which moves the gradients of the points
    a few cells around by up to 5e-3 of the largest (found by comparing the
    GPU's point gradients with the oracle's per point); the L2 error stays
    below 4e-4."""
    from oracle import discretize as D
    from oracle import pipeline as P
    from paper_2609_20964_amd.serving import Server
    rng = np.random.default_rng(611)
    spec = [(32, 5000, "grad"), (64, 20000, None), (128, 30000, "full"), (48, 8000, None), (64, 12000, "grad")]
    reqs = []
    for i, (n, npts, kind) in enumerate(spec):
        c = synth.draw_star_coeffs(620 + i)
        semi, p = rng.uniform(0.12, 0.28, 3), rng.uniform(2, 5)
        x, nn = synth.star(c, npts, [621, i], semi_axes=semi, p=p)
        q = _band_queries(c, semi, p, 2048, [622, i])
        gphi = (rng.standard_normal(len(q)) / len(q)).astype(np.float32) if kind else None
        gnrm = (rng.standard_normal((len(q), 3)) / len(q)).astype(np.float32) if kind == "full" else None
        reqs.append((n, x, nn, q, gphi, gnrm))
    srv = Server(hbm_budget_bytes=8 << 30, max_inflight=4)
    tickets = [srv.submit(n, _cuda(x), _cuda(nn), _cuda(q), gphi=None if gp is None else _cuda(gp),
                          gnrm=None if gn is None else _cuda(gn), want_gq=gn is not None, rel_tol=1e-10,
                          max_iters=5000) for n, x, nn, q, gp, gn in reqs]
    results = _wait(srv, tickets, timeout=300.0)
    srv.close()
    spans = [(info["t_start"], info["t_done"]) for _, _, info in results]
    assert any(a[0] < b[0] < a[1] for a in spans for b in spans if a is not b), spans   # some ran beside others
    for (n, x, nn, q, gphi, gnrm), (st, outs, info) in zip(reqs, results):
        print(f"request {n}^3, {len(x)} points, grad {gphi is not None}, normal term {gnrm is not None}", flush=True)
        assert st == 0, info
        assert info["stats"]["rel_res"] <= 1e-10
        ref = P.Recon(D.Grid.unit(n), x, nn)
        phi_ref, n_ref = ref.sample(q)
        err = np.abs(outs["phi"].cpu().numpy() - phi_ref).max() * n
        ok = np.linalg.norm(n_ref, axis=1) > 0
        ang = angle(outs["nrm"].cpu().numpy()[ok], n_ref[ok])
        print(f"    phi {err:.2e} h, normal angle p99 {np.percentile(ang, 99):.2e}", flush=True)
        assert err <= 1e-4
        assert np.percentile(ang, 99) <= 1e-3 and ang.max() <= 2e-2
        if gphi is not None:
            gx_ref, gn_ref, gq_ref = ref.backward(q, gphi.astype(np.float64),
                                                   None if gnrm is None else gnrm.astype(np.float64))
            assert _close(outs["g_xyz"].cpu().numpy(), gx_ref)
            assert _close(outs["g_nrm"].cpu().numpy(), gn_ref)
            if gnrm is not None:
                assert _close(outs["g_q"].cpu().numpy(), gq_ref, comp_tol=3e-3)


def test_served_exact_quadrature_requests():
    """Requests for the exact-quadrature system beside 7-point ones: each
    served result against the oracle of its own system (phi at the queries
    within 1e-4 h; point gradients within 1e-3 relative in L2)."""
    from oracle import discretize as D
    from oracle import pipeline as P
    from paper_2609_20964_amd.serving import Server
    rng = np.random.default_rng(631)
    spec = [(32, 5000, "exact"), (40, 6000, "vertex"), (48, 8000, "exact")]
    reqs = []
    for i, (n, npts, quad) in enumerate(spec):
        c = synth.draw_star_coeffs(640 + i)
        semi, p = rng.uniform(0.15, 0.28, 3), rng.uniform(2, 4)
        x, nn = synth.star(c, npts, [641, i], semi_axes=semi, p=p)
        q = _band_queries(c, semi, p, 1024, [642, i])
        gphi = (rng.standard_normal(len(q)) / len(q)).astype(np.float32)
        reqs.append((n, x, nn, q, gphi, quad))
    srv = Server(hbm_budget_bytes=4 << 30, max_inflight=3)
    tickets = [srv.submit(n, _cuda(x), _cuda(nn), _cuda(q), gphi=_cuda(gp), rel_tol=1e-10, max_iters=5000,
                          quadrature=quad) for n, x, nn, q, gp, quad in reqs]
    results = _wait(srv, tickets, timeout=300.0)
    srv.close()
    for (n, x, nn, q, gphi, quad), (st, outs, info) in zip(reqs, results):
        assert st == 0, info
        ref = P.Recon(D.Grid.unit(n), x, nn, exact=quad == "exact")
        phi_ref, _ = ref.sample(q)
        err = np.abs(outs["phi"].cpu().numpy() - phi_ref).max() * n
        gx_ref, gn_ref, _ = ref.backward(q, gphi.astype(np.float64))
        print(f"{quad} {n}^3: phi {err:.2e} h", flush=True)
        assert err <= 1e-4
        assert _close(outs["g_xyz"].cpu().numpy(), gx_ref)
        assert _close(outs["g_nrm"].cpu().numpy(), gn_ref)
