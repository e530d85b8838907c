"""wg_poisson_solve_noalloc: the no-allocation Poisson solve against the handle's
wg_poisson_solve on the same right-hand sides (through the C ABI).

Both run the same kernels in the same launch configuration with deterministic
reductions, so the solutions should agree to the last bit; the test holds them
to the field tolerance (1e-5 relative) and reports exact equality.  Two calls
in a row on one device, the second on a smaller grid, so the second runs on the
scratch the first one left behind."""
import ctypes as C

import numpy as np
import pytest

from paper_2609_20964_amd import _lib as L


def _noalloc(grid, b, x, bc, opts, stream):
    st = L.WgStats()
    rc = L.lib().wg_poisson_solve_noalloc(C.byref(grid), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), bc,
                                          C.byref(opts), C.byref(st), C.c_void_p(stream))
    return rc, st


def test_noalloc_rejects_grids_beyond_its_scratch():
    # host-side size check: refused before any device work (fake pointers are never touched)
    g = L.make_grid(128)
    o = L.make_opts(1e-8, 500, False)
    st = L.WgStats()
    rc = L.lib().wg_poisson_solve_noalloc(C.byref(g), C.c_void_p(16), C.c_void_p(16), L.WG_BC_NEUMANN,
                                          C.byref(o), C.byref(st), None)
    assert rc == L.WG_EINVAL
    assert "maximum" in L.last_error()


@pytest.mark.gpu
def test_noalloc_matches_handle_solve_twice():
    import torch

    from paper_2609_20964_amd.recon import Recon

    rng = np.random.default_rng(707)
    stream = torch.cuda.current_stream().cuda_stream
    cases = [((64, 64, 64), L.WG_BC_NEUMANN), ((40, 28, 20), L.WG_BC_DIRICHLET)]
    for n, bc in cases:
        print(f"noalloc case grid {n} bc {bc}", flush=True)
        N = n[0] * n[1] * n[2]
        b = torch.from_numpy(rng.standard_normal(N).astype(np.float32)).cuda()
        o = L.make_opts(1e-10, 2000, False)
        r = Recon(n, 0)
        x_ref, st_ref = r.poisson(b, bc="neumann" if bc == L.WG_BC_NEUMANN else "dirichlet", rel_tol=1e-10,
                                  max_iters=2000)
        torch.cuda.synchronize()
        r.close()
        x = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
        rc, st = _noalloc(L.make_grid(n), b, x, bc, o, stream)
        assert rc == L.WG_OK, L.last_error()
        torch.cuda.synchronize()
        xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
        assert np.isfinite(xn).all()
        err = np.abs(xn - xr).max() / np.abs(xr).max()
        print(f"  iters {st.iters} vs {st_ref['iters']}, rel res {st.rel_res:.2e}, max rel diff {err:.2e}, "
              f"bit-identical {np.array_equal(xn, xr)}", flush=True)
        assert st.rel_res <= 1e-10
        assert st.iters == st_ref["iters"]
        assert err <= 1e-5
