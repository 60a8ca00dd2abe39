"""tvdeblur_solve_noalloc (work buffers in the library's static device array)
against tvdeblur_solve (work buffers in the handle) through the C-ABI: the
same kernels in the same order, so the images and statistics must agree
exactly (bit for bit), on two calls in a row where the second is smaller."""

import numpy as np
import pytest

from paper_1011_5964_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def prepared(p, prec):
    from paper_1011_5964_amd.lib import TVDeblur
    h = TVDeblur(p.v.shape[0], p.v.shape[1], prec)
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    h.transform()  # builds the handle (allocates its tables) ahead of the call
    return h


@pytest.mark.parametrize("prec", ["f32_mixed", "f64"])
def test_noalloc_matches_solve_two_calls(prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    big = synth.small_problem(n=96, ny=80, psf_size=9, sigma=1.5, n_outer=4, alpha=2e-3, beta=0.1)
    small = synth.small_problem(n=40, ny=36, psf_size=7, sigma=1.3, n_outer=3, alpha=1e-3, beta=0.1, seed=11)
    small.bc = "reflective"
    for label, p in (("96x80 AR", big), ("40x36 reflective (smaller, second call)", small)):
        print(f"case noalloc {prec} {label}", flush=True)
        h = prepared(p, prec)
        v = torch.tensor(p.v, dtype=dt, device="cuda")
        u_ref, st_ref = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        out = torch.full_like(v, float("nan"))
        u, st = h.solve_noalloc(v, out, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        print(f"  iters {st['inner_iters']} (solve: {st_ref['inner_iters']})", flush=True)
        assert u.data_ptr() == out.data_ptr()
        assert st["inner_iters"] == st_ref["inner_iters"]
        assert st["relres"] == st_ref["relres"]
        assert torch.equal(u, u_ref)
        # the handle's own path still gives the same result afterwards
        u2, _ = h.solve(v, p.alpha, p.beta, p.n_outer, p.inner_tol, p.max_inner, "x_d")
        assert torch.equal(u2, u_ref)


def test_noalloc_rejections():
    from paper_1011_5964_amd.lib import TVDeblur, TvdError
    p = synth.small_problem(n=32, n_outer=2)
    v = torch.tensor(p.v, dtype=torch.float32, device="cuda")
    out = torch.empty_like(v)
    # not built yet: refused instead of allocating
    h = TVDeblur(32, 32, "f32_mixed")
    h.set_psf(p.psf)
    h.set_bc(p.bc)
    with pytest.raises(TvdError) as e:
        h.solve_noalloc(v, out, p.alpha, p.beta, 2)
    assert e.value.name == "TVD_ESTATE"
    h.transform()
    h.set_profiling(1)
    with pytest.raises(TvdError) as e:
        h.solve_noalloc(v, out, p.alpha, p.beta, 2)
    assert e.value.name == "TVD_EINVAL"
    h.set_profiling(0)
    with pytest.raises(TvdError) as e:
        h.solve_noalloc(v, v, p.alpha, p.beta, 2)
    assert e.value.name == "TVD_EINVAL"
    u, st = h.solve_noalloc(v, out, p.alpha, p.beta, 2)
    assert st["outer_steps"] == 2 and np.isfinite(u.cpu().numpy()).all()
    # an image whose work buffers exceed the static array
    hb = TVDeblur(1024, 1024, "f32_mixed")
    hb.set_psf(synth.gaussian_psf(5, 1.0))
    hb.set_bc("antireflective")
    hb.transform()
    vb = torch.zeros((1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(TvdError) as e:
        hb.solve_noalloc(vb, torch.empty_like(vb), 1e-3, 0.1, 1)
    assert e.value.name == "TVD_ESIZE"
