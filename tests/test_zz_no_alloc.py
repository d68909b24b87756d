"""The allocation-free residual entry point against rt_eval_residual on
grids of the same parameters: bit-identical fields and norm, on two calls
in a row (the second on a smaller grid, so the shared static partials hold
the first call's larger contents), and its rejections."""
import numpy as np
import pytest
import torch

from paper_0901_1110_amd.binding import (RT_EINVAL, RtError, RtGrid, eval_residual_noalloc,
                                         params_from_workload)

from tests.gpu_cases import dev, host, random_case

pytestmark = pytest.mark.gpu


def grid_residual(w, c):
    """rt_eval_residual on a grid (the existing entry point)."""
    p = params_from_workload(w)
    g = RtGrid(p)
    g.rt_set_medium(dev(c["nH"]), dev(c["eh"]))
    g.rt_set_sources(c["cells"], c["Q"])
    gn = g.rt_time_level(dev(c["Un"]), c["dt"], c["cosmo"])
    f, rms = g.rt_eval_residual(dev(c["U"]), gn, c["dt"], c["cosmo"])
    return p, g, gn, host(f), rms


@pytest.mark.parametrize("ns", [1, 3])
def test_noalloc_residual_matches_grid_entry_point(ns):
    results = []
    for n, seed in ((64, 71), (32, 72)):
        w, c = random_case(ns, n, 1.0 if n == 64 else 0.6, 1.0, seed)
        p, g, gn, f_ref, rms_ref = grid_residual(w, c)
        nH, eh, U = dev(c["nH"]), dev(c["eh"]), dev(c["U"])
        f = torch.full_like(U, float("nan"))
        f_out, rms = eval_residual_noalloc(p, nH, eh, U, gn, c["dt"], c["cosmo"], f)
        assert f_out is f
        f_h = host(f)
        assert np.isfinite(f_h).all()
        assert np.array_equal(f_h, f_ref)
        assert rms == rms_ref and np.isfinite(rms)
        # without the norm: the same field, no read-back
        f2, none = eval_residual_noalloc(p, nH, eh, U, gn, c["dt"], c["cosmo"], norm=False)
        assert none is None and np.array_equal(host(f2), f_ref)
        results.append(rms)
        g.close()
    assert results[0] != results[1]


def test_noalloc_rejections():
    w, c = random_case(1, 16, 1.0, 1.0, 73)
    p, g, gn, _, _ = grid_residual(w, c)
    nH, eh, U = dev(c["nH"]), dev(c["eh"]), dev(c["U"])
    lag = params_from_workload(w.replace(limiter_lag=1))
    with pytest.raises(RtError) as e:
        eval_residual_noalloc(lag, nH, eh, U, gn, c["dt"], c["cosmo"])
    assert e.value.status == RT_EINVAL and "limiter_lag" in str(e.value)
    # a grid whose partials exceed the static array: rejected before any
    # device work (the buffers passed are those of the small grid and are
    # never touched)
    big = params_from_workload(w)
    big.nx, big.ny, big.nz = 1024, 512, 512   # 2^20 stencil blocks, 32-bit indexable
    with pytest.raises(RtError) as e:
        eval_residual_noalloc(big, nH, eh, U, gn, c["dt"], c["cosmo"])
    assert e.value.status == RT_EINVAL and "static scratch" in str(e.value)
    g.close()
