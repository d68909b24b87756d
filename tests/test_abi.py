"""Host-side checks of the C ABI (no GPU needed).

The library loads, exports every function include/rt.h declares, the ctypes
struct layouts match the header's field order, parameter validation rejects
bad input before touching a device, and the library's own spectrum
quadrature agrees with the oracle's (scipy) integrals.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import model as om
from paper_0901_1110_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "rt.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(rt_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported():
    lib = b.load_library()
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in b.SIGNATURES, name


def test_params_layout_matches_header():
    txt = open(os.path.join(ROOT, "include", "rt.h")).read()
    body = txt[txt.index("typedef struct rt_params {"):txt.index("} rt_params;")]
    fields = []
    for line in body.splitlines()[1:]:
        line = line.split("/*")[0].strip().rstrip(";")
        if not line:
            continue
        decl = line.split(None, 1)[1]
        for part in decl.split(","):
            fields.append(part.strip().split("[")[0])
    assert fields == [f[0] for f in b.RtParams._fields_]


def test_workspace_bytes_and_validation():
    lib = b.load_library()
    p = b.params_from_workload(synth.CFG_256)
    n = ctypes.c_uint64()
    assert lib.rt_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == b.RT_OK
    N = 256 ** 3
    # the FP64 fields the step needs (about 40 per cell, with the colour-split
    # copies of the FP64 finest level), plus the 2 m + 1
    # Krylov vectors of FGMRES(m)
    m = p.krylov_restart
    assert m == 30
    assert (38 + 2 * m + 1) * 8 * N < n.value < (50 + 2 * m + 1) * 8 * N
    for field, bad in (("nspecies", 2), ("nx", 250), ("theta", 0.0), ("mg_levels", 8),
                       ("u_E", -1.0), ("newton_maxit", 99), ("limiter_mode", 5),
                       ("nspecies", 0), ("lte", 1), ("lte", 2), ("boundary", 3),
                       ("boundary", -1), ("pcg_forcing", -1e-6), ("box_size", 20),
                       ("box_size", 512), ("krylov_restart", -1), ("krylov_restart", 31),
                       ("box_s_sweeps", -1), ("box_s_sweeps", 257)):
        q = b.params_from_workload(synth.CFG_256, **{field: bad})
        assert lib.rt_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == b.RT_EINVAL, field
        h = ctypes.c_void_p()
        assert lib.rt_create_grid(ctypes.byref(q), ctypes.c_void_p(256), 1 << 40, None,
                                  ctypes.byref(h)) == b.RT_EINVAL
    # the box sweeps on S make the preconditioner non-symmetric: FGMRES only
    q = b.params_from_workload(synth.CFG_256, box_s_sweeps=2, krylov_restart=0)
    assert lib.rt_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == b.RT_EINVAL
    q = b.params_from_workload(synth.CFG_256, box_s_sweeps=2)
    assert lib.rt_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == b.RT_OK
    # combinations: LTE needs nspecies = 0 and finite coefficients; a held
    # face needs a finite, non-negative value
    for over in (dict(lte=1, nspecies=0, mu_lte=0.0), dict(lte=1, nspecies=0, kappa_lte=-1.0),
                 dict(lte=1, nspecies=0, kappaP_lte=float("nan")),
                 dict(boundary=2, E_dirichlet=-1.0), dict(boundary=2, E_dirichlet=float("inf")),
                 dict(box_size=32, box_levels=2, box_coarse_sweeps=-1),
                 dict(box_size=32, box_levels=2, box_inner=0)):
        q = b.params_from_workload(synth.CFG_256, **over)
        assert lib.rt_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == b.RT_EINVAL, over
    for over in (dict(lte=1, nspecies=0, kappa_lte=1e-6, kappaP_lte=1e-6, mu_lte=0.6),
                 dict(boundary=1), dict(boundary=2, E_dirichlet=1.0)):
        q = b.params_from_workload(synth.CFG_256, **over)
        assert lib.rt_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == b.RT_OK, over
    # a workspace that is too short is rejected before any device work
    h = ctypes.c_void_p()
    assert lib.rt_create_grid(ctypes.byref(p), ctypes.c_void_p(256), 1024, None,
                              ctypes.byref(h)) == b.RT_EINVAL


@pytest.mark.parametrize("grey,T_B", [(0, 1e5), (1, 1e5), (1, 3e4)])
def test_spectrum_constants_match_oracle(grey, T_B):
    Kg, Kk, Kh, hnu = b.spectrum_constants(grey, T_B)
    oKg, oKk, oKh, ohnu = om.spectrum_constants(grey, T_B)
    for got, ref in ((Kg, oKg), (Kk, oKk), (Kh, oKh)):
        assert np.allclose(got, ref, rtol=1e-9, atol=0)
    assert abs(hnu / ohnu - 1) < 1e-9
