"""Thin ctypes binding of the C ABI in include/rt.h.

Argument marshalling only: every step of the method runs in the HIP library
(librt_gfx950.so).  PyTorch provides device memory (tensor.data_ptr()) and the
HIP stream.  Import fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt_gfx950.so")

RT_OK, RT_EINVAL, RT_EDEVICE, RT_ENOCONV, RT_ELINESEARCH, RT_ENONFINITE = 0, -1, -2, -3, -4, -5
RT_MAX_NEWTON = 32
STATUS_NAMES = {0: "RT_OK", -1: "RT_EINVAL", -2: "RT_EDEVICE", -3: "RT_ENOCONV",
                -4: "RT_ELINESEARCH", -5: "RT_ENONFINITE"}


class RtParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nspecies", ctypes.c_int32),
        ("dx", ctypes.c_double), ("theta", ctypes.c_double),
        ("u_e", ctypes.c_double), ("u_E", ctypes.c_double),
        ("grey", ctypes.c_int32), ("isothermal", ctypes.c_int32),
        ("T_iso", ctypes.c_double), ("y_he", ctypes.c_double),
        ("K_gamma", ctypes.c_double * 3), ("K_kappa", ctypes.c_double * 3),
        ("K_heat", ctypes.c_double * 3), ("hnu_mean", ctypes.c_double),
        ("limiter_mode", ctypes.c_int32), ("D0", ctypes.c_double),
        ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
        ("pcg_rtol", ctypes.c_double), ("pcg_maxit", ctypes.c_int32),
        ("mg_levels", ctypes.c_int32), ("mg_pre", ctypes.c_int32), ("mg_post", ctypes.c_int32),
        ("mg_coarse_sweeps", ctypes.c_int32), ("mg_fp32", ctypes.c_int32),
        ("max_sources", ctypes.c_int32), ("pcg_forcing", ctypes.c_double),
        ("box_size", ctypes.c_int32), ("box_levels", ctypes.c_int32), ("box_inner", ctypes.c_int32),
        ("box_coarse_sweeps", ctypes.c_int32),
        ("lte", ctypes.c_int32), ("kappa_lte", ctypes.c_double), ("kappaP_lte", ctypes.c_double),
        ("mu_lte", ctypes.c_double), ("boundary", ctypes.c_int32),
        ("E_dirichlet", ctypes.c_double), ("krylov_restart", ctypes.c_int32),
        ("limiter_lag", ctypes.c_int32), ("box_s_sweeps", ctypes.c_int32),
    ]


class RtCosmo(ctypes.Structure):
    _fields_ = [("a_old", ctypes.c_double), ("H_old", ctypes.c_double),
                ("a_new", ctypes.c_double), ("H_new", ctypes.c_double)]


class RtNewtonStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("newton_its", ctypes.c_int32),
        ("cg_its_total", ctypes.c_int32), ("vcycles", ctypes.c_int32),
        ("ls_trials", ctypes.c_int32), ("used_alt_guess", ctypes.c_int32),
        ("fnorm_guess", ctypes.c_double), ("fnorm_alt", ctypes.c_double),
        ("fnorm_final", ctypes.c_double),
        ("cg_its", ctypes.c_int32 * RT_MAX_NEWTON),
        ("lambda_", ctypes.c_double * RT_MAX_NEWTON),
        ("fnorm", ctypes.c_double * (RT_MAX_NEWTON + 1)),
    ]

    def as_dict(self):
        k = self.newton_its
        return dict(status=self.status, newton_its=k, cg_its_total=self.cg_its_total,
                    vcycles=self.vcycles, ls_trials=self.ls_trials,
                    used_alt_guess=self.used_alt_guess, fnorm_guess=self.fnorm_guess,
                    fnorm_alt=self.fnorm_alt, fnorm_final=self.fnorm_final,
                    cg_its=list(self.cg_its[:k]), lambdas=list(self.lambda_[:k]),
                    fnorms=list(self.fnorm[:k + 1]))


RT_K_NAMES = ["timelevel", "residual", "trial", "schur", "rbgs_fine", "rbgs_coarse",
              "mg_transfer", "mg_setup", "spmv", "cg_vector", "reduce", "box", "other"]


class RtKernelTiming(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32 * len(RT_K_NAMES)),
                ("total_ms", ctypes.c_double * len(RT_K_NAMES)),
                ("bytes", ctypes.c_double * len(RT_K_NAMES))]

    def as_dict(self):
        return {n: (self.count[i], self.total_ms[i], self.bytes[i])
                for i, n in enumerate(RT_K_NAMES)}


_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32
SIGNATURES = {
    "rt_workspace_bytes": [ctypes.POINTER(RtParams), ctypes.POINTER(ctypes.c_uint64)],
    "rt_create_grid": [ctypes.POINTER(RtParams), _P, ctypes.c_uint64, _P, ctypes.POINTER(_P)],
    "rt_destroy_grid": [_P],
    "rt_last_error": [_P],
    "rt_set_medium": [_P, _P, _P],
    "rt_set_sources": [_P, _I, _P, _P],
    "rt_time_level": [_P, _P, _D, ctypes.POINTER(RtCosmo), _P],
    "rt_eval_residual": [_P, _P, _P, _D, ctypes.POINTER(RtCosmo), _P, ctypes.POINTER(_D)],
    "rt_eval_residual_noalloc": [ctypes.POINTER(RtParams), _P, _P, _P, _P, _D,
                                 ctypes.POINTER(RtCosmo), _P, _P, ctypes.POINTER(_D),
                                 ctypes.c_char_p, ctypes.c_size_t],
    "rt_local_jacobian": [_P, _P, _D, ctypes.POINTER(RtCosmo), _P, _P, _P, _P],
    "rt_schur_form": [_P, _P, _P, _D, ctypes.POINTER(RtCosmo), _P],
    "rt_schur_get": [_P, _P, _P, _P, _P, _P, _P],
    "rt_schur_get_full": [_P, _P, _P, _P],
    "rt_set_operator": [_P, _P, _P, _P, _P],
    "rt_mg_vcycle": [_P, _P, _P],
    "rt_mg_pcg_solve": [_P, _P, _P, _D, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)],
    "rt_newton_step": [_P, _P, _P, _P, _D, ctypes.POINTER(RtCosmo),
                       ctypes.POINTER(RtNewtonStats)],
    "rt_fold_energy": [_P, _P, _P],
    "rt_timing": [_P, _I, ctypes.POINTER(RtKernelTiming)],
    "rt_timing_classes": [_P, ctypes.c_uint32],
    "rt_predict": [_P, _P, _D, ctypes.POINTER(RtCosmo), _P],
    "rt_time_error": [_P, _P, _P, _D, ctypes.POINTER(ctypes.c_double)],
    "rt_use_graphs": [_P, ctypes.c_int32],
    "rt_spectrum_constants": [_I, _D, _P, _P, _P, ctypes.POINTER(_D)],
    "rt_net_workspace_bytes": [_I, _I, _I, _I, ctypes.POINTER(ctypes.c_uint64)],
    "rt_net_create": [_I, _I, _I, _I, _P, ctypes.c_uint64, _P, ctypes.POINTER(_P)],
    "rt_net_destroy": [_P],
    "rt_net_last_error": [_P],
    "rt_net_num_params": [_P],
    "rt_net_set_params": [_P, _P, _I],
    "rt_net_get_params": [_P, _P, _I],
    "rt_net_forward": [_P, _P, _P, _P, _P, _P, _D, _D, _D, _P, _P],
    "rt_net_get_output": [_P, _P, _P],
    "rt_net_train_step": [_P, _P, _P, _P, _P, _P, _D, _D, _D, _P, _P, ctypes.c_float,
                          ctypes.POINTER(ctypes.c_float), _P],
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            "HIP library %s is missing: build it with `python -m paper_0901_1110_amd.build` "
            "(there is no fallback implementation)" % path)
    lib = ctypes.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name.endswith("last_error") else ctypes.c_int
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def spectrum_constants(grey: int, T_B: float = 1e5):
    Kg, Kk, Kh = (ctypes.c_double * 3)(), (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    hnu = ctypes.c_double()
    st = lib().rt_spectrum_constants(int(grey), float(T_B), Kg, Kk, Kh, ctypes.byref(hnu))
    if st != RT_OK:
        raise RtError(st, "rt_spectrum_constants")
    return list(Kg), list(Kk), list(Kh), hnu.value


def params_from_workload(w, **overrides) -> RtParams:
    """rt_params for a synth.Workload (spectrum constants from the library)."""
    Kg, Kk, Kh, hnu = spectrum_constants(w.grey, w.T_B)
    p = RtParams()
    p.nx = p.ny = p.nz = w.n
    p.nspecies = w.nspecies
    p.dx = w.dx
    p.theta = w.theta
    p.u_e, p.u_E = w.u_e, w.u_E
    p.grey = w.grey
    p.isothermal = w.isothermal
    p.T_iso = w.T_iso
    p.y_he = w.y_he
    p.K_gamma[:] = Kg
    p.K_kappa[:] = Kk
    p.K_heat[:] = Kh
    p.hnu_mean = hnu
    p.limiter_mode = 0
    p.D0 = 0.0
    p.newton_tol, p.newton_maxit = w.newton_tol, w.newton_maxit
    p.pcg_rtol, p.pcg_maxit = w.pcg_rtol, w.pcg_maxit
    p.mg_levels, p.mg_pre, p.mg_post = w.mg_levels, w.mg_pre, w.mg_post
    p.mg_coarse_sweeps, p.mg_fp32 = w.mg_coarse_sweeps, w.mg_fp32
    p.max_sources = max(64, w.nsources)
    p.pcg_forcing = w.pcg_forcing
    p.box_size, p.box_levels, p.box_inner = w.box_size, w.box_levels, w.box_inner
    p.box_coarse_sweeps = w.box_coarse_sweeps
    p.lte, p.kappa_lte, p.kappaP_lte, p.mu_lte = w.lte, w.kappa_lte, w.kappaP_lte, w.mu_lte
    p.boundary, p.E_dirichlet = w.boundary, w.E_dirichlet
    p.krylov_restart = w.krylov_restart
    p.limiter_lag = w.limiter_lag
    p.box_s_sweeps = w.box_s_sweeps
    for k, v in overrides.items():
        if k in ("K_gamma", "K_kappa", "K_heat"):
            getattr(p, k)[:] = list(v)
        else:
            setattr(p, k, v)
    return p


def cosmo(c) -> RtCosmo:
    return RtCosmo(*[float(v) for v in c])


def eval_residual_noalloc(params: RtParams, nH, eh, U, gn, dt, c, f=None, norm=True,
                          stream=None):
    """rt_eval_residual_noalloc: the residual (and its RMS norm) without a
    grid or workspace; f is allocated here only when not given."""
    f = torch.empty_like(U) if f is None else f
    st = stream if stream is not None else torch.cuda.current_stream(U.device)
    cc = cosmo(c)
    r = ctypes.c_double()
    msg = ctypes.create_string_buffer(512)
    status = lib().rt_eval_residual_noalloc(ctypes.byref(params), _ptr(nH), _ptr(eh), _ptr(U),
                                            _ptr(gn), float(dt), ctypes.byref(cc),
                                            ctypes.c_void_p(st.cuda_stream), _ptr(f),
                                            ctypes.byref(r) if norm else None, msg,
                                            len(msg))
    if status != RT_OK:
        raise RtError(status, "rt_eval_residual_noalloc: %s" % msg.value.decode())
    return f, (r.value if norm else None)


class RtGrid:
    """Owner of an rt_grid and its caller-allocated device workspace."""

    def __init__(self, params: RtParams, device="cuda", stream=None):
        L = lib()
        nbytes = ctypes.c_uint64()
        st = L.rt_workspace_bytes(ctypes.byref(params), ctypes.byref(nbytes))
        if st != RT_OK:
            raise RtError(st, "rt_workspace_bytes: invalid parameters")
        self.params = params
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = L.rt_create_grid(ctypes.byref(params), _ptr(self.ws), self.ws.numel(),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != RT_OK:
            raise RtError(st, "rt_create_grid")
        self.h = h
        self.N = params.nx * params.ny * params.nz
        self.nv = params.nspecies + 2
        self.nb = params.nspecies + 1
        self.shape = (params.nx, params.ny, params.nz)
        self._keep = []

    def _check(self, st, name):
        if st != RT_OK:
            raise RtError(st, "%s: %s" % (name, lib().rt_last_error(self.h).decode()))
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().rt_destroy_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_state(self):
        return torch.empty((self.nv,) + self.shape, dtype=torch.float64, device=self.device)

    def new_field(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    # -- entry points (same names as the C ABI) --
    def rt_set_medium(self, nH, eh):
        self._keep = [nH, eh]
        return self._check(lib().rt_set_medium(self.h, _ptr(nH), _ptr(eh)), "rt_set_medium")

    def rt_set_sources(self, cells, Q):
        import numpy as np
        c = np.ascontiguousarray(cells, dtype=np.int64)
        q = np.ascontiguousarray(Q, dtype=np.float64)
        return self._check(lib().rt_set_sources(self.h, int(c.size),
                                                c.ctypes.data_as(ctypes.c_void_p),
                                                q.ctypes.data_as(ctypes.c_void_p)),
                           "rt_set_sources")

    def rt_time_level(self, Un, dt, c, gn=None):
        gn = self.new_state() if gn is None else gn
        cc = cosmo(c)
        self._check(lib().rt_time_level(self.h, _ptr(Un), float(dt), ctypes.byref(cc), _ptr(gn)),
                    "rt_time_level")
        return gn

    def rt_predict(self, Un, dt, c, Up=None):
        """Explicit predictor of the step (projected forward Euler update)."""
        Up = self.new_state() if Up is None else Up
        cc = cosmo(c)
        self._check(lib().rt_predict(self.h, _ptr(Un), float(dt), ctypes.byref(cc), _ptr(Up)),
                    "rt_predict")
        return Up

    def rt_time_error(self, Unew, Upred, p=0.0):
        """Time-error estimate between the new state and the predictor (p <= 0: max norm)."""
        out = ctypes.c_double(0.0)
        self._check(lib().rt_time_error(self.h, _ptr(Unew), _ptr(Upred), float(p), ctypes.byref(out)),
                    "rt_time_error")
        return out.value

    def rt_eval_residual(self, U, gn, dt, c, f=None, norm=True):
        f = self.new_state() if f is None else f
        cc = cosmo(c)
        r = ctypes.c_double()
        self._check(lib().rt_eval_residual(self.h, _ptr(U), _ptr(gn), float(dt), ctypes.byref(cc),
                                           _ptr(f), ctypes.byref(r) if norm else None),
                    "rt_eval_residual")
        return f, (r.value if norm else None)

    def rt_local_jacobian(self, U, dt, c):
        nb = self.nb
        M = torch.empty((nb, nb) + self.shape, dtype=torch.float64, device=self.device)
        Uc = torch.empty((nb,) + self.shape, dtype=torch.float64, device=self.device)
        Lr = torch.empty((nb,) + self.shape, dtype=torch.float64, device=self.device)
        dl = self.new_field()
        cc = cosmo(c)
        self._check(lib().rt_local_jacobian(self.h, _ptr(U), float(dt), ctypes.byref(cc), _ptr(M),
                                            _ptr(Uc), _ptr(Lr), _ptr(dl)), "rt_local_jacobian")
        return M, Uc, Lr, dl

    def rt_schur_form(self, U, f, dt, c, b=None):
        b = self.new_field() if b is None else b
        cc = cosmo(c)
        self._check(lib().rt_schur_form(self.h, _ptr(U), _ptr(f), float(dt), ctypes.byref(cc),
                                        _ptr(b)), "rt_schur_form")
        return b

    def rt_schur_get(self):
        nb = self.nb
        ftM = torch.empty((nb,) + self.shape, dtype=torch.float64, device=self.device)
        W = torch.empty_like(ftM)
        out = [self.new_field() for _ in range(4)]
        self._check(lib().rt_schur_get(self.h, _ptr(ftM), _ptr(W), *[_ptr(t) for t in out]),
                    "rt_schur_get")
        return dict(ftM=ftM, W=W, diag=out[0], cx=out[1], cy=out[2], cz=out[3])

    def rt_schur_get_full(self):
        fw = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        bw = torch.empty_like(fw)
        pdiag = self.new_field()
        self._check(lib().rt_schur_get_full(self.h, _ptr(fw), _ptr(bw), _ptr(pdiag)),
                    "rt_schur_get_full")
        return dict(fw=fw, bw=bw, pdiag=pdiag)

    def rt_set_operator(self, diag, cx, cy, cz):
        return self._check(lib().rt_set_operator(self.h, _ptr(diag), _ptr(cx), _ptr(cy), _ptr(cz)),
                           "rt_set_operator")

    def rt_mg_vcycle(self, r, z=None):
        z = self.new_field() if z is None else z
        self._check(lib().rt_mg_vcycle(self.h, _ptr(r), _ptr(z)), "rt_mg_vcycle")
        return z

    def rt_mg_pcg_solve(self, b, rtol, maxit, s=None):
        s = self.new_field() if s is None else s
        its, rr = ctypes.c_int32(), ctypes.c_double()
        self._check(lib().rt_mg_pcg_solve(self.h, _ptr(b), _ptr(s), float(rtol), int(maxit),
                                          ctypes.byref(its), ctypes.byref(rr)), "rt_mg_pcg_solve")
        return s, its.value, rr.value

    def rt_timing(self, enable):
        """enable=True starts per-launch event timing; False returns
        {class: (launches, ms, algorithmic bytes)}."""
        out = RtKernelTiming()
        self._check(lib().rt_timing(self.h, 1 if enable else 0, None if enable else ctypes.byref(out)),
                    "rt_timing")
        return None if enable else out.as_dict()

    def rt_timing_classes(self, classes=None):
        """Time only the named kernel classes (None: all) from now on."""
        if classes is None:
            mask = 0xFFFFFFFF
        else:
            mask = 0
            for c in classes:
                mask |= 1 << RT_K_NAMES.index(c)
        self._check(lib().rt_timing_classes(self.h, mask), "rt_timing_classes")

    def rt_use_graphs(self, enable):
        """False: the subdomain correction is issued launch by launch (no graph)."""
        self._check(lib().rt_use_graphs(self.h, 1 if enable else 0), "rt_use_graphs")

    def rt_fold_energy(self, U, eh):
        return self._check(lib().rt_fold_energy(self.h, _ptr(U), _ptr(eh)), "rt_fold_energy")

    def rt_newton_step(self, Un, U, dt, c, Ualt=None, raise_on_fail=False):
        """Returns the stats dict; U (in: guess) holds U^{n+1} afterwards."""
        cc = cosmo(c)
        st = RtNewtonStats()
        code = lib().rt_newton_step(self.h, _ptr(Un), _ptr(U), _ptr(Ualt), float(dt),
                                    ctypes.byref(cc), ctypes.byref(st))
        if code == RT_EINVAL or code == RT_EDEVICE or (raise_on_fail and code != RT_OK):
            self._check(code, "rt_newton_step")
        return st.as_dict()


class RtNet:
    """Owner of an rt_net (learned initial guess) and its device workspace."""

    def __init__(self, nspecies, shape, device="cuda", stream=None):
        L = lib()
        nx, ny, nz = shape
        nbytes = ctypes.c_uint64()
        st = L.rt_net_workspace_bytes(nspecies, nx, ny, nz, ctypes.byref(nbytes))
        if st != RT_OK:
            raise RtError(st, "rt_net_workspace_bytes: unsupported shape %s" % (shape,))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        st = L.rt_net_create(nspecies, nx, ny, nz, _ptr(self.ws), self.ws.numel(),
                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != RT_OK:
            raise RtError(st, "rt_net_create")
        self.h = h
        self.ns = nspecies
        self.shape = tuple(shape)
        self.N = nx * ny * nz
        self.nin = 2 * (nspecies + 2) + 1
        self.nout = nspecies + 2
        self.P = L.rt_net_num_params(h)

    def _check(self, st, name):
        if st != RT_OK:
            raise RtError(st, "%s: %s" % (name, lib().rt_net_last_error(self.h).decode()))

    def close(self):
        if getattr(self, "h", None):
            lib().rt_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        import numpy as np
        t = np.ascontiguousarray(theta, dtype=np.float32)
        self._check(lib().rt_net_set_params(self.h, t.ctypes.data_as(ctypes.c_void_p), int(t.size)),
                    "rt_net_set_params")

    def get_params(self):
        import numpy as np
        t = np.empty(self.P, dtype=np.float32)
        self._check(lib().rt_net_get_params(self.h, t.ctypes.data_as(ctypes.c_void_p), self.P),
                    "rt_net_get_params")
        return t

    def forward(self, Un, Unm1, en, enm1, nH, nH_mean, u_e, u_E, eh, Uguess):
        self._check(lib().rt_net_forward(self.h, _ptr(Un), _ptr(Unm1), _ptr(en), _ptr(enm1),
                                         _ptr(nH), float(nH_mean), float(u_e), float(u_E),
                                         _ptr(eh), _ptr(Uguess)), "rt_net_forward")
        return Uguess

    def get_output(self):
        out = torch.empty((self.nout,) + self.shape, dtype=torch.float32, device=self.device)
        feat = torch.empty((16,) + self.shape, dtype=torch.float32, device=self.device)
        self._check(lib().rt_net_get_output(self.h, _ptr(out), _ptr(feat)), "rt_net_get_output")
        return out, feat

    def train_step(self, Un, Unm1, en, enm1, nH, nH_mean, u_e, u_E, Unp1, enp1, lr, want_grad=False):
        import numpy as np
        loss = ctypes.c_float()
        grad = np.empty(self.P, dtype=np.float32) if want_grad else None
        self._check(lib().rt_net_train_step(
            self.h, _ptr(Un), _ptr(Unm1), _ptr(en), _ptr(enm1), _ptr(nH), float(nH_mean),
            float(u_e), float(u_E), _ptr(Unp1), _ptr(enp1), float(lr), ctypes.byref(loss),
            grad.ctypes.data_as(ctypes.c_void_p) if want_grad else None), "rt_net_train_step")
        return (loss.value, grad) if want_grad else loss.value
