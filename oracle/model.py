"""Oracle parameters, constants and spectrum integrals.

The paper fixes gamma = 5/3 (Sec. 2, ideal-gas EOS), the hydrogen threshold
h nu_0 = 13.6 eV (Sec. 2.2), and alpha_B(1e4 K) = 2.59e-13 cm^3/s (Sec. 4.5).
Everything else here (cross sections, helium data, the recombination
temperature exponent) is not printed in the paper and is a stated reading.

The grey/monochromatic reduction (Sec. 2.2, Eq. 11; Sec. 3.2.5, Eq. 45):
every term of the form integral f(nu) E_nu dnu becomes E times a constant
integral of f(nu) chi_E(nu) normalised by integral chi_E(nu), which is
computed once here with adaptive quadrature (scipy.integrate.quad).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import integrate

# CGS constants
C_LIGHT = 2.99792458e10
K_B = 1.380649e-16
M_H = 1.6735575e-24
EV = 1.602176634e-12
H_PLANCK = 6.62607015e-27
GAMMA = 5.0 / 3.0
ALPHA_B_1E4 = 2.59e-13       # case-B H recombination at 1e4 K (Sec. 4.5)
ALPHA_T_EXP = -0.7           # reading: alpha ~ T^-0.7 (not printed)
ALPHA_HEII_1E4 = 2.72e-13    # reading (placeholder He data)
ALPHA_HEIII_1E4 = 2.0 * ALPHA_B_1E4 * 4.0 ** 0.7   # hydrogenic Z=2 scaling
BETA_COOL = 0.75             # recombination cooling, reading
HNU_HI = 13.6 * EV
HNU_HEI = 24.6 * EV
HNU_HEII = 54.4 * EV
SIGMA_HI = 6.30e-18          # threshold cross sections (cm^2), readings
SIGMA_HEI = 7.42e-18
SIGMA_HEII = 1.575e-18
SIGMA_SB = 5.670374419e-5    # Stefan-Boltzmann constant (erg cm^-2 s^-1 K^-4)
A_RAD = 4.0 * SIGMA_SB / C_LIGHT   # radiation constant a_r
KAPPA_FLOOR_CELLS = 1.0e-3   # face opacity floor: 1e-3 per proper cell width
E_FLOOR = 1.0e-300           # guards E_face in R = |dE| / E


@dataclasses.dataclass
class Model:
    nspecies: int
    n: tuple                 # (nx, ny, nz)
    dx: float
    theta: float
    u_e: float
    u_E: float
    m: int                   # 0 monochromatic, 1 grey
    y_he: float
    isothermal: int
    T_iso: float
    K_gamma: np.ndarray      # (3,) photoionization constants per species
    K_kappa: np.ndarray      # (3,) opacity constants
    K_heat: np.ndarray       # (3,) photo-heating constants
    hnu_mean: float          # erg per source photon
    limiter_mode: int = 0    # 0: flux limiter; 1: constant D0 (test mode)
    D0: float = 0.0
    # LTE coupling (Sec. 2.1, Eq. 9): no species equations (nspecies = 0),
    # constant proper absorption and Planck-mean coefficients, fixed mean
    # particle mass mu m_H
    lte: int = 0
    kappa_lte: float = 0.0
    kappaP_lte: float = 0.0
    mu_lte: float = 0.6
    boundary: int = 0        # 0 periodic; 1 reflecting walls (zero flux on the domain faces);
                             # 2 x-left face at E_dirichlet (ghost cell), other faces reflect
    E_dirichlet: float = 0.0
    newton_tol: float = 1e-6
    newton_maxit: int = 20
    pcg_rtol: float = 1e-8
    pcg_maxit: int = 200
    mg_levels: int = 3
    mg_pre: int = 2
    mg_post: int = 2
    mg_coarse_sweeps: int = 8
    mg_fp32: int = 0
    pcg_forcing: float = 0.0 # inexact-Newton forcing factor (Sec. 3.2.1), 0: off
    krylov_restart: int = 30 # Schur solve: FGMRES restart length; 0: flexible PCG
    limiter_lag: int = 0     # 1: the flux limiter held at time level n for the step (a reading)
    box_size: int = 0        # source-subdomain correction in the preconditioner, 0: off
    box_levels: int = 3
    box_inner: int = 6
    box_coarse_sweeps: int = 0   # coarsest box level's sweeps, 0: mg_coarse_sweeps
    box_s_sweeps: int = 0    # red-black sweeps on the Schur matrix itself over each box

    @property
    def nv(self):
        return self.nspecies + 2

    @property
    def nb(self):
        return self.nspecies + 1

    @property
    def scales(self):
        """Unit constants u_v per unknown (e_c, x_1..x_Ns, E) (Sec. 3.2.2)."""
        return np.array([self.u_e] + [1.0] * self.nspecies + [self.u_E])


def _sigma(species, nu):
    thr = (HNU_HI, HNU_HEI, HNU_HEII)[species] / H_PLANCK
    s0 = (SIGMA_HI, SIGMA_HEI, SIGMA_HEII)[species]
    return 0.0 if nu < thr else s0 * (nu / thr) ** -3


def spectrum_constants(grey: int, T_B: float = 1e5):
    """(K_gamma, K_kappa, K_heat, hnu_mean) for the assumed spectrum chi_E.

    Monochromatic at 13.6 eV (delta spectrum): K_gamma = sigma_HI/(h nu_0),
    K_kappa = sigma_HI, no photo-heating (the photons sit at threshold), helium
    not ionized.  Grey: a T_B blackbody chi ~ nu^3/(exp(h nu/k T_B) - 1)
    restricted to nu >= nu_0 (Sec. 2.2), integrated per Eq. 45.
    """
    if not grey:
        return (np.array([SIGMA_HI / HNU_HI, 0.0, 0.0]),
                np.array([SIGMA_HI, 0.0, 0.0]),
                np.zeros(3), HNU_HI)
    nu0 = HNU_HI / H_PLANCK
    kT = K_B * T_B

    def chi(nu):
        return nu ** 3 / math.expm1(H_PLANCK * nu / kT)

    nu_hi = 60.0 * kT / H_PLANCK + 100 * nu0

    def quad(fn, lo):
        # split at the helium thresholds so the integrands are smooth per piece
        edges = [lo] + [e for e in (HNU_HEI / H_PLANCK, HNU_HEII / H_PLANCK) if e > lo] + [nu_hi]
        return sum(integrate.quad(fn, a, b, epsabs=0, epsrel=1e-13, limit=400)[0]
                   for a, b in zip(edges[:-1], edges[1:]))

    norm = quad(chi, nu0)
    Kg, Kk, Kh = np.zeros(3), np.zeros(3), np.zeros(3)
    for s in range(3):
        thr = (HNU_HI, HNU_HEI, HNU_HEII)[s] / H_PLANCK
        Kg[s] = quad(lambda nu: _sigma(s, nu) * chi(nu) / (H_PLANCK * nu), thr) / norm
        Kk[s] = quad(lambda nu: _sigma(s, nu) * chi(nu), thr) / norm
        Kh[s] = quad(lambda nu: _sigma(s, nu) * (1.0 - thr / nu) * chi(nu), thr) / norm
    photons = quad(lambda nu: chi(nu) / (H_PLANCK * nu), nu0)
    return Kg, Kk, Kh, norm / photons


def model_from_workload(w, **overrides) -> Model:
    Kg, Kk, Kh, hnu = spectrum_constants(w.grey, w.T_B)
    if w.nspecies == 1:
        Kg, Kk, Kh = Kg.copy(), Kk.copy(), Kh.copy()
        Kg[1:] = Kk[1:] = Kh[1:] = 0.0
    m = Model(nspecies=w.nspecies, n=(w.n, w.n, w.n), dx=w.dx, theta=w.theta,
              u_e=w.u_e, u_E=w.u_E, m=w.grey, y_he=w.y_he,
              isothermal=w.isothermal, T_iso=w.T_iso, K_gamma=Kg, K_kappa=Kk,
              K_heat=Kh, hnu_mean=hnu, newton_tol=w.newton_tol,
              newton_maxit=w.newton_maxit, pcg_rtol=w.pcg_rtol,
              pcg_maxit=w.pcg_maxit, mg_levels=w.mg_levels, mg_pre=w.mg_pre,
              mg_post=w.mg_post, mg_coarse_sweeps=w.mg_coarse_sweeps,
              mg_fp32=w.mg_fp32, pcg_forcing=w.pcg_forcing,
              krylov_restart=w.krylov_restart, limiter_lag=w.limiter_lag,
              box_size=w.box_size,
              box_levels=w.box_levels, box_inner=w.box_inner,
              box_coarse_sweeps=w.box_coarse_sweeps, box_s_sweeps=w.box_s_sweeps,
              lte=w.lte, kappa_lte=w.kappa_lte,
              kappaP_lte=w.kappaP_lte, mu_lte=w.mu_lte, boundary=w.boundary,
              E_dirichlet=w.E_dirichlet)
    return dataclasses.replace(m, **overrides) if overrides else m
