"""Seeded synthetic workloads shared by the oracle, the tests and the bench.

This module only *describes* inputs: grid sizes, physical parameters, solver
settings, and seeded random fields / source lists.  It holds none of the
arithmetic of the implicit method (no rates, no residual, no solver), so that
the CPU oracle and the HIP path can both consume the same inputs while sharing
no code of the method itself.

Physical inputs follow the paper's ionization tests: the isothermal HII region
of Sec. 4.5 (N_gamma = 5e48 photons/s at 13.6 eV, n_H = 1e-3 cm^-3,
E0 = 1e-20 erg cm^-3, T = 1e4 K) and the cosmological I-front / weak-scaling
setup of Secs. 4.6 and 4.8 (64^3 cells per 80 kpc subgrid, so 1.25 kpc
proper cells, starting at a = 0.1 here).  The density field, source
placement and source luminosities are synthetic stand-ins for those
workloads (no data set is used).

All densities and radiation energies are *comoving* (proper value times a^3);
cell widths are comoving centimetres.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

KPC_CM = 3.0857e21          # cm per kiloparsec
# Specific gas energy (erg/g) of gamma=5/3 hydrogen at T = 1e4 K with neutral
# fraction 0.9999 (mean molecular weight 1/(2 - 0.9999)); a literal input value.
E_GAS_1E4K_X09999 = 1.2375915362035662e12
# Hubble constant used for the expanding-universe workloads: 50 km/s/Mpc (the
# q0 = 0.5 cases of Sec. 4.6), in 1/s.
H0_S = 50.0e5 / (1.0e3 * KPC_CM)


def eds_time(a: float) -> float:
    """Cosmic time of scale factor a in an Einstein-de Sitter universe."""
    return 2.0 / (3.0 * H0_S) * a ** 1.5


def eds_scale_factor(t: float) -> float:
    """Inverse of eds_time."""
    return (1.5 * H0_S * t) ** (2.0 / 3.0)


def eds_hubble(a: float) -> float:
    """adot/a in an Einstein-de Sitter universe."""
    return H0_S * a ** -1.5


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                      # cells per side (cubic, periodic)
    dx: float                   # comoving cell width (cm)
    nspecies: int = 1           # 1: HI ; 3: HI, HeI, HeII
    grey: int = 0               # 0: monochromatic 13.6 eV (m=0); 1: T_B blackbody (m=1)
    T_B: float = 1.0e5          # blackbody temperature of the grey spectrum (K)
    y_he: float = 0.0           # n_He / n_H
    theta: float = 1.0
    dt: float = 1.0e11          # s (fixed step)
    steps: int = 1
    nH_mean: float = 1.0e-3     # comoving cm^-3
    sigma_ln: float = 0.0       # lognormal width; 0 -> uniform medium
    seed: int = 0
    nsources: int = 1
    Q: float = 5.0e48           # photons/s (single centred source)
    logQ_range: Tuple[float, float] = (47.0, 49.0)
    centred: bool = True
    x0: Tuple[float, ...] = (0.9999,)
    E0: float = 1.0e-20         # comoving erg cm^-3
    eh0: float = E_GAS_1E4K_X09999
    a_start: float = 1.0        # scale factor at the first step (1: static)
    a_end: Optional[float] = None   # scale factor after the last step (None: static)
    u_e: float = E_GAS_1E4K_X09999
    u_E: float = 1.0e-20
    isothermal: int = 0
    T_iso: float = 1.0e4
    newton_tol: float = 1.0e-6
    newton_maxit: int = 20
    pcg_rtol: float = 1.0e-8
    pcg_maxit: int = 200
    pcg_forcing: float = 0.0   # > 0: the Krylov solve also stops at ||r|| <= pcg_forcing ||f(U_k)||
    krylov_restart: int = 30   # Schur solve: FGMRES restart length; 0: flexible PCG
    limiter_lag: int = 0       # 1: the flux limiter held at time level n for the step
    box_size: int = 0          # > 0: subdomain correction on a box around each source
    box_levels: int = 3
    box_inner: int = 6
    box_coarse_sweeps: int = 0  # coarsest box level's sweeps (0: mg_coarse_sweeps)
    box_s_sweeps: int = 0       # red-black sweeps on the Schur matrix over each box
    lte: int = 0                # 1: LTE coupling, no species (nspecies = 0)
    kappa_lte: float = 0.0      # LTE absorption coefficient (proper, 1/cm)
    kappaP_lte: float = 0.0     # LTE Planck-mean coefficient (proper, 1/cm)
    mu_lte: float = 0.6         # LTE mean particle mass (units of m_H)
    boundary: int = 0           # 0: periodic; 1: reflecting walls; 2: x-left Dirichlet
    E_dirichlet: float = 0.0    # boundary 2: comoving E of the x-left ghost cell
    corner_source: bool = False  # single source in cell (0, 0, 0) instead of the centre
    mg_levels: int = 3
    mg_pre: int = 2
    mg_post: int = 2
    mg_coarse_sweeps: int = 8
    mg_fp32: int = 0

    @property
    def nv(self) -> int:
        return self.nspecies + 2

    @property
    def ncells(self) -> int:
        return self.n ** 3

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    def cosmology(self, step: int):
        """(a_old, H_old, a_new, H_new) for time step `step` (0-based)."""
        if self.a_end is None:
            return (1.0, 0.0, 1.0, 0.0) if self.a_start == 1.0 else (
                self.a_start, 0.0, self.a_start, 0.0)
        t0 = eds_time(self.a_start)
        a_o = eds_scale_factor(t0 + step * self.dt)
        a_n = eds_scale_factor(t0 + (step + 1) * self.dt)
        return (a_o, eds_hubble(a_o), a_n, eds_hubble(a_n))

    def cosmology_at(self, t: float, dt: float):
        """(a_old, H_old, a_new, H_new) for a step of length dt starting a time
        t after the first step's start (variable steps)."""
        if self.a_end is None:
            return self.cosmology(0)
        t0 = eds_time(self.a_start)
        a_o = eds_scale_factor(t0 + t)
        a_n = eds_scale_factor(t0 + t + dt)
        return (a_o, eds_hubble(a_o), a_n, eds_hubble(a_n))


# --- the five workloads -----------------------------------------------------
# Periodic 13.2 kpc box (twice the 6.6 kpc octant of Sec. 4.5, so a centred
# source in a periodic box mirrors the paper's corner source).
_BOX_ILIEV = 13.2 * KPC_CM

# 32^3, one step, plain FP64.
CFG_SMALL = Workload(name="hii_32", n=32, dx=_BOX_ILIEV / 32, mg_levels=3)

# 128^3 expanding lognormal medium with 16 sources, 20 steps from a = 0.1.
# Cells are 1.25 kpc proper at a = 0.1 (12.5 kpc comoving); comoving density
# and radiation energy are the proper values times a^3 = 1e-3.  A step spans
# hundreds of light-crossings of a cell; Newton on the residual with the
# flux limiter at the iterate does not converge here (it stalls in the line
# search), so this workload holds the limiter at time level n for each step.
_A0 = 0.1
_DT_COSMO = 5.0e13
CFG_COSMO = Workload(
    name="cosmo_lognormal_128", n=128, dx=1.25 * KPC_CM / _A0, dt=_DT_COSMO,
    steps=20, nH_mean=1.0e-3 * _A0 ** 3, sigma_ln=1.0, seed=2, nsources=16,
    centred=False, E0=1.0e-20 * _A0 ** 3, u_E=1.0e-20 * _A0 ** 3,
    a_start=_A0, a_end=None, mg_levels=4, limiter_lag=1)
# a_end is filled so that the cosmology helper integrates EdS over the steps.
CFG_COSMO = CFG_COSMO.replace(
    a_end=eds_scale_factor(eds_time(_A0) + CFG_COSMO.steps * _DT_COSMO))

# 256^3 single centred source; the measured workload (plain and mixed).
CFG_256 = Workload(name="hii_256", n=256, dx=_BOX_ILIEV / 256, steps=200,
                   mg_levels=5)

# 512^3 H+He, lognormal sigma 1.5, 64 sources, a = 0.1 -> 0.125 over 50 steps
# (the limiter held at time level n, as for the 128^3 expanding medium).
_A1 = 0.125
_DT_HHE = (2.0 / (3.0 * H0_S)) * (_A1 ** 1.5 - _A0 ** 1.5) / 50
CFG_HHE = Workload(
    name="hhe_lognormal_512", n=512, dx=1.25 * KPC_CM / _A0, nspecies=3,
    grey=1, y_he=0.24 / (4 * 0.76), dt=_DT_HHE, steps=50,
    nH_mean=1.0e-3 * _A0 ** 3, sigma_ln=1.5, seed=5, nsources=64,
    centred=False, x0=(0.9999, 0.9999, 1.0e-4), E0=1.0e-20 * _A0 ** 3,
    u_E=1.0e-20 * _A0 ** 3, a_start=_A0, a_end=_A1, mg_levels=6, mg_fp32=1, limiter_lag=1)

# Cosmological I-front of Sec. 4.6, case q0 = 0.5, z_i = 4: uniform hydrogen
# of proper density 1.175e-28 g/cm^3 at z_i (n_H = rho / m_H), isothermal at
# 1e4 K, the single 5e48 photons/s source of Sec. 4.5, E = 1e-35 erg/cm^3 and
# no ionization at the start; Einstein-de Sitter expansion from a = 0.2.  The
# paper's 80 kpc (proper at z_i) box, periodic with a centred source, 50
# steps of 2e15 s (to z = 1.08, while the front stays inside the box).  A
# step spans thousands of light-crossings of a cell: the limiter is held at
# time level n (as for the expanding lognormal medium).
_A_SG = 0.2
_M_H_G = 1.6735575e-24       # g per hydrogen atom (input conversion only)
_DT_SG = 2.0e15
CFG_SG = Workload(
    name="sg_q05_z4", n=128, dx=80.0 * KPC_CM / _A_SG / 128, dt=_DT_SG, steps=50,
    nH_mean=1.175e-28 / _M_H_G * _A_SG ** 3, x0=(1.0,), E0=1.0e-35 * _A_SG ** 3,
    u_E=1.0e-20 * _A_SG ** 3, isothermal=1, T_iso=1.0e4, a_start=_A_SG,
    a_end=eds_scale_factor(eds_time(_A_SG) + 50 * _DT_SG), mg_levels=4, limiter_lag=1)

# Matter-radiation equilibration of Sec. 4.2 (LTE coupling, Eq. 9): a uniform
# medium of one opacity 4e-8 /cm (absorption and Planck mean), density
# 1e-7 g/cm^3 (n_H = rho / m_H), mean particle mass 0.6 m_H, E = 1e12
# erg/cm^3, gas energy density 1e10 (hot start) or 1e2 (cold start) erg/cm^3,
# 4^3 periodic cells, no sources, 250 steps of 1e-9 s to t = 2.5e-7 s.
_RHO_TS = 1.0e-7
CFG_TS_HOT = Workload(
    name="ts_hot", n=4, dx=1.0, nspecies=0, x0=(), lte=1, kappa_lte=4.0e-8, kappaP_lte=4.0e-8,
    mu_lte=0.6, nH_mean=_RHO_TS / _M_H_G, Q=0.0, E0=1.0e12, u_E=1.0e12,
    eh0=1.0e10 / _RHO_TS, u_e=1.0e15, dt=1.0e-9, steps=250, mg_levels=1, newton_tol=1e-10)
CFG_TS_COLD = CFG_TS_HOT.replace(name="ts_cold", eh0=1.0e2 / _RHO_TS)

# Free-streaming radiation of Sec. 4.1: a transparent medium (constant
# opacities 1e-6 /cm; the LTE terms are then negligible), E = 1e-4 erg/cm^3,
# E = 1 erg/cm^3 held on the x-left face, the other faces reflecting, a 1 cm
# cube, to t = 8.3391 ps (a quarter of the light-crossing time) in 100 steps.
# The gas (1e-7 g/cm^3, mu = 0.6, ~1e4 K) only sets the LTE terms.
CFG_FS = Workload(
    name="free_stream_128", n=128, dx=1.0 / 128, nspecies=0, x0=(), lte=1, kappa_lte=1.0e-6,
    kappaP_lte=1.0e-6, mu_lte=0.6, nH_mean=_RHO_TS / _M_H_G, Q=0.0, E0=1.0e-4, u_E=1.0,
    eh0=2.07e12, u_e=2.07e12, dt=8.3391e-14, steps=100, mg_levels=5, boundary=2,
    E_dirichlet=1.0)

WORKLOADS = {w.name: w for w in (CFG_SMALL, CFG_COSMO, CFG_256, CFG_HHE, CFG_SG, CFG_TS_HOT,
                                 CFG_TS_COLD, CFG_FS)}


# --- generators ---------------------------------------------------------------
def lognormal_density(n: int, sigma_ln: float, mean: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Lognormal density with a Gaussian random field of power P(k) ~ k^-2.

    White noise is filtered by 1/|k| in Fourier space (zero mode removed),
    standardised, scaled by sigma_ln, exponentiated, and normalised so that
    the box mean is exactly `mean`.
    """
    if sigma_ln == 0.0:
        return np.full((n, n, n), mean)
    w = rng.standard_normal((n, n, n))
    W = np.fft.rfftn(w)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    k = 2.0 * np.pi * np.sqrt(k2) / n
    with np.errstate(divide="ignore"):
        filt = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k, 1.0), 0.0)
    g = np.fft.irfftn(W * filt, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std() * sigma_ln
    rho = np.exp(g)
    return mean * rho / rho.mean()


def sources_for(w: Workload, rng: Optional[np.random.Generator] = None):
    """(flat cell indices int64, luminosities photons/s) of the point sources.

    Flat index is (i*n + j)*n + k with k (z) fastest.  A centred source sits at
    cell (n/2, n/2, n/2).  Random sources are distinct cells drawn after the
    density field, with log10 Q uniform in `logQ_range`.
    """
    n = w.n
    if w.corner_source:
        return np.array([0], dtype=np.int64), np.array([w.Q], dtype=np.float64)
    if w.centred:
        c = n // 2
        return (np.array([(c * n + c) * n + c], dtype=np.int64),
                np.array([w.Q], dtype=np.float64))
    cells = rng.choice(n ** 3, size=w.nsources, replace=False).astype(np.int64)
    logQ = rng.uniform(w.logQ_range[0], w.logQ_range[1], size=w.nsources)
    return cells, 10.0 ** logQ


def initial_state(w: Workload):
    """Initial fields of a workload.

    Returns dict with
      U   : (nv, n, n, n) float64, rows (e_c, x_1..x_Ns, E); e_c = 0
      nH  : (n, n, n) comoving hydrogen number density
      eh  : (n, n, n) specific gas energy from the (frozen) hydrodynamic state
      src_cells, src_Q : point sources
    """
    rng = np.random.default_rng(w.seed)
    n = w.n
    nH = lognormal_density(n, w.sigma_ln, w.nH_mean, rng)
    cells, Q = sources_for(w, rng)
    U = np.empty((w.nv, n, n, n))
    U[0] = 0.0
    for s in range(w.nspecies):
        U[1 + s] = w.x0[s]
    U[-1] = w.E0
    eh = np.full((n, n, n), w.eh0)
    return dict(U=U, nH=nH, eh=eh, src_cells=cells, src_Q=Q)


def random_physical_state(n: int, nspecies: int, rng: np.random.Generator,
                          E_range=(1e-21, 1e-14), T_range=(5e3, 2e4),
                          nH_mean=1e-3, sigma_ln=0.5):
    """Random but physical cell states for Jacobian / residual parity cases.

    1 - x_HI is log-uniform in [1e-4, 0.9999]; E is log-uniform in E_range;
    helium fractions are a random split; e_h is drawn through a random target
    temperature using the same literal 1e4 K energy as a unit (so the gas
    specific energy spans roughly T_range).  e_c is a small random correction.
    """
    shape = (n, n, n)
    U = np.empty((nspecies + 2,) + shape)
    ion = 10.0 ** rng.uniform(-4.0, math.log10(0.9999), shape)
    U[1] = 1.0 - ion
    if nspecies == 3:
        u1 = rng.uniform(0.0, 1.0, shape)
        u2 = rng.uniform(0.0, 1.0, shape)
        U[2] = u1
        U[3] = (1.0 - u1) * u2
    U[-1] = 10.0 ** rng.uniform(math.log10(E_range[0]), math.log10(E_range[1]), shape)
    Tfac = rng.uniform(T_range[0], T_range[1], shape) / 1.0e4
    eh = E_GAS_1E4K_X09999 * Tfac
    U[0] = eh * rng.uniform(-0.05, 0.05, shape)
    g = rng.standard_normal(shape) * sigma_ln
    nH = nH_mean * np.exp(g)
    return U, nH, eh
