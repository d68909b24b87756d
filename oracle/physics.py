"""Cell-local physics: temperature, rate coefficients and the local operators.

Paper Sec. 2.1 (model coupling) names the dependencies (kappa(n_i),
eta(T, n_i), G(E, n_i), Lambda(T, n_i), alpha(T), Gamma(E)) but gives the
non-LTE formulas only by reference, so the concrete rate model below is a
stated reading ("rate model v1").  The operators follow Sec. 3.2, Eqs. 26-28:

  L_e = 2 (adot/a) e_c - G + Lambda
  L_n = n_i Gamma_i - alpha_ij n_e n_j          (per species, as fractions)
  L_E = m (adot/a) E - 4 pi eta + c kappa E     (4 pi eta handled separately)

The unknowns are U = (e_c, x_1..x_Ns, E) with x_i = n_i / n_H (HI; and HeI,
HeII as fractions of n_He).  Rates use proper densities n/a^3 and E/a^3
(Eq. 37); comoving tendencies are a^3 times proper ones, so the fraction
equations carry no extra a-factor.  Every function accepts complex arrays so
that the Jacobian can be taken by complex-step differentiation.
"""
from __future__ import annotations

import numpy as np

from .model import (A_RAD, ALPHA_B_1E4, ALPHA_HEII_1E4, ALPHA_HEIII_1E4, ALPHA_T_EXP,
                    BETA_COOL, C_LIGHT, GAMMA, K_B, M_H)


def species_fractions(U, nspecies):
    """(x_HI, x_HeI, x_HeII, x_HeIII) from U; helium absent -> zeros."""
    xHI = U[1]
    if nspecies == 3:
        xHeI, xHeII = U[2], U[3]
        xHeIII = 1.0 - xHeI - xHeII
    else:
        xHeI = xHeII = xHeIII = 0.0 * xHI
    return xHI, xHeI, xHeII, xHeIII


def electron_fraction(xHI, xHeII, xHeIII, y):
    """n_e / n_H for ionized hydrogen and singly/doubly ionized helium."""
    return (1.0 - xHI) + y * (xHeII + 2.0 * xHeIII)


def temperature(e, xHI, xHeII, xHeIII, model):
    """Gas temperature from the specific gas energy (Sec. 2.1, Eq. 8).

    Reading of the garbled Eq. 8 with the EOS of Eq. 7 at v = 0:
    T = (gamma - 1) mu m_H e / k_B, mu = (1 + 4y) / (particles per H nucleus),
    particles per H nucleus = 1 + y + n_e/n_H.
    """
    y = model.y_he
    particles = 1.0 + y + electron_fraction(xHI, xHeII, xHeIII, y)
    return (GAMMA - 1.0) * (1.0 + 4.0 * y) * M_H * e / (K_B * particles)


def recombination_coefficients(T):
    """Case-B alpha(T) for HII, HeII, HeIII: anchor(1e4 K) * (T/1e4)^-0.7."""
    f = (T / 1.0e4) ** ALPHA_T_EXP
    return ALPHA_B_1E4 * f, ALPHA_HEII_1E4 * f, ALPHA_HEIII_1E4 * f


def opacity(U, nH, a, model):
    """Proper absorption coefficient kappa (1/cm) from the species fractions
    (LTE: the constant coefficient)."""
    if model.lte:
        return model.kappa_lte + 0.0 * U[0].real
    xHI, xHeI, xHeII, _ = species_fractions(U, model.nspecies)
    n_p = nH / a ** 3
    K = model.K_kappa
    k = K[0] * n_p * xHI
    if model.nspecies == 3:
        k = k + model.y_he * n_p * (K[1] * xHeI + K[2] * xHeII)
    return k


def opacity_derivatives(U, nH, a, model):
    """d kappa / d x_s for every species fraction s (list, empty for LTE)."""
    if model.lte:
        return []
    n_p = nH / a ** 3
    K = model.K_kappa
    out = [K[0] * n_p]
    if model.nspecies == 3:
        out += [model.y_he * n_p * K[1], model.y_he * n_p * K[2]]
    return out


def local_operators_lte(U, nH, eh, a, H, model):
    """LTE coupling (Sec. 2.1, Eq. 9): eta = kappa_P sigma_SB T^4 / pi,
    G = c kappa E / rho, Lambda = 4 pi eta / rho, with T from the ideal gas
    (Eq. 7) at the fixed mean particle mass mu m_H; U = (e_c, E).  Here
    4 pi eta = c kappa_P a_r T^4 depends on U and stays in L_E."""
    ec, E = U[0], U[-1]
    a3 = a ** 3
    rho_p = M_H * (nH / a3) * (1.0 + 4.0 * model.y_he)
    T = (GAMMA - 1.0) * model.mu_lte * M_H * (eh + ec) / K_B
    emit = C_LIGHT * model.kappaP_lte * A_RAD * T ** 4        # 4 pi eta (proper)
    absorb = C_LIGHT * model.kappa_lte * E                     # comoving
    L = np.empty(U.shape, dtype=np.result_type(U, nH, eh, complex if np.iscomplexobj(U) else float))
    L[0] = 2.0 * H * ec - absorb / a3 / rho_p + emit / rho_p
    L[-1] = model.m * H * E + absorb - a3 * emit
    return L


def local_operators(U, nH, eh, a, H, model):
    """Return L with rows (L_e, L_x1..L_xNs, L_E_local), same shape as U.

    L_E_local excludes the diffusion term and the source emissivity (the
    emissivity does not depend on U; it enters the constant vector g).
    """
    if model.lte:
        return local_operators_lte(U, nH, eh, a, H, model)
    ns = model.nspecies
    y = model.y_he
    ec, E = U[0], U[-1]
    xHI, xHeI, xHeII, xHeIII = species_fractions(U, ns)
    n_p = nH / a ** 3
    E_p = E / a ** 3
    ne = n_p * electron_fraction(xHI, xHeII, xHeIII, y)
    if model.isothermal:
        T = model.T_iso + 0.0 * ec
    else:
        T = temperature(eh + ec, xHI, xHeII, xHeIII, model)
    aH, aHeII, aHeIII = recombination_coefficients(T)
    Kg = model.K_gamma
    G_HI = C_LIGHT * Kg[0] * E_p

    L = np.empty(U.shape, dtype=np.result_type(U, nH, eh, complex if np.iscomplexobj(U) else float))
    # species: dx/dt = -L_x  (Eq. 27 written per fraction)
    L[1] = xHI * G_HI - aH * ne * (1.0 - xHI)
    if ns == 3:
        G_HeI = C_LIGHT * Kg[1] * E_p
        G_HeII = C_LIGHT * Kg[2] * E_p
        L[2] = xHeI * G_HeI - aHeII * ne * xHeII
        L[3] = (xHeII * G_HeII - xHeI * G_HeI + aHeII * ne * xHeII
                - aHeIII * ne * xHeIII)
    # gas energy correction (Eq. 26)
    rho_p = M_H * n_p * (1.0 + 4.0 * y)
    if model.isothermal:
        # fixed-temperature gas: heating and cooling are taken up by the
        # agent that holds T fixed (Sec. 4.5); only the expansion term stays
        L[0] = 2.0 * H * ec
    else:
        Kh = model.K_heat
        heat = C_LIGHT * E_p * n_p * (Kh[0] * xHI + y * (Kh[1] * xHeI + Kh[2] * xHeII)) / rho_p
        recomb = n_p * (aH * (1.0 - xHI) + y * (aHeII * xHeII + aHeIII * xHeIII))
        cool = BETA_COOL * K_B * T * ne * recomb / rho_p
        L[0] = 2.0 * H * ec - heat + cool
    # radiation, local part (Eq. 28 without 4 pi eta)
    L[-1] = model.m * H * E + C_LIGHT * opacity(U, nH, a, model) * E
    return L
