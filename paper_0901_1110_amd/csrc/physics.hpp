// Cell-local physics of the implicit radiation / ionization / energy system.
//
// Rate model (the paper names the dependencies in Sec. 2.1 but gives the
// non-LTE formulas only by reference; this is the library's stated reading):
//   T       = (gamma-1) (1+4y) m_H e / (k_B (1 + y + n_e/n_H))      (Eq. 8)
//   alpha_s = alpha_s(1e4 K) (T/1e4)^-0.7, alpha_HII(1e4) = 2.59e-13 (Sec. 4.5)
//   Gamma_s = c K_gamma_s E/a^3,  kappa = sum_s K_kappa_s n_s/a^3
//   G       = c E/a^3 sum_s K_heat_s n_s / rho,   Lambda = 0.75 k_B T n_e
//             sum_ions alpha n_ion / rho (recombination cooling)
// and the local operators of Sec. 3.2 (Eqs. 26-28), per fraction:
//   L_e  = 2 H e_c - G + Lambda
//   L_HI = x_HI Gamma_HI - alpha_HII n_e (1 - x_HI)
//   L_HeI  = x_HeI Gamma_HeI - alpha_HeII n_e x_HeII
//   L_HeII = x_HeII Gamma_HeII - x_HeI Gamma_HeI + alpha_HeII n_e x_HeII
//            - alpha_HeIII n_e x_HeIII
//   L_E,loc = m H E + c kappa E     (emissivity folded into the time level)
// LTE coupling (Sec. 2.1, Eq. 9; no species, U = (e_c, E)): with T from the
// ideal gas at the fixed mean particle mass mu m_H and 4 pi eta =
// c kappa_P a_r T^4 (4 sigma_SB = c a_r),
//   L_e     = 2 H e_c - c kappa E_p / rho_p + c kappa_P a_r T^4 / rho_p
//   L_E,loc = m H E + c kappa E - a^3 c kappa_P a_r T^4
// The functions are templates on the scalar type so that the same text gives
// values (double) and exact first derivatives (forward-mode dual numbers).
#pragma once

#include <hip/hip_runtime.h>

namespace rtk {

constexpr double C_LIGHT = 2.99792458e10;
constexpr double K_BOLTZ = 1.380649e-16;
constexpr double M_HYD = 1.6735575e-24;
constexpr double GAMMA_GAS = 5.0 / 3.0;
constexpr double T_EXP = -0.7;
constexpr double BETA_COOL = 0.75;
constexpr double SIGMA_SB = 5.670374419e-5;
constexpr double A_RAD = 4.0 * SIGMA_SB / C_LIGHT;
constexpr double KAPPA_FLOOR = 1.0e-3;   // face opacity floor per proper cell width
constexpr double E_TINY = 1.0e-300;

// Parameters copied to the device by value with every launch.
struct DevParams {
  int nx, ny, nz, ns, nv, nb;
  int N;
  int iso, lim_mode;
  double dx, theta, u_e, u_E, m, y, T_iso, D0;
  double Kg[3], Kk[3], Kh[3];
  double hnu;
  double alpha0[3];   // HII, HeII, HeIII at 1e4 K
  double kap_lte, kapP_lte, mu_lte;   // LTE coupling (ns = 0)
  int bc;                             // 0 periodic, 1 reflecting walls, 2 x-left Dirichlet
  double Eb;                          // bc 2: E of the x-left ghost cell
};

// ---- forward-mode dual numbers ------------------------------------------
template <int K>
struct Dual {
  double v;
  double d[K];
  __device__ Dual() {}
  __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int i = 0; i < K; ++i) d[i] = 0.0;
  }
};

template <int K>
__device__ inline Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v + b.v;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int K>
__device__ inline Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v - b.v;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int K>
__device__ inline Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; r.v = a.v * b.v;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int K>
__device__ inline Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r; const double inv = 1.0 / b.v; r.v = a.v * inv;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r;
}
template <int K> __device__ inline Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K> __device__ inline Dual<K> operator+(double b, const Dual<K>& a) { return a + b; }
template <int K> __device__ inline Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K> __device__ inline Dual<K> operator-(double b, const Dual<K>& a) {
  Dual<K> r; r.v = b - a.v;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int K> __device__ inline Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r; r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int K> __device__ inline Dual<K> operator*(double b, const Dual<K>& a) { return a * b; }
template <int K> __device__ inline Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> __device__ inline Dual<K> operator/(double b, const Dual<K>& a) { return Dual<K>(b) / a; }

__device__ inline double val(double x) { return x; }
template <int K> __device__ inline double val(const Dual<K>& x) { return x.v; }

// x^p for a constant exponent p
__device__ inline double powc(double x, double p) { return pow(x, p); }
template <int K>
__device__ inline Dual<K> powc(const Dual<K>& x, double p) {
  Dual<K> r; r.v = pow(x.v, p);
  const double s = p * r.v / x.v;
#pragma unroll
  for (int i = 0; i < K; ++i) r.d[i] = s * x.d[i];
  return r;
}

// ---- local operators ------------------------------------------------------
// u: the nv unknowns of one cell (e_c, x_1..x_Ns, E); returns L in the same
// order (L_e, L_x..., L_E,loc), all unscaled.
template <int NS, class S>
__device__ inline void local_ops(const S* u, double nH, double eh, double a, double H,
                                 const DevParams& P, S* L) {
  if constexpr (NS == 0) {
    const S ec = u[0];
    const S E = u[1];
    const double a3 = a * a * a;
    const double rho = M_HYD * (nH / a3) * (1.0 + 4.0 * P.y);
    const S T = ((GAMMA_GAS - 1.0) * P.mu_lte * M_HYD / K_BOLTZ) * (eh + ec);
    const S T2 = T * T;
    const S emit = (C_LIGHT * P.kapP_lte * A_RAD) * (T2 * T2);
    const S absorb = (C_LIGHT * P.kap_lte) * E;
    L[0] = (2.0 * H) * ec - absorb / a3 / rho + emit / rho;
    L[1] = (P.m * H) * E + absorb - a3 * emit;
    return;
  } else {
  const S ec = u[0];
  const S E = u[NS + 1];
  const S xHI = u[1];
  const double y = P.y;
  const double a3 = a * a * a;
  const double np = nH / a3;
  const S Ep = E / a3;
  S xHeI(0.0), xHeII(0.0), xHeIII(0.0);
  if constexpr (NS == 3) {
    xHeI = u[2];
    xHeII = u[3];
    xHeIII = 1.0 - xHeI - xHeII;
  }
  const S nefrac = (1.0 - xHI) + y * (xHeII + 2.0 * xHeIII);
  const S ne = np * nefrac;
  S T(P.T_iso);
  if (!P.iso) {
    T = ((GAMMA_GAS - 1.0) * (1.0 + 4.0 * y) * M_HYD) * (eh + ec) /
        (K_BOLTZ * (1.0 + y + nefrac));
  }
  const S tf = powc(T / 1.0e4, T_EXP);
  const S aH = P.alpha0[0] * tf;
  const S GamHI = (C_LIGHT * P.Kg[0]) * Ep;
  L[1] = xHI * GamHI - aH * ne * (1.0 - xHI);
  S kappa = (P.Kk[0] * np) * xHI;
  S heat_n = P.Kh[0] * xHI;
  S recomb = aH * (1.0 - xHI);
  if constexpr (NS == 3) {
    const S aHeII = P.alpha0[1] * tf;
    const S aHeIII = P.alpha0[2] * tf;
    const S GamHeI = (C_LIGHT * P.Kg[1]) * Ep;
    const S GamHeII = (C_LIGHT * P.Kg[2]) * Ep;
    L[2] = xHeI * GamHeI - aHeII * ne * xHeII;
    L[3] = xHeII * GamHeII - xHeI * GamHeI + aHeII * ne * xHeII - aHeIII * ne * xHeIII;
    kappa = kappa + (y * np) * (P.Kk[1] * xHeI + P.Kk[2] * xHeII);
    heat_n = heat_n + y * (P.Kh[1] * xHeI + P.Kh[2] * xHeII);
    recomb = recomb + y * (aHeII * xHeII + aHeIII * xHeIII);
  }
  if (P.iso) {
    L[0] = (2.0 * H) * ec;
  } else {
    const double rho = M_HYD * np * (1.0 + 4.0 * y);
    const S heat = C_LIGHT * Ep * np * heat_n / rho;
    const S cool = (BETA_COOL * K_BOLTZ) * T * ne * (np * recomb) / rho;
    L[0] = (2.0 * H) * ec - heat + cool;
  }
  L[NS + 1] = (P.m * H) * E + C_LIGHT * kappa * E;
  }
}

// Proper opacity of one cell (for the face coefficients).
template <int NS>
__device__ inline double opacity(const double* x, double nH, double a, const DevParams& P) {
  if constexpr (NS == 0) return P.kap_lte;
  const double np = nH / (a * a * a);
  double k = P.Kk[0] * np * x[0];
  if constexpr (NS == 3) k += P.y * np * (P.Kk[1] * x[1] + P.Kk[2] * x[2]);
  return k;
}

// Flux-limited diffusion coefficient of Eq. 12 (kappa_T = kappa).
__device__ inline double limiter(double k, double R) {
  return C_LIGHT * (2.0 * k + R) / (6.0 * k * k + 3.0 * k * R + R * R);
}

// Face coefficient between two cells P, Q = P + e_d (Sec. 2.2, a reading of
// the face discretization): mean E and kappa, floored kappa, one-sided R.
__device__ inline double face_D(double EP, double EQ, double kP, double kQ, double a,
                                const DevParams& P) {
  if (P.lim_mode == 1) return P.D0;
  const double adx = a * P.dx;
  const double Ef = 0.5 * (EP + EQ);
  const double kf = fmax(0.5 * (kP + kQ), KAPPA_FLOOR / adx);
  const double R = fabs(EQ - EP) / (adx * fmax(Ef, E_TINY));
  return limiter(kf, R);
}

// Face flux F = D_f (E_Q - E_P) and its derivatives for the exact Newton
// matrix: with T = R dD/dR = -c R^2 (4 kappa + R) / P^2 (P the limiter's
// denominator),
//   dF/dE_Q =  D + T - (E_Q - E_P) T / (2 E_f),
//   dF/dE_P = -D - T - (E_Q - E_P) T / (2 E_f),
//   dF/dkappa_f = (E_Q - E_P) dD/dkappa, dD/dkappa = -c (12 kappa^2 +
//   12 kappa R + R^2) / P^2 (zero where the opacity floor binds);
// DT = D + T is the derivative with respect to E_Q - E_P at fixed E_f and
// kappa_f (>= 0).  kappa_f is the mean of kP and kQ (mean = true) or kQ.
struct FaceJac {
  double D, DT, dEP, dEQ, dk;
};
__device__ inline FaceJac face_jac(double EP, double EQ, double kP, double kQ, double a,
                                   const DevParams& P, bool mean = true) {
  FaceJac J;
  if (P.lim_mode == 1) {
    J.D = P.D0; J.DT = P.D0; J.dEP = -P.D0; J.dEQ = P.D0; J.dk = 0.0;
    return J;
  }
  const double adx = a * P.dx;
  const double Ef = 0.5 * (EP + EQ);
  const double dE = EQ - EP;
  const double km = mean ? 0.5 * (kP + kQ) : kQ;
  const double kfl = KAPPA_FLOOR / adx;
  const double kf = fmax(km, kfl);
  const double Efl = fmax(Ef, E_TINY);
  const double R = fabs(dE) / (adx * Efl);
  const double Pd = 6.0 * kf * kf + 3.0 * kf * R + R * R;
  const double Pd2 = Pd * Pd;
  J.D = C_LIGHT * (2.0 * kf + R) / Pd;
  const double T = -C_LIGHT * R * R * (4.0 * kf + R) / Pd2;
  const double tail = Ef > E_TINY ? dE * T / (2.0 * Efl) : 0.0;
  J.DT = J.D + T;
  J.dEQ = J.D + T - tail;
  J.dEP = -J.D - T - tail;
  J.dk = km > kfl ? dE * (-C_LIGHT * (12.0 * kf * kf + 12.0 * kf * R + R * R) / Pd2) : 0.0;
  return J;
}

// d kappa / d x_s of one cell (proper), for the species fractions s
template <int NS>
__device__ inline void opacity_derivs(double nH, double a, const DevParams& P,
                                      double (&dk)[NS > 0 ? NS : 1]) {
  if constexpr (NS == 0) {
    dk[0] = 0.0;
  } else {
    const double np = nH / (a * a * a);
    dk[0] = P.Kk[0] * np;
    if constexpr (NS == 3) {
      dk[1] = P.y * np * P.Kk[1];
      dk[2] = P.y * np * P.Kk[2];
    }
  }
}

}  // namespace rtk
