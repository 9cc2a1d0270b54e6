/*
 * Oracle (test infrastructure): compressible Navier-Stokes fluxes and the Roe Riemann solver.
 *
 * Non-dimensional equations of the paper's Appendix A: conserved q = (rho, rho u, rho v, rho w, rho e),
 * advective fluxes f^a, g^a, h^a, viscous fluxes with the 1/Re factor, Stokes hypothesis
 * (lambda = -2/3 mu), heat-flux coefficient kappa / ((gamma - 1) Pr M^2), Sutherland viscosity.
 * Reference state rho = 1, |v| = 1, T = 1, so p_inf = 1 / (gamma M^2) and T = gamma M^2 p / rho.
 */
#include <math.h>

#include "oracle.h"

void or_prim(const or_phys* ph, const double q[5], double* rho, double v[3], double* p, double* T) {
  *rho = q[0];
  v[0] = q[1] / q[0];
  v[1] = q[2] / q[0];
  v[2] = q[3] / q[0];
  *p = (ph->gamma - 1.0) * (q[4] - 0.5 * (q[1] * v[0] + q[2] * v[1] + q[3] * v[2]));
  *T = ph->gamma * ph->mach * ph->mach * (*p) / q[0];
}

/* Sutherland's law in reference units: mu = T^{3/2} (1 + S) / (T + S); kappa = mu. */
double or_mu(const or_phys* ph, double T) {
  if (ph->viscosity == 1) return 1.0;
  return T * sqrt(T) * (1.0 + ph->suth) / (T + ph->suth);
}

/* F[c][v]: Cartesian direction c = x, y, z; variable v. */
void or_flux_adv(const or_phys* ph, const double q[5], double F[3][5]) {
  double rho, v[3], p, T;
  or_prim(ph, q, &rho, v, &p, &T);
  for (int c = 0; c < 3; c++) {
    F[c][0] = q[0] * v[c];
    F[c][1] = q[1] * v[c];
    F[c][2] = q[2] * v[c];
    F[c][3] = q[3] * v[c];
    F[c][1 + c] += p;
    F[c][4] = v[c] * (q[4] + p);
  }
}

/* gW[k][c] = d W_k / d x_c with W = (u, v, w, T).  Viscous flux (without the minus sign of F^a - F^v). */
static void visc(const or_phys* ph, const double q[5], const double gW[4][3], int wall, double F[3][5]) {
  double rho, v[3], p, T;
  or_prim(ph, q, &rho, v, &p, &T);
  double mu = or_mu(ph, T);
  double div = gW[0][0] + gW[1][1] + gW[2][2];
  double tau[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) tau[i][j] = mu * (gW[i][j] + gW[j][i]);
  for (int i = 0; i < 3; i++) tau[i][i] += -2.0 / 3.0 * mu * div;
  double kap = mu / ((ph->gamma - 1.0) * ph->prandtl * ph->mach * ph->mach);
  double invRe = 1.0 / ph->reynolds;
  for (int c = 0; c < 3; c++) {
    F[c][0] = 0.0;
    F[c][1] = invRe * tau[c][0];
    F[c][2] = invRe * tau[c][1];
    F[c][3] = invRe * tau[c][2];
    if (wall) F[c][4] = 0.0; /* adiabatic no-slip wall: wall velocity 0 and no heat flux */
    else F[c][4] = invRe * (v[0] * tau[c][0] + v[1] * tau[c][1] + v[2] * tau[c][2] + kap * gW[3][c]);
  }
}

void or_flux_visc(const or_phys* ph, const double q[5], const double gW[4][3], double F[3][5]) {
  visc(ph, q, gW, 0, F);
}

void or_flux_visc_wall(const or_phys* ph, const double q[5], const double gW[4][3], double F[3][5]) {
  visc(ph, q, gW, 1, F);
}

/*
 * Roe flux along the unit normal n from state L to state R:
 *   F* = 1/2 (F(qL) + F(qR)) . n - 1/2 sum_k |lambda_k| alpha_k r_k
 * with sqrt(rho)-weighted averages of v and H = (rho e + p) / rho and no entropy fix.
 */
void or_roe(const or_phys* ph, const double qL[5], const double qR[5], const double n[3], double Fn[5]) {
  const double g = ph->gamma;
  double rL, vL[3], pL, TL, rR, vR[3], pR, TR;
  or_prim(ph, qL, &rL, vL, &pL, &TL);
  or_prim(ph, qR, &rR, vR, &pR, &TR);
  double HL = (qL[4] + pL) / rL, HR = (qR[4] + pR) / rR;
  double sL = sqrt(rL), sR = sqrt(rR);
  double rh = sL * sR;
  double vh[3];
  for (int c = 0; c < 3; c++) vh[c] = (sL * vL[c] + sR * vR[c]) / (sL + sR);
  double Hh = (sL * HL + sR * HR) / (sL + sR);
  double v2 = vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2];
  double c2 = (g - 1.0) * (Hh - 0.5 * v2);
  double ch = sqrt(c2);
  double un = vh[0] * n[0] + vh[1] * n[1] + vh[2] * n[2];
  double dr = rR - rL, dp = pR - pL, dv[3];
  for (int c = 0; c < 3; c++) dv[c] = vR[c] - vL[c];
  double dun = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];

  double a1 = (dp - rh * ch * dun) / (2.0 * c2);
  double a5 = (dp + rh * ch * dun) / (2.0 * c2);
  double a2 = dr - dp / c2;
  double l1 = fabs(un - ch), l5 = fabs(un + ch), l2 = fabs(un);

  double diss[5];
  diss[0] = l1 * a1 + l5 * a5 + l2 * a2;
  for (int c = 0; c < 3; c++)
    diss[1 + c] = l1 * a1 * (vh[c] - ch * n[c]) + l5 * a5 * (vh[c] + ch * n[c]) + l2 * a2 * vh[c] +
                  l2 * rh * (dv[c] - dun * n[c]);
  diss[4] = l1 * a1 * (Hh - un * ch) + l5 * a5 * (Hh + un * ch) + l2 * a2 * 0.5 * v2 +
            l2 * rh * (vh[0] * dv[0] + vh[1] * dv[1] + vh[2] * dv[2] - un * dun);

  double FL[3][5], FR[3][5];
  or_flux_adv(ph, qL, FL);
  or_flux_adv(ph, qR, FR);
  for (int v = 0; v < 5; v++) {
    double fl = FL[0][v] * n[0] + FL[1][v] * n[1] + FL[2][v] * n[2];
    double fr = FR[0][v] * n[0] + FR[1][v] * n[1] + FR[2][v] * n[2];
    Fn[v] = 0.5 * (fl + fr) - 0.5 * diss[v];
  }
}

/* Free stream: rho = 1, v = (1, 0, 0), p = 1 / (gamma M^2). */
void or_freestream(const or_phys* ph, double q[5]) {
  double p = 1.0 / (ph->gamma * ph->mach * ph->mach);
  q[0] = 1.0; q[1] = 1.0; q[2] = 0.0; q[3] = 0.0;
  q[4] = p / (ph->gamma - 1.0) + 0.5;
}
