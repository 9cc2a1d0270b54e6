/*
 * Oracle (test infrastructure): 1-D nodal spectral basis.
 *
 * The DGSEM basis is a tensor product of 1-D Lagrange polynomials on the quadrature nodes (paper, Sec. 2,
 * nodal expansion).  The paper uses Legendre-Gauss nodes; the Gauss-Lobatto family is provided as well.
 * Lagrange polynomials and their derivatives are evaluated by their defining products, not by any
 * barycentric shortcut, so the tables can be checked by eye.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

/* Legendre polynomial P_n and its derivative at x: three-term recurrence. */
static void legendre(int n, double x, double* P, double* dP) {
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  for (int k = 2; k <= n; k++) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1; /* P'_k = P'_{k-2} + (2k-1) P_{k-1} */
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

/* Gauss nodes of order N (N+1 points): roots of P_{N+1}; w = 2 / ((1-x^2) P'_{N+1}(x)^2). */
static void gauss(int N, double* x, double* w) {
  int n = N + 1;
  for (int k = 0; k < n; k++) {
    double xk = -cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    for (int it = 0; it < 100; it++) {
      double P, dP;
      legendre(n, xk, &P, &dP);
      double dx = P / dP;
      xk -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    double P, dP;
    legendre(n, xk, &P, &dP);
    x[k] = xk;
    w[k] = 2.0 / ((1.0 - xk * xk) * dP * dP);
  }
}

/* Gauss-Lobatto nodes of order N: -1, +1 and the roots of P'_N; w = 2 / (N (N+1) P_N(x)^2). */
static void gauss_lobatto(int N, double* x, double* w) {
  x[0] = -1.0; x[N] = 1.0;
  for (int k = 1; k < N; k++) {
    double xk = -cos(M_PI * k / N);
    for (int it = 0; it < 100; it++) {
      double P, dP;
      legendre(N, xk, &P, &dP);
      /* Legendre equation: (1-x^2) P'' = 2x P' - N(N+1) P */
      double d2P = (2.0 * xk * dP - N * (N + 1.0) * P) / (1.0 - xk * xk);
      double dx = dP / d2P;
      xk -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    x[k] = xk;
  }
  for (int k = 0; k <= N; k++) {
    double P, dP;
    legendre(N, x[k], &P, &dP);
    w[k] = 2.0 / (N * (N + 1.0) * P * P);
  }
}

/* l_j(x) = prod_{k != j} (x - x_k) / (x_j - x_k) */
double or_lagrange(int n, const double* xn, int j, double x) {
  double v = 1.0;
  for (int k = 0; k < n; k++)
    if (k != j) v *= (x - xn[k]) / (xn[j] - xn[k]);
  return v;
}

/* l_j'(x) = sum_{m != j} 1/(x_j - x_m) prod_{k != j, m} (x - x_k) / (x_j - x_k) */
double or_lagrange_deriv(int n, const double* xn, int j, double x) {
  double s = 0.0;
  for (int m = 0; m < n; m++) {
    if (m == j) continue;
    double v = 1.0 / (xn[j] - xn[m]);
    for (int k = 0; k < n; k++)
      if (k != j && k != m) v *= (x - xn[k]) / (xn[j] - xn[k]);
    s += v;
  }
  return s;
}

void or_make_basis(int order, int family, or_basis1d* b) {
  memset(b, 0, sizeof(*b));
  b->n = order + 1;
  if (family == 1) gauss_lobatto(order, b->x, b->w);
  else gauss(order, b->x, b->w);
  for (int i = 0; i < b->n; i++)
    for (int j = 0; j < b->n; j++) b->D[i][j] = or_lagrange_deriv(b->n, b->x, j, b->x[i]);
  for (int j = 0; j < b->n; j++) {
    b->lm[j] = or_lagrange(b->n, b->x, j, -1.0);
    b->lp[j] = or_lagrange(b->n, b->x, j, 1.0);
  }
}

/* I[p][j] = l_j^{from}(pts[p]) */
void or_interp_matrix(const or_basis1d* from, const double* pts, int npts, double* I) {
  for (int p = 0; p < npts; p++)
    for (int j = 0; j < from->n; j++) I[p * from->n + j] = or_lagrange(from->n, from->x, j, pts[p]);
}

/* Gaussian elimination with partial pivoting: solves A X = B in place (B is n x nrhs, row-major). */
int or_solve_dense(int n, double* A, double* B, int nrhs) {
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++)
      if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return -1;
    if (piv != c) {
      for (int k = 0; k < n; k++) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
      for (int k = 0; k < nrhs; k++) { double t = B[c * nrhs + k]; B[c * nrhs + k] = B[piv * nrhs + k]; B[piv * nrhs + k] = t; }
    }
    for (int r = c + 1; r < n; r++) {
      double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; k++) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < nrhs; k++) B[r * nrhs + k] -= f * B[c * nrhs + k];
    }
  }
  for (int c = n - 1; c >= 0; c--) {
    for (int k = 0; k < nrhs; k++) {
      double s = B[c * nrhs + k];
      for (int j = c + 1; j < n; j++) s -= A[c * n + j] * B[j * nrhs + k];
      B[c * nrhs + k] = s / A[c * n + c];
    }
  }
  return 0;
}

/*
 * L2 projection from the (fine) basis onto the (coarse) basis, computed with the fine quadrature:
 *   R = (P^T W P)^{-1} P^T W,  P[b][a] = l_a^{coarse}(x_b^{fine}),  W = diag(w^{fine}).
 * This is the restriction operator of the FAS cycle (an L2 projection to the lower order) and the
 * mortar-to-face projection; it is exact whenever the fine set has more nodes than the coarse one.
 */
void or_projection_matrix(const or_basis1d* coarse, const or_basis1d* fine, double* R) {
  int nc = coarse->n, nf = fine->n;
  double P[OR_MAXN * OR_MAXN], M[OR_MAXN * OR_MAXN], B[OR_MAXN * OR_MAXN];
  or_interp_matrix(coarse, fine->x, nf, P); /* P[b*nc + a] */
  for (int a = 0; a < nc; a++)
    for (int c = 0; c < nc; c++) {
      double s = 0.0;
      for (int b = 0; b < nf; b++) s += P[b * nc + a] * fine->w[b] * P[b * nc + c];
      M[a * nc + c] = s;
    }
  for (int a = 0; a < nc; a++)
    for (int b = 0; b < nf; b++) B[a * nf + b] = P[b * nc + a] * fine->w[b];
  or_solve_dense(nc, M, B, nf);
  memcpy(R, B, sizeof(double) * nc * nf);
}
