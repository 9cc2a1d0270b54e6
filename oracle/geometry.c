/*
 * Oracle (test infrastructure): geometry of one discretisation level.
 *
 * Paper, Sec. 2: high-order mapping x^e(xi) of order M; covariant vectors a_i = dx/dxi_i;
 * J = a_i . (a_j x a_k); contravariant metric J a^i by the invariant curl form
 *   J a^i_n = -1/2 xhat_i . curl_xi [ I^N ( X_l grad_xi X_m - X_m grad_xi X_l ) ],  (n, m, l) cyclic,
 * with I^N the interpolant at the element's own solution nodes at this level's orders.  The metric terms
 * are recomputed for every order tensor (every multigrid level), never restricted.
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int64_t vidx(const int n[3], int i, int j, int k) { return i + (int64_t)n[0] * (j + (int64_t)n[1] * k); }

/* derivative along axis d of a nodal field f (npe values) of one element */
static void deriv(const or_basis1d* b[3], const int n[3], int d, const double* f, double* df) {
  for (int k = 0; k < n[2]; k++)
    for (int j = 0; j < n[1]; j++)
      for (int i = 0; i < n[0]; i++) {
        int ijk[3] = {i, j, k};
        double s = 0.0;
        for (int m = 0; m < n[d]; m++) {
          int q[3] = {i, j, k};
          q[d] = m;
          s += b[d]->D[ijk[d]][m] * f[vidx(n, q[0], q[1], q[2])];
        }
        df[vidx(n, i, j, k)] = s;
      }
}

or_level* or_level_create(const or_problem* P, const int32_t* ord) {
  or_level* L = (or_level*)calloc(1, sizeof(or_level));
  int64_t K = P->K;
  L->K = K;
  L->ord = (int32_t*)malloc(sizeof(int32_t) * 3 * K);
  memcpy(L->ord, ord, sizeof(int32_t) * 3 * K);
  L->off = (int64_t*)malloc(sizeof(int64_t) * (K + 1));
  L->fo = (int64_t*)malloc(sizeof(int64_t) * 6 * K);
  L->off[0] = 0;
  int64_t nf = 0;
  for (int64_t e = 0; e < K; e++) {
    int n[3] = {ord[3 * e] + 1, ord[3 * e + 1] + 1, ord[3 * e + 2] + 1};
    L->off[e + 1] = L->off[e] + (int64_t)n[0] * n[1] * n[2];
    int fs[3] = {n[1] * n[2], n[0] * n[2], n[0] * n[1]};
    for (int f = 0; f < 6; f++) {
      L->fo[6 * e + f] = nf;
      nf += fs[f / 2];
    }
  }
  L->nn = L->off[K];
  L->nf = nf;
  int64_t nn = L->nn;
  L->X = (double*)malloc(sizeof(double) * 3 * nn);
  L->Ja = (double*)malloc(sizeof(double) * 9 * nn);
  L->J = (double*)malloc(sizeof(double) * nn);
  L->Nout = (double*)malloc(sizeof(double) * 3 * nf);

  const int M1 = P->M[0], M2 = P->M[1], M3 = P->M[2];
  double eq[3][OR_MAXN];
  int Mv[3] = {M1, M2, M3};
  for (int d = 0; d < 3; d++)
    for (int a = 0; a <= Mv[d]; a++) eq[d][a] = (Mv[d] == 0) ? 0.0 : -1.0 + 2.0 * a / Mv[d];

  for (int64_t e = 0; e < K; e++) {
    int n[3] = {ord[3 * e] + 1, ord[3 * e + 1] + 1, ord[3 * e + 2] + 1};
    const or_basis1d* b[3] = {&P->basis[n[0] - 1], &P->basis[n[1] - 1], &P->basis[n[2] - 1]};
    int npe = n[0] * n[1] * n[2];
    double* X = (double*)malloc(sizeof(double) * 3 * npe);
    double* dX = (double*)malloc(sizeof(double) * 9 * npe); /* dX[(m*3 + d)*npe + node] = dX_m/dxi_d */
    double* V = (double*)malloc(sizeof(double) * 3 * npe);
    double* dV = (double*)malloc(sizeof(double) * npe);
    const double* g = P->gnodes + (int64_t)e * (M1 + 1) * (M2 + 1) * (M3 + 1) * 3;

    /* X at the solution nodes: the degree-M mapping on equispaced reference nodes.  The Lagrange weights sum
     * to one, so the mapping of the nodes taken relative to the element's first mapping node x0 is X - x0
     * exactly; evaluated that way, X - x0 and its derivatives carry round-off relative to the element's size,
     * not to its distance from the origin (which on a thin wall cell far from the origin is larger by the
     * ratio of the two). */
    const double x0[3] = {g[0], g[1], g[2]};
    for (int k = 0; k < n[2]; k++)
      for (int j = 0; j < n[1]; j++)
        for (int i = 0; i < n[0]; i++) {
          double x[3] = {0, 0, 0};
          for (int c3 = 0; c3 <= M3; c3++) {
            double l3 = or_lagrange(M3 + 1, eq[2], c3, b[2]->x[k]);
            for (int c2 = 0; c2 <= M2; c2++) {
              double l2 = or_lagrange(M2 + 1, eq[1], c2, b[1]->x[j]);
              for (int c1 = 0; c1 <= M1; c1++) {
                double l1 = or_lagrange(M1 + 1, eq[0], c1, b[0]->x[i]);
                const double* gp = g + (((int64_t)c3 * (M2 + 1) + c2) * (M1 + 1) + c1) * 3;
                for (int c = 0; c < 3; c++) x[c] += l1 * l2 * l3 * (gp[c] - x0[c]);
              }
            }
          }
          for (int c = 0; c < 3; c++) X[c * npe + vidx(n, i, j, k)] = x[c];
        }
    /* covariant derivatives of I^N X (from X - x0: the derivative of a constant vanishes) */
    for (int m = 0; m < 3; m++)
      for (int d = 0; d < 3; d++) deriv(b, n, d, X + m * npe, dX + (m * 3 + d) * npe);

    double* Ja = (double*)calloc(9 * npe, sizeof(double)); /* Ja[(i*3 + comp)*npe + node] */
    /* The curl form is unchanged when X is shifted by a constant (the discrete curl of a discrete gradient
     * vanishes), so it is evaluated on X - x0 as held in X. */
    /* invariant curl form, component n_ of every J a^i */
    for (int nc = 0; nc < 3; nc++) {
      int mc = (nc + 1) % 3, lc = (nc + 2) % 3;
      /* V_c = X_l dX_m/dxi_c - X_m dX_l/dxi_c at the nodes (I^N of the product) */
      for (int c = 0; c < 3; c++)
        for (int p = 0; p < npe; p++)
          V[c * npe + p] = X[lc * npe + p] * dX[(mc * 3 + c) * npe + p] - X[mc * npe + p] * dX[(lc * 3 + c) * npe + p];
      /* (curl V)_1 = d2 V3 - d3 V2; (curl V)_2 = d3 V1 - d1 V3; (curl V)_3 = d1 V2 - d2 V1 */
      for (int i = 0; i < 3; i++) {
        int a = (i + 1) % 3, bb = (i + 2) % 3;
        deriv(b, n, a, V + bb * npe, dV);
        for (int p = 0; p < npe; p++) Ja[(i * 3 + nc) * npe + p] += -0.5 * dV[p];
        deriv(b, n, bb, V + a * npe, dV);
        for (int p = 0; p < npe; p++) Ja[(i * 3 + nc) * npe + p] -= -0.5 * dV[p];
      }
    }
    int64_t o = L->off[e];
    for (int p = 0; p < npe; p++) {
      double a1[3], a2[3], a3[3];
      for (int c = 0; c < 3; c++) {
        a1[c] = dX[(c * 3 + 0) * npe + p];
        a2[c] = dX[(c * 3 + 1) * npe + p];
        a3[c] = dX[(c * 3 + 2) * npe + p];
      }
      double cr[3] = {a2[1] * a3[2] - a2[2] * a3[1], a2[2] * a3[0] - a2[0] * a3[2], a2[0] * a3[1] - a2[1] * a3[0]};
      L->J[o + p] = a1[0] * cr[0] + a1[1] * cr[1] + a1[2] * cr[2];
      for (int c = 0; c < 3; c++) L->X[c * nn + o + p] = X[c * npe + p] + x0[c];
      for (int q = 0; q < 9; q++) L->Ja[q * nn + o + p] = Ja[q * npe + p];
    }
    /* face metric: J a^d traced to face d+- with l(+-1); outward sign */
    for (int f = 0; f < 6; f++) {
      int d = f / 2, side = f % 2;
      int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
      const double* lf = side ? b[d]->lp : b[d]->lm;
      double sgn = side ? 1.0 : -1.0;
      for (int bq = 0; bq < n[t2]; bq++)
        for (int aq = 0; aq < n[t1]; aq++) {
          double N[3] = {0, 0, 0};
          for (int q = 0; q < n[d]; q++) {
            int ijk[3];
            ijk[d] = q; ijk[t1] = aq; ijk[t2] = bq;
            int64_t p = vidx(n, ijk[0], ijk[1], ijk[2]);
            for (int c = 0; c < 3; c++) N[c] += lf[q] * Ja[(d * 3 + c) * npe + p];
          }
          int64_t fi = L->fo[6 * e + f] + aq + (int64_t)n[t1] * bq;
          for (int c = 0; c < 3; c++) L->Nout[c * nf + fi] = sgn * N[c];
        }
    }
    free(X); free(dX); free(V); free(dV); free(Ja);
  }
  return L;
}

void or_level_destroy(or_level* L) {
  if (!L) return;
  free(L->ord); free(L->off); free(L->fo); free(L->X); free(L->Ja); free(L->J); free(L->Nout);
  free(L);
}
