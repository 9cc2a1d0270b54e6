/*
 * Oracle (test infrastructure): the DGSEM spatial operator A(Q) = [M]^{-1} F(Q) and its isolated variant.
 *
 * Paper, Sec. 2 (weak form, element system with mass matrix and F^e) and Sec. 3.1 (A = M^{-1} F):
 * weak-form DGSEM on Gauss (or Gauss-Lobatto) nodes, Roe advective flux, Bassi-Rebay 1 viscous flux,
 * non-conforming faces through a mortar (exact interpolation of both traces to the mortar, L2 projection
 * back), boundary ghost states.  The isolated operator (Sec. 3.2.1) replaces every numerical flux by the
 * element's own physical flux of its trace, so no neighbour or boundary enters.
 *
 * Weak-form identities used (per direction d, node index i along d, tangential face node t):
 *   J grad W_i = sum_d { [ l_i(+1) W*_{d+} N_{d+} + l_i(-1) W*_{d-} N_{d-} ] / w_i + sum_m Dhat_im (J a^d W)_m }
 *   J A_i      = sum_d { [ l_i(+1) Phi_{d+}   + l_i(-1) Phi_{d-} ] / w_i   + sum_m Dhat_im Ftilde^d_m }
 * with Dhat_im = -D_mi w_m / w_i, N the outward normal scaled by the surface Jacobian (own side),
 * Phi the outward numerical flux times the surface Jacobian, Ftilde^d = J a^d . (F^a - F^v).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int64_t vidx(const int n[3], int i, int j, int k) { return i + (int64_t)n[0] * (j + (int64_t)n[1] * k); }

static void elem_n(const or_level* L, int64_t e, int n[3]) {
  n[0] = L->ord[3 * e] + 1; n[1] = L->ord[3 * e + 1] + 1; n[2] = L->ord[3 * e + 2] + 1;
}

static void face_axes(int f, int* d, int* t1, int* t2) {
  *d = f / 2;
  *t1 = (*d == 0) ? 1 : 0;
  *t2 = (*d == 2) ? 1 : 2;
}

/* Trace of an nvar-component nodal field U[v][nn] onto every element face: Uf[v][nf] */
static void face_traces(const or_problem* P, const or_level* L, const double* U, int nvar, double* Uf) {
  for (int64_t e = 0; e < L->K; e++) {
    int n[3];
    elem_n(L, e, n);
    for (int f = 0; f < 6; f++) {
      int d, t1, t2;
      face_axes(f, &d, &t1, &t2);
      const or_basis1d* bd = &P->basis[n[d] - 1];
      const double* lf = (f % 2) ? bd->lp : bd->lm;
      for (int b = 0; b < n[t2]; b++)
        for (int a = 0; a < n[t1]; a++) {
          int64_t fi = L->fo[6 * e + f] + a + (int64_t)n[t1] * b;
          for (int v = 0; v < nvar; v++) {
            double s = 0.0;
            for (int q = 0; q < n[d]; q++) {
              int ijk[3];
              ijk[d] = q; ijk[t1] = a; ijk[t2] = b;
              s += lf[q] * U[v * L->nn + L->off[e] + vidx(n, ijk[0], ijk[1], ijk[2])];
            }
            Uf[v * L->nf + fi] = s;
          }
        }
    }
  }
}

static void qvec(const double* Uf, int64_t nf, int64_t fi, double q[5]) {
  for (int v = 0; v < 5; v++) q[v] = Uf[v * nf + fi];
}
static void gvec(const double* Gf, int64_t nf, int64_t fi, double g[4][3]) {
  for (int k = 0; k < 4; k++)
    for (int c = 0; c < 3; c++) g[k][c] = Gf[(k * 3 + c) * nf + fi];
}
static void prim_w(const or_phys* ph, const double q[5], double W[4]) {
  double rho, v[3], p, T;
  or_prim(ph, q, &rho, v, &p, &T);
  W[0] = v[0]; W[1] = v[1]; W[2] = v[2]; W[3] = T;
}

/* ghost state of a boundary node with outward unit normal n */
static void ghost(const or_phys* ph, int bc, const double q[5], const double n[3], double qg[5]) {
  if (bc == 1) { /* no-slip adiabatic wall: mirrored velocity, same density and energy */
    qg[0] = q[0]; qg[1] = -q[1]; qg[2] = -q[2]; qg[3] = -q[3]; qg[4] = q[4];
  } else if (bc == 3) { /* free slip: normal momentum reflected */
    double mn = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    qg[0] = q[0];
    for (int c = 0; c < 3; c++) qg[1 + c] = q[1 + c] - 2.0 * mn * n[c];
    qg[4] = q[4];
  } else if (bc == 4) { /* subsonic outflow: interior density and velocity, the far-field pressure */
    double pinf = 1.0 / (ph->gamma * ph->mach * ph->mach);
    double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    for (int c = 0; c < 4; c++) qg[c] = q[c];
    qg[4] = pinf / (ph->gamma - 1.0) + ke;
  } else { /* far field */
    or_freestream(ph, qg);
  }
}

/* ----------------------------------------------------------------------------------------------------
 * Mortar of one interior face, built from its master side (lower element id; for a self-periodic face
 * the lower face index).  Mortar orders are the larger of the two sides' orders along each master
 * face axis; mortar nodes are the node family of that order, in master face coordinates.
 * -------------------------------------------------------------------------------------------------- */
typedef struct {
  int64_t e, g;   /* master, slave element */
  int f, h, o;    /* master face, slave face, orientation master -> slave */
  int nm;         /* mortar nodes */
  int nM, nS;     /* master / slave face nodes */
  double* WM;     /* [nm][nM]  interpolation master face -> mortar */
  double* WS;     /* [nm][nS]  interpolation slave face -> mortar */
  double* PM;     /* [nM][nm]  L2 projection mortar -> master face */
  double* PS;     /* [nS][nm]  L2 projection mortar -> slave face */
} or_mortar;

static void orient_map(int o, double s, double t, double* s2, double* t2) {
  double u = (o & 4) ? t : s, v = (o & 4) ? s : t;
  *s2 = (o & 1) ? -u : u;
  *t2 = (o & 2) ? -v : v;
}

/* side basis (n1 x n2 nodes on its own face axes); mortar nodes given in the side's own coordinates */
static void side_matrices(const or_problem* P, int n1, int n2, int nm, const double* ms, const double* mt,
                          const double* mw, const or_basis1d* B1, const or_basis1d* B2, double* W, double* Pr) {
  const or_basis1d* b1 = &P->basis[n1 - 1];
  const or_basis1d* b2 = &P->basis[n2 - 1];
  int ns = n1 * n2;
  for (int mu = 0; mu < nm; mu++)
    for (int b = 0; b < n2; b++)
      for (int a = 0; a < n1; a++)
        W[mu * ns + a + n1 * b] = or_lagrange(n1, b1->x, a, ms[mu]) * or_lagrange(n2, b2->x, b, mt[mu]);
  /* 1-D mass matrices of the side basis under the mortar quadrature along the matching mortar axis */
  double M1[OR_MAXN * OR_MAXN], M2[OR_MAXN * OR_MAXN], I1[OR_MAXN * OR_MAXN], I2[OR_MAXN * OR_MAXN];
  for (int a = 0; a < n1; a++)
    for (int c = 0; c < n1; c++) {
      double s = 0.0;
      for (int k = 0; k < B1->n; k++)
        s += B1->w[k] * or_lagrange(n1, b1->x, a, B1->x[k]) * or_lagrange(n1, b1->x, c, B1->x[k]);
      M1[a * n1 + c] = s;
      I1[a * n1 + c] = (a == c) ? 1.0 : 0.0;
    }
  for (int a = 0; a < n2; a++)
    for (int c = 0; c < n2; c++) {
      double s = 0.0;
      for (int k = 0; k < B2->n; k++)
        s += B2->w[k] * or_lagrange(n2, b2->x, a, B2->x[k]) * or_lagrange(n2, b2->x, c, B2->x[k]);
      M2[a * n2 + c] = s;
      I2[a * n2 + c] = (a == c) ? 1.0 : 0.0;
    }
  or_solve_dense(n1, M1, I1, n1); /* I1 = M1^{-1} */
  or_solve_dense(n2, M2, I2, n2);
  /* Pr[(a,b)][mu] = sum_{a2,b2} M1^{-1}[a][a2] M2^{-1}[b][b2] w_mu l_a2(s_mu) l_b2(t_mu) */
  for (int b = 0; b < n2; b++)
    for (int a = 0; a < n1; a++)
      for (int mu = 0; mu < nm; mu++) {
        double s = 0.0;
        for (int b2 = 0; b2 < n2; b2++)
          for (int a2 = 0; a2 < n1; a2++) s += I1[a * n1 + a2] * I2[b * n2 + b2] * W[mu * ns + a2 + n1 * b2];
        Pr[(a + n1 * b) * nm + mu] = s * mw[mu];
      }
}

static void mortar_build(const or_problem* P, const or_level* L, int64_t e, int f, or_mortar* m) {
  m->e = e; m->f = f;
  m->g = P->nbr[6 * e + f];
  m->h = P->nbrf[6 * e + f];
  m->o = P->orient[6 * e + f];
  int n[3], ng[3];
  elem_n(L, e, n);
  elem_n(L, m->g, ng);
  int d, t1, t2, dg, s1, s2;
  face_axes(f, &d, &t1, &t2);
  face_axes(m->h, &dg, &s1, &s2);
  int nMs = n[t1], nMt = n[t2];
  int nS1 = ng[s1], nS2 = ng[s2];
  /* slave orders along master axes s and t */
  int slave_s = (m->o & 4) ? nS2 : nS1;
  int slave_t = (m->o & 4) ? nS1 : nS2;
  int ms = nMs > slave_s ? nMs : slave_s;
  int mt = nMt > slave_t ? nMt : slave_t;
  const or_basis1d* Bs = &P->basis[ms - 1];
  const or_basis1d* Bt = &P->basis[mt - 1];
  m->nm = ms * mt;
  m->nM = nMs * nMt;
  m->nS = nS1 * nS2;
  double *sM = malloc(sizeof(double) * m->nm), *tM = malloc(sizeof(double) * m->nm);
  double *sS = malloc(sizeof(double) * m->nm), *tS = malloc(sizeof(double) * m->nm);
  double* w = malloc(sizeof(double) * m->nm);
  for (int be = 0; be < mt; be++)
    for (int al = 0; al < ms; al++) {
      int mu = al + ms * be;
      sM[mu] = Bs->x[al];
      tM[mu] = Bt->x[be];
      w[mu] = Bs->w[al] * Bt->w[be];
      orient_map(m->o, sM[mu], tM[mu], &sS[mu], &tS[mu]);
    }
  m->WM = malloc(sizeof(double) * m->nm * m->nM);
  m->PM = malloc(sizeof(double) * m->nm * m->nM);
  m->WS = malloc(sizeof(double) * m->nm * m->nS);
  m->PS = malloc(sizeof(double) * m->nm * m->nS);
  side_matrices(P, nMs, nMt, m->nm, sM, tM, w, Bs, Bt, m->WM, m->PM);
  /* the slave's first axis runs along the master's t axis when the code transposes */
  const or_basis1d* B1 = (m->o & 4) ? Bt : Bs;
  const or_basis1d* B2 = (m->o & 4) ? Bs : Bt;
  side_matrices(P, nS1, nS2, m->nm, sS, tS, w, B1, B2, m->WS, m->PS);
  free(sM); free(tM); free(sS); free(tS); free(w);
}

static void mortar_free(or_mortar* m) { free(m->WM); free(m->WS); free(m->PM); free(m->PS); }

static int is_master(const or_problem* P, int64_t e, int f) {
  int64_t g = P->nbr[6 * e + f];
  if (g < 0) return 1;
  if (e < g) return 1;
  if (e == g && f < P->nbrf[6 * e + f]) return 1;
  return 0;
}

/* interpolate nvar components of a side's face field to mortar node mu */
static void to_mortar(const double* W, int nside, int mu, const double* Uf, int64_t nf, int64_t fo, int nvar, double* out) {
  for (int v = 0; v < nvar; v++) {
    double s = 0.0;
    for (int k = 0; k < nside; k++) s += W[mu * nside + k] * Uf[v * nf + fo + k];
    out[v] = s;
  }
}

/* ---------------------------------------------------------------------------------------------------- */
void or_gradient(const or_problem* P, const or_level* L, int isolated, const double* Q, double* gW) {
  const or_phys* ph = &P->ph;
  const int64_t nn = L->nn, nf = L->nf;
  double* qf = malloc(sizeof(double) * 5 * nf);
  double* Ws = malloc(sizeof(double) * 4 * nf);   /* W* per side face node */

  /* (1) traces of q */
  face_traces(P, L, Q, 5, qf);

  /* (2) BR1 interface state W* */
  for (int64_t e = 0; e < L->K; e++)
    for (int f = 0; f < 6; f++) {
      int n[3], d, t1, t2;
      elem_n(L, e, n);
      face_axes(f, &d, &t1, &t2);
      int nside = n[t1] * n[t2];
      int64_t fo = L->fo[6 * e + f];
      if (isolated) {
        for (int k = 0; k < nside; k++) {
          double q[5], W[4];
          qvec(qf, nf, fo + k, q);
          prim_w(ph, q, W);
          for (int v = 0; v < 4; v++) Ws[v * nf + fo + k] = W[v];
        }
        continue;
      }
      if (!is_master(P, e, f)) continue;
      int bc = P->bc[6 * e + f];
      if (P->nbr[6 * e + f] < 0) {
        for (int k = 0; k < nside; k++) {
          double q[5], qg[5], W[4], Wg[4], N[3], Js, nh[3];
          qvec(qf, nf, fo + k, q);
          for (int c = 0; c < 3; c++) N[c] = L->Nout[c * nf + fo + k];
          Js = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          for (int c = 0; c < 3; c++) nh[c] = N[c] / Js;
          ghost(ph, bc, q, nh, qg);
          prim_w(ph, q, W);
          prim_w(ph, qg, Wg);
          for (int v = 0; v < 4; v++) Ws[v * nf + fo + k] = 0.5 * (W[v] + Wg[v]);
        }
        continue;
      }
      or_mortar m;
      mortar_build(P, L, e, f, &m);
      int64_t foS = L->fo[6 * m.g + m.h];
      double* wstar = malloc(sizeof(double) * 4 * m.nm);
      for (int mu = 0; mu < m.nm; mu++) {
        double qm[5], qs[5], Wm[4], Wsl[4];
        to_mortar(m.WM, m.nM, mu, qf, nf, fo, 5, qm);
        to_mortar(m.WS, m.nS, mu, qf, nf, foS, 5, qs);
        prim_w(ph, qm, Wm);
        prim_w(ph, qs, Wsl);
        for (int v = 0; v < 4; v++) wstar[v * m.nm + mu] = 0.5 * (Wm[v] + Wsl[v]);
      }
      for (int k = 0; k < m.nM; k++)
        for (int v = 0; v < 4; v++) {
          double s = 0.0;
          for (int mu = 0; mu < m.nm; mu++) s += m.PM[k * m.nm + mu] * wstar[v * m.nm + mu];
          Ws[v * nf + fo + k] = s;
        }
      for (int k = 0; k < m.nS; k++)
        for (int v = 0; v < 4; v++) {
          double s = 0.0;
          for (int mu = 0; mu < m.nm; mu++) s += m.PS[k * m.nm + mu] * wstar[v * m.nm + mu];
          Ws[v * nf + foS + k] = s;
        }
      free(wstar);
      mortar_free(&m);
    }

  /* (3) BR1 gradient of W = (u, v, w, T) at the nodes */
  for (int64_t e = 0; e < L->K; e++) {
    int n[3];
    elem_n(L, e, n);
    const or_basis1d* b[3] = {&P->basis[n[0] - 1], &P->basis[n[1] - 1], &P->basis[n[2] - 1]};
    int64_t o = L->off[e];
    int npe = n[0] * n[1] * n[2];
    double* Wn = malloc(sizeof(double) * 4 * npe);
    for (int p = 0; p < npe; p++) {
      double q[5], W[4];
      for (int v = 0; v < 5; v++) q[v] = Q[v * nn + o + p];
      prim_w(ph, q, W);
      for (int v = 0; v < 4; v++) Wn[v * npe + p] = W[v];
    }
    for (int k3 = 0; k3 < n[2]; k3++)
      for (int j = 0; j < n[1]; j++)
        for (int i = 0; i < n[0]; i++) {
          int ijk[3] = {i, j, k3};
          int64_t p = vidx(n, i, j, k3);
          double G[4][3] = {{0}};
          for (int d = 0; d < 3; d++) {
            const or_basis1d* bd = b[d];
            int id = ijk[d];
            /* volume term: sum_m Dhat_im (J a^d W)_m, Dhat_im = -D_mi w_m / w_i */
            for (int m = 0; m < n[d]; m++) {
              int q3[3] = {i, j, k3};
              q3[d] = m;
              int64_t pm = vidx(n, q3[0], q3[1], q3[2]);
              double Dh = -bd->D[m][id] * bd->w[m] / bd->w[id];
              for (int v = 0; v < 4; v++)
                for (int c = 0; c < 3; c++) G[v][c] += Dh * L->Ja[(d * 3 + c) * nn + o + pm] * Wn[v * npe + pm];
            }
            /* surface terms of faces d- and d+ */
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int64_t fk = ijk[t1] + (int64_t)n[t1] * ijk[t2];
            for (int side = 0; side < 2; side++) {
              int64_t fi = L->fo[6 * e + 2 * d + side] + fk;
              double l = side ? bd->lp[id] : bd->lm[id];
              for (int v = 0; v < 4; v++)
                for (int c = 0; c < 3; c++) G[v][c] += l * Ws[v * nf + fi] * L->Nout[c * nf + fi] / bd->w[id];
            }
          }
          for (int v = 0; v < 4; v++)
            for (int c = 0; c < 3; c++) gW[(v * 3 + c) * nn + o + p] = G[v][c] / L->J[o + p];
        }
    free(Wn);
  }

  free(qf);
  free(Ws);
}

/* A(Q); when 'scale' is given it receives, per node and variable, the round-off scale of that entry (divided
 * by J like A itself): the sum over the terms that make it up of a bound on each term's magnitude.  A term
 * that contracts a flux with a metric vector (J a^d in the volume, the scaled normal N on a face) is bounded
 * by Cauchy-Schwarz, |sum_c F_c V_c| <= |V| sum_c |F_c|: the metric components are differences of products
 * of the mapping's derivatives, so each carries rounding of the order of its vector's length, and a
 * component that vanishes exactly (the z-components of an extruded mesh) still moves the entry by that
 * much.  A face term also counts the magnitude of the numerical flux itself. */
/* operator evaluations since the last reset (a count for the tests' round-off bars; no arithmetic) */
long long or_n_evals = 0;

void or_operator_ex(const or_problem* P, const or_level* L, int isolated, const double* Q, double* A, double* scale) {
  const or_phys* ph = &P->ph;
  or_n_evals++;
  const int64_t nn = L->nn, nf = L->nf;
  double* qf = malloc(sizeof(double) * 5 * nf);
  double* gW = malloc(sizeof(double) * 12 * nn);  /* grad W at nodes, [k*3 + c][nn] */
  double* gf = malloc(sizeof(double) * 12 * nf);
  double* Phi = malloc(sizeof(double) * 5 * nf);  /* outward numerical flux x surface Jacobian */

  /* (1)-(3) traces, BR1 interface state, gradient */
  or_gradient(P, L, isolated, Q, gW);
  face_traces(P, L, Q, 5, qf);

  /* (4) traces of grad W */
  face_traces(P, L, gW, 12, gf);

  /* (5) numerical flux: Roe - {{F^v}} . n, times the surface Jacobian, on every face */
  for (int64_t e = 0; e < L->K; e++)
    for (int f = 0; f < 6; f++) {
      int n[3], d, t1, t2;
      elem_n(L, e, n);
      face_axes(f, &d, &t1, &t2);
      int nside = n[t1] * n[t2];
      int64_t fo = L->fo[6 * e + f];
      if (isolated) {
        for (int k = 0; k < nside; k++) {
          double q[5], g[4][3], Fa[3][5], Fv[3][5], N[3];
          qvec(qf, nf, fo + k, q);
          gvec(gf, nf, fo + k, g);
          for (int c = 0; c < 3; c++) N[c] = L->Nout[c * nf + fo + k];
          or_flux_adv(ph, q, Fa);
          or_flux_visc(ph, q, g, Fv);
          for (int v = 0; v < 5; v++) {
            double s = 0.0;
            for (int c = 0; c < 3; c++) s += (Fa[c][v] - Fv[c][v]) * N[c];
            Phi[v * nf + fo + k] = s;
          }
        }
        continue;
      }
      if (!is_master(P, e, f)) continue;
      int bc = P->bc[6 * e + f];
      if (P->nbr[6 * e + f] < 0) {
        for (int k = 0; k < nside; k++) {
          double q[5], qg[5], g[4][3], Fn[5], Fv[3][5], N[3], nh[3];
          qvec(qf, nf, fo + k, q);
          gvec(gf, nf, fo + k, g);
          for (int c = 0; c < 3; c++) N[c] = L->Nout[c * nf + fo + k];
          double Js = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          for (int c = 0; c < 3; c++) nh[c] = N[c] / Js;
          ghost(ph, bc, q, nh, qg);
          or_roe(ph, q, qg, nh, Fn);
          if (bc == 1) or_flux_visc_wall(ph, q, g, Fv);
          else if (bc == 3) memset(Fv, 0, sizeof(Fv));
          else or_flux_visc(ph, q, g, Fv);
          for (int v = 0; v < 5; v++) {
            double fv = Fv[0][v] * nh[0] + Fv[1][v] * nh[1] + Fv[2][v] * nh[2];
            Phi[v * nf + fo + k] = (Fn[v] - fv) * Js;
          }
        }
        continue;
      }
      or_mortar m;
      mortar_build(P, L, e, f, &m);
      int64_t foS = L->fo[6 * m.g + m.h];
      double* flux = malloc(sizeof(double) * 5 * m.nm);
      for (int mu = 0; mu < m.nm; mu++) {
        double qm[5], qs[5], gm[12], gs[12], N[3], nh[3], Fn[5], FvM[3][5], FvS[3][5];
        double GM[4][3], GS[4][3];
        to_mortar(m.WM, m.nM, mu, qf, nf, fo, 5, qm);
        to_mortar(m.WS, m.nS, mu, qf, nf, foS, 5, qs);
        to_mortar(m.WM, m.nM, mu, gf, nf, fo, 12, gm);
        to_mortar(m.WS, m.nS, mu, gf, nf, foS, 12, gs);
        to_mortar(m.WM, m.nM, mu, L->Nout, nf, fo, 3, N); /* master geometry on the mortar */
        for (int k = 0; k < 4; k++)
          for (int c = 0; c < 3; c++) { GM[k][c] = gm[k * 3 + c]; GS[k][c] = gs[k * 3 + c]; }
        double Js = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        for (int c = 0; c < 3; c++) nh[c] = N[c] / Js;
        or_roe(ph, qm, qs, nh, Fn);
        or_flux_visc(ph, qm, GM, FvM);
        or_flux_visc(ph, qs, GS, FvS);
        for (int v = 0; v < 5; v++) {
          double fv = 0.0;
          for (int c = 0; c < 3; c++) fv += 0.5 * (FvM[c][v] + FvS[c][v]) * nh[c];
          flux[v * m.nm + mu] = (Fn[v] - fv) * Js;
        }
      }
      for (int k = 0; k < m.nM; k++)
        for (int v = 0; v < 5; v++) {
          double s = 0.0;
          for (int mu = 0; mu < m.nm; mu++) s += m.PM[k * m.nm + mu] * flux[v * m.nm + mu];
          Phi[v * nf + fo + k] = s;
        }
      for (int k = 0; k < m.nS; k++)
        for (int v = 0; v < 5; v++) {
          double s = 0.0;
          for (int mu = 0; mu < m.nm; mu++) s += m.PS[k * m.nm + mu] * flux[v * m.nm + mu];
          Phi[v * nf + foS + k] = -s;
        }
      free(flux);
      mortar_free(&m);
    }

  /* round-off scale of each face term: |N| sum_c |(F^a - F^v)_c| of the own traces */
  double* fsc = NULL;
  if (scale) {
    fsc = malloc(sizeof(double) * 5 * nf);
    for (int64_t fi = 0; fi < nf; fi++) {
      double q[5], g[4][3], Fa[3][5], Fv[3][5];
      qvec(qf, nf, fi, q);
      gvec(gf, nf, fi, g);
      or_flux_adv(ph, q, Fa);
      or_flux_visc(ph, q, g, Fv);
      double N2 = 0.0;
      for (int c = 0; c < 3; c++) N2 += L->Nout[c * nf + fi] * L->Nout[c * nf + fi];
      for (int v = 0; v < 5; v++) {
        double a = 0.0;
        for (int c = 0; c < 3; c++) a += fabs(Fa[c][v] - Fv[c][v]);
        fsc[v * nf + fi] = sqrt(N2) * a;
      }
    }
  }

  /* (6) divergence of F^a - F^v: volume term + surface lift, divided by J */
  for (int64_t e = 0; e < L->K; e++) {
    int n[3];
    elem_n(L, e, n);
    const or_basis1d* b[3] = {&P->basis[n[0] - 1], &P->basis[n[1] - 1], &P->basis[n[2] - 1]};
    int64_t o = L->off[e];
    int npe = n[0] * n[1] * n[2];
    double* Ft = malloc(sizeof(double) * 15 * npe); /* Ftilde^d_v at the nodes: [(d*5 + v)][p] */
    double* Fs = malloc(sizeof(double) * 15 * npe); /* |J a^d| sum_c |F_c,v|: round-off scale of Ftilde^d_v */
    for (int p = 0; p < npe; p++) {
      double q[5], g[4][3], Fa[3][5], Fv[3][5];
      for (int v = 0; v < 5; v++) q[v] = Q[v * nn + o + p];
      for (int k = 0; k < 4; k++)
        for (int c = 0; c < 3; c++) g[k][c] = gW[(k * 3 + c) * nn + o + p];
      or_flux_adv(ph, q, Fa);
      or_flux_visc(ph, q, g, Fv);
      for (int d = 0; d < 3; d++) {
        double a2 = 0.0;
        for (int c = 0; c < 3; c++) a2 += L->Ja[(d * 3 + c) * nn + o + p] * L->Ja[(d * 3 + c) * nn + o + p];
        for (int v = 0; v < 5; v++) {
          double s = 0.0, f = 0.0;
          for (int c = 0; c < 3; c++) {
            s += L->Ja[(d * 3 + c) * nn + o + p] * (Fa[c][v] - Fv[c][v]);
            f += fabs(Fa[c][v] - Fv[c][v]);
          }
          Ft[(d * 5 + v) * npe + p] = s;
          Fs[(d * 5 + v) * npe + p] = sqrt(a2) * f;
        }
      }
    }
    for (int k3 = 0; k3 < n[2]; k3++)
      for (int j = 0; j < n[1]; j++)
        for (int i = 0; i < n[0]; i++) {
          int ijk[3] = {i, j, k3};
          int64_t p = vidx(n, i, j, k3);
          double s[5] = {0, 0, 0, 0, 0}, sa[5] = {0, 0, 0, 0, 0};
          for (int d = 0; d < 3; d++) {
            const or_basis1d* bd = b[d];
            int id = ijk[d];
            for (int m = 0; m < n[d]; m++) {
              int q3[3] = {i, j, k3};
              q3[d] = m;
              int64_t pm = vidx(n, q3[0], q3[1], q3[2]);
              double Dh = -bd->D[m][id] * bd->w[m] / bd->w[id];
              for (int v = 0; v < 5; v++) {
                s[v] += Dh * Ft[(d * 5 + v) * npe + pm];
                sa[v] += fabs(Dh) * Fs[(d * 5 + v) * npe + pm];
              }
            }
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int64_t fk = ijk[t1] + (int64_t)n[t1] * ijk[t2];
            for (int side = 0; side < 2; side++) {
              int64_t fi = L->fo[6 * e + 2 * d + side] + fk;
              double l = side ? bd->lp[id] : bd->lm[id];
              for (int v = 0; v < 5; v++) {
                s[v] += l * Phi[v * nf + fi] / bd->w[id];
                if (fsc) sa[v] += fabs(l / bd->w[id]) * (fabs(Phi[v * nf + fi]) + fsc[v * nf + fi]);
              }
            }
          }
          for (int v = 0; v < 5; v++) A[v * nn + o + p] = s[v] / L->J[o + p];
          if (scale)
            for (int v = 0; v < 5; v++) scale[v * nn + o + p] = sa[v] / fabs(L->J[o + p]);
        }
    free(Ft);
    free(Fs);
  }
  free(qf); free(gW); free(gf); free(Phi); free(fsc);
}

void or_operator(const or_problem* P, const or_level* L, int isolated, const double* Q, double* A) {
  or_operator_ex(P, L, isolated, Q, A, NULL);
}

/*
 * CFL time step (paper, Sec. 2): dt = min(dt^a, dt^nu) over every node and direction, with
 *   dt^a = C^a h_d / ((|v| + c) N_d^2),  dt^nu = C^nu h_d^2 / (nu N_d^4),
 * h_d = 2 J / |J a^d| (the element size along xi_d), nu = mu(T) / (rho Re).  The most restrictive wins.
 */
double or_timestep(const or_problem* P, const or_level* L, const double* Q) {
  const or_phys* ph = &P->ph;
  double dt = INFINITY;
  for (int64_t e = 0; e < L->K; e++) {
    int64_t o = L->off[e];
    int64_t npe = L->off[e + 1] - o;
    for (int64_t p = 0; p < npe; p++) {
      double q[5], rho, v[3], pr, T;
      for (int c = 0; c < 5; c++) q[c] = Q[c * L->nn + o + p];
      or_prim(ph, q, &rho, v, &pr, &T);
      double speed = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + sqrt(ph->gamma * pr / rho);
      double nu = or_mu(ph, T) / (rho * ph->reynolds);
      for (int d = 0; d < 3; d++) {
        double a0 = L->Ja[(d * 3 + 0) * L->nn + o + p];
        double a1 = L->Ja[(d * 3 + 1) * L->nn + o + p];
        double a2 = L->Ja[(d * 3 + 2) * L->nn + o + p];
        double h = 2.0 * L->J[o + p] / sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        double N = L->ord[3 * e + d];
        double dta = ph->cfl_adv * h / (speed * N * N);
        double dtv = ph->cfl_visc * h * h / (nu * N * N * N * N);
        if (dta < dt) dt = dta;
        if (dtv < dt) dt = dtv;
      }
    }
  }
  return dt;
}

/*
 * Force of the fluid on the no-slip walls (the drag and lift coefficients of Secs. 4.1 and 4.2 are its
 * components over the dynamic pressure and a reference area): the surface integral over every wall face of
 * p n - tau . n, with n the element's outward unit normal (into the wall), p and the viscous stress
 * tau = (mu / Re)(grad v + grad v^T - 2/3 div v I) from the element's own traces of the state and of its BR1
 * gradient, and the Gauss quadrature of the face nodes with the surface Jacobian.
 * out[0..2]: pressure part, out[3..5]: viscous part, out[6..11]: the round-off scale of each component, the
 * sum over the nodes of the magnitude of the node's vector term (w J_s |p| for the pressure part, w J_s |tau . n|
 * for the viscous part): rounding moves a node's term relative to its length, whatever its direction.
 */
void or_wall_force(const or_problem* P, const or_level* L, const double* Q, double out[12]) {
  const or_phys* ph = &P->ph;
  const int64_t nn = L->nn, nf = L->nf;
  double* qf = malloc(sizeof(double) * 5 * nf);
  double* gW = malloc(sizeof(double) * 12 * nn);
  double* gf = malloc(sizeof(double) * 12 * nf);
  or_gradient(P, L, 0, Q, gW);
  face_traces(P, L, Q, 5, qf);
  face_traces(P, L, gW, 12, gf);
  for (int i = 0; i < 12; i++) out[i] = 0.0;
  for (int64_t e = 0; e < L->K; e++)
    for (int f = 0; f < 6; f++) {
      if (P->nbr[6 * e + f] >= 0 || P->bc[6 * e + f] != 1) continue;
      int n[3], d, t1, t2;
      elem_n(L, e, n);
      face_axes(f, &d, &t1, &t2);
      const or_basis1d* bs = &P->basis[n[t1] - 1];
      const or_basis1d* bt = &P->basis[n[t2] - 1];
      for (int b = 0; b < n[t2]; b++)
        for (int a = 0; a < n[t1]; a++) {
          int64_t fi = L->fo[6 * e + f] + a + (int64_t)n[t1] * b;
          double q[5], g[4][3], N[3], nh[3], Fv[3][5], rho, v[3], p, T;
          qvec(qf, nf, fi, q);
          gvec(gf, nf, fi, g);
          for (int c = 0; c < 3; c++) N[c] = L->Nout[c * nf + fi];
          double Js = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
          for (int c = 0; c < 3; c++) nh[c] = N[c] / Js;
          or_prim(ph, q, &rho, v, &p, &T);
          or_flux_visc(ph, q, g, Fv);
          double w = bs->w[a] * bt->w[b] * Js, tn[3];
          for (int i = 0; i < 3; i++) {
            tn[i] = Fv[0][1 + i] * nh[0] + Fv[1][1 + i] * nh[1] + Fv[2][1 + i] * nh[2];
            out[i] += w * p * nh[i];
            out[3 + i] -= w * tn[i];
          }
          double tl = sqrt(tn[0] * tn[0] + tn[1] * tn[1] + tn[2] * tn[2]);
          for (int i = 0; i < 3; i++) {
            out[6 + i] += fabs(w * p);
            out[9 + i] += w * tl;
          }
        }
    }
  free(qf);
  free(gW);
  free(gf);
}
