/*
 * Oracle (test infrastructure): smoother, transfers, FAS V-cycle, in-cycle truncation error, solve driver.
 *
 * Paper, Sec. 3.1: steady problem A(Q) = S, nonlinear residual r = S - A(Q~); FAS two-level scheme with
 * coarse source S^N = A^N(I Q~) + I r, iteration error eps = Q~^N - Q~^N_0 (the equation's sign; the last
 * line of the printed algorithm writes the opposite sign, which would undo the coarse correction), fine
 * correction Q <- Q + I eps; recursive V-cycle with pre- and post-smoothing (Algorithm "FAS: V-Cycle");
 * Williamson's low-storage RK3 as smoother; L2 projection as restriction of both solution and residual,
 * exact interpolation as prolongation; Delta N = 1 with high-order coarsening (Sec. 3.3.3): the level with
 * cap l keeps every order <= l and lowers the others to l, in all directions (isotropic cycle) or in one
 * direction (anisotropic cycle).  Residual-based smoothing tuning and FMG start (Secs. 3.1.1-3.1.2).
 * Truncation error estimate inside the cycle (Secs. 3.2.1 and 3.3.1): at the entry of every coarse level,
 *   tau = S_phys - A^N(I Q~)   (non-isolated, reusing the A^N(I Q~) of the coarse source), or
 *   tau^ = S_phys - A^^N(I Q~) (isolated, one extra isolated operator evaluation),
 * with the physical source restricted level by level; one value per element, direction and order: the
 * maximum over nodes and variables of |tau|.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#include "oracle_mg.h"

static const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

void or_residual(const or_problem* P, const or_level* L, int isolated, const double* Q, const double* S, double* R) {
  or_operator(P, L, isolated, Q, R);
  int64_t n = 5 * L->nn;
  for (int64_t i = 0; i < n; i++) R[i] = (S ? S[i] : 0.0) - R[i];
}

double or_norm_inf(const double* R, int64_t n) {
  double m = 0.0;
  for (int64_t i = 0; i < n; i++) {
    double a = fabs(R[i]);
    if (a > m || a != a) m = a;
  }
  return m;
}

/* One sweep of Williamson's 3-stage low-storage RK3 with the step frozen for the sweep:
 *   G <- a_s G + dt R(Q);  Q <- Q + b_s G,  a = (0, -5/9, -153/128),  b = (1/3, 15/16, 8/15). */
typedef void (*or_rhs_fn)(void* ctx, const double* Q, double* R);

void or_rk3_sweep(or_rhs_fn rhs, void* ctx, double* Q, int64_t n, double dt, double* G, double* R) {
  memset(G, 0, sizeof(double) * n);
  for (int s = 0; s < 3; s++) {
    rhs(ctx, Q, R);
    for (int64_t i = 0; i < n; i++) {
      G[i] = RK_A[s] * G[i] + dt * R[i];
      Q[i] = Q[i] + RK_B[s] * G[i];
    }
  }
}

typedef struct { const or_problem* P; const or_level* L; const double* S; } dg_rhs_ctx;
static void dg_rhs(void* c, const double* Q, double* R) {
  dg_rhs_ctx* x = (dg_rhs_ctx*)c;
  or_residual(x->P, x->L, 0, Q, x->S, R);
}

/* beta smoothing sweeps; the CFL step is taken from Q at the start of each sweep */
void or_smooth(const or_problem* P, const or_level* L, double* Q, const double* S, int sweeps) {
  int64_t n = 5 * L->nn;
  double* G = malloc(sizeof(double) * n);
  double* R = malloc(sizeof(double) * n);
  dg_rhs_ctx ctx = {P, L, S};
  for (int it = 0; it < sweeps; it++) {
    double dt = or_timestep(P, L, Q);
    or_rk3_sweep(dg_rhs, &ctx, Q, n, dt, G, R);
  }
  free(G);
  free(R);
}

/* Tensor-product transfer of an nvar-field between two order tensors on the same mesh.
 * prolong = 0: L2 projection (fine -> coarse); prolong = 1: interpolation (coarse -> fine);
 * prolong = 2: direction by direction, interpolation where the order rises and L2 projection where it falls
 * (the state carried over to the new orders after an adaptation, Sec. 3.3). */
static void transfer(const or_problem* P, const or_level* Lfrom, const or_level* Lto, const double* U, double* V,
                     int nvar, int prolong) {
  for (int64_t e = 0; e < Lfrom->K; e++) {
    int a[3], b[3];
    for (int d = 0; d < 3; d++) { a[d] = Lfrom->ord[3 * e + d] + 1; b[d] = Lto->ord[3 * e + d] + 1; }
    double T[3][OR_MAXN * OR_MAXN]; /* T[d][to][from] */
    for (int d = 0; d < 3; d++) {
      const or_basis1d* bf = &P->basis[a[d] - 1];
      const or_basis1d* bt = &P->basis[b[d] - 1];
      if (a[d] == b[d]) {
        for (int i = 0; i < b[d]; i++)
          for (int j = 0; j < a[d]; j++) T[d][i * a[d] + j] = (i == j) ? 1.0 : 0.0;
      } else if (prolong == 1 || (prolong == 2 && b[d] > a[d])) {
        or_interp_matrix(bf, bt->x, bt->n, T[d]); /* T[to][from] = l_from(x_to) */
      } else {
        or_projection_matrix(bt, bf, T[d]);       /* R[coarse][fine] */
      }
    }
    int64_t of = Lfrom->off[e], ot = Lto->off[e];
    for (int v = 0; v < nvar; v++)
      for (int k = 0; k < b[2]; k++)
        for (int j = 0; j < b[1]; j++)
          for (int i = 0; i < b[0]; i++) {
            double s = 0.0;
            for (int kk = 0; kk < a[2]; kk++)
              for (int jj = 0; jj < a[1]; jj++)
                for (int ii = 0; ii < a[0]; ii++)
                  s += T[0][i * a[0] + ii] * T[1][j * a[1] + jj] * T[2][k * a[2] + kk] *
                       U[v * Lfrom->nn + of + ii + (int64_t)a[0] * (jj + (int64_t)a[1] * kk)];
            V[v * Lto->nn + ot + i + (int64_t)b[0] * (j + (int64_t)b[1] * k)] = s;
          }
  }
}

void or_restrict(const or_problem* P, const or_level* Lf, const or_level* Lc, const double* Uf, double* Uc) {
  transfer(P, Lf, Lc, Uf, Uc, 5, 0);
}
void or_prolong(const or_problem* P, const or_level* Lc, const or_level* Lf, const double* Uc, double* Uf) {
  transfer(P, Lc, Lf, Uc, Uf, 5, 1);
}
void or_remap(const or_problem* P, const or_level* La, const or_level* Lb, const double* Ua, double* Ub) {
  transfer(P, La, Lb, Ua, Ub, 5, 2);
}

/* ---------------------------------------------------------------------------------------------------- */
or_mg* or_mg_create(const or_problem* P, const int32_t* ord, int nlev, const int* caps, int aniso_dir) {
  or_mg* mg = calloc(1, sizeof(or_mg));
  mg->nlev = nlev;
  mg->dir = aniso_dir;
  mg->caps = malloc(sizeof(int) * nlev);
  mg->L = calloc(nlev, sizeof(or_level*));
  mg->Q = calloc(nlev, sizeof(double*));
  mg->Q0 = calloc(nlev, sizeof(double*));
  mg->S = calloc(nlev, sizeof(double*));
  mg->r = calloc(nlev, sizeof(double*));
  mg->Sphys = calloc(nlev, sizeof(double*));
  int64_t K = P->K;
  int32_t* o = malloc(sizeof(int32_t) * 3 * K);
  /* caps[0] is the finest level; level index l = nlev-1 (finest) ... 0 (coarsest) */
  for (int l = 0; l < nlev; l++) {
    int cap = caps[nlev - 1 - l];
    mg->caps[l] = cap;
    for (int64_t e = 0; e < K; e++)
      for (int d = 0; d < 3; d++) {
        int p = ord[3 * e + d];
        int capped = (aniso_dir < 0 || aniso_dir == d) && p > cap;
        o[3 * e + d] = (l == nlev - 1) ? p : (capped ? cap : p);
      }
    mg->L[l] = or_level_create(P, o);
    int64_t n = 5 * mg->L[l]->nn;
    mg->Q[l] = calloc(n, sizeof(double));
    mg->Q0[l] = calloc(n, sizeof(double));
    mg->S[l] = calloc(n, sizeof(double));
    mg->r[l] = calloc(n, sizeof(double));
    mg->Sphys[l] = calloc(n, sizeof(double));
  }
  free(o);
  return mg;
}

void or_mg_destroy(or_mg* mg) {
  for (int l = 0; l < mg->nlev; l++) {
    or_level_destroy(mg->L[l]);
    free(mg->Q[l]); free(mg->Q0[l]); free(mg->S[l]); free(mg->r[l]); free(mg->Sphys[l]);
  }
  free(mg->L); free(mg->Q); free(mg->Q0); free(mg->S); free(mg->r); free(mg->Sphys); free(mg->caps);
  free(mg->reps); free(mg->fmg_cycles);
  free(mg);
}

static void record_tau(const or_problem* P, const or_mg* mg, int l, const double* tau, double* tau_map, int nt) {
  const or_level* L = mg->L[l];
  const or_level* Ltop = mg->L[mg->nlev - 1];
  int cap = mg->caps[l];
  for (int64_t e = 0; e < L->K; e++) {
    int Pd = Ltop->ord[3 * e + mg->dir];
    if (cap >= Pd || cap < 1 || cap > nt) continue;
    double m = 0.0;
    for (int v = 0; v < 5; v++)
      for (int64_t p = L->off[e]; p < L->off[e + 1]; p++) {
        double a = fabs(tau[v * L->nn + p]);
        if (a > m || a != a) m = a;
      }
    tau_map[(e * 3 + mg->dir) * nt + (cap - 1)] = m;
  }
}

/* Smoothing with the residual-based tuning of Sec. 3.1.2 when prm->tuning is set. */
static void pre_smooth(const or_problem* P, or_mg* mg, int l, const or_mg_params* prm, double* Rfine, double* rnorm_pre) {
  const or_level* L = mg->L[l];
  int64_t n = 5 * L->nn;
  if (!prm->tuning || l == 0) {
    or_smooth(P, L, mg->Q[l], mg->S[l], l == 0 ? prm->beta_coarse : prm->beta_pre);
    or_residual(P, L, 0, mg->Q[l], mg->S[l], Rfine);
    *rnorm_pre = or_norm_inf(Rfine, n);
    if (mg->reps) mg->reps[2 * l] = 1;
    return;
  }
  /* pre-smoothing stops once ||r^P|| < eta ||I r^P|| (residual checked in the next coarser representation) */
  const or_level* Lc = mg->L[l - 1];
  double* rc = malloc(sizeof(double) * 5 * Lc->nn);
  int blocks = 0;
  for (int rep = 0; rep < prm->max_repeats; rep++) {
    or_smooth(P, L, mg->Q[l], mg->S[l], prm->beta_pre);
    blocks++;
    or_residual(P, L, 0, mg->Q[l], mg->S[l], Rfine);
    or_restrict(P, L, Lc, Rfine, rc);
    if (or_norm_inf(Rfine, n) < prm->eta * or_norm_inf(rc, 5 * Lc->nn)) break;
  }
  if (mg->reps) mg->reps[2 * l] = blocks;
  *rnorm_pre = or_norm_inf(Rfine, n);
  free(rc);
}

static void post_smooth(const or_problem* P, or_mg* mg, int l, const or_mg_params* prm, double rnorm_pre) {
  const or_level* L = mg->L[l];
  if (!prm->tuning) {
    or_smooth(P, L, mg->Q[l], mg->S[l], prm->beta_post);
    if (mg->reps) mg->reps[2 * l + 1] = 1;
    return;
  }
  /* post-smoothing stops once ||r_post|| <= ||r_pre|| */
  int64_t n = 5 * L->nn;
  double* R = malloc(sizeof(double) * n);
  int blocks = 0;
  for (int rep = 0; rep < prm->max_repeats; rep++) {
    or_smooth(P, L, mg->Q[l], mg->S[l], prm->beta_post);
    blocks++;
    or_residual(P, L, 0, mg->Q[l], mg->S[l], R);
    if (or_norm_inf(R, n) <= rnorm_pre) break;
  }
  if (mg->reps) mg->reps[2 * l + 1] = blocks;
  free(R);
}

/* Recursive FAS V-cycle on level l (Algorithm "FAS: V-Cycle"); mg->Q[l], mg->r[l] are inputs. */
static void vcycle(const or_problem* P, or_mg* mg, int l, int top, const or_mg_params* prm, double* tau_map, int nt) {
  const or_level* L = mg->L[l];
  int64_t n = 5 * L->nn;
  double* tmp = malloc(sizeof(double) * n);
  if (l < top) {
    /* coarse source S = A(Q~) + r, and the truncation error from the same A(Q~) */
    or_operator(P, L, 0, mg->Q[l], tmp);
    for (int64_t i = 0; i < n; i++) mg->S[l][i] = tmp[i] + mg->r[l][i];
    if (tau_map) {
      if (prm->isolated) or_operator(P, L, 1, mg->Q[l], tmp);
      for (int64_t i = 0; i < n; i++) tmp[i] = mg->Sphys[l][i] - tmp[i];
      record_tau(P, mg, l, tmp, tau_map, nt);
      if (mg->tau_nodal && mg->caps[l] == mg->tau_nodal_cap) memcpy(mg->tau_nodal, tmp, sizeof(double) * n);
    }
  }
  memcpy(mg->Q0[l], mg->Q[l], sizeof(double) * n);
  double rpre = 0.0;
  pre_smooth(P, mg, l, prm, tmp, &rpre); /* tmp <- S - A(Q~) after pre-smoothing */
  if (l > 0) {
    const or_level* Lc = mg->L[l - 1];
    or_restrict(P, L, Lc, mg->Q[l], mg->Q[l - 1]);
    or_restrict(P, L, Lc, tmp, mg->r[l - 1]);
    vcycle(P, mg, l - 1, top, prm, tau_map, nt);
    int64_t nc = 5 * Lc->nn;
    double* eps = malloc(sizeof(double) * nc);
    for (int64_t i = 0; i < nc; i++) eps[i] = mg->Q[l - 1][i] - mg->Q0[l - 1][i];
    or_prolong(P, Lc, L, eps, tmp);
    for (int64_t i = 0; i < n; i++) mg->Q[l][i] += tmp[i];
    free(eps);
    post_smooth(P, mg, l, prm, rpre);
  }
  free(tmp);
}

/* Restrict the physical source level by level (S_phys at the top; zero when absent). */
static void set_sources(const or_problem* P, or_mg* mg, const double* S) {
  int top = mg->nlev - 1;
  int64_t n = 5 * mg->L[top]->nn;
  for (int64_t i = 0; i < n; i++) mg->Sphys[top][i] = S ? S[i] : 0.0;
  for (int l = top; l > 0; l--) or_restrict(P, mg->L[l], mg->L[l - 1], mg->Sphys[l], mg->Sphys[l - 1]);
}

double or_mg_vcycles(const or_problem* P, or_mg* mg, double* Q, const double* S, int ncycles, const or_mg_params* prm,
                     double* tau_map, int nt) {
  int top = mg->nlev - 1;
  int64_t n = 5 * mg->L[top]->nn;
  set_sources(P, mg, S);
  memcpy(mg->Q[top], Q, sizeof(double) * n);
  memcpy(mg->S[top], mg->Sphys[top], sizeof(double) * n);
  for (int c = 0; c < ncycles; c++) vcycle(P, mg, top, top, prm, tau_map, nt);
  memcpy(Q, mg->Q[top], sizeof(double) * n);
  double* R = malloc(sizeof(double) * n);
  or_residual(P, mg->L[top], 0, Q, S, R);
  double r = or_norm_inf(R, n);
  free(R);
  return r;
}

/* Steady solve: optional FMG start (raise a level once ||r|| < fmg_threshold), then V-cycles to tol. */
int or_mg_solve(const or_problem* P, or_mg* mg, double* Q, const double* S, double tol, int max_cycles,
                const or_mg_params* prm, double* res_out, double* history) {
  int top = mg->nlev - 1;
  int64_t n = 5 * mg->L[top]->nn;
  set_sources(P, mg, S);
  memcpy(mg->Q[top], Q, sizeof(double) * n);
  int cycles = 0;
  double r = 0.0;
  if (prm->fmg) {
    for (int l = top; l > 0; l--) or_restrict(P, mg->L[l], mg->L[l - 1], mg->Q[l], mg->Q[l - 1]);
    for (int l = 0; l < top; l++) {
      int64_t nl = 5 * mg->L[l]->nn;
      double* R = malloc(sizeof(double) * nl);
      memcpy(mg->S[l], mg->Sphys[l], sizeof(double) * nl);
      for (;;) {
        or_residual(P, mg->L[l], 0, mg->Q[l], mg->Sphys[l], R);
        r = or_norm_inf(R, nl);
        if (r < prm->fmg_threshold || cycles >= max_cycles) break;
        vcycle(P, mg, l, l, prm, NULL, 0);
        cycles++;
        if (mg->fmg_cycles) mg->fmg_cycles[l]++;
      }
      free(R);
      or_prolong(P, mg->L[l], mg->L[l + 1], mg->Q[l], mg->Q[l + 1]);
    }
  }
  memcpy(mg->S[top], mg->Sphys[top], sizeof(double) * n);
  double* R = malloc(sizeof(double) * n);
  for (;;) {
    or_residual(P, mg->L[top], 0, mg->Q[top], S, R);
    r = or_norm_inf(R, n);
    if (history && cycles < max_cycles) history[cycles] = r;
    if (r < tol || cycles >= max_cycles) break;
    vcycle(P, mg, top, top, prm, NULL, 0);
    cycles++;
  }
  free(R);
  memcpy(Q, mg->Q[top], sizeof(double) * n);
  *res_out = r;
  return cycles;
}
