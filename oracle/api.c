/*
 * Oracle (test infrastructure): flat entry points for the Python test harness (ctypes).
 * Arrays are host arrays in the layouts of the C-ABI: Q[5][n_nodes], orders[K][3], tau[K][3][nt].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#include "oracle_mg.h"

or_problem* ora_create(int64_t K, const int32_t* M, const double* gnodes, const int64_t* nbr, const int32_t* nbrf,
                       const int32_t* orient, const int32_t* bc, const or_phys* ph) {
  or_problem* P = calloc(1, sizeof(or_problem));
  P->K = K;
  for (int d = 0; d < 3; d++) P->M[d] = M[d];
  int64_t ng = K * (M[0] + 1) * (M[1] + 1) * (M[2] + 1) * 3;
  P->gnodes = malloc(sizeof(double) * ng);
  memcpy(P->gnodes, gnodes, sizeof(double) * ng);
  P->nbr = malloc(sizeof(int64_t) * 6 * K);
  P->nbrf = malloc(sizeof(int32_t) * 6 * K);
  P->orient = malloc(sizeof(int32_t) * 6 * K);
  P->bc = malloc(sizeof(int32_t) * 6 * K);
  memcpy(P->nbr, nbr, sizeof(int64_t) * 6 * K);
  memcpy(P->nbrf, nbrf, sizeof(int32_t) * 6 * K);
  memcpy(P->orient, orient, sizeof(int32_t) * 6 * K);
  memcpy(P->bc, bc, sizeof(int32_t) * 6 * K);
  P->ph = *ph;
  for (int o = 0; o < OR_MAXN; o++) {
    if (o == 0 && ph->family == 1) continue;
    or_make_basis(o, ph->family, &P->basis[o]);
  }
  return P;
}

void ora_destroy(or_problem* P) {
  if (!P) return;
  free(P->gnodes); free(P->nbr); free(P->nbrf); free(P->orient); free(P->bc);
  free(P);
}

void ora_basis(int order, int family, double* x, double* w, double* D, double* lm, double* lp) {
  or_basis1d b;
  or_make_basis(order, family, &b);
  for (int i = 0; i < b.n; i++) {
    x[i] = b.x[i]; w[i] = b.w[i]; lm[i] = b.lm[i]; lp[i] = b.lp[i];
    for (int j = 0; j < b.n; j++) D[i * b.n + j] = b.D[i][j];
  }
}

void ora_projection(int nc_order, int nf_order, int family, double* R) {
  or_basis1d c, f;
  or_make_basis(nc_order, family, &c);
  or_make_basis(nf_order, family, &f);
  or_projection_matrix(&c, &f, R);
}

void ora_interp(int from_order, int to_order, int family, double* I) {
  or_basis1d a, b;
  or_make_basis(from_order, family, &a);
  or_make_basis(to_order, family, &b);
  or_interp_matrix(&a, b.x, b.n, I);
}

int64_t ora_level_sizes(or_problem* P, const int32_t* ord, int64_t* nf_out) {
  or_level* L = or_level_create(P, ord);
  int64_t nn = L->nn;
  *nf_out = L->nf;
  or_level_destroy(L);
  return nn;
}

void ora_geometry(or_problem* P, const int32_t* ord, double* X, double* Ja, double* J, double* Nout) {
  or_level* L = or_level_create(P, ord);
  memcpy(X, L->X, sizeof(double) * 3 * L->nn);
  memcpy(Ja, L->Ja, sizeof(double) * 9 * L->nn);
  memcpy(J, L->J, sizeof(double) * L->nn);
  memcpy(Nout, L->Nout, sizeof(double) * 3 * L->nf);
  or_level_destroy(L);
}

void ora_operator(or_problem* P, const int32_t* ord, int isolated, const double* Q, double* A) {
  or_level* L = or_level_create(P, ord);
  or_operator(P, L, isolated, Q, A);
  or_level_destroy(L);
}

void ora_residual(or_problem* P, const int32_t* ord, int isolated, const double* Q, const double* S, double* R) {
  or_level* L = or_level_create(P, ord);
  or_residual(P, L, isolated, Q, S, R);
  or_level_destroy(L);
}

double ora_timestep(or_problem* P, const int32_t* ord, const double* Q) {
  or_level* L = or_level_create(P, ord);
  double dt = or_timestep(P, L, Q);
  or_level_destroy(L);
  return dt;
}

void ora_smooth(or_problem* P, const int32_t* ord, double* Q, const double* S, int sweeps) {
  or_level* L = or_level_create(P, ord);
  or_smooth(P, L, Q, S, sweeps);
  or_level_destroy(L);
}

void ora_transfer(or_problem* P, const int32_t* ord_from, const int32_t* ord_to, int prolong, const double* U, double* V) {
  or_level* A = or_level_create(P, ord_from);
  or_level* B = or_level_create(P, ord_to);
  if (prolong == 2) or_remap(P, A, B, U, V);
  else if (prolong) or_prolong(P, A, B, U, V);
  else or_restrict(P, A, B, U, V);
  or_level_destroy(A);
  or_level_destroy(B);
}

void ora_roe(const or_phys* ph, const double* qL, const double* qR, const double* n, double* F) { or_roe(ph, qL, qR, n, F); }

void ora_flux(const or_phys* ph, const double* q, const double* gW, double* Fa, double* Fv) {
  double A[3][5], V[3][5], g[4][3];
  for (int k = 0; k < 4; k++)
    for (int c = 0; c < 3; c++) g[k][c] = gW[k * 3 + c];
  or_flux_adv(ph, q, A);
  or_flux_visc(ph, q, g, V);
  for (int c = 0; c < 3; c++)
    for (int v = 0; v < 5; v++) { Fa[c * 5 + v] = A[c][v]; Fv[c * 5 + v] = V[c][v]; }
}

/* caps[0] = finest cap ... caps[nlev-1] = coarsest; dir = -1 isotropic */
double ora_vcycles(or_problem* P, const int32_t* ord, int nlev, const int32_t* caps, int dir, const or_mg_params* prm,
                   double* Q, const double* S, int ncycles) {
  int* c = malloc(sizeof(int) * nlev);
  for (int l = 0; l < nlev; l++) c[l] = caps[l];
  or_mg* mg = or_mg_create(P, ord, nlev, c, dir);
  double r = or_mg_vcycles(P, mg, Q, S, ncycles, prm, NULL, 0);
  or_mg_destroy(mg);
  free(c);
  return r;
}

/* Anisotropic 3V cycle: one V-cycle per direction, coarsening that direction only (caps P_d^max .. 1),
 * each starting from the result of the previous one.  tau_map[K][3][nt] (NaN where not estimated). */
void ora_tau_3v(or_problem* P, const int32_t* ord, const or_mg_params* prm, double* Q, const double* S, double* tau_map,
                int nt) {
  int64_t K = P->K;
  for (int64_t i = 0; i < K * 3 * nt; i++) tau_map[i] = NAN;
  for (int d = 0; d < 3; d++) {
    int pmax = 1;
    for (int64_t e = 0; e < K; e++)
      if (ord[3 * e + d] > pmax) pmax = ord[3 * e + d];
    int nlev = pmax;
    if (nlev < 2) continue;
    int* caps = malloc(sizeof(int) * nlev);
    for (int l = 0; l < nlev; l++) caps[l] = pmax - l;
    or_mg* mg = or_mg_create(P, ord, nlev, caps, d);
    or_mg_vcycles(P, mg, Q, S, 1, prm, tau_map, nt);
    or_mg_destroy(mg);
    free(caps);
  }
}

/* One anisotropic V-cycle in direction d (levels max N_d down to 1, as in ora_tau_3v) that also copies the
 * pointwise truncation error of the level capped at 'cap' into tau_nodal ([5][nn of that level]). */
void ora_tau_nodal(or_problem* P, const int32_t* ord, const or_mg_params* prm, double* Q, const double* S, int d,
                   int cap, double* tau_nodal) {
  int64_t K = P->K;
  int pmax = 1;
  for (int64_t e = 0; e < K; e++)
    if (ord[3 * e + d] > pmax) pmax = ord[3 * e + d];
  int nlev = pmax;
  if (nlev < 2) return;
  int nt = pmax - 1;
  double* tau_map = malloc(sizeof(double) * K * 3 * nt);
  for (int64_t i = 0; i < K * 3 * nt; i++) tau_map[i] = NAN;
  int* caps = malloc(sizeof(int) * nlev);
  for (int l = 0; l < nlev; l++) caps[l] = pmax - l;
  or_mg* mg = or_mg_create(P, ord, nlev, caps, d);
  mg->tau_nodal = tau_nodal;
  mg->tau_nodal_cap = cap;
  or_mg_vcycles(P, mg, Q, S, 1, prm, tau_map, nt);
  mg->tau_nodal = NULL;
  or_mg_destroy(mg);
  free(caps);
  free(tau_map);
}

/* Steady solve; reps (nullable, 2 * nlev): smoothing blocks of the last visit of each level (pre, post; level
   index 0 = coarsest); fmg_cycles (nullable, nlev): V-cycles the FMG start ran on each level. */
int ora_solve_ex(or_problem* P, const int32_t* ord, int nlev, const int32_t* caps, const or_mg_params* prm, double* Q,
                 const double* S, double tol, int max_cycles, double* res_out, double* history, int32_t* reps,
                 int32_t* fmg_cycles) {
  int* c = malloc(sizeof(int) * nlev);
  for (int l = 0; l < nlev; l++) c[l] = caps[l];
  or_mg* mg = or_mg_create(P, ord, nlev, c, -1);
  mg->reps = calloc(2 * nlev, sizeof(int));
  mg->fmg_cycles = calloc(nlev, sizeof(int));
  int cyc = or_mg_solve(P, mg, Q, S, tol, max_cycles, prm, res_out, history);
  for (int l = 0; l < nlev; l++) {
    if (reps) { reps[2 * l] = mg->reps[2 * l]; reps[2 * l + 1] = mg->reps[2 * l + 1]; }
    if (fmg_cycles) fmg_cycles[l] = mg->fmg_cycles[l];
  }
  or_mg_destroy(mg);
  free(c);
  return cyc;
}

int ora_solve(or_problem* P, const int32_t* ord, int nlev, const int32_t* caps, const or_mg_params* prm, double* Q,
              const double* S, double tol, int max_cycles, double* res_out, double* history) {
  return ora_solve_ex(P, ord, nlev, caps, prm, Q, S, tol, max_cycles, res_out, history, NULL, NULL);
}

/* Test hook: one RK3 sweep of the linear residual R(Q) = lambda Q. */
typedef void (*or_rhs_fn)(void* ctx, const double* Q, double* R);
void or_rk3_sweep(or_rhs_fn rhs, void* ctx, double* Q, int64_t n, double dt, double* G, double* R);
static void lin_rhs(void* c, const double* Q, double* R) { R[0] = *(const double*)c * Q[0]; }
double ora_rk3_linear(double lambda, double dt, double q0) {
  double Q = q0, G, R;
  or_rk3_sweep(lin_rhs, &lambda, &Q, 1, dt, &G, &R);
  return Q;
}

/* BR1 gradient of W = (u, v, w, T) at the nodes, [12][nn] with row k*3 + c = dW_k/dx_c. */
void or_gradient(const or_problem* P, const or_level* L, int isolated, const double* Q, double* gW);
void ora_gradient(or_problem* P, const int32_t* ord, int isolated, const double* Q, double* gW) {
  or_level* L = or_level_create(P, ord);
  or_gradient(P, L, isolated, Q, gW);
  or_level_destroy(L);
}

/* Operator and the per-entry magnitude of its terms (round-off scale). */
void or_operator_ex(const or_problem* P, const or_level* L, int isolated, const double* Q, double* A, double* scale);
void ora_operator_scale(or_problem* P, const int32_t* ord, int isolated, const double* Q, double* A, double* scale) {
  or_level* L = or_level_create(P, ord);
  or_operator_ex(P, L, isolated, Q, A, scale);
  or_level_destroy(L);
}

/* Force on the no-slip walls: pressure part, viscous part, and the absolute sums of their terms (12 values). */
void ora_wall_force(or_problem* P, const int32_t* ord, const double* Q, double* out) {
  or_level* L = or_level_create(P, ord);
  or_wall_force(P, L, Q, out);
  or_level_destroy(L);
}

/* operator evaluations made since the last call (every level, isolated or not) */
extern long long or_n_evals;
int64_t ora_take_eval_count(void) {
  int64_t n = (int64_t)or_n_evals;
  or_n_evals = 0;
  return n;
}
