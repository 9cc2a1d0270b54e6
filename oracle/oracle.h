/*
 * Plain FP64 CPU oracle of the DGSEM / FAS p-multigrid hot path (test infrastructure only).
 *
 * This is the slow, obviously-correct reference the HIP library is checked against.  It shares no code,
 * header, table or helper with the HIP library.  Only tests, the smoke check and the benchmark's CPU
 * baseline may call it.  Every routine follows the paper's definitions step by step, in its order and
 * notation, with scalar loops and a fixed summation order (built with -ffp-contract=off).
 */
#ifndef PMG_ORACLE_H
#define PMG_ORACLE_H

#include <stdint.h>

#define OR_MAXN 16 /* nodes per direction (order <= 15) */

typedef struct {
  double mach, reynolds, prandtl, gamma, suth, cfl_adv, cfl_visc;
  int32_t family;    /* 0 Legendre-Gauss, 1 Legendre-Gauss-Lobatto */
  int32_t viscosity; /* 0 Sutherland, 1 constant */
} or_phys;

/* 1-D nodal basis of one order */
typedef struct {
  int n; /* nodes = order + 1 */
  double x[OR_MAXN], w[OR_MAXN];
  double D[OR_MAXN][OR_MAXN]; /* D[i][j] = l_j'(x_i) */
  double lm[OR_MAXN], lp[OR_MAXN]; /* l_j(-1), l_j(+1) */
} or_basis1d;

typedef struct or_problem_s or_problem;
typedef struct or_level_s or_level;

struct or_problem_s {
  int64_t K;
  int M[3];
  double* gnodes;
  int64_t* nbr;
  int32_t* nbrf;
  int32_t* orient;
  int32_t* bc;
  or_phys ph;
  or_basis1d basis[OR_MAXN]; /* by order 0..15 (order 0 unused for LGL) */
};

struct or_level_s {
  int64_t K;
  int32_t* ord;  /* K*3 */
  int64_t* off;  /* K+1 node offsets */
  int64_t nn;
  int64_t* fo;   /* K*6 face-node offsets */
  int64_t nf;
  double* X;     /* [3][nn] */
  double* Ja;    /* [3 (contravariant i)][3 (component)][nn] */
  double* J;     /* [nn] */
  double* Nout;  /* [3][nf]: outward face normal scaled by the surface Jacobian, own side */
};

/* basis.c */
void or_make_basis(int order, int family, or_basis1d* b);
double or_lagrange(int n, const double* xn, int j, double x);
double or_lagrange_deriv(int n, const double* xn, int j, double x);
void or_projection_matrix(const or_basis1d* coarse, const or_basis1d* fine, double* R /*nc x nf*/);
void or_interp_matrix(const or_basis1d* from, const double* pts, int npts, double* I /*npts x nfrom*/);
int or_solve_dense(int n, double* A, double* b, int nrhs);

/* physics.c */
void or_prim(const or_phys* ph, const double q[5], double* rho, double v[3], double* p, double* T);
double or_mu(const or_phys* ph, double T);
void or_flux_adv(const or_phys* ph, const double q[5], double F[3][5]);
void or_flux_visc(const or_phys* ph, const double q[5], const double gW[4][3], double F[3][5]);
void or_flux_visc_wall(const or_phys* ph, const double q[5], const double gW[4][3], double F[3][5]);
void or_roe(const or_phys* ph, const double qL[5], const double qR[5], const double n[3], double Fn[5]);
void or_freestream(const or_phys* ph, double q[5]);

/* geometry.c */
or_level* or_level_create(const or_problem* P, const int32_t* ord);
void or_level_destroy(or_level* L);

/* residual.c */
void or_gradient(const or_problem* P, const or_level* L, int isolated, const double* Q, double* gW);
void or_wall_force(const or_problem* P, const or_level* L, const double* Q, double out[12]);
void or_operator(const or_problem* P, const or_level* L, int isolated, const double* Q, double* A);
double or_timestep(const or_problem* P, const or_level* L, const double* Q);

#endif
