/* Oracle (test infrastructure): multigrid declarations. */
#ifndef PMG_ORACLE_MG_H
#define PMG_ORACLE_MG_H

#include "oracle.h"

typedef struct {
  int32_t beta_pre, beta_post, beta_coarse;
  int32_t tuning;      /* 0 fixed sweeps, 1 residual-based tuning */
  double eta;          /* pre-smoothing tuning factor (1.1) */
  int32_t max_repeats; /* cap on tuning repetitions */
  int32_t fmg;
  double fmg_threshold;
  int32_t isolated;    /* truncation error: 0 non-isolated, 1 isolated */
} or_mg_params;

typedef struct {
  int nlev;
  int dir;  /* -1 isotropic, else the coarsened direction */
  int* caps; /* per level index (0 = coarsest) */
  or_level** L;
  double **Q, **Q0, **S, **r, **Sphys;
  /* optional copy of the pointwise truncation error [5][nn] of the level whose cap is tau_nodal_cap */
  double* tau_nodal;
  int tau_nodal_cap;
  /* optional records for the tests: smoothing blocks of the last visit of each level (pre at [2 l], post at
     [2 l + 1]; with fixed sweeps each phase counts one block), and V-cycles the FMG start ran on each level */
  int* reps;
  int* fmg_cycles;
} or_mg;

void or_residual(const or_problem* P, const or_level* L, int isolated, const double* Q, const double* S, double* R);
double or_norm_inf(const double* R, int64_t n);
void or_smooth(const or_problem* P, const or_level* L, double* Q, const double* S, int sweeps);
void or_restrict(const or_problem* P, const or_level* Lf, const or_level* Lc, const double* Uf, double* Uc);
void or_prolong(const or_problem* P, const or_level* Lc, const or_level* Lf, const double* Uc, double* Uf);
/* per direction: interpolation where the order rises, L2 projection where it falls */
void or_remap(const or_problem* P, const or_level* La, const or_level* Lb, const double* Ua, double* Ub);
or_mg* or_mg_create(const or_problem* P, const int32_t* ord, int nlev, const int* caps, int aniso_dir);
void or_mg_destroy(or_mg* mg);
double or_mg_vcycles(const or_problem* P, or_mg* mg, double* Q, const double* S, int ncycles, const or_mg_params* prm,
                     double* tau_map, int nt);
int or_mg_solve(const or_problem* P, or_mg* mg, double* Q, const double* S, double tol, int max_cycles,
                const or_mg_params* prm, double* res_out, double* history);

#endif
