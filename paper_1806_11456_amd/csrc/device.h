// Device-side building blocks: basis tables in constant memory, level descriptors, and the pointwise
// physics of the compressible Navier-Stokes equations (paper, Appendix A) with the Roe flux (Sec. 2).
// Operator kernels are templated on the working precision T (double on the fine level and for the
// truncation error; float on the coarse levels of the mixed-precision cycle).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PMG_MAXN 8        // nodes per direction (order <= 7)
#define PMG_BLOCK 256     // threads per element / face tile
#define PMG_TILE_MAX 512  // nodes per element tile (one element of 8x8x8)
#define PMG_NPT 2         // nodes per thread of a PMG_BLOCK block over a PMG_TILE_MAX tile (the library launches
                          // PMG_TILE_MAX-thread blocks for such tiles instead)
#define PMG_FACE_TILE 256 // mortar nodes per face tile
#define PMG_MAX_TILE_ELEMS 64

// 1-D tables of one node family, indexed by the number of nodes n = order + 1 (1..8).
struct BasisTables {
  double x[PMG_MAXN + 1][PMG_MAXN];
  double w[PMG_MAXN + 1][PMG_MAXN];
  double D[PMG_MAXN + 1][PMG_MAXN][PMG_MAXN];     // D[n][i][j] = l_j'(x_i)
  double Dhat[PMG_MAXN + 1][PMG_MAXN][PMG_MAXN];  // Dhat[n][i][m] = -D[m][i] w_m / w_i (weak form)
  double lm[PMG_MAXN + 1][PMG_MAXN], lp[PMG_MAXN + 1][PMG_MAXN];  // l_i(-1), l_i(+1)
  double Lm[PMG_MAXN + 1][PMG_MAXN], Lp[PMG_MAXN + 1][PMG_MAXN];  // surface lift l_i(-+1) / w_i
};

__constant__ BasisTables c_tab[2];  // [family]

// Transfer matrices T(from, to) of one family, row-major [to][from]: exact interpolation when to > from,
// L2 projection with the 'from' quadrature when to < from, identity when equal.  Global memory.
__device__ __forceinline__ const double* tmat(const double* T, int from, int to) {
  return T + ((from * (PMG_MAXN + 1) + to) * PMG_MAXN * PMG_MAXN);
}
#define TMAT_STRIDE ((PMG_MAXN + 1) * (PMG_MAXN + 1) * PMG_MAXN * PMG_MAXN)

struct Phys {
  double gamma, gm1, gM2, Re, invRe, kcoef, suth, suth1, cfl_adv, cfl_visc;
  double pinf, rhoE_inf;
  int visc_const, family;
};

// Interface between two element faces (master = lower element id; the lower face on self-periodic faces).
struct FaceRec {
  int eM, fM, eS, fS;  // eS = -1 on boundary faces
  int o, bc;
  int foM, foS;        // first face node of each side in the face arrays
  int nMs, nMt;        // master face nodes along its (s, t) axes
  int nS1, nS2;        // slave face nodes along its own axes
  int ms, mt;          // mortar nodes along the master (s, t) axes
  int mbase;           // first mortar node
  int flags;           // bit0 master side equals the mortar, bit1 slave side equals the mortar
};

// One discretisation level as the kernels see it; geometry arrays in the working precision T.
template <class T>
struct LevelDevT {
  int K, nn, nf, nm, fam;
  const Phys* __restrict__ ptab;      // physics of each problem of the batch
  const int* __restrict__ eprob;      // problem of each element
  const int* __restrict__ node_elem;  // element of each node
  const double* __restrict__ dt;      // per-problem explicit step (read by the RK epilogue)
  const int* __restrict__ active;     // per-problem: 0 = frozen (its RK updates use a zero step)
  const int* __restrict__ skip;       // nullable; tiles of problems p with skip[p] == 0 return at once
  const int* __restrict__ ord;        // K*3 orders
  const int* __restrict__ off;        // K+1 node offsets
  const int* __restrict__ fo;         // K*6 face-node offsets
  const T* __restrict__ Ja;           // [9][nn]  (J a^d)_c at [(d*3 + c)]
  const T* __restrict__ invJ;         // [nn]
  const T* __restrict__ J;            // [nn]
  const T* __restrict__ Nout;         // [3][nf] outward normal x surface Jacobian, own side
  // per element tile, two int4: {first elist entry, elements, packed n1|n2<<8|n3<<16, nodes} and
  // {problem, first node, first face node, 0} (the bases -1 unless the tile's elements are consecutive)
  const int4* __restrict__ tiles;
  const int* __restrict__ elist;
  const int* __restrict__ eoff;       // per elist entry: first node of the element (off[elist[k]])
  const int* __restrict__ efo;        // per elist entry: first face node of the element (fo[6 elist[k]])
  const FaceRec* __restrict__ faces;
  const int* __restrict__ mface;      // mortar node -> face
  const int* __restrict__ ftile;      // face tile boundaries in mortar nodes
  const int* __restrict__ ftprob;     // problem of each face tile
  const T* __restrict__ mgeo;         // [4][nm] unit normal (master outward) and surface Jacobian
  // [nf] where the BR1 interface state of each face node comes from: >= 0 the face node facing it across a
  // conforming interface (same nodes on both sides); PMG_WLINK_MORTAR a p-nonconforming face (the mortar
  // pass writes it); <= -2 a boundary face node, -2 - (8 * mortar node + boundary code)
  const int* __restrict__ wlink;
  // [nf] on conforming interior faces: the mortar node (interface point) of each face node, -1 elsewhere
  const int* __restrict__ mlink;
  // [nm] on conforming and boundary faces: {master face node, slave face node or -1 - boundary code} of each
  // mortar node (the mortar nodes are the face nodes of both sides there)
  const int2* __restrict__ cmap;
  const double* __restrict__ T_;      // transfer tables of this family
};
#define PMG_WLINK_MORTAR (-1)
using LevelDev = LevelDevT<double>;

// Dynamic LDS of a templated kernel, viewed in its working type.
#define PMG_DYN_LDS(T, name)                             \
  extern __shared__ __align__(16) unsigned char name##_raw[]; \
  T* name = reinterpret_cast<T*>(name##_raw)

// ------------------------------------------------------------------------------------------------
// Pointwise physics
// ------------------------------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void prim(const Phys& P, const T q[5], T& rho, T v[3], T& p, T& Tt) {
  rho = q[0];
  T ir = T(1) / q[0];
  v[0] = q[1] * ir;
  v[1] = q[2] * ir;
  v[2] = q[3] * ir;
  p = T(P.gm1) * (q[4] - T(0.5) * (q[1] * v[0] + q[2] * v[1] + q[3] * v[2]));
  Tt = T(P.gM2) * p * ir;
}

template <class T>
__device__ __forceinline__ T mu_of(const Phys& P, T Tt) {
  if (P.visc_const) return T(1);
  return Tt * sqrt(Tt) * T(P.suth1) / (Tt + T(P.suth));
}

template <class T>
__device__ __forceinline__ void prim_w(const Phys& P, const T q[5], T W[4]) {
  T rho, v[3], p, Tt;
  prim(P, q, rho, v, p, Tt);
  W[0] = v[0]; W[1] = v[1]; W[2] = v[2]; W[3] = Tt;
}

// F^a . N for an arbitrary vector N (5 components)
template <class T>
__device__ __forceinline__ void flux_adv_n(const Phys& P, const T q[5], const T N[3], T out[5]) {
  T rho, v[3], p, Tt;
  prim(P, q, rho, v, p, Tt);
  T vn = v[0] * N[0] + v[1] * N[1] + v[2] * N[2];
  out[0] = q[0] * vn;
  out[1] = q[1] * vn + p * N[0];
  out[2] = q[2] * vn + p * N[1];
  out[3] = q[3] * vn + p * N[2];
  out[4] = vn * (q[4] + p);
}

// Viscous flux tensor F^v[c][v] (row v = 0 is zero and not stored: F[c][0..3] = momentum, energy)
// g[k*3 + c] = dW_k / dx_c, W = (u, v, w, T).  wall: no-slip adiabatic wall flux (no work, no heat flux).
template <class T>
__device__ __forceinline__ void flux_visc(const Phys& P, const T q[5], const T g[12], bool wall, T F[3][4]) {
  T rho, v[3], p, Tt;
  prim(P, q, rho, v, p, Tt);
  T mu = mu_of(P, Tt);
  T div = g[0] + g[4] + g[8];
  T lam = T(-2.0 / 3.0) * mu * div;
  T tau[3][3];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) tau[i][j] = mu * (g[i * 3 + j] + g[j * 3 + i]);
  tau[0][0] += lam; tau[1][1] += lam; tau[2][2] += lam;
  T kap = mu * T(P.kcoef);
  const T invRe = T(P.invRe);
#pragma unroll
  for (int c = 0; c < 3; c++) {
    F[c][0] = invRe * tau[c][0];
    F[c][1] = invRe * tau[c][1];
    F[c][2] = invRe * tau[c][2];
    F[c][3] = wall ? T(0) : invRe * (v[0] * tau[c][0] + v[1] * tau[c][1] + v[2] * tau[c][2] + kap * g[9 + c]);
  }
}

// Roe flux along the unit normal n (from L to R), standard Roe averages, no entropy fix.
template <class T>
__device__ __forceinline__ void roe_flux(const Phys& P, const T qL[5], const T qR[5], const T n[3], T Fn[5]) {
  T rL, vL[3], pL, TL, rR, vR[3], pR, TR;
  prim(P, qL, rL, vL, pL, TL);
  prim(P, qR, rR, vR, pR, TR);
  T HL = (qL[4] + pL) / rL, HR = (qR[4] + pR) / rR;
  T sL = sqrt(rL), sR = sqrt(rR);
  T isum = T(1) / (sL + sR);
  T rh = sL * sR;
  T vh[3] = {(sL * vL[0] + sR * vR[0]) * isum, (sL * vL[1] + sR * vR[1]) * isum, (sL * vL[2] + sR * vR[2]) * isum};
  T Hh = (sL * HL + sR * HR) * isum;
  T v2 = vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2];
  T c2 = T(P.gm1) * (Hh - T(0.5) * v2);
  T ch = sqrt(c2);
  T un = vh[0] * n[0] + vh[1] * n[1] + vh[2] * n[2];
  T dr = rR - rL, dp = pR - pL;
  T dv[3] = {vR[0] - vL[0], vR[1] - vL[1], vR[2] - vL[2]};
  T dun = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
  T i2c2 = T(1) / (T(2) * c2);
  T a1 = (dp - rh * ch * dun) * i2c2;
  T a5 = (dp + rh * ch * dun) * i2c2;
  T a2 = dr - dp / c2;
  T l1 = fabs(un - ch), l5 = fabs(un + ch), l2 = fabs(un);
  T d[5];
  d[0] = l1 * a1 + l5 * a5 + l2 * a2;
#pragma unroll
  for (int c = 0; c < 3; c++)
    d[1 + c] = l1 * a1 * (vh[c] - ch * n[c]) + l5 * a5 * (vh[c] + ch * n[c]) + l2 * a2 * vh[c] +
               l2 * rh * (dv[c] - dun * n[c]);
  d[4] = l1 * a1 * (Hh - un * ch) + l5 * a5 * (Hh + un * ch) + l2 * a2 * T(0.5) * v2 +
         l2 * rh * (vh[0] * dv[0] + vh[1] * dv[1] + vh[2] * dv[2] - un * dun);
  T fl[5], fr[5];
  flux_adv_n(P, qL, n, fl);
  flux_adv_n(P, qR, n, fr);
#pragma unroll
  for (int k = 0; k < 5; k++) Fn[k] = T(0.5) * (fl[k] + fr[k]) - T(0.5) * d[k];
}

template <class T>
__device__ __forceinline__ void freestream(const Phys& P, T q[5]) {
  q[0] = T(1); q[1] = T(1); q[2] = T(0); q[3] = T(0); q[4] = T(P.rhoE_inf);
}

// ghost state of a boundary node (unit outward normal n): 1 no-slip adiabatic wall, 2 far field (uniform
// inflow), 3 free slip, 4 subsonic outflow with the far-field pressure
template <class T>
__device__ __forceinline__ void ghost_state(const Phys& P, int bc, const T q[5], const T n[3], T g[5]) {
  if (bc == 1) {
    g[0] = q[0]; g[1] = -q[1]; g[2] = -q[2]; g[3] = -q[3]; g[4] = q[4];
  } else if (bc == 3) {
    T mn = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    g[0] = q[0]; g[1] = q[1] - T(2) * mn * n[0]; g[2] = q[2] - T(2) * mn * n[1]; g[3] = q[3] - T(2) * mn * n[2];
    g[4] = q[4];
  } else if (bc == 4) {
    // subsonic outflow: the interior density and velocity with the far-field pressure
    g[0] = q[0]; g[1] = q[1]; g[2] = q[2]; g[3] = q[3];
    g[4] = T(P.pinf) / T(P.gm1) + T(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
  } else {
    freestream(P, g);
  }
}

// Numerical flux x surface Jacobian at one interface point with master outward unit normal n: the Roe flux
// minus the BR1 viscous flux {{F^v}} . n.  bc == 0: interior, the slave state qs and gradient gs are given;
// bc > 0: a boundary, the second state is the ghost state of qm and the viscous flux is the interior one
// (the adiabatic no-slip wall's without work and heat flux, none on free slip).
template <class T>
__device__ __forceinline__ void interface_flux(const Phys& P, int bc, const T qm[5], const T gm[12], const T qs_in[5],
                                               const T gs[12], const T n[3], T Js, T out[5]) {
  T qs[5], fv[4], Fm[3][4], Fn[5];
  if (bc == 0) {
    T Fs[3][4];
#pragma unroll
    for (int v = 0; v < 5; v++) qs[v] = qs_in[v];
    flux_visc(P, qm, gm, false, Fm);
    flux_visc(P, qs, gs, false, Fs);
#pragma unroll
    for (int v = 0; v < 4; v++)
      fv[v] = T(0.5) * (Fm[0][v] + Fs[0][v]) * n[0] + T(0.5) * (Fm[1][v] + Fs[1][v]) * n[1] +
              T(0.5) * (Fm[2][v] + Fs[2][v]) * n[2];
  } else {
    ghost_state(P, bc, qm, n, qs);
    if (bc == 3) {
#pragma unroll
      for (int v = 0; v < 4; v++) fv[v] = T(0);
    } else {
      flux_visc(P, qm, gm, bc == 1, Fm);
#pragma unroll
      for (int v = 0; v < 4; v++) fv[v] = Fm[0][v] * n[0] + Fm[1][v] * n[1] + Fm[2][v] * n[2];
    }
  }
  roe_flux(P, qm, qs, n, Fn);
  out[0] = Fn[0] * Js;
#pragma unroll
  for (int v = 0; v < 4; v++) out[v + 1] = (Fn[v + 1] - fv[v]) * Js;
}

// The same with the viscous part given: fv = {{F^v}} . n (interior) or the boundary's F^v . n, already formed
// from each side's viscous flux dotted with the master unit normal; bc > 0: the second state is the ghost.
template <class T>
__device__ __forceinline__ void interface_flux_fv(const Phys& P, int bc, const T qm[5], const T qs_in[5],
                                                  const T n[3], T Js, const T fv[4], T out[5]) {
  T qs[5], Fn[5];
  if (bc == 0) {
#pragma unroll
    for (int v = 0; v < 5; v++) qs[v] = qs_in[v];
  } else {
    ghost_state(P, bc, qm, n, qs);
  }
  roe_flux(P, qm, qs, n, Fn);
  out[0] = Fn[0] * Js;
#pragma unroll
  for (int v = 0; v < 4; v++) out[v + 1] = (Fn[v + 1] - fv[v]) * Js;
}

__device__ __forceinline__ void unpack3(int p, int& n1, int& n2, int& n3) {
  n1 = p & 255; n2 = (p >> 8) & 255; n3 = p >> 16;
}
