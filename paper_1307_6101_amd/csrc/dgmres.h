// GMRES with its Krylov scalars on the device.  Each system of a batch has a
// record holding its Hessenberg matrix, Givens rotations, residual estimate
// and stopping state; small single-wavefront kernels (one lane per system)
// update the records from the inner products that the batched reduction
// writes to device memory, and write the coefficients and scales that the
// batched vector kernels read.  A restarted GMRES thereby becomes a fixed
// sequence of launches with no host round trip, which a HIP graph can
// capture.  The arithmetic is that of the host-driven GMRES: classical
// Gram-Schmidt with the Daniel-Gragg-Kaufman-Stewart second pass, Givens
// rotations, back substitution; a system that has met its tolerance keeps
// running through the remaining launches with zero coefficients and zero
// basis vectors, which changes nothing.
#pragma once

#include "blas.h"

namespace ddamg {

struct GmSys {
  double2 H[(KMAX + 1) * KMAX];   // row-major (m+1) x m
  double2 g[KMAX + 1];
  double2 cs[KMAX], sn[KMAX];
  double2 h1[KMAX + 1];           // first Gram-Schmidt pass of the current step
  double beta, target, ww1;
  int active, live, conv, again, jend, pad;
};

// device buffers of one batch (NBMAX systems)
struct DevGmres {
  GmSys* sys = nullptr;
  double2* res = nullptr;        // [NBMAX][KMAX+1] inner products
  double2* coef = nullptr;       // [NBMAX][KMAX]
  double* scale = nullptr;       // [NBMAX]
  long long* iters = nullptr;    // [NBMAX] iterations, accumulated
  int* flag = nullptr;           // device alias of a coherent host word: set by
                                 // gm_begin / gm_step / gm_solve (see below)
  BArg arg() const {
    BArg a;
    a.inl = 0;
    a.c = coef;
    a.sc = scale;
    return a;
  }
};

// iters[r] = 0
void gm_reset(const DevGmres& d, int nb, hipStream_t s);
// start of a restart cycle from the norms ||r_r||^2 in res[r][0]: first = 1
// (first cycle) sets the targets tol * ||b_r||; first = 0 continues the
// systems whose Arnoldi estimate has not met the target; first = 2 decides
// by the recomputed residual instead: a system continues while that
// residual is finite and above its target.  scale[r] = 1 / ||r_r|| (0 for
// systems that are done); flag = some system is active
void gm_begin(const DevGmres& d, int m, int nb, double tol, int first, hipStream_t s);
// after the first Gram-Schmidt pass of step j (res = <V_i, w>, <w, w>):
// decide the second pass, coef = its coefficients (zero where none)
void gm_cgs1(const DevGmres& d, int j, int nb, hipStream_t s);
// after the second pass: Hessenberg column, Givens rotation, stopping test;
// coef / scale = the update w += V c and V_{j+1} = w / h_{j+1,j}; flag =
// some system is still live
void gm_step(const DevGmres& d, int j, int m, int nb, hipStream_t s);
// end of a cycle: coef = y = R^-1 g of every active system (zero beyond its
// last step); flag = some system needs another cycle
void gm_solve(const DevGmres& d, int m, int nb, hipStream_t s);

}  // namespace ddamg
