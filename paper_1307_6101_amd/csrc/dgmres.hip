// Device-side Krylov scalars of the batched GMRES (declarations and the
// algorithm in dgmres.h).  Every kernel runs one wavefront; lane r serves
// system r of the batch.
#include "dgmres.h"

namespace ddamg {

namespace {

__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double cabs1(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

__global__ void k_gm_reset(long long* iters, int nb) {
  const int r = threadIdx.x;
  if (r < nb) iters[r] = 0;
}

// lane 0 stores whether any lane's predicate holds; called once by every
// lane of the wavefront, outside divergent code
__device__ inline void set_flag(int* flag, bool pred) {
  const unsigned long long any = __ballot(pred);
  if (threadIdx.x == 0) *flag = any != 0ull;
}

// the per-system bodies return the lane's part of the flag
__device__ inline bool gm_begin_body(DevGmres& d, int r, int m, double tol, int first) {
  GmSys& S = d.sys[r];
  const double beta = sqrt(fmax(d.res[(size_t)r * (KMAX + 1)].x, 0.0));
  if (first == 1) {
    S.target = tol * beta;
    S.active = beta > 0.0;
  } else if (first == 2) {
    S.active = S.active && isfinite(beta) && beta > S.target;
  } else {
    S.active = S.active && !S.conv && beta > 0.0;
  }
  S.conv = 0;
  S.live = S.active;
  S.jend = 0;
  // step j writes rows 0..j+1 of Hessenberg column j and g[j+1], so nothing
  // of an earlier cycle is read again
  S.g[0] = make_double2(S.active ? beta : 0.0, 0.0);
  d.scale[r] = S.active ? 1.0 / beta : 0.0;
  return S.active;
}

__global__ void k_gm_begin(DevGmres d, int m, int nb, double tol, int first) {
  const int r = threadIdx.x;
  const bool live = r < nb ? gm_begin_body(d, r, m, tol, first) : false;
  set_flag(d.flag, live);
}

__global__ void k_gm_cgs1(DevGmres d, int j, int nb) {
  const int r = threadIdx.x;
  if (r >= nb) return;
  GmSys& S = d.sys[r];
  const double2* h = d.res + (size_t)r * (KMAX + 1);
  const double ww = h[j + 1].x;
  double proj = 0;
  for (int i = 0; i <= j; ++i) {
    S.h1[i] = h[i];
    proj += cabs2(h[i]);
  }
  S.ww1 = ww;
  const int again = S.live && !(ww - proj > 0.5 * ww);
  S.again = again;
  for (int i = 0; i <= j; ++i) d.coef[(size_t)r * KMAX + i] = again ? cneg(h[i]) : make_double2(0.0, 0.0);
}

__device__ inline bool gm_step_body(DevGmres& d, int r, int j, int m) {
  GmSys& S = d.sys[r];
  double2* cf = d.coef + (size_t)r * KMAX;
  if (!S.live) {
    for (int i = 0; i <= j; ++i) cf[i] = make_double2(0.0, 0.0);
    d.scale[r] = 0.0;
    return false;
  }
  const double2* h2 = d.res + (size_t)r * (KMAX + 1);
  double proj = 0;
  for (int i = 0; i <= j; ++i) proj += cabs2(S.h1[i]);
  double hn = sqrt(fmax(S.ww1 - proj, 0.0));
  // Hessenberg column j (first pass, plus the second where it ran)
  double2* H = S.H;
  for (int i = 0; i <= j; ++i) {
    double2 hi = S.h1[i];
    if (S.again) hi = cadd(hi, h2[i]);
    H[(size_t)i * m + j] = hi;
    cf[i] = cneg(S.again ? h2[i] : S.h1[i]);
  }
  if (S.again) {
    double nn = h2[j + 1].x;
    for (int i = 0; i <= j; ++i) nn -= cabs2(h2[i]);
    hn = sqrt(fmax(nn, 0.0));
  }
  // Givens rotations of the earlier columns, then the new one
  H[(size_t)(j + 1) * m + j] = make_double2(hn, 0.0);
  for (int i = 0; i < j; ++i) {
    const double2 a = H[(size_t)i * m + j], bq = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cadd(cmul(S.cs[i], a), cmul(S.sn[i], bq));
    H[(size_t)(i + 1) * m + j] = csub(cmul(S.cs[i], bq), cmul(cconj(S.sn[i]), a));
  }
  const double2 a = H[(size_t)j * m + j];
  const double aa = cabs1(a);
  const double rho = sqrt(cabs2(a) + hn * hn);
  if (rho == 0.0) {
    S.cs[j] = make_double2(1.0, 0.0);
    S.sn[j] = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    S.cs[j] = make_double2(0.0, 0.0);
    S.sn[j] = make_double2(1.0, 0.0);
  } else {
    S.cs[j] = make_double2(aa / rho, 0.0);
    S.sn[j] = make_double2(a.x / aa * hn / rho, a.y / aa * hn / rho);
  }
  H[(size_t)j * m + j] = cadd(cmul(S.cs[j], a), cscale(S.sn[j], hn));
  H[(size_t)(j + 1) * m + j] = make_double2(0.0, 0.0);
  const double2 gj = S.g[j];
  S.g[j + 1] = cneg(cmul(cconj(S.sn[j]), gj));
  S.g[j] = cmul(S.cs[j], gj);
  const double est = cabs1(S.g[j + 1]);
  ++d.iters[r];
  S.jend = j + 1;
  if (!isfinite(est)) {
    // nothing more for this system; its iterate stays what it was
    S.live = 0;
    S.active = 0;
    S.jend = 0;
  } else if (est <= S.target || hn == 0.0) {
    S.live = 0;
    S.conv = 1;
  }
  d.scale[r] = S.live ? 1.0 / hn : 0.0;
  return S.live;
}

__global__ void k_gm_step(DevGmres d, int j, int m, int nb) {
  const int r = threadIdx.x;
  const bool live = r < nb ? gm_step_body(d, r, j, m) : false;
  set_flag(d.flag, live);
}

__device__ inline bool gm_solve_body(DevGmres& d, int r, int m) {
  GmSys& S = d.sys[r];
  const bool again = S.active && !S.conv;
  double2* y = d.coef + (size_t)r * KMAX;
  for (int i = 0; i < m; ++i) y[i] = make_double2(0.0, 0.0);
  if (!S.active || S.jend == 0) return again;
  const double2* H = S.H;
  for (int i = S.jend - 1; i >= 0; --i) {
    double2 acc = S.g[i];
    for (int k = i + 1; k < S.jend; ++k) acc = csub(acc, cmul(H[(size_t)i * m + k], y[k]));
    y[i] = cdiv(acc, H[(size_t)i * m + i]);
  }
  return again;
}

__global__ void k_gm_solve(DevGmres d, int m, int nb) {
  const int r = threadIdx.x;
  const bool again = r < nb ? gm_solve_body(d, r, m) : false;
  set_flag(d.flag, again);
}

}  // namespace

void gm_reset(const DevGmres& d, int nb, hipStream_t s) {
  k_gm_reset<<<1, 64, 0, s>>>(d.iters, nb);
  DD_LAUNCH_CHECK();
}

void gm_begin(const DevGmres& d, int m, int nb, double tol, int first, hipStream_t s) {
  DD_REQUIRE(m >= 1 && m <= KMAX && nb >= 1 && nb <= NBMAX && NBMAX <= 64, "bad device GMRES shape");
  k_gm_begin<<<1, 64, 0, s>>>(d, m, nb, tol, first);
  DD_LAUNCH_CHECK();
}

void gm_cgs1(const DevGmres& d, int j, int nb, hipStream_t s) {
  k_gm_cgs1<<<1, 64, 0, s>>>(d, j, nb);
  DD_LAUNCH_CHECK();
}

void gm_step(const DevGmres& d, int j, int m, int nb, hipStream_t s) {
  DD_REQUIRE(j >= 0 && j < m && m <= KMAX, "bad device GMRES step");
  k_gm_step<<<1, 64, 0, s>>>(d, j, m, nb);
  DD_LAUNCH_CHECK();
}

void gm_solve(const DevGmres& d, int m, int nb, hipStream_t s) {
  k_gm_solve<<<1, 64, 0, s>>>(d, m, nb);
  DD_LAUNCH_CHECK();
}

}  // namespace ddamg
