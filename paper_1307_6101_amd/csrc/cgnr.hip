// CGNR: conjugate gradients on the normal equations D^H D z = D^H b with the
// residual r = b - D z, entirely in FP64 -- the Krylov method the paper
// compares DD-alpha-AMG against and whose iteration count it uses as the
// conditioning indicator of a configuration (Sec. 4, Tab. 2 and Tab. 5).
// D^H is applied as Gamma5 D Gamma5 (gamma5-hermiticity of the
// Wilson-clover operator).  A batch of systems advances together with its
// own scalars and stopping test per system.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "cgnr.h"

namespace ddamg {

namespace {

void norms2(Reducer& red, const double2* v, long long n, int nb, std::vector<double>& out, hipStream_t s) {
  red.bdots<double>(nullptr, v, 0, 0, const_cast<double2*>(v), n, nb, s);
  std::vector<std::complex<double>> r(nb);
  red.bfetch(1, nb, r.data(), s);
  out.resize(nb);
  for (int k = 0; k < nb; ++k) out[k] = r[k].real();
}

}  // namespace

void cgnr(Context& ctx, const double2* b, double2* x, int nb, double tol, int max_iter, ddamg_solve_stats* st,
          hipStream_t s) {
  DD_REQUIRE(nb >= 1 && nb <= NBMAX, "batch out of range");
  const FineGeom& g = ctx.g;
  const long long n = (long long)g.nblk * 192, vs = n * nb;
  const FineOpView<double> D = ctx.view<double>();
  Reducer red;
  DevArray<double2> r, p, w, z, t;
  r.alloc(vs);
  p.alloc(vs);
  w.alloc(vs);
  z.alloc(vs);
  t.alloc(vs);
  // z = D^H v = Gamma5 D Gamma5 v
  auto apply_dh = [&](const double2* v, double2* out) {
    gamma5(g, v, t.p, nb, s);
    dslash<double>(D, t.p, out, s, nb);
    gamma5(g, out, out, nb, s);
  };
  auto bupdate = [&](const std::vector<double>& c, const double2* Z, double2* y) {
    std::vector<std::complex<double>> cc((size_t)nb * KMAX, 0.0);
    for (int k = 0; k < nb; ++k) cc[(size_t)k * KMAX] = c[k];
    const BArg a = red.upload(cc, std::vector<double>(), nb, s);
    blincomb<double, double>(a, 1, Z, vs, y, n, nb, nullptr, s);
  };
  std::vector<double> bn, rho, gam, gam1, del;
  norms2(red, b, n, nb, bn, s);
  // r = b - D x, z = D^H r, p = z
  dslash<double>(D, x, r.p, s, nb);
  vbmy<double>(b, r.p, vs, s);
  apply_dh(r.p, z.p);
  vcopy<double, double>(z.p, p.p, vs, s);
  norms2(red, r.p, n, nb, rho, s);
  norms2(red, z.p, n, nb, gam, s);
  std::vector<char> live(nb);
  std::vector<int> status(nb, DDAMG_ENOCONV);
  for (int k = 0; k < nb; ++k) {
    st[k] = ddamg_solve_stats{};
    if (!std::isfinite(bn[k]) || !std::isfinite(rho[k])) status[k] = DDAMG_ENONFINITE;
    else if (rho[k] <= tol * tol * bn[k]) status[k] = DDAMG_OK;
    live[k] = status[k] == DDAMG_ENOCONV;
  }
  std::vector<double> alpha(nb), malpha(nb), beta(nb);
  for (int it = 0; it < max_iter; ++it) {
    bool any = false;
    for (int k = 0; k < nb; ++k) any = any || live[k];
    if (!any) break;
    dslash<double>(D, p.p, w.p, s, nb);  // w = D p
    norms2(red, w.p, n, nb, del, s);
    for (int k = 0; k < nb; ++k) {
      alpha[k] = live[k] && del[k] > 0 ? gam[k] / del[k] : 0.0;
      malpha[k] = -alpha[k];
    }
    bupdate(alpha, p.p, x);     // x += alpha p
    bupdate(malpha, w.p, r.p);  // r -= alpha w
    norms2(red, r.p, n, nb, rho, s);
    for (int k = 0; k < nb; ++k) {
      if (!live[k]) continue;
      ++st[k].outer_iters;
      if (!std::isfinite(rho[k])) {
        status[k] = DDAMG_ENONFINITE;
        live[k] = 0;
      } else if (rho[k] <= tol * tol * bn[k]) {
        status[k] = DDAMG_OK;
        live[k] = 0;
      }
    }
    apply_dh(r.p, z.p);  // z = D^H r
    norms2(red, z.p, n, nb, gam1, s);
    for (int k = 0; k < nb; ++k) {
      beta[k] = live[k] && gam[k] > 0 ? gam1[k] / gam[k] : 0.0;
      gam[k] = gam1[k];
    }
    // p = z + beta p
    {
      const BArg a = red.upload(std::vector<std::complex<double>>(), beta, nb, s);
      bscale<double>(a, p.p, p.p, n, nb, s);
    }
    std::vector<double> one(nb, 1.0);
    bupdate(one, z.p, p.p);
  }
  // the true residual of every system
  dslash<double>(D, x, r.p, s, nb);
  vbmy<double>(b, r.p, vs, s);
  norms2(red, r.p, n, nb, rho, s);
  for (int k = 0; k < nb; ++k) {
    const double rel = bn[k] > 0 ? std::sqrt(std::max(rho[k], 0.0) / bn[k]) : 0.0;
    st[k].true_relres = rel;
    if (status[k] == DDAMG_OK && !(rel <= tol)) status[k] = DDAMG_ENOCONV;
    st[k].status = status[k];
  }
}

}  // namespace ddamg
