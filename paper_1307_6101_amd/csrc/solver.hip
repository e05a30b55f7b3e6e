// Host orchestration: cycles, FGMRES, odd-even coarsest solve, setup.
//
// Readings of the paper used here (each is also the oracle's):
//  * Alg. 3 starts from the random test vectors on the finest level (its
//    "l = 0" test means the first level) and keeps the smoothed iterate
//    unnormalised as the level's test vector.
//  * Alg. 4 runs the level-l cycle with the level's own test vector as
//    right-hand side; the test vectors of coarser levels k > l become the
//    approximate level-k solutions computed last during that cycle.
//  * Setup driver: initial phase on the finest level, then the iterative
//    phase for i = 1..n_inv.
//  * The K-cycle's "maximal restarts 2" allows at most 2 restart cycles of
//    length 5.
//  * The coarsest tolerance eps is relative to the right-hand side of the
//    odd-even reduced (Schur) system, solved by GMRES from zero.
#include "solver.h"

#include <chrono>
#include <cmath>
#include <cstring>

namespace ddamg {

using cd = std::complex<double>;

template <> FineOpView<double> Context::view<double>() const {
  return FineOpView<double>{U64.p, A64.p, nbr.p, g.nblk};
}
template <> FineOpView<float> Context::view<float>() const {
  return FineOpView<float>{U32.p, A32.p, nbr.p, g.nblk};
}
template <> CoarseOpView<double> LevelStore::cview<double>() const {
  return CoarseOpView<double>{K64.p, c_nbr9.p, (int)V, d};
}
template <> CoarseOpView<float> LevelStore::cview<float>() const {
  return CoarseOpView<float>{K32.p, c_nbr9.p, (int)V, d};
}
template <> Work<double>& Hierarchy::work<double>(int l) { return w64[l]; }
template <> Work<float>& Hierarchy::work<float>(int l) { return w32[l]; }
template <> const C<double>* Hierarchy::P<double>(int l) const { return lv[l].P64.p; }
template <> const C<float>* Hierarchy::P<float>(int l) const { return lv[l].P32.p; }
template <> C<double>* Hierarchy::tv<double>(int l) { return lv[l].tv64.p; }
template <> C<float>* Hierarchy::tv<float>(int l) { return lv[l].tv32.p; }

template <typename T, typename F> void Hierarchy::fine_op(F&& f) const {
  if constexpr (std::is_same<T, float>::value)
    if (half) return f(ctx->view16());
  f(ctx->view<T>());
}
template <typename T, typename F> void Hierarchy::coarse_op(int l, F&& f) const {
  if constexpr (std::is_same<T, float>::value)
    if (half) return f(lv[l].cview16());
  f(lv[l].cview<T>());
}
template <typename T, typename F> void Hierarchy::interp(int l, F&& f) const {
  if constexpr (std::is_same<T, float>::value)
    if (half) return f(static_cast<const __half2*>(lv[l].P16.p));
  f(P<T>(l));
}

static inline double2 d2(cd z) { return make_double2(z.real(), z.imag()); }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
Context* create_context(const ddamg_lattice* lat, const double2* links, hipStream_t s) {
  DD_REQUIRE(lat != nullptr && links != nullptr, "null lattice or links");
  for (int mu = 0; mu < 4; ++mu)
    DD_REQUIRE(lat->dims[mu] >= 4 && lat->dims[mu] % 4 == 0,
               "every lattice extent must be a positive multiple of 4");
  DD_REQUIRE(std::isfinite(lat->m0) && std::isfinite(lat->csw), "non-finite m0 or csw");
  std::unique_ptr<Context> c(new Context);
  c->g = make_fine_geom(lat->dims);
  c->m0 = lat->m0;
  c->csw = lat->csw;
  const FineGeom& g = c->g;
  std::vector<int> nbr((size_t)g.nblk * 8), cblk(g.nblk);
  fine_tables(g, nbr.data(), cblk.data());
  c->nbr.upload(nbr, s);
  c->cblk.upload(cblk, s);
  c->U64.alloc((size_t)g.V * 36);
  c->U32.alloc((size_t)g.V * 36);
  c->A64.alloc((size_t)g.V * 36);
  c->A32.alloc((size_t)g.V * 36);
  links_to_native<double>(g, links, c->U64.p, s);
  links_to_native<float>(g, links, c->U32.p, s);
  clover_build(g, links, lat->m0, lat->csw, c->A64.p, s);
  vcopy<double, float>(c->A64.p, c->A32.p, (long long)g.V * 36, s);
  DD_CHECK_HIP(hipStreamSynchronize(s));
  return c.release();
}

void Context::make_half(hipStream_t s) {
  if (U16.p) return;
  U16.alloc((size_t)g.V * 36);
  A16.alloc((size_t)g.V * 36);
  to_half(U64.p, U16.p, (long long)g.V * 36, s);
  to_half(A64.p, A16.p, (long long)g.V * 36, s);
}

// ---------------------------------------------------------------------------
// level operations
// ---------------------------------------------------------------------------
template <typename T> void Hierarchy::apply(int l, const C<T>* in, C<T>* out) {
  if (l == 0) fine_op<T>([&](const auto& op) { dslash(op, in, out, s); });
  else coarse_op<T>(l, [&](const auto& op) { coarse_apply(op, in, out, s); });
}

template <typename T> SapScratch<T>& sap_scratch(LevelStore& L_);
template <> SapScratch<double>& sap_scratch<double>(LevelStore& L_) { return L_.ss64; }
template <> SapScratch<float>& sap_scratch<float>(LevelStore& L_) { return L_.ss32; }

template <typename T> void Hierarchy::sap(int l, const C<T>* b, C<T>* z, int nsweeps) {
  for (int it = 0; it < nsweeps; ++it)
    for (int col = 0; col < 2; ++col) {
      if (l == 0) {
        fine_op<T>([&](const auto& op) { sap_colour(op, ctx->cblk.p, col, p.mr_iters, b, z, s); });
      } else {
        LevelStore& L_ = lv[l];
        coarse_op<T>(l, [&](const auto& op) {
          coarse_sap_colour(op, L_.c_blk_sites.p, L_.c_site_blk.p, L_.cg.nblk, L_.cg.bs, col, p.mr_iters, b,
                            z, sap_scratch<T>(L_), s);
        });
      }
    }
}

template <typename T> void Hierarchy::restrict_to(int l, const C<T>* fine, C<T>* coarse) {
  const LevelStore& L_ = lv[l];
  interp<T>(l, [&](const auto* P_) {
    if (l == 0) restrict_fine<T>(ctx->g, L_.at, L_.ad(), L_.N, P_, fine, coarse, s);
    else restrict_coarse<T>(L_.at, L_.ad(), L_.d, L_.N, L_.V, P_, fine, coarse, s);
  });
}

template <typename T> void Hierarchy::prolong_add(int l, const C<T>* coarse, C<T>* fine) {
  const LevelStore& L_ = lv[l];
  interp<T>(l, [&](const auto* P_) {
    if (l == 0) prolong_fine<T>(ctx->g, L_.ad(), L_.N, P_, coarse, fine, s);
    else prolong_coarse<T>(L_.ad(), L_.d, L_.N, L_.V, P_, coarse, fine, s);
  });
}

double Hierarchy::norm(const double2* v, long long n) {
  red->dots<double>(v, 0, 0, v, n, true, s);
  cd r;
  red->fetch(1, &r, s);
  return std::sqrt(r.real());
}

// ---------------------------------------------------------------------------
// Flexible GMRES(m) on level l from x = 0, at most max_cycles restart
// cycles, stop when the Arnoldi residual estimate <= tol ||b||.  Arnoldi
// with classical Gram-Schmidt and one re-orthogonalisation pass (two fused
// inner-product launches per step); Givens rotations on the host.
// ---------------------------------------------------------------------------
// One Arnoldi orthogonalisation step against V_0..V_j (classical Gram-Schmidt,
// second pass only when the first removed more than half of ||w||^2, the
// criterion of Daniel, Gragg, Kaufman and Stewart).  Fills h[0..j] with the
// Hessenberg column, returns ||w_perp||, and leaves in `c` the coefficients
// that the caller applies as w += V c together with V_{j+1} = w / hn.
template <typename T>
static double gs_step(Reducer& red, const C<T>* V, long long n, int j, C<T>* w, std::vector<cd>& h,
                      std::vector<cd>& h2, Coefs& c, hipStream_t s) {
  red.dots<T>(V, n, j + 1, w, n, true, s);
  red.fetch(j + 2, h.data(), s);
  const double ww = h[j + 1].real();
  double proj = 0;
  for (int i = 0; i <= j; ++i) {
    proj += std::norm(h[i]);
    c.c[i] = d2(-h[i]);
  }
  if (ww - proj > 0.5 * ww) return std::sqrt(ww - proj);
  red.update_dots<T>(c, V, n, j + 1, w, n, s);
  red.fetch(j + 2, h2.data(), s);
  double nn = h2[j + 1].real();
  for (int i = 0; i <= j; ++i) {
    c.c[i] = d2(-h2[i]);
    nn -= std::norm(h2[i]);
    h[i] += h2[i];
  }
  return std::sqrt(std::max(nn, 0.0));
}

template <typename T, typename Op, typename Pre>
int Hierarchy::fgmres(int l, Op op, Pre pre, bool use_pre, const C<T>* b, C<T>* x, int m,
                      int max_cycles, double tol) {
  Work<T>& W = work<T>(l);
  const long long n = lv[l].n;
  DD_REQUIRE(m <= W.m, "Krylov basis too short");
  C<T>* V = W.V.p;
  C<T>* Z = use_pre ? W.Z.p : W.V.p;
  C<T>* w = W.w.p;
  vzero<T>(x, n, s);
  red->dots<T>(b, 0, 0, b, n, true, s);
  cd bb;
  red->fetch(1, &bb, s);
  const double bnorm = std::sqrt(bb.real());
  if (!(bnorm > 0)) return 0;
  const double target = tol * bnorm;
  vcopy<T, T>(b, V, n, s);
  vscale<T>(make_double2(1.0 / bnorm, 0), V, n, s);
  double beta = bnorm;
  int iters = 0;
  std::vector<cd> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), h(KMAX + 1), h2(KMAX + 1);
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    std::fill(H.begin(), H.end(), cd(0));
    std::fill(g.begin(), g.end(), cd(0));
    g[0] = beta;
    int jend = 0;
    bool conv = false;
    for (int j = 0; j < m; ++j) {
      C<T>* Vj = V + (size_t)j * n;
      C<T>* Zj = Z + (size_t)j * n;
      if (use_pre) pre(Vj, Zj);
      op(Zj, w);
      Coefs c;
      const double hn = gs_step<T>(*red, V, n, j, w, h, h2, c, s);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
      H[(size_t)(j + 1) * m + j] = hn;
      // apply previous rotations, then a new one that zeroes H[j+1][j]
      for (int i = 0; i < j; ++i) {
        cd a = H[(size_t)i * m + j], bq = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
        H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * bq;
      }
      {
        cd a = H[(size_t)j * m + j];
        const double bq = hn;
        const double rho = std::sqrt(std::norm(a) + bq * bq);
        if (rho == 0.0) { cs[j] = 1; sn[j] = 0; }
        else if (std::abs(a) == 0.0) { cs[j] = 0; sn[j] = 1; }
        else {
          cs[j] = std::abs(a) / rho;
          sn[j] = (a / std::abs(a)) * bq / rho;
        }
        H[(size_t)j * m + j] = cs[j] * a + sn[j] * bq;
        H[(size_t)(j + 1) * m + j] = 0;
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
      }
      ++iters;
      jend = j + 1;
      const double est = std::abs(g[j + 1]);
      if (!std::isfinite(est)) throw Error(DDAMG_ENONFINITE, "non-finite residual in GMRES");
      if (est <= target || hn == 0.0) { conv = true; break; }
      // w += V c and V_{j+1} = w / hn in one pass
      if (j + 1 < m) vlincomb_scale<T>(c, j + 1, V, n, w, n, 1.0 / hn, V + (size_t)(j + 1) * n, s);
    }
    // y = R^{-1} g, x += Z y
    std::vector<cd> y(jend);
    for (int i = jend - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)i * m + k] * y[k];
      y[i] = acc / H[(size_t)i * m + i];
    }
    Coefs c;
    for (int i = 0; i < jend; ++i) c.c[i] = d2(y[i]);
    vlincomb<T, T>(c, jend, Z, n, x, n, s);
    if (conv || cyc + 1 == max_cycles) break;
    // restart from the true residual
    op(x, w);
    vbmy<T>(b, w, n, s);
    red->dots<T>(w, 0, 0, w, n, true, s);
    cd rr;
    red->fetch(1, &rr, s);
    beta = std::sqrt(rr.real());
    if (!(beta > 0)) break;
    vlincomb_scale<T>(Coefs{}, 0, V, n, w, n, 1.0 / beta, V, s);
  }
  return iters;
}

// ---------------------------------------------------------------------------
// coarsest level: odd-even reduced system
// ---------------------------------------------------------------------------
template <typename T> const C<T>* einv(const LevelStore& L_);
template <> const C<double>* einv<double>(const LevelStore& L_) { return L_.Einv64.p; }
template <> const C<float>* einv<float>(const LevelStore& L_) { return L_.Einv32.p; }

template <typename T> void Hierarchy::schur(const C<T>* v, C<T>* out) {
  const int c = L - 1;
  const LevelStore& L_ = lv[c];
  Work<T>& W = work<T>(c);
  const int ne = (int)L_.cg.even.size(), no = (int)L_.cg.odd.size();
  // t3_e = D_eo v_o ; t4_e = D_ee^-1 t3_e ; out_o = D_oo v_o - D_oe t4_e
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_even.p, ne, T(0), nullptr, T(0), nullptr, T(1), v, W.t3.p, s);
    site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, W.t3.p, W.t4.p, s);
    vzero<T>(out, L_.n, s);
    coarse_site_apply(op, L_.c_odd.p, no, T(0), nullptr, T(1), v, T(-1), W.t4.p, out, s);
  });
}

template <typename T> void Hierarchy::coarsest_solve(const C<T>* b, C<T>* z) {
  const int c = L - 1;
  const LevelStore& L_ = lv[c];
  Work<T>& W = work<T>(c);
  const long long n = L_.n;
  if (!L_.cg.bipartite) {
    cs_iters += fgmres<T>(
        c, [&](const C<T>* a, C<T>* o) { apply<T>(c, a, o); }, [](const C<T>*, C<T>*) {}, false, b,
        z, p.coarse_restart, p.coarse_max_restarts, p.coarse_eps);
    return;
  }
  const int ne = (int)L_.cg.even.size(), no = (int)L_.cg.odd.size();
  // u_e = D_ee^-1 b_e
  vzero<T>(W.t1.p, n, s);
  site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, b, W.t1.p, s);
  // rhs_o = b_o - D_oe u_e (zero on even sites)
  vzero<T>(W.t2.p, n, s);
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_odd.p, no, T(1), b, T(0), nullptr, T(-1), W.t1.p, W.t2.p, s);
  });
  cs_iters += fgmres<T>(
      c, [&](const C<T>* a, C<T>* o) { schur<T>(a, o); }, [](const C<T>*, C<T>*) {}, false, W.t2.p, z,
      p.coarse_restart, p.coarse_max_restarts, p.coarse_eps);
  // z_e = D_ee^-1 (b_e - D_eo z_o)
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_even.p, ne, T(1), b, T(0), nullptr, T(-1), z, W.t1.p, s);
  });
  site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, W.t1.p, z, s);
}

// ---------------------------------------------------------------------------
// the level-l cycle (Alg. 1; Alg. 2 replaces the recursive call by FGMRES)
// ---------------------------------------------------------------------------
template <typename T> void Hierarchy::cycle(int l, const C<T>* b, C<T>* z) {
  Work<T>& W = work<T>(l);
  Work<T>& Wc = work<T>(l + 1);
  const long long n = lv[l].n;
  vzero<T>(z, n, s);
  if (p.mu > 0) {
    sap<T>(l, b, z, p.mu);
    apply<T>(l, z, W.r.p);
    vbmy<T>(b, W.r.p, n, s);
    restrict_to<T>(l, W.r.p, Wc.bin.p);
  } else {
    restrict_to<T>(l, b, Wc.bin.p);
  }
  if (l + 1 == L - 1) {
    coarsest_solve<T>(Wc.bin.p, Wc.z.p);
  } else if (p.cycle == DDAMG_KCYCLE) {
    const int c = l + 1;
    kc_iters += fgmres<T>(
        c, [&](const C<T>* a, C<T>* o) { apply<T>(c, a, o); },
        [&](const C<T>* a, C<T>* o) { cycle<T>(c, a, o); }, true, Wc.bin.p, Wc.z.p, p.kc_len,
        p.kc_restarts, p.kc_tol);
  } else {
    cycle<T>(l + 1, Wc.bin.p, Wc.z.p);
  }
  if (recording) vcopy<T, T>(Wc.z.p, Wc.rec.p, lv[l + 1].n, s);
  prolong_add<T>(l, Wc.z.p, z);
  if (p.nu > 0) sap<T>(l, b, z, p.nu);
}

// ---------------------------------------------------------------------------
// outer FGMRES in FP64, right-preconditioned by the level-0 cycle at T
// ---------------------------------------------------------------------------
template <typename T> C<T>* outerZ(Hierarchy& H);
template <> C<double>* outerZ<double>(Hierarchy& H) { return H.oZ64.p; }
template <> C<float>* outerZ<float>(Hierarchy& H) { return H.oZ32.p; }

template <typename T> int Hierarchy::outer(const double2* b, double2* x, ddamg_solve_stats* st) {
  const long long n = lv[0].n;
  const int m = p.nkv;
  const FineOpView<double> D = ctx->view<double>();
  double2* V = oV.p;
  C<T>* Z = outerZ<T>(*this);
  double2* w = ow.p;
  const double bnorm = norm(b, n);
  if (!std::isfinite(bnorm)) {
    st->status = DDAMG_ENONFINITE;
    return DDAMG_ENONFINITE;
  }
  if (bnorm == 0.0) {
    vzero<double>(x, n, s);
    st->true_relres = 0;
    st->status = DDAMG_OK;
    return DDAMG_OK;
  }
  const double target = p.tol * bnorm;
  // r = b - D x
  dslash<double>(D, x, w, s);
  vbmy<double>(b, w, n, s);
  double beta = norm(w, n);
  std::vector<cd> Hm((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), h(KMAX + 1), h2(KMAX + 1);
  int iters = 0, restarts = 0;
  int status = DDAMG_ENOCONV;
  if (beta <= target) status = DDAMG_OK;
  Work<T>& W0 = work<T>(0);
  while (status == DDAMG_ENOCONV && restarts < p.max_restarts) {
    if (!std::isfinite(beta)) { status = DDAMG_ENONFINITE; break; }
    vlincomb_scale<double>(Coefs{}, 0, V, n, w, n, 1.0 / beta, V, s);
    std::fill(Hm.begin(), Hm.end(), cd(0));
    std::fill(g.begin(), g.end(), cd(0));
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double2* Vj = V + (size_t)j * n;
      C<T>* Zj = Z + (size_t)j * n;
      if constexpr (std::is_same<T, double>::value) {
        cycle<double>(0, Vj, Zj);
        dslash<double>(D, Zj, w, s);
      } else {
        vcopy<double, T>(Vj, W0.bin.p, n, s);
        cycle<T>(0, W0.bin.p, Zj);
        vcopy<T, double>(Zj, ot.p, n, s);
        dslash<double>(D, ot.p, w, s);
      }
      Coefs c;
      const double hn = gs_step<double>(*red, V, n, j, w, h, h2, c, s);
      for (int i = 0; i <= j; ++i) Hm[(size_t)i * m + j] = h[i];
      for (int i = 0; i < j; ++i) {
        cd a = Hm[(size_t)i * m + j], bq = Hm[(size_t)(i + 1) * m + j];
        Hm[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
        Hm[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * bq;
      }
      {
        cd a = Hm[(size_t)j * m + j];
        const double rho = std::sqrt(std::norm(a) + hn * hn);
        if (rho == 0.0) { cs[j] = 1; sn[j] = 0; }
        else if (std::abs(a) == 0.0) { cs[j] = 0; sn[j] = 1; }
        else {
          cs[j] = std::abs(a) / rho;
          sn[j] = (a / std::abs(a)) * hn / rho;
        }
        Hm[(size_t)j * m + j] = cs[j] * a + sn[j] * hn;
        g[j + 1] = -std::conj(sn[j]) * g[j];
        g[j] = cs[j] * g[j];
      }
      ++iters;
      jend = j + 1;
      const double est = std::abs(g[j + 1]);
      if (!std::isfinite(est)) { status = DDAMG_ENONFINITE; break; }
      if (est <= target || hn == 0.0) break;
      if (j + 1 < m) vlincomb_scale<double>(c, j + 1, V, n, w, n, 1.0 / hn, V + (size_t)(j + 1) * n, s);
    }
    if (status == DDAMG_ENONFINITE) break;
    std::vector<cd> y(jend);
    for (int i = jend - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= Hm[(size_t)i * m + k] * y[k];
      y[i] = acc / Hm[(size_t)i * m + i];
    }
    Coefs c;
    for (int i = 0; i < jend; ++i) c.c[i] = d2(y[i]);
    vlincomb<double, T>(c, jend, Z, n, x, n, s);
    ++restarts;
    // true residual in FP64
    dslash<double>(D, x, w, s);
    vbmy<double>(b, w, n, s);
    beta = norm(w, n);
    if (!std::isfinite(beta)) { status = DDAMG_ENONFINITE; break; }
    if (beta <= target) status = DDAMG_OK;
  }
  st->status = status;
  st->outer_iters = iters;
  st->restarts = restarts;
  st->true_relres = beta / bnorm;
  return status;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
template <typename T> std::vector<Work<T>>& work_vec(Hierarchy& H);
template <> std::vector<Work<double>>& work_vec<double>(Hierarchy& H) { return H.w64; }
template <> std::vector<Work<float>>& work_vec<float>(Hierarchy& H) { return H.w32; }

template <typename T> void Hierarchy::alloc_work() {
  std::vector<Work<T>>& W = work_vec<T>(*this);
  W.clear();
  W.resize(L);
  for (int l = 0; l < L; ++l) {
    const long long n = lv[l].n;
    Work<T>& w = W[l];
    w.bin.alloc(n);
    w.z.alloc(n);
    w.r.alloc(n);
    w.rec.alloc(n);
    w.x.alloc(n);
    w.w.alloc(n);
    if (l == L - 1) {
      w.t1.alloc(n);
      w.t2.alloc(n);
      w.t3.alloc(n);
      w.t4.alloc(n);
      w.m = p.coarse_restart;
      w.V.alloc((size_t)(w.m + 1) * n);
    } else if (l > 0) {
      w.m = p.kc_len;
      w.V.alloc((size_t)(w.m + 1) * n);
      w.Z.alloc((size_t)w.m * n);
    }
  }
}

void Hierarchy::build_level(int l, bool from32) {
  LevelStore& F = lv[l];
  LevelStore& Cc = lv[l + 1];
  const long long n = F.n;
  const int N = F.N;
  // the FP64 test vectors (for an FP32 setup: their FP64 copy) feed the
  // orthonormalisation, which writes P in FP64
  if (from32) vcopy<float, double>(F.tv32.p, F.tv64.p, (long long)N * n, s);
  if (l == 0) orthonormalise_fine(ctx->g, F.at, F.ad(), N, F.tv64.p, F.P64.p, s);
  else orthonormalise_coarse(F.at, F.ad(), F.d, N, F.V, F.tv64.p, F.P64.p, s);
  if (F.P32.p) vcopy<double, float>(F.P64.p, F.P32.p, (long long)N * n, s);
  if (F.P16.p) to_half(F.P64.p, F.P16.p, (long long)N * n, s);
  // Galerkin in FP64
  if (l == 0) galerkin_fine(ctx->g, F.at, F.ad(), N, ctx->view<double>(), F.P64.p, Cc.D64.p, s);
  else galerkin_coarse(F.cg, F.at, F.ad(), N, F.cview<double>(), F.P64.p, Cc.D64.p, s);
  expand_coarse<double2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K64.p, s);
  if (Cc.K32.p) expand_coarse<float2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K32.p, s);
  if (Cc.K16.p) expand_coarse<__half2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K16.p, s);
  if (l + 1 == L - 1 && Cc.cg.bipartite) {
    const int ne = (int)Cc.cg.even.size();
    self_block_inverse(Cc.D64.p, Cc.c_even.p, ne, Cc.d, Cc.Einv64.p, s);
    if (Cc.Einv32.p) vcopy<double, float>(Cc.Einv64.p, Cc.Einv32.p, (long long)ne * Cc.d * Cc.d, s);
  }
  DD_CHECK_HIP(hipStreamSynchronize(s));
}

template <typename T> void Hierarchy::initial_setup(int l) {
  LevelStore& F = lv[l];
  const long long n = F.n;
  const int N = F.N;
  Work<T>& W = work<T>(l);
  if (l > 0) {
    const int Np = lv[l - 1].N;
    for (int j = 0; j < N && j < Np; ++j)
      restrict_to<T>(l - 1, tv<T>(l - 1) + (size_t)j * lv[l - 1].n, tv<T>(l) + (size_t)j * n);
    if (N > Np) {
      DD_REQUIRE(tv_extra != nullptr, "extra test vectors needed for a level with more test vectors");
      long long off = 0;
      for (int k = 1; k < l; ++k)
        if (lv[k].N > lv[k - 1].N) off += (long long)(lv[k].N - lv[k - 1].N) * lv[k].n;
      vcopy<double, T>(tv_extra + off, tv<T>(l) + (size_t)Np * n, (long long)(N - Np) * n, s);
    }
  }
  for (int eta = 1; eta <= 3; ++eta)
    for (int j = 0; j < N; ++j) {
      C<T>* v = tv<T>(l) + (size_t)j * n;
      vzero<T>(W.x.p, n, s);
      sap<T>(l, v, W.x.p, eta);
      vcopy<T, T>(W.x.p, v, n, s);
    }
  build_level(l, std::is_same<T, float>::value);
  if (l < L - 2) initial_setup<T>(l + 1);
}

template <typename T> void Hierarchy::iterative_setup(int l, int i) {
  if (l >= L - 1) return;
  const int N = lv[l].N;
  for (int j = 0; j < N; ++j) {
    recording = true;
    cycle<T>(l, tv<T>(l) + (size_t)j * lv[l].n, work<T>(l).rec.p);
    recording = false;
    for (int k = l; k < L - 1; ++k) {
      if (j >= lv[k].N) continue;
      const long long nk = lv[k].n;
      C<T>* src = work<T>(k).rec.p;
      red->dots<T>(src, 0, 0, src, nk, true, s);
      cd rr;
      red->fetch(1, &rr, s);
      const double nrm = std::sqrt(rr.real());
      DD_REQUIRE(nrm > 0 && std::isfinite(nrm), "setup produced a zero or non-finite test vector");
      C<T>* dst = tv<T>(k) + (size_t)j * nk;
      vcopy<T, T>(src, dst, nk, s);
      vscale<T>(make_double2(1.0 / nrm, 0), dst, nk, s);
    }
  }
  for (int k = l; k < L - 1; ++k) build_level(k, std::is_same<T, float>::value);
  for (int q = 1; q <= i; ++q) iterative_setup<T>(l + 1, q);
}

template <typename T> void Hierarchy::setup(const double2* tvc) {
  fine_to_native<T>(ctx->g, tvc, tv<T>(0), lv[0].N, s);
  initial_setup<T>(0);
  for (int i = 1; i <= p.n_inv; ++i) iterative_setup<T>(0, i);
  DD_CHECK_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
void validate_params(const Context& ctx, const ddamg_params& p) {
  DD_REQUIRE(p.levels >= 2 && p.levels <= 4, "levels must be 2..4");
  DD_REQUIRE(p.precond_prec == DDAMG_F32 || p.precond_prec == DDAMG_F64, "bad precond_prec");
  DD_REQUIRE(p.cycle == DDAMG_KCYCLE || p.cycle == DDAMG_VCYCLE, "bad cycle");
  DD_REQUIRE(p.half_storage == 0 || p.half_storage == 1, "half_storage must be 0 or 1");
  DD_REQUIRE(p.half_storage == 0 || p.precond_prec == DDAMG_F32,
             "FP16 operator storage needs the FP32 preconditioner");
  DD_REQUIRE(p.mu >= 0 && p.nu >= 0 && p.mr_iters >= 0 && p.n_inv >= 0, "negative iteration count");
  DD_REQUIRE(p.nkv >= 1 && p.nkv <= KMAX - 1, "nkv out of range");
  DD_REQUIRE(p.kc_len >= 1 && p.kc_len <= KMAX - 1 && p.kc_restarts >= 1, "bad K-cycle length");
  DD_REQUIRE(p.coarse_restart >= 1 && p.coarse_restart <= KMAX - 1 && p.coarse_max_restarts >= 1,
             "bad coarsest GMRES restart");
  DD_REQUIRE(p.tol > 0 && p.kc_tol > 0 && p.coarse_eps > 0, "tolerances must be positive");
  DD_REQUIRE(p.max_restarts >= 1, "max_restarts must be >= 1");
  int dims[4] = {ctx.g.dims[0], ctx.g.dims[1], ctx.g.dims[2], ctx.g.dims[3]};
  for (int mu = 0; mu < 4; ++mu)
    DD_REQUIRE(p.sap_block[mu] >= 1, "bad SAP block");
  int d = 12;
  for (int l = 0; l < p.levels - 1; ++l) {
    // SAP validity on level l
    for (int mu = 0; mu < 4; ++mu) {
      if (l == 0) DD_REQUIRE(p.sap_block[mu] == 2, "the fine SAP blocks are 2^4");
      DD_REQUIRE(dims[mu] % p.sap_block[mu] == 0 && (dims[mu] / p.sap_block[mu]) % 2 == 0,
                 "SAP blocks must tile level " + std::to_string(l) + " with an even count per direction");
      DD_REQUIRE(p.agg[l][mu] >= 1 && dims[mu] % p.agg[l][mu] == 0,
                 "aggregates must tile level " + std::to_string(l));
    }
    int asz = p.agg[l][0] * p.agg[l][1] * p.agg[l][2] * p.agg[l][3];
    if (l == 0)
      DD_REQUIRE(asz == 256 && p.agg[0][0] % 2 == 0 && p.agg[0][1] % 2 == 0 && p.agg[0][2] % 2 == 0 &&
                     p.agg[0][3] % 2 == 0,
                 "fine aggregates must hold 256 sites made of 2^4 blocks (e.g. 4^4)");
    else
      DD_REQUIRE(asz * d <= 1024, "coarse aggregate too large");
    if (l > 0) {
      int bs = p.sap_block[0] * p.sap_block[1] * p.sap_block[2] * p.sap_block[3];
      DD_REQUIRE(bs * d <= 1024, "coarse SAP block too large");
    }
    DD_REQUIRE(p.ntv[l] >= 1 && p.ntv[l] <= 32, "ntv must be 1..32");
    DD_REQUIRE(p.ntv[l] <= asz * d / 2, "more test vectors than an aggregate's dimension");
    for (int mu = 0; mu < 4; ++mu) dims[mu] /= p.agg[l][mu];
    d = 2 * p.ntv[l];
  }
  DD_REQUIRE(d <= 64, "coarsest dof per site must be <= 64");
}

Hierarchy* create_hierarchy(Context* ctx, const ddamg_params* pp, const double2* tvc,
                            const double2* tv_extra, hipStream_t s) {
  DD_REQUIRE(ctx && pp && tvc, "null argument");
  validate_params(*ctx, *pp);
  std::unique_ptr<Hierarchy> H(new Hierarchy);
  H->ctx = ctx;
  H->p = *pp;
  H->L = pp->levels;
  H->s = s;
  H->tv_extra = tv_extra;
  H->red.reset(new Reducer);
  H->half = pp->half_storage == 1;
  const ddamg_params& p = H->p;
  if (H->half) ctx->make_half(s);
  const int L = H->L;
  H->lv.resize(L);
  int dims[4];
  for (int mu = 0; mu < 4; ++mu) dims[mu] = ctx->g.dims[mu];
  int d = 12;
  for (int l = 0; l < L; ++l) {
    LevelStore& S = H->lv[l];
    S.fine = l == 0;
    for (int mu = 0; mu < 4; ++mu) S.dims[mu] = dims[mu];
    S.d = d;
    S.V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    S.n = S.V * d;
    if (l > 0) {
      int sap[4] = {0, 0, 0, 0};
      if (l < L - 1) for (int mu = 0; mu < 4; ++mu) sap[mu] = p.sap_block[mu];
      S.cg = make_coarse_geom(dims, d, sap);
      S.c_nbr9.upload(S.cg.nbr9, s);
      S.c_blk_sites.upload(S.cg.blk_sites, s);
      S.c_site_blk.upload(S.cg.site_blk, s);
      S.c_even.upload(S.cg.even, s);
      S.c_odd.upload(S.cg.odd, s);
      S.D64.alloc((size_t)S.V * 5 * d * d);
      S.K64.alloc((size_t)S.V * 9 * d * d);
      if (!H->half) S.K32.alloc((size_t)S.V * 9 * d * d);
      if (H->half) S.K16.alloc((size_t)S.V * 9 * d * d);
      if (l < L - 1) {
        const size_t nv = (size_t)S.V * d;
        S.sr64.alloc(2 * nv);
        S.sq64.alloc(2 * nv);
        S.sr32.alloc(2 * nv);
        S.sq32.alloc(2 * nv);
        S.sp64.alloc(2 * (size_t)S.V * 4);
        S.sp32.alloc(2 * (size_t)S.V * 4);
        for (int k = 0; k < 2; ++k) {
          S.ss64.rho[k] = S.sr64.p + k * nv;
          S.ss64.q[k] = S.sq64.p + k * nv;
          S.ss64.part[k] = S.sp64.p + k * (size_t)S.V * 4;
          S.ss32.rho[k] = S.sr32.p + k * nv;
          S.ss32.q[k] = S.sq32.p + k * nv;
          S.ss32.part[k] = S.sp32.p + k * (size_t)S.V * 4;
        }
      }
      if (l == L - 1 && S.cg.bipartite) {
        S.Einv64.alloc(S.cg.even.size() * (size_t)d * d);
        S.Einv32.alloc(S.cg.even.size() * (size_t)d * d);
      }
    }
    if (l < L - 1) {
      S.N = p.ntv[l];
      S.at = l == 0 ? make_fine_agg(ctx->g, p.agg[l]) : make_coarse_agg(S.cg, p.agg[l]);
      S.a_members.upload(S.at.members, s);
      S.a_member_agg.upload(S.at.member_agg, s);
      S.P64.alloc((size_t)S.N * S.n);
      if (!H->half) S.P32.alloc((size_t)S.N * S.n);
      if (H->half) S.P16.alloc((size_t)S.N * S.n);
      S.tv64.alloc((size_t)S.N * S.n);
      if (p.precond_prec == DDAMG_F32) S.tv32.alloc((size_t)S.N * S.n);
      for (int mu = 0; mu < 4; ++mu) dims[mu] = S.at.cdims[mu];
      d = 2 * S.N;
    }
  }
  const long long n0 = H->lv[0].n;
  H->oV.alloc((size_t)(p.nkv + 1) * n0);
  H->ow.alloc(n0);
  H->ob.alloc(n0);
  H->ox.alloc(n0);
  if (p.precond_prec == DDAMG_F32) {
    H->alloc_work<float>();
    H->oZ32.alloc((size_t)p.nkv * n0);
    H->ot.alloc(n0);
    H->setup<float>(tvc);
  } else {
    H->alloc_work<double>();
    H->oZ64.alloc((size_t)p.nkv * n0);
    H->setup<double>(tvc);
  }
  H->tv_extra = nullptr;
  return H.release();
}

// explicit instantiations used by the C ABI
template void Hierarchy::apply<double>(int, const C<double>*, C<double>*);
template void Hierarchy::apply<float>(int, const C<float>*, C<float>*);
template void Hierarchy::sap<double>(int, const C<double>*, C<double>*, int);
template void Hierarchy::sap<float>(int, const C<float>*, C<float>*, int);
template void Hierarchy::restrict_to<double>(int, const C<double>*, C<double>*);
template void Hierarchy::restrict_to<float>(int, const C<float>*, C<float>*);
template void Hierarchy::prolong_add<double>(int, const C<double>*, C<double>*);
template void Hierarchy::prolong_add<float>(int, const C<float>*, C<float>*);
template void Hierarchy::cycle<double>(int, const C<double>*, C<double>*);
template void Hierarchy::cycle<float>(int, const C<float>*, C<float>*);
template int Hierarchy::outer<double>(const double2*, double2*, ddamg_solve_stats*);
template int Hierarchy::outer<float>(const double2*, double2*, ddamg_solve_stats*);
template void Hierarchy::setup<double>(const double2*);
template void Hierarchy::setup<float>(const double2*);
template void Hierarchy::alloc_work<double>();
template void Hierarchy::alloc_work<float>();

}  // namespace ddamg
