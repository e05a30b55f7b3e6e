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

#include <atomic>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
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

// polled mode of the device-scalar GMRES: the first read of the liveness
// flag comes after the number of steps the previous solve of the level
// needed (a read costs a host round trip, a step past convergence a few
// launches), then one read per step
constexpr int COARSE_POLL = 1;

// the outer FGMRES stops a system whose recomputed residual a restart cycle
// has reduced by less than this factor (stagnation)
constexpr double OUTER_STAGNATION = 0.999;

// largest coarsest Schur system (unknowns) stored as a dense matrix: 2048^2
// complex entries are 64 MiB in FP64 and 32 MiB in FP32
constexpr long long DENSE_SCHUR_MAX = 2048;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static void check_lattice(const ddamg_lattice* lat) {
  DD_REQUIRE(lat != nullptr, "null lattice");
  for (int mu = 0; mu < 4; ++mu)
    DD_REQUIRE(lat->dims[mu] >= 4 && lat->dims[mu] % 4 == 0,
               "every lattice extent must be a positive multiple of 4");
  DD_REQUIRE(std::isfinite(lat->m0) && std::isfinite(lat->csw), "non-finite m0 or csw");
}

// geometry, neighbour tables and the operator arrays of a context (no
// kernels); with a workspace also the FP16 copies and the canonical-layout
// scratch that would otherwise be made on first use
static void context_layout(Context& c, const ddamg_lattice* lat, bool half, int nrhs_max, hipStream_t s) {
  c.g = make_fine_geom(lat->dims);
  c.m0 = lat->m0;
  c.csw = lat->csw;
  const FineGeom& g = c.g;
  std::vector<int> nbr((size_t)g.nblk * 8), cblk(g.nblk);
  fine_tables(g, nbr.data(), cblk.data());
  c.nbr.upload(nbr, s);
  c.cblk.upload(cblk, s);
  c.U64.alloc((size_t)g.V * 36);
  c.U32.alloc((size_t)g.V * 36);
  c.A64.alloc((size_t)g.V * 36);
  c.A32.alloc((size_t)g.V * 36);
  if (current_workspace()) {
    if (half) {
      c.U16.alloc((size_t)g.V * 36);
      c.A16.alloc((size_t)g.V * 36);
    }
    if (nrhs_max > 0) {
      c.s64a.alloc((size_t)g.V * 12 * nrhs_max);
      c.s64b.alloc((size_t)g.V * 12 * nrhs_max);
    }
  }
}

Context* create_context(const ddamg_lattice* lat, const double2* links, hipStream_t s,
                        std::unique_ptr<Workspace> ws, bool half, int nrhs_max) {
  check_lattice(lat);
  DD_REQUIRE(links != nullptr, "null links");
  std::unique_ptr<Context> c(new Context);
  c->ws = std::move(ws);
  const WorkspaceScope scope(c->ws.get());
  context_layout(*c, lat, half, nrhs_max, s);
  const FineGeom& g = c->g;
  links_to_native<double>(g, links, c->U64.p, s);
  links_to_native<float>(g, links, c->U32.p, s);
  clover_build(g, links, lat->m0, lat->csw, c->A64.p, s);
  vcopy<double, float>(c->A64.p, c->A32.p, (long long)g.V * 36, s);
  if (c->U16.p) c->make_half(s);
  DD_CHECK_HIP(hipStreamSynchronize(s));
  return c.release();
}

void Context::make_half(hipStream_t s) {
  if (half_ready) return;
  // the copies belong to the context: from its workspace, if it has one
  const WorkspaceScope scope(ws.get());
  if (!U16.p) {
    U16.alloc((size_t)g.V * 36);
    A16.alloc((size_t)g.V * 36);
  }
  to_half(U64.p, U16.p, (long long)g.V * 36, s);
  to_half(A64.p, A16.p, (long long)g.V * 36, s);
  half_ready = true;
}

// ---------------------------------------------------------------------------
// level operations
// ---------------------------------------------------------------------------
void Hierarchy::lt_mark(int level) {
  hipEvent_t e = nullptr;
  if (lt_pool.empty()) {
    DD_CHECK_HIP(hipEventCreate(&e));
  } else {
    e = lt_pool.back();
    lt_pool.pop_back();
  }
  lt_marks.emplace_back(e, level);
  DD_CHECK_HIP(hipEventRecord(e, s));
}
void Hierarchy::lt_push(int l) {
  if (!lt_on) return;
  lt_stack.push_back(l);
  lt_mark(l);
}
void Hierarchy::lt_pop() {
  if (!lt_on) return;
  lt_stack.pop_back();
  lt_mark(lt_stack.empty() ? 0 : lt_stack.back());
}
void Hierarchy::lt_begin() {
  lt_on = p.profile_levels == 1 && !p.graph;
  for (auto& m : lt_marks) lt_pool.push_back(m.first);
  lt_marks.clear();
  lt_stack.assign(1, 0);
  if (lt_on) lt_mark(0);
}
void Hierarchy::lt_end(double out[4]) {
  for (int k = 0; k < 4; ++k) out[k] = 0;
  if (!lt_on) return;
  lt_mark(0);
  DD_CHECK_HIP(hipEventSynchronize(lt_marks.back().first));
  for (size_t i = 0; i + 1 < lt_marks.size(); ++i) {
    float ms = 0;
    DD_CHECK_HIP(hipEventElapsedTime(&ms, lt_marks[i].first, lt_marks[i + 1].first));
    out[std::min(lt_marks[i].second, 3)] += ms * 1e-3;
  }
  for (auto& m : lt_marks) lt_pool.push_back(m.first);
  lt_marks.clear();
  lt_on = false;
}

template <typename T> void Hierarchy::apply(int l, const C<T>* in, C<T>* out, int nb) {
  const double V = (double)lv[l].V, vz = sizeof(C<T>), ob = op_bytes<T>();
  if (l == 0) {
    // spinor in and out (24 complex), four links and the clover (72 complex)
    meter(V * (24 * vz * nb + 72 * ob), 1870.0 * V * nb);
    fine_op<T>([&](const auto& op) { dslash(op, in, out, s, nb); });
  } else {
    const double d = lv[l].d;
    meter(V * (9 * d * d * ob + 2 * d * vz * nb), 72.0 * d * d * V * nb);
    coarse_op<T>(l, [&](const auto& op) { coarse_apply(op, in, out, s, nb); });
  }
}

// coarse SAP work buffers of level l for a batch of nb (grown on demand)
template <typename T, typename E>
static SapScratch<T>& sap_buffers(DevArray<C<T>>& rho, DevArray<C<T>>& q, DevArray<E>& part, SapScratch<T>& ss,
                                  long long nv, long long V, int nb) {
  if (rho.n < 2 * (size_t)nv * nb) {
    rho.alloc(2 * (size_t)nv * nb);
    q.alloc(2 * (size_t)nv * nb);
    part.alloc(2 * (size_t)V * 4 * nb);
    for (int k = 0; k < 2; ++k) {
      ss.rho[k] = rho.p + (size_t)k * nv * nb;
      ss.q[k] = q.p + (size_t)k * nv * nb;
      ss.part[k] = part.p + (size_t)k * V * 4 * nb;
    }
  }
  return ss;
}
template <typename T> SapScratch<T>& sap_scratch(LevelStore& L_, int nb);
template <> SapScratch<double>& sap_scratch<double>(LevelStore& L_, int nb) {
  return sap_buffers<double>(L_.sr64, L_.sq64, L_.sp64, L_.ss64, L_.n, L_.V, nb);
}
template <> SapScratch<float>& sap_scratch<float>(LevelStore& L_, int nb) {
  return sap_buffers<float>(L_.sr32, L_.sq32, L_.sp32, L_.ss32, L_.n, L_.V, nb);
}

template <typename T> const void* sap_scratch_base(const LevelStore& L_);
template <> const void* sap_scratch_base<double>(const LevelStore& L_) { return L_.sr64.p; }
template <> const void* sap_scratch_base<float>(const LevelStore& L_) { return L_.sr32.p; }

template <typename T> void Hierarchy::sap(int l, const C<T>* b, C<T>* z, int nsweeps, int nb) {
  {
    const double V = (double)lv[l].V, vz = sizeof(C<T>), ob = op_bytes<T>();
    if (l == 0) {
      // per sweep: b, z in, z out (36 complex per site and field), links and
      // clover (72 complex); residual + mr_iters block-MR steps
      meter(nsweeps * V * (36 * vz * nb + 72 * ob), nsweeps * (1870.0 + p.mr_iters * 2280.0) * V * nb);
    } else {
      // per sweep about 1 + mr_iters applications of the level operator
      const double d = lv[l].d;
      meter(nsweeps * (1.0 + p.mr_iters) * V * (9 * d * d * ob + 2 * d * vz * nb),
            nsweeps * (1.0 + p.mr_iters) * 72.0 * d * d * V * nb);
    }
  }
  for (int it = 0; it < nsweeps; ++it)
    for (int col = 0; col < 2; ++col) {
      if (l == 0) {
        fine_op<T>([&](const auto& op) { sap_colour(op, ctx->cblk.p, col, p.mr_iters, b, z, s, nb); });
      } else {
        LevelStore& L_ = lv[l];
        const void* before = sap_scratch_base<T>(L_);
        SapScratch<T>& ws = sap_scratch<T>(L_, nb);
        if (sap_scratch_base<T>(L_) != before) ++gen;
        coarse_op<T>(l, [&](const auto& op) {
          coarse_sap_colour(op, L_.sap_tables(), col, p.mr_iters, b, z, ws, s, nb);
        });
      }
    }
}

template <typename T> void Hierarchy::restrict_to(int l, const C<T>* fine, C<T>* coarse, int nb) {
  const LevelStore& L_ = lv[l];
  meter(L_.N * (double)L_.n * op_bytes<T>() + ((double)L_.n + 2.0 * L_.N * lv[l + 1].V) * sizeof(C<T>) * nb,
        8.0 * L_.N * (double)L_.n * nb);
  interp<T>(l, [&](const auto* P_) {
    if (l == 0) restrict_fine<T>(ctx->g, L_.at, L_.ad(), L_.N, P_, fine, coarse, s, nb);
    else restrict_coarse<T>(L_.at, L_.ad(), L_.d, L_.N, L_.V, P_, fine, coarse, s, nb);
  });
}

template <typename T> void Hierarchy::prolong_add(int l, const C<T>* coarse, C<T>* fine, int nb) {
  const LevelStore& L_ = lv[l];
  meter(L_.N * (double)L_.n * op_bytes<T>() + (2.0 * L_.n + 2.0 * L_.N * lv[l + 1].V) * sizeof(C<T>) * nb,
        8.0 * L_.N * (double)L_.n * nb);
  interp<T>(l, [&](const auto* P_) {
    if (l == 0) prolong_fine<T>(ctx->g, L_.at, L_.ad(), L_.N, P_, coarse, fine, s, nb);
    else prolong_coarse<T>(L_.at, L_.ad(), L_.d, L_.N, L_.V, P_, coarse, fine, s, nb);
  });
}


// ---------------------------------------------------------------------------
// Batched Krylov building blocks.  Every system r of a batch has its own
// Hessenberg matrix, Givens rotations and stopping test on the host; the
// vector work of all systems goes through one launch per operation.  A
// system that has stopped is carried along with zero basis vectors (scale
// 0), so it costs work but never changes again.
// ---------------------------------------------------------------------------
// norms ||v_r|| of a batch
template <typename T>
void bnorms(Reducer& red, const C<T>* v, long long n, int nb, std::vector<double>& out, hipStream_t s) {
  red.bdots<T>(nullptr, v, 0, 0, const_cast<C<T>*>(v), n, nb, s);
  std::vector<cd> r(nb);
  red.bfetch(1, nb, r.data(), s);
  out.resize(nb);
  for (int k = 0; k < nb; ++k) out[k] = std::sqrt(std::max(r[k].real(), 0.0));
}

// dst_r = scale_r * src_r
template <typename T>
static void bscale_host(Reducer& red, const std::vector<double>& scale, const C<T>* src, C<T>* dst, long long n,
                        int nb, hipStream_t s) {
  const BArg a = red.upload(std::vector<cd>(), scale, nb, s);
  bscale<T>(a, src, dst, n, nb, s);
}

// Arnoldi step with classical Gram-Schmidt; a second pass for the systems
// whose first pass removed more than half of ||w||^2 (the criterion of
// Daniel, Gragg, Kaufman and Stewart).
template <typename T>
void Hierarchy::arnoldi(const C<T>* V, long long vstride, long long n, int nb, int j, C<T>* w,
                        const std::vector<char>& live, std::vector<cd>& h, std::vector<double>& hn,
                        std::vector<cd>& cf) {
  const int k1 = j + 2;
  // the inner products read V_0..V_j and w; the update reads them again and
  // writes the next basis vector.  The second pass takes the products of
  // w - V h1 without storing it: the basis vector is then formed from w with
  // the summed coefficients -(h1 + h2)
  meter((2.0 * k1 + 1) * n * sizeof(C<T>) * nb, 16.0 * k1 * n * nb);
  std::vector<cd> h1((size_t)nb * k1), h2((size_t)nb * k1), c1((size_t)nb * KMAX, cd(0));
  red->bdots<T>(nullptr, V, vstride, j + 1, w, n, nb, s);
  red->bfetch(k1, nb, h1.data(), s);
  h.assign((size_t)nb * (KMAX + 1), cd(0));
  hn.assign(nb, 0.0);
  cf.assign((size_t)nb * KMAX, cd(0));
  std::vector<char> again(nb, 0);
  bool any = false;
  for (int r = 0; r < nb; ++r) {
    const cd* hr = &h1[(size_t)r * k1];
    const double ww = hr[j + 1].real();
    double proj = 0;
    for (int i = 0; i <= j; ++i) proj += std::norm(hr[i]);
    for (int i = 0; i <= j; ++i) {
      h[(size_t)r * (KMAX + 1) + i] = hr[i];
      cf[(size_t)r * KMAX + i] = -hr[i];
    }
    hn[r] = std::sqrt(std::max(ww - proj, 0.0));
    if (live[r] && !(ww - proj > 0.5 * ww)) {
      again[r] = 1;
      any = true;
      for (int i = 0; i <= j; ++i) c1[(size_t)r * KMAX + i] = -hr[i];
    }
  }
  if (!any) return;
  const BArg a = red->upload(c1, std::vector<double>(), nb, s);
  red->bdots<T>(&a, V, vstride, j + 1, w, n, nb, s, nullptr, false);
  red->bfetch(k1, nb, h2.data(), s);
  for (int r = 0; r < nb; ++r) {
    if (!again[r]) continue;
    const cd* hr = &h2[(size_t)r * k1];
    double nn = hr[j + 1].real();
    for (int i = 0; i <= j; ++i) {
      nn -= std::norm(hr[i]);
      h[(size_t)r * (KMAX + 1) + i] += hr[i];
      cf[(size_t)r * KMAX + i] = -h[(size_t)r * (KMAX + 1) + i];
    }
    hn[r] = std::sqrt(std::max(nn, 0.0));
  }
}

// Givens update of column j of system r's Hessenberg matrix H (row-major
// (m+1) x m) and of its right-hand side g; returns |g[j+1]|
static double givens_column(cd* H, cd* g, cd* cs, cd* sn, int m, int j, const cd* h, double hn) {
  for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
  H[(size_t)(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const cd a = H[(size_t)i * m + j], bq = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
    H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * bq;
  }
  const cd a = H[(size_t)j * m + j];
  const double rho = std::sqrt(std::norm(a) + hn * hn);
  if (rho == 0.0) { cs[j] = 1; sn[j] = 0; }
  else if (std::abs(a) == 0.0) { cs[j] = 0; sn[j] = 1; }
  else {
    cs[j] = std::abs(a) / rho;
    sn[j] = (a / std::abs(a)) * hn / rho;
  }
  H[(size_t)j * m + j] = cs[j] * a + sn[j] * hn;
  H[(size_t)(j + 1) * m + j] = 0;
  g[j + 1] = -std::conj(sn[j]) * g[j];
  g[j] = cs[j] * g[j];
  return std::abs(g[j + 1]);
}

// y = R^{-1} g for the leading jend x jend triangle
static void back_substitute(const cd* H, const cd* g, int m, int jend, cd* y) {
  for (int i = jend - 1; i >= 0; --i) {
    cd acc = g[i];
    for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)i * m + k] * y[k];
    y[i] = acc / H[(size_t)i * m + i];
  }
}

// ---------------------------------------------------------------------------
// Flexible GMRES(m) on level l for a batch, from x = 0, at most max_cycles
// restart cycles per system, system r stops when its Arnoldi residual
// estimate <= tol ||b_r||.
// ---------------------------------------------------------------------------
template <typename T, typename Op, typename Pre>
void Hierarchy::fgmres(int l, Op op, Pre pre, bool use_pre, const C<T>* b, C<T>* x, int m, int max_cycles,
                       double tol, int nb, long long* iters) {
  Work<T>& W = work<T>(l);
  const long long n = lv[l].n, vs = (long long)nb * n;
  DD_REQUIRE(m <= W.m && nb <= W.cap, "Krylov basis too short for the batch");
  C<T>* V = W.V.p;
  C<T>* Z = use_pre ? W.Z.p : W.V.p;
  C<T>* w = W.w.p;
  vzero<T>(x, vs, s);
  std::vector<double> beta, target(nb), scale(nb);
  bnorms<T>(*red, b, n, nb, beta, s);
  std::vector<char> active(nb);
  bool any = false;
  for (int r = 0; r < nb; ++r) {
    active[r] = beta[r] > 0;
    target[r] = tol * beta[r];
    scale[r] = active[r] ? 1.0 / beta[r] : 0.0;
    any = any || active[r];
  }
  if (!any) return;
  bscale_host<T>(*red, scale, b, V, n, nb, s);
  std::vector<cd> H((size_t)nb * (m + 1) * m), g((size_t)nb * (m + 1)), cs((size_t)nb * m), sn((size_t)nb * m);
  std::vector<cd> h, cf, y(m), cy((size_t)nb * KMAX);
  std::vector<double> hn;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    std::fill(H.begin(), H.end(), cd(0));
    std::fill(g.begin(), g.end(), cd(0));
    for (int r = 0; r < nb; ++r) g[(size_t)r * (m + 1)] = active[r] ? beta[r] : 0.0;
    std::vector<int> jend(nb, 0);
    std::vector<char> live = active, conv(nb, 0);
    for (int j = 0; j < m; ++j) {
      C<T>* Vj = V + (size_t)j * vs;
      C<T>* Zj = Z + (size_t)j * vs;
      if (use_pre) {
        // a stopped system is carried with zero input: not a visit of the
        // levels below for the setup's record
        const std::vector<char> outer_visit = visit;
        for (int r = 0; r < nb && r < (int)visit.size(); ++r) visit[r] = visit[r] && live[r];
        pre(Vj, Zj);
        visit = outer_visit;
      }
      op(Zj, w);
      arnoldi<T>(V, vs, n, nb, j, w, live, h, hn, cf);
      bool still = false;
      for (int r = 0; r < nb; ++r) {
        if (!live[r]) continue;
        const double est = givens_column(&H[(size_t)r * (m + 1) * m], &g[(size_t)r * (m + 1)], &cs[(size_t)r * m],
                                         &sn[(size_t)r * m], m, j, &h[(size_t)r * (KMAX + 1)], hn[r]);
        if (iters) ++iters[r];
        jend[r] = j + 1;
        if (!std::isfinite(est)) throw Error(DDAMG_ENONFINITE, "non-finite residual in GMRES");
        if (est <= target[r] || hn[r] == 0.0) {
          live[r] = 0;
          conv[r] = 1;
        }
        still = still || live[r];
      }
      if (!still) break;
      // w += V c and V_{j+1} = w / hn in one pass (zero for stopped systems)
      if (j + 1 < m) {
        for (int r = 0; r < nb; ++r) scale[r] = live[r] ? 1.0 / hn[r] : 0.0;
        const BArg a = red->upload(cf, scale, nb, s);
        blincomb<T, T>(a, j + 1, V, vs, w, n, nb, V + (size_t)(j + 1) * vs, s);
      }
    }
    // x_r += Z_r y_r
    int kmax = 0;
    std::fill(cy.begin(), cy.end(), cd(0));
    for (int r = 0; r < nb; ++r) {
      if (!active[r] || jend[r] == 0) continue;
      back_substitute(&H[(size_t)r * (m + 1) * m], &g[(size_t)r * (m + 1)], m, jend[r], y.data());
      for (int i = 0; i < jend[r]; ++i) cy[(size_t)r * KMAX + i] = y[i];
      kmax = std::max(kmax, jend[r]);
    }
    if (kmax > 0) {
      const BArg a = red->upload(cy, std::vector<double>(), nb, s);
      blincomb<T, T>(a, kmax, Z, vs, x, n, nb, nullptr, s);
    }
    bool more = false;
    for (int r = 0; r < nb; ++r) {
      active[r] = active[r] && !conv[r];
      more = more || active[r];
    }
    if (!more || cyc + 1 == max_cycles) break;
    // restart the unfinished systems from their true residuals
    op(x, w);
    vbmy<T>(b, w, vs, s);
    bnorms<T>(*red, w, n, nb, beta, s);
    more = false;
    for (int r = 0; r < nb; ++r) {
      active[r] = active[r] && beta[r] > 0;
      scale[r] = active[r] ? 1.0 / beta[r] : 0.0;
      more = more || active[r];
    }
    if (!more) break;
    bscale_host<T>(*red, scale, w, V, n, nb, s);
  }
}

// ---------------------------------------------------------------------------
// coarsest level: odd-even reduced system
// ---------------------------------------------------------------------------
template <typename T> const C<T>* einv(const LevelStore& L_);
template <> const C<double>* einv<double>(const LevelStore& L_) { return L_.Einv64.p; }
template <> const C<float>* einv<float>(const LevelStore& L_) { return L_.Einv32.p; }

template <typename T> void Hierarchy::schur(const C<T>* v, C<T>* out, int nb) {
  const int c = L - 1;
  const LevelStore& L_ = lv[c];
  if (L_.sm > 0) {
    const C<T>* S;
    if constexpr (std::is_same<T, double>::value) S = L_.S64.p;
    else S = L_.S32.p;
    meter((double)L_.sm * L_.sm * sizeof(C<T>) + 2.0 * L_.sm * sizeof(C<T>) * nb, 8.0 * L_.sm * L_.sm * nb);
    dense_schur_apply<T>(S, L_.sm, L_.s_oidx.p, L_.s_eidx.p, L_.n, v, out, s, nb);
    return;
  }
  Work<T>& W = work<T>(c);
  const int ne = (int)L_.cg.even.size(), no = (int)L_.cg.odd.size();
  {
    // two half-lattice sweeps of the stencil and the even self-block inverses
    const double d = L_.d;
    meter(L_.V * (9 * d * d * op_bytes<T>() + 4 * d * sizeof(C<T>) * nb) + ne * d * d * sizeof(C<T>),
          (72.0 + 8.0) * d * d * L_.V * nb);
  }
  // t3_e = D_eo v_o ; t4_e = D_ee^-1 t3_e ; out_o = D_oo v_o - D_oe t4_e
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_even.p, ne, T(0), nullptr, T(0), nullptr, T(1), v, W.t3.p, s, nb);
    site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, L_.n, W.t3.p, W.t4.p, s, nb);
    vzero<T>(out, L_.n * nb, s);
    coarse_site_apply(op, L_.c_odd.p, no, T(0), nullptr, T(1), v, T(-1), W.t4.p, out, s, nb);
  });
}

// ---------------------------------------------------------------------------
// GMRES(m) from x = 0 with the scalars on the device: the host-driven
// fgmres above (unpreconditioned) as a fixed sequence of launches
// ---------------------------------------------------------------------------
DevGmres Hierarchy::gm() {
  if (!gm_sys.p) {
    gm_sys.alloc(NBMAX);
    gm_res.alloc((size_t)NBMAX * (KMAX + 1));
    gm_coef.alloc((size_t)NBMAX * KMAX);
    gm_scale.alloc(NBMAX);
    gm_iters.alloc(NBMAX);
    ++gen;
  }
  if (!gm_flag_host && !counting_only()) {
    DD_CHECK_HIP(hipHostMalloc(&gm_flag_host, sizeof(int), hipHostMallocCoherent));
    DD_CHECK_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&gm_flag_dev), gm_flag_host, 0));
  }
  DevGmres d;
  d.sys = gm_sys.p;
  d.res = gm_res.p;
  d.coef = gm_coef.p;
  d.scale = gm_scale.p;
  d.iters = gm_iters.p;
  d.flag = gm_flag_dev;
  return d;
}

// ---------------------------------------------------------------------------
// outer FGMRES of one right-hand side with the scalars on the device: the
// host-driven outer() above as a fixed launch sequence per step, so that the
// steps of several hierarchies can be captured into one graph
// (ddamg_solve_batch).  Right preconditioning by the level-0 cycle at FP32
// (fixed launch sequence: V- or W-cycle, coarsest GMRES with device scalars),
// FP64 basis V and residuals, FP32 directions Z.  A system whose estimate has
// met the target runs the remaining steps with zero coefficients and zero
// basis vectors; at the end of a cycle the recomputed FP64 residual decides
// whether it continues (gm_begin mode 2), as the host-driven solver's
// certification does.
// ---------------------------------------------------------------------------
DevGmres Hierarchy::gmo() {
  if (!go_sys.p) {
    go_sys.alloc(NBMAX);
    go_res.alloc((size_t)NBMAX * (KMAX + 1));
    go_coef.alloc((size_t)NBMAX * KMAX);
    go_scale.alloc(NBMAX);
    go_iters.alloc(NBMAX);
    ++gen;
  }
  if (!go_flag_host && !counting_only()) {
    DD_CHECK_HIP(hipHostMalloc(&go_flag_host, sizeof(int), hipHostMallocCoherent));
    DD_CHECK_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&go_flag_dev), go_flag_host, 0));
  }
  DevGmres d;
  d.sys = go_sys.p;
  d.res = go_res.p;
  d.coef = go_coef.p;
  d.scale = go_scale.p;
  d.iters = go_iters.p;
  d.flag = go_flag_dev;
  return d;
}

void Hierarchy::outer_dev_prepare() {
  DD_REQUIRE(p.precond_prec == DDAMG_F32 && !hs && p.half_directions == 0,
             "the batched graph solve needs the FP32 preconditioner with FP32 spinors and directions");
  DD_REQUIRE(p.graph == 1, "the batched graph solve needs hierarchies built with graph = 1");
  ensure_batch<float>(1);
  gmo();
  gm();
  const long long n = lv[0].n;
  if (go_zeroed != gen) {
    // the tail combines all n_kv directions (zero coefficients past the
    // last step): every slot must hold finite values from the start
    vzero<double>(oV.p, (long long)(p.nkv + 1) * n, s);
    vzero<float>(oZ32.p, (long long)p.nkv * n, s);
  }
  // one eager cycle makes the lazily allocated scratch exist before capture
  Work<float>& W0 = work<float>(0);
  vzero<float>(W0.bin.p, n, s);
  dev_scalars = true;
  try {
    cycle<float>(0, W0.bin.p, oZ32.p, 1);
  } catch (...) {
    dev_scalars = false;
    throw;
  }
  dev_scalars = false;
  DD_CHECK_HIP(hipStreamSynchronize(s));
  go_zeroed = gen;
}

void Hierarchy::outer_dev_begin() {
  const long long n = lv[0].n;
  const DevGmres d = gmo();
  const BArg a = d.arg();
  const FineOpView<double> D = ctx->view<double>();
  gm_reset(d, 1, s);
  // targets tol * ||b||
  red->bdots<double>(nullptr, ob.p, 0, 0, ob.p, n, 1, s, d.res);
  gm_begin(d, p.nkv, 1, p.tol, 1, s);
  // r_0 = b - D x_0 decides whether the system starts at all
  dslash<double>(D, ox.p, ow.p, s, 1);
  vbmy<double>(ob.p, ow.p, n, s);
  red->bdots<double>(nullptr, ow.p, 0, 0, ow.p, n, 1, s, d.res);
  gm_begin(d, p.nkv, 1, p.tol, 2, s);
  bscale<double>(a, ow.p, oV.p, n, 1, s);
}

void Hierarchy::outer_dev_step(int j) {
  const long long n = lv[0].n;
  const int m = p.nkv;
  const DevGmres d = gmo();
  const BArg a = d.arg();
  const FineOpView<double> D = ctx->view<double>();
  Work<float>& W0 = work<float>(0);
  double2* Vj = oV.p + (size_t)j * n;
  float2* Zj = oZ32.p + (size_t)j * n;
  vcopy<double, float>(Vj, W0.bin.p, n, s);
  const bool ds = dev_scalars;
  dev_scalars = true;
  try {
    cycle<float>(0, W0.bin.p, Zj, 1);
  } catch (...) {
    dev_scalars = ds;
    throw;
  }
  dev_scalars = ds;
  vcopy<float, double>(Zj, ot.p, n, s);
  meter((double)ctx->g.V * (24 * 16.0 + 72 * 16.0), 1870.0 * ctx->g.V);
  dslash<double>(D, ot.p, ow.p, s, 1);
  meter((2.0 * (j + 2) + 1) * n * 16.0, 16.0 * (j + 2) * n);
  red->bdots<double>(nullptr, oV.p, n, j + 1, ow.p, n, 1, s, d.res);
  gm_cgs1(d, j, 1, s);
  red->bdots<double>(&a, oV.p, n, j + 1, ow.p, n, 1, s, d.res);
  gm_step(d, j, m, 1, s);
  if (j + 1 < m) blincomb<double, double>(a, j + 1, oV.p, n, ow.p, n, 1, oV.p + (size_t)(j + 1) * n, s);
}

void Hierarchy::outer_dev_tail() {
  const long long n = lv[0].n;
  const int m = p.nkv;
  const DevGmres d = gmo();
  const BArg a = d.arg();
  const FineOpView<double> D = ctx->view<double>();
  gm_solve(d, m, 1, s);
  blincomb<double, float>(a, m, oZ32.p, n, ox.p, n, 1, nullptr, s);
  dslash<double>(D, ox.p, ow.p, s, 1);
  vbmy<double>(ob.p, ow.p, n, s);
  red->bdots<double>(nullptr, ow.p, 0, 0, ow.p, n, 1, s, d.res);
  gm_begin(d, m, 1, p.tol, 2, s);
  bscale<double>(a, ow.p, oV.p, n, 1, s);
}

Hierarchy::BatchGraphs::~BatchGraphs() {
  auto drop = [](BatchGraph& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.g) (void)hipGraphDestroy(b.g);
  };
  for (auto& b : step) drop(b);
  drop(tail);
}

template <typename T, typename Op>
void Hierarchy::gmres_dev(int l, Op op, const C<T>* b, C<T>* x, int m, int cycles, double tol, int nb,
                          int poll) {
  Work<T>& W = work<T>(l);
  const long long n = lv[l].n, vs = (long long)nb * n;
  DD_REQUIRE(m <= W.m && nb <= W.cap, "Krylov basis too short for the batch");
  const DevGmres d = gm();
  const BArg a = d.arg();
  C<T>* V = W.V.p;
  C<T>* w = W.w.p;
  vzero<T>(x, vs, s);
  // the liveness flag, read after the stream has drained
  auto flag_set = [&]() {
    DD_CHECK_HIP(hipStreamSynchronize(s));
    return *static_cast<volatile int*>(gm_flag_host) != 0;
  };
  for (int c = 0; c < cycles; ++c) {
    // r = b (first cycle) or b - A x: its norm starts the cycle
    const C<T>* r0 = b;
    if (c > 0) {
      if (poll > 0 && !flag_set()) break;   // no system needs another cycle
      op(x, w);
      vbmy<T>(b, w, vs, s);
      r0 = w;
    }
    red->bdots<T>(nullptr, r0, 0, 0, const_cast<C<T>*>(r0), n, nb, s, d.res);
    gm_begin(d, m, nb, tol, c == 0, s);
    bscale<T>(a, r0, V, n, nb, s);
    int steps = 0, polls = 0;
    const int first_poll = std::max(poll, pred_steps);
    for (int j = 0; j < m; ++j) {
      op(V + (size_t)j * vs, w);
      red->bdots<T>(nullptr, V, vs, j + 1, w, n, nb, s, d.res);
      gm_cgs1(d, j, nb, s);
      red->bdots<T>(&a, V, vs, j + 1, w, n, nb, s, d.res);
      gm_step(d, j, m, nb, s);
      steps = j + 1;
      if (j + 1 < m) blincomb<T, T>(a, j + 1, V, vs, w, n, nb, V + (size_t)(j + 1) * vs, s);
      if (poll > 0 && j + 1 < m && j + 1 >= first_poll) {
        ++polls;
        if (!flag_set()) break;
      }
    }
    if (poll > 0) {
      // next time the first read comes one step earlier if it already found
      // every system done, else at the step where they were
      pred_steps = polls <= 1 ? std::max(1, steps - 1) : steps;
    }
    gm_solve(d, m, nb, s);
    // only the basis vectors written in this cycle
    blincomb<T, T>(a, steps, V, vs, x, n, nb, nullptr, s);
  }
}

template <typename T> void Hierarchy::coarsest_solve(const C<T>* b, C<T>* z, int nb, int poll) {
  const TraceRange range("ddamg coarsest solve");
  const int c = L - 1;
  const LevelStore& L_ = lv[c];
  Work<T>& W = work<T>(c);
  const long long n = L_.n;
  if (!L_.cg.bipartite) {
    gmres_dev<T>(
        c, [&](const C<T>* a, C<T>* o) { apply<T>(c, a, o, nb); }, b, z, p.coarse_restart,
        p.coarse_max_restarts, p.coarse_eps, nb, poll);
    return;
  }
  const int ne = (int)L_.cg.even.size(), no = (int)L_.cg.odd.size();
  vzero<T>(W.t1.p, n * nb, s);
  site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, L_.n, b, W.t1.p, s, nb);
  vzero<T>(W.t2.p, n * nb, s);
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_odd.p, no, T(1), b, T(0), nullptr, T(-1), W.t1.p, W.t2.p, s, nb);
  });
  gmres_dev<T>(
      c, [&](const C<T>* a, C<T>* o) { schur<T>(a, o, nb); }, W.t2.p, z, p.coarse_restart,
      p.coarse_max_restarts, p.coarse_eps, nb, poll);
  coarse_op<T>(c, [&](const auto& op) {
    coarse_site_apply(op, L_.c_even.p, ne, T(1), b, T(0), nullptr, T(-1), z, W.t1.p, s, nb);
  });
  site_matvec<T>(einv<T>(L_), L_.c_even.p, ne, L_.d, L_.n, W.t1.p, z, s, nb);
}

void Hierarchy::drop_graphs() {
  for (auto& g : graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

// The level-0 cycle captured into a HIP graph.  The first call for a batch
// size (or after buffers were reallocated) runs the cycle eagerly, which
// also grows any scratch it needs, and then captures the same launches;
// later calls replay the graph.  The capture is thread-local, so other
// threads may keep using the device meanwhile.
template <typename T> void Hierarchy::apply_pre_graph(int nb) {
  Work<T>& W0 = work<T>(0);
  const bool f32 = std::is_same<T, float>::value;
  PreGraph* G = nullptr;
  for (auto& g : graphs)
    if (g.nb == nb && g.f32 == f32) G = &g;
  if (G && G->gen == gen && G->exec) {
    DD_CHECK_HIP(hipGraphLaunch(G->exec, s));
    return;
  }
  if (G && G->gen != gen) {
    // buffers changed: every graph is stale
    drop_graphs();
    G = nullptr;
  }
  dev_scalars = true;
  try {
    cycle<T>(0, W0.bin.p, W0.x.p, nb);
    hipGraph_t graph = nullptr;
    DD_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      cycle<T>(0, W0.bin.p, W0.x.p, nb);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      (void)hipGetLastError();
      throw;
    }
    DD_CHECK_HIP(hipStreamEndCapture(s, &graph));
    PreGraph ng;
    ng.nb = nb;
    ng.f32 = f32;
    ng.gen = gen;
    const hipError_t e = hipGraphInstantiate(&ng.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    DD_CHECK_HIP(e);
    graphs.push_back(ng);
  } catch (...) {
    dev_scalars = false;
    throw;
  }
  dev_scalars = false;
}

// ---------------------------------------------------------------------------
// the level-l cycle (Alg. 1; Alg. 2 replaces the recursive call by FGMRES)
// ---------------------------------------------------------------------------
static const char* const CYCLE_RANGE[4] = {"ddamg cycle level 0", "ddamg cycle level 1", "ddamg cycle level 2",
                                            "ddamg cycle level 3"};

template <typename T> void Hierarchy::cycle(int l, const C<T>* b, C<T>* z, int nb) {
  const TraceRange range(CYCLE_RANGE[l]);
  lt_push(l);
  Work<T>& W = work<T>(l);
  Work<T>& Wc = work<T>(l + 1);
  DD_REQUIRE(nb <= W.cap && nb <= Wc.cap, "batch larger than the work buffers");
  const long long n = lv[l].n;
  vzero<T>(z, n * nb, s);
  if (p.mu > 0) {
    sap<T>(l, b, z, p.mu, nb);
    apply<T>(l, z, W.r.p, nb);
    vbmy<T>(b, W.r.p, n * nb, s);
    restrict_to<T>(l, W.r.p, Wc.bin.p, nb);
  } else {
    restrict_to<T>(l, b, Wc.bin.p, nb);
  }
  coarse_correction<T>(l, nb);
  prolong_add<T>(l, Wc.z.p, z, nb);
  if (p.nu > 0) sap<T>(l, b, z, p.nu, nb);
  lt_pop();
}

template <typename T> void Hierarchy::coarse_correction(int l, int nb) {
  Work<T>& Wc = work<T>(l + 1);
  if (l + 1 == L - 1) {
    // under graph capture the fixed launch sequence, else with the host
    // reading the device's liveness flag
    lt_push(l + 1);
    coarsest_solve<T>(Wc.bin.p, Wc.z.p, nb, dev_scalars ? 0 : COARSE_POLL);
    lt_pop();
  } else if (p.cycle == DDAMG_KCYCLE) {
    const int c = l + 1;
    lt_push(c);
    fgmres<T>(
        c, [&](const C<T>* a, C<T>* o) { apply<T>(c, a, o, nb); },
        [&](const C<T>* a, C<T>* o) { cycle<T>(c, a, o, nb); }, true, Wc.bin.p, Wc.z.p, p.kc_len,
        p.kc_restarts, p.kc_tol, nb, kc_it.data());
    lt_pop();
  } else if (p.cycle == DDAMG_WCYCLE) {
    // two cycles on level l+1, the second on the residual of the first
    const long long nc = lv[l + 1].n;
    cycle<T>(l + 1, Wc.bin.p, Wc.z.p, nb);
    lt_push(l + 1);
    apply<T>(l + 1, Wc.z.p, Wc.x.p, nb);
    vbmy<T>(Wc.bin.p, Wc.x.p, nc * nb, s);
    lt_pop();
    cycle<T>(l + 1, Wc.x.p, Wc.w.p, nb);
    vadd<T>(Wc.w.p, Wc.z.p, nc * nb, s);
  } else {
    cycle<T>(l + 1, Wc.bin.p, Wc.z.p, nb);
  }
  if (recording) {
    const long long nc = lv[l + 1].n;
    for (int r = 0; r < nb; ++r)
      if (visit[r]) vcopy<T, T>(Wc.z.p + r * nc, Wc.rec.p + r * nc, nc, s);
  }
}

// ---------------------------------------------------------------------------
// the level-0 cycle on FP16 fine spinors (mu = 0: restriction of b, the
// coarse correction, z = P e, then the post-smoothing SAP sweeps)
// ---------------------------------------------------------------------------
void Hierarchy::ensure_hs(int nb) {
  if (hcap >= nb) return;
  const size_t n0 = (size_t)lv[0].n * nb, v0 = (size_t)lv[0].V * nb;
  h16a.alloc(n0);
  h16b.alloc(n0);
  h16as.alloc(v0);
  h16bs.alloc(v0);
  hcap = nb;
}

void Hierarchy::restrict_hs(const __half2* fine, const float* fsc, C<float>* coarse, int nb) {
  const LevelStore& L_ = lv[0];
  // FP16 P and fine field (plus a scale per site), FP32 coarse field
  meter(L_.N * (double)L_.n * 4.0 + ((double)L_.n * 4.0 + L_.V * 4.0 + 2.0 * L_.N * lv[1].V * 8.0) * nb,
        8.0 * L_.N * (double)L_.n * nb);
  restrict_fine_hs(ctx->g, L_.at, L_.ad(), L_.N, L_.P16.p, fine, fsc, coarse, s, nb);
}

void Hierarchy::prolong_hs(const C<float>* coarse, __half2* fine, float* fsc, int nb) {
  const LevelStore& L_ = lv[0];
  meter(L_.N * (double)L_.n * 4.0 + ((double)L_.n * 4.0 + L_.V * 4.0 + 2.0 * L_.N * lv[1].V * 8.0) * nb,
        8.0 * L_.N * (double)L_.n * nb);
  prolong_fine_hs(ctx->g, L_.at, L_.ad(), L_.N, L_.P16.p, coarse, fine, fsc, s, nb);
}

void Hierarchy::sap_hs(const __half2* b, const float* bs, __half2* z, float* zs, int nsweeps, int nb) {
  // per sweep: b, z in, z out (36 FP16 complex and 3 scales per site and
  // field), FP16 links and clover (72 complex)
  const double V = (double)lv[0].V;
  meter(nsweeps * V * ((36 * 4.0 + 12.0) * nb + 72 * 4.0), nsweeps * (1870.0 + p.mr_iters * 2280.0) * V * nb);
  for (int it = 0; it < nsweeps; ++it)
    for (int col = 0; col < 2; ++col) sap_colour_hs(ctx->view16(), ctx->cblk.p, col, p.mr_iters, b, bs, z, zs, s, nb);
}

void Hierarchy::cycle_hs(const __half2* b, const float* bs, __half2* z, float* zs, int nb) {
  lt_push(0);
  Work<float>& Wc = work<float>(1);
  DD_REQUIRE(nb <= Wc.cap && nb <= hcap, "batch larger than the work buffers");
  restrict_hs(b, bs, Wc.bin.p, nb);
  coarse_correction<float>(0, nb);
  prolong_hs(Wc.z.p, z, zs, nb);
  if (p.nu > 0) sap_hs(b, bs, z, zs, p.nu, nb);
  lt_pop();
}

// ---------------------------------------------------------------------------
// outer FGMRES in FP64 for a batch, right-preconditioned by the level-0
// cycle at T; every system is certified by its true residual, recomputed in
// FP64, and restarted until it meets tol (or max_restarts).
// ---------------------------------------------------------------------------
template <typename T> DevArray<C<T>>& outerZ(Hierarchy& H);
template <> DevArray<C<double>>& outerZ<double>(Hierarchy& H) { return H.oZ64; }
template <> DevArray<C<float>>& outerZ<float>(Hierarchy& H) { return H.oZ32; }

template <typename T> void Hierarchy::outer(const double2* b, double2* x, ddamg_solve_stats* st, int nb) {
  const TraceRange range("ddamg outer FGMRES");
  const long long n = lv[0].n, vs = (long long)nb * n;
  const int m = p.nkv;
  ensure_batch<T>(nb);
  const FineOpView<double> D = ctx->view<double>();
  // the FP64 operator of the outer iteration (residuals and Arnoldi)
  const auto applyD64 = [&](const double2* in, double2* out) {
    meter((double)ctx->g.V * (24 * 16.0 * nb + 72 * 16.0), 1870.0 * ctx->g.V * nb);
    dslash<double>(D, in, out, s, nb);
  };
  double2* V = oV.p;
  C<T>* Z = outerZ<T>(*this).p;
  // FP16 directions with per-site scales (FP16 storage, FP32 cycle)
  const bool zh = std::is_same<T, float>::value && (p.half_directions == 1 || hs);
  gm_reset(gm(), nb, s);
  double2* w = ow.p;
  std::vector<double> bnorm, beta, target(nb), scale(nb);
  bnorms<double>(*red, b, n, nb, bnorm, s);
  std::vector<int> status(nb, DDAMG_ENOCONV);
  std::vector<char> active(nb, 0);
  for (int r = 0; r < nb; ++r) {
    st[r].outer_iters = 0;
    st[r].restarts = 0;
    st[r].true_relres = 0;
    if (!std::isfinite(bnorm[r])) status[r] = DDAMG_ENONFINITE;
    else if (bnorm[r] == 0.0) status[r] = DDAMG_OK;
    target[r] = p.tol * bnorm[r];
  }
  // systems with b_r = 0 have the solution 0
  {
    std::vector<double> keep(nb);
    for (int r = 0; r < nb; ++r) keep[r] = (bnorm[r] == 0.0) ? 0.0 : 1.0;
    bscale_host<double>(*red, keep, x, x, n, nb, s);
  }
  // r = b - D x
  applyD64(x, w);
  vbmy<double>(b, w, vs, s);
  bnorms<double>(*red, w, n, nb, beta, s);
  for (int r = 0; r < nb; ++r) {
    if (status[r] != DDAMG_ENOCONV) continue;
    if (!std::isfinite(beta[r])) status[r] = DDAMG_ENONFINITE;
    else if (beta[r] <= target[r]) status[r] = DDAMG_OK;
    active[r] = status[r] == DDAMG_ENOCONV;
  }
  std::vector<cd> H((size_t)nb * (m + 1) * m), g((size_t)nb * (m + 1)), cs((size_t)nb * m), sn((size_t)nb * m);
  std::vector<cd> h, cf, y(m), cy((size_t)nb * KMAX);
  std::vector<double> hn;
  Work<T>& W0 = work<T>(0);
  for (int restart = 0; restart < p.max_restarts; ++restart) {
    bool any = false;
    for (int r = 0; r < nb; ++r) {
      scale[r] = active[r] ? 1.0 / beta[r] : 0.0;
      any = any || active[r];
    }
    if (!any) break;
    const std::vector<double> beta_start = beta;
    bscale_host<double>(*red, scale, w, V, n, nb, s);
    std::fill(H.begin(), H.end(), cd(0));
    std::fill(g.begin(), g.end(), cd(0));
    for (int r = 0; r < nb; ++r) g[(size_t)r * (m + 1)] = active[r] ? beta[r] : 0.0;
    std::vector<int> jend(nb, 0);
    std::vector<char> live = active;
    // FP16 spinors: the FP16 form of V_j, made by the previous step's update
    bool vj_encoded = false;
    for (int j = 0; j < m; ++j) {
      double2* Vj = V + (size_t)j * vs;
      C<T>* Zj = Z + (size_t)j * vs;
      if (p.graph) {
        vcopy<double, T>(Vj, W0.bin.p, vs, s);
        apply_pre_graph<T>(nb);
        if (zh) {
          encode_sites(ctx->g, reinterpret_cast<const float2*>(W0.x.p), oZ16.p + (size_t)j * vs,
                       oZs.p + (size_t)j * nb * ctx->g.V, ot.p, nb, s);
          applyD64(ot.p, w);
        } else if constexpr (std::is_same<T, double>::value) {
          vcopy<double, double>(W0.x.p, Zj, vs, s);
          applyD64(Zj, w);
        } else {
          vcopy<T, T>(W0.x.p, Zj, vs, s);
          vcopy<T, double>(W0.x.p, ot.p, vs, s);
          applyD64(ot.p, w);
        }
      } else if constexpr (std::is_same<T, double>::value) {
        cycle<double>(0, Vj, Zj, nb);
        applyD64(Zj, w);
      } else if (hs) {
        // FP16 fine spinors: the cycle writes the stored direction itself
        __half2* zj = oZ16.p + (size_t)j * vs;
        float* zjs = oZs.p + (size_t)j * nb * ctx->g.V;
        if (!vj_encoded) encode_h<double>(ctx->g, Vj, h16a.p, h16as.p, nb, s);
        vj_encoded = false;
        cycle_hs(h16a.p, h16as.p, zj, zjs, nb);
        // D in FP64 on exactly the stored FP16 direction
        // (FP16 spinor and its scale in, FP64 spinor out, FP64 links and clover)
        meter((double)ctx->g.V * ((52.0 + 192.0) * nb + 72 * 16.0), 1870.0 * ctx->g.V * nb);
        dslash_hs(D, zj, zjs, w, s, nb);
      } else if (zh) {
        vcopy<double, T>(Vj, W0.bin.p, vs, s);
        cycle<T>(0, W0.bin.p, W0.x.p, nb);
        // the stored direction is the FP16 one: D is applied to its decoded value
        encode_sites(ctx->g, reinterpret_cast<const float2*>(W0.x.p), oZ16.p + (size_t)j * vs,
                     oZs.p + (size_t)j * nb * ctx->g.V, ot.p, nb, s);
        applyD64(ot.p, w);
      } else {
        vcopy<double, T>(Vj, W0.bin.p, vs, s);
        cycle<T>(0, W0.bin.p, Zj, nb);
        vcopy<T, double>(Zj, ot.p, vs, s);
        applyD64(ot.p, w);
      }
      arnoldi<double>(V, vs, n, nb, j, w, live, h, hn, cf);
      bool still = false;
      for (int r = 0; r < nb; ++r) {
        if (!live[r]) continue;
        const double est = givens_column(&H[(size_t)r * (m + 1) * m], &g[(size_t)r * (m + 1)], &cs[(size_t)r * m],
                                         &sn[(size_t)r * m], m, j, &h[(size_t)r * (KMAX + 1)], hn[r]);
        ++st[r].outer_iters;
        jend[r] = j + 1;
        if (!std::isfinite(est)) {
          status[r] = DDAMG_ENONFINITE;
          live[r] = 0;
          active[r] = 0;
          jend[r] = 0;
        } else if (est <= target[r] || hn[r] == 0.0) {
          live[r] = 0;
        }
        still = still || live[r];
      }
      if (!still) break;
      if (j + 1 < m) {
        for (int r = 0; r < nb; ++r) scale[r] = live[r] ? 1.0 / hn[r] : 0.0;
        const BArg a = red->upload(cf, scale, nb, s);
        if (hs && !p.graph && !std::is_same<T, double>::value) {
          // the next basis vector and its FP16 form for the next cycle
          blincomb_encode(a, j + 1, V, vs, w, V + (size_t)(j + 1) * vs, h16a.p, h16as.p, ctx->g.nblk, nb, s);
          vj_encoded = true;
        } else {
          blincomb<double, double>(a, j + 1, V, vs, w, n, nb, V + (size_t)(j + 1) * vs, s);
        }
      }
    }
    int kmax = 0;
    std::fill(cy.begin(), cy.end(), cd(0));
    for (int r = 0; r < nb; ++r) {
      if (!active[r] || jend[r] == 0) continue;
      back_substitute(&H[(size_t)r * (m + 1) * m], &g[(size_t)r * (m + 1)], m, jend[r], y.data());
      for (int i = 0; i < jend[r]; ++i) cy[(size_t)r * KMAX + i] = y[i];
      kmax = std::max(kmax, jend[r]);
      ++st[r].restarts;
    }
    if (kmax > 0) {
      const BArg a = red->upload(cy, std::vector<double>(), nb, s);
      if (zh) blincomb_sites(a, kmax, oZ16.p, oZs.p, x, ctx->g.nblk, nb, s);
      else blincomb<double, T>(a, kmax, Z, vs, x, n, nb, nullptr, s);
    }
    // true residuals in FP64
    applyD64(x, w);
    vbmy<double>(b, w, vs, s);
    bnorms<double>(*red, w, n, nb, beta, s);
    for (int r = 0; r < nb; ++r) {
      if (!active[r]) continue;
      if (!std::isfinite(beta[r])) {
        status[r] = DDAMG_ENONFINITE;
        active[r] = 0;
      } else if (beta[r] <= target[r]) {
        status[r] = DDAMG_OK;
        active[r] = 0;
      } else if (beta[r] > OUTER_STAGNATION * beta_start[r]) {
        // a whole restart cycle left the recomputed residual where it was
        // (a tolerance below what the arithmetic reaches, or a useless
        // preconditioner): more cycles would not change it
        status[r] = DDAMG_ENOCONV;
        active[r] = 0;
      }
    }
  }
  for (int r = 0; r < nb; ++r) {
    st[r].status = status[r];
    st[r].true_relres = bnorm[r] > 0 ? beta[r] / bnorm[r] : 0.0;
  }
  {
    std::vector<long long> it(nb);
    DD_CHECK_HIP(hipMemcpyAsync(it.data(), gm_iters.p, sizeof(long long) * nb, hipMemcpyDeviceToHost, s));
    DD_CHECK_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nb; ++r) cs_it[r] += it[r];
  }
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
template <typename T> std::vector<Work<T>>& work_vec(Hierarchy& H);
template <> std::vector<Work<double>>& work_vec<double>(Hierarchy& H) { return H.w64; }
template <> std::vector<Work<float>>& work_vec<float>(Hierarchy& H) { return H.w32; }

template <typename T> void Hierarchy::alloc_work(int cap) {
  ++gen;
  std::vector<Work<T>>& W = work_vec<T>(*this);
  W.clear();
  W.resize(L);
  for (int l = 0; l < L; ++l) {
    const size_t n = (size_t)lv[l].n * cap;
    Work<T>& w = W[l];
    w.cap = cap;
    w.bin.alloc(n);
    w.rec.alloc(n);
    if (l == 0) {
      w.x.alloc(n);
      if (p.mu > 0) w.r.alloc(n);
      continue;
    }
    w.z.alloc(n);
    w.r.alloc(n);
    w.x.alloc(n);
    w.w.alloc(n);
    if (l == L - 1) {
      w.t1.alloc(n);
      w.t2.alloc(n);
      w.t3.alloc(n);
      w.t4.alloc(n);
      w.m = p.coarse_restart;
      w.V.alloc((size_t)(w.m + 1) * n);
    } else {
      w.m = p.kc_len;
      w.V.alloc((size_t)(w.m + 1) * n);
      w.Z.alloc((size_t)w.m * n);
    }
  }
}

// work buffers at precision T for a batch of nb
template <typename T> void Hierarchy::ensure_work(int nb) {
  DD_REQUIRE(nb >= 1 && nb <= NBMAX, "batch size out of range");
  if (work_vec<T>(*this).empty() || work_vec<T>(*this)[0].cap < nb) alloc_work<T>(nb);
  if ((int)kc_it.size() < nb) kc_it.resize(nb, 0);
  if ((int)cs_it.size() < nb) cs_it.resize(nb, 0);
}

// work buffers and outer-solver buffers for a batch of nb
template <typename T> void Hierarchy::ensure_batch(int nb) {
  ensure_work<T>(nb);
  if (ocap >= nb) return;
  const size_t n0 = (size_t)lv[0].n * nb;
  oV.alloc((size_t)(p.nkv + 1) * n0);
  ow.alloc(n0);
  ob.alloc(n0);
  ox.alloc(n0);
  if (std::is_same<T, float>::value) {
    // FP16 preconditioned directions with one FP32 scale per site
    if (hs) ensure_hs(nb);
    if (p.half_directions == 1 || hs) {
      oZ16.alloc((size_t)p.nkv * n0);
      oZs.alloc((size_t)p.nkv * nb * ctx->g.V);
    } else {
      oZ32.alloc((size_t)p.nkv * n0);
    }
    ot.alloc(n0);
  } else {
    oZ64.alloc((size_t)p.nkv * n0);
  }
  ocap = nb;
}

void Hierarchy::build_level(int l, bool from32) {
  const TraceRange range("ddamg P and Galerkin operator");
  ++gen;
  LevelStore& F = lv[l];
  LevelStore& Cc = lv[l + 1];
  const long long n = F.n;
  const int N = F.N;
  // the FP64 test vectors (for an FP32 setup: their FP64 copy) feed the
  // orthonormalisation, which writes P in FP64
  if (from32) vcopy<float, double>(F.tv32.p, F.tv64.p, (long long)N * n, s);
  if (!setup_flags.p) setup_flags.alloc(2);
  DD_CHECK_HIP(hipMemsetAsync(setup_flags.p, 0, 2 * sizeof(int), s));
  if (l == 0) orthonormalise_fine(ctx->g, F.at, F.ad(), N, F.tv64.p, F.P64.p, setup_flags.p, s);
  else orthonormalise_coarse(F.at, F.ad(), F.d, N, F.V, F.tv64.p, F.P64.p, setup_flags.p, s);
  if (F.P32.p) vcopy<double, float>(F.P64.p, F.P32.p, (long long)N * n, s);
  if (F.P16.p) to_half(F.P64.p, F.P16.p, (long long)N * n, s);
  // Galerkin in FP64
  if (l == 0) galerkin_fine(ctx->g, F.at, F.ad(), N, ctx->view<double>(), F.P64.p, Cc.D64.p, s);
  else galerkin_coarse(F.cg, F.at, F.ad(), N, F.cview<double>(), F.P64.p, Cc.D64.p, s, p.galerkin_cols);
  expand_coarse<double2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K64.p, s);
  if (Cc.K32.p) expand_coarse<float2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K32.p, s);
  if (Cc.K16.p) expand_coarse<__half2>(Cc.D64.p, Cc.c_nbr9.p, (int)Cc.V, Cc.d, Cc.K16.p, s);
  if (l + 1 == L - 1 && Cc.cg.bipartite) {
    const int ne = (int)Cc.cg.even.size();
    self_block_inverse(Cc.D64.p, Cc.c_even.p, ne, Cc.d, Cc.Einv64.p, setup_flags.p + 1, s);
    if (Cc.Einv32.p) vcopy<double, float>(Cc.Einv64.p, Cc.Einv32.p, (long long)ne * Cc.d * Cc.d, s);
    if (Cc.sm > 0) build_dense_schur(l + 1);
  }
  int fl[2] = {0, 0};
  DD_CHECK_HIP(hipMemcpyAsync(fl, setup_flags.p, sizeof(fl), hipMemcpyDeviceToHost, s));
  DD_CHECK_HIP(hipStreamSynchronize(s));
  DD_REQUIRE(!fl[0], "the test vectors of level " + std::to_string(l) +
                         " are linearly dependent on an aggregate to within rounding (Gram ratio below 1e-12): "
                         "P cannot be orthonormalised accurately");
  DD_REQUIRE(!fl[1], "an even-site self block of the coarsest level is singular or not finite");
}

void Hierarchy::build_dense_schur(int c) {
  LevelStore& C_ = lv[c];
  const int m = C_.sm, ne = (int)C_.cg.even.size(), no = (int)C_.cg.odd.size(), d = C_.d;
  const long long n = C_.n;
  constexpr int chunk = NBMAX;
  // temporaries: kept with a workspace (reserved up front), freed otherwise
  DevArray<double2> &e = ds_e, &t3 = ds_t3, &t4 = ds_t4, &o = ds_o;
  const size_t need = (size_t)n * chunk;
  if (e.n < need) {
    e.alloc(need);
    t3.alloc(need);
    t4.alloc(need);
    o.alloc(need);
  }
  const CoarseOpView<double> op = C_.cview<double>();
  for (int j0 = 0; j0 < m; j0 += chunk) {
    const int nbc = std::min(chunk, m - j0);
    schur_unit_cols(e.p, n, nbc, C_.s_oidx.p, j0, s);
    // the sparse product of schur(): D_eo, D_ee^-1, then D_oo - D_oe
    coarse_site_apply(op, C_.c_even.p, ne, 0.0, nullptr, 0.0, nullptr, 1.0, e.p, t3.p, s, nbc);
    site_matvec<double>(C_.Einv64.p, C_.c_even.p, ne, d, n, t3.p, t4.p, s, nbc);
    coarse_site_apply(op, C_.c_odd.p, no, 0.0, nullptr, 1.0, e.p, -1.0, t4.p, o.p, s, nbc);
    schur_gather_cols(o.p, n, nbc, C_.s_oidx.p, m, j0, C_.S64.p, s);
  }
  vcopy<double, float>(C_.S64.p, C_.S32.p, (long long)m * m, s);
  if (!ws) {
    // freeing them waits for the stream to drain
    DD_CHECK_HIP(hipStreamSynchronize(s));
    e.release(), t3.release(), t4.release(), o.release();
  }
}

// The N test vectors of a level form a batch: Alg. 3 smooths each of them
// on its own and Alg. 4 cycles each with the hierarchy fixed until all are
// done, so the N updates are independent and run together (in chunks of
// the work capacity).
template <typename T> void Hierarchy::initial_setup(int l) {
  const TraceRange range("ddamg initial setup (Alg. 3)");
  LevelStore& F = lv[l];
  const long long n = F.n;
  const int N = F.N;
  Work<T>& W = work<T>(l);
  if (l > 0) {
    const int Np = lv[l - 1].N;
    const int nr = std::min(N, Np);
    for (int j0 = 0; j0 < nr; j0 += W.cap)
      restrict_to<T>(l - 1, tv<T>(l - 1) + (size_t)j0 * lv[l - 1].n, tv<T>(l) + (size_t)j0 * n,
                     std::min(W.cap, nr - j0));
    if (N > Np) {
      DD_REQUIRE(tv_extra != nullptr, "extra test vectors needed for a level with more test vectors");
      long long off = 0;
      for (int k = 1; k < l; ++k)
        if (lv[k].N > lv[k - 1].N) off += (long long)(lv[k].N - lv[k - 1].N) * lv[k].n;
      vcopy<double, T>(tv_extra + off, tv<T>(l) + (size_t)Np * n, (long long)(N - Np) * n, s);
    }
  }
  for (int eta = 1; eta <= 3; ++eta)
    for (int j0 = 0; j0 < N; j0 += W.cap) {
      const int nb = std::min(W.cap, N - j0);
      C<T>* v = tv<T>(l) + (size_t)j0 * n;
      vzero<T>(W.x.p, n * nb, s);
      sap<T>(l, v, W.x.p, eta, nb);
      vcopy<T, T>(W.x.p, v, n * nb, s);
    }
  build_level(l, std::is_same<T, float>::value);
  if (l < L - 2) initial_setup<T>(l + 1);
}

template <typename T> void Hierarchy::iterative_setup(int l, int i) {
  const TraceRange range("ddamg iterative setup (Alg. 4)");
  if (l >= L - 1) return;
  const int N = lv[l].N;
  const int cap = work<T>(l).cap;
  for (int j0 = 0; j0 < N; j0 += cap) {
    const int nb = std::min(cap, N - j0);
    recording = true;
    visit.assign(nb, 1);
    cycle<T>(l, tv<T>(l) + (size_t)j0 * lv[l].n, work<T>(l).rec.p, nb);
    recording = false;
    visit.clear();
    for (int k = l; k < L - 1; ++k) {
      // test vectors j0 .. j0+cnt-1 of level k are replaced
      const int cnt = std::min(nb, lv[k].N - j0);
      if (cnt <= 0) continue;
      const long long nk = lv[k].n;
      C<T>* src = work<T>(k).rec.p;
      std::vector<double> nrm;
      bnorms<T>(*red, src, nk, cnt, nrm, s);
      std::vector<double> scale(cnt);
      for (int r = 0; r < cnt; ++r) {
        DD_REQUIRE(nrm[r] > 0 && std::isfinite(nrm[r]), "setup produced a zero or non-finite test vector");
        scale[r] = 1.0 / nrm[r];
      }
      bscale_host<T>(*red, scale, src, tv<T>(k) + (size_t)j0 * nk, nk, cnt, s);
    }
  }
  for (int k = l; k < L - 1; ++k) build_level(k, std::is_same<T, float>::value);
  for (int q = 1; q <= i; ++q) iterative_setup<T>(l + 1, q);
}

// With DDAMG_VERBOSE set in the environment the setup reports each phase on
// stderr as it completes (long setups on large lattices).
static bool verbose() {
  static const bool v = std::getenv("DDAMG_VERBOSE") != nullptr;
  return v;
}

template <typename T> void Hierarchy::setup(const double2* tvc) {
  const auto t0 = std::chrono::steady_clock::now();
  auto report = [&](const char* what, int i) {
    if (!verbose()) return;
    DD_CHECK_HIP(hipStreamSynchronize(s));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[ddamg] setup: %s %d done at %.2f s\n", what, i, sec);
    std::fflush(stderr);
  };
  fine_to_native<T>(ctx->g, tvc, tv<T>(0), lv[0].N, s);
  initial_setup<T>(0);
  report("initial phase, levels", L);
  for (int i = 1; i <= p.n_inv; ++i) {
    iterative_setup<T>(0, i);
    report("iterative phase, iteration", i);
  }
  DD_CHECK_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// SAP block shape of level l: the per-level row where it is set, else sap_block
void sap_block_of(const ddamg_params& p, int l, int out[4]) {
  bool own = l >= 1 && l <= 3;
  for (int mu = 0; own && mu < 4; ++mu) own = p.sap_block_l[l - 1][mu] > 0;
  for (int mu = 0; mu < 4; ++mu) out[mu] = own ? p.sap_block_l[l - 1][mu] : p.sap_block[mu];
}

void validate_params(const Context& ctx, const ddamg_params& p) {
  DD_REQUIRE(p.levels >= 2 && p.levels <= 4, "levels must be 2..4");
  DD_REQUIRE(p.precond_prec == DDAMG_F32 || p.precond_prec == DDAMG_F64, "bad precond_prec");
  DD_REQUIRE(p.cycle == DDAMG_KCYCLE || p.cycle == DDAMG_VCYCLE || p.cycle == DDAMG_WCYCLE, "bad cycle");
  DD_REQUIRE(p.half_storage == 0 || p.half_storage == 1, "half_storage must be 0 or 1");
  DD_REQUIRE(p.half_storage == 0 || p.precond_prec == DDAMG_F32,
             "FP16 operator storage needs the FP32 preconditioner");
  DD_REQUIRE(p.half_directions == 0 || p.half_directions == 1, "half_directions must be 0 or 1");
  DD_REQUIRE(p.half_directions == 0 || p.precond_prec == DDAMG_F32,
             "FP16 directions need the FP32 preconditioner");
  DD_REQUIRE(p.graph == 0 || p.graph == 1, "graph must be 0 or 1");
  DD_REQUIRE(p.coarse_dense == 0 || p.coarse_dense == 1, "coarse_dense must be 0 or 1");
  DD_REQUIRE(p.galerkin_cols == 0 || p.galerkin_cols == 1 || p.galerkin_cols == 4,
             "galerkin_cols must be 0, 1 or 4");
  DD_REQUIRE(p.profile_levels == 0 || p.profile_levels == 1, "profile_levels must be 0 or 1");
  DD_REQUIRE(p.half_spinors == 0 || p.half_spinors == 1, "half_spinors must be 0 or 1");
  DD_REQUIRE(p.half_spinors == 0 || (p.precond_prec == DDAMG_F32 && p.half_storage == 1),
             "FP16 spinors need the FP32 preconditioner with FP16 operator storage (half_storage = 1)");
  DD_REQUIRE(p.half_spinors == 0 || (p.mu == 0 && p.graph == 0),
             "FP16 spinors need mu = 0 and graph = 0");
  DD_REQUIRE(p.graph == 0 || p.levels == 2 || p.cycle != DDAMG_KCYCLE,
             "a graph-captured preconditioner needs the V- or W-cycle (levels >= 3)");
  DD_REQUIRE(p.mu >= 0 && p.nu >= 0 && p.mr_iters >= 0 && p.n_inv >= 0, "negative iteration count");
  DD_REQUIRE(p.nkv >= 1 && p.nkv <= KMAX - 1, "nkv out of range");
  DD_REQUIRE(p.kc_len >= 1 && p.kc_len <= KMAX - 1 && p.kc_restarts >= 1, "bad K-cycle length");
  DD_REQUIRE(p.coarse_restart >= 1 && p.coarse_restart <= KMAX - 1 && p.coarse_max_restarts >= 1,
             "bad coarsest GMRES restart");
  DD_REQUIRE(p.tol > 0 && p.kc_tol > 0 && p.coarse_eps > 0, "tolerances must be positive");
  DD_REQUIRE(p.max_restarts >= 1, "max_restarts must be >= 1");
  DD_REQUIRE(p.batch >= 1 && p.batch <= NBMAX, "batch must be 1..32");
  int dims[4] = {ctx.g.dims[0], ctx.g.dims[1], ctx.g.dims[2], ctx.g.dims[3]};
  for (int mu = 0; mu < 4; ++mu)
    DD_REQUIRE(p.sap_block[mu] >= 1, "bad SAP block");
  for (int l = 0; l < 3; ++l)
    for (int mu = 0; mu < 4; ++mu) DD_REQUIRE(p.sap_block_l[l][mu] >= 0, "bad per-level SAP block");
  int d = 12;
  for (int l = 0; l < p.levels - 1; ++l) {
    // SAP validity on level l
    int blk[4];
    sap_block_of(p, l, blk);
    for (int mu = 0; mu < 4; ++mu) {
      if (l == 0) DD_REQUIRE(blk[mu] == 2, "the fine SAP blocks are 2^4");
      DD_REQUIRE(dims[mu] % blk[mu] == 0 && (dims[mu] / blk[mu]) % 2 == 0,
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
    DD_REQUIRE(p.ntv[l] >= 1 && p.ntv[l] <= 32, "ntv must be 1..32");
    DD_REQUIRE(p.ntv[l] <= asz * d / 2, "more test vectors than an aggregate's dimension");
    for (int mu = 0; mu < 4; ++mu) dims[mu] /= p.agg[l][mu];
    d = 2 * p.ntv[l];
  }
  DD_REQUIRE(d <= 64, "coarsest dof per site must be <= 64");
}

void Hierarchy::set_sap_block(int l, const int blk[4]) {
  DD_REQUIRE(l >= 1 && l <= L - 2, "only the coarse levels 1..L-2 are smoothed by SAP");
  ddamg_params q = p;
  for (int mu = 0; mu < 4; ++mu) q.sap_block_l[l - 1][mu] = blk[mu];
  validate_params(*ctx, q);
  LevelStore& S = lv[l];
  int sap[4];
  sap_block_of(q, l, sap);
  CoarseGeom g = make_coarse_geom(S.dims, S.d, sap);
  S.cg.sap[0] = g.sap[0], S.cg.sap[1] = g.sap[1], S.cg.sap[2] = g.sap[2], S.cg.sap[3] = g.sap[3];
  S.cg.nblk = g.nblk;
  S.cg.bs = g.bs;
  S.cg.blk_sites = std::move(g.blk_sites);
  S.cg.site_blk = std::move(g.site_blk);
  S.cg.site_pos = std::move(g.site_pos);
  S.cg.inmask = std::move(g.inmask);
  S.cg.kmax = g.kmax;
  S.c_blk_sites.upload(S.cg.blk_sites, s);
  S.c_site_blk.upload(S.cg.site_blk, s);
  S.c_site_pos.upload(S.cg.site_pos, s);
  S.c_inmask.upload(S.cg.inmask, s);
  DD_CHECK_HIP(hipStreamSynchronize(s));
  p = q;
  ++gen;
}

void Hierarchy::layout() {
  lv.resize(L);
  int dims[4];
  for (int mu = 0; mu < 4; ++mu) dims[mu] = ctx->g.dims[mu];
  int d = 12;
  for (int l = 0; l < L; ++l) {
    LevelStore& S = lv[l];
    S.fine = l == 0;
    for (int mu = 0; mu < 4; ++mu) S.dims[mu] = dims[mu];
    S.d = d;
    S.V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    S.n = S.V * d;
    if (l > 0) {
      int sap[4] = {0, 0, 0, 0};
      if (l < L - 1) sap_block_of(p, l, sap);
      S.cg = make_coarse_geom(dims, d, sap);
      S.c_nbr9.upload(S.cg.nbr9, s);
      S.c_blk_sites.upload(S.cg.blk_sites, s);
      S.c_site_blk.upload(S.cg.site_blk, s);
      S.c_site_pos.upload(S.cg.site_pos, s);
      S.c_inmask.upload(S.cg.inmask, s);
      S.c_even.upload(S.cg.even, s);
      S.c_odd.upload(S.cg.odd, s);
      S.D64.alloc((size_t)S.V * 5 * d * d);
      S.K64.alloc((size_t)S.V * 9 * d * d);
      if (!half) S.K32.alloc((size_t)S.V * 9 * d * d);
      if (half) S.K16.alloc((size_t)S.V * 9 * d * d);
      if (l == L - 1 && S.cg.bipartite) {
        S.Einv64.alloc(S.cg.even.size() * (size_t)d * d);
        S.Einv32.alloc(S.cg.even.size() * (size_t)d * d);
        // a dense Schur complement where it is small: at most DENSE_SCHUR_MAX
        // unknowns and at most twice the entries of the sparse blocks
        const long long m = (long long)S.cg.odd.size() * d, sparse = S.V * 9LL * d * d;
        if (p.coarse_dense && S.cg.odd.size() == S.cg.even.size() && m <= DENSE_SCHUR_MAX && m * m <= 2 * sparse) {
          S.sm = (int)m;
          S.s_oidx_h.resize(m);
          S.s_eidx_h.resize(m);
          for (size_t k = 0; k < S.cg.odd.size(); ++k)
            for (int a = 0; a < d; ++a) {
              S.s_oidx_h[k * d + a] = S.cg.odd[k] * d + a;
              S.s_eidx_h[k * d + a] = S.cg.even[k] * d + a;
            }
          S.s_oidx.upload(S.s_oidx_h, s);
          S.s_eidx.upload(S.s_eidx_h, s);
          S.S64.alloc((size_t)m * m);
          S.S32.alloc((size_t)m * m);
        }
      }
    }
    if (l < L - 1) {
      S.N = p.ntv[l];
      S.at = l == 0 ? make_fine_agg(ctx->g, p.agg[l]) : make_coarse_agg(S.cg, p.agg[l]);
      S.a_members.upload(S.at.members, s);
      S.a_member_agg.upload(S.at.member_agg, s);
      S.P64.alloc((size_t)S.N * S.n);
      if (!half) S.P32.alloc((size_t)S.N * S.n);
      if (half) S.P16.alloc((size_t)S.N * S.n);
      S.tv64.alloc((size_t)S.N * S.n);
      if (p.precond_prec == DDAMG_F32) S.tv32.alloc((size_t)S.N * S.n);
      for (int mu = 0; mu < 4; ++mu) dims[mu] = S.at.cdims[mu];
      d = 2 * S.N;
    }
  }
  red.reset(new Reducer);
}

// the batch the setup runs its test vectors in: at most `batch` at once
static int setup_batch(const ddamg_params& p) {
  int cap = 1;
  for (int l = 0; l < p.levels - 1; ++l) cap = std::max(cap, p.ntv[l]);
  return std::min(cap, p.batch);
}

void Hierarchy::reserve(int nrhs) {
  nrhs_max = nrhs;
  const int solve = std::min(nrhs, p.batch), cap = std::max(setup_batch(p), solve);
  auto at = [&](auto zero) {
    using T = decltype(zero);
    ensure_work<T>(cap);
    ensure_batch<T>(solve);
    for (int l = 1; l <= L - 2; ++l) sap_scratch<T>(lv[l], cap);
  };
  if (p.precond_prec == DDAMG_F32) at(0.f);
  else at(0.0);
  gm();
  // the outer solver's device records of the batch graph solve
  if (p.graph == 1) gmo();
  setup_flags.alloc(2);
  // canonical-layout level calls and the preconditioner call: two fields of
  // the finest level per right-hand side at the hierarchy's precision
  const size_t c2 = p.precond_prec == DDAMG_F32 ? 2 : 1;
  sc64a.alloc(((size_t)lv[0].n * nrhs + c2 - 1) / c2);
  sc64b.alloc(((size_t)lv[0].n * nrhs + c2 - 1) / c2);
  const LevelStore& Lc = lv[L - 1];
  if (Lc.sm > 0) {
    const size_t nc = (size_t)Lc.n * NBMAX;
    ds_e.alloc(nc);
    ds_t3.alloc(nc);
    ds_t4.alloc(nc);
    ds_o.alloc(nc);
  }
}

Hierarchy* create_hierarchy(Context* ctx, const ddamg_params* pp, const double2* tvc,
                            const double2* tv_extra, hipStream_t s, std::unique_ptr<Workspace> ws,
                            int nrhs_max) {
  DD_REQUIRE(ctx && pp && tvc, "null argument");
  validate_params(*ctx, *pp);
  static std::atomic<long long> next_uid{1};
  std::unique_ptr<Hierarchy> H(new Hierarchy);
  H->uid = next_uid++;
  H->ws = std::move(ws);
  H->ctx = ctx;
  H->p = *pp;
  H->L = pp->levels;
  H->s = s;
  H->tv_extra = tv_extra;
  H->half = pp->half_storage == 1;
  H->hs = pp->half_spinors == 1;
  if (H->half) ctx->make_half(s);
  const WorkspaceScope scope(H->ws.get());
  H->layout();
  if (H->ws) H->reserve(nrhs_max);
  const int cap = setup_batch(H->p);
  const auto t0 = std::chrono::steady_clock::now();
  if (H->p.precond_prec == DDAMG_F32) {
    H->ensure_work<float>(cap);
    H->setup<float>(tvc);
  } else {
    H->ensure_work<double>(cap);
    H->setup<double>(tvc);
  }
  DD_CHECK_HIP(hipStreamSynchronize(s));
  H->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  H->tv_extra = nullptr;
  return H.release();
}

void workspace_bytes(const ddamg_lattice* lat, const ddamg_params* pp, int nrhs_max, size_t* ctx_bytes,
                     size_t* hier_bytes) {
  check_lattice(lat);
  DD_REQUIRE(nrhs_max >= 1 && nrhs_max <= 1 << 20, "nrhs_max must be >= 1");
  const bool half = pp && pp->half_storage == 1;
  // the counters outlive the arrays that report back to them
  Workspace count_ctx, count;
  Context c;
  {
    const WorkspaceScope scope(&count_ctx);
    context_layout(c, lat, half, nrhs_max, nullptr);
    if (ctx_bytes) *ctx_bytes = count_ctx.peak();
  }
  if (!hier_bytes) return;
  *hier_bytes = 0;
  if (!pp) return;
  validate_params(c, *pp);
  {
    const WorkspaceScope scope(&count);
    Hierarchy H;
    H.ctx = &c;
    H.p = *pp;
    H.L = pp->levels;
    H.half = half;
    H.hs = pp->half_spinors == 1;
    H.layout();
    H.reserve(nrhs_max);
  }
  *hier_bytes = count.peak();
}

// explicit instantiations used by the C ABI
template void bnorms<double>(Reducer&, const C<double>*, long long, int, std::vector<double>&, hipStream_t);
template void Hierarchy::apply<double>(int, const C<double>*, C<double>*, int);
template void Hierarchy::apply<float>(int, const C<float>*, C<float>*, int);
template void Hierarchy::sap<double>(int, const C<double>*, C<double>*, int, int);
template void Hierarchy::sap<float>(int, const C<float>*, C<float>*, int, int);
template void Hierarchy::restrict_to<double>(int, const C<double>*, C<double>*, int);
template void Hierarchy::restrict_to<float>(int, const C<float>*, C<float>*, int);
template void Hierarchy::prolong_add<double>(int, const C<double>*, C<double>*, int);
template void Hierarchy::prolong_add<float>(int, const C<float>*, C<float>*, int);
template void Hierarchy::cycle<double>(int, const C<double>*, C<double>*, int);
template void Hierarchy::cycle<float>(int, const C<float>*, C<float>*, int);
template void Hierarchy::outer<double>(const double2*, double2*, ddamg_solve_stats*, int);
template void Hierarchy::outer<float>(const double2*, double2*, ddamg_solve_stats*, int);
template void Hierarchy::ensure_batch<double>(int);
template void Hierarchy::ensure_batch<float>(int);
template void Hierarchy::ensure_work<double>(int);
template void Hierarchy::ensure_work<float>(int);
template void Hierarchy::setup<double>(const double2*);
template void Hierarchy::setup<float>(const double2*);
template void Hierarchy::alloc_work<double>(int);
template void Hierarchy::alloc_work<float>(int);

}  // namespace ddamg
