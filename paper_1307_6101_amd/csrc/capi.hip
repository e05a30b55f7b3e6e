// extern "C" entry points declared in include/ddamg.h.  Each checks its
// arguments on the host, converts canonical <-> native layouts where asked,
// and calls into the hierarchy / kernels on the caller's stream.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "cgnr.h"
#include "handles.h"
#include "solver.h"
#include "tune.h"

using namespace ddamg;

namespace {
thread_local std::string g_err;
}  // namespace

int ddamg::guarded_call(void (*f)(void*), void* arg) {
  try {
    f(arg);
    g_err.clear();
    return DDAMG_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_err = e.what();
    return DDAMG_EHIP;
  } catch (...) {
    g_err = "unknown failure";
    return DDAMG_EHIP;
  }
}

namespace {

void check_prec(int prec, bool f16s = false) {
  DD_REQUIRE(prec == DDAMG_F64 || prec == DDAMG_F32 || prec == DDAMG_F16 || (f16s && prec == DDAMG_F16S),
             f16s ? "prec must be DDAMG_F64, DDAMG_F32, DDAMG_F16 or DDAMG_F16S"
                  : "prec must be DDAMG_F64, DDAMG_F32 or DDAMG_F16");
}
// DDAMG_F16S: level 0 of a hierarchy with FP16 spinors; the native layout
// where the call reads and writes only FP16 fine fields
void check_f16s(const Hierarchy& H, int prec, int level, int layout, bool native_ok) {
  if (prec != DDAMG_F16S) return;
  DD_REQUIRE(H.hs, "DDAMG_F16S needs a hierarchy built with half_spinors = 1");
  DD_REQUIRE(level == 0, "DDAMG_F16S applies to level 0");
  DD_REQUIRE(native_ok || layout == DDAMG_CANONICAL, "this DDAMG_F16S call takes the canonical layout");
}
// DDAMG_F16 on a hierarchy: its FP32 level operations read the FP16 copies
// of the operator data, which exist when it was built with half_storage
void check_half(const Hierarchy& H, int prec) {
  DD_REQUIRE(prec != DDAMG_F16 || H.half, "DDAMG_F16 needs a hierarchy built with half_storage = 1");
}
void check_layout(int layout) {
  DD_REQUIRE(layout == DDAMG_CANONICAL || layout == DDAMG_NATIVE, "layout must be DDAMG_CANONICAL or DDAMG_NATIVE");
}

// scratch for canonical-layout calls: n complex numbers of precision T in a
// raw array of FP64 elements that both precisions share
// (grown by allocating the new array first, so that a failed growth leaves
// the old one in place)
template <typename T> C<T>* scratch(DevArray<double2>& a, size_t n) {
  const size_t need = (n * sizeof(C<T>) + sizeof(double2) - 1) / sizeof(double2);
  if (a.n < need) {
    DevArray<double2> t;
    t.alloc(need);
    a = std::move(t);
  }
  return reinterpret_cast<C<T>*>(a.p);
}
template <typename T> C<T>* ctx_scratch(Context& c, int w, size_t n) { return scratch<T>(w ? c.s64b : c.s64a, n); }
template <typename T> C<T>* hier_scratch(Hierarchy& h, int w, size_t n) { return scratch<T>(w ? h.sc64b : h.sc64a, n); }

// canonical complex128 <-> native at T for nrhs level-l fields (n complex each)
template <typename T>
void to_nat(Context& c, int l, long long n, int nrhs, const double2* in, C<T>* out, hipStream_t s) {
  if (l == 0) fine_to_native<T>(c.g, in, out, nrhs, s);
  else vcopy<double, T>(in, out, n * nrhs, s);
}
template <typename T>
void from_nat(Context& c, int l, long long n, int nrhs, const C<T>* in, double2* out, hipStream_t s) {
  if (l == 0) fine_from_native<T>(c.g, in, out, nrhs, s);
  else vcopy<T, double>(in, out, n * nrhs, s);
}

// Every entry point hands the whole batch of nrhs fields to one batched
// call; with the canonical layout the batch is converted through scratch
// fields first.
template <typename T, bool HALF = false>
void apply_D_impl(Context& c, const void* in, void* out, int nrhs, int layout, hipStream_t s) {
  const long long n = c.g.V * 12;
  const auto op = [&] {
    if constexpr (HALF) {
      c.make_half(s);
      return c.view16();
    } else {
      return c.view<T>();
    }
  }();
  if (layout == DDAMG_NATIVE) {
    dslash<T>(op, static_cast<const C<T>*>(in), static_cast<C<T>*>(out), s, nrhs);
  } else {
    C<T>* a = ctx_scratch<T>(c, 0, n * nrhs);
    C<T>* b = ctx_scratch<T>(c, 1, n * nrhs);
    to_nat<T>(c, 0, n, nrhs, static_cast<const double2*>(in), a, s);
    dslash<T>(op, a, b, s, nrhs);
    from_nat<T>(c, 0, n, nrhs, b, static_cast<double2*>(out), s);
  }
}

Hierarchy& H_(ddamg_hier h) {
  DD_REQUIRE(h != nullptr && h->h, "null hierarchy");
  return *h->h;
}

template <typename T>
void apply_Dc_impl(Hierarchy& H, int level, const void* in, void* out, int nrhs, int layout) {
  const long long n = H.lv[level].n;
  if (layout == DDAMG_NATIVE) {
    H.apply<T>(level, static_cast<const C<T>*>(in), static_cast<C<T>*>(out), nrhs);
  } else {
    C<T>* a = hier_scratch<T>(H, 0, n * nrhs);
    C<T>* b = hier_scratch<T>(H, 1, n * nrhs);
    to_nat<T>(*H.ctx, level, n, nrhs, static_cast<const double2*>(in), a, H.s);
    H.apply<T>(level, a, b, nrhs);
    from_nat<T>(*H.ctx, level, n, nrhs, b, static_cast<double2*>(out), H.s);
  }
}

template <typename T>
void restrict_impl(Hierarchy& H, int level, const void* fine, void* coarse, int nrhs, int layout) {
  const long long nf = H.lv[level].n, nc = H.lv[level + 1].n;
  if (layout == DDAMG_NATIVE) {
    H.restrict_to<T>(level, static_cast<const C<T>*>(fine), static_cast<C<T>*>(coarse), nrhs);
  } else {
    C<T>* a = hier_scratch<T>(H, 0, nf * nrhs);
    C<T>* b = hier_scratch<T>(H, 1, nf * nrhs);
    to_nat<T>(*H.ctx, level, nf, nrhs, static_cast<const double2*>(fine), a, H.s);
    H.restrict_to<T>(level, a, b, nrhs);
    from_nat<T>(*H.ctx, level + 1, nc, nrhs, b, static_cast<double2*>(coarse), H.s);
  }
}

template <typename T>
void prolong_impl(Hierarchy& H, int level, const void* coarse, void* fine, int nrhs, int layout) {
  const long long nf = H.lv[level].n, nc = H.lv[level + 1].n;
  if (layout == DDAMG_NATIVE) {
    H.prolong_add<T>(level, static_cast<const C<T>*>(coarse), static_cast<C<T>*>(fine), nrhs);
  } else {
    C<T>* a = hier_scratch<T>(H, 0, nf * nrhs);
    C<T>* b = hier_scratch<T>(H, 1, nf * nrhs);
    to_nat<T>(*H.ctx, level, nf, nrhs, static_cast<const double2*>(fine), a, H.s);
    to_nat<T>(*H.ctx, level + 1, nc, nrhs, static_cast<const double2*>(coarse), b, H.s);
    H.prolong_add<T>(level, b, a, nrhs);
    from_nat<T>(*H.ctx, level, nf, nrhs, a, static_cast<double2*>(fine), H.s);
  }
}

template <typename T>
void sap_impl(Hierarchy& H, int level, const void* b, void* z, int nsweeps, int nrhs, int layout) {
  const long long n = H.lv[level].n;
  if (layout == DDAMG_NATIVE) {
    H.sap<T>(level, static_cast<const C<T>*>(b), static_cast<C<T>*>(z), nsweeps, nrhs);
  } else {
    C<T>* a = hier_scratch<T>(H, 0, n * nrhs);
    C<T>* c = hier_scratch<T>(H, 1, n * nrhs);
    to_nat<T>(*H.ctx, level, n, nrhs, static_cast<const double2*>(b), a, H.s);
    to_nat<T>(*H.ctx, level, n, nrhs, static_cast<const double2*>(z), c, H.s);
    H.sap<T>(level, a, c, nsweeps, nrhs);
    from_nat<T>(*H.ctx, level, n, nrhs, c, static_cast<double2*>(z), H.s);
  }
}

// The native form of nrhs FP16 fine fields (DDAMG_F16S, DDAMG_NATIVE): the
// FP16 entries of all fields ([nrhs][V/16][12][16] __half2) followed by their
// site scales ([nrhs][V] float), in one buffer.
struct HsPacked {
  __half2* h;
  float* s;
};
HsPacked hs_packed(const void* p, long long n0, int nrhs) {
  __half2* h = static_cast<__half2*>(const_cast<void*>(p));
  return HsPacked{h, reinterpret_cast<float*>(h + n0 * nrhs)};
}

// Level calls on FP16 fine spinors (DDAMG_F16S): the canonical FP64 fields
// are converted to native FP64 and encoded into the hierarchy's FP16
// buffers, and the results decoded back, a batch of at most params.batch
// at a time
template <typename F> void f16s_chunks(Hierarchy& H, int nrhs, F&& f) {
  const int cap = std::min(nrhs, H.p.batch);
  H.ensure_work<float>(cap);
  H.ensure_hs(cap);
  const long long n = H.lv[0].n;
  double2* a = hier_scratch<double>(H, 0, n * cap);
  double2* c = hier_scratch<double>(H, 1, n * cap);
  for (int r0 = 0; r0 < nrhs; r0 += cap) f(r0, std::min(cap, nrhs - r0), a, c);
}

void sap_f16s(Hierarchy& H, const void* b, void* z, int nsweeps, int nrhs, int layout) {
  const FineGeom& g = H.ctx->g;
  const long long n = H.lv[0].n;
  if (layout == DDAMG_NATIVE) {
    const HsPacked pb = hs_packed(b, n, nrhs), pz = hs_packed(z, n, nrhs);
    H.sap_hs(pb.h, pb.s, pz.h, pz.s, nsweeps, nrhs);
    return;
  }
  f16s_chunks(H, nrhs, [&](int r0, int nb, double2* a, double2*) {
    fine_to_native<double>(g, static_cast<const double2*>(b) + r0 * n, a, nb, H.s);
    encode_h<double>(g, a, H.h16a.p, H.h16as.p, nb, H.s);
    fine_to_native<double>(g, static_cast<const double2*>(z) + r0 * n, a, nb, H.s);
    encode_h<double>(g, a, H.h16b.p, H.h16bs.p, nb, H.s);
    H.sap_hs(H.h16a.p, H.h16as.p, H.h16b.p, H.h16bs.p, nsweeps, nb);
    decode_h<double>(g, H.h16b.p, H.h16bs.p, a, nb, H.s);
    fine_from_native<double>(g, a, static_cast<double2*>(z) + r0 * n, nb, H.s);
  });
}

void restrict_f16s(Hierarchy& H, const void* fine, void* coarse, int nrhs, int layout) {
  const FineGeom& g = H.ctx->g;
  const long long n = H.lv[0].n, nc = H.lv[1].n;
  if (layout == DDAMG_NATIVE) {
    const HsPacked pf = hs_packed(fine, n, nrhs);
    H.restrict_hs(pf.h, pf.s, static_cast<float2*>(coarse), nrhs);
    return;
  }
  f16s_chunks(H, nrhs, [&](int r0, int nb, double2* a, double2* c) {
    fine_to_native<double>(g, static_cast<const double2*>(fine) + r0 * n, a, nb, H.s);
    encode_h<double>(g, a, H.h16a.p, H.h16as.p, nb, H.s);
    float2* cf = reinterpret_cast<float2*>(c);
    H.restrict_hs(H.h16a.p, H.h16as.p, cf, nb);
    vcopy<float, double>(cf, static_cast<double2*>(coarse) + r0 * nc, nc * nb, H.s);
  });
}

void prolong_f16s(Hierarchy& H, const void* coarse, void* fine, int nrhs) {
  const FineGeom& g = H.ctx->g;
  const long long n = H.lv[0].n, nc = H.lv[1].n;
  f16s_chunks(H, nrhs, [&](int r0, int nb, double2* a, double2* c) {
    float2* cf = reinterpret_cast<float2*>(c);
    vcopy<double, float>(static_cast<const double2*>(coarse) + r0 * nc, cf, nc * nb, H.s);
    H.prolong_hs(cf, H.h16b.p, H.h16bs.p, nb);
    // fine += the decoded FP16 result
    decode_h<double>(g, H.h16b.p, H.h16bs.p, a, nb, H.s);
    fine_from_native<double>(g, a, c, nb, H.s);
    vadd<double>(c, static_cast<double2*>(fine) + r0 * n, n * nb, H.s);
  });
}

// the solve's preconditioner on a hierarchy with FP16 spinors: b encoded,
// the FP16 cycle, z decoded (T: the precision of native-layout fields)
template <typename T>
void precondition_hs(Hierarchy& H, const void* b, void* z, int nrhs, int layout) {
  const FineGeom& g = H.ctx->g;
  const long long n = H.lv[0].n;
  f16s_chunks(H, nrhs, [&](int r0, int nb, double2* a, double2*) {
    std::fill(H.kc_it.begin(), H.kc_it.end(), 0);
    std::fill(H.cs_it.begin(), H.cs_it.end(), 0);
    if (layout == DDAMG_NATIVE) {
      encode_h<T>(g, static_cast<const C<T>*>(b) + r0 * n, H.h16a.p, H.h16as.p, nb, H.s);
    } else {
      fine_to_native<double>(g, static_cast<const double2*>(b) + r0 * n, a, nb, H.s);
      encode_h<double>(g, a, H.h16a.p, H.h16as.p, nb, H.s);
    }
    H.cycle_hs(H.h16a.p, H.h16as.p, H.h16b.p, H.h16bs.p, nb);
    if (layout == DDAMG_NATIVE) {
      decode_h<T>(g, H.h16b.p, H.h16bs.p, static_cast<C<T>*>(z) + r0 * n, nb, H.s);
    } else {
      decode_h<double>(g, H.h16b.p, H.h16bs.p, a, nb, H.s);
      fine_from_native<double>(g, a, static_cast<double2*>(z) + r0 * n, nb, H.s);
    }
  });
}

template <typename T>
void precondition_impl(Hierarchy& H, const void* b, void* z, int nrhs, int layout) {
  const long long n = H.lv[0].n;
  H.ensure_work<T>(std::min(nrhs, H.p.batch));
  const int cap = H.work<T>(0).cap;
  for (int r0 = 0; r0 < nrhs; r0 += cap) {
    const int nb = std::min(cap, nrhs - r0);
    std::fill(H.kc_it.begin(), H.kc_it.end(), 0);
    std::fill(H.cs_it.begin(), H.cs_it.end(), 0);
    // the cycle writes z before reading b's copy; b must stay intact
    C<T>* a = hier_scratch<T>(H, 0, n * nb);
    if (layout == DDAMG_NATIVE) {
      vcopy<T, T>(static_cast<const C<T>*>(b) + r0 * n, a, n * nb, H.s);
      H.cycle<T>(0, a, static_cast<C<T>*>(z) + r0 * n, nb);
    } else {
      C<T>* c = hier_scratch<T>(H, 1, n * nb);
      to_nat<T>(*H.ctx, 0, n, nb, static_cast<const double2*>(b) + r0 * n, a, H.s);
      H.cycle<T>(0, a, c, nb);
      from_nat<T>(*H.ctx, 0, n, nb, c, static_cast<double2*>(z) + r0 * n, H.s);
    }
  }
}

}  // namespace

extern "C" {

const char* ddamg_last_error(void) { return g_err.c_str(); }

const char* ddamg_version(void) { return "ddamg-gfx950 0.1"; }

void ddamg_params_default(ddamg_params* p, int levels) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->levels = levels;
  for (int l = 0; l < 3; ++l)
    for (int mu = 0; mu < 4; ++mu) p->agg[l][mu] = l == 0 ? 4 : 2;
  for (int l = 0; l < 3; ++l) p->ntv[l] = 20;
  for (int mu = 0; mu < 4; ++mu) p->sap_block[mu] = 2;
  p->mu = 0;
  p->nu = 5;
  p->mr_iters = 3;
  p->n_inv = 6;
  p->coarse_eps = 5e-2;
  p->coarse_restart = 30;
  p->coarse_max_restarts = 10;
  p->kc_len = 5;
  p->kc_restarts = 2;
  p->kc_tol = 1e-1;
  p->nkv = 10;
  p->tol = 1e-10;
  p->max_restarts = 100;
  p->precond_prec = DDAMG_F32;
  p->cycle = DDAMG_KCYCLE;
  p->half_storage = 0;
  p->batch = 16;
  p->half_directions = 0;
  p->graph = 0;
  p->coarse_dense = 1;
  p->galerkin_cols = 0;
  p->profile_levels = 0;
  p->half_spinors = 0;
}

int ddamg_create(const ddamg_lattice* lat, const void* links, void* stream, ddamg_ctx* out) {
  return guarded([&] {
    DD_REQUIRE(out != nullptr, "null output handle");
    *out = nullptr;
    std::unique_ptr<ddamg_ctx_s> h(new ddamg_ctx_s);
    h->c.reset(create_context(lat, static_cast<const double2*>(links), as_stream(stream)));
    *out = h.release();
  });
}

void ddamg_destroy(ddamg_ctx ctx) { delete ctx; }

int ddamg_workspace_bytes(const ddamg_lattice* lat, const ddamg_params* params, int nrhs_max,
                          size_t* ctx_bytes, size_t* hier_bytes) {
  return guarded([&] {
    DD_REQUIRE(ctx_bytes || hier_bytes, "no output");
    workspace_bytes(lat, params, nrhs_max, ctx_bytes, hier_bytes);
  });
}

// the caller's workspace for a handle, checked against what the handle's
// layout counts
static std::unique_ptr<Workspace> caller_workspace(void* workspace, size_t ws_bytes, size_t need) {
  DD_REQUIRE(workspace != nullptr, "null workspace");
  DD_REQUIRE(reinterpret_cast<uintptr_t>(workspace) % Workspace::ALIGN == 0,
             "the workspace must be aligned to 256 bytes");
  DD_REQUIRE(ws_bytes >= need, "the workspace holds " + std::to_string(ws_bytes) + " bytes; " +
                                   std::to_string(need) + " are needed");
  return std::unique_ptr<Workspace>(new Workspace(workspace, ws_bytes));
}

int ddamg_create_ws(const ddamg_lattice* lat, const void* links, const ddamg_params* params, int nrhs_max,
                    void* workspace, size_t ws_bytes, void* stream, ddamg_ctx* out) {
  return guarded([&] {
    DD_REQUIRE(out != nullptr, "null output handle");
    *out = nullptr;
    size_t need = 0;
    workspace_bytes(lat, params, nrhs_max, &need, nullptr);
    const bool half = params && params->half_storage == 1;
    std::unique_ptr<ddamg_ctx_s> h(new ddamg_ctx_s);
    h->c.reset(create_context(lat, static_cast<const double2*>(links), as_stream(stream),
                              caller_workspace(workspace, ws_bytes, need), half, nrhs_max));
    *out = h.release();
  });
}


int ddamg_apply_D(ddamg_ctx ctx, const void* in, void* out, int nrhs, int prec, int layout,
                  void* stream) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c, "null context");
    const WorkspaceScope wsc(ctx->c->ws.get());
    DD_REQUIRE(in && out && in != out, "in/out must be distinct device pointers");
    DD_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    check_prec(prec);
    check_layout(layout);
    if (prec == DDAMG_F64) apply_D_impl<double>(*ctx->c, in, out, nrhs, layout, as_stream(stream));
    else if (prec == DDAMG_F16) apply_D_impl<float, true>(*ctx->c, in, out, nrhs, layout, as_stream(stream));
    else apply_D_impl<float>(*ctx->c, in, out, nrhs, layout, as_stream(stream));
  });
}

int ddamg_to_native(ddamg_ctx ctx, ddamg_hier hier, int level, const void* in, void* out, int nrhs,
                    int prec, void* stream) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c && in && out && nrhs >= 1, "bad argument");
    check_prec(prec, true);
    DD_REQUIRE(prec != DDAMG_F16S || level == 0, "DDAMG_F16S applies to level 0");
    hipStream_t s = as_stream(stream);
    Context& c = *ctx->c;
    const WorkspaceScope wsc(c.ws.get());
    if (prec == DDAMG_F16S) {
      const long long n = c.g.V * 12;
      double2* a = ctx_scratch<double>(c, 0, n * nrhs);
      fine_to_native<double>(c.g, static_cast<const double2*>(in), a, nrhs, s);
      const HsPacked po = hs_packed(out, n, nrhs);
      encode_h<double>(c.g, a, po.h, po.s, nrhs, s);
    } else if (level == 0) {
      if (prec == DDAMG_F64) fine_to_native<double>(c.g, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, s);
      else fine_to_native<float>(c.g, static_cast<const double2*>(in), static_cast<float2*>(out), nrhs, s);
    } else {
      Hierarchy& H = H_(hier);
      DD_REQUIRE(level < H.L, "level out of range");
      const long long n = H.lv[level].n * nrhs;
      if (prec == DDAMG_F64) vcopy<double, double>(static_cast<const double2*>(in), static_cast<double2*>(out), n, s);
      else vcopy<double, float>(static_cast<const double2*>(in), static_cast<float2*>(out), n, s);
    }
  });
}

int ddamg_from_native(ddamg_ctx ctx, ddamg_hier hier, int level, const void* in, void* out, int nrhs,
                      int prec, void* stream) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c && in && out && nrhs >= 1, "bad argument");
    check_prec(prec, true);
    DD_REQUIRE(prec != DDAMG_F16S || level == 0, "DDAMG_F16S applies to level 0");
    hipStream_t s = as_stream(stream);
    Context& c = *ctx->c;
    const WorkspaceScope wsc(c.ws.get());
    if (prec == DDAMG_F16S) {
      const long long n = c.g.V * 12;
      double2* a = ctx_scratch<double>(c, 0, n * nrhs);
      const HsPacked pi = hs_packed(in, n, nrhs);
      decode_h<double>(c.g, pi.h, pi.s, a, nrhs, s);
      fine_from_native<double>(c.g, a, static_cast<double2*>(out), nrhs, s);
      return;
    }
    if (level == 0) {
      if (prec == DDAMG_F64) fine_from_native<double>(c.g, static_cast<const double2*>(in), static_cast<double2*>(out), nrhs, s);
      else fine_from_native<float>(c.g, static_cast<const float2*>(in), static_cast<double2*>(out), nrhs, s);
    } else {
      Hierarchy& H = H_(hier);
      DD_REQUIRE(level < H.L, "level out of range");
      const long long n = H.lv[level].n * nrhs;
      if (prec == DDAMG_F64) vcopy<double, double>(static_cast<const double2*>(in), static_cast<double2*>(out), n, s);
      else vcopy<float, double>(static_cast<const float2*>(in), static_cast<double2*>(out), n, s);
    }
  });
}

int ddamg_build_hierarchy(ddamg_ctx ctx, const ddamg_params* params, const void* tv,
                          const void* tv_extra, void* stream, ddamg_hier* out) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c, "null context");
    DD_REQUIRE(out != nullptr, "null output handle");
    *out = nullptr;
    std::unique_ptr<ddamg_hier_s> h(new ddamg_hier_s);
    h->owner = ctx;
    h->h.reset(create_hierarchy(ctx->c.get(), params, static_cast<const double2*>(tv),
                                static_cast<const double2*>(tv_extra), as_stream(stream)));
    *out = h.release();
  });
}

void ddamg_destroy_hierarchy(ddamg_hier hier) { delete hier; }

int ddamg_build_hierarchy_ws(ddamg_ctx ctx, const ddamg_params* params, const void* tv, const void* tv_extra,
                             int nrhs_max, void* workspace, size_t ws_bytes, void* stream, ddamg_hier* out) {
  return guarded([&] {
    DD_REQUIRE(ctx && ctx->c, "null context");
    DD_REQUIRE(out != nullptr && params != nullptr, "null argument");
    *out = nullptr;
    ddamg_lattice lat{};
    for (int mu = 0; mu < 4; ++mu) lat.dims[mu] = ctx->c->g.dims[mu];
    lat.m0 = ctx->c->m0;
    lat.csw = ctx->c->csw;
    size_t need = 0;
    workspace_bytes(&lat, params, nrhs_max, nullptr, &need);
    std::unique_ptr<ddamg_hier_s> h(new ddamg_hier_s);
    h->owner = ctx;
    h->h.reset(create_hierarchy(ctx->c.get(), params, static_cast<const double2*>(tv),
                                static_cast<const double2*>(tv_extra), as_stream(stream),
                                caller_workspace(workspace, ws_bytes, need), nrhs_max));
    *out = h.release();
  });
}


int ddamg_level_info(ddamg_hier hier, int level, int dims_out[4], int* dof_out) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L, "level out of range");
    if (dims_out) for (int mu = 0; mu < 4; ++mu) dims_out[mu] = H.lv[level].dims[mu];
    if (dof_out) *dof_out = H.lv[level].d;
  });
}

int ddamg_apply_Dc(ddamg_hier hier, int level, const void* in, void* out, int nrhs, int prec,
                   int layout, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L, "level out of range");
    DD_REQUIRE(in && out && in != out && nrhs >= 1, "bad argument");
    check_prec(prec);
    check_layout(layout);
    H.s = as_stream(stream);
    check_half(H, prec);
    if (prec == DDAMG_F64) apply_Dc_impl<double>(H, level, in, out, nrhs, layout);
    else apply_Dc_impl<float>(H, level, in, out, nrhs, layout);
  });
}

int ddamg_restrict(ddamg_hier hier, int level, const void* fine, void* coarse, int nrhs, int prec,
                   int layout, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L - 1, "level out of range");
    DD_REQUIRE(fine && coarse && nrhs >= 1, "bad argument");
    check_prec(prec, true);
    check_layout(layout);
    H.s = as_stream(stream);
    check_half(H, prec);
    check_f16s(H, prec, level, layout, true);
    if (prec == DDAMG_F16S) restrict_f16s(H, fine, coarse, nrhs, layout);
    else if (prec == DDAMG_F64) restrict_impl<double>(H, level, fine, coarse, nrhs, layout);
    else restrict_impl<float>(H, level, fine, coarse, nrhs, layout);
  });
}

int ddamg_prolong(ddamg_hier hier, int level, const void* coarse, void* fine, int nrhs, int prec,
                  int layout, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L - 1, "level out of range");
    DD_REQUIRE(fine && coarse && nrhs >= 1, "bad argument");
    check_prec(prec, true);
    check_layout(layout);
    H.s = as_stream(stream);
    check_half(H, prec);
    check_f16s(H, prec, level, layout, false);
    if (prec == DDAMG_F16S) prolong_f16s(H, coarse, fine, nrhs);
    else if (prec == DDAMG_F64) prolong_impl<double>(H, level, coarse, fine, nrhs, layout);
    else prolong_impl<float>(H, level, coarse, fine, nrhs, layout);
  });
}

int ddamg_sap_smooth(ddamg_hier hier, int level, const void* b, void* z, int nsweeps, int nrhs,
                     int prec, int layout, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L - 1, "SAP is defined on levels 0..L-2");
    DD_REQUIRE(b && z && b != z && nrhs >= 1 && nsweeps >= 0, "bad argument");
    check_prec(prec, true);
    check_layout(layout);
    H.s = as_stream(stream);
    check_half(H, prec);
    check_f16s(H, prec, level, layout, true);
    if (prec == DDAMG_F16S) sap_f16s(H, b, z, nsweeps, nrhs, layout);
    else if (prec == DDAMG_F64) sap_impl<double>(H, level, b, z, nsweeps, nrhs, layout);
    else sap_impl<float>(H, level, b, z, nsweeps, nrhs, layout);
  });
}

int ddamg_precondition(ddamg_hier hier, const void* b, void* z, int nrhs, int layout, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(b && z && b != z && nrhs >= 1, "bad argument");
    check_layout(layout);
    H.s = as_stream(stream);
    if (H.p.precond_prec == DDAMG_F64) precondition_impl<double>(H, b, z, nrhs, layout);
    else if (H.hs) precondition_hs<float>(H, b, z, nrhs, layout);
    else precondition_impl<float>(H, b, z, nrhs, layout);
  });
}

namespace {

// Solves the nrhs systems of one hierarchy on stream s, params.batch at a
// time; fills stats (per system) and returns the worst per-system outcome
// (DDAMG_OK, DDAMG_ENOCONV or DDAMG_ENONFINITE).  Failures of the library
// itself throw.
int solve_batches(Hierarchy& H, const void* b, void* z, int nrhs, ddamg_solve_stats* stats, hipStream_t s,
                  const void* z_ref = nullptr) {
  int worst = DDAMG_OK;
  if (H.p.graph && (!H.own_s || s != H.own_s)) {
    // graphs are captured on the hierarchy's own stream (the caller's may be
    // the null stream, which cannot be captured), ordered after the caller's
    if (!H.own_s) DD_CHECK_HIP(hipStreamCreateWithFlags(&H.own_s, hipStreamNonBlocking));
    hipEvent_t ready = nullptr;
    DD_CHECK_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    const hipError_t e1 = hipEventRecord(ready, s);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(H.own_s, ready, 0) : e1;
    (void)hipEventDestroy(ready);
    DD_CHECK_HIP(e2);
    s = H.own_s;
  }
  H.s = s;
  const long long n = H.lv[0].n;
  const int bmax = std::min(nrhs, H.p.batch);
  if (H.p.precond_prec == DDAMG_F64) H.ensure_batch<double>(bmax);
  else H.ensure_batch<float>(bmax);
  std::vector<ddamg_solve_stats> st(bmax);
  for (int r0 = 0; r0 < nrhs; r0 += bmax) {
    const int nb = std::min(bmax, nrhs - r0);
    auto t0 = std::chrono::steady_clock::now();
    for (auto& e : st) std::memset(&e, 0, sizeof(e));
    std::fill(H.kc_it.begin(), H.kc_it.end(), 0);
    std::fill(H.cs_it.begin(), H.cs_it.end(), 0);
    H.m_bytes = H.m_flops = 0;
    H.lt_begin();
    fine_to_native<double>(H.ctx->g, static_cast<const double2*>(b) + r0 * n, H.ob.p, nb, H.s);
    fine_to_native<double>(H.ctx->g, static_cast<const double2*>(z) + r0 * n, H.ox.p, nb, H.s);
    if (H.p.precond_prec == DDAMG_F64) H.outer<double>(H.ob.p, H.ox.p, st.data(), nb);
    else H.outer<float>(H.ob.p, H.ox.p, st.data(), nb);
    fine_from_native<double>(H.ctx->g, H.ox.p, static_cast<double2*>(z) + r0 * n, nb, H.s);
    double tl[4];
    H.lt_end(tl);
    // the error against the reference solution, in FP64 on the device
    std::vector<double> err(nb, -1.0);
    if (z_ref) {
      const double2* zr = static_cast<const double2*>(z_ref) + r0 * n;
      std::vector<double> dn, rn;
      vcopy<double, double>(zr, H.ow.p, n * nb, H.s);
      vbmy<double>(static_cast<const double2*>(z) + r0 * n, H.ow.p, n * nb, H.s);
      bnorms<double>(*H.red, H.ow.p, n, nb, dn, H.s);
      bnorms<double>(*H.red, zr, n, nb, rn, H.s);
      for (int r = 0; r < nb; ++r) err[r] = rn[r] > 0 ? dn[r] / rn[r] : dn[r];
    }
    DD_CHECK_HIP(hipStreamSynchronize(H.s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < nb; ++r) {
      st[r].kcycle_iters = H.kc_it[r];
      st[r].coarsest_iters = H.cs_it[r];
      st[r].seconds = secs;
      st[r].err_vs_ref = err[r];
      st[r].t_setup_s = H.t_setup;
      for (int k = 0; k < 4; ++k) st[r].t_level_s[k] = tl[k];
      st[r].bytes = H.m_bytes;
      st[r].flops = H.m_flops;
      st[r].coarsest_dense = H.lv[H.L - 1].sm;
      if (stats) stats[r0 + r] = st[r];
      if (st[r].status != DDAMG_OK && worst == DDAMG_OK) worst = st[r].status;
    }
  }
  return worst;
}

int report_worst(int worst) {
  if (worst == DDAMG_ENOCONV) g_err = "outer FGMRES reached max_restarts before tol";
  if (worst == DDAMG_ENONFINITE) g_err = "non-finite value in b or in a residual";
  return worst;
}

}  // namespace

int ddamg_solve(ddamg_hier hier, const void* b, void* z, int nrhs, ddamg_solve_stats* stats,
                void* stream) {
  int worst = DDAMG_OK;
  int rc = guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(b && z && b != z && nrhs >= 1, "bad argument");
    worst = solve_batches(H, b, z, nrhs, stats, as_stream(stream));
  });
  if (rc != DDAMG_OK) return rc;
  return report_worst(worst);
}

int ddamg_solve_ex(ddamg_hier hier, const void* b, void* z, int nrhs, const void* z_ref,
                   ddamg_solve_stats* stats, void* stream) {
  int worst = DDAMG_OK;
  int rc = guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(b && z && b != z && nrhs >= 1, "bad argument");
    DD_REQUIRE(z_ref != z && z_ref != b, "z_ref must not alias b or z");
    worst = solve_batches(H, b, z, nrhs, stats, as_stream(stream), z_ref);
  });
  if (rc != DDAMG_OK) return rc;
  return report_worst(worst);
}

int ddamg_solve_many(int n, const ddamg_hier* hiers, const void* const* b, void* const* z, const int* nrhs,
                     ddamg_solve_stats* stats, void* stream) {
  std::vector<int> worst(n > 0 ? n : 0, DDAMG_OK), rcs(n > 0 ? n : 0, DDAMG_OK);
  std::vector<std::string> msgs(n > 0 ? n : 0);
  int rc = guarded([&] {
    DD_REQUIRE(n >= 1 && n <= DDAMG_MAX_SYSTEMS, "n must be in 1..DDAMG_MAX_SYSTEMS");
    DD_REQUIRE(hiers && b && z && nrhs, "null argument array");
    std::vector<long long> off(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      DD_REQUIRE(hiers[i] != nullptr, "null hierarchy");
      DD_REQUIRE(b[i] && z[i] && b[i] != z[i] && nrhs[i] >= 1, "bad argument for system " + std::to_string(i));
      for (int k = 0; k < i; ++k)
        DD_REQUIRE(hiers[k] != hiers[i], "a hierarchy appears twice (its solves would share buffers)");
      off[i + 1] = off[i] + nrhs[i];
    }
    int dev = 0;
    DD_CHECK_HIP(hipGetDevice(&dev));
    // the inputs are ordered after the work already on the caller's stream
    struct Ev {
      hipEvent_t e = nullptr;
      ~Ev() { if (e) (void)hipEventDestroy(e); }
    } ready;
    DD_CHECK_HIP(hipEventCreateWithFlags(&ready.e, hipEventDisableTiming));
    DD_CHECK_HIP(hipEventRecord(ready.e, as_stream(stream)));
    for (int i = 0; i < n; ++i) {
      Hierarchy& H = H_(hiers[i]);
      if (!H.own_s) DD_CHECK_HIP(hipStreamCreateWithFlags(&H.own_s, hipStreamNonBlocking));
      DD_CHECK_HIP(hipStreamWaitEvent(H.own_s, ready.e, 0));
    }
    // one host thread per system: each drives its hierarchy's solver on the
    // hierarchy's own stream, so the kernels of different systems overlap
    // and one system's host round trips hide behind the others' work
    struct Joiner {
      std::vector<std::thread> t;
      ~Joiner() { for (auto& x : t) if (x.joinable()) x.join(); }
    } th;
    th.t.reserve(n);
    for (int i = 0; i < n; ++i)
      th.t.emplace_back([&, i] {
        try {
          Hierarchy& H = H_(hiers[i]);
          const WorkspaceScope wsc(H.ws.get());
          DD_CHECK_HIP(hipSetDevice(dev));
          worst[i] = solve_batches(H, b[i], z[i], nrhs[i], stats ? stats + off[i] : nullptr, H.own_s);
        } catch (const Error& e) {
          rcs[i] = e.status;
          msgs[i] = e.what();
        } catch (const std::exception& e) {
          rcs[i] = DDAMG_EHIP;
          msgs[i] = e.what();
        } catch (...) {
          rcs[i] = DDAMG_EHIP;
          msgs[i] = "unknown failure";
        }
      });
    for (auto& t : th.t) t.join();
    for (int i = 0; i < n; ++i)
      if (rcs[i] != DDAMG_OK) throw Error(rcs[i], "system " + std::to_string(i) + ": " + msgs[i]);
  });
  if (rc != DDAMG_OK) return rc;
  int w = DDAMG_OK;
  for (int i = 0; i < n; ++i)
    if (worst[i] != DDAMG_OK && w == DDAMG_OK) w = worst[i];
  return report_worst(w);
}

}  // extern "C"

namespace {

// One graph over several hierarchies.  f(H) is captured for each hierarchy
// on its own stream into a graph of its own; their kernel nodes are then
// copied into one graph, each system's nodes with their own dependencies
// and none between systems, so the replay runs the systems side by side.
// The node lists per system let the host disable a system's nodes once it
// has converged (disabled nodes do nothing).
template <typename F>
Hierarchy::BatchGraph capture_all(const std::vector<Hierarchy*>& hs, F&& f) {
  Hierarchy::BatchGraph bg;
  const size_t n = hs.size();
  struct Graphs {
    std::vector<hipGraph_t> g;
    ~Graphs() {
      for (hipGraph_t x : g)
        if (x) (void)hipGraphDestroy(x);
    }
  } parts;
  parts.g.assign(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    Hierarchy& H = *hs[i];
    H.s = H.own_s;
    const WorkspaceScope wsc(H.ws.get());
    DD_CHECK_HIP(hipStreamBeginCapture(H.own_s, hipStreamCaptureModeThreadLocal));
    try {
      f(H);
    } catch (...) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(H.own_s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      (void)hipGetLastError();
      throw;
    }
    DD_CHECK_HIP(hipStreamEndCapture(H.own_s, &parts.g[i]));
  }
  DD_CHECK_HIP(hipGraphCreate(&bg.g, 0));
  try {
    bg.nodes.resize(n);
    bg.on.assign(n, 1);
    for (size_t i = 0; i < n; ++i) {
      size_t cnt = 0;
      DD_CHECK_HIP(hipGraphGetNodes(parts.g[i], nullptr, &cnt));
      std::vector<hipGraphNode_t> src(cnt);
      if (cnt) DD_CHECK_HIP(hipGraphGetNodes(parts.g[i], src.data(), &cnt));
      // copy in dependency order (each node after the nodes it waits for)
      std::map<hipGraphNode_t, hipGraphNode_t> dst;
      std::vector<std::vector<hipGraphNode_t>> deps(cnt);
      for (size_t k = 0; k < cnt; ++k) {
        size_t nd = 0;
        DD_CHECK_HIP(hipGraphNodeGetDependencies(src[k], nullptr, &nd));
        deps[k].resize(nd);
        if (nd) DD_CHECK_HIP(hipGraphNodeGetDependencies(src[k], deps[k].data(), &nd));
      }
      size_t done = 0;
      std::vector<char> copied(cnt, 0);
      while (done < cnt) {
        bool progress = false;
        for (size_t k = 0; k < cnt; ++k) {
          if (copied[k]) continue;
          std::vector<hipGraphNode_t> dd;
          bool ready = true;
          for (hipGraphNode_t d : deps[k]) {
            auto it = dst.find(d);
            if (it == dst.end()) {
              ready = false;
              break;
            }
            dd.push_back(it->second);
          }
          if (!ready) continue;
          hipGraphNodeType type;
          DD_CHECK_HIP(hipGraphNodeGetType(src[k], &type));
          hipGraphNode_t nn = nullptr;
          if (type == hipGraphNodeTypeKernel) {
            hipKernelNodeParams kp{};
            DD_CHECK_HIP(hipGraphKernelNodeGetParams(src[k], &kp));
            DD_CHECK_HIP(hipGraphAddKernelNode(&nn, bg.g, dd.data(), dd.size(), &kp));
            bg.nodes[i].push_back(nn);
          } else if (type == hipGraphNodeTypeEmpty) {
            DD_CHECK_HIP(hipGraphAddEmptyNode(&nn, bg.g, dd.data(), dd.size()));
          } else {
            throw Error(DDAMG_EHIP, "a captured outer step holds a graph node other than a kernel");
          }
          dst[src[k]] = nn;
          copied[k] = 1;
          ++done;
          progress = true;
        }
        DD_REQUIRE(progress, "cyclic dependencies in a captured graph");
      }
    }
    DD_CHECK_HIP(hipGraphInstantiate(&bg.exec, bg.g, nullptr, nullptr, 0));
  } catch (...) {
    if (bg.exec) (void)hipGraphExecDestroy(bg.exec);
    if (bg.g) (void)hipGraphDestroy(bg.g);
    throw;
  }
  return bg;
}

// enable the nodes of exactly the systems in `want`
void set_systems(Hierarchy::BatchGraph& bg, const std::vector<char>& want) {
  for (size_t i = 0; i < want.size(); ++i) {
    if (bg.on[i] == want[i]) continue;
    for (hipGraphNode_t nd : bg.nodes[i]) DD_CHECK_HIP(hipGraphNodeSetEnabled(bg.exec, nd, want[i] ? 1u : 0u));
    bg.on[i] = want[i];
  }
}

bool flag_of(const Hierarchy& H) { return *static_cast<volatile int*>(H.go_flag_host) != 0; }

}  // namespace

extern "C" {

int ddamg_solve_batch(int n, const ddamg_hier* hiers, const void* const* b, void* const* z,
                      ddamg_solve_stats* stats, void* stream) {
  int worst = DDAMG_OK;
  int rc = guarded([&] {
    const TraceRange range("ddamg solve batch");
    DD_REQUIRE(n >= 1 && n <= DDAMG_MAX_SYSTEMS, "n must be 1..DDAMG_MAX_SYSTEMS");
    DD_REQUIRE(hiers && b && z, "null argument");
    std::vector<Hierarchy*> hs(n);
    for (int i = 0; i < n; ++i) {
      DD_REQUIRE(hiers[i] != nullptr, "null hierarchy");
      DD_REQUIRE(b[i] && z[i] && b[i] != z[i], "bad argument for system " + std::to_string(i));
      hs[i] = &H_(hiers[i]);
      for (int k = 0; k < i; ++k) DD_REQUIRE(hs[k] != hs[i], "a hierarchy appears twice (its solves would share buffers)");
      DD_REQUIRE(hs[i]->p.nkv == hs[0]->p.nkv, "every hierarchy of the batch needs the same n_kv");
    }
    const int m = hs[0]->p.nkv;
    for (Hierarchy* H : hs)
      if (!H->own_s) DD_CHECK_HIP(hipStreamCreateWithFlags(&H->own_s, hipStreamNonBlocking));
    // everything runs on the first hierarchy's own stream (a capture cannot
    // start on the caller's stream, which may be the null stream), after
    // the work already enqueued on the caller's
    hipStream_t S = hs[0]->own_s;
    {
      struct Ev {
        hipEvent_t e = nullptr;
        ~Ev() { if (e) (void)hipEventDestroy(e); }
      } ready;
      DD_CHECK_HIP(hipEventCreateWithFlags(&ready.e, hipEventDisableTiming));
      DD_CHECK_HIP(hipEventRecord(ready.e, as_stream(stream)));
      DD_CHECK_HIP(hipStreamWaitEvent(S, ready.e, 0));
    }
    int max_restarts = 0;
    for (Hierarchy* H : hs) {
      const WorkspaceScope wsc(H->ws.get());
      H->s = S;
      H->outer_dev_prepare();
      max_restarts = std::max(max_restarts, H->p.max_restarts);
    }
    // the step and tail graphs of this list of hierarchies, kept by the first
    Hierarchy& H0 = *hs[0];
    std::vector<long long> uids(n), gens(n);
    for (int i = 0; i < n; ++i) uids[i] = hs[i]->uid, gens[i] = hs[i]->gen;
    if (!H0.bgraphs || H0.bgraphs->uids != uids || H0.bgraphs->gens != gens) {
      H0.bgraphs.reset();
      std::unique_ptr<Hierarchy::BatchGraphs> bg(new Hierarchy::BatchGraphs);
      bg->uids = uids;
      bg->gens = gens;
      for (int j = 0; j < m; ++j) bg->step.push_back(capture_all(hs, [&](Hierarchy& H) { H.outer_dev_step(j); }));
      bg->tail = capture_all(hs, [&](Hierarchy& H) { H.outer_dev_tail(); });
      H0.bgraphs = std::move(bg);
    }
    const auto t0 = std::chrono::steady_clock::now();
    // inputs after the work already on S; targets, r_0 and V_0 eagerly
    for (int i = 0; i < n; ++i) {
      Hierarchy& H = *hs[i];
      const WorkspaceScope wsc(H.ws.get());
      H.s = S;
      fine_to_native<double>(H.ctx->g, static_cast<const double2*>(b[i]), H.ob.p, 1, S);
      fine_to_native<double>(H.ctx->g, static_cast<const double2*>(z[i]), H.ox.p, 1, S);
      H.outer_dev_begin();
    }
    DD_CHECK_HIP(hipStreamSynchronize(S));
    std::vector<int> restarts(n, 0);
    std::vector<char> active(n);
    for (int i = 0; i < n; ++i) active[i] = flag_of(*hs[i]);
    for (int c = 0; c < max_restarts; ++c) {
      bool any = false;
      for (int i = 0; i < n; ++i) {
        any = any || active[i];
        restarts[i] += active[i];
      }
      if (!any) break;
      // one graph per outer step of every system; the host reads the
      // systems' device-written liveness flags after each, disables the
      // nodes of the systems that have stopped in the graphs still to run,
      // and ends the cycle when none is left
      std::vector<char> live = active;
      for (int j = 0; j < m; ++j) {
        Hierarchy::BatchGraph& G = H0.bgraphs->step[j];
        set_systems(G, live);
        DD_CHECK_HIP(hipGraphLaunch(G.exec, S));
        DD_CHECK_HIP(hipStreamSynchronize(S));
        bool anylive = false;
        for (int i = 0; i < n; ++i) {
          live[i] = live[i] && flag_of(*hs[i]);
          anylive = anylive || live[i];
        }
        if (!anylive) break;
      }
      set_systems(H0.bgraphs->tail, active);
      DD_CHECK_HIP(hipGraphLaunch(H0.bgraphs->tail.exec, S));
      DD_CHECK_HIP(hipStreamSynchronize(S));
      for (int i = 0; i < n; ++i) active[i] = flag_of(*hs[i]);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // certification and results, system by system
    for (int i = 0; i < n; ++i) {
      Hierarchy& H = *hs[i];
      const WorkspaceScope wsc(H.ws.get());
      const long long nn = H.lv[0].n;
      H.s = S;
      std::vector<double> bn, rn;
      bnorms<double>(*H.red, H.ob.p, nn, 1, bn, S);
      dslash<double>(H.ctx->view<double>(), H.ox.p, H.ow.p, S, 1);
      vbmy<double>(H.ob.p, H.ow.p, nn, S);
      bnorms<double>(*H.red, H.ow.p, nn, 1, rn, S);
      long long its = 0;
      DD_CHECK_HIP(hipMemcpyAsync(&its, H.go_iters.p, sizeof(its), hipMemcpyDeviceToHost, S));
      fine_from_native<double>(H.ctx->g, H.ox.p, static_cast<double2*>(z[i]), 1, S);
      DD_CHECK_HIP(hipStreamSynchronize(S));
      ddamg_solve_stats st{};
      st.outer_iters = (int)its;
      st.restarts = restarts[i];
      st.true_relres = bn[0] > 0 ? rn[0] / bn[0] : 0.0;
      st.seconds = secs;
      st.err_vs_ref = -1;
      st.t_setup_s = H.t_setup;
      if (!std::isfinite(rn[0])) st.status = DDAMG_ENONFINITE;
      else if (rn[0] <= H.p.tol * bn[0]) st.status = DDAMG_OK;
      else st.status = DDAMG_ENOCONV;
      if (st.status != DDAMG_OK && worst == DDAMG_OK) worst = st.status;
      if (stats) stats[i] = st;
    }
  });
  if (rc != DDAMG_OK) return rc;
  return report_worst(worst);
}

int ddamg_set_sap_block(ddamg_hier hier, int level, const int block[4]) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(block != nullptr, "null block shape");
    H.set_sap_block(level, block);
  });
}

int ddamg_set_batch(ddamg_hier hier, int batch) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(batch >= 1 && batch <= NBMAX, "batch must be 1..32");
    H.p.batch = batch;
  });
}

int ddamg_tune(ddamg_hier hier, const void* b, int nrhs, const char* cache_path, ddamg_tune_result* out,
               void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(b && nrhs >= 1, "bad argument");
    const std::string path = cache_path ? cache_path : "";
    const std::string key = tune_key(H, nrhs);
    TuneChoice best;
    auto apply = [&](const TuneChoice& c) {
      for (int l = 1; l <= H.L - 2; ++l) H.set_sap_block(l, c.sap[l - 1]);
      if (c.batch >= 1) H.p.batch = c.batch;
    };
    auto current = [&]() {
      TuneChoice c;
      for (int l = 1; l <= H.L - 2; ++l)
        for (int mu = 0; mu < 4; ++mu) c.sap[l - 1][mu] = H.lv[l].cg.sap[mu];
      c.batch = H.p.batch;
      return c;
    };
    bool cached = !path.empty() && tune_cache_lookup(path, key, best);
    if (!cached) {
      hipStream_t s = as_stream(stream);
      const long long n = H.lv[0].n;
      DevArray<double2> z;
      z.alloc((size_t)n * nrhs);
      // best of two timed solves after a warm-up one; a solve that does not
      // converge does not count
      auto measure = [&]() {
        double t = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
          vzero<double>(z.p, n * nrhs, s);
          DD_CHECK_HIP(hipStreamSynchronize(s));
          const auto t0 = std::chrono::steady_clock::now();
          const int w = solve_batches(H, b, z.p, nrhs, nullptr, s);
          const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          if (w != DDAMG_OK) return 1e300;
          if (rep > 0) t = std::min(t, dt);
        }
        return t;
      };
      best = current();
      best.batch = std::min(best.batch, nrhs);   // the same grouping, stated as used
      H.p.batch = best.batch;
      best.seconds = measure();
      for (int l = 1; l <= H.L - 2; ++l) {
        for (const auto& cand : sap_candidates(H, l)) {
          TuneChoice c = best;
          for (int mu = 0; mu < 4; ++mu) c.sap[l - 1][mu] = cand[mu];
          try {
            apply(c);
          } catch (const Error&) {
            apply(best);
            continue;
          }
          c.seconds = measure();
          if (c.seconds < best.seconds) best = c;
        }
        apply(best);
      }
      if (nrhs > 1) {
        for (int bt : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}) {
          if (bt > nrhs || bt == best.batch) continue;
          TuneChoice c = best;
          c.batch = bt;
          apply(c);
          c.seconds = measure();
          if (c.seconds < best.seconds) best = c;
        }
      }
      DD_REQUIRE(best.seconds < 1e299, "no candidate configuration converged");
      if (!path.empty()) tune_cache_store(path, key, best);
    }
    apply(best);
    if (out) {
      for (int l = 0; l < 3; ++l)
        for (int mu = 0; mu < 4; ++mu) out->sap_block_l[l][mu] = best.sap[l][mu];
      out->batch = H.p.batch;
      out->seconds = best.seconds;
      out->from_cache = cached ? 1 : 0;
    }
  });
}

int ddamg_cgnr(ddamg_ctx ctx, const void* b, void* z, int nrhs, double tol, int max_iter,
               ddamg_solve_stats* stats, void* stream) {
  int worst = DDAMG_OK;
  int rc = guarded([&] {
    DD_REQUIRE(ctx && ctx->c, "null context");
    DD_REQUIRE(b && z && b != z && nrhs >= 1, "bad argument");
    DD_REQUIRE(tol > 0 && max_iter >= 0, "tol must be > 0 and max_iter >= 0");
    Context& c = *ctx->c;
    const WorkspaceScope wsc(c.ws.get());
    hipStream_t s = as_stream(stream);
    const long long n = c.g.V * 12;
    const int bmax = std::min(nrhs, 16);
    DevArray<double2> nb_, nx_;
    nb_.alloc((size_t)n * bmax);
    nx_.alloc((size_t)n * bmax);
    std::vector<ddamg_solve_stats> st(bmax);
    for (int r0 = 0; r0 < nrhs; r0 += bmax) {
      const int nb = std::min(bmax, nrhs - r0);
      auto t0 = std::chrono::steady_clock::now();
      fine_to_native<double>(c.g, static_cast<const double2*>(b) + r0 * n, nb_.p, nb, s);
      fine_to_native<double>(c.g, static_cast<const double2*>(z) + r0 * n, nx_.p, nb, s);
      cgnr(c, nb_.p, nx_.p, nb, tol, max_iter, st.data(), s);
      fine_from_native<double>(c.g, nx_.p, static_cast<double2*>(z) + r0 * n, nb, s);
      DD_CHECK_HIP(hipStreamSynchronize(s));
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int r = 0; r < nb; ++r) {
        st[r].seconds = secs;
        if (stats) stats[r0 + r] = st[r];
        if (st[r].status != DDAMG_OK && worst == DDAMG_OK) worst = st[r].status;
      }
    }
  });
  if (rc != DDAMG_OK) return rc;
  if (worst == DDAMG_ENOCONV) g_err = "CGNR reached max_iter before tol";
  if (worst == DDAMG_ENONFINITE) g_err = "non-finite value in b or in a residual";
  return worst;
}

int ddamg_export_interpolation(ddamg_hier hier, int level, void* out, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L - 1, "level out of range");
    DD_REQUIRE(out != nullptr, "null output");
    hipStream_t s = as_stream(stream);
    const LevelStore& S = H.lv[level];
    if (level == 0) fine_from_native<double>(H.ctx->g, S.P64.p, static_cast<double2*>(out), S.N, s);
    else vcopy<double, double>(S.P64.p, static_cast<double2*>(out), (long long)S.N * S.n, s);
  });
}

int ddamg_export_coarse_op(ddamg_hier hier, int level, void* out, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 1 && level < H.L, "level out of range (coarse levels are 1..L-1)");
    DD_REQUIRE(out != nullptr, "null output");
    export_coarse(H.lv[level].cview<double>(), static_cast<double2*>(out), as_stream(stream));
  });
}

int ddamg_import_test_vectors(ddamg_hier hier, int level, const void* tv, void* stream) {
  return guarded([&] {
    Hierarchy& H = H_(hier);
    const WorkspaceScope wsc(H.ws.get());
    DD_REQUIRE(level >= 0 && level < H.L - 1, "level out of range");
    DD_REQUIRE(tv != nullptr, "null test vectors");
    H.s = as_stream(stream);
    LevelStore& S = H.lv[level];
    const double2* in = static_cast<const double2*>(tv);
    if (level == 0) fine_to_native<double>(H.ctx->g, in, S.tv64.p, S.N, H.s);
    else vcopy<double, double>(in, S.tv64.p, (long long)S.N * S.n, H.s);
    if (H.p.precond_prec == DDAMG_F32) vcopy<double, float>(S.tv64.p, S.tv32.p, (long long)S.N * S.n, H.s);
    H.build_level(level, false);
  });
}

}  // extern "C"
