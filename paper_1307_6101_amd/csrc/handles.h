// The opaque handle types of the C ABI (include/ddamg.h): a context owns
// one lattice operator, a hierarchy handle owns one multilevel hierarchy and
// remembers the context it was built on.
#pragma once

#include <memory>

#include "solver.h"

struct ddamg_ctx_s {
  std::unique_ptr<ddamg::Context> c;
};
struct ddamg_hier_s {
  std::unique_ptr<ddamg::Hierarchy> h;
  ddamg_ctx_s* owner;
};

namespace ddamg {
// Run f, turning a thrown ddamg::Error into its status and the calling
// thread's last-error message (every entry point goes through this).
int guarded_call(void (*f)(void*), void* arg);
template <typename F> int guarded(F&& f) {
  return guarded_call([](void* a) { (*static_cast<F*>(a))(); }, &f);
}
}  // namespace ddamg
