// CGNR on the fine Wilson-clover operator (the paper's Krylov comparison
// method, Sec. 4): declarations.
#pragma once

#include "solver.h"

namespace ddamg {

// x (in: initial guess, out: solution) for nb native FP64 fine fields b;
// stops system k when ||b_k - D x_k|| <= tol ||b_k|| (recursive residual,
// confirmed by the recomputed one) or after max_iter iterations; st[k]
// receives status, iterations (outer_iters) and the true relative residual.
void cgnr(Context& ctx, const double2* b, double2* x, int nb, double tol, int max_iter, ddamg_solve_stats* st,
          hipStream_t s);

}  // namespace ddamg
