"""The DD-alpha-AMG multilevel method: cycles (Alg. 1, Alg. 2), setup
(Alg. 3, Alg. 4, Fig. 1) and the outer FGMRES solve (Sec. 2, Sec. 3, Tab. 1).

Levels are numbered from 0 here (level 0 is the paper's level 1, D_1 = D).

Readings where the paper is silent or garbled (the same in the GPU library):

* Alg. 3 tests "l = 0" for the random start; levels start at 1, so the
  random test vectors enter on the finest level.
* Alg. 3 stores the smoothed iterate as the level's test vector, unnormalised.
* Alg. 4 runs the K-cycle of level l with that level's own test vector as
  right-hand side (Fig. 1: the current test vector is the right-hand side),
  and z_k for k > l is the approximate level-k solution computed last during
  that cycle (the result of the most recent coarse solve on level k).
* The setup driver is initial_setup(finest) followed by
  iterative_setup(finest, i) for i = 1..n_inv.
* The K-cycle's "maximal restarts 2" is read as at most 2 restart cycles of
  length 5 (at most 10 iterations).
* When a level has more test vectors than the one above, the extra ones are
  fresh random vectors (passed in).
"""
from __future__ import annotations

import numpy as np

from .aggregation import Aggregation
from .galerkin import galerkin
from .krylov import OddEvenCoarsest, fgmres, norm
from .sap import sap_sweep, validate_blocks


class Hierarchy:
    def __init__(self, fine_op, params, cycle="K"):
        self.p = dict(params)
        self.L = int(self.p["levels"])
        self.ops = [fine_op] + [None] * (self.L - 1)
        self.aggs = [None] * (self.L - 1)
        self.tv = [None] * (self.L - 1)
        self.coarsest = None
        self.cycle_type = cycle
        # SAP block shape per smoothed level (levels 0..L-2); a level whose
        # 2^4 blocks would come in odd counts takes e.g. 3^4 blocks
        base = tuple(self.p.get("sap_block", (2, 2, 2, 2)))
        self.blocks = [tuple(b) for b in self.p.get("sap_blocks", [base] * (self.L - 1))]
        dims = fine_op.dims
        for l in range(self.L - 1):
            validate_blocks(dims, self.blocks[l])
            agg = self.p["agg"][l]
            dims = tuple(d // a for d, a in zip(dims, agg))
        self.counters = {"coarsest_iters": 0, "kcycle_iters": 0}
        # Optional replacement of the SAP block solves: a callable
        # (level, operator, block shape) -> block solver for sap_sweep.  The
        # tests pass exact dense block inverses, which make the smoother a
        # linear map with a closed form; None keeps the MR block solves.
        self.block_solver_factory = None

    # -- smoothing ---------------------------------------------------------
    def smooth(self, l, b, z, n):
        bs = None
        if self.block_solver_factory is not None and n > 0:
            bs = self.block_solver_factory(l, self.ops[l], self.blocks[l])
        for _ in range(n):
            z = sap_sweep(self.ops[l], b, z, self.blocks[l], self.p["mr_iters"], block_solver=bs)
        return z

    # -- Alg. 1 / Alg. 2 -----------------------------------------------------
    def cycle(self, l, b, record=None):
        """One application of the level-l cycle to b: K-cycle (Alg. 2), V-cycle
        (Alg. 1) or W-cycle (Alg. 1 with two level-(l+1) cycles, the second
        on the residual of the first)."""
        op = self.ops[l]
        z = np.zeros_like(b)
        z = self.smooth(l, b, z, self.p["mu"])
        r = b - op.apply(z) if self.p["mu"] > 0 else b
        bc = self.aggs[l].restrict(r)
        if l + 1 == self.L - 1:
            st = {}
            zc = self.coarsest.solve(bc, stats=st)
            self.counters["coarsest_iters"] += st.get("iters", 0)
        elif self.cycle_type == "K":
            st = {}
            zc = fgmres(self.ops[l + 1].apply, bc,
                        lambda v: self.cycle(l + 1, v, record),
                        self.p["kc_len"], self.p["kc_restarts"], self.p["kc_tol"], stats=st)
            self.counters["kcycle_iters"] += st.get("iters", 0)
        elif self.cycle_type == "W":
            # two cycles on level l+1, the second on the residual of the first
            zc = self.cycle(l + 1, bc, record)
            zc = zc + self.cycle(l + 1, bc - self.ops[l + 1].apply(zc), record)
        else:
            zc = self.cycle(l + 1, bc, record)
        if record is not None:
            record[l + 1] = zc
        z = z + self.aggs[l].prolong(zc)
        return self.smooth(l, b, z, self.p["nu"])

    # -- construct P_l and D_{l+1} -------------------------------------------
    def build_level(self, l):
        self.aggs[l] = Aggregation(self.ops[l].dims, self.p["agg"][l], self.tv[l])
        self.ops[l + 1] = galerkin(self.ops[l], self.aggs[l])
        if l + 1 == self.L - 1:
            self.coarsest = OddEvenCoarsest(self.ops[l + 1], self.p["coarse_eps"],
                                            self.p.get("coarse_restart", 30),
                                            self.p.get("coarse_max_restarts", 10))


def initial_setup(H, l, tv0, extra=None):
    """Alg. 3 on level l: restrict (or take random) test vectors, smooth each
    one eta-fold from zero for eta = 1, 2, 3, construct P_l and D_{l+1},
    recurse."""
    N = H.p["ntv"][l]
    if l == 0:
        v = [np.array(x, dtype=np.complex128) for x in tv0[:N]]
    else:
        v = [H.aggs[l - 1].restrict(x) for x in H.tv[l - 1]][:N]
        if len(v) < N:
            v += [np.array(x, dtype=np.complex128) for x in extra[l]][: N - len(v)]
    for eta in (1, 2, 3):
        for j in range(N):
            x = np.zeros_like(v[j])
            x = H.smooth(l, v[j], x, eta)
            v[j] = x
    H.tv[l] = np.stack(v)
    H.build_level(l)
    if l < H.L - 2:
        initial_setup(H, l + 1, tv0, extra)


def iterative_setup(H, l, i):
    """Alg. 4 on level l, iteration i: one cycle per test vector updates the
    test vectors of levels l..L-2, P and D are rebuilt there, then the next
    level runs i times."""
    if l >= H.L - 1:
        return
    N = H.p["ntv"][l]
    for j in range(N):
        rec = {}
        rec[l] = H.cycle(l, H.tv[l][j], rec)
        for k in range(l, H.L - 1):
            if j < H.tv[k].shape[0]:
                H.tv[k][j] = rec[k] / norm(rec[k])
    for k in range(l, H.L - 1):
        H.build_level(k)
    for q in range(1, i + 1):
        iterative_setup(H, l + 1, q)


def build_hierarchy(fine_op, params, tv0, extra=None, cycle="K"):
    H = Hierarchy(fine_op, params, cycle)
    initial_setup(H, 0, tv0, extra)
    for i in range(1, int(H.p["n_inv"]) + 1):
        iterative_setup(H, 0, i)
    return H


def solve(H, b, x0=None, max_restarts=200, stats=None):
    """Outer FGMRES (restart n_kv, tolerance tol, true-residual check)
    preconditioned by the level-0 cycle."""
    st = {} if stats is None else stats
    H.counters = {"coarsest_iters": 0, "kcycle_iters": 0}
    x = fgmres(H.ops[0].apply, b, lambda v: H.cycle(0, v), H.p["nkv"], max_restarts,
               H.p["tol"], x0=x0, check_true_residual=True, stats=st)
    st.update(H.counters)
    st["true_relres"] = norm(b - H.ops[0].apply(x)) / norm(b)
    return x
