/*
 * ddamg.h -- C ABI of the MI355X (gfx950) DD-alpha-AMG library.
 *
 * Solves the lattice Wilson(-clover) Dirac system D z = b (Frommer, Kahl,
 * Krieg, Leder, Rottmann, arXiv:1307.6101, Sec. 1 eq. (1)) with FGMRES
 * preconditioned by the adaptive-aggregation domain-decomposition multilevel
 * method (Sec. 2: Alg. 1 V-cycle, Alg. 2 K-cycle, Alg. 3 / Alg. 4 setup;
 * Sec. 3 and Tab. 1: parameters, single-precision preconditioner inside a
 * double-precision outer FGMRES, odd-even GMRES on the coarsest level).
 *
 * Conventions used by every call
 * ------------------------------
 * Lattice.  dims = {X, Y, Z, T}, periodic in all four directions; direction
 *   mu = 0,1,2,3 is x,y,z,t.  Canonical site index i = x + X*(y + Y*(z + Z*t)).
 * Operator.  (D psi)(x) = (m0+4) psi(x)
 *     - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^H psi(x-mu)]
 *     - c_sw/32 sum_{mu,nu} g_mu g_nu (Q_mu,nu(x) - Q_nu,mu(x)) psi(x),
 *   chiral gamma basis with Gamma5 = diag(1,1,-1,-1) (the paper's Gamma5:
 *   +1 on spins 1,2, -1 on spins 3,4), Q_mu,nu the four-leaf clover.
 * Complex numbers are interleaved (re, im).
 * Canonical layouts (DDAMG_CANONICAL, always complex128):
 *   links        [V][4 mu][3][3] row-major (U_mu(x) couples x to x+mu)
 *   fine spinor  [nrhs][V][4 spin][3 colour]
 *   level-l field [nrhs][V_l][2N]: components 0..N-1 carry Gamma5 = +1,
 *                N..2N-1 carry Gamma5 = -1 (coarse site = aggregate, in the
 *                canonical order of the coarse lattice)
 *   coarse operator [V_l][9][2N][2N] row-major, blocks self, +x,+y,+z,+t,
 *                -x,-y,-z,-t: (D_l v)(x) = sum_k B_k(x) v(x + d_k)
 * Native layouts (DDAMG_NATIVE) are the library's internal ones, at the
 *   precision of the call (F64: complex128, F32: complex64):
 *   fine field   [nrhs][V/16][12][16]: 2^4 blocks of sites; site (x,y,z,t)
 *                has local index (x&1)+2(y&1)+4(z&1)+8(t&1) in block
 *                (x/2,y/2,z/2,t/2); blocks are numbered tile-major: a tile is
 *                the 2x2x2x2 blocks of one 4^4 brick (block bits in the same
 *                order inside the tile); tiles in a Morton-like order: level
 *                by level, each direction whose remaining tile count is even
 *                gives one binary digit (finest level first, x lowest), the
 *                rest lexicographic (x fastest)
 *   level-l field (l >= 1) [nrhs][V_l][2N] (canonical order)
 *   Use ddamg_to_native / ddamg_from_native to convert.
 * Levels are numbered from 0 (the fine lattice; the paper's level 1).
 * Memory.  Every pointer argument named in/out/b/z/links/tv is a DEVICE
 *   pointer owned by the caller; the library never frees it.  Handles made by
 *   ddamg_create / ddamg_build_hierarchy own the library's device memory
 *   (operators, interpolations, Krylov bases) and free it on destroy.
 *   Handles made by ddamg_create_ws / ddamg_build_hierarchy_ws instead carve
 *   all their device memory out of a caller-owned workspace, whose size
 *   ddamg_workspace_bytes returns; they own only small host state (pinned
 *   staging words, events, captured graphs).
 * Streams.  `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 *   on it and return without waiting, except ddamg_create,
 *   ddamg_build_hierarchy and ddamg_solve, which return when done.
 * Errors.  Every int-returning call returns DDAMG_OK or a negative status;
 *   arguments are checked on the host before anything is launched, and
 *   ddamg_last_error() then describes the failure (thread-local string).
 */
#ifndef DDAMG_H
#define DDAMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DDAMG_OK = 0,
  DDAMG_EINVAL = -1,        /* bad argument, shape or parameter */
  DDAMG_ENOMEM = -2,        /* device allocation failed */
  DDAMG_EHIP = -3,          /* a HIP runtime call failed */
  DDAMG_ENOCONV = -4,       /* solve hit max_restarts before tol */
  DDAMG_ENONFINITE = -5,    /* NaN / Inf in b or in a residual */
  DDAMG_EUNSUPPORTED = -6   /* valid request this build does not implement */
};

/* Precision of a call.  F64 and F32: arithmetic (and storage) precision.
 * F16: IEEE binary16 storage of the operator data (links, clover, P_l, D_l)
 * with FP32 arithmetic and FP32 native vectors (Sec. 3 runs the
 * preconditioner in single precision; the half-precision storage is this
 * library's); on a hierarchy it needs half_storage = 1. */
/* F16S: F16 with the fine-level spinors too in binary16, one FP32 scale per
 * site (the storage of params.half_spinors), for level 0 only: in
 * ddamg_to_native / ddamg_from_native (canonical complex128 <-> the native
 * FP16 form), and in ddamg_sap_smooth, ddamg_restrict (canonical or native
 * layout) and ddamg_prolong (canonical layout; fine += the FP16-encoded
 * P coarse) on a hierarchy built with half_spinors = 1.  The native FP16
 * form of nrhs fine fields is one buffer: the entries of all fields
 * ([nrhs][V/16][12][16] binary16 pairs (re, im), each site's 12 components
 * divided by their largest |re|, |im|) followed by the site scales
 * ([nrhs][V/16][16] float, that largest value); a restriction's coarse
 * output is native FP32. */
enum { DDAMG_F64 = 0, DDAMG_F32 = 1, DDAMG_F16 = 2, DDAMG_F16S = 3 };
enum { DDAMG_CANONICAL = 0, DDAMG_NATIVE = 1 };   /* vector layout */
enum { DDAMG_KCYCLE = 0, DDAMG_VCYCLE = 1, DDAMG_WCYCLE = 2 };  /* Alg. 2 / Alg. 1 / Alg. 1 with
                                                                 two coarse cycles per level */

typedef struct ddamg_ctx_s* ddamg_ctx;    /* one lattice operator D */
typedef struct ddamg_hier_s* ddamg_hier;  /* a multilevel hierarchy for D */

typedef struct {
  int dims[4];     /* X, Y, Z, T; each a multiple of 4 */
  double m0;       /* bare mass */
  double csw;      /* clover coefficient (0 = Wilson) */
} ddamg_lattice;

/* Method parameters; ddamg_params_default() fills the paper's Tab. 1. */
typedef struct {
  int levels;                 /* L >= 2 */
  int agg[3][4];              /* aggregate (lattice-block) shape, level l -> l+1 */
  int ntv[3];                 /* test vectors N on level l (l < L-1) */
  int sap_block[4];           /* SAP block shape (2^4; the fine level always 2^4) */
  int mu, nu;                 /* pre- / post-smoothing steps (0 / 5) */
  int mr_iters;               /* MR iterations per SAP block solve (3) */
  int n_inv;                  /* iterative setup iterations (6) */
  double coarse_eps;          /* coarsest relative residual (5e-2) */
  int coarse_restart;         /* coarsest GMRES restart length (30) */
  int coarse_max_restarts;    /* coarsest GMRES restart cycles (10) */
  int kc_len;                 /* K-cycle FGMRES length (5) */
  int kc_restarts;            /* K-cycle FGMRES restart cycles (2) */
  double kc_tol;              /* K-cycle relative residual (1e-1) */
  int nkv;                    /* outer FGMRES restart length (10) */
  double tol;                 /* outer relative residual (1e-10) */
  int max_restarts;           /* outer restart cycles before DDAMG_ENOCONV */
  int precond_prec;           /* DDAMG_F32 (mixed) or DDAMG_F64 (plain) */
  int cycle;                  /* DDAMG_KCYCLE, DDAMG_VCYCLE, or DDAMG_WCYCLE: on an
                                 intermediate level the coarse system gets two
                                 cycles, the second on the residual of the
                                 first (a fixed count, like the V-cycle) */
  int half_storage;           /* 0: the preconditioner's operator data (fine
                                 links and clover, every P_l, every coarse D_l)
                                 are stored at precond_prec.  1: stored as IEEE
                                 binary16 and widened to FP32 on load, the
                                 arithmetic staying FP32 (needs precond_prec =
                                 DDAMG_F32); the hierarchy's FP32 level
                                 operations (apply_Dc, restrict, prolong,
                                 sap_smooth with prec = DDAMG_F32) then read
                                 these FP16 copies too.  Orthonormalisation,
                                 Galerkin products and the outer solver
                                 always use the FP64 masters. */
  int batch;                  /* largest number of systems advanced together
                                 (1..32, default 16): the right-hand sides of
                                 one ddamg_solve call go through the solver in
                                 batches of this size, and so do the test
                                 vectors of a level in the setup.  Batched
                                 systems share every launch but keep their own
                                 Krylov scalars and stopping tests. */
  int sap_block_l[3][4];      /* SAP block shape on coarse level l = 1..3 (row
                                 l-1); a row with a zero entry takes
                                 sap_block.  Lets a level whose extents give
                                 an odd count of 2^4 blocks use e.g. 3^4
                                 blocks (Sec. 2: the blocks of one colour
                                 must not touch). */
  int half_directions;        /* 1: the outer FGMRES keeps its preconditioned
                                 directions Z_j in FP16 with one FP32 scale
                                 per site (the largest |re|, |im| of the
                                 site's 12 components) instead of FP32, and
                                 applies D to exactly the stored values (the
                                 flexible Arnoldi relation stays exact); about
                                 half the memory of Z, for the largest
                                 lattices, at the price of more outer
                                 iterations.  Needs precond_prec = DDAMG_F32.
                                 0 (default): FP32 directions. */
  int graph;                  /* 1: ddamg_solve applies the preconditioner by
                                 replaying a HIP graph captured once per batch
                                 size (no host round trip inside a cycle).
                                 The coarsest GMRES then keeps its Krylov
                                 scalars (Hessenberg matrix, Givens rotations,
                                 stopping test) on the device and issues a
                                 fixed sequence of launches: coarse_restart
                                 steps in each of coarse_max_restarts cycles,
                                 the steps after a system has reached
                                 coarse_eps changing nothing, so results equal
                                 those of the host-driven solve up to
                                 rounding while costing the full launch
                                 count.  Needs the V- or W-cycle when levels >= 3
                                 (the K-cycle's stopping tests are data
                                 dependent).  0 (default): host-driven. */
  int coarse_dense;           /* 1 (default): on a coarsest level whose
                                 odd-even Schur system S = D_oo - D_oe
                                 D_ee^-1 D_eo (Sec. 3) is small (at most
                                 2048 unknowns and at most twice the entries
                                 of the level's sparse blocks) the setup forms
                                 S as a dense matrix (FP64, with an FP32 copy
                                 that the FP32 and FP16-storage solves use)
                                 and the coarsest GMRES applies it with one
                                 launch instead of the three-launch sparse
                                 product; results agree up to rounding.
                                 0: always the sparse product. */
  int galerkin_cols;          /* columns of P a workgroup of the coarse
                                 Galerkin product D_{l+1} = P_l^H D_l P_l
                                 (l >= 1) applies each loaded operator entry
                                 to: 1 or 4; 0 (default) takes 4 where the
                                 level has aggregates enough to fill the
                                 device with a quarter of the workgroups,
                                 else 1.  The result is the same up to
                                 rounding either way. */
  int profile_levels;         /* 1: ddamg_solve records GPU events where
                                 the work moves between levels and reports
                                 the time consumed on each level (the
                                 per-level times of the paper's Tab. 4) in
                                 ddamg_solve_stats.t_level_s; costs a few
                                 microseconds per level change.  Not with
                                 graph = 1 (the times stay 0).  0: off. */
  int half_spinors;           /* 1: the fine-level vectors of the solve's
                                 preconditioner (the cycle's right-hand side
                                 and its result, which the SAP colour passes,
                                 the restriction and the prolongation read
                                 and write) are stored in FP16 with one FP32
                                 scale per site, like half_directions (which
                                 it implies), and the arithmetic stays FP32.
                                 The FP16 storage of links and spinors that
                                 halves the bytes of the smoother (Sec. 3
                                 puts the whole preconditioner in single
                                 precision; going to half precision storage
                                 is this library's).  Needs precond_prec =
                                 DDAMG_F32, half_storage = 1, mu = 0 and
                                 graph = 0; the setup keeps FP32 vectors.
                                 0 (default): FP32 vectors. */
} ddamg_params;

typedef struct {
  int status;                 /* DDAMG_OK, DDAMG_ENOCONV or DDAMG_ENONFINITE */
  int outer_iters;            /* outer FGMRES iterations (preconditioner calls) */
  int restarts;               /* outer restart cycles */
  long long kcycle_iters;     /* FGMRES iterations on levels 1..L-2 */
  long long coarsest_iters;   /* GMRES iterations on the coarsest level */
  double true_relres;         /* ||b - D z|| / ||b||, recomputed in FP64 */
  double seconds;             /* wall time of the call */
  double err_vs_ref;          /* ||z - z_ref|| / ||z_ref|| in FP64 for
                                 ddamg_solve_ex with a reference solution
                                 (Sec. 3.4 reports the error against a known
                                 solution), else -1 */
  double t_setup_s;           /* wall time of the hierarchy's setup */
  double t_level_s[4];        /* GPU time consumed on level 0..3 during the
                                 solve of this record's batch (with
                                 params.profile_levels), else 0 */
  double bytes;               /* algorithmic bytes of the batch's solve: the
                                 compulsory traffic of every operator, smoother,
                                 transfer and Krylov vector operation counted
                                 from their per-site sizes (an estimate, not
                                 a measurement) */
  double flops;               /* algorithmic flops of the batch's solve,
                                 counted the same way */
  int coarsest_dense;         /* order of the dense Schur matrix of the
                                 coarsest level (0: sparse product) */
} ddamg_solve_stats;

/* Fill p with the defaults of Tab. 1 for `levels` levels (agg 4^4 then 2^4,
 * N = 20, SAP blocks 2^4, 3 MR steps, mu = 0, nu = 5, n_inv = 6, eps = 5e-2,
 * K-cycle length 5 / 2 cycles / 1e-1, n_kv = 10, tol = 1e-10, FP32
 * preconditioner, K-cycle). */
void ddamg_params_default(ddamg_params* p, int levels);

/* Description of the last failure on the calling thread ("" if none). */
const char* ddamg_last_error(void);

/* Library version string. */
const char* ddamg_version(void);

/* Create the operator D (Sec. 1 eq. (1)) on one lattice.  `links` is a device
 * pointer to the canonical complex128 links; they are copied (the caller may
 * free them afterwards).  The clover term is built on the device in FP64 and
 * kept in FP64 and FP32 next to the links.  EINVAL unless every extent is a
 * positive multiple of 4. */
int ddamg_create(const ddamg_lattice* lat, const void* links, void* stream, ddamg_ctx* out);

/* Workspace sizes for caller-owned device memory.  *ctx_bytes (if non-NULL)
 * receives the bytes a context on `lat` made by ddamg_create_ws keeps: the
 * links and clover term in FP64 and FP32 (Sec. 1 eq. (1)), their FP16 copies
 * when params is non-NULL with half_storage = 1, the neighbour tables, and
 * scratch for canonical-layout ddamg_apply_D calls of up to nrhs_max fields.
 * *hier_bytes (if non-NULL; needs params) receives the bytes a hierarchy built
 * with these params by ddamg_build_hierarchy_ws keeps: P_l, D_{l+1} and the
 * test vectors of every level (Sec. 2), the setup's work (Alg. 3 and 4), and
 * the work of solves, preconditioner and canonical-layout level calls at the
 * hierarchy's precision on batches of up to nrhs_max right-hand sides (the
 * outer FGMRES bases of Sec. 3, the K-cycle bases of Alg. 2, the coarsest
 * GMRES basis, SAP scratch).  The count runs the same allocation sequence
 * as the build, against a counter, so it is exact; it needs no GPU.  EINVAL
 * for an invalid lattice or params, or nrhs_max < 1. */
int ddamg_workspace_bytes(const ddamg_lattice* lat, const ddamg_params* params, int nrhs_max,
                          size_t* ctx_bytes, size_t* hier_bytes);

/* ddamg_create with all device memory carved out of `workspace` (a device
 * pointer aligned to 256 bytes, ws_bytes long, owned by the caller, which must
 * keep it allocated until ddamg_destroy has returned).  params (nullable) and
 * nrhs_max must be those given to ddamg_workspace_bytes; EINVAL if ws_bytes is
 * below its *ctx_bytes.  Calls that need more than was counted (ddamg_cgnr's
 * vectors, ddamg_apply_D on more than nrhs_max fields in canonical layout)
 * take it from the rest of the workspace and fail with ENOMEM when it runs
 * out. */
int ddamg_create_ws(const ddamg_lattice* lat, const void* links, const ddamg_params* params, int nrhs_max,
                    void* workspace, size_t ws_bytes, void* stream, ddamg_ctx* out);
void ddamg_destroy(ddamg_ctx ctx);

/* out = D in for nrhs fine fields (eq. (1)), computed at `prec`.  With
 * DDAMG_CANONICAL, in/out are complex128 canonical spinors; with
 * DDAMG_NATIVE they are native fine fields at `prec`.  in and out must not
 * overlap. */
int ddamg_apply_D(ddamg_ctx ctx, const void* in, void* out, int nrhs, int prec, int layout,
                  void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as ddamg_apply_D with DDAMG_CANONICAL, but the native staging
 * fields live in a fixed array of DDAMG_NOALLOC_SCRATCH_BYTES bytes in the
 * library's device data (one per GPU, held until the process ends) instead
 * of memory the library allocates.  No call allocates.  in/out: device
 * pointers to nrhs canonical complex128 spinors, caller-owned, distinct.
 * EINVAL when 2 * nrhs * V * 12 * (16 bytes for F64, 8 for F32) exceeds
 * DDAMG_NOALLOC_SCRATCH_BYTES.  Every call on a GPU uses that GPU's one
 * array, whatever the context: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  The
 * staging is fully overwritten by each call (nothing needs clearing). */
#define DDAMG_NOALLOC_SCRATCH_BYTES (64u << 20)
int ddamg_apply_D_noalloc(ddamg_ctx ctx, const void* in, void* out, int nrhs, int prec, void* stream);

/* Canonical complex128 <-> native (at prec) conversion of nrhs fields of
 * level `level` (level 0 needs only ctx; level >= 1 needs hier, else pass
 * NULL). */
int ddamg_to_native(ddamg_ctx ctx, ddamg_hier hier, int level, const void* in, void* out,
                    int nrhs, int prec, void* stream);
int ddamg_from_native(ddamg_ctx ctx, ddamg_hier hier, int level, const void* in, void* out,
                      int nrhs, int prec, void* stream);

/* Build the multilevel hierarchy (Sec. 2.2: Alg. 3 initial phase on every
 * level, then Alg. 4 iterative phase for i = 1..n_inv).  `tv` holds the
 * ntv[0] random initial test vectors as canonical complex128 fine spinors
 * ([ntv[0]][V][12], device); where a coarser level has more test vectors than
 * the level above, the extra ones are taken from `tv_extra` (canonical
 * complex128 fields of that level, concatenated level by level; NULL if
 * none).  Smoothing and cycles run at params->precond_prec; orthonormalisation
 * and the Galerkin products D_{l+1} = P_l^H D_l P_l run in FP64.  EINVAL
 * when a level's extents are not divisible by its aggregate or SAP block
 * shape, a SAP block count per direction is odd, or N exceeds an aggregate's
 * dimension. */
int ddamg_build_hierarchy(ddamg_ctx ctx, const ddamg_params* params, const void* tv,
                          const void* tv_extra, void* stream, ddamg_hier* out);

/* ddamg_build_hierarchy with all of the hierarchy's device memory carved out
 * of `workspace` (device, 256-byte aligned, ws_bytes long, caller-owned and
 * kept allocated until ddamg_destroy_hierarchy has returned): what
 * ddamg_workspace_bytes(lattice of ctx, params, nrhs_max) counts in
 * *hier_bytes, all of it allocated before the setup starts, so that solves
 * and preconditioner calls on up to nrhs_max right-hand sides allocate
 * nothing.  EINVAL if ws_bytes is below that count.  Work beyond the count
 * (level calls at the other precision, ddamg_tune's solution vectors, a
 * larger SAP block set by ddamg_set_sap_block) takes memory from the rest of
 * the workspace and fails with ENOMEM when it runs out. */
int ddamg_build_hierarchy_ws(ddamg_ctx ctx, const ddamg_params* params, const void* tv, const void* tv_extra,
                             int nrhs_max, void* workspace, size_t ws_bytes, void* stream, ddamg_hier* out);
void ddamg_destroy_hierarchy(ddamg_hier hier);

/* Lattice extents and components per site of level `level` (Sec. 2: level
 * l+1 has one site per aggregate of level l and 2 N_l components, the two
 * chirality halves of the N_l test vectors). */
int ddamg_level_info(ddamg_hier hier, int level, int dims_out[4], int* dof_out);

/* out = D_level in for nrhs level-`level` fields (level >= 1: the Galerkin
 * operator of Sec. 1; level 0: D).  Layout as for ddamg_apply_D. */
int ddamg_apply_Dc(ddamg_hier hier, int level, const void* in, void* out, int nrhs, int prec,
                   int layout, void* stream);

/* coarse = P_level^H fine (Alg. 1, restriction) and fine += P_level coarse
 * (Alg. 1, interpolation), level = 0 .. L-2. */
int ddamg_restrict(ddamg_hier hier, int level, const void* fine, void* coarse, int nrhs,
                   int prec, int layout, void* stream);
int ddamg_prolong(ddamg_hier hier, int level, const void* coarse, void* fine, int nrhs,
                  int prec, int layout, void* stream);

/* nsweeps SAP steps z <- z + M (b - D z) on level `level` (Sec. 2; Tab. 1:
 * red-black lattice blocks, mr_iters MR steps per block solve, colour 0
 * first).  z is read and overwritten. */
int ddamg_sap_smooth(ddamg_hier hier, int level, const void* b, void* z, int nsweeps, int nrhs,
                     int prec, int layout, void* stream);

/* One application of the level-0 cycle (the preconditioner) to b: z = C(b)
 * (Alg. 2, or Alg. 1 with params.cycle = DDAMG_VCYCLE), for nrhs fields
 * (batches of at most params.batch). */
int ddamg_precondition(ddamg_hier hier, const void* b, void* z, int nrhs, int layout,
                       void* stream);

/* Solve D z = b (Sec. 1 eq. (1)) for nrhs canonical complex128 right-hand
 * sides with FGMRES (restart nkv, double precision) preconditioned by the
 * cycle computed in single precision (Sec. 3, opening paragraph), to
 * ||b - D z|| <= tol ||b|| (checked on the recomputed residual).  z holds the
 * initial guess on entry (zeros for none) and the solution on return.
 * The right-hand sides go through in batches of params.batch: every launch
 * serves the whole batch while each system keeps its own Krylov scalars,
 * stopping tests and restarts (at every level), so each result is the one
 * a solve of that system alone gives, up to rounding.  stats (host, may be
 * NULL) receives one record per right-hand side; `seconds` is the wall
 * time of its batch.  A restart cycle that reduces a system's recomputed
 * residual by less than 0.1 % ends that system (stagnation: a tolerance
 * below what FP64 reaches, or a preconditioner that does not help) with
 * DDAMG_ENOCONV instead of running out its restarts.  Returns DDAMG_ENOCONV
 * / DDAMG_ENONFINITE if any right-hand side did (a non-finite inner
 * residual fails the whole batch). */
int ddamg_solve(ddamg_hier hier, const void* b, void* z, int nrhs, ddamg_solve_stats* stats,
                void* stream);

/* ddamg_solve with a reference solution (the error protocol of Sec. 3.4:
 * b = D z_ref for a known z_ref): z_ref (device, nrhs canonical complex128
 * fields, or NULL) gives stats[r].err_vs_ref = ||z_r - z_ref_r|| /
 * ||z_ref_r||, computed in FP64 on the device after the solve.  Otherwise
 * identical to ddamg_solve. */
int ddamg_solve_ex(ddamg_hier hier, const void* b, void* z, int nrhs, const void* z_ref,
                   ddamg_solve_stats* stats, void* stream);

/* ddamg_solve (Sec. 1 eq. (1), Sec. 3) for several independent systems on
 * different lattices (an uneven batch: the sizes,
 * links, masses and hierarchy parameters of the n hierarchies may all
 * differ), solved concurrently.  System i is ddamg_solve(hiers[i], b[i],
 * z[i], nrhs[i], ...) with the same arguments, layout, ownership and result:
 * b[i], z[i] are device pointers to nrhs[i] canonical complex128 fields of
 * hiers[i]'s fine lattice, z[i] holding the initial guess.  Each hierarchy
 * runs on a stream of its own (created on first use, default priority,
 * destroyed with the hierarchy) driven by its own host thread, so the
 * kernels of the systems overlap on the device; all of them start after
 * the work already enqueued on `stream`.  stats (host, may be NULL) holds
 * sum(nrhs) records, those of system i after those of systems 0..i-1.
 * Synchronous: returns when every system is done.  1 <= n <=
 * DDAMG_MAX_SYSTEMS; every hierarchy at most once (DDAMG_EINVAL otherwise);
 * hierarchies may share a context.  Returns the first failure of the
 * library (message names the system), else DDAMG_ENOCONV /
 * DDAMG_ENONFINITE if any system did, else DDAMG_OK.  The hierarchies must
 * not be used by other calls while this one runs. */
#define DDAMG_MAX_SYSTEMS 64
int ddamg_solve_many(int n, const ddamg_hier* hiers, const void* const* b, void* const* z, const int* nrhs,
                     ddamg_solve_stats* stats, void* stream);

/* The uneven batch as one graph (the per-system solve of ddamg_solve, Sec. 1
 * eq. (1) and Sec. 3, with Alg. 1's V-cycle or the W-cycle as
 * preconditioner): n systems on their own lattices and hierarchies, one
 * canonical complex128 right-hand side b[i] and initial guess / solution
 * z[i] (device) each.  Every system's outer FGMRES keeps its Krylov scalars
 * (Hessenberg matrix, Givens rotations, stopping test) on the device, so one
 * outer step -- preconditioner, D, Gram-Schmidt -- is a fixed launch
 * sequence; the steps of all n systems are captured into one HIP graph per
 * step index (the systems side by side on the hierarchies' own streams), and
 * the end of a restart cycle (solution update, recomputed FP64 residual,
 * restart decision) into one more.  The host replays them, reading after
 * each step the systems' device-written convergence flags: a system that has
 * converged keeps running with zero coefficients and zero basis vectors,
 * and the cycle ends when none is live.  Accepts only the recomputed
 * residual ||b - D z|| <= tol ||b|| (as ddamg_solve).  Needs every hierarchy
 * built with graph = 1 (V- or W-cycle for levels >= 3), precond_prec =
 * DDAMG_F32, half_spinors = half_directions = 0 and one n_kv for all.  The
 * graphs are captured on the first call for a list of hierarchies and kept
 * (by hiers[0]) for the next calls with the same list.  stats (host, may be
 * NULL) receives n records.  Synchronous.  Returns as ddamg_solve_many. */
int ddamg_solve_batch(int n, const ddamg_hier* hiers, const void* const* b, void* const* z,
                      ddamg_solve_stats* stats, void* stream);

/* Change the SAP block shape of coarse level `level` (1 .. levels-2, the
 * coarse levels smoothed by SAP; Tab. 1's default is 2^4 blocks on every
 * level, Sec. 2 only requires a red-black block decomposition)
 * smoothed coarse levels) for the solves from now on; the hierarchy (test
 * vectors, P, D_c), built with the earlier shape, is kept.  The shape must
 * tile the level with an even block count per direction (Sec. 2).  Not
 * stream-ordered: waits for the device. */
int ddamg_set_sap_block(ddamg_hier hier, int level, const int block[4]);
/* Change params.batch (1..32), the number of right-hand sides of ddamg_solve
 * that advance together, for the solves from now on. */
int ddamg_set_batch(ddamg_hier hier, int batch);

typedef struct {
  int sap_block_l[3][4];   /* chosen SAP block of coarse levels 1..3 (rows
                              beyond levels-2 are 0) */
  int batch;               /* chosen batch size */
  double seconds;          /* solve time measured for the choice */
  int from_cache;          /* 1: read from the cache, no measurement */
} ddamg_tune_result;

/* Autotuner of choices the method leaves open (the coarse-level SAP block
 * shapes, for which Tab. 1 gives only the default, and the right-hand side
 * batch).
 * Times complete solves of the nrhs canonical complex128
 * right-hand sides b (device) with every candidate SAP block shape of each
 * smoothed coarse level (equal extents in x, y, z and a free extent in t,
 * dividing the level with an even count per direction, block volume 8..512;
 * one level after the other), then, for nrhs > 1, every batch size up to
 * min(nrhs, 32); keeps the fastest choice that converges (best of two
 * timed solves after a warm-up) and applies it to the hierarchy.  With a
 * cache file (may be NULL) the choice is looked up first under a key made
 * of the device architecture, lattice, precisions, levels, aggregates,
 * test-vector counts, cycle and nrhs, and stored there after a search
 * (a JSON object, one entry per line).  Synchronous; allocates a work
 * field of nrhs fine fields.  out (host, may be NULL) receives the choice. */
int ddamg_tune(ddamg_hier hier, const void* b, int nrhs, const char* cache_path, ddamg_tune_result* out,
               void* stream);

/* CGNR, the Krylov method the paper compares against (Sec. 4, Tab. 5; its
 * iteration count is the conditioning indicator of Tab. 2): conjugate
 * gradients on D^H D z = D^H b with the residual r = b - D z, all in double
 * precision, D^H applied as Gamma5 D Gamma5.  b, z: device pointers to nrhs
 * canonical complex128 fine fields of the context's lattice; z holds the
 * initial guess on entry and the solution on return.  Stops a system when
 * ||b - D z|| <= tol ||b|| (the recursive residual, confirmed by the
 * recomputed one) or after max_iter iterations.  Right-hand sides advance
 * in batches of up to 16 with their own scalars.  stats (host, may be NULL)
 * receives one record per right-hand side (outer_iters = CG iterations,
 * true_relres, seconds of its batch).  Synchronous; work buffers are
 * allocated per call.  Returns DDAMG_ENOCONV / DDAMG_ENONFINITE if any
 * system did. */
int ddamg_cgnr(ddamg_ctx ctx, const void* b, void* z, int nrhs, double tol, int max_iter,
               ddamg_solve_stats* stats, void* stream);

/* Export the orthonormalised interpolation basis of level `level` (P_l of
 * Sec. 2: the test vectors split by chirality on each aggregate and
 * orthonormalised) as
 * ntv[level] canonical complex128 fields of that level ([N][V_l][d_l]), and
 * the coarse operator D_{level} (level >= 1) in the canonical coarse layout. */
int ddamg_export_interpolation(ddamg_hier hier, int level, void* out, void* stream);
int ddamg_export_coarse_op(ddamg_hier hier, int level, void* out, void* stream);

/* Replace the test vectors of level `level` (canonical complex128,
 * [ntv][V_l][d_l]) and rebuild P_level and D_{level+1} = P^H D_level P from
 * them in FP64 (the construction that ends each setup step of Alg. 3 and
 * Alg. 4).  EINVAL if the vectors are linearly dependent on an aggregate to
 * within rounding. */
int ddamg_import_test_vectors(ddamg_hier hier, int level, const void* tv, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DDAMG_H */
