// Host orchestration of the DD-alpha-AMG method on one GPU: the operator
// context, the multilevel hierarchy, the K-/V-cycle (Alg. 2 / Alg. 1), the
// flexible GMRES solvers, the odd-even coarsest solve and the two setup
// phases (Alg. 3, Alg. 4).  Everything numerical runs in the kernels of
// fine/coarse/transfer/blas; this layer only sequences launches and keeps
// the small Krylov scalars (Hessenberg matrix, Givens rotations) on the host.
#pragma once

#include <complex>
#include <memory>
#include <vector>

#include "../../include/ddamg.h"
#include "blas.h"
#include "coarse.h"
#include "dgmres.h"
#include "fine.h"
#include "memory.h"
#include "transfer.h"

namespace ddamg {

struct Context {
  // the caller's workspace the arrays below are carved from (nullptr: each
  // is a hipMalloc of its own); declared first so that it outlives them
  std::unique_ptr<Workspace> ws;
  FineGeom g;
  double m0 = 0, csw = 0;
  DevArray<double2> U64, A64;
  DevArray<float2> U32, A32;
  DevArray<__half2> U16, A16;     // FP16 storage, made on first request
  bool half_ready = false;
  DevArray<int> nbr, cblk;
  // scratch for canonical-layout calls, raw bytes shared by both precisions
  DevArray<double2> s64a, s64b;
  template <typename T> FineOpView<T> view() const;
  FineOpView<float, __half2> view16() const { return {U16.p, A16.p, nbr.p, g.nblk}; }
  void make_half(hipStream_t s);
};

// Work fields of one level for a batch of up to `cap` systems (each buffer
// [cap][n]; the Krylov bases [m+1][cap][n])
template <typename T>
struct Work {
  DevArray<C<T>> bin, z, r, rec, x, w, t1, t2, t3, t4;
  DevArray<C<T>> V, Z;     // Krylov bases of this level
  int m = 0;               // basis length
  int cap = 0;             // batch capacity
};

struct LevelStore {
  bool fine = false;
  int dims[4] = {0, 0, 0, 0};
  int d = 12;
  long long V = 0, n = 0;
  // coarse operator (level >= 1)
  CoarseGeom cg;
  DevArray<int> c_nbr9, c_blk_sites, c_site_blk, c_site_pos, c_even, c_odd;
  DevArray<unsigned> c_inmask;
  SapTables sap_tables() const { return SapTables{c_blk_sites.p, c_site_pos.p, c_inmask.p, cg.nblk, cg.bs, cg.kmax}; }
  DevArray<double2> D64;           // Galerkin output: self + forward blocks, row-major
  DevArray<double2> K64, Einv64;   // nine-block column-major apply copies
  DevArray<float2> K32, Einv32;
  DevArray<__half2> K16;
  // dense Schur complement of a small coarsest level (sm = its order, 0 when
  // the sparse product is used): FP64 master, FP32 copy, index tables
  int sm = 0;
  std::vector<int> s_oidx_h, s_eidx_h;
  DevArray<int> s_oidx, s_eidx;
  DevArray<double2> S64;
  DevArray<float2> S32;
  // coarse SAP work buffers (rho, q ping-pong; per-site inner products),
  // sized for the largest batch seen
  DevArray<double2> sr64, sq64;
  DevArray<float2> sr32, sq32;
  DevArray<double> sp64;
  DevArray<float> sp32;
  SapScratch<double> ss64;
  SapScratch<float> ss32;
  // interpolation to the next level
  int N = 0;
  AggTables at;
  DevArray<int> a_members, a_member_agg;
  DevArray<double2> P64;
  DevArray<float2> P32;
  DevArray<__half2> P16;
  DevArray<double2> tv64;  // test vectors (FP64 storage; setup in the preconditioner precision uses tv32)
  DevArray<float2> tv32;
  AggDev ad() const { return AggDev{a_members.p, a_member_agg.p}; }
  template <typename T> CoarseOpView<T> cview() const;
  CoarseOpView<float, __half2> cview16() const { return {K16.p, c_nbr9.p, (int)V, d}; }
};

struct Hierarchy {
  // the caller's workspace (see Context::ws); declared first
  std::unique_ptr<Workspace> ws;
  int nrhs_max = 0;                // batches the workspace was sized for (0: no workspace)
  Context* ctx = nullptr;
  ddamg_params p{};
  int L = 0;
  std::vector<LevelStore> lv;
  std::vector<Work<double>> w64;
  std::vector<Work<float>> w32;
  // outer FGMRES (FP64 basis, preconditioned directions at the preconditioner precision)
  DevArray<double2> oV, oZ64, ob, ox, ow, ot;
  DevArray<float2> oZ32;
  DevArray<__half2> oZ16;          // FP16 directions with per-site scales (FP16 storage)
  DevArray<float> oZs;
  DevArray<double2> sc64a, sc64b;   // scratch for canonical-layout calls (raw bytes, both precisions)
  DevArray<double2> ds_e, ds_t3, ds_t4, ds_o;   // dense Schur construction, kept with a workspace
  std::unique_ptr<Reducer> red;
  hipStream_t s = nullptr;
  hipStream_t own_s = nullptr;     // the hierarchy's own stream (concurrent solves), made on first use
  bool recording = false;
  // setup record: visit[r] says whether system r is really being visited
  // (live in every enclosing FGMRES), so its record may be overwritten
  std::vector<char> visit;
  bool half = false;               // FP16 operator storage for the FP32 levels
  // FP16 fine-level spinors of the solve's preconditioner (half_spinors):
  // two batches of fields [cap][n0] with their site scales [cap][V0], the
  // cycle's right-hand side (a) and a result for the level calls (b)
  bool hs = false;
  int hcap = 0;
  DevArray<__half2> h16a, h16b;
  DevArray<float> h16as, h16bs;
  void ensure_hs(int nb);
  int ocap = 0;                    // batch capacity of the outer solver's buffers
  std::vector<long long> kc_it, cs_it;   // per system of the batch: K-cycle / coarsest iterations
  const double2* tv_extra = nullptr;
  DevArray<int> setup_flags;       // [0] dependent test vectors, [1] singular coarsest self block
  double t_setup = 0;              // wall time of the setup
  // Algorithmic bytes and flops of the level operations since the last
  // reset: each operation adds what its definition must move and compute
  // (per-site sizes of its vectors and operator data, at the precision and
  // storage it runs with); an estimate of the compulsory work, not a
  // measurement.
  double m_bytes = 0, m_flops = 0;
  void meter(double bytes, double flops) { m_bytes += bytes; m_flops += flops; }
  // bytes per stored complex number of the operator data read by precision T
  template <typename T> double op_bytes() const { return sizeof(T) == 8 ? 16.0 : (half ? 4.0 : 8.0); }
  // GPU time per level (params.profile_levels): an event is recorded on the
  // stream wherever the work moves from one level to another (lt_push on
  // entering a level, lt_pop on returning), and the time between two marks
  // is charged to the level current after the first
  std::vector<std::pair<hipEvent_t, int>> lt_marks;
  std::vector<hipEvent_t> lt_pool;
  std::vector<int> lt_stack;
  bool lt_on = false;
  void lt_mark(int level);
  void lt_push(int l);
  void lt_pop();
  void lt_begin();
  void lt_end(double out[4]);
  // device-side GMRES scalars (graph mode) and the captured preconditioner
  // graphs, one per (precision, batch size); `gen` counts reallocations of
  // the buffers a graph has baked in
  DevArray<GmSys> gm_sys;
  DevArray<double2> gm_res, gm_coef;
  DevArray<double> gm_scale;
  DevArray<long long> gm_iters;
  int* gm_flag_host = nullptr;     // coherent pinned word, written by the kernels
  int* gm_flag_dev = nullptr;
  bool dev_scalars = false;
  int pred_steps = 4;              // steps the last polled device-scalar GMRES cycle needed
  long long gen = 0;
  struct PreGraph {
    hipGraphExec_t exec = nullptr;
    int nb = 0;
    bool f32 = false;
    long long gen = -1;
  };
  std::vector<PreGraph> graphs;
  DevGmres gm();
  void drop_graphs();
  // outer FGMRES of one right-hand side with its scalars on the device
  // (ddamg_solve_batch): its own GMRES record and liveness flag, the
  // preconditioner, D and the Gram-Schmidt step as a fixed launch sequence
  // (capturable), fields in ob (b), ox (x, native FP64)
  DevArray<GmSys> go_sys;
  DevArray<double2> go_res, go_coef;
  DevArray<double> go_scale;
  DevArray<long long> go_iters;
  int* go_flag_host = nullptr;
  int* go_flag_dev = nullptr;
  long long go_zeroed = -1;        // gen at which the outer bases were cleared
  DevGmres gmo();
  void outer_dev_prepare();        // buffers, warm-up of lazy allocations (eager)
  void outer_dev_begin();          // targets, r_0 = b - D x_0, V_0 (eager)
  void outer_dev_step(int j);      // step j: Z_j = M V_j, w = D Z_j, Gram-Schmidt, V_{j+1}
  void outer_dev_tail();           // x += Z y, r = b - D x, restart decision, V_0
  long long uid = 0;               // unique per hierarchy (graph caches key on it)
  // graphs of ddamg_solve_batch over a list of hierarchies (kept by the
  // first one): one per outer step, one for the cycle's tail
  struct BatchGraph {
    hipGraph_t g = nullptr;        // kept: its nodes name the ones to disable
    hipGraphExec_t exec = nullptr;
    std::vector<std::vector<hipGraphNode_t>> nodes;   // kernel nodes per system
    std::vector<char> on;                             // per system: enabled
  };
  struct BatchGraphs {
    std::vector<long long> uids, gens;
    std::vector<BatchGraph> step;  // one per outer step index
    BatchGraph tail;
    ~BatchGraphs();
  };
  std::unique_ptr<BatchGraphs> bgraphs;

  template <typename T> Work<T>& work(int l);
  template <typename T> const C<T>* P(int l) const;
  // call f with the operator view / interpolation the precision-T kernels
  // read (the FP16 copies for T = float when `half` is set)
  template <typename T, typename F> void fine_op(F&& f) const;
  template <typename T, typename F> void coarse_op(int l, F&& f) const;
  template <typename T, typename F> void interp(int l, F&& f) const;
  template <typename T> const C<T>* tv(int l) const;
  template <typename T> C<T>* tv(int l);

  // level operations at precision T
  // (nb fields of the level, contiguous, processed by batched launches)
  template <typename T> void apply(int l, const C<T>* in, C<T>* out, int nb = 1);
  template <typename T> void sap(int l, const C<T>* b, C<T>* z, int nsweeps, int nb = 1);
  template <typename T> void restrict_to(int l, const C<T>* fine, C<T>* coarse, int nb = 1);
  template <typename T> void prolong_add(int l, const C<T>* coarse, C<T>* fine, int nb = 1);
  // Solvers on batches of nb systems advancing together (fields n apart);
  // every system keeps its own Krylov scalars and stopping test, so the
  // result for each equals that of a solve on its own.
  template <typename T> void cycle(int l, const C<T>* b, C<T>* z, int nb = 1);
  // the part of the cycle below level l: work<T>(l+1).bin -> work<T>(l+1).z
  template <typename T> void coarse_correction(int l, int nb);
  // the level-0 cycle and its pieces on FP16 fine spinors with site scales
  // (b, bs: right-hand side; z, zs: result), FP32 arithmetic on FP16
  // operator data; the coarse levels run as in cycle<float>
  void cycle_hs(const __half2* b, const float* bs, __half2* z, float* zs, int nb);
  void sap_hs(const __half2* b, const float* bs, __half2* z, float* zs, int nsweeps, int nb);
  void restrict_hs(const __half2* fine, const float* fs, C<float>* coarse, int nb);
  void prolong_hs(const C<float>* coarse, __half2* fine, float* fs, int nb);   // fine = P coarse
  // Coarsest solve (odd-even reduced GMRES) with the GMRES scalars on the
  // device: with poll > 0 the host reads the device's liveness flag (a
  // round trip each) first after max(poll, pred_steps) steps, then every
  // step, and at each restart, and stops when no system is left; poll = 0
  // issues the fixed launch sequence (graph capture)
  template <typename T> void coarsest_solve(const C<T>* b, C<T>* z, int nb, int poll);
  template <typename T, typename Op>
  void gmres_dev(int l, Op op, const C<T>* b, C<T>* x, int m, int cycles, double tol, int nb, int poll);
  // level-0 cycle of the batch, work<T>(0).bin -> work<T>(0).x, by replaying
  // the captured graph (captured on first use after an eager run)
  template <typename T> void apply_pre_graph(int nb);
  template <typename T> void schur(const C<T>* v, C<T>* out, int nb);
  // FGMRES(m) from x = 0; iters[r] += iterations of system r
  template <typename T, typename Op, typename Pre>
  void fgmres(int l, Op op, Pre pre, bool use_pre, const C<T>* b, C<T>* x, int m, int max_cycles,
              double tol, int nb, long long* iters);
  // one Arnoldi step of every system: w_r orthogonalised against
  // V_{0..j, r}; h[r * (KMAX + 1) + i] the Hessenberg column, hn[r] the
  // norm left; cf[r * KMAX + i] the coefficients of w + V c
  template <typename T>
  void arnoldi(const C<T>* V, long long vstride, long long n, int nb, int j, C<T>* w,
               const std::vector<char>& live, std::vector<std::complex<double>>& h, std::vector<double>& hn,
               std::vector<std::complex<double>>& cf);
  // outer FP64 FGMRES for nb right-hand sides (native FP64 fields)
  template <typename T> void outer(const double2* b, double2* x, ddamg_solve_stats* st, int nb);
  template <typename T> void ensure_batch(int nb);
  template <typename T> void ensure_work(int nb);

  // setup
  template <typename T> void setup(const double2* tv_canonical);
  template <typename T> void initial_setup(int l);
  template <typename T> void iterative_setup(int l, int i);
  // construct P_l (FP64 orthonormalisation) and D_{l+1} (FP64 Galerkin);
  // from32: the FP32 test vectors are the current ones
  void build_level(int l, bool from32);
  // the dense Schur complement of coarsest level c, column by column from
  // unit vectors through the sparse FP64 product
  void build_dense_schur(int c);
  template <typename T> void alloc_work(int cap);
  // the level structure: geometry, index tables and the arrays of the
  // operators, interpolations and test vectors (no kernels: it also runs
  // against a counting workspace)
  void layout();
  // with a workspace: everything a setup and the solves of batches of up to
  // nrhs right-hand sides grow on demand otherwise, allocated up front
  void reserve(int nrhs);
  // replace the SAP block shape of coarse level l (1 <= l <= L-2) for the
  // solves from now on (the setup already done is kept)
  void set_sap_block(int l, const int blk[4]);

  Hierarchy() = default;
  Hierarchy(const Hierarchy&) = delete;
  Hierarchy& operator=(const Hierarchy&) = delete;
  ~Hierarchy() {
    for (auto& m : lt_marks) lt_pool.push_back(m.first);
    for (hipEvent_t e : lt_pool) (void)hipEventDestroy(e);
    drop_graphs();
    bgraphs.reset();
    if (own_s) (void)hipStreamDestroy(own_s);
    if (gm_flag_host) (void)hipHostFree(gm_flag_host);
    if (go_flag_host) (void)hipHostFree(go_flag_host);
  }
};

// out[r] = ||v_r|| (FP64 sum) for nb fields of n complex numbers each
template <typename T>
void bnorms(Reducer& red, const C<T>* v, long long n, int nb, std::vector<double>& out, hipStream_t s);

// ws: the caller's workspace (nullptr: the library allocates); half and
// nrhs_max size what a workspace reserves up front (the FP16 operator
// copies, canonical-layout scratch for nrhs_max fields)
Context* create_context(const ddamg_lattice* lat, const double2* links, hipStream_t s,
                        std::unique_ptr<Workspace> ws = nullptr, bool half = false, int nrhs_max = 0);
Hierarchy* create_hierarchy(Context* ctx, const ddamg_params* p, const double2* tv,
                            const double2* tv_extra, hipStream_t s,
                            std::unique_ptr<Workspace> ws = nullptr, int nrhs_max = 0);
// device bytes of a context and, with params, of a hierarchy on it, as the
// workspace entry points allocate them
void workspace_bytes(const ddamg_lattice* lat, const ddamg_params* p, int nrhs_max, size_t* ctx_bytes,
                     size_t* hier_bytes);
void validate_params(const Context& ctx, const ddamg_params& p);
void sap_block_of(const ddamg_params& p, int l, int out[4]);

}  // namespace ddamg
