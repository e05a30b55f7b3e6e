#!/usr/bin/env python3
"""Benchmark of the DD-alpha-AMG hot path on one MI355X.

A step is one complete solve of D z = b to relative residual 1e-10 on the
48^3x96 four-level Wilson-clover workload (aggregates 4^4, 2^4, 2^4; N = 20 /
20 / 28; c_sw 1, eps 0.55, m0 -0.43; one complex Gaussian right-hand side):
outer FP64 FGMRES, FP32 K-cycle preconditioner on FP16-stored operator data,
the hierarchy built beforehand (setup timed separately) and b resident in
HBM.  `value` is solves per second.

Also reported on the same inputs: the plain FP64 GPU solve (everything FP64)
for the time-to-solution comparison, the setup times, the solve's error
measured by the FP64 oracle (its site-by-site operator on sampled sites), two
and three levels against four on the same lattice, CGNR, the SAP colour
pass (the solve's dominant kernel) and the Wilson-clover stencil against the
HBM roofline (HIP events around launches on the stream the library uses),
and the FP64 CPU oracle timed on a bounded sample of the same workload.

Other workloads (--workload): the 16^3x32 three-level lattice with its
batched, FP16 and CGNR variants; the 32^3x64 lattice with the 12 point
sources in one batch; the uneven batch of eight lattices; the bare-mass scan.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.time()
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
BATCH_RHS = 12          # batch size of the batched-kernel timings (the 12 spin-colour sources)
# HBM traffic per launch of the FP32 stencil on the 16^3x32 lattice: None,
# the kernel's arithmetic has changed since the FETCH_SIZE / WRITE_SIZE runs
# of profiles/dslash_clover16x32_counters.md
DSLASH_F32_TRAFFIC_BYTES = None
# HBM traffic per launch of the SAP colour pass on FP16-stored links and
# clover on the 48^3x96 lattice, from the FETCH_SIZE / WRITE_SIZE counter
# runs summarised in profiles/ (None until taken for the current kernel)
SAP_F16_PASS_TRAFFIC_BYTES = 5.572e9
# the same for the pass on FP16 spinors (b, z with one FP32 scale per site)
SAP_F16S_PASS_TRAFFIC_BYTES = 4.122e9
# FP32 vector peak without packed FP32 instructions (which the library does
# not emit): 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
VALU_F32_PEAK_TFLOPS = 78.6
# flops of one SAP update of a site (a complex multiply 6, a complex add 2,
# real times complex 2): the residual b - D z (8 spin-projected hops of 168
# flops: 12 for the projection, 132 for U times two half spinors, 24 to
# rebuild and add; the two Hermitian 6x6 clover blocks 504; combining 72)
# = 1920, then per MR step the block operator (4 hops, clover, combining:
# 1224), the inner products (144) and the two updates (192) = 1560, three
# steps 4680, and z += x (24): 6624
SAP_FLOPS_PER_UPDATED_SITE = 6624
WORKLOAD = "clover16x32_3lvl"
HEADLINE = "clover48x96_4lvl"
METRIC = "Dψ HBM GB/s + time-to-1e-10 solve, mixed/batched vs FP64 plain, 1 GPU"
BATCH_WORKLOAD = "clover32x64_3lvl_12rhs"
FOUR_LEVEL_WORKLOAD = "clover48x96_4lvl"
UNEVEN_WORKLOAD = "uneven8_3lvl"
SCAN_WORKLOAD = "m0_scan_16x32"
# bare masses of the scan on the 16^3x32 lattice (eps 0.5: the critical mass
# estimated on 4^4 is about -0.49)
SCAN_M0 = (-0.30, -0.35, -0.40, -0.43, -0.45, -0.46)
# the shorter scan reported next to the default line
SCAN_M0_SHORT = (-0.30, -0.40, -0.45)
# coarsest GMRES of the graph-captured V-cycle: restart length, cycles (a
# fixed launch sequence, steps after convergence doing nothing)
GRAPH_COARSE = (8, 1)
# compulsory bytes of one Wilson-clover apply per site: spinor in (24 reals),
# 4 links (72 reals: each link serves two sites), clover (72 reals), spinor out
# (24 reals) -> 192 reals
DPSI_REALS_PER_SITE = 192
DPSI_SPINOR_REALS_PER_SITE = 48
# one SAP sweep (both colours) per site: b, z in, z out (72 reals), links and
# clover (144 reals)
SAP_REALS_PER_SITE = 216
SAP_SPINOR_REALS_PER_SITE = 72
# with FP16 spinors each of the three spinor reads / writes of a site also
# moves its FP32 scale
SAP_SCALE_BYTES_PER_SITE = 12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched point-source solve")
    ap.add_argument("--no-half", action="store_true",
                    help="skip the FP16-operator-storage variant of the mixed solve")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default SAP blocks and batch size (no autotuner search)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the Wilson-clover stencil loops and a reference copy of known size "
                         "(for hardware-counter runs)")
    ap.add_argument("--profile-window", type=float, nargs=2, default=None, metavar=("START", "DURATION"),
                    help="after the warmup, wait until START seconds after the bench started and solve "
                         "repeatedly for DURATION seconds (for a rocprofv3 --collection-period window that "
                         "holds nothing but solves)")
    ap.add_argument("--no-levels", action="store_true",
                    help="skip the two- and three-level comparison on the headline lattice")
    ap.add_argument("--fp32-spinors", action="store_true",
                    help="FP32 fine-level spinors in the headline preconditioner (default: FP16 with site scales)")
    ap.add_argument("--no-other-spinors", action="store_true",
                    help="skip the solve with the other fine-spinor storage (and its per-level times)")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the short bare-mass scan (16^3x32, two and three levels against CGNR) "
                         "reported next to the default line")
    ap.add_argument("--workload", default=HEADLINE, choices=[WORKLOAD, BATCH_WORKLOAD, FOUR_LEVEL_WORKLOAD, UNEVEN_WORKLOAD,
                                                      SCAN_WORKLOAD],
                    help="the 48^3x96 four-level lattice (default), the 16^3x32 three-level lattice with "
                         "its batched and FP16 variants, the 32^3x64 lattice with the 12 point sources "
                         "solved in one batch, the uneven batch of eight lattices (four 16^4, two 24^3x48, "
                         "two 32^3x64) solved concurrently, or the bare-mass scan towards criticality on the "
                         "16^3x32 lattice (two and three levels against CGNR)")
    ap.add_argument("--lattice", default=None,
                    help="X,Y,Z,T lattice for --kernels-only (default: the bench workload's)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_1307_6101_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_1307_6101_amd import ddamg as dd

    cfg = W.CONFIGS[WORKLOAD]
    if args.kernels_only:
        kernels_only(args, W.CONFIGS[args.workload], dd, W, np, torch)
        return
    if args.workload == HEADLINE:
        headline_workload(args, dd, W, np, torch)
        return
    if args.workload == UNEVEN_WORKLOAD:
        uneven_workload(args, dd, W, np, torch)
        return
    if args.workload == SCAN_WORKLOAD:
        scan_workload(args, cfg, dd, W, np, torch)
        return
    if args.workload != WORKLOAD:
        big_workload(args, args.workload, W.CONFIGS[args.workload], dd, W, np, torch)
        return
    dims = cfg["dims"]
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    log(f"[bench] workload {WORKLOAD} dims={dims} V={V}")
    t0 = time.time()
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    b = W.gaussian_spinor(dims, cfg["seed_rhs"])
    tv = W.test_vectors(dims, 12, cfg["ntv"][0], cfg["seed_tv"])
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s")
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(b).to(dev)
    tvd = torch.from_numpy(tv).to(dev)
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], Ud)
    del Ud

    def params(prec, half=False):
        p = dd.params_default(cfg["levels"])
        for l, a in enumerate(cfg["agg"]):
            for mu in range(4):
                p.agg[l][mu] = a[mu]
        for l, n in enumerate(cfg["ntv"]):
            p.ntv[l] = n
        p.nu = cfg["nu"]
        p.precond_prec = prec
        p.half_storage = 1 if half else 0
        return p

    def setup(prec, half=False):
        torch.cuda.synchronize()
        t = time.time()
        H = dd.build_hierarchy(ctx, params(prec, half), tvd)
        torch.cuda.synchronize()
        return H, time.time() - t

    H32, t_setup32 = setup(dd.F32)
    log(f"[bench] mixed-precision setup {t_setup32:.2f}s")
    z = torch.zeros_like(bd)

    def one_solve(H):
        z.zero_()
        rc, st = dd.solve(H, bd, z)
        if rc != dd.OK:
            raise RuntimeError(f"solve failed rc={rc} {st}")
        return st[0]

    # the autotuner picks the level-1 SAP block shape (timed solves; every
    # hierarchy below is tuned the same way, the plain FP64 one included)
    def tune(H, rhs, nrhs=1):
        if args.no_tune:
            return None
        one_solve(H) if nrhs == 1 else None
        t = time.time()
        r = dd.tune(H, rhs, nrhs=nrhs)
        return dict(sap_block_level1=r["sap_block_l"][0], batch=r["batch"], search_s=round(time.time() - t, 3))

    one_solve(H32)
    t_untuned = float(np.median([one_solve(H32)["seconds"] for _ in range(3)]))
    tuned32 = tune(H32, bd.reshape(1, -1))
    if tuned32 is not None:
        tuned32["untuned_time_to_solution_s"] = round(t_untuned, 4)
    log(f"[bench] autotuned: {tuned32}")

    for i in range(args.warmup):
        st = one_solve(H32)
        log(f"[bench] warmup {i}: {st['outer_iters']} its, {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    t = time.time()
    stats = []
    for i in range(args.steps):
        st = one_solve(H32)
        stats.append(st)
        log(f"[bench] step {i}: {st['outer_iters']} its, relres {st['true_relres']:.2e}, "
            f"{st['seconds']:.3f}s")
    torch.cuda.synchronize()
    elapsed = time.time() - t
    ms = 1000.0 * elapsed / args.steps
    z_mixed = z.clone()

    # plain FP64 GPU method on the same inputs
    plain = None
    if not args.no_plain:
        H64, t_setup64 = setup(dd.F64)
        log(f"[bench] plain FP64 setup {t_setup64:.2f}s")
        tuned64 = tune(H64, bd.reshape(1, -1))
        log(f"[bench] plain FP64 autotuned: {tuned64}")
        one_solve(H64)
        torch.cuda.synchronize()
        t = time.time()
        pst = [one_solve(H64) for _ in range(max(1, min(args.steps, 3)))]
        torch.cuda.synchronize()
        t_plain = (time.time() - t) / len(pst)
        plain = dict(time_to_solution_s=t_plain, setup_s=t_setup64,
                     outer_iters=pst[-1]["outer_iters"], true_relres=pst[-1]["true_relres"], autotuned=tuned64)
        log(f"[bench] plain FP64 solve {t_plain:.3f}s, {pst[-1]['outer_iters']} its")
        diff = torch.linalg.vector_norm(z - z_mixed) / torch.linalg.vector_norm(z)
        plain["rel_diff_vs_mixed_solution"] = float(diff)

    # CGNR in FP64 (the paper's comparison method, Sec. 4) on the same system
    cg = None
    if not args.no_plain:
        zc = torch.zeros_like(bd)
        torch.cuda.synchronize()
        t = time.time()
        rc, cst = dd.cgnr(ctx, bd.reshape(1, -1), zc.reshape(1, -1), tol=cfg["tol"], max_iter=100000)
        torch.cuda.synchronize()
        t_cg = time.time() - t
        cg = dict(time_to_solution_s=round(t_cg, 4), iterations=cst[0]["outer_iters"],
                  true_relres=cst[0]["true_relres"], status=rc,
                  speedup_mixed_vs_cgnr=round(t_cg / (ms / 1000.0), 2))
        log(f"[bench] CGNR FP64: {cst[0]['outer_iters']} its, {t_cg:.3f}s")

    # the 12 spin-colour point sources on the same lattice: one batch through
    # the mixed-precision solver, against the plain FP64 method solving them
    # one at a time
    batched = None
    if not args.no_batch:
        bps = torch.from_numpy(W.point_sources(dims)).to(dev)
        zps = torch.zeros_like(bps)

        def batch_solve(H, nb):
            zps.zero_()
            torch.cuda.synchronize()
            t = time.time()
            rc, st = dd.solve(H, bps, zps, nrhs=nb)
            torch.cuda.synchronize()
            if rc != dd.OK:
                raise RuntimeError(f"batched solve failed rc={rc}")
            return time.time() - t, st

        tuned_b = tune(H32, bps, BATCH_RHS)
        log(f"[bench] 12 point sources autotuned: {tuned_b}")
        batch_solve(H32, BATCH_RHS)
        t_b, st_b = batch_solve(H32, BATCH_RHS)
        log(f"[bench] 12 point sources, one mixed batch: {t_b:.3f}s "
            f"({1000 * t_b / BATCH_RHS:.2f} ms per rhs), its {[x['outer_iters'] for x in st_b]}")
        batched = dict(rhs=BATCH_RHS, sources="12 spin-colour point sources at x = 0",
                       mixed_batch_s=round(t_b, 4), mixed_per_rhs_s=round(t_b / BATCH_RHS, 5),
                       outer_iters=[x["outer_iters"] for x in st_b],
                       max_true_relres=max(x["true_relres"] for x in st_b), autotuned=tuned_b)
        if not args.no_plain:
            p1 = params(dd.F64)
            p1.batch = 1
            H64b = dd.build_hierarchy(ctx, p1, tvd)
            tune(H64b, bps[:1], 1)
            t_p, st_p = batch_solve(H64b, BATCH_RHS)
            log(f"[bench] 12 point sources, plain FP64 one at a time: {t_p:.3f}s")
            batched.update(plain_fp64_one_at_a_time_s=round(t_p, 4),
                           speedup_vs_plain_fp64=round(t_p / t_b, 3))
            del H64b
    if not args.no_plain:
        del H64

    # the mixed solve with the preconditioner's operator data stored in FP16
    half = None
    H16 = None
    if not args.no_half:
        H16, t_setup16 = setup(dd.F32, half=True)
        log(f"[bench] FP16-storage setup {t_setup16:.2f}s")
        tune(H16, bd.reshape(1, -1))
        one_solve(H16)
        torch.cuda.synchronize()
        t = time.time()
        hst = [one_solve(H16) for _ in range(max(1, min(args.steps, 3)))]
        torch.cuda.synchronize()
        t_half = (time.time() - t) / len(hst)
        half = dict(time_to_solution_s=round(t_half, 4), setup_s=round(t_setup16, 3),
                    outer_iters=hst[-1]["outer_iters"], true_relres=hst[-1]["true_relres"],
                    speedup_vs_fp32_storage=round((ms / 1000.0) / t_half, 3))
        log(f"[bench] FP16-storage solve {t_half:.3f}s, {hst[-1]['outer_iters']} its")
        # and with the outer directions in FP16 with per-site scales
        pd = params(dd.F32, True)
        pd.half_directions = 1
        Hd = dd.build_hierarchy(ctx, pd, tvd)
        tune(Hd, bd.reshape(1, -1))
        one_solve(Hd)
        torch.cuda.synchronize()
        t = time.time()
        dst = [one_solve(Hd) for _ in range(max(1, min(args.steps, 3)))]
        torch.cuda.synchronize()
        t_dir = (time.time() - t) / len(dst)
        half["with_fp16_directions"] = dict(time_to_solution_s=round(t_dir, 4),
                                            outer_iters=dst[-1]["outer_iters"],
                                            true_relres=dst[-1]["true_relres"])
        log(f"[bench] FP16 storage + FP16 directions solve {t_dir:.3f}s, {dst[-1]['outer_iters']} its")
        del Hd

    # dominant fine kernels, timed with events on the stream the library uses
    kern = {}
    stream = torch.cuda.current_stream()
    nat32 = torch.zeros(V * 12, dtype=torch.complex64, device=dev)
    out32 = torch.zeros_like(nat32)
    dd.to_native(ctx, None, 0, bd, nat32, prec=dd.F32)
    nat64 = torch.zeros(V * 12, dtype=torch.complex128, device=dev)
    out64 = torch.zeros_like(nat64)
    dd.to_native(ctx, None, 0, bd, nat64, prec=dd.F64)

    def time_launches(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1000.0 / reps

    t_d32 = time_launches(lambda: dd.apply_D(ctx, nat32, out32, prec=dd.F32, layout=dd.NATIVE),
                          args.kernel_reps)
    t_d64 = time_launches(lambda: dd.apply_D(ctx, nat64, out64, prec=dd.F64, layout=dd.NATIVE),
                          args.kernel_reps)
    zs = torch.zeros_like(nat32)
    t_sap32 = time_launches(lambda: dd.sap_smooth(H32, 0, nat32, zs, 1, prec=dd.F32,
                                                  layout=dd.NATIVE), args.kernel_reps)
    for name, tk, bytes_per_real in (("dslash_f32", t_d32, 4), ("dslash_f64", t_d64, 8)):
        nbytes = DPSI_REALS_PER_SITE * bytes_per_real * V
        kern[name] = dict(seconds=tk, algorithmic_bytes=nbytes, gbs=nbytes / tk / 1e9)
    if H16 is not None:
        t_d16 = time_launches(lambda: dd.apply_Dc(H16, 0, nat32, out32, prec=dd.F32, layout=dd.NATIVE),
                              args.kernel_reps)
        # FP32 spinor in and out, FP16 links and clover
        nbytes = (DPSI_SPINOR_REALS_PER_SITE * 4 + (DPSI_REALS_PER_SITE - DPSI_SPINOR_REALS_PER_SITE) * 2) * V
        kern["dslash_f16store"] = dict(seconds=t_d16, algorithmic_bytes=nbytes, gbs=nbytes / t_d16 / 1e9)
        t_s16 = time_launches(lambda: dd.sap_smooth(H16, 0, nat32, zs, 1, prec=dd.F32, layout=dd.NATIVE),
                              args.kernel_reps)
        # b, z in, z out in FP32; links and clover in FP16
        sb16 = (SAP_SPINOR_REALS_PER_SITE * 4 + (SAP_REALS_PER_SITE - SAP_SPINOR_REALS_PER_SITE) * 2) * V
        kern["sap_sweep_f16store"] = dict(seconds=t_s16, algorithmic_bytes=sb16, gbs=sb16 / t_s16 / 1e9,
                                          launches=2)
    sbytes = SAP_REALS_PER_SITE * 4 * V
    kern["sap_sweep_f32"] = dict(seconds=t_sap32, algorithmic_bytes=sbytes, gbs=sbytes / t_sap32 / 1e9,
                                 launches=2)
    # batched right-hand sides: one launch per operation for NB fields
    NB = BATCH_RHS
    natb = torch.zeros((NB, V * 12), dtype=torch.complex64, device=dev)
    for r in range(NB):
        natb[r].copy_(nat32)
    outb = torch.zeros_like(natb)
    t_db = time_launches(lambda: dd.apply_D(ctx, natb, outb, nrhs=NB, prec=dd.F32, layout=dd.NATIVE),
                         args.kernel_reps)
    nbytes = (DPSI_SPINOR_REALS_PER_SITE * NB + DPSI_REALS_PER_SITE - DPSI_SPINOR_REALS_PER_SITE) * 4 * V
    kern[f"dslash_f32_x{NB}"] = dict(seconds=t_db, algorithmic_bytes=nbytes, gbs=nbytes / t_db / 1e9)
    zb = torch.zeros_like(natb)
    t_sb = time_launches(lambda: dd.sap_smooth(H32, 0, natb, zb, 1, nrhs=NB, prec=dd.F32, layout=dd.NATIVE),
                         max(2, args.kernel_reps // 5))
    sbb = (SAP_SPINOR_REALS_PER_SITE * NB + SAP_REALS_PER_SITE - SAP_SPINOR_REALS_PER_SITE) * 4 * V
    kern[f"sap_sweep_f32_x{NB}"] = dict(seconds=t_sb, algorithmic_bytes=sbb, gbs=sbb / t_sb / 1e9, launches=2)
    # coarse operator of level 1 on the matrix cores
    (cdims, cd) = dd.level_info(H32, 1)
    cV = int(np.prod(cdims))
    cin = torch.randn((NB, cV * cd), dtype=torch.complex64, device=dev)
    cout = torch.zeros_like(cin)
    t_cb = time_launches(lambda: dd.apply_Dc(H32, 1, cin, cout, nrhs=NB, prec=dd.F32, layout=dd.NATIVE),
                         args.kernel_reps)
    flops = 9 * cd * cd * 8 * NB * cV
    kbytes = 9 * cd * cd * 8 * cV + 2 * NB * cd * 8 * cV       # nine stored blocks + vectors
    kern[f"coarse_apply_mfma_f32_x{NB}"] = dict(seconds=t_cb, algorithmic_bytes=kbytes, gbs=kbytes / t_cb / 1e9,
                                                tflops=flops / t_cb / 1e12,
                                                mfma_frac=flops / t_cb / 1e12 / MFMA_F32_PEAK_TFLOPS)
    t_c1 = time_launches(lambda: dd.apply_Dc(H32, 1, cin[0], cout[0], nrhs=1, prec=dd.F32, layout=dd.NATIVE),
                         args.kernel_reps)
    kern["coarse_apply_f32_x1"] = dict(seconds=t_c1, algorithmic_bytes=9 * cd * cd * 8 * cV + 2 * cd * 8 * cV,
                                       gbs=(9 * cd * cd * 8 * cV + 2 * cd * 8 * cV) / t_c1 / 1e9)
    for k, v in kern.items():
        extra = f", {v['tflops']:.1f} TFLOP/s ({100 * v['mfma_frac']:.1f}% of FP32 MFMA peak)" if "tflops" in v else ""
        log(f"[bench] {k}: {v['seconds'] * 1e6:.1f} us, {v['gbs']:.0f} GB/s{extra}")

    dom = kern["dslash_f32"]
    roofline = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4), "traffic": DSLASH_F32_TRAFFIC_BYTES,
                "kernel": "k_dslash<float> (Wilson-clover, FP32)",
                "note": "16^3x32 working set ~175 MB fits the 256 MB Infinity Cache"}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, U, b, stats[-1]["outer_iters"], V)

    mean_its = float(np.mean([s["outer_iters"] for s in stats]))
    line = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 outer",
        "data": "synthetic (seeded SU(3) links exp(i eps H), Gaussian rhs)",
        "config": {"workload": "16^3x32 Wilson-clover, 3 levels (4^4, 2^4 aggregates, N=20), "
                               "c_sw=1, eps=0.5, m0=-0.4, 1 rhs, tol 1e-10",
                   "parallelism": "1 GPU"},
        "time_to_solution_s": round(ms / 1000.0, 4),
        "setup_s": round(t_setup32, 3),
        "autotuned": tuned32,
        "outer_iters": mean_its,
        "true_relres": stats[-1]["true_relres"],
        "kcycle_iters": stats[-1]["kcycle_iters"],
        "coarsest_iters": stats[-1]["coarsest_iters"],
        "cgnr_fp64": cg,
        "plain_fp64": plain,
        "fp16_storage": half,
        "batched_point_sources": batched,
        "speedup_vs_plain_fp64": (round(plain["time_to_solution_s"] / (ms / 1000.0), 3) if plain else None),
        "kernels": {k: dict({"us": round(v["seconds"] * 1e6, 2), "GB/s": round(v["gbs"], 1)},
                            **({"TFLOP/s": round(v["tflops"], 2), "mfma_frac": round(v["mfma_frac"], 4)}
                               if "tflops" in v else {})) for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def fill_params(dd, cfg, prec, half=False, batch=None, levels=None, spinors16=False, profile=False):
    """ddamg_params of a workload (Tab. 1 defaults otherwise); `levels` keeps
    only the first levels of its hierarchy; spinors16: FP16 fine-level
    spinors in the preconditioner; profile: per-level GPU times."""
    L = cfg["levels"] if levels is None else levels
    p = dd.params_default(L)
    for l, a in enumerate(cfg["agg"][:L - 1]):
        for mu in range(4):
            p.agg[l][mu] = a[mu]
    for l, n in enumerate(cfg["ntv"][:L - 1]):
        p.ntv[l] = n
    for l, blk in enumerate(cfg.get("sap_blocks", [])[1:L - 1]):
        for mu in range(4):
            p.sap_block_l[l][mu] = blk[mu]
    p.nu = cfg["nu"]
    p.precond_prec = prec
    p.half_storage = 1 if half else 0
    p.half_spinors = 1 if spinors16 else 0
    p.profile_levels = 1 if profile else 0
    if batch is not None:
        p.batch = batch
    return p


def device_fields(torch, W, dims, dof, n, seed):
    """W.gaussian_field(dims, dof, seed, nrhs=n) built on the device one
    field at a time (host memory for one field)."""
    X, Y, Z, T = dims
    out = torch.empty((n, T, Z, Y, X, dof), dtype=torch.complex128, device="cuda")
    for k, f in enumerate(W.gaussian_fields_iter(dims, dof, n, seed)):
        out[k].copy_(torch.from_numpy(f))
    return out


def time_launches(torch, fn, reps):
    """Mean seconds per call of fn (after one untimed call), from HIP events
    recorded on torch's current stream, which the binding passes to the
    library: the events bracket exactly the launches of the timed calls."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1000.0 / reps


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def headline_workload(args, dd, W, np, torch):
    """The 48^3x96 four-level workload (the default bench line)."""
    name = HEADLINE
    cfg = W.CONFIGS[name]
    dims = cfg["dims"]
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    log(f"[bench] workload {name} dims={dims} V={V}")
    t0 = time.time()
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    log(f"[bench] links in {time.time() - t0:.1f}s")
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], torch.from_numpy(U).to(dev))
    tvd = device_fields(torch, W, dims, 12, cfg["ntv"][0], cfg["seed_tv"])
    log(f"[bench] test vectors in {time.time() - t0:.1f}s")
    # fresh random vectors for level 2, which has more test vectors than level 1
    d2 = 2 * cfg["ntv"][1]
    cd2 = tuple(x // (a1 * a2) for x, a1, a2 in zip(dims, cfg["agg"][0], cfg["agg"][1]))
    extra = torch.from_numpy(W.test_vectors(cd2, d2, cfg["ntv"][2] - cfg["ntv"][1], cfg["seed_tv"] + 7)).to(dev)
    b = W.gaussian_spinor(dims, cfg["seed_rhs"])
    bd = torch.from_numpy(b).to(dev).unsqueeze(0)
    z = torch.zeros_like(bd)
    log(f"[bench] inputs in {time.time() - t0:.1f}s")

    def build(prec, half, levels=None, spinors16=False, profile=False):
        torch.cuda.synchronize()
        t = time.time()
        H = dd.build_hierarchy(ctx, fill_params(dd, cfg, prec, half, batch=8, levels=levels, spinors16=spinors16,
                                                profile=profile),
                               tvd, extra if (levels or cfg["levels"]) == 4 else None)
        torch.cuda.synchronize()
        return H, time.time() - t

    def one_solve(H):
        z.zero_()
        rc, st = dd.solve(H, bd, z)
        if rc != dd.OK:
            raise RuntimeError(f"solve failed rc={rc} {st}")
        return st[0]

    spinors16 = not args.fp32_spinors
    H, t_setup = build(dd.F32, True, spinors16=spinors16)
    log(f"[bench] mixed FP16-storage setup {t_setup:.2f}s (FP16 fine spinors: {spinors16})")
    for i in range(args.warmup):
        st = one_solve(H)
        log(f"[bench] warmup {i}: {st['outer_iters']} its, {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    if args.profile_window is not None:
        start, dur = args.profile_window
        while time.time() - T_START < start:
            time.sleep(0.05)
        n = 0
        while time.time() - T_START < start + dur:
            one_solve(H)
            n += 1
        log(f"[bench] profile window: {n} solves from {start:.0f}s to {time.time() - T_START:.1f}s")
    t = time.time()
    stats = []
    for i in range(args.steps):
        st = one_solve(H)
        stats.append(st)
        log(f"[bench] step {i}: {st['outer_iters']} its, relres {st['true_relres']:.2e}, {st['seconds']:.3f}s")
    torch.cuda.synchronize()
    ms = 1000.0 * (time.time() - t) / args.steps
    zz = z[0].cpu().numpy()

    # the solve's error measured by the FP64 oracle: its site-by-site
    # operator (its own index arithmetic and clover leaves) on sampled sites;
    # sqrt(V) times the rms residual there estimates ||b - D z||
    from oracle.dirac import apply_at_sites
    rng = np.random.Generator(np.random.PCG64(4811))
    sites = [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(64)]
    dz = apply_at_sites(U, cfg["m0"], cfg["csw"], zz, sites)
    r = np.array([b[s[3], s[2], s[1], s[0]] for s in sites]) - dz
    bnorm = float(np.linalg.norm(b))
    oracle_est = float(np.sqrt(np.mean(np.sum(np.abs(r) ** 2, axis=1)) * V)) / bnorm
    oracle_max = float(np.max(np.linalg.norm(r, axis=1))) / bnorm
    log(f"[bench] oracle residual on 64 sampled sites: estimate {oracle_est:.2e}, largest site {oracle_max:.2e}")
    del zz

    # kernels of the solve, timed with events on the stream the library uses
    kern = {}
    nat32 = torch.zeros(V * 12, dtype=torch.complex64, device=dev)
    dd.to_native(ctx, None, 0, bd, nat32, prec=dd.F32)
    zs = torch.zeros_like(nat32)
    out32 = torch.zeros_like(nat32)
    reps = args.kernel_reps
    t_sap = time_launches(torch, lambda: dd.sap_smooth(H, 0, nat32, zs, 1, prec=dd.F32, layout=dd.NATIVE), reps)
    # one colour pass handles half the sites: b, z in, z out at FP32 and the
    # links and clover at FP16, per site of the lattice and sweep
    sweep_bytes = (SAP_SPINOR_REALS_PER_SITE * 4 + (SAP_REALS_PER_SITE - SAP_SPINOR_REALS_PER_SITE) * 2) * V
    kern["sap_colour_pass_f16store"] = dict(seconds=t_sap / 2, algorithmic_bytes=sweep_bytes / 2,
                                            gbs=sweep_bytes / t_sap / 1e9)
    if spinors16:
        # the pass the solve runs: b, z as FP16 with site scales (native form:
        # entries, then scales, in one buffer)
        hb = torch.empty(V * 12 + V, dtype=torch.float32, device=dev)
        hz = torch.empty_like(hb)
        dd.to_native(ctx, None, 0, bd, hb, prec=dd.F16S)
        hz.zero_()
        t_sh = time_launches(torch, lambda: dd.sap_smooth(H, 0, hb, hz, 1, prec=dd.F16S, layout=dd.NATIVE), reps)
        sw16 = (SAP_REALS_PER_SITE * 2 + SAP_SCALE_BYTES_PER_SITE) * V
        kern["sap_colour_pass_f16spinors"] = dict(seconds=t_sh / 2, algorithmic_bytes=sw16 / 2,
                                                  gbs=sw16 / t_sh / 1e9)
        del hb, hz
    t_d16 = time_launches(torch, lambda: dd.apply_Dc(H, 0, nat32, out32, prec=dd.F32, layout=dd.NATIVE), reps)
    d16 = (DPSI_SPINOR_REALS_PER_SITE * 4 + (DPSI_REALS_PER_SITE - DPSI_SPINOR_REALS_PER_SITE) * 2) * V
    kern["dslash_f16store"] = dict(seconds=t_d16, algorithmic_bytes=d16, gbs=d16 / t_d16 / 1e9)
    t_d32 = time_launches(torch, lambda: dd.apply_D(ctx, nat32, out32, prec=dd.F32, layout=dd.NATIVE), reps)
    kern["dslash_f32"] = dict(seconds=t_d32, algorithmic_bytes=DPSI_REALS_PER_SITE * 4 * V,
                              gbs=DPSI_REALS_PER_SITE * 4 * V / t_d32 / 1e9)
    del nat32, zs, out32
    nat64 = torch.zeros(V * 12, dtype=torch.complex128, device=dev)
    out64 = torch.zeros_like(nat64)
    dd.to_native(ctx, None, 0, bd, nat64, prec=dd.F64)
    t_d64 = time_launches(torch, lambda: dd.apply_D(ctx, nat64, out64, prec=dd.F64, layout=dd.NATIVE), reps)
    kern["dslash_f64"] = dict(seconds=t_d64, algorithmic_bytes=DPSI_REALS_PER_SITE * 8 * V,
                              gbs=DPSI_REALS_PER_SITE * 8 * V / t_d64 / 1e9)
    del nat64, out64
    # level-1 coarse operator (12^3x24 sites, 40 components, FP16-stored):
    # one field per launch, and 12 fields on the matrix cores
    (cdims, cd) = dd.level_info(H, 1)
    cV = int(np.prod(cdims))
    cin = torch.randn((BATCH_RHS, cV * cd), dtype=torch.complex64, device=dev)
    cout = torch.zeros_like(cin)
    t_c1 = time_launches(torch, lambda: dd.apply_Dc(H, 1, cin[0], cout[0], prec=dd.F32, layout=dd.NATIVE), reps)
    cbytes = (9 * cd * cd * 4 + 2 * cd * 8) * cV
    kern["coarse_apply_f16store_x1"] = dict(seconds=t_c1, algorithmic_bytes=cbytes, gbs=cbytes / t_c1 / 1e9)
    t_cb = time_launches(torch, lambda: dd.apply_Dc(H, 1, cin, cout, nrhs=BATCH_RHS, prec=dd.F32,
                                                    layout=dd.NATIVE), reps)
    flops = 9 * cd * cd * 8 * BATCH_RHS * cV
    cbb = (9 * cd * cd * 4 + 2 * BATCH_RHS * cd * 8) * cV
    kern[f"coarse_apply_mfma_f16store_x{BATCH_RHS}"] = dict(
        seconds=t_cb, algorithmic_bytes=cbb, gbs=cbb / t_cb / 1e9, tflops=flops / t_cb / 1e12,
        mfma_frac=flops / t_cb / 1e12 / MFMA_F32_PEAK_TFLOPS)
    del cin, cout
    for k, v in kern.items():
        ext = f", {v['tflops']:.1f} TFLOP/s" if "tflops" in v else ""
        log(f"[bench] {k}: {v['seconds'] * 1e6:.1f} us, {v['gbs']:.0f} GB/s{ext}")
    mixed = dict(outer_iters=[s["outer_iters"] for s in stats][-1], true_relres=stats[-1]["true_relres"],
                 kcycle_iters=stats[-1]["kcycle_iters"], coarsest_iters=stats[-1]["coarsest_iters"])
    del H
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # the other spinor storage on the same lattice (FP16 operators), with the
    # per-level GPU times of its solve (event marks where the work changes
    # level: the consumed time per level of the paper's Tab. 4)
    other = None
    if not args.no_other_spinors:
        Ho, t_o = build(dd.F32, True, spinors16=not spinors16, profile=True)
        one_solve(Ho)
        torch.cuda.synchronize()
        to = time.time()
        sto = one_solve(Ho)
        torch.cuda.synchronize()
        to = time.time() - to
        other = dict(spinors="fp32" if spinors16 else "fp16", setup_s=round(t_o, 3), solve_s=round(to, 4),
                     outer_iters=sto["outer_iters"], true_relres=sto["true_relres"],
                     t_level_s=[round(x, 4) for x in sto["t_level_s"]])
        log(f"[bench] {other['spinors']} spinors: solve {to:.3f}s, {sto['outer_iters']} its, "
            f"per-level {other['t_level_s']}")
        del Ho
        torch.cuda.empty_cache()

    # fewer levels on the same lattice (mixed, FP16 storage), one solve each
    levels_cmp = None
    if not args.no_levels:
        levels_cmp = {"4": dict(setup_s=round(t_setup, 3), solve_s=round(ms / 1000.0, 4),
                                outer_iters=mixed["outer_iters"])}
        for L in (3, 2):
            Hl, t_l = build(dd.F32, True, levels=L, spinors16=spinors16)
            one_solve(Hl)
            torch.cuda.synchronize()
            tl = time.time()
            st = one_solve(Hl)
            torch.cuda.synchronize()
            tl = time.time() - tl
            levels_cmp[str(L)] = dict(setup_s=round(t_l, 3), solve_s=round(tl, 4), outer_iters=st["outer_iters"],
                                      kcycle_iters=st["kcycle_iters"], coarsest_iters=st["coarsest_iters"])
            log(f"[bench] {L} levels: setup {t_l:.2f}s, solve {tl:.3f}s, {st['outer_iters']} its, "
                f"{st['coarsest_iters']} coarsest its")
            del Hl
            torch.cuda.empty_cache()

    # plain FP64 GPU method on the same inputs
    plain = None
    if not args.no_plain:
        H64, t_setup64 = build(dd.F64, False)
        one_solve(H64)
        torch.cuda.synchronize()
        tp = time.time()
        pst = one_solve(H64)
        torch.cuda.synchronize()
        tp = time.time() - tp
        plain = dict(time_to_solution_s=round(tp, 4), setup_s=round(t_setup64, 3), outer_iters=pst["outer_iters"],
                     true_relres=pst["true_relres"])
        log(f"[bench] plain FP64: setup {t_setup64:.2f}s, solve {tp:.3f}s, {pst['outer_iters']} its")
        del H64
        torch.cuda.empty_cache()
        # CGNR (the paper's comparison method, Sec. 4; the conditioning indicator)
        zc = torch.zeros_like(bd)
        torch.cuda.synchronize()
        tc = time.time()
        rc, cst = dd.cgnr(ctx, bd, zc, tol=cfg["tol"], max_iter=100000)
        torch.cuda.synchronize()
        tc = time.time() - tc
        plain["cgnr"] = dict(time_s=round(tc, 4), iterations=cst[0]["outer_iters"], true_relres=cst[0]["true_relres"],
                             status=rc)
        log(f"[bench] CGNR FP64: {cst[0]['outer_iters']} its, {tc:.3f}s")

    # the short bare-mass scan towards criticality on the 16^3x32 lattice
    scan = None
    if not args.no_scan:
        rows, _ = m0_scan(W.CONFIGS[WORKLOAD], dd, W, np, torch, SCAN_M0_SHORT,
                          ((3, None, "3lvl"), (2, None, "2lvl")), 1)
        scan = {"lattice": "16^3x32, eps=0.5, c_sw=1, tol 1e-10, b = D z*", "rows": rows}

    if spinors16:
        dom = kern["sap_colour_pass_f16spinors"]
        traffic = SAP_F16S_PASS_TRAFFIC_BYTES
        kname = ("k_sap_colour<float, __half2, __half2> (one SAP colour pass, FP32 arithmetic on FP16 "
                 "links, clover and spinors)")
    else:
        dom = kern["sap_colour_pass_f16store"]
        traffic = SAP_F16_PASS_TRAFFIC_BYTES
        kname = ("k_sap_colour<float, __half2, float2> (one SAP colour pass, FP32 arithmetic on FP16 "
                 "links and clover)")
    sap_flops = SAP_FLOPS_PER_UPDATED_SITE * V / 2
    roofline = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                "algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
                "us_per_launch": round(dom["seconds"] * 1e6, 2),
                # the same launch against the FP32 vector units: its arithmetic
                # intensity (6624 flop per 444 B) lies above their balance point
                "alu": {"achieved": round(sap_flops / dom["seconds"] / 1e12, 2), "peak": VALU_F32_PEAK_TFLOPS,
                        "unit": "TFLOP/s",
                        "frac": round(sap_flops / dom["seconds"] / 1e12 / VALU_F32_PEAK_TFLOPS, 4),
                        "flops_per_launch": sap_flops}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_headline(cfg, U, b, mixed["outer_iters"], V, ms / 1000.0)

    aggs = ", ".join("x".join(str(a) for a in ag) for ag in cfg["agg"])
    line = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 preconditioner on f16-stored operators and fine spinors, f64 outer" if spinors16 else
                  "f32 preconditioner on f16-stored operators, f64 outer"),
        "data": "synthetic (seeded SU(3) links exp(i eps H), one complex Gaussian rhs)",
        "config": {"workload": f"{'x'.join(map(str, dims))} Wilson-clover, {cfg['levels']} levels "
                               f"(aggregates {aggs}, N={cfg['ntv']}, level-2 SAP blocks 3^4), c_sw={cfg['csw']}, "
                               f"eps={cfg['eps']}, m0={cfg['m0']}, 1 rhs, tol 1e-10",
                   "parallelism": "1 GPU"},
        "time_to_solution_s": round(ms / 1000.0, 4),
        "setup_s": round(t_setup, 3),
        **mixed,
        "oracle_sampled_relres": oracle_est,
        "oracle_sampled_max_site_relres": oracle_max,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": (round(plain["time_to_solution_s"] / (ms / 1000.0), 3) if plain else None),
        "other_spinor_storage": other,
        "levels_2_3_4": levels_cmp,
        "m0_scan_16x32": scan,
        "kernels": {k: dict({"us": round(v["seconds"] * 1e6, 2), "GB/s": round(v["gbs"], 1)},
                            **({"TFLOP/s": round(v["tflops"], 2), "mfma_frac": round(v["mfma_frac"], 4)}
                               if "tflops" in v else {})) for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_headline(cfg, U, b, outer_iters, V, gpu_solve_s):
    """The FP64 numpy oracle, unmodified, timed on a bounded sample of the
    headline workload: the 16^3x32 corner of its lattice (its links and
    right-hand side, closed periodically) carries one outer iteration's
    fine-level work (nu = 5 SAP sweeps, one Wilson-clover apply, P^H and P
    with N = 20), scaled to the whole lattice (x V / V_sample) and solve
    (x outer iterations of the GPU run).  The three coarse levels and the
    setup are left out: an upper bound on the oracle's solves per second."""
    import numpy as np

    import workloads as W
    from oracle.aggregation import Aggregation
    from oracle.dirac import WilsonClover
    from oracle.sap import sap_sweep
    sd = (16, 16, 16, 32)
    Us = np.ascontiguousarray(U[:sd[3], :sd[2], :sd[1], :sd[0]])
    bs = np.ascontiguousarray(b[:sd[3], :sd[2], :sd[1], :sd[0]])
    Vs = int(np.prod(sd))
    op = WilsonClover(Us, cfg["m0"], cfg["csw"])
    agg = Aggregation(sd, cfg["agg"][0], W.test_vectors(sd, 12, cfg["ntv"][0], cfg["seed_tv"]))
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t = time.time()
    zc = agg.restrict(bs)
    zf = agg.prolong(zc)
    for _ in range(cfg["nu"]):
        zf = sap_sweep(op, bs, zf, (2, 2, 2, 2), cfg["mr_iters"])
    op.apply(zf)
    wall = time.time() - t
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu_s = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    cores = max(1, int(round(cpu_s / wall)))
    per_solve = wall * (V / Vs) * outer_iters
    model, nproc = cpu_info()
    log(f"[bench] oracle sample {wall:.1f}s wall, {cpu_s:.1f}s cpu; scaled {per_solve:.0f}s per solve")
    return {"value": round(1.0 / per_solve, 8), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"one outer iteration's fine-level work (P^H, P with N=20, 5 SAP sweeps, 1 Dpsi; FP64 "
                      f"numpy) on the 16^3x32 corner of the 48^3x96 lattice took {wall:.2f}s; x{V // Vs} "
                      f"volume, x{outer_iters} outer iterations; coarse levels and setup excluded (upper bound)",
            "host": {"cpu_model": model, "nproc": nproc},
            "core_minutes_per_solve": round(per_solve * cores / 60.0, 2),
            "gpu_speedup": round(per_solve / gpu_solve_s, 1),
            "paper_context": "Tab. 5: 3-level DD-alpha-AMG 160 core-minutes (128 Nehalem cores, 64^4 BMW-c "
                             "ensemble, 75.2 s), CGNR 111,446 core-minutes"}

def big_workload(args, name, cfg, dd, W, np, torch):
    """The larger lattices, run on request: a step is one solve with the
    FP32 preconditioner on FP16-stored operator data and FP16 fine spinors
    (FP32 spinors with --fp32-spinors).  On the 32^3x64
    lattice the 12 spin-colour point sources go through in one batch (the
    coarse operator on the matrix cores); on the 48^3x96 lattice (four
    levels) one Gaussian right-hand side.  The plain FP64 method solves
    sources one at a time for comparison (its own hierarchy, built after the
    first one is freed)."""
    dims = cfg["dims"]
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    nsrc = BATCH_RHS if name == BATCH_WORKLOAD else 1
    log(f"[bench] workload {name} dims={dims} V={V}")
    t0 = time.time()
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    log(f"[bench] links in {time.time() - t0:.1f}s")
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], torch.from_numpy(U).to(dev))
    del U
    tv = W.test_vectors(dims, 12, cfg["ntv"][0], cfg["seed_tv"])
    tvd = torch.from_numpy(tv).to(dev)
    del tv
    log(f"[bench] test vectors in {time.time() - t0:.1f}s")
    extra = None
    if cfg["levels"] == 4 and cfg["ntv"][2] > cfg["ntv"][1]:
        # fresh random test vectors for the level with more of them (level 2)
        d2 = 2 * cfg["ntv"][1]
        cd2 = tuple(x // (a1 * a2) for x, a1, a2 in zip(dims, cfg["agg"][0], cfg["agg"][1]))
        extra = torch.from_numpy(W.test_vectors(cd2, d2, cfg["ntv"][2] - cfg["ntv"][1],
                                                cfg["seed_tv"] + 7)).to(dev)
    if nsrc > 1:
        b = torch.from_numpy(W.point_sources(dims)).to(dev)
        src = "12 spin-colour point sources in one batch"
    else:
        b = torch.from_numpy(W.gaussian_spinor(dims, cfg["seed_rhs"])).unsqueeze(0).to(dev)
        src = "one complex Gaussian rhs"
    z = torch.zeros_like(b)
    log(f"[bench] inputs in {time.time() - t0:.1f}s")

    def params(prec, half, batch):
        p = dd.params_default(cfg["levels"])
        for l, a in enumerate(cfg["agg"]):
            for mu in range(4):
                p.agg[l][mu] = a[mu]
        for l, n in enumerate(cfg["ntv"]):
            p.ntv[l] = n
        for l, blk in enumerate(cfg.get("sap_blocks", [])[1:]):
            for mu in range(4):
                p.sap_block_l[l][mu] = blk[mu]
        p.nu = cfg["nu"]
        p.precond_prec = prec
        p.half_storage = 1 if half else 0
        p.half_spinors = 1 if half and spinors16 else 0
        p.batch = batch
        return p

    def build(prec, half, batch):
        torch.cuda.synchronize()
        t = time.time()
        H = dd.build_hierarchy(ctx, params(prec, half, batch), tvd, extra)
        torch.cuda.synchronize()
        return H, time.time() - t

    spinors16 = not args.fp32_spinors

    def solve(Hh, nb):
        z.zero_()
        torch.cuda.synchronize()
        t = time.time()
        rc, st = dd.solve(Hh, b[:nb], z[:nb], nrhs=nb)
        torch.cuda.synchronize()
        if rc != dd.OK:
            raise RuntimeError(f"solve failed rc={rc}")
        return time.time() - t, st

    # batch: the 20 setup test vectors in one batch (and the 12 sources in
    # one batched solve) on 32^3x64; 8 on the four-level lattice
    H, t_setup = build(dd.F32, True, 8 if cfg["levels"] == 4 else max(BATCH_RHS, cfg["ntv"][0]))
    log(f"[bench] mixed FP16-storage setup {t_setup:.2f}s")
    for i in range(args.warmup):
        tw, st = solve(H, nsrc)
        log(f"[bench] warmup {i}: {tw:.3f}s")
    times, stats = [], None
    for i in range(args.steps):
        tt, stats = solve(H, nsrc)
        times.append(tt)
        log(f"[bench] step {i}: {nsrc} rhs in {tt:.3f}s, its {[x['outer_iters'] for x in stats]}")
    ms = 1000.0 * float(np.mean(times))
    plain = None
    if not args.no_plain:
        del H
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        H64, t_setup64 = build(dd.F64, False, 1)
        n_plain = min(2, nsrc)
        tp, stp = solve(H64, n_plain)
        plain = dict(setup_s=round(t_setup64, 3), sources_timed=n_plain,
                     per_source_s=round(tp / n_plain, 4), outer_iters=[x["outer_iters"] for x in stp])
        log(f"[bench] plain FP64: setup {t_setup64:.2f}s, {tp / n_plain:.3f}s per source")
    aggs = ", ".join("x".join(str(a) for a in ag) for ag in cfg["agg"])
    line = {
        "metric": METRIC,
        "value": round(nsrc / (ms / 1000.0), 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 preconditioner on f16-stored operators and fine spinors, f64 outer" if spinors16 else
                  "f32 preconditioner on f16-stored operators, f64 outer"),
        "data": "synthetic (seeded SU(3) links exp(i eps H), " + src + ")",
        "config": {"workload": f"{'x'.join(map(str, dims))} Wilson-clover, {cfg['levels']} levels "
                               f"(aggregates {aggs}, N={cfg['ntv']}), c_sw={cfg['csw']}, eps={cfg['eps']}, "
                               f"m0={cfg['m0']}, {src}, tol 1e-10",
                   "parallelism": "1 GPU"},
        "setup_s": round(t_setup, 3),
        "outer_iters": [x["outer_iters"] for x in stats],
        "max_true_relres": max(x["true_relres"] for x in stats),
        "plain_fp64": plain,
        "speedup_vs_plain_fp64_per_source": (round(plain["per_source_s"] / (ms / 1000.0 / nsrc), 3)
                                             if plain else None),
    }
    print(json.dumps(line), flush=True)


def kernels_only(args, cfg, dd, W, np, torch):
    """The fine kernels alone, for hardware-counter runs: the Wilson-clover
    stencil in FP32 and FP64, one SAP sweep (two colour passes) on FP16-stored
    links and clover, one in FP32 and one on FP16 links, clover and spinors,
    each from a cheap two-level hierarchy
    (the fine smoother reads only the fine operator), and a 1 GiB device copy
    (the reference for scaling FETCH_SIZE / WRITE_SIZE counters)."""
    dims = tuple(int(x) for x in args.lattice.split(",")) if args.lattice else cfg["dims"]
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    t0 = time.time()
    U = W.links(dims, cfg["eps"], cfg["seed_links"])
    b = W.gaussian_spinor(dims, cfg["seed_rhs"])
    log(f"[bench] kernels-only dims={dims} inputs in {time.time() - t0:.1f}s")
    ctx = dd.create(dims, cfg["m0"], cfg["csw"], torch.from_numpy(U).to(dev))
    del U
    bd = torch.from_numpy(b).to(dev)
    out = {}
    for name, prec, cdt, bpr in (("dslash_f32", dd.F32, torch.complex64, 4),
                                 ("dslash_f64", dd.F64, torch.complex128, 8)):
        x = torch.zeros(V * 12, dtype=cdt, device=dev)
        y = torch.zeros_like(x)
        dd.to_native(ctx, None, 0, bd, x, prec=prec)
        t = time_launches(torch, lambda: dd.apply_D(ctx, x, y, prec=prec, layout=dd.NATIVE), args.kernel_reps)
        nbytes = DPSI_REALS_PER_SITE * bpr * V
        out[name] = {"us": round(t * 1e6, 2), "GB/s": round(nbytes / t / 1e9, 1), "algorithmic_bytes": nbytes}
        log(f"[bench] {name}: {t * 1e6:.1f} us, {nbytes / t / 1e9:.0f} GB/s")
        del x, y
    tv = device_fields(torch, W, dims, 12, 2, cfg["seed_tv"])
    x = torch.zeros(V * 12, dtype=torch.complex64, device=dev)
    dd.to_native(ctx, None, 0, bd, x, prec=dd.F32)
    zf = torch.zeros_like(x)
    for name, half in (("sap_colour_pass_f16store", True), ("sap_colour_pass_f32", False)):
        p = dd.params_default(2)
        p.ntv[0] = 2
        p.n_inv = 0
        p.precond_prec = dd.F32
        p.half_storage = 1 if half else 0
        H = dd.build_hierarchy(ctx, p, tv)
        t = time_launches(torch, lambda: dd.sap_smooth(H, 0, x, zf, 1, prec=dd.F32, layout=dd.NATIVE),
                          args.kernel_reps) / 2
        nbytes = ((SAP_SPINOR_REALS_PER_SITE * 4 + (SAP_REALS_PER_SITE - SAP_SPINOR_REALS_PER_SITE) * 2) * V / 2
                  if half else SAP_REALS_PER_SITE * 4 * V / 2)
        out[name] = {"us": round(t * 1e6, 2), "GB/s": round(nbytes / t / 1e9, 1), "algorithmic_bytes": nbytes}
        log(f"[bench] {name}: {t * 1e6:.1f} us per colour pass, {nbytes / t / 1e9:.0f} GB/s")
        del H
    # the pass on FP16 spinors (native form: entries, then site scales)
    p = dd.params_default(2)
    p.ntv[0] = 2
    p.n_inv = 0
    p.precond_prec = dd.F32
    p.half_storage = 1
    p.half_spinors = 1
    H = dd.build_hierarchy(ctx, p, tv)
    hb = torch.empty(V * 13, dtype=torch.float32, device=dev)
    hz = torch.zeros_like(hb)
    dd.to_native(ctx, None, 0, bd, hb, prec=dd.F16S)
    t = time_launches(torch, lambda: dd.sap_smooth(H, 0, hb, hz, 1, prec=dd.F16S, layout=dd.NATIVE),
                      args.kernel_reps) / 2
    nbytes = (SAP_REALS_PER_SITE * 2 + SAP_SCALE_BYTES_PER_SITE) * V / 2
    out["sap_colour_pass_f16spinors"] = {"us": round(t * 1e6, 2), "GB/s": round(nbytes / t / 1e9, 1),
                                         "algorithmic_bytes": nbytes}
    log(f"[bench] sap_colour_pass_f16spinors: {t * 1e6:.1f} us per colour pass, {nbytes / t / 1e9:.0f} GB/s")
    del H, hb, hz
    # reference copy of known size: 1 GiB read + 1 GiB written
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"lattice": dims, "kernels": out, "copy_bytes_each_way": a.numel() * 8}), flush=True)


def cpu_baseline(cfg, U, b, outer_iters, V):
    """The FP64 numpy oracle, unmodified, on a bounded sample of the same
    workload: one outer iteration's fine-level work (nu = 5 SAP sweeps and one
    Wilson-clover apply) on the full 16^3x32 lattice, scaled to a whole solve
    by the GPU run's outer iteration count.  Coarse levels and setup are left
    out, so the figure is an upper bound on the oracle's solves per second."""
    import numpy as np

    from oracle.dirac import WilsonClover
    from oracle.sap import sap_sweep
    t_build = time.time()
    op = WilsonClover(U, cfg["m0"], cfg["csw"])
    log(f"[bench] oracle operator built in {time.time() - t_build:.1f}s")
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t = time.time()
    z = np.zeros_like(b)
    for _ in range(cfg["nu"]):
        z = sap_sweep(op, b, z, (2, 2, 2, 2), cfg["mr_iters"])
    op.apply(z)
    wall = time.time() - t
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu_s = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    per_solve = wall * outer_iters
    log(f"[bench] oracle sample {wall:.1f}s wall, {cpu_s:.1f}s cpu")
    return {"value": round(1.0 / per_solve, 6), "unit": "solves/s",
            "cores": max(1, int(round(cpu_s / wall))), "kind": "oracle",
            "sample": f"fine-level work of one outer iteration (5 SAP sweeps + 1 Dpsi, FP64 numpy) on the "
                      f"full 16^3x32 lattice took {wall:.2f}s; x{outer_iters} outer iterations; coarse "
                      f"levels and setup excluded (upper bound)"}


def uneven_workload(args, dd, W, np, torch):
    """The uneven batch: eight independent lattices (four 16^4, two 24^3x48,
    two 32^3x64; own links, eps 0.45-0.6, m0 -0.45..-0.3), each with its own
    three-level hierarchy (FP32 preconditioner, FP64 outer FGMRES, one
    complex Gaussian right-hand side).  A step solves all eight with
    ddamg_solve_many (concurrently, one stream per hierarchy) using the
    K-cycle, after the autotuner has chosen each hierarchy's level-1 SAP
    block shape.  Also timed: the same eight one after another; the V-cycle,
    host-driven and graph-captured (coarsest GMRES with device-side scalars
    and a fixed launch sequence); the plain FP64 method one after another."""
    dev = torch.device("cuda:0")
    n = len(W.UNEVEN_BATCH)
    cfgs = [W.uneven_batch_config(j) for j in range(n)]
    sites = sum(int(np.prod(c["dims"])) for c in cfgs)
    log(f"[bench] workload {UNEVEN_WORKLOAD}: {n} lattices, {sites} fine sites")

    def params(cfg, prec, cycle, graph=False):
        p = dd.params_default(cfg["levels"])
        for l, a in enumerate(cfg["agg"]):
            for mu in range(4):
                p.agg[l][mu] = a[mu]
        for l, k in enumerate(cfg["ntv"]):
            p.ntv[l] = k
        for l, blk in enumerate(cfg["sap_blocks"][1:]):
            for mu in range(4):
                p.sap_block_l[l][mu] = blk[mu]
        p.nu = cfg["nu"]
        p.cycle = dd.VCYCLE if cycle == "V" else dd.KCYCLE
        p.precond_prec = prec
        p.batch = 1
        if graph:
            p.graph = 1
            p.coarse_restart, p.coarse_max_restarts = GRAPH_COARSE
        return p

    ctxs, tvs, bs, zs = [], [], [], []
    for j, cfg in enumerate(cfgs):
        t = time.time()
        dims = cfg["dims"]
        U = W.links(dims, cfg["eps"], cfg["seed_links"])
        ctxs.append(dd.create(dims, cfg["m0"], cfg["csw"], torch.from_numpy(U).to(dev)))
        del U
        tvs.append(torch.from_numpy(W.test_vectors(dims, 12, cfg["ntv"][0], cfg["seed_tv"])).to(dev))
        bs.append(torch.from_numpy(W.gaussian_spinor(dims, cfg["seed_rhs"])).unsqueeze(0).to(dev))
        zs.append(torch.zeros_like(bs[-1]))
        log(f"[bench] lattice {j} {dims} eps={cfg['eps']} m0={cfg['m0']}: inputs {time.time() - t:.1f}s")

    def build_set(prec, cycle, graph=False):
        hs, su = [], []
        for j, cfg in enumerate(cfgs):
            torch.cuda.synchronize()
            t = time.time()
            hs.append(dd.build_hierarchy(ctxs[j], params(cfg, prec, cycle, graph), tvs[j]))
            torch.cuda.synchronize()
            su.append(round(time.time() - t, 3))
        return hs, su

    def zero_all():
        for z in zs:
            z.zero_()
        torch.cuda.synchronize()

    def together(hs, one_graph=False):
        zero_all()
        t = time.time()
        rc, st = (dd.solve_batch if one_graph else dd.solve_many)(hs, bs, zs)
        torch.cuda.synchronize()
        return time.time() - t, rc, st

    def one_by_one(hs):
        zero_all()
        per, stats = [], []
        for H, b, z in zip(hs, bs, zs):
            t = time.time()
            rc, st = dd.solve(H, b, z)
            torch.cuda.synchronize()
            per.append(time.time() - t)
            stats += st
        return per, stats

    def summary(st):
        return dict(status=[x["status"] for x in st], outer_iters=[x["outer_iters"] for x in st],
                    coarsest_iters=[x["coarsest_iters"] for x in st],
                    max_true_relres=max(x["true_relres"] for x in st))

    def run_set(name, prec, cycle, graph, reps, tune=False, one_graph=False):
        hs, su = build_set(prec, cycle, graph)
        log(f"[bench] {name}: setup {su}")
        tuned = None
        if tune:
            t_untuned, _, st0 = together(hs)
            log(f"[bench] {name}, together before tuning: {t_untuned:.3f}s")
            t = time.time()
            choice = [dd.tune(H, b, nrhs=1) for H, b in zip(hs, bs)]
            tuned = dict(search_s=round(time.time() - t, 2), together_before_s=round(t_untuned, 4),
                         sap_block_level1=[c["sap_block_l"][0] for c in choice])
            log(f"[bench] {name}: tuned in {tuned['search_s']}s, level-1 SAP blocks {tuned['sap_block_level1']}")
        times, st = [], None
        for i in range(reps):
            tt, rc, st = together(hs, one_graph)
            times.append(tt)
            log(f"[bench] {name}, together #{i}: {tt:.3f}s rc={rc} its {[x['outer_iters'] for x in st]} "
                f"coarsest {[x['coarsest_iters'] for x in st]}")
        per, st1 = one_by_one(hs)
        log(f"[bench] {name}, one after another: {sum(per):.3f}s {[round(x, 4) for x in per]} "
            f"its {[x['outer_iters'] for x in st1]}")
        out = dict(setup_s=su, together_s=round(float(np.mean(times[-max(1, reps - 1):])), 4),
                   one_after_another_s=round(sum(per), 4), per_system_alone_s=[round(x, 4) for x in per],
                   **summary(st))
        if tuned:
            out["autotuned"] = tuned
        del hs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return out, times

    reps = args.warmup + args.steps
    kres, ktimes = run_set("mixed K-cycle", dd.F32, "K", False, reps, tune=True)
    vres, _ = run_set("mixed V-cycle", dd.F32, "V", False, 2)
    gres, _ = run_set("mixed V-cycle, graph-captured", dd.F32, "V", True, 3)
    gres["coarsest_budget"] = {"restart": GRAPH_COARSE[0], "cycles": GRAPH_COARSE[1]}
    # the same hierarchies through ddamg_solve_batch: one graph per outer
    # step over all eight systems, the outer scalars and convergence flags
    # on the device
    bres, _ = run_set("mixed V-cycle, one graph over all systems", dd.F32, "V", True, 3, one_graph=True)
    bres["coarsest_budget"] = gres["coarsest_budget"]
    plain = None
    if not args.no_plain:
        per, its, su, stat = [], [], [], []
        for j, cfg in enumerate(cfgs):
            torch.cuda.synchronize()
            t = time.time()
            H64 = dd.build_hierarchy(ctxs[j], params(cfg, dd.F64, "K"), tvs[j])
            torch.cuda.synchronize()
            su.append(round(time.time() - t, 3))
            zs[j].zero_()
            torch.cuda.synchronize()
            t = time.time()
            rc, st = dd.solve(H64, bs[j], zs[j])
            torch.cuda.synchronize()
            per.append(time.time() - t)
            its.append(st[0]["outer_iters"])
            stat.append(st[0]["status"])
            del H64
            log(f"[bench] plain FP64 lattice {j}: setup {su[-1]:.2f}s, solve {per[-1]:.3f}s rc={rc}, its {its[-1]}")
        plain = dict(total_s=round(sum(per), 4), per_system_s=[round(x, 4) for x in per], outer_iters=its,
                     status=stat, setup_s=su)
    # CGNR iteration counts: the conditioning indicator of the paper's Tab. 2
    cgn = None
    if not args.no_plain:
        cgn = dict(iterations=[], seconds=[])
        for j in range(n):
            zs[j].zero_()
            rc, st = dd.cgnr(ctxs[j], bs[j], zs[j], tol=1e-10, max_iter=20000)
            cgn["iterations"].append(st[0]["outer_iters"])
            cgn["seconds"].append(round(st[0]["seconds"], 3))
            log(f"[bench] CGNR lattice {j}: {st[0]['outer_iters']} its, {st[0]['seconds']:.2f}s rc={rc}")
    ms = 1000.0 * float(np.mean(ktimes[args.warmup:] or ktimes))
    line = {
        "metric": METRIC,
        "value": round(n / (ms / 1000.0), 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 outer",
        "data": "synthetic (seeded SU(3) links exp(i eps H) per lattice, one Gaussian rhs each)",
        "config": {"workload": "uneven batch of 8 independent Wilson-clover lattices (4 x 16^4, 2 x 24^3x48, "
                               "2 x 32^3x64; eps 0.45-0.6, m0 -0.45..-0.3, massive side of criticality, c_sw=1), "
                               "3 levels each, K-cycle, tol 1e-10, solved concurrently",
                   "parallelism": "1 GPU"},
        "fine_sites": sites,
        "kcycle": kres,
        "vcycle": vres,
        "vcycle_graph_captured": gres,
        "vcycle_one_graph_all_systems": bres,
        "plain_fp64": plain,
        "cgnr_fp64": cgn,
        "speedup_vs_plain_fp64": round(plain["total_s"] / (ms / 1000.0), 3) if plain else None,
    }
    print(json.dumps(line), flush=True)


def m0_scan(cfg, dd, W, np, torch, masses, variants, reps):
    """Critical slowing down on synthetic links: the 16^3x32 workload's links
    (eps 0.5) with the bare mass m0 moved towards the critical value; for
    each m0 the mixed-precision multigrid solves of `variants` (levels,
    cycle, key) and FP64 CGNR, with b = D z* for a Gaussian z* so that the
    error ||z - z*|| / ||z*|| is reported next to the residual (the paper's
    m0 scans, 2 vs 3 levels and comparison with CGNR).  Returns the rows
    and the mean first-variant solve time."""
    dims = cfg["dims"]
    dev = torch.device("cuda:0")
    U = torch.from_numpy(W.links(dims, cfg["eps"], cfg["seed_links"])).to(dev)
    zstar = torch.from_numpy(W.gaussian_spinor(dims, cfg["seed_rhs"])).unsqueeze(0).to(dev)
    b = torch.zeros_like(zstar)
    tv = torch.from_numpy(W.test_vectors(dims, 12, cfg["ntv"][0], cfg["seed_tv"])).to(dev)
    z = torch.zeros_like(b)

    def params(levels, cycle=None):
        p = dd.params_default(levels)
        for l in range(levels - 1):
            for mu in range(4):
                p.agg[l][mu] = cfg["agg"][l][mu]
            p.ntv[l] = cfg["ntv"][l]
        p.nu = cfg["nu"]
        p.precond_prec = dd.F32
        if cycle is not None:
            p.cycle = cycle
        return p

    def timed_solve(H):
        z.zero_()
        torch.cuda.synchronize()
        t = time.time()
        rc, st = dd.solve(H, b, z)
        torch.cuda.synchronize()
        return time.time() - t, rc, st[0]

    def error(x):
        return float(torch.linalg.vector_norm(x - zstar) / torch.linalg.vector_norm(zstar))

    rows, t_first = [], []
    for m0 in masses:
        ctx = dd.create(dims, m0, cfg["csw"], U)
        dd.apply_D(ctx, zstar, b, prec=dd.F64)
        row = {"m0": m0}
        for levels, cyc, key in variants:
            torch.cuda.synchronize()
            t = time.time()
            H = dd.build_hierarchy(ctx, params(levels, cyc), tv)
            torch.cuda.synchronize()
            t_setup = time.time() - t
            timed_solve(H)
            ts = [timed_solve(H) for _ in range(max(1, reps))]
            t_solve = min(x[0] for x in ts)
            rc, st = ts[-1][1], ts[-1][2]
            row[key] = dict(setup_s=round(t_setup, 3), solve_s=round(t_solve, 4),
                            outer_iters=st["outer_iters"], status=rc, true_relres=st["true_relres"],
                            rel_error=error(z))
            if key == variants[0][2]:
                t_first.append(t_solve)
            del H
        zc = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.time()
        rc, cst = dd.cgnr(ctx, b, zc, tol=cfg["tol"], max_iter=200000)
        torch.cuda.synchronize()
        row["cgnr"] = dict(iterations=cst[0]["outer_iters"], solve_s=round(time.time() - t, 3), status=rc,
                           rel_error=error(zc))
        rows.append(row)
        log(f"[bench] m0={m0}: " + ", ".join(f"{k} {v.get('outer_iters', v.get('iterations'))} its "
                                               f"{v['solve_s']}s err {v['rel_error']:.1e}"
                                               for k, v in row.items() if k != "m0"))
        del ctx
    return rows, float(np.mean(t_first))


def scan_workload(args, cfg, dd, W, np, torch):
    """The bare-mass scan as a workload of its own: three levels (K-, V- and
    W-cycle) and two levels against CGNR at every mass of SCAN_M0.  A step is
    one pass over the masses; `value` is the three-level K-cycle solves per
    second over the scan."""
    log(f"[bench] workload {SCAN_WORKLOAD} dims={cfg['dims']} m0={SCAN_M0}")
    rows, t3 = m0_scan(cfg, dd, W, np, torch, SCAN_M0,
                       ((3, None, "3lvl"), (2, None, "2lvl"), (3, dd.VCYCLE, "3lvl_vcycle"),
                        (3, dd.WCYCLE, "3lvl_wcycle")), args.steps)
    ms = 1000.0 * t3
    line = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 outer",
        "data": "synthetic (seeded SU(3) links exp(i eps H), b = D z* for a Gaussian z*)",
        "config": {"workload": f"16^3x32 Wilson-clover, eps=0.5, c_sw=1, m0 scan {list(SCAN_M0)}, "
                               "3 levels (K-, V-, W-cycle) and 2 levels against FP64 CGNR, tol 1e-10",
                   "parallelism": "1 GPU"},
        "scan": rows,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
