"""The C-ABI library loads, exports every symbol include/ddamg.h declares,
its structs match the header's layout, and host-side argument checks reject
bad input before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddamg.h")


@pytest.fixture(scope="module")
def dd():
    from paper_1307_6101_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_1307_6101_amd import ddamg
    ddamg.load_library()
    return ddamg


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddamg_[a-zA-Z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(dd):
    lib = dd.load_library()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(dd._SIGS), set(names) ^ set(dd._SIGS)


def test_struct_layout_matches_header(tmp_path, dd):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "ddamg.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(ddamg_lattice), sizeof(ddamg_params), sizeof(ddamg_solve_stats));
  printf("%zu %zu %zu %zu\n", offsetof(ddamg_params, coarse_eps), offsetof(ddamg_params, kc_tol),
         offsetof(ddamg_params, tol), offsetof(ddamg_params, cycle));
  printf("%zu %zu\n", offsetof(ddamg_solve_stats, true_relres), offsetof(ddamg_solve_stats, seconds));
  printf("%zu %zu %zu %zu\n", sizeof(ddamg_tune_result), offsetof(ddamg_tune_result, batch),
         offsetof(ddamg_tune_result, seconds), offsetof(ddamg_tune_result, from_cache));
  printf("%zu %zu %zu %zu %zu\n", offsetof(ddamg_params, half_storage), offsetof(ddamg_params, batch),
         offsetof(ddamg_params, sap_block_l), offsetof(ddamg_params, half_directions),
         offsetof(ddamg_params, graph));
  printf("%zu %zu %zu %zu\n", offsetof(ddamg_params, coarse_dense), offsetof(ddamg_params, galerkin_cols),
         offsetof(ddamg_params, profile_levels), offsetof(ddamg_params, half_spinors));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(ddamg_solve_stats, err_vs_ref), offsetof(ddamg_solve_stats, t_setup_s),
         offsetof(ddamg_solve_stats, t_level_s), offsetof(ddamg_solve_stats, bytes),
         offsetof(ddamg_solve_stats, flops), offsetof(ddamg_solve_stats, coarsest_dense));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(dd.Lattice)
    assert vals[1] == ctypes.sizeof(dd.Params)
    assert vals[2] == ctypes.sizeof(dd.SolveStats)
    assert vals[3] == dd.Params.coarse_eps.offset
    assert vals[4] == dd.Params.kc_tol.offset
    assert vals[5] == dd.Params.tol.offset
    assert vals[6] == dd.Params.cycle.offset
    assert vals[7] == dd.SolveStats.true_relres.offset
    assert vals[8] == dd.SolveStats.seconds.offset
    assert vals[9] == ctypes.sizeof(dd.TuneResult)
    assert vals[10] == dd.TuneResult.batch.offset
    assert vals[11] == dd.TuneResult.seconds.offset
    assert vals[12] == dd.TuneResult.from_cache.offset
    assert vals[13] == dd.Params.half_storage.offset
    assert vals[14] == dd.Params.batch.offset
    assert vals[15] == dd.Params.sap_block_l.offset
    assert vals[16] == dd.Params.half_directions.offset
    assert vals[17] == dd.Params.graph.offset
    assert vals[18] == dd.Params.coarse_dense.offset
    assert vals[19] == dd.Params.galerkin_cols.offset
    assert vals[20] == dd.Params.profile_levels.offset
    assert vals[21] == dd.Params.half_spinors.offset
    assert vals[22:28] == [dd.SolveStats.err_vs_ref.offset, dd.SolveStats.t_setup_s.offset,
                           dd.SolveStats.t_level_s.offset, dd.SolveStats.bytes.offset,
                           dd.SolveStats.flops.offset, dd.SolveStats.coarsest_dense.offset]


def test_params_default_is_table1(dd):
    p = dd.params_default(3)
    assert p.levels == 3
    assert list(p.agg[0]) == [4, 4, 4, 4] and list(p.agg[1]) == [2, 2, 2, 2]
    assert list(p.ntv) == [20, 20, 20]
    assert list(p.sap_block) == [2, 2, 2, 2]
    assert (p.mu, p.nu, p.mr_iters, p.n_inv) == (0, 5, 3, 6)
    assert (p.kc_len, p.kc_restarts, p.nkv) == (5, 2, 10)
    assert p.coarse_eps == 5e-2 and p.kc_tol == 1e-1 and p.tol == 1e-10
    assert p.precond_prec == dd.F32 and p.cycle == dd.KCYCLE
    assert p.half_storage == 0 and p.batch == 16 and p.half_directions == 0
    # beyond Tab. 1: host-driven coarsest GMRES, dense Schur product where small
    assert p.graph == 0 and p.coarse_dense == 1
    assert p.galerkin_cols == 0 and p.profile_levels == 0 and p.half_spinors == 0


def test_host_validation_rejects_bad_lattice(dd):
    lib = dd.load_library()
    h = ctypes.c_void_p()
    for dims in ((6, 8, 8, 8), (8, 8, 8, 0), (8, 8, 2, 8)):
        lat = dd.Lattice((ctypes.c_int * 4)(*dims), -0.3, 1.0)
        rc = lib.ddamg_create(ctypes.byref(lat), ctypes.c_void_p(16), None, ctypes.byref(h))
        assert rc == dd.EINVAL
        assert b"multiple of 4" in lib.ddamg_last_error()
    lat = dd.Lattice((ctypes.c_int * 4)(8, 8, 8, 8), -0.3, 1.0)
    assert lib.ddamg_create(ctypes.byref(lat), None, None, ctypes.byref(h)) == dd.EINVAL
    assert lib.ddamg_create(None, ctypes.c_void_p(16), None, ctypes.byref(h)) == dd.EINVAL


def test_null_handles_rejected(dd):
    lib = dd.load_library()
    assert lib.ddamg_apply_D(None, ctypes.c_void_p(16), ctypes.c_void_p(32), 1, 0, 0, None) == dd.EINVAL
    assert lib.ddamg_solve(None, ctypes.c_void_p(16), ctypes.c_void_p(32), 1, None, None) == dd.EINVAL
    assert lib.ddamg_apply_Dc(None, 1, ctypes.c_void_p(16), ctypes.c_void_p(32), 1, 0, 0, None) == dd.EINVAL
    assert b"null" in lib.ddamg_last_error()


def test_solve_many_validation(dd):
    """Checked on the host before any device call."""
    lib = dd.load_library()
    P = ctypes.c_void_p
    one = (P * 1)(P(16))
    bz = (P * 1)(P(32))
    zz = (P * 1)(P(48))
    n1 = (ctypes.c_int * 1)(1)
    assert lib.ddamg_solve_many(0, one, bz, zz, n1, None, None) == dd.EINVAL
    assert lib.ddamg_solve_many(65, one, bz, zz, n1, None, None) == dd.EINVAL
    assert lib.ddamg_solve_many(1, None, bz, zz, n1, None, None) == dd.EINVAL
    assert lib.ddamg_solve_many(1, (P * 1)(None), bz, zz, n1, None, None) == dd.EINVAL
    assert b"null" in lib.ddamg_last_error()
    two = (P * 2)(P(16), P(16))
    b2 = (P * 2)(P(32), P(64))
    z2 = (P * 2)(P(48), P(80))
    n2 = (ctypes.c_int * 2)(1, 1)
    assert lib.ddamg_solve_many(2, two, b2, z2, n2, None, None) == dd.EINVAL
    assert b"twice" in lib.ddamg_last_error()
    assert lib.ddamg_solve_many(1, one, bz, bz, n1, None, None) == dd.EINVAL
    assert lib.ddamg_solve_many(1, one, bz, zz, (ctypes.c_int * 1)(0), None, None) == dd.EINVAL


def _round(b):
    return (b + 255) // 256 * 256


def test_workspace_bytes_counts_the_layout(dd):
    """The workspace query runs the handles' allocation sequence against a
    counter on the host: it needs no GPU, and its totals follow the array
    sizes of the layout exactly."""
    dims = (16, 16, 16, 16)
    V = 16 ** 4
    c1, h0 = dd.workspace_bytes(dims, -0.3, 1.0, None, 1)
    assert h0 == 0
    # links and clover in FP64 and FP32, neighbour tables, two scratch fields
    ops = 2 * _round(V * 36 * 16) + 2 * _round(V * 36 * 8)
    scr = 2 * _round(V * 12 * 16)
    tables = _round(V // 16 * 8 * 4) + _round(V // 16 * 4)
    assert c1 == ops + scr + tables
    c3, _ = dd.workspace_bytes(dims, -0.3, 1.0, None, 3)
    assert c3 - c1 == 2 * (_round(3 * V * 12 * 16) - _round(V * 12 * 16))
    p = dd.params_default(3)
    p.ntv[0], p.ntv[1] = 8, 8
    p.agg[1][:] = [2, 2, 2, 2]
    c_nohalf, h1 = dd.workspace_bytes(dims, -0.3, 1.0, p, 1)
    assert c_nohalf == c1
    # at least P_0, P_1 (FP64 + FP32), the test vectors (FP64 + FP32) and
    # the coarse operators (five FP64 blocks, nine in FP64 and FP32)
    n0, V1, d1 = V * 12, V // 256, 16
    n1 = V1 * d1
    V2, d2 = V1 // 16, 16
    lower = (8 * n0 + 8 * n1) * (16 + 8) * 2 + (V1 * d1 * d1 + V2 * d2 * d2) * (5 * 16 + 9 * 24)
    assert h1 > lower
    _, h4 = dd.workspace_bytes(dims, -0.3, 1.0, p, 4)
    assert h4 > h1
    p.half_storage = 1
    c_half, h1h = dd.workspace_bytes(dims, -0.3, 1.0, p, 1)
    assert c_half - c1 == 2 * _round(V * 36 * 4)
    assert h1h < h1      # FP16 copies of P and D_c in place of the FP32 ones


def test_workspace_validation_on_host(dd):
    lib = dd.load_library()
    lat = dd.Lattice((ctypes.c_int * 4)(8, 8, 8, 8), -0.3, 1.0)
    cb = ctypes.c_size_t(0)
    assert lib.ddamg_workspace_bytes(ctypes.byref(lat), None, 0, ctypes.byref(cb), None) == dd.EINVAL
    p = dd.params_default(2)
    p.agg[0][:] = [3, 4, 4, 4]
    hb = ctypes.c_size_t(0)
    assert lib.ddamg_workspace_bytes(ctypes.byref(lat), ctypes.byref(p), 1, ctypes.byref(cb),
                                     ctypes.byref(hb)) == dd.EINVAL
    # a workspace smaller than the count, or misaligned, is refused before any device work
    need, _ = dd.workspace_bytes((8, 8, 8, 8), -0.3, 1.0, None, 1)
    h = ctypes.c_void_p()
    rc = lib.ddamg_create_ws(ctypes.byref(lat), ctypes.c_void_p(256), None, 1, ctypes.c_void_p(1 << 20),
                             ctypes.c_size_t(need - 1), None, ctypes.byref(h))
    assert rc == dd.EINVAL and b"needed" in lib.ddamg_last_error()
    rc = lib.ddamg_create_ws(ctypes.byref(lat), ctypes.c_void_p(256), None, 1, ctypes.c_void_p((1 << 20) + 64),
                             ctypes.c_size_t(need), None, ctypes.byref(h))
    assert rc == dd.EINVAL and b"aligned" in lib.ddamg_last_error()
    assert lib.ddamg_build_hierarchy_ws(None, ctypes.byref(p), ctypes.c_void_p(256), None, 1,
                                        ctypes.c_void_p(1 << 20), ctypes.c_size_t(1 << 30), None,
                                        ctypes.byref(h)) == dd.EINVAL
