"""Seeded synthetic inputs for the DD-alpha-AMG hot path.

This module is shared by the CPU oracle and by the GPU path.  It only draws
random numbers and builds test inputs (gauge links, right-hand sides, initial
test vectors); it holds none of the solver's arithmetic.

The paper (Sec. 3, Tab. 2) measures on real gauge ensembles (BMW-c 48^4 and
64^4, CLS 128x64^3) that are not available here.  Synthetic links of the same
structure stand in for them: every link is an SU(3) matrix U = exp(i eps H)
with H a traceless Hermitian Gaussian matrix.

Conventions shared by everything in this repository:

* a lattice is given by ``dims = (X, Y, Z, T)``; direction mu = 0, 1, 2, 3 is
  x, y, z, t; the canonical site index is ``x + X*(y + Y*(z + Z*t))``, so a
  field is a C-ordered numpy array of shape ``(T, Z, Y, X, ...)``;
* a fine spinor has 12 complex components per site, index ``spin*3 + colour``;
* links have shape ``(T, Z, Y, X, 4, 3, 3)`` (direction, row, column).
"""
from __future__ import annotations

import os

import numpy as np

BASE_SEED = 13076101

# Gell-Mann matrices lambda_1..lambda_8 (standard normalisation tr(l_a l_b) = 2 delta_ab).
_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def _shape(dims):
    X, Y, Z, T = dims
    return (T, Z, Y, X)


def volume(dims) -> int:
    return int(np.prod(dims))


def su3_exp(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices, via eigh."""
    w, W = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ab,...b,...cb->...ac", W, ph, W.conj())


def _links_from_normals(h: np.ndarray, eps: float) -> np.ndarray:
    H = np.einsum("...a,aij->...ij", h, _GELL_MANN) / 2.0
    return su3_exp(H, eps)


# Lattices with at least this many links are exponentiated by a pool of
# worker processes (each matrix is exponentiated on its own, so the result
# is the same bit for bit as in one process).
PARALLEL_LINKS = 1 << 22


def links(dims, eps: float, seed: int, workers: int | None = None) -> np.ndarray:
    """Gauge links U_mu(x) = exp(i eps H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1).

    The normals are drawn in canonical site order, then direction, with 8 per
    link.  Returns complex128 of shape (T, Z, Y, X, 4, 3, 3).  ``workers``
    (default: up to 16 where the lattice has PARALLEL_LINKS links or more,
    else 1) processes share the exponentials.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal(_shape(dims) + (4, 8))
    nlinks = h.size // 8
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if nlinks >= PARALLEL_LINKS else 1
    if workers <= 1:
        return _links_from_normals(h, eps)
    return _parallel_links(h, eps, workers)


def _links_worker(argv):
    """Child-process entry: exponentiate links lo..hi of the memory-mapped
    normals file into the memory-mapped links file."""
    hpath, upath = argv[0], argv[1]
    n, lo, hi = int(argv[2]), int(argv[3]), int(argv[4])
    eps = float(argv[5])
    h = np.memmap(hpath, dtype=np.float64, mode="r", shape=(n, 8))
    u = np.memmap(upath, dtype=np.complex128, mode="r+", shape=(n, 3, 3))
    step = 1 << 16
    for a in range(lo, hi, step):
        b = min(hi, a + step)
        u[a:b] = _links_from_normals(np.asarray(h[a:b]), eps)
    u.flush()
    del h, u


def _parallel_links(h: np.ndarray, eps: float, workers: int) -> np.ndarray:
    """The exponentials of _links_from_normals shared by `workers` child
    processes (each started as a fresh interpreter running _links_worker on
    one slice) through two memory-mapped files in a private temporary
    directory (in memory where /dev/shm exists), removed afterwards.  A
    failing child raises here."""
    import shutil
    import subprocess
    import sys
    import tempfile
    shape = h.shape[:-1] + (3, 3)
    n = h.size // 8
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, sys.argv[1]); import workloads; "
            "workloads._links_worker(sys.argv[2:])")
    tmp = tempfile.mkdtemp(prefix="ddamg_links_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    procs = []
    try:
        hpath, upath = os.path.join(tmp, "h"), os.path.join(tmp, "u")
        hm = np.memmap(hpath, dtype=np.float64, mode="w+", shape=(n, 8))
        hm[:] = h.reshape(n, 8)
        hm.flush()
        del hm
        um = np.memmap(upath, dtype=np.complex128, mode="w+", shape=(n, 3, 3))
        del um
        cuts = np.linspace(0, n, workers + 1).astype(np.int64)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
        for k in range(workers):
            procs.append(subprocess.Popen(
                [sys.executable, "-c", code, root, hpath, upath, str(n), str(int(cuts[k])),
                 str(int(cuts[k + 1])), repr(float(eps))], env=env))
        rcs = [p.wait(timeout=1800) for p in procs]
        if any(rcs):
            raise RuntimeError(f"link exponentiation workers failed: exit codes {rcs}")
        out = np.array(np.memmap(upath, dtype=np.complex128, mode="r", shape=(n, 3, 3))).reshape(shape)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
        shutil.rmtree(tmp, ignore_errors=True)
    return out


def random_su3(dims, seed: int, eps: float = np.pi) -> np.ndarray:
    """One random SU(3) matrix per site (used for gauge transformations in tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal(_shape(dims) + (8,))
    H = np.einsum("...a,aij->...ij", h, _GELL_MANN) / 2.0
    return su3_exp(H, eps)


def gaussian_field(dims, dof: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian field, Re and Im ~ N(0,1), canonical order.

    Shape (T, Z, Y, X, dof), or (nrhs, T, Z, Y, X, dof) when nrhs is given.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lead = () if nrhs is None else (nrhs,)
    g = rng.standard_normal(lead + _shape(dims) + (dof, 2))
    return g[..., 0] + 1j * g[..., 1]


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    return gaussian_field(dims, 12, seed, nrhs)


def point_sources(dims) -> np.ndarray:
    """The 12 spin-colour point sources b^(s,c)(x) = delta_{x,0} e_s (x) e_c."""
    b = np.zeros((12,) + _shape(dims) + (12,), dtype=np.complex128)
    for k in range(12):
        b[k, 0, 0, 0, 0, k] = 1.0
    return b


def test_vectors(dims, dof: int, n: int, seed: int) -> np.ndarray:
    """The n random initial test vectors of the setup, shape (n, T, Z, Y, X, dof)."""
    return gaussian_field(dims, dof, seed, nrhs=n)


def gaussian_fields_iter(dims, dof: int, n: int, seed: int):
    """The n fields of gaussian_field(dims, dof, seed, nrhs=n) one at a time
    (the same values: the normals are drawn in the same order), so that large
    lattices need one field of host memory instead of n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(n):
        g = rng.standard_normal(_shape(dims) + (dof, 2))
        yield g[..., 0] + 1j * g[..., 1]


# --------------------------------------------------------------------------
# Workloads.  Defaults follow the paper's parameter table (Tab. 1); sizes,
# link spread eps and bare mass m0 define the synthetic stand-ins.
# --------------------------------------------------------------------------

DEFAULT_PARAMS = dict(
    n_inv=6,            # setup iterations (Tab. 1)
    coarse_eps=5e-2,    # coarsest-system relative residual (Tab. 1)
    nkv=10,             # outer FGMRES restart length (Tab. 1)
    tol=1e-10,          # outer relative residual (Tab. 1)
    mu=0, nu=5,         # pre/post smoothing (Tab. 1)
    sap_block=(2, 2, 2, 2),
    mr_iters=3,
    kc_len=5, kc_restarts=2, kc_tol=1e-1,   # K-cycle (Tab. 1)
    coarse_restart=30, coarse_max_restarts=10,
)


def _cfg(k, **kw):
    p = dict(DEFAULT_PARAMS)
    p.update(kw)
    p["seed_links"] = BASE_SEED + 100 * k
    p["seed_rhs"] = BASE_SEED + 100 * k + 1
    p["seed_tv"] = BASE_SEED + 100 * k + 2
    p["seed_gauge"] = BASE_SEED + 100 * k + 3
    return p


CONFIGS = {
    # two-level, 8^4, Wilson only
    "wilson8_2lvl": _cfg(0, dims=(8, 8, 8, 8), eps=0.4, m0=-0.3, csw=0.0,
                         levels=2, agg=[(4, 4, 4, 4)], ntv=[8], nu=2),
    # three-level, 16^3x32, clover
    "clover16x32_3lvl": _cfg(1, dims=(16, 16, 16, 32), eps=0.5, m0=-0.4, csw=1.0,
                             levels=3, agg=[(4, 4, 4, 4), (2, 2, 2, 2)], ntv=[20, 20]),
    # three-level, 32^3x64, 12 point sources
    "clover32x64_3lvl_12rhs": _cfg(2, dims=(32, 32, 32, 64), eps=0.5, m0=-0.42, csw=1.0,
                                   levels=3, agg=[(4, 4, 4, 4), (2, 2, 2, 2)], ntv=[20, 20]),
    # four-level, 48^3x96
    # (level 2 is 6^3x12: 2^4 SAP blocks would come in odd counts, 3^4 blocks
    # give 2^3x4 of them)
    "clover48x96_4lvl": _cfg(4, dims=(48, 48, 48, 96), eps=0.55, m0=-0.43, csw=1.0,
                             levels=4, agg=[(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)],
                             ntv=[20, 20, 28],
                             sap_blocks=[(2, 2, 2, 2), (2, 2, 2, 2), (3, 3, 3, 3)]),
}

# the uneven batch of eight lattices: (dims, eps, m0).  Every pair lies on
# the massive side of the critical mass estimated for its eps (on 4^4 with
# this link normalisation: about -0.40 at eps 0.45, -0.49 at 0.50, -0.59 at
# 0.55, -0.69 at 0.60), by 0.09 to 0.29; with eps <= 0.40 every m0 in
# [-0.45, -0.30] is at or below it (indefinite systems that the method, in
# plain FP64 too, does not solve in 1000 outer iterations).
UNEVEN_BATCH = [
    ((16, 16, 16, 16), 0.45, -0.30), ((16, 16, 16, 16), 0.50, -0.35),
    ((16, 16, 16, 16), 0.55, -0.45), ((16, 16, 16, 16), 0.60, -0.45),
    ((24, 24, 24, 48), 0.50, -0.40), ((24, 24, 24, 48), 0.55, -0.35),
    ((32, 32, 32, 64), 0.45, -0.30), ((32, 32, 32, 64), 0.60, -0.40),
]


def uneven_batch_seed(j: int) -> int:
    return BASE_SEED + 400 + 10 * j


def uneven_batch_config(j: int) -> dict:
    """Parameters of lattice j of the uneven batch: three levels (aggregates
    4^4 then 2^4), N = 20/20, c_sw = 1, V-cycle.  A 24^3x48 lattice has a
    6^3x12 second level, where 2^4 SAP blocks would come in odd counts: its
    SAP blocks there are 3^4 (2^3x4 of them), and its coarsest lattice 3^3x6
    has odd extents (no odd-even split)."""
    dims, eps, m0 = UNEVEN_BATCH[j]
    level2 = [x // 4 for x in dims]
    blocks = (2, 2, 2, 2) if all((e // 2) % 2 == 0 for e in level2) else (3, 3, 3, 3)
    p = dict(DEFAULT_PARAMS)
    p.update(dims=dims, eps=eps, m0=m0, csw=1.0, levels=3, agg=[(4, 4, 4, 4), (2, 2, 2, 2)], ntv=[20, 20],
             sap_blocks=[(2, 2, 2, 2), blocks, (2, 2, 2, 2)], cycle="V")
    seed = uneven_batch_seed(j)
    p.update(seed_links=seed, seed_rhs=seed + 1, seed_tv=seed + 2, seed_gauge=seed + 3)
    return p
