"""Helpers shared by the GPU parity tests: moving numpy fields to and from
the device, translating a parameter dict into the C struct, and rebuilding
an oracle hierarchy from the GPU's exported interpolation bases."""
import sys

import numpy as np
import torch

from oracle import multigrid as mg
from oracle.lattice import shape


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty(shape_, dtype=torch.complex128):
    return torch.zeros(shape_, dtype=dtype, device="cuda")


def fields_on_device(dims, dof, n, seed):
    """gaussian_field(dims, dof, seed, nrhs=n) built on the device one field
    at a time (one field of host memory for the largest lattices)."""
    import workloads as W
    out = torch.empty((n,) + shape(dims) + (dof,), dtype=torch.complex128, device="cuda")
    for k, f in enumerate(W.gaussian_fields_iter(dims, dof, n, seed)):
        out[k].copy_(torch.from_numpy(f))
    return out


def sampled_residual(U, m0, csw, b_at, z, sites):
    """(sqrt(V) * rms over the sampled sites of |b - D z|, an estimate of
    ||b - D z||; the largest |b - D z| of a sampled site, a lower bound of
    it), with D the oracle's site-by-site operator; b_at(site) gives b at a
    site (x, y, z, t), z is the host solution field."""
    from oracle.dirac import apply_at_sites
    dz = apply_at_sites(U, m0, csw, z, sites)
    r = np.array([b_at(s) for s in sites]) - dz
    V = int(np.prod(U.shape[:4]))
    return (float(np.sqrt(np.mean(np.sum(np.abs(r) ** 2, axis=1)) * V)),
            float(np.max(np.linalg.norm(r, axis=1))))


def sample_sites(dims, n, seed, extra=()):
    rng = np.random.Generator(np.random.PCG64(seed))
    return list(extra) + [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(n)]


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_params(dd, p, prec=None, cycle="K", half=False, half_dirs=False):
    P = dd.params_default(int(p["levels"]))
    for l, a in enumerate(p["agg"]):
        for mu in range(4):
            P.agg[l][mu] = a[mu]
    for l, n in enumerate(p["ntv"]):
        P.ntv[l] = n
    for mu in range(4):
        P.sap_block[mu] = p.get("sap_block", (2, 2, 2, 2))[mu]
    for l, blk in enumerate(p.get("sap_blocks", [])[1:]):
        for mu in range(4):
            P.sap_block_l[l][mu] = blk[mu]
    P.mu, P.nu = p["mu"], p["nu"]
    P.mr_iters = p["mr_iters"]
    P.n_inv = p["n_inv"]
    P.coarse_eps = p["coarse_eps"]
    P.coarse_restart = p.get("coarse_restart", 30)
    P.coarse_max_restarts = p.get("coarse_max_restarts", 10)
    P.kc_len, P.kc_restarts, P.kc_tol = p["kc_len"], p["kc_restarts"], p["kc_tol"]
    P.nkv, P.tol = p["nkv"], p["tol"]
    P.max_restarts = p.get("max_restarts", 100)
    P.precond_prec = dd.F64 if prec is None else prec
    P.cycle = {"K": dd.KCYCLE, "V": dd.VCYCLE, "W": dd.WCYCLE}[cycle]
    P.half_storage = 1 if half else 0
    P.half_directions = 1 if half_dirs else 0
    return P


def export_P(dd, H, level, N):
    dims, d = dd.level_info(H, level)
    V = int(np.prod(dims))
    out = empty((N, V, d))
    dd.export_interpolation(H, level, out)
    return host(out).reshape((N,) + shape(dims) + (d,))


def export_Dc(dd, H, level):
    dims, d = dd.level_info(H, level)
    V = int(np.prod(dims))
    out = empty((V, 9, d, d))
    dd.export_coarse_op(H, level, out)
    return host(out).reshape(shape(dims) + (9, d, d))


def oracle_from_gpu(dd, H, op, p, cycle="K"):
    """Oracle hierarchy on the GPU's interpolation bases (exported P columns
    used as test vectors: re-orthonormalising an orthonormal set returns it)."""
    OH = mg.Hierarchy(op, p, cycle)
    for l in range(OH.L - 1):
        OH.tv[l] = export_P(dd, H, l, p["ntv"][l])
        OH.build_level(l)
    return OH
