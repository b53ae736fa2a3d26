"""Helpers shared by the GPU parity tests (inputs from synth, expected values
from the oracle, results from the library through its C ABI)."""
import numpy as np
import torch

import synth
from oracle import space as S, operator as O


def case(cfg, n, k=None, noise=None, nq=None, seed=0):
    """Oracle space and coefficient vector for workload `cfg` on a small mesh."""
    mesh, field, c = synth.make_config(cfg, n_override=n)
    k = k or c["k"]
    sp = S.Space(mesh.elem_vid, mesh.elem_xyz, k)
    x = sp.interpolate(field, nq1d=nq or (k + 4))
    sig = c["noise"] if noise is None else noise
    if sig:
        x = x + sig * np.random.default_rng(6698 + cfg + seed).standard_normal(sp.n_dof)
    return mesh, sp, x, c


def gpu_space(mesh, k):
    from paper_2408_06698_amd.hopu import Hopu
    return Hopu(mesh.dim, k, mesh.elem_vid, mesh.elem_xyz)


def dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_dual(sp, r, ref):
    """||r - ref||_{M^-1} / ||ref||_{M^-1} (residuals are dual vectors)."""
    e = r - ref
    den = ref @ O.mass_solve(sp, ref)
    return float(np.sqrt(max(e @ O.mass_solve(sp, e), 0.0) / den)) if den > 0 else float(np.abs(e).max())


def rel_primal(sp, x, ref):
    e = x - ref
    return float(np.sqrt(max(e @ O.mass_apply(sp, e), 0.0) / (ref @ O.mass_apply(sp, ref))))
