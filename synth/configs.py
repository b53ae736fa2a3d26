"""The five synthetic workloads (meshes, fields, step counts and seeds).

Seeds: numpy default_rng(6698 + c) for the field and coefficient noise of
workload c, 66980 + c for vertex jitter, 669800 + c for finite-difference
directions.  Everything here is input description only.
"""
import numpy as np
from .mesh import kuhn_mesh, graded_nodes, symmetric_graded_nodes
from . import fields

TWO_PI = 2.0 * np.pi

CONFIGS = {
    1: dict(name="2d_periodic_tg_k2", dim=2, k=2, n=(16, 16), lengths=(1.0, 1.0),
            periodic=(True, True), field="tg2d", noise=1e-3, dt=1e-3, steps=10,
            l=1),
    2: dict(name="3d_periodic_tg_k3", dim=3, k=3, n=(32, 32, 32),
            lengths=(TWO_PI,) * 3, periodic=(True, True, True), field="tg3d",
            noise=1e-3, dt=5e-4, steps=50, l=2),
    3: dict(name="3d_graded_wall_k4", dim=3, k=4, n=(48, 48, 48),
            lengths=(1.0, None, 1.0), periodic=(True, False, True),
            field="curl_wall", noise=0.0, dt=1e-4, steps=10, l=3,
            grading=("one_sided", 1.1, 1.0415e-3), jitter=0.05),
    4: dict(name="3d_periodic_curl_k3_adjoint", dim=3, k=3, n=(24, 24, 24),
            lengths=(TWO_PI,) * 3, periodic=(True, True, True),
            field="curl_periodic", noise=0.0, dt=1e-3, steps=20, l=2,
            ckpt_every=5, fd_dirs=32, fd_h=1e-6),
    5: dict(name="3d_channel_spectral_k5", dim=3, k=5, n=(96, 64, 48),
            lengths=(4.0, 1.0, 2.0), periodic=(True, False, True),
            field="spectral_wall", noise=0.0, dt=1e-4, steps=100, l=4,
            grading=("symmetric", 1.151811)),
}


def _y_nodes(cfg):
    g = cfg.get("grading")
    ny = cfg["n"][1]
    if g is None:
        return None
    if g[0] == "one_sided":
        y = graded_nodes(ny, g[1], g[2])
        return y / y[-1]  # normalise exactly onto [0, 1]
    return symmetric_graded_nodes(ny, g[1], 1.0)


def make_config(c, n_override=None, with_jitter=True):
    """Return (mesh, field_fn, cfg) for workload c.  n_override shrinks the
    mesh (same recipe) for fast tests."""
    cfg = dict(CONFIGS[c])
    if n_override is not None:
        cfg["n"] = tuple(n_override)
    lengths = tuple(1.0 if L is None else L for L in cfg["lengths"])
    nodes = [None] * cfg["dim"]
    if cfg.get("grading") is not None:
        if n_override is not None and cfg["grading"][0] == "one_sided":
            # keep the ratio; rescale so the box stays [0,1]
            y = graded_nodes(cfg["n"][1], cfg["grading"][1], 1.0)
            nodes[1] = y / y[-1]
        elif n_override is not None:
            nodes[1] = symmetric_graded_nodes(cfg["n"][1] + (cfg["n"][1] % 2),
                                              cfg["grading"][1], 1.0)
            if cfg["n"][1] % 2:
                nodes[1] = np.linspace(0, 1, cfg["n"][1] + 1)
        else:
            nodes[1] = _y_nodes(cfg)
    jit = cfg.get("jitter", 0.0) if with_jitter else 0.0
    mesh = kuhn_mesh(cfg["dim"], cfg["n"], lengths, cfg["periodic"], nodes,
                     jitter=jit, jitter_seed=66980 + c)
    seed = 6698 + c
    fname = cfg["field"]
    if fname == "tg2d":
        f = fields.taylor_green_2d()
    elif fname == "tg3d":
        f = fields.taylor_green_3d()
    elif fname == "curl_periodic":
        f = fields.curl_fourier_periodic(seed)
    elif fname == "curl_wall":
        f = fields.curl_fourier_wall(seed)
    elif fname == "spectral_wall":
        f = fields.spectral_wall_field(seed, lengths=lengths)
    else:
        raise KeyError(fname)
    cfg["lengths"] = lengths
    cfg["seed"] = seed
    return mesh, f, cfg


def coefficient_noise(c, n_dof, sigma):
    """Seeded N(0, sigma^2) noise for the free coefficients of workload c."""
    rng = np.random.default_rng(6698 + c + 1000)
    return sigma * rng.standard_normal(n_dof)


def fd_directions(c, n_dirs, n_dof):
    rng = np.random.default_rng(669800 + c)
    return rng.standard_normal((n_dirs, n_dof))
