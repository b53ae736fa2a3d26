"""Structured simplex meshes (Kuhn subdivision) with periodic identification,
geometric grading and seeded vertex jitter, plus tiny hand-made meshes.

Output convention (what both the oracle and the library consume):
  elem_vid : int64 [E][d+1]  global vertex ids, periodic images identified
  elem_xyz : float64 [E][d+1][d]  *unwrapped* coordinates of each element's
             vertices (an element never straddles a period; its coordinates
             are those of one connected copy)
Vertex order inside an element is the generator's order; consumers sort by id.
"""
from dataclasses import dataclass, field
import itertools
import numpy as np


@dataclass
class Mesh:
    dim: int
    elem_vid: np.ndarray
    elem_xyz: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def n_elems(self):
        return self.elem_vid.shape[0]


def graded_nodes(n, ratio, h0):
    """y_j = h0 (ratio^j - 1)/(ratio - 1), j = 0..n (one-sided grading)."""
    j = np.arange(n + 1, dtype=np.float64)
    return h0 * (ratio ** j - 1.0) / (ratio - 1.0)


def symmetric_graded_nodes(n, ratio, length=1.0):
    """Nodes on [0, length] graded geometrically toward both ends (n even)."""
    assert n % 2 == 0
    half = n // 2
    steps = ratio ** np.arange(half, dtype=np.float64)
    steps = np.concatenate([steps, steps[::-1]])
    steps *= length / steps.sum()
    return np.concatenate([[0.0], np.cumsum(steps)])


def _axis_nodes(n, length, nodes):
    if nodes is None:
        return np.linspace(0.0, length, n + 1)
    nodes = np.asarray(nodes, dtype=np.float64)
    assert nodes.shape == (n + 1,)
    return nodes


def kuhn_mesh(dim, n, lengths=None, periodic=None, nodes=None, jitter=0.0,
              jitter_seed=None):
    """Kuhn triangulation of a box.

    dim      : 2 or 3
    n        : cells per direction (tuple of length dim)
    lengths  : box lengths (defaults to 1)
    periodic : per-direction flags
    nodes    : per-direction optional node coordinate arrays (length n_i + 1)
    jitter   : relative amplitude: each coordinate of each movable node is
               displaced by U(-jitter, jitter) times the smaller adjacent
               spacing in that direction.  Nodes on a non-periodic boundary
               keep that coordinate; periodic images move together.

    Cubes are numbered ix + nx (iy + ny iz); each cube gives d! simplices in
    lexicographic order of the axis permutation pi, with vertices
    v0, v0 + e_pi1, v0 + e_pi1 + e_pi2, ..., v0 + (1,..,1).
    """
    n = tuple(int(v) for v in n)
    assert len(n) == dim
    lengths = tuple(float(v) for v in (lengths or (1.0,) * dim))
    periodic = tuple(bool(v) for v in (periodic or (True,) * dim))
    nodes = nodes or (None,) * dim
    for a in range(dim):
        if periodic[a] and n[a] < 3:
            raise ValueError("a periodic direction needs at least 3 cells")
    ax = [_axis_nodes(n[a], lengths[a], nodes[a]) for a in range(dim)]
    nid = [n[a] if periodic[a] else n[a] + 1 for a in range(dim)]

    # displacement per identified node
    disp = np.zeros(tuple(nid) + (dim,))
    if jitter > 0.0:
        rng = np.random.default_rng(jitter_seed)
        u = rng.uniform(-jitter, jitter, size=disp.shape)
        for a in range(dim):
            h = np.diff(ax[a])
            if periodic[a]:
                left = np.concatenate([[h[-1]], h[:-1]])  # spacing before node j
                right = h
                small = np.minimum(left, right)  # length n
            else:
                small = np.empty(n[a] + 1)
                small[0] = h[0]
                small[-1] = h[-1]
                small[1:-1] = np.minimum(h[:-1], h[1:])
            shape = [1] * dim
            shape[a] = nid[a]
            d = u[..., a] * small.reshape(shape)
            if not periodic[a]:
                sl = [slice(None)] * dim
                sl[a] = 0
                d[tuple(sl)] = 0.0
                sl[a] = -1
                d[tuple(sl)] = 0.0
            disp[..., a] = d

    perms = list(itertools.permutations(range(dim)))
    cells = np.stack(np.meshgrid(*[np.arange(n[a]) for a in range(dim)],
                                 indexing="ij"), axis=-1)
    # order cubes as ix + nx (iy + ny iz): x fastest
    cells = cells.transpose(tuple(range(dim))[::-1] + (dim,)).reshape(-1, dim)
    n_cells = cells.shape[0]
    E = n_cells * len(perms)
    vid = np.empty((n_cells, len(perms), dim + 1), dtype=np.int64)
    xyz = np.empty((n_cells, len(perms), dim + 1, dim), dtype=np.float64)
    for p, perm in enumerate(perms):
        offs = [np.zeros(dim, dtype=np.int64)]
        for a in perm:
            o = offs[-1].copy()
            o[a] += 1
            offs.append(o)
        for v, o in enumerate(offs):
            g = cells + o  # unwrapped grid index
            ident = np.empty_like(g)
            for a in range(dim):
                ident[:, a] = g[:, a] % n[a] if periodic[a] else g[:, a]
            flat = np.zeros(n_cells, dtype=np.int64)
            mul = 1
            for a in range(dim):
                flat += ident[:, a] * mul
                mul *= nid[a]
            vid[:, p, v] = flat
            for a in range(dim):
                if periodic[a]:
                    wraps = g[:, a] // n[a]
                    coord = ax[a][g[:, a] % n[a]] + wraps * lengths[a]
                else:
                    coord = ax[a][g[:, a]]
                xyz[:, p, v, a] = coord + disp[tuple(ident.T)][:, a]
    info = dict(n=n, lengths=lengths, periodic=periodic, nodes=ax)
    return Mesh(dim, vid.reshape(E, dim + 1), xyz.reshape(E, dim + 1, dim), info)


def two_element_mesh(dim):
    """Two simplices sharing one facet; every other facet is a wall."""
    if dim == 2:
        pts = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
        tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    else:
        pts = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.0, 0.1],
                        [0.1, 0.2, 1.0], [0.9, 0.8, 0.7]])
        tris = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int64)
    return Mesh(dim, tris, pts[tris], dict(n=None, periodic=(False,) * dim))
