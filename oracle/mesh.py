"""Topology and geometry of an affine simplex mesh (oracle; test
infrastructure only).

Facet sets (section 2.1): F^I holds facets with two neighbouring elements
(interior and periodic facets); F^W holds facets with one element (walls,
homogeneous Dirichlet, where the normal velocity is zero in the space).

Conventions (the paper does not fix them):
  * sorted-vertex convention: local vertex i of T is its i-th smallest
    (periodic-identified) global vertex id; the affine map is
    F_T(x^) = x_0 + J x^ with columns x_i - x_0; det J is signed;
  * local facet i is opposite local vertex i; it is parametrised from its
    own vertices in ascending id order, so both neighbours of a facet use
    the same parametrisation and no permutation tables are needed;
  * facet normal N_F = (x_b - x_a) x (x_c - x_a) (3D) or R(x_b - x_a) with
    R(t) = (t2, -t1) (2D), unit normal n_F = N_F / |N_F|;
  * global facet numbering: interior facets in lexicographic order of their
    sorted vertex-id tuple; wall facets are listed separately.
"""
from dataclasses import dataclass
import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class Topo:
    dim: int
    n_elems: int
    vid: np.ndarray        # [E][d+1] sorted vertex ids
    xyz: np.ndarray        # [E][d+1][d] coordinates in sorted order
    J: np.ndarray          # [E][d][d]
    detJ: np.ndarray       # [E]
    elem_facet: np.ndarray  # [E][d+1] interior facet index or -1 (wall)
    nbr: np.ndarray        # [E][d+1] neighbour element or -1
    nbr_face: np.ndarray   # [E][d+1] neighbour's local facet index or -1
    facet_elems: np.ndarray   # [F][2] (lower element id first)
    facet_local: np.ndarray   # [F][2] local facet index in each element
    facet_vids: np.ndarray    # [F][d] sorted vertex ids
    wall_elems: np.ndarray    # [W] element of each wall facet
    wall_local: np.ndarray    # [W] local facet index
    NF: np.ndarray            # [E][d+1][d] facet normal computed from T
    NF_norm: np.ndarray       # [E][d+1]
    sigma: np.ndarray         # [E][d+1] outward sign of N_F for T

    @property
    def n_facets(self):
        return self.facet_elems.shape[0]


def facet_vectors(xyz_f, dim):
    """Normal N = (x_b - x_a) x (x_c - x_a) or R(x_b - x_a)."""
    if dim == 2:
        t = xyz_f[..., 1, :] - xyz_f[..., 0, :]
        return np.stack([t[..., 1], -t[..., 0]], -1)
    return np.cross(xyz_f[..., 1, :] - xyz_f[..., 0, :],
                    xyz_f[..., 2, :] - xyz_f[..., 0, :])


def build(elem_vid, elem_xyz):
    elem_vid = np.asarray(elem_vid, dtype=np.int64)
    elem_xyz = np.asarray(elem_xyz, dtype=np.float64)
    E, dp1 = elem_vid.shape
    dim = dp1 - 1
    order = np.argsort(elem_vid, axis=1, kind="stable")
    vid = np.take_along_axis(elem_vid, order, 1)
    if np.any(vid[:, 1:] == vid[:, :-1]):
        raise MeshError("element with a repeated vertex")
    xyz = np.take_along_axis(elem_xyz, order[:, :, None], 1)
    J = np.stack([xyz[:, i + 1] - xyz[:, 0] for i in range(dim)], -1)
    detJ = np.linalg.det(J)
    if np.any(detJ == 0.0):
        raise MeshError("degenerate element")

    # facets: tuple of sorted vertex ids without local vertex i
    keys = np.stack([np.delete(vid, i, axis=1) for i in range(dp1)], 1)  # [E][d+1][d]
    flat = keys.reshape(-1, dim)
    uniq, inv, counts = np.unique(flat, axis=0, return_inverse=True,
                                  return_counts=True)
    inv = inv.reshape(E, dp1)
    if np.any(counts > 2):
        raise MeshError("facet shared by more than two elements")
    interior = counts == 2
    # interior facets keep lexicographic order (np.unique sorts rows)
    new_index = -np.ones(len(uniq), dtype=np.int64)
    new_index[interior] = np.arange(interior.sum())
    elem_facet = new_index[inv]
    F = int(interior.sum())
    facet_elems = -np.ones((F, 2), dtype=np.int64)
    facet_local = -np.ones((F, 2), dtype=np.int64)
    nbr = -np.ones((E, dp1), dtype=np.int64)
    nbr_face = -np.ones((E, dp1), dtype=np.int64)
    wall_e, wall_l = [], []
    for e in range(E):  # elements in ascending order: lower id fills slot 0
        for i in range(dp1):
            f = elem_facet[e, i]
            if f < 0:
                wall_e.append(e)
                wall_l.append(i)
                continue
            slot = 0 if facet_elems[f, 0] < 0 else 1
            facet_elems[f, slot] = e
            facet_local[f, slot] = i
    for f in range(F):
        (e0, e1), (i0, i1) = facet_elems[f], facet_local[f]
        if e0 == e1:
            raise MeshError("element is its own neighbour (too few periodic cells)")
        nbr[e0, i0], nbr_face[e0, i0] = e1, i1
        nbr[e1, i1], nbr_face[e1, i1] = e0, i0

    NF = np.empty((E, dp1, dim))
    for i in range(dp1):
        lv = [v for v in range(dp1) if v != i]
        NF[:, i] = facet_vectors(xyz[:, lv], dim)
    NFn = np.linalg.norm(NF, axis=-1)
    sigma = np.array([(-1.0) ** i for i in range(dp1)])[None, :] * np.sign(detJ)[:, None]
    # geometric check of the outward sign: N_F . (facet point - opposite vertex)
    for i in range(dp1):
        lv = [v for v in range(dp1) if v != i]
        c = xyz[:, lv].mean(1) - xyz[:, i]
        geo = np.sign(np.einsum("ed,ed->e", NF[:, i], c))
        if not np.array_equal(geo, sigma[:, i]):
            raise MeshError("outward sign mismatch")
    uniq_vids = uniq[interior]
    return Topo(dim, E, vid, xyz, J, detJ, elem_facet, nbr, nbr_face,
                facet_elems, facet_local, uniq_vids,
                np.array(wall_e, dtype=np.int64), np.array(wall_l, dtype=np.int64),
                NF, NFn, sigma)
