"""Sizes of the five synthetic workloads at full size, from the host library's
mesh builder and space sizes, against closed forms: Kuhn meshes split every
cell into d! simplices and every wall cell face into (d-1)! facets; each
interior facet has two sides; the velocity space is BDM_k = (P^k)^d per
element (section 2.2, read as BDM_k on simplices) with P^k facet moments."""
import ctypes as C
from math import comb, factorial, prod

import numpy as np
import pytest

import synth
from synth.configs import CONFIGS
from paper_2408_06698_amd import _lib as L


def _host_mesh(m, which, dtype, count):
    out = np.zeros(count, dtype=dtype)
    n = L.lib().hopu_host_mesh(m.dim, m.n_elems, m.elem_vid.ctypes.data_as(C.c_void_p),
                               m.elem_xyz.ctypes.data_as(C.c_void_p), which,
                               out.ctypes.data_as(C.c_void_p), out.size)
    assert n >= 0
    return out[:n]


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5])
def test_full_size_counts(c):
    cfg = CONFIGS[c]
    d, k, n = cfg["dim"], cfg["k"], cfg["n"]
    E = factorial(d) * prod(n)
    W = sum(2 * factorial(d - 1) * prod(n) // n[j] for j in range(d) if not cfg["periodic"][j])
    F = ((d + 1) * E - W) // 2
    nf = comb(k + d - 1, d - 1)
    nloc = d * comb(k + d, d)
    nint = nloc - (d + 1) * nf

    assert L.lib().hopu_host_sizes(d, k, 0) == nloc
    assert L.lib().hopu_host_sizes(d, k, 1) == nf
    assert L.lib().hopu_host_sizes(d, k, 2) == nint

    m, _, _ = synth.make_config(c)
    m.elem_vid = np.ascontiguousarray(m.elem_vid)
    m.elem_xyz = np.ascontiguousarray(m.elem_xyz)
    assert m.n_elems == E
    nbr = _host_mesh(m, 1, np.int32, (d + 1) * E)
    fe = _host_mesh(m, 4, np.int32, (d + 1) * E)
    assert int((nbr < 0).sum()) == W
    assert fe.size == 2 * F
    n_dof = F * nf + E * nint
    print(f"workload {c}: E {E}, F {F}, walls {W}, n_loc {nloc}, DoFs {n_dof}")
    if c == 5:
        # BDM_5 on a tetrahedron: 168 local DoFs (RT_5 would have 189)
        assert nloc == 168 and n_dof == 222_759_936
    if c == 2:
        assert n_dof == 7_864_320
