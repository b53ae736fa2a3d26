"""CPU tests of the library's host side through its C ABI: symbols, host
tables and mesh topology/geometry against the oracle (no GPU needed)."""
import ctypes as C
import re
import os
import numpy as np
import pytest

import synth
from synth.mesh import two_element_mesh
from oracle import basis as B, quadrature as Q, mesh as OM, space as S

from paper_2408_06698_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "hopu.h")).read()
    names = set(re.findall(r"\b(hopu_[a-z0-9_]+)\s*\(", hdr))
    assert "hopu_create" in names and len(names) >= 18
    lib = C.CDLL(L.LIB_PATH)
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(L.SIGNATURES) == names


def _table(dim, k, which):
    n = L.lib().hopu_host_tables(dim, k, which, None, 0)
    buf = np.zeros(max(int(n), 1))
    # the call copies min(cap, size) values
    n = L.lib().hopu_host_tables(dim, k, which, buf.ctypes.data_as(C.c_void_p), buf.size)
    return buf[:n]


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 4), (3, 1), (3, 3), (3, 5)])
def test_host_quadrature_matches_oracle(dim, k):
    nqv = L.lib().hopu_host_sizes(dim, k, 4)
    nqf = L.lib().hopu_host_sizes(dim, k, 5)
    xv = _table(dim, k, 0).reshape(nqv, dim)
    wv = _table(dim, k, 1)
    xo, wo = Q.simplex_rule(dim, Q.volume_points_per_dir(k))
    # same rule: compare as sets (sorted rows)
    oi = np.lexsort(xo.T[::-1]); hi = np.lexsort(xv.T[::-1])
    assert np.abs(xv[hi] - xo[oi]).max() < 1e-14
    assert np.abs(wv[hi] - wo[oi]).max() < 1e-15
    sf = _table(dim, k, 3).reshape(nqf, dim - 1)
    so, wso = Q.simplex_rule(dim - 1, Q.facet_points_per_dir(k))
    oi = np.lexsort(so.T[::-1]); hi = np.lexsort(sf.T[::-1])
    assert np.abs(sf[hi] - so[oi]).max() < 1e-14
    assert np.abs(_table(dim, k, 4)[hi] - wso[oi]).max() < 1e-15
    # facet polynomials at the host's facet points
    psi_h = _table(dim, k, 5).reshape(nqf, -1)
    assert np.abs(psi_h - B.psi(dim, k, sf)).max() < 1e-13


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (3, 3), (3, 4), (3, 5)])
def test_host_dual_basis_matches_oracle(dim, k):
    """The dual basis is independent of the internal modal basis: compare
    phi^_i at the host's volume points."""
    nqv = L.lib().hopu_host_sizes(dim, k, 4)
    n = L.lib().hopu_host_sizes(dim, k, 0)
    nP = L.lib().hopu_host_sizes(dim, k, 3)
    xv = _table(dim, k, 0).reshape(nqv, dim)
    V = _table(dim, k, 2).reshape(nqv, nP)
    Dinv = _table(dim, k, 7).reshape(n, n)
    phi_h = np.stack([V @ Dinv[a * nP:(a + 1) * nP, :] for a in range(dim)], -1)  # [q][n][d]
    phi_o, _ = B.dual_basis(dim, k, xv)
    scale = np.abs(phi_o).max(axis=(0, 2))  # per basis function
    err = np.abs(phi_h - phi_o).max(axis=(0, 2)) / scale
    assert err.max() < 1e-11, err.max()


def _host_mesh(m, which, dtype, count):
    out = np.zeros(count, dtype=dtype)
    n = L.lib().hopu_host_mesh(m.dim, m.n_elems, m.elem_vid.ctypes.data_as(C.c_void_p),
                               m.elem_xyz.ctypes.data_as(C.c_void_p), which,
                               out.ctypes.data_as(C.c_void_p), out.size)
    assert n >= 0
    return out[:n]


@pytest.mark.parametrize("cfg,n", [(1, (5, 4)), (3, (3, 4, 3)), (4, (3, 3, 3))])
def test_host_mesh_matches_oracle(cfg, n):
    m, f, c = synth.make_config(cfg, n_override=n)
    m.elem_vid = np.ascontiguousarray(m.elem_vid)
    m.elem_xyz = np.ascontiguousarray(m.elem_xyz)
    t = OM.build(m.elem_vid, m.elem_xyz)
    E, dp1, d = t.n_elems, t.dim + 1, t.dim
    fid = _host_mesh(m, 0, np.int32, E * dp1).reshape(E, dp1)
    nbr = _host_mesh(m, 1, np.int32, E * dp1).reshape(E, dp1)
    nbf = _host_mesh(m, 2, np.int32, E * dp1).reshape(E, dp1)
    geo = _host_mesh(m, 3, np.float64, E * 32).reshape(E, 32)
    fe = _host_mesh(m, 4, np.int32, 2 * t.n_facets).reshape(-1, 2)
    assert np.array_equal(fid, t.elem_facet)
    assert np.array_equal(nbr, t.nbr)
    assert np.array_equal(nbf, t.nbr_face)
    assert np.array_equal(fe, t.facet_elems)
    assert np.allclose(geo[:, :d * d].reshape(E, d, d), t.J, rtol=0, atol=1e-15)
    assert np.allclose(geo[:, 9], t.detJ, rtol=1e-14, atol=0)
    assert np.allclose(geo[:, 10:10 + dp1], t.NF_norm, rtol=1e-14, atol=0)
    nrm = geo[:, 14:14 + dp1 * d].reshape(E, dp1, d)
    ref = t.sigma[:, :, None] * t.NF / t.NF_norm[:, :, None]
    assert np.abs(nrm - ref).max() < 1e-14
    # batches: every element exactly once, one signature per batch
    bel = _host_mesh(m, 5, np.int32, E * 16 + 16 * 64).reshape(-1, 16)
    got = np.sort(bel[bel >= 0])
    assert np.array_equal(got, np.arange(E))
    for row in bel:
        els = row[row >= 0]
        sig = {tuple(np.where(t.nbr[e] < 0, 15, t.nbr_face[e])) for e in els}
        assert len(sig) == 1


def test_host_mesh_errors():
    m = two_element_mesh(2)
    bad = np.ascontiguousarray(np.array([[0, 0, 1], [0, 2, 3]], dtype=np.int64))
    n = L.lib().hopu_host_mesh(2, 2, bad.ctypes.data_as(C.c_void_p),
                               np.ascontiguousarray(m.elem_xyz).ctypes.data_as(C.c_void_p), 0, None, 0)
    assert n == -2
    # three elements on one facet
    vid = np.ascontiguousarray(np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]], dtype=np.int64))
    xyz = np.ascontiguousarray(np.random.default_rng(0).standard_normal((3, 3, 2)))
    assert L.lib().hopu_host_mesh(2, 3, vid.ctypes.data_as(C.c_void_p), xyz.ctypes.data_as(C.c_void_p), 0,
                                  None, 0) == -2


def _bf16_terms_to_f32(bits):
    """Raw bfloat16 bit patterns -> float32 values."""
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 3), (3, 5)])
def test_host_bf16_split_tables(dim, k):
    """The split-BF16 copies of the FP32-layout fragment tables (of the
    convection kernel and of the transpose-Jacobian kernel): four steps of
    a lane per fragment, terms that are successive 8-bit truncations of the
    FP32 value (hi + mid + lo equal to it, hi + lo within 2^-15), zero past
    the last step."""
    nP = L.lib().hopu_host_sizes(dim, k, 3)
    nqv = L.lib().hopu_host_sizes(dim, k, 4)
    nqf = L.lib().hopu_host_sizes(dim, k, 5)
    NQVT, NAT, NQFT = -(-nqv // 16), -(-nP // 16), -(-nqf // 16)
    NPK = -(-nP // 4)
    cases = [(8, 10, 3, NQVT, 4, dim * NAT), (8, 9, 2, NQVT, 4, dim * NAT), (11, 12, 3, (dim + 1) * NQFT, NPK, 1),
             # the transpose-Jacobian kernel's volume tables
             (13, 15, 3, NQVT * dim, NPK, 1), (14, 16, 3, NQVT, 4, NAT)]
    for w32, wbf, ns, outer, steps, inner in cases:
        t32 = _table(dim, k, w32).astype(np.float32).reshape(outer, steps, inner, 64)
        ng = -(-steps // 4)
        bits = _table(dim, k, wbf)
        assert np.all(bits == np.round(bits)) and bits.min() >= 0 and bits.max() < 65536
        b = bits.astype(np.uint32).reshape(outer, ng, inner, 64, ns, 4)
        terms = _bf16_terms_to_f32(b)                      # [outer][ng][inner][64][ns][4]
        for sg in range(ng):
            for j in range(4):
                st = 4 * sg + j
                got = terms[:, sg, :, :, :, j]             # [outer][inner][64][ns]
                if st >= steps:
                    assert np.all(got == 0)
                    continue
                f = t32[:, st, :, :]
                # each term: the FP32 remainder truncated to its leading 8 bits
                r = f.copy()
                for tt in range(ns):
                    h = (r.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
                    assert np.array_equal(got[..., tt], h)
                    r = (r - h).astype(np.float32)
                tot = got.astype(np.float64).sum(axis=-1)
                if ns == 3:
                    assert np.array_equal(tot, f.astype(np.float64))
                else:
                    assert np.all(np.abs(tot - f) <= 2.0 ** -15 * np.abs(f))


def test_build_flags():
    """Every HIP source is compiled for gfx950 with packed FP32 instructions
    switched off (the compiler would otherwise form v_pk_* FP32 ops from
    ordinary float code), and every source file in csrc is built."""
    import glob
    import os
    from paper_2408_06698_amd import build as B
    assert "--offload-arch=gfx950" in B.FLAGS
    i = B.FLAGS.index("-packed-fp32-ops")
    assert B.FLAGS[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]
    srcs = glob.glob(os.path.join(B.CSRC, "*.hip")) + glob.glob(os.path.join(B.CSRC, "*.cpp"))
    assert {os.path.basename(p) for p in srcs} == set(B.SOURCES)
