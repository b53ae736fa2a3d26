"""The Stokes set-up kernel's arithmetic, emulated in numpy from the
library's own host tables and element frames (hopu_host_tables 20-25,
hopu_host_mesh 6), against the oracle's element Schur complements S_T
(paper section 2.3, static condensation of sigma and gamma).

This checks the tables and the formulas the kernel evaluates (the rows of G,
the multiplier form of the nt condition, the scaling of the condensed
blocks) on the CPU; the GPU tests check the kernel itself.  No GPU needed.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import stokes as OST
from oracle.space import Space
from paper_2408_06698_amd import _lib as L


def _table(d, k, which):
    n = L.lib().hopu_host_tables(d, k, which, None, 0)
    assert n > 0
    out = np.zeros(n)
    L.lib().hopu_host_tables(d, k, which, out.ctypes.data_as(C.c_void_p), n)
    return out


def _frames(m):
    vid = np.ascontiguousarray(m.elem_vid, dtype=np.int64)
    xyz = np.ascontiguousarray(m.elem_xyz, dtype=np.float64)
    args = (m.dim, vid.shape[0], vid.ctypes.data_as(C.c_void_p), xyz.ctypes.data_as(C.c_void_p), 6)
    n = L.lib().hopu_host_mesh(*args, None, 0)
    out = np.zeros(n)
    L.lib().hopu_host_mesh(*args, out.ctypes.data_as(C.c_void_p), n)
    return out.reshape(-1, 64)


def _dp(d, k):
    if k < 0:
        return 0
    if d == 1:
        return k + 1
    return (k + 1) * (k + 2) // 2 if d == 2 else (k + 1) * (k + 2) * (k + 3) // 6


def emulate_ST(d, k, geo, nu, dt, tabs):
    """S_T as the set-up kernel forms it, for one element frame."""
    Ea, Gc, MpG, TV, Phi, Mref = tabs
    nE, nG = d * d - 1, d * (d - 1) // 2
    nP1, nPk = _dp(d, k + 1), _dp(d, k)
    nft, nf = _dp(d - 1, k + 1), _dp(d - 1, k)
    ntop = nft - nf
    n = d * nPk
    nfl = (d + 1) * nf
    Ea = Ea.reshape(nE, d, d)
    Gc = Gc.reshape(nG, d, d)
    MpG = MpG.reshape(nPk, nP1)
    TV = TV.reshape(nP1, n, d, d)
    Phi = Phi.reshape(d + 1, nP1, nft)
    Mref = Mref.reshape(n, n, d, d)
    J = geo[0:9].reshape(3, 3)[:d, :d]
    Ji = geo[9:18].reshape(3, 3)[:d, :d]
    det = geo[18]
    adet, sgn = abs(det), np.sign(det)
    fr = [geo[20 + 11 * f:31 + 11 * f] for f in range(d + 1)]
    nout = [f[0:d] for f in fr]
    tang = [[f[3:3 + d], f[6:6 + d]][:d - 1] for f in fr]
    NFn = [f[9] for f in fr]
    inter = [f[10] > 0.5 for f in fr]
    H = np.einsum("rp,aqp,qs->ars", Ji, Ea, J)
    rows = []
    # gamma rows
    ge = np.einsum("cij,aij->ca", Gc, Ea)
    for c in range(nG):
        for be in range(nPk):
            rows.append((-adet * ge[c][:, None] * MpG[be][None, :]).ravel())
    # nt multipliers
    for f in range(d + 1):
        for c in range(d - 1):
            ent = np.einsum("p,apq,q->a", nout[f], Ea, tang[f][c])
            for m in range(ntop):
                r = adet * ent[:, None] * Phi[f, :, nf + m][None, :] if inter[f] else np.zeros((nE, nP1))
                rows.append(r.ravel())
    # velocity rows
    vol = np.einsum("ars,pirs->iap", H, TV)        # [n][a][alpha]
    pint = adet ** ((d - 1) / d)
    for i in range(n):
        if i < nfl:
            f, j = divmod(i, nf)
            sf = (-1.0 if f % 2 else 1.0) * sgn
            enn = np.einsum("p,apq,q->a", nout[f], Ea, nout[f])
            r = -NFn[f] * sgn * vol[i] + sf * NFn[f] * enn[:, None] * Phi[f, :, j][None, :]
        else:
            r = -pint * sgn * vol[i]
        rows.append(r.ravel())
    # u^ rows
    for f in range(d + 1):
        for c in range(d - 1):
            etn = np.einsum("p,apq,q->a", tang[f][c], Ea, nout[f])
            for j in range(nf):
                r = NFn[f] * etn[:, None] * Phi[f, :, j][None, :] if inter[f] else np.zeros((nE, nP1))
                rows.append(r.ravel())
    G = np.array(rows)
    n1 = nG * nPk + (d + 1) * (d - 1) * ntop
    K = -(2.0 * nu / adet) * G @ G.T
    K11, K21, K22 = K[:n1, :n1], K[n1:, :n1], K[n1:, n1:]
    keep = np.abs(K11).sum(1) > 0          # wall multipliers drop out
    K11, K21 = K11[np.ix_(keep, keep)], K21[:, keep]
    S = -K22 + K21 @ np.linalg.solve(K11, K21.T)
    Gm = J.T @ J
    Sc = np.array([NFn[i // nf] if i < nfl else pint for i in range(n)])
    S[:n, :n] += np.einsum("rs,ijrs->ij", Gm, Mref) * np.outer(Sc, Sc) / adet / dt
    return S


@pytest.mark.parametrize("d,k,walls", [(2, 1, False), (2, 2, True), (2, 3, False), (2, 4, True),
                                       (3, 1, False), (3, 2, True), (3, 3, False), (3, 4, True)])
def test_emulated_setup_matches_oracle_schur_blocks(d, k, walls):
    per = tuple(a != 1 for a in range(d)) if walls else (True,) * d
    m = synth.kuhn_mesh(d, (3,) * d, periodic=per, jitter=0.15, jitter_seed=4)
    sp = Space(m.elem_vid, m.elem_xyz, k)
    nu, dt = 0.03, 0.01
    tabs = [_table(d, k, w) for w in range(20, 26)]
    geo = _frames(m)
    elems = list(range(0, sp.topo.n_elems, max(1, sp.topo.n_elems // 6)))
    hg = OST.uhat_gdof(sp)
    loc = np.concatenate([sp.gdof, np.where(hg >= 0, sp.n_dof + hg, -1)], 1)
    # the element matrices' conditioning grows with k (the oracle's monomial
    # stress basis and null-space reduction as much as the condensation):
    # up to 1.1e-10 relative at 3D k = 3 (jittered), 8.8e-10 at 2D k = 4,
    # 1e-9 to 6e-9 at 3D k = 4
    tol = {1: 1e-10, 2: 1e-10, 3: 5e-10, 4: 2e-8}[k]
    for T in elems:
        S = emulate_ST(d, k, geo[T], nu, dt, tabs)
        ref_T = OST._schur_block(sp, OST.element_blocks(sp, T, nu), T, dt, hg.shape[1])
        keep = loc[T] >= 0
        ref = ref_T[np.ix_(keep, keep)]
        got = S[np.ix_(keep, keep)]
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (T, np.abs(got - ref).max())
