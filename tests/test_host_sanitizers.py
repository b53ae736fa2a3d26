"""The library's host-side mesh and table code (host_tables.cpp) built with
g++ and AddressSanitizer + UndefinedBehaviorSanitizer (host code only), run
on 2D and 3D meshes (periodic, walled, graded, jittered, relabelled): no
sanitizer report, the same mesh arrays as the library builds, and the
builder's error paths."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from paper_2408_06698_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_06698_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("asan") / "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "host_check.cpp"),
           os.path.join(CSRC, "host_tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _relabel(mesh, seed):
    rng = np.random.default_rng(seed)
    E, d = mesh.elem_vid.shape[0], mesh.dim
    perm = rng.permutation(E)
    vmap = rng.permutation(int(mesh.elem_vid.max()) + 1)
    lp = np.argsort(rng.random((E, d + 1)), axis=1)
    vid = np.take_along_axis(vmap[mesh.elem_vid[perm]], lp, 1)
    xyz = np.take_along_axis(mesh.elem_xyz[perm], lp[:, :, None], 1)
    return d, np.ascontiguousarray(vid, dtype=np.int64), np.ascontiguousarray(xyz)


def _library_array(dim, vid, xyz, which, dtype):
    args = (dim, vid.shape[0], vid.ctypes.data_as(C.c_void_p), xyz.ctypes.data_as(C.c_void_p), which)
    n = L.lib().hopu_host_mesh(*args, None, 0)
    out = np.zeros(n, dtype=dtype)
    L.lib().hopu_host_mesh(*args, out.ctypes.data_as(C.c_void_p), n)
    return out


@pytest.mark.parametrize("cfg,n,kmax,relabel", [(1, (4, 5), 4, False), (3, (3, 4, 3), 5, False),
                                                (3, (3, 4, 3), 3, True), (2, (3, 3, 3), 2, True)])
def test_host_code_under_sanitizers(checker, tmp_path, cfg, n, kmax, relabel):
    mesh, _, _ = synth.make_config(cfg, n_override=n)
    if relabel:
        dim, vid, xyz = _relabel(mesh, 17)
    else:
        dim, vid, xyz = mesh.dim, np.ascontiguousarray(mesh.elem_vid, np.int64), np.ascontiguousarray(mesh.elem_xyz)
    mf, of = tmp_path / "mesh.bin", tmp_path / "out.bin"
    with open(mf, "wb") as f:
        f.write(np.array([dim, vid.shape[0]], dtype=np.int64).tobytes() + vid.tobytes() + xyz.tobytes())
    r = subprocess.run([checker, str(mf), str(of), str(kmax)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("ok")
    raw = open(of, "rb").read()
    nf, nn, ng, nb = np.frombuffer(raw[:32], dtype=np.int64)
    o = 32
    fid = np.frombuffer(raw[o:o + 4 * nf], dtype=np.int32); o += 4 * nf
    nbr = np.frombuffer(raw[o:o + 4 * nn], dtype=np.int32); o += 4 * nn
    geo = np.frombuffer(raw[o:o + 8 * ng], dtype=np.float64); o += 8 * ng
    bat = np.frombuffer(raw[o:o + 4 * nb], dtype=np.int32)
    assert np.array_equal(fid, _library_array(dim, vid, xyz, 0, np.int32))
    assert np.array_equal(nbr, _library_array(dim, vid, xyz, 1, np.int32))
    assert np.array_equal(geo, _library_array(dim, vid, xyz, 3, np.float64))
    assert np.array_equal(bat, _library_array(dim, vid, xyz, 5, np.int32))
