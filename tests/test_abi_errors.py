"""C-ABI argument and mesh errors, forced from the host.  hopu_create
validates the mesh before any HIP call, so these run without a GPU."""
import ctypes as C
import os
import subprocess
import sys
import numpy as np
import pytest

import synth
from paper_2408_06698_amd import _lib as L


def _create(dim, k, vid, xyz):
    h = C.c_void_p()
    vid = np.ascontiguousarray(vid, dtype=np.int64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    st = L.lib().hopu_create(C.byref(h), dim, k, vid.shape[0], vid.ctypes.data_as(C.c_void_p),
                             xyz.ctypes.data_as(C.c_void_p), None)
    return st, h, L.lib().hopu_last_error(None).decode()


def test_bad_arguments():
    m, f, c = synth.make_config(1, n_override=(4, 4))
    assert _create(4, 2, m.elem_vid, m.elem_xyz)[0] == L.HOPU_EINVAL
    assert _create(2, 0, m.elem_vid, m.elem_xyz)[0] == L.HOPU_EINVAL
    assert _create(2, 7, m.elem_vid, m.elem_xyz)[0] == L.HOPU_EINVAL
    st, h, msg = _create(3, 6, np.zeros((1, 4)), np.zeros((1, 4, 3)))
    assert st == L.HOPU_EUNSUPPORTED and "order" in msg
    st = L.lib().hopu_create(None, 2, 2, 1, None, None, None)
    assert st == L.HOPU_EINVAL
    assert L.lib().hopu_sizes(None, None, None, None, None, None, None) == L.HOPU_EINVAL
    L.lib().hopu_destroy(None)


def test_malformed_meshes():
    m, f, c = synth.make_config(1, n_override=(4, 4))
    vid = m.elem_vid.copy()
    vid[3, 1] = vid[3, 0]
    st, h, msg = _create(2, 2, vid, m.elem_xyz)
    assert st == L.HOPU_EMESH and "repeated" in msg
    xyz = m.elem_xyz.copy()
    xyz[5, 2] = xyz[5, 0]
    st, h, msg = _create(2, 2, m.elem_vid, xyz)
    assert st == L.HOPU_EMESH and "degenerate" in msg
    vid = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]])
    st, h, msg = _create(2, 1, vid, np.random.default_rng(0).standard_normal((3, 3, 2)))
    assert st == L.HOPU_EMESH and "more than two" in msg
    # a periodic direction with 2 cells: an element meets itself
    # build a 2-cell periodic strip by identifying x-nodes modulo 2
    xs = np.linspace(0, 1, 3)
    elems, coords = [], []
    for j in range(2):
        for i in range(2):
            a = (i % 2) + 2 * j
            b = ((i + 1) % 2) + 2 * j
            cc = (i % 2) + 2 * (j + 1)
            d = ((i + 1) % 2) + 2 * (j + 1)
            p = lambda ii, jj: [xs[ii], xs[jj]]
            elems += [[a, b, d], [a, cc, d]]
            coords += [[p(i, j), p(i + 1, j), p(i + 1, j + 1)], [p(i, j), p(i, j + 1), p(i + 1, j + 1)]]
    st, h, msg = _create(2, 1, np.array(elems), np.array(coords))
    assert st == L.HOPU_EMESH


def test_alloc_failure_is_reported():
    """HOPU_TEST_FAIL_ALLOC=1 makes every device allocation fail, so the
    first one in create does: create returns HOPU_ENOMEM, frees what it
    holds and leaves the handle NULL (run in a child process with the env
    set)."""
    code = (
        "import ctypes as C, numpy as np, synth\n"
        "from paper_2408_06698_amd import _lib as L\n"
        "m, f, c = synth.make_config(1, n_override=(4, 4))\n"
        "h = C.c_void_p()\n"
        "v = np.ascontiguousarray(m.elem_vid); x = np.ascontiguousarray(m.elem_xyz)\n"
        "st = L.lib().hopu_create(C.byref(h), 2, 2, v.shape[0], v.ctypes.data_as(C.c_void_p), "
        "x.ctypes.data_as(C.c_void_p), None)\n"
        "print(st, L.lib().hopu_last_error(None).decode())\n"
        "assert st == L.HOPU_ENOMEM and h.value is None\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, HOPU_TEST_FAIL_ALLOC="1", PYTHONPATH=root)
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=root)
    assert res.returncode == 0, res.stderr + res.stdout


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No CPU fallback: without libhopu.so the binding's entry to the
    library raises, naming the build command, and so does reading the
    error of a failed call."""
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libhopu.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError, match="build"):
        L.lib()
    with pytest.raises(ImportError):
        L.check(L.HOPU_OK + 1)


def test_binding_checks_buffers_before_the_library():
    """Device pointers cannot be checked by the library, so the binding
    refuses short, host-resident, mistyped or non-tensor buffers first."""
    import torch
    from paper_2408_06698_amd.hopu import _dev
    with pytest.raises(TypeError):
        _dev(np.zeros(4), 4)
    with pytest.raises(ValueError, match="expected 4 entries"):
        _dev(torch.zeros(3, dtype=torch.float64), 4)
    with pytest.raises(ValueError, match="on the GPU"):
        _dev(torch.zeros(4, dtype=torch.float64), 4)
    with pytest.raises(ValueError, match="expected 5 entries"):
        _dev(torch.zeros(4, dtype=torch.int8), 5, torch.int8, "l_per_facet")


def test_stokes_entry_points_reject_a_null_context():
    """The implicit Stokes step's calls validate their context first (no HIP
    call is made), and the host tables of every supported order build."""
    lib = L.lib()
    assert lib.hopu_stokes_sizes(None, None, None, None) == L.HOPU_EINVAL
    assert lib.hopu_stokes_setup(None, 0.1, 0.1, 0) == L.HOPU_EINVAL
    assert lib.hopu_stokes_apply(None, None, None) == L.HOPU_EINVAL
    assert lib.hopu_stokes_precond(None, None, None) == L.HOPU_EINVAL
    assert lib.hopu_stokes_step(None, None, 0, None, 1e-10, 10, None) == L.HOPU_EINVAL
    for d, k in [(2, 1), (2, 4), (3, 1), (3, 4)]:
        for which in range(20, 26):
            assert lib.hopu_host_tables(d, k, which, None, 0) > 0
