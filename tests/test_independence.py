"""The oracle and the library share no code: neither imports the other, the
library's Python files never import the oracle, and the oracle imports no
compiled extension.  Only the seeded input generators (synth) serve both,
and synth imports neither."""
import ast
import glob
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            out.add(node.module.split(".")[0])
    return out


def _files(sub):
    return glob.glob(os.path.join(ROOT, sub, "**", "*.py"), recursive=True)


def test_oracle_imports_no_library_code():
    for f in _files("oracle"):
        bad = _imports(f) & {"paper_2408_06698_amd", "ctypes", "torch"}
        assert not bad, (f, bad)


def test_library_imports_no_oracle():
    for f in _files("paper_2408_06698_amd"):
        assert "oracle" not in _imports(f), f


def test_synth_imports_neither():
    for f in _files("synth"):
        assert not (_imports(f) & {"oracle", "paper_2408_06698_amd"}), f


def test_native_sources_do_not_reference_the_oracle():
    for f in glob.glob(os.path.join(ROOT, "paper_2408_06698_amd", "csrc", "*")):
        assert "oracle" not in open(f, errors="replace").read().lower(), f
