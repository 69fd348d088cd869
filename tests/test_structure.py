"""Structure of the repository that the parity claims rest on: the oracle and
the GPU package share no code and import nothing from each other, the input
generators hold no arithmetic of the method and import neither, and the
package refuses to work without its compiled library (no CPU fallback)."""

import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(folder):
    """Top-level module names imported by the Python files of a folder."""
    found = {}
    for dirpath, _, files in os.walk(os.path.join(ROOT, folder)):
        for f in files:
            if not f.endswith(".py"):
                continue
            tree = ast.parse(open(os.path.join(dirpath, f)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    names = [a.name for a in node.names]
                elif isinstance(node, ast.ImportFrom) and node.level == 0:
                    names = [node.module or ""]
                else:
                    continue
                for n in names:
                    found.setdefault(n.split(".")[0], set()).add(os.path.join(dirpath, f))
    return found


def test_oracle_and_package_import_nothing_from_each_other():
    assert "paper_2502_12350_amd" not in _imports("oracle")
    assert "oracle" not in _imports("paper_2502_12350_amd")


def test_input_generators_import_neither_side():
    imp = _imports("seisgen")
    assert "oracle" not in imp and "paper_2502_12350_amd" not in imp


def test_package_fails_loudly_without_its_library(tmp_path):
    # a fresh interpreter pointed at a library that does not exist
    env = dict(os.environ, WFD_LIB=str(tmp_path / "missing.so"))
    code = ("import paper_2502_12350_amd._lib as L\n"
            "try:\n    L.lib()\nexcept ImportError as e:\n    print('refused:', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=120)
    assert "refused:" in out.stdout, out.stdout + out.stderr
