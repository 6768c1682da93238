"""The product path has no CPU fallback: the binding refuses to run without
the HIP library, and no module of the package imports the oracle."""

import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2608_30239_amd")


def test_binding_fails_loudly_without_the_library(tmp_path):
    # a fresh interpreter, so that no library is loaded yet
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2608_30239_amd import native as N\n"
            "try:\n"
            "    N.load(%r)\n"
            "except FileNotFoundError as e:\n"
            "    print('refused:', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(1)\n") % (ROOT, str(tmp_path / "libmcpd.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "refused" in r.stdout, r.stdout + r.stderr


def test_package_never_imports_the_oracle():
    for name in os.listdir(PKG):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            else:
                continue
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (name, mods)
