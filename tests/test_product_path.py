"""CPU tests of the product path's boundary: without the HIP library it fails
loudly (no fallback), and no module of the package reaches the oracle."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2104_00794_amd")


def test_missing_library_raises():
    code = ("from paper_2104_00794_amd import tpx\n"
            "tpx.LIB_PATH = '/nonexistent/libtpx.so'\n"
            "try:\n"
            "    tpx.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    raise SystemExit(3)\n"
            "raise SystemExit(0)\n")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert p.returncode == 3, p.stdout + p.stderr
    assert "not built" in p.stdout


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_package_never_imports_the_oracle():
    files = [os.path.join(PKG, f) for f in os.listdir(PKG) if f.endswith(".py")]
    assert len(files) >= 6
    for f in files:
        for name in _imports(f):
            assert not name.split(".")[0] == "oracle", (f, name)


def test_bench_uses_the_oracle_only_for_the_cpu_baseline():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    owners = []
    for fn in [n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)]:
        for node in ast.walk(fn):
            if isinstance(node, (ast.Import, ast.ImportFrom)):
                names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                if any(n.split(".")[0] == "oracle" for n in names):
                    owners.append(fn.name)
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    assert not any("oracle" in ast.dump(n) for n in top)
    assert owners == ["cpu_baseline"]
