"""The oracle and the product path share nothing (no GPU): read from the
sources' syntax trees, the library's Python modules never import the oracle,
the oracle imports nothing of the package, and the benchmark and the entry
module import the oracle only inside the functions that time or check
against it."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2103_14870_amd")


def imports(path):
    """(module name, enclosing top-level function or None) of every import."""
    tree = ast.parse(open(path).read(), filename=path)
    out = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = func
            if func is None and isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)):
                f = child.name
            if isinstance(child, ast.Import):
                out.extend((a.name, f) for a in child.names)
            elif isinstance(child, ast.ImportFrom):
                out.append((child.module or "", f))
            visit(child, f)

    visit(tree, None)
    return out


def test_package_never_imports_the_oracle():
    for name in sorted(os.listdir(PKG)):
        if name.endswith(".py"):
            mods = [m for m, _ in imports(os.path.join(PKG, name))]
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), name


def test_oracle_imports_nothing_of_the_package():
    for name in sorted(os.listdir(os.path.join(ROOT, "oracle"))):
        if name.endswith(".py"):
            mods = [m for m, _ in imports(os.path.join(ROOT, "oracle", name))]
            assert not any(m.startswith("paper_2103_14870_amd") for m in mods), name
            assert all(m.split(".")[0] in ("__future__", "itertools", "dataclasses", "numpy", "scipy", "math")
                       for m in mods), (name, mods)


def test_oracle_is_imported_only_where_it_is_the_baseline_or_the_check():
    allowed = {"bench.py": {"cpu_baseline", "cpu_baseline_qs"}, "__graft_entry__.py": {"smoke"}}
    for name, funcs in allowed.items():
        for mod, func in imports(os.path.join(ROOT, name)):
            if mod == "oracle" or mod.startswith("oracle."):
                assert func in funcs, (name, mod, func)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No fallback: with no built library the binding raises instead of
    computing anything elsewhere."""
    import subprocess
    import sys

    code = f"from paper_2103_14870_amd import gfem; gfem.load({str(tmp_path / 'libgfem.so')!r})"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "FileNotFoundError" in r.stderr and "is not built" in r.stderr


def test_binding_holds_one_library(tmp_path):
    """Once a library is loaded, calls without a path reuse it and naming
    another file raises instead of mixing two builds in one process."""
    import subprocess
    import sys

    code = (
        "from paper_2103_14870_amd import gfem\n"
        "a = gfem.load()\n"
        "assert gfem.load() is a and gfem.load(gfem.LIB_PATH) is a\n"
        "try:\n"
        f"    gfem.load({str(tmp_path / 'other.so')!r})\n"
        "except RuntimeError as e:\n"
        "    assert 'already loaded' in str(e)\n"
        "    print('refused')\n"
    )
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "refused"
