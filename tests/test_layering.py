"""The oracle is test infrastructure: the product path (the package, the shared input
generators) never imports it, and bench.py reaches it only from its CPU-baseline leg.
Checked on the sources with the ast module (no GPU, nothing imported)."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _oracle_imports(path):
    """(line, enclosing function) of every import of the oracle package in a source file."""
    tree = ast.parse(open(path).read(), filename=path)
    found = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else func
            if isinstance(child, ast.Import):
                if any(a.name == "oracle" or a.name.startswith("oracle.") for a in child.names):
                    found.append((child.lineno, func))
            elif isinstance(child, ast.ImportFrom):
                if child.module and (child.module == "oracle" or child.module.startswith("oracle.")):
                    found.append((child.lineno, func))
            visit(child, f)

    visit(tree, None)
    return found


def _py_files(sub):
    for dirpath, _, files in os.walk(os.path.join(ROOT, sub)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(dirpath, f)


def test_product_path_never_imports_the_oracle():
    offenders = [(p, hit) for sub in ("paper_2601_08374_amd", "synthetic") for p in _py_files(sub)
                 for hit in _oracle_imports(p)]
    assert offenders == []


def test_bench_imports_the_oracle_only_in_its_cpu_baseline_leg():
    hits = _oracle_imports(os.path.join(ROOT, "bench.py"))
    assert hits, "bench.py times the oracle on the host"
    assert {func for _, func in hits} <= {"cpu_baseline", "cpu_baseline_forms"}


def test_graft_entry_imports_the_oracle_only_in_smoke():
    hits = _oracle_imports(os.path.join(ROOT, "__graft_entry__.py"))
    assert {func for _, func in hits} <= {"smoke"}


def test_missing_library_fails_loudly():
    """With no built library the binding raises; there is no fallback path to run instead."""
    import subprocess
    import sys
    env = dict(os.environ, PAELAST_LIB=os.path.join(ROOT, "no_such_dir", "libpaelast.so"))
    code = ("import sys\n"
            "from paper_2601_08374_amd import capi\n"
            "try:\n"
            "    capi.pa_elast_ndofs\n"
            "except RuntimeError as e:\n"
            "    print(e); sys.exit(3)\n"
            "sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 3, r.stdout + r.stderr
    assert "not built" in r.stdout
