"""Host-side checks of bench.py (no GPU): its entry point parses the
documented options and does not shadow a module-level import with a local
name (a conditional local import of a module makes every later use of that
name in the function fail when the branch was not taken)."""
import ast
import os
import sys

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)


def _module_imports(tree):
    names = set()
    for node in tree.body:
        if isinstance(node, ast.Import):
            names.update(a.asname or a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            names.update(a.asname or a.name for a in node.names)
    return names


def test_main_does_not_shadow_module_imports():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    top = _module_imports(tree)
    main = [n for n in tree.body if isinstance(n, ast.FunctionDef) and n.name == "main"][0]
    local = set()
    for node in ast.walk(main):
        if isinstance(node, (ast.Import, ast.ImportFrom)):
            local.update(a.asname or a.name.split(".")[0] for a in node.names)
    assert not (local & top), sorted(local & top)


def test_options_parse():
    import bench
    argv = sys.argv
    try:
        sys.argv = ["bench.py", "--steps", "3", "--warmup", "1", "--no-sweep", "--no-compensated"]
        a = bench.parse()
        assert (a.steps, a.warmup, a.gpus, a.levels, a.size) == (3, 1, 1, 1, 16384)
        sys.argv = ["bench.py", "--mfma-probe"]
        assert bench.parse().mfma_probe
    finally:
        sys.argv = argv
