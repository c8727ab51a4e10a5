"""The functions of bench.py and of the package's Python modules read only
names they define, import or receive, their module's own names and builtins
(a static check on the CPU: rarely run branches, such as bench.py --extras,
would otherwise fail only on the GPU)."""
import ast
import builtins
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bound(node):
    """Names a function binds anywhere inside it (nested scopes included)."""
    out = set()
    for n in ast.walk(node):
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            out.add(n.id)
        elif isinstance(n, ast.arg):
            out.add(n.arg)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                out.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            out.add(n.name)
        elif isinstance(n, ast.ExceptHandler) and n.name:
            out.add(n.name)
    return out


FILES = ["bench.py", "__graft_entry__.py", "paper_1310_2078_amd/sl1m.py",
         "paper_1310_2078_amd/serve.py", "paper_1310_2078_amd/refine.py",
         "paper_1310_2078_amd/coarse.py", "paper_1310_2078_amd/workloads.py",
         "paper_1310_2078_amd/build.py"]


@pytest.mark.parametrize("path", FILES)
def test_functions_use_defined_names(path):
    tree = ast.parse(open(os.path.join(ROOT, path), encoding="utf-8").read())
    module = set(dir(builtins))
    for n in tree.body:
        if isinstance(n, (ast.FunctionDef, ast.ClassDef)):
            module.add(n.name)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                module.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, (ast.Assign, ast.AnnAssign)):
            for t in (n.targets if isinstance(n, ast.Assign) else [n.target]):
                for x in ast.walk(t):
                    if isinstance(x, ast.Name):
                        module.add(x.id)
    missing = []
    fns = [n for n in tree.body if isinstance(n, ast.FunctionDef)]
    for c in (n for n in tree.body if isinstance(n, ast.ClassDef)):
        fns += [n for n in c.body if isinstance(n, ast.FunctionDef)]
    for fn in fns:
        known = module | _bound(fn)
        for x in ast.walk(fn):
            if isinstance(x, ast.Name) and isinstance(x.ctx, ast.Load) and x.id not in known:
                missing.append(f"{fn.name}: {x.id} (line {x.lineno})")
    assert not missing, missing
