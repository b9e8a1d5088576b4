"""Static checks of the Python binding that need no GPU: every name a
function reads is bound in that function, an enclosing one, the module or
builtins (catches a keyword used in a function that does not take it)."""
import ast
import builtins
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["paper_2010_09913_amd/__init__.py", "paper_2010_09913_amd/_native.py",
         "paper_2010_09913_amd/scheduler.py", "bench.py", "__graft_entry__.py"]


def _bound_in(node):
    names = set()
    for sub in ast.walk(node):
        if isinstance(sub, ast.arg):
            names.add(sub.arg)
        elif isinstance(sub, ast.Name) and isinstance(sub.ctx, (ast.Store, ast.Del)):
            names.add(sub.id)
        elif isinstance(sub, (ast.FunctionDef, ast.ClassDef, ast.AsyncFunctionDef)):
            names.add(sub.name)
        elif isinstance(sub, (ast.Import, ast.ImportFrom)):
            for a in sub.names:
                names.add((a.asname or a.name).split(".")[0])
        elif isinstance(sub, ast.ExceptHandler) and sub.name:
            names.add(sub.name)
        elif isinstance(sub, (ast.Global, ast.Nonlocal)):
            names.update(sub.names)
    return names


def _module_bound(tree):
    names = set(dir(builtins)) | {"__file__", "__name__"}
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            names.add(node.name)
        else:
            names |= _bound_in(node)
    return names


@pytest.mark.parametrize("path", FILES)
def test_functions_read_only_bound_names(path):
    tree = ast.parse(open(os.path.join(ROOT, path)).read())
    module = _module_bound(tree)
    problems = []

    fns = (ast.FunctionDef, ast.AsyncFunctionDef, ast.Lambda)

    def visit(fn, outer):
        scope = outer | _bound_in(fn)
        stack = list(ast.iter_child_nodes(fn))
        while stack:
            node = stack.pop()
            if isinstance(node, fns):
                visit(node, scope)      # nested: sees this function's names
                continue
            if isinstance(node, ast.Name) and isinstance(node.ctx, ast.Load) and \
                    node.id not in scope and node.id not in module:
                problems.append(f"{path}:{node.lineno} {getattr(fn, 'name', 'lambda')}: "
                                f"{node.id}")
            stack.extend(ast.iter_child_nodes(node))

    stack = list(ast.iter_child_nodes(tree))
    while stack:
        node = stack.pop()
        if isinstance(node, fns):
            visit(node, set())
        else:
            stack.extend(ast.iter_child_nodes(node))
    assert not problems, problems


def test_header_constants_match_the_binding():
    # every status code and flag the header defines has the same value in the
    # ctypes binding (a drifted flag would silently select another mode)
    import re
    from paper_2010_09913_amd import _native
    hdr = open(os.path.join(ROOT, "include", "slimsell.h")).read()
    consts = {m.group(1): int(m.group(2))
              for m in re.finditer(r"^#define\s+(SS_[A-Z_]+)\s+(-?\d+)", hdr, re.M)}
    consts.update({m.group(1): int(m.group(2))
                   for m in re.finditer(r"^\s+(SS_E[A-Z]+|SS_OK)\s*=\s*(-?\d+)", hdr, re.M)})
    flags = {k: v for k, v in consts.items()
             if k.startswith(("SS_STATS_", "SS_RUN_", "SS_SELL_", "SS_NO_")) or k.startswith("SS_E")
             or k == "SS_OK"}
    assert {"SS_NO_SUMMARY", "SS_SELL_VAL", "SS_EITER", "SS_OK"} <= set(flags)
    for name, value in flags.items():
        assert getattr(_native, name) == value, name
    # flags are distinct single bits
    bits = [v for k, v in flags.items() if not (k.startswith("SS_E") or k == "SS_OK")]
    assert len(set(bits)) == len(bits) and all(b > 0 and b & (b - 1) == 0 for b in bits)
