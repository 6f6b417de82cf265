"""CPU-only checks of the top-level scripts (bench.py, __graft_entry__.py):
every global name that one of their functions refers to is defined at module
level or is a builtin, so that no leg of a run stops on a missing helper.
Nothing is run on a GPU."""
import builtins
import os
import symtable

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _globals_used(table, out):
    if table.get_type() == "function":
        for sym in table.get_symbols():
            if sym.is_global() and sym.is_referenced():
                out.add((table.get_name(), sym.get_name()))
    for child in table.get_children():
        _globals_used(child, out)


@pytest.mark.parametrize("script", ["bench.py", "__graft_entry__.py"])
def test_script_functions_refer_only_to_defined_names(script):
    path = os.path.join(ROOT, script)
    with open(path) as fh:
        src = fh.read()
    top = symtable.symtable(src, path, "exec")
    defined = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    used = set()
    _globals_used(top, used)
    missing = sorted((fn, n) for fn, n in used if n not in defined and not hasattr(builtins, n))
    assert not missing, missing
