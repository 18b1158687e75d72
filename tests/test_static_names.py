"""Every global name a function of the host-side Python modules reads is
defined at module level or is a builtin (catches stray references that only
fail when a rarely used path runs, e.g. a benchmark workload)."""
import builtins
import os
import symtable

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["bench.py", "__graft_entry__.py", "paper_2408_06880_amd/lbm.py",
         "paper_2408_06880_amd/server.py", "paper_2408_06880_amd/autotune.py",
         "paper_2408_06880_amd/inputs.py", "paper_2408_06880_amd/build.py",
         "oracle/__init__.py"]


def _module_names(top):
    names = set(dir(builtins)) | {"__file__", "__name__"}
    for sym in top.get_symbols():
        if sym.is_assigned() or sym.is_imported() or sym.is_namespace():
            names.add(sym.get_name())
    return names


def _undefined(table, defined, path=""):
    out = []
    for child in table.get_children():
        where = f"{path}.{child.get_name()}"
        if child.get_type() == "function":
            for sym in child.get_symbols():
                if sym.is_global() and sym.is_referenced() and sym.get_name() not in defined:
                    out.append(f"{where}: {sym.get_name()}")
        out += _undefined(child, defined, where)
    return out


@pytest.mark.parametrize("rel", FILES)
def test_no_undefined_globals(rel):
    path = os.path.join(ROOT, rel)
    src = open(path).read()
    top = symtable.symtable(src, path, "exec")
    assert _undefined(top, _module_names(top)) == []
