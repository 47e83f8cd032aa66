"""The C-ABI library loads on a host without a GPU, exports every function that
include/lagot.h declares, and the ctypes structures of the binding have the C
layout (checked against a C program compiled from the header). No compute call
is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lagot.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2601_05765_amd as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2601_05765_amd import build
        build.build()
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lagot_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for f in ("lagot_cells", "lagot_newton_step", "lagot_solve", "lagot_create", "lagot_destroy"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    import paper_2601_05765_amd as L
    names = declared_functions()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == names


def test_strerror_and_defaults(lib):
    import paper_2601_05765_amd as L
    assert L.strerror(0) == "ok"
    assert "capacity" in L.strerror(L.ECAPACITY)
    o = L.default_opts()
    assert o.tol == 1e-5 and o.max_newton == 100 and o.max_halvings == 30 and o.cg_max_iter == 1000


def test_struct_layout_matches_header(tmp_path):
    import paper_2601_05765_amd as L
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "lagot.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(lagot_box), sizeof(lagot_opts), sizeof(lagot_stats));
  printf("%zu %zu %zu %zu\n", offsetof(lagot_opts, cg_rtol), offsetof(lagot_opts, threads_per_cell),
         offsetof(lagot_stats, max_rel_err), offsetof(lagot_stats, ms_linear));
  return 0; }
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b = subprocess.check_output([str(exe)]).decode().split("\n")[:2]
    sizes = [int(v) for v in a.split()]
    offs = [int(v) for v in b.split()]
    assert sizes == [ctypes.sizeof(L.Box), ctypes.sizeof(L.Opts), ctypes.sizeof(L.Stats)]
    assert offs == [L.Opts.cg_rtol.offset, L.Opts.threads_per_cell.offset, L.Stats.max_rel_err.offset,
                    L.Stats.ms_linear.offset]


def test_product_path_has_no_oracle_dependency():
    """The package never imports or links the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2601_05765_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "lagot_oracle" not in text, f


def test_fluid_params_defaults_and_layout(lib, tmp_path):
    """lagot_fluid_params: the binding's structure matches the header, and the library's
    defaults are the documented ones (host-only call, no GPU needed)."""
    import ctypes
    import paper_2601_05765_amd as L
    p = L.default_fluid_params()
    assert (p.dt, p.eps, p.gamma, p.mu, list(p.gravity), p.cg_rtol, p.cg_max_iter) == \
        (1e-3, 1.0, 0.0, 0.0, [0.0, 0.0, -9.81], 1e-10, 2000)
    src = tmp_path / "fl.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "lagot.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(lagot_fluid_params), offsetof(lagot_fluid_params, gravity),
         offsetof(lagot_fluid_params, cg_rtol), offsetof(lagot_fluid_params, cg_max_iter));
  return 0; }
''')
    exe = tmp_path / "fl"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).decode().split()]
    F = L.FluidParams
    assert got == [ctypes.sizeof(F), F.gravity.offset, F.cg_rtol.offset, F.cg_max_iter.offset]


def test_constants_match_header():
    """The binding's copies of the header's constants (parameter count, row limit of the
    allocation-free forward)."""
    import paper_2601_05765_amd as L
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(LAGOT_[A-Z0-9_]+)\s+(-?\d+)\b", text))
    assert int(defs["LAGOT_MLP_NPARAMS"]) == L.MLP_NPARAMS
    assert int(defs["LAGOT_NOALLOC_MAX_ROWS"]) == L.NOALLOC_MAX_ROWS
