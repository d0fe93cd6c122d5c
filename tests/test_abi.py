"""The C-ABI library loads and exports every symbol include/vrph.h declares,
and the Python record layouts match the C structs (no GPU calls)."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrph.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vrph_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vrph_create", "vrph_pdist", "vrph_barcode_from_dist", "vrph_barcode_from_points",
                 "vrph_batch_plan", "vrph_batch_forward", "vrph_backward"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2502_05063_amd import vrph

    L = vrph.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_c():
    from paper_2502_05063_amd import vrph
    import ctypes

    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "vrph.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(vrph_pair), sizeof(vrph_stats),
         offsetof(vrph_pair, birth_edge), offsetof(vrph_stats, tau_eff),
         offsetof(vrph_stats, total_ms));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    assert vals[0] == vrph.PAIR_DTYPE.itemsize
    assert vals[1] == ctypes.sizeof(vrph.Stats)
    assert vals[2] == vrph.PAIR_DTYPE.fields["birth_edge"][1]
    assert vals[3] == vrph.Stats.tau_eff.offset
    assert vals[4] == vrph.Stats.total_ms.offset


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2502_05063_amd import vrph

    monkeypatch.setattr(vrph, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(vrph, "_lib", None)
    with pytest.raises(ImportError):
        vrph.lib()
