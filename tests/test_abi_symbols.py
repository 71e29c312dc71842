"""The C-ABI library loads and exports every function include/sidm.h
declares; the binding declares the same names.  No compute call (CPU only)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sidm.h")
LIB = os.path.join(ROOT, "paper_2506_06269_amd", "libsidm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sidm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("sidm_create", "sidm_destroy", "sidm_status_string", "sidm_last_error",
                     "sidm_gravity", "sidm_knn_h", "sidm_scatter", "sidm_kdk_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsidm.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (sidm_[a-z_]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = C.CDLL(LIB)
    for n in declared():
        assert getattr(lib, n) is not None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsidm.so not built")
def test_binding_names_match_header():
    import paper_2506_06269_amd as S
    assert set(S.EXPORTED) == set(declared())
    for n in declared():
        assert callable(getattr(S, n)), n
    assert S.lib().sidm_status_string(S.SIDM_ERR_CAPACITY) == b"device capacity exceeded"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsidm.so not built")
def test_struct_layouts_match_header():
    """Field sizes of the binding's ctypes structures against the C compiler's."""
    import tempfile
    import paper_2506_06269_amd as S
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "sidm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(sidm_halo),
         sizeof(sidm_state), sizeof(sidm_diag), sizeof(sidm_event), offsetof(sidm_halo, seed),
         offsetof(sidm_diag, n_events), offsetof(sidm_diag, status), sizeof(sidm_center),
         offsetof(sidm_center, index), offsetof(sidm_halo, eta), offsetof(sidm_halo, max_bin),
         offsetof(sidm_halo, tree_alpha), offsetof(sidm_diag, n_grav_terms));
  return 0; }
'''
    d = tempfile.mkdtemp()
    c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert got == [C.sizeof(S.SidmHalo), C.sizeof(S.SidmState), C.sizeof(S.SidmDiag),
                   S.EVENT_BYTES, S.SidmHalo.seed.offset, S.SidmDiag.n_events.offset,
                   S.SidmDiag.status.offset, C.sizeof(S.SidmCenter), S.SidmCenter.index.offset,
                   S.SidmHalo.eta.offset, S.SidmHalo.max_bin.offset,
                   S.SidmHalo.tree_alpha.offset, S.SidmDiag.n_grav_terms.offset]
