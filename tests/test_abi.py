"""CPU checks of the C-ABI boundary: the library loads, exports every declared entry
point, its structures have the layout the binding assumes, and it fails cleanly
(an error code, no abort) when no GPU is present."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2505_06021_amd import rpa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpa.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(rpa_\w+)\s*\(", src, re.M)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(rpa.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rpa.LIB_PATH):
        pytest.skip("librpa.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", rpa.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = set(re.findall(r" T (rpa_\w+)", out))
    missing = [f for f in declared_functions() if f not in syms]
    assert not missing, missing
    rpa.load()   # and the dynamic loader resolves it


def test_struct_layouts_match_header():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "rpa.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(rpa_system), offsetof(rpa_system, kq),
         offsetof(rpa_system, philox_seed), offsetof(rpa_system, vhalf), offsetof(rpa_system, nk_occ),
         offsetof(rpa_system, S_ao), offsetof(rpa_system, eps_d),
         sizeof(rpa_freq), sizeof(rpa_result), sizeof(rpa_stats));
  return 0;
}
'''
    import ctypes as C
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    want = [C.sizeof(rpa.RpaSystemC), rpa.RpaSystemC.kq.offset, rpa.RpaSystemC.philox_seed.offset,
            rpa.RpaSystemC.vhalf.offset, rpa.RpaSystemC.nk_occ.offset, rpa.RpaSystemC.S_ao.offset,
            rpa.RpaSystemC.eps_d.offset, C.sizeof(rpa.RpaFreqC),
            C.sizeof(rpa.RpaResultC),
            C.sizeof(rpa.RpaStatsC)]
    assert got == want


def test_init_without_gpu_returns_error_code():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    if not os.path.exists(rpa.LIB_PATH):
        pytest.skip("librpa.so not built")
    with pytest.raises(rpa.RpaError) as e:
        rpa.Context()
    assert e.value.code in (rpa.RPA_E_DEVICE, rpa.RPA_E_ARG)
