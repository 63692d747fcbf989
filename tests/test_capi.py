"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/icnnm.h, and its host logic behaves without a GPU."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2604_17001_amd import icnnm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "icnnm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(icnnm_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["icnnm_create", "icnnm_destroy", "icnnm_last_error", "icnnm_learn_eigvecs", "icnnm_solve",
              "icnnm_solve_batch", "icnnm_submit", "icnnm_poll", "icnnm_params_default"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = icnnm.load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(icnnm.EXPORTS) == _declared()


def test_params_default():
    lib = icnnm.load_library()
    p = icnnm.Params()
    lib.icnnm_params_default(C.byref(p))
    assert math.isinf(p.lam) and p.theta0 == 0 and p.rho == 1.1 and p.theta_max == 1e10
    assert p.max_iter == 100 and p.tol == 0 and p.precision == 0 and p.refresh_every == 10 and p.check_v == 0


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets as the C compiler lays out include/icnnm.h
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text("""#include <stdio.h>
#include <stddef.h>
#include "icnnm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(icnnm_shape), sizeof(icnnm_params), sizeof(icnnm_info),
         offsetof(icnnm_info, t_device_s), offsetof(icnnm_info, tile), offsetof(icnnm_params, check_v));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(icnnm.Shape), C.sizeof(icnnm.Params), C.sizeof(icnnm.Info),
                   icnnm.Info.t_device_s.offset, icnnm.Info.tile.offset, icnnm.Params.check_v.offset]


def test_null_context_is_rejected():
    lib = icnnm.load_library()
    assert lib.icnnm_solve(None, None, None, None, None, None, None, None, None) == icnnm.E_INVALID
    assert lib.icnnm_poll(None, C.c_uint64(1), None) == icnnm.E_INVALID
    assert lib.icnnm_create(0, 0, None) == icnnm.E_INVALID
    assert lib.icnnm_last_error(None) == b"NULL context"


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = icnnm.load_library()
    h = C.c_void_p()
    assert lib.icnnm_create(0, 0, C.byref(h)) == icnnm.E_DEVICE
    assert not h.value
