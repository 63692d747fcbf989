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


def test_plan_of_a_video_tensor():
    # 64x64x16 with an 8x8x4 kernel: the state holds the scaled multiplier and the
    # Z-step operand, m x kp floats each, plus smaller partials
    pl = icnnm.plan((64, 64, 16), (8, 8, 4))
    assert pl["padded_k"] == 256
    b = pl["tile"]
    assert pl["ntiles"] == int(math.prod(pl["tiles_per_dim"]))
    assert tuple(-(-m // t) for m, t in zip((64, 64, 16), b)) == pl["tiles_per_dim"]
    assert pl["ntiles"] * math.prod(b) >= 64 * 64 * 16
    assert pl["state_bytes"] >= 2 * 64 * 64 * 16 * 256 * 4
    # the reduced precisions keep the multiplier U in 16 bits (two bytes per state entry
    # fewer) and add two m-float arrays (running adjoint and delta of L)
    lo = icnnm.plan((64, 64, 16), (8, 8, 4), precision="bf16")
    m, kp = 64 * 64 * 16, 256
    assert lo["state_bytes"] == pl["state_bytes"] - 2 * m * kp + 2 * m * 4


def _gather_codes_fit(pl, dims, kdims):
    """Every gather-table entry (tile << shift) | box position of the plan fits a
    non-negative int32, with shift the bits of the largest box extent."""
    lead = 3 - len(dims)
    kd = (1,) * lead + tuple(kdims)
    E = [b + k - 1 for b, k in zip(pl["tile"], kd)]
    shift = max(1, (max(E) - 1).bit_length())
    return max(pl["tiles_per_dim"]) << shift < 2 ** 31


def test_plan_keeps_tile_indices_in_the_gather_encoding():
    # gather-table entries pack (tile << shift) | position into an int32; an order-1
    # tensor of 10M entries (39063 tiles of 256 rows, more than a 16-bit field holds)
    # must get codes that fit, never wrapped ones
    n = 10_000_000
    for joint in (False, True):
        pl = icnnm.plan((n,), (4,), joint=joint)
        assert pl["tile"][:2] == (1, 1) and pl["tiles_per_dim"][2] * pl["tile"][2] >= n
        assert _gather_codes_fit(pl, (n,), (4,))
    # 2^24 entries, the largest order-1 extent
    pl = icnnm.plan((1 << 24,), (3,))
    assert _gather_codes_fit(pl, (1 << 24,), (3,))
    # a long innermost dimension beside a large kernel
    pl = icnnm.plan((4, 1 << 20), (4, 31))
    assert _gather_codes_fit(pl, (4, 1 << 20), (4, 31))


def test_plan_rejects_bad_shapes():
    with pytest.raises(icnnm.IcnnmError) as e:
        icnnm.plan((8, 8), (9, 2))
    assert e.value.code == icnnm.E_INVALID
    lib = icnnm.load_library()
    s = icnnm.make_shape((8, 8, 8), (2, 2, 2))
    s.ndim = 4
    p = icnnm.make_params(lib)
    out = icnnm.PlanInfo()
    assert lib.icnnm_plan(C.byref(s), C.byref(p), 0, C.byref(out)) == icnnm.E_INVALID
    # NULL shape
    assert lib.icnnm_plan(None, C.byref(p), 0, C.byref(out)) == icnnm.E_INVALID
