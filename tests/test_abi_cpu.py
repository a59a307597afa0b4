"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/ofrr.h, its structs have the header's layout, and
the no-device / NULL-argument paths answer with the documented status."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2505_00281_amd import ofrr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofrr.h")


def _declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ofrr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_and_library_exports_every_entry_point():
    lib = ofrr.load_library()
    declared = _declared_functions()
    assert "ofrr_eig_partial" in declared and "ofrr_svd_partial" in declared
    assert sorted(declared) == sorted(ofrr.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ofrr.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (ofrr_[a-z0-9_]+)", out))
    assert set(declared) <= exported


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "ofrr.h"
int main(void) {
  printf("%zu %zu %zu\\n", sizeof(ofrr_matrix), sizeof(ofrr_plan), sizeof(ofrr_info));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(ofrr_plan, lo), offsetof(ofrr_plan, max_iters),
         offsetof(ofrr_plan, b_split), offsetof(ofrr_plan, profile), offsetof(ofrr_plan, tail_product));
  printf("%zu %zu\\n", offsetof(ofrr_matrix, values), offsetof(ofrr_matrix, nnz));
  printf("%zu\\n", offsetof(ofrr_info, max_resid));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0:3] == [ctypes.sizeof(ofrr.Matrix), ctypes.sizeof(ofrr.Plan), ctypes.sizeof(ofrr.Info)]
    assert vals[3:8] == [ofrr.Plan.lo.offset, ofrr.Plan.max_iters.offset, ofrr.Plan.b_split.offset,
                         ofrr.Plan.profile.offset, ofrr.Plan.tail_product.offset]
    assert vals[8:10] == [ofrr.Matrix.values.offset, ofrr.Matrix.nnz.offset]
    assert vals[10] == ofrr.Info.max_resid.offset


def test_plan_defaults():
    p = ofrr.Plan()
    ofrr.load_library().ofrr_plan_default(ctypes.byref(p))
    assert (p.basis_dtype, p.gram_accum, p.refine, p.filter, p.degree) == (ofrr.F64, ofrr.ACC_F64, 0,
                                                                          ofrr.POWER, 1)
    assert (p.max_iters, p.stall_iters, p.b_split, p.profile, p.tail_product) == (20, 3, 1, 0, 0)


def test_descriptors_keep_their_tensors_alive():
    """A descriptor built from temporaries must keep them alive: it holds raw
    pointers, and freed device memory is recycled by the caching allocator
    (regression: a CSR descriptor built from temporaries pointed at reused
    memory)."""
    import gc
    import weakref
    import torch
    refs = []

    def make():
        rp = torch.tensor([0, 1, 2], dtype=torch.int32)
        ci = torch.tensor([0, 1], dtype=torch.int32)
        v = torch.tensor([1.0, 2.0])
        refs.extend(weakref.ref(t) for t in (rp, ci, v))
        return ofrr.csr_matrix(rp, ci, v)

    m = make()
    gc.collect()
    assert all(r() is not None for r in refs)
    assert m.row_ptr == refs[0]().data_ptr() and m.col_idx == refs[1]().data_ptr()
    d = ofrr.dense_matrix(torch.eye(3, dtype=torch.float64) * 2, symmetric=True)
    gc.collect()
    assert d._keep[0].data_ptr() == d.values
    with pytest.raises(ofrr.OfrrError):
        ofrr.csr_matrix(torch.tensor([0, 1]), torch.tensor([0]), torch.tensor([1.0]))  # int64 indices


def test_null_context_and_no_device_status():
    lib = ofrr.load_library()
    assert lib.ofrr_eig_partial(None, None, 1, 1, 0, None, None, None, None, None, None) == ofrr.ERR_INVALID_ARG
    assert lib.ofrr_destroy(None) == ofrr.ERR_INVALID_ARG
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    st = lib.ofrr_create(ctypes.byref(h), 0, None)
    assert st == ofrr.ERR_NO_DEVICE
    assert b"device" in lib.ofrr_last_error(None)
    with pytest.raises(ofrr.OfrrError):
        ofrr.Context(0)
