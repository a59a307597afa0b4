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
  printf("%zu %zu %zu %zu\\n", offsetof(ofrr_info, max_resid), offsetof(ofrr_plan, gram_switch_t),
         offsetof(ofrr_info, gram_t_max), offsetof(ofrr_info, grams_f64));
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
    assert vals[10:14] == [ofrr.Info.max_resid.offset, ofrr.Plan.gram_switch_t.offset,
                           ofrr.Info.gram_t_max.offset, ofrr.Info.grams_f64.offset]


def test_plan_defaults():
    p = ofrr.Plan()
    ofrr.load_library().ofrr_plan_default(ctypes.byref(p))
    assert (p.basis_dtype, p.gram_accum, p.refine, p.filter, p.degree) == (ofrr.F64, ofrr.ACC_F64, 0,
                                                                          ofrr.POWER, 1)
    assert (p.max_iters, p.stall_iters, p.b_split, p.profile, p.tail_product) == (20, 3, 1, 0, 0)
    assert p.gram_switch_t == 0.0


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


def _unbound_context():
    """A Context object that never reached the library (no GPU here): the
    binding's argument checks run before any library call, so they can be
    exercised on the CPU."""
    import torch
    c = ofrr.Context.__new__(ofrr.Context)
    c.lib, c.h, c.device = None, None, torch.device("cuda", 0)
    return c


def test_binding_rejects_host_tensors_and_short_blocks():
    import torch
    c = _unbound_context()
    A = torch.eye(8, dtype=torch.float64).t()  # column-major view
    with pytest.raises(ofrr.OfrrError) as e:   # V has 7 rows, A has 8 columns
        c.block_product(A, torch.zeros(7, 4, dtype=torch.float64))
    assert e.value.status == ofrr.ERR_INVALID_ARG and "rows" in str(e.value)
    with pytest.raises(ofrr.OfrrError) as e:   # trans: A^T V needs rows(A) = 8 rows
        c.block_product_sliced(torch.zeros(8, 5, dtype=torch.float64).t().contiguous().t(),
                               torch.zeros(5, 4, dtype=torch.float64), trans=True)
    assert "rows" in str(e.value)
    with pytest.raises(ofrr.OfrrError) as e:   # right shape, but host memory
        c.block_product(A, torch.zeros(8, 4, dtype=torch.float64))
    assert e.value.status == ofrr.ERR_INVALID_ARG and "cuda" in str(e.value)
    with pytest.raises(ofrr.OfrrError):
        c.eig_partial(A, 2, 4)
    with pytest.raises(ofrr.OfrrError):
        c.svd_partial(A, 2, 4)
    with pytest.raises(ofrr.OfrrError):
        c.hessenberg(torch.zeros(8, 4), 0.0)
    with pytest.raises(ofrr.OfrrError):
        c.project(torch.zeros(8, 4), torch.zeros(8, 4))
    with pytest.raises(ofrr.OfrrError):
        c.quantize(torch.zeros(16))
    with pytest.raises(ofrr.OfrrError):
        c.pencil_eig(torch.eye(4, dtype=torch.float64), torch.eye(4, dtype=torch.float64))
    rp = torch.tensor([0, 1, 2], dtype=torch.int32)
    csr = ofrr.csr_matrix(rp, torch.tensor([0, 1], dtype=torch.int32), torch.tensor([1.0, 2.0]))
    with pytest.raises(ofrr.OfrrError):        # host CSR arrays
        c.block_product(csr, torch.zeros(2, 4, dtype=torch.float32), v_dtype="f32")


def test_binding_rejects_mismatched_element_types():
    import torch
    c = _unbound_context()
    A = torch.eye(8, dtype=torch.float32).t()
    with pytest.raises(ofrr.OfrrError) as e:   # 4-byte V declared as FP64
        c.block_product(A, torch.zeros(8, 4, dtype=torch.float32), v_dtype="f64")
    assert "elements" in str(e.value)
