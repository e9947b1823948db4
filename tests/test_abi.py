"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function that include/mstab.h declares, and rejects bad arguments
before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1604_06043_amd import mstab

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mstab.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mstab_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return mstab.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mstab.EXPORTS) == names


def test_options_defaults(lib):
    o = mstab.mstab_options_default()
    assert o.struct_size == ctypes.sizeof(mstab.mstab_options)
    assert o.tol == 1e-8 and o.max_replacements == 3 and o.method == mstab.METHOD_MSTAB
    assert o.fetch == mstab.FETCH_THRESHOLD and abs(o.fetch_rel - 1e-4) < 1e-18


def test_status_strings(lib):
    for st in (0, 1, -1, -2, -3, -4, -5):
        assert lib.mstab_status_str(st)
    assert lib.mstab_status_str(-99) == b"unknown status"


def test_convdiff_nnz_closed_form(lib, orc):
    for dim, n in ((2, 1), (2, 7), (2, 64), (3, 5), (3, 128), (3, 256)):
        assert lib.mstab_convdiff_nnz(dim, n) == orc._load().orc_convdiff_nnz(dim, n)
    assert lib.mstab_convdiff_nnz(4, 3) == -1


def test_create_rejects_bad_arguments_without_a_device(lib):
    h = ctypes.c_void_p()
    assert lib.mstab_create(None, 4, 2, None, None, ctypes.byref(h)) == mstab.E_INVALID
    assert h.value is None
    csr = mstab.mstab_csr(10, 28, 8, 8, 8)   # non-null dummies: rejected on s, l, n first
    for s, ell in ((0, 1), (9, 1), (2, 0), (2, 9)):
        assert lib.mstab_create(ctypes.byref(csr), s, ell, None, None, ctypes.byref(h)) == mstab.E_INVALID
    csr.n = 3
    assert lib.mstab_create(ctypes.byref(csr), 4, 1, None, None, ctypes.byref(h)) == mstab.E_INVALID
    o = mstab.mstab_options_default()
    o.struct_size = 3
    csr.n = 100
    assert lib.mstab_create(ctypes.byref(csr), 4, 1, ctypes.byref(o), None, ctypes.byref(h)) == mstab.E_INVALID
    assert b"struct_size" in lib.mstab_last_error(None)
    assert lib.mstab_destroy(None) == mstab.OK
    assert lib.mstab_solve_next(None, None, None, None) == mstab.E_INVALID


def test_workgroup_engine_option_checks_without_a_device(lib):
    """ENGINE_WORKGROUP refuses what its kernel does not do, before any device
    work (dummy matrix pointers are never dereferenced)."""
    h = ctypes.c_void_p()
    csr = mstab.mstab_csr(100, 280, 8, 8, 8)
    for over in (dict(engine=2), dict(engine=1, precision=mstab.PREC_F32_MATRIX),
                 dict(engine=1, precond=mstab.PRECOND_JACOBI), dict(engine=1, reorder=mstab.REORDER_RCM),
                 dict(engine=1, orthonormalize_recycle=1)):
        o = mstab.mstab_options_default(**over)
        assert lib.mstab_create(ctypes.byref(csr), 4, 2, ctypes.byref(o), None, ctypes.byref(h)) == mstab.E_INVALID
        assert h.value is None
        assert b"engine" in lib.mstab_last_error(None).lower() or b"ENGINE" in lib.mstab_last_error(None)
    csr.n = (1 << 20) + 1
    o = mstab.mstab_options_default(engine=1)
    assert lib.mstab_create(ctypes.byref(csr), 4, 2, ctypes.byref(o), None, ctypes.byref(h)) == mstab.E_INVALID


def test_struct_layouts_match_header(tmp_path):
    """ctypes layouts equal what a C compiler makes of include/mstab.h."""
    import subprocess
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mstab.h"', 'int main(void) {']
    for cls in (mstab.mstab_csr, mstab.mstab_options, mstab.mstab_info):
        name = cls.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ['return 0; }']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for cls in (mstab.mstab_csr, mstab.mstab_options, mstab.mstab_info):
        name = cls.__name__
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_solve_batch_rejects_bad_arguments_without_a_device(lib):
    P = ctypes.c_void_p
    assert lib.mstab_solve_batch(None, 0, None, None, None) == mstab.OK
    assert lib.mstab_solve_batch(None, -1, None, None, None) == mstab.E_INVALID
    assert lib.mstab_solve_batch(None, mstab.MAX_BATCH + 1, None, None, None) == mstab.E_INVALID
    assert lib.mstab_solve_batch(None, 2, None, None, None) == mstab.E_INVALID
    nulls = (P * 2)(None, None)
    assert lib.mstab_solve_batch(nulls, 2, nulls, nulls, None) == mstab.E_INVALID
    assert b"NULL entry" in lib.mstab_last_error(None)


def test_csr_check_refuses_malformed_patterns(lib):
    """The structure check that mstab_create, mstab_spmv and mstab_jacobi_split
    run before any product (here its host entry point)."""
    import numpy as np
    rp = np.array([0, 2, 4, 5], dtype=np.int32)
    ci = np.array([0, 1, 0, 2, 2], dtype=np.int32)
    mstab.mstab_csr_check(rp, ci)                        # well formed
    bad = [
        (np.array([1, 2, 4, 5]), ci),                    # row_ptr[0] != 0
        (np.array([0, 3, 2, 5]), ci),                    # decreasing row pointer
        (np.array([0, 2, 4, 4]), ci),                    # row_ptr[n] != nnz
        (rp, np.array([0, 1, 0, 3, 2])),                 # a column equal to n
        (rp, np.array([0, 1, -1, 2, 2])),                # a negative column
        (rp, np.array([1, 0, 0, 2, 2])),                 # columns not increasing
        (rp, np.array([0, 0, 0, 2, 2])),                 # a repeated column
    ]
    for r, c in bad:
        with pytest.raises(mstab.MstabError) as e:
            mstab.mstab_csr_check(r, c)
        assert e.value.status == mstab.E_INVALID
    # the host order computation refuses the same patterns
    with pytest.raises(mstab.MstabError):
        mstab.mstab_rcm_order(rp, np.array([0, 1, 0, 3, 2], dtype=np.int32))
