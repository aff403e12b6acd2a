"""The C ABI without a GPU: the library loads, exports every function that
include/lpcg.h declares (and no other lpcg_ function), and the binding's
ctypes structures have the layout the C compiler gives the header's."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpcg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(lpcg_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = _declared()
    for must in ("lpcg_analyze", "lpcg_pcg_solve", "lpcg_gnn_predict_L", "lpcg_ic0", "lpcg_sptrsv",
                 "lpcg_spmv", "lpcg_llt_loss", "lpcg_gnn_backward", "lpcg_adam_step"):
        assert must in names, must


def test_library_exports_every_declared_symbol():
    from paper_2305_16432_amd import lpcg
    L = lpcg.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lpcg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if re.search(r" T lpcg_\w+$", ln)})
    assert exported == _declared()
    assert L.lpcg_version  # callable without a device
    L.lpcg_version.restype = ctypes.c_char_p
    assert L.lpcg_version().decode()


def test_binding_struct_layout_matches_header():
    from paper_2305_16432_amd import lpcg
    structs = {"lpcg_csr": lpcg._CSR, "lpcg_info": lpcg._Info, "lpcg_precond": lpcg._Precond,
               "lpcg_solve_opts": lpcg._Opts, "lpcg_result": lpcg._Result, "lpcg_gnn": lpcg._Gnn,
               "lpcg_trsv_cfg": lpcg._TrsvCfg, "lpcg_blk_schedule": lpcg._BlkSchedule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lpcg.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write("\n".join(lines))
        cc = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                             "-I", "/opt/rocm/include", c, "-o", exe], capture_output=True, text=True)
        if cc.returncode != 0:
            pytest.fail(cc.stderr[-2000:])
        got = dict(ln.split() for ln in subprocess.run([exe], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def test_colour_ordering_row_limit():
    """The colour ordering's row limit: the binding's constant is the header's,
    and a larger analysis is refused (EINVAL) on the host, before any device
    work, so this runs without a GPU (the array pointers are never read)."""
    from paper_2305_16432_amd import lpcg
    m = re.search(r"#define\s+LPCG_COLOR_MAX_ROWS\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == lpcg.COLOR_MAX_ROWS
    L = lpcg.lib()
    dummy = (ctypes.c_int32 * 4)()
    dval = (ctypes.c_double * 4)()
    for n, ordering in ((lpcg.COLOR_MAX_ROWS + 1, lpcg.ORDER_COLOR), (1 << 22, lpcg.ORDER_COLOR)):
        A = lpcg._CSR(n, 7 * n, ctypes.cast(dummy, ctypes.c_void_p), ctypes.cast(dummy, ctypes.c_void_p),
                      ctypes.cast(dval, ctypes.c_void_p))
        out = ctypes.c_void_p()
        rc = L.lpcg_analyze(ctypes.byref(A), None, ctypes.c_int32(1), ctypes.c_int32(ordering),
                            ctypes.byref(out), None)
        assert rc == lpcg.EINVAL and not out.value
        L.lpcg_last_error.restype = ctypes.c_char_p
        assert b"colour ordering" in L.lpcg_last_error()
