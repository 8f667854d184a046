"""C-ABI boundary checks that need no GPU: the library loads and exports
every function that include/pms.h declares; without a device, creation
fails cleanly with a status instead of crashing."""
import ctypes
import os

import pytest

import paper_2403_00306_amd as pms


def test_header_lists_the_boundary():
    names = pms.header_functions()
    for must in ["pms_create", "pms_solve", "pms_destroy", "pms_last_error",
                 "pms_solve_device", "pms_solve_batch", "pms_submit",
                 "pms_poll", "pms_release", "pms_autotune"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = pms.load_library()
    missing = [n for n in pms.header_functions() if not hasattr(lib, n)]
    assert missing == []


def test_status_strings():
    lib = pms.load_library()
    assert lib.pms_status_string(0) == b"PMS_OK"
    assert lib.pms_status_string(-2) == b"PMS_EBASE"
    assert lib.pms_status_string(-5) == b"PMS_EBUSY"
    assert lib.pms_status_string(42) == b"PMS_UNKNOWN"


def test_null_arguments_rejected_without_device():
    lib = pms.load_library()
    assert lib.pms_create(None, None) == pms.PMS_EINVAL
    assert lib.pms_last_error(None) == b"out is NULL"
    lib.pms_destroy(None)   # NULL-safe
    s = pms.Stats()
    assert lib.pms_last_stats(None, ctypes.byref(s)) == pms.PMS_EINVAL
    assert lib.pms_solve(None, b"A", 1, 1, 1, 0, None, None) == pms.PMS_EINVAL


def test_structure_layout_matches_header(tmp_path):
    # compile a probe against include/pms.h and compare every field offset
    # with the ctypes mirrors used by the binding
    structs = {"pms_options": pms.Options, "pms_instance": pms.CInstance,
               "pms_result": pms.CResult, "pms_stats": pms.Stats,
               "pms_serve_stats": pms.ServeStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pms.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));'
                         % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include")
    subprocess.check_call(["gcc", "-I", inc, "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)])
               .decode().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_create_without_gpu_fails_cleanly():
    with pytest.raises(pms.PmsError) as e:
        pms.Context()
    assert e.value.status in (pms.PMS_EDEVICE, pms.PMS_EINVAL)
