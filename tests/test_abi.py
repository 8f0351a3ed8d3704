"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/pase.h, and validates arguments without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2502_04589_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pase.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pase_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nat.LIB_PATH):
        pytest.fail("libpase.so is not built (run __graft_entry__.build())")
    return nat.load()


def test_header_declares_the_core_api():
    names = declared_functions()
    for core in ("pase_setup", "pase_solve", "pase_destroy", "pase_workspace_bytes"):
        assert core in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = declared_functions()
    bound = {s[0] for s in nat.SIGNATURES}
    for name in names:
        assert hasattr(lib, name), f"{name} not exported"
        assert name in bound, f"{name} has no ctypes signature"


def test_options_default_and_status_strings(lib):
    opt = nat.Options()
    lib.pase_options_default(C.byref(opt))
    assert opt.precision == 0 and opt.cg_steps == 2 and opt.nu == 2
    assert abs(opt.omega - 2.0 / 3.0) < 1e-15
    for code in range(7):
        assert lib.pase_status_string(code)


def _problem(dim, levels):
    p = nat.Problem()
    p.dim = dim
    p.nlevels = len(levels)
    for i, n in enumerate(levels):
        p.n[i] = n
    p.kappa = None
    return p


def test_workspace_query_validates_arguments(lib):
    opt = nat.Options()
    lib.pase_options_default(C.byref(opt))
    opt.nev_max = 10
    nbytes = C.c_size_t(0)
    assert lib.pase_workspace_bytes(C.byref(_problem(2, [128, 64, 32, 16])), C.byref(opt), C.byref(nbytes)) == 0
    # ten fine multi-vectors of 127^2 x 10 doubles at least
    assert nbytes.value >= 10 * 127 * 127 * 10 * 8
    bad = [_problem(4, [8, 4]), _problem(2, [8, 3]), _problem(2, [8]), _problem(3, [9, 4])]
    for p in bad:
        assert lib.pase_workspace_bytes(C.byref(p), C.byref(opt), C.byref(nbytes)) == 1
        assert lib.pase_last_error(None)
    opt.nev_max = 0
    assert lib.pase_workspace_bytes(C.byref(_problem(2, [8, 4])), C.byref(opt), C.byref(nbytes)) == 1
    opt.nev_max = 4
    opt.precision = 1
    assert lib.pase_workspace_bytes(C.byref(_problem(2, [8, 4])), C.byref(opt), C.byref(nbytes)) in (0, 6)


def test_setup_rejects_null_and_small_workspace_without_gpu_work(lib):
    opt = nat.Options()
    lib.pase_options_default(C.byref(opt))
    h = C.c_void_p()
    p = _problem(2, [8, 4])
    assert lib.pase_setup(C.byref(p), C.byref(opt), None, 0, None, C.byref(h)) == 1
    # a host buffer with a too-small size is rejected before any device call
    buf = (C.c_uint8 * 512)()
    addr = (C.addressof(buf) + 255) & ~255
    assert lib.pase_setup(C.byref(p), C.byref(opt), C.c_void_p(addr), 256, None, C.byref(h)) == 3
    assert not h.value


def test_entry_points_reject_null_handle(lib):
    assert lib.pase_apply(None, 0, 1, None, None, None) == 1
    assert lib.pase_solve(None, 1, 1e-8, None, None, None, None) == 1
    assert lib.pase_destroy(None) == 0
    assert lib.pase_unet_save(None, b"/nonexistent/x") == 1
    assert lib.pase_unet_load(None, b"/nonexistent/x") == 1


def _c_layout(type_name, fields):
    """sizeof(type) and offsetof(type, f) for each field, from the C compiler on the real header."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    prog = "#include <stdio.h>\n#include <stddef.h>\n#include \"pase.h\"\nint main(void){\n"
    prog += f'printf("%zu\\n", sizeof({type_name}));\n'
    for f in fields:
        prog += f'printf("%zu\\n", offsetof({type_name}, {f}));\n'
    prog += "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(prog)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cls, cname", [(nat.Report, "pase_report"), (nat.Options, "pase_options"),
                                        (nat.Problem, "pase_problem")])
def test_ctypes_structs_match_the_header_layout(cls, cname):
    """The binding's structures have the C layout of include/pase.h (size and every field offset)."""
    names = [f[0] for f in cls._fields_]
    got = _c_layout(cname, names)
    assert got[0] == C.sizeof(cls)
    for name, off in zip(names, got[1:]):
        assert getattr(cls, name).offset == off, name
