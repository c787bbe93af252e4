"""CPU-only checks of the C-ABI library: it loads, exports every function the
header declares, and validates arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skew_evd.h")
LIB = os.path.join(ROOT, "paper_1912_04062_amd", "libskewevd.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(?:int|void|const char \*)\s*\*?\s*(skew_evd\w*)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1912_04062_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for must in ["skew_evd", "skew_evd_ex", "skew_evd_batched", "skew_evd_create",
                 "skew_evd_destroy", "skew_evd_status_string", "skew_evd_band_reduce",
                 "skew_evd_tridiagonalize", "skew_evd_tridiag_eig", "skew_evd_default_opts",
                 "skew_evd_version", "skew_evd_autotune"]:
        assert must in names


def test_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_argument_validation_without_device(lib):
    vp = ctypes.c_void_p
    lib.skew_evd.argtypes = [ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    assert lib.skew_evd(-1, None, 1, 0, None, None, None) == -1
    assert lib.skew_evd(4, None, 4, 1, None, None, None) == -2
    assert lib.skew_evd(4, vp(8), 3, 1, None, None, None) == -3
    assert lib.skew_evd(4, vp(8), 4, 3, None, None, None) == -4
    assert lib.skew_evd(4, vp(8), 4, 2, None, None, None) == -5
    assert lib.skew_evd(4, vp(8), 4, 2, vp(8), None, None) == -6
    assert lib.skew_evd(4, vp(8), 4, 2, vp(8), vp(8), None) == -7
    assert lib.skew_evd(0, None, 1, 0, None, None, None) == 0
    lib.skew_evd_ex.restype = ctypes.c_int
    assert lib.skew_evd_ex(None, 4, vp(8), 4, 1, vp(8), vp(8), 4, vp(8), 4, None, None) == -1
    lib.skew_evd_autotune.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
    assert lib.skew_evd_autotune(None, 100, 0, vp(8), None) == -1


def test_status_strings(lib):
    lib.skew_evd_status_string.restype = ctypes.c_char_p
    lib.skew_evd_status_string.argtypes = [ctypes.c_int]
    for code in range(0, 7):
        assert lib.skew_evd_status_string(code)
    assert b"invalid" in lib.skew_evd_status_string(-3)
    assert lib.skew_evd_version() >= 100


def test_oracle_shares_nothing_with_the_library():
    """The oracle is plain C with no include of the library's sources."""
    src = open(os.path.join(ROOT, "oracle", "skew_oracle.c")).read()
    assert "skew_evd.h" not in src and "csrc" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_1912_04062_amd", "csrc")):
        txt = open(os.path.join(ROOT, "paper_1912_04062_amd", "csrc", f)).read()
        assert "oracle" not in txt.lower()


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's ctypes mirrors of skew_evd_opts / skew_evd_info have the
    C layout: sizes and field offsets from a program compiled against the header."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    from paper_1912_04062_amd import skewevd as s
    fields = {"skew_evd_opts": (s.Opts, ["precision", "band", "max_refine_sweeps", "refine_tol",
                                         "workspace_limit", "profile", "autotune",
                                         "no_fp64_fallback", "debug", "all_pairs", "panel_method",
                                         "reduction", "tridiag_method"]),
              "skew_evd_info": (s.Info, ["ms_total", "ms_stage", "band", "refine_sweeps",
                                         "refine_residual", "workspace_bytes", "kern"])}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "skew_evd.h"', "int main(void) {"]
    for cname, (_, names) in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f in names:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for _, (cls, names) in fields.items():
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f in names]
    assert got == want


def test_noalloc_argument_validation_without_device(lib):
    """The allocation-free entry point checks its arguments, and refuses orders
    above its fixed array's limit, before any device call."""
    vp, ip = ctypes.c_void_p, ctypes.c_int
    f = lib.skew_evd_noalloc
    f.argtypes = [ip, vp, ip, ip, vp, vp, ip, vp, ip, vp]
    f.restype = ip
    nmax = int(re.search(r"#define SKEW_EVD_NOALLOC_NMAX (\d+)", open(HEADER).read()).group(1))
    assert nmax >= 512
    assert f(-1, None, 1, 0, None, None, 1, None, 1, None) == -1
    assert f(4, None, 4, 1, None, None, 4, None, 4, None) == -2
    assert f(4, vp(8), 3, 1, None, None, 4, None, 4, None) == -3
    assert f(4, vp(8), 4, 3, None, None, 4, None, 4, None) == -4
    assert f(4, vp(8), 4, 2, None, None, 4, None, 4, None) == -5
    assert f(4, vp(8), 4, 2, vp(8), None, 4, None, 4, None) == -6
    assert f(4, vp(8), 4, 2, vp(8), vp(8), 3, None, 4, None) == -7
    assert f(4, vp(8), 4, 2, vp(8), vp(8), 4, None, 4, None) == -8
    assert f(4, vp(8), 4, 2, vp(8), vp(8), 4, vp(8), 3, None) == -9
    assert f(0, None, 1, 0, None, None, 1, None, 1, None) == 0
    n = nmax + 1
    assert f(n, vp(8), n, 1, vp(8), vp(8), n, vp(8), n, None) == 4       # NOMEM, no device touched
    lib.skew_evd_status_string.restype = ctypes.c_char_p
    assert b"allocation-free" in lib.skew_evd_status_string(4)
