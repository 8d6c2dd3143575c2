"""The C-ABI library loads and exports every function that include/bingo.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "bingo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bingo_[a-z0-9_]+)\s*\(", text)))


def _lib_path():
    from paper_2504_10233_amd import build_lib, lib_path
    if not os.path.exists(lib_path()):
        build_lib.build()
    return lib_path()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["bingo_build", "bingo_update_batch", "bingo_walk", "bingo_ppr"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2504_10233_amd import binding
    assert sorted(binding.EXPORTS) == _declared()


def test_strerror_without_gpu():
    lib = ctypes.CDLL(_lib_path())
    lib.bingo_strerror.restype = ctypes.c_char_p
    assert lib.bingo_strerror(0) == b"ok"
    assert b"range" in lib.bingo_strerror(-2)


def test_build_rejects_bad_arguments_without_gpu():
    # argument checks happen before any device call
    lib = ctypes.CDLL(_lib_path())
    out = ctypes.c_void_p()
    assert lib.bingo_build(None, 10, 0, None, None, None, None, ctypes.byref(out)) == -1


def test_probe_rejects_bad_arguments_without_gpu():
    lib = ctypes.CDLL(_lib_path())
    f = lib.bingo_probe_random_reads
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]
    ms = ctypes.c_float()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its argument checks
    assert f(None, 1 << 20, 256, 4, 0, 64, 1, fake, ctypes.byref(ms), None) == -1
    assert f(fake, 1 << 20, 256, 4, 0, 32, 1, fake, ctypes.byref(ms), None) == -1   # line width
    assert f(fake, 1 << 10, 256, 4, 0, 64, 1, fake, ctypes.byref(ms), None) == -1   # table too small
    assert f(fake, 1 << 20, 100, 4, 0, 64, 1, fake, ctypes.byref(ms), None) == -1   # lanes
    assert f(fake, 1 << 20, 256, 3, 0, 64, 1, fake, ctypes.byref(ms), None) == -1   # reads


def test_replay_probe_rejects_bad_arguments_without_gpu():
    lib = ctypes.CDLL(_lib_path())
    f = lib.bingo_probe_replay
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                  ctypes.c_void_p]
    ms = ctypes.c_float()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its argument checks
    assert f(None, fake, 10, 5, 256, 256, 1, 1, fake, ctypes.byref(ms), None) == -1     # no graph
    assert f(fake, None, 10, 5, 256, 256, 1, 1, fake, ctypes.byref(ms), None) == -1     # no visits
    assert f(fake, fake, 10, 5, 256, 256, 1, 1, None, ctypes.byref(ms), None) == -1     # no counters


def test_quantize_rejects_bad_arguments_without_gpu():
    lib = ctypes.CDLL(_lib_path())
    f = lib.bingo_quantize_biases
    f.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint32, ctypes.c_void_p,
                  ctypes.c_void_p]
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its argument checks
    assert f(8, None, 1.0, 8, fake, None) == -1
    assert f(8, fake, 1.0, 8, None, None) == -1
    assert f(8, fake, 1.0, 0, fake, None) == -1      # frac_bits 1..16
    assert f(8, fake, 1.0, 17, fake, None) == -1
    assert f(8, fake, 0.0, 8, fake, None) == -1      # lambda > 0
    assert f(8, fake, float("nan"), 8, fake, None) == -1
    assert f(8, fake, float("inf"), 8, fake, None) == -1


def test_build_rejects_bad_frac_bits_without_gpu():
    from paper_2504_10233_amd.binding import _Config
    lib = ctypes.CDLL(_lib_path())
    out = ctypes.c_void_p()
    for fb, al in ((17, 0), (8, 1), (0, 2)):  # too many fraction bits; alias with fixed point; bad flag
        cfg = _Config(ctypes.sizeof(_Config), 1, 40, 10, 0, fb, al)
        assert lib.bingo_build(ctypes.byref(cfg), 10, 0, None, None, None, None, ctypes.byref(out)) == -1


def test_build_rejects_bad_radix_without_gpu():
    from paper_2504_10233_amd.binding import _Config
    lib = ctypes.CDLL(_lib_path())
    out = ctypes.c_void_p()
    # base 3; base 4 with fixed-point biases or alias rows; a nonzero reserved word
    for fb, al, rb, rs in ((0, 0, 3, 0), (8, 0, 4, 0), (0, 1, 4, 0), (0, 0, 4, 1)):
        cfg = _Config(ctypes.sizeof(_Config), 1, 40, 10, 0, fb, al, rb, rs)
        assert lib.bingo_build(ctypes.byref(cfg), 10, 0, None, None, None, None, ctypes.byref(out)) == -1


def test_missing_library_fails_loudly(tmp_path):
    # the package without its shared library: the first call raises, nothing falls back to the host
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2504_10233_amd"
    pkg.mkdir()
    src = os.path.join(ROOT, "paper_2504_10233_amd")
    for f in ("__init__.py", "binding.py"):
        shutil.copy(os.path.join(src, f), pkg / f)
    code = ("import numpy as np, paper_2504_10233_amd as b\n"
            "try:\n"
            "    b.Graph(4, np.array([0]), np.array([1]), np.array([1]), device='cpu')\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=tmp_path)
    assert r.returncode == 0, r.stderr
    assert "raised: libbingo.so is not built" in r.stdout


def test_header_is_plain_c(tmp_path):
    # the boundary is a C ABI: the header compiles as C99 with every warning on
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler on this host")
    c = tmp_path / "h.c"
    c.write_text('#include "bingo.h"\nint main(void) { bingo_walk_query q; bingo_config g; bingo_server_config s;\n'
                 '(void)q; (void)g; (void)s; return bingo_strerror(0) == 0; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-c", str(c), "-o", str(tmp_path / "h.o")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
