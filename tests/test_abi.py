"""The C-ABI library loads and exports every function its header declares
(CPU only: nothing is called that needs a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mick.h")
LIB = os.path.join(ROOT, "paper_2601_15401_amd", "libmick.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mick_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("mick_keygen", "mick_encrypt", "mick_mul_k", "mick_relin_k", "mick_rescale_multi",
              "mick_mul_relin_rescale", "mick_decrypt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libmick.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.mick_strerror.restype = ctypes.c_char_p
    assert lib.mick_strerror(0) == b"ok"
    assert lib.mick_strerror(-3) == b"k exceeds the key set"
    # argument validation happens before any device work
    out = ctypes.c_void_p()
    assert lib.mick_params_create(12, 3, 1, 3, ctypes.byref(out)) == -1
    assert lib.mick_params_create(13, 3, 9, 3, ctypes.byref(out)) == -1
    assert lib.mick_params_create(16, 32, 8, 2, ctypes.byref(out)) == -1
