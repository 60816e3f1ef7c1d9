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
    assert lib.mick_params_create(13, 3, 25, 3, ctypes.byref(out)) == -1   # K > 24
    assert lib.mick_params_create(16, 40, 8, 1, ctypes.byref(out)) == -1   # digit of 40 primes
    assert lib.mick_params_create(16, 34, 8, 34, ctypes.byref(out)) == -1  # 34 digits


def test_queue_schedule_allocator_validate_without_gpu():
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    out = vp()
    # queue: NULL arrays, bad set counts, tiny capacity
    lib.mick_queue_create.argtypes = [vp, vp, ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
    assert lib.mick_queue_create(None, None, 1, 1 << 20, ctypes.byref(out)) == -1
    arr = (vp * 1)(None)
    assert lib.mick_queue_create(ctypes.cast(arr, vp), ctypes.cast(arr, vp), 0, 1 << 20, ctypes.byref(out)) == -1
    assert lib.mick_queue_create(ctypes.cast(arr, vp), ctypes.cast(arr, vp), 17, 1 << 20, ctypes.byref(out)) == -1
    assert lib.mick_queue_create(ctypes.cast(arr, vp), ctypes.cast(arr, vp), 1, 64, ctypes.byref(out)) == -1
    assert lib.mick_queue_create(ctypes.cast(arr, vp), ctypes.cast(arr, vp), 1, 1 << 20, ctypes.byref(out)) == -1
    assert out.value is None
    lib.mick_queue_push.argtypes = [vp, vp, ctypes.c_int]
    assert lib.mick_queue_push(None, None, 1) == -1
    lib.mick_queue_run.argtypes = [vp, vp]
    assert lib.mick_queue_run(None, None) == -1
    lib.mick_queue_drain.argtypes = [vp, vp]
    assert lib.mick_queue_drain(None, None) == -1
    lib.mick_queue_info.argtypes = [vp, vp, vp, vp]
    assert lib.mick_queue_info(None, None, None, None) == -1
    lib.mick_queue_job_bytes.restype = ctypes.c_size_t
    lib.mick_queue_job_bytes.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    assert lib.mick_queue_job_bytes(None, 0, 2, 3) == 0
    lib.mick_queue_destroy.argtypes = [vp]
    lib.mick_queue_destroy(None)  # NULL-safe
    # schedule
    lib.mick_params_schedule.argtypes = [vp]
    assert lib.mick_params_schedule(None) == -1
    lib.mick_params_set_schedule.argtypes = [vp, ctypes.c_int]
    assert lib.mick_params_set_schedule(None, 8) == -1
    lib.mick_autotune.argtypes = [vp, ctypes.c_char_p]
    assert lib.mick_autotune(None, None) == -1
    # allocator: both functions or neither
    lib.mick_set_allocator.argtypes = [vp, vp, vp]
    cb = ctypes.CFUNCTYPE(vp, ctypes.c_size_t, vp)(lambda n, c: None)
    assert lib.mick_set_allocator(ctypes.cast(cb, vp), None, None) == -1
    assert lib.mick_set_allocator(None, None, None) == 0


def test_tree_planner_and_shapes_without_gpu():
    """The library's planner and shape report (host code) against the oracle's
    planner and Table II counting."""
    from oracle import tree as T
    from paper_2601_15401_amd import mick
    for n in range(2, 18):
        got = mick.tree_plan(n)
        assert got == T.plan(n), n
        assert mick.tree_shape(got) == (n, T.depth(got), T.rs_units(got)[0])
        b = T.binary_plan(n)
        assert mick.tree_shape(b) == (n, T.depth(b), T.rs_units(b)[0])
    for t in [(2, 2, 2), ((3, 2), 1), (1, 1), 5, ((2, 2), (2, 1))]:
        assert mick.tree_shape(t) == (T.n_inputs(t), T.depth(t), T.rs_units(t)[0])
    lib = ctypes.CDLL(LIB)
    arr = (ctypes.c_int * 3)(-2, 2, 0)
    assert lib.mick_tree_shape(arr, 3, None, None, None) == -1          # group of 0
    arr = (ctypes.c_int * 2)(-2, 2)
    assert lib.mick_tree_shape(arr, 2, None, None, None) == -1          # missing child
    arr = (ctypes.c_int * 3)(2, 2, 2)
    assert lib.mick_tree_shape(arr, 3, None, None, None) == -1          # tokens left over
    arr = (ctypes.c_int * 2)(-1, 2)
    assert lib.mick_tree_shape(arr, 2, None, None, None) == -1          # node of one child
    arr = (ctypes.c_int * 1)(-(1 << 31))
    assert lib.mick_tree_shape(arr, 1, None, None, None) == -1
    buf = (ctypes.c_int * 2)()
    assert lib.mick_tree_plan(12, buf, 2) == -1                         # too few token slots
    assert lib.mick_tree_plan(1, buf, 2) == -1


def test_profile_site_selection_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.mick_profile_select.argtypes = [ctypes.c_char_p]
    assert lib.mick_profile_select(b"modup_bconv_passA") == 0
    assert lib.mick_profile_select(b"passB_kip,intt_d.passA") == 0
    assert lib.mick_profile_select(b"no_such_site") == -1
    assert lib.mick_profile_select(b"tensor,") == -1  # an empty name is not a site
    assert lib.mick_profile_select(None) == 0
    assert lib.mick_profile_select(b"") == 0


def test_job_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures against the C compiler's layout of
    mick_job and mick_qjob (a layout mismatch would hand the library shifted
    pointers)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        import pytest
        pytest.skip("gcc not available")
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "mick.h"\n'
                   'int main(void) {\n'
                   ' printf("%zu %zu %zu %zu %zu\\n", sizeof(mick_job), offsetof(mick_job, level), '
                   'offsetof(mick_job, cts), offsetof(mick_job, out), offsetof(mick_job, status));\n'
                   ' printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(mick_qjob), offsetof(mick_qjob, set), '
                   'offsetof(mick_qjob, level), offsetof(mick_qjob, cts), offsetof(mick_qjob, out), '
                   'offsetof(mick_qjob, status));\n return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True, check=True).stdout.split("\n")
    from paper_2601_15401_amd import mick
    J, Q = mick.Job, mick.QJob
    assert [int(x) for x in lines[0].split()] == [ctypes.sizeof(J), J.level.offset, J.cts.offset, J.out.offset,
                                                  J.status.offset]
    assert [int(x) for x in lines[1].split()] == [ctypes.sizeof(Q), Q.set.offset, Q.level.offset, Q.cts.offset,
                                                  Q.out.offset, Q.status.offset]


def test_status_words_and_cancel_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.mick_strerror.restype = ctypes.c_char_p
    assert lib.mick_strerror(-8) != b"unknown status" and lib.mick_strerror(-9) == b"cancelled"
    assert lib.mick_strerror(1) == b"pending"
    lib.mick_queue_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    assert lib.mick_queue_cancel(None, 5) == -1
    lib.mick_output_scale.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int] * 2 + [ctypes.c_void_p]
    assert lib.mick_output_scale(None, None, 3, 3, None) == -1
