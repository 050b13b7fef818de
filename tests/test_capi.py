"""The C-ABI library loads and exports every symbol the public header declares;
argument checks that run before any HIP call.  No GPU needed."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ngfreg.h")
LIB = os.path.join(ROOT, "paper_1812_06765_amd", "libngfreg.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ngf_status|void|const char\*)\s+(ngf_\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1812_06765_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("ngf_build_pyramid", "ngf_eval_J_grad", "ngf_lbfgs_step", "ngf_register",
              "ngf_eval_pair"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_argument_checks_without_gpu(lib):
    lib.ngf_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.ngf_version()
    from paper_1812_06765_amd.ngf import Params, E_ARG
    lib.ngf_create.argtypes = [ctypes.POINTER(Params), ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]
    lib.ngf_create.restype = ctypes.c_int32
    h = ctypes.c_void_p()
    good = dict(alpha=0.1, tau=1.0, rho=1.0, levels=3, ratio=2, max_iter=5, lbfgs_mem=5,
                tol_J=1e-6, early_stop=0, reserved=0)
    for key, bad in (("alpha", -1.0), ("tau", 0.0), ("rho", float("nan")), ("levels", 0),
                     ("levels", 13), ("ratio", 3), ("lbfgs_mem", 0), ("lbfgs_mem", 9),
                     ("max_iter", -1)):
        p = Params(**{**good, key: bad})
        assert lib.ngf_create(ctypes.byref(p), None, ctypes.byref(h)) == E_ARG, key
    assert lib.ngf_create(None, None, ctypes.byref(h)) == E_ARG
    p = Params(**good)
    assert lib.ngf_create(ctypes.byref(p), None, None) == E_ARG
    # batched form: worker count and null arguments are checked first
    lib.ngf_batch_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.ngf_batch_create.restype = ctypes.c_int32
    for w in (0, -1, 17):
        assert lib.ngf_batch_create(ctypes.byref(p), w, ctypes.byref(h)) == E_ARG, w
    assert lib.ngf_batch_create(None, 4, ctypes.byref(h)) == E_ARG
    assert lib.ngf_batch_create(ctypes.byref(p), 4, None) == E_ARG
    lib.ngf_batch_register.restype = ctypes.c_int32
    assert lib.ngf_batch_register(None, 0, None, None, None, None, None, None) == E_ARG
    lib.ngf_eval_J_grad_f64.restype = ctypes.c_int32
    assert lib.ngf_eval_J_grad_f64(None, 0, None, None, None, None) == E_ARG


def test_build_sources_and_flags():
    from paper_1812_06765_amd import build
    srcs = [os.path.basename(s) for s in build.sources()]
    assert {"k_eval.hip", "k_grid.hip", "k_lbfgs.hip", "ngf_api.hip"} <= set(srcs)
    assert "--offload-arch=gfx950" in build.CFLAGS
    i = build.CFLAGS.index("-target-feature")
    assert build.CFLAGS[i + 2] == "-packed-fp32-ops"


def _build_c_check(tmp_path):
    """Compile tests/c/ngf_c_check.c as C99 against the public header and
    link it with the library (no Python or torch on the caller's side)."""
    import subprocess
    pkg = os.path.join(ROOT, "paper_1812_06765_amd")
    exe = str(tmp_path / "ngf_c_check")
    rocm = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "c", "ngf_c_check.c"), f"-L{pkg}", "-lngfreg",
           f"-Wl,-rpath,{pkg}", f"-L{rocm}", "-lamdhip64", f"-Wl,-rpath,{rocm}", "-lm",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_caller_compiles_links_and_checks_arguments(tmp_path):
    import subprocess
    exe = _build_c_check(tmp_path)
    r = subprocess.run([exe, "cpu"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cpu checks ok" in r.stdout


def test_iteration_record_layout_and_jsonl(tmp_path):
    """The binding's record matches the header's 64-byte ngf_iter_record
    field by field, and the JSON-lines writer keeps every field."""
    import json

    from paper_1812_06765_amd.ngf import ITER_FIELDS, IterRecord, write_jsonl
    assert ctypes.sizeof(IterRecord) == 64
    offs = {name: getattr(IterRecord, name).offset for name, _ in IterRecord._fields_}
    assert offs == {"level": 0, "iter": 4, "evals": 8, "reserved": 12, "J": 16, "D": 24,
                    "S": 32, "gmax": 40, "t": 48, "us": 56}
    recs = [dict(level=1, iter=0, evals=1, J=3.5, D=3.0, S=5.0, gmax=0.25, t=0.0, us=0.0),
            dict(level=0, iter=7, evals=9, J=1.25, D=1.0, S=2.5, gmax=1e-3, t=0.5, us=12.5)]
    path = tmp_path / "log.jsonl"
    write_jsonl(recs, str(path))
    back = [json.loads(line) for line in open(path)]
    assert back == [{k: r[k] for k in ITER_FIELDS} for r in recs]


def test_aux_calls_check_arguments_without_gpu(lib):
    """Log and checkpoint calls reject a null context before any HIP call."""
    from paper_1812_06765_amd.ngf import E_ARG
    for name in ("ngf_set_iteration_log", "ngf_iteration_log", "ngf_lbfgs_state_size",
                 "ngf_lbfgs_save", "ngf_lbfgs_load"):
        getattr(lib, name).restype = ctypes.c_int32
    n = ctypes.c_int32()
    sz = ctypes.c_size_t()
    buf = ctypes.create_string_buffer(8)
    assert lib.ngf_set_iteration_log(None, 1) == E_ARG
    assert lib.ngf_iteration_log(None, None, 0, ctypes.byref(n)) == E_ARG
    assert lib.ngf_lbfgs_state_size(None, ctypes.byref(sz)) == E_ARG
    assert lib.ngf_lbfgs_save(None, buf, ctypes.c_size_t(8)) == E_ARG
    assert lib.ngf_lbfgs_load(None, buf, ctypes.c_size_t(8)) == E_ARG
