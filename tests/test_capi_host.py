"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/slepian.h declares, and rejects bad arguments before
touching a device."""

import ctypes as C
import os
import re

import pytest

from paper_1611_04950_amd import slepian as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "slepian.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slepian_[a-z0-9_]+)\s*\(", text)))


def test_header_functions_are_exported():
    names = _declared_functions()
    assert len(names) >= 17
    lib = C.CDLL(S.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(S.EXPORTED) == names


def test_status_strings():
    for st in range(-8, 1):
        assert S.slepian_status_string(st) != "unknown status"
    assert S.slepian_status_string(-99) == "unknown status"


@pytest.mark.parametrize("N,W,eps,code", [
    (1, 0.1, 1e-6, S.SLEPIAN_EINVAL),
    (100, 0.0, 1e-6, S.SLEPIAN_EINVAL),
    (100, 0.5, 1e-6, S.SLEPIAN_EINVAL),
    (100, 0.1, 0.0, S.SLEPIAN_EINVAL),
    (100, 0.1, 0.5, S.SLEPIAN_EINVAL),
    (100, float("nan"), 1e-6, S.SLEPIAN_EINVAL),
    (1 << 22, 0.1, 1e-6, S.SLEPIAN_ENOTSUP),
])
def test_plan_domain_checked_before_any_device_work(N, W, eps, code):
    h = C.c_void_p()
    assert S._lib.slepian_plan(N, W, eps, C.byref(h)) == code
    assert h.value is None


def test_plan_options_checked():
    h = C.c_void_p()
    for opts in (S.PlanOpts(-1.0, 0, 0, -1), S.PlanOpts(0.0, 100, 0, -1), S.PlanOpts(0.0, -2, 0, -1),
                 S.PlanOpts(0.0, 0, 7, -1)):
        assert S._lib.slepian_plan_ex(100, 0.1, 1e-6, C.byref(opts), C.byref(h)) == S.SLEPIAN_EINVAL


def test_plan_batch_checked_before_any_device_work():
    """A bad triple anywhere in the batch fails the whole call before any
    device work, and no handle is written."""
    n = 3
    Ns = (C.c_int64 * n)(100, 200, 1)
    Ws = (C.c_double * n)(0.1, 0.1, 0.1)
    Es = (C.c_double * n)(1e-6, 1e-6, 1e-6)
    hs = (C.c_void_p * n)()
    assert S._lib.slepian_plan_batch(n, Ns, Ws, Es, None, hs) == S.SLEPIAN_EINVAL
    assert all(h is None for h in hs)
    assert S._lib.slepian_plan_batch(-1, Ns, Ws, Es, None, hs) == S.SLEPIAN_EINVAL
    assert S._lib.slepian_plan_batch(0, None, None, None, None, None) == S.SLEPIAN_OK


def test_null_handles():
    lib = S._lib
    assert lib.slepian_plan_destroy(None) == S.SLEPIAN_OK
    assert lib.slepian_group_destroy(None) == S.SLEPIAN_OK
    n = C.c_size_t()
    assert lib.slepian_workspace_size(None, 0, 4, C.byref(n)) == S.SLEPIAN_EINVAL
    assert lib.slepian_project(None, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_lsq(None, 0, 0.0, None, 0, None, 0, 1, 0.0, 0, None, 0, None, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_coeffs(None, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_plan_info_get(None, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_plan_save(None, b"/tmp/x") == S.SLEPIAN_EINVAL
    h = C.c_void_p()
    assert lib.slepian_plan_load(b"/nonexistent/plan.bin", -1, C.byref(h)) == S.SLEPIAN_EIO
    assert lib.slepian_group_create(None, 0, None, C.byref(h)) == S.SLEPIAN_EINVAL
    # multiband entry points: no plan, no band set
    f = (C.c_double * 2)(0.0, 0.25)
    assert lib.slepian_project_multiband(None, 2, f, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_bands_create(None, 2, f, C.byref(h)) == S.SLEPIAN_EINVAL
    assert h.value is None
    assert lib.slepian_bands_create(None, 2, f, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_bands_destroy(None) == S.SLEPIAN_OK
    assert lib.slepian_bands_workspace_size(None, 4, C.byref(n)) == S.SLEPIAN_EINVAL
    assert lib.slepian_project_bands(None, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL
    # fast factorization: no plan, no factorization
    h = C.c_void_p()
    assert lib.slepian_factor_create(None, C.byref(h)) == S.SLEPIAN_EINVAL
    assert h.value is None
    assert lib.slepian_factor_create(None, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_destroy(None) == S.SLEPIAN_OK
    assert lib.slepian_factor_info(None, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_mu(None, None, 0) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_workspace_size(None, 4, C.byref(n)) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_compress(None, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL
    assert lib.slepian_factor_recover(None, None, 0, None, 0, 1, None, 0, None) == S.SLEPIAN_EINVAL


def test_plan_load_rejects_garbage(tmp_path):
    p = tmp_path / "bad.plan"
    p.write_bytes(b"not a plan file at all" * 10)
    h = C.c_void_p()
    assert S._lib.slepian_plan_load(str(p).encode(), -1, C.byref(h)) == S.SLEPIAN_EIO


def test_synth_is_seeded_and_float32():
    from paper_1611_04950_amd import synth
    a = synth.config_signals(2, 512, 3, 0.125)
    b = synth.config_signals(2, 512, 3, 0.125)
    assert a.dtype.is_floating_point and a.dtype.itemsize == 4
    assert a.shape == (3, 512)
    assert (a == b).all()
    c = synth.config_signals(1, 100, 2, 0.1)
    assert abs(float(c.double().std()) - 1.0) < 0.2


def test_header_is_plain_c():
    """include/slepian.h is a C header (the boundary takes no C++ or torch
    types): it compiles as C99 and as C++ with warnings as errors."""
    import shutil
    import subprocess
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "slepian.h")
    for cc, args in (("gcc", ["-std=c99", "-x", "c"]), ("g++", ["-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, "-fsyntax-only", "-Wall", "-Wextra", "-Werror", *args, hdr], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    """The library's host code (argument checks, plan-file parser) built with
    AddressSanitizer and UndefinedBehaviorSanitizer (host pass only) and
    driven by tests/host_sanitize_main.c: null and out-of-domain arguments on
    every entry point, and malformed plan files.  No GPU is needed: the
    checks run before any device work."""
    import shutil
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang) and shutil.which("gcc")):
        pytest.skip("ROCm compilers not available")
    from paper_1611_04950_amd import build as B
    objdir = os.path.join(root, "_build")
    plain = [os.path.join(objdir, os.path.splitext(f)[0] + ".o") for f in B.SOURCES
             if f not in ("capi.cpp", "trace.cpp")]
    if not all(os.path.exists(o) for o in plain):
        B.build()
    out = tmp_path
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", f"-I{os.path.join(root, 'include')}", f"-I{B.CSRC}", "-Wno-unused-result",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in ("capi.cpp", "trace.cpp"):
        o = str(out / (src + ".o"))
        r = subprocess.run([hipcc, *flags, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o", o],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(o)
    main_o = str(out / "main.o")
    r = subprocess.run(["gcc", "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        f"-I{os.path.join(root, 'include')}", "-c", os.path.join(root, "tests", "host_sanitize_main.c"),
                        "-o", main_o], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    exe = str(out / "host_check")
    r = subprocess.run([clang, "-fsanitize=address,undefined", main_o, *objs, *plain, "-L/opt/rocm/lib",
                        "-lamdhip64", "-lhipblaslt", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(out)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
