"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C certificate (oracle/certificate.c, OpenMP) built with gcc's
  sanitizers and run by tests/sanitize/oracle_driver.c on small clouds with
  the certificate's edge cases, each result against a brute force.
* The library's host side: csrc/api.hip compiled with the sanitizers on its
  host pass only (-Xarch_host before each -fsanitize=; the device code is
  unchanged), linked with the other objects into a separate shared library,
  loaded in a child interpreter with clang's ASan runtime preloaded, and
  driven through every host-only path this container can reach without a
  GPU: argument validation of every entry point, the size limits, the
  no-allocation entry point's scratch check, the workspace-mode switch,
  status strings and the thread-local error text.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow


def _clean(env=None):
    e = dict(os.environ)
    e.update(env or {})
    return e


def test_oracle_certificate_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_driver"
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fopenmp", os.path.join(ROOT, "oracle", "certificate.c"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", str(exe), "-lm"])
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120,
                         env=_clean({"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"}))
    assert res.returncode == 0, res.stderr
    assert "ERROR" not in res.stderr and "runtime error" not in res.stderr, res.stderr
    assert "all checks passed" in res.stdout


_HOST_CHECK = r'''
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_1609_05388_amd import adagio
lib = ctypes.CDLL(LIB)
for name, (res, args) in adagio.SIGNATURES.items():
    fn = getattr(lib, name)
    fn.restype = res
    fn.argtypes = args
fake = ctypes.c_void_p(0x1000)
r, s, c = ctypes.c_int32(), ctypes.c_int32(), adagio.Cert()
ks = adagio.KnnStats()
R, S, C = ctypes.byref(r), ctypes.byref(s), ctypes.byref(c)
checks = [
    (lambda: lib.adagio_fit(fake, 1, 8, 0.1, 1, None, fake, R, S, C, None), -1, b"n >= 2"),
    (lambda: lib.adagio_fit(fake, 10, 8, 1.5, 1, None, fake, R, S, C, None), -1, b"eps"),
    (lambda: lib.adagio_fit(fake, 10, 8, 0.1, 1, None, None, R, S, C, None), -1, b"NULL"),
    (lambda: lib.adagio_fit(fake, 700001, 8, 0.1, 1, None, fake, R, S, C, None), -5, b"700000"),
    (lambda: lib.adagio_certify_map(fake, 600000, 8192, fake, 3, None, C, None), -5, b"n x d"),
    (lambda: lib.adagio_max_distortion(None, 10, 8, fake, 3, None, C, None), -1, b"NULL"),
    (lambda: lib.adagio_max_distortion(fake, 10, 32769, fake, 3, None, C, None), -5, b"32768"),
    (lambda: lib.adagio_max_distortion_noalloc(fake, 20000, 784, fake, 256, None, C, None), -5, b"64 MiB"),
    (lambda: lib.adagio_project(fake, 10, 8, 9, 1, fake, None), -1, b"r must be"),
    (lambda: lib.adagio_project_axes(fake, 8, 0, 1, fake, None), -1, b"r must be"),
    (lambda: lib.adagio_project_family(fake, 8, 3, 9, 1, fake, None), -1, b"family"),
    (lambda: lib.adagio_pca(fake, 10, 0, fake, fake, None), -1, b"d >= 1"),
    (lambda: lib.adagio_pca_randomized(fake, 10, 8, 9, 1, 1, fake, fake, None), -1, b"ell"),
    (lambda: lib.adagio_knn(fake, 10, fake, 10, 4, 33, 0, fake, fake, ctypes.byref(ks), None), -1, b"k must be"),
    (lambda: lib.adagio_knn_vote(fake, 10, 3, fake, 10, 0, 5, fake, None), -1, b"n_labels"),
    (lambda: lib.adagio_mlp_forward(fake, fake, 0, fake, None), -1, b"batch"),
    (lambda: lib.adagio_mlp_grad(fake, fake, fake, 4, 1.5, fake, fake, None), -1, b"tau"),
    (lambda: lib.adagio_mlp_train_step(fake, fake, fake, 0, 0.1, fake, fake, 4, 0.5, fake, None), -1, b"step"),
    (lambda: lib.adagio_keep_workspace(2), -1, b"keep must be"),
    (lambda: lib.adagio_keep_workspace(0), 0, b""),
]
o1, o2 = adagio.Opts(), adagio.Opts()
o1.screen = 7
o2.refine = 3
checks.append((lambda: lib.adagio_certify_map(fake, 10, 8, fake, 3, ctypes.byref(o1), C, None), -1, b"screen"))
checks.append((lambda: lib.adagio_fit(fake, 10, 8, 0.1, 1, ctypes.byref(o2), fake, R, S, C, None), -1, b"refine"))
for call, want, text in checks:
    got = call()
    err = lib.adagio_last_error()
    assert got == want and text in err, (got, want, text, err)
for code in range(-9, 1):
    assert lib.adagio_status_string(code)
assert lib.adagio_mlp_param_count() > 0
print("host paths ok:", len(checks))
'''


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1609_05388_amd import build
    build.build()
    asan_rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    assert asan_rt, "clang's ASan runtime not found"
    csrc = os.path.join(ROOT, "paper_1609_05388_amd", "csrc")
    obj = tmp_path / "api_asan.o"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc] + san +
                          ["-c", os.path.join(csrc, "api.hip"), "-o", str(obj)],
                          stderr=subprocess.DEVNULL)
    others = [o for o in sorted(glob.glob(os.path.join(build.OBJ, "*.o"))) if not o.endswith("api.hip.o")]
    lib = tmp_path / "libadagio_asan.so"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + san[:4] +
                          ["-Xarch_host", "-shared-libasan", "-o", str(lib), str(obj)] + others)
    code = "ROOT = %r\nLIB = %r\n" % (ROOT, str(lib)) + _HOST_CHECK
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         env=_clean({"LD_PRELOAD": asan_rt[-1], "ASAN_OPTIONS": "detect_leaks=0"}))
    assert res.returncode == 0, res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    assert "host paths ok" in res.stdout
