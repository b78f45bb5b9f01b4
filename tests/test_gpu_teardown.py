"""Process exit with the library loaded through ctypes alone (no Python
binding, so no help from it at exit).

Each case runs in a fresh child interpreter that loads libadagio.so with
ctypes.CDLL, runs one small adagio_fit and exits; the child must end with
status 0 and write nothing to stderr (the one line libdrm prints when its
GPU name table is missing on the host is dropped first: it comes from the
driver stack at start-up, not from the library).

* default workspace (freed before the call returns), device memory from torch
  (imported first, so that the library binds to the HIP runtime torch
  loaded: a process must not hold two HIP runtimes);
* kept workspace (adagio_keep_workspace(1)) left allocated at exit, device
  memory from the HIP runtime through ctypes, no torch in the process: the
  library's own exit handler frees the workspace, its streams and events;
* two fits with per-call workspaces, no torch: the device's library streams
  that both fits used are still held at exit, and the exit handler destroys
  them.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1609_05388_amd", "libadagio.so")

_COMMON = r'''
import ctypes, sys
import numpy as np
if USE_TORCH:
    import torch
sys.path.insert(0, ROOT)
from paper_1609_05388_amd import gen
lib = ctypes.CDLL(LIB)
P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
lib.adagio_fit.restype = ctypes.c_int
lib.adagio_fit.argtypes = [P, I64, I64, ctypes.c_double, ctypes.c_uint64, P, P, P, P, P, P]
lib.adagio_keep_workspace.restype = ctypes.c_int
lib.adagio_keep_workspace.argtypes = [ctypes.c_int]
lib.adagio_last_error.restype = ctypes.c_char_p
cert = (ctypes.c_char * 512)()        # adagio_cert_t is far smaller
X = gen.low_rank_pixels(n=600, d=64, rank=6, seed=5)
n, d = X.shape
r = I32(); s = I32()
'''

_TORCH_DEFAULT = _COMMON + r'''
Xd = torch.from_numpy(X).cuda()
Pi = torch.empty((d, d), dtype=torch.float32, device="cuda")
rc = lib.adagio_fit(Xd.data_ptr(), n, d, 0.1, 5388, None, Pi.data_ptr(), ctypes.byref(r), ctypes.byref(s),
                    cert, None)
torch.cuda.synchronize()
print("rc", rc, "r", r.value, lib.adagio_last_error().decode(), flush=True)
sys.exit(0 if rc == 0 else 3)
'''

_HIP_KEEP = _COMMON + r'''
hip = ctypes.CDLL("libamdhip64.so.7")   # the runtime the library links
hip.hipMalloc.argtypes = [ctypes.POINTER(P), ctypes.c_size_t]
hip.hipMemcpy.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int]
hip.hipDeviceSynchronize.argtypes = []
xd, pd = P(), P()
assert hip.hipMalloc(ctypes.byref(xd), X.nbytes) == 0
assert hip.hipMalloc(ctypes.byref(pd), d * d * 4) == 0
assert hip.hipMemcpy(xd, X.ctypes.data, X.nbytes, 1) == 0      # host to device
assert lib.adagio_keep_workspace(1) == 0
rc = lib.adagio_fit(xd, n, d, 0.1, 5388, None, pd, ctypes.byref(r), ctypes.byref(s), cert, None)
rc2 = lib.adagio_fit(xd, n, d, 0.1, 5388, None, pd, ctypes.byref(r), ctypes.byref(s), cert, None)
assert hip.hipDeviceSynchronize() == 0
print("rc", rc, rc2, "r", r.value, lib.adagio_last_error().decode(), flush=True)
sys.exit(0 if rc == 0 and rc2 == 0 else 3)
'''


_HIP_PER_CALL = _HIP_KEEP.replace("assert lib.adagio_keep_workspace(1) == 0\n", "")


def _run_child(body, use_torch):
    code = "ROOT = %r\nLIB = %r\nUSE_TORCH = %r\n" % (ROOT, LIB, use_torch) + body
    print("child interpreter: adagio_fit through ctypes, then exit", flush=True)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    err = "\n".join(l for l in res.stderr.splitlines() if "amdgpu.ids" not in l).strip()
    return res, err


def test_exit_after_fit_with_per_call_workspace():
    res, err = _run_child(_TORCH_DEFAULT, True)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    assert err == "", res.stderr
    assert "rc 0" in res.stdout


def test_exit_with_kept_workspace_and_no_torch():
    res, err = _run_child(_HIP_KEEP, False)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    assert err == "", res.stderr
    assert "rc 0 0" in res.stdout


def test_exit_after_per_call_fits_and_no_torch():
    assert "adagio_keep_workspace(1)" not in _HIP_PER_CALL
    res, err = _run_child(_HIP_PER_CALL, False)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    assert err == "", res.stderr
    assert "rc 0 0" in res.stdout
