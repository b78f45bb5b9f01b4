"""The C ABI boundary, checked without a GPU: the library loads, exports
every entry point declared in include/adagio.h, its Python binding covers
them, and argument errors are reported before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adagio.h")
LIB = os.path.join(ROOT, "paper_1609_05388_amd", "libadagio.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adagio_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1609_05388_amd import build
        build.build()
    from paper_1609_05388_amd import adagio
    return adagio.load(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("adagio_fit", "adagio_embed", "adagio_max_distortion", "adagio_pca",
                     "adagio_project", "adagio_project_axes", "adagio_certify_map"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1609_05388_amd import adagio
    assert set(declared_functions()) == set(adagio.SIGNATURES)


def test_struct_layouts_match_header():
    """Field order and sizes of the ctypes mirrors follow the header."""
    from paper_1609_05388_amd import adagio
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cname, py in (("adagio_cert", adagio.Cert), ("adagio_stats", adagio.Stats),
                      ("adagio_opts", adagio.Opts), ("adagio_knn_stats", adagio.KnnStats)):
        body = re.search(r"typedef struct %s \{(.*?)\}" % cname, text, flags=re.S).group(1)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
            for nm in names.split(","):
                fields.append(re.sub(r"\[.*\]", "", nm).strip().lstrip("*"))
        assert fields == [f for f, _ in py._fields_], cname


def test_struct_offsets_match_c_compiler(tmp_path):
    """sizeof/offsetof of every field as gcc lays out the header's structs."""
    from paper_1609_05388_amd import adagio
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "adagio.h"', "int main(void) {"]
    for ctype, py in (("adagio_cert_t", adagio.Cert), ("adagio_stats_t", adagio.Stats),
                      ("adagio_opts_t", adagio.Opts), ("adagio_knn_stats_t", adagio.KnnStats)):
        lines.append('printf("%%zu\\n", sizeof(%s));' % ctype)
        for f, _ in py._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (ctype, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = []
    for py in (adagio.Cert, adagio.Stats, adagio.Opts, adagio.KnnStats):
        want.append(ctypes.sizeof(py))
        want.extend(getattr(py, f).offset for f, _ in py._fields_)
    assert got == want


def test_status_strings(lib):
    assert lib.adagio_status_string(0) == b"ok"
    assert lib.adagio_status_string(-1) == b"invalid argument"
    assert lib.adagio_status_string(-999) == b"unknown status"


def test_invalid_arguments_rejected_without_gpu(lib):
    """Validation runs before any HIP call (this container has no GPU)."""
    from paper_1609_05388_amd import adagio
    fake = ctypes.c_void_p(0x1000)
    r = ctypes.c_int32()
    s = ctypes.c_int32()
    c = adagio.Cert()
    # n < 2
    assert lib.adagio_fit(fake, 1, 8, 0.1, 1, None, fake, ctypes.byref(r), ctypes.byref(s), ctypes.byref(c), None) == -1
    assert b"n >= 2" in lib.adagio_last_error()
    # eps outside (0, 1)
    assert lib.adagio_fit(fake, 10, 8, 1.5, 1, None, fake, ctypes.byref(r), ctypes.byref(s), ctypes.byref(c), None) == -1
    assert lib.adagio_fit(fake, 10, 8, 0.0, 1, None, fake, ctypes.byref(r), ctypes.byref(s), ctypes.byref(c), None) == -1
    # NULL X
    assert lib.adagio_max_distortion(None, 10, 8, fake, 3, None, ctypes.byref(c), None) == -1
    # r outside [1, d]
    assert lib.adagio_project(fake, 10, 8, 9, 1, fake, None) == -1
    assert lib.adagio_project_axes(fake, 8, 0, 1, fake, None) == -1
    # d < 1
    assert lib.adagio_pca(fake, 10, 0, fake, fake, None) == -1
    # unsupported screen precision value
    o = adagio.Opts()
    o.screen = 7
    assert lib.adagio_certify_map(fake, 10, 8, fake, 3, ctypes.byref(o), ctypes.byref(c), None) == -1
    # kNN: k out of range, exclude_self with more queries than rows, NULL output
    ks = adagio.KnnStats()
    assert lib.adagio_knn(fake, 10, fake, 10, 4, 0, 0, fake, fake, ctypes.byref(ks), None) == -1
    assert lib.adagio_knn(fake, 10, fake, 10, 4, 33, 0, fake, fake, ctypes.byref(ks), None) == -1
    assert lib.adagio_knn(fake, 11, fake, 10, 4, 3, 1, fake, fake, ctypes.byref(ks), None) == -1
    assert lib.adagio_knn(fake, 10, fake, 10, 4, 3, 0, None, fake, ctypes.byref(ks), None) == -1
    assert lib.adagio_knn_vote(fake, 10, 3, fake, 10, 0, 5, fake, None) == -1
    assert lib.adagio_knn_vote(fake, 10, 3, fake, 10, 4, 0, fake, None) == -1
    # sizes beyond the launch geometry (one 256-thread workgroup per tile slot
    # of the screens, one work-item per element of n x d and d x d arrays, at
    # most 2^32 work-items per dispatch) are refused before any device work
    assert lib.adagio_fit(fake, 700001, 8, 0.1, 1, None, fake, ctypes.byref(r), ctypes.byref(s), ctypes.byref(c),
                          None) == -5
    assert b"700000" in lib.adagio_last_error()
    assert lib.adagio_max_distortion(fake, 10, 32769, fake, 3, None, ctypes.byref(c), None) == -5
    assert lib.adagio_certify_map(fake, 600000, 8192, fake, 3, None, ctypes.byref(c), None) == -5
    assert b"n x d" in lib.adagio_last_error()


def test_workspace_mode_argument(lib):
    """adagio_keep_workspace takes 0 or 1; other values are refused before any
    device work (keep = 0 with nothing kept touches no device)."""
    assert lib.adagio_keep_workspace(2) == -1
    assert b"keep must be 0 or 1" in lib.adagio_last_error()
    assert lib.adagio_keep_workspace(-1) == -1
    assert lib.adagio_keep_workspace(0) == 0


def test_mfma_ceiling_arguments(lib):
    """The MFMA ceiling measurement takes kinds 0-2 and host outputs; others
    are refused before any device work."""
    t, g = ctypes.c_double(), ctypes.c_double()
    assert lib.adagio_mfma_ceiling(3, ctypes.byref(t), ctypes.byref(g), None) == -1
    assert b"kind must be" in lib.adagio_last_error()
    assert lib.adagio_mfma_ceiling(-1, ctypes.byref(t), ctypes.byref(g), None) == -1
    assert lib.adagio_mfma_ceiling(0, None, ctypes.byref(g), None) == -1


def test_noalloc_certificate_refuses_before_device_work(lib):
    """The no-allocation certificate refuses inputs beyond its fixed scratch
    array, and screens other than FP32, on the host."""
    from paper_1609_05388_amd import adagio
    fake = ctypes.c_void_p(0x1000)
    c = adagio.Cert()
    assert lib.adagio_max_distortion_noalloc(fake, 20000, 784, fake, 256, None, ctypes.byref(c), None) == -5
    assert b"64 MiB" in lib.adagio_last_error()
    o = adagio.Opts()
    o.screen = 1
    assert lib.adagio_max_distortion_noalloc(fake, 100, 8, fake, 3, ctypes.byref(o), ctypes.byref(c), None) == -5
    assert b"FP32 screen only" in lib.adagio_last_error()
    assert lib.adagio_max_distortion_noalloc(fake, 100, 8, None, 3, None, ctypes.byref(c), None) == -1
