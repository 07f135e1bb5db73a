"""CPU checks of the boundary: the HIP library loads and exports every
function include/lsr.h declares; host-side validation works without a GPU;
the product package never reaches the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1801_01572_amd")


def _declared():
    src = open(os.path.join(ROOT, "include", "lsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsr_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("lsr_register_pair", "lsr_register_batch", "lsr_align_loss", "lsr_align_loss_backward",
                 "lsr_create", "lsr_destroy", "lsr_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(PKG, "liblsr.so")
    if not os.path.exists(path):
        from paper_1801_01572_amd.build import build
        build()
    lib = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(lib, name), name


def test_defaults_and_create_without_device():
    import paper_1801_01572_amd as L
    p = L.default_params()
    assert abs(p.r_feature - 0.05) < 1e-8 and abs(p.tau - 0.9) < 1e-7 and p.precision == L.FP32
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert L.lib().lsr_create(ctypes.byref(h), 0, 0) != 0       # no device: an error code, not a crash


def test_product_path_does_not_use_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt and "from oracle" not in txt, f


def test_oracle_library_builds():
    from oracle.build import build
    assert os.path.exists(build())


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of lsr_cloud, lsr_params, lsr_result and lsr_tune have
    the header's sizes and field offsets (a mismatch would shift every field
    the binding reads back)."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    from paper_1801_01572_amd import _lib
    pairs = [("lsr_cloud", _lib.Cloud), ("lsr_params", _lib.Params), ("lsr_result", _lib.Result),
             ("lsr_tune", _lib.Tune), ("lsr_trace", _lib.Trace), ("lsr_ransac_result", _lib.RansacResult),
             ("lsr_ransac_trace", _lib.RansacTrace), ("lsr_camera", _lib.Camera),
             ("lsr_edge", _lib.Edge), ("lsr_loop_params", _lib.LoopParams), ("lsr_loop_result", _lib.LoopResult)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lsr.h"', "int main(void) {"]
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:   # a trailing underscore marks a C name that is a Python keyword
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname.rstrip("_")}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run([gcc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
