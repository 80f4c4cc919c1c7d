"""The C ABI library loads on the CPU host and exports every symbol that the
public headers declare (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_18966_amd", "libsvds.so")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("svds.h", "svds_ops.h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:int|void|const char \*)\s*(svds_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsvds.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_headers_declare_the_boundary():
    names = _declared()
    for must in ["svds_plan_create_csr", "svds_plan_create_dense", "svds_plan_execute",
                 "svds_plan_destroy", "svds_csr_solve", "svds_dense_solve", "svds_csr_solve_batched",
                 "svds_residuals_csr", "svds_strerror", "svds_op_spmv_csr", "svds_op_csc_build",
                 "svds_op_cgs2", "svds_op_small_svd", "svds_op_rotate", "svds_op_philox_normal",
                 "svds_op_csr_matvec"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_version_need_no_gpu(lib):
    lib.svds_strerror.restype = ctypes.c_char_p
    lib.svds_version.restype = ctypes.c_char_p
    assert b"invalid" in lib.svds_strerror(-1)
    assert b"gfx950" in lib.svds_version()


def test_validation_rejects_bad_sizes_before_touching_the_device(lib):
    """k/p validation is host logic: EINVAL without any device call."""
    from paper_2405_18966_amd.svds import svds_csr, svds_opts  # noqa: F401  (struct layout)
    import importlib
    mod = importlib.import_module("paper_2405_18966_amd.svds")
    fake = 4096  # never dereferenced: validation fails first
    A = mod.svds_csr(10, 5, 0, fake, fake, fake, 0)
    h = ctypes.c_void_p()
    for k, p in [(0, 3), (3, 3), (2, 5), (2, 11)]:
        o = mod.svds_opts(k, p, 0.0, 0, 0, 0, None, None, 0)
        assert mod.lib.svds_plan_create_csr(ctypes.byref(A), ctypes.byref(o), ctypes.byref(h)) == -1
    o = mod.svds_opts(2, 4, 0.0, 0, 7, 0, None, None, 0)  # unknown precision
    assert mod.lib.svds_plan_create_csr(ctypes.byref(A), ctypes.byref(o), ctypes.byref(h)) == -1


def test_smallest_triplets_unsupported_forms_rejected_on_the_host(lib):
    """SVDS_FLAG_SMALLEST is FP64-only: mixed precision and the batched solver
    return EUNSUPPORTED before any device call; so does the batched solver for
    SVDS_FLAG_SELECTIVE_REORTH."""
    import importlib
    mod = importlib.import_module("paper_2405_18966_amd.svds")
    fake = 4096  # never dereferenced
    A = mod.svds_csr(100, 50, 0, fake, fake, fake, 0)
    h = ctypes.c_void_p()
    o = mod.svds_opts(2, 6, 0.0, 0, mod.SVDS_PREC_MIXED, 0, None, None, mod.SVDS_FLAG_SMALLEST)
    assert mod.lib.svds_plan_create_csr(ctypes.byref(A), ctypes.byref(o), ctypes.byref(h)) == -4
    outs = (ctypes.c_void_p * 1)(fake)
    info = mod.svds_info()
    for flag in (mod.SVDS_FLAG_SMALLEST, mod.SVDS_FLAG_SELECTIVE_REORTH):
        o = mod.svds_opts(2, 6, 0.0, 0, mod.SVDS_PREC_FP64, 0, None, None, flag)
        assert mod.lib.svds_csr_solve_batched(1, ctypes.byref(A), ctypes.byref(o), outs, outs, outs,
                                              ctypes.byref(info)) == -4


def test_ctypes_structs_match_the_c_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets that a
    C compiler gives the header's structs (a field added on one side only
    would shift every later field)."""
    import shutil
    import subprocess
    mod = __import__("paper_2405_18966_amd.svds", fromlist=["x"])
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"svds_csr": mod.svds_csr, "svds_dense": mod.svds_dense, "svds_opts": mod.svds_opts,
               "svds_info": mod.svds_info, "svds_tuning": mod.svds_tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "svds.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.split("\n") if l)
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def test_binding_constants_match_the_header():
    """Every SVDS_FLAG_*, SVDS_PREC_* and dtype value the binding defines is
    the one include/svds.h gives it, and every flag of the header is bound."""
    import paper_2405_18966_amd.svds as mod
    text = re.sub(r"/\*.*?\*/", "", open(HEADERS[0]).read(), flags=re.S)
    header = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(SVDS_(?:FLAG|PREC)_\w+)\s*=\s*(\d+)", text)}
    flags = [n for n in header if n.startswith("SVDS_FLAG_")]
    assert len(flags) >= 14
    for name, value in header.items():
        assert hasattr(mod, name), name
        assert getattr(mod, name) == value, (name, getattr(mod, name), value)
