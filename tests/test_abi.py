"""The C-ABI library loads and exports every entry point include/rmb.h
declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmb.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for name in ("rmb_ctx_create", "rmb_mobility_matvec"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (one HIP runtime for torch and the library)
    import paper_1602_02170_amd as rmb
    if not os.path.exists(rmb.LIB_PATH):
        pytest.fail("librmb.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(rmb.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(rmb.EXPORTS) == declared_symbols()
    lib.rmb_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rmb_version()


def test_binding_refuses_to_run_without_library(tmp_path):
    import paper_1602_02170_amd as rmb
    old = rmb._LIB
    rmb._LIB = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            rmb.library(str(tmp_path / "missing.so"))
    finally:
        rmb._LIB = old


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program compiled against include/rmb.h prints them)."""
    import subprocess
    import paper_1602_02170_amd as rmb
    structs = {"rmb_system": rmb.rmb_system, "rmb_shapes": rmb.rmb_shapes, "rmb_solve_opts": rmb.rmb_solve_opts,
               "rmb_solve_info": rmb.rmb_solve_info, "rmb_tune_record": rmb.rmb_tune_record}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rmb.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for line in out:
        if line:
            n, f, v = line.split()
            got[(n, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_server_refuses_a_tag_already_in_flight():
    """A tag reused before its request is polled would drop the only
    references to the first request's output tensors while the library still
    writes them; the binding refuses it before calling into the library."""
    import paper_1602_02170_amd as rmb

    class NoLib:
        def __getattr__(self, name):
            raise AssertionError(f"{name} must not be called")

    class Ctx:
        lib = NoLib()
        h = None

    srv = rmb.Server.__new__(rmb.Server)
    srv.ctx, srv.h, srv.stream = Ctx(), None, None
    srv.live = {7: ("request 7",)}
    with pytest.raises(ValueError, match="already in flight"):
        srv.submit(7, None, None)
    assert srv.live == {7: ("request 7",)}


def test_tile_shapes_are_described():
    import paper_1602_02170_amd as rmb
    shapes = rmb.tile_shapes()
    assert len(shapes) >= 1
    for s in shapes:
        assert s["panel"] in (16, 32, 64, 128) and s["row_tiles"] >= 1 and s["chunk"] >= 4
    p = ctypes.c_int32()
    assert rmb.library().rmb_tile_shape_info(len(shapes), ctypes.byref(p), ctypes.byref(p),
                                             ctypes.byref(p)) == rmb.RMB_EINVAL
