"""The C-ABI library builds, loads and exports every entry point declared in
include/atos.h.  These tests make no compute call, so they run without a GPU."""
import ctypes
import os
import re

import pytest

import paper_2112_00132_amd as atos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "atos.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(atos_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(atos.library_path()):
        from paper_2112_00132_amd import build
        build.build()
    return ctypes.CDLL(atos.library_path())


def test_header_declares_the_core_calls():
    names = _declared_functions()
    for required in ("atos_graph_load", "atos_graph_free", "atos_bfs", "atos_pagerank",
                     "atos_color", "atos_workspace_bytes", "atos_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_strerror_and_version(lib):
    lib.atos_strerror.restype = ctypes.c_char_p
    lib.atos_version.restype = ctypes.c_char_p
    assert lib.atos_strerror(0) == b"ok"
    assert lib.atos_strerror(3) == b"worklist ring overflow"
    assert lib.atos_strerror(12345) == b"unknown status"
    assert re.fullmatch(rb"\d+\.\d+\.\d+", lib.atos_version())


def test_null_handles_are_rejected_without_touching_the_gpu(lib):
    EINVAL = 1
    assert lib.atos_graph_free(None) == EINVAL
    assert lib.atos_graph_info(None, None, None, None) == EINVAL
    size = ctypes.c_size_t()
    assert lib.atos_workspace_bytes(None, 1, None, ctypes.byref(size)) == EINVAL
    assert lib.atos_bfs(None, ctypes.c_int64(0), None, None, ctypes.c_size_t(0), None, None,
                        None) == EINVAL
    assert lib.atos_workspace_stats(None, None, None) == EINVAL
    out = ctypes.c_void_p()
    # negative sizes and unknown flags are argument errors, caught before any HIP call
    assert lib.atos_graph_load(ctypes.c_void_p(16), 0, ctypes.c_void_p(16), ctypes.c_int64(-1),
                               ctypes.c_int64(0), 0, None, ctypes.byref(out)) == EINVAL
    assert lib.atos_graph_load(ctypes.c_void_p(16), 0, ctypes.c_void_p(16), ctypes.c_int64(4),
                               ctypes.c_int64(4), 0x80, None, ctypes.byref(out)) == EINVAL


def test_binding_raises_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(atos, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(atos, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        atos._load()


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of the ABI's structs have the C compiler's sizes and
    field offsets (a C program compiled against include/atos.h prints them)."""
    import subprocess
    structs = {
        "atos_config": atos._Config, "atos_stats": atos._Stats,
        "atos_batch_instance": atos._BatchInstance, "atos_tune_result": atos._TuneResult,
        "atos_server_config": atos._ServerConfig, "atos_query": atos._Query,
        "atos_completion": atos._Completion,
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "atos.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
