"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/viecut.h, and its host-only entry points behave."""
import ctypes
import os
import re

import pytest

import paper_1708_06127_amd as vc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "viecut.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(viecut_[a-z_0-9]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_library_exports_every_declared_function():
    lib = vc.load()
    names = declared_functions()
    assert "viecut_mincut" in names and "viecut_mincut_batch" in names and "viecut_session_step" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(vc.EXPORTED) == names


def test_default_params():
    p = vc.params()
    assert (p.lp_iters, p.n0, p.max_rounds, p.flags, p.seed) == (2, 10000, 64, 0, 0)


def test_strerror():
    assert vc.strerror(0) == "ok"
    for code in range(-8, 0):
        assert vc.strerror(code) and vc.strerror(code) != "unknown error"
    assert vc.strerror(-99) == "unknown error"


def test_workspace_bytes():
    assert vc.workspace_bytes(1, 0) == 0
    a = vc.workspace_bytes(1000, 32000)
    b = vc.workspace_bytes(2000, 64000)
    assert 0 < a < b
    # the 2^20-vertex, 33.6 M-arc workload fits easily in 288 GB
    assert vc.workspace_bytes(1 << 20, 33_635_268) < 8 * 2**30


def test_invalid_arguments_rejected_on_host():
    lib = vc.load()
    res = vc.Result()
    g = vc.Csr()
    g.n, g.nnz = 1, 0
    p = vc.params()
    assert lib.viecut_mincut(ctypes.byref(g), ctypes.byref(p), None, 0, None, ctypes.byref(res), None) == vc.EINVAL
    g.n = 5
    p.lp_iters = -1
    assert lib.viecut_mincut(ctypes.byref(g), ctypes.byref(p), None, 0, None, ctypes.byref(res), None) == vc.EINVAL


def test_vertex_limit_rejected_on_host():
    """More than 2^30 vertices (label gathers use 32-bit byte offsets) is
    refused with EOVERFLOW by the host checks, before any device call: the
    pointers here are never dereferenced, and no GPU is needed."""
    lib = vc.load()
    res = vc.Result()
    p = vc.params()
    g = vc.Csr()
    g.n, g.nnz = (1 << 30) + 1, 0
    g.row_ptr = ctypes.c_void_p(0x1000)
    side = ctypes.c_void_p(0x2000)
    assert lib.viecut_mincut(ctypes.byref(g), ctypes.byref(p), None, 0, None, ctypes.byref(res), side) == \
        vc.EOVERFLOW
    assert lib.viecut_validate(ctypes.byref(g), 0, None) == vc.EOVERFLOW
    assert vc.workspace_bytes((1 << 30) + 1, 0) == 0
    # a batch whose graphs together exceed the limit: the union is refused
    gs = (vc.Csr * 3)()
    for i in range(3):
        gs[i].n, gs[i].nnz, gs[i].row_ptr = (1 << 29) - 4, 0, ctypes.c_void_p(0x1000)
    outs = (vc.Result * 3)()
    sides = (ctypes.c_void_p * 3)(0x2000, 0x2000, 0x2000)
    assert lib.viecut_batch_workspace_bytes(gs, 3, ctypes.byref(p)) == 0
    assert lib.viecut_mincut_batch(gs, 3, ctypes.byref(p), None, 0, None, outs, sides) == vc.EOVERFLOW


def test_noalloc_rejects_graphs_beyond_the_scratch_on_host():
    """viecut_mincut_noalloc refuses, before any device call, a graph whose
    workspace exceeds the static scratch (ETOOBIG), and takes the same host
    argument checks as viecut_mincut."""
    lib = vc.load()
    res = vc.Result()
    p = vc.params()
    g = vc.Csr()
    g.row_ptr, g.col, g.w = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000)
    side = ctypes.c_void_p(0x2000)
    g.n, g.nnz = 1 << 20, 1 << 22
    assert vc.workspace_bytes(g.n, g.nnz) > vc.NOALLOC_SCRATCH_BYTES
    assert lib.viecut_mincut_noalloc(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(res), side) == vc.ETOOBIG
    g.n = 1
    assert lib.viecut_mincut_noalloc(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(res), side) == vc.EINVAL
    g.n, g.nnz = 8192, 8192 * 64
    assert vc.workspace_bytes(g.n, g.nnz) <= vc.NOALLOC_SCRATCH_BYTES  # the largest planted batch member fits
    assert lib.viecut_mincut_noalloc(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(res), None) == vc.EINVAL


def test_tuning_table_on_host(tmp_path):
    """The launch-shape table: keys and ranges checked, buckets kept in
    order, the file format read back (no GPU: only host state)."""
    vc.tuning_clear()
    assert "bucket -1" in vc.tuning_get()
    vc.tuning_set(1 << 26, "long_split", 384)
    vc.tuning_set(-1, "radix_large_from", 1 << 24)
    vc.tuning_set(1 << 20, "emit_wave", 0)
    text = vc.tuning_get()
    lines = [l for l in text.splitlines() if l.startswith("bucket")]
    assert [int(l.split()[1]) for l in lines] == [1 << 20, 1 << 26, -1]
    assert "long_split=384" in lines[1] and "radix_large_from=16777216" in lines[2] and "emit_wave=0" in lines[0]
    for key, bad in [("long_split", 800), ("long_split", 100), ("emit_wave", 2), ("lp_group", 0), ("lp_group", 5),
                     ("emit_group", 0), ("emit_group", 3), ("first_group", 0), ("huge_part", 2),
                     ("nonsense", 1)]:
        with pytest.raises(vc.ViecutError):
            vc.tuning_set(-1, key, bad)
    vc.tuning_clear()
    assert "long_split=512" in vc.tuning_get()


def test_tuning_file_read_at_load(tmp_path):
    """A fresh process reads the table from the file VIECUT_TUNING names."""
    import os
    import subprocess
    import sys
    f = tmp_path / "t.txt"
    f.write_text("# tuned\nbucket 1000000 long_split=320 emit_wave=0\nbucket -1 radix_large_from=123\n"
                 "bucket 5 long_split=9999\n")  # out of range: ignored
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = "import paper_1708_06127_amd as vc; print(vc.tuning_get())"
    p = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, VIECUT_TUNING=str(f)))
    assert p.returncode == 0, p.stderr
    lines = [l for l in p.stdout.splitlines() if l.startswith("bucket")]
    assert lines[0].startswith("bucket 5 ") and "long_split=512" in lines[0]
    assert lines[1].startswith("bucket 1000000 ") and "long_split=320" in lines[1] and "emit_wave=0" in lines[1]
    assert lines[2].startswith("bucket -1 ") and "radix_large_from=123" in lines[2]
    assert str(f) in p.stdout
