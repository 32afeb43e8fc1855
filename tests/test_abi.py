"""The C-ABI library loads and exports every function include/bh.h declares
(no GPU work: only symbol lookup), and the binding knows each of them."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bh.h")
LIB = os.path.join(ROOT, "paper_1907_02289_amd", "libbh.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bh_status|const char \*)\s*(bh_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("bh_build_tree", "bh_make_lists", "bh_forces", "bh_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1907_02289_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_lists_every_symbol():
    from paper_1907_02289_amd import bh
    assert sorted(bh.SYMBOLS) == declared()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_binding_rejects_tensors_the_library_cannot_take():
    """The binding hands the library only contiguous CUDA float64 tensors of
    the expected length; anything else raises before a pointer is passed."""
    import torch
    from paper_1907_02289_amd import bh
    assert bh._ptr(None) is None
    for t in (torch.zeros(4, dtype=torch.float64), torch.zeros(4, dtype=torch.float32), [0.0] * 4):
        with pytest.raises(TypeError):
            bh._ptr(t, 4, "x")


def test_bench_uses_the_papers_printed_values():
    """The benchmark's paper-convention flop count and its collision
    restitution are the values the paper prints (tests/golden)."""
    import inspect

    import bench
    from golden import paper_values
    pv = paper_values()
    assert bench.PAPER_FLOPS_PER_INTERACTION == pv["flops_particle_cell"]
    assert inspect.signature(bench.collision_params).parameters["restitution"].default == pv["restitution_radial"]


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without the built library the binding raises: there is no other
    implementation to fall back on."""
    from paper_1907_02289_amd import bh
    monkeypatch.setattr(bh, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        bh.load_library(str(tmp_path / "libbh.so"))


def test_bench_percentile_is_nearest_rank():
    """p99 by nearest rank: of 100 values the 99th smallest, of 4096 the
    4056th (ceil(0.99 * 4096) = 4056), of 1 value that value."""
    import numpy as np

    import bench
    v = np.arange(1, 101, dtype=float)[::-1].copy()
    assert bench.p99_nearest_rank(v) == 99.0
    w = np.random.default_rng(0).permutation(4096).astype(float)
    assert bench.p99_nearest_rank(w) == 4055.0
    assert bench.p99_nearest_rank(np.array([3.5])) == 3.5


def test_binding_checks_a_supplied_training_set():
    """mlp_set_dataset refuses features, labels and pairs of different
    lengths before the library is called."""
    import numpy as np
    from paper_1907_02289_amd import bh
    ctx = bh.Context.__new__(bh.Context)          # no library context: the checks come first
    with pytest.raises(ValueError):
        ctx.mlp_set_dataset(np.zeros((5, 4)), np.zeros(4))
    with pytest.raises(ValueError):
        ctx.mlp_set_dataset(np.zeros((5, 4)), np.zeros(5), pairs=np.zeros((4, 2)))


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of bh_params, bh_sizes and bh_train_opts have the C
    layout: sizes and every field offset as a C compiler lays them out from
    include/bh.h."""
    import ctypes
    import subprocess
    from paper_1907_02289_amd import bh
    structs = {"bh_params": bh.Params, "bh_sizes": bh.Sizes, "bh_train_opts": bh.TrainOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bh.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
