"""The C ABI library loads without a GPU, exports every function declared in
include/bf.h, and the binding's struct layouts match the C compiler's."""
import ctypes
import os
import subprocess

import pytest

from paper_1604_01093_amd import bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_header_functions():
    lib = bf.load()
    names = bf.header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(bf._SIGS), set(names) ^ set(bf._SIGS)


def test_params_default_and_status_strings():
    p = bf.bf_params_default()
    assert p.w_sparse == 1.0 and p.tau_dist == 0.15 and p.tau_normal == 0.9 and p.max_angle_deg == 60.0
    assert p.depth_min == 0.1 and p.depth_max == 10.0 and p.dense_ramp == 1
    lib = bf.load()
    assert lib.bf_status_string(0) == b"ok"
    assert lib.bf_status_string(4) == b"matrix not positive definite"


def test_null_arguments_are_rejected_without_a_device():
    lib = bf.load()
    assert lib.bf_create(None, None) == bf.BF_ERR_INVALID_ARG
    out = (ctypes.c_double * 8)()
    assert lib.bf_last_timings(None, out) == bf.BF_ERR_INVALID_ARG
    assert lib.bf_pcg_solve(None, None, 1, None, None) == bf.BF_ERR_INVALID_ARG
    assert lib.bf_graph_captures(None) == -1


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    structs = {"bf_intrinsics": bf.bf_intrinsics, "bf_frames": bf.bf_frames, "bf_corrs": bf.bf_corrs,
               "bf_pairs": bf.bf_pairs, "bf_params": bf.bf_params, "bf_structure": bf.bf_structure}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bf.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
