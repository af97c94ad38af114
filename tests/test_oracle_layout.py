"""The oracle's ctypes mirrors have the layout its C header gives the structs."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_struct_layouts_match_the_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    checks = {
        "orc_cfg": (oracle.OrcCfg, ["two_ring_levels", "eta", "r_list", "adapt_dt", "grow_iters",
                                    "shrink_iters", "dt_min", "shrink"]),
        "orc_pci_state": (oracle.OrcPciState, ["major_len", "minor_steps", "hist", "dt_cur",
                                               "peak_iters", "last_a2max", "snap", "snap_t",
                                               "snap_clean", "last_rollback", "trace_p",
                                               "trace_e", "trace_cap", "trace_len"]),
        "orc_info": (oracle.OrcInfo, ["TV", "lmax", "delta"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rts_oracle.h"',
             "int main(void) {"]
    for name, (_, fields) in checks.items():
        lines.append(f'printf("%zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("%zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = []
    for name, (cls, fields) in checks.items():
        want.append(C.sizeof(cls))
        want += [getattr(cls, f).offset for f in fields]
    assert got == want
