"""The C-ABI library loads and exports every entry point that include/rts.h
declares; host-only calls validate configurations (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2009_14514_amd import _rts, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rts.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rts_[a-z_]+)\s*\(", text)))


def test_header_declares_the_bound_entry_points():
    assert declared_functions() == sorted(_rts.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_rts.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_config_and_workspace_size():
    c = _rts.default_config()
    assert c.n_levels == 4 and c.lambda_v == 0.4 and c.lambda_f == 0.25 and c.alpha_rts == 0.4
    sc = scenes.dam_break_small()
    cfg = _rts.config_from_params(sc.params)
    small = _rts.workspace_size(cfg, sc.n, sc.nw)
    big = _rts.workspace_size(cfg, 10 * sc.n, sc.nw)
    assert 0 < small < big


@pytest.mark.parametrize("field,value,status", [
    ("block_edge", 0.01, _rts.RTS_E_INVALID),     # block smaller than the support
    ("gamma", 5.0, _rts.RTS_E_UNSUPPORTED),
    ("n_levels", 9, _rts.RTS_E_INVALID),
    ("cand_cap", 100, _rts.RTS_E_INVALID),       # not a multiple of 128
    ("c0", -1.0, _rts.RTS_E_INVALID),
    ("mode", 7, _rts.RTS_E_INVALID),
])
def test_invalid_configurations_are_rejected(field, value, status):
    sc = scenes.dam_break_small()
    cfg = _rts.config_from_params(sc.params)
    setattr(cfg, field, value)
    with pytest.raises(_rts.RtsError) as e:
        _rts.workspace_size(cfg, sc.n, sc.nw)
    assert e.value.status == status


def test_create_rejects_a_bad_workspace_without_touching_the_device():
    sc = scenes.dam_break_small()
    cfg = _rts.config_from_params(sc.params)
    with pytest.raises(_rts.RtsError) as e:
        _rts.create(cfg, sc.n, sc.nw, 0, 0, 0)                 # NULL workspace
    assert e.value.status == _rts.RTS_E_INVALID
    with pytest.raises(_rts.RtsError) as e:
        _rts.create(cfg, sc.n, sc.nw, 4096 + 8, 1 << 30, 0)     # misaligned
    assert e.value.status == _rts.RTS_E_INVALID


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C compiler gives
    the header's structs."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    checks = {
        "rts_config": (_rts.RtsConfig, ["n_minor", "nbr_cap", "two_ring_levels", "pci_adapt_dt",
                                        "eta", "r_list", "beta_ratio", "pci_grow_iters", "pci_shrink_iters",
                                        "pci_dt_min", "pci_shrink"]),
        "rts_stats": (_rts.RtsStats, ["bad_index", "pci_iters", "pci_errmax", "pci_iters_total",
                                      "pci_rollbacks", "pci_dt_next"]),
        "rts_tune": (_rts.RtsTune, ["search_threads", "force_threads", "force_lanes", "candidates",
                                    "ms_per_step"]),
        "rts_diff_desc": (_rts.RtsDiffDesc, ["list_cap", "dt", "alpha"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rts.h"', "int main(void) {"]
    for name, (_, fields) in checks.items():
        lines.append(f'printf("%zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("%zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = []
    for name, (cls, fields) in checks.items():
        want.append(C.sizeof(cls))
        want += [getattr(cls, f).offset for f in fields]
    assert got == want


@pytest.mark.parametrize("field,value", [("n_minor", 0), ("nbr_cap", 4), ("eta", 0.0),
                                         ("mode", 2), ("r_list", 1.0)])
def test_invalid_pcisph_configurations_are_rejected(field, value):
    sc = scenes.pcisph_dam_break_small()
    cfg = _rts.config_from_params(sc.params)
    setattr(cfg, field, value)
    with pytest.raises(_rts.RtsError):
        _rts.workspace_size(cfg, sc.n, sc.nw)


@pytest.mark.parametrize("over", [dict(pci_grow=0.9), dict(pci_shrink=0.0),
                                  dict(pci_shrink=1.5), dict(delta=1.0),
                                  dict(pci_dt_min=2e-3), dict(pci_dt_max=5e-4),
                                  dict(pci_adapt_dt=2)])
def test_invalid_adaptive_step_configurations_are_rejected(over):
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3)
    kw = dict(pci_adapt_dt=1)
    kw.update(over)
    cfg = _rts.config_from_params(sc.params, **kw)
    with pytest.raises(_rts.RtsError):
        _rts.workspace_size(cfg, sc.n, sc.nw)
    ok = _rts.config_from_params(sc.params, pci_adapt_dt=1)
    assert _rts.workspace_size(ok, sc.n, sc.nw) > 0
