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
