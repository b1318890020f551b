"""The C-ABI library loads without a GPU and exports every function declared
in include/*.h; host-side argument validation needs no device."""
import ctypes
import glob
import os
import re

import pytest

from paper_2603_13618_amd import lks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lks_[a-z0-9_]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(lks.LIB_PATH)
    names = _declared()
    assert len(names) >= 17
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_config_validation_on_host():
    L = lks.lib()
    ok = lks.make_config(9, 64, 64, "f32", tau=0.6, max_steps=10)
    assert lks.scratch_bytes(ok) > 256
    bad = [lks.make_config(9, 64, 64, "f32", tau=0.5),
           lks.make_config(9, 0, 64, "f32", tau=0.6),
           lks.make_config(9, 64, 64, "f32", tau=0.6, max_steps=0),
           lks.make_config(9, 64, 64, "f32", tau=0.6, flag_mask=8),
           lks.make_config(9, 64, 64, "f32", tau=0.6, bc=(1, 0)),
           lks.make_config(25, 64, 64, "f32", mu=0.0, dt=1e-3, dx=0.1),
           lks.make_config(7, 64, 64, "f32", tau=0.6),
           lks.make_config(9, 64, 64, 9, tau=0.6),
           lks.make_config(9, 64, 64, "f32", tau=0.6, thr=[[1.0, 0.5]] * 4)]
    for c in bad:
        assert lks.scratch_bytes(c) == 0
    # create rejects NULL buffers before touching the device
    ctx = ctypes.c_void_p()
    buf = lks.Buffers()
    st = L.lks_create(ctypes.byref(ok), ctypes.byref(buf), None, ctypes.byref(ctx))
    assert st == 1 and not ctx.value
    assert b"NULL" in L.lks_last_error(None)
    assert L.lks_status_str(4) == b"non-positive populations"


def test_abi_struct_layout_matches_header():
    # offsets of the ctypes mirror against the C declaration order/alignment
    assert ctypes.sizeof(lks.Config) == 4 * 6 + 8 * 5 + 4 + 4 + 8 * 8 + 4 + 4
    assert lks.Config.thr.offset == 72
    assert ctypes.sizeof(lks.Buffers) == 8 * 7


@pytest.mark.parametrize("name", ["lks_step", "lks_moments", "lks_check", "lks_init_equilibrium"])
def test_null_context_is_rejected(name):
    fn = getattr(lks.lib(), name)
    args = [None] * len(fn.argtypes)
    if name == "lks_step":
        args = [None, 1, 1]
    assert fn(*args) == 1
