"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point that include/gs.h declares, sizes workspaces, and rejects bad
arguments before any device work is enqueued."""
import ctypes
import math
import os
import re

import pytest

from paper_1907_04834_amd import gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gs.lib()
    names = declared_symbols()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(gs.EXPORTS)


def test_version_and_defaults():
    assert "gfx950" in gs.gs_version()
    p = gs.Params()
    gs.lib().gs_params_default(ctypes.byref(p))
    assert (p.sigma, p.cutoff_sigmas, p.theta, p.leaf_cap, p.nt) == (1.0, 3.0, 0.5, 1, 40)


def test_workspace_sizes():
    prm = gs.params(0.05, nt=40)
    small = gs.gs_workspace_bytes(1000, prm, gs.GS_EXACT, gs.GS_OP_RHS)
    big = gs.gs_workspace_bytes(200000, prm, gs.GS_EXACT, gs.GS_OP_RHS)
    assert 0 < small < big
    assert gs.gs_workspace_bytes(200000, prm, gs.GS_BH, gs.GS_OP_RHS) > 0
    assert gs.gs_workspace_bytes(200000, prm, gs.GS_EXACT, gs.GS_OP_SHOOT) >= big
    assert gs.gs_workspace_bytes(-1, prm, gs.GS_EXACT, gs.GS_OP_RHS) == 0
    assert gs.gs_workspace_bytes(10, prm, 7, gs.GS_OP_RHS) == 0


def _call(name, *args):
    return getattr(gs.lib(), name)(*args)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("field,value", [("sigma", 0.0), ("sigma", -1.0),
                                         ("sigma", math.nan), ("sigma", math.inf)])
def test_rejects_bad_sigma(field, value):
    prm = gs.params(0.1)
    setattr(prm, field, value)
    st = _call("gs_rhs_exact", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, 1 << 30,
               None)
    assert st == -1
    assert "sigma" in gs.lib().gs_last_error().decode()


@pytest.mark.parametrize("field,value", [("theta", -0.1), ("theta", math.nan),
                                         ("cutoff_sigmas", 0.0), ("leaf_cap", 0),
                                         ("leaf_cap", 65), ("nt", 0)])
def test_rejects_bad_tree_params(field, value):
    prm = gs.params(0.1)
    setattr(prm, field, value)
    st = _call("gs_shoot", FAKE, FAKE, 10, ctypes.byref(prm), gs.GS_BH, FAKE, FAKE, None,
               FAKE, 1 << 30, None)
    assert st == -1


def test_rejects_negative_n_null_and_small_workspace():
    prm = gs.params(0.1)
    assert _call("gs_rhs_exact", FAKE, FAKE, -5, ctypes.byref(prm), FAKE, FAKE, FAKE, 1 << 30,
                 None) == -1
    assert _call("gs_rhs_exact", None, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, 1 << 30,
                 None) == -1
    st = _call("gs_rhs_exact", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, 16, None)
    assert st == -2
    assert "workspace" in gs.lib().gs_last_error().decode()
    st = _call("gs_shoot", FAKE, FAKE, 10, ctypes.byref(prm), 3, FAKE, FAKE, None, FAKE,
               1 << 30, None)
    assert st == -1


def test_zero_points_is_a_noop():
    prm = gs.params(0.1)
    assert _call("gs_rhs_exact", None, None, 0, ctypes.byref(prm), None, None, None, 0,
                 None) == 0
    assert _call("gs_shoot", None, None, 0, ctypes.byref(prm), gs.GS_BH, None, None, None,
                 None, 0, None) == 0


def _off(vals):
    return (ctypes.c_int64 * len(vals))(*vals)


def test_exact_items_parameter():
    prm = gs.params(0.05, nt=4)
    for bad in (-1, 100, 255, (1 << 22) + 1):
        prm.exact_items = bad
        st = _call("gs_rhs_exact", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, 1 << 30,
                   None)
        assert st == -1 and "exact_items" in gs.lib().gs_last_error().decode()
    # more work items per launch: smaller source chunks, more partial sums
    sizes = []
    for items in (6144, 24576, 49152):
        prm.exact_items = items
        sizes.append(gs.gs_workspace_bytes(200000, prm, gs.GS_EXACT, gs.GS_OP_RHS))
    assert sizes[0] < sizes[1] < sizes[2]
    prm.exact_items = 0
    assert gs.gs_workspace_bytes(200000, prm, gs.GS_EXACT, gs.GS_OP_RHS) == sizes[1]
    # the tuner needs a workspace that fits at least one candidate
    st = _call("gs_autotune_exact", FAKE, FAKE, _off([0, 5000]), 1, ctypes.byref(prm), FAKE,
               FAKE, FAKE, 4096, None, None)
    assert st == -2


def test_batch_workspace_sizes():
    prm = gs.params(0.05, nt=40, theta=0.5, leaf_cap=16)
    offs = [0, 5000, 5000, 12000, 40000]
    for method in (gs.GS_EXACT, gs.GS_BH):
        rhs = gs.gs_batch_workspace_bytes(offs, prm, method, gs.GS_OP_RHS)
        sh = gs.gs_batch_workspace_bytes(offs, prm, method, gs.GS_OP_SHOOT)
        assert 0 < rhs <= sh
    # a one-set batch needs about what the single-set call needs
    one = gs.gs_batch_workspace_bytes([0, 20000], prm, gs.GS_BH, gs.GS_OP_SHOOT)
    single = gs.gs_workspace_bytes(20000, prm, gs.GS_BH, gs.GS_OP_SHOOT)
    assert abs(one - single) < 0.05 * single
    # the backward stage: GS_OP_ADJOINT sizes for checkpoints every 8 steps
    for method in (gs.GS_EXACT, gs.GS_BH):
        adj = gs.gs_batch_workspace_bytes(offs, prm, method, gs.GS_OP_ADJOINT)
        assert adj == gs.lib().gs_adjoint_batch_workspace_bytes(_off(offs), len(offs) - 1,
                                                                ctypes.byref(prm), method, 8)
        assert adj > gs.gs_batch_workspace_bytes(offs, prm, method, gs.GS_OP_SHOOT) // 2
        # a one-set batch is what the single-set call uses
        assert (gs.lib().gs_adjoint_batch_workspace_bytes(_off([0, 7000]), 1, ctypes.byref(prm),
                                                          method, 5)
                == gs.lib().gs_adjoint_workspace_bytes(7000, ctypes.byref(prm), method, 5))
    assert gs.lib().gs_adjoint_batch_workspace_bytes(_off(offs), len(offs) - 1,
                                                     ctypes.byref(prm), gs.GS_BH, 0) == 0


@pytest.mark.parametrize("offs,nsub,msg", [
    ([1, 5, 9], 2, "offsets[0]"),
    ([0, 9, 5], 2, "non-decreasing"),
    ([0, 4], 0, "nsub"),
])
def test_batch_rejects_bad_offsets(offs, nsub, msg):
    prm = gs.params(0.1)
    st = _call("gs_rhs_batch", FAKE, FAKE, _off(offs), nsub, ctypes.byref(prm), gs.GS_EXACT,
               FAKE, FAKE, FAKE, 1 << 30, None)
    assert st == -1
    assert msg in gs.lib().gs_last_error().decode()
    assert _call("gs_batch_workspace_bytes", _off(offs), nsub, ctypes.byref(prm), gs.GS_EXACT,
                 gs.GS_OP_RHS) == 0


def test_batch_rejects_null_offsets_bad_method_and_small_workspace():
    prm = gs.params(0.1, nt=4)
    st = _call("gs_shoot_batch", FAKE, FAKE, None, 1, ctypes.byref(prm), gs.GS_BH, FAKE, FAKE,
               None, FAKE, 1 << 30, None)
    assert st == -1
    st = _call("gs_shoot_batch", FAKE, FAKE, _off([0, 10]), 1, ctypes.byref(prm), 3, FAKE, FAKE,
               None, FAKE, 1 << 30, None)
    assert st == -1
    st = _call("gs_shoot_batch", FAKE, FAKE, _off([0, 10, 30]), 2, ctypes.byref(prm),
               gs.GS_BH, FAKE, FAKE, None, FAKE, 4096, None)
    assert st == -2
    # all sets empty: a no-op that touches nothing
    st = _call("gs_shoot_batch", None, None, _off([0, 0, 0]), 2, ctypes.byref(prm), gs.GS_BH,
               None, None, None, None, 0, None)
    assert st == 0


def test_adjoint_batch_rejects_bad_arguments():
    prm = gs.params(0.1, nt=4)
    off = _off([0, 10, 30])

    def call(offs, nsub, lam=0.01, ck=2, method=gs.GS_EXACT, ws_bytes=1 << 30, q=FAKE):
        return _call("gs_shoot_adjoint_batch", q, FAKE, FAKE, offs, nsub, ctypes.byref(prm),
                     method, ctypes.c_double(lam), ck, FAKE, FAKE, FAKE, ws_bytes, None)

    assert call(off, 2, lam=math.nan) == -1 and "lambda" in gs.lib().gs_last_error().decode()
    assert call(off, 2, ck=0) == -1 and "ckpt" in gs.lib().gs_last_error().decode()
    assert call(_off([0, 9, 5]), 2) == -1
    assert call(off, 2, method=5) == -1
    assert call(off, 2, q=None) == -1
    assert call(off, 2, method=gs.GS_BH, ws_bytes=4096) == -2
    # all sets empty: a no-op that touches nothing
    assert _call("gs_shoot_adjoint_batch", None, None, None, _off([0, 0]), 1,
                 ctypes.byref(prm), gs.GS_BH, ctypes.c_double(0.01), 2, None, None, None, 0,
                 None) == 0


def test_rejects_unknown_flags():
    prm = gs.params(0.1, flags=2)  # no such flag
    st = _call("gs_rhs_exact", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, 1 << 30,
               None)
    assert st == -1 and "flags" in gs.lib().gs_last_error().decode()


def test_f64_rhs_checks_its_workspace():
    """gs_rhs_exact_f64 needs the (header-only) workspace that
    gs_workspace_bytes reports for GS_FLAG_F64, like every other call."""
    prm = gs.params(0.1, flags=gs.GS_FLAG_F64)
    need = gs.gs_workspace_bytes(10, prm, gs.GS_EXACT, gs.GS_OP_RHS)
    assert need > 0
    st = _call("gs_rhs_exact_f64", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, None, 0, None)
    assert st == -2
    st = _call("gs_rhs_exact_f64", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, FAKE, need - 1,
               None)
    assert st == -2


def test_field_workspace_grows_with_both_sizes():
    prm = gs.params(0.05)
    f = gs.lib().gs_field_workspace_bytes
    assert 0 < f(1000, 1000, ctypes.byref(prm)) < f(200000, 1000, ctypes.byref(prm))
    assert f(1000, 1000, ctypes.byref(prm)) < f(1000, 200000, ctypes.byref(prm))
    assert f(-1, 10, ctypes.byref(prm)) == 0
    # GS_OP_FIELD sizes the square case
    assert gs.gs_workspace_bytes(5000, prm, gs.GS_EXACT, gs.GS_OP_FIELD) == f(
        5000, 5000, ctypes.byref(prm))


def test_status_codes_are_distinct():
    assert gs.STATUS[-6] == "GS_ERR_OVERFLOW" and gs.STATUS[-4] == "GS_ERR_NONFINITE"


def test_static_workspace_entry_checks_before_device_work():
    """gs_rhs_exact_static: size limit, parameter and pointer checks, n = 0,
    all before any device work; every n up to the limit fits the array with
    the smallest work-item target."""
    prm = gs.params(0.05)
    st = _call("gs_rhs_exact_static", FAKE, FAKE, gs.GS_STATIC_MAX_N + 1, ctypes.byref(prm),
               FAKE, FAKE, None)
    assert st == -2 and "GS_STATIC_MAX_N" in gs.lib().gs_last_error().decode()
    assert _call("gs_rhs_exact_static", None, None, 0, ctypes.byref(prm), None, None,
                 None) == 0
    assert _call("gs_rhs_exact_static", FAKE, FAKE, 10, None, FAKE, FAKE, None) == -1
    assert _call("gs_rhs_exact_static", None, FAKE, 10, ctypes.byref(prm), FAKE, FAKE,
                 None) == -1
    bad = gs.params(-1.0)
    assert _call("gs_rhs_exact_static", FAKE, FAKE, 10, ctypes.byref(bad), FAKE, FAKE,
                 None) == -1
    prm.exact_items = 100
    st = _call("gs_rhs_exact_static", FAKE, FAKE, 10, ctypes.byref(prm), FAKE, FAKE, None)
    assert st == -1 and "exact_items" in gs.lib().gs_last_error().decode()
    prm.exact_items = 256
    assert gs.gs_workspace_bytes(gs.GS_STATIC_MAX_N, prm, gs.GS_EXACT,
                                 gs.GS_OP_RHS) <= gs.GS_STATIC_SCRATCH_BYTES
