"""Host-only checks of the C ABI library: it loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsnet.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsnet_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2509_19785_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared


def test_defaults():
    from paper_2509_19785_amd import _lib
    p = _lib.tsnet_params()
    _lib.tsnet_default_params(ctypes.byref(p))
    assert (p.lambda_kl, p.lambda_c, p.lambda_r, p.eps_r) == (1.0, 1.2, 0.01, 0.05)
    assert (p.interval_width, p.min_intervals, p.max_intervals, p.nodes_per_interval) == (0.25, 50, 512, 3)
    assert (p.repulsion, p.entropy, p.theta, p.far_trim) == (0, 0, 0.5, 64)
    # the Python mirror of the struct has the C layout (size and defaults)
    from paper_2509_19785_amd import api
    assert ctypes.sizeof(_lib.tsnet_params) == 80
    assert api.Params().far_trim == p.far_trim
    q = api.Params.variant("BH-tsNET", theta=0.3).to_c()
    assert (q.repulsion, q.entropy, q.theta) == (1, 1, 0.3)
    s = _lib.tsnet_step_params()
    _lib.tsnet_default_step_params(ctypes.byref(s))
    assert (s.momentum_early, s.momentum_late, s.momentum_switch_iter) == (0.5, 0.8, 250)
    assert (s.min_gain, s.gain_up, s.gain_down, s.eta) == (0.01, 0.2, 0.8, 0.0)


def test_null_arguments_are_rejected():
    from paper_2509_19785_amd import _lib
    assert _lib.lib.tsnet_ctx_create(None, 0) == _lib.TSNET_EINVAL
    assert b"NULL" in _lib.lib.tsnet_last_error()
    assert _lib.lib.tsnet_grad(None, None, None, None, None, None, None) == _lib.TSNET_EINVAL
    assert _lib.lib.tsnet_P_free(None) == 0 and _lib.lib.tsnet_ctx_destroy(None) == 0
    assert _lib.lib.tsnet_stage_count() == 16
    assert _lib.lib.tsnet_stage_name(6) == b"attract_assemble"
    assert _lib.lib.tsnet_stage_name(11) == b"pmds"
    assert _lib.lib.tsnet_stage_name(12) == b"np" and _lib.lib.tsnet_stage_name(13) == b"stress"
    assert _lib.lib.tsnet_stage_name(14) == b"quadtree"
    assert _lib.lib.tsnet_stage_name(15) == b"far_points"


def test_pmds_arguments_checked_on_the_host():
    import ctypes
    from paper_2509_19785_amd import _lib
    prm = _lib.tsnet_pmds_params()
    _lib.lib.tsnet_default_pmds_params(ctypes.byref(prm))
    assert (prm.pivots, prm.seed, prm.scale) == (50, 0, 1e-2)
    L = _lib.lib
    # NULL context / params / X, bad sizes: rejected before any device work
    assert L.tsnet_pmds(None, None, None, 1, 0, None, 1, ctypes.byref(prm), None, None, None, None,
                        None) == _lib.TSNET_EINVAL
    fake_ctx, fake_ptr = ctypes.c_void_p(1), ctypes.c_void_p(8)
    assert L.tsnet_pmds(fake_ctx, fake_ptr, fake_ptr, 0, 0, None, 1, ctypes.byref(prm), fake_ptr,
                        None, None, None, None) == _lib.TSNET_EINVAL
    assert b"n must be" in L.tsnet_last_error()
    for bad in ({"pivots": 0}, {"pivots": 129}, {"scale": 0.0}, {"scale": float("inf")}):
        q = _lib.tsnet_pmds_params()
        L.tsnet_default_pmds_params(ctypes.byref(q))
        for k, v in bad.items():
            setattr(q, k, v)
        assert L.tsnet_pmds(fake_ctx, fake_ptr, fake_ptr, 10, 0, None, 1, ctypes.byref(q),
                            fake_ptr, None, None, None, None) == _lib.TSNET_EINVAL
    # graph offsets that do not cover n
    offs = (ctypes.c_int32 * 3)(0, 4, 9)
    assert L.tsnet_pmds(fake_ctx, fake_ptr, fake_ptr, 10, 0, offs, 2, ctypes.byref(prm), fake_ptr,
                        None, None, None, None) == _lib.TSNET_EINVAL


def test_metric_arguments_checked_on_the_host():
    import ctypes
    from paper_2509_19785_amd import _lib
    L = _lib.lib
    fake_ctx, fake_ptr = ctypes.c_void_p(1), ctypes.c_void_p(8)
    # NULL context / X / outputs, bad sizes: rejected before any device work
    assert L.tsnet_np(None, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, None, 4, fake_ptr,
                      fake_ptr, None, None) == _lib.TSNET_EINVAL
    assert L.tsnet_np(fake_ctx, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, None, 4, None,
                      fake_ptr, None, None) == _lib.TSNET_EINVAL
    assert L.tsnet_np(fake_ctx, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, None, 3, fake_ptr,
                      fake_ptr, None, None) == _lib.TSNET_EINVAL
    assert b"num_vertices" in L.tsnet_last_error()
    assert L.tsnet_np(fake_ctx, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, fake_ptr, 0, fake_ptr,
                      fake_ptr, None, None) == _lib.TSNET_EINVAL
    offs = (ctypes.c_int32 * 3)(0, 2, 3)
    assert L.tsnet_np(fake_ctx, fake_ptr, fake_ptr, 4, 0, offs, 2, fake_ptr, None, 4, fake_ptr,
                      fake_ptr, None, None) == _lib.TSNET_EINVAL
    sums = (ctypes.c_double * 6)()
    assert L.tsnet_stress(fake_ctx, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, None, 1, sums,
                          None, None) == _lib.TSNET_EINVAL
    assert b"sources" in L.tsnet_last_error()
    assert L.tsnet_stress(fake_ctx, fake_ptr, fake_ptr, 4, 0, None, 1, fake_ptr, fake_ptr, 1, None,
                          None, None) == _lib.TSNET_EINVAL
    assert L.tsnet_stress(fake_ctx, fake_ptr, fake_ptr, 0, 0, None, 1, fake_ptr, fake_ptr, 1, sums,
                          None, None) == _lib.TSNET_EINVAL
    assert b"n must be" in L.tsnet_last_error()


def test_stage_names_unique():
    from paper_2509_19785_amd import _lib
    names = [_lib.lib.tsnet_stage_name(i) for i in range(_lib.lib.tsnet_stage_count())]
    assert len(set(names)) == len(names) and _lib.lib.tsnet_stage_name(99) == b""
