"""The C-ABI library loads and exports every symbol include/aaa.h declares
(no compute calls: these run without a GPU), and host-side argument checks
fail cleanly."""
import ctypes as C
import os
import re

import pytest

from paper_2504_12811_amd import _lib as L
from paper_2504_12811_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "aaa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aaa_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.aaa_version().decode().startswith("aaa-gfx950")


def _abi_scene(n=10, deg=0):
    s = L.Scene()
    s.n = n
    s.sh_degree = deg
    fake = 0x1000
    s.means = s.log_scales = s.quats = s.opacity_logits = s.sh = fake
    return s


def test_workspace_size_host_checks():
    lib = L.lib()
    sc, cam = S.small_scene(n=16)
    c = L.make_camera(cam)
    st = L.make_settings(S.Settings())
    need = C.c_size_t()
    assert lib.aaa_workspace_size(C.byref(_abi_scene()), C.byref(c), C.byref(st), 1000, C.byref(need)) == L.AAA_OK
    assert need.value > 0
    bad = L.make_settings(S.Settings(ray_window=3))
    assert lib.aaa_workspace_size(C.byref(_abi_scene()), C.byref(c), C.byref(bad), 1000, C.byref(need)) == L.AAA_ERR_INVALID
    assert b"ray_window" in lib.aaa_last_error()
    assert lib.aaa_workspace_size(C.byref(_abi_scene(deg=4)), C.byref(c), C.byref(st), 1000, C.byref(need)) == L.AAA_ERR_UNSUPPORTED
    # an opacity clamp of 1 (or one that rounds to 1 in float) is rejected:
    # the backward divides by 1 - alpha
    for amax in (1.0, 1.0 - 1e-9, 1.5):
        bad = L.make_settings(S.Settings(alpha_max=amax, t_min=0.0))
        assert lib.aaa_workspace_size(C.byref(_abi_scene()), C.byref(c), C.byref(bad), 1000,
                                      C.byref(need)) == L.AAA_ERR_INVALID, amax
        assert b"alpha_max" in lib.aaa_last_error()
    ok = L.make_settings(S.Settings(alpha_max=0.999, t_min=0.0))
    assert lib.aaa_workspace_size(C.byref(_abi_scene()), C.byref(c), C.byref(ok), 1000, C.byref(need)) == L.AAA_OK
    c.width = 0
    assert lib.aaa_workspace_size(C.byref(_abi_scene()), C.byref(c), C.byref(st), 1000, C.byref(need)) == L.AAA_ERR_INVALID


def test_render_rejects_null_context_and_small_workspace():
    lib = L.lib()
    sc, cam = S.small_scene(n=16)
    c = L.make_camera(cam)
    st = L.make_settings(S.Settings())
    assert lib.aaa_render(None, C.byref(_abi_scene()), C.byref(c), C.byref(st), None, 0, 10, None, None, None, None) == L.AAA_ERR_INVALID


def test_sort_tmp_size_and_bad_bits():
    lib = L.lib()
    need = C.c_size_t()
    assert lib.aaa_sort_tmp_size(1 << 20, C.byref(need)) == L.AAA_OK and need.value > (1 << 20) * 12
    assert lib.aaa_sort_pairs(None, None, 10, 0, None, 0, None) == L.AAA_ERR_INVALID
    assert lib.aaa_sort_pairs(None, None, 10, 65, None, 0, None) == L.AAA_ERR_INVALID
