"""The C-ABI library loads and exports every function that include/*.h declares
(no GPU needed; no compute call is made)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_1810_13100_amd", "libncs.so")


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(ncs_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("ncs_setup", "ncs_iterate", "ncs_solve", "ncs_destroy", "ncs_last_error", "ncs_prefilter",
              "ncs_cnn_create", "ncs_cnn_forward", "ncs_cnn_train_step", "ncs_conv3x3_bf16",
              "ncs_cone_setup", "ncs_cone_iterate", "ncs_cone_adjoint"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libncs.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (same HIP runtime as the binding)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1810_13100_amd import cnn, cone, ncs
    assert sorted(ncs.EXPORTED + cnn.EXPORTED + cone.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libncs.so not built")
def test_last_error_is_empty_string_initially():
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB)
    lib.ncs_last_error.restype = ctypes.c_char_p
    assert lib.ncs_last_error() == b""


@pytest.mark.skipif(not os.path.exists(LIB), reason="libncs.so not built")
def test_null_arguments_are_rejected_without_gpu_work():
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB)
    lib.ncs_setup.restype = ctypes.c_int32
    lib.ncs_iterate.restype = ctypes.c_int32
    lib.ncs_last_error.restype = ctypes.c_char_p
    assert lib.ncs_setup(None, None, 0, None, None, None, None) == -1
    assert b"null" in lib.ncs_last_error()
    lib.ncs_iterate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    assert lib.ncs_iterate(None, 1, None) == -1
    lib.ncs_cone_setup.restype = ctypes.c_int32
    assert lib.ncs_cone_setup(None, None, 0, None, None, None) == -1
    assert b"null" in lib.ncs_last_error()
    lib.ncs_cone_iterate.restype = ctypes.c_int32
    lib.ncs_cone_iterate.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    assert lib.ncs_cone_iterate(None, 1, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libncs.so not built")
def test_cone_geometry_and_parameters_are_validated_before_gpu_work():
    """ncs_cone_setup checks its geometry and parameters before any HIP call
    (include/ncs_cone.h: the limits of the geometry and of the parameters)."""
    import torch  # noqa: F401
    from paper_1810_13100_amd import cone, ncs
    lib = ctypes.CDLL(LIB)
    lib.ncs_cone_setup.restype = ctypes.c_int32
    lib.ncs_last_error.restype = ctypes.c_char_p
    good = (32, 16, 24, 48, 11, 0, 60.0)
    ok_params = (0.01, 0.03, 1.0, 0.01, 0.0, ncs.METHOD_NCS, 0, 0, 0)
    cases = [
        ((32, 16, 24, 48, 11, 0, 25.0), ok_params, b"source_radius"),     # source inside the margin
        ((24, 16, 24, 48, 11, 0, 60.0), ok_params, b"n_side"),            # N not a power of two
        ((32, 512, 24, 48, 11, 0, 60.0), ok_params, b"n_slices"),         # N_z above 256
        ((32, 16, 24, 48, 1, 0, 60.0), ok_params, b"n_rows >= 2"),        # one detector row
        ((32, 16, 65536, 48, 11, 0, 60.0), ok_params, b"65535"),          # N_v above 65535
        ((32, 16, 24, 4097, 4096, 0, 60.0), ok_params, b"2^24"),          # N_r N_s above 2^24
        ((32, 16, 24, 48, 11, 1, 60.0), ok_params, b"reserved"),          # reserved field set
        (good, (0.0,) + ok_params[1:], b"alpha > 0"),                     # alpha = 0
        (good, ok_params[:5] + (ncs.METHOD_ADMM_CG,) + ok_params[6:], b"NCS_METHOD"),
        (good, ok_params[:7] + (2, 0), b"positivity"),                    # positivity not 0 or 1
    ]
    for geo, par, msg in cases:
        g = cone._ConeGeometry(*geo)
        p = cone._ConeParams(*par)
        h = ctypes.c_void_p()
        st = lib.ncs_cone_setup(ctypes.byref(g), ctypes.byref(p), ncs.NCS_F32, None, None, ctypes.byref(h))
        assert st == ncs.NCS_ERR_INVALID_ARG, (geo, par)
        assert h.value is None
        assert msg in lib.ncs_last_error(), (geo, par, lib.ncs_last_error())
    g = cone._ConeGeometry(*good)
    p = cone._ConeParams(*ok_params)
    h = ctypes.c_void_p()
    assert lib.ncs_cone_setup(ctypes.byref(g), ctypes.byref(p), 7, None, None, ctypes.byref(h)) == -1   # dtype
    assert b"dtype" in lib.ncs_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libncs.so not built")
def test_slice_geometry_and_parameters_are_validated_before_gpu_work():
    """ncs_setup checks geometry, parameters and dtype before any HIP call
    (include/ncs.h: the fields of ncs_geometry and ncs_params)."""
    import torch  # noqa: F401
    from paper_1810_13100_amd import ncs
    lib = ctypes.CDLL(LIB)
    lib.ncs_setup.restype = ctypes.c_int32
    lib.ncs_last_error.restype = ctypes.c_char_p
    geo = dict(n_side=64, n_angles=90, n_bins=92, beam=0, source_radius=0.0)
    par = dict(alpha=0.01, beta=0.03, gamma=1.0, lambda_=0.01, c_r=0.0, mu_dc=0.0, data_term=0, tv_term=0,
               check_every=0, diverge_checks=0, projector=0, graph_chunk=0, dual_ramp=0.0, backprojector=0,
               method=0, cg_iters=0, cg_precondition=0, positivity=0, probes=0)
    cases = [
        (dict(n_side=48), {}, b"n_side"),
        (dict(n_side=2048), {}, b"n_side"),
        (dict(n_angles=0), {}, b"n_angles"),
        (dict(n_bins=1), {}, b"n_bins"),
        (dict(beam=2), {}, b"beam"),
        (dict(beam=1, source_radius=40.0), {}, b"source_radius"),          # inside 1.01 N / sqrt 2
        ({}, dict(alpha=0.0), b"alpha > 0"),
        ({}, dict(lambda_=float("nan")), b"lambda >= 0"),
        ({}, dict(probes=5000), b"probes"),
        ({}, dict(data_term=7), b"data_term"),
        ({}, dict(tv_term=5), b"tv_term"),
        ({}, dict(method=3), b"method"),
        ({}, dict(method=2, cg_iters=2000), b"cg_iters"),
        ({}, dict(positivity=2), b"positivity"),
        ({}, dict(method=2, positivity=1), b"ADMM-CG"),
        ({}, dict(method=1, gamma=0.0), b"PDHG needs gamma"),
        ({}, dict(backprojector=4), b"backprojector"),
        ({}, dict(projector=4), b"projector"),
        (dict(beam=1, source_radius=128.0), dict(projector=1), b"fan beam"),
        (dict(beam=1, source_radius=128.0), dict(method=2, cg_precondition=1), b"fan beams run"),
        ({}, dict(method=2, cg_precondition=0), b"double precision only"),   # FP32 plain CG
    ]
    for gk, pk, msg in cases:
        g = ncs._Geometry(**{**geo, **gk})
        p = ncs._Params(**{**par, **pk})
        h = ctypes.c_void_p()
        st = lib.ncs_setup(ctypes.byref(g), ctypes.byref(p), ncs.NCS_F32, None, None, None, ctypes.byref(h))
        assert st == ncs.NCS_ERR_INVALID_ARG, (gk, pk)
        assert h.value is None
        assert msg in lib.ncs_last_error(), (gk, pk, lib.ncs_last_error())
    g, p, h = ncs._Geometry(**geo), ncs._Params(**par), ctypes.c_void_p()
    assert lib.ncs_setup(ctypes.byref(g), ctypes.byref(p), 9, None, None, None, ctypes.byref(h)) == -1
    assert b"dtype" in lib.ncs_last_error()
