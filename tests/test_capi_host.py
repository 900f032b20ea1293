"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function that include/ctm.h declares,
size workspaces and reject invalid configurations without touching a device.
"""
import ctypes
import os
import re

import pytest

import paper_2607_15158_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ctm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(ctm_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_move_api():
    names = declared_functions()
    for n in ["ctm_init", "ctm_move", "ctm_converge", "ctm_observable", "ctm_destroy",
              "ctm_workspace_bytes", "ctm_set_isometries", "ctm_qr_f64", "ctm_svd_f64",
              "ctm_gemm_f64", "ctm_profile", "ctm_profile_read"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_status_strings():
    assert P._lib.ctm_status_str(0) == b"ok"
    assert P._lib.ctm_status_str(5) == b"numerical failure"


def test_workspace_bytes_scale_and_config3_fits_hbm():
    small = P.workspace_bytes(P.Config(d=2, D=2, chi=8, p=4))
    big = P.workspace_bytes(P.Config(d=2, D=6, chi=144, p=16))
    assert 0 < small < big
    assert big < 16 * 2 ** 30      # a few GiB of the 288 GB HBM
    f32 = P.workspace_bytes(P.Config(d=2, D=6, chi=144, p=16, prec="f32"))
    bf16 = P.workspace_bytes(P.Config(d=2, D=6, chi=144, p=16, prec="bf16"))
    assert bf16 < f32 < big


@pytest.mark.parametrize("kw", [dict(chi=0), dict(D=0), dict(p=-1), dict(n_si=-1),
                                dict(chi=180, p=13),
                                dict(D=4, chi=176, p=16)])   # k = 192, N = 2816: no leaf split
def test_invalid_configs_are_rejected(kw):
    base = dict(d=2, D=2, chi=8, p=4)
    base.update(kw)
    with pytest.raises(P.CtmError):
        P.workspace_bytes(P.Config(**base))


def test_unknown_projector_and_precision_rejected():
    c = P.Config(d=2, D=2, chi=8).c()
    c.proj = 7
    n = ctypes.c_size_t()
    assert P._lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == P.CTM_E_ARG
    c = P.Config(d=2, D=2, chi=8).c()
    c.prec = 9
    assert P._lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == P.CTM_E_ARG
    c = P.Config(d=2, D=2, chi=8).c()
    c.growth = 2
    assert P._lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == P.CTM_E_ARG
    c = P.Config(d=2, D=2, chi=8).c()
    c.svd_driver = 3
    assert P._lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == P.CTM_E_ARG


def test_recycling_configs():
    """Recycling keeps two more sets of blocks; it needs min_si_moves >= 1, a
    numeric threshold and the four-direction move."""
    base = dict(d=2, D=3, chi=18, p=6)
    plain = P.workspace_bytes(P.Config(**base))
    rec = P.workspace_bytes(P.Config(**base, recycle_sin2=1e-3))
    N, k, chi = 18 * 9, 24, 18
    assert rec - plain >= 8 * (N * k + chi * chi) * 8
    n = ctypes.c_size_t()
    for kw in (dict(recycle_sin2=1e-3, min_si_moves=0),
               dict(recycle_sin2=float("nan")),
               dict(recycle_sin2=1e-3, sym="c4v")):
        c = P.Config(**base, **kw).c()
        assert P._lib.ctm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == P.CTM_E_ARG, kw


def test_null_arguments_are_errors_not_crashes():
    assert P._lib.ctm_workspace_bytes(None, None) == P.CTM_E_ARG
    h = ctypes.c_void_p()
    c = P.Config(d=2, D=2, chi=8).c()
    assert P._lib.ctm_init(ctypes.byref(h), ctypes.byref(c), None, None, None, 0, None) == P.CTM_E_ARG
    assert P._lib.ctm_move(None, None) == P.CTM_E_ARG
    assert P._lib.ctm_observable(None, 0, None, None) == P.CTM_E_ARG


def test_single_hip_runtime_in_process():
    """The library shares torch's HIP/HSA runtime instead of loading a second one.

    Two runtimes in one process cannot share the device: whichever initialises
    second reports that no GPU is present.
    """
    maps = open("/proc/self/maps").read().splitlines()
    for stem in ("libamdhip64", "libhsa-runtime64"):
        files = {ln.split()[-1] for ln in maps if stem in ln.split()[-1]}
        assert len(files) <= 1, files
