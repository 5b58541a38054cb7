"""The measurement probes: the contraction probe (r = 5 FP32 volume
contraction in the VALU sum-factorised and the MFMA dense form: both forms
compute the same numbers, and both time positively) and the launch and memory
floor probe (every variant times positively, eagerly and as graph nodes, and
bad arguments are refused)."""
import ctypes
import os
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2303_11767_amd",
                   "libdgsw_probe.so")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ctypes.CDLL(LIB)
    lib.dgp_contraction_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.dgp_contraction_check.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.dgp_floor_time.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)]
    return lib


@pytest.mark.parametrize("n", [1, 37, 4096])
def test_forms_agree(lib, n):
    rel = ctypes.c_double()
    assert lib.dgp_contraction_check(n, ctypes.byref(rel)) == 0
    print("[case] contraction forms", n, "max relative difference", rel.value, flush=True)
    sys.stdout.flush()
    assert rel.value <= 1e-5


def test_forms_time(lib):
    for variant in (0, 1):
        ms = ctypes.c_double()
        assert lib.dgp_contraction_time(variant, 6480, 3, ctypes.byref(ms)) == 0
        assert ms.value > 0.0


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_floor_probe_times(lib, variant, graph):
    us = ctypes.c_double(-1.0)
    print("[case] floor", variant, graph, flush=True)
    assert lib.dgp_floor_time(variant, 13, 7, graph, 10, ctypes.byref(us)) == 0
    assert 0.0 < us.value < 1e5


def test_floor_probe_refuses_bad_arguments(lib):
    us = ctypes.c_double()
    assert lib.dgp_floor_time(3, 13, 7, 0, 10, ctypes.byref(us)) == -1
    assert lib.dgp_floor_time(0, 0, 7, 0, 10, ctypes.byref(us)) == -1
    assert lib.dgp_floor_time(0, 13, 7, 2, 10, ctypes.byref(us)) == -1
    assert lib.dgp_floor_time(0, 13, 7, 0, 0, ctypes.byref(us)) == -1
