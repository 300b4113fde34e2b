"""The C-ABI library loads and exports every entry point include/em.h declares.

No compute call is made here: these run without a GPU.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "em.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(em_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("em_init", "em_iterate", "em_loglik", "em_destroy", "em_workspace_bytes",
                     "em_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import ctypes
    em = pytest.importorskip("paper_2302_05804_amd.em")
    lib = ctypes.CDLL(em.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding covers the same set
    assert set(em.exported_symbols()) >= set(declared_functions())


def test_workspace_bytes_host_logic():
    em = pytest.importorskip("paper_2302_05804_amd.em")
    P = em.Problem.make
    good = P(4, 128, 128, 15)
    nb = em.workspace_bytes(good)
    # u and r planes alone need 2 * n * Hf * Wf floats
    assert nb >= 2 * 4 * 128 * 128 * 4
    assert nb % 256 == 0
    assert em.workspace_bytes(P(33, 4096, 4096, 43)) > em.workspace_bytes(P(8, 1024, 1024, 43))
    sr2 = em.workspace_bytes(P(16, 2048, 2048, 43, sr=2))
    assert sr2 >= 2 * 16 * 2048 * 2048 * 4 + 4096 * 4096 * 4
    for bad in (P(0, 8, 8, 3), P(1, 0, 8, 3), P(1, 8, 8, 4), P(1, 8, 8, 45), P(1, 8, 8, 3, sr=3),
                P(1, 8, 8, 3, precision=9), P(1, 8, 8, 3, weight_mode=7), P(1, 8, 8, -1)):
        assert em.workspace_bytes(bad) == 0


def test_version_string():
    em = pytest.importorskip("paper_2302_05804_amd.em")
    assert "gfx950" in em.version()


def test_launch_plans_match_their_grids():
    """Host-only check of every launch descriptor for many shapes: both grids
    (frame / latent), both super-resolution factors, every precision and kernel
    variant, the serving plan and the stand-alone operators."""
    em = pytest.importorskip("paper_2302_05804_amd.em")
    import itertools
    sizes = [(1, 1), (3, 2), (17, 130), (64, 64), (65, 129), (128, 128), (257, 1023),
             (1024, 1024), (2048, 2048), (4096, 4096)]
    for (h, w), n, k, sr, prec in itertools.product(sizes, (1, 3, 8, 16, 33), (1, 15, 43), (1, 2),
                                                     (em.FP32, em.BF16_SPLIT, em.FP16_SPLIT, em.BF16)):
        em.check_plan(em.Problem.make(n, h, w, k, sr=sr, precision=prec))
    # the typeset weighting (sr = 1): one frame per adjoint group, never fused
    for (h, w), n, prec in itertools.product(sizes[:7], (1, 3, 33),
                                             (em.FP32, em.BF16_SPLIT, em.FP16_SPLIT)):
        em.check_plan(em.Problem.make(n, h, w, 43, precision=prec, weight_mode=em.W_LITERAL))
    # Student-t noise (its forward writes u w m and u w y, no binary16 r planes)
    for (h, w), n, sr, prec in itertools.product(sizes[:8], (3, 16), (1, 2),
                                                 (em.FP32, em.BF16_SPLIT, em.FP16_SPLIT)):
        em.check_plan(em.Problem.make(n, h, w, 43, sr=sr, precision=prec, nu=4.0))
