"""The C-ABI library loads and exports every function that include/fmmbem.h declares (no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fmmbem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmmbem_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("fmmbem_create", "fmmbem_set_mesh", "fmmbem_matvec", "fmmbem_solve", "fmmbem_eval_field"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_16073_amd import fmmbem as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    import ctypes
    L = ctypes.CDLL(F.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding covers the same names
    assert set(_declared()) <= set(F.EXPORTS)


def test_create_without_device_fails_cleanly():
    """No GPU here: create must report an error code, not crash or fall back."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2103_16073_amd import fmmbem as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(F.FmmbemError):
        F.Context(0)
