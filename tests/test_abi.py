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


def test_binding_structs_match_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's field offsets and size (a C program built
    from include/fmmbem.h prints them), so an option or report field never lands in another's slot."""
    import ctypes
    import shutil
    import subprocess
    from paper_2103_16073_amd import fmmbem as F
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    pairs = {"fmmbem_options": F.Options, "fmmbem_solve_opts": F.SolveOpts, "fmmbem_solve_report": F.SolveReport,
             "fmmbem_train_opts": F.TrainOpts, "fmmbem_train_report": F.TrainReport, "fmmbem_info": F.Info,
             "fmmbem_batch_shape": F.BatchShape, "fmmbem_kstat": F.KStat}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmmbem.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, cls in pairs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with an error and a message, before any
    device work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
