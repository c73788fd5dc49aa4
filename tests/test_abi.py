"""CPU checks of the C-ABI library: it builds for gfx950, loads, and exports every entry
point the public header declares.  No compute call is made (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlte.h")
LIB = os.path.join(ROOT, "paper_1912_08445_amd", "libnlte.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nlte_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(LIB):
        from paper_1912_08445_amd import build
        build.build()
    return LIB


def test_header_declares_entry_points():
    names = declared()
    assert "nlte_formal_solve" in names and "nlte_run_ali" in names and len(names) >= 20


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (nlte_[a-z_]+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_covers_header(libpath):
    from paper_1912_08445_amd import binding
    assert sorted(binding.EXPORTS) == declared()
    L = binding.lib()
    for n in binding.EXPORTS:
        assert getattr(L, n) is not None


def test_library_is_gfx950_code_object(libpath):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", libpath], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_create_without_gpu_reports_hip_error(libpath):
    """Without a visible device the library refuses to create a context (no CPU path)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1912_08445_amd import binding
    h = ctypes.c_void_p()
    assert binding.lib().nlte_create(ctypes.byref(h), 0) == binding.NLTE_E_HIP
