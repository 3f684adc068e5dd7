"""The C-ABI library loads (without a GPU) and exports every function the headers declare."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_18314_amd", "libnncert.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(nnc_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_the_interface():
    names = declared_functions()
    for required in ("nnc_create", "nnc_init_certificates", "nnc_step", "nnc_repair", "nnc_rebuild",
                     "nnc_oracle_verify", "nnc_frontier_entropy", "nnc_destroy", "nnc_strerror"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnncert.so not built")
def test_library_exports_every_declared_function():
    import torch  # noqa: F401  (the library must share torch's HIP runtime)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnncert.so not built")
def test_binding_export_list_matches_headers():
    from paper_2606_18314_amd import binding
    assert set(binding.EXPORTS) <= set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnncert.so not built")
def test_strerror_without_gpu():
    from paper_2606_18314_amd import binding
    binding.load()
    assert binding.strerror(-4).startswith("measured step")
    assert binding.strerror(0) == "ok"
