"""The C-ABI library loads and exports every entry point include/tk.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_11404_amd", "libtk.so")


def declared():
    text = open(os.path.join(ROOT, "include", "tk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tk_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (binds torch's HIP runtime first, as the binding does)
    L = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")
def test_host_only_entry_points():
    from paper_2603_11404_amd import tk
    L = tk.lib()
    assert L.tk_version() == 100
    assert L.tk_status_string(1) == b"TK_ERR_INVALID_ARGUMENT"
    assert tk.cmaes_state_bytes(9, 16) > 0 and tk.cmaes_state_bytes(9, 16) % 256 == 0
    assert tk.cmaes_state_bytes(0, 16) == 0 and tk.cmaes_state_bytes(19, 16) == 0
    assert tk.cmaes_state_bytes(9, 1025) == 0
    lay = tk.cmaes_layout(18, 1024)
    assert lay["order"] + 4 * 1024 <= lay["total_bytes"]
    with pytest.raises(tk.TkError) as e:
        tk.cmaes_layout(0, 16)
    assert e.value.status == 1


def test_binding_exports_match_header():
    from paper_2603_11404_amd import tk
    assert sorted(tk.EXPORTS) == declared()
