"""CPU-side checks of the HIP library: it loads, exports every entry point
the header declares, and its host-only planner arithmetic (exact chain norms)
matches the oracle bit for bit.  No device work is done here."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2609_04573_amd import apc
    return apc


def test_library_exports_every_header_symbol():
    apc = _lib()
    header = open(os.path.join(ROOT, "include", "apc.h")).read()
    names = set(re.findall(r"^(?:apc_status|void|const char\*|int32_t|int64_t)\s+(apc_[a-z_]+)\s*\(", header, re.M))
    assert names, "no declarations found"
    lib = apc.library()
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} not exported"
    assert set(apc.EXPORTED) <= names


def test_strerror_and_bad_arguments():
    apc = _lib()
    lib = apc.library()
    assert lib.apc_strerror(apc.APC_E_BELOW_FLOOR).decode().startswith("target below")
    with pytest.raises(apc.ApcError):
        apc.axis_norms(0, 3, 3)
    with pytest.raises(apc.ApcError):
        apc.axis_norms(10, 3, 2)


@pytest.mark.parametrize("n", [1, 2, 3, 9, 17, 64, 100, 500, 512, 513, 1800])
@pytest.mark.parametrize("degree", [1, 3])
def test_axis_norms_match_oracle(n, degree):
    from oracle import grid, weights
    apc = _lib()
    L = grid.num_levels((n,)) + 1
    li, l1 = weights.axis_norms(n, L, degree)
    gi, g1 = apc.axis_norms(n, L, degree)
    assert gi == li
    assert g1 == l1


def test_oracle_is_not_imported_by_the_package():
    pkg = os.path.join(ROOT, "paper_2609_04573_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
