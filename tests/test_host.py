"""CPU-side checks of the library boundary: the shared library loads and
exports every symbol the header declares; host-only helpers."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fppr.h")).read()
    return sorted(set(re.findall(r"FPPR_API\s+[\w\s\*]+?\b(fppr_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1903_11749_amd import fppr

    lib_path = fppr.LIB_PATH
    assert os.path.exists(lib_path), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (fppr_\w+)", out))
    declared = declared_symbols()
    assert declared, "no declarations found"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    # the binding knows every declared call, with the same names
    assert sorted(set(fppr.exported_symbols())) == declared
    fppr.lib()  # loads (no GPU needed to load)


def test_alpha_threshold_and_guarantee_helpers():
    from paper_1903_11749_amd import fppr

    assert fppr.fppr_alpha_threshold(0.15) == 644245094
    assert fppr.fppr_alpha_threshold(0.5) == 2**31
    assert fppr.fppr_alpha_threshold(1e-12) == 1
    assert fppr.fppr_alpha_threshold(0.0) == 0 and fppr.fppr_alpha_threshold(1.0) == 0
    eps, delta, pf = 0.5, 0.5, 1e-6
    want = math.ceil((2 + 2 * eps / 3) * math.log(2 / pf) / (eps**2 * delta))
    assert fppr.fppr_walks_for_guarantee(eps, delta, pf) == want
    assert fppr.fppr_walks_for_guarantee(0, 0.5, 0.1) == 0


def test_threshold_agrees_with_oracle_definition():
    """Both sides define T(alpha) independently; they agree on a sweep."""
    from oracle import oracle as O
    from paper_1903_11749_amd import fppr

    for a in np.concatenate([np.linspace(1e-6, 1 - 1e-6, 997), [0.1, 0.15, 0.2, 0.5]]):
        assert fppr.fppr_alpha_threshold(float(a)) == O.alpha_threshold(float(a))
