"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/af.h declares, and fails loudly (no fallback) without a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def declared_functions():
    src = open(os.path.join(ROOT, "include", "af.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("af_create", "af_destroy", "af_set_state", "af_get_state", "af_step", "af_residual",
                     "af_norms", "af_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2510_11527_amd import af
    L = af.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(af.EXPORTS) == declared_functions()


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2510_11527_amd import af
    from paper_2510_11527_amd import workloads as W
    spec, _ = W.config2(n=8)
    with pytest.raises(af.AFError) as e:
        af.Context(spec)
    assert e.value.status in (af.AF_ERR_DEVICE, af.AF_ERR_ALLOC)


def test_invalid_problem_rejected_before_device_use():
    from paper_2510_11527_amd import af
    from paper_2510_11527_amd import workloads as W
    spec, _ = W.config2(n=8)
    with pytest.raises(af.AFError) as e:
        af.Context(dict(spec, n=[2, 8]))
    assert e.value.status == af.AF_ERR_ARG
    with pytest.raises(af.AFError) as e:
        af.Context(dict(spec, cfl=0.5))
    assert e.value.status == af.AF_ERR_CFL
    with pytest.raises(af.AFError) as e:
        af.Context([spec, dict(spec, precision=32)])
    assert e.value.status == af.AF_ERR_UNSUPPORTED


def test_package_has_no_oracle_dependency():
    """The product path never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2510_11527_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".hpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liborc" not in txt and "af_oracle" not in txt, f
