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


def test_empty_batch_rejected_before_device_use():
    """A batch of no instances, or a missing problem array or handle, is an
    argument error, returned before any device call."""
    import ctypes
    from paper_2510_11527_amd import af
    from paper_2510_11527_amd import workloads as W
    spec, _ = W.config2(n=8)
    arr = (af.AfProblem * 1)(af.make_problem(spec, None, "ssprk3"))
    h = ctypes.c_void_p()
    assert af.lib().af_create(0, arr, ctypes.byref(h)) == af.AF_ERR_ARG
    assert af.lib().af_create(1, None, ctypes.byref(h)) == af.AF_ERR_ARG
    assert af.lib().af_create(1, arr, None) == af.AF_ERR_ARG
    assert not h.value


def test_package_has_no_oracle_dependency():
    """The product path never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2510_11527_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".hpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liborc" not in txt and "af_oracle" not in txt, f


def test_new_problem_fields_validated_before_device_use():
    """The diffusion form and the ends are checked by af_create before any
    device call."""
    from paper_2510_11527_amd import af
    from paper_2510_11527_amd import workloads as W
    s2, _ = W.config2(n=8)
    s1, _ = W.config_ek(n_inst=1, n=16)[0]
    s3, _ = W.config5(n=4)
    cases = [
        (dict(s2, diffusion_form="nodc"), af.AF_ERR_UNSUPPORTED),       # App. A is 1D
        (dict(s1, bc=("periodic", "outflow")), af.AF_ERR_ARG),          # both ends periodic or neither
        (dict(s1, bc=(("dirichlet", 1.5), "outflow")), af.AF_ERR_BOUNDS),
        (dict(s1, bc=(("dirichlet", float("nan")), "outflow")), af.AF_ERR_ARG),
        (dict(s3, bc=("outflow", "outflow")), af.AF_ERR_UNSUPPORTED),   # no 3D open ends
        (dict(s2, si=True, bcs=[("outflow", "outflow"), ("periodic", "periodic")]), af.AF_ERR_UNSUPPORTED),
        (dict(s1, bcs=[("outflow", "outflow"), ("outflow", "outflow")]), af.AF_ERR_ARG),  # unused axis
    ]
    for spec, status in cases:
        with pytest.raises(af.AFError) as e:
            af.Context(spec)
        assert e.value.status == status, (spec.get("bc"), spec.get("bcs"), e.value)


def test_problem_struct_layout_matches_the_header(tmp_path):
    """The ctypes mirror of af_problem / af_norms_t has the C layout: a C
    program compiled against include/af.h prints sizes and offsets."""
    import subprocess
    from paper_2510_11527_amd import af
    fields = [f for f, _ in af.AfProblem._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "af.h"', 'int main(void) {',
           '  printf("%zu %zu\\n", sizeof(af_problem), sizeof(af_norms_t));']
    src += ['  printf("%%zu\\n", offsetof(af_problem, %s));' % f for f in fields]
    src += ['  return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == ctypes.sizeof(af.AfProblem)
    assert int(out[1]) == ctypes.sizeof(af.AfNorms)
    for f, off in zip(fields, out[2:]):
        assert int(off) == getattr(af.AfProblem, f).offset, f
