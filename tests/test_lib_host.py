"""CPU checks of the C-ABI library: it loads without a GPU, exports every declared symbol, and
its host-side tables (Daubechies filters, Kaiser-Bessel kernel) match the oracle's."""
import os
import re

import numpy as np
import pytest

from oracle.kb import kb_beta, kb_psi, kb_psi_hat
from oracle.sara import daubechies_lowpass
from paper_1801_02417_amd import psara as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "psara.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(psara_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared_symbols()
    assert len(names) >= 25
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(P.EXPORTS)


def test_wavelet_filters_match_oracle():
    for p in range(1, 9):
        assert np.max(np.abs(P.psara_wavelet_filter(p) - daubechies_lowpass(p))) < 1e-14
    with pytest.raises(ValueError):
        P.psara_wavelet_filter(9)


@pytest.mark.parametrize("taps", [4, 6, 8])
def test_kaiser_bessel_tables_match_oracle(taps):
    b = P.psara_kb_beta(taps, 2.0)
    assert abs(b - kb_beta(taps, 2.0)) < 1e-13
    for t in np.linspace(-taps / 2, taps / 2, 37):
        assert abs(P.psara_kb_value(taps, b, float(t)) - float(kb_psi(t, taps, b))) < 1e-14
    for nu in np.linspace(-0.25, 0.25, 21):
        assert abs(P.psara_kb_deapod(taps, b, float(nu)) * float(kb_psi_hat(nu, taps, b)) - 1.0) < 1e-13


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.PsaraError):
        P.psara_create(0)


def test_footprint_formula_scales():
    a = P.psara_footprint(256, 200000, 8, 4)
    b = P.psara_footprint(512, 1000000, 8, 4)
    assert 30e6 < a < 200e6
    assert b > 3 * a
    assert P.psara_footprint(100, 10, 8, 4) == 0          # not a power of two


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the C-ABI structs have the sizes and field offsets a C compiler
    gives the declarations in include/psara.h."""
    import ctypes as C
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    checks = {"psara_report": (P.PsaraReport, ["residual", "rel_var", "n_p", "iterations"]),
              "psara_stop": (P.PsaraStop, ["theta", "rel_var", "np_max"]),
              "psara_request": (P.PsaraRequest, ["M", "uv", "epsilon", "iters_per_stage", "opnorm_rtol",
                                                 "check_every", "stop"]),
              "psara_result": (P.PsaraResult, ["t_submit", "n", "report"])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "psara.h"', "int main(void) {"]
    for name, (_, fields) in checks.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, (cls, fields) in checks.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f in fields:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
