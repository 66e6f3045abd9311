"""Host-side checks of libkxg that need no GPU: the shared library loads,
exports every entry point that include/kxg.h declares, computes its
Gauss-Legendre rule correctly, and rejects bad arguments before any device
work."""
import os
import re

import numpy as np
import pytest

from paper_2607_00755_amd import kxg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "kxg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kxg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = kxg.lib()
    syms = declared_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(kxg.EXPORTED)


def test_library_gauss_legendre_matches_numpy():
    for n in (1, 2, 7, 18, 64, 257):
        x, w = kxg.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 2e-15
        # eigenvector-based weights lose a few digits as n grows
        assert np.max(np.abs(w - wr)) < 1e-14 * max(1.0, n / 8.0) ** 2


@pytest.mark.parametrize("kwargs,msg", [
    (dict(p=[1.0, 2.0, 3.0]), "n=3"),
    (dict(p=[1.0, 2.0, 2.0, 3.0]), "strictly increasing"),
    (dict(p=[-1.0, 2.0, 3.0, 4.0]), "p[0]"),
    (dict(p=[1.0, 2.0, 3.0, 4.0], mass=0.0), "mass"),
    (dict(p=[1.0, 2.0, 3.0, 4.0], n_mu=0), "n_mu"),
    (dict(p=[1.0, 2.0, 3.0, 4.0], b_cap=0), "b_cap"),
    (dict(p=[1.0, 2.0, 3.0, 4.0], dp=[1.0, -1.0, 1.0, 1.0]), "dp[1]"),
    (dict(p=list(np.linspace(1, 2, 1025))), "n=1025"),
])
def test_build_rejects_bad_arguments(kwargs, msg):
    with pytest.raises(kxg.KxgError) as ei:
        kxg.Kernel(**kwargs)
    assert ei.value.status == kxg.EINVAL
    assert msg in str(ei.value)


def test_null_handles_are_rejected():
    L = kxg.lib()
    assert L.kxg_eval(None, 0, None, 1, None, 0, None, None) == kxg.EINVAL
    assert L.kxg_eval_noalloc(None, 0, None, 1, None, 0, None, None) == kxg.EINVAL
    assert L.kxg_stepper_advance(None, 1, None) == kxg.EINVAL
    assert L.kxg_kernel_bytes(None, 0) == 0
    L.kxg_kernel_free(None)
    L.kxg_stepper_free(None)
    assert L.kxg_gauss_legendre(0, None, None) == kxg.EINVAL
    assert b"kxg_gauss_legendre" in L.kxg_last_error()


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2607_00755_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "kxg_oracle" not in src and "liboracle" not in src, fn
