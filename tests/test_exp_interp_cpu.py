"""The FP64 exponential of the exact-form stream's log interpolation (Tang's
table-driven method, written out in kxg_eval.hip as `exp_interp`): its
reduction constants and polynomial, read from the source and run here in
numpy with the kernel's operation order, against numpy's exp over the whole
range the interpolation reaches (ln 1e-300 .. ln 1e3).  The GPU parity tests
check the kernel's results against the oracle; this pins the method's own
error bound on the CPU."""
import os
import re
from decimal import Decimal, getcontext

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2607_00755_amd", "csrc", "kxg_eval.hip")
LN2 = Decimal("0.693147180559945309417232121458176568075500134360255254120680009")


def _constants(kind):
    text = open(SRC).read()
    head = "__device__ inline %s exp_interp(%s x" % (kind, kind)
    body = text[text.index(head):]
    body = body[:body.index("\n}\n")]
    nums = re.findall(r"(?<![\w.])(\d+\.\d+(?:e[-+]?\d+)?)f?", body)
    return body, [float(x) for x in nums]


def test_reduction_constants_split_ln2_over_32():
    getcontext().prec = 60
    for kind, bits in (("double", 38),):
        body, nums = _constants(kind)
        inv, l1, l2 = nums[0], nums[1], nums[2]
        assert abs(Decimal(inv) - 32 / LN2) / (32 / LN2) < Decimal("1e-7")
        # L1 + L2 = ln2/32 to the working precision, L1 short enough that
        # N L1 is exact for |N| < 2^15
        assert abs(Decimal(l1) + Decimal(l2) - LN2 / 32) < Decimal("1e-22")
        m, e = np.frexp(l1)
        assert float(m * 2.0 ** bits).is_integer()


def _tang(x, kind):
    body, nums = _constants(kind)
    dt = np.float64 if kind == "double" else np.float32
    inv, l1, l2 = (dt(v) for v in nums[:3])
    coef = [dt(1.0 / 120.0), dt(1.0 / 24.0), dt(1.0 / 6.0), dt(0.5), dt(1.0)]
    t32 = np.array([2.0 ** (j / 32.0) for j in range(32)]).astype(dt)
    x = x.astype(dt)
    nd = np.rint(x * inv).astype(dt)
    r = (x - nd * l1).astype(dt)
    r = (r - nd * l2).astype(dt)
    p = coef[0]
    for c in coef[1:]:
        p = (p * r + c).astype(dt)
    p = (p * r).astype(dt)
    n = nd.astype(np.int64)
    tj = t32[n & 31]
    return np.ldexp((tj + tj * p).astype(dt), (n >> 5).astype(np.int32)).astype(dt)


def test_fp64_error_bound():
    rng = np.random.default_rng(7)
    x = np.concatenate([np.linspace(np.log(1e-300), np.log(1e3), 400001),
                        rng.uniform(np.log(1e-300), np.log(1e3), 200000)])
    rel = np.abs(_tang(x, "double") - np.exp(x)) / np.exp(x)
    assert rel.max() < 1e-14
