"""Accuracy of the FP32 log1p and expm1 that the FP32 constitutive update and
its adjoint use (hardware base-2 logarithm and exponential with the Goldberg
and Kahan corrections), through the C-ABI, against numpy's float64 routines on
the same float32 inputs: relative error within a few float32 ulp over the
ranges the kernels see (principal strains and their differences, |x| up to
about 1) and beyond, exact results where the identities make them exact."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -23
BOUND_ULP = 4.0


def _inputs(lo, hi, n=200_000, seed=1):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return (sign * mag).astype(np.float32)


@pytest.fixture(scope="module")
def ddm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_17335_amd as m
    return m


def _eval(ddm, fn, x):
    import torch
    y = ddm.eval_math(fn, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _ulp_error(got, want):
    # error in units of the float32 spacing at the exact result
    return np.abs(got.astype(np.float64) - want) / (np.abs(want) * EPS32)


@pytest.mark.parametrize("fn,lo,hi", [("log1p", 1e-12, 0.999), ("log1p", 1.0, 1e30),
                                      ("expm1", 1e-12, 1.0), ("expm1", 1.0, 80.0)])
def test_relative_error_within_bound(ddm, fn, lo, hi):
    x = _inputs(lo, hi)
    if fn == "log1p" and lo >= 1.0:
        x = np.abs(x)                       # log1p needs x > -1
    want = getattr(np, fn)(x.astype(np.float64))
    got = _eval(ddm, fn, x)
    err = _ulp_error(got, want)
    k = int(np.argmax(err))
    print(f"{fn} |x| in [{lo:g}, {hi:g}]: max error {err[k]:.2f} ulp at x = {x[k]!r}", flush=True)
    sys.stdout.flush()
    assert err[k] <= BOUND_ULP, (fn, x[k], got[k], want[k])


def test_special_values(ddm):
    x = np.array([0.0, -0.0, 1e-30, -1e-30, np.inf, np.nan, -1.0, -2.0], dtype=np.float32)
    lp = _eval(ddm, "log1p", x)
    assert lp[0] == 0.0 and lp[2] == np.float32(1e-30) and lp[3] == np.float32(-1e-30)
    assert lp[4] == np.inf and np.isnan(lp[5]) and lp[6] == -np.inf and np.isnan(lp[7])
    x = np.array([0.0, 1e-30, -1e-30, 100.0, -100.0, np.inf, -np.inf, np.nan], dtype=np.float32)
    em = _eval(ddm, "expm1", x)
    assert em[0] == 0.0 and em[1] == np.float32(1e-30) and em[2] == np.float32(-1e-30)
    assert em[3] == np.inf and em[4] == -1.0 and em[5] == np.inf and em[6] == -1.0 and np.isnan(em[7])


def test_empty_and_errors(ddm):
    import torch
    y = ddm.eval_math("log1p", torch.zeros(0, device="cuda"))
    assert y.numel() == 0
    with pytest.raises(ValueError):
        ddm.eval_math("log1p", torch.zeros(4, dtype=torch.float64, device="cuda"))
