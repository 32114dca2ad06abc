"""Tolerances of the parity tests.

Images (polar, fan, camera): per element |gpu - oracle| <= 1e-5 * max(|oracle|,
1e-3 * max|oracle|), i.e. 1e-5 relative with a floor at 1e-3 of the image's
peak for elements near zero.  Bin indices: bit-exact.

Gradients: per component |gpu - reference| <= 1e-3 * max(|reference|, 1e-3 *
max|reference|) against FP64 central differences and against the FP64
oracle's analytic gradient (which is itself pinned to central differences);
the floor (1e-3 of the largest component of the same vector) only governs
vectors of like quantities (the reflectivity table), scalar parameters are
each held to 1e-3 of their own magnitude.  Parameter gradients are sums of
many float32 terms of both signs, so the parity tests also hold each
component to 1e-5 of the sum of the magnitudes of its terms (the condition of
the sum, reported by the oracle), a bound that is tighter than 1e-3 relative
wherever the sum does not cancel more than a hundredfold.
"""
import numpy as np

IMG_RTOL = 1e-5
IMG_FLOOR = 1e-3
GRAD_RTOL_ORACLE = 1e-5
GRAD_RTOL_FD = 1e-3


def rel_report(got, want, rtol=IMG_RTOL, floor=IMG_FLOOR, mask=None):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    if mask is not None:
        got, want = got[mask], want[mask]
    if want.size == 0:
        return 0, 0.0
    peak = np.abs(want).max()
    scale = np.maximum(np.abs(want), floor * peak)
    err = np.abs(got - want)
    bad = err > rtol * scale
    with np.errstate(divide="ignore", invalid="ignore"):
        worst = float(np.nanmax(np.where(scale > 0, err / scale, np.where(err > 0, np.inf, 0.0))))
    return int(bad.sum()), worst


def assert_image_close(got, want, what="", rtol=IMG_RTOL, floor=IMG_FLOOR, mask=None):
    nbad, worst = rel_report(got, want, rtol, floor, mask)
    assert nbad == 0, "%s: %d elements beyond %.1e relative (worst %.3e)" % (what, nbad, rtol, worst)
    return worst


def assert_grad_close(got, want, rtol, what=""):
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    peak = np.abs(want).max() if want.size else 0.0
    scale = np.maximum(np.abs(want), 1e-3 * peak)
    err = np.abs(got - want)
    ok = err <= rtol * scale + 1e-30
    assert ok.all(), "%s: got %s want %s (rel %s)" % (what, got[~ok], want[~ok], (err / np.maximum(scale, 1e-300))[~ok])


def assert_grad_scalars(got, want, rtol=GRAD_RTOL_FD, what=""):
    """|got - want| <= rtol * |want| per component (scalar parameters of
    different units: no shared floor; an exact zero must come out zero)."""
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    err = np.abs(got - want)
    ok = err <= rtol * np.abs(want) + 1e-30
    assert ok.all(), "%s: got %s want %s (rel %s)" % (what, got[~ok], want[~ok],
                                                     (err / np.maximum(np.abs(want), 1e-300))[~ok])


def assert_grad_cond(got, want, cond, rtol=GRAD_RTOL_ORACLE, what=""):
    """|got - want| <= rtol * cond per component, cond = sum of |terms|."""
    got = np.asarray(got, np.float64).ravel()
    want = np.asarray(want, np.float64).ravel()
    cond = np.asarray(cond, np.float64).ravel()
    err = np.abs(got - want)
    ok = err <= rtol * cond + 1e-30
    assert ok.all(), "%s: got %s want %s err/cond %s" % (what, got[~ok], want[~ok],
                                                        (err / np.maximum(cond, 1e-300))[~ok])
