"""Kernel resources of the built library, from the compiler's
kernel-resource-usage remarks that the build records next to the objects
(`_build/*.resources.json`; skipped when the library has not been built here).

A kernel whose per-thread arrays end up in per-lane stack memory runs many
times slower (a fan-operator backward variant once kept 608 bytes per lane and
ran 12x slower on large batches), so every kernel must keep its state in
registers: the only stack allowed is a couple of register spills under an
explicit occupancy bound.
"""
import glob
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = sorted(glob.glob(os.path.join(ROOT, "_build", "*.hip.resources.json")))


def _kernels():
    out = {}
    for path in REPORTS:
        with open(path) as fh:
            out.update(json.load(fh))
    return out


@pytest.mark.skipif(not REPORTS, reason="library not built in this tree")
def test_no_kernel_keeps_arrays_on_the_stack():
    ks = _kernels()
    assert len(ks) > 20
    big = {k: v.get("scratch_bytes_per_lane", 0) for k, v in ks.items() if v.get("scratch_bytes_per_lane", 0) > 16}
    assert not big, big


@pytest.mark.skipif(not REPORTS, reason="library not built in this tree")
def test_plan_hot_kernels_have_no_spills():
    ks = _kernels()
    hot = [k for k in ks if any(n in k for n in ("k_fant_bwd", "k_ret_uw_bwd", "k_bin_uw", "k_cam_", "6k_tileI", "5k_fanI",
                                                  "k_uw_bwd", "4k_uwI"))]
    assert len(hot) >= 10
    for k in hot:
        assert ks[k].get("scratch_bytes_per_lane", 0) == 0, k
        assert ks[k].get("vgpr_spills", 0) == 0, k
        assert ks[k].get("waves_per_simd", 0) >= 2, k
