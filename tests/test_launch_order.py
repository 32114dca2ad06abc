"""Workgroup numbering of the tile launches, checked on the host.

The kernels that walk polar tiles renumber their workgroups so that each XCD
takes runs of consecutive tiles (`xcd_grouped_id`), and the fused launches
interleave tile and camera workgroups through the dispatch order
(`fused_slot`).  Both decide which work a workgroup does, so each must be a
bijection: every tile and every camera group taken exactly once, whatever the
grid size.  The helpers are host-callable; this test compiles them for the
host with hipcc (no GPU code, no GPU needed) and checks those properties.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_01074_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "device.hpp"
#include <cstdio>
#include <vector>

using namespace osim;

template <int G>
static int check_grouped(int n) {
    std::vector<int> seen(n, 0);
    for (int b = 0; b < n; ++b) {
        const int x = xcd_grouped_id<G>(b, n);
        if (x < 0 || x >= n || seen[x]++) return 1;
    }
    // within every full round of kXcds * G workgroups, the workgroups one XCD
    // receives (b % kXcds equal) take G consecutive ids, in dispatch order
    const int round = kXcds * G;
    for (int r0 = 0; r0 + round <= n; r0 += round)
        for (int xcd = 0; xcd < kXcds; ++xcd)
            for (int k = 0; k < G; ++k)
                if (xcd_grouped_id<G>(r0 + xcd + k * kXcds, n) != r0 + xcd * G + k) return 2;
    return 0;
}

static int check_fused(int n_tile, int n_cam) {
    const int n = n_tile + n_cam;
    std::vector<int> tiles(n_tile, 0), cams(n_cam, 0);
    long long last_cam = -1, max_gap = 0;
    for (long long x = 0; x < n; ++x) {
        const FusedSlot s = fused_slot(x, n_tile, n_cam);
        if (s.cam) {
            if (s.index < 0 || s.index >= n_cam || cams[s.index]++) return 3;
            if (last_cam >= 0 && x - last_cam > max_gap) max_gap = x - last_cam;
            last_cam = x;
        } else {
            if (s.index < 0 || s.index >= n_tile || tiles[s.index]++) return 4;
        }
    }
    for (int v : tiles) if (v != 1) return 5;
    for (int v : cams) if (v != 1) return 6;
    // camera workgroups evenly spread: consecutive ones at most ceil(N / C) apart
    if (n_cam > 0 && max_gap > (n + n_cam - 1) / n_cam) return 7;
    return 0;
}

int main() {
    for (int n = 0; n <= 4200; ++n) {
        if (int e = check_grouped<8>(n)) { printf("grouped<8> n=%d error %d\n", n, e); return 1; }
        if (int e = check_grouped<16>(n)) { printf("grouped<16> n=%d error %d\n", n, e); return 1; }
    }
    const int big[] = {32768, 32771, 1000003};
    for (int n : big)
        if (check_grouped<16>(n)) { printf("grouped<16> n=%d\n", n); return 1; }
    const int tiles[] = {0, 1, 2, 7, 64, 255, 1000, 32768};
    const int cams[] = {0, 1, 3, 64, 257, 1000, 4096};
    for (int t : tiles)
        for (int c : cams)
            if (t + c > 0)
                if (int e = check_fused(t, c)) { printf("fused t=%d c=%d error %d\n", t, c, e); return 1; }
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_workgroup_numbering_is_a_bijection(tmp_path):
    src = tmp_path / "launch_order.hip"
    exe = tmp_path / "launch_order"
    src.write_text(PROGRAM)
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O2", "-I", CSRC,
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
