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


SEG_PROGRAM = r"""
#include "device.hpp"
#include <cstdio>
#include <cstdint>
#include <vector>

using namespace osim;

// a small deterministic generator (xorshift64*) for the segment lengths
static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint32_t rnd() { st ^= st >> 12; st ^= st << 25; st ^= st >> 27; return (uint32_t)((st * 2685821657736338717ull) >> 32); }

template <int NT>
static int check(const std::vector<int> &len) {
    std::vector<int> seg_end(NT);
    long long acc = 0;
    for (int c = 0; c < NT; ++c) { acc += len[c]; seg_end[c] = (int)acc; }
    const int total = (int)acc;
    std::vector<unsigned short> map(2 * NT, 0xffff);
    const int shift = seg_map_shift(total, 2 * NT);
    if (total > 0 && ((total - 1) >> shift) + 1 > 2 * NT - 1) return 1;   // end slot inside the map
    // the segments fill their entries from different threads at once: no
    // entry may be written by two of them
    std::vector<int> writes(2 * NT, 0);
    for (int c = 0; c < NT; ++c) {
        std::vector<unsigned short> own(2 * NT, 0xffff);
        seg_map_fill(own.data(), c, seg_end[c] - len[c], seg_end[c], total, shift);
        for (int j = 0; j < 2 * NT; ++j)
            if (own[j] != 0xffff) {
                if (writes[j]++) return 3;
                map[j] = own[j];
            }
    }
    const int step = total > 4000000 ? 997 : 1;
    for (long long k = 0; k < total; k += step) {
        int want = 0;
        while (seg_end[want] <= k) ++want;   // brute force: first c with seg_end[c] > k
        if (seg_find<NT>(seg_end.data(), map.data(), shift, (int)k) != want) return 2;
    }
    return 0;
}

template <int NT>
static int run() {
    for (int trial = 0; trial < 400; ++trial) {
        std::vector<int> len(NT);
        const int kind = trial % 8;
        for (int c = 0; c < NT; ++c) {
            const uint32_t r = rnd();
            switch (kind) {
                case 0: len[c] = (int)(r % 33); break;                          // ~16 per segment
                case 1: len[c] = (r % 4 == 0) ? (int)(r % 200) : 0; break;      // mostly empty
                case 2: len[c] = (r % 64 == 0) ? (int)(r % 5000) : 0; break;    // sparse and long
                case 3: len[c] = (int)(r % 3); break;                           // very short
                case 4: len[c] = c == (int)(r % NT) ? 100000 : 0; break;        // at most one segment
                case 5: len[c] = (c < NT / 2) ? 0 : (int)(r % 50); break;       // half the chunks absent
                case 6: len[c] = (int)(r % 9000); break;                        // long everywhere
                default: len[c] = (c % 97 == 3) ? 1 : 0; break;                 // isolated single pairs
            }
        }
        if (int e = check<NT>(len)) { printf("NT=%d trial %d kind %d error %d\n", NT, trial, kind, e); return 1; }
    }
    // one huge window (shift > 10) and the empty window
    std::vector<int> big(NT, 0), none(NT, 0);
    for (int c = 0; c < NT; c += 3) big[c] = 400000;
    if (check<NT>(big) || check<NT>(none)) { printf("NT=%d big/none\n", NT); return 1; }
    return 0;
}

int main() {
    if (run<256>() || run<512>()) return 1;
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_segment_map_finds_every_index(tmp_path):
    """The pair walk's coarse segment map and search, against a brute-force
    scan over every flat index, for windows of mixed, mostly empty, very long
    and isolated segments."""
    src = tmp_path / "seg_map.hip"
    exe = tmp_path / "seg_map"
    src.write_text(SEG_PROGRAM)
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-O2", "-I", CSRC,
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
