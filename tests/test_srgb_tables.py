"""The sRGB encode tables the GPU kernel uses (paper_2503_01074_amd/csrc/
srgb_tables.hpp, written by gen_srgb_tables.py, independently of the
oracle): the kernel's lookup (a first-guess code from the float's exponent
and top seven mantissa bits, then one threshold comparison) emulated in
numpy on the CPU gives the oracle's 8-bit code on every threshold and its
neighbours, octave boundaries, random values and special values."""
import os
import re

import numpy as np

from oracle import camera_io as cio

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2503_01074_amd", "csrc",
                   "srgb_tables.hpp")


def _tables():
    text = open(HDR).read()

    def block(name):
        m = re.search(r"%s\[\d+\] = \{(.*?)\};" % name, text, re.S)
        return [v.strip() for v in m.group(1).replace("\n", " ").split(",") if v.strip()]

    thr = np.array([float.fromhex(v.rstrip("f")) for v in block("kSrgbThreshold")], np.float32)
    guess = np.array([int(v) for v in block("kSrgbGuess")], np.int64)
    e0 = int(re.search(r"kSrgbGuessE0 = (\d+);", text).group(1))
    return thr, guess, e0


def _kernel_codes(x):
    thr, guess, e0 = _tables()
    thr = np.concatenate([thr, [np.float32(np.inf)]])
    x = np.asarray(x, np.float32)
    with np.errstate(invalid="ignore"):
        idx = (x.view(np.uint32) >> 16).astype(np.int64) - (e0 << 7)
        idx = np.clip(idx, 0, guess.shape[0] - 1)
        q = guess[idx]
        q = q + (x >= thr[q + 1])
        return np.where(x >= 1.0, 255, np.where(x >= np.float32(2.0 ** -13), q, 0))


def test_lookup_matches_oracle_codes():
    thr, _, _ = _tables()
    t = thr[1:]
    up, down = np.float32(np.inf), np.float32(-np.inf)
    pts = [t, np.nextafter(t, down), np.nextafter(t, up)]
    octaves = np.float32(2.0) ** np.arange(-20, 2, dtype=np.float32)
    pts += [octaves, np.nextafter(octaves, down), np.nextafter(octaves, up)]
    rs = np.random.default_rng(5)
    pts.append(rs.uniform(-0.1, 1.1, 200000).astype(np.float32))
    pts.append(np.exp(rs.uniform(np.log(1e-6), 0.0, 200000)).astype(np.float32))
    pts.append(np.array([0.0, -0.0, 1.0, np.nextafter(np.float32(1.0), down), np.inf, -np.inf, np.nan, -1.0,
                         1e-30, 2.0 ** -13, 3.4e38], np.float32))
    x = np.concatenate(pts).astype(np.float32)
    want = cio.encode_codes(x)
    got = _kernel_codes(x)
    np.testing.assert_array_equal(got, want)


def test_one_comparison_suffices():
    thr, guess, e0 = _tables()
    # every bucket: the code of its largest float is at most one above its guess
    i = np.arange(guess.shape[0], dtype=np.uint32)
    hi = (((e0 << 7) + i) << 16 | 0xFFFF).astype(np.uint32).view(np.float32)
    assert np.all(cio.encode_codes(hi) - guess <= 1)
