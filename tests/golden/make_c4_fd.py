"""Writes c4_central_differences.json: FP64 central differences of the
oracle's forward pass on the differentiable batch (see tests/_fd.py for the
loss, the parameters and the step sizes).  Calls only the oracle and the
seeded input generators.

    python tests/golden/make_c4_fd.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import _fd  # noqa: E402


def main():
    fd = _fd.c4_central_differences()
    rec = {
        "what": "FP64 central differences of L = sum <w, polar> + <w, fan> + <w, camera> on the differentiable "
                "batch (32 sonar frames 512x64 returns, 64 materials, 512x512 bins, 512x1024 fan, paper speckle; "
                "32 camera frames 960x540, one water row); loss weights keys (202, k), (203, k), (204, k)",
        "sonar_keys": list(_fd.SONAR_KEYS),
        "sonar": [float(v) for v in fd["sonar"]],
        "refl": {str(m): float(v) for m, v in fd["refl"].items()},
        "water_keys": ["beta_d0", "beta_d1", "beta_d2", "beta_b0", "beta_b1", "beta_b2",
                       "b_inf0", "b_inf1", "b_inf2"],
        "water": [float(v) for v in fd["water"]],
    }
    with open(os.path.join(HERE, "c4_central_differences.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
