"""Writes synth_manifest.json: the SHA-256 of every synthetic image of the
workload presets, so a run on another machine can check it feeds the same
bytes (numpy's generator or FFT could differ).  Calls only the input
generator.  Run from the repository root: python tests/golden/make_synth_manifest.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1502_00324_amd.configs import WORKLOADS  # noqa: E402
from paper_1502_00324_amd.synth import make_image, sha256  # noqa: E402


def main():
    out = {}
    for name, wl in sorted(WORKLOADS.items()):
        out[name] = [{"seed": s, "width": w, "height": h, "n_rect": n, "sha256": sha256(make_image(s, w, h, n))}
                     for (s, w, h, n) in wl.images]
    with open(os.path.join(HERE, "synth_manifest.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
