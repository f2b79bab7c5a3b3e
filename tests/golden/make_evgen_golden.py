"""Writes evgen_sha256.json: the SHA-256 of the seeded 128x128 stream.

Run from the repository root:  python tests/golden/make_evgen_golden.py
The digest covers (t, x, y, polarity, is_noise) in that order.
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import evgen  # noqa: E402


def main():
    s, _, _, _ = evgen.dvs128(seed=1, n_batches=20)
    h = hashlib.sha256()
    for a in (s.events.t, s.events.x, s.events.y, s.events.p, s.events.is_noise):
        h.update(np.ascontiguousarray(a).tobytes())
    out = {"dvs128_seed1": h.hexdigest(), "n_events": len(s.events)}
    with open(os.path.join(HERE, "evgen_sha256.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(out)


if __name__ == "__main__":
    main()
