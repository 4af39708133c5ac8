"""Write the seeded mock images the GPU tests and the benchmark load.

Calls only the oracle's mock-data synthesis and the seeded draws; run from
the repository root:  python tests/data/make_inputs.py
Each workload file holds d (ny, nx), sigma, psf (K, K) and the true lens;
MANIFEST.json records their SHA-256.
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthgen  # noqa: E402
from oracle import mock  # noqa: E402


def main():
    manifest = {}
    for name in ("c1", "c2", "c4"):
        w = synthgen.WORKLOADS[name]
        D = mock.workload_data(w)
        path = os.path.join(HERE, f"{name}.npz")
        np.savez(path, d=D["d"], sigma=np.float64(D["sigma"]), psf=D["psf"], lens=D["lens"])
        with open(path, "rb") as f:
            manifest[f"{name}.npz"] = hashlib.sha256(f.read()).hexdigest()
    with open(os.path.join(HERE, "MANIFEST.json"), "w") as f:
        json.dump(manifest, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
