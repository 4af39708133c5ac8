"""Write the seeded mock images the GPU tests and the benchmark load.

Calls only the oracle's mock-data synthesis and the seeded draws; run from
the repository root:  python tests/data/make_inputs.py [name ...]
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


def main(names=("c1", "c2", "c4", "large")):
    mpath = os.path.join(HERE, "MANIFEST.json")
    manifest = {}
    if os.path.exists(mpath):
        with open(mpath) as f:
            manifest = json.load(f)
    for name in names:
        w = synthgen.WORKLOADS[name]
        D = mock.workload_data(w)
        path = os.path.join(HERE, f"{name}.npz")
        # the large image is stored rounded to FP32 (half the bytes); both the
        # oracle and the GPU read these stored values
        d = D["d"].astype(np.float32) if name == "large" else D["d"]
        np.savez(path, d=d, sigma=np.float64(D["sigma"]), psf=D["psf"], lens=D["lens"])
        with open(path, "rb") as f:
            manifest[f"{name}.npz"] = hashlib.sha256(f.read()).hexdigest()
    with open(mpath, "w") as f:
        json.dump(manifest, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("c1", "c2", "c4", "large"))
