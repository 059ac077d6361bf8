"""Write the FP64 oracle's image of the headline workload (128 x 128 warped
sensors with +-5 % jitter on a 25 mm plane, 2048 samples at 60 MHz, 40-tube
vessel phantom, 256^3 output; seed 1002) for the full-image GPU parity test.

Only the oracle computes it: the seeded input generator, then
oracle.reconstruct, the plain non-uniform DFT of Section 2, eq. disc_rec,
followed by the equispaced inverse transform (the direct-FT ground truth of
Section 5.1). Nothing here touches the GPU path.

Output, next to this script:
  headline_oracle_image.npy   float32 [256, 256, 256] (about 64 MiB; not kept
                              in version control, regenerate with this script)
  headline_oracle_image.json  SHA-256 of the .npy, the FP64 image's L2 norm and
                              largest magnitude, the rounding of the float32
                              copy, the host and the time taken (kept in
                              version control)

The float32 copy differs from the FP64 image by at most half a unit in the
last place (about 3e-8 relative), far below the 1e-5 bound it is used for.
Run: python tests/golden/make_headline_image.py   (about 5 minutes on 8 cores)
"""
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1510_01078_amd import inputs  # noqa: E402

NPY = os.path.join(HERE, "headline_oracle_image.npy")
META = os.path.join(HERE, "headline_oracle_image.json")


def sha256(path):
    h = hashlib.sha256()
    with open(path, "rb") as fh:
        for blk in iter(lambda: fh.read(1 << 22), b""):
            h.update(blk)
    return h.hexdigest()


def main():
    t0 = time.time()
    p = inputs.config_problem(2)
    t1 = time.time()
    f = oracle.reconstruct(p.xy, p.h, p.g, p.dt, p.c, p.shape, p.extent)
    t2 = time.time()
    f32 = f.astype(np.float32)
    np.save(NPY, f32)
    meta = {
        "workload": "128x128 warped sensors (+-5% jitter) on 25 mm, 2048 samples at 60 MHz, "
                    "40-tube vessel phantom -> 256^3 (seed 1002)",
        "file": os.path.basename(NPY),
        "dtype": "float32",
        "shape": list(f32.shape),
        "sha256": sha256(NPY),
        "l2_norm_fp64": float(np.linalg.norm(f.ravel())),
        "max_abs_fp64": float(np.abs(f).max()),
        "float32_copy_rel_l2": float(np.linalg.norm((f32.astype(np.float64) - f).ravel()) / np.linalg.norm(f.ravel())),
        "seconds_inputs": round(t1 - t0, 1),
        "seconds_oracle": round(t2 - t1, 1),
        "host": f"{platform.processor() or platform.machine()}, {os.cpu_count()} CPUs",
        "command": "python tests/golden/make_headline_image.py",
    }
    with open(META, "w") as fh:
        json.dump(meta, fh, indent=1)
        fh.write("\n")
    print(json.dumps(meta, indent=1))


if __name__ == "__main__":
    main()
