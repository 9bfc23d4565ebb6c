"""Writes the full-size oracle fixtures the GPU parity tests compare against.

Calls only the FP64 oracle (oracle/) on the seeded synthetic inputs
(paper_1807_02137_amd.synth, which holds no arithmetic of the method):

  c2_oracle_1024.npz  the 1024x1024 twelve-ellipse image (seed 2000), 9 grids,
                      solved to a relative residual of 1e-6: the cycle history,
                      the final segmentation mask (packed bits) and phi at
                      4096 seeded sample pixels;
  c4_oracle_8192_2cycles.npz
                      the 8192x8192 star-polygon image (seed 4000), 14 grids:
                      the relative residuals of the first two cycles, the mask
                      after two cycles (packed bits) and phi at 16384 seeded
                      sample pixels.

Run from the repository root: python tests/golden/make_fullsize.py [c2] [c4]
(c4 takes several minutes and about 12 GB of host memory).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import Oracle, OracleParams  # noqa: E402
from paper_1807_02137_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def samples(n, m, k, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, k), rng.integers(0, m, k)


def c2():
    inst = synth.config2(2000, 1024)
    t0 = time.time()
    o = Oracle(inst.image, inst.markers, OracleParams(levels=9))
    k, hist = o.solve(1e-6, 80)
    phi = o.get("phi")
    si, sj = samples(1024, 1024, 4096, 77)
    np.savez_compressed(os.path.join(HERE, "c2_oracle_1024.npz"), cycles=k, hist=hist,
                        mask=np.packbits(phi > 0), si=si, sj=sj, phi_s=phi[si, sj])
    print(f"c2: {k} cycles, rel {hist[-1]:.3e}, {time.time() - t0:.0f} s", flush=True)


def c4():
    inst = synth.config4(4000, 8192)
    t0 = time.time()
    o = Oracle(inst.image, inst.markers, OracleParams(levels=14))
    print(f"c4: setup {time.time() - t0:.0f} s", flush=True)
    hist = []
    for _ in range(2):
        rel, _ = o.vcycle()
        hist.append(rel)
        print(f"c4: cycle rel {rel:.4e} at {time.time() - t0:.0f} s", flush=True)
    phi = o.get("phi")
    si, sj = samples(8192, 8192, 16384, 78)
    np.savez_compressed(os.path.join(HERE, "c4_oracle_8192_2cycles.npz"), hist=np.array(hist),
                        mask=np.packbits(phi > 0), si=si, sj=sj, phi_s=phi[si, sj])


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c4"]
    if "c2" in which:
        c2()
    if "c4" in which:
        c4()
