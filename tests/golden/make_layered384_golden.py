"""Write tests/golden/layered384_oracle_planes.npz: the FP64 oracle's state of the
384 x 384 x 256 layered workload (one double-couple source) after NT steps, on three
planes through the source, every second cell of a 128 x 128 window (all 24 split
fields, stored rounded to float32).

At NT = 150 steps (0.12 s) the source has radiated its whole 25 Hz Ricker pulse
and the wavefield reaches about 30 cells from the source, well inside the windows;
the receivers at the seabed have not seen it yet, so the state is what is compared.

Calls only the oracle and the seeded input generators.  Run from the repo root
(about 42 s per step on 8 host threads, 15 GB of memory):
    python tests/golden/make_layered384_golden.py [--nt 150]
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1705_04874_amd import inputs  # noqa: E402

HALF = 64      # window half-width in cells
STRIDE = 2     # every second cell of the window


def planes(w):
    """(name, z-slice, y-slice, x-slice) of the three sampled planes through the source."""
    i, j, k = (int(v) for v in w.src_ijk[0])
    nz, ny, nx = w.model.shape

    def win(c, n):
        a = max(0, c - HALF)
        return slice(a, min(n, a + 2 * HALF), STRIDE)

    return [("xy", slice(k, k + 1), win(j, ny), win(i, nx)),
            ("xz", win(k, nz), slice(j, j + 1), win(i, nx)),
            ("yz", win(k, nz), win(j, ny), slice(i, i + 1))]


def main():
    from tests.golden.make_layered128_golden import model_digest
    ap = argparse.ArgumentParser()
    ap.add_argument("--nt", type=int, default=150)
    ap.add_argument("--out", default=os.path.join(ROOT, "tests", "golden", "layered384_oracle_planes.npz"))
    a = ap.parse_args()
    w = inputs.layered384_workload(nt=a.nt)
    s = oracle.Solver.from_workload(w, rec=w.rec[:1])
    s.set_sources(w.src_ijk, w.src_m, w.wavelet)
    t = time.time()
    done = 0
    while done < a.nt:
        k = min(10, a.nt - done)
        s.run(k)
        done += k
        print(f"step {done}/{a.nt}  {time.time() - t:.0f}s", flush=True)
    st = s.get_state()
    s.close()
    out = {"nt": a.nt, "digest": model_digest(w)}
    for name, zs, ys, xs in planes(w):
        out[name] = st[:, zs, ys, xs].astype(np.float32)
    del st
    np.savez_compressed(a.out, **out)
    print("wrote", a.out, {k: v.shape for k, v in out.items() if hasattr(v, "shape")}, f"{time.time() - t:.0f}s")


if __name__ == "__main__":
    main()
