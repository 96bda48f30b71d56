"""Write tests/golden/layered128_oracle_traces.npz: FP64 oracle traces of the 128^3 layered
workload (2000 steps, one double-couple source) at a fixed sample of receivers.

Calls only the oracle and the seeded input generators. Run from the repo root:
    python tests/golden/make_layered128_golden.py [--nt 2000]
"""
import argparse
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1705_04874_amd import inputs  # noqa: E402

# every 130th receiver of the 64x64 block (32 receivers spread over the plane)
SAMPLE = np.arange(0, 4096, 130)[:32]


def model_digest(w):
    h = hashlib.sha256()
    for a in (w.model.vp, w.model.vs, w.model.rho, w.src_ijk, w.src_m, w.wavelet, w.rec):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nt", type=int, default=2000)
    ap.add_argument("--out", default=os.path.join(ROOT, "tests", "golden", "layered128_oracle_traces.npz"))
    a = ap.parse_args()
    w = inputs.layered128_workload(nt=a.nt)
    s = oracle.Solver.from_workload(w, rec=w.rec[SAMPLE])
    s.set_sources(w.src_ijk, w.src_m, w.wavelet)
    t = time.time()
    chunks = []
    done = 0
    while done < a.nt:
        k = min(100, a.nt - done)
        chunks.append(s.run(k))
        done += k
        print(f"step {done}/{a.nt}  {time.time() - t:.0f}s", flush=True)
    tr = np.concatenate(chunks, axis=2)
    np.savez_compressed(a.out, traces=tr, receivers=SAMPLE, nt=a.nt, digest=model_digest(w))
    print("wrote", a.out, tr.shape, f"{time.time() - t:.0f}s")


if __name__ == "__main__":
    main()
