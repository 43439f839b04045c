"""Writes alg1_nedelec_hex_64.txt: the oracle's Algorithm 1 on the full-size
Nedelec benchmark problem (nedelec_hex(64), 262,144 patches of 12 dofs,
spectral criterion, eps = 1e-8), run once as the sequential loop: the entry
count, the number of criterion evaluations, and SHA-256 digests of phi and
of the entries' patch ids (int32, little-endian), so that a test can compare
every one of the 262,144 assignments without storing them.

Calls only the generators and the oracle.  About half an hour on one core:
    python tests/golden/make_alg1_nedelec64.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle as O  # noqa: E402

EPS = 1e-8


def main():
    t0 = time.time()
    P = gen.nedelec_hex(64)
    tiles = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(tiles, EPS, "spectral")
    phi = np.asarray(res["phi"], dtype="<i4")
    reps = np.asarray(res["reps"], dtype="<i4")
    lines = [
        "# Algorithm 1 (spectral criterion, eps = 1e-8) on nedelec_hex(64) by the",
        "# oracle's sequential loop; written by make_alg1_nedelec64.py.",
        "# phi_sha256 / reps_sha256: SHA-256 of the int32 little-endian arrays.",
        f"n_p {P.n_p}",
        f"m_p {len(reps)}",
        f"evals {res['evals']}",
        f"margin {res['margin']:.6e}",
        f"phi_sha256 {hashlib.sha256(phi.tobytes()).hexdigest()}",
        f"reps_sha256 {hashlib.sha256(reps.tobytes()).hexdigest()}",
        "reps_head " + ",".join(str(int(v)) for v in reps[:16]),
        "reps_tail " + ",".join(str(int(v)) for v in reps[-8:]),
    ]
    with open(os.path.join(HERE, "alg1_nedelec_hex_64.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines), f"\n{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
