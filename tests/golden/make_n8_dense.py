"""Writes n8_dense_exact.json: exact expectation values of the n = 8 workload
(depth-8 Haar SU(4) brickwork, seed 0, two-qubit depolarizing) from the dense
density-matrix oracle, at the base strength p = 1e-3 and without noise.

These are the references of the extrapolation error: a fit over the amplified
levels is compared with the value at p, and a fit over all levels evaluated at
zero noise with the noiseless value.  Only the oracle computes them.

    python tests/golden/make_n8_dense.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, ptm                               # noqa: E402
from paper_2501_13237_amd import workloads                  # noqa: E402


def main():
    w = workloads.plain_fp64_n8(seed=0)
    layers = [[(k, U) for k, U in zip(ls, us)] for ls, us in w.circuit()]
    p = w.noise["dep"]
    rho_p = dense.run_circuit(w.n, layers, ptm.Noise(dep=p))
    rho_0 = dense.run_circuit(w.n, layers, ptm.Noise())
    out = {
        "workload": w.name, "seed": 0, "n": w.n, "p": p,
        "observables": ["".join("IXYZ"[c] for c in o) for o in w.observables],
        "exact_at_p": [float(dense.expectation(rho_p, w.n, o).real) for o in w.observables],
        "exact_noiseless": [float(dense.expectation(rho_0, w.n, o).real) for o in w.observables],
        "source": "oracle.dense (complex128 density matrix, Kraus channels)",
    }
    with open(os.path.join(HERE, "n8_dense_exact.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
