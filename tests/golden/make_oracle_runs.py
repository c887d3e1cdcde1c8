"""Writes oracle results of the larger workloads, which the oracle needs
minutes for, as stored expectations for the GPU parity tests:

* ``n32_d20_oracle.json``: the n = 32 chain, depth-20 Haar SU(4) brickwork
  (seed 0) with two-qubit depolarizing 1e-3 followed by amplitude damping
  5e-4 on each qubit, one noise level, chi in {64, 128, 256}: every <Z_i>,
  the emulation fidelity, the trace and the smallest relative cut gap.
* ``n50_d24_oracle.json``: the n = 50 chain, depth-24 brickwork (seed 0)
  with two-qubit depolarizing at the eight levels (1 + 15 j / 7) x 1e-3,
  chi = 256: every <Z_i> and <X_1 X_2> at every level, fidelities, traces,
  smallest cut gaps.

Both runs use the float64 oracle (``oracle.mpo``) with the mixed path's
truncation tie tolerance 1e-5, and count the cuts where the tie rule lowered
the rank: when there are none, the float64 path's tie tolerance (1e-10) gives
the same truncations and the same results.  The inputs come from
``paper_2501_13237_amd.workloads``.

    python tests/golden/make_oracle_runs.py n32
    python tests/golden/make_oracle_runs.py n50 [levels...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np                                          # noqa: E402

from oracle import mpo as ompo, ptm                         # noqa: E402
from paper_2501_13237_amd import workloads                  # noqa: E402


def _names(obs):
    return ["".join("IXYZ"[c] for c in o) for o in obs]


_TIES = [0]
_rank = ompo.truncation_rank


def _counting_rank(s, chi_max, tau, tie_tol):
    """oracle.mpo.truncation_rank, counting the cuts where the tie
    tolerance 1e-5 keeps another rank than 1e-10."""
    r = _rank(s, chi_max, tau, tie_tol)
    if r != _rank(s, chi_max, tau, 1e-10):
        _TIES[0] += 1
    return r


ompo.truncation_rank = _counting_rank


def _run(n, layers, noise, c, chi, tie):
    _TIES[0] = 0
    nz = ptm.Noise(**noise).scaled(c)
    m = ompo.PauliMPO(n, chi, tau=1e-14, tie_tol=tie)
    for ls, us in layers:
        m.apply_layer(ls, [ptm.ptm_noisy_gate(U, nz) for U in us])
    return m


def _record(m, obs):
    return {"values": [float(v) for v in m.expectations(obs)],
            "fidelity": float(m.fidelity), "trace": float(m.trace()),
            "min_cut_gap": float(min(m.cut_gaps)) if m.cut_gaps else 1.0,
            "bonds": [int(b) for b in m.bond_dims()],
            "tie_rule_cuts": int(_TIES[0])}


def n32():
    out = {"workload": "haar-n32-d20-dep1e-3-ad5e-4 (seed 0), one level",
           "source": "oracle.mpo (float64, LAPACK SVD)", "runs": {}}
    for chi in (64, 128, 256):
        w = workloads.mixed_n32(chi=chi, seed=0)
        layers = w.circuit()
        out["observables"] = _names(w.observables)
        t0 = time.time()
        m = _run(w.n, layers, w.noise, 1.0, chi, 1e-5)
        out["runs"][f"chi{chi}"] = _record(m, w.observables)
        print(f"chi={chi} F={m.fidelity:.3e} ties={_TIES[0]} {time.time() - t0:.0f}s",
              flush=True)
    with open(os.path.join(HERE, "n32_d20_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def n50(levels):
    w = workloads.noise_sweep_n50(seed=0)
    obs = workloads.z_singles(w.n) + [workloads.pauli_string(w.n, {1: "X", 2: "X"})]
    path = os.path.join(HERE, "n50_d24_oracle.json")
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    else:
        out = {"workload": w.name + " (seed 0)", "factors": w.factors, "p0": 1e-3,
               "observables": _names(obs),
               "source": "oracle.mpo (float64, LAPACK SVD)", "levels": {}}
    layers = w.circuit()
    for j in levels:
        t0 = time.time()
        m = _run(w.n, layers, w.noise, w.factors[j], w.chi, 1e-5)
        out["levels"][str(j)] = _record(m, obs)
        print(f"level {j} F={m.fidelity:.3e} ties={_TIES[0]} {time.time() - t0:.0f}s",
              flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    if sys.argv[1] == "n32":
        n32()
    else:
        n50([int(a) for a in sys.argv[2:]] or list(range(8)))
