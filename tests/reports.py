"""GPU-against-oracle reports on the larger workloads (not collected by
pytest; needs a GPU and the built library).

    python tests/reports.py --precision          # n = 32, chi 64/128/256
    python tests/reports.py --clifford 30        # n = 64 random Cliffords
    python tests/reports.py --clifford 12 --mirror

Each prints one JSON object on stdout and its progress on stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def precision_report(nze, workloads, chis=(64, 128, 256), oracle_chis=(64,)):
    """n = 32, depth 20, depolarizing 1e-3 + amplitude damping 5e-4, one level:
    all <Z_i> from the mixed and float64 GPU paths and (for oracle_chis) the
    CPU oracle."""
    from oracle import mpo as ompo
    from oracle import ptm as optm
    out = []
    for chi in chis:
        w = workloads.mixed_n32(chi=chi, seed=0)
        layers = w.circuit()
        res = {}
        for name, prec in (("mixed", nze.NZE_MIXED), ("fp64", nze.NZE_FP64)):
            m = nze.MPO(w.n, chi, 1, prec)
            t0 = time.perf_counter()
            nze.run_circuit(m, layers, w.noise, w.factors)
            vals, fid, tr = m.expect(w.observables)
            st, _ = m.stats()
            res[name] = (vals[0], fid[0], time.perf_counter() - t0, st[0]["min_cut_gap"])
            m.close()
        rec = {"chi": chi, "F_mixed": res["mixed"][1], "F_fp64": res["fp64"][1],
               "max_abs_mixed_vs_fp64": float(np.max(np.abs(res["mixed"][0] - res["fp64"][0]))),
               "mean_abs_mixed_vs_fp64": float(np.mean(np.abs(res["mixed"][0] - res["fp64"][0]))),
               "min_cut_gap_fp64": res["fp64"][3],
               "seconds_mixed": res["mixed"][2], "seconds_fp64": res["fp64"][2]}
        if chi in oracle_chis:
            m = ompo.PauliMPO(w.n, chi)
            nz = optm.Noise(**w.noise)
            for ls, us in layers:
                m.apply_layer(ls, [optm.ptm_noisy_gate(U, nz) for U in us])
            ref = m.expectations(w.observables)
            rec["max_abs_mixed_vs_oracle"] = float(np.max(np.abs(res["mixed"][0] - ref)))
            rec["max_abs_fp64_vs_oracle"] = float(np.max(np.abs(res["fp64"][0] - ref)))
            rec["F_oracle"] = m.fidelity
        out.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    return out


def clifford_report(nze, workloads, depth=30, precision=None, mirror=False):
    """n = 64 random Clifford brickwork, Pauli noise 3e-4 per qubit, six
    levels, chi = 512: every weight-1 and nearest-neighbour weight-2 Pauli
    against exact Pauli propagation.  mirror: depth/2 random layers followed
    by their inverses, whose <Z_i> are nonzero products of noise factors."""
    from oracle import pauliprop
    from oracle import ptm as optm
    precision = nze.NZE_MIXED if precision is None else precision
    w = workloads.clifford_n64(seed=0)
    if mirror:
        w.depth = depth // 2
        half = w.circuit()
        layers = half + [(ls, [np.ascontiguousarray(U.conj().T) for U in us])
                         for ls, us in reversed(half)]
    else:
        w.depth = depth
        layers = w.circuit()
    m = nze.MPO(w.n, w.chi, len(w.factors), precision)
    t0 = time.perf_counter()
    for t, (ls, us) in enumerate(layers):
        m.apply_layer(ls, nze.layer_ptms(us, w.noise, w.factors))
        m.sync()
        print(f"clifford layer {t + 1}/{len(layers)} at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    vals, fid, tr = m.expect(w.observables)
    secs = time.perf_counter() - t0
    st, bonds = m.stats()
    m.close()
    gates = [(k, U) for ls, us in layers for k, U in zip(ls, us)]
    tables = pauliprop.gate_tables(gates)
    recs = []
    for j, c in enumerate(w.factors):
        nz = optm.Noise(**w.noise).scaled(c)
        ref = np.array([pauliprop.expectation(w.n, gates, nz, o, tables=tables)
                        for o in w.observables])
        print(f"clifford exact level {j + 1}/{len(w.factors)} done", file=sys.stderr, flush=True)
        fin = np.isfinite(vals[j])
        nzmask = (np.abs(ref) > 1e-12) & fin
        err = np.abs(vals[j] - ref)
        recs.append({"factor": c, "F": float(fid[j]), "trace": float(tr[j]),
                     "non_finite": int((~fin).sum()),
                     "max_abs_err": float(np.max(err[fin])) if fin.any() else None,
                     "nonzero_exact": int((np.abs(ref) > 1e-12).sum()),
                     "max_abs_err_nonzero": float(np.max(err[nzmask])) if nzmask.any() else None,
                     "max_bond": int(st[j]["max_bond"]),
                     "updates": int(st[j]["updates"])})
    # NZNE: quadratic fit over the six levels, evaluated at zero noise,
    # against the noiseless exact value (observables finite at every level)
    lam = np.array(w.factors) * w.noise["px"]
    exact0 = np.array([pauliprop.expectation(w.n, gates, optm.Noise(), o, tables=tables)
                       for o in w.observables])
    ok = np.all(np.isfinite(vals), axis=0)
    zne = np.full(vals.shape[1], np.nan)
    for i in np.nonzero(ok)[0]:
        zne[i] = nze.extrapolate(lam, vals[:, i], fid)[0]
    nz0 = (np.abs(exact0) > 1e-12) & ok
    e0 = np.abs(zne - exact0)
    return {"variant": "mirror" if mirror else "random", "depth": len(layers),
            "seconds": secs, "updates_per_s": sum(r["updates"] for r in recs) / secs,
            "levels": recs, "observables_finite_at_all_levels": int(ok.sum()),
            "nzne_max_abs_err": float(np.max(e0[ok])) if ok.any() else None,
            "nzne_max_abs_err_nonzero": float(np.max(e0[nz0])) if nz0.any() else None,
            "level1_max_abs_err_nonzero": float(np.max(np.abs(vals[0] - exact0)[nz0])) if nz0.any() else None,
            "nonzero_exact_noiseless": int((np.abs(exact0) > 1e-12).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", action="store_true")
    ap.add_argument("--clifford", type=int, default=0,
                    help="n = 64 Clifford check at this depth")
    ap.add_argument("--mirror", action="store_true",
                    help="Clifford check on half the depth plus its inverse")
    args = ap.parse_args()
    import torch
    from paper_2501_13237_amd import nze, workloads
    torch.cuda.set_device(0)
    out = {}
    if args.precision:
        out["precision_n32"] = precision_report(nze, workloads)
    if args.clifford:
        out["clifford_n64"] = clifford_report(nze, workloads, args.clifford,
                                              mirror=args.mirror)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
