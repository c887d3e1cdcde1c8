"""Throughput of the NZNE hot path on one MI355X.

One step = one whole noise-extrapolation job of the headline workload:
build the 16x16 PTMs of every gate at every noise level (host, float64), create
the MPOs of all levels in the product state, apply every brickwork layer (one
persistent kernel launch per layer, all levels batched), read out the Pauli
expectation values and fidelities, and extrapolate each observable with the
quadratic and exponential fits.  Inputs are seeded and synthetic.

Workload: 1D chain n = 50, depth-24 brickwork of Haar-random SU(4) gates,
two-qubit depolarizing noise p0 = 1e-3 amplified to 8 levels
lambda_j = (1 + 15 j / 7) p0, chi = 256; observables <Z_25>, <X_1 X_2>.
588 gates x 8 levels = 4704 two-site updates per job.

Prints one JSON line (rank 0).  `value` is two-site updates/s of the mixed
(float32 MFMA) path; the plain float64 path is timed beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
METRIC = ("MPO two-site updates/s at chi=256 vs plain FP64; extrap. error; "
          "p50/p99 job latency")


def run_job(nze, w, layers, precision, return_mpo=False):
    """One full job; returns (values[L][n_obs], fidelities, stats, layer_ms)."""
    import torch
    factors = w.factors
    m = nze.MPO(w.n, w.chi, len(factors), precision)
    stream = torch.cuda.current_stream()
    ev = []
    for ls, us in layers:
        ptms = nze.layer_ptms(us, w.noise, factors)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.apply_layer(ls, ptms)
        e1.record(stream)
        ev.append((e0, e1))
    vals, fid, tr = m.expect(w.observables)
    lam = np.array(factors) * w.noise["dep"]
    fits = {}
    for o in range(vals.shape[1]):
        q, *_ = nze.extrapolate(lam, vals[:, o], fid, lam[0], nze.NZE_POLY,
                                degree=2)
        q0, *_ = nze.extrapolate(lam, vals[:, o], fid, 0.0, nze.NZE_POLY,
                                 degree=2)
        try:
            e, *_ = nze.extrapolate(lam, vals[:, o], fid, lam[0], nze.NZE_EXP3)
        except nze.NzeError:
            e = None
        fits[o] = {"quad_at_p0": q, "quad_at_0": q0, "exp_at_p0": e}
    stats, bonds = m.stats()
    layer_ms = [a.elapsed_time(b) for a, b in ev]
    out = (vals, fid, tr, stats, layer_ms, fits)
    if return_mpo:
        return out + (m,)
    m.close()
    return out


def saturated_rate(layers, layer_ms, levels, first=6):
    """Updates/s over the layers whose bonds are all saturated (every layer
    from the seventh on at chi = 256, n = 50), from the per-layer events."""
    upd = sum(len(ls) for ls, _ in layers[first:]) * levels
    ms = sum(layer_ms[first:])
    return {"from_layer": first + 1, "updates": upd, "kernel_ms": ms,
            "updates_per_s": 1e3 * upd / ms if ms > 0 else None}


def cpu_baseline(w, layers, timed_layer=5, budget_s=40.0):
    """The oracle on noise level 1: evolve the first layers (bonds grow to
    chi), then time one layer whose bonds are saturated."""
    from oracle import mpo as ompo
    from oracle import ptm
    nz = ptm.Noise(**w.noise)
    m = ompo.PauliMPO(w.n, w.chi)
    t_start = time.perf_counter()
    for t, (ls, us) in enumerate(layers):
        ptms = [ptm.ptm_noisy_gate(U, nz) for U in us]
        t0 = time.perf_counter()
        m.apply_layer(ls, ptms)
        dt = time.perf_counter() - t0
        if t >= timed_layer or time.perf_counter() - t_start > budget_s:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(ls) / dt, "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"CPU float64 oracle (NumPy/LAPACK) on noise level 1 "
                       f"of {len(w.factors)}: layers 1-{t} evolved untimed, "
                       f"layer {t + 1} timed ({len(ls)} updates in "
                       f"{dt:.2f} s, bonds up to {max(m.bond_dims())})")}


def serve_jobs(count, seed, workloads, nze):
    """Synthetic job stream: n ~ U{16..64}, depth ~ U{10..30},
    chi ~ U{64, 128, 256}, 4-8 levels evenly spaced in [1, 16] x 1e-3
    (two-qubit depolarizing), Haar brickwork seeded per job, observables
    <Z_(n/2)> and <X_1 X_2>.  Inputs (PTMs) are prepared before the clock."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        n = int(rng.integers(16, 65))
        depth = int(rng.integers(10, 31))
        chi = int(rng.choice([64, 128, 256]))
        L = int(rng.integers(4, 9))
        factors = list(np.linspace(1.0, 16.0, L))
        layers = workloads.brickwork(n, depth, seed=10000 * seed + i)
        ptms = [nze.layer_ptms(us, {"dep": 1e-3}, factors) for _, us in layers]
        obs = [workloads.pauli_string(n, {n // 2: "Z"}),
               workloads.pauli_string(n, {1: "X", 2: "X"})]
        upd = workloads.n_gates(layers) * L
        jobs.append(dict(n=n, depth=depth, chi=chi, L=L, layers=[ls for ls, _ in layers],
                         ptms=ptms, obs=obs, updates=upd))
    return jobs


def serve_run(nze, jobs, rate, seed, precision):
    """Poisson arrivals at `rate` jobs/s into the serving loop; latency is
    arrival -> result available on the host."""
    rng = np.random.default_rng(seed + 7)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(jobs)))
    srv = nze.Server(64 << 30, max_active=64)
    t0 = time.perf_counter()
    ids, lat, done_upd = {}, {}, 0
    nxt = 0
    while len(lat) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and arrivals[nxt] <= now:
            j = jobs[nxt]
            ids[srv.submit(j["n"], j["chi"], precision, j["layers"], j["ptms"],
                           j["obs"])] = nxt
            nxt += 1
        a, q, d = srv.step()
        if a == 0 and q == 0 and nxt < len(jobs):
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
        for jid, k in ids.items():
            if k in lat:
                continue
            st, vals, fid, _ = srv.poll(jid)
            if st == 2:
                lat[k] = (time.perf_counter() - t0) - arrivals[k]
                done_upd += jobs[k]["updates"]
            elif st < 0:
                raise RuntimeError(f"job {k} failed with {st}")
    wall = time.perf_counter() - t0
    hw, launches = srv.stats()
    srv.close()
    la = np.array([lat[k] for k in range(len(jobs))])
    return {"offered_rate_jobs_per_s": rate, "jobs": len(jobs),
            "p50_latency_s": float(np.percentile(la, 50)),
            "p99_latency_s": float(np.percentile(la, 99)),
            "completed_jobs_per_s": len(jobs) / wall,
            "updates_per_s": done_upd / wall, "wall_s": wall,
            "launches": int(launches), "arena_high_water_gib": hw / 2 ** 30}


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
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--depth", type=int, default=None,
                    help="override the depth (diagnostics only)")
    ap.add_argument("--serve", type=int, default=0,
                    help="also run the serving loop on this many jobs")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-sustainable-rate", type=float, default=0.0)
    ap.add_argument("--skip-main", action="store_true",
                    help="only the serving / report runs")
    ap.add_argument("--precision-report", action="store_true")
    ap.add_argument("--clifford-report", type=int, default=0,
                    help="run the n=64 Clifford check at this depth")
    ap.add_argument("--clifford-mirror", action="store_true",
                    help="Clifford check on half the depth plus its inverse")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus must be 1 "
              "(the levels and jobs of a multi-GPU run would be sharded "
              "without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_13237_amd import nze, workloads
    torch.cuda.set_device(0)
    nze.lib()
    w = workloads.noise_sweep_n50(seed=0)
    if args.depth:
        w.depth = args.depth
    layers = w.circuit()
    upd_per_job = workloads.n_gates(layers) * len(w.factors)

    if args.skip_main:
        out = {"metric": "reports", "n_gpus": 1, "data": "synthetic"}
        if args.precision_report:
            out["precision_n32"] = precision_report(nze, workloads)
        if args.clifford_report:
            out["clifford_n64"] = clifford_report(nze, workloads, args.clifford_report,
                                                  mirror=args.clifford_mirror)
        if args.serve:
            jobs = serve_jobs(args.serve, 1, workloads, nze)
            out["serving"] = serve_run(nze, jobs, args.serve_rate, 1, nze.NZE_MIXED)
        if args.serve_sustainable_rate > 0:
            out["serving_sustainable"] = serve_run(
                nze, jobs, args.serve_sustainable_rate, 1, nze.NZE_MIXED)
        print(json.dumps(out), flush=True)
        return

    def timed(precision, steps, warmup):
        for _ in range(warmup):
            run_job(nze, w, layers, precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for _ in range(steps):
            res = run_job(nze, w, layers, precision)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, res

    dt, res = timed(nze.NZE_MIXED, args.steps, args.warmup)
    vals, fid, tr, stats, layer_ms, fits = res
    flops_job = sum(s["flops"] for s in stats)
    kernel_s = sum(layer_ms) / 1e3
    achieved = flops_job / kernel_s / 1e12
    value = upd_per_job * args.steps / dt

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Haar-random SU(4) brickwork)",
        "config": {"workload": (f"brickwork n={w.n} depth={w.depth} Haar SU(4), "
                                f"depolarizing p0=1e-3 at {len(w.factors)} levels "
                                f"(1..16)xp0, chi={w.chi}, mixed precision"),
                   "n": w.n, "depth": w.depth, "levels": len(w.factors),
                   "chi": w.chi, "updates_per_step": upd_per_job,
                   "observables": ["Z_25", "X_1 X_2"]},
        "roofline": {"bound": "mfma", "achieved": achieved,
                     "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["f32"], "traffic": None,
                     "kernel": "k_layer (persistent, one launch per layer)",
                     "mean_layer_ms": float(np.mean(layer_ms)),
                     "algorithmic_tflop_per_step": flops_job / 1e12},
        "saturated_layers": saturated_rate(layers, layer_ms, len(w.factors)),
        "fidelity": [float(x) for x in fid],
        "jacobi_sweeps_total": int(sum(s["sweeps_total"] for s in stats)),
        "extrapolation": {str(k): v for k, v in fits.items()},
    }
    if args.fp64_steps > 0:
        dt64, res64 = timed(nze.NZE_FP64, args.fp64_steps, 0)
        v64 = upd_per_job * args.fp64_steps / dt64
        vals64, fid64 = res64[0], res64[1]
        st64 = res64[3]
        fl64 = sum(s["flops"] for s in st64) / (sum(res64[4]) / 1e3) / 1e12
        out["fp64"] = {"value": v64, "unit": "updates/s",
                       "ms_per_step": 1e3 * dt64 / args.fp64_steps,
                       "achieved_tflops": fl64,
                       "frac_of_fp64_peak": fl64 / PEAK_TFLOPS["f64"]}
        out["speedup_mixed_vs_fp64"] = value / v64
        out["mixed_vs_fp64_max_abs_obs"] = float(np.max(np.abs(vals - vals64)))
        out["mixed_vs_fp64_max_rel_fid"] = float(np.max(np.abs(fid - fid64) / fid64))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, layers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
