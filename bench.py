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
path (float32 MFMA Jacobi, float64 refinement); the plain float64 path is
timed beside it, and both paths' readouts are compared with the stored
float64 oracle runs of the same job.  Also reported: p50/p99 job latency of
the serving loop on a Poisson stream of mixed jobs at the offered 20 jobs/s
(overload) and at 70 % of the completion rate it measured (sustainable), the
NZNE error of the n = 8 workload against dense values, and the oracle on the
host cores (all threads, and one thread).  Legs after the timed steps run
only while the run stays inside --budget-s.  Steady-state saturated updates at
several batch sizes are measured with --saturated-batches.
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


KERNEL_SOURCES = ["nze_device.h", "nze_phases.h", "nze_mpo.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_layer_traffic_mixed_n50_d24_chi256.md")
MFMA_FILE = os.path.join(ROOT, "profiles", "k_layer_mfma_counters_mixed_n50_d24_chi256.md")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_13237_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _profile_field(path, key):
    """A per-launch figure from a committed counter summary, or None when
    the kernel sources changed after the counters were taken."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.split(":", 1)[0].strip() in (key, "kernel_sources_sha256"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes (calibrated FETCH_SIZE + WRITE_SIZE) per k_layer launch."""
    return _profile_field(TRAFFIC_FILE, "traffic_bytes_per_launch")


def measured_mfma_flops():
    """Executed FP32 MFMA flops per k_layer launch (SQ_INSTS_VALU_MFMA_MOPS_F32)."""
    return _profile_field(MFMA_FILE, "mfma_flops_per_launch")


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


def saturated_batches(nze, workloads, batches, first=6, timed=2):
    """Steady-state two-site updates at saturated chi = 256: B independent
    n = 50 MPOs (noise levels evenly spaced in [1, 16] x p0, B = 1 at p0) are
    evolved through the first `first` layers untimed, then `timed` layers are
    timed, all B MPOs in one launch per layer.  Reports updates/s and the
    algorithmic FP32 MFMA rate of those launches."""
    import torch
    out = {}
    for B in batches:
        w = workloads.noise_sweep_n50(seed=0)
        w.depth = first + timed
        layers = w.circuit()
        factors = list(np.linspace(1.0, 16.0, B)) if B > 1 else [1.0]
        m = nze.MPO(w.n, w.chi, B, nze.NZE_MIXED)
        try:
            stream = torch.cuda.current_stream()
            for ls, us in layers[:first]:
                m.apply_layer(ls, nze.layer_ptms(us, w.noise, factors))
            ptms = [nze.layer_ptms(us, w.noise, factors) for _, us in layers[first:]]
            torch.cuda.synchronize()
            fl0 = sum(st["flops"] for st in m.stats()[0])
            ev = []
            for (ls, _), p in zip(layers[first:], ptms):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                m.apply_layer(ls, p)
                e1.record(stream)
                ev.append((e0, e1))
            torch.cuda.synchronize()
            ms = sum(a.elapsed_time(b) for a, b in ev)
            stats, bonds = m.stats()
            fl = sum(st["flops"] for st in stats) - fl0
            upd = sum(len(ls) for ls, _ in layers[first:]) * B
            tf = fl / (ms / 1e3) / 1e12
            out[str(B)] = {"updates": upd, "kernel_ms": ms,
                           "updates_per_s": 1e3 * upd / ms,
                           "achieved_tflops": tf,
                           "frac": tf / PEAK_TFLOPS["f32"],
                           "bonds_at_chi": int(np.sum(bonds[0] == w.chi))}
        finally:
            m.close()
        print(f"# saturated batch B={B}: {out[str(B)]['updates_per_s']:.1f} updates/s",
              file=sys.stderr, flush=True)
    return out


def lattice_run(nze, workloads, rows, cols, rounds, chi, levels=8, seed=0):
    """A rows x cols lattice with open boundaries (qubits numbered
    column-major), `rounds` rounds of one Haar SU(4) gate per edge, routed
    onto the chain with noiseless SWAPs (layout restored after every gate) and
    run at `levels` depolarizing levels (1..16) x 1e-3 in mixed precision.
    Reports logical gates and chain updates (gates + SWAPs) per second of the
    layer launches."""
    import torch
    rng = np.random.default_rng(seed)
    q = lambda r, c: c * rows + r
    edges = []
    for c in range(cols):
        for r in range(rows):
            if r + 1 < rows:
                edges.append((q(r, c), q(r + 1, c)))
            if c + 1 < cols:
                edges.append((q(r, c), q(r, c + 1)))
    gates = [(a, b, workloads.haar_su4(rng)) for _ in range(rounds) for a, b in edges]
    n = rows * cols
    factors = list(np.linspace(1.0, 16.0, levels))
    layers, perm = nze.routed_layers(n, gates, {"dep": 1e-3}, factors, restore=True)
    ops = sum(len(ls) for ls, _ in layers)
    m = nze.MPO(n, chi, levels, nze.NZE_MIXED)
    try:
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for ls, ptms in layers:
            m.apply_layer(ls, ptms)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st, bonds = m.stats()
    finally:
        m.close()
    return {"lattice": f"{rows}x{cols}", "rounds": rounds, "chi": chi, "levels": levels,
            "logical_gates": len(gates), "chain_ops": ops, "swaps": ops - len(gates),
            "layer_launches": len(layers), "kernel_ms": ms,
            "logical_gates_per_s": 1e3 * len(gates) * levels / ms,
            "chain_updates_per_s": 1e3 * ops * levels / ms,
            "fidelity_min": float(min(x["fidelity"] for x in st))}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, layers, timed_layer=5, budget_s=30.0, one_thread_updates=3):
    """The oracle on noise level 1: evolve the first layers (bonds grow to
    chi), then time one layer whose bonds are saturated with every host
    thread, and the first updates of the next layer with one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import mpo as ompo
    from oracle import ptm
    nz = ptm.Noise(**w.noise)
    m = ompo.PauliMPO(w.n, w.chi)
    t_start = time.perf_counter()
    t = 0
    for t, (ls, us) in enumerate(layers):
        ptms = [ptm.ptm_noisy_gate(U, nz) for U in us]
        t0 = time.perf_counter()
        m.apply_layer(ls, ptms)
        dt = time.perf_counter() - t0
        if t >= timed_layer or time.perf_counter() - t_start > budget_s:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # one thread: gates from the middle of the next layer (saturated bonds),
    # in its zig-zag order, after an untimed centre move to the first of them
    nls, nus = layers[t + 1]
    ltr = nls[0] % 2 == 0
    mid = len(nls) // 2
    order = (list(range(mid, mid + one_thread_updates)) if ltr
             else list(range(mid, mid - one_thread_updates, -1)))
    m.move_centre(nls[order[0]] if ltr else nls[order[0]] + 1)
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        for i in order:
            m.apply_gate(nls[i], ptm.ptm_noisy_gate(nus[i], nz), ltr)
        dt1 = time.perf_counter() - t1
    return {"value": len(ls) / dt, "unit": "updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "one_thread_updates_per_s": len(order) / dt1,
            "sample": (f"CPU float64 oracle (NumPy/LAPACK) on noise level 1 "
                       f"of {len(w.factors)}: layers 1-{t} evolved untimed, "
                       f"layer {t + 1} timed with {cores} threads ({len(ls)} updates "
                       f"in {dt:.2f} s, bonds up to {max(m.bond_dims())}), then "
                       f"{len(order)} updates from the middle of layer {t + 2} "
                       f"with one thread in {dt1:.2f} s")}


def serve_jobs(count, seed, workloads, nze, chis=(64, 128, 256)):
    """Synthetic job stream: n ~ U{16..64}, depth ~ U{10..30},
    chi ~ U{64, 128, 256} (or U{chis}), 4-8 levels evenly spaced in
    [1, 16] x 1e-3 (two-qubit depolarizing), Haar brickwork seeded per job,
    observables <Z_(n/2)> and <X_1 X_2>.  Inputs (PTMs) are prepared before
    the clock."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(count):
        n = int(rng.integers(16, 65))
        depth = int(rng.integers(10, 31))
        chi = int(rng.choice(list(chis)))
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
                print(f"serve: job {k} done after {lat[k]:.2f} s "
                      f"({len(lat)}/{len(jobs)})", file=sys.stderr, flush=True)
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


def copy_probe(torch, mib):
    """A plain device copy of known size: the HBM counters of one dispatch
    read mib MiB fetched and mib MiB written when they count exactly."""
    torch.cuda.set_device(0)
    x = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "bytes_read": mib * 2 ** 20,
                      "bytes_written": mib * 2 ** 20}), flush=True)


def extrapolation_error(nze, workloads):
    """n = 8 workload (exact at chi = 256): quadratic NZNE from the GPU path
    against the dense density-matrix values stored with the tests, under both
    readings of the extrapolation: (i) fit levels {2,4,8}p, evaluate at p;
    (ii) fit {1,2,4,8}p, evaluate at zero noise."""
    path = os.path.join(ROOT, "tests", "golden", "n8_dense_exact.json")
    with open(path) as f:
        ref = json.load(f)
    w = workloads.plain_fp64_n8(seed=0)
    layers = w.circuit()
    out = {"workload": ref["workload"]}
    for name, prec in (("fp64", nze.NZE_FP64), ("mixed", nze.NZE_MIXED)):
        m = nze.MPO(w.n, w.chi, len(w.factors), prec)
        nze.run_circuit(m, layers, w.noise, w.factors)
        vals, fid, _ = m.expect(w.observables)
        m.close()
        p = w.noise["dep"]
        lam = np.array(w.factors) * p
        ea, eb, e_raw_p, e_raw_0 = [], [], [], []
        for o in range(len(w.observables)):
            va, *_ = nze.extrapolate(lam[1:], vals[1:, o], fid[1:], p, nze.NZE_POLY, degree=2)
            vb, *_ = nze.extrapolate(lam, vals[:, o], fid, 0.0, nze.NZE_POLY, degree=2)
            ea.append(abs(va - ref["exact_at_p"][o]))
            eb.append(abs(vb - ref["exact_noiseless"][o]))
            e_raw_p.append(abs(vals[1, o] - ref["exact_at_p"][o]))
            e_raw_0.append(abs(vals[0, o] - ref["exact_noiseless"][o]))
        out[name] = {"nzne_levels_2_4_8_to_p_max_abs_err": max(ea),
                     "unmitigated_2p_vs_p_max_abs_err": max(e_raw_p),
                     "zne_levels_1_2_4_8_to_0_max_abs_err": max(eb),
                     "unmitigated_p_vs_0_max_abs_err": max(e_raw_0)}
    return out


def oracle_error(vals, fid, precision_name):
    """The job's readout against the stored float64 oracle runs of the same
    workload (tests/golden/n50_d24_oracle.json, written by the oracle): max
    |d<O>| over the two observables and every level, max relative dF."""
    path = os.path.join(ROOT, "tests", "golden", "n50_d24_oracle.json")
    try:
        with open(path) as f:
            g = json.load(f)
    except OSError:
        return None
    names = g["observables"]
    idx = [names.index("I" * 25 + "Z" + "I" * 24), names.index("IXX" + "I" * 47)]
    errs, ferr = [], []
    for key, ref in g["levels"].items():
        j = int(key)
        errs.append(max(abs(vals[j][o] - ref["values"][i]) for o, i in enumerate(idx)))
        ferr.append(abs(fid[j] / ref["fidelity"] - 1.0))
    return {"path": precision_name, "levels": len(errs),
            "max_abs_obs": float(max(errs)), "max_rel_fidelity": float(max(ferr))}


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--depth", type=int, default=None,
                    help="override the depth (diagnostics only)")
    ap.add_argument("--serve", type=int, default=10,
                    help="also run the serving loop on this many jobs "
                         "(0 to skip)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-sustainable-rate", type=float, default=-1.0,
                    help="offered rate of the second serving leg; -1: 70 %% of "
                         "the completion rate measured in the first leg; 0: skip")
    ap.add_argument("--serve-sustainable-jobs", type=int, default=6)
    ap.add_argument("--serve-chi", type=int, default=0,
                    help="draw every serving job with this chi (0: the mix of 64, 128, 256)")
    ap.add_argument("--budget-s", type=float, default=570.0,
                    help="wall-time budget of the whole run: legs after the "
                         "timed steps are skipped (and say so) when their "
                         "estimated time does not fit")
    ap.add_argument("--no-extrapolation-error", action="store_true",
                    help="skip the n=8 extrapolation-error leg (profiling runs)")
    ap.add_argument("--skip-main", action="store_true",
                    help="only the serving runs")
    ap.add_argument("--saturated-batches", default="",
                    help="batch sizes of the saturated-update microbenchmark "
                         "(comma list; empty to skip)")
    ap.add_argument("--lattice", default="",
                    help="also run a routed 2D lattice: ROWSxCOLSxROUNDS (e.g. 2x25x8)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many MiB device-to-device five times "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the levels and jobs "
              "of a multi-GPU run shard across GPUs without communication, so "
              "the one-GPU throughput is the per-GPU share", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
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
        chis = (args.serve_chi,) if args.serve_chi else (64, 128, 256)
        if args.serve:
            jobs = serve_jobs(args.serve, 1, workloads, nze, chis)
            out["serving"] = serve_run(nze, jobs, args.serve_rate, 1, nze.NZE_MIXED)
        if args.serve_sustainable_rate > 0:
            jobs = jobs if args.serve else serve_jobs(200, 1, workloads, nze, chis)
            out["serving_sustainable"] = serve_run(
                nze, jobs, args.serve_sustainable_rate, 1, nze.NZE_MIXED)
        print(json.dumps(out), flush=True)
        return

    def timed(precision, steps, warmup):
        name = "fp64" if precision == nze.NZE_FP64 else "mixed"
        for i in range(warmup):
            run_job(nze, w, layers, precision)
            print(f"# {name} warmup job {i + 1}/{warmup} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for i in range(steps):
            res = run_job(nze, w, layers, precision)
            # run_job reads the results back, so the job has finished here
            print(f"# {name} timed job {i + 1}/{steps} done at {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
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
                     "frac": achieved / PEAK_TFLOPS["f32"],
                     "traffic": measured_traffic(),
                     "mfma_counter_tflops": (None if measured_mfma_flops() is None else
                                             measured_mfma_flops() / (np.mean(layer_ms) / 1e3) / 1e12),
                     "kernel": "k_layer (persistent, one launch per layer)",
                     "mean_layer_ms": float(np.mean(layer_ms)),
                     "algorithmic_tflop_per_step": flops_job / 1e12},
        "saturated_layers": saturated_rate(layers, layer_ms, len(w.factors)),
        "fidelity": [float(x) for x in fid],
        "jacobi_sweeps_total": int(sum(s["sweeps_total"] for s in stats)),
        "cap_hits": int(sum(s["cap_hits"] for s in stats)),
        "ns_scaled": int(sum(s["ns_scaled"] for s in stats)),
        "error_vs_oracle": oracle_error(vals, fid, "mixed"),
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
        out["fp64"]["error_vs_oracle"] = oracle_error(vals64, fid64, "fp64")
    job_s = dt / args.steps

    def fits(est_s):
        return time.perf_counter() - t_start + est_s <= args.budget_s

    # the serving legs are reported beside the headline; an error in one of
    # them is reported in its field, not raised
    if args.serve:
        # a job of the mix is on average about a third of the n = 50 job
        est = args.serve * job_s * 0.35 + 10.0
        if not fits(est):
            out["serving"] = {"skipped": f"time budget ({est:.0f} s estimated)"}
        else:
            try:
                jobs = serve_jobs(args.serve, 1, workloads, nze)
                out["serving"] = serve_run(nze, jobs, args.serve_rate, 1, nze.NZE_MIXED)
            except Exception as e:  # noqa: BLE001
                out["serving"] = {"error": repr(e)}
        sus = args.serve_sustainable_rate
        cap = out["serving"].get("completed_jobs_per_s") if isinstance(out["serving"], dict) else None
        if sus < 0:
            sus = 0.7 * cap if cap else 0.0
        if sus > 0:
            k = args.serve_sustainable_jobs
            est = k / sus + 0.5 * k * job_s * 0.35 + 10.0
            if not fits(est):
                out["serving_sustainable"] = {"skipped": f"time budget ({est:.0f} s estimated)",
                                              "offered_rate_jobs_per_s": sus}
            else:
                try:
                    jobs = serve_jobs(k, 2, workloads, nze)
                    out["serving_sustainable"] = serve_run(nze, jobs, sus, 2, nze.NZE_MIXED)
                except Exception as e:  # noqa: BLE001
                    out["serving_sustainable"] = {"error": repr(e)}
    if args.saturated_batches:
        try:
            out["saturated_batch"] = saturated_batches(
                nze, workloads, [int(b) for b in args.saturated_batches.split(",")])
        except Exception as e:  # noqa: BLE001
            out["saturated_batch"] = {"error": repr(e)}
    if args.lattice:
        r, c, k = (int(x) for x in args.lattice.split("x"))
        try:
            out["lattice_2d"] = lattice_run(nze, workloads, r, c, k, w.chi)
        except Exception as e:  # noqa: BLE001
            out["lattice_2d"] = {"error": repr(e)}
    if not args.no_extrapolation_error:
        out["extrapolation_error_n8"] = extrapolation_error(nze, workloads)
    if not args.no_cpu_baseline:
        if fits(45.0):
            out["cpu_baseline"] = cpu_baseline(w, layers)
        else:
            out["cpu_baseline"] = {"skipped": "time budget"}
    out["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
