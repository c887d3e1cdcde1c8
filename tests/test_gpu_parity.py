"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the same
seeded inputs.  Only gauge-invariant outputs are compared: expectation values,
emulation fidelity, trace, bond dimensions where nothing is truncated."""
import sys

import numpy as np
import pytest

from oracle import mpo as ompo
from oracle import pauliprop, ptm
from paper_2501_13237_amd import nze, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_run(n, layers, noise, factors, chi, tau=1e-14, tie=1e-10):
    out = []
    for c in factors:
        nz = ptm.Noise(**noise).scaled(c)
        m = ompo.PauliMPO(n, chi, tau=tau, tie_tol=tie)
        for ls, us in layers:
            m.apply_layer(ls, [ptm.ptm_noisy_gate(U, nz) for U in us])
        out.append(m)
    return out


def _gpu_run(n, layers, noise, factors, chi, precision, **kw):
    m = nze.MPO(n, chi, len(factors), precision, **kw)
    nze.run_circuit(m, layers, noise, factors)
    return m


def _compare(n, layers, noise, factors, chi, obs, precision, tol, **kw):
    _say(f"case n={n} depth={len(layers)} chi={chi} L={len(factors)} "
         f"prec={precision} noise={noise}")
    g = _gpu_run(n, layers, noise, factors, chi, precision, **kw)
    vals, fid, tr = g.expect(obs)
    orc = _oracle_run(n, layers, noise, factors, chi,
                      tie=(1e-10 if precision == nze.NZE_FP64 else 1e-5))
    for j, m in enumerate(orc):
        ref = m.expectations(obs)
        err = np.max(np.abs(vals[j] - ref))
        _say(f"  level {j}: max|dO|={err:.3e} F_gpu={fid[j]:.12f} "
             f"F_orc={m.fidelity:.12f} tr_gpu={tr[j]:.12f} tr_orc={m.trace():.12f}")
        assert err < tol
        assert abs(fid[j] - m.fidelity) < tol * max(1.0, m.fidelity)
        assert abs(tr[j] - m.trace()) < 10 * tol
    return g, orc


@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, FP64_TOL),
                                           (nze.NZE_MIXED, MIXED_TOL)])
def test_plain_n8_exact(precision, tol):
    w = workloads.plain_fp64_n8(seed=0)
    layers = w.circuit()
    g, orc = _compare(w.n, layers, w.noise, w.factors, w.chi, w.observables,
                      precision, tol)
    stats, bonds = g.stats()
    assert all(abs(s["fidelity"] - 1.0) < tol for s in stats)
    # numerical ranks at the 1e-14 s_1 threshold are implementation-dependent;
    # the invariant is the exact cap 4^min(k, n-k) of every bond.  In the mixed
    # path the float32 rounding directions (~1e-6 s_1) lie above tau = 1e-7 and
    # fill the bonds of an exactly low-rank state, so only float64 is checked.
    caps = np.array([4 ** min(k + 1, w.n - k - 1) for k in range(w.n - 1)])
    assert precision == nze.NZE_MIXED or np.all(bonds <= caps[None, :])


def test_small_chain_two_sites():
    layers = workloads.brickwork(2, 3, seed=5)
    obs = workloads.weight1_all(2) + workloads.weight2_neighbours(2)
    _compare(2, layers, {"dep": 0.05}, [1.0, 2.0], 4, obs, nze.NZE_FP64,
             FP64_TOL)


@pytest.mark.parametrize("chi", [16, 20])
def test_truncated_fp64(chi):
    n = 10
    layers = workloads.brickwork(n, 10, seed=3)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    g, orc = _compare(n, layers, {"dep": 1e-2}, [1.0, 4.0], chi, obs,
                      nze.NZE_FP64, FP64_TOL)
    assert orc[0].fidelity < 0.999


def test_odd_chain_ragged_amplitude_damping():
    n = 7
    layers = workloads.brickwork(n, 9, seed=8)
    obs = workloads.weight1_all(n)
    _compare(n, layers, {"dep": 2e-3, "ad": 5e-3}, [1.0, 3.0, 5.0], 40, obs,
             nze.NZE_FP64, FP64_TOL)


def test_chi_one_product_truncation():
    n = 6
    layers = workloads.brickwork(n, 4, seed=2)
    obs = workloads.z_singles(n)
    _compare(n, layers, {"dep": 0.05}, [1.0], 1, obs, nze.NZE_FP64, FP64_TOL)


def test_mixed_truncated_ad():
    n = 12
    layers = workloads.brickwork(n, 10, seed=4)
    obs = workloads.z_singles(n)
    _compare(n, layers, {"dep": 1e-3, "ad": 5e-4}, [1.0], 32, obs,
             nze.NZE_MIXED, MIXED_TOL)


def test_clifford_exact_vs_pauli_propagation():
    n = 16
    layers = workloads.brickwork(n, 4, seed=6, kind="clifford")
    noise = {"px": 3e-3, "py": 3e-3, "pz": 3e-3}
    obs = workloads.weight1_all(n) + workloads.weight2_neighbours(n)
    for prec, tol in ((nze.NZE_FP64, FP64_TOL), (nze.NZE_MIXED, MIXED_TOL)):
        _say(f"clifford prec={prec}")
        g = _gpu_run(n, layers, noise, [1.0, 4.0], 256, prec)
        vals, fid, tr = g.expect(obs)
        gates = [(k, U) for ls, us in layers for k, U in zip(ls, us)]
        for j, c in enumerate([1.0, 4.0]):
            nz = ptm.Noise(**noise).scaled(c)
            ref = np.array([pauliprop.expectation(n, gates, nz, o) for o in obs])
            err = np.max(np.abs(vals[j] - ref))
            _say(f"  level {j}: max err vs Pauli propagation {err:.3e}")
            assert err < tol
            assert abs(fid[j] - 1.0) < tol


def test_batch_matches_separate_bitwise():
    n = 10
    la = workloads.brickwork(n, 6, seed=11)
    lb = workloads.brickwork(n + 2, 5, seed=12)
    obs_a = workloads.z_singles(n)
    obs_b = workloads.z_singles(n + 2)
    noise = {"dep": 5e-3}
    sep_a = _gpu_run(n, la, noise, [1.0, 2.0], 16, nze.NZE_FP64)
    sep_b = _gpu_run(n + 2, lb, noise, [1.0], 16, nze.NZE_FP64)
    ma = nze.MPO(n, 16, 2, nze.NZE_FP64)
    mb = nze.MPO(n + 2, 16, 1, nze.NZE_FP64)
    for t in range(max(len(la), len(lb))):
        mpos, lss, ptms = [], [], []
        if t < len(la):
            mpos.append(ma)
            lss.append(la[t][0])
            ptms.append(nze.layer_ptms(la[t][1], noise, [1.0, 2.0]))
        if t < len(lb):
            mpos.append(mb)
            lss.append(lb[t][0])
            ptms.append(nze.layer_ptms(lb[t][1], noise, [1.0]))
        nze.apply_layer_batch(mpos, lss, ptms)
    va, fa, _ = ma.expect(obs_a)
    vb, fb, _ = mb.expect(obs_b)
    ra, rfa, _ = sep_a.expect(obs_a)
    rb, rfb, _ = sep_b.expect(obs_b)
    assert np.array_equal(va, ra) and np.array_equal(fa, rfa)
    assert np.array_equal(vb, rb) and np.array_equal(fb, rfb)


@pytest.mark.parametrize("precision", [nze.NZE_FP64, nze.NZE_MIXED])
def test_xcd_groups_match_device_groups_bitwise(precision):
    # eight levels in one launch take the XCD-local workgroup groups; each
    # level alone (one MPO) takes device-wide groups.  A pair visit computes
    # the same numbers whichever workgroup runs it, so both must agree bitwise.
    n = 12
    layers = workloads.brickwork(n, 8, seed=31)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    noise = {"dep": 2e-3}
    factors = [1.0 + 15.0 * j / 7 for j in range(8)]
    _say(f"xcd vs device groups prec={precision}")
    m8 = _gpu_run(n, layers, noise, factors, 24, precision)
    v8, f8, t8 = m8.expect(obs)
    st8, _ = m8.stats()
    assert min(s["fidelity"] for s in st8) < 0.999     # truncation happened
    for j, c in enumerate(factors):
        m1 = _gpu_run(n, layers, noise, [c], 24, precision)
        v1, f1, t1 = m1.expect(obs)
        assert np.array_equal(v8[j], v1[0]) and f8[j] == f1[0] and t8[j] == t1[0]


@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, FP64_TOL),
                                           (nze.NZE_MIXED, MIXED_TOL)])
def test_bond_spectra_and_entropy(precision, tol):
    # Schmidt values at every bond (canonical form there) and the MPO
    # entanglement entropy, exact (n = 8, chi = 256) and truncated
    # (n = 10, chi = 24) runs, against the oracle's LAPACK spectra
    for n, chi, depth, seed in ((8, 256, 8, 41), (10, 24, 8, 42)):
        layers = workloads.brickwork(n, depth, seed=seed)
        noise = {"dep": 2e-3}
        factors = [1.0, 4.0]
        _say(f"bond spectra n={n} chi={chi} prec={precision}")
        g = _gpu_run(n, layers, noise, factors, chi, precision)
        orc = _oracle_run(n, layers, noise, factors, chi,
                          tie=(1e-10 if precision == nze.NZE_FP64 else 1e-5))
        for j, m in enumerate(orc):
            for b in range(n - 1):
                sg = g.bond_spectrum(j, b)
                so = m.bond_spectrum(b)
                so = so / np.linalg.norm(so)
                k = min(sg.size, so.size)
                assert sg.size >= 1 and abs(np.linalg.norm(sg) - 1.0) < 10 * tol
                assert np.max(np.abs(sg[:k] - so[:k])) < tol
                # values the GPU does not report are numerical zeros
                assert so.size <= k or so[k] < 1e3 * tol
                assert abs(g.entanglement_entropy(j, b) - m.entanglement_entropy(b)) < 100 * tol
        # the moves change the gauge only: readout is unchanged
        obs = workloads.z_singles(n)
        vals, fid, _ = g.expect(obs)
        for j, m in enumerate(orc):
            assert np.max(np.abs(vals[j] - m.expectations(obs))) < tol


def _torch_dev(a, precision):
    import torch
    dt = torch.float64 if precision == nze.NZE_FP64 else torch.float32
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("precision", [nze.NZE_FP64, nze.NZE_MIXED])
@pytest.mark.parametrize("dims", [(256, 256, 256), (37, 50, 29), (1, 4, 16)])
def test_kernel_theta_against_oracle(precision, dims):
    # one two-site contraction with the noisy-gate superoperator, at the
    # saturated chi = 256 of the n = 50 workload and at ragged shapes, both
    # orientations, against the oracle's Theta'
    cl, cm, cr = dims
    rng = np.random.default_rng(100 + cl)
    A = rng.standard_normal((cl, 4, cm)) / np.sqrt(4 * cm)
    B = rng.standard_normal((cm, 4, cr)) / np.sqrt(cm)
    U = workloads.haar_su4(rng)
    R = ptm.ptm_noisy_gate(U, ptm.Noise(dep=1e-3, ad=5e-4))
    m = ompo.PauliMPO(2, 1)
    m.sites = [A, B]
    ref = m.two_site_block(0, R)
    tol = 1e-12 if precision == nze.NZE_FP64 else 1e-5
    for ltr in (True, False):
        _say(f"theta dims={dims} prec={precision} ltr={ltr}")
        X = nze.kernel_theta(_torch_dev(A.reshape(4 * cl, cm), precision),
                             _torch_dev(B.reshape(cm, 4 * cr), precision), R, ltr)
        got = X.double().cpu().numpy()
        if not ltr:
            got = got.T
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        _say(f"  max rel err {err:.2e}")
        assert err < tol


@pytest.mark.parametrize("precision", [nze.NZE_FP64, nze.NZE_MIXED])
@pytest.mark.parametrize("shape", [(1024, 1024), (2048, 2048), (1000, 996), (37, 64)])
def test_kernel_rowortho_known_spectrum(precision, shape):
    # the block one-sided Jacobi of the layer kernel on X = U diag(s) V^T with
    # a known spectrum: graded over eight decades with clusters of equal
    # values, sizes of the chi = 256 and chi = 512 updates and ragged ones
    R, C = shape
    k = min(R, C)
    rng = np.random.default_rng(R + C)
    Uq, _ = np.linalg.qr(rng.standard_normal((R, k)))
    Vq, _ = np.linalg.qr(rng.standard_normal((C, k)))
    s = np.logspace(0, -8, k)
    s[10:14] = s[10]                      # an exactly degenerate cluster
    s[k // 2:k // 2 + 3] = s[k // 2]
    Xin = (Uq * s) @ Vq.T
    _say(f"rowortho R={R} C={C} prec={precision}")
    X = _torch_dev(Xin, precision)
    fp64 = precision == nze.NZE_FP64
    W, norms, sweeps = nze.kernel_rowortho(X, 1e-13 if fp64 else 2e-6,
                                           1e-15 if fp64 else 1e-6, max_sweeps=40)
    Wn = W.double().cpu().numpy()
    Xo = X.double().cpu().numpy()
    sv = np.sort(np.sqrt(np.maximum(norms, 0.0)))[::-1]
    err = np.max(np.abs(sv[:k] - s))
    orth = np.max(np.abs(Wn @ Wn.T - np.eye(R)))
    resid = np.max(np.abs(Wn @ Xin - Xo))
    _say(f"  sweeps={sweeps} max|sigma-s|={err:.2e} |WW^T-I|={orth:.2e} |W X - X_out|={resid:.2e}")
    # float32: every visit rotates a row by a 32-term sum (~sqrt(32) 2^-24
    # relative), and a row takes ~sweeps x rounds visits, so the singular
    # values carry ~1e-5 relative rounding after the ~1000 visits of a hard
    # 1024-row input; float64 stays at the 1e-13 level
    tol = 1e-11 if fp64 else 5e-5
    assert err < tol and orth < tol and resid < tol
    assert np.all(sv[k:] < tol)           # rows beyond the rank are zero
    # rows of the result are mutually orthogonal: the cosine bound is
    # tol (1 + (tol_abs/tol) ||X|| / ||row||), so check rows well above the
    # absolute floor
    nr = np.sqrt(np.einsum("ij,ij->i", Xo, Xo))
    big = nr > (1e-2 if fp64 else 0.1)
    G = Xo[big] @ Xo[big].T / np.outer(nr[big], nr[big])
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < (1e-11 if fp64 else 1e-4)


def test_full_size_first_layers_against_oracle():
    # the n = 50, chi = 256, eight-level workload in the launch configuration
    # the benchmark times (all levels in one launch per layer), first six
    # layers: the middle bonds reach chi and are truncated from layer 5 on.
    # Sampled levels 0 and 7 against the oracle, float64 path, every <Z_i>
    # and the workload's two observables.
    w = workloads.noise_sweep_n50(seed=0)
    layers = w.circuit()[:6]
    obs = workloads.z_singles(w.n) + list(w.observables)
    _say("full size n=50 chi=256 L=8 depth 6 fp64")
    g = _gpu_run(w.n, layers, w.noise, w.factors, w.chi, nze.NZE_FP64)
    vals, fid, tr = g.expect(obs)
    st, bonds = g.stats()
    assert bonds.max() == w.chi
    for j in (0, 7):
        nz = ptm.Noise(**w.noise).scaled(w.factors[j])
        m = ompo.PauliMPO(w.n, w.chi)
        for ls, us in layers:
            m.apply_layer(ls, [ptm.ptm_noisy_gate(U, nz) for U in us])
        err = np.max(np.abs(vals[j] - m.expectations(obs)))
        _say(f"  level {j}: max|dO|={err:.3e} F_gpu={fid[j]:.12f} F_orc={m.fidelity:.12f} "
             f"min gap {st[j]['min_cut_gap']:.2e}")
        assert err < FP64_TOL
        assert abs(fid[j] - m.fidelity) < FP64_TOL


def _cat_tfim_1d(n, steps, lam, th_zz, th_x):
    """1D transverse-field Ising Trotter circuit under the cat-qubit noise
    model: per step exp(-i th_zz Z Z / 2) on even then odd pairs as
    CX . Z(th_zz) on the target . CX, then exp(-i th_x X / 2) on every qubit
    as H . Z(th_x) . H, each gate followed by its cat-model Pauli errors.
    Returns the MPO layers (left sites, PTMs with every single-qubit gate
    folded into a neighbouring two-qubit subcircuit through the library's
    host calls) and the plain gate list for the dense simulator."""
    assert n % 2 == 0
    L1 = {"I": 0, "X": 1, "Y": 2, "Z": 3}

    def r1(gate):
        r = np.zeros(4)
        for k, v in ptm.CAT_RATES[gate].items():
            r[L1[k]] = v
        return r

    r2 = np.zeros(16)
    for k, v in ptm.CAT_RATES["CX"].items():
        r2[4 * L1[k[0]] + L1[k[1]]] = v
    cx = nze.build_ptm_pauli(ptm.CX_LEFT, r2, lam)
    zz = nze.ptm_compose(nze.compose_1q(cx, ptm.rz(th_zz), r1("Z"), lam, 1, True), cx)
    gates, layers = [], []
    pending = {}                      # qubit -> number of X blocks to fold
    for step in range(steps):
        for parity in (0, 1):
            ls = list(range(parity, n - 1, 2))
            ptms = []
            for k in ls:
                R = zz.copy()
                for side, q in ((0, k), (1, k + 1)):
                    for _ in range(pending.pop(q, 0)):     # X block of the step before
                        for u, g in ((ptm.H1, "H"), (ptm.rz(th_x), "Z"), (ptm.H1, "H"))[::-1]:
                            R = nze.compose_1q(R, u, r1(g), lam, side, False)
                ptms.append(R)
                gates += [("2q", k, ptm.CX_LEFT, "CX"), ("1q", k + 1, ptm.rz(th_zz), "Z"),
                          ("2q", k, ptm.CX_LEFT, "CX")]
            layers.append((np.array(ls, dtype=np.int32), ptms))
        for q in range(n):
            pending[q] = pending.get(q, 0) + 1
            gates += [("1q", q, ptm.H1, "H"), ("1q", q, ptm.rz(th_x), "Z"), ("1q", q, ptm.H1, "H")]
    # the last X blocks fold after the last two-qubit subcircuit on their qubit
    for li in (len(layers) - 1, len(layers) - 2):
        ls, ptms = layers[li]
        for i, k in enumerate(ls):
            for side, q in ((0, k), (1, k + 1)):
                if pending.pop(q, 0):
                    for u, g in ((ptm.H1, "H"), (ptm.rz(th_x), "Z"), (ptm.H1, "H")):
                        ptms[i] = nze.compose_1q(ptms[i], u, r1(g), lam, side, True)
    assert not pending
    return layers, gates


def _dense_cat(n, gates, lam):
    from oracle import dense
    rho = dense.product_state([0] * n)
    for kind, k, U, g in gates:
        if kind == "2q":
            rho = dense.apply_two_qubit(rho, n, k, U)
            ks = ptm.kraus_pauli_channel(ptm.cat_probs(g, lam))
            rho = sum(dense.apply_two_qubit(rho, n, k, K) for K in ks)
        else:
            ks = [K @ U for K in ptm.kraus_pauli_channel(ptm.cat_probs(g, lam))]
            if k < n - 1:
                rho = sum(dense.apply_two_qubit(rho, n, k, np.kron(K, ptm.I2)) for K in ks)
            else:
                rho = sum(dense.apply_two_qubit(rho, n, k - 1, np.kron(ptm.I2, K)) for K in ks)
    return rho


@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, FP64_TOL),
                                           (nze.NZE_MIXED, MIXED_TOL)])
def test_cat_noise_tfim_with_one_qubit_gates_against_dense(precision, tol):
    # single-qubit gates and the cat-qubit noise model (App. C.2 table),
    # folded into the two-qubit subcircuits on the host, against the dense
    # density matrix of the same gate list (n = 8, exact at chi = 256)
    from oracle import dense
    n, steps, lam = 8, 3, 2e-3
    layers, gates = _cat_tfim_1d(n, steps, lam, 0.4, 0.3)
    _say(f"cat tfim n={n} steps={steps} prec={precision}")
    m = nze.MPO(n, 256, 1, precision)
    for ls, ptms in layers:
        m.apply_layer(ls, np.array(ptms)[None])
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    vals, fid, _ = m.expect(obs)
    rho = _dense_cat(n, gates, lam)
    ref = np.array([dense.expectation(rho, n, o).real for o in obs])
    err = np.max(np.abs(vals[0] - ref))
    _say(f"  max|dO|={err:.3e} F={fid[0]:.12f}")
    assert err < tol and abs(fid[0] - 1.0) < tol


def test_long_chain_and_empty_layers():
    # a long chain (n = 600: 300 gates per layer in one launch, bonds
    # truncated at chi = 16, F ~ 6e-6, smallest cut gap ~ 1e-5) against the
    # oracle, with an empty layer in between (no gates: a no-op).  Observed:
    # 6e-14 (FP64), 8e-7 (mixed).
    n, chi = 600, 16
    layers = workloads.brickwork(n, 4, seed=51)
    noise = {"dep": 4e-3, "ad": 1e-3}
    obs = [workloads.pauli_string(n, {q: "Z"}) for q in (0, 1, 299, 300, 598, 599)] + \
          [workloads.pauli_string(n, {q: "Z", q + 1: "Z"}) for q in (0, 300, 598)]
    for prec, tol in ((nze.NZE_FP64, FP64_TOL), (nze.NZE_MIXED, MIXED_TOL)):
        _say(f"long chain n={n} chi={chi} prec={prec}")
        m = nze.MPO(n, chi, 2, prec)
        for t, (ls, us) in enumerate(layers):
            m.apply_layer(ls, nze.layer_ptms(us, noise, [1.0, 3.0]))
            if t == 1:
                m.apply_layer(np.zeros(0, dtype=np.int32), np.zeros((2, 0, 16, 16)))
        vals, fid, _ = m.expect(obs)
        orc = _oracle_run(n, layers, noise, [1.0, 3.0], chi,
                          tie=(1e-10 if prec == nze.NZE_FP64 else 1e-5))
        for j, o in enumerate(orc):
            err = np.max(np.abs(vals[j] - o.expectations(obs)))
            _say(f"  level {j}: max|dO|={err:.3e} F_gpu={fid[j]:.6e} F_orc={o.fidelity:.6e}")
            assert err < tol
            assert abs(fid[j] - o.fidelity) < tol * max(1.0, o.fidelity) * 10


def test_many_groups_kernel_matches_bitwise():
    # ten chi = 256 levels ask for 320 groups, more than one per CU: the
    # launch takes the float kernel built for two workgroups per CU (scalar
    # rotations).  Each level alone takes the one-per-CU kernel (vector
    # rotations).  Same arithmetic per element, so identical results.
    n = 8
    layers = workloads.brickwork(n, 8, seed=61)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    noise = {"dep": 2e-3}
    factors = list(np.linspace(1.0, 10.0, 10))
    _say("many groups: 10 levels chi=256 mixed")
    m10 = _gpu_run(n, layers, noise, factors, 256, nze.NZE_MIXED)
    v10, f10, t10 = m10.expect(obs)
    for j in (0, 9):
        m1 = _gpu_run(n, layers, noise, [factors[j]], 256, nze.NZE_MIXED)
        v1, f1, t1 = m1.expect(obs)
        assert np.array_equal(v10[j], v1[0]) and f10[j] == f1[0] and t10[j] == t1[0]


def test_invalid_layer_rejected():
    m = nze.MPO(6, 8, 1, nze.NZE_FP64)
    with pytest.raises(nze.NzeError) as e:
        m.apply_layer(np.array([2, 1], dtype=np.int32), np.zeros((1, 2, 16, 16)))
    assert e.value.code == nze.NZE_EINVAL
    with pytest.raises(nze.NzeError) as e:
        m.apply_layer(np.array([5], dtype=np.int32), np.zeros((1, 1, 16, 16)))
    assert e.value.code == nze.NZE_EINVAL


def test_eight_levels_one_launch_fp64_truncated():
    # eight MPOs in one launch, truncated (F = 0.43)
    n = 10
    layers = workloads.brickwork(n, 8, seed=21)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    factors = [1.0 + 15.0 * j / 7 for j in range(8)]
    _compare(n, layers, {"dep": 1e-3}, factors, 24, obs, nze.NZE_FP64, FP64_TOL)


def test_eight_levels_one_launch_mixed_exact():
    # eight MPOs in one launch, nothing truncated (chi = 256 at n = 8)
    n = 8
    layers = workloads.brickwork(n, 8, seed=22)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    factors = [1.0 + 15.0 * j / 7 for j in range(8)]
    _compare(n, layers, {"dep": 1e-3}, factors, 256, obs, nze.NZE_MIXED, MIXED_TOL)


def test_mixed_truncated_per_level():
    # Truncated mixed run at a cut with a small gap: the smallest relative cut
    # gaps of this circuit are 4.6e-6 (noise 1 x p) and 2.0e-5 (4 x p).  The
    # float64 band polish around the cut resolves the near-degenerate pairs
    # the float32 Jacobi (default thresholds 3e-7 relative, 1e-9 absolute)
    # leaves mixed there, so each level meets the mixed tolerance against
    # the float64 oracle.
    n, chi = 10, 64
    layers = workloads.brickwork(n, 8, seed=21)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    _compare(n, layers, {"dep": 1e-3}, [1.0, 4.0], chi, obs, nze.NZE_MIXED,
             MIXED_TOL)


def test_eight_levels_one_launch_mixed_truncated():
    # the truncated eight-level case of the float64 test above, mixed path
    n = 10
    layers = workloads.brickwork(n, 8, seed=21)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n)
    factors = [1.0 + 15.0 * j / 7 for j in range(8)]
    _compare(n, layers, {"dep": 1e-3}, factors, 24, obs, nze.NZE_MIXED, MIXED_TOL)


@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, FP64_TOL),
                                           (nze.NZE_MIXED, MIXED_TOL)])
def test_server_alone_vs_mix_bitwise(precision, tol):
    # jobs of uneven width, run through the serving loop together and alone:
    # each result is bitwise the same (every MPO runs on its own workgroups
    # with the same arithmetic), and equal to the oracle's within the path's
    # tolerance
    noise = {"dep": 2e-3}
    specs = [(8, 16, 4, 5, 31), (11, 24, 3, 6, 32), (14, 8, 2, 4, 33)]
    jobs = []
    for n, chi, L, depth, seed in specs:
        layers = workloads.brickwork(n, depth, seed=seed)
        factors = list(np.linspace(1.0, 4.0, L))
        ptms = [nze.layer_ptms(us, noise, factors) for _, us in layers]
        obs = workloads.z_singles(n)
        jobs.append((n, chi, [ls for ls, _ in layers], ptms, obs, layers, factors))

    def run(selection):
        srv = nze.Server(256 << 20, max_active=8)
        ids = [srv.submit(n, chi, precision, lss, ptms, obs)
               for (n, chi, lss, ptms, obs, _, _) in selection]
        # a job that could never run is refused at submission and leaves
        # the others untouched
        with pytest.raises(nze.NzeError):
            n0, chi0, lss0, ptms0, obs0 = selection[0][:5]
            srv.submit(n0, chi0, precision, [[0, 1]] + lss0[1:], ptms0, obs0)
        for _ in range(100):
            a, q, d = srv.step()
            if d == len(ids):
                break
        out = [srv.poll(i) for i in ids]
        srv.close()
        return out

    mixed = run(jobs)
    for j, job in enumerate(jobs):
        alone = run([job])[0]
        assert mixed[j][0] == 2 and alone[0] == 2
        assert np.array_equal(mixed[j][1], alone[1])
        assert np.array_equal(mixed[j][2], alone[2])
    # and the mixed run agrees with the oracle
    for j, (n, chi, lss, ptms, obs, layers, factors) in enumerate(jobs):
        orc = _oracle_run(n, layers, noise, factors, chi,
                          tie=(1e-10 if precision == nze.NZE_FP64 else 1e-5))
        for lv, m in enumerate(orc):
            assert np.max(np.abs(mixed[j][1][lv] - m.expectations(obs))) < tol


@pytest.mark.parametrize("precision", [nze.NZE_FP64, nze.NZE_MIXED])
def test_server_backfill_admits_a_fitting_job_past_a_waiting_one(precision):
    # an arena of exactly the second job's footprint: while the first job is
    # resident the second cannot be admitted, and the third, which fits
    # beside the first, is admitted before it (backfill); the second still
    # runs once the first has released its memory, and every result equals
    # the job run alone
    noise = {"dep": 2e-3}
    specs = [(8, 16, 4, 5, 41), (12, 64, 8, 6, 42), (8, 16, 2, 4, 43)]
    jobs = []
    for n, chi, L, depth, seed in specs:
        layers = workloads.brickwork(n, depth, seed=seed)
        factors = list(np.linspace(1.0, 4.0, L))
        ptms = [nze.layer_ptms(us, noise, factors) for _, us in layers]
        jobs.append((n, chi, [ls for ls, _ in layers], ptms, workloads.z_singles(n)))
    fp = [nze.footprint(nze.make_config(n, chi, ptms[0].shape[0], precision))
          for (n, chi, _, ptms, _) in jobs]
    arena = fp[1]
    assert fp[0] + fp[2] <= arena < fp[0] + fp[1]

    def run(selection, arena_bytes):
        srv = nze.Server(arena_bytes, max_active=8)
        ids = [srv.submit(n, chi, precision, lss, ptms, obs)
               for (n, chi, lss, ptms, obs) in selection]
        for _ in range(200):
            a, q, d = srv.step()
            if d == len(ids):
                break
        out = [srv.poll(i) for i in ids]
        srv.close()
        return out

    _say(f"backfill prec={precision}: footprints {fp}, arena {arena}")
    mixed = run(jobs, arena)
    assert all(st == 2 for st, _, _, _ in mixed)
    t_admit = [t[1] for _, _, _, t in mixed]
    t_done = [t[2] for _, _, _, t in mixed]
    assert t_admit[2] < t_admit[1]          # the third job passed the second
    assert t_admit[1] >= t_done[0]          # which waited for the first's memory
    for j, job in enumerate(jobs):
        alone = run([job], 64 << 20)[0]
        assert np.array_equal(mixed[j][1], alone[1])
        assert np.array_equal(mixed[j][2], alone[2])


def test_plain_n8_extrapolation_both_readings():
    # n = 8 workload: extrapolated values from the GPU pipeline (readout +
    # host fit) equal the oracle's; their error against the dense density
    # matrix is the method's accuracy (reported).
    from oracle import dense, fits
    w = workloads.plain_fp64_n8(seed=0)
    layers = w.circuit()
    g = _gpu_run(w.n, layers, w.noise, w.factors, w.chi, nze.NZE_FP64)
    vals, fid, _ = g.expect(w.observables)
    lam = np.array(w.factors) * w.noise["dep"]
    dl = [[(k, U) for k, U in zip(ls, us)] for ls, us in layers]
    p = w.noise["dep"]
    rho_p = dense.run_circuit(w.n, dl, ptm.Noise(dep=p))
    rho_0 = dense.run_circuit(w.n, dl, ptm.Noise())
    err_a, err_b = [], []
    for o, obs in enumerate(w.observables):
        # (i) fit the amplified levels {2,4,8}p, evaluate at lambda* = p
        va, *_ = nze.extrapolate(lam[1:], vals[1:, o], fid[1:], p, nze.NZE_POLY, degree=2)
        ra, _ = fits.fit_poly(lam[1:], vals[1:, o], 2, p)
        # (ii) fit all of {1,2,4,8}p, evaluate at 0
        vb, *_ = nze.extrapolate(lam, vals[:, o], fid, 0.0, nze.NZE_POLY, degree=2)
        rb, _ = fits.fit_poly(lam, vals[:, o], 2, 0.0)
        assert abs(va - ra) < 1e-10 and abs(vb - rb) < 1e-10
        err_a.append(abs(va - dense.expectation(rho_p, w.n, obs).real))
        err_b.append(abs(vb - dense.expectation(rho_0, w.n, obs).real))
    _say(f"n=8 quadratic NZNE (levels 2,4,8 -> p): max err vs dense {max(err_a):.2e}; "
         f"ZNE (levels 1,2,4,8 -> 0): max err vs dense {max(err_b):.2e}")
    assert max(err_a) < 1e-4 and max(err_b) < 1e-3


@pytest.mark.parametrize("precision", [nze.NZE_FP64, nze.NZE_MIXED])
def test_rowortho_sweep_cap_reports_noconv(precision):
    # three sweeps cannot orthogonalise a graded 1024 x 1024 block; the last
    # sweep the cap allows always measures the largest off-diagonal (no
    # forced cross-block-only sweep there), so the cap is an error, not a
    # benign hit at the rounding floor
    R = C = 1024
    rng = np.random.default_rng(5)
    Xin = rng.standard_normal((R, C)) * np.logspace(0, -4, R)[:, None]
    _say(f"rowortho cap R={R} prec={precision}")
    X = _torch_dev(Xin, precision)
    fp64 = precision == nze.NZE_FP64
    with pytest.raises(nze.NzeError) as e:
        nze.kernel_rowortho(X, 1e-13 if fp64 else 1e-7, 1e-15 if fp64 else 1e-8,
                            max_sweeps=3)
    assert e.value.code == nze.NZE_ENOCONV
