"""Pins of the MPO oracle: dense density matrices, exact Pauli propagation,
basis invariance, the partial-fidelity definition and special cases."""
import numpy as np
import pytest

from oracle import dense, mpo, mpo_ketbra, pauliprop, ptm
from paper_2501_13237_amd import workloads


def _ptm_layers(layers, noise):
    return [(ls, [ptm.ptm_noisy_gate(U, noise) for U in us])
            for ls, us in layers]


def _dense_layers(layers):
    return [[(k, U) for k, U in zip(ls, us)] for ls, us in layers]


def _random_strings(n, count, rng):
    return [rng.integers(0, 4, size=n).astype(np.uint8) for _ in range(count)]


@pytest.mark.parametrize("noise", [ptm.Noise(dep=0.05),
                                   ptm.Noise(dep=1e-3, ad=0.03),
                                   ptm.Noise(px=0.01, py=0.02, pz=0.03)])
def test_mpo_exact_vs_dense_small(noise):
    n, depth = 6, 6
    layers = workloads.brickwork(n, depth, seed=11)
    m = mpo.run(n, _ptm_layers(layers, noise), chi_max=64)
    rho = dense.run_circuit(n, _dense_layers(layers), noise)
    rng = np.random.default_rng(0)
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n) \
        + _random_strings(n, 20, rng)
    got = m.expectations(obs)
    ref = np.array([dense.expectation(rho, n, o).real for o in obs])
    assert np.max(np.abs(got - ref)) < 1e-12
    assert abs(m.fidelity - 1.0) < 1e-12
    assert abs(m.trace() - 1.0) < 1e-12


def test_mpo_pauli_vector_vs_dense():
    n = 5
    noise = ptm.Noise(dep=0.02, ad=0.01)
    layers = workloads.brickwork(n, 5, seed=3)
    m = mpo.run(n, _ptm_layers(layers, noise), chi_max=64)
    rho = dense.run_circuit(n, _dense_layers(layers), noise)
    v = m.pauli_vector()
    for idx in range(4 ** n):
        digits = [(idx >> (2 * (n - 1 - q))) & 3 for q in range(n)]
        ref = dense.expectation(rho, n, digits).real
        assert abs(v[idx] - ref) < 1e-12


def test_plain_fp64_n8_workload_exact():
    w = workloads.plain_fp64_n8(seed=0)
    layers = w.circuit()
    assert workloads.n_gates(layers) == 28
    for c in w.factors[:2]:
        noise = ptm.Noise(dep=w.noise["dep"] * c)
        m = mpo.run(w.n, _ptm_layers(layers, noise), chi_max=w.chi)
        rho = dense.run_circuit(w.n, _dense_layers(layers), noise)
        got = m.expectations(w.observables)
        ref = np.array([dense.expectation(rho, w.n, o).real
                        for o in w.observables])
        assert np.max(np.abs(got - ref)) < 1e-12
        assert abs(m.fidelity - 1.0) < 1e-12
        assert abs(m.trace() - 1.0) < 1e-12
        # bond dimensions reach the exact caps 4^min(k, n-k) at depth 8
        assert max(m.bond_dims()) <= 256


def test_pauli_propagation_vs_dense():
    n = 6
    noise = ptm.Noise(px=0.02, py=0.01, pz=0.03)
    layers = workloads.brickwork(n, 5, seed=7, kind="clifford")
    rho = dense.run_circuit(n, _dense_layers(layers), noise)
    gates = [g for layer in _dense_layers(layers) for g in layer]
    rng = np.random.default_rng(1)
    for o in workloads.weight1_all(n) + _random_strings(n, 30, rng):
        ref = dense.expectation(rho, n, o).real
        got = pauliprop.expectation(n, gates, noise, o)
        assert abs(got - ref) < 1e-13


def test_clifford_mpo_vs_pauli_propagation():
    # depth 4: each bond is crossed by at most two gates, so chi <= 256 keeps
    # everything exact at any n.
    n = 14
    noise = ptm.Noise(px=3e-3, py=3e-3, pz=3e-3)
    layers = workloads.brickwork(n, 4, seed=5, kind="clifford")
    m = mpo.run(n, _ptm_layers(layers, noise), chi_max=256)
    gates = [g for layer in _dense_layers(layers) for g in layer]
    obs = workloads.weight1_all(n) + workloads.weight2_neighbours(n)
    got = m.expectations(obs)
    ref = np.array([pauliprop.expectation(n, gates, noise, o) for o in obs])
    assert np.max(np.abs(got - ref)) < 1e-12
    assert abs(m.fidelity - 1.0) < 1e-12


def test_mirror_circuit_noise_factors():
    # Clifford layers followed by their inverses: without noise <Z_i> = 1;
    # with Pauli noise it is a nonzero product of channel eigenvalues.
    n = 8
    fwd = workloads.brickwork(n, 3, seed=9, kind="clifford")
    inv = [(ls, [U.conj().T for U in us]) for ls, us in reversed(fwd)]
    layers = fwd + inv
    noise = ptm.Noise(px=1e-2, py=2e-2, pz=5e-3)
    gates = [g for layer in _dense_layers(layers) for g in layer]
    m = mpo.run(n, _ptm_layers(layers, noise), chi_max=256)
    ref = np.array([pauliprop.expectation(n, gates, noise, o)
                    for o in workloads.z_singles(n)])
    assert np.all(np.abs(ref) > 0.3)
    assert np.max(np.abs(m.expectations(workloads.z_singles(n)) - ref)) < 1e-12
    m0 = mpo.run(n, _ptm_layers(layers, ptm.Noise()), chi_max=256)
    assert np.max(np.abs(m0.expectations(workloads.z_singles(n)) - 1)) < 1e-12


@pytest.mark.parametrize("chi", [4, 8, 16])
def test_basis_invariance_truncated(chi):
    n = 8
    noise = ptm.Noise(dep=0.01, ad=0.005)
    layers = workloads.brickwork(n, 6, seed=21)
    pm = mpo.PauliMPO(n, chi)
    km = mpo_ketbra.KetBraMPO(n, chi)
    for ls, us in layers:
        pm.apply_layer(ls, [ptm.ptm_noisy_gate(U, noise) for U in us])
        km.apply_layer(ls, [mpo_ketbra.superop_noisy_gate(U, noise)
                            for U in us])
    assert pm.fidelity < 1.0 - 1e-6          # the truncated regime
    assert np.max(np.abs(np.array(pm.partial_fidelities)
                         - np.array(km.partial_fidelities))) < 1e-10
    obs = workloads.z_singles(n) + workloads.zz_neighbours(n) \
        + _random_strings(n, 10, np.random.default_rng(2))
    assert np.max(np.abs(pm.expectations(obs) - km.expectations(obs))) < 1e-10
    for l in range(n - 1):
        sp, sk = pm.bond_spectrum(l), km.bond_spectrum(l)
        sp, sk = sp / sp[0], sk / sk[0]
        assert np.max(np.abs(sp - sk)) < 1e-10


def _dense_from_pauli_vector(v, n):
    dim = 2 ** n
    rho = np.zeros((dim, dim), dtype=np.complex128)
    for idx in range(4 ** n):
        if v[idx] == 0:
            continue
        P = np.ones((1, 1))
        for q in range(n):
            P = np.kron(P, ptm.PAULI1[(idx >> (2 * (n - 1 - q))) & 3])
        rho += v[idx] * P
    return rho / dim


def test_partial_fidelity_definition():
    # Sec. 2.1.2: f_l = |<<rho_l | C_l rho_{l-1}>>|^2 /
    #                   (||rho_l||^2 ||C_l rho_{l-1}||^2), evaluated densely.
    n, chi = 5, 3
    noise = ptm.Noise(dep=0.02)
    layers = workloads.brickwork(n, 4, seed=13)
    m = mpo.PauliMPO(n, chi)
    for ls, us in layers:
        ltr = ls[0] % 2 == 0
        order = range(len(ls)) if ltr else range(len(ls) - 1, -1, -1)
        for i in order:
            rho_prev = _dense_from_pauli_vector(m.pauli_vector(), n)
            target = dense.apply_noisy_gate(rho_prev, n, ls[i], us[i], noise)
            f = m.apply_gate(ls[i], ptm.ptm_noisy_gate(us[i], noise), ltr)
            rho_now = _dense_from_pauli_vector(m.pauli_vector(), n)
            num = abs(dense.frobenius_inner(rho_now, target)) ** 2
            den = (dense.frobenius_inner(rho_now, rho_now).real
                   * dense.frobenius_inner(target, target).real)
            assert abs(f - num / den) < 1e-12
    assert m.fidelity < 0.9999


def test_fidelity_improves_with_chi_and_converges():
    n = 8
    noise = ptm.Noise(dep=5e-3)
    layers = workloads.brickwork(n, 8, seed=4)
    rho = dense.run_circuit(n, _dense_layers(layers), noise)
    obs = workloads.z_singles(n)
    ref = np.array([dense.expectation(rho, n, o).real for o in obs])
    fids, errs = [], []
    for chi in (4, 16, 64, 256):
        m = mpo.run(n, _ptm_layers(layers, noise), chi_max=chi)
        fids.append(m.fidelity)
        errs.append(np.max(np.abs(m.expectations(obs) - ref)))
    assert fids[0] < fids[1] < fids[2] <= 1.0 + 1e-12
    assert abs(fids[3] - 1.0) < 1e-12 and errs[3] < 1e-12
    assert errs[0] > 1e-6


def test_special_cases():
    n = 6
    layers = workloads.brickwork(n, 4, seed=1)
    # noiseless: the state stays pure, purity 2^-n sum v_P^2 = 1
    m = mpo.run(n, _ptm_layers(layers, ptm.Noise()), chi_max=256)
    v = m.pauli_vector()
    assert abs(np.sum(v * v) / 2 ** n - 1.0) < 1e-12
    # full depolarizing on (2, 3): the pair's reduced state is maximally mixed
    R = ptm.ptm_noisy_gate(np.eye(4), ptm.Noise(dep=1.0))
    m.apply_layer([2], [R])
    z = m.expectations([workloads.pauli_string(n, {2: "Z"}),
                        workloads.pauli_string(n, {3: "Z"}),
                        workloads.pauli_string(n, {2: "X", 3: "Y"})])
    assert np.max(np.abs(z)) < 1e-13
    # identity gate leaves every expectation unchanged
    obs = workloads.weight1_all(n)
    before = m.expectations(obs)
    m.apply_layer([0, 4], [np.eye(16), np.eye(16)])
    assert np.max(np.abs(m.expectations(obs) - before)) < 1e-14


def test_truncation_rank_rule():
    s = np.array([1.0, 0.5, 0.25, 0.25 * (1 + 1e-12), 0.1, 1e-15])
    s = np.sort(s)[::-1]
    # plain chi cut
    assert mpo.truncation_rank(s, 2, 1e-14, 1e-10) == 2
    # cut inside the tied pair at positions 2, 3 -> drop the whole cluster
    assert mpo.truncation_rank(s, 3, 1e-14, 1e-10) == 2
    # tau removes numerical zeros
    assert mpo.truncation_rank(s, 10, 1e-14, 1e-10) == 5
    # a cluster containing s_1 that exceeds chi keeps chi values
    assert mpo.truncation_rank(np.ones(8), 4, 1e-14, 1e-10) == 4
