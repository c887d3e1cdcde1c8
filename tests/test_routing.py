"""Routing of gates on arbitrary qubit pairs onto the chain (nze_route_chain,
nze_ptm_swap_qubits) for 2D-lattice circuits laid out along the chain
(Sec. 3 orders lattice qubits column- or row-major).  Pinned against the
dense density-matrix simulation with the gates applied on their own qubit
pairs (no routing), through the oracle MPO on the routed sequence."""
import numpy as np
import pytest

from oracle import dense, ptm
from oracle import mpo as ompo
from paper_2501_13237_amd import nze, workloads

SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                dtype=np.complex128)


def lattice_edges(rows, cols, periodic_rows=False):
    """Nearest-neighbour edges of a rows x cols lattice, qubit index
    c * rows + r (column-major), optionally periodic along the columns."""
    q = lambda r, c: c * rows + r
    edges = []
    for c in range(cols):
        for r in range(rows):
            if r + 1 < rows:
                edges.append((q(r, c), q(r + 1, c)))
            if c + 1 < cols:
                edges.append((q(r, c), q(r, c + 1)))
            elif periodic_rows and cols > 2:
                edges.append((q(r, c), q(r, 0)))
    return edges


def lattice_circuit(rows, cols, steps, seed, periodic=True):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(steps):
        for a, b in lattice_edges(rows, cols, periodic):
            if rng.random() < 0.5:
                a, b = b, a
            gates.append((a, b, workloads.haar_su4(rng)))
    return gates


@pytest.mark.parametrize("restore", [False, True])
def test_route_chain_ops_are_adjacent_and_oriented(restore):
    rng = np.random.default_rng(3)
    for n in (2, 3, 7, 12):
        pairs = []
        for _ in range(40):
            a, b = rng.choice(n, size=2, replace=False)
            pairs.append((int(a), int(b)))
        ops, perm = nze.route_chain(n, pairs, restore)
        at = list(range(n))
        seen = 0
        for s, g, f in ops:
            assert 0 <= s < n - 1
            if g < 0:
                at[s], at[s + 1] = at[s + 1], at[s]
                continue
            assert g == seen
            a, b = pairs[g]
            assert (at[s], at[s + 1]) == ((b, a) if f else (a, b))
            seen += 1
        assert seen == len(pairs)
        assert [at.index(q) for q in range(n)] == list(perm)
        if restore:
            assert list(perm) == list(range(n))


def test_route_chain_rejects_bad_input():
    with pytest.raises(nze.NzeError):
        nze.route_chain(4, [(0, 4)])
    with pytest.raises(nze.NzeError):
        nze.route_chain(4, [(2, 2)])


@pytest.mark.parametrize("noise", [{}, {"dep": 0.01}, {"dep": 0.01, "ad": 0.02},
                                   {"px": 0.01, "py": 0.002, "pz": 0.03}])
def test_ptm_swap_qubits_is_the_exchanged_gate(noise):
    # the exchanged PTM equals the oracle PTM of SWAP U SWAP with the same
    # (exchange-symmetric) channel, and exchanging twice is the identity
    rng = np.random.default_rng(11)
    U = workloads.haar_su4(rng)
    got = nze.ptm_swap_qubits(nze.build_ptm(U, noise))
    ref = ptm.ptm_noisy_gate(SWAP @ U @ SWAP, ptm.Noise(**noise))
    assert np.max(np.abs(got - ref)) < 1e-14
    assert np.max(np.abs(nze.ptm_swap_qubits(got) - nze.build_ptm(U, noise))) == 0.0


def oracle_routed(n, gates, noise, chi, restore=False):
    """The oracle MPO on the routed op sequence (oracle PTMs; noiseless
    SWAPs), with the ops grouped as the binding groups them."""
    ops, perm = nze.route_chain(n, [(a, b) for a, b, _ in gates], restore)
    nz = ptm.Noise(**noise)
    m = ompo.PauliMPO(n, chi)
    cur = []

    def flush():
        if cur:
            cur.sort(key=lambda o: o[0])
            rs = []
            for s, g, f in cur:
                if g < 0:
                    rs.append(ptm.ptm_noisy_gate(SWAP, ptm.Noise()))
                else:
                    U = gates[g][2]
                    rs.append(ptm.ptm_noisy_gate(SWAP @ U @ SWAP if f else U, nz))
            m.apply_layer([o[0] for o in cur], rs)
        cur.clear()

    used = set()
    for op in ops:
        if op[0] in used or op[0] + 1 in used:
            flush()
            used.clear()
        cur.append(op)
        used.update((op[0], op[0] + 1))
    flush()
    return m, perm


@pytest.mark.parametrize("rows,cols,restore", [(2, 3, False), (3, 2, False), (2, 3, True)])
def test_routed_lattice_circuit_matches_dense(rows, cols, restore):
    n = rows * cols
    gates = lattice_circuit(rows, cols, 2, seed=rows * 10 + cols)
    noise = {"dep": 0.01, "ad": 0.005}
    m, perm = oracle_routed(n, gates, noise, chi=4 ** (n // 2), restore=restore)
    rho = dense.product_state([0] * n)
    for a, b, U in gates:
        rho = dense.apply_noisy_gate_pair(rho, n, a, b, U, ptm.Noise(**noise))
    obs = workloads.z_singles(n) + [workloads.pauli_string(n, {a: "Z", b: "Z"})
                                    for a, b in lattice_edges(rows, cols, True)]
    obs += [workloads.pauli_string(n, {0: "X", n - 1: "Y"})]
    ref = np.array([dense.expectation(rho, n, o).real for o in obs])
    got = m.expectations([nze.permute_paulis(o, perm) for o in obs])
    assert np.max(np.abs(got - ref)) < 1e-12
    assert abs(m.fidelity - 1.0) < 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [(nze.NZE_FP64, 1e-10), (nze.NZE_MIXED, 1e-5)])
def test_routed_lattice_gpu_matches_dense(precision, tol):
    # a 2 x 4 lattice, periodic along the columns, two rounds of Haar gates on
    # every edge, routed onto the chain and run through the HIP path at two
    # noise levels (bond dimension 256: nothing is truncated), against the
    # dense simulation with the gates on their own qubit pairs
    rows, cols = 2, 4
    n = rows * cols
    gates = lattice_circuit(rows, cols, 2, seed=41)
    noise = {"dep": 1e-3}
    factors = [1.0, 4.0]
    print(f"routed lattice {rows}x{cols} precision={precision}", flush=True)
    layers, perm = nze.routed_layers(n, gates, noise, factors, restore=True)
    m = nze.MPO(n, 256, len(factors), precision)
    try:
        for ls, ptms in layers:
            m.apply_layer(ls, ptms)
        obs = workloads.z_singles(n) + [workloads.pauli_string(n, {a: "Z", b: "Z"})
                                        for a, b in lattice_edges(rows, cols, True)]
        obs += [workloads.pauli_string(n, {1: "X", 6: "X"})]
        vals, fid, tr = m.expect([nze.permute_paulis(o, perm) for o in obs])
    finally:
        m.close()
    for j, c in enumerate(factors):
        rho = dense.product_state([0] * n)
        nz = ptm.Noise(**noise).scaled(c)
        for a, b, U in gates:
            rho = dense.apply_noisy_gate_pair(rho, n, a, b, U, nz)
        ref = np.array([dense.expectation(rho, n, o).real for o in obs])
        err = np.max(np.abs(vals[j] - ref))
        print(f"  level {j}: max|dO| = {err:.2e}, F = {fid[j]:.15f}", flush=True)
        assert err < tol
        assert abs(fid[j] - 1.0) < tol


def test_route_chain_swap_counts():
    # with the layout restored after every gate, a gate at chain distance d
    # costs 2 (d - 1) SWAPs; nearest-neighbour gates (a brickwork) cost none
    rng = np.random.default_rng(5)
    n = 9
    pairs = [tuple(int(x) for x in rng.choice(n, size=2, replace=False)) for _ in range(30)]
    ops, perm = nze.route_chain(n, pairs, restore=True)
    assert sum(1 for _, g, _ in ops if g < 0) == sum(2 * (abs(a - b) - 1) for a, b in pairs)
    assert list(perm) == list(range(n))
    brick = [(k, k + 1) for t in range(4) for k in range(t % 2, n - 1, 2)]
    for restore in (False, True):
        ops, perm = nze.route_chain(n, brick, restore)
        assert all(g >= 0 for _, g, _ in ops) and len(ops) == len(brick)


def test_permute_paulis_moves_each_letter_to_its_site():
    perm = np.array([2, 0, 3, 1])
    got = nze.permute_paulis(np.array([1, 2, 3, 0], dtype=np.uint8), perm)
    assert list(got) == [2, 0, 1, 3]
