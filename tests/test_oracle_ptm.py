"""Pins of the oracle's Pauli-transfer matrices against closed forms.

Every expected value below is a closed form written out by hand from the
channel's definition, not a call back into the oracle's trace formula.
"""
import numpy as np
import pytest

from oracle import ptm
from paper_2501_13237_amd import workloads


def test_depolarizing_closed_form():
    # App. C.2.1: the Kraus form equals rho -> (1 - lam) rho + lam I / 4, whose
    # PTM is diag(1, 1 - lam, ..., 1 - lam).
    for lam in (0.0, 1e-3, 0.3, 1.0):
        R = ptm.ptm_kraus(ptm.kraus_depolarizing2(lam))
        expect = np.diag([1.0] + [1.0 - lam] * 15)
        assert np.max(np.abs(R - expect)) < 1e-14


def test_amplitude_damping_closed_form():
    g = 0.37
    a1 = np.array([[1, 0, 0, 0],
                   [0, np.sqrt(1 - g), 0, 0],
                   [0, 0, np.sqrt(1 - g), 0],
                   [g, 0, 0, 1 - g]])
    k = ptm.kraus_amplitude_damping1(g)
    R = ptm.ptm_kraus(ptm.kraus_product(k, k))
    assert np.max(np.abs(R - np.kron(a1, a1))) < 1e-14
    # non-unital: first column is not e_0, first row still is (trace kept)
    assert abs(R[15, 0] - g * g) < 1e-14
    assert np.max(np.abs(R[0] - np.eye(16)[0])) < 1e-14


def test_pauli_channel_closed_form():
    px, py, pz = 0.01, 0.02, 0.03
    d1 = np.array([1, 1 - 2 * (py + pz), 1 - 2 * (px + pz), 1 - 2 * (px + py)])
    k = ptm.kraus_pauli1(px, py, pz)
    R = ptm.ptm_kraus(ptm.kraus_product(k, k))
    assert np.max(np.abs(R - np.diag(np.kron(d1, d1)))) < 1e-14


def test_matchgate_depolarizing_is_diagonal_and_unital():
    # App. C.3.1: K_0 = sqrt(1 - lam) I, K = sqrt(lam / 7) sigma for the seven
    # matchgate Paulis.  P is kept with weight (1 - lam) + (lam/7) * sum of
    # +-1 (commute / anticommute) -- counted here by hand from the Pauli
    # multiplication table (XY anticommute etc.).
    lam = 0.2
    names = ["ZI", "IZ", "XX", "XY", "YY", "YX", "ZZ"]
    code = {"I": 0, "X": 1, "Y": 2, "Z": 3}
    ks = [np.sqrt(1 - lam) * np.eye(4)]
    for nm in names:
        ks.append(np.sqrt(lam / 7) * ptm.pauli2(4 * code[nm[0]] + code[nm[1]]))
    R = ptm.ptm_kraus(ks)

    def comm1(a, b):     # single-qubit Paulis commute iff equal or one is I
        return 1 if (a == 0 or b == 0 or a == b) else -1

    for P in range(16):
        s = sum(comm1(P // 4, code[nm[0]]) * comm1(P % 4, code[nm[1]])
                for nm in names)
        assert abs(R[P, P] - ((1 - lam) + lam / 7 * s)) < 1e-14
    assert np.max(np.abs(R - np.diag(np.diag(R)))) < 1e-14


def test_unitary_ptm_orthogonal_and_unital():
    rng = np.random.default_rng(3)
    for _ in range(5):
        R = ptm.ptm_unitary(workloads.haar_su4(rng))
        assert np.max(np.abs(R.T @ R - np.eye(16))) < 1e-13
        assert np.max(np.abs(R[0] - np.eye(16)[0])) < 1e-14
        assert np.max(np.abs(R[:, 0] - np.eye(16)[0])) < 1e-14


def test_clifford_ptm_signed_permutation():
    rng = np.random.default_rng(4)
    for _ in range(20):
        R = ptm.ptm_unitary(workloads.random_clifford2(rng))
        A = np.abs(R)
        assert np.allclose(A.sum(axis=0), 1, atol=1e-13)
        assert np.allclose(A.sum(axis=1), 1, atol=1e-13)
        assert np.allclose(A * (1 - A), 0, atol=1e-13)


def test_cnot_ptm_known_entries():
    # CNOT (control = left qubit): X_c I -> X_c X_t, I Z_t -> Z_c Z_t,
    # Z_c I -> Z_c I, I X_t -> I X_t (textbook Heisenberg action).
    CX = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])
    R = ptm.ptm_unitary(CX)
    idx = lambda a, b: 4 * a + b  # noqa: E731
    assert abs(R[idx(1, 1), idx(1, 0)] - 1) < 1e-14
    assert abs(R[idx(3, 3), idx(0, 3)] - 1) < 1e-14
    assert abs(R[idx(3, 0), idx(3, 0)] - 1) < 1e-14
    assert abs(R[idx(0, 1), idx(0, 1)] - 1) < 1e-14


def test_zero_noise_is_the_gate():
    rng = np.random.default_rng(5)
    U = workloads.haar_su4(rng)
    R0 = ptm.ptm_noisy_gate(U, ptm.Noise(dep=0.0, ad=0.0))
    assert np.max(np.abs(R0 - ptm.ptm_unitary(U))) < 1e-15


def test_composition_order_gate_then_channel():
    # U -> C o U (Sec. 2.2.1): for a non-unital C the two orders differ; the
    # oracle must use R_C R_U.  Check on the state |00>: amplitude damping after
    # an X on both qubits moves population back towards |00>.
    X2 = np.kron(ptm.X, ptm.X)
    g = 0.25
    R = ptm.ptm_noisy_gate(X2, ptm.Noise(ad=g))
    v0 = np.zeros(16)
    v0[0], v0[3], v0[12], v0[15] = 1, 1, 1, 1       # |00><00| in Pauli coords
    v = R @ v0
    # after X x X: <Z> = -1 on each qubit, then damping: <Z> = -1 + 2 g
    assert abs(v[12] - (-1 + 2 * g)) < 1e-14
    assert abs(v[3] - (-1 + 2 * g)) < 1e-14


def test_clifford_group_order():
    assert len(workloads.clifford_group2()) == 11520


@pytest.mark.parametrize("seed", [0, 1])
def test_ptm_matches_dense_action(seed):
    # v'_P = Tr(P U rho U^dag) computed densely vs R @ v.
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    rho = A @ A.conj().T
    rho /= np.trace(rho)
    U = workloads.haar_su4(rng)
    v = np.array([np.trace(ptm.PAULI2[P] @ rho).real for P in range(16)])
    rho2 = U @ rho @ U.conj().T
    v2 = np.array([np.trace(ptm.PAULI2[P] @ rho2).real for P in range(16)])
    assert np.max(np.abs(ptm.ptm_unitary(U) @ v - v2)) < 1e-14


# ------------------------------------------- cat-qubit noise, 1-qubit gates


def _anticommute(a, b):
    return not np.allclose(a @ b, b @ a)


def test_cat_pauli_channels_closed_form():
    # A Pauli channel is diagonal in the Pauli basis with
    # f_t = sum_s p_s (-1)^[s, t anticommute]; the commutation is checked on
    # the matrices themselves, not on the index arithmetic.
    lam = 0.013
    for gate, nq in (("Z", 1), ("H", 1), ("CX", 2)):
        probs = ptm.cat_probs(gate, lam)
        assert abs(sum(probs.values()) - {"Z": 1, "H": 5, "CX": 4}[gate] * lam) < 1e-15
        ks = ptm.kraus_pauli_channel(probs)
        basis = ptm.PAULI1 if nq == 1 else ptm.PAULI2
        ops = {k: (ptm.PAULI1[ptm._LETTER[k]] if nq == 1 else
                   np.kron(ptm.PAULI1[ptm._LETTER[k[0]]], ptm.PAULI1[ptm._LETTER[k[1]]]))
               for k in probs}
        p0 = 1.0 - sum(probs.values())
        for ti, t in enumerate(basis):
            f = p0 + sum(p * (-1.0 if _anticommute(ops[k], t) else 1.0)
                         for k, p in probs.items())
            out = sum(K @ t @ K.conj().T for K in ks)
            assert np.max(np.abs(out - f * t)) < 1e-14


def test_cat_hadamard_ptm_closed_form():
    # H maps X <-> Z and Y -> -Y; then Z (3 lam) and X (2 lam) errors scale
    # X by 1 - 6 lam, Y by 1 - 10 lam, Z by 1 - 4 lam (on the left qubit,
    # identity on the right one)
    lam = 0.01
    R = ptm.ptm_1q_on_pair(ptm.H1, ptm.cat_probs("H", lam), 0)
    r = R[0::4, 0::4]                    # right qubit in I
    want = np.array([[1, 0, 0, 0], [0, 0, 0, 1 - 6 * lam],
                     [0, 0, -(1 - 10 * lam), 0], [0, 1 - 4 * lam, 0, 0]])
    assert np.max(np.abs(r - want)) < 1e-14
    # identity on the other qubit: R = r (x) I
    assert np.max(np.abs(R - np.kron(r, np.eye(4)))) < 1e-14


@pytest.mark.parametrize("qubit", [0, 1])
def test_one_qubit_gate_on_pair_matches_dense_action(qubit):
    rng = np.random.default_rng(7 + qubit)
    A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    rho = A @ A.conj().T
    rho /= np.trace(rho)
    u = ptm.rz(0.37) @ ptm.H1
    probs = ptm.cat_probs("H", 0.02)
    ks = [K @ u for K in ptm.kraus_pauli_channel(probs)]
    ks2 = [np.kron(K, ptm.I2) if qubit == 0 else np.kron(ptm.I2, K) for K in ks]
    rho2 = sum(K @ rho @ K.conj().T for K in ks2)
    v = np.array([np.trace(ptm.PAULI2[P] @ rho).real for P in range(16)])
    v2 = np.array([np.trace(ptm.PAULI2[P] @ rho2).real for P in range(16)])
    R = ptm.ptm_1q_on_pair(u, probs, qubit)
    assert np.max(np.abs(R @ v - v2)) < 1e-14
