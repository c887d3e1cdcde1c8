"""Pauli-transfer matrices (PTMs) of two-qubit gates and noise channels.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Conventions (readings of the paper, each recorded in the design notes):

* Single-qubit Paulis are sigma_0..sigma_3 = I, X, Y, Z, the order App. C.2.1
  uses for the depolarizing Kraus operators.
* A two-qubit Pauli is indexed P = 4*p_left + p_right; its 4x4 matrix is
  kron(sigma_p_left, sigma_p_right), the left (lower-index) qubit being the
  most significant bit of the computational-basis index.
* The PTM of a linear map E on two qubits is R[P, Q] = Tr(P E(Q)) / 4.  With
  Pauli coordinates v_P = Tr(P rho) (so rho = sum_P v_P P / 4) this gives
  v'_P = sum_Q R[P, Q] v_Q, the superoperator that acts on the vectorised state
  of Sec. 2.1.1 once that state is written in the Pauli basis.
* A noisy gate is U -> C o U (Sec. 2.2.1, "Parametrised noise models"): the
  unitary acts first, then the channel, so R = R_C @ R_U.
* A noise level scales every parameter of the channel family by one factor
  (the family is one-parameter, Sec. 2.2.1).  Channels compose in the order
  two-qubit depolarizing, then amplitude damping on each qubit, then a Pauli
  channel on each qubit.

Every PTM here is built from the definition (trace formula over Kraus
operators); the closed forms quoted in the paper are checked against it in the
tests, not used here.
"""
from dataclasses import dataclass

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI1 = [I2, X, Y, Z]


def pauli2(P):
    """4x4 matrix of the two-qubit Pauli with index P = 4*p_left + p_right."""
    return np.kron(PAULI1[P // 4], PAULI1[P % 4])


PAULI2 = [pauli2(P) for P in range(16)]


def ptm_of_map(apply_map):
    """R[P, Q] = Tr(P E(Q)) / 4 for a linear map E on two qubits (real part;
    the imaginary part vanishes for Hermiticity-preserving maps)."""
    R = np.empty((16, 16), dtype=np.complex128)
    for Q in range(16):
        EQ = apply_map(PAULI2[Q])
        for P in range(16):
            R[P, Q] = np.trace(PAULI2[P] @ EQ) / 4.0
    assert np.max(np.abs(R.imag)) < 1e-12
    return R.real.copy()


def ptm_unitary(U):
    """PTM of rho -> U rho U^dagger."""
    U = np.asarray(U, dtype=np.complex128)
    Ud = U.conj().T
    return ptm_of_map(lambda A: U @ A @ Ud)


def ptm_kraus(kraus):
    """PTM of rho -> sum_k K rho K^dagger."""
    ks = [np.asarray(K, dtype=np.complex128) for K in kraus]
    return ptm_of_map(lambda A: sum(K @ A @ K.conj().T for K in ks))


# ---------------------------------------------------------------- channels


def kraus_depolarizing2(lam):
    """Two-qubit depolarizing channel, App. C.2.1: K_0 = sqrt(1 - 15 lam/16) I,
    K_ij = sqrt(lam/16) sigma_i sigma_j for (i, j) != (0, 0)."""
    ks = [np.sqrt(1.0 - 15.0 * lam / 16.0) * np.eye(4, dtype=np.complex128)]
    for P in range(1, 16):
        ks.append(np.sqrt(lam / 16.0) * PAULI2[P])
    return ks


def kraus_amplitude_damping1(gamma):
    """Textbook single-qubit amplitude damping (not in the paper; it is part of
    one of the synthetic workloads)."""
    K0 = np.array([[1, 0], [0, np.sqrt(1.0 - gamma)]], dtype=np.complex128)
    K1 = np.array([[0, np.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return [K0, K1]


def kraus_pauli1(px, py, pz):
    """Single-qubit Pauli channel rho -> (1-px-py-pz) rho + px X rho X + ..."""
    return [np.sqrt(1.0 - px - py - pz) * I2, np.sqrt(px) * X,
            np.sqrt(py) * Y, np.sqrt(pz) * Z]


def kraus_product(k_left, k_right):
    """Kraus operators of the product channel (left qubit) x (right qubit)."""
    return [np.kron(a, b) for a in k_left for b in k_right]


@dataclass(frozen=True)
class Noise:
    """Noise family attached after every two-qubit gate.

    dep: two-qubit depolarizing strength lambda (App. C.2.1)
    ad:  amplitude-damping gamma on each of the two qubits
    px, py, pz: single-qubit Pauli channel on each of the two qubits
    """
    dep: float = 0.0
    ad: float = 0.0
    px: float = 0.0
    py: float = 0.0
    pz: float = 0.0

    def scaled(self, c):
        return Noise(self.dep * c, self.ad * c, self.px * c, self.py * c,
                     self.pz * c)


def noise_kraus_sequence(noise):
    """The channels of ``noise`` in application order, as Kraus lists."""
    seq = []
    if noise.dep != 0.0:
        seq.append(kraus_depolarizing2(noise.dep))
    if noise.ad != 0.0:
        k = kraus_amplitude_damping1(noise.ad)
        seq.append(kraus_product(k, k))
    if noise.px != 0.0 or noise.py != 0.0 or noise.pz != 0.0:
        k = kraus_pauli1(noise.px, noise.py, noise.pz)
        seq.append(kraus_product(k, k))
    return seq


def ptm_noisy_gate(U, noise):
    """R = R_C @ R_U: the gate U followed by its noise channel C (Sec. 2.2.1)."""
    R = ptm_unitary(U)
    for ks in noise_kraus_sequence(noise):
        R = ptm_kraus(ks) @ R
    return R


# ------------------------------------------- cat-qubit noise, 1-qubit gates

# Cat-qubit noise model (App. C.2, table of errors per gate at strength lam):
# probability per unit lam of each Pauli error after the gate.  CX: control
# first ("1"), target second ("2").
CAT_RATES = {
    "Z": {"Z": 1.0},                              # Z(theta): Z with lam
    "H": {"Z": 3.0, "X": 2.0},                    # H: Z 3 lam, X 2 lam
    "CX": {"ZI": 3.0, "IZ": 0.5, "ZZ": 0.5},      # CX: Z1 3 lam, Z2 lam/2, Z1Z2 lam/2
}

_LETTER = {"I": 0, "X": 1, "Y": 2, "Z": 3}


def kraus_pauli_channel(probs):
    """Kraus operators sqrt(p_s) s of the Pauli channel rho -> sum_s p_s s rho s
    on one qubit (probs keyed by 'X', ...) or two (keyed by 'ZI', ...); the
    identity keeps 1 - sum p_s."""
    nq = len(next(iter(probs))) if probs else 1
    ks = []
    rest = 1.0
    for key, p in probs.items():
        if p == 0.0:
            continue
        if nq == 1:
            m = PAULI1[_LETTER[key]]
        else:
            m = np.kron(PAULI1[_LETTER[key[0]]], PAULI1[_LETTER[key[1]]])
        ks.append(np.sqrt(p) * m)
        rest -= p
    eye = np.eye(2 ** nq, dtype=np.complex128)
    return [np.sqrt(rest) * eye] + ks


def cat_probs(gate, lam):
    """Error probabilities of a gate of the cat-qubit model at strength lam."""
    return {k: v * lam for k, v in CAT_RATES[gate].items()}


def ptm_gate_pauli(U, probs2):
    """Two-qubit gate U followed by the two-qubit Pauli channel probs2."""
    return ptm_kraus(kraus_pauli_channel(probs2)) @ ptm_unitary(U)


def ptm_1q_on_pair(u, probs1, qubit):
    """16x16 PTM of the single-qubit gate u followed by the Pauli channel
    probs1, on qubit 0 (left) or 1 (right) of a pair, identity on the other:
    built from the two-qubit Kraus operators (sqrt(p_s) s u) (x) I."""
    u = np.asarray(u, dtype=np.complex128)
    ks = [K @ u for K in kraus_pauli_channel(probs1)]
    if qubit == 0:
        ks2 = [np.kron(K, I2) for K in ks]
    else:
        ks2 = [np.kron(I2, K) for K in ks]
    return ptm_kraus(ks2)


def rz(theta):
    """Z(theta) = exp(-i theta Z / 2)."""
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)])


H1 = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
CX_LEFT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                   dtype=np.complex128)   # control on the left qubit
