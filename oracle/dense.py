"""Brute-force density-matrix simulation in the computational basis.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is the exact reference the MPO emulation is checked against at small n:
rho is a dense 2^n x 2^n complex128 matrix, gates act as U rho U^dagger and
noise channels as sum_k K rho K^dagger with the Kraus operators of App. C.2 (and
the textbook channels of ``oracle.ptm``).  No Pauli-transfer matrix and no
Pauli-basis coordinate is used anywhere in this module, so it is independent of
the PTM convention it pins.  Qubit 0 is the most significant bit of the index.
"""
import numpy as np

from .ptm import PAULI1, noise_kraus_sequence


def product_state(bits):
    """Density matrix of the computational-basis product state |bits><bits|."""
    n = len(bits)
    idx = 0
    for b in bits:
        idx = 2 * idx + int(b)
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[idx, idx] = 1.0
    return rho


def apply_two_qubit(rho, n, k, K):
    """rho -> K_(k,k+1) rho K_(k,k+1)^dagger for a 4x4 operator K on qubits
    k (left, more significant) and k+1."""
    a, c = 2 ** k, 2 ** (n - k - 2)
    t = rho.reshape(a, 4, c, a, 4, c)
    t = np.einsum('ij,ajbckd->aibckd', K, t)
    t = np.einsum('ij,ckdajb->ckdaib', K.conj(), t)
    return t.reshape(2 ** n, 2 ** n)


def apply_channel(rho, n, k, kraus):
    out = np.zeros_like(rho)
    for K in kraus:
        out += apply_two_qubit(rho, n, k, K)
    return out


def apply_noisy_gate(rho, n, k, U, noise):
    """The noisy gate C o U on qubits (k, k+1) (Sec. 2.2.1)."""
    rho = apply_two_qubit(rho, n, k, np.asarray(U, dtype=np.complex128))
    for kraus in noise_kraus_sequence(noise):
        rho = apply_channel(rho, n, k, kraus)
    return rho


def apply_pair(rho, n, a, b, K):
    """rho -> K rho K^dagger for a 4x4 operator K on any two distinct qubits
    (a, b), a being the more significant index of K: the action of a
    two-qubit gate on the dense density matrix, for circuits whose gates are
    not nearest neighbours on the chain (2D lattices, Sec. 3)."""
    K4 = np.asarray(K, dtype=np.complex128).reshape(2, 2, 2, 2)
    t = rho.reshape((2,) * (2 * n))
    t = np.tensordot(K4, t, axes=([2, 3], [a, b]))
    t = np.moveaxis(t, [0, 1], [a, b])
    t = np.tensordot(K4.conj(), t, axes=([2, 3], [n + a, n + b]))
    t = np.moveaxis(t, [0, 1], [n + a, n + b])
    return t.reshape(2 ** n, 2 ** n)


def apply_noisy_gate_pair(rho, n, a, b, U, noise):
    """The noisy gate C o U (Sec. 2.2.1) on qubits (a, b), any a != b."""
    rho = apply_pair(rho, n, a, b, U)
    for kraus in noise_kraus_sequence(noise):
        out = np.zeros_like(rho)
        for K in kraus:
            out += apply_pair(rho, n, a, b, K)
        rho = out
    return rho


def run_circuit(n, layers, noise, init_bits=None):
    """Simulate a list of layers; each layer is a list of (k, U) gates acting
    on qubits (k, k+1).  Gates of one layer act on disjoint pairs, so their
    order inside a layer does not matter here."""
    rho = product_state(init_bits if init_bits is not None else [0] * n)
    for layer in layers:
        for k, U in layer:
            rho = apply_noisy_gate(rho, n, k, U, noise)
    return rho


def expectation(rho, n, paulis):
    """Tr(P rho) for the Pauli string ``paulis`` (0=I, 1=X, 2=Y, 3=Z per
    qubit), computed by applying each single-qubit Pauli to the row index."""
    t = rho.reshape((2,) * (2 * n))
    for q, p in enumerate(paulis):
        if p:
            t = np.tensordot(PAULI1[p], t, axes=([1], [q]))
            t = np.moveaxis(t, 0, q)
    m = t.reshape(2 ** n, 2 ** n)
    return np.trace(m)


def frobenius_inner(a, b):
    """<<a|b>> = Tr(a^dagger b), the Frobenius inner product of Sec. 2.1.2."""
    return np.vdot(a, b)
