"""Exact Heisenberg-picture Pauli propagation for Clifford circuits under
Pauli-diagonal noise.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

<O>_rho_T = Tr(O C_T(...C_1(rho_0))) = Tr(C_1^dag(...C_T^dag(O)) rho_0), and for
a noisy gate C = N o U (Sec. 2.2.1) the adjoint is C^dag(O) = U^dag N^dag(O) U.
A Pauli-diagonal channel maps a Pauli string sigma to f_sigma * sigma and a
Clifford U maps it to +-(another Pauli string), so one string and one real
coefficient carry the whole computation and the result is exact.  The
conjugation U^dag sigma U is done by explicit 4x4 matrix products and the
eigenvalue f_sigma from the Kraus operators, so no Pauli-transfer matrix is
involved.
"""
import numpy as np

from .ptm import PAULI2, noise_kraus_sequence


def conjugation_table(U):
    """For each two-qubit Pauli index P: (Q, sign) with U^dag P U = sign * Q."""
    U = np.asarray(U, dtype=np.complex128)
    Ud = U.conj().T
    table = []
    for P in range(16):
        M = Ud @ PAULI2[P] @ U
        coeffs = np.array([np.trace(PAULI2[Q] @ M) / 4.0 for Q in range(16)])
        Q = int(np.argmax(np.abs(coeffs)))
        c = coeffs[Q]
        if abs(abs(c) - 1.0) > 1e-9 or abs(c.imag) > 1e-9:
            raise ValueError("gate is not a Clifford: U^dag P U is not a Pauli")
        others = np.abs(np.delete(coeffs, Q))
        if others.max() > 1e-9:
            raise ValueError("gate is not a Clifford")
        table.append((Q, float(np.sign(c.real))))
    return table


def channel_eigenvalues(kraus_list_seq):
    """f_P with N^dag(P) = f_P P for a composition of Pauli-diagonal two-qubit
    channels (given as a list of Kraus lists)."""
    f = np.ones(16)
    for ks in kraus_list_seq:
        for P in range(16):
            M = sum(K.conj().T @ PAULI2[P] @ K for K in ks)
            coeffs = np.array([np.trace(PAULI2[Q] @ M) / 4.0
                               for Q in range(16)])
            off = np.abs(np.delete(coeffs, P)).max()
            if off > 1e-12:
                raise ValueError("channel is not Pauli-diagonal")
            f[P] *= coeffs[P].real
    return f


def gate_tables(gates):
    """conjugation_table of every gate of a flat (k, U) list, in order."""
    return [conjugation_table(U) for _, U in gates]


def expectation(n, gates, noise, paulis, init_bits=None, tables=None):
    """Exact <paulis> after the gate sequence ``gates`` (a flat list of
    (k, U) in application order, gate on qubits (k, k+1)) with ``noise`` after
    every gate, starting from the product state |init_bits>.  ``tables`` may
    hold gate_tables(gates) when many strings share one circuit."""
    init_bits = init_bits if init_bits is not None else [0] * n
    f = channel_eigenvalues(noise_kraus_sequence(noise))
    tables = tables if tables is not None else gate_tables(gates)
    string = list(paulis)
    coef = 1.0
    for (k, _), table in zip(reversed(gates), reversed(tables)):
        P = 4 * string[k] + string[k + 1]
        coef *= f[P]                       # N^dag first ...
        Q, sign = table[P]                 # ... then U^dag . U
        coef *= sign
        string[k], string[k + 1] = Q // 4, Q % 4
    for q, p in enumerate(string):
        if p in (1, 2):                    # <b|X|b> = <b|Y|b> = 0
            return 0.0
        if p == 3 and init_bits[q]:
            coef = -coef
    return coef
