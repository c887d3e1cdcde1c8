"""Pins of the oracle's diagnostics and noise tables against values worked
out by hand: the MPO entanglement entropy (App. A.1) and the cat-qubit CX row
of the noise table (App. C.2)."""
import numpy as np
import pytest

from oracle import mpo as ompo
from oracle import ptm


def _two_site_mpo(s):
    """n = 2 MPO whose single bond has Schmidt values s: M0 = U, M1 = S V^T
    with orthonormal U (4 x k) and V^T (k x 4)."""
    k = len(s)
    rng = np.random.default_rng(k)
    U, _ = np.linalg.qr(rng.standard_normal((4, k)))
    V, _ = np.linalg.qr(rng.standard_normal((4, k)))
    m = ompo.PauliMPO(2, 16)
    m.sites = [U.reshape(1, 4, k), (np.asarray(s)[:, None] * V.T).reshape(k, 4, 1)]
    m.centre = 1
    return m


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_entropy_of_equal_schmidt_values_is_ln_k(k):
    m = _two_site_mpo([0.7] * k)
    assert abs(m.entanglement_entropy(0) - np.log(k)) < 1e-13


def test_entropy_weights_are_squared_values():
    # s = (sqrt(1/2), sqrt(1/4), sqrt(1/4)) gives p = (1/2, 1/4, 1/4) and
    # S = (1/2) ln 2 + (1/2) ln 4 = (3/2) ln 2; taking p from s instead of s^2,
    # or another logarithm base, changes the value
    m = _two_site_mpo([np.sqrt(0.5), 0.5, 0.5])
    assert abs(m.entanglement_entropy(0) - 1.5 * np.log(2.0)) < 1e-13


def test_entropy_of_product_and_bell_states():
    # |00><00| is a product across the bond: S = 0.  The Bell pair
    # (|00> + |11>)/sqrt(2) has Pauli coordinates v_II = v_XX = v_ZZ = 1,
    # v_YY = -1 (a 4 x 4 matrix with four equal singular values): S = ln 4.
    m = ompo.PauliMPO(2, 16)
    assert abs(m.entanglement_entropy(0)) < 1e-14
    H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    CX = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                  dtype=np.complex128)
    bell = CX @ np.kron(H, np.eye(2))
    m.apply_gate(0, ptm.ptm_unitary(bell), True)
    v = m.pauli_vector().reshape(4, 4)
    assert np.allclose(v, np.diag([1.0, 1.0, -1.0, 1.0]), atol=1e-14)
    assert abs(m.entanglement_entropy(0) - np.log(4.0)) < 1e-13
    # the maximally mixed pair: only v_II, S = 0
    m2 = ompo.PauliMPO(2, 16)
    m2.apply_gate(0, ptm.ptm_noisy_gate(np.eye(4), ptm.Noise(dep=1.0)), True)
    assert abs(m2.entanglement_entropy(0)) < 1e-14


def test_cat_cx_rates_by_hand():
    # CX row of the cat-qubit table (App. C.2): Z on the control (qubit 1,
    # the left site) 3 lam, Z on the target lam / 2, ZZ lam / 2.  The
    # channel is diagonal in the Pauli basis, f_t = 1 - 2 (sum of the rates
    # of the errors that anticommute with t).  For t = a (x) b, with
    # "a flips" meaning a in {X, Y}:
    #   a in {I,Z}, b in {I,Z}: nothing anticommutes           -> 1
    #   a flips,    b in {I,Z}: Z_1 and Z_1 Z_2 (3 + 1/2) lam  -> 1 - 7 lam
    #   a in {I,Z}, b flips:    Z_2 and Z_1 Z_2 (1/2 + 1/2)    -> 1 - 2 lam
    #   a flips,    b flips:    Z_1 and Z_2 (3 + 1/2)          -> 1 - 7 lam
    # Exchanging control and target swaps the two middle rows.
    lam = 0.01
    flips = {0: False, 1: True, 2: True, 3: False}
    expect = np.empty(16)
    for a in range(4):
        for b in range(4):
            fa, fb = flips[a], flips[b]
            expect[4 * a + b] = {(False, False): 1.0, (True, False): 1 - 7 * lam,
                                 (False, True): 1 - 2 * lam,
                                 (True, True): 1 - 7 * lam}[(fa, fb)]
    R = ptm.ptm_gate_pauli(np.eye(4), ptm.cat_probs("CX", lam))
    assert np.max(np.abs(R - np.diag(expect))) < 1e-15
