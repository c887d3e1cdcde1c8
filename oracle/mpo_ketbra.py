"""The same MPO emulation in the paper's own basis: the complex ket-bra
superket index (i_k, j_k) of eq. ``vectorized_dm`` (Sec. 2.1.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Gates act by the complex 16x16 superoperator S[(i1 j1)(i2 j2), (k1 l1)(k2 l2)]
= U[i1 i2, k1 k2] * conj(U[j1 j2, l1 l2]) (summed over Kraus operators for a
channel), built here directly from the operators, never from a Pauli-transfer
matrix.  The map from this basis to Pauli coordinates is a per-site unitary up
to the factor sqrt(2), so the normalised singular values of every two-site
block, the truncation decisions, the partial fidelities and the expectation
values must equal those of ``oracle.mpo.PauliMPO`` -- an independent pin of the
Pauli-basis oracle, including its truncated regime.  Schedule, truncation rule
and normalisation follow ``oracle.mpo`` (same readings).
"""
import numpy as np

from .mpo import truncation_rank
from .ptm import PAULI1, noise_kraus_sequence


def superop(ops):
    """sum over K in ops of K (x) conj(K), regrouped to local (i, j) pairs."""
    S = np.zeros((16, 16), dtype=np.complex128)
    for K in ops:
        K4 = np.asarray(K, dtype=np.complex128).reshape(2, 2, 2, 2)
        # K4[i1, i2, k1, k2]; S[(i1,j1,i2,j2),(k1,l1,k2,l2)]
        T = np.einsum('acbd,egfh->aecgbfdh', K4, K4.conj())
        S += T.reshape(16, 16)
    return S


def superop_noisy_gate(U, noise):
    S = superop([U])
    for kraus in noise_kraus_sequence(noise):
        S = superop(kraus) @ S
    return S


class KetBraMPO:
    def __init__(self, n, chi_max, tau=1e-14, tie_tol=1e-10, init_bits=None):
        self.n, self.chi_max, self.tau, self.tie_tol = n, chi_max, tau, tie_tol
        bits = init_bits if init_bits is not None else [0] * n
        self.sites = []
        for b in bits:
            v = np.zeros(4, dtype=np.complex128)
            v[3 if b else 0] = 1.0            # |b><b| -> index (b, b)
            self.sites.append(v.reshape(1, 4, 1))
        self.log_scale = 0.0
        self.centre = 0
        self.fidelity = 1.0
        self.partial_fidelities = []

    def move_centre(self, target):
        while self.centre < target:
            c = self.centre
            M = self.sites[c]
            cl, _, cr = M.shape
            Q, R = np.linalg.qr(M.reshape(cl * 4, cr))
            self.sites[c] = Q.reshape(cl, 4, Q.shape[1])
            self.sites[c + 1] = np.einsum('ij,jqb->iqb', R, self.sites[c + 1])
            self.centre += 1
        while self.centre > target:
            c = self.centre
            M = self.sites[c]
            cl, _, cr = M.shape
            Q, R = np.linalg.qr(M.reshape(cl, 4 * cr).T)
            self.sites[c] = Q.T.reshape(Q.shape[1], 4, cr)
            self.sites[c - 1] = np.einsum('apj,jk->apk', self.sites[c - 1],
                                          R.T)
            self.centre -= 1

    def apply_gate(self, k, S, left_to_right):
        self.move_centre(k if left_to_right else k + 1)
        A, B = self.sites[k], self.sites[k + 1]
        cl, cr = A.shape[0], B.shape[2]
        theta = np.einsum('apc,cqb->apqb', A, B).reshape(cl, 16, cr)
        theta = np.einsum('PQ,aQb->aPb', S, theta).reshape(cl * 4, 4 * cr)
        U, s, Vt = np.linalg.svd(theta, full_matrices=False)
        r = truncation_rank(s, self.chi_max, self.tau, self.tie_tol)
        s2 = s * s
        kept = s2[:r].sum()
        f = kept / s2.sum()
        nrm = np.sqrt(kept)
        if left_to_right:
            self.sites[k] = U[:, :r].reshape(cl, 4, r)
            self.sites[k + 1] = ((s[:r, None] * Vt[:r]) / nrm).reshape(r, 4, cr)
            self.centre = k + 1
        else:
            self.sites[k] = ((U[:, :r] * s[:r]) / nrm).reshape(cl, 4, r)
            self.sites[k + 1] = Vt[:r].reshape(r, 4, cr)
            self.centre = k
        self.log_scale += np.log(nrm)
        self.fidelity *= f
        self.partial_fidelities.append(f)

    def apply_layer(self, left_sites, superops):
        ls = list(left_sites)
        ltr = (ls[0] % 2 == 0)
        order = range(len(ls)) if ltr else range(len(ls) - 1, -1, -1)
        for i in order:
            self.apply_gate(ls[i], superops[i], ltr)

    def contract(self, paulis):
        v = np.ones(1, dtype=np.complex128)
        for k, p in enumerate(paulis):
            # Tr(P rho_local) = sum_ij P[j, i] rho[i, j]
            w = PAULI1[int(p)].T.reshape(4)
            v = v @ np.einsum('apb,p->ab', self.sites[k], w)
        return v[0]

    def expectations(self, observables):
        cI = self.contract([0] * self.n)
        return np.array([(self.contract(o) / cI).real for o in observables])

    def bond_spectrum(self, l):
        saved = ([s.copy() for s in self.sites], self.centre)
        self.move_centre(l)
        M = self.sites[l]
        s = np.linalg.svd(M.reshape(M.shape[0] * 4, M.shape[2]),
                          compute_uv=False)
        self.sites, self.centre = saved
        return s
